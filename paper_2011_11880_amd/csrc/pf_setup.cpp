// Host-side setup of a plan: validation, per-bus admittance rows, the fixed
// Jacobian pattern with its slot maps, per-generator tables, wavefront
// tiles and bus orders.  Everything here runs once per plan; evaluation
// calls only read what it produced.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <deque>
#include <limits>
#include <numeric>

#include "pf_internal.hpp"

namespace pf {

static thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[768];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

void clear_error() { g_err.clear(); }

const char *last_error() { return g_err.c_str(); }

namespace {

bool finite(double v) { return std::isfinite(v); }

// Checks one network's data (the models of Section II-A) before any
// structure is built from it.
int validate(const pf_network &n, int g) {
    if (n.n_bus < 1) return fail(PF_EINVAL, "grid %d: n_bus must be >= 1", g);
    if (n.n_branch < 0 || n.n_load < 0 || n.n_pv < 0 || n.n_slack < 0 || n.n_shunt < 0)
        return fail(PF_EINVAL, "grid %d: negative group size", g);
    if (n.n_branch > 0 && (!n.br_from || !n.br_to || !n.br_r || !n.br_x || !n.br_b ||
                           !n.br_tap || !n.br_shift_deg))
        return fail(PF_EINVAL, "grid %d: missing branch arrays", g);
    if (n.n_load > 0 && (!n.load_bus || !n.load_p || !n.load_q))
        return fail(PF_EINVAL, "grid %d: missing load arrays", g);
    if (n.n_pv > 0 && (!n.pv_bus || !n.pv_p || !n.pv_v))
        return fail(PF_EINVAL, "grid %d: missing PV arrays", g);
    if (n.n_slack > 0 && (!n.slack_bus || !n.slack_v || !n.slack_theta))
        return fail(PF_EINVAL, "grid %d: missing slack arrays", g);
    if (n.n_shunt > 0 && (!n.shunt_bus || !n.shunt_g || !n.shunt_b))
        return fail(PF_EINVAL, "grid %d: missing shunt arrays", g);
    const int N = n.n_bus;
    std::vector<int> live_deg(N, 0);
    for (int e = 0; e < n.n_branch; ++e) {
        const int f = n.br_from[e], t = n.br_to[e];
        if (f < 0 || f >= N || t < 0 || t >= N)
            return fail(PF_EINVAL, "grid %d: branch %d has a bus index out of range", g, e);
        if (f == t) return fail(PF_ETOPO, "grid %d: branch %d is a self-loop at bus %d", g, e, f);
        const double r = n.br_r[e], x = n.br_x[e];
        if (!finite(r) || !finite(x) || !finite(n.br_b[e]) || !finite(n.br_shift_deg[e]))
            return fail(PF_EINVAL, "grid %d: branch %d has non-finite data", g, e);
        if (r == 0.0 && x == 0.0)
            return fail(PF_EINVAL, "grid %d: branch %d has zero impedance", g, e);
        if (!finite(n.br_tap[e]) || !(n.br_tap[e] > 0.0))
            return fail(PF_EINVAL, "grid %d: branch %d has tap <= 0", g, e);
        const int st = n.br_status ? n.br_status[e] : 1;
        if (st != 0 && st != 1) return fail(PF_EINVAL, "grid %d: branch %d status must be 0/1", g, e);
        if (st) {
            live_deg[f]++;
            live_deg[t]++;
        }
    }
    for (int k = 0; k < n.n_load; ++k) {
        if (n.load_bus[k] < 0 || n.load_bus[k] >= N)
            return fail(PF_EINVAL, "grid %d: load %d bus out of range", g, k);
        if (!finite(n.load_p[k]) || !finite(n.load_q[k]))
            return fail(PF_EINVAL, "grid %d: load %d has non-finite data", g, k);
    }
    std::vector<int> gen_at(N, -1);
    for (int k = 0; k < n.n_pv + n.n_slack; ++k) {
        const bool pv = k < n.n_pv;
        const int bus = pv ? n.pv_bus[k] : n.slack_bus[k - n.n_pv];
        if (bus < 0 || bus >= N)
            return fail(PF_EINVAL, "grid %d: generator %d bus out of range", g, k);
        const double a = pv ? n.pv_p[k] : n.slack_theta[k - n.n_pv];
        const double v = pv ? n.pv_v[k] : n.slack_v[k - n.n_pv];
        if (!finite(a) || !finite(v))
            return fail(PF_EINVAL, "grid %d: generator %d has non-finite data", g, k);
        if (gen_at[bus] >= 0)
            return fail(PF_ETOPO, "grid %d: bus %d has two voltage controllers", g, bus);
        gen_at[bus] = k;
    }
    for (int k = 0; k < n.n_shunt; ++k) {
        if (n.shunt_bus[k] < 0 || n.shunt_bus[k] >= N)
            return fail(PF_EINVAL, "grid %d: shunt %d bus out of range", g, k);
        if (!finite(n.shunt_g[k]) || !finite(n.shunt_b[k]))
            return fail(PF_EINVAL, "grid %d: shunt %d has non-finite data", g, k);
    }
    if (N > 1)
        for (int i = 0; i < N; ++i)
            if (live_deg[i] == 0)
                return fail(PF_ETOPO, "grid %d: bus %d has no in-service branch", g, i);
    return PF_OK;
}

}  // namespace

int build_host_plan(const pf_network *nets, int32_t n_grids, HostPlan &hp) {
    if (!nets || n_grids < 1) return fail(PF_EINVAL, "need at least one network");
    int64_t tot_bus = 0, tot_br = 0, tot_ld = 0, tot_pv = 0, tot_sl = 0, tot_sh = 0;
    for (int g = 0; g < n_grids; ++g) {
        int rc = validate(nets[g], g);
        if (rc) return rc;
        tot_bus += nets[g].n_bus;
        tot_br += nets[g].n_branch;
        tot_ld += nets[g].n_load;
        tot_pv += nets[g].n_pv;
        tot_sl += nets[g].n_slack;
        tot_sh += nets[g].n_shunt;
    }
    const int64_t lim = std::numeric_limits<int32_t>::max() / 4;
    if (tot_bus > lim || tot_br > lim / 2 || tot_ld > lim || tot_pv + tot_sl > lim || tot_sh > lim)
        return fail(PF_EINVAL, "network too large for 32-bit indexing");
    hp.Nt = int32_t(tot_bus);
    hp.Bt = int32_t(tot_br);
    hp.NLt = int32_t(tot_ld);
    hp.NPVt = int32_t(tot_pv);
    hp.NSt = int32_t(tot_sl);
    hp.NGt = int32_t(tot_pv + tot_sl);
    hp.NSHt = int32_t(tot_sh);
    hp.grids.assign(n_grids, GridInfo{});
    hp.yptr.assign(1, 0);
    hp.rowptr.assign(1, 0);
    hp.bus4.clear();
    hp.bus2.clear();
    hp.busx.clear();
    hp.ytr.clear();
    hp.ycol.clear();
    hp.colidx.clear();
    hp.cptr.assign(1, 0);
    hp.clist.clear();
    hp.gen4.clear();
    hp.gen2.clear();
    hp.genpv.clear();
    hp.pv_gen.clear();
    hp.pv_vset.clear();
    hp.pv_mode.assign(size_t(hp.NPVt), 0);
    hp.pv_qt.assign(size_t(hp.NPVt), 0.0);
    hp.br_f.resize(hp.Bt);
    hp.br_t.resize(hp.Bt);
    hp.br_on.resize(hp.Bt);
    hp.params.assign(size_t(hp.n_params()), 0.0);
    hp.pv_p.resize(hp.NPVt);
    hp.shunt_g.resize(hp.NSHt);
    hp.shunt_b.resize(hp.NSHt);
    hp.load_bus.resize(hp.NLt);
    hp.shptr.assign(size_t(hp.Nt) + 1, 0);
    hp.ldptr.assign(size_t(hp.Nt) + 1, 0);
    hp.shlist.resize(hp.NSHt);
    hp.ldlist.resize(hp.NLt);

    const int64_t B = hp.Bt, NL = hp.NLt;
    int64_t xoff = 0, joff = 0;
    int32_t bus_off = 0, br_off = 0, ld_off = 0, pv_off = 0, gen_off = 0, sh_off = 0, y_off = 0;
    for (int g = 0; g < n_grids; ++g) {
        const pf_network &n = nets[g];
        GridInfo &gi = hp.grids[g];
        const int N = n.n_bus, NPV = n.n_pv, NS = n.n_slack, NG = NPV + NS;
        gi.N = N;
        gi.NPV = NPV;
        gi.NS = NS;
        gi.NG = NG;
        gi.NB = n.n_branch;
        gi.NL = n.n_load;
        gi.NSH = n.n_shunt;
        gi.xoff = xoff;
        gi.joff = joff;
        gi.bus_off = bus_off;
        gi.br_off = br_off;
        gi.load_off = ld_off;
        gi.pv_off = pv_off;
        gi.gen_off = gen_off;
        gi.shunt_off = sh_off;
        gi.y_off = y_off;

        // sorted neighbour sets {i} U adj(i) over in-service branches
        std::vector<int32_t> nptr(N + 1, 0);
        for (int e = 0; e < n.n_branch; ++e) {
            if (n.br_status && !n.br_status[e]) continue;
            nptr[n.br_from[e] + 1]++;
            nptr[n.br_to[e] + 1]++;
        }
        for (int i = 0; i < N; ++i) nptr[i + 1] += nptr[i] + 1;  // +1: the bus itself
        std::vector<int32_t> nb(nptr[N]);
        std::vector<int32_t> fillp(nptr.begin(), nptr.end() - 1);
        for (int i = 0; i < N; ++i) nb[fillp[i]++] = i;
        for (int e = 0; e < n.n_branch; ++e) {
            if (n.br_status && !n.br_status[e]) continue;
            const int f = n.br_from[e], t = n.br_to[e];
            nb[fillp[f]++] = t;
            nb[fillp[t]++] = f;
        }
        // per bus: sort, unique -> admittance row; start/len
        std::vector<int32_t> rs(N), rl(N);
        std::vector<int32_t> rowcols;
        rowcols.reserve(nb.size());
        for (int i = 0; i < N; ++i) {
            auto b0 = nb.begin() + nptr[i], b1 = nb.begin() + nptr[i + 1];
            std::sort(b0, b1);
            auto end = std::unique(b0, b1);
            rs[i] = int32_t(rowcols.size());
            rl[i] = int32_t(end - b0);
            rowcols.insert(rowcols.end(), b0, end);
        }
        const int32_t ny = int32_t(rowcols.size());
        gi.n_y = ny;
        if (int64_t(y_off) + ny > lim) return fail(PF_EINVAL, "network too large");

        // generator at each bus (local generator index g: PV first, then slack)
        std::vector<int32_t> gen_at(N, -1), slack_at(N, -1);
        for (int k = 0; k < NPV; ++k) gen_at[n.pv_bus[k]] = k;
        for (int s = 0; s < NS; ++s) {
            gen_at[n.slack_bus[s]] = NPV + s;
            slack_at[n.slack_bus[s]] = s;
        }

        // Jacobian row lengths: P_i, Q_i, then V rows, then theta rows
        const int64_t nloc = 2LL * N + NG + NS;
        std::vector<int64_t> rp(nloc + 1, 0);
        for (int i = 0; i < N; ++i) {
            rp[i + 1] = 2LL * rl[i] + (slack_at[i] >= 0 ? 1 : 0);
            rp[N + i + 1] = 2LL * rl[i] + (gen_at[i] >= 0 ? 1 : 0);
        }
        for (int k = 0; k < NG + NS; ++k) rp[2LL * N + k + 1] = (hp.q_slots && k < NPV) ? 2 : 1;
        for (int64_t r = 0; r < nloc; ++r) rp[r + 1] += rp[r];
        const int64_t nnz = rp[nloc];
        if (joff + nnz >= std::numeric_limits<int32_t>::max())
            return fail(PF_EINVAL, "Jacobian too large for 32-bit indexing");
        gi.nnz = nnz;

        // pattern (absolute indices)
        hp.colidx.resize(size_t(joff + nnz));
        for (int64_t r = 0; r < nloc; ++r) hp.rowptr.push_back(int32_t(joff + rp[r + 1]));
        for (int i = 0; i < N; ++i) {
            for (int pass = 0; pass < 2; ++pass) {   // P row then Q row
                int64_t p = joff + rp[pass * N + i];
                for (int q = 0; q < rl[i]; ++q) hp.colidx[p++] = int32_t(xoff + rowcols[rs[i] + q]);
                for (int q = 0; q < rl[i]; ++q) hp.colidx[p++] = int32_t(xoff + N + rowcols[rs[i] + q]);
                if (pass == 0 && slack_at[i] >= 0)
                    hp.colidx[p++] = int32_t(xoff + 2LL * N + NG + slack_at[i]);
                if (pass == 1 && gen_at[i] >= 0)
                    hp.colidx[p++] = int32_t(xoff + 2LL * N + gen_at[i]);
            }
        }
        for (int k = 0; k < NG; ++k) {
            const int bus = k < NPV ? n.pv_bus[k] : n.slack_bus[k - NPV];
            hp.colidx[size_t(joff + rp[2LL * N + k])] = int32_t(xoff + N + bus);
            if (hp.q_slots && k < NPV)   // the unit's own Q_g column (the diagonal)
                hp.colidx[size_t(joff + rp[2LL * N + k]) + 1] = int32_t(xoff + 2LL * N + k);
        }
        for (int s = 0; s < NS; ++s)
            hp.colidx[size_t(joff + rp[2LL * N + NG + s])] = int32_t(xoff + n.slack_bus[s]);

        // admittance rows and per-bus slot maps
        for (int i = 0; i < N; ++i) {
            const int32_t ys = y_off + rs[i];
            int32_t pd = -1;
            for (int q = 0; q < rl[i]; ++q) {
                const int32_t c = rowcols[rs[i] + q];
                if (c == i) pd = q;
                hp.ycol.push_back(q == 0 ? (c | kRowStart) : c);
            }
            hp.yptr.push_back(ys + rl[i]);
            hp.bus4.push_back(ys);
            hp.bus4.push_back(ys + rl[i]);
            hp.bus4.push_back(int32_t(joff + rp[i]));
            hp.bus4.push_back(int32_t(joff + rp[N + i]));
            hp.bus2.push_back(pd);
            hp.bus2.push_back(gen_at[i] >= 0 ? gen_off + gen_at[i] : -1);
            hp.busx.push_back(int32_t(xoff + i));
            hp.busx.push_back(int32_t(xoff + N + i));
        }
        // transpose partner of every off-diagonal entry (the pattern is
        // structurally symmetric)
        for (int i = 0; i < N; ++i) {
            for (int q = 0; q < rl[i]; ++q) {
                const int32_t c = rowcols[rs[i] + q];
                if (c == i) {
                    hp.ytr.push_back(-1);
                    continue;
                }
                auto b0 = rowcols.begin() + rs[c], b1 = b0 + rl[c];
                const int32_t pos = int32_t(std::lower_bound(b0, b1, i) - rowcols.begin());
                hp.ytr.push_back(y_off + pos);
            }
        }

        // contributions of each in-service branch to the four entries it
        // touches, appended in ascending branch order
        auto pos = [&](int i, int c) -> int32_t {
            auto b0 = rowcols.begin() + rs[i], b1 = b0 + rl[i];
            return int32_t(std::lower_bound(b0, b1, c) - rowcols.begin());
        };
        std::vector<int32_t> cnt(size_t(ny) + 1, 0);
        for (int e = 0; e < n.n_branch; ++e) {
            if (n.br_status && !n.br_status[e]) continue;
            const int f = n.br_from[e], t = n.br_to[e];
            cnt[pos(f, f) + 1]++;
            cnt[pos(f, t) + 1]++;
            cnt[pos(t, f) + 1]++;
            cnt[pos(t, t) + 1]++;
        }
        for (int q = 0; q < ny; ++q) cnt[q + 1] += cnt[q];
        const int32_t cbase = hp.cptr.back();
        for (int q = 0; q < ny; ++q) hp.cptr.push_back(cbase + cnt[q + 1]);
        hp.clist.resize(size_t(cbase) + cnt[ny]);
        std::vector<int32_t> cf(cnt.begin(), cnt.end() - 1);
        for (int e = 0; e < n.n_branch; ++e) {
            if (n.br_status && !n.br_status[e]) continue;
            const int f = n.br_from[e], t = n.br_to[e];
            const int32_t gb = br_off + e;
            hp.clist[cbase + cf[pos(f, f)]++] = (gb << 2) | K_FF;
            hp.clist[cbase + cf[pos(f, t)]++] = (gb << 2) | K_FT;
            hp.clist[cbase + cf[pos(t, f)]++] = (gb << 2) | K_TF;
            hp.clist[cbase + cf[pos(t, t)]++] = (gb << 2) | K_TT;
        }

        // raw data
        for (int e = 0; e < n.n_branch; ++e) {
            const int64_t ge = br_off + e;
            hp.br_f[ge] = bus_off + n.br_from[e];
            hp.br_t[ge] = bus_off + n.br_to[e];
            hp.br_on[ge] = n.br_status ? n.br_status[e] : 1;
            hp.params[ge] = n.br_r[e];
            hp.params[B + ge] = n.br_x[e];
            hp.params[2 * B + ge] = n.br_b[e];
            hp.params[3 * B + ge] = n.br_tap[e];
            hp.params[4 * B + ge] = n.br_shift_deg[e];
        }
        for (int k = 0; k < n.n_load; ++k) {
            hp.load_bus[ld_off + k] = bus_off + n.load_bus[k];
            hp.params[5 * B + ld_off + k] = n.load_p[k];
            hp.params[5 * B + NL + ld_off + k] = n.load_q[k];
        }
        for (int k = 0; k < NPV; ++k) hp.pv_p[pv_off + k] = n.pv_p[k];
        for (int k = 0; k < n.n_shunt; ++k) {
            hp.shunt_g[sh_off + k] = n.shunt_g[k];
            hp.shunt_b[sh_off + k] = n.shunt_b[k];
        }
        // generator tables
        for (int k = 0; k < NG; ++k) {
            const bool pv = k < NPV;
            const int s = k - NPV;
            hp.gen4.push_back(int32_t(xoff + 2LL * N + k));
            hp.gen4.push_back(int32_t(joff + rp[2LL * N + k]));
            hp.gen4.push_back(pv ? (hp.q_slots ? kGenVoltageSlot : kGenVoltage)
                                 : int32_t(xoff + 2LL * N + NG + s));
            hp.gen4.push_back(pv ? -1 : int32_t(joff + rp[2LL * N + NG + s]));
            hp.gen2.push_back(pv ? n.pv_v[k] : n.slack_v[s]);
            hp.gen2.push_back(pv ? 0.0 : n.slack_theta[s]);
            hp.genpv.push_back(pv ? pv_off + k : -1);
            if (pv) {
                hp.pv_gen.push_back(gen_off + k);
                hp.pv_vset.push_back(n.pv_v[k]);
            }
        }
        // shunts and loads per bus (stable: input order within a bus)
        for (int k = 0; k < n.n_shunt; ++k) hp.shptr[bus_off + n.shunt_bus[k] + 1]++;
        for (int k = 0; k < n.n_load; ++k) hp.ldptr[bus_off + n.load_bus[k] + 1]++;

        xoff += nloc;
        joff += nnz;
        bus_off += N;
        br_off += n.n_branch;
        ld_off += n.n_load;
        pv_off += NPV;
        gen_off += NG;
        sh_off += n.n_shunt;
        y_off += ny;
    }
    for (int i = 0; i < hp.Nt; ++i) {
        hp.shptr[i + 1] += hp.shptr[i];
        hp.ldptr[i + 1] += hp.ldptr[i];
    }
    {
        std::vector<int32_t> fs(hp.shptr.begin(), hp.shptr.end() - 1);
        std::vector<int32_t> fl(hp.ldptr.begin(), hp.ldptr.end() - 1);
        int32_t so = 0, lo = 0;
        for (int g = 0; g < n_grids; ++g) {
            const pf_network &n = nets[g];
            const int32_t bo = hp.grids[g].bus_off;
            for (int k = 0; k < n.n_shunt; ++k) hp.shlist[fs[bo + n.shunt_bus[k]]++] = so + k;
            for (int k = 0; k < n.n_load; ++k) hp.ldlist[fl[bo + n.load_bus[k]]++] = lo + k;
            so += n.n_shunt;
            lo += n.n_load;
        }
    }
    hp.n = xoff;
    hp.nnz = joff;
    hp.n_y = y_off;

    // bus processing orders (batched kernel): natural and breadth-first
    hp.order_natural.resize(hp.Nt);
    std::iota(hp.order_natural.begin(), hp.order_natural.end(), 0);
    hp.order_bfs.clear();
    hp.order_bfs.reserve(hp.Nt);
    std::vector<char> seen(hp.Nt, 0);
    std::deque<int32_t> dq;
    for (int g = 0; g < n_grids; ++g) {
        const GridInfo &gi = hp.grids[g];
        for (int s = 0; s < gi.N; ++s) {
            const int32_t root = gi.bus_off + s;
            if (seen[root]) continue;
            seen[root] = 1;
            dq.push_back(root);
            while (!dq.empty()) {
                const int32_t b = dq.front();
                dq.pop_front();
                hp.order_bfs.push_back(b);
                for (int32_t e = hp.yptr[b]; e < hp.yptr[b + 1]; ++e) {
                    const int32_t nbg = gi.bus_off + (hp.ycol[e] & kColMask);
                    if (!seen[nbg]) {
                        seen[nbg] = 1;
                        dq.push_back(nbg);
                    }
                }
            }
        }
    }
    build_adjoint_order(hp);
    return PF_OK;
}

// Adjoint work lists.  Each grid's buses fill positions [bus_off, bus_off +
// N) of order_bfs, so tiles of whole rows taken along that order (at most
// kAdjTileEntries entries unless one row is longer) never cross grids.  Each
// in-service branch is assigned to the position of its (from, to) entry.
void build_adjoint_order(HostPlan &hp) {
    hp.adj_src.clear();
    hp.adj_tiles.clear();
    hp.adj_src.reserve(size_t(hp.n_y));
    for (int g = 0; g < int(hp.grids.size()); ++g) {
        const GridInfo &gi = hp.grids[g];
        int32_t q = gi.bus_off;
        const int32_t qend = gi.bus_off + gi.N;
        while (q < qend) {
            const int32_t q0 = q;
            const int32_t e0 = int32_t(hp.adj_src.size());
            int32_t cnt = 0;
            while (q < qend) {
                const int32_t b = hp.order_bfs[q];
                const int32_t len = hp.yptr[b + 1] - hp.yptr[b];
                if (cnt > 0 && cnt + len > kAdjTileEntries) break;
                for (int32_t e = hp.yptr[b]; e < hp.yptr[b + 1]; ++e) hp.adj_src.push_back(e);
                cnt += len;
                ++q;
            }
            hp.adj_tiles.push_back(e0);
            hp.adj_tiles.push_back(e0 + cnt);
            hp.adj_tiles.push_back(q0);
            hp.adj_tiles.push_back(g);
        }
    }
    std::vector<int32_t> at(size_t(hp.n_y));
    for (size_t q = 0; q < hp.adj_src.size(); ++q) at[size_t(hp.adj_src[q])] = int32_t(q);
    hp.adj_own.assign(size_t(hp.n_y), -1);
    hp.adj_left.clear();
    for (const GridInfo &gi : hp.grids) {
        for (int32_t e = gi.br_off; e < gi.br_off + gi.NB; ++e) {
            if (!hp.br_on[e]) {
                hp.adj_left.push_back(e);
                continue;
            }
            const int32_t f = hp.br_f[e], tl = hp.br_t[e] - gi.bus_off;
            int32_t q = hp.yptr[f];
            while (q < hp.yptr[f + 1] && (hp.ycol[q] & kColMask) != tl) ++q;
            int32_t *own = q < hp.yptr[f + 1] ? &hp.adj_own[size_t(at[size_t(q)])] : nullptr;
            if (own && *own < 0)
                *own = e;
            else
                hp.adj_left.push_back(e);
        }
    }
}

int attach_batch(const pf_batch_spec *spec, HostPlan &hp) {
    if (!spec) return fail(PF_EINVAL, "batch spec is NULL");
    if (spec->n_inst < 1) return fail(PF_EINVAL, "n_inst must be >= 1");
    const int64_t I = spec->n_inst;
    if (spec->inst_stride != 0 && spec->inst_stride < spec->n_inst)
        return fail(PF_EINVAL, "inst_stride must be 0 or >= n_inst");
    if (spec->layout != PF_LAYOUT_ROWS && spec->layout != PF_LAYOUT_PANELS)
        return fail(PF_EINVAL, "unknown batched layout %d", spec->layout);
    hp.kind = KIND_BATCH;
    hp.n_inst = spec->n_inst;
    hp.panels = spec->layout == PF_LAYOUT_PANELS;
    // panels: the overlay tables keep a row pitch of n_inst internally
    hp.ld = (spec->inst_stride && !hp.panels) ? spec->inst_stride : spec->n_inst;
    const int64_t LD = hp.ld;
    if (int64_t(hp.nnz) * LD > (int64_t(1) << 40))
        return fail(PF_EINVAL, "batch too large");
    hp.load_scale_t.clear();
    hp.pv_scale_t.clear();
    hp.outage.clear();
    if (spec->load_scale && hp.NLt > 0) {
        hp.load_scale_t.assign(size_t(hp.NLt) * LD, 1.0);
        for (int64_t k = 0; k < I; ++k)
            for (int64_t l = 0; l < hp.NLt; ++l) {
                const double s = spec->load_scale[k * hp.NLt + l];
                if (!finite(s)) return fail(PF_EINVAL, "load_scale[%lld][%lld] is not finite",
                                            (long long)k, (long long)l);
                hp.load_scale_t[l * LD + k] = s;
            }
    }
    if (spec->pv_scale && hp.NPVt > 0) {
        hp.pv_scale_t.assign(size_t(hp.NPVt) * LD, 1.0);
        for (int64_t k = 0; k < I; ++k)
            for (int64_t l = 0; l < hp.NPVt; ++l) {
                const double s = spec->pv_scale[k * hp.NPVt + l];
                if (!finite(s)) return fail(PF_EINVAL, "pv_scale[%lld][%lld] is not finite",
                                            (long long)k, (long long)l);
                hp.pv_scale_t[l * LD + k] = s;
            }
    }
    if (spec->outage) {
        hp.outage.resize(size_t(I));
        bool any = false;
        for (int64_t k = 0; k < I; ++k) {
            const int32_t o = spec->outage[k];
            if (o < -1 || o >= hp.Bt)
                return fail(PF_EINVAL, "outage[%lld] = %d out of range", (long long)k, o);
            if (o >= 0 && !hp.br_on[o])
                return fail(PF_EINVAL, "outage[%lld]: branch %d is already out of service",
                            (long long)k, o);
            hp.outage[k] = o;
            any = any || o >= 0;
        }
        if (!any) hp.outage.clear();
    }
    return PF_OK;
}

int normalise_schedule(const HostPlan &hp, const pf_schedule *in, pf_schedule &s) {
    pf_schedule d{};
    if (in) d = *in;
    // defaults: the fastest schedules measured on MI355X for the 70,000-bus
    // grid (single instance) and its 1000-state batch (batched: groups of 8
    // instance chunks, 4 buses per work item in breadth-first order, 8 waves
    // per block, contiguous work per XCD)
    const bool batch = hp.kind == KIND_BATCH;
    if (d.tile_entries == 0) d.tile_entries = 64;
    if (d.batch_buses == 0) d.batch_buses = batch ? 4 : 1;
    if (d.batch_order == 0) d.batch_order = batch ? 2 : 1;
    if (d.xcd_remap == 0) d.xcd_remap = 1;
    if (d.batch_group == 0) d.batch_group = batch ? 8 : 64;
    if (d.waves_per_block == 0) d.waves_per_block = batch ? 8 : 2;
    if (d.grid_blocks == 0) d.grid_blocks = -1;
    if (d.tile_entries < 64 || d.tile_entries % 64 || d.tile_entries > (1 << 20))
        return fail(PF_EINVAL, "tile_entries must be a multiple of 64 in [64, 2^20]");
    if (d.waves_per_block < 1 || d.waves_per_block > 8)
        return fail(PF_EINVAL, "waves_per_block must be in [1, 8]");
    if (d.grid_blocks < -1 || d.grid_blocks > (1 << 20))
        return fail(PF_EINVAL, "grid_blocks must be -1, 0 or in [1, 2^20]");
    if (d.batch_buses < 1 || d.batch_buses > (1 << 16))
        return fail(PF_EINVAL, "batch_buses must be in [1, 65536]");
    if (d.batch_order < 1 || d.batch_order > 2) return fail(PF_EINVAL, "batch_order must be 1 or 2");
    if (d.xcd_remap < 1 || d.xcd_remap > 2) return fail(PF_EINVAL, "xcd_remap must be 1 or 2");
    if (d.batch_group < 1 || d.batch_group > 64)
        return fail(PF_EINVAL, "batch_group must be in [1, 64]");
    s = d;
    return PF_OK;
}

// Wavefront tiles of whole admittance rows: greedy, at most tile_entries
// entries unless a single row is longer.  Tiles never cross grids.  Each
// tile records its entry range, first bus, grid, and the contiguous ranges
// of Jacobian values its P rows and Q rows occupy.
void build_tiles(HostPlan &hp) {
    hp.tiles.clear();
    const int32_t cap = hp.sched.tile_entries;
    for (int g = 0; g < int(hp.grids.size()); ++g) {
        const GridInfo &gi = hp.grids[g];
        int32_t b = gi.bus_off;
        const int32_t bend = gi.bus_off + gi.N;
        while (b < bend) {
            const int32_t b0 = b;
            const int32_t e0 = hp.yptr[b];
            int32_t e1 = hp.yptr[b + 1];
            ++b;
            while (b < bend && hp.yptr[b + 1] - e0 <= cap) {
                e1 = hp.yptr[b + 1];
                ++b;
            }
            const int64_t r_first = gi.xoff + (b0 - gi.bus_off);
            const int64_t r_last = gi.xoff + (b - 1 - gi.bus_off);
            hp.tiles.push_back(e0);
            hp.tiles.push_back(e1);
            hp.tiles.push_back(b0);
            hp.tiles.push_back(g);
            // Jacobian value ranges of the tile's P rows and Q rows
            hp.tiles.push_back(hp.rowptr[r_first]);
            hp.tiles.push_back(hp.rowptr[r_last + 1]);
            hp.tiles.push_back(hp.rowptr[r_first + gi.N]);
            hp.tiles.push_back(hp.rowptr[r_last + 1 + gi.N]);
        }
    }
}

}  // namespace pf
