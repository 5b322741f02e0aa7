// Drives libpf's host setup and C ABI through valid and malformed networks
// (host-only plans); built with AddressSanitizer and UBSan by the test.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "pf.h"

namespace {
int failures = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                  \
        }                                                                \
    } while (0)

struct Net {
    int N;
    std::vector<int32_t> f, t, st, lbus, pvbus, sbus, shbus;
    std::vector<double> r, x, b, tap, sh, lp, lq, pvp, pvv, sv, sth, shg, shb;
    pf_network view() {
        pf_network n{};
        n.n_bus = N;
        n.n_branch = int32_t(f.size());
        n.n_load = int32_t(lbus.size());
        n.n_pv = int32_t(pvbus.size());
        n.n_slack = int32_t(sbus.size());
        n.n_shunt = int32_t(shbus.size());
        n.br_from = f.data();
        n.br_to = t.data();
        n.br_r = r.data();
        n.br_x = x.data();
        n.br_b = b.data();
        n.br_tap = tap.data();
        n.br_shift_deg = sh.data();
        n.br_status = st.empty() ? nullptr : st.data();
        n.load_bus = lbus.data();
        n.load_p = lp.data();
        n.load_q = lq.data();
        n.pv_bus = pvbus.data();
        n.pv_p = pvp.data();
        n.pv_v = pvv.data();
        n.slack_bus = sbus.data();
        n.slack_v = sv.data();
        n.slack_theta = sth.data();
        n.shunt_bus = shbus.data();
        n.shunt_g = shg.data();
        n.shunt_b = shb.data();
        return n;
    }
};

// A ring of N buses plus chords (some parallel), a slack, PV units, loads, shunts.
Net ring(int N, unsigned seed) {
    Net n;
    n.N = N;
    std::srand(seed);
    auto add = [&](int a, int c) {
        n.f.push_back(a);
        n.t.push_back(c);
        n.r.push_back(0.01 + 0.001 * (std::rand() % 10));
        n.x.push_back(0.1 + 0.01 * (std::rand() % 10));
        n.b.push_back(0.02);
        n.tap.push_back(std::rand() % 4 ? 1.0 : 1.03);
        n.sh.push_back(std::rand() % 5 ? 0.0 : 2.5);
    };
    for (int i = 0; i < N; ++i) add(i, (i + 1) % N);
    for (int i = 0; i + 3 < N; i += 3) add(i, i + 3);
    add(0, 1);  // parallel to the ring edge
    n.sbus = {0};
    n.sv = {1.0};
    n.sth = {0.0};
    for (int i = 1; i < N; i += 4) {
        n.pvbus.push_back(i);
        n.pvp.push_back(0.5);
        n.pvv.push_back(1.02);
    }
    for (int i = 2; i < N; i += 2) {
        n.lbus.push_back(i);
        n.lp.push_back(0.3);
        n.lq.push_back(0.1);
    }
    if (N > 2) {  // a second load on one bus
        n.lbus.push_back(2);
        n.lp.push_back(0.1);
        n.lq.push_back(0.05);
    }
    for (int i = 0; i < N; i += 7) {
        n.shbus.push_back(i);
        n.shg.push_back(0.001);
        n.shb.push_back(0.1);
    }
    return n;
}

pf_setup_opts host_only() {
    pf_setup_opts o{};
    o.host_only = 1;
    o.device = -1;
    return o;
}

void check_plan(pf_plan *p, int64_t n_expect) {
    int64_t n = 0, nnz = 0;
    CHECK(pf_info(p, &n, &nnz) == PF_OK);
    CHECK(n == n_expect);
    std::vector<int32_t> rp(static_cast<size_t>(n) + 1), ci(static_cast<size_t>(nnz));
    CHECK(pf_pattern(p, rp.data(), ci.data()) == PF_OK);
    CHECK(rp[0] == 0 && rp[size_t(n)] == nnz);
    for (int64_t r = 0; r < n; ++r)
        for (int32_t q = rp[r] + 1; q < rp[r + 1]; ++q) CHECK(ci[q - 1] < ci[q]);
    pf_info_t info{};
    CHECK(pf_info_ex(p, &info) == PF_OK);
    CHECK(info.n == n && info.nnz == nnz);
    CHECK(pf_eval(p, nullptr, nullptr, nullptr, nullptr) == PF_EINVAL);
}

void expect_fail(Net net, int code) {
    pf_network v = net.view();
    pf_setup_opts o = host_only();
    pf_plan *p = nullptr;
    const int rc = pf_setup(&v, &o, &p);
    CHECK(rc == code);
    CHECK(p == nullptr);
    CHECK(pf_last_error()[0] != '\0');
}
}  // namespace

int main() {
    for (int N : {1, 2, 5, 40, 301}) {
        Net net = ring(N, unsigned(N));
        if (N == 1) {
            net.f.clear(); net.t.clear(); net.r.clear(); net.x.clear(); net.b.clear();
            net.tap.clear(); net.sh.clear();
        }
        if (N == 2) {  // ring(2) has two parallel edges and a chord-free layout
            net.pvbus.clear(); net.pvp.clear(); net.pvv.clear();
        }
        pf_network v = net.view();
        pf_setup_opts o = host_only();
        pf_plan *p = nullptr;
        const int rc = pf_setup(&v, &o, &p);
        CHECK(rc == PF_OK);
        if (rc != PF_OK) {
            std::fprintf(stderr, "N=%d: %s\n", N, pf_last_error());
            continue;
        }
        const int64_t NG = int64_t(v.n_pv) + v.n_slack;
        check_plan(p, 2LL * N + NG + v.n_slack);
        for (int te : {64, 128, 4096}) {
            pf_schedule s{};
            s.tile_entries = te;
            CHECK(pf_set_schedule(p, &s) == PF_OK);
            pf_schedule g{};
            CHECK(pf_get_schedule(p, &g) == PF_OK && g.tile_entries == te);
        }
        pf_schedule bad{};
        bad.tile_entries = 65;
        CHECK(pf_set_schedule(p, &bad) == PF_EINVAL);
        pf_destroy(p);
    }
    {   // batch specs
        Net net = ring(40, 7);
        pf_network v = net.view();
        pf_setup_opts o = host_only();
        std::vector<double> ls(3 * size_t(v.n_load), 1.1), ps(3 * size_t(v.n_pv), 0.9);
        std::vector<int32_t> out = {-1, 3, 0};
        pf_batch_spec spec{3, ls.data(), ps.data(), out.data(), 0, PF_LAYOUT_ROWS};
        pf_plan *p = nullptr;
        CHECK(pf_setup_batch(&v, &spec, &o, &p) == PF_OK);
        pf_destroy(p);
        spec.layout = PF_LAYOUT_PANELS;
        CHECK(pf_setup_batch(&v, &spec, &o, &p) == PF_OK);
        pf_destroy(p);
        spec.layout = 7;
        CHECK(pf_setup_batch(&v, &spec, &o, &p) == PF_EINVAL);
        spec.layout = PF_LAYOUT_ROWS;
        out[1] = v.n_branch;
        CHECK(pf_setup_batch(&v, &spec, &o, &p) == PF_EINVAL);
        out[1] = 3;
        ls[5] = NAN;
        CHECK(pf_setup_batch(&v, &spec, &o, &p) == PF_EINVAL);
        ls[5] = 1.0;
        spec.inst_stride = 2;
        CHECK(pf_setup_batch(&v, &spec, &o, &p) == PF_EINVAL);
        spec.n_inst = 0;
        CHECK(pf_setup_batch(&v, &spec, &o, &p) == PF_EINVAL);
    }
    {   // multi-grid
        std::vector<Net> nets = {ring(5, 1), ring(40, 2), ring(17, 3)};
        std::vector<pf_network> v;
        int64_t n_tot = 0;
        for (auto &n : nets) {
            v.push_back(n.view());
            n_tot += 2LL * n.N + v.back().n_pv + 2LL * v.back().n_slack;
        }
        pf_setup_opts o = host_only();
        pf_plan *p = nullptr;
        CHECK(pf_setup_multi(v.data(), int32_t(v.size()), &o, &p) == PF_OK);
        if (p) {
            check_plan(p, n_tot);
            std::vector<int64_t> xo(v.size() + 1), jo(v.size() + 1);
            CHECK(pf_info_multi(p, xo.data(), jo.data()) == PF_OK);
            CHECK(xo.back() == n_tot);
        }
        pf_destroy(p);
        CHECK(pf_setup_multi(v.data(), 0, &o, &p) == PF_EINVAL);
    }
    {   // row orders for diagonal pivots, with and without Q_g slots
        Net net = ring(40, 5);
        pf_network v = net.view();
        pf_setup_opts o = host_only();
        o.q_limits = 1;
        pf_plan *p = nullptr;
        CHECK(pf_setup(&v, &o, &p) == PF_OK);
        if (p) {
            int64_t n = 0, nnz = 0;
            CHECK(pf_info(p, &n, &nnz) == PF_OK);
            std::vector<int32_t> ord(size_t(n), -1), sw(size_t(n), -1), qv(2 * size_t(v.n_pv), -1);
            std::vector<char> seen(size_t(n), 0);
            CHECK(pf_jacobian_row_order(p, ord.data()) == PF_OK);
            CHECK(pf_jacobian_switch_order(p, sw.data(), qv.data()) == PF_OK);
            for (int64_t r = 0; r < n; ++r) {
                CHECK(sw[size_t(r)] >= 0 && sw[size_t(r)] < n);
                if (sw[size_t(r)] >= 0 && sw[size_t(r)] < n) seen[size_t(sw[size_t(r)])] = 1;
                CHECK(sw[size_t(r)] == ord[size_t(r)]);   // every unit under voltage control
            }
            for (int64_t r = 0; r < n; ++r) CHECK(seen[size_t(r)]);
            for (int32_t k = 0; k < v.n_pv; ++k) {
                CHECK(qv[2 * size_t(k)] == 2 * 40 + k);
                CHECK(qv[2 * size_t(k) + 1] == 40 + net.pvbus[size_t(k)]);
                CHECK(sw[size_t(qv[2 * size_t(k)])] == qv[2 * size_t(k) + 1]);
            }
            CHECK(pf_jacobian_switch_order(p, nullptr, nullptr) == PF_EINVAL);
        }
        pf_destroy(p);
        o.q_limits = 0;
        CHECK(pf_setup(&v, &o, &p) == PF_OK);
        if (p) {
            std::vector<int32_t> sw(size_t(2 * 40 + v.n_pv + 2 * v.n_slack));
            CHECK(pf_jacobian_switch_order(p, sw.data(), nullptr) == PF_EINVAL);
        }
        pf_destroy(p);
    }
    {   // malformed networks
        Net n = ring(40, 9);
        n.t[3] = n.f[3];
        expect_fail(n, PF_ETOPO);
        n = ring(40, 9);
        n.t[3] = 40;
        expect_fail(n, PF_EINVAL);
        n = ring(40, 9);
        n.f[0] = -2;
        expect_fail(n, PF_EINVAL);
        n = ring(40, 9);
        n.r[2] = 0.0;
        n.x[2] = 0.0;
        expect_fail(n, PF_EINVAL);
        n = ring(40, 9);
        n.tap[2] = -1.0;
        expect_fail(n, PF_EINVAL);
        n = ring(40, 9);
        n.x[2] = INFINITY;
        expect_fail(n, PF_EINVAL);
        n = ring(40, 9);
        n.pvbus[1] = n.pvbus[0];
        expect_fail(n, PF_ETOPO);
        n = ring(40, 9);
        n.st.assign(n.f.size(), 1);
        n.st[0] = 0;
        n.st[39] = 0;   // bus 0 keeps its chord to bus 3 and the parallel edge
        n.st.back() = 0;
        n.st[40] = 0;   // now bus 0 has no in-service branch
        expect_fail(n, PF_ETOPO);
        n = ring(40, 9);
        n.lbus[0] = 99;
        expect_fail(n, PF_EINVAL);
        n = ring(40, 9);
        n.N = 0;
        expect_fail(n, PF_EINVAL);
        pf_plan *p = nullptr;
        CHECK(pf_setup(nullptr, nullptr, &p) == PF_EINVAL);
        pf_network v = ring(5, 1).view();
        CHECK(pf_setup(&v, nullptr, nullptr) == PF_EINVAL);
        // without host_only the stub device layer reports no GPU
        Net keep = ring(5, 1);
        v = keep.view();
        CHECK(pf_setup(&v, nullptr, &p) == PF_EDEVICE);
        CHECK(p == nullptr);
    }
    pf_destroy(nullptr);
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
