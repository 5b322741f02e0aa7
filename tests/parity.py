"""Shared comparison helpers for the GPU parity tests.

Tolerance (floating point): an entry passes when
    |gpu - oracle| <= 1e-12 |oracle| + 1e-14            (primary bar)
or, for sums whose terms cancel,
    |gpu - oracle| <= 1e-12 S + 1e-14                   (fallback)
where S is the sum of the absolute values of the terms the oracle added for
that entry.  Both sides compute in FP64 but fold in different orders (the
oracle per branch and model, the library per admittance entry), so a
cancelling sum can lose relative accuracy on either side; S bounds that
loss.  Such entries are rare (a random sum lands within 1e-4 S of zero about
once in 10^4 entries), so every comparison also asserts that at most
FALLBACK_FRAC of its entries (at least one) needed the fallback, and records
the count; the session summary prints the totals.  Helpers return how many
entries needed the fallback.
"""

import numpy as np

RTOL = 1e-12
ATOL = 1e-14
FALLBACK_FRAC = 1e-4

# (what, entries compared, entries that needed the fallback) per comparison
RECORD = []


def check_close(gpu, ora, scale, what="", max_fallback=None):
    gpu = np.asarray(gpu, dtype=np.float64)
    ora = np.asarray(ora, dtype=np.float64)
    scale = np.asarray(scale, dtype=np.float64)
    assert gpu.shape == ora.shape == scale.shape, (what, gpu.shape, ora.shape, scale.shape)
    assert np.all(np.isfinite(gpu)), what + ": non-finite values"
    err = np.abs(gpu - ora)
    prim = err <= RTOL * np.abs(ora) + ATOL
    fb = err <= RTOL * scale + ATOL
    bad = ~(prim | fb)
    if np.any(bad):
        k = int(np.argmax(np.where(bad, err / (np.abs(ora) + scale + 1e-300), 0)))
        raise AssertionError(
            f"{what}: {int(bad.sum())} of {bad.size} entries off; worst at {k}: "
            f"gpu={gpu[k]!r} oracle={ora[k]!r} scale={scale[k]!r}")
    n_fb = int(np.sum(~prim & fb))
    limit = max(1, int(FALLBACK_FRAC * gpu.size)) if max_fallback is None else max_fallback
    RECORD.append((what, int(gpu.size), n_fb))
    assert n_fb <= limit, (f"{what}: {n_fb} of {gpu.size} entries passed only through the "
                           f"cancellation fallback (at most {limit} allowed)")
    return n_fb


def oracle_on_pattern(rp, ci, J_ora, A_ora):
    """Oracle Jacobian values and scales laid out on the library pattern
    (rp, ci).  Entries of the pattern that the oracle lacks get 0 (those
    must come out exactly 0 from the library, e.g. an outaged pair)."""
    n = rp.shape[0] - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    keys = rows * n + ci.astype(np.int64)
    J_ora = J_ora.tocsr()
    J_ora.sort_indices()
    A_ora = A_ora.tocsr()
    A_ora.sort_indices()
    orow = np.repeat(np.arange(n, dtype=np.int64), np.diff(J_ora.indptr))
    okeys = orow * n + J_ora.indices.astype(np.int64)
    pos = np.searchsorted(keys, okeys)
    assert np.all(pos < keys.size) and np.all(keys[pos] == okeys), \
        "oracle has entries outside the library pattern"
    v = np.zeros(keys.size)
    s = np.zeros(keys.size)
    present = np.zeros(keys.size, bool)
    v[pos] = J_ora.data
    s[pos] = A_ora.data
    present[pos] = True
    return v, s, present


def check_jacobian(rp, ci, vals, J_ora, A_ora, what="J"):
    v, s, present = oracle_on_pattern(rp, ci, J_ora, A_ora)
    vals = np.asarray(vals)
    absent = ~present
    if np.any(absent):
        assert np.all(vals[absent] == 0.0), what + ": entries absent from the oracle are not 0"
    return check_close(vals[present], v[present], s[present], what)


def pattern_keys(rp, ci):
    """Sorted keys row * n + col of a CSR pattern with sorted columns."""
    n = rp.shape[0] - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    return rows * n + ci.astype(np.int64)


def triplet_positions(keys, n, rows, cols):
    """Position in the pattern (keys from pattern_keys) of every oracle
    triplet; reusable for every instance whose triplets share one structure."""
    tk = rows.astype(np.int64) * n + cols.astype(np.int64)
    pos = np.searchsorted(keys, tk)
    assert np.all(pos < keys.size) and np.all(keys[pos] == tk), \
        "oracle has entries outside the library pattern"
    return pos


def check_jacobian_triplets(vals, keys, pos, trip_vals, trip_scales, what="J"):
    """The oracle's Jacobian as its triplets summed per pattern slot (values,
    and the triplets' sums of |products| as the scale, in triplet order),
    compared with the library's values on the same pattern; slots no
    triplet reaches must be exactly 0."""
    m = keys.size
    v = np.bincount(pos, weights=trip_vals, minlength=m)
    s = np.bincount(pos, weights=trip_scales, minlength=m)
    present = np.bincount(pos, minlength=m) > 0
    vals = np.asarray(vals)
    if not np.all(present):
        assert np.all(vals[~present] == 0.0), what + ": entries absent from the oracle are not 0"
    return check_close(vals[present], v[present], s[present], what)
