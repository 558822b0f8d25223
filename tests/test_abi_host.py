"""C ABI on the CPU: the library loads, exports every declared symbol, and its
host-only logic (thresholds, schedule offsets, validation) is right."""
import ctypes as C
import os
import re
from decimal import Decimal, getcontext

import numpy as np
import pytest

import paper_1004_0024_amd as pa
from gen import LayeredSystem, chimera_template, make_chimera_system, make_random_system

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for hdr in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not hdr.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", hdr)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(\w+)\s*\([^;]*\)\s*;", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "for")))


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(pa.lib_path())
    names = declared_functions()
    assert {"ising_load_graph", "ising_sweep", "pt_swap", "ising_observables"} <= set(names)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def _exact_threshold(beta, d):
    """ceil(2^32 * exp(-2 beta d)) with 60-digit arithmetic (beta taken as its exact double)."""
    getcontext().prec = 60
    x = -2 * Decimal(beta) * d
    v = x.exp() * (Decimal(2) ** 32)
    return int(v.to_integral_value(rounding="ROUND_CEILING"))


def test_threshold_row_closed_form():
    rng = np.random.default_rng(0)
    betas = list(rng.uniform(0.01, 3.5, 120)) + [0.1, 3.0, 1e-3]
    for beta in betas:
        row = pa.threshold_row(beta, 63)
        assert row[0] == 0xFFFFFFFF
        for d in range(1, 64):
            t = _exact_threshold(beta, d)
            # the library rounds exp() in double first; it may differ from the exact
            # real only when 2^32 e^x lies within a double ulp of an integer
            assert abs(int(row[d]) + 1 - t) <= 1, (beta, d)
            if abs(int(row[d]) + 1 - t) == 1:
                pass
        assert all(row[d] >= row[d + 1] for d in range(1, 63))  # monotone in d


def test_threshold_matches_probability_comparison():
    """u <= thr[d]  <=>  u * 2^-32 < exp(-2.0*beta*d) for every u near the cut."""
    for beta in (0.1, 0.37, 1.3, 3.0):
        row = pa.threshold_row(beta, 30)
        for d in range(1, 31):
            p = np.exp(-2.0 * beta * d)
            for u in (int(row[d]) - 1, int(row[d]), int(row[d]) + 1):
                if 0 <= u < 2 ** 32:
                    assert (u <= row[d]) == (u * 2.0 ** -32 < p), (beta, d, u)


def test_level_offsets_chimera_closed_form():
    for L in (1, 2, 3, 5, 8):
        sysm = make_chimera_system(L, 3, seed=L, K=2)
        f, depth = pa.level_offsets(sysm)
        for y in range(L):
            for x in range(L):
                c = (y * L + x) * 8
                assert all(f[c + k] == y for k in range(4))
                assert all(f[c + k] == y + 1 + x for k in range(4, 8))
        assert depth == 2 * L


def test_level_offsets_longest_chain_brute_force():
    for seed in range(5):
        sysm = make_random_system(9, 14, seed=seed, K=1)
        f, depth = pa.level_offsets(sysm)
        adj = {q: set() for q in range(9)}
        for a, b in zip(sysm.eu, sysm.ev):
            adj[int(a)].add(int(b))
            adj[int(b)].add(int(a))

        def longest(q):  # longest increasing-index path ending at q, by recursion
            return max([longest(p) + 1 for p in adj[q] if p < q], default=0)

        assert [longest(q) for q in range(9)] == list(f)
        assert depth == max(f) + 1


def _bad(**kw):
    base = make_chimera_system(1, 3, seed=1, K=2)
    d = dict(S=base.S, M=base.M, ring=base.ring, eu=base.eu, ev=base.ev, eJ=base.eJ, h=base.h,
             J_tau=base.J_tau, beta=base.beta)
    d.update(kw)
    return LayeredSystem(**d)


@pytest.mark.parametrize("kw,code", [
    (dict(M=2, ring=True), -2),                                           # ring needs M >= 3
    (dict(beta=np.array([0.5, -1.0])), -2),                               # beta > 0
    (dict(eu=np.array([0, 0], np.int32), ev=np.array([1, 1], np.int32),
          eJ=np.array([1, 1], np.int8)), -1),                             # duplicate edge
    (dict(eu=np.array([0], np.int32), ev=np.array([0], np.int32), eJ=np.array([1], np.int8)), -1),
    (dict(eu=np.array([0], np.int32), ev=np.array([9], np.int32), eJ=np.array([1], np.int8)), -1),
    (dict(h=np.full(8, 100, np.int8)), -2),                               # |h|+sum|J| > 63
    (dict(beta=np.full(300, 1.0)), -2),                                   # K > 256
])
def test_validation_error_codes(kw, code):
    with pytest.raises(pa.IsingError) as e:
        pa.level_offsets(_bad(**kw))
    assert e.value.code == code


def test_cold_ladder_range():
    """A flip probability exp(-2 beta d) that would underflow to 0 in double has no
    uint32 threshold (u <= thr cannot say "never"; a wrapped ceil - 1 would say
    "always").  Rows stay exact up to 2 beta d_max = 700 and are rejected beyond, and
    a system is checked with its own d_max, not the table's 63."""
    for beta, dmax in ((12.0, 27), (5.5, 63), (350.0, 1), (20.0, 17)):
        row = pa.threshold_row(beta, dmax)
        assert row[0] == 0xFFFFFFFF
        assert all(0 <= int(row[d]) < 0xFFFFFFFF for d in range(1, dmax + 1))
        assert all(row[d] >= row[d + 1] for d in range(1, dmax))
        assert int(row[dmax]) == _exact_threshold(beta, dmax) - 1 or int(row[dmax]) == 0
    for beta, dmax in ((20.0, 27), (5.6, 63), (350.1, 1)):
        with pytest.raises(pa.IsingError) as e:
            pa.threshold_row(beta, dmax)
        assert e.value.code == -2
    # the system of _bad() has d_max = max over spins of |h| + sum|J| + 2 |J_tau| <= 21
    pa.level_offsets(_bad(beta=np.array([0.5, 6.0])))  # 2 * 6 * 21 <= 700
    with pytest.raises(pa.IsingError) as e:
        pa.level_offsets(_bad(beta=np.array([0.5, 60.0])))
    assert e.value.code == -2


def test_validation_degree():
    S = 12
    eu = np.array([0] * 9, np.int32)
    ev = np.arange(1, 10, dtype=np.int32)
    sysm = LayeredSystem(S=S, M=1, ring=False, eu=eu, ev=ev, eJ=np.ones(9, np.int8), h=np.zeros(S, np.int8),
                         J_tau=np.zeros(S, np.int8), beta=np.array([1.0]))
    with pytest.raises(pa.IsingError) as e:
        pa.level_offsets(sysm)
    assert e.value.code == -2
    # Chimera with a ring: 6 in-slice + 2 tau = 8 is accepted
    S_, eu_, ev_ = chimera_template(3)
    assert S_ == 72
    f, depth = pa.level_offsets(make_chimera_system(3, 4, seed=0, K=1))
    assert depth == 6


def test_acceptance_rows_match_oracle():
    """Thresholds of the approximate flip tests (Fig. 7): the library's host code and the
    oracle's, written separately, agree bit for bit."""
    import numpy as np
    import oracle
    import paper_1004_0024_amd as pa
    from gen import beta_ladder
    betas = list(beta_ladder(32, 0.1, 3.0)) + [0.05, 0.731, 1.0, 2.5]
    for kind in (pa.ACCEPT_FAST, pa.ACCEPT_ACCURATE):
        for beta in betas:
            row = pa.acceptance_row(beta, 63, kind)
            assert row[0] == 0xFFFFFFFF
            ref = [oracle.approx_threshold(beta, d, kind) for d in range(1, 64)]
            assert [int(v) for v in row[1:]] == ref, (kind, beta)
    assert np.array_equal(pa.acceptance_row(0.7, 63, pa.ACCEPT_EXACT), pa.threshold_row(0.7, 63))


def test_acceptance_kind_rejected():
    import pytest
    import paper_1004_0024_amd as pa
    with pytest.raises(pa.IsingError):
        pa.acceptance_row(0.5, 10, 7)


def test_two_field_rows_match_the_flip_rule():
    """Two-field thresholds: entry (d_sp, d_t) is the largest u with u * 2^-32 < exp(-2x),
    x = a d_sp + c d_t in double (products rounded separately), every u passing at x <= 0;
    under the Fig. 7 variants the rows equal the oracle's thresholds bit for bit."""
    import oracle
    rng = np.random.default_rng(5)
    ds, dt = 21, 6
    weights = [(0.05, 0.9), (0.3, 2.1), (0.8, 0.02), (1.5, 0.4)] + \
        [tuple(rng.uniform(0.01, 2.0, 2)) for _ in range(6)] + [(0.125, 0.125), (-0.2, 0.3)]
    for a, c in weights:
        row = pa.two_field_row(a, c, ds, dt, pa.ACCEPT_EXACT)
        for i in range(-ds, ds + 1):
            for j in range(-dt, dt + 1):
                x = a * i + c * j
                t = int(row[i + ds, j + dt])
                if x <= 0:
                    assert t == 0xFFFFFFFF, (a, c, i, j)
                    continue
                p = np.exp(-2.0 * x)
                assert t * 2.0 ** -32 < p and not ((t + 1) * 2.0 ** -32 < p), (a, c, i, j)
        for kind in (pa.ACCEPT_FAST, pa.ACCEPT_ACCURATE):
            row = pa.two_field_row(a, c, ds, dt, kind)
            for i in range(-ds, ds + 1):
                for j in range(-dt, dt + 1):
                    x = a * i + c * j
                    want = 0xFFFFFFFF if x <= 0 else oracle.approx_threshold_x(x, kind)
                    assert int(row[i + ds, j + dt]) == want, (kind, a, c, i, j)
    # a = c = beta: the row over d_sp + d_t is the one-field row (dyadic beta: exact products)
    for beta in (0.125, 0.375, 1.0):
        row = pa.two_field_row(beta, beta, ds, dt, pa.ACCEPT_EXACT)
        one = pa.threshold_row(beta, ds + dt)
        for i in range(-ds, ds + 1):
            for j in range(-dt, dt + 1):
                assert row[i + ds, j + dt] == one[max(i + j, 0)], (beta, i, j)


def test_two_field_row_rejects_out_of_range():
    with pytest.raises(pa.IsingError):
        pa.two_field_row(30.0, 1.0, 21, 6)  # exp(-2x) would underflow
    with pytest.raises(pa.IsingError):
        pa.two_field_row(0.5, 0.5, 40, 40)  # row longer than the supported 1024 words


def test_trotter_weights_match_oracle():
    import oracle
    from gen import beta_ladder
    beta = beta_ladder(32, 0.1, 3.0)
    for M, G in ((64, 1.0), (32, 0.3), (8, 2.5)):
        a, c = pa.trotter_weights(beta, M, G)
        ra, rc = oracle.trotter_weights(beta, M, G)
        assert np.array_equal(a, ra)
        assert np.allclose(c, rc, rtol=2e-15, atol=0), (M, G)  # libm and numpy: a few ulp
    with pytest.raises(pa.IsingError):
        pa.trotter_weights(beta, 8, 0.0)
