"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bar (set by the estimator's definition, eqs. (2)-(3) of arXiv:1811.11722):
lattice indices bit-exact; every per-shift Q_k within 1e-12 relative of the
oracle's on identical seeded inputs.  The oracle runs on the host of the GPU
box with all its cores.
"""
import math
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1811_11722_amd import synth
from parity_bounds import complex_sector_check

pytestmark = pytest.mark.gpu

TOL = 1e-12
THREADS = min(16, os.cpu_count() or 1)


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def Q():
    O.build(force=False)
    from paper_1811_11722_amd import qmc
    qmc.lib()
    return qmc


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def _both(Q, family, d, n, g, sh, tk="none", alpha=0, launch=None, jit=None, **kw):
    """(gpu result, gpu per-shift, oracle estimate)"""
    okw = dict(kw)
    plan = Q.Plan(d, n, g, sh, tk, alpha)
    if launch:
        plan.set_launch(*launch)
    if jit is not None:
        plan.set_jit(jit)
    res, q = plan.integrate(Q.Params(family, d, **kw))
    est = O.estimate(n, g, sh, O.Params(family, d, **okw), tk, alpha, threads=THREADS)
    assert est.status == 0
    plan.close()
    return res, np.asarray(q), est


# ------------------------------------------------------------ device math
def test_device_log_exp_ulps(Q):
    """qlog / qexp against long-double libm on random and edge arguments."""
    rng = np.random.default_rng(7)
    x = np.concatenate([10.0 ** rng.uniform(-300, 300, 200000), rng.uniform(0.5, 2.0, 200000),
                        [1.0, 2.0, 0.5, 1e-308, 1.7e308, np.nextafter(1.0, 2), np.nextafter(1.0, 0)]])
    _say("device log")
    y = Q.math_eval("log", x)
    ref = np.log(x.astype(np.longdouble))
    err = np.abs((y - ref).astype(np.float64))
    assert np.all(err <= 2.5 * np.spacing(np.maximum(np.abs(ref.astype(np.float64)), 1.0)))
    assert np.all(np.isnan(Q.math_eval("log", np.array([0.0, -1.0, np.nan]))))
    t = np.concatenate([rng.uniform(-700, 700, 200000), rng.uniform(-1, 1, 200000), [0.0, -745.0, 709.7]])
    _say("device exp")
    y = Q.math_eval("exp", t)
    ref = np.exp(t.astype(np.longdouble))
    rel = np.abs(((y - ref) / ref).astype(np.float64))
    ok = ref > 2.3e-308
    assert np.all(rel[ok] <= 2.5 * 2.0 ** -52)
    assert Q.math_eval("exp", np.array([800.0]))[0] == np.inf
    assert Q.math_eval("exp", np.array([-800.0]))[0] == 0.0


def test_device_atan2_sincos(Q):
    """qatan2 / qsincos against long-double libm: every quadrant, the sector
    phase's own arguments (-delta, F) with F of both signs, the octant
    boundary tan(pi/8), and phases up to |x| = 1e5."""
    rng = np.random.default_rng(11)
    mag = 10.0 ** rng.uniform(-6, 6, 100000)
    ang = rng.uniform(-np.pi, np.pi, 100000)
    yy = np.concatenate([mag * np.sin(ang), -10.0 ** rng.uniform(-4, 0, 50000),
                         [0.0, -0.0, 1.0, -1.0, np.tan(np.pi / 8), -1e-300, 2.0]])
    xx = np.concatenate([mag * np.cos(ang), rng.choice([-1.0, 1.0], 50000) * 10.0 ** rng.uniform(-3, 3, 50000),
                         [1.0, -1.0, 0.0, -0.0, 1.0, -1.0, 2.0]])
    _say("device atan2")
    a = Q.math_eval("atan2", yy, xx)
    ref = np.arctan2(yy.astype(np.longdouble), xx.astype(np.longdouble))
    err = np.abs((a - ref).astype(np.float64))
    assert np.all(err <= 2.5 * np.spacing(np.abs(ref.astype(np.float64))) + 1e-300), err.max()
    assert np.array_equal(np.signbit(a[-7:-3]), np.signbit(np.arctan2(yy[-7:-3], xx[-7:-3])))
    t = np.concatenate([rng.uniform(-4.5, 4.5, 200000), rng.uniform(-1e5, 1e5, 100000),
                        [0.0, np.pi / 4, np.pi / 2, -np.pi, 1e-300]])
    _say("device sincos")
    sc = Q.math_eval("sincos", t)
    tl = t.astype(np.longdouble)
    for col, ref in ((0, np.sin(tl)), (1, np.cos(tl))):
        err = np.abs((sc[:, col] - ref).astype(np.float64))
        # absolute error of a few ulps of 1 (the reduced argument carries
        # the rounding of |x| for the large arguments)
        bound = 4.0 * 2.0 ** -53 * np.maximum(1.0, np.abs(t) * 2.0 ** -20)
        assert np.all(err <= bound), (col, err.max())


def test_korobov_constant_error_decay(Q):
    """Sec. 2, Fig. 3: integrating 1 with the Korobov weight-3 transform in
    d = 6, the reported error falls far faster than 1/n, and the per-shift
    sums stay within the oracle's parity bar."""
    d, m = 6, 16
    sh = synth.shifts(81, m, d)
    errs = []
    for n, a in ((1021, 76), (16381, 5029), (262139, 100135)):
        g = O.korobov_vector(n, d, a)
        _say(f"fig3 n={n}")
        res, q, est = _both(Q, "const", d, n, g, sh, "korobov", 3, c=1.0)
        assert np.all(np.abs(q - est.q_re) <= 1e-12 * np.abs(est.q_re))
        errs.append(res.err_re)
    assert errs[1] < errs[0] / 50 and errs[2] < errs[1] / 50, errs


# ---------------------------------------------------------- lattice indices
def test_indices_bit_exact_all_points(Q):
    n, d = 131071, 4
    g = O.korobov_vector(n, d, 48724)
    plan = Q.Plan(d, n, g, synth.shifts(1, 16, d), "korobov", 3)
    _say(f"dump all indices n={n} d={d}")
    idx, sums = plan.lattice_dump(0, n)
    want = O.lattice_indices(n, g, np.arange(n))
    assert np.array_equal(idx.astype(np.uint64), want)
    assert np.all(sums[:, 0] == n * (n - 1) // 2)
    assert np.all(sums[:, 1] == ((n - 1) * n * (2 * n - 1) // 6) % 2 ** 64)


@pytest.mark.parametrize("n,d", [(1073741789, 10), (16777213, 6), (2, 1), (257, 3), (1021, 16)])
def test_indices_sampled_large(Q, n, d):
    a = 3 if n > 3 else 1
    g = O.korobov_vector(n, d, a)
    plan = Q.Plan(d, n, g, synth.shifts(2, 2, d), "baker")
    rng = np.random.default_rng(n)
    ranges = [(0, min(n, 4096)), (max(0, n - 4096), min(n, 4096))]
    if n > 100000:
        ranges.append((int(rng.integers(0, n - 4096)), 4096))
    for lo, cnt in ranges:
        _say(f"dump n={n} d={d} j in [{lo}, {lo + cnt})")
        idx, sums = plan.lattice_dump(lo, cnt)
        want = O.lattice_indices(n, g, np.arange(lo, lo + cnt))
        assert np.array_equal(idx.astype(np.uint64), want)
    # every coordinate is a permutation of 0..n-1 (gcd(g_i, n) = 1, n prime or g_i = 1)
    for i in range(d):
        if math.gcd(int(g[i]), n) == 1:
            assert int(sums[i, 0]) == n * (n - 1) // 2
            assert int(sums[i, 1]) == ((n - 1) * n * (2 * n - 1) // 6) % 2 ** 64


# ------------------------------------------------------ generating vector
def test_korobov_search_config_product_peak(Q):
    w = synth.product_peak_workload()
    _say("korobov search n=131071 d=4 64 candidates")
    a_gpu, p2_gpu, all_gpu = Q.korobov_search(w.n, w.d, w.candidates)
    a_or, p2_or, all_or = O.korobov_search(w.n, w.d, w.candidates, threads=THREADS)
    assert np.all(_rel(all_gpu, all_or) < 1e-9)
    if a_gpu != a_or:  # a near-tie: both choices must be minimal within rounding
        assert abs(p2_gpu - p2_or) <= 1e-9 * p2_or
    assert p2_gpu == all_gpu.min()


@pytest.mark.parametrize("n,cands", [(4093, [3, 17, 76, 1234, 2001]), (4096, [3, 17, 77, 1235, 2001]),
                                     (4096, [3, 18, 77, 1234]), (2, [1]), (3, [1, 2])])
def test_korobov_search_half_range(Q, n, cands):
    """The P2 sum formed from j <= n/2 (odd n; even n with odd candidates,
    whose point n/2 is (1/2, ..., 1/2)) and over all n points (even n with an
    even candidate) against the oracle's plain sum over all points."""
    d = 5
    c = np.array(cands, dtype=np.uint64)
    _say(f"korobov search n={n} candidates={cands}")
    _, _, all_gpu = Q.korobov_search(n, d, c)
    _, _, all_or = O.korobov_search(n, d, c, threads=THREADS)
    rel = _rel(all_gpu, all_or)
    print(f"max relative difference {rel.max():.2e}")
    assert np.all(rel < 1e-12), rel.max()


# ------------------------------------------------------------- estimates
def test_product_peak_config(Q):
    """Genz product peak, d = 4, Korobov 3, n = 131071, m = 16."""
    w = synth.product_peak_workload()
    a, _, _ = O.korobov_search(w.n, w.d, w.candidates, threads=THREADS)
    g = O.korobov_vector(w.n, w.d, a)
    _say("product peak d=4 korobov3 n=131071 m=16")
    res, q, est = _both(Q, "genz_product_peak", w.d, w.n, g, w.shifts, "korobov", 3,
                        a=w.genz_a, u=w.genz_u)
    assert np.all(_rel(q, est.q_re) < TOL), _rel(q, est.q_re).max()
    mean, er, _ = est.mean_error()
    assert abs(res.mean_re - mean.real) <= TOL * abs(mean.real)
    assert abs(res.err_re - er) <= 1e-6 * er


@pytest.mark.parametrize("launch", [(2, 1), (4, 3), (8, 8), (8, 1)])
def test_product_peak_launch_shapes(Q, launch):
    """Shift tile and grid size change only the summation order."""
    w = synth.product_peak_workload(n=16381, m=11)
    g = O.korobov_vector(w.n, w.d, 1234)
    _say(f"product peak launch {launch}")
    res, q, est = _both(Q, "genz_product_peak", w.d, w.n, g, w.shifts, "korobov", 3,
                        launch=launch, a=w.genz_a, u=w.genz_u)
    assert np.all(_rel(q, est.q_re) < TOL)


@pytest.mark.parametrize("a_scale", [1e-4, 1.0, 100.0])
@pytest.mark.parametrize("launch", [(8, 1), (4, 3), (2, 2)])
def test_product_peak_tile_reciprocal(Q, a_scale, launch):
    """The shifts of a tile share one reciprocal of their denominators'
    product unless a denominator could leave 2^-62 .. 2^62.  With a in
    2..8 scaled by 1e-4 the four factors a^-2 + s^2 multiply to about 2^90,
    scaled by 100 the lower bound a^-2 of each multiplies to 2^-69, so those
    take one reciprocal per shift; unscaled (2^-16 .. 2^-1.4) they share one.
    Both against the oracle, per shift."""
    w = synth.product_peak_workload(n=16381, m=11)
    g = O.korobov_vector(w.n, w.d, 1234)
    a = w.genz_a * a_scale
    _say(f"product peak tile reciprocal a x {a_scale} launch {launch}")
    res, q, est = _both(Q, "genz_product_peak", w.d, w.n, g, w.shifts, "korobov", 3,
                        launch=launch, a=a, u=w.genz_u)
    rel = _rel(q, est.q_re)
    print(f"max relative difference {rel.max():.2e}")
    assert np.all(np.isfinite(q)) and np.all(rel < TOL), rel.max()


@pytest.mark.parametrize("family", ["genz_product_peak", "genz_oscillatory", "genz_gaussian",
                                    "genz_continuous", "genz_corner_peak", "const", "p2kernel"])
@pytest.mark.parametrize("tk,alpha", [("none", 0), ("baker", 0), ("korobov", 1), ("korobov", 3),
                                      ("korobov", 6)])
def test_families_and_transforms(Q, family, tk, alpha):
    d, n, m = 3, 4093, 5
    a, u = synth.genz_params(17, d)
    a = a / 3.0
    g = O.korobov_vector(n, d, 76)
    sh = synth.shifts(17, m, d)
    kw = dict(a=a, u=u) if family.startswith("genz") else ({"c": 1.7} if family == "const" else {})
    _say(f"{family} {tk}{alpha} d={d} n={n} m={m}")
    res, q, est = _both(Q, family, d, n, g, sh, tk, alpha, **kw)
    assert np.all(_rel(q, est.q_re) < TOL), (_rel(q, est.q_re).max())


@pytest.mark.parametrize("d", [1, 2, 5, 7, 8, 9, 11, 12, 13, 16])
def test_dimensions(Q, d):
    n, m = 1021, 6
    a, u = synth.genz_params(d, d)
    g = O.korobov_vector(n, d, 76)
    sh = synth.shifts(d, m, d)
    _say(f"product peak d={d}")
    res, q, est = _both(Q, "genz_product_peak", d, n, g, sh, "korobov", 2, a=a, u=u)
    assert np.all(_rel(q, est.q_re) < TOL)


@pytest.mark.parametrize("n", [2, 3, 255, 256, 257, 65537])
def test_small_and_ragged_n(Q, n):
    d, m = 2, 3
    g = np.array([1, 1 if n <= 3 else 3], dtype=np.uint64)
    a, u = np.array([3.0, 4.0]), np.array([0.2, 0.8])
    sh = synth.shifts(n, m, d)
    _say(f"ragged n={n}")
    res, q, est = _both(Q, "genz_gaussian", d, n, g, sh, "baker", a=a, u=u)
    assert np.all(_rel(q, est.q_re) < TOL)


def test_trig_dual_lattice(Q):
    n, d, m = 1021, 3, 6
    g = O.korobov_vector(n, d, 76)
    sh = synth.shifts(9, m, d)
    gl = [int(v) for v in g]
    hs = [(1, 0, 0), (0, 2, -1), (3, 1, 1), (-gl[1], 1, 0)]
    ch, phi = [0.7, -0.3, 0.25, 0.9], [0.1, 1.2, -0.4, 0.3]
    _say("trig dual lattice")
    res, q, est = _both(Q, "trig", d, n, g, sh, "none", trig=(0.5, hs, ch, phi))
    want = 0.5 + 0.9 * np.cos(2 * np.pi * (sh @ np.array(hs[3], dtype=float)) + 0.3)
    assert np.all(np.abs(q - want) < 1e-11)
    assert np.all(np.abs(q - est.q_re) < 1e-12)


def test_constant_exact_baker(Q):
    n, d, m = 65521, 6, 4
    g = O.korobov_vector(n, d, 17364)
    plan = Q.Plan(d, n, g, synth.shifts(3, m, d), "baker")
    _say("constant baker")
    res, q = plan.integrate(Q.Params("const", d, c=2.75))
    assert np.all(np.abs(q - 2.75) <= 4 * np.spacing(2.75))
    assert res.err_re <= 1e-15


# ------------------------------------------------------------ sector family
def _sector_case(Q, d, n, m, n_u, n_f, seed, complex_kinematics=False, launch=None, jit=None):
    tab = synth.sector_tables(seed, d, n_u, n_f, complex_kinematics=complex_kinematics)
    ab, _, _ = O.korobov_search(n, d, synth.korobov_candidates(seed, n, 8), threads=THREADS)
    g = O.korobov_vector(n, d, ab)
    sh = synth.shifts(seed, m, d)
    _say(f"sector d={d} n={n} m={m} nU={n_u} nF={n_f} complex={complex_kinematics} launch={launch} "
         f"jit={jit}")
    return _both(Q, "sector", d, n, g, sh, "baker", launch=launch, jit=jit, sector=tab)


@pytest.mark.parametrize("jit", [0, 2])
@pytest.mark.parametrize("launch", [None, (1, 0), (2, 4), (4, 0)])
def test_sector_real(Q, launch, jit):
    res, q, est = _sector_case(Q, 6, 65521, 8, 12, 30, 101, launch=launch, jit=jit)
    assert np.all(_rel(q, est.q_re) < TOL), _rel(q, est.q_re).max()


@pytest.mark.parametrize("jit", [0, 2])
@pytest.mark.parametrize("d,n_u,n_f", [(2, 4, 5), (3, 17, 31), (8, 12, 30), (9, 40, 40), (14, 12, 30)])
def test_sector_real_shapes(Q, d, n_u, n_f, jit):
    res, q, est = _sector_case(Q, d, 16381, 5, n_u, n_f, 200 + d, jit=jit)
    assert np.all(_rel(q, est.q_re) < TOL)


@pytest.mark.parametrize("jit", [0, 2])
@pytest.mark.parametrize("u_case", ["bounded", "no_constant_term", "negative_coefficient"])
def test_sector_u_edge_cases(Q, u_case, jit):
    """U^-2 where U is bounded away from 0 (non-negative coefficients, a
    positive constant term), where it vanishes at a corner (no constant
    term) and with a negative coefficient.  Each against the oracle, per
    shift, at shift tile 4."""
    import dataclasses
    d, n, m = 6, 16381, 8
    tab = synth.sector_tables(101, d, 12, 30)
    eu = np.asarray(tab.exp_u).reshape(tab.n_u, d)
    const = [t for t in range(tab.n_u) if not eu[t].any()]
    assert const, "the synthetic U has a constant term"
    if u_case == "no_constant_term":
        keep = [t for t in range(tab.n_u) if t not in const]
        tab = dataclasses.replace(tab, coef_u=np.asarray(tab.coef_u)[keep], exp_u=eu[keep])
    elif u_case == "negative_coefficient":
        cu = np.array(tab.coef_u, dtype=np.float64)
        t = next(t for t in range(tab.n_u) if t not in const)
        cu[t] = -0.01 * cu[t]
        tab = dataclasses.replace(tab, coef_u=cu)
    g = O.korobov_vector(n, d, 5029)
    sh = synth.shifts(56, m, d)
    _say(f"sector U edge case {u_case} jit={jit}")
    res, q, est = _both(Q, "sector", d, n, g, sh, "baker", launch=(4, 0), jit=jit, sector=tab)
    rel = _rel(q, est.q_re)
    print(f"max relative difference {rel.max():.2e}")
    assert np.all(rel < TOL), rel.max()


def test_sector_same_structure_new_values(Q):
    """One plan, one specialised kernel (found by the monomial structure),
    three integrands that share it: new coefficients and powers, and the
    monomials given in another order (the packer stores them in the order the
    code reads them).  Each estimate against the oracle's, and the first one
    again, bit for bit."""
    import dataclasses
    d, n, m = 6, 16381, 4
    g = O.korobov_vector(n, d, 5029)
    sh = synth.shifts(55, m, d)
    a = synth.sector_tables(55, d, 12, 30)
    rng = np.random.default_rng(55)
    b = dataclasses.replace(a, coef_u=a.coef_u * rng.uniform(0.5, 2.0, a.n_u),
                            coef_f=a.coef_f * rng.uniform(0.5, 2.0, a.n_f), pow_f=-1.1)
    pu, pf = rng.permutation(a.n_u), rng.permutation(a.n_f)
    c = dataclasses.replace(a, coef_u=a.coef_u[pu], exp_u=a.exp_u[pu], coef_f=a.coef_f[pf], exp_f=a.exp_f[pf])
    plan = Q.Plan(d, n, g, sh, "baker")
    plan.set_jit(2)
    first = None
    for name, tab in (("a", a), ("b", b), ("c", c), ("a", a)):
        _say(f"same structure, integrand {name}")
        res, q = plan.integrate(Q.Params("sector", d, sector=tab))
        est = O.estimate(n, g, sh, O.Params("sector", d, sector=tab), "baker", threads=THREADS)
        assert np.all(_rel(q, est.q_re) < TOL), (name, _rel(q, est.q_re).max())
        if name == "a":
            if first is None:
                first = np.array(q)
            else:
                assert np.array_equal(np.array(q), first)
    plan.close()


@pytest.mark.parametrize("d,cplx,want", [(6, False, 4), (3, False, 4), (8, False, 4), (9, False, 2), (6, True, 2)])
def test_specialised_default_tile(Q, d, cplx, want):
    """The default shift tile of the specialised kernel: four shifts per
    thread for real sectors up to d = 8, two for wider or complex ones; the
    estimate matches the oracle's either way (m = 6 leaves a ragged last
    tile at T = 4)."""
    n, m = 16381, 6
    tab = synth.sector_tables(300 + d, d, 12, 30, complex_kinematics=cplx)
    g = O.korobov_vector(n, d, 5029)
    sh = synth.shifts(300 + d, m, d)
    plan = Q.Plan(d, n, g, sh, "baker")
    _say(f"default tile d={d} complex={cplx}")
    res, q = plan.integrate(Q.Params("sector", d, sector=tab))
    T, _, used = plan.last_launch()
    assert used and T == want
    if cplx:
        # a mixed-sign complex F: the bound of its rounding condition
        complex_sector_check(q, n, g, sh, tab, label=f"default tile d={d}")
    else:
        est = O.estimate(n, g, sh, O.Params("sector", d, sector=tab), "baker", threads=THREADS)
        assert np.all(_rel(q, est.q_re) < TOL), _rel(q, est.q_re).max()
    plan.close()


@pytest.mark.parametrize("d,want", [(6, 4), (8, 2)])
def test_orders_default_tile(Q, d, want):
    """Expansion orders: four shifts per thread up to d = 6, two above; the
    three orders match the oracle's coefficients f L^k / k! either way
    (m = 6 leaves a ragged last tile at T = 4)."""
    n, m = 16381, 6
    tab = synth.sector_tables(320 + d, d, 12, 30)
    g = O.korobov_vector(n, d, 5029)
    sh = synth.shifts(320 + d, m, d)
    plan = Q.Plan(d, n, g, sh, "baker")
    _say(f"orders default tile d={d}")
    res, per = plan.integrate_orders(Q.Params("sector", d, sector=tab, orders=(3, 0.7, -1.2)))
    T, _, used = plan.last_launch()
    assert used and T == want
    for k in range(3):
        est = O.estimate(n, g, sh, O.Params("sector", d, sector=tab, eps=(0.7, -1.2, k)), "baker",
                         threads=THREADS)
        assert np.all(_rel(per[:, k], est.q_re) < TOL), (k, _rel(per[:, k], est.q_re).max())
    plan.close()


@pytest.mark.parametrize("jit", [0, 2])
@pytest.mark.parametrize("launch", [None, (1, 0), (2, 0)])
def test_sector_complex(Q, launch, jit):
    """Complex kinematics (mixed-sign F, F - 0.01i), d = 10 (workload 5's
    shape), against the long-double oracle within the rounding-condition
    bound of complex_sector_check."""
    n, m, d = 16381, 6, 10
    tab = synth.sector_tables(505, d, 20, 60, complex_kinematics=True)
    ab, _, _ = O.korobov_search(n, d, synth.korobov_candidates(505, n, 8), threads=THREADS)
    g = O.korobov_vector(n, d, ab)
    sh = synth.shifts(505, m, d)
    plan = Q.Plan(d, n, g, sh, "baker")
    if launch:
        plan.set_launch(*launch)
    plan.set_jit(jit)
    _say(f"complex sector d={d} launch={launch} jit={jit}")
    res, q = plan.integrate(Q.Params("sector", d, sector=tab))
    plan.close()
    complex_sector_check(q, n, g, sh, tab, label=f"launch={launch} jit={jit}")


def test_xmy_toy_integral(Q):
    """eq. (7) as a complex sector: U = 1, F = x1 - x2, delta = 1e-2."""
    d, n, m = 2, 65521, 8
    s = synth.SectorTables(d=2, coef_u=np.array([1.0]), exp_u=np.zeros((1, 2), np.uint8),
                           coef_f=np.array([1.0, -1.0]), exp_f=np.array([[1, 0], [0, 1]], np.uint8),
                           nu=np.zeros(2, np.uint8), pow_u=-2.0, pow_f=-1.7, delta_im=1e-2,
                           is_complex=True)
    g = O.korobov_vector(n, d, 17364)
    sh = synth.shifts(8, m, d)
    _say("x - y toy integral")
    res, q, est = _both(Q, "sector", d, n, g, sh, "baker", sector=s)
    qo = est.q
    assert np.all(np.abs(q - qo) <= TOL * np.abs(qo))


def test_sector_nonfinite_status(Q):
    """A real sector whose F vanishes inside the domain gives ENONFINITE."""
    s = synth.SectorTables(d=2, coef_u=np.array([1.0]), exp_u=np.zeros((1, 2), np.uint8),
                           coef_f=np.array([1.0, -1.0]), exp_f=np.array([[1, 0], [0, 1]], np.uint8),
                           nu=np.zeros(2, np.uint8))
    plan = Q.Plan(2, 1021, O.korobov_vector(1021, 2, 76), synth.shifts(1, 4, 2), "baker")
    _say("non-finite sector")
    st, res, _ = plan.integrate_status(Q.Params("sector", 2, sector=s))
    assert st == Q.QMC_ENONFINITE and math.isnan(res.mean_re)


def test_determinism(Q):
    w = synth.sector_workload(n=65521, m=8)
    g = O.korobov_vector(w.n, w.d, 17364)
    plan = Q.Plan(w.d, w.n, g, w.shifts, "baker")
    p = Q.Params("sector", w.d, sector=w.sector)
    _say("determinism")
    _, q1 = plan.integrate(p)
    _, q2 = plan.integrate(p)
    assert np.array_equal(q1, q2)


# ------------------------------------------------------ full-size sampled
def test_sector_full_size_sampled_shifts(Q):
    """The benchmark workload (d = 6, n = 16777213, m = 32, baker) in the
    launch the benchmark uses; the oracle recomputes 3 of the 32 shifts."""
    w = synth.sector_workload()
    a, _, _ = Q.korobov_search(w.n, w.d, w.candidates)
    g = O.korobov_vector(w.n, w.d, a)
    plan = Q.Plan(w.d, w.n, g, w.shifts, "baker")
    _say("sector full size")
    res, q = plan.integrate(Q.Params("sector", w.d, sector=w.sector))
    assert plan.last_launch()[2], "the default path should run the specialised kernel"
    pick = [0, 17, 31]
    est = O.estimate(w.n, g, w.shifts[pick], O.Params("sector", w.d, sector=w.sector), "baker",
                     threads=THREADS)
    assert np.all(_rel(q[pick], est.q_re) < TOL), _rel(q[pick], est.q_re).max()


# ----------------------------------------------------------- expansion orders
@pytest.mark.parametrize("cplx", [False, True])
def test_sector_orders_match_oracle(Q, cplx):
    """Coefficients of e^0..e^3 of x^nu U^(-2 + 0.7 e) (F - i delta)^(-1.3 - 1.2 e)
    in one pass, each order's per-shift sums against the oracle's."""
    d, n, m = 5, 16381, 8
    tab = synth.sector_tables(91, d, 7, 12)
    if cplx:
        tab.delta_im, tab.is_complex = 0.02, True
    g = O.korobov_vector(n, d, 17364)
    sh = synth.shifts(91, m, d)
    plan = Q.Plan(d, n, g, sh, "baker")
    _say(f"orders complex={cplx}")
    res, per = plan.integrate_orders(Q.Params("sector", d, sector=tab, orders=(4, 0.7, -1.2)))
    assert len(res) == 4 and per.shape == (m, 4)
    for k in range(4):
        est = O.estimate(n, g, sh, O.Params("sector", d, sector=tab, eps=(0.7, -1.2, k)), "baker", threads=THREADS)
        ref = est.q_re + 1j * est.q_im if cplx else est.q_re
        assert np.all(np.abs(per[:, k] - ref) <= 1e-12 * np.abs(ref)), (k, np.max(np.abs(per[:, k] - ref) / np.abs(ref)))
        mean, err, _ = est.mean_error()
        got = complex(res[k].mean_re, res[k].mean_im)
        assert abs(got - mean) <= 1e-12 * abs(mean)
    # order 0 of the expansion is the plain integrand
    r0, q0 = plan.integrate(Q.Params("sector", d, sector=tab))
    assert abs(complex(r0.mean_re, r0.mean_im) - complex(res[0].mean_re, res[0].mean_im)) <= 1e-12 * abs(r0.mean_re)


def test_sector_orders_validation(Q):
    d, n = 3, 1021
    tab = synth.sector_tables(92, d, 3, 4)
    plan = Q.Plan(d, n, O.korobov_vector(n, d, 76), synth.shifts(92, 2, d), "baker")
    with pytest.raises(Q.QMCError) as e:
        plan.integrate(Q.Params("sector", d, sector=tab, orders=(2, 1.0, 1.0)))
    assert e.value.status == Q.QMC_EINVAL
    with pytest.raises(Q.QMCError) as e:
        plan.integrate_orders(Q.Params("sector", d, sector=tab, orders=(5, 1.0, 1.0)))
    assert e.value.status == Q.QMC_EUNSUPPORTED
    plan.set_jit(0)
    with pytest.raises(Q.QMCError) as e:
        plan.integrate_orders(Q.Params("sector", d, sector=tab, orders=(2, 1.0, 1.0)))
    assert e.value.status == Q.QMC_EUNSUPPORTED
    # one order is the plain integrand through either entry point
    plan.set_jit(1)
    one, _ = plan.integrate_orders(Q.Params("sector", d, sector=tab, orders=(1, 1.0, 1.0)))
    plain, _ = plan.integrate(Q.Params("sector", d, sector=tab))
    assert one[0].mean_re == plain.mean_re


# ------------------------------------------------------------ Sidi transform
@pytest.mark.parametrize("family", ["genz_product_peak", "const"])
@pytest.mark.parametrize("m_", [1, 2, 3, 4, 5, 6])
def test_sidi_transform_families(Q, family, m_):
    """Sidi's sin^m transform compiled ahead of time, against the oracle."""
    d, n, m = 3, 4093, 5
    a, u = synth.genz_params(17, d)
    g = O.korobov_vector(n, d, 76)
    sh = synth.shifts(17, m, d)
    kw = dict(a=a / 3.0, u=u) if family.startswith("genz") else {"c": 1.7}
    _say(f"{family} sidi{m_}")
    res, q, est = _both(Q, family, d, n, g, sh, "sidi", m_, **kw)
    assert np.all(_rel(q, est.q_re) < TOL), (_rel(q, est.q_re).max())


@pytest.mark.parametrize("m_", [1, 2, 3, 6])
@pytest.mark.parametrize("cplx", [False, True])
def test_sidi_transform_sectors(Q, m_, cplx):
    """Sectors with Sidi's transform through the specialised kernel."""
    d, n, m = 6, 16381, 5
    tab = synth.sector_tables(231, d, 12, 30)
    if cplx:
        tab.delta_im, tab.is_complex = 0.02, True
    g = O.korobov_vector(n, d, 17364)
    sh = synth.shifts(231, m, d)
    _say(f"sector sidi{m_} complex={cplx}")
    res, q, est = _both(Q, "sector", d, n, g, sh, "sidi", m_, sector=tab)
    assert np.all(_rel(q, est.q) < TOL), (_rel(q, est.q).max())
