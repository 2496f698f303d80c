"""GPU parity of the contour-deformed sector integrand (Sec. 3 of
arXiv:1811.11722): z_k = x_k - i lam x_k (1 - x_k) dF/dx_k, integrand
f(z) det(dz/dx), through the C ABI against the CPU oracle.

The oracle takes det(dz/dx) by LU with partial pivoting on the Jacobian
itself; the kernel takes it from the LDL^T pivots of a symmetrised, similar
matrix, so agreement also checks that similarity.

Bar: |Q_k - Q_k(oracle)| <= 1e-12 max(|Q_k|, (1/n) sum_j |fhat(x_j)|).  The
deformed values are complex with phases that cancel in the sum (for a
Euclidean F the imaginary part integrates to zero), and each point carries a
relative rounding of a few ulp on both sides, so the difference of the sums
is bounded by the sum of the magnitudes, not by |Q_k|.  Where F's own terms
cancel (mixed-sign kinematics) the bar widens to 4x the oracle's spread when
F's monomials are summed in other orders.
"""
import dataclasses
import math
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1811_11722_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-12
THREADS = min(16, os.cpu_count() or 1)


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def Q():
    O.build(force=False)
    return Q_()


def Q_():
    from paper_1811_11722_amd import qmc
    qmc.lib()
    return qmc


def _oracle_q(n, g, sh, tab, lam, tk, alpha, eps=None):
    est = O.estimate(n, g, sh, O.Params("sector", tab.d, sector=tab, deform=lam, eps=eps), tk, alpha,
                     threads=THREADS)
    assert est.status == 0
    return est


def _floor(n, g, sh, tab, lam, tk, alpha):
    """Largest relative move of the oracle's Q_k when F's monomials are summed
    in three other orders (same polynomial, different rounding)."""
    base = _oracle_q(n, g, sh, tab, lam, tk, alpha).q
    worst = 0.0
    for s in range(3):
        perm = np.random.default_rng(s).permutation(tab.n_f)
        t2 = dataclasses.replace(tab, coef_f=tab.coef_f[perm], exp_f=tab.exp_f[perm])
        q2 = _oracle_q(n, g, sh, t2, lam, tk, alpha).q
        worst = max(worst, float(np.max(np.abs(q2 - base) / np.abs(base))))
    return worst


def _ok(q, est, floor=0.0):
    """The bar above; returns (passed, worst ratio of difference to bar)."""
    qo = est.q
    bar = np.maximum(TOL * np.maximum(np.abs(qo), est.q_abs), 4 * floor * np.abs(qo))
    r = np.abs(np.asarray(q) - qo) / bar
    return bool(np.all(r <= 1.0)), float(r.max())


def _gpu(Q, d, n, g, sh, tab, lam, tk, alpha, launch=None):
    plan = Q.Plan(d, n, g, sh, tk, alpha)
    if launch:
        plan.set_launch(*launch)
    res, q = plan.integrate(Q.Params("sector", d, sector=tab, deform=lam), allow_crossing=True)
    assert plan.last_launch()[2], "deformation runs on the specialised kernel"
    plan.close()
    _crossings_match(res.contour_crossed, n, g, sh, tab, lam, tk, alpha)
    return res, np.asarray(q)


def _crossings_match(crossed, n, g, sh, tab, lam, tk, alpha):
    """The crossing count of the estimate's own pass equals the oracle's sign
    check (at most 2^22 points; beyond, the GPU's separate check)."""
    if n * len(sh) <= 1 << 22:
        chk = O.estimate(n, g, sh, O.Params("sector", tab.d, sector=tab, deform=lam, deform_check=True), tk, alpha,
                         threads=THREADS)
        want = int(np.rint(chk.q_re * n).sum())
    else:
        plan = Q_().Plan(tab.d, n, g, sh, tk, alpha)
        frac, per = plan.deform_check(Q_().Params("sector", tab.d, sector=tab, deform=lam))
        plan.close()
        want = int(np.rint(per * n).sum())
    assert round(crossed * len(sh) * n) == want, (crossed, want)


@pytest.mark.parametrize("lam", [0.005, 0.02])
@pytest.mark.parametrize("tk,alpha", [("baker", 0), ("korobov", 3)])
def test_deform_euclidean_matches_oracle_and_cauchy(Q, lam, tk, alpha):
    """A Euclidean sector (F > 0): per-shift sums against the oracle, and the
    mean against the undeformed integral (unchanged by Cauchy's theorem).
    |grad F| reaches ~240 on this sector, so lambda up to 0.02 keeps the
    contour on the -i0 side everywhere (sign check 0); larger lambda leaves
    the first-order regime."""
    d, n, m = 6, 65521, 8
    tab = synth.sector_tables(301, d, 12, 30)
    g = O.korobov_vector(n, d, 17364)
    sh = synth.shifts(301, m, d)
    _say(f"deform euclidean lam={lam} {tk}{alpha}")
    res, q = _gpu(Q, d, n, g, sh, tab, lam, tk, alpha)
    est = _oracle_q(n, g, sh, tab, lam, tk, alpha)
    assert q.dtype.kind == "c" and res.is_complex
    ok, worst = _ok(q, est)
    assert ok, worst
    plan = Q.Plan(d, n, g, sh, tk, alpha)
    plain, _ = plan.integrate(Q.Params("sector", d, sector=tab))
    frac, _ = plan.deform_check(Q.Params("sector", d, sector=tab, deform=lam))
    plan.close()
    assert frac == 0.0
    assert abs(res.mean_re - plain.mean_re) < 6 * (res.err_re + plain.err_re)
    assert abs(res.mean_im) < 6 * res.err_im


@pytest.mark.parametrize("d,n_u,n_f", [(3, 5, 9), (6, 12, 30), (10, 20, 60), (16, 16, 40)])
@pytest.mark.parametrize("launch", [None, (2, 0)])
def test_deform_mixed_sign_kinematics(Q, d, n_u, n_f, launch):
    """Mixed-sign F (it vanishes inside the cube) at delta = 0: only the
    deformation makes the integrand finite."""
    n, m, lam = (16381, 6, 0.5) if d <= 10 else (4093, 4, 0.5)
    tab = synth.sector_tables(400 + d, d, n_u, n_f, complex_kinematics=True)
    tab = dataclasses.replace(tab, delta_im=0.0, is_complex=True)
    ab, _, _ = O.korobov_search(n, d, synth.korobov_candidates(400 + d, n, 8), threads=THREADS)
    g = O.korobov_vector(n, d, ab)
    sh = synth.shifts(400 + d, m, d)
    _say(f"deform mixed d={d} nU={n_u} nF={n_f} launch={launch}")
    res, q = _gpu(Q, d, n, g, sh, tab, lam, "korobov", 3, launch)
    est = _oracle_q(n, g, sh, tab, lam, "korobov", 3)
    fl = _floor(n, g, sh, tab, lam, "korobov", 3)
    assert fl < 2.5e-10
    ok, worst = _ok(q, est, fl)
    assert ok, (worst, fl)


@pytest.mark.parametrize("p", [-0.7, -1.5])
def test_deform_circle_threshold(Q, p):
    """F = (x1 - 1/2)^2 + (x2 - 1/2)^2 - 0.09 vanishes on a circle inside the
    square: against the oracle per shift, and against the closed -i0 value
    (the smooth deformed integrand reaches it to rounding)."""
    sys.path.insert(0, os.path.dirname(__file__))
    from test_oracle_pins import _circle_closed, circle_sector
    d, n, m, R = 2, 65521, 8, 0.3
    tab = circle_sector(R, p)
    a, _, _ = O.korobov_search(n, d, synth.korobov_candidates(8, n, 16), threads=THREADS)
    g = O.korobov_vector(n, d, a)
    sh = synth.shifts(3, m, d)
    _say(f"deform circle p={p}")
    res, q = _gpu(Q, d, n, g, sh, tab, 0.5, "korobov", 3)
    ok, worst = _ok(q, _oracle_q(n, g, sh, tab, 0.5, "korobov", 3))
    assert ok, worst
    want = _circle_closed(p, R)
    assert abs(complex(res.mean_re, res.mean_im) - want) < 1e-12 * abs(want)


def test_deform_xmy_closed_form(Q):
    """eq. (7) at delta = 0 through the deformation: I = [1 + e^(-i pi eps)] /
    (eps (eps - 1)); Korobov weight 3 tames the corner singularities.  The
    deformed integrand is unbounded at the corners (0, 0) and (1, 1), where a
    double resolves z and 1 - z only to absolute rounding, so the per-shift
    sums of any two FP64 implementations differ by more than 1e-12 there
    (up to ~1e-6 of the summed magnitudes); both must still give the closed
    form within their error."""
    d, n, m, eps = 2, 262139, 16, 0.3
    tab = synth.SectorTables(d=d, coef_u=np.array([1.0]), exp_u=np.zeros((1, d), np.uint8),
                             coef_f=np.array([1.0, -1.0]), exp_f=np.array([[1, 0], [0, 1]], np.uint8),
                             nu=np.zeros(d, np.uint8), pow_u=-2.0, pow_f=-2.0 + eps, delta_im=0.0,
                             is_complex=True)
    a, _, _ = O.korobov_search(n, d, synth.korobov_candidates(8, n, 16), threads=THREADS)
    g = O.korobov_vector(n, d, a)
    sh = synth.shifts(8, m, d)
    _say("deform xmy")
    res, q = _gpu(Q, d, n, g, sh, tab, 1.0, "korobov", 3)
    est = _oracle_q(n, g, sh, tab, 1.0, "korobov", 3)
    mo, eo_re, eo_im = est.mean_error()
    want = (1 + np.exp(-1j * np.pi * eps)) / (eps * (eps - 1))
    assert abs(mo - want) < 1e-3 * abs(want)
    assert np.all(np.abs(q - est.q) <= 1e-5 * est.q_abs)
    got = complex(res.mean_re, res.mean_im)
    assert abs(got.real - want.real) < 6 * res.err_re
    assert abs(got.imag - want.imag) < 6 * res.err_im
    assert abs(got - want) < 1e-3 * abs(want)


@pytest.mark.parametrize("n", [2, 7, 1021])
def test_deform_small_and_one_dimensional(Q, n):
    """d = 1 threshold F = x - a (closed form at large n), and ragged tiny n."""
    a = 0.37
    tab = synth.SectorTables(d=1, coef_u=np.array([1.0]), exp_u=np.zeros((1, 1), np.uint8),
                             coef_f=np.array([-a, 1.0]), exp_f=np.array([[0], [1]], np.uint8),
                             nu=np.zeros(1, np.uint8), pow_u=-2.0, pow_f=-1.5, delta_im=0.0,
                             is_complex=True)
    g = np.array([1], np.uint32)
    sh = synth.shifts(5, 4, 1)
    _say(f"deform d=1 n={n}")
    res, q = _gpu(Q, 1, n, g, sh, tab, 0.5, "korobov", 3)
    ok, worst = _ok(q, _oracle_q(n, g, sh, tab, 0.5, "korobov", 3))
    assert ok, worst


def test_deform_orders_match_oracle(Q):
    """Expansion orders of the deformed integrand in one pass."""
    d, n, m = 5, 16381, 6
    tab = synth.sector_tables(93, d, 7, 12, complex_kinematics=True)
    tab = dataclasses.replace(tab, delta_im=0.0, is_complex=True)
    g = O.korobov_vector(n, d, 17364)
    sh = synth.shifts(93, m, d)
    plan = Q.Plan(d, n, g, sh, "korobov", 3)
    _say("deform orders")
    res, per = plan.integrate_orders(Q.Params("sector", d, sector=tab, orders=(3, 0.7, -1.2), deform=0.5),
                                     allow_crossing=True)
    plan.close()
    assert len(res) == 3 and per.shape == (m, 3)
    assert len({r.contour_crossed for r in res}) == 1
    _crossings_match(res[0].contour_crossed, n, g, sh, tab, 0.5, "korobov", 3)
    fl = _floor(n, g, sh, tab, 0.5, "korobov", 3)
    for k in range(3):
        ok, worst = _ok(per[:, k], _oracle_q(n, g, sh, tab, 0.5, "korobov", 3, eps=(0.7, -1.2, k)), fl)
        assert ok, (k, worst, fl)


def test_deform_validation(Q):
    d, n = 3, 1021
    tab = synth.sector_tables(92, d, 3, 4)
    g = O.korobov_vector(n, d, 76)
    sh = synth.shifts(92, 2, d)
    plan = Q.Plan(d, n, g, sh, "baker")
    with pytest.raises(Q.QMCError) as e:
        plan.integrate(Q.Params("sector", d, sector=tab, deform=float("nan")))
    assert e.value.status == Q.QMC_EINVAL
    bad = dataclasses.replace(tab, pow_u=2.0e5)
    with pytest.raises(Q.QMCError) as e:
        plan.integrate(Q.Params("sector", d, sector=bad, deform=0.5))
    assert e.value.status == Q.QMC_EUNSUPPORTED
    plan.set_jit(0)
    with pytest.raises(Q.QMCError) as e:
        plan.integrate(Q.Params("sector", d, sector=tab, deform=0.5))
    assert e.value.status == Q.QMC_EUNSUPPORTED
    plan.set_jit(1)
    with pytest.raises(Q.QMCError) as e:
        plan.cv_train(Q.Params("sector", d, sector=tab, deform=0.5), 4, 4)
    assert e.value.status == Q.QMC_EUNSUPPORTED
    with pytest.raises(Q.QMCError) as e:
        Q.integrate_batch([plan], [Q.Params("sector", d, sector=tab, deform=0.5)])
    assert e.value.status == Q.QMC_EUNSUPPORTED
    plan.close()


def test_deform_in_specialised_batch(Q):
    """Deformed sectors batched with the specialised schedule equal their
    single-plan estimates."""
    d, n = 5, 4093
    tabs = [dataclasses.replace(synth.sector_tables(500 + s, d, 7, 12, complex_kinematics=True),
                                delta_im=0.0, is_complex=True) for s in range(4)]
    g = O.korobov_vector(n, d, 1234)
    plans = [Q.Plan(d, n, g, synth.shifts(500 + s, 4, d), "korobov", 3) for s in range(4)]
    params = [Q.Params("sector", d, sector=t, deform=0.05) for t in tabs]
    _say("deform specialised batch")
    out = Q.integrate_batch(plans, params, schedule="specialised")
    for p, pa, r in zip(plans, params, out):
        single, _ = p.integrate(pa)
        assert (r.mean_re, r.mean_im, r.err_re, r.err_im) == (single.mean_re, single.mean_im, single.err_re,
                                                              single.err_im)
        p.close()


def test_deform_full_size_sampled(Q):
    """The benchmark's sector shape (d = 6, n_U = 12, n_F = 30, m = 32) with
    mixed-sign F and the deformation at n = 2^24 - 3 in the default launch;
    the oracle recomputes 2 of the 32 shifts at n = 2^20 - 3 on a second plan
    (the oracle's cost per deformed point is ~50x the plain one)."""
    w = synth.sector_workload()
    tab = synth.sector_tables(777, w.d, 12, 30, complex_kinematics=True)
    tab = dataclasses.replace(tab, delta_im=0.0, is_complex=True)
    a, _, _ = Q.korobov_search(w.n, w.d, w.candidates)
    g = O.korobov_vector(w.n, w.d, a)
    _say("deform full size")
    res, q = _gpu(Q, w.d, w.n, g, w.shifts, tab, 0.5, "korobov", 3)
    assert np.all(np.isfinite(q)) and res.is_complex
    n2 = 1048573
    g2 = O.korobov_vector(n2, w.d, 1234)
    pick = [0, 31]
    _, q2 = _gpu(Q, w.d, n2, g2, w.shifts, tab, 0.5, "korobov", 3)
    est = _oracle_q(n2, g2, w.shifts[pick], tab, 0.5, "korobov", 3)
    fl = _floor(16381, O.korobov_vector(16381, w.d, 1234), w.shifts[pick], tab, 0.5, "korobov", 3)
    ok, worst = _ok(q2[pick], est, fl)
    assert ok, (worst, fl)


@pytest.mark.parametrize("lam", [3.0, 20.0])
def test_deform_crossing_reported(Q, lam):
    """qmc_integrate counts the sign check in its own pass: at lambda = 20 the
    quartic F = x1^2 x2^2 - 0.05 crosses the cut on a region, and the call
    returns ECONTOUR with the result filled in and the fraction equal to the
    separate check's (and the oracle's); at lambda = 3 it does not.  Orders
    and the specialised batch report it the same way."""
    n, d = 65521, 2
    g = O.korobov_vector(n, d, 17364)
    sh = synth.shifts(21, 4, d)
    tab = synth.SectorTables(d=d, coef_u=np.array([1.0]), exp_u=np.zeros((1, d), np.uint8),
                             coef_f=np.array([-0.05, 1.0]), exp_f=np.array([[0, 0], [2, 2]], np.uint8),
                             nu=np.zeros(d, np.uint8), pow_u=-2.0, pow_f=-1.5, delta_im=0.0, is_complex=True)
    pa = Q.Params("sector", d, sector=tab, deform=lam)
    plan = Q.Plan(d, n, g, sh, "none")
    _say(f"deform crossing lam={lam}")
    frac, _ = plan.deform_check(pa)
    st, res, per = plan.integrate_status(pa)
    if lam == 3.0:
        assert st == Q.QMC_OK and res.contour_crossed == 0.0 and frac == 0.0
    else:
        assert st == Q.QMC_ECONTOUR and frac > 0.01
        assert abs(res.contour_crossed - frac) <= 1e-15
        assert np.all(np.isfinite(per[: 2 * len(sh)])) and np.isfinite(res.mean_re) and res.err_re > 0
        with pytest.raises(Q.QMCError) as e:
            plan.integrate(pa)
        assert e.value.status == Q.QMC_ECONTOUR
    r2, q2 = plan.integrate(pa, allow_crossing=True)
    assert (r2.mean_re, r2.mean_im, r2.contour_crossed) == (res.mean_re, res.mean_im, res.contour_crossed)
    assert np.array_equal(q2, per[0::2] + 1j * per[1::2])
    _crossings_match(res.contour_crossed, n, g, sh, tab, lam, "none", 0)
    po = Q.Params("sector", d, sector=tab, deform=lam, orders=(2, 0.3, -0.4))
    ro, _ = plan.integrate_orders(po, allow_crossing=True)
    assert all(abs(r.contour_crossed - frac) <= 1e-15 for r in ro)
    rb = Q.integrate_batch([plan], [pa], schedule="specialised", allow_crossing=True)
    assert abs(rb[0].contour_crossed - frac) <= 1e-15
    plan.close()


@pytest.mark.parametrize("lam", [3.0, 6.0, 20.0])
def test_deform_check_quartic_counts(Q, lam):
    """Sign check of F = x1^2 x2^2 - 0.05 (violated on a region for large
    lambda, none at 3): per-shift violation counts equal the oracle's."""
    n, d = 65521, 2
    g = O.korobov_vector(n, d, 17364)
    sh = synth.shifts(21, 4, d)
    tab = synth.SectorTables(d=d, coef_u=np.array([1.0]), exp_u=np.zeros((1, d), np.uint8),
                             coef_f=np.array([-0.05, 1.0]), exp_f=np.array([[0, 0], [2, 2]], np.uint8),
                             nu=np.zeros(d, np.uint8), pow_u=-2.0, pow_f=-1.5, delta_im=0.0, is_complex=True)
    plan = Q.Plan(d, n, g, sh, "none")
    _say(f"deform check quartic lam={lam}")
    frac, per = plan.deform_check(Q.Params("sector", d, sector=tab, deform=lam))
    plan.close()
    est = O.estimate(n, g, sh, O.Params("sector", d, sector=tab, deform=lam, deform_check=True), threads=THREADS)
    assert np.array_equal(np.rint(per * n), np.rint(est.q_re * n)), (per * n, est.q_re * n)
    assert (frac == 0.0) == (lam == 3.0)
    assert abs(frac - est.q_re.mean()) <= 1e-15


@pytest.mark.parametrize("lam", [0.05, 0.1, 0.2, 0.5])
def test_deform_check_sector_counts(Q, lam):
    """Sign check of a mixed-sign d = 6 sector under the Korobov transform:
    per-shift counts equal the oracle's."""
    d, n, m = 6, 65521, 4
    tab = synth.sector_tables(406, d, 12, 30, complex_kinematics=True)
    tab = dataclasses.replace(tab, delta_im=0.0, is_complex=True)
    g = O.korobov_vector(n, d, 17364)
    sh = synth.shifts(406, m, d)
    plan = Q.Plan(d, n, g, sh, "korobov", 3)
    _say(f"deform check sector lam={lam}")
    frac, per = plan.deform_check(Q.Params("sector", d, sector=tab, deform=lam))
    plan.close()
    est = O.estimate(n, g, sh, O.Params("sector", d, sector=tab, deform=lam, deform_check=True), "korobov", 3,
                     threads=THREADS)
    assert np.array_equal(np.rint(per * n), np.rint(est.q_re * n)), (per * n, est.q_re * n)


def test_deform_select_rule(Q):
    """The selection returns the ladder lambda with no violation and the
    smallest error, and its result is qmc_integrate's at that lambda."""
    d, n, m = 6, 65521, 8
    tab = synth.sector_tables(406, d, 12, 30, complex_kinematics=True)
    tab = dataclasses.replace(tab, delta_im=0.0, is_complex=True)
    g = O.korobov_vector(n, d, 17364)
    sh = synth.shifts(406, m, d)
    plan = Q.Plan(d, n, g, sh, "korobov", 3)
    _say("deform select")
    lam, res = plan.deform_select(Q.Params("sector", d, sector=tab), lam_max=0.8, shrink=0.5, count=7)
    ladder = [0.8 * 0.5 ** i for i in range(7)]
    assert lam in ladder
    errs = {}
    for L in ladder:
        p = Q.Params("sector", d, sector=tab, deform=L)
        frac, _ = plan.deform_check(p)
        if frac == 0.0:
            st, r, _ = plan.integrate_status(p)
            if st == Q.QMC_OK:
                errs[L] = math.hypot(r.err_re, r.err_im)
    assert errs and lam == min(errs, key=errs.get)
    r, _ = plan.integrate(Q.Params("sector", d, sector=tab, deform=lam))
    assert (r.mean_re, r.mean_im, r.err_re, r.err_im) == (res.mean_re, res.mean_im, res.err_re, res.err_im)
    with pytest.raises(Q.QMCError) as e:
        plan.deform_select(Q.Params("sector", d, sector=tab), lam_max=0.8, shrink=1.5, count=7)
    assert e.value.status == Q.QMC_EINVAL
    with pytest.raises(Q.QMCError) as e:
        plan.deform_check(Q.Params("sector", d, sector=tab))
    assert e.value.status == Q.QMC_EINVAL
    plan.close()
