"""Control variate on the GPU: FP64 residual against the oracle, and the
MFMA-assembled least-squares training on an exactly representable model."""
import math
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1811_11722_amd import synth

pytestmark = pytest.mark.gpu
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


@pytest.mark.parametrize("R,K", [(8, 4), (16, 8), (32, 12)])
def test_cv_residual_matches_oracle(Q, R, K):
    """Same FP64 weights on both sides: plain and residual Q_k agree, and
    int g matches the oracle's closed form."""
    d, n, m = 5, 16381, 6
    tab = synth.sector_tables(41, d, 8, 14)
    g = O.korobov_vector(n, d, 17364)
    sh = synth.shifts(41, m, d)
    rng = np.random.default_rng(R * 100 + K)
    W = rng.normal(size=(R, d, K)) / np.sqrt(K)
    W[:, :, 0] += 1.0
    c = rng.normal(size=R) * 1e-3
    plan = Q.Plan(d, n, g, sh, "baker")
    _say(f"cv residual R={R} K={K}")
    out, plain, qp, qr = plan.integrate_cv(Q.Params("sector", d, sector=tab), W, c)
    ep = O.estimate(n, g, sh, O.Params("sector", d, sector=tab), "baker", threads=THREADS)
    er = O.estimate(n, g, sh, O.Params("sector", d, sector=tab, cv=(W, c)), "baker", threads=THREADS)
    scale = np.maximum(np.abs(ep.q_re), np.abs(er.q_re))
    assert np.all(np.abs(qp - ep.q_re) <= 1e-12 * np.abs(ep.q_re))
    assert np.all(np.abs(qr - er.q_re) <= 1e-12 * scale), np.max(np.abs(qr - er.q_re) / scale)
    ig = Q.cv_integral(W, c)
    assert abs(ig - O.cv_integral(W, c)) <= 1e-14 * max(1.0, abs(ig))
    assert abs(plain.mean_re - ep.mean_error()[0].real) <= 1e-12 * abs(plain.mean_re)


def test_cv_zero_model_is_plain_bitwise(Q):
    """W = 0 makes g = 0: the residual sums are the plain sums bit for bit."""
    d, n, m = 4, 4093, 4
    tab = synth.sector_tables(43, d, 5, 9)
    plan = Q.Plan(d, n, O.korobov_vector(n, d, 1077), synth.shifts(43, m, d), "baker")
    _say("cv zero model")
    W = np.zeros((8, d, 4))
    c = np.ones(8)
    out, plain, qp, qr = plan.integrate_cv(Q.Params("sector", d, sector=tab), W, c)
    assert np.array_equal(qp, qr)
    assert Q.cv_integral(W, c) == 0.0


def _monomial_legendre(nu):
    """Coefficients of z^nu (nu <= 2) in the orthonormal shifted Legendre basis
    P~_k(z) = sqrt(2k+1) P_k(2z - 1), k < 4."""
    return {0: [1.0, 0.0, 0.0, 0.0],
            1: [0.5, 0.5 / math.sqrt(3.0), 0.0, 0.0],
            2: [1.0 / 3.0, 0.5 / math.sqrt(3.0), 1.0 / (6.0 * math.sqrt(5.0)), 0.0]}[nu]


def test_cv_exact_model_gives_zero_error(Q):
    """f = C prod z^nu is itself a rank-1 Legendre model: with the exact
    coefficients the residual is rounding noise, the error collapses and the
    estimate is the closed form int g = C prod 1/(nu_i + 1)."""
    d = 4
    nu = [1, 2, 0, 1]
    s = synth.SectorTables(d=d, coef_u=np.array([1.5]), exp_u=np.zeros((1, d), np.uint8),
                           coef_f=np.array([0.7]), exp_f=np.zeros((1, d), np.uint8),
                           nu=np.array(nu, np.uint8))
    C = 1.5 ** -2 * 0.7 ** -1.3
    exact = C / (2 * 3 * 1 * 2)
    W = np.zeros((8, d, 4))
    for i, v in enumerate(nu):
        W[0, i] = _monomial_legendre(v)
    c = np.zeros(8)
    c[0] = C
    n = 16381
    plan = Q.Plan(d, n, O.korobov_vector(n, d, 5029), synth.shifts(4, 8, d), "baker")
    _say("cv exact model")
    out, plain, qp, qr = plan.integrate_cv(Q.Params("sector", d, sector=s), W, c)
    assert out.used_cv == 1
    assert out.err_re <= 1e-14 * exact
    assert abs(out.mean_re - exact) <= 1e-14 * exact
    assert abs(Q.cv_integral(W, c) - exact) <= 1e-15 * exact


def test_cv_training_recovers_separable_integrand(Q):
    """U and F constant: f = c_U^-2 c_F^-1.3 prod z^nu is a rank-1 product of
    polynomials of degree <= 2, so the fitted model reproduces it, the
    residual variance collapses and int g + Q[f - g] hits the closed form."""
    d = 4
    s = synth.SectorTables(d=d, coef_u=np.array([1.5]), exp_u=np.zeros((1, d), np.uint8),
                           coef_f=np.array([0.7]), exp_f=np.zeros((1, d), np.uint8),
                           nu=np.array([1, 2, 0, 1], np.uint8))
    exact = 1.5 ** -2 * 0.7 ** -1.3 / (2 * 3 * 1 * 2)
    nt = 65521
    gt = O.korobov_vector(nt, d, 17364)
    train = Q.Plan(d, nt, gt, synth.shifts(3, 2, d, stream=3), "baker")
    p = Q.Params("sector", d, sector=s)
    _say("cv train separable")
    W, c, rep = train.cv_train(p, 8, 4, max_sweeps=6)
    assert rep.sweeps >= 1 and rep.rel_loss < 1e-6, (rep.sweeps, rep.rel_loss)
    n = 16381
    plan = Q.Plan(d, n, O.korobov_vector(n, d, 5029), synth.shifts(4, 8, d), "baker")
    out, plain, qp, qr = plan.integrate_cv(p, W, c)
    assert out.used_cv == 1
    # the ridge (1e-5 of the mean diagonal) bounds how closely the fit can
    # approach the exact rank-1 model (relative loss ~1e-7), and the
    # lattice error of what remains is what the shifts measure
    print(f"  rel loss {rep.rel_loss:.3g}, error ratio cv / plain {out.err_re / plain.err_re:.3g}, "
          f"plain rel err {plain.err_re / exact:.3g}, cv rel err {out.err_re / exact:.3g}, "
          f"|mean - exact| / exact {abs(out.mean_re - exact) / exact:.3g}")
    assert out.err_re <= 1e-2 * plain.err_re
    assert abs(out.mean_re - exact) <= 6 * out.err_re + 1e-13 * exact


def test_cv_training_sector_reduces_variance(Q):
    """A generic positive sector in d = 4: the fit lowers the training loss
    and the control-variate estimate agrees with the plain one."""
    d = 4
    tab = synth.sector_tables(55, d, 6, 10)
    nt = 65521
    train = Q.Plan(d, nt, O.korobov_vector(nt, d, 17364), synth.shifts(5, 2, d, stream=3), "baker")
    p = Q.Params("sector", d, sector=tab)
    _say("cv train generic sector")
    W, c, rep = train.cv_train(p, 16, 8, max_sweeps=8)
    assert rep.rel_loss < 0.05, rep.rel_loss
    n = 16381
    g = O.korobov_vector(n, d, 5029)
    sh = synth.shifts(6, 8, d)
    plan = Q.Plan(d, n, g, sh, "baker")
    out, plain, qp, qr = plan.integrate_cv(p, W, c)
    assert abs(out.mean_re - plain.mean_re) <= 6 * math.hypot(out.err_re, plain.err_re)
    er = O.estimate(n, g, sh, O.Params("sector", d, sector=tab, cv=(W, c)), "baker", threads=THREADS)
    assert np.all(np.abs(qr - er.q_re) <= 1e-12 * np.maximum(np.abs(qp), np.abs(er.q_re)))


def test_cv_validation(Q):
    d = 2
    plan = Q.Plan(d, 1021, O.korobov_vector(1021, d, 5), synth.shifts(1, 2, d), "baker")
    pg = Q.Params("genz_gaussian", d, a=[1.0, 2.0], u=[0.2, 0.3])
    with pytest.raises(Q.QMCError) as e:
        plan.cv_train(pg, 8, 4)
    assert e.value.status == Q.QMC_EUNSUPPORTED
    tab = synth.sector_tables(1, d, 2, 3)
    with pytest.raises(Q.QMCError) as e:
        plan.cv_train(Q.Params("sector", d, sector=tab), 7, 4)
    assert e.value.status == Q.QMC_EUNSUPPORTED


def _complex_positive_sector(seed, d, n_u, n_f, delta=0.01):
    """Positive U and F (well conditioned) with F -> F - i delta."""
    t = synth.sector_tables(seed, d, n_u, n_f)
    t.delta_im, t.is_complex = delta, True
    return t


def test_cv_complex_residual_matches_oracle(Q):
    """Two models (real and imaginary part), same FP64 weights on both sides."""
    d, n, m, R, K = 5, 16381, 6, 16, 8
    tab = _complex_positive_sector(61, d, 7, 12)
    g = O.korobov_vector(n, d, 17364)
    sh = synth.shifts(61, m, d)
    rng = np.random.default_rng(7)
    W = rng.normal(size=(2, R, d, K)) / np.sqrt(K)
    W[:, :, :, 0] += 1.0
    c = rng.normal(size=(2, R)) * 1e-3
    plan = Q.Plan(d, n, g, sh, "baker")
    _say("cv complex residual")
    out, plain, qp, qr = plan.integrate_cv(Q.Params("sector", d, sector=tab), W, c)
    ep = O.estimate(n, g, sh, O.Params("sector", d, sector=tab), "baker", threads=THREADS)
    er = O.estimate(n, g, sh, O.Params("sector", d, sector=tab, cv=(W, c)), "baker", threads=THREADS)
    ep_q = ep.q_re + 1j * ep.q_im
    er_q = er.q_re + 1j * er.q_im
    assert np.all(np.abs(qp - ep_q) <= 1e-12 * np.abs(ep_q))
    scale = np.maximum(np.abs(ep_q), np.abs(er_q))
    assert np.all(np.abs(qr - er_q) <= 1e-12 * scale), np.max(np.abs(qr - er_q) / scale)
    assert plain.is_complex == 1


def test_cv_complex_exact_models(Q):
    """f = U0^-2 (F0 - i delta)^p prod z^nu: exact real and imaginary models
    make the residual vanish; the estimate is the closed form."""
    d = 4
    nu = [1, 2, 0, 1]
    s = synth.SectorTables(d=d, coef_u=np.array([1.5]), exp_u=np.zeros((1, d), np.uint8),
                           coef_f=np.array([0.7]), exp_f=np.zeros((1, d), np.uint8),
                           nu=np.array(nu, np.uint8), delta_im=0.05, is_complex=True)
    Cc = 1.5 ** -2 * complex(0.7, -0.05) ** -1.3
    exact = Cc / (2 * 3 * 1 * 2)
    W = np.zeros((2, 8, d, 4))
    c = np.zeros((2, 8))
    for i, v in enumerate(nu):
        W[0, 0, i] = W[1, 0, i] = _monomial_legendre(v)
    c[0, 0], c[1, 0] = Cc.real, Cc.imag
    n = 16381
    plan = Q.Plan(d, n, O.korobov_vector(n, d, 5029), synth.shifts(4, 8, d), "baker")
    _say("cv complex exact models")
    out, plain, qp, qr = plan.integrate_cv(Q.Params("sector", d, sector=s), W, c)
    assert out.used_cv == 1 and out.is_complex == 1
    assert math.hypot(out.err_re, out.err_im) <= 1e-14 * abs(exact)
    assert abs(complex(out.mean_re, out.mean_im) - exact) <= 1e-14 * abs(exact)


def test_cv_complex_training(Q):
    """Training fits both components; the estimate agrees with the plain one
    and the trained residual matches the oracle's."""
    d = 4
    tab = _complex_positive_sector(55, d, 6, 10)  # the table of the real training test
    nt = 65521
    train = Q.Plan(d, nt, O.korobov_vector(nt, d, 17364), synth.shifts(8, 2, d, stream=3), "baker")
    p = Q.Params("sector", d, sector=tab)
    _say("cv complex training")
    W, c, rep = train.cv_train(p, 16, 8, max_sweeps=6)
    assert W.shape == (2, 16, d, 8) and c.shape == (2, 16)
    assert rep.rel_loss < 0.05, rep.rel_loss
    n = 16381
    g = O.korobov_vector(n, d, 5029)
    sh = synth.shifts(9, 8, d)
    plan = Q.Plan(d, n, g, sh, "baker")
    out, plain, qp, qr = plan.integrate_cv(p, W, c)
    e = math.hypot(math.hypot(out.err_re, out.err_im), math.hypot(plain.err_re, plain.err_im))
    assert abs(complex(out.mean_re, out.mean_im) - complex(plain.mean_re, plain.mean_im)) <= 6 * e
    er = O.estimate(n, g, sh, O.Params("sector", d, sector=tab, cv=(W, c)), "baker", threads=THREADS)
    er_q = er.q_re + 1j * er.q_im
    assert np.all(np.abs(qr - er_q) <= 1e-12 * np.maximum(np.abs(qp), np.abs(er_q)))
