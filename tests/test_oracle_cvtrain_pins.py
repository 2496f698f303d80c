"""Pins of the oracle's control-variate training routines (CPU only).

Each routine is tied to something other than itself:
- bfloat16 rounding against its definition (8 significant bits, nearest,
  ties to even) evaluated through frexp / rint, and known-answer ties;
- the step's design-matrix columns against monomial models whose Legendre
  coefficients are known in closed form, against the pinned model g(z), and
  the Legendre values against scipy;
- the normal equations against numpy products of the same quantised design
  matrix;
- the Cholesky solve against numpy's dense solver, including the ridge
  escalation on an indefinite matrix;
- the exact least-squares step against numpy's normal-equation solution and
  its optimality (gradient zero, objective not above the starting point).
"""
import math

import numpy as np
import pytest
from scipy.special import eval_legendre

from oracle import oracle as O


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def bf16_by_frexp(x):
    """Round float32 values to 8 significant bits, nearest with ties to even,
    by scaling the frexp significand (in [1/2, 1)) to [128, 256)."""
    x = np.asarray(x, dtype=np.float32).astype(np.float64)
    m, e = np.frexp(x)
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


def test_bf16_known_ties():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties to the even 1
    assert O.bf16(1.0 + 2.0 ** -8) == 1.0
    # 1 + 3 * 2^-8 lies halfway between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    assert O.bf16(1.0 + 3.0 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert O.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7  # above the tie
    assert O.bf16(-3.0) == -3.0
    assert O.bf16(0.0) == 0.0
    assert math.isinf(O.bf16(float(np.finfo(np.float32).max)))  # rounds up past the largest bf16
    assert math.isnan(O.bf16(float("nan")))


def test_bf16_matches_definition():
    rng = np.random.default_rng(1)
    x = (rng.standard_normal(20000) * np.exp(rng.uniform(-40, 40, 20000))).astype(np.float32)
    got = np.array([O.bf16(float(v)) for v in x])
    assert np.array_equal(got, bf16_by_frexp(x))


def _monomial_legendre(nu, K):
    """Coefficients of z^nu (nu <= 2) in P~_k(z) = sqrt(2k+1) P_k(2z - 1)."""
    c = {0: [1.0], 1: [0.5, 0.5 / math.sqrt(3.0)],
         2: [1.0 / 3.0, 0.5 / math.sqrt(3.0), 1.0 / (6.0 * math.sqrt(5.0))]}[nu]
    return np.array(c + [0.0] * (K - len(c)))


def _samples(seed, n, d):
    rng = np.random.default_rng(seed)
    z = rng.random((n, d)).astype(np.float32)
    sw = rng.uniform(0.5, 1.5, n).astype(np.float32)
    return rng, z, sw


def test_features_of_monomial_models():
    """W[r, i', :] = Legendre coefficients of z^nu[r, i']: rho_j[r] is
    sw_j prod_{i' != i} z^nu exactly (up to rounding)."""
    n, d, R, K, i = 300, 4, 5, 4, 2
    rng, z, sw = _samples(2, n, d)
    nu = rng.integers(0, 3, (R, d))
    W = np.zeros((R, d, K))
    for r in range(R):
        for ii in range(d):
            W[r, ii] = _monomial_legendre(int(nu[r, ii]), K)
    rho, phi, env = O.cv_features(z, sw, W, i)
    zz = z.astype(np.float64)
    want = sw[:, None].astype(np.float64) * np.prod(
        [zz[:, [ii]] ** nu[:, ii][None, :] for ii in range(d) if ii != i], axis=0)
    # the Legendre form of z^2 cancels for small z: the bound is on the scale
    # of the terms (the envelope), not of the value
    assert np.all(np.abs(rho - want) <= 1e-14 * env)
    assert np.all(env >= np.abs(rho))


def test_features_reproduce_model_and_scipy_legendre():
    n, d, R, K = 200, 5, 6, 7
    rng, z, sw = _samples(3, n, d)
    W = rng.standard_normal((R, d, K))
    for i in range(d):
        rho, phi, env = O.cv_features(z, sw, W, i)
        for j in range(0, n, 17):
            # sw g(z) = sum_{r,k} rho[r] W[r,i,k] phi[k], c = 1
            g = O.cv_g(W, np.ones(R), z[j].astype(np.float64))
            lin = float(np.einsum("r,rk,k->", rho[j], W[:, i, :], phi[j]))
            assert abs(lin - float(sw[j]) * g) <= 1e-12 * max(1.0, np.sum(env[j]))
        t = 2.0 * z[:, i].astype(np.float64) - 1.0
        ref = np.stack([math.sqrt(2 * k + 1) * eval_legendre(k, t) for k in range(K)], axis=1)
        assert np.allclose(phi, ref, rtol=0, atol=1e-13)
        assert np.all(env >= np.abs(rho) * (1 - 1e-15))


def test_normal_equations_against_numpy():
    n, R, K = 700, 6, 5
    rng = np.random.default_rng(4)
    rho = rng.standard_normal((n, R)) * np.exp(rng.uniform(-3, 3, (n, R)))
    phi = rng.uniform(-2, 2, (n, K))
    y = rng.standard_normal(n)
    G, b, Ga, ba = O.cv_normal(rho, phi, y, threads=4)
    # the matrix: single-precision factors multiplied in single precision,
    # then rounded to bfloat16
    A32 = (rho.astype(np.float32)[:, :, None] * phi.astype(np.float32)[:, None, :]).reshape(n, R * K)
    assert A32.dtype == np.float32
    A16 = bf16_by_frexp(A32)
    Gref = A16.T @ A16
    Gabs = np.abs(A16).T @ np.abs(A16)
    assert np.all(np.abs(G - Gref) <= 4 * n * 2.0 ** -52 * Gabs)
    assert np.allclose(Ga, Gabs, rtol=1e-13, atol=0)
    # the right-hand side: the double design matrix
    A64 = (rho[:, :, None] * phi[:, None, :]).reshape(n, R * K)
    bref = A64.T @ y
    babs = np.abs(A64).T @ np.abs(y)
    assert np.all(np.abs(b - bref) <= 4 * n * 2.0 ** -52 * babs)
    assert np.array_equal(G, G.T)
    assert np.min(np.linalg.eigvalsh(G)) >= -1e-12 * np.max(np.diag(G))
    # sampled entries are the same sums
    us = rng.integers(0, R * K, 20)
    vs = rng.integers(0, R * K, 20)
    g2, ga2, b2, ba2 = O.cv_normal_at(rho, phi, y, us, vs)
    assert np.array_equal(g2, G[us, vs]) and np.array_equal(b2, b[us])
    assert np.array_equal(ga2, Ga[us, vs]) and np.array_equal(ba2, ba[us])


def test_solve_against_numpy_and_escalation():
    rng = np.random.default_rng(5)
    F = 40
    M = rng.standard_normal((F, 3 * F))
    G = M @ M.T
    b = rng.standard_normal(F)
    x, lam, esc = O.cv_solve(G, b, 1e-5)
    assert esc == 0
    assert lam == pytest.approx(1e-5 * np.trace(G) / F, rel=1e-14)
    ref = np.linalg.solve(G + lam * np.eye(F), b)
    assert np.allclose(x, ref, rtol=1e-10, atol=1e-12 * np.max(np.abs(ref)))
    # indefinite: the second pivot is negative until lam > 0.5; trace / F = 0.25,
    # so the ridges 1e-5, 1e-3, 1e-1 fail and 10 (lam = 2.5) succeeds
    G2 = np.diag([1.0, -0.5])
    x2, lam2, esc2 = O.cv_solve(G2, np.array([1.0, 2.0]), 1e-5)
    assert esc2 == 3 and lam2 == pytest.approx(2.5, rel=1e-12)
    assert np.allclose(x2, [1.0 / 3.5, 2.0 / 2.0], rtol=1e-14)
    _, _, esc3 = O.cv_solve(np.diag([1.0, -5.0]), np.ones(2), 1e-5)
    assert esc3 == -1


def test_step_is_the_ridge_least_squares_solution():
    n, d, R, K = 2000, 4, 4, 5
    rng, z, sw = _samples(6, n, d)
    zz = z.astype(np.float64)
    y = sw * (1.0 / (1.0 + np.sum(zz, axis=1))) + 0.01 * rng.standard_normal(n)
    W = rng.standard_normal((R, d, K)) * 0.3
    W[:, :, 0] += 0.7
    ridge = 1e-5
    for i in range(d):
        Wn, lam = O.cv_step(z, sw, y, W, i, ridge, threads=4)
        rho, phi, _ = O.cv_features(z, sw, W, i)
        A = (rho[:, :, None] * phi[:, None, :]).reshape(n, R * K)
        N = A.T @ A
        lref = ridge * np.trace(N) / (R * K)
        assert lam == pytest.approx(lref, rel=1e-12)
        w = np.linalg.solve(N + lref * np.eye(R * K), A.T @ y.astype(np.float64))
        got = Wn[:, i, :].reshape(-1)
        assert np.allclose(got, w, rtol=1e-8, atol=1e-10 * np.max(np.abs(w)))
        # the other dimensions are untouched
        mask = np.ones(d, bool)
        mask[i] = False
        assert np.array_equal(Wn[:, mask, :], W[:, mask, :])
        # optimality: the gradient of the ridge objective vanishes, and the
        # objective is not above the starting factors'
        grad = A.T @ (A @ got - y) + lam * got
        assert np.max(np.abs(grad)) <= 1e-9 * np.max(np.abs(A.T @ y))
        J0, _ = O.cv_objective(z, sw, y, W, i, lam)
        J1, sy = O.cv_objective(z, sw, y, Wn, i, lam)
        assert J1 <= J0 * (1 + 1e-12)
        # the objective agrees with the pinned model g(z)
        gs = np.array([O.cv_g(Wn, np.ones(R), zz[j]) for j in range(0, n, 97)])
        e = y[::97] - sw[::97].astype(np.float64) * gs
        Jsub = np.sum(e * e)
        Jo, _ = O.cv_objective(z[::97], sw[::97], y[::97], Wn, i, 0.0)
        assert Jo == pytest.approx(Jsub, rel=1e-10)
        W = Wn
