"""Control-variate training on the GPU against the CPU oracle, step by step.

Each training step is called through its own C entry point on inputs made
on the host (seeded, by the oracle), and compared element by element with
the oracle's FP64 / long-double computation of the same quantity:
- samples (z, J, fhat of the training lattice): the oracle's values rounded
  to single precision, within one unit in the last place;
- design-matrix factors rho, phi: FP64 on both sides (different operation
  order), bound from the length of the recurrences and products (below);
- normal equations: the BF16 matrix and FP64 right-hand side summed exactly
  by the oracle, bound = accumulation length x unit roundoff (FP32 for the
  matrix, FP64 for the right-hand side) x the sum of absolute products, at a
  small size in full and at the training size (n = 1048573, d = 8, R = 32,
  K = 12) on sampled entries;
- the FP64 solve (Cholesky on the oracle side, the explicit inverse from
  the blocked Cholesky on the GPU): the same matrix on both sides, bound
  from the condition number and the methods' stability;
- one whole step with refinement: the exact ridge minimum of the oracle's
  FP64 step and the GPU step's objective (property check, printed).
Shapes: workload 4 (d = 8, R = 32, K = 12, F = 384), workload 5's model
(d = 10, R = 64, K = 12, F = 768) and a small R < 32 case.
"""
import math
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1811_11722_amd import synth

pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 1)
U32 = 2.0 ** -24  # unit roundoff of single precision
U64 = 2.0 ** -53


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def Q():
    O.build(force=False)
    from paper_1811_11722_amd import qmc
    qmc.lib()
    return qmc


def _training_set(seed, d, n, tkind="baker", alpha=0, complex_f=False):
    """Samples of a workload-4-shaped sector (12 / 30 monomials) on a Korobov
    lattice with the training shift (stream 3), computed by the oracle."""
    tab = synth.sector_tables(seed, d, 12, 30, complex_kinematics=complex_f)
    g = O.korobov_vector(n, d, 17364 % n)
    shift = synth.shifts(seed, 1, d, stream=3)[0]
    z, jac, f = O.cv_samples(n, g, shift, O.Params("sector", d, sector=tab), tkind, alpha)
    return tab, g, shift, z, jac, f


def _init_factors(seed, R, d, K):
    """Factors shaped like the training's starting point (near-constant
    rank-1 terms with perturbations)."""
    rng = np.random.default_rng(seed)
    base = (1.0 / R) ** (1.0 / d)
    W = 0.1 * base * (rng.random((R, d, K)) - 0.5) / (np.arange(K) + 1.0)
    W[:, :, 0] = base * (1.0 + 0.5 * (rng.random((R, d)) - 0.5))
    return W


@pytest.mark.parametrize("tk,alpha,cplx", [("baker", 0, False), ("korobov", 3, False), ("baker", 0, True)])
def test_samples_match_oracle(Q, tk, alpha, cplx):
    d, n = 8, 16381
    tab, g, shift, z, jac, f = _training_set(71, d, n, tk, alpha, cplx)
    plan = Q.Plan(d, n, g, shift[None, :].repeat(2, axis=0), tk, alpha)
    p = Q.Params("sector", d, sector=tab)
    for part in ([0, 1] if cplx else [0]):
        _say(f"cv samples {tk}{alpha} complex={cplx} part={part}")
        zg, swg, ywg = plan.cv_samples(p, part)
        want = f.real if part == 0 else f.imag
        # the GPU point idx * (1/n) + shift is within an ulp of the oracle's
        # idx / n + shift.  The GPU's Korobov map is a polynomial in x - 1/2
        # (absolute error a few units of 2^-53, so near 0 its relative error
        # grows), the oracle's the binomial tail; the FP64 values then agree
        # to ~1e-12 relative (J, fhat) or 2^-44 absolute (z), and both round
        # to single precision: at most one unit in the last place apart, plus
        # that FP64 gap
        def ulp32(v):
            return np.spacing(np.abs(v).astype(np.float32)).astype(np.float64)

        dz = np.abs(zg.astype(np.float64) - z.astype(np.float32).astype(np.float64))
        assert np.all(dz <= ulp32(z) + 2.0 ** -44)
        # Near a face the point's own rounding dominates: the GPU's x =
        # {idx (1/n) + shift} is within dx = 2^-52 of the oracle's, a
        # relative change dx / min(x, 1 - x); the Korobov weight grows like
        # x^alpha and z like x^(alpha+1) there, so z^nu J moves by
        # (nu (alpha + 1) + alpha) dx / min(x, 1 - x) per coordinate
        # (counted 4x below)
        # Besides, the GPU evaluates the Korobov map as a polynomial in
        # x - 1/2, accurate to a few units of 2^-53 absolute: the factor z^nu
        # of fhat moves by nu 2^-50 / z relative (counted 4x)
        rel = np.full(n, 1e-12)
        if tk == "korobov":
            x = np.array([O.point(n, g, j, shift) for j in range(n)])
            grow = tab.nu.astype(np.float64) * (alpha + 1) + alpha
            rel += np.sum(grow[None, :] * 2.0 ** -50 / np.minimum(x, 1.0 - x), axis=1)
            rel += np.sum(tab.nu.astype(np.float64)[None, :] * 2.0 ** -48 / np.maximum(z, 1e-300), axis=1)
        # values below the smallest normal single (weights of points near a
        # face, multiplied over 8 coordinates) may come back flushed to zero
        tiny = float(np.finfo(np.float32).tiny)
        dsw = np.abs(swg.astype(np.float64) - jac.astype(np.float32).astype(np.float64))
        assert np.all(dsw <= ulp32(jac) + rel * np.abs(jac) + tiny)
        dy = np.abs(ywg.astype(np.float64) - want.astype(np.float32).astype(np.float64))
        bad = dy > ulp32(want) + rel * np.abs(want) + tiny
        assert not np.any(bad), (np.flatnonzero(bad)[:5], want[bad][:5], ywg[bad][:5])
        print(f"  max |dz| {dz.max():.3g}, max |dy|/|y| {np.max(dy / np.maximum(np.abs(want), 1e-300)):.3g}")


def _feature_bounds(d, K, env, k):
    """|rho_gpu - rho| <= B_rho env and |phi_gpu[k] - phi[k]| <= B_phi sqrt(2k+1).

    FP64 on both sides from the same single-precision z: t = 2z - 1 (exact),
    the Legendre recurrence to degree K - 1 in two operation orders (absolute
    error below 8 (k + 1)^2 u each, a generous cover of the recurrence's at
    most quadratic growth on [-1, 1]), the weights times sqrt(2k+1) (one
    rounding), a K-term Horner sum (K roundings relative to
    sum_k |w_k| sqrt(2k+1)), then d - 1 products and the weight sw (one
    rounding each).  Per factor eta = (16 K^2 + 3 K + 2) u relative to the
    factor's envelope; the product bound is (1 + eta)^(d-1) (1 + u)^d - 1."""
    eta = (16 * K * K + 3 * K + 2) * U64
    B_rho = (1 + eta) ** (d - 1) * (1 + U64) ** d - 1
    B_phi = 16 * (k + 1) ** 2 * U64 + 2 * U64
    return B_rho, B_phi


@pytest.mark.parametrize("d,R,K,n", [(8, 32, 12, 16381 + 130), (10, 64, 12, 4093), (5, 8, 4, 1021)])
def test_features_match_oracle(Q, d, R, K, n):
    tab, g, shift, z, jac, f = _training_set(72, d, n)
    z32, sw32 = z.astype(np.float32), jac.astype(np.float32)
    W = _init_factors(d * 1000 + R, R, d, K)
    for i in sorted({0, d // 2, d - 1}):
        _say(f"cv features d={d} R={R} K={K} n={n} i={i}")
        rho_g, phi_g = Q.cv_features(z32, sw32, W, i)
        rho, phi, env = O.cv_features(z32, sw32, W, i)
        k = np.arange(K)
        B_rho, B_phi = _feature_bounds(d, K, env, k)
        err_rho = np.abs(rho_g - rho)
        err_phi = np.abs(phi_g - phi)
        print(f"  i={i}: max |drho|/env {np.max(err_rho / env):.3g} (bound {B_rho:.3g}), "
              f"max |dphi|/sqrt(2k+1) {np.max(err_phi / np.sqrt(2 * k + 1)):.3g}")
        assert np.all(err_rho <= B_rho * env)
        assert np.all(err_phi <= B_phi[None, :] * np.sqrt(2 * k + 1)[None, :])


def _design_inputs(d, R, K, n, seed, i=0):
    """Factors and target for the normal equations: the oracle's FP64
    features and y = fhat / mean |fhat|."""
    tab, g, shift, z, jac, f = _training_set(seed, d, n)
    W = _init_factors(seed, R, d, K)
    rho, phi, env = O.cv_features(z.astype(np.float32), jac.astype(np.float32), W, i)
    y = f.real / np.mean(np.abs(f.real))
    return rho, phi, y


@pytest.mark.parametrize("d,R,K,n", [(8, 32, 12, 16381 + 77), (10, 64, 12, 4093), (5, 8, 4, 2039),
                                     (6, 16, 8, 33)])
def test_normal_equations_match_oracle(Q, d, R, K, n):
    rho, phi, y = _design_inputs(d, R, K, n, 73)
    _say(f"cv normal d={d} R={R} K={K} n={n}")
    G, b, acc = Q.cv_normal(rho, phi, y)
    Go, bo, Ga, ba = O.cv_normal(rho, phi, y, threads=THREADS)
    # FP32 accumulation of at most acc points per partial (products of two
    # BF16 values are exact in FP32), FP64 over the partials; the right-hand
    # side in FP64 (one rounding of rho phi, then fused multiply-adds)
    bG = (int(acc[0]) + 16) * U32 + n * U64
    bb = (int(acc[1]) + 2) * U64 + n * U64
    eG = np.abs(G - Go)
    eb = np.abs(b - bo)
    print(f"  acc {acc.tolist()}: max |dG|/|G|abs {np.max(eG / np.maximum(Ga, 1e-300)):.3g} (bound {bG:.3g}), "
          f"max |db|/|b|abs {np.max(eb / np.maximum(ba, 1e-300)):.3g} (bound {bb:.3g})")
    assert np.array_equal(G, G.T)
    assert np.all(eG <= bG * Ga)
    assert np.all(eb <= bb * ba)


def test_normal_equations_training_size_sampled(Q):
    """Workload 4's training set size (n = 1048573, d = 8, R = 32, K = 12),
    the same launch as training: 96 sampled entries against the oracle."""
    d, R, K, n = 8, 32, 12, 1048573
    rho, phi, y = _design_inputs(d, R, K, n, 74, i=3)
    _say(f"cv normal training size n={n}")
    G, b, acc = Q.cv_normal(rho, phi, y)
    rng = np.random.default_rng(9)
    F = R * K
    us = np.concatenate([rng.integers(0, F, 88), [0, F - 1, F - 1, 31, 32, 200, 383, 100]])
    vs = np.concatenate([rng.integers(0, F, 88), [0, F - 1, 0, 32, 31, 200, 0, 383]])
    go, ga, bo, ba = O.cv_normal_at(rho, phi, y, us, vs)
    bG = (int(acc[0]) + 16) * U32 + n * U64
    bb = (int(acc[1]) + 2) * U64 + n * U64
    eG = np.abs(G[us, vs] - go)
    eb = np.abs(b[us] - bo)
    print(f"  acc {acc.tolist()}: max |dG|/|G|abs {np.max(eG / ga):.3g} (bound {bG:.3g}), "
          f"max |db|/|b|abs {np.max(eb / ba):.3g} (bound {bb:.3g})")
    assert np.all(eG <= bG * ga)
    assert np.all(eb <= bb * ba)


@pytest.mark.parametrize("d,R,K,n", [(8, 32, 12, 16381), (10, 64, 12, 4093), (5, 8, 4, 2039), (6, 16, 8, 4093),
                                     (6, 32, 16, 8191)])
def test_solve_matches_oracle(Q, d, R, K, n):
    rho, phi, y = _design_inputs(d, R, K, n, 75)
    G, b, _, _ = O.cv_normal(rho, phi, y, threads=THREADS)
    _say(f"cv solve R={R} K={K}")
    x, lam, esc = Q.cv_solve(G, b, R, K, 1e-5)
    xo, lamo, esco = O.cv_solve(G, b, 1e-5)
    assert esc == esco == 0
    # the trace is summed in the same order on both sides
    assert lam == lamo
    F = R * K
    ev = np.linalg.eigvalsh(G + lamo * np.eye(F))
    kappa = ev[-1] / ev[0]
    rel = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    # the oracle's Cholesky solve is backward stable (|dA| <= ~3F u |L||L^T|),
    # so it lies within ~3F kappa u of the exact solution; the GPU multiplies
    # by the explicit inverse M^T M (M = L^-1 by block forward substitution
    # with the inverted diagonal blocks), whose forward error is of the same
    # order (each of M's columns a substitution, then one product): the two
    # differ by at most ~2 kappa 3F u, doubled
    bound = 12 * F * kappa * U64
    print(f"  kappa {kappa:.3g}: |x - x_oracle| / |x| = {rel:.3g} (bound {bound:.3g})")
    assert rel <= bound


def test_solve_escalation_matches_oracle(Q):
    """An indefinite matrix: the ridge is raised 100x per failed attempt on
    both sides; one that stays indefinite is reported."""
    R, K = 8, 4
    F = R * K
    rng = np.random.default_rng(3)
    M = rng.standard_normal((F, F))
    G = M @ M.T
    G[5, 5] = -0.2 * np.trace(G) / F  # negative pivot until lam > 0.2 mean diagonal
    b = rng.standard_normal(F)
    _say("cv solve escalation")
    x, lam, esc = Q.cv_solve(G, b, R, K, 1e-5)
    xo, lamo, esco = O.cv_solve(G, b, 1e-5)
    assert esc == esco and esc > 0 and lam == lamo
    assert np.allclose(x, xo, rtol=1e-9, atol=1e-12 * np.max(np.abs(xo)))
    G2 = np.diag(np.r_[np.ones(F - 1), -1e9])
    with pytest.raises(Q.QMCError) as e:
        Q.cv_solve(G2, b, R, K, 1e-5)
    assert e.value.status == Q.QMC_ENONFINITE


@pytest.mark.parametrize("d,R,K,n", [(8, 32, 12, 65521), (5, 16, 8, 16381)])
def test_als_step_reaches_ridge_minimum(Q, d, R, K, n):
    """One step with two refinements against the oracle's exact FP64 ridge
    step from the same factors: the GPU step's objective must lie within
    1e-9 of the exact minimum (relative) and below the starting value, and
    the refinements must not raise it.  Property check (the BF16 matrix is a
    preconditioner of the FP64 refinement, so there is no elementwise bound
    on W from one step); the achieved excess is printed."""
    tab, g, shift, z, jac, f = _training_set(76, d, n)
    z32, sw32 = z.astype(np.float32), jac.astype(np.float32)
    scale = float(np.mean(np.abs(f.real)))
    yw = f.real.astype(np.float32)
    y = yw.astype(np.float64) / scale
    W = _init_factors(77, R, d, K)
    for i in (0, d - 1):
        _say(f"cv als step d={d} R={R} K={K} n={n} i={i}")
        Wo, lamo = O.cv_step(z32, sw32, y, W, i, 1e-5, threads=THREADS)
        W0, lam0 = Q.cv_als_step(z32, sw32, yw, scale, W, i, 1e-5, refine=0)
        W2, lam2 = Q.cv_als_step(z32, sw32, yw, scale, W, i, 1e-5, refine=2)
        assert lam0 == lam2
        assert abs(lam2 - lamo) <= 2.0 ** -7 * lamo  # BF16 against FP64 diagonal
        Jo, sy = O.cv_objective(z32, sw32, y, Wo, i, lamo)
        Jin, _ = O.cv_objective(z32, sw32, y, W, i, lamo)
        J0, _ = O.cv_objective(z32, sw32, y, W0, i, lamo)
        J2, _ = O.cv_objective(z32, sw32, y, W2, i, lamo)
        print(f"  i={i}: J/sum y^2 start {Jin / sy:.6g}, exact {Jo / sy:.9g}, "
              f"gpu refine 0 excess {(J0 - Jo) / Jo:.3g}, refine 2 excess {(J2 - Jo) / Jo:.3g}")
        assert J2 <= Jin
        assert (J2 - Jo) <= 1e-9 * Jo
        assert J2 <= J0 * (1 + 1e-12)
        mask = np.ones(d, bool)
        mask[i] = False
        assert np.array_equal(W2[:, mask, :], W[:, mask, :])
