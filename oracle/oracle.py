"""ctypes binding of the CPU oracle (``qmc_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg.  The GPU library never imports it.

Family and transform names map to the oracle's own integer codes below; the
GPU library numbers its own codes independently.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qmc_oracle.c")
SRC_CV = os.path.join(HERE, "qmc_oracle_cvtrain.c")
# ORACLE_LIB names another build of the same sources (the sanitizer test's)
LIB = os.environ.get("ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

FAMILIES = {
    "const": 0, "trig": 1, "p2kernel": 2, "genz_product_peak": 3, "genz_oscillatory": 4,
    "genz_gaussian": 5, "genz_continuous": 6, "genz_corner_peak": 7, "sector": 8,
}
TRANSFORMS = {"none": 0, "korobov": 1, "baker": 2, "sidi": 3}


def build(force: bool = True) -> str:
    """Compile the oracle with plain gcc (no fast-math, no FP contraction);
    with ORACLE_LIB set, use that build as it is."""
    if os.environ.get("ORACLE_LIB"):
        return LIB
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", SRC, SRC_CV, "-o", LIB + ".tmp", "-lm", "-lpthread"]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


def build_sanitized(out: str) -> str:
    """The same sources with AddressSanitizer and UndefinedBehaviorSanitizer
    (clang, shared sanitizer runtime; any finding aborts), for a CPU test run
    with that runtime preloaded and ORACLE_LIB pointing at `out`."""
    cmd = ["/opt/rocm/llvm/bin/clang", "-O1", "-g", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-shared-libsan",
           "-shared", SRC, SRC_CV, "-o", out, "-lm", "-lpthread"]
    subprocess.check_call(cmd)
    return out


class _Params(C.Structure):
    _fields_ = [
        ("family", C.c_int32),
        ("c", C.c_double),
        ("n_terms", C.c_uint32),
        ("c0", C.c_double),
        ("h", C.c_void_p),
        ("ch", C.c_void_p),
        ("phi", C.c_void_p),
        ("a", C.c_void_p),
        ("u", C.c_void_p),
        ("n_u", C.c_uint32),
        ("n_f", C.c_uint32),
        ("coef_u", C.c_void_p),
        ("exp_u", C.c_void_p),
        ("coef_f", C.c_void_p),
        ("exp_f", C.c_void_p),
        ("nu", C.c_void_p),
        ("pow_u", C.c_double),
        ("pow_f", C.c_double),
        ("delta_im", C.c_double),
        ("is_complex", C.c_int32),
        ("cv_w", C.c_void_p),
        ("cv_c", C.c_void_p),
        ("cv_r", C.c_uint32),
        ("cv_k", C.c_uint32),
        ("cv_w_im", C.c_void_p),
        ("cv_c_im", C.c_void_p),
        ("eps_u", C.c_double),
        ("eps_f", C.c_double),
        ("eps_order", C.c_int32),
        ("deform_lambda", C.c_double),
        ("deform_check", C.c_int32),
        ("point_mode", C.c_int32),
        ("precise", C.c_int32),
    ]


_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = C.CDLL(LIB)
        vp, u64, u32, i32, dbl = C.c_void_p, C.c_uint64, C.c_uint32, C.c_int32, C.c_double
        L.or_lattice_index.restype = u64
        L.or_lattice_index.argtypes = [u64, u64, u64]
        L.or_lattice_indices.argtypes = [u32, u64, vp, vp, u64, vp]
        L.or_point.argtypes = [u32, u64, vp, u64, vp, i32, vp]
        L.or_transform.argtypes = [i32, i32, dbl, vp, vp]
        L.or_poly.restype = dbl
        L.or_poly.argtypes = [u32, u32, vp, vp, vp]
        L.or_legendre.argtypes = [u32, dbl, vp]
        L.or_cv_g.restype = dbl
        L.or_cv_g.argtypes = [u32, u32, u32, vp, vp, vp]
        L.or_cv_integral.restype = dbl
        L.or_cv_integral.argtypes = [u32, u32, u32, vp, vp]
        L.or_integrand.argtypes = [vp, u32, vp, vp, vp]
        L.or_fhat.argtypes = [vp, u32, i32, i32, vp, vp, vp]
        L.or_estimate.restype = C.c_int
        L.or_estimate.argtypes = [u32, u64, vp, u32, vp, i32, i32, vp, i32, vp, vp, vp]
        L.or_estimate_cond.restype = C.c_int
        L.or_estimate_cond.argtypes = [u32, u64, vp, u32, vp, i32, i32, vp, i32, vp, vp, vp, vp]
        L.or_sector_condition.restype = dbl
        L.or_sector_condition.argtypes = [vp, u32, vp]
        L.or_mean_error.argtypes = [u32, vp, vp]
        L.or_korobov_vector.argtypes = [u64, u32, u64, vp]
        L.or_p2.restype = dbl
        L.or_p2.argtypes = [u32, u64, vp, i32]
        L.or_korobov_search.restype = C.c_int
        L.or_korobov_search.argtypes = [u64, u32, vp, u32, i32, vp, vp, vp]
        L.or_cbc.restype = C.c_int
        L.or_cbc.argtypes = [u64, u32, vp, i32, vp, vp]
        L.or_cv_samples.restype = C.c_int
        L.or_cv_samples.argtypes = [u32, u64, vp, vp, i32, i32, vp, vp, vp, vp, vp]
        L.or_bf16.restype = C.c_float
        L.or_bf16.argtypes = [C.c_float]
        L.or_cv_features.restype = C.c_int
        L.or_cv_features.argtypes = [u32, u32, u32, u32, u32, vp, vp, vp, vp, vp, vp]
        L.or_cv_normal.restype = C.c_int
        L.or_cv_normal.argtypes = [u32, u32, u32, vp, vp, vp, i32, vp, vp, vp, vp]
        L.or_cv_normal_at.restype = C.c_int
        L.or_cv_normal_at.argtypes = [u32, u32, u32, vp, vp, vp, u32, vp, vp, vp, vp, vp, vp]
        L.or_cv_solve.restype = C.c_int
        L.or_cv_solve.argtypes = [u32, vp, vp, dbl, vp, vp]
        L.or_cv_step.restype = C.c_int
        L.or_cv_step.argtypes = [u32, u32, u32, u32, u32, vp, vp, vp, vp, dbl, i32, vp, vp]
        L.or_cv_objective.restype = C.c_int
        L.or_cv_objective.argtypes = [u32, u32, u32, u32, u32, vp, vp, vp, vp, dbl, vp, vp]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Params:
    """Integrand description; keeps the numpy arrays alive for the call."""

    def __init__(self, family: str, d: int, *, c: float = 1.0, a=None, u=None, trig=None,
                 sector=None, cv=None, point_mode: int = 0, eps=None, deform: float = 0.0,
                 deform_check: bool = False, precise: bool = False):
        """eps (sector): (eps_u, eps_f, k) selects the coefficient of e^k of the
        integrand with exponents pow_u + eps_u e, pow_f + eps_f e.  precise
        (plain sector): U, F, the powers and logarithms in long double."""
        self.keep = []
        p = _Params()
        p.family = FAMILIES[family]
        p.c = float(c)
        p.point_mode = int(point_mode)
        p.precise = int(bool(precise))
        if eps is not None:
            p.eps_u, p.eps_f, p.eps_order = float(eps[0]), float(eps[1]), int(eps[2])
        p.deform_lambda = float(deform)  # contour deformation of a sector (0 = none)
        p.deform_check = int(bool(deform_check))  # 1 where Im(F(z) - i delta) > 0, unweighted

        def arr(x, dt):
            v = np.ascontiguousarray(np.asarray(x, dtype=dt))
            self.keep.append(v)
            return v

        if a is not None:
            p.a = _ptr(arr(a, np.float64))
        if u is not None:
            p.u = _ptr(arr(u, np.float64))
        if trig is not None:
            c0, h, ch, phi = trig
            h = arr(h, np.int64).reshape(-1, d)
            p.n_terms = h.shape[0]
            p.c0 = float(c0)
            p.h = _ptr(h)
            p.ch = _ptr(arr(ch, np.float64))
            p.phi = _ptr(arr(phi, np.float64))
        if sector is not None:
            s = sector
            p.n_u, p.n_f = s.n_u, s.n_f
            p.coef_u = _ptr(arr(s.coef_u, np.float64))
            p.exp_u = _ptr(arr(s.exp_u, np.uint8))
            p.coef_f = _ptr(arr(s.coef_f, np.float64))
            p.exp_f = _ptr(arr(s.exp_f, np.uint8))
            p.nu = _ptr(arr(s.nu, np.uint8))
            p.pow_u, p.pow_f = float(s.pow_u), float(s.pow_f)
            p.delta_im = float(s.delta_im)
            p.is_complex = int(bool(s.is_complex))
        if cv is not None:
            # (W (R, d, K), c (R,)) for the real part; a leading axis of 2
            # adds the imaginary-part model of a complex integrand
            W, cc = cv
            W = arr(W, np.float64)
            cc = arr(cc, np.float64)
            if W.ndim == 3:
                W, cc = W[None], cc[None]
            p.cv_w = _ptr(arr(W[0], np.float64))
            p.cv_c = _ptr(arr(cc[0], np.float64))
            p.cv_r, p.cv_k = W.shape[1], W.shape[3]
            if W.shape[0] == 2:
                p.cv_w_im = _ptr(arr(W[1], np.float64))
                p.cv_c_im = _ptr(arr(cc[1], np.float64))
        self.struct = p

    @property
    def ref(self):
        return C.byref(self.struct)


def lattice_index(j: int, gi: int, n: int) -> int:
    return int(lib().or_lattice_index(j, gi, n))


def lattice_indices(n: int, g, js) -> np.ndarray:
    g = np.ascontiguousarray(np.asarray(g, dtype=np.uint64))
    js = np.ascontiguousarray(np.asarray(js, dtype=np.uint64))
    out = np.zeros((js.size, g.size), dtype=np.uint64)
    lib().or_lattice_indices(g.size, n, _ptr(g), _ptr(js), js.size, _ptr(out))
    return out


def point(n: int, g, j: int, shift, mode: int = 0) -> np.ndarray:
    g = np.ascontiguousarray(np.asarray(g, dtype=np.uint64))
    sh = np.ascontiguousarray(np.asarray(shift, dtype=np.float64))
    x = np.zeros(g.size)
    lib().or_point(g.size, n, _ptr(g), j, _ptr(sh), mode, _ptr(x))
    return x


def transform(kind: str, alpha: int, x: float):
    z, w = C.c_double(), C.c_double()
    lib().or_transform(TRANSFORMS[kind], alpha, float(x), C.byref(z), C.byref(w))
    return z.value, w.value


def poly(coef, exps, z) -> float:
    coef = np.ascontiguousarray(np.asarray(coef, dtype=np.float64))
    exps = np.ascontiguousarray(np.asarray(exps, dtype=np.uint8))
    z = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
    return float(lib().or_poly(z.size, coef.size, _ptr(coef), _ptr(exps), _ptr(z)))


def legendre(K: int, x: float) -> np.ndarray:
    out = np.zeros(K)
    lib().or_legendre(K, float(x), _ptr(out))
    return out


def cv_g(W, c, z) -> float:
    W = np.ascontiguousarray(np.asarray(W, dtype=np.float64))
    c = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
    z = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
    R, d, K = W.shape
    return float(lib().or_cv_g(d, R, K, _ptr(W), _ptr(c), _ptr(z)))


def cv_integral(W, c) -> float:
    W = np.ascontiguousarray(np.asarray(W, dtype=np.float64))
    c = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
    R, d, K = W.shape
    return float(lib().or_cv_integral(d, R, K, _ptr(W), _ptr(c)))


def integrand(params: Params, z) -> complex:
    z = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
    re, im = C.c_double(), C.c_double()
    lib().or_integrand(params.ref, z.size, _ptr(z), C.byref(re), C.byref(im))
    return complex(re.value, im.value)


def fhat(params: Params, x, tkind: str = "none", alpha: int = 0) -> complex:
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    re, im = C.c_double(), C.c_double()
    lib().or_fhat(params.ref, x.size, TRANSFORMS[tkind], alpha, _ptr(x), C.byref(re), C.byref(im))
    return complex(re.value, im.value)


class Estimate:
    def __init__(self, q_re, q_im, q_abs, status, q_cond=None):
        self.q_re, self.q_im, self.q_abs, self.status = q_re, q_im, q_abs, status
        self.q_cond = q_cond

    @property
    def q(self) -> np.ndarray:
        return self.q_re + 1j * self.q_im

    def mean_error(self):
        mr, er = mean_error(self.q_re)
        mi, ei = mean_error(self.q_im)
        return complex(mr, mi), er, ei


def estimate(n: int, g, shifts, params: Params, tkind: str = "none", alpha: int = 0,
             threads: int = 0, condition: bool = False) -> Estimate:
    """Per-shift Q_k of eq. (2) for every shift row.  condition (sectors):
    also q_cond[k] = (1/n) sum_j |fhat_j| c_j, c_j the sector's rounding
    condition at the point (sector_condition)."""
    g = np.ascontiguousarray(np.asarray(g, dtype=np.uint64))
    sh = np.ascontiguousarray(np.asarray(shifts, dtype=np.float64))
    m, d = sh.shape
    assert d == g.size
    if threads <= 0:
        threads = os.cpu_count() or 1
    q_re, q_im, q_abs = np.zeros(m), np.zeros(m), np.zeros(m)
    q_cond = np.zeros(m) if condition else None
    st = lib().or_estimate_cond(d, n, _ptr(g), m, _ptr(sh), TRANSFORMS[tkind], alpha, params.ref,
                                threads, _ptr(q_re), _ptr(q_im), _ptr(q_abs), _ptr(q_cond))
    return Estimate(q_re, q_im, q_abs, st, q_cond)


def sector_condition(params: Params, z) -> float:
    """|pU| S_U / |U| + |pF| S_F / |F - i delta| at z (S: sums of the terms'
    magnitudes): the relative change of the sector's value per unit
    roundoff in the terms of U and F."""
    z = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
    return float(lib().or_sector_condition(params.ref, z.size, _ptr(z)))


def mean_error(q) -> tuple:
    q = np.ascontiguousarray(np.asarray(q, dtype=np.float64))
    out = np.zeros(2)
    lib().or_mean_error(q.size, _ptr(q), _ptr(out))
    return float(out[0]), float(out[1])


def korobov_vector(n: int, d: int, a: int) -> np.ndarray:
    g = np.zeros(d, dtype=np.uint64)
    lib().or_korobov_vector(n, d, a, _ptr(g))
    return g


def p2(n: int, g, threads: int = 0) -> float:
    g = np.ascontiguousarray(np.asarray(g, dtype=np.uint64))
    if threads <= 0:
        threads = os.cpu_count() or 1
    return float(lib().or_p2(g.size, n, _ptr(g), threads))


def korobov_search(n: int, d: int, cand, threads: int = 0):
    cand = np.ascontiguousarray(np.asarray(cand, dtype=np.uint64))
    if threads <= 0:
        threads = os.cpu_count() or 1
    a = C.c_uint64()
    pb = C.c_double()
    allp = np.zeros(cand.size)
    st = lib().or_korobov_search(n, d, _ptr(cand), cand.size, threads, C.byref(a), C.byref(pb),
                                 _ptr(allp))
    if st != 0:
        raise ValueError("bad korobov search arguments")
    return int(a.value), float(pb.value), allp


def cbc(n: int, d: int, gamma=None, threads: int = 0):
    """Component-by-component generating vector: (z (d,), e2 (d,)), e2[s] the
    squared worst-case error after component s."""
    gamma = np.ones(d) if gamma is None else np.ascontiguousarray(np.asarray(gamma, dtype=np.float64))
    if threads <= 0:
        threads = os.cpu_count() or 1
    z = np.zeros(d, dtype=np.uint64)
    e2 = np.zeros(d)
    if lib().or_cbc(n, d, _ptr(gamma), threads, _ptr(z), _ptr(e2)) != 0:
        raise ValueError("bad cbc arguments")
    return z, e2



# --------------------------------------------------------------- control-variate training
def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def cv_samples(n: int, g, shift, params: Params, tkind: str = "none", alpha: int = 0):
    """(z (n, d), J (n,), fhat (n,) complex) at the points {j g / n + shift}."""
    g = np.ascontiguousarray(np.asarray(g, dtype=np.uint64))
    sh = _f64(shift)
    d = g.size
    z, jac, fr, fi = np.zeros((n, d)), np.zeros(n), np.zeros(n), np.zeros(n)
    if lib().or_cv_samples(d, n, _ptr(g), _ptr(sh), TRANSFORMS[tkind], alpha, params.ref, _ptr(z), _ptr(jac),
                           _ptr(fr), _ptr(fi)):
        raise ValueError("bad cv_samples arguments")
    return z, jac, fr + 1j * fi


def bf16(x: float) -> float:
    """x rounded to bfloat16 (nearest, ties to even), as a float."""
    return float(lib().or_bf16(float(x)))


def cv_features(z, sw, W, i: int):
    """(rho (n, R), phi (n, K), env (n, R)) of the least-squares step for
    dimension i, in double; z (n, d) and sw (n,) single precision."""
    z, sw, W = _f32(z), _f32(sw), _f64(W)
    n, d = z.shape
    R, _, K = W.shape
    rho, phi, env = np.zeros((n, R)), np.zeros((n, K)), np.zeros((n, R))
    if lib().or_cv_features(n, d, R, K, i, _ptr(z), _ptr(sw), _ptr(W), _ptr(rho), _ptr(phi), _ptr(env)):
        raise ValueError("bad cv_features arguments")
    return rho, phi, env


def cv_normal(rho, phi, y, threads: int = 0):
    """Normal equations as the GPU assembles them from double rho, phi, y
    (bfloat16 matrix of the single-precision factors, double right-hand
    side), summed in long double: (G, b, |G|, |b|), rows and columns
    u = r K + k."""
    rho, phi, y = _f64(rho), _f64(phi), _f64(y)
    n, R = rho.shape
    K = phi.shape[1]
    F = R * K
    if threads <= 0:
        threads = os.cpu_count() or 1
    G, Ga, b, ba = np.zeros((F, F)), np.zeros((F, F)), np.zeros(F), np.zeros(F)
    if lib().or_cv_normal(n, R, K, _ptr(rho), _ptr(phi), _ptr(y), threads, _ptr(G), _ptr(b), _ptr(Ga),
                          _ptr(ba)):
        raise ValueError("bad cv_normal arguments")
    return G, b, Ga, ba


def cv_normal_at(rho, phi, y, us, vs):
    """Entries G[us, vs] and b[us] with their envelopes (sampled form)."""
    rho, phi, y = _f64(rho), _f64(phi), _f64(y)
    us = np.ascontiguousarray(np.asarray(us, dtype=np.uint32))
    vs = np.ascontiguousarray(np.asarray(vs, dtype=np.uint32))
    n, R = rho.shape
    K = phi.shape[1]
    c = us.size
    G, Ga, b, ba = np.zeros(c), np.zeros(c), np.zeros(c), np.zeros(c)
    if lib().or_cv_normal_at(n, R, K, _ptr(rho), _ptr(phi), _ptr(y), c, _ptr(us), _ptr(vs), _ptr(G), _ptr(Ga),
                             _ptr(b), _ptr(ba)):
        raise ValueError("bad cv_normal_at arguments")
    return G, Ga, b, ba


def cv_solve(G, b, ridge: float):
    """(x, lam, escalations) of (G + lam I) x = b, lam = ridge trace(G) / F
    (escalated 100x per non-positive pivot); escalations = -1 if it fails."""
    G, b = _f64(G), _f64(b)
    F = b.size
    x = np.zeros(F)
    lam = C.c_double()
    esc = lib().or_cv_solve(F, _ptr(G), _ptr(b), float(ridge), C.byref(lam), _ptr(x))
    return x, lam.value, int(esc)


def cv_step(z, sw, y, W, i: int, ridge: float, threads: int = 0):
    """One exact ridge least-squares step for dimension i: (W_new, lam);
    y (n,) the double target."""
    z, sw, y, W = _f32(z), _f32(sw), _f64(y), _f64(W)
    n, d = z.shape
    R, _, K = W.shape
    if threads <= 0:
        threads = os.cpu_count() or 1
    out = np.zeros_like(W)
    lam = C.c_double()
    st = lib().or_cv_step(n, d, R, K, i, _ptr(z), _ptr(sw), _ptr(y), _ptr(W), float(ridge), threads, _ptr(out),
                          C.byref(lam))
    if st:
        raise ValueError(f"cv_step failed ({st})")
    return out, lam.value


def cv_objective(z, sw, y, W, i: int, lam: float):
    """(J, sum y^2): J = sum_j (y_j - sw_j g(z_j))^2 + lam |W[., i, .]|^2, c = 1."""
    z, sw, y, W = _f32(z), _f32(sw), _f64(y), _f64(W)
    n, d = z.shape
    R, _, K = W.shape
    J, sy = C.c_double(), C.c_double()
    if lib().or_cv_objective(n, d, R, K, i, _ptr(z), _ptr(sw), _ptr(y), _ptr(W), float(lam), C.byref(J),
                             C.byref(sy)):
        raise ValueError("bad cv_objective arguments")
    return J.value, sy.value
