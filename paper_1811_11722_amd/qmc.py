"""Thin ctypes binding of libqmc.so (declarations in include/qmc.h).

Argument marshalling only: every step of the estimator runs in the HIP
library.  Importing this module loads the library and raises if it has not
been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# QMC_LIB names another build of the library (the host-sanitizer test's)
LIB_PATH = os.environ.get("QMC_LIB") or os.path.join(HERE, "libqmc.so")

# status codes
QMC_OK, QMC_EINVAL, QMC_EUNSUPPORTED, QMC_ENOMEM, QMC_EDEVICE, QMC_ENONFINITE, QMC_ECONTOUR = range(7)
# transforms
QMC_T_NONE, QMC_T_KOROBOV, QMC_T_BAKER, QMC_T_SIDI = 0, 1, 2, 3
QMC_T_TENT = QMC_T_BAKER
# families
(QMC_F_CONST, QMC_F_TRIG, QMC_F_P2KERNEL, QMC_F_GENZ_PRODUCT_PEAK, QMC_F_GENZ_OSCILLATORY,
 QMC_F_GENZ_GAUSSIAN, QMC_F_GENZ_CONTINUOUS, QMC_F_GENZ_CORNER_PEAK, QMC_F_SECTOR) = range(9)

FAMILY = {
    "const": QMC_F_CONST, "trig": QMC_F_TRIG, "p2kernel": QMC_F_P2KERNEL,
    "genz_product_peak": QMC_F_GENZ_PRODUCT_PEAK, "genz_oscillatory": QMC_F_GENZ_OSCILLATORY,
    "genz_gaussian": QMC_F_GENZ_GAUSSIAN, "genz_continuous": QMC_F_GENZ_CONTINUOUS,
    "genz_corner_peak": QMC_F_GENZ_CORNER_PEAK, "sector": QMC_F_SECTOR,
}
TRANSFORM = {"none": QMC_T_NONE, "korobov": QMC_T_KOROBOV, "baker": QMC_T_BAKER,
             "tent": QMC_T_TENT, "sidi": QMC_T_SIDI}


class qmc_transform(C.Structure):
    _fields_ = [("kind", C.c_int32), ("alpha", C.c_int32)]


class qmc_const_params(C.Structure):
    _fields_ = [("c", C.c_double)]


class qmc_trig_params(C.Structure):
    _fields_ = [("n_terms", C.c_uint32), ("c0", C.c_double), ("h", C.c_void_p),
                ("c", C.c_void_p), ("phi", C.c_void_p)]


class qmc_genz_params(C.Structure):
    _fields_ = [("a", C.c_void_p), ("u", C.c_void_p)]


class qmc_sector_params(C.Structure):
    _fields_ = [("n_u", C.c_uint32), ("n_f", C.c_uint32), ("coef_u", C.c_void_p),
                ("exp_u", C.c_void_p), ("coef_f", C.c_void_p), ("exp_f", C.c_void_p),
                ("nu", C.c_void_p), ("pow_u", C.c_double), ("pow_f", C.c_double),
                ("delta_im", C.c_double), ("is_complex", C.c_int32), ("n_orders", C.c_uint32),
                ("eps_u", C.c_double), ("eps_f", C.c_double), ("deform_lambda", C.c_double)]


class qmc_result(C.Structure):
    _fields_ = [("mean_re", C.c_double), ("mean_im", C.c_double), ("err_re", C.c_double),
                ("err_im", C.c_double), ("is_complex", C.c_int32), ("used_cv", C.c_int32),
                ("contour_crossed", C.c_double)]


class qmc_cv_train_opts(C.Structure):
    _fields_ = [("max_sweeps", C.c_uint32), ("ridge", C.c_double), ("tol", C.c_double),
                ("seed", C.c_uint64), ("refine", C.c_uint32)]


class qmc_cv_train_report(C.Structure):
    _fields_ = [("sweeps", C.c_uint32), ("rel_loss", C.c_double), ("scale", C.c_double),
                ("seconds", C.c_double)]


class qmc_launch(C.Structure):
    _fields_ = [("shift_tile", C.c_uint32), ("blocks_per_cu", C.c_uint32)]


class qmc_batch_opts(C.Structure):
    _fields_ = [("use_graph", C.c_int32), ("per_plan_launches", C.c_int32),
                ("tile_points", C.c_uint32), ("schedule", C.c_int32)]


BATCH_SCHEDULE = {"default": 0, "persistent": 1, "per_tile": 2, "specialised": 3}


# every symbol include/qmc.h declares, with its ctypes signature
_vp, _u32, _u64, _i32, _dbl = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int32, C.c_double
SIGNATURES = {
    "qmc_plan_create": (C.c_int, [_u32, _u64, _vp, _u32, _vp, qmc_transform, _vp]),
    "qmc_plan_set_stream": (C.c_int, [_vp, _vp]),
    "qmc_plan_set_launch": (C.c_int, [_vp, _vp]),
    "qmc_integrate": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "qmc_plan_set_jit": (C.c_int, [_vp, _i32]),
    "qmc_plan_get_launch": (C.c_int, [_vp, _vp, _vp]),
    "qmc_plan_set_timing": (C.c_int, [_vp, _i32]),
    "qmc_plan_kernel_time": (C.c_int, [_vp, _vp, _vp, _i32]),
    "qmc_lattice_dump": (C.c_int, [_vp, _u64, _u64, _vp, _vp]),
    "qmc_korobov_vector": (C.c_int, [_u64, _u32, _u64, _vp]),
    "qmc_korobov_search": (C.c_int, [_u64, _u32, _vp, _u32, _vp, _vp, _vp]),
    "qmc_integrate_batch": (C.c_int, [_u32, _vp, C.c_int, _vp, _vp, _vp]),
    "qmc_batch_autotune": (C.c_int, [_u32, _vp, C.c_int, _vp, _vp, _vp]),
    "qmc_autotune": (C.c_int, [_vp, C.c_int, _vp, _vp]),
    "qmc_batch_per_shift": (C.c_int, [_u32, _vp, _vp]),
    "qmc_batch_stats": (C.c_int, [_vp]),
    "qmc_math_eval": (C.c_int, [_i32, _u64, _vp, _vp]),
    "qmc_cv_train": (C.c_int, [_vp, C.c_int, _vp, _u32, _u32, _vp, _vp, _vp, _vp]),
    "qmc_cv_integral": (C.c_int, [_u32, _u32, _u32, _vp, _vp, _vp]),
    "qmc_integrate_cv": (C.c_int, [_vp, C.c_int, _vp, _u32, _u32, _vp, _vp, _vp, _vp, _vp]),
    "qmc_integrate_orders": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "qmc_deform_check": (C.c_int, [_vp, _vp, _vp, _vp]),
    "qmc_integrate_sum": (C.c_int, [_vp, C.c_uint32, _vp, _vp, _vp]),
    "qmc_cbc_search": (C.c_int, [C.c_uint64, C.c_uint32, _vp, _vp, C.c_uint32, _vp, _vp]),
    "qmc_korobov_search_extensible": (C.c_int, [C.c_uint32, C.c_uint32, C.c_uint32, _vp, C.c_uint32, _vp, _vp,
                                                _vp]),
    "qmc_lattice_merge": (C.c_int, [C.c_uint32, C.c_uint32, _vp, _vp, _vp, _vp]),
    "qmc_lattice_moved_shifts": (C.c_int, [_u64, _u32, _vp, _u32, _vp, _vp]),
    "qmc_deform_select": (C.c_int, [_vp, _vp, C.c_double, C.c_double, C.c_uint32, _vp, _vp]),
    "qmc_cv_samples": (C.c_int, [_vp, C.c_int, _vp, _u32, _vp, _vp, _vp]),
    "qmc_cv_features": (C.c_int, [_u32, _u32, _u32, _u32, _u32, _vp, _vp, _vp, _vp, _vp]),
    "qmc_cv_normal": (C.c_int, [_u32, _u32, _u32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "qmc_cv_solve": (C.c_int, [_u32, _u32, _vp, _vp, _dbl, _vp, _vp, _vp]),
    "qmc_cv_als_step": (C.c_int, [_u32, _u32, _u32, _u32, _u32, _vp, _vp, _vp, _dbl, _vp, _dbl, _u32, _vp,
                                  _vp]),
    "qmc_integrate_static": (C.c_int, [_u32, _u64, _vp, _u32, _vp, qmc_transform, C.c_int, _vp, _vp, _vp, _vp]),
    "qmc_plan_destroy": (None, [_vp]),
    "qmc_status_string": (C.c_char_p, [C.c_int]),
    "qmc_last_error": (C.c_char_p, []),
}

_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1811_11722_amd.build` (no CPU fallback exists)")
        # PyTorch ships its own HIP runtime under the same soname as the system
        # one, and a process holds only the first one loaded.  Loading torch
        # first makes the library share torch's runtime, so torch streams can
        # be handed to it and torch keeps working in the same process.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class QMCError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib().qmc_last_error().decode(errors="replace")
        name = lib().qmc_status_string(status).decode()
        super().__init__(f"{where}: {name} ({status}): {msg}")


def check(status: int, where: str):
    if status != QMC_OK:
        raise QMCError(status, where)


def _arr(x, dt):
    return np.ascontiguousarray(np.asarray(x, dtype=dt))


def _p(a: np.ndarray):
    # the buffer's address as an int (what a c_void_p argument takes);
    # half the cost of a ctypes pointer object per call
    return a.ctypes.data


class Params:
    """Family parameter struct plus the arrays it points into."""

    def __init__(self, family: str, d: int, *, c: float = 1.0, a=None, u=None, trig=None,
                 sector=None, orders=None, deform: float = 0.0):
        """orders (sector only): (n_orders, eps_u, eps_f) for qmc_integrate_orders.
        deform (sector only): contour-deformation parameter lambda (0 = none);
        a deformed sector's result is complex."""
        self.family = FAMILY[family]
        self.n_orders = 0
        self.keep = []

        def keep(x, dt):
            v = _arr(x, dt)
            self.keep.append(v)
            return v

        if self.family == QMC_F_CONST:
            self.struct = qmc_const_params(float(c))
        elif self.family == QMC_F_TRIG:
            c0, h, ch, phi = trig
            h = keep(h, np.int64).reshape(-1, d)
            self.struct = qmc_trig_params(h.shape[0], float(c0), _p(h), _p(keep(ch, np.float64)),
                                          _p(keep(phi, np.float64)))
        elif self.family == QMC_F_P2KERNEL:
            self.struct = None
        elif self.family == QMC_F_SECTOR:
            s = sector
            self.struct = qmc_sector_params(
                s.n_u, s.n_f, _p(keep(s.coef_u, np.float64)), _p(keep(s.exp_u, np.uint8)),
                _p(keep(s.coef_f, np.float64)), _p(keep(s.exp_f, np.uint8)),
                _p(keep(s.nu, np.uint8)), float(s.pow_u), float(s.pow_f), float(s.delta_im),
                int(bool(s.is_complex)), int(orders[0]) if orders else 0,
                float(orders[1]) if orders else 0.0, float(orders[2]) if orders else 0.0,
                float(deform))
            self.n_orders = int(orders[0]) if orders else 0
        else:
            self.struct = qmc_genz_params(_p(keep(a, np.float64)), _p(keep(u, np.float64)))
        # the struct's address, formed once: a batch passes hundreds of these
        # per call, and a ctypes cast per parameter block cost about 1 us each
        self._addr = None if self.struct is None else C.addressof(self.struct)

    @property
    def ptr(self):
        return self._addr

    @property
    def is_complex(self) -> bool:
        return self.family == QMC_F_SECTOR and (bool(self.struct.is_complex)
                                                or self.struct.deform_lambda != 0.0)


class Plan:
    """Owner of a qmc_plan_t."""

    def __init__(self, d: int, n: int, g: Sequence[int], shifts, transform: str = "none",
                 alpha: int = 0):
        g = _arr(g, np.uint64)
        sh = _arr(shifts, np.float64)
        self.d, self.n, self.m = int(d), int(n), int(sh.shape[0])
        self.handle = C.c_void_p()
        check(lib().qmc_plan_create(self.d, self.n, _p(g), self.m, _p(sh),
                                    qmc_transform(TRANSFORM[transform], alpha),
                                    C.byref(self.handle)), "qmc_plan_create")

    def close(self):
        if self.handle:
            lib().qmc_plan_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream_handle: int):
        check(lib().qmc_plan_set_stream(self.handle, C.c_void_p(stream_handle)), "set_stream")

    def set_launch(self, shift_tile: int = 0, blocks_per_cu: int = 0):
        cfg = qmc_launch(shift_tile, blocks_per_cu)
        check(lib().qmc_plan_set_launch(self.handle, C.byref(cfg)), "set_launch")

    def set_jit(self, mode: int):
        """0 tables, 1 specialise when possible (default), 2 always specialise."""
        check(lib().qmc_plan_set_jit(self.handle, int(mode)), "set_jit")

    def last_launch(self):
        cfg, used = qmc_launch(), C.c_int32()
        check(lib().qmc_plan_get_launch(self.handle, C.byref(cfg), C.byref(used)), "get_launch")
        return cfg.shift_tile, cfg.blocks_per_cu, bool(used.value)

    def set_timing(self, on: bool = True):
        check(lib().qmc_plan_set_timing(self.handle, int(on)), "set_timing")

    def kernel_time(self, reset: bool = False):
        ms, cnt = C.c_double(), C.c_uint64()
        check(lib().qmc_plan_kernel_time(self.handle, C.byref(ms), C.byref(cnt), int(reset)),
              "kernel_time")
        return ms.value, cnt.value

    def integrate(self, params: Params, allow_crossing: bool = False):
        """Returns (qmc_result, per-shift array: real (m,) or complex (m,)).
        A deformed contour that crosses the cut raises QMCError (ECONTOUR)
        unless allow_crossing, which returns the result with
        res.contour_crossed > 0."""
        res = qmc_result()
        per = np.zeros(2 * self.m)
        st = lib().qmc_integrate(self.handle, params.family, params.ptr, C.byref(res), _p(per))
        if not (allow_crossing and st == QMC_ECONTOUR):
            check(st, "qmc_integrate")
        if res.is_complex:
            return res, per[0::2] + 1j * per[1::2]
        return res, per[: self.m].copy()

    def integrate_status(self, params: Params):
        """Like integrate but returns (status, result, per_shift) without raising."""
        res = qmc_result()
        per = np.zeros(2 * self.m)
        st = lib().qmc_integrate(self.handle, params.family, params.ptr, C.byref(res), _p(per))
        return st, res, per

    def cv_train(self, params: Params, R: int, K: int, max_sweeps: int = 0, ridge: float = 0.0,
                 tol: float = 1e-4, seed: int = 1, refine: int = 0):
        """Fit the Legendre control variate on this plan's lattice (first shift).
        Returns (W, c, report): W (R, d, K) and c (R,) for a real integrand,
        W (2, R, d, K) and c (2, R) (real-part model, imaginary-part model)
        for a complex one."""
        nm = 2 if params.is_complex else 1
        W = np.zeros((nm, R, self.d, K))
        c = np.zeros((nm, R))
        opts = qmc_cv_train_opts(max_sweeps, ridge, tol, seed, refine)
        rep = qmc_cv_train_report()
        check(lib().qmc_cv_train(self.handle, params.family, params.ptr, R, K, C.byref(opts), _p(W),
                                 _p(c), C.byref(rep)), "qmc_cv_train")
        if nm == 1:
            return W[0], c[0], rep
        return W, c, rep

    def cv_samples(self, params: Params, part: int = 0):
        """Training samples of this plan's lattice with its first shift:
        (z (n, d), sw (n,), yw (n,)) in single precision."""
        z = np.zeros((self.n, self.d), np.float32)
        sw = np.zeros(self.n, np.float32)
        yw = np.zeros(self.n, np.float32)
        check(lib().qmc_cv_samples(self.handle, params.family, params.ptr, part, _p(z), _p(sw), _p(yw)),
              "qmc_cv_samples")
        return z, sw, yw

    def integrate_cv(self, params: Params, W, c):
        """Returns (result, plain result, plain per-shift Q_k, residual
        per-shift Q_k); complex integrands give complex Q_k arrays."""
        W = _arr(W, np.float64)
        c = _arr(c, np.float64)
        nm = 2 if params.is_complex else 1
        if W.ndim == 3:
            W = W[None]
            c = c.reshape(1, -1)
        if W.shape[0] != nm or c.shape != (nm, W.shape[1]):
            raise ValueError("W must be (R, d, K) for a real integrand and (2, R, d, K) for a complex one")
        _, R, d, K = W.shape
        out, plain = qmc_result(), qmc_result()
        per = np.zeros(2 * nm * self.m)
        check(lib().qmc_integrate_cv(self.handle, params.family, params.ptr, R, K, _p(W), _p(c),
                                     C.byref(out), C.byref(plain), _p(per)), "qmc_integrate_cv")
        if nm == 1:
            return out, plain, per[0::2].copy(), per[1::2].copy()
        per = per.reshape(self.m, 4)
        return out, plain, per[:, 0] + 1j * per[:, 1], per[:, 2] + 1j * per[:, 3]

    def integrate_orders(self, params: Params, allow_crossing: bool = False):
        """Expansion coefficients in one pass: (list of n_orders results,
        per-shift array (m, n_orders), complex for complex sectors);
        allow_crossing as in integrate."""
        no = max(params.n_orders, 1)
        out = (qmc_result * no)()
        parts = no * (2 if params.is_complex else 1)
        per = np.zeros(self.m * parts)
        st = lib().qmc_integrate_orders(self.handle, params.family, params.ptr, out, _p(per))
        if not (allow_crossing and st == QMC_ECONTOUR):
            check(st, "qmc_integrate_orders")
        per = per.reshape(self.m, parts)
        if params.is_complex:
            per = per[:, 0::2] + 1j * per[:, 1::2]
        return list(out), per

    def integrate_sum(self, params: Sequence[Params]):
        """The sum of several sector integrals in one pass: (result, per-shift
        array (m,), complex for complex sectors)."""
        ptrs = (C.c_void_p * len(params))(*[pa.ptr for pa in params])
        res = qmc_result()
        per = np.zeros(2 * self.m)
        check(lib().qmc_integrate_sum(self.handle, len(params), ptrs, C.byref(res), _p(per)), "qmc_integrate_sum")
        if res.is_complex:
            return res, per[0::2] + 1j * per[1::2]
        return res, per[: self.m].copy()

    def deform_check(self, params: Params):
        """Fraction of lattice points where the deformed F - i delta has a
        positive imaginary part: (overall, per-shift array (m,))."""
        frac = C.c_double()
        per = np.zeros(self.m)
        check(lib().qmc_deform_check(self.handle, params.ptr, C.byref(frac), _p(per)), "qmc_deform_check")
        return frac.value, per

    def deform_select(self, params: Params, lam_max: float = 1.0, shrink: float = 0.5, count: int = 10):
        """(lambda, result): the ladder lam_max * shrink^i lambda with no sign
        violation and the smallest estimated error on this plan."""
        lam = C.c_double()
        res = qmc_result()
        check(lib().qmc_deform_select(self.handle, params.ptr, float(lam_max), float(shrink), int(count),
                                      C.byref(lam), C.byref(res)), "qmc_deform_select")
        return lam.value, res

    def lattice_dump(self, j_lo: int, count: int):
        idx = np.zeros((count, self.d), dtype=np.uint32)
        sums = np.zeros(2 * self.d, dtype=np.uint64)
        check(lib().qmc_lattice_dump(self.handle, j_lo, count, _p(idx), _p(sums)), "lattice_dump")
        return idx, sums.reshape(self.d, 2)

    def autotune(self, params: Params):
        best = qmc_launch()
        check(lib().qmc_autotune(self.handle, params.family, params.ptr, C.byref(best)),
              "qmc_autotune")
        return best.shift_tile, best.blocks_per_cu


def math_eval(fn: str, x, x2=None) -> np.ndarray:
    """Device math on arrays: 'log', 'exp', 'atan2' (math_eval('atan2', y, x))
    or 'sincos' (returns an (n, 2) array of sin, cos)."""
    code = {"log": 0, "exp": 1, "atan2": 2, "sincos": 3}[fn]
    x = _arr(x, np.float64)
    n = x.size
    if code == 2:
        x = _arr(np.stack([x, _arr(x2, np.float64)], axis=-1), np.float64)
    y = np.zeros((n, 2) if code == 3 else n)
    check(lib().qmc_math_eval(code, n, _p(x), _p(y)), "qmc_math_eval")
    return y


def cv_integral(W, c) -> float:
    W = _arr(W, np.float64)
    c = _arr(c, np.float64)
    R, d, K = W.shape
    out = C.c_double()
    check(lib().qmc_cv_integral(R, d, K, _p(W), _p(c), C.byref(out)), "qmc_cv_integral")
    return out.value


def integrate_static(d: int, n: int, g, shifts, params: "Params", transform: str = "none", alpha: int = 0,
                     stream: int = 0, status_only: bool = False):
    """One estimate through qmc_integrate_static (no device allocation):
    (result, per-shift Q_k), complex Q_k for complex sectors.  With
    status_only the status is returned in front instead of raised."""
    g = _arr(g, np.uint64)
    sh = _arr(shifts, np.float64)
    m = int(sh.shape[0])
    res = qmc_result()
    per = np.zeros(2 * m)
    st = lib().qmc_integrate_static(int(d), int(n), _p(g), m, _p(sh), qmc_transform(TRANSFORM[transform], alpha),
                                    params.family, params.ptr, C.c_void_p(stream), C.byref(res), _p(per))
    if status_only:
        return st, res, per
    check(st, "qmc_integrate_static")
    if res.is_complex:
        return res, per[0::2] + 1j * per[1::2]
    return res, per[:m].copy()


def cv_features(z, sw, W, i: int):
    """(rho (n, R), phi (n, K)) in FP64 of the training step for dimension i."""
    z, sw, W = _arr(z, np.float32), _arr(sw, np.float32), _arr(W, np.float64)
    n, d = z.shape
    R, _, K = W.shape
    rho = np.zeros((n, R))
    phi = np.zeros((n, K))
    check(lib().qmc_cv_features(n, d, R, K, i, _p(z), _p(sw), _p(W), _p(rho), _p(phi)), "qmc_cv_features")
    return rho, phi


def cv_normal(rho, phi, y):
    """(G (F, F), b (F,), acc_len (2,)) of the BF16 normal matrix and the
    FP64 right-hand side, u = r K + k."""
    rho, phi, y = _arr(rho, np.float64), _arr(phi, np.float64), _arr(y, np.float64)
    n, R = rho.shape
    K = phi.shape[1]
    G = np.zeros((R * K, R * K))
    b = np.zeros(R * K)
    acc = np.zeros(2, np.uint32)
    check(lib().qmc_cv_normal(n, R, K, _p(rho), _p(phi), _p(y), _p(G), _p(b), _p(acc)), "qmc_cv_normal")
    return G, b, acc


def cv_solve(G, b, R: int, K: int, ridge: float):
    """(x, lam, escalations) of (G + lam I) x = b on the device."""
    G, b = _arr(G, np.float64), _arr(b, np.float64)
    x = np.zeros(R * K)
    lam = C.c_double()
    esc = C.c_int32()
    check(lib().qmc_cv_solve(R, K, _p(G), _p(b), float(ridge), C.byref(lam), _p(x), C.byref(esc)), "qmc_cv_solve")
    return x, lam.value, esc.value


def cv_als_step(z, sw, yw, scale: float, W, i: int, ridge: float, refine: int = 2):
    """One training step for dimension i: (W_new, lam)."""
    z, sw, yw, W = _arr(z, np.float32), _arr(sw, np.float32), _arr(yw, np.float32), _arr(W, np.float64)
    n, d = z.shape
    R, _, K = W.shape
    out = np.zeros_like(W)
    lam = C.c_double()
    check(lib().qmc_cv_als_step(n, d, R, K, i, _p(z), _p(sw), _p(yw), float(scale), _p(W), float(ridge), refine,
                                _p(out), C.byref(lam)), "qmc_cv_als_step")
    return out, lam.value


def korobov_vector(n: int, d: int, a: int) -> np.ndarray:
    g = np.zeros(d, dtype=np.uint64)
    check(lib().qmc_korobov_vector(n, d, a, _p(g)), "qmc_korobov_vector")
    return g


def korobov_search(n: int, d: int, cand):
    cand = _arr(cand, np.uint64)
    a = C.c_uint64()
    p2 = C.c_double()
    allp = np.zeros(cand.size)
    check(lib().qmc_korobov_search(n, d, _p(cand), cand.size, C.byref(a), C.byref(p2), _p(allp)),
          "qmc_korobov_search")
    return int(a.value), float(p2.value), allp


def integrate_batch(plans: Sequence[Plan], params: Sequence[Params], use_graph: bool = True,
                    per_plan_launches: bool = False, tile_points: int = 0, schedule: str = "default",
                    allow_crossing: bool = False):
    """schedule: "default", "persistent" (workgroups loop over the work list),
    "per_tile" (one workgroup per tile) or "specialised" (sectors: one launch
    per plan of its run-time specialised kernel, compiled once per exponent
    structure); allow_crossing as in Plan.integrate."""
    fam = params[0].family
    handles = (C.c_void_p * len(plans))(*[p.handle for p in plans])
    pp = (C.c_void_p * len(params))(*[p.ptr for p in params])
    opts = qmc_batch_opts(int(use_graph), int(per_plan_launches), tile_points, BATCH_SCHEDULE[schedule])
    out = (qmc_result * len(plans))()
    st = lib().qmc_integrate_batch(len(plans), handles, fam, pp, C.byref(opts), out)
    if not (allow_crossing and st == QMC_ECONTOUR):
        check(st, "qmc_integrate_batch")
    return list(out)


def batch_autotune(plans: Sequence[Plan], params: Sequence[Params]):
    """Fastest table-driven batch options by timing: (dict of
    integrate_batch keyword arguments, milliseconds)."""
    fam = params[0].family
    handles = (C.c_void_p * len(plans))(*[p.handle for p in plans])
    pp = (C.c_void_p * len(params))(*[p.ptr for p in params])
    best = qmc_batch_opts()
    ms = C.c_double()
    check(lib().qmc_batch_autotune(len(plans), handles, fam, pp, C.byref(best), C.byref(ms)), "qmc_batch_autotune")
    sched = {v: k for k, v in BATCH_SCHEDULE.items()}[best.schedule]
    return {"use_graph": bool(best.use_graph), "tile_points": best.tile_points, "schedule": sched}, ms.value


def batch_per_shift(plans: Sequence[Plan], complex_parts: bool = False):
    """Per-shift Q_k of the last graph/persistent batch run over these plans."""
    handles = (C.c_void_p * len(plans))(*[p.handle for p in plans])
    bufs = [np.zeros(p.m * (2 if complex_parts else 1)) for p in plans]
    ptrs = (C.c_void_p * len(plans))(*[_p(b) for b in bufs])
    check(lib().qmc_batch_per_shift(len(plans), handles, ptrs), "qmc_batch_per_shift")
    if complex_parts:
        return [b[0::2] + 1j * b[1::2] for b in bufs]
    return bufs


def batch_stats() -> dict:
    """Counters of the batch machinery since the library was loaded."""
    out = np.zeros(4, dtype=np.uint64)
    check(lib().qmc_batch_stats(_p(out)), "qmc_batch_stats")
    return {"contexts_built": int(out[0]), "graph_launches": int(out[1]),
            "specialised_captures": int(out[2]), "specialised_launches": int(out[3])}


def cbc_search(n: int, d: int, gamma=None, cand=None):
    """Component-by-component generating vector on the GPU: (z (d,) uint64,
    e2 (d,) squared worst-case error after each component)."""
    g = None if gamma is None else _arr(gamma, np.float64)
    c = None if cand is None else _arr(cand, np.uint64)
    z = np.zeros(d, dtype=np.uint64)
    e2 = np.zeros(d)
    check(lib().qmc_cbc_search(int(n), int(d), None if g is None else _p(g), None if c is None else _p(c),
                               0 if c is None else c.size, _p(z), _p(e2)), "qmc_cbc_search")
    return z, e2


def korobov_search_extensible(kmin: int, kmax: int, d: int, cand):
    """(a, mean log P2 over the rungs, P2 per rung) for odd candidates a."""
    cand = _arr(cand, np.uint64)
    a = C.c_uint64()
    score = C.c_double()
    p2 = np.zeros(kmax - kmin + 1)
    check(lib().qmc_korobov_search_extensible(kmin, kmax, d, _p(cand), cand.size, C.byref(a), C.byref(score),
                                              _p(p2)), "qmc_korobov_search_extensible")
    return int(a.value), float(score.value), p2


class ExtensibleLattice:
    """Embedded rank-1 lattices of 2^k points, g = (1, a, a^2, ...) mod 2^kmax,
    with fixed shifts.  ladder() integrates the rungs 2^kmin .. 2^kmax and
    evaluates each lattice point once: rung k + 1 adds the 2^k-point lattice
    with the shifts moved by (g mod 2^(k+1)) / 2^(k+1) and merges."""

    def __init__(self, d: int, a: int, kmax: int, shifts, transform: str = "baker", alpha: int = 0):
        if a % 2 == 0:
            raise ValueError("a must be odd")
        self.d, self.a, self.kmax = d, int(a), int(kmax)
        self.shifts = _arr(shifts, np.float64).reshape(-1, d)
        self.m = self.shifts.shape[0]
        self.transform, self.alpha = transform, alpha
        self.g = korobov_vector(1 << self.kmax, d, self.a)

    def moved_shifts(self, k: int) -> np.ndarray:
        """Shifts that turn the 2^k-point lattice into the odd points of 2^(k+1)."""
        out = np.empty_like(self.shifts)
        check(lib().qmc_lattice_moved_shifts(1 << (k + 1), self.d, _p(self.g), self.m, _p(self.shifts), _p(out)),
              "qmc_lattice_moved_shifts")
        return out

    def ladder(self, params: "Params", kmin: int, kmax: int = None, setup=None):
        """[(n, result, per-shift)] for n = 2^kmin .. 2^kmax; setup(plan) may
        set launch options on every plan."""
        kmax = self.kmax if kmax is None else kmax
        if not (1 <= kmin <= kmax <= self.kmax):
            raise ValueError("need 1 <= kmin <= kmax <= kmax of the lattice")
        np_ = 2 if params.is_complex else 1

        def run(k, shifts):
            # the plan reads g mod 2^k itself
            plan = Plan(self.d, 1 << k, self.g, shifts, self.transform, self.alpha)
            if setup:
                setup(plan)
            res, q = plan.integrate(params)
            plan.close()
            flat = np.column_stack([q.real, q.imag]).ravel() if np_ == 2 else np.asarray(q, np.float64)
            return res, np.ascontiguousarray(flat)

        res, flat = run(kmin, self.shifts)
        out = [(1 << kmin, res, flat)]
        for k in range(kmin, kmax):
            _, extra = run(k, self.moved_shifts(k))
            merged = np.zeros_like(flat)
            res = qmc_result()
            check(lib().qmc_lattice_merge(self.m, np_, _p(flat), _p(extra), _p(merged), C.byref(res)),
                  "qmc_lattice_merge")
            flat = merged
            out.append((1 << (k + 1), res, flat))
        return [(n, r, (f[0::2] + 1j * f[1::2]) if np_ == 2 else f) for n, r, f in out]

