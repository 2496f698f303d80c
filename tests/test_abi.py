"""C ABI on the CPU: the library loads, exports every function include/qmc.h
declares, and rejects bad arguments before touching a device."""
import ctypes as C
import os
import re
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qmc.h")


@pytest.fixture(scope="module")
def Q():
    from paper_1811_11722_amd import qmc
    qmc.lib()
    return qmc


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qmc_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(Q):
    names = _declared()
    assert len(names) >= 14
    for name in names:
        assert hasattr(Q.lib(), name), name
        assert name in Q.SIGNATURES, f"binding lacks {name}"


def _plan_status(Q, d, n, g, m, shifts, kind=0, alpha=0):
    h = C.c_void_p()
    g = np.ascontiguousarray(np.asarray(g, dtype=np.uint64))
    sh = np.ascontiguousarray(np.asarray(shifts, dtype=np.float64))
    return Q.lib().qmc_plan_create(d, n, g.ctypes.data_as(C.c_void_p), m,
                                   sh.ctypes.data_as(C.c_void_p), Q.qmc_transform(kind, alpha),
                                   C.byref(h))


def test_plan_create_validation(Q):
    g2 = [1, 5]
    z = np.zeros((2, 2))
    cases = [
        ((0, 7, g2, 2, z), Q.QMC_EINVAL),                      # d = 0
        ((17, 7, [1] * 17, 2, np.zeros((2, 17))), Q.QMC_EUNSUPPORTED),
        ((2, 1, g2, 2, z), Q.QMC_EINVAL),                      # n < 2
        ((2, 2 ** 31 + 1, g2, 2, z), Q.QMC_EUNSUPPORTED),      # n > 2^31
        ((2, 7, [1, 7], 2, z), Q.QMC_EINVAL),                  # g_i = 0 mod n
        ((2, 7, g2, 1, z[:1]), Q.QMC_EINVAL),                  # m < 2
        ((2, 7, g2, 2, np.full((2, 2), 1.0)), Q.QMC_EINVAL),   # shift = 1
        ((2, 7, g2, 2, np.full((2, 2), -0.1)), Q.QMC_EINVAL),  # shift < 0
        ((2, 7, g2, 2, np.full((2, 2), np.nan)), Q.QMC_EINVAL),
        ((2, 7, g2, 5000, np.zeros((5000, 2))), Q.QMC_EUNSUPPORTED),
    ]
    for args, want in cases:
        assert _plan_status(Q, *args) == want, args
    assert _plan_status(Q, 2, 7, g2, 2, z, kind=9) == Q.QMC_EINVAL
    assert _plan_status(Q, 2, 7, g2, 2, z, kind=1, alpha=0) == Q.QMC_EINVAL
    assert _plan_status(Q, 2, 7, g2, 2, z, kind=1, alpha=7) == Q.QMC_EUNSUPPORTED
    h = C.c_void_p()
    g = np.array(g2, dtype=np.uint64)
    assert Q.lib().qmc_plan_create(2, 7, g.ctypes.data_as(C.c_void_p), 2, None,
                                   Q.qmc_transform(0, 0), C.byref(h)) == Q.QMC_EINVAL
    assert Q.lib().qmc_plan_create(2, 7, None, 2, z.ctypes.data_as(C.c_void_p),
                                   Q.qmc_transform(0, 0), C.byref(h)) == Q.QMC_EINVAL
    assert b"m must be" in Q.lib().qmc_last_error() or True


def test_korobov_search_validation(Q):
    cand = np.array([3, 5], dtype=np.uint64)
    a, p = C.c_uint64(), C.c_double()
    L = Q.lib()
    cp = cand.ctypes.data_as(C.c_void_p)
    assert L.qmc_korobov_search(101, 2, cp, 0, C.byref(a), C.byref(p), None) == Q.QMC_EINVAL
    assert L.qmc_korobov_search(101, 0, cp, 2, C.byref(a), C.byref(p), None) == Q.QMC_EINVAL
    assert L.qmc_korobov_search(101, 17, cp, 2, C.byref(a), C.byref(p), None) == Q.QMC_EUNSUPPORTED
    assert L.qmc_korobov_search(1, 2, cp, 2, C.byref(a), C.byref(p), None) == Q.QMC_EINVAL
    assert L.qmc_korobov_search(2 ** 31 + 11, 2, cp, 2, C.byref(a), C.byref(p), None) == Q.QMC_EUNSUPPORTED
    bad = np.array([3, 101], dtype=np.uint64)
    assert L.qmc_korobov_search(101, 2, bad.ctypes.data_as(C.c_void_p), 2, C.byref(a), C.byref(p),
                                None) == Q.QMC_EINVAL
    assert L.qmc_korobov_search(101, 2, None, 2, C.byref(a), C.byref(p), None) == Q.QMC_EINVAL


def test_korobov_vector_host(Q):
    g = Q.korobov_vector(131071, 6, 48724)
    assert [int(v) for v in g] == [pow(48724, i, 131071) for i in range(6)]
    with pytest.raises(Q.QMCError):
        Q.korobov_vector(1, 2, 3)


def test_null_plan_and_status_strings(Q):
    L = Q.lib()
    r = Q.qmc_result()
    assert L.qmc_integrate(None, 0, None, C.byref(r), None) == Q.QMC_EINVAL
    assert L.qmc_plan_set_launch(None, None) == Q.QMC_EINVAL
    assert L.qmc_lattice_dump(None, 0, 0, None, None) == Q.QMC_EINVAL
    L.qmc_plan_destroy(None)
    for s in range(7):
        assert L.qmc_status_string(s) != b"unknown status"
    assert L.qmc_status_string(99) == b"unknown status"
    assert L.qmc_batch_stats(None) == Q.QMC_EINVAL
    stats = Q.batch_stats()  # no device work
    assert set(stats) == {"contexts_built", "graph_launches", "specialised_captures", "specialised_launches"}
    assert all(isinstance(v, int) and v >= 0 for v in stats.values())


def test_construction_and_merge_validation(Q):
    """The lattice-construction entry points reject bad arguments before any
    device work."""
    L = Q.lib()
    z = np.zeros(4, dtype=np.uint64)
    e2 = np.zeros(4)
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    assert L.qmc_cbc_search(1021, 0, None, None, 0, p(z), p(e2)) == Q.QMC_EINVAL        # d = 0
    assert L.qmc_cbc_search(1021, 17, None, None, 0, p(z), p(e2)) == Q.QMC_EUNSUPPORTED  # d > 16
    assert L.qmc_cbc_search(1, 2, None, None, 0, p(z), p(e2)) == Q.QMC_EINVAL           # n < 2
    assert L.qmc_cbc_search(2 ** 31 + 1, 2, None, None, 0, p(z), p(e2)) == Q.QMC_EUNSUPPORTED
    bad_g = np.array([1.0, -1.0])
    assert L.qmc_cbc_search(1021, 2, p(bad_g), None, 0, p(z), p(e2)) == Q.QMC_EINVAL    # gamma < 0
    cand = np.array([4, 8], dtype=np.uint64)
    assert L.qmc_cbc_search(1024, 2, None, p(cand), 2, p(z), p(e2)) == Q.QMC_EINVAL     # not units
    assert L.qmc_cbc_search(1021, 2, None, None, 0, None, p(e2)) == Q.QMC_EINVAL        # null output
    assert L.qmc_cbc_search(2 ** 31 - 1, 2, None, None, 0, p(z), p(e2)) == Q.QMC_EUNSUPPORTED  # too much work
    a, sc = C.c_uint64(), C.c_double()
    odd = np.array([3, 5], dtype=np.uint64)
    assert L.qmc_korobov_search_extensible(0, 4, 2, p(odd), 2, C.byref(a), C.byref(sc), None) == Q.QMC_EINVAL
    assert L.qmc_korobov_search_extensible(5, 4, 2, p(odd), 2, C.byref(a), C.byref(sc), None) == Q.QMC_EINVAL
    assert L.qmc_korobov_search_extensible(4, 32, 2, p(odd), 2, C.byref(a), C.byref(sc), None) == Q.QMC_EUNSUPPORTED
    assert L.qmc_korobov_search_extensible(4, 8, 2, p(cand), 2, C.byref(a), C.byref(sc), None) == Q.QMC_EINVAL
    q = np.zeros(4)
    res = Q.qmc_result()
    assert L.qmc_lattice_merge(2, 3, p(q), p(q), p(q), C.byref(res)) == Q.QMC_EINVAL
    assert L.qmc_lattice_merge(2, 1, None, p(q), p(q), C.byref(res)) == Q.QMC_EINVAL
    nanq = np.array([np.nan, 1.0])
    assert L.qmc_lattice_merge(2, 1, p(nanq), p(nanq), p(q[:2].copy()), C.byref(res)) == Q.QMC_ENONFINITE
    lam, r = C.c_double(), Q.qmc_result()
    assert L.qmc_deform_select(None, None, 1.0, 0.5, 4, C.byref(lam), C.byref(r)) == Q.QMC_EINVAL
    frac = C.c_double()
    assert L.qmc_deform_check(None, None, C.byref(frac), None) == Q.QMC_EINVAL


def test_moved_shifts_exact(Q):
    """qmc_lattice_moved_shifts (host code): {shift + (g mod 2n)/2n} against
    exact rationals, and the nesting it serves: the n-point lattice with the
    moved shifts is exactly the odd half of the 2n-point lattice."""
    from fractions import Fraction as Fr
    L = Q.lib()
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    d, m, a = 3, 5, 1093
    rng = np.random.default_rng(7)
    sh = rng.random((m, d))
    sh[0, 0] = 1.0 - 2.0 ** -53       # a sum that rounds up to 1 wraps to 0
    for k in (1, 5, 12, 31):
        n2 = 1 << (k + 1)
        g = np.array([pow(a, i, 1 << 40) for i in range(d)], dtype=np.uint64)   # read mod n2
        out = np.empty_like(sh)
        assert L.qmc_lattice_moved_shifts(n2, d, p(g), m, p(sh), p(out)) == Q.QMC_OK
        for kk in range(m):
            for i in range(d):
                want = float(Fr(float(sh[kk, i])) + Fr(int(g[i]) % n2, n2))   # one rounding
                want = want - 1.0 if want >= 1.0 else want                   # then the wrap
                assert out[kk, i] == want, (k, kk, i)
    # nesting, in exact rationals on a tiny lattice with dyadic shifts
    n, d = 16, 2
    g = np.array([1, 5], dtype=np.uint64)
    sh = np.array([[0.25, 0.5], [0.125, 0.875]])
    out = np.empty_like(sh)
    assert L.qmc_lattice_moved_shifts(2 * n, d, p(g), 2, p(sh), p(out)) == Q.QMC_OK
    for kk in range(2):
        pts = lambda N, s: {tuple((Fr(j * int(gi), N) + Fr(float(si))) % 1 for gi, si in zip(g, s)) for j in range(N)}
        odd = {tuple((Fr((2 * j + 1) * int(gi), 2 * n) + Fr(float(si))) % 1 for gi, si in zip(g, sh[kk]))
               for j in range(n)}
        assert pts(n, out[kk]) == odd
        assert pts(n, sh[kk]) | odd == pts(2 * n, sh[kk])
    # validation
    assert L.qmc_lattice_moved_shifts(24, d, p(g), 2, p(sh), p(out)) == Q.QMC_EINVAL        # not a power of 2
    assert L.qmc_lattice_moved_shifts(1, d, p(g), 2, p(sh), p(out)) == Q.QMC_EINVAL
    assert L.qmc_lattice_moved_shifts(1 << 33, d, p(g), 2, p(sh), p(out)) == Q.QMC_EUNSUPPORTED
    assert L.qmc_lattice_moved_shifts(32, 0, p(g), 2, p(sh), p(out)) == Q.QMC_EINVAL
    assert L.qmc_lattice_moved_shifts(32, 17, p(g), 2, p(sh), p(out)) == Q.QMC_EUNSUPPORTED
    assert L.qmc_lattice_moved_shifts(32, d, None, 2, p(sh), p(out)) == Q.QMC_EINVAL
    bad = np.array([[0.5, 1.0], [0.0, 0.0]])
    assert L.qmc_lattice_moved_shifts(32, d, p(g), 2, p(bad), p(out)) == Q.QMC_EINVAL


def _math_table():
    text = open(os.path.join(ROOT, "paper_1811_11722_amd", "csrc", "qmc_device.hpp")).read()
    body = text[text.index("kMathTab[1024]"):]
    body = body[body.index("{") + 1: body.index("};")]
    body = "\n".join(line.split("//")[0] for line in body.split("\n"))
    vals = [float.fromhex(v) for v in re.findall(r"(-?0x[0-9a-fp.+-]+),", body)]
    assert len(vals) == 1024
    return vals


def test_device_polynomials_are_the_generators_output():
    """The coefficients of qatan2 and qsincos in qmc_device.hpp are exactly
    what make_math_tables.py --poly writes (Chebyshev interpolants of the
    atan, sin and cos remainders in 50-digit arithmetic, and the split of
    pi/2)."""
    sys.path.insert(0, os.path.join(ROOT, "paper_1811_11722_amd", "csrc"))
    import make_math_tables as M
    want = M.polynomials()
    text = open(os.path.join(ROOT, "paper_1811_11722_amd", "csrc", "qmc_device.hpp")).read()

    def consts(fn):
        body = text[text.index(f"__device__ __forceinline__ {fn}"):]
        body = body[: body.index("\n}\n")]
        return [float.fromhex(v) for v in re.findall(r"(-?0x[0-9a-f]\.[0-9a-f]+p[+-]\d+)", body)]

    at = consts("double qatan2")
    # kTanPi8, pi/4, pi/2, pi, then the polynomial from its leading term
    import mpmath
    with mpmath.workdps(40):
        assert at[:4] == [float(mpmath.tan(mpmath.pi / 8)), float(mpmath.pi / 4), float(mpmath.pi / 2),
                          float(mpmath.pi)]
    assert at[4:] == want["atan"]
    sc = consts("void qsincos")
    assert sc[0] == want["two_over_pi"][0]
    assert sc[1:4] == want["half_pi_split"]
    assert sc[4:10] == want["sin"] and sc[10:16] == want["cos"]


def test_device_log_table():
    """The logarithm half of the table compiled into the device code: entry
    2j holds 1/(1/2 + (j + 1/2)/512) rounded to double and entry 2j + 1 -ln
    of that value rounded to double (checked in 40-digit arithmetic)."""
    import mpmath
    vals = _math_table()
    mpmath.mp.dps = 40
    for j in range(256):
        ic, nl = vals[2 * j], vals[2 * j + 1]
        assert ic == 1.0 / (0.5 + (j + 0.5) / 512.0)
        exact = -mpmath.log(mpmath.mpf(ic))
        assert abs(mpmath.mpf(nl) - exact) <= mpmath.mpf(np.spacing(abs(nl))) / 2


def test_device_exp_table():
    """The exponential half of the table: entry 512 + j holds 2^(j/512)
    rounded to double (checked in 40-digit arithmetic); and the split of
    ln 2 / 512 used in the reduction: the high part times any |k| < 2^21 is
    exact and high + low equals ln 2 / 512 to 1e-27."""
    import mpmath
    vals = _math_table()
    mpmath.mp.dps = 40
    for j in range(512):
        t = vals[512 + j]
        exact = mpmath.power(2, mpmath.mpf(j) / 512)
        assert abs(mpmath.mpf(t) - exact) <= mpmath.mpf(np.spacing(t)) / 2
    hi, lo = 6.93147180369123816490e-01 / 512.0, 1.90821492927058770002e-10 / 512.0
    assert float.fromhex("0x1.62e42feep-1") / 512.0 == hi
    assert int(float.hex(hi).split("p")[0].split(".")[1], 16) % (1 << 20) == 0  # 32 significant bits
    assert abs(mpmath.mpf(hi) + mpmath.mpf(lo) - mpmath.log(2) / 512) < mpmath.mpf(1e-27)
