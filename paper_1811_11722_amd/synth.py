"""Seeded synthetic inputs for the shifted rank-1 lattice estimator.

This module only *draws* inputs: random shifts, integrand parameters, sparse
polynomial tables, Korobov candidates and the prime ladder of lattice sizes.
It holds none of the estimator's arithmetic (no lattice points, no transforms,
no integrands, no sums), so the GPU library and the CPU oracle can both be fed
from it without sharing any of the method.

Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), written here from its
published definition.  A draw is addressed by a 128-bit counter
``(t, stream, sub, 0)`` and a 64-bit key (the config seed), so every value is
reproducible on its own.  Stream numbers:

* 0      integrand parameters (Genz a, u; sector tables of a single sector)
* 1      Korobov multiplier candidates
* 2      estimation shifts (counter t = k*d + i)
* 3      the independent shift of the control-variate training lattice
* 16 + s tables (sub 0) and shifts (sub 1) of sector s of a sector batch
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import List, Optional, Sequence

import numpy as np

# --------------------------------------------------------------------------
# Philox4x32-10
# --------------------------------------------------------------------------
_M0 = 0xD2511F53
_M1 = 0xCD9E8D57
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK32 = 0xFFFFFFFF

SEED_BASE = 18111172200


def philox4x32_10(counters: np.ndarray, key: Sequence[int]) -> np.ndarray:
    """Philox4x32 with 10 rounds on an (N, 4) array of uint32 counters."""
    c = np.asarray(counters, dtype=np.uint64).reshape(-1, 4)
    c0, c1, c2, c3 = (c[:, 0].copy(), c[:, 1].copy(), c[:, 2].copy(), c[:, 3].copy())
    k0, k1 = int(key[0]) & _MASK32, int(key[1]) & _MASK32
    m32 = np.uint64(_MASK32)
    for _ in range(10):
        p0 = c0 * np.uint64(_M0)
        p1 = c2 * np.uint64(_M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & m32
        hi1, lo1 = p1 >> np.uint64(32), p1 & m32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
        k0 = (k0 + _W0) & _MASK32
        k1 = (k1 + _W1) & _MASK32
    return np.stack([c0, c1, c2, c3], axis=1).astype(np.uint32)


def _key(seed: int):
    seed = int(seed)
    return (seed & _MASK32, (seed >> 32) & _MASK32)


def _counters(count: int, stream: int, offset: int, sub: int) -> np.ndarray:
    t = np.arange(offset, offset + count, dtype=np.uint64)
    ctr = np.zeros((count, 4), dtype=np.uint64)
    ctr[:, 0] = t & np.uint64(_MASK32)
    ctr[:, 1] = stream
    ctr[:, 2] = sub
    ctr[:, 3] = t >> np.uint64(32)
    return ctr


def u64s(seed: int, stream: int, count: int, offset: int = 0, sub: int = 0) -> np.ndarray:
    """64-bit words (w1 << 32 | w0) of the draws (offset .. offset+count-1)."""
    w = philox4x32_10(_counters(count, stream, offset, sub), _key(seed)).astype(np.uint64)
    return (w[:, 1] << np.uint64(32)) | w[:, 0]


def uniforms(seed: int, stream: int, count: int, offset: int = 0, sub: int = 0) -> np.ndarray:
    """Doubles in [0, 1): the top 53 bits of each 64-bit word times 2^-53."""
    return (u64s(seed, stream, count, offset, sub) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


class _Draws:
    """Sequential reader over one (seed, stream, sub) Philox stream."""

    def __init__(self, seed: int, stream: int, sub: int = 0):
        self.seed, self.stream, self.sub, self.pos = seed, stream, sub, 0

    def uniform(self, count: int) -> np.ndarray:
        out = uniforms(self.seed, self.stream, count, self.pos, self.sub)
        self.pos += count
        return out

    def word(self, count: int) -> np.ndarray:
        out = u64s(self.seed, self.stream, count, self.pos, self.sub)
        self.pos += count
        return out


# --------------------------------------------------------------------------
# Lattice sizes
# --------------------------------------------------------------------------
def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 3.3e24."""
    if n < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)
    for p in small:
        if n % p == 0:
            return n == p
    dd, s = n - 1, 0
    while dd % 2 == 0:
        dd //= 2
        s += 1
    for a in small:
        x = pow(a, dd, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def largest_prime_below(limit: int) -> int:
    n = limit - 1
    while not is_prime(n):
        n -= 1
    return n


def prime_ladder(kmin: int, kmax: int) -> List[int]:
    """Largest prime below 2^k for k = kmin..kmax."""
    return [largest_prime_below(1 << k) for k in range(kmin, kmax + 1)]


# --------------------------------------------------------------------------
# Integrand parameters
# --------------------------------------------------------------------------
def shifts(seed: int, m: int, d: int, stream: int = 2, sub: int = 0) -> np.ndarray:
    """m i.i.d. uniform shifts in [0,1)^d, row-major (m, d); draw t = k*d + i."""
    return uniforms(seed, stream, m * d, 0, sub).reshape(m, d)


def genz_params(seed: int, d: int, stream: int = 0):
    """Genz parameters a_i ~ U[2, 8], u_i ~ U[0, 1)."""
    dr = _Draws(seed, stream)
    a = 2.0 + 6.0 * dr.uniform(d)
    u = dr.uniform(d)
    return a, u


def korobov_candidates(seed: int, n: int, count: int = 64, stream: int = 1) -> np.ndarray:
    """Korobov multipliers a_c = 2 + (word_c mod (n - 3)) in [2, n - 2].

    a and n - a generate reflections of the same lattice, so each candidate is
    stored as min(a, n - a).
    """
    w = u64s(seed, stream, count)
    a = 2 + (w % np.uint64(n - 3)).astype(np.int64)
    a = np.minimum(a, n - a)
    return a.astype(np.uint64)


def exponent_vectors(d: int, max_exp: int = 2, min_deg: int = 1, max_deg: int = 3) -> List[tuple]:
    """All exponent vectors with entries <= max_exp and total degree in
    [min_deg, max_deg], in lexicographic order."""
    out = []
    for e in itertools.product(range(max_exp + 1), repeat=d):
        if min_deg <= sum(e) <= max_deg:
            out.append(e)
    return out


def _pick_distinct(dr: _Draws, pool: list, count: int) -> list:
    """Partial Fisher-Yates shuffle of `pool` driven by the stream."""
    pool = list(pool)
    count = min(count, len(pool))
    for t in range(count):
        r = int(dr.word(1)[0] % np.uint64(len(pool) - t))
        pool[t], pool[t + r] = pool[t + r], pool[t]
    return pool[:count]


@dataclasses.dataclass
class SectorTables:
    """One sector integrand  prod_i z_i^nu_i * U(z)^pow_u * (F(z) - i*delta)^pow_f.

    coef_u/exp_u hold U row-major (n_u, d); monomial 0 is the constant term.
    coef_f/exp_f hold F likewise.  Exponents are uint8 in {0, 1, 2}.
    """
    d: int
    coef_u: np.ndarray
    exp_u: np.ndarray
    coef_f: np.ndarray
    exp_f: np.ndarray
    nu: np.ndarray
    pow_u: float = -2.0
    pow_f: float = -1.3
    delta_im: float = 0.0
    is_complex: bool = False
    clamped: bool = False

    @property
    def n_u(self) -> int:
        return int(self.coef_u.shape[0])

    @property
    def n_f(self) -> int:
        return int(self.coef_f.shape[0])


def sector_tables(seed: int, d: int, n_u: int, n_f: int, *, stream: int = 0, sub: int = 0,
                  eps0: float = 0.3, complex_kinematics: bool = False,
                  delta_im: float = 1e-2) -> SectorTables:
    """Synthetic sector integrand tables.

    nu_i ~ U{0,1,2}.  U and F each start with the constant monomial, followed
    by distinct exponent vectors (entries 0..2, total degree 1..3) drawn
    without replacement.  Coefficients are 10^U(-2, 2).  With
    complex_kinematics every F coefficient also gets a sign +-1 with
    probability 1/2 and the integrand uses F - i*delta_im.
    """
    dr = _Draws(seed, stream, sub)
    pool = exponent_vectors(d)
    nu = np.floor(3.0 * dr.uniform(d)).astype(np.uint8)
    clamped = False
    tabs = []
    for count in (n_u, n_f):
        if count - 1 > len(pool):
            clamped = True
        picks = _pick_distinct(dr, pool, count - 1)
        exps = np.zeros((len(picks) + 1, d), dtype=np.uint8)
        if picks:
            exps[1:] = np.array(picks, dtype=np.uint8)
        coef = 10.0 ** (4.0 * dr.uniform(len(picks) + 1) - 2.0)
        tabs.append((coef, exps))
    (cu, eu), (cf, ef) = tabs
    if complex_kinematics:
        sign = np.where(dr.uniform(cf.shape[0]) < 0.5, -1.0, 1.0)
        cf = cf * sign
    return SectorTables(d=d, coef_u=cu, exp_u=eu, coef_f=cf, exp_f=ef, nu=nu,
                        pow_u=-2.0, pow_f=-1.0 - eps0,
                        delta_im=delta_im if complex_kinematics else 0.0,
                        is_complex=bool(complex_kinematics), clamped=clamped)


# --------------------------------------------------------------------------
# Workload descriptions
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    seed: int
    d: int
    n: int
    m: int
    transform: tuple            # (kind, alpha): kind 0 none, 1 Korobov, 2 baker
    family: str
    shifts: np.ndarray
    candidates: np.ndarray      # Korobov multiplier candidates
    genz_a: Optional[np.ndarray] = None
    genz_u: Optional[np.ndarray] = None
    sector: Optional[SectorTables] = None
    extra: dict = dataclasses.field(default_factory=dict)


N_LADDER = {k: largest_prime_below(1 << k) for k in (10, 12, 14, 16, 17, 18, 20, 22, 24, 30)}


def product_peak_workload(n: int = 131071, m: int = 16, d: int = 4, seed: int = SEED_BASE + 1,
                          alpha: int = 3) -> Workload:
    """Genz product peak, Korobov alpha periodisation (defaults: n = 131071, d = 4, m = 16)."""
    a, u = genz_params(seed, d)
    return Workload(name=f"genz_product_peak_d{d}_korobov{alpha}_n{n}_m{m}", seed=seed, d=d, n=n,
                    m=m, transform=(1, alpha), family="genz_product_peak",
                    shifts=shifts(seed, m, d), candidates=korobov_candidates(seed, n),
                    genz_a=a, genz_u=u)


def sector_workload(n: int = 16777213, m: int = 32, d: int = 6, n_u: int = 12, n_f: int = 30,
                    seed: int = SEED_BASE + 2, complex_kinematics: bool = False,
                    name: Optional[str] = None) -> Workload:
    """Sector integrand x^nu U^-2 F^-1.3 (optionally F - 0.01i), baker periodisation."""
    tab = sector_tables(seed, d, n_u, n_f, complex_kinematics=complex_kinematics)
    kind = "complex" if complex_kinematics else "real"
    return Workload(name=name or f"sector_{kind}_d{d}_nu{n_u}_nf{n_f}_baker_n{n}_m{m}", seed=seed,
                    d=d, n=n, m=m, transform=(2, 0), family="sector",
                    shifts=shifts(seed, m, d), candidates=korobov_candidates(seed, n), sector=tab)


def sector_batch_draws(seed: int = SEED_BASE + 3, count: int = 2000):
    """Per-sector (d, n_u, n_f) for a batch: d ~ U{2..9}, counts ~ U{4..40}."""
    out = []
    for s in range(count):
        dr = _Draws(seed, 16 + s, 2)
        r = dr.uniform(3)
        out.append((2 + int(8 * r[0]), 4 + int(37 * r[1]), 4 + int(37 * r[2])))
    return out


def sector_batch(seed: int = SEED_BASE + 3, count: int = 2000) -> List[SectorTables]:
    tabs = []
    for s, (d, nu_, nf_) in enumerate(sector_batch_draws(seed, count)):
        tabs.append(sector_tables(seed, d, nu_, nf_, stream=16 + s, sub=0))
    return tabs


def sector_batch_shifts(seed: int, s: int, m: int, d: int) -> np.ndarray:
    return shifts(seed, m, d, stream=16 + s, sub=1)
