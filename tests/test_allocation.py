"""The total-error-goal allocation of lattice sizes over sectors (host
logic, no GPU): optimality against brute force over a small ladder, the
Lagrange condition of the continuous solution, and the constraint."""
import itertools
import math

import numpy as np
import pytest

from paper_1811_11722_amd.drivers import allocate_total


def _err(s0, n0, ns, rate):
    return math.sqrt(sum((s * (n0 / n) ** rate) ** 2 for s, n in zip(s0, ns)))


def test_continuous_solution_is_stationary_and_tight():
    rng = np.random.default_rng(3)
    s0 = 10.0 ** rng.uniform(-8, -4, 7)
    c = rng.uniform(1.0, 9.0, 7)
    n0, goal, rate = 16381, 3e-9, 2.0
    _, cont, _ = allocate_total(s0, c, n0, goal, rate, ladder=[1 << 40])
    # constraint holds with equality
    assert abs(_err(s0, n0, cont, rate) - goal) <= 1e-12 * goal
    # Lagrange: c_s / (2 rate sigma_s^2(n) / n_s) is the same for every s
    lam = c / (2 * rate * (s0 * (n0 / cont) ** rate) ** 2 / cont)
    assert np.all(np.abs(lam / lam[0] - 1) < 1e-10)


@pytest.mark.parametrize("seed", range(6))
def test_rounded_allocation_against_brute_force(seed):
    """On a ladder of 8 sizes and 3 sectors: the rounded allocation meets the
    goal whenever the ladder can, and costs at most the ladder's step factor
    more than the cheapest feasible choice (the continuous optimum is a lower
    bound for every feasible choice)."""
    rng = np.random.default_rng(seed)
    ladder = [1021 * 2 ** k for k in range(8)]
    s0 = 10.0 ** rng.uniform(-7, -5, 3)
    c = rng.uniform(1.0, 5.0, 3)
    n0, rate = 1021, 2.0
    goal = float(np.sqrt(np.sum(s0 ** 2))) * 10.0 ** rng.uniform(-3.5, -1)
    sizes, cont, pred = allocate_total(s0, c, n0, goal, rate, ladder=ladder)
    best = None
    for ns in itertools.product(ladder, repeat=3):
        if _err(s0, n0, ns, rate) <= goal:
            cost = sum(ci * ni for ci, ni in zip(c, ns))
            best = cost if best is None else min(best, cost)
    if best is None:  # the ladder cannot reach the goal: every sector at the top
        assert all(n == ladder[-1] for n in sizes) or pred > goal
        return
    assert pred <= goal * (1 + 1e-12)
    cost = sum(ci * ni for ci, ni in zip(c, sizes))
    lower = sum(ci * ni for ci, ni in zip(c, cont))
    assert lower <= best * (1 + 1e-12)
    assert cost <= 2.0 * lower * (1 + 1e-12)


def test_zero_error_sectors_take_the_smallest_lattice():
    sizes, _, pred = allocate_total([0.0, 1e-6], [1.0, 1.0], 1021, 1e-8, 2.0, ladder=[1021, 2039, 4093, 1 << 30])
    assert sizes[0] == 1021 and pred <= 1e-8


def test_invalid_inputs():
    with pytest.raises(ValueError):
        allocate_total([1e-6], [0.0], 1021, 1e-8)
    with pytest.raises(ValueError):
        allocate_total([np.nan], [1.0], 1021, 1e-8)


def test_per_sector_rates_stationary_and_tight():
    """Different rates per sector: the bisection meets the goal and the
    Lagrange condition cost_s n_s / (2 rate_s sigma_s(n_s)^2) is common."""
    rng = np.random.default_rng(8)
    s0 = 10.0 ** rng.uniform(-8, -4, 9)
    c = rng.uniform(1.0, 9.0, 9)
    r = rng.uniform(0.5, 2.5, 9)
    n0, goal = 65521, 1e-9
    _, cont, _ = allocate_total(s0, c, n0, goal, r, ladder=[1 << 62])
    err = np.sqrt(np.sum((s0 * (n0 / cont) ** r) ** 2))
    assert abs(err - goal) <= 1e-9 * goal
    lam = c * cont / (2 * r * (s0 * (n0 / cont) ** r) ** 2)
    assert np.all(np.abs(lam / lam[0] - 1) < 1e-8)
    # with equal rates the bisection reproduces the closed form
    _, cont2, _ = allocate_total(s0, c, n0, goal, 2.0, ladder=[1 << 62])
    a = (s0 ** 2 * n0 ** 4.0 / c) ** (1 / 5)
    K = (np.sum(s0 ** 2 * n0 ** 4.0 * a ** -4.0) / goal ** 2) ** 0.25
    assert np.allclose(cont2, K * a, rtol=1e-9)


def test_estimate_rates():
    from paper_1811_11722_amd.drivers import estimate_rates
    r = estimate_rates([1e-4, 1e-4, 1e-4, 0.0], [1e-6, 1e-3, 1e-4 * 4 ** -1.5, 0.0], 1000, 4000)
    assert np.allclose(r[:3], [2.5, 0.25, 1.5])
    assert r[3] == 0.25


def test_jsonl_rows_resume(tmp_path):
    """The sweep record: rows written are found again by key after a reopen,
    a last line cut short by a crash is dropped (and the file truncated to
    the last whole row, so the next append starts a clean line), and a
    missing path keeps rows in memory only."""
    from paper_1811_11722_amd.drivers import JsonlRows
    path = str(tmp_path / "rows.jsonl")
    r = JsonlRows(path, ("phase", "sector"))
    assert r.resumed == 0 and r.get("pilot", 0) is None
    for s in range(3):
        r.add({"phase": "pilot", "sector": s, "n": 16381, "rel_err": 0.1 * s})
    with open(path, "a") as f:
        f.write('{"phase": "pilot", "sector": 3, "n"')          # interrupted write
    r2 = JsonlRows(path, ("phase", "sector"))
    assert r2.resumed == 3 and r2.get("pilot", 3) is None
    assert r2.get("pilot", 2) == {"phase": "pilot", "sector": 2, "n": 16381, "rel_err": 0.2}
    r2.add({"phase": "pilot", "sector": 3, "n": 16381, "rel_err": 0.3})
    r3 = JsonlRows(path, ("phase", "sector"))
    assert r3.resumed == 4 and r3.get("pilot", 3)["rel_err"] == 0.3
    mem = JsonlRows(None, ("form", "n"))
    mem.add({"form": "plain", "n": 5})
    assert mem.get("plain", 5) == {"form": "plain", "n": 5} and mem.resumed == 0
