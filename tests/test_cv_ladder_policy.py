"""The control variate's ladder policy (host logic, no GPU): the residual
pass runs until a given number of consecutive rungs have fallen back to the
plain estimate, the plain kernel from then on."""
from paper_1811_11722_amd.drivers import CvLadderPolicy


def _run(drop_after, used):
    """passes taken for a sequence of per-rung outcomes of the residual pass"""
    p, taken = CvLadderPolicy(drop_after), []
    for u in used:
        cv = p.residual_pass()
        taken.append(cv)
        if cv:
            p.record(u)
    return taken


def test_drops_after_consecutive_fallbacks():
    assert _run(2, [1, 1, 0, 0, 1, 1]) == [True, True, True, True, False, False]


def test_a_used_rung_resets_the_count():
    assert _run(2, [0, 1, 0, 1, 0, 0, 1]) == [True] * 6 + [False]


def test_zero_keeps_the_residual_pass():
    assert _run(0, [0] * 8) == [True] * 8


def test_drop_after_one():
    assert _run(1, [1, 0, 1]) == [True, True, False]
