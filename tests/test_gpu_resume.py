"""Resumable sweeps: the sector-batch and convergence drivers append one JSON
line per result, and a rerun on a file cut short (as by a crash) reproduces
the uninterrupted record exactly, recomputing only what is missing."""
import json
import sys

import pytest

from paper_1811_11722_amd import drivers

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _rows(path):
    return [json.loads(x) for x in open(path).read().splitlines() if x.strip()]


def _cut(src, dst, keep, partial=True):
    lines = open(src).read().splitlines(keepends=True)
    with open(dst, "w") as f:
        f.writelines(lines[:keep])
        if partial:
            f.write(lines[keep][: len(lines[keep]) // 2])


def _key(r, fields):
    return tuple(r[f] for f in fields)


def test_sector_batch_rows_resume(tmp_path):
    full, cut = str(tmp_path / "full.jsonl"), str(tmp_path / "cut.jsonl")
    _say("sector batch rows, 30 sectors, uninterrupted")
    a = drivers.sector_batch_rows(full, count=30, chunk=8)
    assert a["sectors_computed"] == 60 and a["rows_resumed"] == 0
    _cut(full, cut, 41)        # every pilot and 11 finals, then half a line
    _say("sector batch rows, resumed")
    b = drivers.sector_batch_rows(cut, count=30, chunk=8)
    assert b["rows_resumed"] == 41 and b["sectors_computed"] == 19
    ra = {_key(r, ("phase", "sector")): r for r in _rows(full)}
    rb = {_key(r, ("phase", "sector")): r for r in _rows(cut)}
    assert ra == rb
    assert len(ra) == 60 and a["rel_err_max"] == b["rel_err_max"]


def test_convergence_resume(tmp_path):
    full, cut = str(tmp_path / "full.jsonl"), str(tmp_path / "cut.jsonl")
    args = dict(kmin=14, kmax=16, cv_kmax=15, R=8, K=4, n_train=16381, max_sweeps=2)
    _say("convergence rows, uninterrupted")
    a = drivers.convergence(out_path=full, **args)
    n_rows = len(_rows(full))
    assert n_rows == 3 + 1 + 2      # plain rungs, the model, cv rungs
    _cut(full, cut, 4)              # the plain rungs and the model
    _say("convergence rows, resumed")
    b = drivers.convergence(out_path=cut, **args)
    assert b["rows_resumed"] == 4
    strip = lambda rows: [{k: v for k, v in r.items() if k not in ("seconds", "evals_per_s", "search_seconds")}
                          for r in rows]
    assert strip(a["rows"]) == strip(b["rows"])
    assert strip(a["cv"]["rows"]) == strip(b["cv"]["rows"])
