"""Loading the stored oracle runs (``tests/golden/oracle_*.json``, written by
``tests/golden/make_oracle_runs.py`` from ``oracle/`` alone) and comparing a
library run with them step by step."""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")
sys.path.insert(0, GOLDEN)
from fingerprint import compare as fp_compare  # noqa: E402
from fingerprint import fingerprint  # noqa: E402


class GoldenRun:
    def __init__(self, name: str):
        path = os.path.join(GOLDEN, f"oracle_{name}.json")
        d = json.load(open(path))
        self.d = d
        self.M, self.K, self.steps = d["M"], d["K"], d["steps"]
        self.eta = np.array([[complex(*z) for z in row] for row in d["eta"]])
        self.rho = np.array([[complex(*z) for z in r] for r in d["rho"]]).reshape(-1, self.M, self.M)
        f = d["stats_fields"]
        self.stats = [None] + [dict(zip(f, row)) for row in d["stats"][1:]]
        self.fp = {int(k): v for k, v in d["fp"].items()}

    @staticmethod
    def exists(name: str) -> bool:
        return os.path.exists(os.path.join(GOLDEN, f"oracle_{name}.json"))

    def ambiguous(self, t_max: int) -> int:
        return sum(self.stats[t]["n_amb_rep"] + self.stats[t]["n_amb_theta"] for t in range(1, t_max + 1))


def fingerprint_of(hist, w) -> dict:
    return fingerprint(hist, w)


def check_fingerprint(got_groups, gold: GoldenRun, t: int, wtol: float):
    why = fp_compare(fingerprint(*got_groups), gold.fp[t], wtol)
    assert why == "", f"groups after step {t}: {why}"


def check_stats(stats, gold: GoldenRun, t0: int = 1):
    """Library counters (list of dicts for steps t0..) against the stored ones.
    The library stores merged groups, so its groups stored after step t are the
    groups the oracle extends at step t+1 (pre-merging keeps the survivors
    themselves and merges them at the next step)."""
    for k, s in enumerate(stats):
        t = t0 + k
        o = gold.stats[t]
        for key in ("n_groups", "n_children", "n_survivors"):
            assert s[key] == o[key], (t, key, s[key], o[key])
        if t + 1 <= gold.steps:
            assert s["n_stored"] == gold.stats[t + 1]["n_groups"], (t, s["n_stored"])
        assert abs(s["dropped_abs"] - o["dropped_abs"]) <= 1e-12 * max(1.0, o["dropped_abs"]), t
