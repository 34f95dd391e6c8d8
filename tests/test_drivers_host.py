"""Host logic of the drivers: the Alg. 2 schedule and the stage ranges."""
import os

import numpy as np

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _drivers():
    from paper_2002_10083_amd import drivers
    return drivers


def test_binary_schedule_matches_hand_trace():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "alg2_schedule_8.txt"))
            if l.strip() and not l.startswith("#")]
    assert _drivers().binary_schedule(8) == [int(r[1]) for r in rows]


def test_binary_schedule_matches_oracle():
    for s in range(1, 40):
        assert _drivers().binary_schedule(s) == oracle.binary_merge_schedule(s)[0]


def test_stage_ranges_cover():
    for n, s in ((10, 3), (1000, 8), (7, 8)):
        r = _drivers().stage_ranges(n, s)
        assert r[0][0] == 0 and r[-1][1] == n and len(r) == s
        assert all(a[1] == b[0] for a, b in zip(r, r[1:]))
        assert max(b - a for a, b in r) - min(b - a for a, b in r) <= 1
