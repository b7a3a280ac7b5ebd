"""The scaling measure and gain that bench.py reports, against Table 1 of the paper (Sec. 4):
recomputed from the printed per-event times, P_n(3), P_n(4) and G_n must reproduce the printed
columns to one unit of their last printed digit (the printed times are rounded to four digits,
and the printed P and G were evidently formed from unrounded times)."""
import os

import pytest

import bench

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table1_timings.txt")


def _rows():
    out = []
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            n, tg, p3, tc, p4, g = line.split()
            out.append((int(n), float(tg), None if p3 == "-" else float(p3), float(tc),
                        None if p4 == "-" else float(p4), int(g)))
    return out


def test_table1_scaling_measures_and_gain():
    rows = _rows()
    assert [r[0] for r in rows] == list(range(4, 13))
    for prev, cur in zip(rows, rows[1:]):
        n = cur[0]
        assert abs(bench.scaling_measure(cur[1], prev[1], n, 3) - cur[2]) <= 0.01, n
        assert abs(bench.scaling_measure(cur[3], prev[3], n, 4) - cur[4]) <= 0.01, n
    for n, tg, _, tc, _, g in rows:
        assert abs(tc / tg - g) <= 1.0, n


def test_scaling_measure_is_one_for_pure_power_laws():
    for m in (3, 4):
        for n in range(5, 13):
            assert bench.scaling_measure(n ** m, (n - 1) ** m, n, m) == pytest.approx(1.0, rel=1e-14)
