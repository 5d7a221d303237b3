"""The Table 1 fixture (Section 3, Table 1) is the transcription every
Table-1 check reads: its printed speedup columns must be the ratios of its
printed IT and CPU columns, to the printed four decimals."""
import json
import os

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1.json")


def load_table1():
    with open(GOLDEN) as f:
        return json.load(f)["rows"]


def test_table1_fixture_is_self_consistent():
    rows = load_table1()
    assert len(rows) == 15
    assert sorted({r["m"] for r in rows}) == [300000, 400000, 500000, 600000, 700000]
    assert sorted({r["n"] for r in rows}) == [50, 100, 150]
    for r in rows:
        assert abs(r["mwrk_it"] / r["csk_it"] - r["it_speedup"]) <= 6e-5, r
        # the CPU ratio was printed from unrounded times
        assert abs(r["mwrk_cpu_s"] / r["csk_cpu_s"] - r["cpu_speedup"]) <= 3e-4 * r["cpu_speedup"], r
