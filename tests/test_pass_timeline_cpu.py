"""Host logic of the pass-timeline tool (paper_1302_0120_amd/pass_timeline.py)
on synthetic records: launches ordered by their first start, kernel
boundaries between consecutive launches, per-phase medians, and the first
and last launch of each pass type left out."""
import numpy as np
import pytest

from paper_1302_0120_amd import pass_timeline as pt


def _records(n_launch, nwg, t0, period, phases, kind):
    rec = np.zeros((2, pt.LAUNCHES, pt.WGS, pt.FIELDS), dtype=np.uint64)
    cnt = np.zeros((2, pt.WGS), dtype=np.uint32)
    for s in range(n_launch):
        start = t0 + s * period
        for g in range(nwg):
            st = start + g % 3  # start spread of 2 ticks
            a = st + phases[0]
            b = a + phases[1]
            c = b + phases[2]
            e = c + phases[3]
            rec[kind, s % pt.LAUNCHES, g] = [st, a, b, c, e, 0, g % 8, s]
    cnt[kind, :nwg] = n_launch
    return rec, cnt


def test_summarise_phases_and_boundaries():
    # column launches at 0, 100, 200, ...; row launches at 50, 150, ...;
    # each launch's work-groups start over 2 ticks and last 38, so a launch
    # ends 40 ticks after its first start and the boundary is 10 ticks.
    rc, cc = _records(6, 16, 0, 100, (10, 20, 5, 3), 0)
    rr, cr = _records(6, 32, 50, 100, (12, 18, 6, 2), 1)
    out = pt.summarise(rc, cc, rr, cr, tick_us=0.01)
    col, row = out["column pass"], out["row pass"]
    assert col["launches"] == 4 and row["launches"] == 4  # first and last of each left out
    assert col["work_groups"] == 16 and row["work_groups"] == 32
    assert col["loads_us"] == pytest.approx(0.10) and col["transforms_us"] == pytest.approx(0.20)
    assert col["stores_us"] == pytest.approx(0.05) and col["partials_us"] == pytest.approx(0.03)
    assert row["loads_us"] == pytest.approx(0.12) and row["transforms_us"] == pytest.approx(0.18)
    assert col["start_spread_us"] == pytest.approx(0.02)
    assert col["boundary_us"] == pytest.approx(0.10) and row["boundary_us"] == pytest.approx(0.10)
    assert col["span_us"] == pytest.approx(0.40) and row["span_us"] == pytest.approx(0.40)


def test_ring_keeps_the_last_launches_and_checks_consistency():
    n = pt.LAUNCHES + 5
    rc, cc = _records(n, 8, 0, 100, (1, 2, 3, 4), 0)
    rr, cr = _records(n, 8, 50, 100, (1, 2, 3, 4), 1)
    out = pt.summarise(rc, cc, rr, cr, tick_us=1.0)
    assert out["column pass"]["launches"] == pt.LAUNCHES - 2
    bad = cc.copy()
    bad[0, 3] += 1  # one work-group saw another launch count
    with pytest.raises(RuntimeError):
        pt.summarise(rc, bad, rr, cr, tick_us=1.0)
