"""Per-work-group timelines of the one-mask GS passes (profiling).

    python -m paper_1302_0120_amd.build --timeline      (once, on any host)
    python -m paper_1302_0120_amd.pass_timeline         (on the GPU)

Loads the timeline build of the library (``libphasemask_timeline.so``, see
``csrc/pm_trace.h``), runs one-mask solves of the 1024 x 1024 (100
iterations) and 800 x 600 (25 iterations) spot workloads, and prints, per
pass type, the medians over the recorded launches of: the kernel boundary
(previous pass's last work-group end to this pass's first work-group
start), the spread of work-group starts, and each work-group's time to its
loads, through its transforms, to its acknowledged stores and to its end.
The forced waits of the instrument slow a solve by about a fifth, so the
phases are upper bounds; the plain library's timings come from ``bench.py``.
"""
from __future__ import annotations

import ctypes
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TIMELINE_LIB = os.path.join(HERE, "libphasemask_timeline.so")
# Layout of the records (csrc/pm_trace.h).
LAUNCHES, WGS, FIELDS = 32, 1024, 8


def _load():
    if not os.path.exists(TIMELINE_LIB):
        raise SystemExit(f"{TIMELINE_LIB} is not built; run `python -m paper_1302_0120_amd.build --timeline`")
    os.environ["PHASEMASK_LIBRARY"] = TIMELINE_LIB
    if "paper_1302_0120_amd.binding" in sys.modules:
        raise SystemExit("run pass_timeline in a fresh process (the plain library is already loaded)")
    from paper_1302_0120_amd import binding
    return binding


def _read(lib, length):
    rec = np.zeros((2, LAUNCHES, WGS, FIELDS), dtype=np.uint64)
    cnt = np.zeros((2, WGS), dtype=np.uint32)
    fn = getattr(lib, f"phasemask_timeline_read_{length}")
    fn.restype = ctypes.c_int
    if fn(ctypes.c_void_p(rec.ctypes.data), ctypes.c_void_p(cnt.ctypes.data)) != 0:
        raise RuntimeError("timeline read failed")
    return rec, cnt


def _reset(lib, length):
    fn = getattr(lib, f"phasemask_timeline_reset_{length}")
    fn.restype = ctypes.c_int
    if fn() != 0:
        raise RuntimeError("timeline reset failed")


def _launches(rec, cnt, kind):
    """Records of the kept launches of pass `kind`, each (nwg, FIELDS)."""
    c = cnt[kind]
    nwg = int((c > 0).sum())
    if nwg == 0:
        return []
    if not ((c[:nwg] == c[0]).all() and (c[nwg:] == 0).all()):
        raise RuntimeError("launches of one pass type with different grids")
    n = int(c[0])
    out = []
    for s in range(max(0, n - LAUNCHES), n):
        r = rec[kind, s % LAUNCHES, :nwg].astype(np.int64)
        if not (r[:, 7] == s).all():
            raise RuntimeError("inconsistent launch records")
        out.append(r)
    return out


def summarise(rec_col, cnt_col, rec_row, cnt_row, tick_us):
    ev = [(int(r[:, 0].min()), 0, r) for r in _launches(rec_col, cnt_col, 0)]
    ev += [(int(r[:, 0].min()), 1, r) for r in _launches(rec_row, cnt_row, 1)]
    ev.sort(key=lambda e: e[0])
    per = {0: [], 1: []}
    prev_end = None
    for t0, kind, r in ev:
        t = r[:, :5].astype(np.float64)
        stored = bool((r[:, 2] > 0).all())
        per[kind].append({
            "boundary_us": None if prev_end is None else (t0 - prev_end) * tick_us,
            "start_spread_us": (r[:, 0].max() - t0) * tick_us,
            "loads_us": float(np.median(t[:, 1] - t[:, 0])) * tick_us,
            "transforms_us": float(np.median(t[:, 2] - t[:, 1])) * tick_us if stored else None,
            "stores_us": float(np.median(t[:, 3] - t[:, 2])) * tick_us if stored else None,
            "stores_max_us": float((t[:, 3] - t[:, 2]).max()) * tick_us if stored else None,
            "partials_us": float(np.median(t[:, 4] - t[:, 3])) * tick_us if stored else None,
            "span_us": (r[:, 4].max() - t0) * tick_us,
            "work_groups": r.shape[0],
        })
        prev_end = int(r[:, 4].max())
    out = {}
    for kind, name in ((0, "column pass"), (1, "row pass")):
        # the first and last launches of a solve run other modes (start, output)
        rows = [d for d in per[kind][1:-1] if d["transforms_us"] is not None and d["boundary_us"] is not None]
        if not rows:
            continue
        out[name] = {k: round(float(np.median([d[k] for d in rows])), 3) for k in rows[0]}
        out[name]["launches"] = len(rows)
    return out


def main():
    binding = _load()
    import torch
    from paper_1302_0120_amd import synth
    lib = binding.lib
    clock = lib.phasemask_timeline_clock_khz
    clock.restype = ctypes.c_int
    khz = clock()
    if khz <= 0:
        raise RuntimeError("no wall clock rate")
    tick_us = 1e3 / khz
    result = {"wall_clock_khz": khz}
    for spec, name in ((synth.SPOTS_1024, "1024x1024, 100 iterations"), (synth.SPOTS_800x600, "800x600, 25 iterations")):
        m, phi0 = synth.spot_problem(spec)
        md, pd = torch.from_numpy(m).cuda(), torch.from_numpy(phi0).cuda()
        plan = binding.PhaseMask(spec.height, spec.width)
        out = torch.empty_like(pd)
        hist = torch.empty(2 * spec.n_iter + 1, dtype=torch.float64, device="cuda")
        for _ in range(3):
            plan.solve(md, pd, spec.n_iter, out=out, history=hist)
        torch.cuda.synchronize()
        lcol, lrow = spec.height, spec.width
        for length in {lcol, lrow}:
            _reset(lib, length)
        plan.solve(md, pd, spec.n_iter, out=out, history=hist)
        torch.cuda.synchronize()
        rc, cc = _read(lib, lcol)
        rr, cr = _read(lib, lrow)
        result[name] = summarise(rc, cc, rr, cr, tick_us)
        print(json.dumps({name: result[name]}), flush=True)
    return result


if __name__ == "__main__":
    main()
