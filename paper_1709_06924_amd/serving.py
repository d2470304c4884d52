"""Open-loop serving harness: replays a seeded Poisson request stream
(inputs.serving_stream) against the library's request loop (scvt.Server)
and reports latency percentiles and throughput.  Scheduling and statistics
only -- every solve runs in the HIP library."""
import time

import numpy as np

from . import inputs
from . import scvt


def depth_series(depth, step_s):
    """(time, waiting, running) samples thinned to one per step_s seconds:
    the largest queue depth and running count seen in each interval."""
    out = []
    for t, w, r in depth:
        b = int(t // step_s)
        if out and out[-1][0] == b * step_s:
            out[-1][1] = max(out[-1][1], w)
            out[-1][2] = max(out[-1][2], r)
        else:
            out.append([b * step_s, w, r])
    return out


def run_stream(requests, tol=1e-8, max_iter=5000, max_slots=8, hbm_budget=64 << 30,
               precision="mixed", m_hist=10, poll_s=0.002, log=None, series_step_s=1.0):
    """Submit each request at its arrival time (seconds from start), wait for
    all to finish.  Returns per-request records and a summary."""
    srv = scvt.Server(hbm_budget, max_slots)
    t0 = time.perf_counter()
    pending = {}
    records = []
    depth = []
    k = 0
    try:
        while k < len(requests) or pending:
            now = time.perf_counter() - t0
            while k < len(requests) and requests[k]["t"] <= now:
                r = requests[k]
                z0 = inputs.uniform_sphere(r["n"], r["z0_seed"])
                rid = srv.submit(z0, r["density"], tol, max_iter, m_hist=m_hist,
                                 precision=precision)
                pending[rid] = r
                k += 1
            for rid in list(pending):
                res = srv.poll(rid, want_z=False)
                if res is None:
                    continue
                r = pending.pop(rid)
                info = res["info"]
                records.append({"id": r["id"], "n": r["n"], "status": res["status"],
                                "latency_s": res["t_done"] - res["t_submit"],
                                "queue_s": res["t_start"] - res["t_submit"],
                                "iters": info["iter"], "evals": info["n_evals"],
                                "step_inf": info["step_inf"], "F": info["F"]})
                srv.release(rid)
                if log:
                    log("serving: request %d n=%d done in %.2f s (%d iterations)"
                        % (r["id"], r["n"], records[-1]["latency_s"], info["iter"]))
            st = srv.stats()
            depth.append((time.perf_counter() - t0, st["waiting"], st["running"]))
            time.sleep(poll_s)
    finally:
        srv.close()
    wall = time.perf_counter() - t0
    lat = np.array([r["latency_s"] for r in records])
    gen_it = sum(r["n"] * r["iters"] for r in records)
    summary = {
        "requests": len(records),
        "failed": sum(1 for r in records if r["status"] < 0),
        "converged": sum(1 for r in records if r["status"] == 0),
        "p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
        "mean_s": float(lat.mean()) if len(lat) else None,
        "wall_s": wall,
        "throughput_rps": len(records) / wall,
        "generator_iterations_per_s": gen_it / wall,
        "max_queue_depth": max((d[1] for d in depth), default=0),
        "max_running": max((d[2] for d in depth), default=0),
        "depth_over_time": depth_series(depth, series_step_s),
    }
    return records, summary
