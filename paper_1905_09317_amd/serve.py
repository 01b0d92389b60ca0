"""Replay a stream of Monte-Carlo queries against the library's serving lanes.

Queries are submitted at their arrival times (c2f_submit); a waiter thread
collects them in order (c2f_wait_info).  Latency is measured by the library's
own clock from submission to delivered outputs, so the waiter's order does
not distort it.  All simulation work runs in libc2f; this module only paces
submissions and summarises the timings.
"""
from __future__ import annotations

import threading
import time

import numpy as np

from .api import Request, Simulator
from .inputs import Query, ServedStream


def load_stream(sim: Simulator, stream: ServedStream) -> tuple[int, dict]:
    """Upload the stream's weather and every query's landscape crop
    (not part of any latency).  Returns (weather id, {qid: landscape id})."""
    wx = sim.set_weather(stream.weather)
    lands = {}
    for q in stream.queries:
        fuel, elev = stream.crop(q)
        lands[q.qid] = sim.load_landscape(fuel, elev, cell_m=stream.cell_m)
    return wx, lands


def request_of(stream: ServedStream, q: Query, landscape: int, weather: int,
               outputs=("burn_count", "burned_cells")) -> Request:
    return Request(landscape=landscape, weather=weather, n_periods=stream.n_periods, reps=q.reps,
                   seed=q.seed, sigma=stream.sigma, rounding=stream.rounding,
                   precision=stream.precision, ignition_mode=1, scenario_mode=1,
                   outputs=outputs)


def run_stream(sim: Simulator, stream: ServedStream, weather: int, lands: dict,
               queries=None, on_result=None, pace: bool = True) -> dict:
    """Submit `queries` (default: all) at their arrival times and wait for
    every result.  on_result(query, outputs, info) is called from the waiter
    thread.  Returns a summary of latencies and throughput."""
    queries = list(stream.queries if queries is None else queries)
    pending: list = []
    cv = threading.Condition()
    infos: list = [None] * len(queries)
    errors: list = []
    done_submitting = [False]

    def waiter():
        k = 0
        while True:
            with cv:
                while k >= len(pending) and not done_submitting[0]:
                    cv.wait()
                if k >= len(pending):
                    return
                q, ticket = pending[k]
            try:
                res, info = sim.wait_info(ticket)
                infos[k] = info
                if on_result is not None:
                    on_result(q, res, info)
            except Exception as exc:  # a failed request is reported, not fatal
                errors.append((q.qid, repr(exc)))
            k += 1

    th = threading.Thread(target=waiter, daemon=True)
    th.start()
    t0 = time.perf_counter()
    for q in queries:
        if pace:
            delay = t0 + q.t - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
        ticket, _ = sim.submit(request_of(stream, q, lands[q.qid], weather))
        with cv:
            pending.append((q, ticket))
            cv.notify()
    with cv:
        done_submitting[0] = True
        cv.notify()
    th.join()
    wall = time.perf_counter() - t0

    ok = [(q, i) for q, i in zip(queries, infos) if i is not None and i["status"] == 0]
    lat = np.array([i["done_ms"] - i["submit_ms"] for _, i in ok])
    queue = np.array([i["start_ms"] - i["submit_ms"] for _, i in ok])
    cu = sum(q.reps * q.side * q.side for q, _ in ok) * stream.n_periods
    first = min(i["submit_ms"] for _, i in ok) if ok else 0.0
    last = max(i["done_ms"] for _, i in ok) if ok else 0.0
    span_s = max(1e-9, (last - first) / 1e3)
    drain_ms = (last - max(i["submit_ms"] for _, i in ok)) if ok else float("nan")
    arrivals_s = queries[-1].t - queries[0].t if len(queries) > 1 else 0.0
    offered = (sum(q.reps * q.side * q.side for q in queries) * stream.n_periods
               / arrivals_s) if arrivals_s > 0 else float("nan")
    batches = {}
    for _, i in ok:
        batches[(i["lane"], i["start_ms"])] = i["batch_requests"]
    pct = (lambda a, p: float(np.percentile(a, p)) if a.size else float("nan"))
    return {
        "queries": len(queries), "completed": len(ok), "failed": len(queries) - len(ok),
        "errors": errors[:5],
        "latency_ms_p50": pct(lat, 50), "latency_ms_p99": pct(lat, 99),
        "latency_ms_mean": float(lat.mean()) if lat.size else float("nan"),
        "latency_ms_max": float(lat.max()) if lat.size else float("nan"),
        "queue_ms_p50": pct(queue, 50), "queue_ms_p99": pct(queue, 99),
        "cell_updates": cu, "span_s": span_s, "cell_updates_per_s": cu / span_s,
        "offered_cell_updates_per_s": offered,
        "arrival_span_s": arrivals_s, "wall_s": wall,
        # backlog left when the last query arrived, drained after it
        "drain_ms": drain_ms,
        "sustained": (drain_ms < max(2000.0, 100.0 * arrivals_s)) if pace and ok else None,
        "batches": len(batches),
        "mean_batch_requests": float(np.mean(list(batches.values()))) if batches else 0.0,
        "lanes_used": len({k[0] for k in batches}),
    }
