"""Driver for the request server: a timed request stream with arrivals.

The server (hoqri_server_* in libhoqri.so) does admission, batching and all
device work; this module only submits requests at their arrival times, calls
the engine step and records when each result came back.
"""
from __future__ import annotations

import time
from typing import Sequence

from . import _lib as H


def run_stream(server: "H.Server", requests: Sequence[dict], arrivals: Sequence[float], stream=None):
    """Submits request i at arrivals[i] seconds after the start (all inputs are
    already on the device) and steps the server until every request finished.

    requests[i] needs: idx, vals, dims, ranks, U (list of factor tensors,
    overwritten), G. Returns (results by id, latency seconds by id, wall
    seconds from the first arrival to the last result, steps).
    """
    order = sorted(range(len(requests)), key=lambda i: arrivals[i])
    results, latency = {}, {}
    nxt = 0
    steps = 0
    t0 = time.perf_counter()
    first_arrival = arrivals[order[0]] if order else 0.0
    last_finish = first_arrival
    while len(results) < len(requests):
        now = time.perf_counter() - t0
        while nxt < len(order) and arrivals[order[nxt]] <= now:
            i = order[nxt]
            q = requests[i]
            server.submit(i, q["idx"], q["vals"], q["dims"], q["ranks"], q["U"], q["G"])
            nxt += 1
        queued, active, _ = server.info()
        if queued == 0 and active == 0:
            # idle until the next arrival
            if nxt < len(order):
                wait = arrivals[order[nxt]] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.001))
            continue
        done = server.step(stream)
        steps += 1
        tnow = time.perf_counter() - t0
        for r in done:
            results[r.id] = r
            latency[r.id] = tnow - arrivals[r.id]
            last_finish = max(last_finish, tnow)
    return results, latency, last_finish - first_arrival, steps
