"""Request loop for the serving path: Poisson arrivals, continuous batching.

``serve(requests, rate, ...)`` replays a request stream against a
``ph0.Server``: request k arrives at the k-th point of a Poisson process of
the given rate; arrivals are offered to the server as soon as they arrive and
again whenever earlier work finishes (a request not admitted yet waits, and
that wait counts in its latency); finished results are collected without
blocking.  Latency = completion time - arrival time.

``plain(requests)`` runs the same requests one at a time through the
single-cloud device path, for comparison.
"""
from __future__ import annotations

import time
from collections import deque

import numpy as np

from . import ph0


def _percentiles(lat):
    a = np.asarray(lat) * 1000.0
    return dict(p50_ms=float(np.percentile(a, 50)), p99_ms=float(np.percentile(a, 99)),
                mean_ms=float(a.mean()), max_ms=float(a.max()))


def serve(requests, rate=None, server=None, mem_budget=8 << 30, slots=4, seed=0,
          keep_results=False):
    """Replay `requests` (list of N x d int8/int16 arrays).

    rate: arrivals per second (None = all arrive at t=0, closed loop).
    Returns a dict with throughput, latency percentiles and, optionally, the
    barcodes by request index.
    """
    own = server is None
    srv = ph0.Server(mem_budget, slots) if own else server
    rng = np.random.default_rng(seed)
    n = len(requests)
    if rate:
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n))
    else:
        arrivals = np.zeros(n)
    waiting = deque()
    results = {}
    lat = np.zeros(n)
    done = 0
    nxt = 0
    t0 = time.perf_counter()
    try:
        while done < n:
            now = time.perf_counter() - t0
            while nxt < n and arrivals[nxt] <= now:
                waiting.append(nxt)
                nxt += 1
            # admit in arrival order while slots and memory allow
            while waiting and srv.submit(requests[waiting[0]], waiting[0]):
                waiting.popleft()
            r = srv.poll()
            while r is not None:
                tag, status, bars = r
                if status != 0:
                    raise RuntimeError("request %d failed with status %d" % (tag, status))
                lat[tag] = time.perf_counter() - t0 - arrivals[tag]
                if keep_results:
                    results[tag] = bars
                done += 1
                r = srv.poll()
            if r is None and done < n:
                time.sleep(20e-6)
        elapsed = time.perf_counter() - t0
    finally:
        if own:
            srv.close()
    out = dict(requests=n, seconds=elapsed, clouds_per_s=n / elapsed,
               rate=rate, slots=slots, **_percentiles(lat))
    if keep_results:
        out["results"] = results
    return out


def plain(requests, device="cuda"):
    """The same requests one at a time through ph0_barcodes_device."""
    import torch

    nmax = max(r.shape[0] for r in requests)
    dmax = max(r.shape[1] for r in requests)
    ws = ph0.alloc_workspace(nmax, dmax, np.int16, device)
    lat = []
    t0 = time.perf_counter()
    results = []
    for r in requests:
        t1 = time.perf_counter()
        x = torch.from_numpy(np.ascontiguousarray(r)).to(device)
        out = ph0.ph0_barcodes_device(x, workspace=ws)
        results.append(out.cpu().numpy().view(np.uint32))
        lat.append(time.perf_counter() - t1)
    elapsed = time.perf_counter() - t0
    return dict(requests=len(requests), seconds=elapsed, clouds_per_s=len(requests) / elapsed,
                results=results, **_percentiles(lat))
