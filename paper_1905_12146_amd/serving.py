"""Serving many gradient sessions on one GPU (continuous batching).

``Server`` wraps the native scheduler of libphylograd (``pg_server_*``):
sessions are admitted by HBM footprint, every admitted session's next call
joins the next batch, and a batch runs as one launch per kernel.

``run_stream`` drives a stream of requests the way MCMC / HMC / optimizer
clients would: each request arrives at its (Poisson) time, opens a session
on its own tree and alignment, makes ``calls`` dependent logL + gradient
calls on perturbed branch lengths (partials stay resident between calls),
and closes.  It reports per-request and per-call latency percentiles and
throughput.
"""
from __future__ import annotations

import threading
import time

import numpy as np

from . import binding as B


class Server:
    def __init__(self, device=0, precision=B.PG_FP32, hbm_budget_bytes=32 << 30, max_sessions=64):
        self.handle = B.pg_server_create(device, precision, hbm_budget_bytes, max_sessions)
        self.precision = precision

    def open(self, w, masks=None):
        """Open a session for a synth.Workload (tree, tip masks, weights, model);
        ``masks`` may hold the workload's tip masks computed beforehand."""
        return B.pg_server_open(self.handle, w.parent, w.tip_masks() if masks is None else masks, w.weights,
                                w.Q, w.pi, w.rates, w.cat_weights)

    def submit(self, session, t, want_grad=True):
        return B.pg_server_submit(self.handle, session, t, want_grad)

    def wait(self, ticket, n_branches):
        return B.pg_server_wait(self.handle, ticket, n_branches)

    def close(self, session):
        B.pg_server_close(self.handle, session)

    def stats(self):
        return B.pg_server_stats(self.handle)

    def shutdown(self):
        if self.handle:
            B.pg_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.shutdown()


def _make(spec):
    from synth.workloads import request_workload
    return request_workload(spec)


def generate_requests(specs, processes=8):
    """Workloads of the request specs, generated in a process pool."""
    if processes <= 1:
        return [_make(s) for s in specs]
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    with ctx.Pool(processes) as pool:
        return pool.map(_make, specs, chunksize=4)


def run_stream(server, specs, workloads, calls=10, perturb=0.01, seed=0, time_origin=None):
    """Serve the requests; returns a dict of latencies (seconds) and counts.

    Each request thread sleeps until its arrival time, then opens, calls and
    closes; call k+1 uses t_k * exp(perturb * N(0, 1)).  Tip masks are built
    before the clock starts (the client's data, not the server's work).
    """
    n = len(specs)
    masks = [w.tip_masks() for w in workloads]
    req_lat = np.full(n, np.nan)
    call_lat = [[] for _ in range(n)]
    errors = []
    results = [None] * n
    start = time.perf_counter() if time_origin is None else time_origin

    def client(i):
        spec, w = specs[i], workloads[i]
        rng = np.random.default_rng(seed * 1_000_003 + spec.rid)
        delay = start + spec.arrival_s - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        t_arr = time.perf_counter()
        try:
            sid = server.open(w, masks[i])
            t = w.t.copy()
            out = []
            for _ in range(calls):
                tk = server.submit(sid, t)
                status, logL, grad, lat = server.wait(tk, len(t))
                if status != B.PG_OK:
                    raise B.PhyloGradError(status, f"request {spec.rid}")
                call_lat[i].append(lat * 1e-9)
                out.append((logL, grad))
                t = t * np.exp(perturb * rng.normal(size=t.shape))
            server.close(sid)
            results[i] = out
            req_lat[i] = time.perf_counter() - t_arr
        except Exception as e:  # reported, never swallowed
            errors.append((spec.rid, repr(e)))

    threads = [threading.Thread(target=client, args=(i,), daemon=True) for i in range(n)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    wall = time.perf_counter() - start
    cl = np.array([x for row in call_lat for x in row])
    done = int(np.isfinite(req_lat).sum())
    return {
        "requests": n, "completed": done, "errors": errors, "calls": int(cl.size), "wall_s": wall,
        "calls_per_s": cl.size / wall if wall > 0 else 0.0,
        "requests_per_s": done / wall if wall > 0 else 0.0,
        "request_p50_ms": float(np.nanpercentile(req_lat, 50) * 1e3) if done else None,
        "request_p99_ms": float(np.nanpercentile(req_lat, 99) * 1e3) if done else None,
        "request_mean_ms": float(np.nanmean(req_lat) * 1e3) if done else None,
        "call_p50_ms": float(np.percentile(cl, 50) * 1e3) if cl.size else None,
        "call_p99_ms": float(np.percentile(cl, 99) * 1e3) if cl.size else None,
        "results": results,
    }
