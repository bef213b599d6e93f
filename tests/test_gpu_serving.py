"""Serving extension: continuous batching of many sessions on one GPU.

The defining check: each request's result is bit-for-bit the same whether
its calls run alone (a batch of one) or batched with other requests, and
the same as the single-context path; plus oracle parity, admission by HBM
footprint under a small budget, and error reporting.
"""
import numpy as np
import pytest

import oracle as O
from paper_1905_12146_amd import binding as B
from synth import make_workload
from tests._fixtures import args_of

pytestmark = pytest.mark.gpu


def _workloads():
    sizes = [(100, 500), (257, 1031), (640, 333), (33, 17), (1200, 2100), (2, 5), (499, 64)]
    return [make_workload("C3", seed=100 + i, n_tips=n, n_patterns=s, tips="uniform")
            for i, (n, s) in enumerate(sizes)]


def _single(w, precision):
    with B.Context(0, precision) as ctx:
        ctx.set_workload(w)
        return ctx.logL_and_grad(w.t)


@pytest.mark.parametrize("precision", [B.PG_FP32, B.PG_FP64])
def test_alone_equals_mixed_bitwise(gpu, precision):
    from paper_1905_12146_amd.serving import Server
    ws = _workloads()
    ref = [_single(w, precision) for w in ws]
    with Server(0, precision, 8 << 30, 64) as srv:
        # alone: one request at a time
        alone = []
        for w in ws:
            sid = srv.open(w)
            st, l, g, _ = srv.wait(srv.submit(sid, w.t), len(w.t))
            assert st == B.PG_OK
            alone.append((l, g))
            srv.close(sid)
        # mixed: everything queued at once, several calls each
        sids = [srv.open(w) for w in ws]
        tickets = [[srv.submit(sid, w.t * f) for f in (1.0, 1.3, 1.0)] for sid, w in zip(sids, ws)]
        mixed = [[srv.wait(tk, len(w.t)) for tk in tks] for tks, w in zip(tickets, ws)]
        stats = srv.stats()
        for sid in sids:
            srv.close(sid)
    assert stats["max_batch"] >= 2, stats
    for (lr, gr), (la, ga), mx in zip(ref, alone, mixed):
        assert la == lr and np.array_equal(ga, gr)
        for k in (0, 2):
            st, l, g, _ = mx[k]
            assert st == B.PG_OK
            assert l == la and np.array_equal(g, ga)


def test_served_result_matches_oracle(gpu):
    from paper_1905_12146_amd.serving import Server
    w = make_workload("C3", seed=7, n_tips=150, n_patterns=600)
    with Server(0, B.PG_FP32, 4 << 30, 8) as srv:
        sid = srv.open(w)
        st, logL, grad, lat = srv.wait(srv.submit(sid, w.t), len(w.t))
        srv.close(sid)
    assert st == B.PG_OK and lat > 0
    lin = O.linear_gradient(*args_of(w))
    rep = O.parity_report(logL, grad, lin["logL"], lin["grad"], lin["abs_grad"], 1e-5)
    print("served FP32 vs oracle", rep, flush=True)
    assert rep["ok"], rep


def test_split_sessions_alone_equal_mixed_and_oracle(gpu):
    """Split-BF16 sessions (61-state codon models and a 4-state one): each
    request's result is bitwise the same alone, batched with the others and
    from a single context, and meets the oracle at the path's 1e-5."""
    from paper_1905_12146_amd.serving import Server
    ws = [make_workload("C4", seed=300 + i, n_tips=n, n_patterns=s) for i, (n, s) in
          enumerate([(40, 120), (97, 61), (16, 300), (3, 9)])]
    ws.append(make_workload("C1", seed=310, n_tips=50, n_patterns=77, n_cats=2))
    ref = [_single(w, B.PG_SPLIT_BF16) for w in ws]
    with Server(0, B.PG_SPLIT_BF16, 8 << 30, 16) as srv:
        alone = []
        for w in ws:
            sid = srv.open(w)
            st, l, g, _ = srv.wait(srv.submit(sid, w.t), len(w.t))
            assert st == B.PG_OK
            alone.append((l, g))
            srv.close(sid)
        sids = [srv.open(w) for w in ws]
        tickets = [[srv.submit(sid, w.t * f) for f in (1.0, 0.7)] for sid, w in zip(sids, ws)]
        mixed = [[srv.wait(tk, len(w.t)) for tk in tks] for tks, w in zip(tickets, ws)]
        stats = srv.stats()
        for sid in sids:
            srv.close(sid)
    assert stats["max_batch"] >= 2, stats
    for (lr, gr), (la, ga), mx, w in zip(ref, alone, mixed, ws):
        assert la == lr and np.array_equal(ga, gr)
        st, l, g, _ = mx[0]
        assert st == B.PG_OK and l == la and np.array_equal(g, ga)
        lin = O.linear_gradient(*args_of(w))
        rep = O.parity_report(la, ga, lin["logL"], lin["grad"], lin["abs_grad"], 1e-5)
        print("served split vs oracle", w.n_tips, w.n_patterns, w.n_states, rep, flush=True)
        assert rep["ok"], rep


def test_admission_by_footprint(gpu):
    from paper_1905_12146_amd.serving import Server
    ws = [make_workload("C3", seed=200 + i, n_tips=400, n_patterns=800, tips="uniform") for i in range(6)]
    fp = B.pg_footprint_bytes(400, 800, 4, 4, B.PG_FP32)
    budget = int(2.5 * fp)          # room for two sessions at a time
    with Server(0, B.PG_FP32, budget, 64) as srv:
        sids = [srv.open(w) for w in ws]
        tickets = [srv.submit(s, w.t) for s, w in zip(sids, ws)]
        for s in sids:
            srv.close(s)
        out = [srv.wait(tk, len(w.t)) for tk, w in zip(tickets, ws)]
        stats = srv.stats()
    assert all(o[0] == B.PG_OK for o in out)
    assert stats["max_waiting"] >= 1, stats
    assert stats["peak_bytes"] <= budget, stats
    assert 0 < stats["peak_held"] <= budget, stats   # pool blocks in use plus cached
    assert stats["admitted_total"] == 6


def test_errors(gpu):
    from paper_1905_12146_amd.serving import Server
    w = make_workload("C3", seed=9, n_tips=300, n_patterns=700, tips="uniform")
    fp = B.pg_footprint_bytes(300, 700, 4, 4, B.PG_FP32)
    with Server(0, B.PG_FP32, fp // 2, 4) as srv:
        with pytest.raises(B.PhyloGradError) as e:
            srv.open(w)
        assert e.value.code == B.PG_E_OOM
    with Server(0, B.PG_FP32, 4 << 30, 4) as srv:
        with pytest.raises(B.PhyloGradError) as e:
            srv.submit(12345, w.t)
        assert e.value.code == B.PG_E_STATE
        sid = srv.open(w)
        bad = w.t.copy()
        bad[0] = np.nan
        with pytest.raises(B.PhyloGradError) as e:
            srv.submit(sid, bad)
        assert e.value.code == B.PG_E_INVALID
        srv.close(sid)


def test_stream_of_requests(gpu):
    """A short Poisson stream through the driver: every request completes and
    its first call equals the single-context result."""
    from paper_1905_12146_amd.serving import Server, run_stream
    from synth import serving_requests
    from synth.workloads import request_workload
    specs = serving_requests(12, qps=200.0, seed=3, n_tips_range=(100, 600), n_patterns_range=(200, 900))
    ws = [request_workload(s) for s in specs]
    with Server(0, B.PG_FP32, 8 << 30, 8) as srv:
        res = run_stream(srv, specs, ws, calls=3)
    assert not res["errors"], res["errors"]
    assert res["completed"] == 12 and res["calls"] == 36
    for w, out in zip(ws[:3], res["results"][:3]):
        l, g = _single(w, B.PG_FP32)
        assert out[0][0] == l and np.array_equal(out[0][1], g)


def test_failed_upload_wakes_waiting_caller(gpu):
    """A session whose device buffers cannot be allocated (about 2 TB in
    FP64) fails its queued calls with PG_E_OOM, and a thread already blocked
    in pg_server_wait on one of them wakes up."""
    import threading

    from paper_1905_12146_amd.serving import Server
    small_w = make_workload("C3", seed=11, n_tips=50, n_patterns=64, tips="uniform")
    N, S, m, K = 1000, 100_000, 20, 64
    huge = make_workload("C3", seed=12, n_tips=N, n_patterns=16, tips="uniform")
    masks = np.full((N, S), (1 << m) - 1, dtype=np.uint64)  # every tip missing
    Q = np.full((m, m), 1.0 / (m - 1))
    np.fill_diagonal(Q, -1.0)
    with Server(0, B.PG_FP64, 1 << 42, 1) as srv:
        first = srv.open(small_w)              # holds the only session slot
        st, _, _, _ = srv.wait(srv.submit(first, small_w.t), len(small_w.t))
        assert st == B.PG_OK
        sid = B.pg_server_open(srv.handle, huge.parent, masks, np.ones(S), Q, np.full(m, 1.0 / m),
                               np.ones(K), np.full(K, 1.0 / K))
        tk = srv.submit(sid, huge.t)
        out = {}
        waiter = threading.Thread(target=lambda: out.update(r=srv.wait(tk, len(huge.t))), daemon=True)
        waiter.start()
        srv.close(first)                       # admits the huge session, whose upload fails
        waiter.join(timeout=60)
        assert not waiter.is_alive(), "the waiting caller was not woken"
        assert out["r"][0] == B.PG_E_OOM, out
        with pytest.raises(B.PhyloGradError) as e:   # the server closed it
            srv.close(sid)
        assert e.value.code == B.PG_E_STATE
        ok = srv.open(small_w)                 # the server keeps serving
        st, _, _, _ = srv.wait(srv.submit(ok, small_w.t), len(small_w.t))
        assert st == B.PG_OK
        srv.close(ok)
