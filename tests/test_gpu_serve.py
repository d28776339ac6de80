"""Continuous-batching server: every request's result is the same alone and in
the mix, equal to the oracle; admission by budget; error and cancel paths."""
import sys
import threading

import numpy as np
import pytest
import torch

import oracle
from tests.libtq import ensure_built
from workloads import datagen

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stderr.flush()


@pytest.fixture(scope="module")
def tq():
    return ensure_built()


@pytest.fixture(scope="module")
def env(tq):
    o = oracle.default()
    w = datagen.WORKLOADS["small"]
    X = datagen.rows("small", datagen.DB, 0, w["n"]).numpy()
    Q = datagen.rows("small", datagen.QUERIES, 0, 300).numpy()
    V, VQ = o.encode(X, w["x"]), o.encode(Q, w["x"])
    db = tq.tq_db_create(torch.from_numpy(o.pack(V).view(np.int32).copy()).cuda(), w["d"], w["x"])
    ei10, es10 = o.knn(VQ, V, 10)
    ei100, es100 = o.knn(VQ, V, 100)
    yield dict(db=db, CQ=o.pack(VQ), oracle={10: (ei10, es10), 100: (ei100, es100)}, W=db.W)
    db.destroy()


def make_requests(seed, count, max_size=32):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        while True:
            nq = int(rng.geometric(1 / 8))
            if nq <= max_size:
                break
        q0 = int(rng.integers(0, 300 - nq + 1))
        out.append((q0, nq, int(rng.choice([10, 100]))))
    return out


def check(env, req, res):
    q0, nq, k = req
    ids, sc, _ = res
    ei, es = env["oracle"][k]
    assert np.array_equal(ids, ei[q0:q0 + nq]) and np.array_equal(sc, es[q0:q0 + nq]), req


@pytest.mark.parametrize("segments", [1, 3, 7])
def test_alone_and_in_the_mix(tq, env, segments):
    reqs = make_requests(segments, 40)
    srv = tq.tq_server(env["db"], max_k=100, n_segments=segments)
    say(f"serve alone, segments={segments}")
    alone = []
    for (q0, nq, k) in reqs:
        t = srv.submit(env["CQ"][q0:q0 + nq], k)
        alone.append(srv.wait(t, 20000))
    say(f"serve mix from 4 threads, segments={segments}")
    tickets = [None] * len(reqs)

    def submitter(part):
        for i in range(part, len(reqs), 4):
            q0, nq, k = reqs[i]
            tickets[i] = srv.submit(env["CQ"][q0:q0 + nq], k)

    th = [threading.Thread(target=submitter, args=(p,)) for p in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    mix = [srv.wait(t, 20000) for t in tickets]
    st = srv.stats()
    srv.destroy()
    for req, a, m in zip(reqs, alone, mix):
        assert a is not None and m is not None
        assert np.array_equal(a[0], m[0]) and np.array_equal(a[1], m[1]), req
        check(env, req, a)
        assert a[2].ticks == segments and m[2].ticks == segments
    for r in alone + mix:
        assert r[2].complete_ns >= r[2].admit_ns >= r[2].submit_ns
    assert st["completed"] == 2 * len(reqs) and st["bytes_in_use"] == 0


def test_budget_admission(tq, env):
    W, nc = env["W"], (env["W"] + 3) // 4
    per_query = (2 * W + 16 * nc) * 4 + 100 * 16
    srv = tq.tq_server(env["db"], max_k=100, n_segments=2, budget_bytes=per_query * 5)
    say("serve budget: oversize request rejected")
    with pytest.raises(tq.TQError) as e:
        srv.submit(env["CQ"][:6], 10)
    assert e.value.status == tq.TQ_ERR_INVALID
    say("serve budget: one request at a time")
    reqs = [(5 * i, 5, 10 if i % 2 else 100) for i in range(12)]
    tickets = [srv.submit(env["CQ"][q0:q0 + nq], k) for (q0, nq, k) in reqs]
    for req, t in zip(reqs, tickets):
        check(env, req, srv.wait(t, 20000))
    srv.destroy()


def test_error_paths(tq, env):
    srv = tq.tq_server(env["db"], max_k=50, max_request_nq=16, n_segments=2)
    say("serve error paths")
    with pytest.raises(tq.TQError):
        srv.submit(env["CQ"][:4], 51)  # k above max_k
    with pytest.raises(tq.TQError):
        srv.submit(env["CQ"][:17], 10)  # nq above max_request_nq
    with pytest.raises(tq.TQError) as e:
        srv.poll(987654321)
    assert e.value.status == tq.TQ_ERR_NOTFOUND
    t = srv.submit(env["CQ"][:3], 10)
    r = srv.wait(t, 20000)
    check(env, (0, 3, 10), r)
    with pytest.raises(tq.TQError) as e:
        srv.poll(t)  # already collected
    assert e.value.status == tq.TQ_ERR_NOTFOUND
    srv.destroy()


def test_cancel(tq, env):
    srv = tq.tq_server(env["db"], max_k=100, n_segments=4, max_slots=64)
    reqs = make_requests(99, 30)
    say("serve cancel")
    tickets = [srv.submit(env["CQ"][q0:q0 + nq], k) for (q0, nq, k) in reqs]
    cancelled = set(range(0, 30, 3))
    for i in cancelled:
        srv.cancel(tickets[i])  # pending, active or finished: all are dropped
    for i, (req, t) in enumerate(zip(reqs, tickets)):
        if i in cancelled:
            with pytest.raises(tq.TQError) as e:
                srv.poll(t)
            assert e.value.status == tq.TQ_ERR_NOTFOUND
        else:
            check(env, req, srv.wait(t, 20000))
    srv.destroy()


def test_destroy_with_work_in_flight(tq, env):
    srv = tq.tq_server(env["db"], max_k=100, n_segments=3, max_slots=128)
    say("serve destroy with pending work")
    for (q0, nq, k) in make_requests(5, 60):
        srv.submit(env["CQ"][q0:q0 + nq], k)
    srv.destroy()


def test_watchdog_stops_the_server(tq, env):
    """A watchdog of 1 us: no tick can finish that fast, so the first wait
    for a tick gives up, the server stops and its requests report
    TQ_ERR_DEVICE with the watchdog's reason; the GPU work itself finishes
    normally and the database serves a new server afterwards."""
    say("serving watchdog of 1 us")
    srv = tq.tq_server(env["db"], max_k=100, tick_timeout_us=1)
    tickets = [srv.submit(env["CQ"][i * 5:i * 5 + 5], 10) for i in range(3)]
    tripped = 0
    for i, t in enumerate(tickets):
        try:
            res = srv.wait(t, 60000)
        except tq.TQError as e:
            assert e.status == tq.TQ_ERR_DEVICE and "watchdog" in str(e), str(e)
            tripped += 1
        else:  # a tick whose event had already fired when first checked
            check(env, (i * 5, 5, 10), res)
    assert tripped >= 1
    with pytest.raises(tq.TQError) as e:
        srv.submit(env["CQ"][:2], 10)
    assert e.value.status == tq.TQ_ERR_STATE
    srv.destroy()
    say("a generous watchdog lets the same requests through")
    srv = tq.tq_server(env["db"], max_k=100, tick_timeout_us=10_000_000)
    for i in range(3):
        check(env, (i * 5, 5, 10), srv.wait(srv.submit(env["CQ"][i * 5:i * 5 + 5], 10), 60000))
    srv.destroy()


def test_device_limit_gives_nomem(tq, env):
    """tq_set_device_limit: creating a database or a server that would take
    the library's device memory past the limit fails with TQ_ERR_NOMEM and
    holds nothing more; lifting the limit makes the same calls succeed."""
    o = oracle.default()
    rng = np.random.default_rng(5)
    d, x = 256, 64
    V = o.encode(rng.standard_normal((5000, d)).astype(np.float32), x)
    codes = torch.from_numpy(o.pack(V).view(np.int32).copy()).cuda()
    held = tq.tq_device_bytes()
    try:
        say("device limit: database that does not fit")
        tq.tq_set_device_limit(held + 4096)
        with pytest.raises(tq.TQError) as e:
            tq.tq_db_create(codes, d, x)
        assert e.value.status == tq.TQ_ERR_NOMEM
        assert tq.tq_device_bytes() == held
        say("device limit: server that does not fit")
        with pytest.raises(tq.TQError) as e:
            tq.tq_server(env["db"], max_k=100, max_slots=4096)
        assert e.value.status == tq.TQ_ERR_NOMEM
        assert tq.tq_device_bytes() == held
    finally:
        tq.tq_set_device_limit(0)
    say("device limit lifted")
    db = tq.tq_db_create(codes, d, x)
    assert tq.tq_device_bytes() > held
    ids, sc = tq.tq_search_knn(db, codes[:3], 5, path=tq.TQ_PATH_PLAIN)
    torch.cuda.synchronize()
    ei, es = o.knn(V[:3], V, 5)
    assert np.array_equal(ids.cpu().numpy(), ei) and np.array_equal(sc.cpu().numpy(), es)
    db.destroy()
    srv = tq.tq_server(env["db"], max_k=100)
    check(env, (0, 4, 100), srv.wait(srv.submit(env["CQ"][:4], 100), 60000))
    srv.destroy()


@pytest.mark.parametrize("engine", ["popcount", "matrix"])
def test_pinned_engine_mix(tq, env, engine):
    """A server pinned to one engine gives the oracle's rows for a mix of
    requests submitted from four threads (k = 10 and 100, 1-32 queries)."""
    eng = tq.TQ_ENGINE_POPCOUNT if engine == "popcount" else tq.TQ_ENGINE_MATRIX
    reqs = make_requests(17, 40)
    srv = tq.tq_server(env["db"], max_k=100, n_segments=2, engine=eng)
    say(f"serve mix on the {engine} engine")
    tickets = [None] * len(reqs)

    def submitter(part):
        for i in range(part, len(reqs), 4):
            q0, nq, k = reqs[i]
            tickets[i] = srv.submit(env["CQ"][q0:q0 + nq], k)

    th = [threading.Thread(target=submitter, args=(p,)) for p in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for req, t in zip(reqs, tickets):
        check(env, req, srv.wait(t, 20000))
    srv.destroy()
    with pytest.raises(tq.TQError):
        tq.tq_server(env["db"], max_k=100, engine=tq.TQ_ENGINE_SPARSE)
