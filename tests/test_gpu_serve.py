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
