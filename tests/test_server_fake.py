"""Scheduling logic of the solve server on the host-only backend (no GPU):
admission in arrival order within the HBM budget and the slot count, exact
step counts, isolation of a failing request, latency bookkeeping."""
import threading

import numpy as np
import pytest

from paper_1903_01168_amd import capi
from paper_1903_01168_amd import serve
from paper_1903_01168_amd import workloads as W


def _req(n=64, **kw):
    return W.params(nx=n, ny=n, A=1e-3, **kw)


def _disk(n):
    return serve.init_disk(n / 2, n / 2, n / 4, 1.0, 0.0, 0.0, 1.0)


def _bytes(p):
    import ctypes as C
    return capi.load().lbm_bytes_required(C.byref(capi.make_params(p)))


def test_all_requests_complete_with_exact_steps():
    with serve.Server(1 << 30, max_slots=4, chunk_steps=10, fake_mlups=100.0) as s:
        ids = [s.enqueue(_req(64 + 64 * (k % 3)), _disk(64), steps) for k, steps in
               enumerate([0, 1, 9, 10, 11, 99, 1000, 37])]
        res = [s.wait(i) for i in ids]
        for r, steps in zip(res, [0, 1, 9, 10, 11, 99, 1000, 37]):
            assert r["status"] == capi.LBM_OK and r["steps_done"] == steps
            assert r["t_arrive"] <= r["t_admit"] <= r["t_done"]
        st = s.stats()
        assert st["completed"] == 8 and st["failed"] == 0 and st["peak_active"] <= 4


def test_admission_in_arrival_order_within_budget():
    p = _req(128)
    b = _bytes(p)
    budget = int(2.5 * b)               # room for two lattices at a time
    with serve.Server(budget, max_slots=8, chunk_steps=4, fake_mlups=50.0) as s:
        ids = [s.enqueue(p, _disk(128), 20 + 7 * k) for k in range(12)]
        res = [s.wait(i) for i in ids]
        st = s.stats()
        assert st["peak_bytes"] <= budget and st["peak_active"] <= 2
        admits = [r["t_admit"] for r in res]
        assert admits == sorted(admits)             # nobody overtakes the head of the queue
        assert all(r["status"] == capi.LBM_OK for r in res)


def test_small_requests_wait_behind_a_large_head():
    small, big = _req(64), _req(512)
    budget = _bytes(big) + _bytes(small)
    with serve.Server(budget, max_slots=8, chunk_steps=10, fake_mlups=10.0) as s:
        first = s.enqueue(small, _disk(64), 5000)
        head = s.enqueue(big, _disk(512), 10)
        tail = [s.enqueue(small, _disk(64), 10) for _ in range(3)]
        r_head = s.wait(head)
        r_tail = [s.wait(t) for t in tail]
        s.wait(first)
        assert all(rt["t_admit"] >= r_head["t_admit"] for rt in r_tail)


def test_request_larger_than_budget_is_rejected_not_blocking():
    p = _req(64)
    with serve.Server(_bytes(p) * 2, max_slots=4, chunk_steps=10, fake_mlups=10.0) as s:
        huge = s.enqueue(_req(1024), _disk(1024), 10)
        ok = s.enqueue(p, _disk(64), 10)
        assert s.wait(huge)["status"] == capi.LBM_E_NOMEM
        assert s.wait(ok)["status"] == capi.LBM_OK


def test_failure_is_isolated():
    # the victim asks for far more steps than can run before the injection
    # lands, so the outcome does not depend on thread timing
    with serve.Server(1 << 30, max_slots=8, chunk_steps=10, fake_mlups=1.0) as s:
        steps = [2000, 2000, 10 ** 12, 2000, 2000]
        ids = [s.enqueue(_req(64), _disk(64), n) for n in steps]
        s.inject_failure(ids[2])
        res = [s.wait(i) for i in ids]
        assert res[2]["status"] == capi.LBM_E_UNSTABLE and res[2]["steps_done"] < 10 ** 12
        for k in (0, 1, 3, 4):
            assert res[k]["status"] == capi.LBM_OK and res[k]["steps_done"] == 2000
        assert s.stats()["failed"] == 1


def test_invalid_request_rejected_at_enqueue():
    with serve.Server(1 << 30, max_slots=2, chunk_steps=10, fake_mlups=10.0) as s:
        with pytest.raises(capi.LbmError) as e:
            s.enqueue(_req(64, tau_r=0.4), _disk(64), 10)
        assert e.value.code == capi.LBM_E_INVAL
        with pytest.raises(capi.LbmError):
            s.enqueue(_req(64), serve.init_bands([5, 10], 1.0, 1.0), 10)
        assert s.poll(123456)["rc"] == capi.LBM_E_NOTFOUND


def test_concurrent_enqueue_from_threads():
    out = []
    lock = threading.Lock()
    with serve.Server(1 << 30, max_slots=16, chunk_steps=8, fake_mlups=100.0) as s:
        def client(k):
            ids = [s.enqueue(_req(64), _disk(64), 10 + k + j) for j in range(20)]
            res = [(i, s.wait(i)) for i in ids]
            with lock:
                out.extend(res)
        th = [threading.Thread(target=client, args=(k,)) for k in range(6)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        assert len(out) == 120 and len({i for i, _ in out}) == 120
        assert all(r["status"] == capi.LBM_OK for _, r in out)
        assert s.stats()["completed"] == 120


def test_poll_busy_then_done_and_release():
    with serve.Server(1 << 30, max_slots=1, chunk_steps=2, fake_mlups=1e-3) as s:
        a = s.enqueue(_req(64), _disk(64), 4)
        b = s.enqueue(_req(64), _disk(64), 4)
        r = s.poll(b)
        assert r["rc"] in (capi.LBM_E_BUSY, capi.LBM_OK)
        s.wait(a)
        assert s.wait(b)["status"] == capi.LBM_OK
        assert s.release(b) == capi.LBM_OK
        assert s.poll(b)["rc"] == capi.LBM_E_NOTFOUND


def test_virtual_latency_reflects_queueing():
    # one slot, identical requests: they run one after the other, each for
    # exactly its own cost on the virtual clock
    with serve.Server(1 << 30, max_slots=1, chunk_steps=10, fake_mlups=1.0) as s:
        ids = [s.enqueue(_req(64), _disk(64), 100) for _ in range(4)]
        res = [s.wait(i) for i in ids]
        per = 64 * 64 * 100 / 1e6
        for r in res:
            assert r["t_done"] - r["t_admit"] == pytest.approx(per, rel=1e-9)
        for a, b in zip(res, res[1:]):
            assert b["t_admit"] >= a["t_done"] - 1e-12
