"""Scheduling logic of the serving loop on the CPU (simulated executor):
completion of every request, footprint admission, coalescing limits, and
oldest-first service.  The GPU execution of the same loop is in
test_gpu_serving.py."""

import time

import pytest

from paper_2406_09144_amd.serving import BATCHABLE, Server, latency_stats, make_trace


class SimExecutor:
    """Each launch 'runs' for a fixed time per image and costs a fixed footprint."""

    def __init__(self, per_image_s=2e-4, bytes_per_image=100, clock=time.perf_counter):
        self.per = per_image_s
        self.bpi = bytes_per_image
        self.clock = clock
        self.inflight_bytes = 0
        self.log = []

    def footprint(self, job, op, B):
        return self.bpi * B + (50 if op == "cg20" else 0)

    def launch(self, job, op, reqs, slot):
        B = sum(r.size for r in reqs)
        self.log.append((job, op, [r.rid for r in reqs], B, slot))
        return self.clock() + self.per * B

    def done(self, handle):
        return self.clock() >= handle


def test_trace_is_seeded_and_poisson_like():
    a = make_trace(8, 200.0, 2.0, seed=1)
    b = make_trace(8, 200.0, 2.0, seed=1)
    assert [(r.t_arrival, r.job, r.op, r.size) for r in a] == [(r.t_arrival, r.job, r.op, r.size) for r in b]
    assert 300 < len(a) < 500  # mean 400
    gaps = [y.t_arrival - x.t_arrival for x, y in zip(a, a[1:])]
    assert abs(sum(gaps) / len(gaps) - 1 / 200.0) < 1e-3


def test_all_requests_complete_with_budget_and_batch_limits():
    trace = make_trace(4, 2000.0, 0.1, seed=3)
    ex = SimExecutor()
    srv = Server(ex, n_slots=3, hbm_budget=1500, max_batch=8)
    out = srv.run(trace, realtime=False)
    assert all(r.t_done is not None and r.t_start is not None for r in out)
    assert all(r.t_done >= r.t_start >= 0 for r in out)
    assert srv.peak_bytes <= 1500
    for job, op, rids, B, slot in ex.log:
        if op not in BATCHABLE:
            assert len(rids) == 1
        assert B <= 8 or len(rids) == 1
        assert 0 <= slot < 3
    # every request launched exactly once
    launched = [rid for _, _, rids, _, _ in ex.log for rid in rids]
    assert sorted(launched) == sorted(r.rid for r in trace)
    st = latency_stats(out, from_release=True)
    assert st["p99_ms"] >= st["p50_ms"] > 0


def test_coalescing_groups_same_job_and_op():
    trace = make_trace(1, 1e5, 0.001, seed=4, mix={"psf_apply": 1.0})
    ex = SimExecutor(per_image_s=1e-3)
    srv = Server(ex, n_slots=1, hbm_budget=10 ** 9, max_batch=8)
    srv.run(trace, realtime=False)
    sizes = [len(rids) for _, _, rids, _, _ in ex.log]
    assert max(sizes) == 8 and sum(sizes) == len(trace)


def test_oldest_group_first():
    trace = make_trace(3, 1e5, 0.002, seed=5, mix={"degrid": 1.0})
    ex = SimExecutor()
    srv = Server(ex, n_slots=1, hbm_budget=10 ** 9)
    srv.run(trace, realtime=False)
    order = [rids[0] for _, _, rids, _, _ in ex.log]
    assert order == sorted(order)


def test_oversized_request_is_rejected():
    trace = make_trace(1, 1000.0, 0.01, seed=6, mix={"cg20": 1.0})
    srv = Server(SimExecutor(), n_slots=2, hbm_budget=100)
    with pytest.raises(RuntimeError):
        srv.run(trace, realtime=False)


def _req(rid, t, op="cg20", job=0, size=1, t_cancel=None):
    from paper_2406_09144_amd.serving import Request
    return Request(rid, t, job, op, size, t_cancel=t_cancel)


def test_request_cancelled_while_pending_is_never_launched_and_frees_nothing_twice():
    # one slot: the long request 0 holds it while 1 and 2 wait; both are cancelled
    # before the slot frees, so only 0 and 3 ever reach the executor
    ex = SimExecutor(per_image_s=0.05)
    srv = Server(ex, n_slots=1, hbm_budget=10_000, max_batch=8)
    trace = [_req(0, 0.0), _req(1, 0.001, t_cancel=0.01), _req(2, 0.001, "psf_apply", t_cancel=0.02),
             _req(3, 0.002)]
    out = srv.run(trace, realtime=True)
    launched = [rid for _, _, rids, _, _ in ex.log for rid in rids]
    assert launched == [0, 3]
    assert [r.cancelled for r in out] == [False, True, True, False]
    assert out[1].t_start is None and out[2].t_start is None
    assert out[1].t_done < out[0].t_done  # dropped at its cancel time, not after the slot freed
    assert sorted(srv.free_slots) == [0] and srv.bytes_in_flight == 0
    st = latency_stats(out)
    assert st["n"] == 2


def test_request_cancelled_on_the_device_frees_its_slot_when_the_launch_ends():
    ex = SimExecutor(per_image_s=0.03)
    srv = Server(ex, n_slots=1, hbm_budget=10_000, max_batch=8)
    trace = [_req(0, 0.0, t_cancel=0.005), _req(1, 0.001)]
    out = srv.run(trace, realtime=True)
    launched = [rid for _, _, rids, _, _ in ex.log for rid in rids]
    assert launched == [0, 1]
    assert out[0].cancelled and not out[1].cancelled
    assert out[1].t_start >= out[0].t_done  # the slot came back when the launch ended
    assert sorted(srv.free_slots) == [0] and srv.bytes_in_flight == 0


def test_cancel_from_another_thread():
    import threading
    ex = SimExecutor(per_image_s=0.05)
    srv = Server(ex, n_slots=1, hbm_budget=10_000, max_batch=8)
    trace = [_req(0, 0.0), _req(1, 0.0), _req(2, 0.0)]
    threading.Timer(0.01, lambda: srv.cancel(2)).start()
    out = srv.run(trace, realtime=True)
    launched = [rid for _, _, rids, _, _ in ex.log for rid in rids]
    assert launched == [0, 1] and out[2].cancelled


def test_overlap_stats_of_launch_intervals():
    from paper_2406_09144_amd.serving import overlap_stats
    st = overlap_stats([(0.0, 2.0), (1.0, 3.0), (5.0, 6.0)])
    assert st["launches"] == 3 and st["max_concurrent"] == 2
    assert abs(st["launch_ms_sum"] - 5.0) < 1e-12 and abs(st["busy_ms"] - 4.0) < 1e-12
    assert abs(st["concurrency"] - 1.25) < 1e-12
    # serial launches: no overlap
    st = overlap_stats([(0.0, 1.0), (1.0, 2.0)])
    assert st["max_concurrent"] == 1 and abs(st["concurrency"] - 1.0) < 1e-12
