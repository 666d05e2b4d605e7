"""Serving scheduler on the CPU (fake executor: stages complete at once).
Checks admission order, the memory budget, slot limits, failure handling and
statistics without a device.  Device pointers are fake and never touched."""
import time

import pytest

import paper_2607_22484_amd as psvt

FAKE_A = 1 << 40
FAKE_Y = 1 << 41


def submit(srv, m, n, tau=0.1):
    return srv.submit_ptr(FAKE_A, FAKE_Y, m, n, n, n, tau)


def test_fake_server_completes_everything():
    srv = psvt.Server(budget_bytes=1 << 30, max_slots=8, fake=True)
    tickets = [submit(srv, 64 + 16 * i, 48 + 8 * i) for i in range(40)]
    srv.drain(timeout=30)
    for t in tickets:
        assert srv.poll(t) == psvt.RQ_DONE
    st = srv.stats()
    assert st["submitted"] == 40 and st["completed"] == 40 and st["failed"] == 0
    assert st["queued"] == 0 and st["active"] == 0
    assert st["p99_ms"] >= st["p50_ms"] >= 0.0
    assert st["ticks"] > 0 and st["launches"] > 0
    srv.close()


def test_mixed_sizes_over_all_lanes():
    """Requests from 64^2 to 4096 x 2048 fall into all four size lanes (s^2 l
    in factors of 8 from 512^3), each lane running its own ticks: every
    request completes."""
    srv = psvt.Server(budget_bytes=64 << 30, max_slots=64, fake=True)
    shapes = [(4096, 2048), (2048, 2048), (1024, 1024), (512, 512), (64, 64)] * 6
    tickets = [submit(srv, m, n) for m, n in shapes]
    srv.drain(timeout=60)
    assert all(srv.poll(t) == psvt.RQ_DONE for t in tickets)
    st = srv.stats()
    assert st["completed"] == len(shapes) and st["failed"] == 0
    srv.close()


@pytest.mark.parametrize("room", [1, 2])
def test_budget_limits_concurrency(room):
    """With room for exactly one or two requests at a time, peak pool use
    never exceeds the budget and every request still completes.  (The fake
    executor finishes stages at once, so how many requests overlap depends
    on thread timing; only the upper bound is deterministic.)"""
    need = psvt.workspace_bytes(psvt.OP_SVT, 256, 256)
    budget = room * ((need + 255) // 256 * 256) + 1024
    srv = psvt.Server(budget_bytes=budget, max_slots=16, fake=True)
    tickets = [submit(srv, 256, 256) for _ in range(10)]
    srv.drain(timeout=30)
    st = srv.stats()
    assert st["completed"] == 10
    assert need <= st["peak_bytes"] <= budget
    assert all(srv.poll(t) == psvt.RQ_DONE for t in tickets)
    srv.close()


def test_request_larger_than_budget_is_rejected():
    srv = psvt.Server(budget_bytes=1 << 20, max_slots=4, fake=True)
    with pytest.raises(psvt.PsvtError) as e:
        submit(srv, 4096, 4096)
    assert e.value.code == psvt.PSVT_EWORKSPACE
    t = submit(srv, 32, 32)  # a small one still fits
    assert srv.wait(t, timeout=10) == psvt.RQ_DONE
    srv.close()


def test_bad_requests_and_arguments():
    srv = psvt.Server(budget_bytes=1 << 26, max_slots=2, fake=True)
    for m, n, tau in [(0, 5, 0.1), (5, 0, 0.1), (8, 8, -1.0), (8, 8, float("nan"))]:
        with pytest.raises(psvt.PsvtError):
            srv.submit_ptr(FAKE_A, FAKE_Y, m, n, max(n, 1), max(n, 1), tau)
    with pytest.raises(psvt.PsvtError):
        srv.poll(12345)
    srv.close()
    lib = psvt.load()
    import ctypes
    h = ctypes.c_void_p()
    assert lib.psvt_server_create(100, 4, None, psvt.SERVER_FAKE, ctypes.byref(h)) == psvt.PSVT_EINVAL
    assert lib.psvt_server_create(1 << 20, 0, None, psvt.SERVER_FAKE, ctypes.byref(h)) == psvt.PSVT_EINVAL
    assert lib.psvt_server_create(1 << 20, 4, None, 0x80, ctypes.byref(h)) == psvt.PSVT_EINVAL


def test_fifo_admission_no_overtaking():
    """A large request at the head of the queue is not overtaken by smaller
    ones that would fit: admission is in arrival order."""
    big = psvt.workspace_bytes(psvt.OP_SVT, 512, 512)
    small = psvt.workspace_bytes(psvt.OP_SVT, 32, 32)
    budget = (big + 255) // 256 * 256 + 2 * ((small + 255) // 256 * 256)
    srv = psvt.Server(budget_bytes=budget, max_slots=8, fake=True)
    ts = [submit(srv, 32, 32), submit(srv, 512, 512), submit(srv, 32, 32), submit(srv, 32, 32)]
    srv.drain(timeout=30)
    assert all(srv.poll(t) == psvt.RQ_DONE for t in ts)
    assert srv.stats()["peak_bytes"] <= budget
    srv.close()


def test_threads_submitting_concurrently():
    import threading
    srv = psvt.Server(budget_bytes=1 << 30, max_slots=32, fake=True)
    out = []

    def client(k):
        for i in range(25):
            out.append(submit(srv, 32 + k, 40 + i))
    th = [threading.Thread(target=client, args=(k,)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    srv.drain(timeout=30)
    assert len(set(out)) == 100
    assert srv.stats()["completed"] == 100
    srv.close()


def test_cohort_admission_completes_everything():
    """Cohort admission (the default): requests admitted while their lane
    runs a started cohort wait for it and then start together; everything
    completes, in every lane, and bad flag sets are rejected."""
    srv = psvt.Server(budget_bytes=64 << 30, max_slots=64, fake=True, cohort=True)
    shapes = [(4096, 2048), (2048, 2048), (1024, 1024), (512, 512), (64, 64)] * 4
    tickets = []
    for i, (m, n) in enumerate(shapes):
        tickets.append(submit(srv, m, n))
        if i % 5 == 4:
            time.sleep(0.002)  # later arrivals meet running cohorts
    srv.drain(timeout=60)
    assert all(srv.poll(t) == psvt.RQ_DONE for t in tickets)
    st = srv.stats()
    assert st["completed"] == len(shapes) and st["failed"] == 0 and st["active"] == 0
    srv.close()
    lib = psvt.load()
    import ctypes
    h = ctypes.c_void_p()
    assert lib.psvt_server_create(1 << 20, 4, None, 0x8, ctypes.byref(h)) == psvt.PSVT_EINVAL
    assert lib.psvt_server_create(1 << 20, 4, None, psvt.SERVER_COHORT | psvt.SERVER_EAGER,
                                  ctypes.byref(h)) == psvt.PSVT_EINVAL


def test_eager_admission_completes_everything():
    srv = psvt.Server(budget_bytes=64 << 30, max_slots=64, fake=True, cohort=False)
    shapes = [(2048, 1024), (512, 512), (64, 64)] * 4
    tickets = [submit(srv, m, n) for m, n in shapes]
    srv.drain(timeout=60)
    assert all(srv.poll(t) == psvt.RQ_DONE for t in tickets)
    srv.close()


@pytest.mark.parametrize("cohort", [True, False])
def test_many_same_lane_requests_share_ticks(cohort):
    """1200 requests of one size class, all admitted at once (more than one
    tick's descriptor segment can describe): ticks take them in rotation,
    every request completes and none fails."""
    srv = psvt.Server(budget_bytes=64 << 30, max_slots=2000, fake=True, cohort=cohort)
    tickets = [submit(srv, 96, 64) for _ in range(1200)]
    srv.drain(timeout=120)
    st = srv.stats()
    assert st["completed"] == 1200 and st["failed"] == 0
    assert all(srv.poll(t) == psvt.RQ_DONE for t in tickets)
    srv.close()


def test_status_flag_rejected_for_served_requests():
    """The status word is one per call: a server config asking for it is
    rejected at creation."""
    import ctypes
    cfg, _ = psvt.make_config(status=1 << 40)
    h = ctypes.c_void_p()
    assert psvt.load().psvt_server_create(1 << 30, 4, ctypes.byref(cfg), psvt.SERVER_FAKE,
                                          ctypes.byref(h)) == psvt.PSVT_EINVAL


def test_planning_failure_fails_only_its_request():
    """Fault injection: the 4th admission's plan fails; only that request
    fails, every other one completes."""
    srv = psvt.Server(budget_bytes=1 << 30, max_slots=8, fake=True)
    srv.inject_fault(psvt.FAULT_PLAN, 3)
    tickets = [submit(srv, 64 + 8 * i, 48) for i in range(10)]
    srv.drain(timeout=30)
    states = [srv.poll(t) for t in tickets]
    assert states[3] == psvt.RQ_FAILED
    assert all(s == psvt.RQ_DONE for i, s in enumerate(states) if i != 3)
    st = srv.stats()
    assert st["failed"] == 1 and st["completed"] == 9 and st["timed_out"] == 0
    srv.close()


def test_launch_failure_fails_its_tick_only():
    """Fault injection: the first tick fails as a launch error would.  The
    requests of that tick fail; requests of the other lanes and requests
    submitted afterwards complete; the workspaces all return to the pool
    (a budget that holds one large request at a time still serves them)."""
    srv = psvt.Server(budget_bytes=1 << 30, max_slots=64, fake=True)
    srv.inject_fault(psvt.FAULT_TICK, 0)
    small = [submit(srv, 64, 48) for _ in range(3)]
    with pytest.raises(psvt.PsvtError, match="launch failed"):
        srv.drain(timeout=30)        # reports the injected launch error ...
    big = [submit(srv, 2048, 1024), submit(srv, 4096, 2048)]   # other lanes
    later = [submit(srv, 64, 48) for _ in range(3)]
    with pytest.raises(psvt.PsvtError):
        srv.drain(timeout=30)
    first = [srv.poll(t) for t in small]
    assert first.count(psvt.RQ_FAILED) >= 1
    assert all(srv.poll(t) == psvt.RQ_DONE for t in big + later)   # ... which stayed with its tick
    st = srv.stats()
    assert st["failed"] == first.count(psvt.RQ_FAILED)
    assert st["active"] == 0 and st["queued"] == 0
    srv.close()
    # one slot of budget: failed requests' workspaces must come back
    budget = 4 * psvt.workspace_bytes(psvt.OP_SVT, 256, 192, psvt.make_config()[0])
    srv = psvt.Server(budget_bytes=budget, max_slots=64, fake=True)
    srv.inject_fault(psvt.FAULT_TICK, 1)
    ts = [submit(srv, 256, 192) for _ in range(12)]
    with pytest.raises(psvt.PsvtError):
        srv.drain(timeout=30)
    assert all(srv.poll(t) in (psvt.RQ_DONE, psvt.RQ_FAILED) for t in ts)
    assert srv.stats()["completed"] >= 8
    srv.close()


def test_deadline_fails_stalled_requests_and_frees_their_memory():
    """Fault injection: fake ticks stall.  With a 0.2 s deadline the running
    and the queued requests fail (timed_out), their memory returns to the
    pool, and after the stall clears new requests complete."""
    budget = 2 * psvt.workspace_bytes(psvt.OP_SVT, 256, 192, psvt.make_config()[0])
    srv = psvt.Server(budget_bytes=budget, max_slots=8, fake=True)
    srv.inject_fault(psvt.FAULT_STALL, 1)
    srv.set_timeout(0.2)
    ts = [submit(srv, 256, 192) for _ in range(5)]   # two run, three wait for memory
    t0 = time.time()
    for t in ts:
        assert srv.wait(t, timeout=10) == psvt.RQ_FAILED
    assert time.time() - t0 < 5
    st = srv.stats()
    assert st["timed_out"] == 5 and st["failed"] == 5 and st["active"] == 0 and st["queued"] == 0
    srv.inject_fault(psvt.FAULT_STALL, 0)
    srv.set_timeout(0)
    ok = [submit(srv, 256, 192) for _ in range(4)]
    srv.drain(timeout=30)
    assert all(srv.poll(t) == psvt.RQ_DONE for t in ok)
    assert srv.stats()["peak_bytes"] <= budget
    srv.close()


def test_fault_injection_is_for_fake_servers_and_checks_arguments():
    srv = psvt.Server(budget_bytes=1 << 30, max_slots=4, fake=True)
    with pytest.raises(psvt.PsvtError):
        srv.inject_fault(99, 0)
    with pytest.raises(psvt.PsvtError):
        srv.set_timeout(-1.0)
    srv.close()


def test_concurrent_clients_with_faults_and_deadlines():
    """Several client threads submit, poll and wait while ticks fail now and
    then and a deadline is set: every request ends done or failed, the
    counters add up, and destroy joins cleanly (also the stress run of the
    thread-sanitizer build)."""
    import threading
    srv = psvt.Server(budget_bytes=1 << 28, max_slots=16, fake=True)
    srv.inject_fault(psvt.FAULT_TICK, 7)
    srv.set_timeout(5.0)
    tickets = []
    lock = threading.Lock()

    def client(k):
        for i in range(40):
            t = submit(srv, 32 + 7 * k + i, 24 + 3 * i)
            with lock:
                tickets.append(t)
            if i % 5 == 0:
                srv.wait(t, timeout=5)
            else:
                srv.poll(t)
    th = [threading.Thread(target=client, args=(k,)) for k in range(6)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    try:
        srv.drain(timeout=30)
    except psvt.PsvtError:
        pass
    states = [srv.poll(t) for t in tickets]
    assert all(s in (psvt.RQ_DONE, psvt.RQ_FAILED) for s in states)
    st = srv.stats()
    assert st["completed"] + st["failed"] == len(tickets) == 240
    srv.close()
