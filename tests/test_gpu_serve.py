"""GPU tests of the serving loop: requests of mixed sizes run concurrently
(continuous batching) and each result equals the same request run alone,
and the single-call result; parity with the oracle at the serving schedule."""
import sys
import time

import numpy as np
import pytest

import oracle
from paper_2607_22484_amd import inputs

pytestmark = pytest.mark.gpu

SCHED = dict(iters=20, n_fp8=6, n_bf16=12)


def _announce(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tdev(gpu_lib):
    import torch
    return torch, torch.device("cuda:0")


def _requests(count, idx):
    shapes = inputs.serve_shapes(count, idx=idx, lo=64, hi=400)
    return [inputs.noisy_lowrank(m, n, rank=r, idx=100 + k, cfg=inputs.CFG_SERVE) for k, (m, n, r) in
            enumerate(shapes)]


@pytest.mark.parametrize("cohort", [False, True])
def test_mix_equals_alone_and_oracle(gpu_lib, tdev, cohort):
    torch, dev = tdev
    pbs = _requests(10, idx=1)
    _announce("serve mix cohort=%s %s" % (cohort, [p.shape for p in pbs]))
    As = [torch.from_numpy(p.A).to(dev) for p in pbs]
    srv = gpu_lib.Server(budget_bytes=1 << 30, max_slots=16, cohort=cohort, **SCHED)
    tickets = []
    for A, p in zip(As, pbs):
        tickets.append(srv.submit(A, p.tau))
        time.sleep(0.0005)  # staggered arrivals: later requests join running ones
    srv.drain(timeout=120)
    mix = [Y.cpu().numpy() for _, Y in tickets]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(pbs) and st["failed"] == 0
    alone_srv = gpu_lib.Server(budget_bytes=1 << 30, max_slots=1, **SCHED)
    worst = 0.0
    for A, p, Ym in zip(As, pbs, mix):
        t, Y = alone_srv.submit(A, p.tau)
        assert alone_srv.wait(t, timeout=60) == gpu_lib.RQ_DONE
        Ya = Y.cpu().numpy()
        assert np.array_equal(Ya, Ym), p.name            # alone == in the mix
        Ys = gpu_lib.svt(A, p.tau, **SCHED).cpu().numpy()
        assert np.array_equal(Ys, Ym), p.name            # == single call
        err = oracle.rel_fro_err(Ym.astype(np.float64), oracle.svt(p.A, p.tau))
        worst = max(worst, err)
    alone_srv.close()
    print("serving schedule worst rel err vs oracle %.3e" % worst)
    assert worst <= 1e-2


def test_budget_admission_on_device(gpu_lib, tdev):
    """A budget with room for two requests: everything completes, the pool
    peak stays within the budget."""
    torch, dev = tdev
    pbs = _requests(6, idx=2)
    _announce("serve budget")
    need = max(gpu_lib.workspace_bytes(gpu_lib.OP_SVT, *p.shape, gpu_lib.make_config(**SCHED)[0]) for p in pbs)
    budget = 2 * ((need + 255) // 256 * 256)
    srv = gpu_lib.Server(budget_bytes=budget, max_slots=8, **SCHED)
    outs = [srv.submit(torch.from_numpy(p.A).to(dev), p.tau) for p in pbs]
    srv.drain(timeout=120)
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(pbs) and st["peak_bytes"] <= budget
    for (_, Y), p in zip(outs, pbs):
        assert oracle.rel_fro_err(Y.cpu().numpy().astype(np.float64), oracle.svt(p.A, p.tau)) <= 1e-2


def test_submit_is_ordered_after_the_callers_stream(gpu_lib, tdev):
    """A request submitted right after in-stream work that writes its input
    (no synchronisation in between) reads the written input: the server
    waits for an event recorded on the caller's stream at submit.  The
    caller's stream is kept busy first, so an unordered read would see the
    stale contents (zeros)."""
    torch, dev = tdev
    pb = inputs.noisy_lowrank(384, 256, rank=16, idx=7, cfg=inputs.CFG_SERVE)
    _announce("serve submit ordering")
    src = torch.from_numpy(pb.A).to(dev)
    single = gpu_lib.svt(src, pb.tau, **SCHED)
    torch.cuda.synchronize()
    srv = gpu_lib.Server(budget_bytes=1 << 30, max_slots=4, **SCHED)
    for trial in range(3):
        A = torch.zeros_like(src)
        big = torch.randn(4096, 4096, device=dev)
        torch.cuda.synchronize()
        for _ in range(8):                # ~ tens of ms of queued work on the caller's stream
            big = big @ big
            big = big / big.norm()
        A.copy_(src)                      # the input is written only after that work
        t, Y = srv.submit(A, pb.tau)      # no synchronisation
        assert srv.wait(t, timeout=60) == gpu_lib.RQ_DONE
        torch.cuda.synchronize()
        assert torch.equal(Y, single), trial
    srv.close()
