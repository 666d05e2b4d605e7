"""GPU tests of psvt_svt_batched / psvt_rank_r_batched (device descriptor
array, no allocation, no host read of the shapes), through the C ABI:

* uneven shapes of both sides: bitwise equal to single calls (FP32 and
  low-precision schedules), and within the tolerance of the oracle;
* capture into a HIP graph, replayed with eager work between replays and
  with the descriptors and inputs changed on the device in between: every
  replay equals the single calls on the current contents;
* descriptors outside the maxima or malformed are skipped (Y untouched,
  PSVT_STATUS_INVALID) while the others complete; status words of converged
  matrices read 0."""
import sys

import numpy as np
import pytest

import oracle
from paper_2607_22484_amd import inputs

pytestmark = pytest.mark.gpu


def _announce(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tdev(gpu_lib):
    import torch
    return torch, torch.device("cuda:0")


def _cases(count, lo, hi, idx):
    return inputs.batch_cases(count=count, idx=idx, lo=lo, hi=hi)


@pytest.mark.parametrize("sched", [dict(), dict(n_bf16=18), dict(n_fp8=6, n_bf16=12)], ids=["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("op", [0, 3], ids=["svt", "rank_r"])
def test_batched_desc_equals_single_calls(gpu_lib, tdev, sched, op):
    torch, dev = tdev
    pbs = _cases(14, 17, 300, idx=21)
    _announce("batched desc %s op=%d %s" % (sched, op, [p.shape for p in pbs]))
    As = [torch.from_numpy(p.A).to(dev) for p in pbs]
    taus = [p.tau for p in pbs]
    Ys = gpu_lib.svt_batched(As, taus, iters=20, op=op, **sched)
    single = gpu_lib.svt if op == 0 else gpu_lib.rank_r
    for A, t, Y, p in zip(As, taus, Ys, pbs):
        ref = single(A, t, iters=20, **sched)
        torch.cuda.synchronize()
        assert torch.equal(Y, ref), p.name
    if op == 0 and not sched:
        worst = max(oracle.rel_fro_err(Y.cpu().numpy().astype(np.float64),
                                       oracle.svt_from_svd(p.U, p.sigma, p.V, p.tau)) for Y, p in zip(Ys, pbs))
        assert worst <= 1e-3


def test_batched_desc_graph_capture_and_replay(gpu_lib, tdev):
    """The call is captured into a graph once; between replays the inputs
    are overwritten and two descriptors are exchanged on the device (the host
    never sees the shapes): each replay equals single calls on the current
    descriptors."""
    torch, dev = tdev
    pbs = _cases(6, 40, 200, idx=22)
    _announce("batched desc graph %s" % [p.shape for p in pbs])
    As = [torch.from_numpy(p.A).to(dev) for p in pbs]
    taus = [p.tau for p in pbs]
    Ys = [torch.zeros_like(A) for A in As]
    cfg, keep = gpu_lib.make_config(iters=20, n_bf16=18)
    max_m = max(A.shape[0] for A in As)
    max_n = max(A.shape[1] for A in As)
    ws = torch.empty(gpu_lib.batched_workspace_bytes(len(As), max_m, max_n, cfg), dtype=torch.uint8, device=dev)
    desc = gpu_lib.device_descriptors(As, taus, Ys)
    desc_alt = gpu_lib.device_descriptors([As[1], As[0]] + As[2:], [taus[1], taus[0]] + taus[2:],
                                          [Ys[1], Ys[0]] + Ys[2:])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):       # warm-up outside the capture (first launches load code objects)
        gpu_lib.svt_batched_raw(desc.data_ptr(), len(As), max_m, max_n, ws, cfg)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gpu_lib.svt_batched_raw(desc.data_ptr(), len(As), max_m, max_n, ws, cfg)
    rng = np.random.default_rng(5)
    for rep in range(4):
        for A in As:                 # new inputs, written eagerly between replays
            A.mul_(float(rng.uniform(0.5, 2.0)))
        if rep == 2:                 # exchange the first two descriptors on the device
            desc.copy_(desc_alt)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        cur = [(As[1], taus[1], Ys[1]), (As[0], taus[0], Ys[0])] if rep >= 2 else [(As[0], taus[0], Ys[0]),
                                                                                    (As[1], taus[1], Ys[1])]
        for A, t, Y in cur + list(zip(As[2:], taus[2:], Ys[2:])):
            ref = gpu_lib.svt(A, t, iters=20, n_bf16=18)
            torch.cuda.synchronize()
            assert torch.equal(Y, ref), rep
    del keep


def test_batched_desc_invalid_and_status(gpu_lib, tdev):
    torch, dev = tdev
    pbs = _cases(5, 32, 160, idx=23)
    _announce("batched desc invalid/status")
    As = [torch.from_numpy(p.A).to(dev) for p in pbs]
    taus = [p.tau for p in pbs]
    max_m = max(A.shape[0] for A in As)
    max_n = max(A.shape[1] for A in As)
    big = torch.from_numpy(inputs.small_case().A).to(dev)       # 256 x 128: beyond the maxima below
    As2 = As + [big]
    taus2 = taus + [0.1]
    Ys = [torch.full_like(A, 7.0) for A in As2]
    st = torch.full((len(As2),), -1, dtype=torch.int32, device=dev)
    statuses = [st[i:i + 1] for i in range(len(As2))]
    taus2[1] = -1.0                                               # malformed: negative tau
    gpu_lib.svt_batched(As2, taus2, iters=20, outs=Ys, statuses=statuses, max_m=max(max_m, 129), max_n=max_n)
    torch.cuda.synchronize()
    words = [int(x) & 0xFFFFFFFF for x in st.cpu().tolist()]
    assert words[1] == gpu_lib.STATUS_INVALID and words[-1] == gpu_lib.STATUS_INVALID
    assert bool((Ys[1] == 7.0).all()) and bool((Ys[-1] == 7.0).all())
    for i in (0, 2, 3, 4):
        assert words[i] == 0
        ref = gpu_lib.svt(As2[i], taus2[i], iters=20)
        torch.cuda.synchronize()
        assert torch.equal(Ys[i], ref)


def test_batched_desc_fullsize_recipe(gpu_lib, tdev):
    """All 512 matrices of the batched recipe (m, n log-uniform in
    [128, 2048]) in one device-described call with the default BF16
    schedule: each against its construction (1e-2) and a sample bitwise
    against single calls."""
    torch, dev = tdev
    pbs = inputs.batch_cases(count=512)
    _announce("batched desc 512")
    As = [torch.from_numpy(p.A).to(dev) for p in pbs]
    taus = [p.tau for p in pbs]
    Ys = gpu_lib.svt_batched(As, taus, iters=20, n_bf16=18)
    for k in (0, 100, 511):
        ref = gpu_lib.svt(As[k], taus[k], iters=20, n_bf16=18)
        torch.cuda.synchronize()
        assert torch.equal(Ys[k], ref)
    worst = 0.0
    for Y, p in zip(Ys, pbs):
        ref = oracle.svt_from_svd(p.U, p.sigma, p.V, p.tau)
        worst = max(worst, float(np.linalg.norm(Y.cpu().numpy().astype(np.float64) - ref) / np.linalg.norm(ref)))
    print("batched desc 512 worst %.3e" % worst)
    assert worst <= 1e-2
