"""GPU tests of the persistent batched executor (PSVT_FLAG_PERSISTENT on
psvt_svt_batched / psvt_rank_r_batched), through the C ABI:

* uneven shapes of both sides, FP32 and low-precision schedules, svt and
  rank_r: bitwise equal to single calls made with the executor's tile set
  (psvt_tune_persistent_tiles), and to the per-stage batched form under the
  same tile set; the abort flag stays clear;
* captured into a HIP graph and replayed with new inputs between replays;
* descriptors beyond the maxima are skipped with PSVT_STATUS_INVALID;
* the abort path, forced from the host with a zero spin limit: the launch
  ends, and every matrix either matches its single call or is marked
  invalid;
* the batched recipe at full size (512 matrices, 128..2048) against its
  construction.
The schedule itself (ticket order, dependency counts, drain) is replayed on
the CPU by tests/test_persist_schedule.py."""
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


@pytest.fixture
def ptiles(gpu_lib):
    gpu_lib.persistent_tiles(True)
    yield
    gpu_lib.persistent_tiles(False)
    gpu_lib.spin_limit(1 << 22)


def _run(gpu_lib, torch, As, taus, op=0, outs=None, statuses=None, max_m=None, max_n=None, **sched):
    """One persistent call; returns (outputs, aborted)."""
    dev = As[0].device
    Ys = list(outs) if outs is not None else [torch.empty_like(A) for A in As]
    max_m = max_m or max(A.shape[0] for A in As)
    max_n = max_n or max(A.shape[1] for A in As)
    flags = sched.pop("flags", 0) | gpu_lib.FLAG_PERSISTENT
    if statuses is not None:
        flags |= gpu_lib.FLAG_STATUS
    cfg, keep = gpu_lib.make_config(flags=flags, **sched)
    ws = torch.empty(gpu_lib.batched_workspace_bytes(len(As), max_m, max_n, cfg, op), dtype=torch.uint8, device=dev)
    d = gpu_lib.device_descriptors(As, taus, Ys, statuses, dev)
    gpu_lib.svt_batched_raw(d.data_ptr(), len(As), max_m, max_n, ws, cfg, op)
    torch.cuda.synchronize()
    del keep
    return Ys, gpu_lib.persistent_aborted(ws)


@pytest.mark.parametrize("sched", [dict(), dict(n_bf16=18), dict(n_fp8=6, n_bf16=12),
                                   dict(n_bf16=18, flags=0x10)], ids=["fp32", "bf16", "fp8", "hform"])
@pytest.mark.parametrize("op", [0, 3], ids=["svt", "rank_r"])
def test_persistent_equals_single_calls(gpu_lib, tdev, ptiles, sched, op):
    torch, dev = tdev
    if op == 3 and sched.get("flags"):
        pytest.skip("the H-form applies to svt only")
    pbs = inputs.batch_cases(count=14, idx=31, lo=17, hi=300)
    _announce("persistent %s op=%d %s" % (sched, op, [p.shape for p in pbs]))
    As = [torch.from_numpy(p.A).to(dev) for p in pbs]
    taus = [p.tau for p in pbs]
    Ys, aborted = _run(gpu_lib, torch, As, taus, op=op, iters=20, **dict(sched))
    assert not aborted
    single = gpu_lib.svt if op == 0 else gpu_lib.rank_r
    staged = gpu_lib.svt_batched(As, taus, iters=20, op=op, **sched)   # per-stage form, same tile set
    for A, t, Y, Z, p in zip(As, taus, Ys, staged, pbs):
        ref = single(A, t, iters=20, **sched)
        torch.cuda.synchronize()
        assert torch.equal(Y, ref), p.name
        assert torch.equal(Z, ref), p.name
    if op == 0 and not sched:
        worst = max(oracle.rel_fro_err(Y.cpu().numpy().astype(np.float64),
                                       oracle.svt_from_svd(p.U, p.sigma, p.V, p.tau)) for Y, p in zip(Ys, pbs))
        assert worst <= 1e-3


def test_persistent_graph_capture_and_replay(gpu_lib, tdev, ptiles):
    torch, dev = tdev
    pbs = inputs.batch_cases(count=6, idx=32, lo=40, hi=200)
    _announce("persistent graph %s" % [p.shape for p in pbs])
    As = [torch.from_numpy(p.A).to(dev) for p in pbs]
    taus = [p.tau for p in pbs]
    Ys = [torch.zeros_like(A) for A in As]
    cfg, keep = gpu_lib.make_config(iters=20, n_bf16=18, flags=gpu_lib.FLAG_PERSISTENT)
    max_m = max(A.shape[0] for A in As)
    max_n = max(A.shape[1] for A in As)
    ws = torch.empty(gpu_lib.batched_workspace_bytes(len(As), max_m, max_n, cfg), dtype=torch.uint8, device=dev)
    desc = gpu_lib.device_descriptors(As, taus, Ys)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):       # warm-up outside the capture
        gpu_lib.svt_batched_raw(desc.data_ptr(), len(As), max_m, max_n, ws, cfg)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gpu_lib.svt_batched_raw(desc.data_ptr(), len(As), max_m, max_n, ws, cfg)
    rng = np.random.default_rng(6)
    for rep in range(3):
        for A in As:
            A.mul_(float(rng.uniform(0.5, 2.0)))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert not gpu_lib.persistent_aborted(ws)
        for A, t, Y in zip(As, taus, Ys):
            ref = gpu_lib.svt(A, t, iters=20, n_bf16=18)
            torch.cuda.synchronize()
            assert torch.equal(Y, ref), rep
    del keep


def test_persistent_invalid_descriptors(gpu_lib, tdev, ptiles):
    torch, dev = tdev
    pbs = inputs.batch_cases(count=5, idx=33, lo=32, hi=160)
    _announce("persistent invalid/status")
    As = [torch.from_numpy(p.A).to(dev) for p in pbs]
    taus = [p.tau for p in pbs]
    max_m = max(A.shape[0] for A in As)
    max_n = max(A.shape[1] for A in As)
    big = torch.from_numpy(inputs.small_case().A).to(dev)       # 256 x 128: beyond the maxima below
    As2 = As + [big]
    taus2 = taus + [0.1]
    taus2[1] = -1.0
    Ys = [torch.full_like(A, 7.0) for A in As2]
    st = torch.full((len(As2),), -1, dtype=torch.int32, device=dev)
    Ys, aborted = _run(gpu_lib, torch, As2, taus2, outs=Ys, statuses=[st[i:i + 1] for i in range(len(As2))],
                       max_m=max(max_m, 129), max_n=max_n, iters=20)
    assert not aborted
    words = [int(x) & 0xFFFFFFFF for x in st.cpu().tolist()]
    assert words[1] == gpu_lib.STATUS_INVALID and words[-1] == gpu_lib.STATUS_INVALID
    assert bool((Ys[1] == 7.0).all()) and bool((Ys[-1] == 7.0).all())
    for i in (0, 2, 3, 4):
        assert words[i] == 0
        ref = gpu_lib.svt(As2[i], taus2[i], iters=20)
        torch.cuda.synchronize()
        assert torch.equal(Ys[i], ref)


def test_persistent_abort_path_ends(gpu_lib, tdev, ptiles):
    """Spin limit 0 (set from the host): any wait not already satisfied
    aborts.  The launch still ends; matrices either match their single call
    or read PSVT_STATUS_INVALID."""
    torch, dev = tdev
    pbs = inputs.batch_cases(count=8, idx=34, lo=64, hi=256)
    _announce("persistent abort path")
    As = [torch.from_numpy(p.A).to(dev) for p in pbs]
    taus = [p.tau for p in pbs]
    st = torch.full((len(As),), -1, dtype=torch.int32, device=dev)
    gpu_lib.spin_limit(0)
    Ys, aborted = _run(gpu_lib, torch, As, taus, statuses=[st[i:i + 1] for i in range(len(As))], iters=20)
    gpu_lib.spin_limit(1 << 22)
    print("abort path: aborted=%s" % aborted)
    words = [int(x) & 0xFFFFFFFF for x in st.cpu().tolist()]
    for i, (A, t, Y) in enumerate(zip(As, taus, Ys)):
        if words[i] == gpu_lib.STATUS_INVALID:
            assert aborted
            continue
        assert words[i] == 0
        ref = gpu_lib.svt(A, t, iters=20)
        torch.cuda.synchronize()
        assert torch.equal(Y, ref)


def test_persistent_fullsize_recipe(gpu_lib, tdev, ptiles):
    """All 512 matrices of the batched recipe in one persistent launch with
    the default BF16 schedule: each against its construction (1e-2), a
    sample bitwise against single calls."""
    torch, dev = tdev
    pbs = inputs.batch_cases(count=512)
    _announce("persistent 512")
    As = [torch.from_numpy(p.A).to(dev) for p in pbs]
    taus = [p.tau for p in pbs]
    Ys, aborted = _run(gpu_lib, torch, As, taus, iters=20, n_bf16=18)
    assert not aborted
    for k in (0, 100, 511):
        ref = gpu_lib.svt(As[k], taus[k], iters=20, n_bf16=18)
        torch.cuda.synchronize()
        assert torch.equal(Ys[k], ref)
    worst = 0.0
    for Y, p in zip(Ys, pbs):
        ref = oracle.svt_from_svd(p.U, p.sigma, p.V, p.tau)
        worst = max(worst, float(np.linalg.norm(Y.cpu().numpy().astype(np.float64) - ref) / np.linalg.norm(ref)))
    print("persistent 512 worst %.3e" % worst)
    assert worst <= 1e-2
