"""psvt_svt_noalloc (static device scratch, no device allocation) against
psvt_svt with a caller workspace, through the C ABI: bitwise equal results
(the same kernels on the same plan), on two calls in a row with the second
one smaller, for FP32 and the low-precision schedules up to the scratch's
largest size; and within the tolerance of the oracle."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_2607_22484_amd import inputs

pytestmark = pytest.mark.gpu


def _announce(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


def _via_c_abi(psvt, torch, A, tau, cfg):
    """One psvt_svt_noalloc call through ctypes, on the current stream."""
    m, n = A.shape
    Y = torch.full((m, n), float("nan"), device=A.device)
    stream = ctypes.c_void_p(torch.cuda.current_stream(A.device).cuda_stream)
    rc = psvt.load().psvt_svt_noalloc(A.data_ptr(), m, n, A.stride(0), float(tau), Y.data_ptr(), Y.stride(0),
                                      ctypes.byref(cfg), stream)
    assert rc == psvt.PSVT_OK, psvt.load().psvt_last_error()
    return Y


@pytest.mark.parametrize("sched", [dict(), dict(n_bf16=18), dict(n_fp8=6, n_bf16=12)], ids=["fp32", "bf16", "fp8"])
def test_noalloc_equals_workspace_entry_point(gpu_lib, sched):
    import torch
    dev = torch.device("cuda:0")
    cfg, keep = gpu_lib.make_config(iters=20, **sched)
    if not sched:
        cases = [inputs.small_case(), inputs.square_case(0.5, n=160, m=224)]   # second call smaller
    elif "n_fp8" in sched:   # the FP8 schedule's input class: low rank + noise (psvt.h)
        cases = [inputs.noisy_lowrank(1024, 1024, rank=64, idx=3, cfg=inputs.CFG_TEST),
                 inputs.noisy_lowrank(300, 200, rank=16, idx=4, cfg=inputs.CFG_TEST)]
    else:
        cases = [inputs.square_case(0.5, n=1024), inputs.small_case()]      # the scratch's largest size first
    for pb in cases:
        _announce("noalloc %s %s" % (sched, pb.A.shape))
        A = torch.from_numpy(pb.A).to(dev)
        Y = _via_c_abi(gpu_lib, torch, A, pb.tau, cfg)
        ref = gpu_lib.svt(A, pb.tau, iters=20, **sched)
        torch.cuda.synchronize()
        assert torch.equal(Y, ref)
        Yh = Y.cpu().numpy().astype(np.float64)
        if pb.U is not None:
            err = oracle.rel_fro_err(Yh, oracle.svt_from_svd(pb.U, pb.sigma, pb.V, pb.tau))
        else:
            exact, cert = oracle.svt_gapped(pb.A, pb.tau, k=pb.rank + 64, return_bound=True)
            err = oracle.rel_fro_err(Yh, exact) + cert
        assert err <= (1e-3 if not sched else 1e-2), err
    del keep


def test_noalloc_python_wrapper_and_status(gpu_lib):
    import torch
    dev = torch.device("cuda:0")
    pb = inputs.small_case(idx=3)
    A = torch.from_numpy(pb.A).to(dev)
    st = torch.full((1,), -1, dtype=torch.int32, device=dev)
    _announce("noalloc wrapper")
    Y = gpu_lib.svt_noalloc(A, pb.tau, status=st)
    assert torch.equal(Y, gpu_lib.svt(A, pb.tau))
    torch.cuda.synchronize()
    assert int(st.item()) == 0
