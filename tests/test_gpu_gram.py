"""GPU tests of the Gram form of the polar factor (PSVT_FLAG_GRAM), through
the C ABI: tall and wide low-rank-plus-noise inputs (both sides) and a
constructed spectrum with tau mid-range against the oracle (FP32: 1e-3;
with the BF16 sign schedule: 1e-2); the device-described batched forms
(per-stage and persistent) bitwise against single calls; the status word."""
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


def _host(torch, Y):
    torch.cuda.synchronize()
    return Y.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("shape,rank", [((1024, 128), 24), ((128, 1024), 24), ((2000, 250), 60),
                                        ((4096, 512), 100)])
@pytest.mark.parametrize("sched,tol", [(dict(), 1e-3), (dict(n_bf16=18), 1e-2)], ids=["fp32", "bf16S"])
def test_gram_form_low_rank_plus_noise(gpu_lib, tdev, shape, rank, sched, tol):
    torch, dev = tdev
    m, n = shape
    pb = inputs.noisy_lowrank(m, n, rank=rank, idx=3, norm_iters=60)
    _announce("gram %s r=%d %s" % (shape, rank, sched))
    A = torch.from_numpy(pb.A).to(dev)
    Y = _host(torch, gpu_lib.svt(A, pb.tau, iters=20, flags=gpu_lib.FLAG_GRAM, **sched))
    ref = oracle.svt(pb.A.astype(np.float64), pb.tau)
    err = oracle.rel_fro_err(Y, ref)
    std = oracle.rel_fro_err(_host(torch, gpu_lib.svt(A, pb.tau, iters=20, **sched)), ref)
    print("gram %s %s: %.3e (standard form %.3e)" % (shape, sched, err, std))
    assert err <= tol


@pytest.mark.parametrize("q,tol", [(0.1, 1e-3), (0.5, 1e-4), (0.9, 1e-4)])
@pytest.mark.parametrize("m,n", [(900, 150), (150, 900), (2000, 400)])
def test_gram_form_constructed_spectrum(gpu_lib, tdev, m, n, q, tol):
    """sigma log-spaced 10 .. 1e-3, tau at the 10 / 50 / 90 % quantile
    (sigma_max / tau about 4000, 100, 3)."""
    torch, dev = tdev
    pb = inputs.square_case(q, idx=5, n=n, m=m)
    _announce("gram constructed %dx%d q=%.1f" % (m, n, q))
    A = torch.from_numpy(pb.A).to(dev)
    Y = _host(torch, gpu_lib.svt(A, pb.tau, iters=20, flags=gpu_lib.FLAG_GRAM))
    err = oracle.rel_fro_err(Y, oracle.svt_from_svd(pb.U, pb.sigma, pb.V, pb.tau))
    print("gram constructed %dx%d q=%.1f: %.3e" % (m, n, q, err))
    assert err <= tol


def test_gram_form_batched_and_status(gpu_lib, tdev):
    torch, dev = tdev
    pbs = inputs.batch_cases(count=8, idx=41, lo=40, hi=400)
    _announce("gram batched %s" % [p.shape for p in pbs])
    As = [torch.from_numpy(p.A).to(dev) for p in pbs]
    taus = [p.tau for p in pbs]
    flags = gpu_lib.FLAG_GRAM
    staged = gpu_lib.svt_batched(As, taus, iters=20, flags=flags)
    gpu_lib.persistent_tiles(True)
    try:
        pers = gpu_lib.svt_batched(As, taus, iters=20, flags=flags, persistent=True)
        for A, t, Z in zip(As, taus, pers):
            ref = gpu_lib.svt(A, t, iters=20, flags=flags)
            torch.cuda.synchronize()
            assert torch.equal(Z, ref)
    finally:
        gpu_lib.persistent_tiles(False)
    for A, t, Z in zip(As, taus, staged):
        ref = gpu_lib.svt(A, t, iters=20, flags=flags)
        torch.cuda.synchronize()
        assert torch.equal(Z, ref)
    st = torch.full((1,), -1, dtype=torch.int32, device=dev)
    gpu_lib.svt(As[0], taus[0], iters=20, flags=flags, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0


def test_gram_form_rejected_outside_svt(gpu_lib, tdev):
    torch, dev = tdev
    A = torch.randn(64, 32, device=dev)
    with pytest.raises(gpu_lib.PsvtError):
        gpu_lib.rank_r(A, 0.1, flags=gpu_lib.FLAG_GRAM)
    with pytest.raises(gpu_lib.PsvtError):
        gpu_lib.polar(A, flags=gpu_lib.FLAG_GRAM)
    with pytest.raises(gpu_lib.PsvtError):
        gpu_lib.svt(A, 0.1, flags=gpu_lib.FLAG_GRAM | gpu_lib.FLAG_HFORM)
