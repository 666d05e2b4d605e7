"""GPU tests on the workload of the paper's Fig. 1 (an i.i.d. Gaussian
301 x 300 matrix): error against the number of polar iterations."""
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
def fig1(gpu_lib):
    import torch
    A = inputs.gaussian(301, 300, cfg=inputs.CFG_FIG1)
    U, s, V = oracle.svd(A)
    # tau with a wide relative gap: the geometric midpoint of the most
    # separated neighbouring pair among the 30 smallest singular values
    low = s[-30:]
    j = int(np.argmax(low[:-1] / low[1:]))
    tau_gap = float(np.sqrt(low[j] * low[j + 1]))
    return torch, torch.from_numpy(A).to("cuda:0"), U, s, V, tau_gap


def _err(gpu_lib, fig1, tau, iters, **kw):
    torch, Ad, U, s, V, _ = fig1
    Y = gpu_lib.svt(Ad, tau, iters=iters, **kw)
    torch.cuda.synchronize()
    return oracle.rel_fro_err(Y.cpu().numpy().astype(np.float64), oracle.svt_from_svd(U, s, V, tau))


def test_gapped_tau_converges(gpu_lib, fig1):
    """With tau >= 5 % away from every singular value, 25 FP32 iterations
    reach 1e-3 and the BF16 schedule (23 BF16 + 2 FP32) 1e-2; the error
    falls steeply over the first iterations."""
    _, _, _, s, _, tau = fig1
    gap = float(np.min(np.abs(s / tau - 1.0)))
    _announce("fig1 gapped tau=%.4g gap=%.3f" % (tau, gap))
    assert gap >= 0.05
    errs = [_err(gpu_lib, fig1, tau, k) for k in (2, 6, 12, 25)]
    print("fig1 tau=%.4g fp32 err at 2/6/12/25 iterations: %s" % (tau, ["%.2e" % e for e in errs]))
    assert errs[-1] <= 1e-3
    assert errs[0] > errs[1] > errs[-1]
    eb = _err(gpu_lib, fig1, tau, 25, n_bf16=23)
    print("fig1 tau=%.4g bf16 schedule err %.2e" % (tau, eb))
    assert eb <= 1e-2


@pytest.mark.parametrize("tau", [1.0, 17.0, 33.0])
def test_error_falls_with_iterations(gpu_lib, fig1, tau):
    """Without a gap guarantee (tau inside the bulk of the spectrum) more
    iterations still never make the FP32 result worse than three do, and it
    stays finite."""
    _announce("fig1 tau=%g" % tau)
    e3, e25 = _err(gpu_lib, fig1, tau, 3), _err(gpu_lib, fig1, tau, 25)
    print("fig1 tau=%g fp32 err 3 its %.2e, 25 its %.2e" % (tau, e3, e25))
    assert np.isfinite(e25) and e25 <= e3
