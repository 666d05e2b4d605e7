"""GPU test on the workload of the paper's Fig. 2: an i.i.d. Gaussian
m x (m+1) matrix (left-sided), 25 iterations, tau mid-spectrum."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2607_22484_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m", [300, 1000])
def test_gaussian_m_by_m_plus_1(gpu_lib, m):
    import torch
    print("[gpu-case] fig2 m=%d" % m, flush=True)
    sys.stdout.flush()
    A = inputs.gaussian(m, m + 1, cfg=inputs.CFG_FIG2, idx=0)
    tau = math.sqrt(m)
    ref = oracle.svt(A, tau)
    Ad = torch.from_numpy(A).to("cuda:0")
    got = {}
    for name, kw, tol in [("fp32", {}, 1e-3), ("bf16", {"n_bf16": 23}, 1e-2)]:
        Y = gpu_lib.svt(Ad, tau, iters=25, **kw)
        torch.cuda.synchronize()
        got[name] = oracle.rel_fro_err(Y.cpu().numpy().astype(np.float64), ref)
        assert got[name] <= tol, (name, got[name])
    print("fig2 m=%d rel err %s" % (m, got))
