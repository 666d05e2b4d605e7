"""GPU tests of the status word (PSVT_FLAG_STATUS) and of norm_safety,
through the C ABI: a converged call reports 0; too few iterations report
non-convergence (||S^2 - I||_F / sqrt(s) above the threshold); a non-finite
input reports both non-finite bits; norm_safety only rescales the start of
the iterations (same result within the tolerance)."""
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


def _status(torch, dev):
    return torch.full((1,), -1, dtype=torch.int32, device=dev)


def _word(st):
    import torch
    torch.cuda.synchronize()
    return int(st.cpu().item()) & 0xFFFFFFFF


@pytest.mark.parametrize("entry", ["svt", "rank_r", "polar", "polar_sym"])
def test_status_converged_is_zero(gpu_lib, tdev, entry):
    torch, dev = tdev
    _announce("status converged %s" % entry)
    pb = inputs.small_case()
    A = torch.from_numpy(pb.A).to(dev)
    st = _status(torch, dev)
    if entry == "svt":
        Y = gpu_lib.svt(A, pb.tau, status=st)
        ref = oracle.svt(pb.A, pb.tau)
    elif entry == "rank_r":
        Y = gpu_lib.rank_r(A, pb.tau, status=st)
        ref = oracle.rank_r(pb.A, pb.tau)
    elif entry == "polar":
        Y = gpu_lib.polar(A, status=st)
        ref = oracle.polar(pb.A)
    else:
        G = (pb.A.astype(np.float64).T @ pb.A - pb.tau ** 2 * np.eye(pb.A.shape[1])).astype(np.float32)
        Y = gpu_lib.polar_sym(torch.from_numpy(G).to(dev), status=st)
        ref = oracle.polar_sym(G)
    assert _word(st) == 0
    assert oracle.rel_fro_err(Y.cpu().numpy().astype(np.float64), ref) <= 1e-3
    # the status pass does not change the result
    Y0 = {"svt": lambda: gpu_lib.svt(A, pb.tau), "rank_r": lambda: gpu_lib.rank_r(A, pb.tau),
          "polar": lambda: gpu_lib.polar(A), "polar_sym": None}[entry]
    if Y0 is not None:
        assert torch.equal(Y0(), Y)


@pytest.mark.parametrize("iters", [2, 4])
def test_status_reports_non_convergence(gpu_lib, tdev, iters):
    """A few iterations leave the small eigenvalues of the shifted Gram
    unconverged (S^2 != I): the bit is set; with 20 it is clear."""
    torch, dev = tdev
    _announce("status not converged iters=%d" % iters)
    pb = inputs.small_case()
    A = torch.from_numpy(pb.A).to(dev)
    st = _status(torch, dev)
    gpu_lib.svt(A, pb.tau, iters=iters, status=st)
    assert _word(st) == gpu_lib.STATUS_NOT_CONVERGED
    gpu_lib.svt(A, pb.tau, iters=20, status=st)
    assert _word(st) == 0
    # a looser threshold accepts the short run
    gpu_lib.svt(A, pb.tau, iters=iters, status=st, status_tol=10.0)
    assert _word(st) == 0


def test_status_reports_non_finite_input(gpu_lib, tdev):
    torch, dev = tdev
    _announce("status non-finite")
    pb = inputs.small_case()
    Ah = pb.A.copy()
    Ah[17, 5] = np.nan
    A = torch.from_numpy(Ah).to(dev)
    st = _status(torch, dev)
    gpu_lib.svt(A, pb.tau, status=st)
    w = _word(st)
    assert w & gpu_lib.STATUS_NONFINITE_INPUT and w & gpu_lib.STATUS_NONFINITE_OUTPUT
    Ah[17, 5] = np.inf
    gpu_lib.polar(torch.from_numpy(Ah).to(dev), status=st)
    assert _word(st) & gpu_lib.STATUS_NONFINITE_INPUT


@pytest.mark.parametrize("safety", [1.0, 1.5, 4.0])
def test_norm_safety(gpu_lib, tdev, safety):
    """norm_safety divides the starting iterate by a larger bound: the
    result stays within 1e-3 of the oracle at 20 iterations (the schedule
    reaches a singular value 4x smaller within them)."""
    torch, dev = tdev
    _announce("norm_safety %g" % safety)
    pb = inputs.small_case()
    A = torch.from_numpy(pb.A).to(dev)
    Y = gpu_lib.svt(A, pb.tau, norm_safety=safety).cpu().numpy().astype(np.float64)
    assert oracle.rel_fro_err(Y, oracle.svt(pb.A, pb.tau)) <= 1e-3
