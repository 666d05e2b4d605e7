"""FP64 CPU oracle for singular value soft-thresholding.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library and never calls it; the GPU library never calls it.

Every quantity is the plain definition written out on top of an SVD computed
by the one-sided Jacobi routine in ``jacobi.c`` (FP64):

* ``svt(A, tau)``      -- A_tau = U max(Sigma - tau I, 0) V^T, the operator of
                          section 2, Eq. (1).
* ``polar(A)``         -- P = U V^T, the polar factor (section 2).  For a
                          rank-deficient A, the partial isometry sum over
                          sigma_j > 0 of u_j v_j^T (the limit of the matmul
                          iterations; it is what the method uses).
* ``polar_sym(G)``     -- polar of a symmetric matrix = sign of its eigenvalues
                          (section 2), obtained by the same routine: for
                          G = Q Lambda Q^T the SVD has U V^T = Q sign(Lambda) Q^T.
                          Exact-zero eigenvalues map to 0.
* ``rank_r(A, tau)``   -- best rank-r approximation, the sum over sigma_j > tau
                          of sigma_j u_j v_j^T (Corollary 1, with the threshold
                          tau strictly between sigma_{r+1} and sigma_r).
* ``svt_from_svd``     -- Eq. (1) for factors already known (constructed
                          spectra): no SVD is computed.
* ``svt_gapped``       -- Eq. (1) for large low-rank-plus-noise inputs, by the
                          Jacobi SVD of a compressed matrix whose range holds
                          every singular vector above tau (checked).

Inputs are widened to float64 before anything else; callers hand in exactly
the FP32 matrix the GPU sees.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jacobi.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile ``liboracle.so`` with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_svd.restype = ctypes.c_int
        lib.oracle_svd.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def threads() -> int:
    """OpenMP threads the oracle uses."""
    return int(_load().oracle_threads())


def svd(A, nthreads: int = 0):
    """Thin SVD A = U diag(s) V^T by one-sided Jacobi in FP64.

    Returns (U, s, V) with s descending; U is m x k, V is n x k, k = min(m, n).
    A wide input is handled through its transpose (A^T = V diag(s) U^T).
    """
    A = np.asarray(A, dtype=np.float64)
    if A.ndim != 2:
        raise ValueError("input must be 2-D")
    m, n = A.shape
    if m == 0 or n == 0:
        k = min(m, n)
        return np.zeros((m, k)), np.zeros(k), np.zeros((n, k))
    if m < n:
        V, s, U = svd(A.T, nthreads)
        return U, s, V
    A = np.ascontiguousarray(A)
    U = np.empty((m, n))
    s = np.empty(n)
    V = np.empty((n, n))
    rc = _load().oracle_svd(m, n, A.ctypes.data, n, U.ctypes.data, s.ctypes.data, V.ctypes.data, int(nthreads))
    if rc < 0:
        raise RuntimeError("oracle_svd failed with code %d" % rc)
    return U, s, V


def svt_from_svd(U, s, V, tau):
    """Eq. (1): U max(Sigma - tau I, 0) V^T for given factors (FP64)."""
    U = np.asarray(U, np.float64)
    V = np.asarray(V, np.float64)
    s = np.asarray(s, np.float64)
    return (U * np.maximum(s - tau, 0.0)) @ V.T


def svt(A, tau, nthreads: int = 0):
    """A_tau of section 2, Eq. (1), via the Jacobi SVD."""
    if tau < 0:
        raise ValueError("tau must be >= 0")
    U, s, V = svd(A, nthreads)
    return svt_from_svd(U, s, V, tau)


def polar(A, nthreads: int = 0):
    """Polar factor U V^T (section 2); partial isometry over sigma > 0."""
    U, s, V = svd(A, nthreads)
    keep = (s > 0).astype(np.float64)
    return (U * keep) @ V.T


def polar_sym(G, nthreads: int = 0):
    """Matrix sign of a symmetric G: Q sign(Lambda) Q^T (section 2).

    The input is symmetrised as (G + G^T)/2 first.  Through the SVD,
    G = U diag(s) V^T with u_j = sign(lambda_j) v_j, so U V^T is the sign.
    """
    G = np.asarray(G, np.float64)
    if G.ndim != 2 or G.shape[0] != G.shape[1]:
        raise ValueError("polar_sym needs a square matrix")
    G = 0.5 * (G + G.T)
    return polar(G, nthreads)


def rank_r(A, tau, nthreads: int = 0):
    """Best rank-r approximation (Corollary 1): keep sigma_j > tau."""
    U, s, V = svd(A, nthreads)
    keep = np.where(s > tau, s, 0.0)
    return (U * keep) @ V.T


def svt_gapped(A, tau, k, power_iters=6, seed=0, nthreads: int = 0):
    """Eq. (1) for a large matrix whose singular values above tau are few and
    separated by a wide gap from the rest (low-rank signal plus noise, tau =
    2 ||N||_2), computed on a compressed matrix:

      Q = orthonormal basis of (A A^T)^q A Omega  (Omega: n x k Gaussian),
      B = Q^T A (k x n),  A_tau = Q (B)_tau  with (B)_tau by the Jacobi SVD.

    Exact when range(Q) contains the left singular vectors of every
    sigma > tau and the rest of A, (I - Q Q^T) A, has spectral norm <= tau;
    the power steps make the first hold to working precision for a gapped
    spectrum, and the second is checked (RuntimeError otherwise).  k must
    exceed the number of singular values above tau."""
    A = np.asarray(A, np.float64)
    m, n = A.shape
    if m < n:
        return svt_gapped(A.T, tau, k, power_iters, seed, nthreads).T
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(A @ rng.standard_normal((n, k)))
    for _ in range(power_iters):
        Q, _ = np.linalg.qr(A @ (A.T @ Q))
    B = Q.T @ A
    R = A - Q @ B
    x = rng.standard_normal(n)
    for _ in range(50):  # ||R||_2 by power iteration (an underestimate: pad 5%)
        x = R.T @ (R @ x)
        x /= np.linalg.norm(x)
    rnorm = float(np.linalg.norm(R @ x))
    if rnorm * 1.05 > tau:
        raise RuntimeError("residual %.3g not below tau %.3g: increase k" % (rnorm, tau))
    return Q @ svt(B, tau, nthreads)


def rel_fro_err(approx, exact, A=None):
    """Relative Frobenius error of the numerical experiments (section 3,
    Fig. 1 caption).  When the exact result is 0 (tau >= sigma_max) the
    error is taken relative to ||A||_F instead, if A is given."""
    approx = np.asarray(approx, np.float64)
    exact = np.asarray(exact, np.float64)
    num = np.linalg.norm(approx - exact)
    den = np.linalg.norm(exact)
    if den == 0.0:
        den = np.linalg.norm(np.asarray(A, np.float64)) if A is not None else 1.0
        if den == 0.0:
            den = 1.0
    return float(num / den)
