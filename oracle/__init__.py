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
                          Jacobi SVD of a compressed matrix, accepted only
                          under a certified bound on its error.
* ``prox_error_bound`` -- a rigorous upper bound on ||Y - A_tau||_F for any
                          candidate Y, from the duality gap of the prox
                          problem whose solution A_tau is (section 2).

Inputs are widened to float64 before anything else; callers hand in exactly
the FP32 matrix the GPU sees.
"""
from __future__ import annotations

import ctypes
import math
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


def _gram_lambda_max_upper(F):
    """An upper bound on lambda_max(F^T F) = ||F||_2^2: LAPACK's largest
    eigenvalue of the computed Gram matrix C (the smaller of F^T F, F F^T)
    plus n u ||C||_F (the computed eigenvalues are those of C plus a
    perturbation of norm of order u ||C||_2; Weyl's inequality) plus
    l u ||F||_F^2 (rounding of the l-term sums that form C)."""
    C = F.T @ F if F.shape[0] >= F.shape[1] else F @ F.T
    nc = C.shape[0]
    if nc == 0:
        return 0.0
    u = float(np.finfo(np.float64).eps)
    return (max(float(np.linalg.eigvalsh(C)[-1]), 0.0) + nc * u * float(np.linalg.norm(C)) +
            max(F.shape) * u * float(np.sum(F * F)))


def prox_error_bound(A, Y, tau, factor=None):
    """Certified upper bound on ||Y - A_tau||_F for any candidate Y.

    A_tau is the proximal point of tau ||.||_* at A (section 2: the
    subroutine of nuclear-norm proximal methods), i.e. the minimiser of the
    1-strongly convex f(X) = ||X - A||_F^2 / 2 + tau ||X||_*, so
    ||Y - A_tau||_F^2 / 2 <= f(Y) - d(Z) for every dual-feasible Z.  The dual
    is d(Z) = <A, Z> - ||Z||_F^2 / 2 over ||Z||_2 <= tau (the spectral norm
    is the dual of the nuclear norm).  With M = A - Y and Z = c M,
    0 <= c <= 1, c ||M||_2 <= tau:

        f(Y) - d(cM) = tau ||Y||_* - c <Y, M> + (1 - c)^2 ||M||_F^2 / 2.

    Any upper bound on ||Y||_* and on ||M||_2 keeps the result an upper
    bound.  ||Y||_*: the singular values of Y (LAPACK), or, for
    factor = (Q, Z) with Y = Q Z and Q (nearly) orthonormal,
    sqrt(1 + ||Q^T Q - I||_2) ||Z||_*.  ||M||_2: the block form of M^T M in
    an orthonormal basis [W, W_perp], W = the right singular vectors of Y's
    nonzero part:

        lambda_max(M^T M) <= lambda_max([[alpha, beta], [beta, gamma]]),
        alpha = lambda_max(W^T M^T M W)          (small eigenproblem)
        beta  = ||W^T M^T M W_perp||_2            (small SVD)
        gamma = lambda_max(W_perp^T M^T M W_perp) = ||M W_perp W_perp^T||_2^2,
        each computed by LAPACK and raised by a bound on its rounding
        error (alpha: an SVD of M W; gamma: ``_gram_lambda_max_upper``),

    since x^T K x <= alpha |a|^2 + 2 beta |a||b| + gamma |b|^2 for
    x = W a + W_perp b.  It is tight when W spans the top right singular
    subspace of M (beta ~ 0, bound ~ alpha).  Returns (bound, parts)."""
    A = np.asarray(A, np.float64)
    Y = np.asarray(Y, np.float64)
    m, n = A.shape
    if m < n:
        f = None if factor is None else (factor[1].T, factor[0].T)
        if f is not None:
            raise ValueError("pass the tall orientation with a factor")
        return prox_error_bound(A.T, Y.T, tau)
    M = A - Y
    if factor is None:
        _, sy, Vyt = np.linalg.svd(Y, full_matrices=False)
        nuc = float(sy.sum())
    else:
        Q, Z = factor
        e = float(np.linalg.norm(Q.T @ Q - np.eye(Q.shape[1]), 2))
        _, sy, Vyt = np.linalg.svd(np.asarray(Z, np.float64), full_matrices=False)
        nuc = math.sqrt(1.0 + e) * float(sy.sum())
    keep = sy > sy[0] * 1e-13 if sy.size and sy[0] > 0 else np.zeros(sy.shape, bool)
    W = Vyt[keep].T
    u = float(np.finfo(np.float64).eps)
    if W.shape[1]:
        W, _ = np.linalg.qr(W)
        MW = M @ W
        # ||M W||_2 by an SVD of M W itself (backward stable: relative error
        # of order max(m, k) u, no rounding of a Gram product)
        alpha = (float(np.linalg.norm(MW, 2)) * (1.0 + max(MW.shape) * u)) ** 2
        G = MW.T @ M
        B = G - (G @ W) @ W.T
        beta = float(np.linalg.norm(B, 2)) + u * (min(B.shape) * max(B.shape) * float(np.linalg.norm(B)) +
                                                  m * float(np.linalg.norm(MW)) * float(np.linalg.norm(M)))
        X = M - MW @ W.T
    else:
        alpha = beta = 0.0
        X = M
    gamma = _gram_lambda_max_upper(X)
    lam = 0.5 * (alpha + gamma) + math.sqrt(0.25 * (alpha - gamma) ** 2 + beta * beta)
    spec_up = math.sqrt(max(lam, 0.0)) * (1.0 + 1e-13)
    c = 1.0 if spec_up <= tau else tau / spec_up
    gap = tau * nuc - c * float(np.sum(Y * M)) + 0.5 * (1.0 - c) ** 2 * float(np.sum(M * M))
    bound = math.sqrt(2.0 * max(gap, 0.0))
    return bound, {"spec_upper": spec_up, "alpha": alpha, "beta": beta, "gamma_upper": gamma, "gap": gap,
                   "nuclear": nuc}


def svt_compressed(A, tau, Q, nthreads: int = 0):
    """Eq. (1) through an orthonormal basis Q (m x k) of a subspace meant to
    hold the left singular vectors of every sigma > tau:
    Y = Q (Q^T A)_tau, with (Q^T A)_tau by the Jacobi SVD of the k x n
    matrix.  Exact when that subspace is exactly invariant and the rest of A
    has spectral norm <= tau; ``prox_error_bound`` certifies it."""
    A = np.asarray(A, np.float64)
    return Q @ svt(Q.T @ A, tau, nthreads)


def svt_gapped(A, tau, k, power_iters=6, seed=0, nthreads: int = 0, max_rel_bound=1e-6, return_bound=False):
    """Eq. (1) for a large matrix whose singular values above tau are few and
    separated by a wide gap from the rest (low-rank signal plus noise, tau =
    2 ||N||_2), computed on a compressed matrix and then certified:

      Q = orthonormal basis of (A A^T)^q A Omega  (Omega: n x k Gaussian),
      Y = Q (Q^T A)_tau,

    accepted only when the duality-gap bound of ``prox_error_bound`` gives
    ||Y - A_tau||_F <= max_rel_bound ||Y||_F (RuntimeError otherwise).  The
    bound holds for any Y, so acceptance does not rest on the randomised
    basis being good.  k must exceed the number of singular values above
    tau."""
    A = np.asarray(A, np.float64)
    m, n = A.shape
    if m < n:
        out = svt_gapped(A.T, tau, k, power_iters, seed, nthreads, max_rel_bound, return_bound)
        return (out[0].T, out[1]) if return_bound else out.T
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(A @ rng.standard_normal((n, k)))
    for _ in range(power_iters):
        Q, _ = np.linalg.qr(A @ (A.T @ Q))
    Z = svt(Q.T @ A, tau, nthreads)
    Y = Q @ Z
    bound, _ = prox_error_bound(A, Y, tau, factor=(Q, Z))
    ny = float(np.linalg.norm(Y))
    rel = bound / ny if ny > 0 else bound
    if not rel <= max_rel_bound:
        raise RuntimeError("certified error bound %.3g exceeds %.3g: increase k or power_iters" % (rel, max_rel_bound))
    return (Y, rel) if return_bound else Y


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
