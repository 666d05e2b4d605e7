"""Seeded synthetic inputs for singular value soft-thresholding.

This module is the one piece shared by the tests, the oracle side and the GPU
side: it builds input matrices and thresholds and holds none of the method's
arithmetic.  Every draw comes from ``numpy.random.default_rng`` seeded with
``[2607_22484, cfg, idx]``; matrices are built in float64 and rounded once to
float32, and the float32 array is what both sides receive.

Workload recipes (the paper's experiments use random test matrices:
an i.i.d. Gaussian 301 x 300 matrix in Fig. 1, Gaussian m x (m+1) in Fig. 2):

* constructed spectra  A = U diag(sigma) V^T with U, V Haar-distributed
  (QR of a Gaussian matrix, columns signed by diag(R)), so the exact SVD of the
  float64 matrix is known;
* low-rank signal plus Gaussian noise  A = U diag(sigma) V^T + N, with
  N_ij ~ N(0, (0.01/sqrt(n))^2) and tau = 2 ||N||_2;
* i.i.d. Gaussian matrices as in Figs. 1 and 2.

``gap_clamp`` keeps every singular value at least 5 % (multiplicatively) away
from tau: values >= tau are raised to at least 1.05 tau and values < tau are
lowered to at most tau / 1.05.  Order and count on each side are preserved.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SEED_ROOT = 2607_22484

# config ids used in seeds
CFG_SMALL = 1      # 256 x 128 constructed, log spectrum 1 .. 1e-2
CFG_SQUARE = 2     # 4096^2 constructed, log spectrum 10 .. 1e-3
CFG_NOISY = 3      # rank-200 signal + noise, 8192 x 4096 / 4096 x 8192
CFG_BATCH = 4      # 512 uneven constructed matrices
CFG_SERVE = 5      # serving request stream
CFG_FIG1 = 6       # 301 x 300 Gaussian
CFG_FIG2 = 7       # m x (m+1) Gaussian
CFG_TEST = 9       # ad-hoc test shapes


def rng_for(cfg: int, idx: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED_ROOT, int(cfg), int(idx)])


def haar_columns(rng: np.random.Generator, n: int, k: int) -> np.ndarray:
    """n x k matrix with Haar-distributed orthonormal columns (k <= n)."""
    G = rng.standard_normal((n, k))
    Q, R = np.linalg.qr(G)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d


def log_spectrum(k: int, hi: float, lo: float) -> np.ndarray:
    """k values log-spaced from hi down to lo (descending)."""
    if k == 1:
        return np.array([hi], dtype=np.float64)
    i = np.arange(k, dtype=np.float64)
    return hi * (lo / hi) ** (i / (k - 1))


def gap_clamp(sigma: np.ndarray, tau: float, gap: float = 1.05) -> np.ndarray:
    s = np.array(sigma, dtype=np.float64, copy=True)
    above = s >= tau
    s[above] = np.maximum(s[above], gap * tau)
    s[~above] = np.minimum(s[~above], tau / gap)
    return s


@dataclasses.dataclass
class Problem:
    """One SVT input.  ``A`` is the float32 matrix both sides receive;
    ``A64`` the float64 matrix it was rounded from; ``U, sigma, V`` the exact
    thin SVD of ``A64`` when it is known (constructed spectra), else None."""
    A: np.ndarray
    tau: float
    A64: np.ndarray
    U: Optional[np.ndarray] = None
    sigma: Optional[np.ndarray] = None
    V: Optional[np.ndarray] = None
    rank: Optional[int] = None
    name: str = ""

    @property
    def shape(self):
        return self.A.shape


def constructed(cfg: int, idx: int, m: int, n: int, sigma: np.ndarray, tau: float, name: str = "",
                rank: Optional[int] = None) -> Problem:
    rng = rng_for(cfg, idx)
    k = min(m, n)
    assert len(sigma) == k
    U = haar_columns(rng, m, k)
    V = haar_columns(rng, n, k)
    A64 = (U * sigma) @ V.T
    return Problem(A=A64.astype(np.float32), tau=float(tau), A64=A64, U=U, sigma=np.asarray(sigma, np.float64),
                   V=V, rank=rank, name=name)


# ---------------------------------------------------------------- recipes

def small_case(idx: int = 0, m: int = 256, n: int = 128) -> Problem:
    """256 x 128, sigma log-spaced 1 .. 1e-2, tau = geometric midpoint of
    sigma_64 and sigma_65 (= 0.1 at the default size), gap-clamped."""
    k = min(m, n)
    sig = log_spectrum(k, 1.0, 1e-2)
    h = k // 2
    tau = math.sqrt(sig[h - 1] * sig[h])
    return constructed(CFG_SMALL, idx, m, n, gap_clamp(sig, tau), tau, name="small_%dx%d" % (m, n))


def square_case(q: float, idx: int = 0, n: int = 4096, m: Optional[int] = None) -> Problem:
    """n x n (or m x n), sigma log-spaced 10 .. 1e-3, tau at quantile q of
    sigma (numpy linear quantile), gap-clamped."""
    m = n if m is None else m
    k = min(m, n)
    sig = log_spectrum(k, 10.0, 1e-3)
    tau = float(np.quantile(sig, q))
    return constructed(CFG_SQUARE, idx + int(round(q * 1000)), m, n, gap_clamp(sig, tau), tau,
                       name="square_%dx%d_q%02d" % (m, n, int(round(q * 100))))


def rank_case(r: int = 256, idx: int = 0, n: int = 4096, m: Optional[int] = None) -> Problem:
    """Same spectrum as ``square_case``; tau = sqrt(sigma_r sigma_{r+1})
    (1-based), gap-clamped, so exactly r values exceed tau."""
    m = n if m is None else m
    k = min(m, n)
    sig = log_spectrum(k, 10.0, 1e-3)
    tau = math.sqrt(sig[r - 1] * sig[r])
    return constructed(CFG_SQUARE, 100000 + idx + r, m, n, gap_clamp(sig, tau), tau, rank=r,
                       name="rank%d_%dx%d" % (r, m, n))


def noise_spectral_norm(N: np.ndarray, iters: int = 200, seed: int = 0) -> float:
    """||N||_2 by power iteration on N^T N in float64 (input recipe only).
    The returned value is the Rayleigh quotient after ``iters`` steps."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(N.shape[1])
    x /= np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = N.T @ (N @ x)
        lam = float(x @ y)
        x = y / np.linalg.norm(y)
    return math.sqrt(lam)


def noisy_lowrank(m: int, n: int, rank: int = 200, idx: int = 0, noise: float = 0.01,
                  sig_lo: float = 1.0, sig_hi: float = 10.0, cfg: int = CFG_NOISY, norm_iters: int = 200) -> Problem:
    """Rank-``rank`` Haar signal with sigma ~ U[sig_lo, sig_hi] plus i.i.d.
    N(0, (noise/sqrt(n))^2), n = column count; tau = 2 ||N||_2."""
    rng = rng_for(cfg, idx)
    U = haar_columns(rng, m, rank)
    V = haar_columns(rng, n, rank)
    sig = np.sort(rng.uniform(sig_lo, sig_hi, size=rank))[::-1]
    N = rng.standard_normal((m, n)) * (noise / math.sqrt(n))
    A64 = (U * sig) @ V.T + N
    tau = 2.0 * noise_spectral_norm(N, iters=norm_iters)
    return Problem(A=A64.astype(np.float32), tau=tau, A64=A64, rank=rank, name="noisy_%dx%d_r%d" % (m, n, rank))


def batch_cases(count: int = 512, idx: int = 0, lo: int = 128, hi: int = 2048) -> List[Problem]:
    """``count`` constructed matrices; m, n = round(exp U[ln lo, ln hi]) drawn
    independently; sigma log-spaced 1 .. 1e-2 over min(m, n) values; tau at a
    quantile q ~ U[0.1, 0.9], gap-clamped."""
    rng = rng_for(CFG_BATCH, idx)
    shapes = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=(count, 2)))).astype(int)
    qs = rng.uniform(0.1, 0.9, size=count)
    out = []
    for j in range(count):
        m, n = int(shapes[j, 0]), int(shapes[j, 1])
        k = min(m, n)
        sig = log_spectrum(k, 1.0, 1e-2)
        tau = float(np.quantile(sig, qs[j]))
        out.append(constructed(CFG_BATCH, 1000 * (idx + 1) + j, m, n, gap_clamp(sig, tau), tau,
                               name="batch%d_%dx%d" % (j, m, n)))
    return out


def gaussian(m: int, n: int, cfg: int = CFG_FIG1, idx: int = 0) -> np.ndarray:
    """i.i.d. standard Gaussian m x n, float32 (Figs. 1 and 2)."""
    return rng_for(cfg, idx).standard_normal((m, n)).astype(np.float32)


def serve_shapes(count: int, idx: int = 0, lo: int = 256, hi: int = 4096):
    """Request shapes for the serving stream: s = round(exp U[ln lo, ln hi]),
    square, or 2:1 rectangular either way with equal probability; rank r
    from {16, 64, 256} capped at s/4."""
    rng = rng_for(CFG_SERVE, idx)
    out = []
    for _ in range(count):
        s = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        kind = rng.integers(0, 3)
        if kind == 0:
            m, n = s, s
        elif kind == 1:
            m, n = s, max(1, s // 2)
        else:
            m, n = max(1, s // 2), s
        r = int(min(rng.choice([16, 64, 256]), min(m, n) // 4))
        out.append((m, n, max(r, 1)))
    return out


CFG_COMPLETION = 10  # matrix-completion problems for the proximal client


@dataclasses.dataclass
class CompletionProblem:
    """A matrix-completion problem: M = rank-r signal (Haar factors, singular
    values uniform in [1, 10]) plus small Gaussian noise, observed on a random
    subset of its entries (each kept with probability p); lam the
    nuclear-norm weight."""
    M: np.ndarray
    mask: np.ndarray
    lam: float
    rank: int
    name: str = ""


def completion_lam(fro_M: float, m: int, n: int, p: float, lam_mult: float) -> float:
    """lam = lam_mult x the sampling noise's spectral edge: observing M on a
    Bernoulli(p) mask gives p M + E, E with independent entries of variance
    about p (1 - p) ||M||_F^2 / (m n), so ||E||_2 is about
    sqrt(p (1 - p)) ||M||_F / sqrt(m n) (sqrt(m) + sqrt(n)).  With lam_mult
    = 2 the thresholding removes that bulk with a factor-2 gap and keeps the
    signal directions above it."""
    return lam_mult * math.sqrt(p * (1.0 - p)) * fro_M / math.sqrt(m * n) * (math.sqrt(m) + math.sqrt(n))


def completion_problem(m: int, n: int, rank: int, p: float = 0.8, idx: int = 0, lam_mult: float = 2.0,
                       noise: float = 0.01, cfg: int = CFG_COMPLETION) -> CompletionProblem:
    """M = U diag(sigma) V^T + N (float32; N i.i.d. N(0, (noise/sqrt(n))^2)),
    mask ~ Bernoulli(p), lam from ``completion_lam``."""
    rng = rng_for(cfg, idx)
    U = haar_columns(rng, m, rank)
    V = haar_columns(rng, n, rank)
    sig = np.sort(rng.uniform(1.0, 10.0, size=rank))[::-1]
    M = (U * sig) @ V.T + rng.standard_normal((m, n)) * (noise / math.sqrt(n))
    mask = (rng.uniform(size=(m, n)) < p).astype(np.float32)
    lam = completion_lam(float(np.linalg.norm(M)), m, n, p, lam_mult)
    return CompletionProblem(M=M.astype(np.float32), mask=mask, lam=lam, rank=rank,
                             name="completion_%dx%d_r%d" % (m, n, rank))


def completion_problem_device(torch, gen, m: int, n: int, rank: int, p: float = 0.8, lam_mult: float = 2.0,
                              noise: float = 0.01):
    """The serving stream's matrix-completion problem (the recipe of
    ``completion_problem``), drawn on the device from the seeded torch
    generator ``gen`` (Haar factors from the QR of Gaussians); returns
    (M_obs = mask * M, mask, lam)."""
    dev = gen.device
    U = torch.linalg.qr(torch.randn(m, rank, device=dev, generator=gen))[0]
    V = torch.linalg.qr(torch.randn(n, rank, device=dev, generator=gen))[0]
    sig = 1.0 + 9.0 * torch.rand(rank, device=dev, generator=gen)
    M = (U * sig) @ V.T + torch.randn(m, n, device=dev, generator=gen) * (noise / math.sqrt(n))
    mask = (torch.rand(m, n, device=dev, generator=gen) < p).to(torch.float32)
    lam = completion_lam(float(M.norm().item()), m, n, p, lam_mult)
    return (mask * M).contiguous(), mask, lam
