"""Pins for the FP64 oracle: checks against what the paper and the
mathematics fix, never against the oracle's own formulas retyped.

Each test names the planted mistake it would catch (dropped term, wrong
sign, transposed operand, wrong shift, wrong sort order, ...).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2607_22484_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-12


def relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


# ----------------------------------------------------------------- golden

def _golden():
    with open(os.path.join(HERE, "golden", "closed_forms.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _golden(), ids=lambda c: c["name"])
def test_golden_closed_forms(case):
    """Hand-derived results (section 2, Eq. (1)); catches a wrong sign of the
    left factor, a dropped (sigma - tau) shrink, or a transposed result."""
    A = np.array(case["A"], dtype=np.float64)
    tau = case["tau"]
    np.testing.assert_allclose(oracle.svt(A, tau), np.array(case["A_tau"]), rtol=0, atol=1e-13)
    if "P" in case:
        np.testing.assert_allclose(oracle.polar(A), np.array(case["P"]), rtol=0, atol=1e-13)
        np.testing.assert_allclose(oracle.svt(A.T, tau), np.array(case["A_tau"]).T, rtol=0, atol=1e-13)


def test_scalar_tau_squared_proposition():
    """P1: A=[0.5], tau=0.4.  The proposition with the Gram shifted by tau^2
    gives 0.1 = A_tau; shifting by tau would give 0 (section 2,
    Proposition 1; the listing shifts by tau**2)."""
    A = np.array([[0.5]])
    tau = 0.4
    P = oracle.polar(A)
    S = oracle.polar_sym(A.T @ A - tau ** 2 * np.eye(1))
    Y = 0.5 * (A + A @ S) - tau / 2 * (P + P @ S)
    assert abs(Y[0, 0] - 0.1) < 1e-15
    assert abs(oracle.svt(A, tau)[0, 0] - 0.1) < 1e-15
    S_wrong = oracle.polar_sym(A.T @ A - tau * np.eye(1))
    Y_wrong = 0.5 * (A + A @ S_wrong) - tau / 2 * (P + P @ S_wrong)
    assert abs(Y_wrong[0, 0]) < 1e-15


# ------------------------------------------------------------ diagonal, 2x2

@pytest.mark.parametrize("shape", [(5, 5), (7, 4), (4, 7)])
def test_diagonal_and_permuted(shape):
    """P2: A = Pm diag(d) Qm with signed d and permutation matrices Pm, Qm:
    A_tau = Pm diag(sign d (|d| - tau)_+) Qm; polar = Pm diag(sign d) Qm;
    S = sign(A^T A - tau^2 I) = Qm^T diag(sign(d^2 - tau^2)) Qm."""
    rng = np.random.default_rng(5)
    m, n = shape
    k = min(m, n)
    d = np.array([3.0, -2.5, 1.5, -0.7, 0.3, 2.2, -1.1])[:k]
    D = np.zeros((m, n))
    D[np.arange(k), np.arange(k)] = d
    Pm = np.eye(m)[rng.permutation(m)]
    Qm = np.eye(n)[rng.permutation(n)]
    A = Pm @ D @ Qm
    tau = 1.2
    Dt = np.zeros((m, n))
    Dt[np.arange(k), np.arange(k)] = np.sign(d) * np.maximum(np.abs(d) - tau, 0)
    np.testing.assert_allclose(oracle.svt(A, tau), Pm @ Dt @ Qm, atol=TOL)
    Ds = np.zeros((m, n))
    Ds[np.arange(k), np.arange(k)] = np.sign(d)
    np.testing.assert_allclose(oracle.polar(A), Pm @ Ds @ Qm, atol=TOL)
    sdiag = np.full(n, -1.0)       # zero columns of A: 0 - tau^2 < 0
    sdiag[:k] = np.sign(d ** 2 - tau ** 2)
    np.testing.assert_allclose(oracle.polar_sym(A.T @ A - tau ** 2 * np.eye(n)), Qm.T @ np.diag(sdiag) @ Qm,
                               atol=TOL)


def _svd2(a, b, c, d):
    """Closed-form singular values and polar factor of [[a,b],[c,d]]."""
    p = math.hypot(a + d, c - b)
    q = math.hypot(a - d, b + c)
    s1, s2 = (p + q) / 2, abs(p - q) / 2
    det = a * d - b * c
    A = np.array([[a, b], [c, d]])
    P = (A + np.sign(det) * np.array([[d, -c], [-b, a]])) / (s1 + s2)
    return s1, s2, P


@pytest.mark.parametrize("seed", range(6))
def test_two_by_two_closed_form(seed):
    """P3: 2x2 closed forms for sigma, P, u1 v1^T and A_tau in all three tau
    regimes; sign of a symmetric indefinite 2x2 = (2G - tr G I)/(l1 - l2)."""
    rng = np.random.default_rng(100 + seed)
    a, b, c, d = rng.standard_normal(4)
    A = np.array([[a, b], [c, d]])
    s1, s2, P = _svd2(a, b, c, d)
    U, s, V = oracle.svd(A)
    np.testing.assert_allclose(s, [s1, s2], rtol=1e-13)
    np.testing.assert_allclose(oracle.polar(A), P, atol=1e-13)
    u1v1 = (A - s2 * P) / (s1 - s2)
    for tau, expect in [(0.5 * s2, A - 0.5 * s2 * P), (0.5 * (s1 + s2), (s1 - 0.5 * (s1 + s2)) * u1v1),
                        (1.5 * s1, np.zeros((2, 2)))]:
        np.testing.assert_allclose(oracle.svt(A, tau), expect, atol=1e-12)
    # symmetric indefinite sign
    g = rng.standard_normal(3)
    G = np.array([[g[0], g[1]], [g[1], -abs(g[2]) - abs(g[0]) - 1.0]])
    tr = np.trace(G)
    disc = math.sqrt((G[0, 0] - G[1, 1]) ** 2 + 4 * G[0, 1] ** 2)
    l1, l2 = (tr + disc) / 2, (tr - disc) / 2
    if l1 > 0 > l2:
        np.testing.assert_allclose(oracle.polar_sym(G), (2 * G - tr * np.eye(2)) / (l1 - l2), atol=1e-13)


# ------------------------------------------------------------ special cases

@pytest.mark.parametrize("shape", [(40, 25), (25, 40), (33, 33)])
def test_tau_zero_and_tau_large(shape):
    """P4: tau = 0 returns A; tau >= sigma_max returns 0."""
    rng = np.random.default_rng(7)
    A = rng.standard_normal(shape)
    np.testing.assert_allclose(oracle.svt(A, 0.0), A, atol=1e-12 * np.linalg.norm(A))
    smax = np.linalg.norm(A, 2)
    assert np.abs(oracle.svt(A, smax * 1.0000001)).max() < 1e-12 * smax
    assert np.abs(oracle.svt(A, 10 * smax)).max() == 0.0


@pytest.mark.parametrize("shape", [(60, 30), (30, 60), (45, 45)])
def test_orthogonality_and_sign_properties(shape):
    """P5: P^T P = I (tall/square) or P P^T = I (wide); S = S^T, S^2 = I,
    S G = G S; Pi = (I+S)/2 is a projector with trace #{sigma > tau}."""
    rng = np.random.default_rng(11)
    m, n = shape
    A = rng.standard_normal(shape)
    P = oracle.polar(A)
    if m >= n:
        np.testing.assert_allclose(P.T @ P, np.eye(n), atol=1e-12)
    else:
        np.testing.assert_allclose(P @ P.T, np.eye(m), atol=1e-12)
    s = np.linalg.svd(A, compute_uv=False)
    tau = float(np.sqrt(s[len(s) // 3] * s[len(s) // 3 + 1]))
    G = A.T @ A - tau ** 2 * np.eye(n)
    S = oracle.polar_sym(G)
    np.testing.assert_allclose(S, S.T, atol=1e-12)
    np.testing.assert_allclose(S @ S, np.eye(n), atol=1e-11)
    np.testing.assert_allclose(S @ G, G @ S, atol=1e-10 * np.linalg.norm(G))
    Pi = 0.5 * (np.eye(n) + S)
    np.testing.assert_allclose(Pi @ Pi, Pi, atol=1e-11)
    assert abs(np.trace(Pi) - np.sum(s > tau)) < 1e-10


@pytest.mark.parametrize("shape", [(50, 30), (30, 50), (40, 40)])
def test_proposition_identity_both_sides(shape):
    """P6: Proposition 1 and its footnote.  With oracle P and
    S = sign(A^T A - tau^2 I) (right) or S = sign(A A^T - tau^2 I) (left),
    (A + AS)/2 - tau/2 (P + PS) and (A + SA)/2 - tau/2 (P + SP) both equal
    A_tau.  Catches a sign error in either term or the wrong side."""
    rng = np.random.default_rng(13)
    m, n = shape
    A = rng.standard_normal(shape)
    s = np.linalg.svd(A, compute_uv=False)
    tau = float(np.sqrt(s[len(s) // 2] * s[len(s) // 2 - 1]))
    At = oracle.svt(A, tau)
    P = oracle.polar(A)
    Sr = oracle.polar_sym(A.T @ A - tau ** 2 * np.eye(n))
    Sl = oracle.polar_sym(A @ A.T - tau ** 2 * np.eye(m))
    right = 0.5 * (A + A @ Sr) - tau / 2 * (P + P @ Sr)
    left = 0.5 * (A + Sl @ A) - tau / 2 * (P + Sl @ P)
    assert relerr(right, At) < 1e-11
    assert relerr(left, At) < 1e-11
    # the fused form (A - tau P)(I + S)/2 used by the GPU epilogue
    assert relerr((A - tau * P) @ (0.5 * (np.eye(n) + Sr)), At) < 1e-11


def test_constructed_spectrum_small_recipe():
    """P7: A = U diag(sigma) V^T built in FP64 (the 256 x 128 recipe):
    oracle A_tau equals U diag(sigma - tau)_+ V^T with no SVD taken."""
    pb = inputs.small_case()
    exact = oracle.svt_from_svd(pb.U, pb.sigma, pb.V, pb.tau)
    assert relerr(oracle.svt(pb.A64, pb.tau), exact) < 1e-12
    # recipe check: tau = 0.1 and the gap clamp
    assert abs(pb.tau - 0.1) < 1e-12
    assert np.min(np.maximum(pb.sigma / pb.tau, pb.tau / pb.sigma)) >= 1.05 - 1e-12


@pytest.mark.parametrize("shape", [(36, 20), (20, 36)])
def test_invariances(shape):
    """P8: (Q A Z)_tau = Q A_tau Z for orthogonal Q, Z; (cA)_{c tau} = c A_tau;
    (A^T)_tau = (A_tau)^T."""
    rng = np.random.default_rng(17)
    m, n = shape
    A = rng.standard_normal(shape)
    tau = 1.3
    At = oracle.svt(A, tau)
    Q = inputs.haar_columns(rng, m, m)
    Z = inputs.haar_columns(rng, n, n)
    assert relerr(oracle.svt(Q @ A @ Z, tau), Q @ At @ Z) < 1e-12
    assert relerr(oracle.svt(3.5 * A, 3.5 * tau), 3.5 * At) < 1e-12
    assert relerr(oracle.svt(A.T, tau), At.T) < 1e-12


@pytest.mark.parametrize("shape", [(30, 20), (20, 30)])
def test_prox_certificate(shape):
    """P9: A_tau is the proximal point of tau ||.||_* (section 2: it is the
    subroutine of nuclear-norm proximal methods).  M = A - A_tau satisfies
    ||M||_2 <= tau and <M, A_tau> = tau ||A_tau||_*; A - A_tau = U min(S, tau)
    V^T; and A_tau beats random perturbations on the prox objective."""
    rng = np.random.default_rng(19)
    A = rng.standard_normal(shape)
    s = np.linalg.svd(A, compute_uv=False)
    tau = float(np.median(s))
    At = oracle.svt(A, tau)
    M = A - At
    assert np.linalg.norm(M, 2) <= tau * (1 + 1e-12)
    nuc = np.linalg.svd(At, compute_uv=False).sum()
    assert abs(np.sum(M * At) - tau * nuc) < 1e-10 * max(1.0, tau * nuc)
    U, sv, Vt = np.linalg.svd(A, full_matrices=False)
    np.testing.assert_allclose(M, (U * np.minimum(sv, tau)) @ Vt, atol=1e-11)

    def f(X):
        return 0.5 * np.linalg.norm(X - A) ** 2 + tau * np.linalg.svd(X, compute_uv=False).sum()
    f0 = f(At)
    for _ in range(20):
        assert f(At + 1e-3 * rng.standard_normal(shape)) > f0


@pytest.mark.parametrize("shape", [(80, 50), (50, 80), (64, 64)])
def test_matches_lapack(shape):
    """P10: thresholding through LAPACK's SVD (numpy.linalg.svd, the
    SVD-based reference approach of the code section) matches the Jacobi
    oracle."""
    rng = np.random.default_rng(23)
    A = rng.standard_normal(shape)
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    for tau in [0.0, float(s[len(s) // 4]) * 1.01, float(np.median(s)) * 0.99, float(s[0]) * 2]:
        ref = (U * np.maximum(s - tau, 0)) @ Vt
        got = oracle.svt(A, tau)
        if np.linalg.norm(ref) == 0:
            assert np.abs(got).max() == 0
        else:
            assert relerr(got, ref) < 1e-12
    Us, ss, Vs = oracle.svd(A)
    np.testing.assert_allclose(ss, s, rtol=1e-12, atol=1e-14 * s[0])


@pytest.mark.parametrize("r", [1, 5, 17])
def test_rank_r_truncation(r):
    """P11: Corollary 1 -- [A]_r from the oracle equals brute-force
    truncation of LAPACK's SVD, and meets Eckart-Young:
    ||A - [A]_r||_F^2 = sum_{i>r} sigma_i^2.  Also (A + AS)/2 with
    S = sign(A^T A - tau^2 I), tau between sigma_{r+1} and sigma_r."""
    rng = np.random.default_rng(29)
    A = rng.standard_normal((45, 30))
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    tau = float(np.sqrt(s[r - 1] * s[r]))
    Ar = oracle.rank_r(A, tau)
    ref = (U[:, :r] * s[:r]) @ Vt[:r]
    assert relerr(Ar, ref) < 1e-12
    assert abs(np.linalg.norm(A - Ar) ** 2 - np.sum(s[r:] ** 2)) < 1e-10 * np.sum(s ** 2)
    S = oracle.polar_sym(A.T @ A - tau ** 2 * np.eye(30))
    assert relerr(0.5 * (A + A @ S), ref) < 1e-11


def test_scalar_identity():
    """P12: max(x, 0) = (|x| + x)/2 on the diagonal path (section 2)."""
    x = np.linspace(-3, 3, 601)
    np.testing.assert_array_equal(np.maximum(x, 0), 0.5 * (np.abs(x) + x))
    d = np.array([2.0, 0.5, -1.0])
    tau = 0.8
    A = np.diag(d)
    expect = np.diag(np.sign(d) * 0.5 * (np.abs(np.abs(d) - tau) + (np.abs(d) - tau)))
    np.testing.assert_allclose(oracle.svt(A, tau), expect, atol=1e-15)


def test_singular_values_sorted_and_rank_deficient():
    """Sort order and the rank tolerance: a rank-3 matrix reports three
    nonzero values in descending order; its polar factor is the partial
    isometry U_3 V_3^T."""
    rng = np.random.default_rng(31)
    L = rng.standard_normal((20, 3)) @ rng.standard_normal((3, 12))
    U, s, V = oracle.svd(L)
    assert np.all(np.diff(s) <= 0)
    assert np.count_nonzero(s) == 3
    Ul, sl, Vlt = np.linalg.svd(L, full_matrices=False)
    np.testing.assert_allclose(oracle.polar(L), Ul[:, :3] @ Vlt[:3], atol=1e-12)


def test_empty_and_vector_shapes():
    for shape in [(0, 5), (5, 0), (0, 0)]:
        assert oracle.svt(np.zeros(shape), 0.5).shape == shape
    a = np.array([[3.0], [4.0]])
    np.testing.assert_allclose(oracle.svt(a, 1.0), a * (4.0 / 5.0), atol=1e-15)
    np.testing.assert_allclose(oracle.svt(a.T, 1.0), a.T * (4.0 / 5.0), atol=1e-15)


def test_svt_gapped_matches_full_jacobi():
    """The compressed route for gapped low-rank + noise inputs equals the
    full Jacobi oracle (it is the same Eq. (1) on an exact invariant
    subspace), and its certificate accepts it."""
    pb = inputs.noisy_lowrank(300, 160, rank=12, idx=5, cfg=inputs.CFG_TEST)
    full = oracle.svt(pb.A, pb.tau)
    Y, bound = oracle.svt_gapped(pb.A, pb.tau, k=32, return_bound=True)
    assert relerr(Y, full) < 1e-11
    assert bound < 1e-6
    assert relerr(oracle.svt_gapped(pb.A.T, pb.tau, k=32), full.T) < 1e-11
    with pytest.raises(RuntimeError):
        oracle.svt_gapped(pb.A, pb.tau * 1e-3, k=8)   # k too small for this tau


def _planted_basis(A, tau, theta, extra=8, j=3, into=20):
    """Orthonormal basis of the exact top left singular subspace (LAPACK),
    with column j turned by angle theta towards the noise direction `into`
    places below the threshold: the subspace misses part of one u_j."""
    U, s, _ = np.linalg.svd(A, full_matrices=False)
    r1 = int(np.sum(s > tau))
    Q = U[:, :r1 + extra].copy()
    Q[:, j] = math.cos(theta) * U[:, j] + math.sin(theta) * U[:, r1 + into]
    Q, _ = np.linalg.qr(Q)
    return Q


def test_certificate_rejects_partial_subspace():
    """A basis that misses part of one retained singular direction passes the
    residual test ||(I - QQ^T) A||_2 < tau (necessary, not sufficient), yet
    gives a wrong A_tau; the duality-gap certificate bounds that error from
    above and rejects it (prox optimality, section 2)."""
    pb = inputs.noisy_lowrank(300, 160, rank=12, idx=5, cfg=inputs.CFG_TEST)
    A = pb.A.astype(np.float64)
    full = oracle.svt(A, pb.tau)
    for theta in (1e-3, 1e-4):
        Q = _planted_basis(A, pb.tau, theta)
        assert np.linalg.norm(A - Q @ (Q.T @ A), 2) * 1.05 < pb.tau   # the old check passes
        Z = oracle.svt(Q.T @ A, pb.tau)
        Y = Q @ Z
        bound, _ = oracle.prox_error_bound(A, Y, pb.tau, factor=(Q, Z))
        actual = np.linalg.norm(Y - full)
        assert actual > 1e-5 * np.linalg.norm(full)                   # and the result is wrong
        assert bound >= actual
        assert bound > 1e-6 * np.linalg.norm(Y)                       # rejected


def test_certificate_with_values_just_below_tau():
    """Completion iterates keep singular values within a fraction of a
    percent below tau outside the retained subspace: the certificate must
    still reach the compressed result's accuracy there (its spectral-norm
    bound on the complement is that block's norm, not a power-mean that
    counts the values near tau), and the certified compressed route must
    equal the full Jacobi oracle."""
    rng = np.random.default_rng(17)
    m, n, tau = 300, 150, 2.0
    U = np.linalg.qr(rng.standard_normal((m, n)))[0]
    V = np.linalg.qr(rng.standard_normal((n, n)))[0]
    sig = np.concatenate([np.linspace(8.0, 2.2, 20), tau * np.array([0.999, 0.998, 0.997, 0.996, 0.995]),
                          np.linspace(0.9, 0.01, n - 25)])
    A = (U * sig) @ V.T
    # the certificate's floor: sqrt(2 delta tau ||Y||_*) / ||Y||_F for the
    # relative rounding margin delta ~ 1e-13 of its spectral-norm bound
    Y, bound = oracle.svt_gapped(A, tau, k=40, power_iters=10, max_rel_bound=2e-6, return_bound=True)
    assert bound < 2e-6
    assert relerr(Y, oracle.svt(A, tau)) < 1e-10
    assert relerr(Y, oracle.svt_from_svd(U, sig, V, tau)) < 1e-10


@pytest.mark.parametrize("kind", ["exact", "scaled", "dense_noise", "low_rank", "dropped_term", "transposed"])
def test_prox_error_bound_is_an_upper_bound(kind):
    """The certificate is an upper bound on ||Y - A_tau||_F for any Y, and
    is small only at A_tau: exact answer (tiny), and planted mistakes (a
    scaled result, noise, a low-rank slip, a dropped singular triple, the
    transposed orientation) each give a bound above their true error."""
    rng = np.random.default_rng(41)
    A = rng.standard_normal((60, 40))
    s = np.linalg.svd(A, compute_uv=False)
    tau = float(np.sqrt(s[9] * s[10]))
    At = oracle.svt(A, tau)
    U, sv, V = oracle.svd(A)
    Y = {"exact": At,
         "scaled": 1.01 * At,
         "dense_noise": At + 1e-4 * rng.standard_normal(At.shape),
         "low_rank": At + 1e-3 * np.outer(rng.standard_normal(60), rng.standard_normal(40)),
         "dropped_term": At - (sv[0] - tau) * np.outer(U[:, 0], V[:, 0]),
         "transposed": oracle.svt(A.T, tau).T + 1e-6 * np.outer(U[:, 12], V[:, 3])}[kind]
    bound, parts = oracle.prox_error_bound(A, Y, tau)
    actual = np.linalg.norm(Y - At)
    assert bound >= actual * (1 - 1e-9)
    if kind == "exact":
        assert bound < 1e-6 * np.linalg.norm(At)
        assert parts["spec_upper"] <= tau * (1 + 1e-10)
    else:
        assert bound > 1e-6 * np.linalg.norm(At)


@pytest.mark.slow
def test_svt_gapped_c3_recipe_matches_full_jacobi():
    """The precision-form recipe (rank-200 Haar signal, sigma ~ U[1, 10],
    noise std 0.01/sqrt(n), tau = 2 ||N||_2) at 4096 x 2048: the certified
    compressed route equals the full Jacobi oracle (about 1.5 min on 8 cores)."""
    pb = inputs.noisy_lowrank(4096, 2048, rank=200, idx=7, cfg=inputs.CFG_TEST, norm_iters=60)
    Y, bound = oracle.svt_gapped(pb.A, pb.tau, k=256, return_bound=True)
    assert bound < 1e-6
    assert relerr(Y, oracle.svt(pb.A, pb.tau)) < 1e-10
