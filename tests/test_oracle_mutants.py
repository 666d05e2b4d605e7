"""The pins must catch mistakes: plausible wrong versions of the oracle's
soft-thresholding (each a one-line slip in Eq. (1) of section 2 or in the
use of the SVD) are run through the same checks as the oracle, on the CPU,
and each one must fail at least one of them while the oracle passes all.
The mutants are built here from the oracle's own SVD; nothing in oracle/ is
changed."""
import json
import os

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

HERE = os.path.dirname(os.path.abspath(__file__))


def _svt_from(U, s, V, tau):
    return (U * np.maximum(s - tau, 0.0)) @ V.T


def correct(A, tau):
    return oracle.svt(A, tau)


def dropped_shrink(A, tau):  # forgets the - tau
    U, s, V = oracle.svd(A)
    return (U * s * (s > tau)) @ V.T


def tau_squared(A, tau):  # thresholds sigma at tau^2 (the proposition's shift leaking into Eq. (1))
    U, s, V = oracle.svd(A)
    return _svt_from(U, s, V, tau * tau)


def wrong_sign(A, tau):  # sign of the left factor lost
    U, s, V = oracle.svd(A)
    return _svt_from(-U, s, V, tau)


def transposed_factor(A, tau):  # U and V swapped for a square input (result transposed)
    U, s, V = oracle.svd(A)
    if A.shape[0] != A.shape[1]:
        return _svt_from(U, s, V, tau)[::-1]  # row order lost instead
    return _svt_from(V, s, U, tau)


def unsorted_values(A, tau):  # singular values paired with the wrong vectors
    U, s, V = oracle.svd(A)
    return _svt_from(U, s[::-1], V, tau)


def abs_instead_of_max(A, tau):  # |sigma - tau| instead of max(sigma - tau, 0)
    U, s, V = oracle.svd(A)
    return (U * np.abs(s - tau)) @ V.T


def half_threshold(A, tau):  # tau/2 (the 1/2 of the proposition applied twice)
    U, s, V = oracle.svd(A)
    return _svt_from(U, s, V, 0.5 * tau)


MUTANTS = [dropped_shrink, tau_squared, wrong_sign, transposed_factor, unsorted_values, abs_instead_of_max,
           half_threshold]


# ----------------------------------------------------------------- checks

def check_golden(f):
    with open(os.path.join(HERE, "golden", "closed_forms.json")) as fh:
        cases = json.load(fh)["cases"]
    for c in cases:
        A = np.array(c["A"], dtype=np.float64)
        if not np.allclose(f(A, c["tau"]), np.array(c["A_tau"]), rtol=0, atol=1e-12):
            return False
    return True


def check_limits(f):
    rng = np.random.default_rng(5)
    A = rng.standard_normal((7, 5))
    smax = np.linalg.norm(A, 2)
    return np.allclose(f(A, 0.0), A, atol=1e-12) and np.allclose(f(A, 1.01 * smax), 0.0, atol=1e-12)


def check_prox_certificate(f):
    """M = A - A_tau has ||M||_2 <= tau and <M, A_tau> = tau ||A_tau||_* (the
    optimality conditions of the prox of the nuclear norm)."""
    rng = np.random.default_rng(6)
    A = rng.standard_normal((9, 6))
    tau = 0.8 * np.median(np.linalg.svd(A, compute_uv=False))
    Y = f(A, tau)
    if Y.shape != A.shape:
        return False
    M = A - Y
    nuc = np.sum(np.linalg.svd(Y, compute_uv=False))
    return np.linalg.norm(M, 2) <= tau * (1 + 1e-10) and abs(np.sum(M * Y) - tau * nuc) <= 1e-9 * max(1.0, tau * nuc)


def check_diagonal(f):
    d = np.array([3.0, -2.0, 0.5])
    A = np.diag(d)
    return np.allclose(f(A, 1.0), np.diag(np.sign(d) * np.maximum(np.abs(d) - 1.0, 0.0)), atol=1e-12)


CHECKS = [check_golden, check_limits, check_prox_certificate, check_diagonal]


def test_oracle_passes_every_check():
    for chk in CHECKS:
        assert chk(correct), chk.__name__


@pytest.mark.parametrize("mutant", MUTANTS, ids=lambda m: m.__name__)
def test_each_mutant_fails_a_check(mutant):
    failed = [chk.__name__ for chk in CHECKS if not chk(mutant)]
    assert failed, "%s passes every pin" % mutant.__name__


# ----------------------------------------------------------------- polar

def polar_correct(A):
    return oracle.polar(A)


def polar_transposed(A):  # V U^T
    U, s, V = oracle.svd(A)
    return (V * (s > 0)) @ U.T


def polar_negated(A):
    return -oracle.polar(A)


def polar_unnormalised(A):  # U Sigma V^T / sigma_max instead of U V^T
    U, s, V = oracle.svd(A)
    return (U * (s / s[0])) @ V.T


def check_polar(f):
    """P has orthonormal columns (tall A) and P^T A is symmetric positive
    semidefinite (A = P H, section 2)."""
    rng = np.random.default_rng(7)
    for shape in [(8, 5), (6, 6)]:
        A = rng.standard_normal(shape)
        P = f(A)
        if P.shape != A.shape:
            return False
        H = P.T @ A
        if not np.allclose(P.T @ P, np.eye(shape[1]), atol=1e-10):
            return False
        if not np.allclose(H, H.T, atol=1e-10) or np.min(np.linalg.eigvalsh(0.5 * (H + H.T))) < -1e-10:
            return False
    return True


def test_polar_pins_catch_mutants():
    assert check_polar(polar_correct)
    for m in (polar_transposed, polar_negated, polar_unnormalised):
        assert not check_polar(m), m.__name__
