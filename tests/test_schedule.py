"""The odd-quintic schedule designer (CPU): minimax optimality of each step,
convergence of the composed map, and agreement of the shipped table."""
import os

import numpy as np
import pytest

from paper_2607_22484_amd import schedule


@pytest.mark.parametrize("lo,hi", [(1e-3, 1.3), (0.1, 2.0), (0.5, 1.6), (0.9, 1.2)])
def test_remez_equioscillates(lo, hi):
    """Chebyshev alternation: the error 1 - p reaches +-E at lo, two interior
    points and hi with alternating signs, and nowhere exceeds E."""
    a, b, c, E = schedule.remez_odd_quintic(lo, hi)
    x = np.linspace(lo, hi, 200001)
    err = 1.0 - schedule.quintic((a, b, c), x)
    assert np.max(np.abs(err)) <= E * (1 + 1e-9)
    assert abs(err[0] - E) < 1e-9 * max(E, 1e-300) + 1e-14
    assert abs(err[-1] + E) < 1e-9 * max(E, 1e-300) + 1e-14
    # two interior extrema with -E then +E
    inner = err[1:-1]
    assert np.min(inner) <= -E * (1 - 1e-6) and np.max(inner) >= E * (1 - 1e-6)


def test_remez_beats_perturbations():
    """No nearby odd quintic has a smaller maximum error on the interval."""
    lo, hi = 0.05, 1.3
    a, b, c, E = schedule.remez_odd_quintic(lo, hi)
    x = np.linspace(lo, hi, 20001)
    rng = np.random.default_rng(0)
    for _ in range(200):
        d = rng.standard_normal(3) * 1e-3
        e = np.max(np.abs(1 - schedule.quintic((a + d[0], b + d[1], c + d[2]), x)))
        assert e >= E - 1e-12


def test_composed_schedule_converges():
    """20 steps of the shipped schedule map every x in [l0, 1] (and values up
    to 30 % above) to within 1e-6 of 1."""
    tab = schedule.design()
    x = np.concatenate([np.geomspace(schedule.DEFAULT_L0, 1.0, 5000), np.linspace(1.0, 1.3, 500)])
    for t in range(20):
        x = schedule.quintic(tab[t], x)
    assert np.max(np.abs(x - 1.0)) < 1e-6


def test_odd_symmetry_and_fixed_point():
    tab = schedule.design()
    for row in tab:
        assert schedule.quintic(row, -0.37) == -schedule.quintic(row, 0.37)
    ns = schedule.NS_QUINTIC
    assert abs(schedule.quintic(ns, 1.0) - 1.0) < 1e-15
    # p'(1) = p''(1) = 0 for the classical quintic
    a, b, c = ns
    assert abs(a + 3 * b + 5 * c) < 1e-15 and abs(6 * b + 20 * c) < 1e-15


def test_header_matches_designer(tmp_path):
    """The committed coefficient header is what the designer produces."""
    path = tmp_path / "coeffs.h"
    schedule.write_header(str(path))
    shipped = open(schedule.header_path()).read()
    assert path.read_text() == shipped
