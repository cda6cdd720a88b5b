"""Pins of the oracle's close evaluation (oracle/close.py) against what the
mathematics fixes: the exact harmonic solution at targets approaching the
curves (where the plain trapezoidal rule fails), the Dirichlet data at the
nodes themselves (the exterior limit of the representation is the boundary
value), the plain rule far from the curves, and exact derivatives of
trigonometric polynomials."""
import numpy as np
import pytest

import synth
from oracle import nystrom, evaluate
from oracle.close import evaluate_close, spectral_derivative
from oracle.geometry import Curves


@pytest.fixture(scope="module")
def solved():
    # 320 nodes per curve resolve these densities to ~1e-13 (at 128 the
    # density's own discretization error is ~1e-6 near the curves)
    isl = synth.star_islands(12, 5, (0.1, 0.25), nodes=320)
    cv = Curves(isl)
    coeffs = synth.random_data_coeffs(13, isl)
    g = synth.exact_harmonic(cv.x, isl.center, coeffs)
    s, a = nystrom.solve_dense(cv, g)
    return isl, cv, coeffs, g, s, a


def test_spectral_derivative_exact_on_trig_polynomials():
    for n in (16, 17, 64):
        t = 2 * np.pi * np.arange(n) / n
        f = 1.5 + np.sin(3 * t) - 0.25 * np.cos(5 * t) + 0.5 * np.sin(7 * t)
        df = 3 * np.cos(3 * t) + 1.25 * np.sin(5 * t) + 3.5 * np.cos(7 * t)
        assert np.abs(spectral_derivative(f) - df).max() < 1e-12


def test_close_targets_reach_the_exact_solution(solved):
    """u = Re sum c_k / (xi - xi_k) at targets 1e-1 .. 1e-6 island radii
    outside the curves: the compensated rule stays within 1e-10 while the
    plain trapezoidal rule loses all accuracy."""
    isl, cv, coeffs, g, s, a = solved
    dists = [1e-1, 1e-2, 1e-3, 1e-4, 1e-6]
    tg, tag = synth.near_curve_targets(isl, 14, dists)
    exact = synth.exact_harmonic(tg, isl.center, coeffs)
    scale = np.abs(exact).max()
    u = evaluate_close(cv, s, a, tg)
    assert np.abs(u - exact).max() < 1e-10 * scale
    plain = evaluate.evaluate(cv, s, a, tg)
    worst = np.abs(plain - exact)[tag <= 1e-3].max()
    assert worst > 1e-4 * scale


def test_nodes_give_the_dirichlet_data(solved):
    """At the nodes the compensated rule returns the exterior boundary
    value, and the representation's exterior limit is the data g."""
    isl, cv, coeffs, g, s, a = solved
    rows = np.arange(0, cv.n, 7)
    u = evaluate_close(cv, s, a, cv.x[rows])
    assert np.abs(u - g[rows]).max() < 1e-10 * np.abs(g).max()


def test_far_targets_match_the_plain_rule(solved):
    isl, cv, coeffs, g, s, a = solved
    tg = synth.sphere_targets(15, 60, isl)
    tg = np.concatenate([tg, [[0.0, 0.0, 1.0]]])
    u = evaluate_close(cv, s, a, tg)
    ref = evaluate.evaluate(cv, s, a, tg)
    assert np.abs(u - ref).max() < 1e-11 * np.abs(ref).max()
