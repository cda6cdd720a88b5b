"""Pins of the oracle's adjoint and shape derivatives (CPU only).

* A circular cap about the south pole with node data cos t has the exterior
  solution u = Re(R / zeta), R = tan(r0 / 2), in the stereographic plane
  (Section 3; the Laplace-Beltrami operator is conformally the planar
  Laplacian).  Moving the curve by delta r(t) with the data attached to the
  parameter t changes u by the harmonic extension of
  -grad u . delta x = cos t delta rho(t) / R on |zeta| = R, where
  delta rho = (1/2) sec^2(r0/2) delta r; for delta r = r0 cos(mt) (or sin)
  this is a sum of two Fourier modes extended as Re((R/zeta)^k) (or
  Re(i (R/zeta)^k)).  The finite-difference gradient of J = w . u must match
  it; a swapped coefficient, a wrong mode index or step would not.
* dJ/dg by the dense adjoint against the exact change of the linear map
  g -> J on random directions.
* The transposed solve against the forward operator by duality.
* The shape gradient by the adjoint assembly (lambda and the derivatives
  of the assembled matrices) against the finite difference of the whole
  pipeline on three islands, for two of them (a transposed system, a wrong
  sign of the lambda term or a swapped island index would not agree).
"""
import numpy as np
import pytest

import synth
from oracle import adjoint, nystrom, evaluate
from oracle.geometry import Curves


def _stereo(x):
    return (x[:, 0] + 1j * x[:, 1]) / (1.0 - x[:, 2])


def _cap_targets(r0, count, seed):
    """Sphere points with colatitude below pi - r0 - 0.35 (off the curve)."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        if np.arccos(v[2]) < np.pi - r0 - 0.35:
            out.append(v)
    return np.array(out)


@pytest.fixture(scope="module")
def cap_case():
    r0, n = 0.5, 96
    isl = synth.cap_island(colat=np.pi, radius=r0, n=n)
    t = 2 * np.pi * np.arange(n) / n
    g = np.cos(t)
    tg = _cap_targets(r0, 30, 7)
    w = np.random.default_rng(8).standard_normal(len(tg))
    return r0, isl, g, tg, w


def test_cap_cos_data_solution(cap_case):
    r0, isl, g, tg, w = cap_case
    cv = Curves(isl)
    sigma, A = nystrom.solve_dense(cv, g)
    u = evaluate.evaluate(cv, sigma, A, tg)
    exact = np.real(np.tan(r0 / 2) / _stereo(tg))
    assert np.abs(u - exact).max() < 1e-12


def test_cap_shape_derivative_closed_form(cap_case):
    r0, isl, g, tg, w = cap_case
    fd = adjoint.grad_shape_fd(isl, g, tg, w)[0]
    R = np.tan(r0 / 2)
    c0 = 0.5 * r0 / np.cos(r0 / 2) ** 2
    q = R / _stereo(tg)
    exp = np.zeros(16)
    for m in range(1, 9):
        ua = np.real(q ** (m + 1)) + np.real(q ** (m - 1))
        ub = np.real(1j * q ** (m + 1)) + np.real(1j * q ** (m - 1))
        exp[m - 1] = c0 / (2 * R) * np.dot(w, ua)
        exp[7 + m] = c0 / (2 * R) * np.dot(w, ub)
    assert np.abs(fd - exp).max() < 1e-8 * np.abs(exp).max()


@pytest.fixture(scope="module")
def stars3():
    isl = synth.star_islands(71, 3, (0.12, 0.25), nodes=[64, 80, 72])
    cv = Curves(isl)
    tg = synth.sphere_targets(72, 25, isl)
    w = np.random.default_rng(73).standard_normal(len(tg))
    g = synth.exact_harmonic(cv.x, isl.center,
                             synth.random_data_coeffs(74, isl))
    return isl, cv, tg, w, g


def test_grad_data_matches_linear_change(stars3):
    isl, cv, tg, w, g = stars3
    grad = adjoint.grad_data(cv, tg, w)
    J0 = adjoint.functional(isl, g, tg, w)
    rng = np.random.default_rng(75)
    for _ in range(3):
        d = rng.standard_normal(cv.n)
        dJ = adjoint.functional(isl, g + d, tg, w) - J0
        assert abs(dJ - grad @ d) < 1e-10 * max(abs(dJ), np.abs(grad).sum())


def test_adjoint_solve_duality(stars3):
    isl, cv, tg, w, g = stars3
    rng = np.random.default_rng(76)
    rs, ra = rng.standard_normal(cv.n), rng.standard_normal(cv.m)
    ls, la = adjoint.adjoint_solve(cv, rs, ra)
    for _ in range(3):
        xs, xa = rng.standard_normal(cv.n), rng.standard_normal(cv.m)
        top, bot = nystrom.apply_system(cv, xs, xa)
        lhs = top @ ls + bot @ la
        rhs = xs @ rs + xa @ ra
        assert abs(lhs - rhs) < 1e-10 * (np.abs(top @ ls) + np.abs(bot @ la))


def test_eval_transpose_duality(stars3):
    isl, cv, tg, w, g = stars3
    rng = np.random.default_rng(77)
    gs, ga = adjoint.eval_transpose(cv, tg, w)
    xs, xa = rng.standard_normal(cv.n), rng.standard_normal(cv.m)
    u = evaluate.evaluate(cv, xs, xa, tg)
    assert abs(w @ u - (gs @ xs + ga @ xa)) < 1e-12 * np.abs(w).sum() * np.abs(u).max()


def test_shape_gradient_adjoint_matches_pipeline_fd(stars3):
    isl, cv, tg, w, g = stars3
    idx = [0, 2]
    adj = adjoint.grad_shape_adjoint(isl, g, tg, w, islands_idx=idx)
    fd = adjoint.grad_shape_fd(isl, g, tg, w, islands_idx=idx)
    scale = np.abs(fd[idx]).max()
    assert scale > 0
    assert np.abs(adj[idx] - fd[idx]).max() < 1e-8 * scale
    assert np.abs(adj[1]).max() == 0.0  # island 1 not asked for
