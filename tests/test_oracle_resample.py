"""Pins of the oracle's arclength resampling (oracle/resample.py) against
curves whose arclength parametrization is known in closed form or by
independent quadrature of the analytic curve, and of oracle Curves built
from node samples against the analytic construction."""
import numpy as np
import pytest
from scipy import integrate

import synth
from oracle import nystrom
from oracle.geometry import Curves, curve_on_sphere, radius_derivs
from oracle.resample import resample


def _cap_points(c, f1, f2, rho, theta):
    return (np.cos(rho) * c[None, :]
            + np.sin(rho) * (np.cos(theta)[:, None] * f1
                             + np.sin(theta)[:, None] * f2))


def test_circle_with_uneven_parameter():
    """A small circle sampled at theta(tau) = tau + 0.3 sin(tau): the
    arclength nodes sit at theta = 2 pi j / N, with t = theta, so x_t and
    x_tt are the theta-derivatives of the circle."""
    c = np.array([0.3, -0.5, 0.8])
    c /= np.linalg.norm(c)
    f1 = np.cross(c, [1.0, 0.0, 0.0])
    f1 /= np.linalg.norm(f1)
    f2 = np.cross(c, f1)
    rho = 0.35
    tau = 2 * np.pi * np.arange(64) / 64
    x_in = _cap_points(c, f1, f2, rho, tau + 0.3 * np.sin(tau))
    x, xt, xtt, L = resample(x_in, c, 48)
    th = 2 * np.pi * np.arange(48) / 48
    assert abs(L - 2 * np.pi * np.sin(rho)) < 1e-13
    assert np.abs(x - _cap_points(c, f1, f2, rho, th)).max() < 1e-13
    dx = np.sin(rho) * (-np.sin(th)[:, None] * f1 + np.cos(th)[:, None] * f2)
    assert np.abs(xt - dx).max() < 1e-12
    ddx = -np.sin(rho) * (np.cos(th)[:, None] * f1 + np.sin(th)[:, None] * f2)
    assert np.abs(xtt - ddx).max() < 1e-10


@pytest.fixture(scope="module")
def star():
    isl = synth.star_islands(21, 1, (0.2, 0.2), k_range=(5, 5), nodes=1024)
    x_in, _, _ = curve_on_sphere(isl.center[0], isl.e1[0], isl.r0[0],
                                 isl.coef[0], 1024)
    return isl, x_in, resample(x_in, isl.center[0], 160)


def test_star_nodes_on_the_curve_equally_spaced(star):
    """Resampled nodes lie on the analytic curve r(phi), and the analytic
    arclength between consecutive nodes (adaptive quadrature of |x'| of the
    analytic curve) is L / N."""
    isl, x_in, (x, xt, xtt, L) = star
    c, e1 = isl.center[0], isl.e1[0]
    e2 = np.cross(e1, c)
    rho = np.arccos(np.clip(x @ c, -1, 1))
    phi = np.unwrap(np.arctan2(x @ e2, x @ e1))
    r, _, _ = radius_derivs(isl.r0[0], isl.coef[0], phi)
    assert np.abs(rho - r).max() < 1e-12

    def speed(t):
        _, xt1, _ = _analytic(isl, np.array([t]))
        return np.linalg.norm(xt1[0])
    phi_c = np.concatenate([phi, [phi[0] + 2 * np.pi]])
    arcs = [integrate.quad(speed, phi_c[j], phi_c[j + 1], epsabs=1e-15,
                           epsrel=1e-13)[0] for j in range(len(phi))]
    assert np.abs(np.array(arcs) - L / len(phi)).max() < 1e-12 * L


def _analytic(isl, t):
    """x, x', x'' of the analytic island curve at parameters t."""
    c, e1 = isl.center[0], isl.e1[0]
    e2 = np.cross(e1, c)
    r, rt, rtt = radius_derivs(isl.r0[0], isl.coef[0], t)
    u = np.cos(t)[:, None] * e1 + np.sin(t)[:, None] * e2
    v = -np.sin(t)[:, None] * e1 + np.cos(t)[:, None] * e2
    cr, sr = np.cos(r)[:, None], np.sin(r)[:, None]
    x = cr * c + sr * u
    xt = rt[:, None] * (-sr * c + cr * u) + sr * v
    return x, xt, None


def test_star_arclength_parameter(star):
    """|x_t| = L / 2 pi at every node, x_t tangent to the sphere, and
    x_t . x_tt = 0 (constant speed)."""
    isl, x_in, (x, xt, xtt, L) = star
    sp = np.linalg.norm(xt, axis=1)
    assert np.abs(sp - L / (2 * np.pi)).max() < 1e-12 * L
    assert np.abs(np.einsum("ij,ij->i", x, xt)).max() < 1e-13
    assert np.abs(np.einsum("ij,ij->i", xt, xtt)).max() < 1e-10 * L ** 2


def test_curves_from_samples_match_analytic():
    """Curves built from node samples (x, x', x'' at the analytic nodes)
    equal the analytic construction, operator included."""
    isl = synth.star_islands(22, 3, (0.1, 0.2), nodes=[64, 80, 48])
    cv = Curves(isl)
    cs = Curves(samples=(cv.x, cv.xt, cv.xtt, isl.center, isl.n))
    assert np.abs(cs.xi - cv.xi).max() == 0.0
    rows = np.arange(cv.n)
    assert np.abs(nystrom.kernel_block(cs, rows)
                  - nystrom.kernel_block(cv, rows)).max() == 0.0


def test_arclength_nodes_solve_to_exact_solution():
    """The Nystrom system on arclength-resampled star curves (Section 6,
    Example 2's discretization) reaches the exact harmonic solution.  The
    curves are gentle (k = 2..3, amplitude 0.2): the arclength
    parametrization of a strongly undulating curve is analytic in a much
    thinner strip than its polar one (at k = 7, amplitude 0.3 its spectrum
    still holds 1e-2 of the derivative at mode 256)."""
    isl = synth.star_islands(23, 4, (0.1, 0.2), k_range=(2, 3), amp=0.2,
                             nodes=512)
    xs, xts, xtts = [], [], []
    for k in range(isl.m):
        x_in, _, _ = curve_on_sphere(isl.center[k], isl.e1[k], isl.r0[k],
                                     isl.coef[k], 512)
        x, xt, xtt, _ = resample(x_in, isl.center[k], 128)
        xs.append(x), xts.append(xt), xtts.append(xtt)
    cs = Curves(samples=(np.concatenate(xs), np.concatenate(xts),
                         np.concatenate(xtts), isl.center, [128] * isl.m))
    coeffs = synth.random_data_coeffs(24, isl)
    g = synth.exact_harmonic(cs.x, isl.center, coeffs)
    s, a = nystrom.solve_dense(cs, g)
    tg = synth.sphere_targets(25, 100, isl)
    from oracle import evaluate
    u = evaluate.evaluate(cs, s, a, tg)
    exact = synth.exact_harmonic(tg, isl.center, coeffs)
    assert np.abs(u - exact).max() < 1e-10 * np.abs(exact).max()
