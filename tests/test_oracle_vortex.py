"""Pin of the oracle's point-vortex decomposition (oracle/vortex.py,
Section 6, Example 2) against the closed-form solution for one circular
cap and one vortex with zero data on the coastline.

Stereographic projection (Section 3) maps the cap to a disk |xi - a| < R
and the domain to its exterior with infinity (the north pole) included.
On the circle, with w = (xi - a)/R, |w| = 1, the data of psi* is
-Gamma G(x, v) = (Gamma / 4 pi) [log 2 + 2 log|xi - eta| - log(1 + |xi|^2)
- log(1 + |eta|^2)] (chord identity), and each term has a bounded harmonic
extension to |w| > 1:

* log|xi - eta| -> log R + log|w_eta| + log|1 - 1 / (conj(w_eta) w)|,
  w_eta = (eta - a)/R (|w_eta| > 1);
* log(1 + |xi|^2) -> log(R |a|) - log|w1| + 2 log|1 - w1 / w|, where
  R conj(a) w^2 + (1 + |a|^2 + R^2) w + R a = R conj(a)(w - w1)(w - 1/conj(w1)),
  |w1| < 1 (on |w| = 1, 1 + |xi|^2 equals that quadratic over w);

using |w - b| = |1 - b / w| for |b| < 1 and |w - b| = |b| |w - 1/conj(b)|
on |w| = 1.  Then psi = psi* + Gamma G(x, v) everywhere in the domain.
"""
import numpy as np
import pytest

import synth
from oracle import vortex
from oracle.geometry import Curves

LOG2 = np.log(2.0)


def _stereo(xyz):
    xyz = np.atleast_2d(xyz)
    return (xyz[:, 0] + 1j * xyz[:, 1]) / (1.0 - xyz[:, 2])


def _greens(x, v):
    d2 = ((x - v[None, :]) ** 2).sum(1)
    return -np.log(d2) / (4 * np.pi) + LOG2 / (4 * np.pi)


def closed_form(targets, colat, rho, v, gamma):
    """psi at targets for the cap (centre at colatitude `colat` in the x-z
    plane, angular radius rho), vortex v of strength gamma, zero data."""
    p, q = 1.0 / np.tan((colat - rho) / 2), 1.0 / np.tan((colat + rho) / 2)
    a, R = 0.5 * (p + q), 0.5 * (p - q)
    xi = _stereo(targets)
    eta = _stereo(v)[0]
    w = (xi - a) / R
    weta = (eta - a) / R
    ext_log_d = np.log(R) + np.log(abs(weta)) + np.log(
        np.abs(1 - 1 / (np.conj(weta) * w)))
    alpha = 1 + abs(a) ** 2 + R ** 2
    roots = np.roots([R * np.conj(a), alpha, R * a])
    w1 = roots[np.argmin(np.abs(roots))]
    ext_log_q = (np.log(R * abs(a)) - np.log(abs(w1))
                 + 2 * np.log(np.abs(1 - w1 / w)))
    psi_star = gamma / (4 * np.pi) * (LOG2 + 2 * ext_log_d - ext_log_q
                                      - np.log(1 + abs(eta) ** 2))
    return psi_star + gamma * _greens(targets, v)


@pytest.mark.parametrize("vcol,vlon", [(1.8, 0.7), (0.6, 2.5)])
def test_cap_with_one_vortex(vcol, vlon):
    colat, rho = 1.0, 0.4
    isl = synth.cap_island(colat, rho, 256)
    cv = Curves(isl)
    v = np.array([np.sin(vcol) * np.cos(vlon), np.sin(vcol) * np.sin(vlon),
                  np.cos(vcol)])
    gamma = 1.7
    s, A = vortex.solve(cv, np.zeros(cv.n), v[None, :], [gamma])
    tg = synth.sphere_targets(7, 80, isl)
    # keep targets away from the vortex itself
    tg = tg[np.linalg.norm(tg - v, axis=1) > 0.05]
    psi = vortex.evaluate_psi(cv, s, A, tg, v[None, :], [gamma])
    exact = closed_form(tg, colat, rho, v, gamma)
    assert np.abs(psi - exact).max() < 1e-11 * np.abs(exact).max()
    # the closed form vanishes on the coastline
    assert np.abs(closed_form(cv.x, colat, rho, v, gamma)).max() < 1e-12


def test_vortex_field_is_the_greens_sum():
    rng = np.random.default_rng(3)
    pts = rng.standard_normal((20, 3))
    pts /= np.linalg.norm(pts, axis=1, keepdims=True)
    vs = rng.standard_normal((4, 3))
    vs /= np.linalg.norm(vs, axis=1, keepdims=True)
    gam = rng.uniform(-2 * np.pi, 2 * np.pi, 4)
    ref = sum(gam[j] * _greens(pts, vs[j]) for j in range(4))
    assert np.abs(vortex.vortex_field(pts, vs, gam) - ref).max() < 1e-14
