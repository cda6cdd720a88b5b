"""Close evaluation of the representation near the curves.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The representation of eq. eqn:u_multi (Section 4.1) is evaluated in the
paper with the same trapezoidal rule as the equation (Section 5).  That rule
is spectrally accurate only a few node spacings away from a curve: the
integrand's near-singularity at a close target is not resolved.  The paper
reports solution errors at sample points only (Section 6) and is silent on
targets near a curve.  Here every island's Cauchy sum is replaced by the
globally compensated trapezoidal rule for exterior Cauchy integrals
(Ioakimidis, Papadakis and Perdios 1991; Helsing and Ojala 2008; Barnett,
Wu and Veerapaneni 2015), which is accurate at every distance:

* The Cauchy part of island k's double layer at a planar point z is
  -s_k Re v(z), v(z) = (1/2 pi i) sum_j sigma_j a_j with
  a_j = h xi'_j / (xi_j - z) (the trapezoidal form of the Cauchy integral
  (1/2 pi i) int sigma(y) / (y - z) dy over the curve).
* v is analytic outside the island and vanishes at infinity, so it is the
  exterior Cauchy integral of its own exterior boundary values V:
  (1/2 pi i) int V(y) / (y - z) dy = -s_k v(z) for z outside.  By the
  Plemelj formulas, V(y_i) = (1/2 pi i) int (sigma(y) - sigma(y_i)) / (y - y_i) dy,
  whose integrand is smooth, so the trapezoidal rule is spectrally accurate:
  V_i = (1/2 pi i) [ sum_{j != i} h (sigma_j - sigma_i) xi'_j / (xi_j - xi_i)
                     + h sigma'_i ],
  with sigma' the derivative of the trigonometric interpolant of sigma.
* The quadrature error of sum_j V_j a_j at a close z is, to leading order,
  V(z) times that of sum_j a_j (whose exact value is 0 outside the island),
  which gives the compensated value
  v(z) = sum_j V_j a_j / (sum_j a_j - 2 pi i s_k),
  exact in the limit z -> xi_i (it tends to V_i).

Every target is evaluated this way against every island (the compensated
sum equals the plain one to rounding far from a curve).  Targets must lie in
the domain (outside every island); the north pole keeps no Cauchy part.
"""
import numpy as np

from .nystrom import greens


def spectral_derivative(f):
    """d f / d t at t_j = 2 pi j / N of the trigonometric interpolant of the
    periodic samples f (the Nyquist mode of even N carries no derivative)."""
    f = np.asarray(f, float)
    n = f.shape[0]
    k = np.fft.fftfreq(n, d=1.0 / n)
    if n % 2 == 0:
        k[n // 2] = 0.0
    return np.real(np.fft.ifft(1j * k * np.fft.fft(f)))


def boundary_values(cv, sigma, k):
    """Exterior boundary values V_i of island k's Cauchy integral of sigma
    at its nodes (complex, one per node)."""
    sel = cv.island == k
    xi, dxi = cv.xi[sel], cv.dxi[sel]
    s = np.asarray(sigma, float)[sel]
    h = cv.h[sel][0]
    n = xi.shape[0]
    ds = spectral_derivative(s)
    V = np.empty(n, complex)
    for i in range(n):
        d = xi - xi[i]
        d[i] = 1.0
        terms = (s - s[i]) * dxi / d
        terms[i] = 0.0
        V[i] = (h * terms.sum() + h * ds[i]) / (2j * np.pi)
    return V


def cauchy_close(cv, sigma, k, z, V=None):
    """Island k's Cauchy part -s_k Re v(z) at planar points z by the
    compensated rule (z on a node gives the boundary value)."""
    sel = cv.island == k
    xi, dxi = cv.xi[sel], cv.dxi[sel]
    h = cv.h[sel][0]
    sk = cv.sign_per_island[k]
    if V is None:
        V = boundary_values(cv, sigma, k)
    z = np.atleast_1d(np.asarray(z, complex))
    out = np.empty(z.shape[0])
    for t, zt in enumerate(z):
        d = xi - zt
        hit = np.flatnonzero(d == 0)
        if hit.size:
            v = V[hit[0]]
        else:
            a = h * dxi / d
            v = (V * a).sum() / (a.sum() - 2j * np.pi * sk)
        out[t] = -sk * np.real(v)
    return out


def evaluate_close(cv, sigma, A, targets):
    """u at sphere targets (eq. eqn:u_multi) with every island's Cauchy sum
    taken by the compensated rule; the correction term and the log sources
    as in evaluate.evaluate."""
    targets = np.asarray(targets, float)
    sigma = np.asarray(sigma, float)
    A = np.asarray(A, float)
    den = 1.0 - targets[:, 2]
    at_pole = den <= 0.0
    z = np.where(at_pole, 0.0, (targets[:, 0] + 1j * targets[:, 1])
                 / np.where(at_pole, 1.0, den))
    w = cv.s * cv.h / (2 * np.pi) * sigma
    corr = np.sum(w * np.imag(np.conj(cv.xi) * cv.dxi /
                              (1 + np.abs(cv.xi) ** 2)))
    out = corr + greens(targets, cv.center) @ A
    live = ~at_pole
    for k in range(cv.m):
        V = boundary_values(cv, sigma, k)
        out[live] += cauchy_close(cv, sigma, k, z[live], V)
    return out
