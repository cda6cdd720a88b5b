"""Resampling of a closed curve on the sphere at points equally spaced in
arclength.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Section 6, Example 2 smooths coastline data, resamples it at equally spaced
points in arclength and alters the discretization of eq. disc_sphere
accordingly: the trapezoidal rule then runs over the arclength parameter
t = 2 pi s / L.  The paper gives no procedure; this is the plain definition
used here (the library's host routine computes the same thing faster):

* The input is n points x_j of a closed smooth curve at equispaced values
  tau_j = 2 pi j / n of some parameter, and a point c inside it.  The curve
  is carried to the plane by the stereographic projection from -c,
  zeta = (x.e1 + i x.e2) / (1 + x.c) (e2 = e1 x c), which maps c to 0 and
  is conformal with |dx| = 2 |d zeta| / (1 + |zeta|^2) on the unit sphere.
* zeta(tau) is the trigonometric interpolant of the samples, keeping the
  modes |k| <= K (K < n / 2; a smaller K low-pass filters the data).
* The arclength s(tau) = int_0^tau 2 |zeta'| / (1 + |zeta|^2) is computed
  by adaptive quadrature, L = s(2 pi), and node j of N sits at the tau_j
  with s(tau_j) = j L / N (root bracketing), so node 0 is the input's
  first point.
* Nodes x(t_j), x'(t_j), x''(t_j) for t = 2 pi s / L follow from the chain
  rule: tau_t = (L / 2 pi) / speed, tau_tt = -(speed' / speed) tau_t^2, then
  zeta_t, zeta_tt, and the inverse projection
  x = (2 Re zeta e1 + 2 Im zeta e2 + (1 - |zeta|^2) c) / (1 + |zeta|^2).
"""
import numpy as np
from scipy import integrate, optimize


def frame(c):
    """e1 = normalize(z x c) (x if c is on the z axis), e2 = e1 x c."""
    c = np.asarray(c, float)
    a = np.cross([0.0, 0.0, 1.0], c)
    if np.linalg.norm(a) < 1e-12:
        a = np.array([1.0, 0.0, 0.0])
    e1 = a / np.linalg.norm(a)
    e1 = e1 - np.dot(e1, c) * c
    e1 /= np.linalg.norm(e1)
    return e1, np.cross(e1, c)


class TrigCurve:
    """The planar image zeta(tau) of the samples as a trigonometric
    polynomial of degree K."""

    def __init__(self, x, c, n_modes=None):
        x = np.asarray(x, float)
        self.c = np.asarray(c, float)
        self.e1, self.e2 = frame(self.c)
        n = x.shape[0]
        zeta = (x @ self.e1 + 1j * (x @ self.e2)) / (1.0 + x @ self.c)
        K = (n - 1) // 2 if n_modes is None else int(n_modes)
        if not (0 < K and 2 * K + 1 <= n):
            raise ValueError("n_modes outside (0, n/2)")
        self.k = np.arange(-K, K + 1)
        tau = 2 * np.pi * np.arange(n) / n
        # c_k = (1/n) sum_j zeta_j exp(-i k tau_j)
        self.ck = np.exp(-1j * np.outer(self.k, tau)) @ zeta / n

    def derivs(self, tau):
        """zeta, zeta', zeta'' at tau (arrays)."""
        tau = np.atleast_1d(np.asarray(tau, float))
        e = np.exp(1j * np.outer(tau, self.k)) * self.ck[None, :]
        ik = 1j * self.k
        return e.sum(1), (e * ik).sum(1), (e * ik ** 2).sum(1)

    def speed(self, tau):
        z, z1, _ = self.derivs(tau)
        return 2.0 * np.abs(z1) / (1.0 + np.abs(z) ** 2)


def arclength(tc, a, b):
    val, _ = integrate.quad(lambda t: tc.speed(t)[0], a, b, epsabs=1e-15,
                            epsrel=1e-14, limit=400)
    return val


def resample(x, c, n_out, n_modes=None):
    """(x, x_t, x_tt) at n_out nodes equally spaced in arclength, each
    (n_out, 3), parameter t = 2 pi s / L; and L."""
    tc = TrigCurve(x, c, n_modes)
    # L by the periodic trapezoidal rule on a fine grid (spectrally exact
    # for the smooth periodic speed)
    m = 8 * max(len(tc.k), n_out)
    L = 2 * np.pi * tc.speed(2 * np.pi * np.arange(m) / m).mean()
    taus = np.zeros(n_out)
    prev, s_prev = 0.0, 0.0
    for j in range(1, n_out):
        target = j * L / n_out

        def f(t):
            return s_prev + arclength(tc, prev, t) - target
        hi = prev + 1e-3
        while f(hi) < 0:
            hi = min(2 * np.pi, hi + 0.1)
        taus[j] = optimize.brentq(f, prev, hi, xtol=1e-15, rtol=1e-15)
        s_prev = target
        prev = taus[j]
    z, z1, z2 = tc.derivs(taus)
    sp = 2.0 * np.abs(z1) / (1.0 + np.abs(z) ** 2)
    # speed' = 2 Re(conj(z') z'') / (|z'| (1 + |z|^2))
    #          - 4 |z'| Re(conj(z) z') / (1 + |z|^2)^2
    q0 = 1.0 + np.abs(z) ** 2
    dsp = (2.0 * np.real(np.conj(z1) * z2) / (np.abs(z1) * q0)
           - 4.0 * np.abs(z1) * np.real(np.conj(z) * z1) / q0 ** 2)
    tt = (L / (2 * np.pi)) / sp
    ttt = -(dsp / sp) * tt ** 2
    zt = z1 * tt
    ztt = z2 * tt ** 2 + z1 * ttt
    q = np.abs(z) ** 2
    qt = 2.0 * np.real(np.conj(z) * zt)
    qtt = 2.0 * np.real(np.conj(z) * ztt) + 2.0 * np.abs(zt) ** 2
    p = 1.0 + q
    w = 2.0 * z / p
    wt = 2.0 * zt / p - 2.0 * z * qt / p ** 2
    wtt = (2.0 * ztt / p - 4.0 * zt * qt / p ** 2 - 2.0 * z * qtt / p ** 2
           + 4.0 * z * qt ** 2 / p ** 3)
    h = 2.0 / p - 1.0
    ht = -2.0 * qt / p ** 2
    htt = -2.0 * qtt / p ** 2 + 4.0 * qt ** 2 / p ** 3

    def lift(wv, hv):
        return (np.real(wv)[:, None] * tc.e1 + np.imag(wv)[:, None] * tc.e2
                + hv[:, None] * tc.c)
    return lift(w, h), lift(wt, ht), lift(wtt, htt), L
