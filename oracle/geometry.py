"""Island curves on the unit sphere and their stereographic images.

Section 3: xi = (x1 + i x2) / (1 - x3) maps the sphere (north pole removed)
to the plane.  Section 5: each curve is sampled at N equispaced parameter
values t_j = 2 pi j / N with spacing h = 2 pi / N, and the Nystrom rule needs
xi, d xi/dt and d^2 xi/dt^2 at the nodes.  Everything here is FP64.
"""
import numpy as np


class SampledIslands:
    """Islands given by their node samples only (Section 6, Example 2):
    a point c_k inside each curve (its log source) and the node counts."""

    def __init__(self, centers, nodes):
        self.center = np.asarray(centers, float)
        self.n = np.asarray(nodes, np.int64)

    @property
    def m(self):
        return int(self.center.shape[0])


class Curves:
    """All nodes of all islands, curve-major (island 0's nodes first).

    Either analytic islands (`islands`: centre, frame, radius function), or
    `samples` = (x, x_t, x_tt, centers, nodes_per_curve): the nodes of
    every curve at t_j = 2 pi j / N_k of its own parameter, with the first
    and second t-derivatives, curve-major."""

    def __init__(self, islands=None, samples=None):
        if samples is not None:
            x, xt, xtt, centers, nodes = samples
            islands = SampledIslands(centers, nodes)
            self.x = np.asarray(x, float)
            self.xt = np.asarray(xt, float)
            self.xtt = np.asarray(xtt, float)
        self.islands = islands
        m = islands.m
        xs, xts, xtts, isl, hs = [], [], [], [], []
        for k in range(m):
            n = int(islands.n[k])
            if samples is None:
                x, xt, xtt = curve_on_sphere(islands.center[k],
                                             islands.e1[k], islands.r0[k],
                                             islands.coef[k], n)
                xs.append(x), xts.append(xt), xtts.append(xtt)
            isl.append(np.full(n, k))
            hs.append(np.full(n, 2 * np.pi / n))
        if samples is None:
            self.x = np.concatenate(xs)
            self.xt = np.concatenate(xts)
            self.xtt = np.concatenate(xtts)
        self.island = np.concatenate(isl)
        self.h = np.concatenate(hs)
        self.xi, self.dxi, self.ddxi = stereographic(self.x, self.xt, self.xtt)
        self.sign_per_island = np.array(
            [orientation_sign(self.xi[self.island == k],
                              self.dxi[self.island == k])
             for k in range(m)])
        self.s = self.sign_per_island[self.island]
        self.center = islands.center
        self.center_xi = (self.center[:, 0] + 1j * self.center[:, 1]) / (
            1.0 - self.center[:, 2])

    @property
    def n(self):
        return self.x.shape[0]

    @property
    def m(self):
        return self.islands.m

    def offsets(self):
        return np.concatenate([[0], np.cumsum(self.islands.n)])


def radius_derivs(r0, coef, t):
    """r(t) = r0 (1 + sum_n a_n cos nt + b_n sin nt) and its t-derivatives."""
    a = np.asarray(coef[:8], float)
    b = np.asarray(coef[8:16], float)
    nn = np.arange(1, 9)[:, None]
    c = np.cos(nn * t[None, :])
    s = np.sin(nn * t[None, :])
    r = r0 * (1.0 + (a[:, None] * c + b[:, None] * s).sum(0))
    rt = r0 * (nn * (-a[:, None] * s + b[:, None] * c)).sum(0)
    rtt = r0 * (nn ** 2 * (-a[:, None] * c - b[:, None] * s)).sum(0)
    return r, rt, rtt


def curve_on_sphere(center, e1, r0, coef, n):
    """Points x(t) at geodesic distance r(t) from the centre c in direction
    u(t) = cos t e1 + sin t e2 (e2 = e1 x c), with x' and x''.

    x = cos r c + sin r u; the derivatives follow from u' = v, v' = -u with
    v = -sin t e1 + cos t e2.
    """
    c = np.asarray(center, float)
    e1 = np.asarray(e1, float)
    e2 = np.cross(e1, c)
    t = 2 * np.pi * np.arange(n) / n
    r, rt, rtt = radius_derivs(r0, coef, t)
    u = np.cos(t)[:, None] * e1 + np.sin(t)[:, None] * e2
    v = -np.sin(t)[:, None] * e1 + np.cos(t)[:, None] * e2
    cr, sr = np.cos(r)[:, None], np.sin(r)[:, None]
    rt_, rtt_ = rt[:, None], rtt[:, None]
    x = cr * c + sr * u
    xt = rt_ * (-sr * c + cr * u) + sr * v
    xtt = (-(rtt_ * sr + rt_ ** 2 * cr) * c
           + (rtt_ * cr - rt_ ** 2 * sr - sr) * u
           + 2 * rt_ * cr * v)
    return x, xt, xtt


def stereographic(x, xt, xtt):
    """xi = w / d with w = x1 + i x2, d = 1 - x3, and its first two
    t-derivatives by the quotient rule (d' = -x3', d'' = -x3'')."""
    w = x[:, 0] + 1j * x[:, 1]
    wt = xt[:, 0] + 1j * xt[:, 1]
    wtt = xtt[:, 0] + 1j * xtt[:, 1]
    d = 1.0 - x[:, 2]
    x3t = xt[:, 2]
    x3tt = xtt[:, 2]
    xi = w / d
    dxi = wt / d + w * x3t / d ** 2
    ddxi = (wtt / d + 2 * wt * x3t / d ** 2 + w * x3tt / d ** 2
            + 2 * w * x3t ** 2 / d ** 3)
    return xi, dxi, ddxi


def orientation_sign(xi, dxi):
    """+1 when the island lies to the left of the planar traversal.

    An island (never containing the north pole: such geometries are
    rejected) is the bounded interior of its planar curve, which lies to the
    left exactly when the curve runs counter-clockwise, i.e. when its signed
    area (1/2) sum Im(conj(xi) xi') is positive.
    """
    area = np.sum(np.imag(np.conj(xi) * dxi))
    return 1.0 if area > 0 else -1.0


def island_area(islands, k, n_quad=4096):
    """Spherical area of island k: integral over t of (1 - cos r(t)) dt,
    by the periodic trapezoidal rule (spectrally accurate)."""
    t = 2 * np.pi * np.arange(n_quad) / n_quad
    r, _, _ = radius_derivs(islands.r0[k], islands.coef[k], t)
    return np.sum(1.0 - np.cos(r)) * (2 * np.pi / n_quad)
