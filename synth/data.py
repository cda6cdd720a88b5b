"""Seeded boundary data, densities and sphere target points.

`exact_harmonic` is the closed-form data of the paper's examples (Section 6,
eq. exact_bcs): u = Re sum_k c_k / (xi - xi_k), with xi the stereographic
image (x1 + i x2) / (1 - x3) of a sphere point (Section 3) and xi_k the image
of island k's centre.  u is the real part of a function analytic off the
islands and at infinity, hence harmonic for the Laplace-Beltrami operator in
the domain, so its trace is exact Dirichlet data and its values at targets
are the exact solution.
"""
import numpy as np


def _stereo(xyz):
    xyz = np.asarray(xyz, float)
    return (xyz[..., 0] + 1j * xyz[..., 1]) / (1.0 - xyz[..., 2])


def exact_harmonic(xyz, centers, coeffs):
    """u(x) = Re sum_k coeffs[k] / (xi(x) - xi(centers[k])).

    xyz: (n, 3) sphere points; centers: (M, 3); coeffs: (M,) complex.
    Returns (n,) float64.  Summed in blocks to bound memory.
    """
    xi = _stereo(xyz)
    pk = _stereo(centers)
    coeffs = np.asarray(coeffs, complex)
    out = np.empty(xi.shape[0])
    blk = max(1, (1 << 22) // max(1, pk.size))
    for a in range(0, xi.shape[0], blk):
        d = xi[a:a + blk, None] - pk[None, :]
        out[a:a + blk] = np.real((coeffs[None, :] / d).sum(axis=1))
    return out


def paper_data_coeffs(m):
    """The paper's data psi = 1/2 sum_k Re 1/(xi - xi_k): c_k = 1/2."""
    return np.full(m, 0.5 + 0j)


def random_data_coeffs(seed, islands):
    """c_k = rho_k (Z1 + i Z2)/sqrt(2), rho_k = planar size of island k.

    rho_k is bounded from the island's bounding cap: the largest distance
    between xi_k and the image of a point at geodesic distance r_max from
    the centre, sampled on 64 directions.
    """
    rng = np.random.default_rng(seed)
    m = islands.m
    z = (rng.standard_normal(m) + 1j * rng.standard_normal(m)) / np.sqrt(2)
    rmax = islands.max_radius()
    t = np.linspace(0, 2 * np.pi, 64, endpoint=False)
    rho = np.empty(m)
    for k in range(m):
        c = islands.center[k]
        e1 = islands.e1[k]
        e2 = np.cross(e1, c)
        u = np.cos(t)[:, None] * e1 + np.sin(t)[:, None] * e2
        x = np.cos(rmax[k]) * c + np.sin(rmax[k]) * u
        rho[k] = np.abs(_stereo(x) - _stereo(c)).max()
    return rho * z


def random_vector(seed, n):
    return np.random.default_rng(seed).standard_normal(n)


def sphere_targets(seed, count, islands, far_factor=1.3, far_nodes=10.0,
                   batch=65536):
    """Uniform points on the sphere, rejected when the angular distance to an
    island centre is below far_factor * r_max_k + far_nodes * l_k, with
    l_k = 2 pi far_factor r_max_k / N_k (trapezoidal evaluation is only
    accurate a few node spacings away from a curve)."""
    rng = np.random.default_rng(seed)
    rmax = islands.max_radius()
    ell = 2 * np.pi * far_factor * rmax / islands.n
    need = np.cos(far_factor * rmax + far_nodes * ell)   # reject if dot > need
    out = []
    got = 0
    while got < count:
        v = rng.standard_normal((batch, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        ok = np.ones(batch, bool)
        for a in range(0, islands.m, 256):
            dots = v @ islands.center[a:a + 256].T
            ok &= ~np.any(dots > need[a:a + 256][None, :], axis=1)
        v = v[ok]
        out.append(v)
        got += v.shape[0]
    return np.concatenate(out)[:count]


def near_curve_targets(islands, seed, dists, per=3):
    """Sphere points just outside the curves: for every island k and every
    d in dists, `per` points on the geodesic ray of a random parameter t
    (between nodes) at polar radius r(t) + d r0_k about the centre.
    Returns (points (n, 3), d of each point)."""
    rng = np.random.default_rng(seed)
    pts, tag = [], []
    nn = np.arange(1, 9)
    for k in range(islands.m):
        c = islands.center[k]
        e1 = islands.e1[k]
        e2 = np.cross(e1, c)
        n = int(islands.n[k])
        for d in dists:
            t = (rng.integers(n, size=per) + rng.uniform(0.1, 0.9, per)) \
                * 2 * np.pi / n
            a, b = islands.coef[k, :8], islands.coef[k, 8:]
            r = islands.r0[k] * (1.0 + (a[:, None] * np.cos(nn[:, None] * t)
                                        + b[:, None] * np.sin(nn[:, None] * t)
                                        ).sum(0))
            rr = r + d * islands.r0[k]
            u = np.cos(t)[:, None] * e1 + np.sin(t)[:, None] * e2
            pts.append(np.cos(rr)[:, None] * c + np.sin(rr)[:, None] * u)
            tag += [d] * per
    return np.concatenate(pts), np.array(tag)


def point_vortices(seed, count, islands):
    """Vortex positions in the domain (sphere_targets' rejection rule) and
    strengths uniform on (-2 pi, 2 pi), the range of Section 6, Example 2."""
    xyz = sphere_targets(seed, count, islands)
    gamma = np.random.default_rng(seed + 1).uniform(-2 * np.pi, 2 * np.pi,
                                                    count)
    return xyz, gamma
