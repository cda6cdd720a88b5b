"""Island geometries on the unit sphere (seeded).

An island is described the way the library's C-ABI takes it:

* ``center`` -- unit vector c, the island's centre and log-source point;
* ``e1``     -- unit vector orthogonal to c giving the t = 0 direction
  (the second frame vector is e2 = e1 x c);
* ``r0``     -- mean geodesic radius in radians;
* ``coef``   -- 16 Fourier shape coefficients a_1..a_8, b_1..b_8 of the
  geodesic polar radius r(t) = r0 (1 + sum_n a_n cos nt + b_n sin nt);
* ``n``      -- number of equispaced nodes on the boundary curve.

The paper's examples use ellipses whose sizes and placement it does not give
(Section 6, Examples 1 and 3); star curves r0 (1 + 0.3 cos kt) placed by
random sequential addition stand in for them.
"""
from dataclasses import dataclass, field
import numpy as np


@dataclass
class IslandSet:
    center: np.ndarray          # (M, 3)
    e1: np.ndarray              # (M, 3)
    r0: np.ndarray              # (M,)
    coef: np.ndarray            # (M, 16)
    n: np.ndarray               # (M,) int
    meta: dict = field(default_factory=dict)

    @property
    def m(self):
        return int(self.r0.shape[0])

    @property
    def n_total(self):
        return int(self.n.sum())

    def subset(self, idx):
        idx = np.asarray(idx)
        return IslandSet(self.center[idx].copy(), self.e1[idx].copy(),
                         self.r0[idx].copy(), self.coef[idx].copy(),
                         self.n[idx].copy(), dict(self.meta))

    def with_nodes(self, n):
        out = IslandSet(self.center.copy(), self.e1.copy(), self.r0.copy(),
                        self.coef.copy(), np.full(self.m, int(n), np.int32)
                        if np.isscalar(n) else np.asarray(n, np.int32).copy(),
                        dict(self.meta))
        return out

    def rotated(self, rot):
        """Rigid rotation of every island (rot: 3x3 orthogonal, det +1)."""
        rot = np.asarray(rot, float)
        return IslandSet(self.center @ rot.T, self.e1 @ rot.T, self.r0.copy(),
                         self.coef.copy(), self.n.copy(), dict(self.meta))

    def max_radius(self):
        """Upper bound of r(t) from the coefficient magnitudes."""
        return self.r0 * (1.0 + np.abs(self.coef).sum(axis=1))


def _frame(center, phi):
    """e1 = cos(phi) a + sin(phi) b with a = normalize(z x c), b = c x a."""
    z = np.array([0.0, 0.0, 1.0])
    a = np.cross(z, center)
    na = np.linalg.norm(a)
    if na < 1e-12:                      # centre on the z axis
        a = np.array([1.0, 0.0, 0.0])
    else:
        a = a / na
    b = np.cross(center, a)
    e1 = np.cos(phi) * a + np.sin(phi) * b
    # remove rounding drift so that |e1| = 1 and e1 . c = 0 to ~1e-16
    e1 = e1 - np.dot(e1, center) * center
    return e1 / np.linalg.norm(e1)


def cap_island(colat=1.0, radius=0.4, n=256):
    """One circular cap: centre at colatitude `colat` in the x-z plane."""
    c = np.array([np.sin(colat), 0.0, np.cos(colat)])
    e1 = _frame(c, 0.0)
    return IslandSet(c[None, :], e1[None, :], np.array([radius]),
                     np.zeros((1, 16)), np.array([n], np.int32),
                     {"kind": "cap", "colat": colat, "radius": radius})


def _unit_random(rng):
    while True:
        v = rng.standard_normal(3)
        nv = np.linalg.norm(v)
        if nv > 1e-8:
            return v / nv


def star_islands(seed, m, r0_range, k_range=(3, 7), nodes=256, amp=0.3,
                 pole_margin=0.1, gap_factor=6.0, max_tries=200000):
    """Random sequential addition of m star islands r0 (1 + amp cos k t).

    Placement rule: a centre is rejected when its colatitude is below
    (1+amp) r0 + pole_margin (so the north pole stays in the domain), or when
    its angular distance to an earlier centre is below
    (1+amp)(r0_a + r0_b) + gap_factor * max(l_a, l_b), with l the node spacing
    2 pi (1+amp) r0 / N of the larger curve.  `nodes` is an int or a
    per-island array.
    """
    rng = np.random.default_rng(seed)
    nodes = np.broadcast_to(np.asarray(nodes, np.int64), (m,)).copy()
    r0 = rng.uniform(r0_range[0], r0_range[1], size=m)
    kk = rng.integers(k_range[0], k_range[1] + 1, size=m)
    phi = rng.uniform(0.0, 2 * np.pi, size=m)
    rmax = (1.0 + amp) * r0
    ell = 2 * np.pi * rmax / nodes
    centers = np.zeros((m, 3))
    placed = 0
    tries = 0
    while placed < m:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random sequential addition did not converge")
        c = _unit_random(rng)
        colat = np.arccos(np.clip(c[2], -1.0, 1.0))
        if colat < rmax[placed] + pole_margin:
            continue
        if placed:
            dots = np.clip(centers[:placed] @ c, -1.0, 1.0)
            ang = np.arccos(dots)
            need = rmax[:placed] + rmax[placed] + gap_factor * np.maximum(
                ell[:placed], ell[placed])
            if np.any(ang < need):
                continue
        centers[placed] = c
        placed += 1
    e1 = np.stack([_frame(centers[i], phi[i]) for i in range(m)])
    coef = np.zeros((m, 16))
    coef[np.arange(m), kk - 1] = amp
    area = 2 * np.pi * (1 - np.cos(rmax))
    meta = {"kind": "star", "seed": seed, "k": kk, "tries": tries,
            "coverage_bound": float(area.sum() / (4 * np.pi))}
    return IslandSet(centers, e1, r0, coef, nodes.astype(np.int32), meta)


def deep_tree_islands(nodes=128, amp=0.3):
    """Seven star islands from near the north pole to within 1e-3 rad of the
    south pole, their radii shrinking from 0.25 to 2e-5 rad.  Stereographic
    projection magnifies the northern ones and shrinks the southern ones
    (the distortion the paper points to in Section 6, Example 3), so the
    quadtree over their images needs 20 or more levels."""
    spec = [  # (colatitude, longitude, r0, k)
        (0.45, 0.0, 0.25, 3),
        (1.2, 1.0, 0.15, 5),
        (2.0, 2.5, 0.08, 4),
        (2.8, 4.0, 0.02, 6),
        (3.1, 0.5, 0.002, 3),
        (3.1365, 2.0, 1e-4, 5),
        (3.1405, 4.5, 2e-5, 3),
    ]
    m = len(spec)
    c = np.array([[np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t)]
                  for t, p, _, _ in spec])
    e1 = np.stack([_frame(c[i], 0.3 * i) for i in range(m)])
    r0 = np.array([sp[2] for sp in spec])
    coef = np.zeros((m, 16))
    for i, sp in enumerate(spec):
        coef[i, sp[3] - 1] = amp
    nodes = np.broadcast_to(np.asarray(nodes, np.int64), (m,)).copy()
    return IslandSet(c, e1, r0, coef, nodes.astype(np.int32),
                     {"kind": "deep"})


# Workload recipes (sizes and distributions of the paper's examples, with
# star curves standing in for its ellipses).
CONFIGS = {
    "cap256": dict(kind="cap", colat=1.0, radius=0.4, n=256),
    "stars40x512": dict(kind="star", seed=2, m=40, r0_range=(0.05, 0.15),
                        nodes=512),
    "stars1000x256": dict(kind="star", seed=3, m=1000, r0_range=(0.01, 0.03),
                          nodes=256),
    "stars2000x512": dict(kind="star", seed=5, m=2000, r0_range=(0.01, 0.03),
                          nodes=512),
}


def config_islands(name, nodes=None):
    cfg = dict(CONFIGS[name])
    if cfg.pop("kind") == "cap":
        if nodes is not None:
            cfg["n"] = nodes
        return cap_island(**cfg)
    if nodes is not None:
        cfg["nodes"] = nodes
    return star_islands(**cfg)


def batch_geometries(n_geoms=64, base_seed=4000, m_range=(10, 400),
                     node_choices=(128, 256, 384, 512),
                     total_range=(4096, 102400)):
    """Uneven batch: M_b ~ U{10..400}, N_k ~ U{128,256,384,512} per island,
    redrawn until the total node count lies in total_range; radii
    r0 ~ U[0.5, 1.5] * 0.25 / sqrt(M_b)."""
    out = []
    for b in range(n_geoms):
        rng = np.random.default_rng(base_seed + b)
        while True:
            m = int(rng.integers(m_range[0], m_range[1] + 1))
            nodes = rng.choice(np.asarray(node_choices), size=m)
            if total_range[0] <= nodes.sum() <= total_range[1]:
                break
        scale = 0.25 / np.sqrt(m)
        out.append(star_islands(base_seed + b, m, (0.5 * scale, 1.5 * scale),
                                nodes=nodes))
    return out
