"""Pins of the CPU oracle against facts fixed by the paper and by mathematics,
not by the oracle itself.  Each test names the part of the oracle a plausible
mistake would break.
"""
import numpy as np
import pytest

import synth
from oracle import nystrom, gmres, evaluate
from oracle.geometry import Curves, island_area, orientation_sign


def _rot(axis, ang):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    k = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]],
                  [-axis[1], axis[0], 0]])
    return np.eye(3) + np.sin(ang) * k + (1 - np.cos(ang)) * k @ k


def _full_k(cv):
    return nystrom.kernel_block(cv, np.arange(cv.n))


@pytest.fixture(scope="module")
def stars6():
    return synth.star_islands(11, 6, (0.1, 0.3), nodes=96)


# --- T1: circular cap, every entry in closed form ---------------------------
@pytest.mark.parametrize("colat,rho,n,rot", [(1.0, 0.4, 256, None),
                                             (2.2, 0.7, 64, (0.3, 1, 0.2)),
                                             (0.9, 0.2, 33, (1, 0, 0))])
def test_cap_every_entry_closed_form(colat, rho, n, rot):
    """On a small circle of geodesic radius rho, (x' - x).n'/|x - x'|^2 equals
    -cos(rho)/(2 sin(rho)) for every pair (Appendix A, eq. kern1), so every
    entry of (I+K) - I, diagonal included, is -cos(rho)/N.  Pins the kernel
    scale 2h/(2 pi), the correction-term sign, the diagonal limit and the
    orientation sign."""
    isl = synth.cap_island(colat, rho, n)
    if rot is not None:
        isl = isl.rotated(_rot(rot, 0.7))
    cv = Curves(isl)
    K = _full_k(cv)
    assert np.abs(K + np.cos(rho) / n).max() < 1e-13


def test_cap_printed_sign_would_fail():
    """The paper's printed '-' sign of the correction term gives a different
    operator: check that the closed form distinguishes the two readings."""
    isl = synth.cap_island(1.0, 0.4, 128)
    cv = Curves(isl)
    K = _full_k(cv)
    corr = np.imag(np.conj(cv.xi) * cv.dxi / (1 + np.abs(cv.xi) ** 2))
    K_minus = K - 2 * (corr * cv.s * cv.h / np.pi)[None, :]
    assert np.abs(K_minus + np.cos(0.4) / 128).max() > 1e-3


# --- T1b: planar kernel equals the sphere form of Appendix A -----------------
def test_planar_kernel_equals_sphere_form(stars6):
    """The stereographic kernel (projection derivatives, correction term,
    orientation signs) must reproduce the double-layer kernel computed from
    3D geometry alone (Appendix A, eq. kern1) entry by entry."""
    cv = Curves(stars6)
    K = _full_k(cv)
    Ks = nystrom.sphere_kernel_block(cv, np.arange(cv.n))
    assert np.abs(K - Ks).max() < 1e-12 * max(1.0, np.abs(K).max())


# --- T2: one cap, discrete solution in closed form --------------------------
def test_cap_solution_closed_form():
    """With (I+K) = I - (cos rho/N) 1 1^T the discrete system gives
    A_0 = 0 and sigma = 2 g + 2 cos(rho) mean(g) / (1 - cos(rho))."""
    rho = 0.4
    isl = synth.config_islands("cap256")
    cv = Curves(isl)
    g = synth.exact_harmonic(cv.x, isl.center, [1.0])
    sig, A = nystrom.solve_dense(cv, g)
    expect = 2 * g + 2 * np.cos(rho) * g.mean() / (1 - np.cos(rho))
    assert abs(A[0]) < 1e-13
    assert np.abs(sig - expect).max() < 1e-12 * np.abs(expect).max()


# --- T3: null-space identity (Section 4.1) ----------------------------------
def test_null_space_identity(stars6):
    """(I+K) zeta_k = (Area_k / 2 pi) 1 on every node of every curve, where
    zeta_k is 1 on curve k and Area_k is island k's spherical area; this is
    the D_k identity of Section 4.1 (with the area element 4/(1+|xi|^2)^2)."""
    isl = stars6.with_nodes(384)
    cv = Curves(isl)
    for k in range(isl.m):
        zeta = (cv.island == k).astype(float)
        y = nystrom.apply_iplusk(cv, zeta)
        expect = island_area(isl, k) / (2 * np.pi)
        assert np.abs(y - expect).max() < 1e-12, k


# --- T4: pure log-source data is reproduced exactly --------------------------
def test_log_source_data_exact(stars6):
    """g = sum_m a_m G(x, c_m) with sum(a) = 0 is harmonic in the domain and
    the discrete system is solved exactly by sigma = 0, A = a."""
    cv = Curves(stars6)
    a = synth.random_vector(5, stars6.m)
    a -= a.mean()
    g = nystrom.greens(cv.x, cv.center) @ a
    sig, A = nystrom.solve_dense(cv, g)
    assert np.abs(sig).max() < 1e-11
    assert np.abs(A - a).max() < 1e-12


# --- T5: constant data ------------------------------------------------------
def test_constant_data(stars6):
    """g = 1: u = 1, represented by A = 0 and sigma = (4 pi / Area_0) zeta_0
    (only island 0 carries no constraint)."""
    isl = stars6.with_nodes(192)
    cv = Curves(isl)
    sig, A = nystrom.solve_dense(cv, np.ones(cv.n))
    expect = (cv.island == 0) * 4 * np.pi / island_area(isl, 0)
    assert np.abs(A).max() < 1e-10
    assert np.abs(sig - expect).max() < 1e-9 * np.abs(expect).max()


# --- T6 / T9: harmonic data, exact solution, spectral convergence ------------
def test_harmonic_data_and_spectral_convergence(stars6):
    """u = Re sum_k c_k/(xi - xi_k) (Section 6, eq. exact_bcs) is the exact
    solution; the error at far targets must drop super-algebraically with
    the node count (Section 5) down to near machine precision."""
    coeffs = synth.random_data_coeffs(3, stars6)
    tg = synth.sphere_targets(9, 60, stars6)
    exact = synth.exact_harmonic(tg, stars6.center, coeffs)
    errs = []
    for n in (24, 48, 96, 192):
        isl = stars6.with_nodes(n)
        cv = Curves(isl)
        g = synth.exact_harmonic(cv.x, isl.center, coeffs)
        sig, A = nystrom.solve_dense(cv, g)
        u = evaluate.evaluate(cv, sig, A, tg)
        errs.append(np.abs(u - exact).max() / np.abs(exact).max())
    assert errs[-1] < 1e-11
    assert errs[0] > 10 * errs[1] > 0
    assert errs[1] > 100 * errs[2] or errs[2] < 1e-11


def test_eval_on_curve_limit_matches_jump(stars6):
    """Evaluating the representation at the north pole (xi = infinity) keeps
    only the correction and log terms; at a point approaching the pole the
    full formula converges to that value."""
    isl = stars6.with_nodes(64)
    cv = Curves(isl)
    sig = synth.random_vector(1, cv.n)
    A = synth.random_vector(2, cv.m)
    pole = np.array([[0.0, 0.0, 1.0]])
    eps = 1e-7
    near = np.array([[np.sin(eps), 0.0, np.cos(eps)]])
    up = evaluate.evaluate(cv, sig, A, pole)
    un = evaluate.evaluate(cv, sig, A, near)
    assert abs(up[0] - un[0]) < 1e-5


# --- T10: preconditioned GMRES ----------------------------------------------
def test_gmres_matches_lu_and_preconditioning_helps(stars6):
    """GMRES on eq. matrix_eqns_c reaches the LU solution; its iteration count
    stays about constant under node refinement (bounded conditioning,
    Section 6 Example 1) and is far below the unpreconditioned count."""
    coeffs = synth.paper_data_coeffs(stars6.m)
    its = []
    for n in (64, 128):
        isl = stars6.with_nodes(n)
        cv = Curves(isl)
        g = synth.exact_harmonic(cv.x, isl.center, coeffs)
        s_lu, a_lu = nystrom.solve_dense(cv, g)
        s_it, a_it, it, _ = gmres.solve_preconditioned(cv, g, tol=1e-13)
        its.append(it)
        assert np.abs(s_it - s_lu).max() < 1e-9 * np.abs(s_lu).max()
        assert np.abs(a_it - a_lu).max() < 1e-9 * max(1, np.abs(a_lu).max())
    assert abs(its[1] - its[0]) <= 3
    cv = Curves(stars6.with_nodes(64))
    g = synth.exact_harmonic(cv.x, stars6.center, coeffs)
    _, _, it_np, _ = gmres.solve_preconditioned(cv, g, tol=1e-13,
                                                precondition=False,
                                                max_iter=400)
    assert it_np > its[0] + 5


def test_preconditioned_condition_bounded(stars6):
    """cond(P^-1 A) stays bounded under refinement while cond(A) grows
    (Section 6, Table 1 pattern)."""
    conds_p, conds = [], []
    for n in (32, 64, 128):
        cv = Curves(stars6.with_nodes(n))
        A = nystrom.system_matrix(cv)
        P = A.copy()
        P[:cv.n, :cv.n] = np.eye(cv.n)
        conds.append(np.linalg.cond(A))
        conds_p.append(np.linalg.cond(np.linalg.solve(P, A)))
    assert max(conds_p) / min(conds_p) < 1.2
    assert conds[2] > 1.5 * conds[0]


# --- T12: rotation invariance -----------------------------------------------
def test_rotation_invariance(stars6):
    """Rotating every island on the sphere changes all planar images but not
    the operator: the kernel depends on chordal geometry only."""
    cv = Curves(stars6)
    R = _rot((0.2, -0.5, 0.4), 0.35)
    rot = stars6.rotated(R)
    assert np.all(np.arccos(rot.center[:, 2]) > rot.max_radius() + 0.05)
    cv2 = Curves(rot)
    K1, K2 = _full_k(cv), _full_k(cv2)
    assert np.abs(K1 - K2).max() < 1e-12
    E1, E2 = nystrom.log_source_block(cv), nystrom.log_source_block(cv2)
    assert np.abs(E1 - E2).max() < 1e-12


# --- orientation rule ------------------------------------------------------
def test_orientation_reversal_leaves_operator(stars6):
    """Traversing a curve backwards negates xi' and flips s_k; the product
    s_k xi' and hence every operator entry must be unchanged."""
    cv = Curves(stars6)
    K = _full_k(cv)
    k = 2
    idx = np.where(cv.island == k)[0]
    rev = idx[::-1]
    cv.xi[idx] = cv.xi[rev].copy()
    cv.dxi[idx] = -cv.dxi[rev].copy()
    cv.ddxi[idx] = cv.ddxi[rev].copy()
    cv.x[idx] = cv.x[rev].copy()
    s = orientation_sign(cv.xi[idx], cv.dxi[idx])
    assert s == -cv.sign_per_island[k]
    cv.s[idx] = s
    K2 = _full_k(cv)
    perm = np.arange(cv.n)
    perm[idx] = rev
    assert np.abs(K2 - K[np.ix_(perm, perm)]).max() < 1e-13


def test_island_area_cap():
    """Area of a cap of radius rho is 2 pi (1 - cos rho)."""
    isl = synth.cap_island(1.0, 0.4, 64)
    assert abs(island_area(isl, 0) - 2 * np.pi * (1 - np.cos(0.4))) < 1e-14


def test_greens_planar_form():
    """G in chordal form equals the planar expression of eq. fundC."""
    rng = np.random.default_rng(0)
    x = rng.standard_normal((20, 3))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    y = rng.standard_normal((7, 3))
    y /= np.linalg.norm(y, axis=1, keepdims=True)
    xi = (x[:, 0] + 1j * x[:, 1]) / (1 - x[:, 2])
    eta = (y[:, 0] + 1j * y[:, 1]) / (1 - y[:, 2])
    d = xi[:, None] - eta[None, :]
    planar = -np.log(2 * np.abs(d) ** 2 / ((1 + np.abs(xi[:, None]) ** 2) *
                                           (1 + np.abs(eta[None, :]) ** 2))
                     ) / (4 * np.pi)
    assert np.abs(planar - nystrom.greens(x, y)).max() < 1e-13
