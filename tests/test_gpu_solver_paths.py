"""GPU parity of the solver's less travelled paths against the CPU oracle:
GMRES restarts (short restart lengths, so that every solve runs several
cycles; FP64 and mixed, with and without captured graphs, one handle and a
batch handle whose systems converge in different cycles), GMRES on the
unpreconditioned system of eq. matrix_eqns, the transposed operator
(I + K)^T, and the true residual the solve reports."""
import numpy as np
import pytest

import synth
from oracle import nystrom
from oracle.geometry import Curves

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(b).max()


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1306_0612_amd import lbs
    lbs.load()
    return torch, lbs


def _t(torch, a):
    return torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda")


def _np(x):
    return x.detach().cpu().numpy()


@pytest.fixture(scope="module")
def single():
    isl = synth.star_islands(71, 10, (0.06, 0.16), nodes=96)
    cv = Curves(isl)
    rhs = []
    for r in range(3):
        g = synth.exact_harmonic(cv.x, isl.center,
                                 synth.random_data_coeffs(700 + r, isl))
        rhs.append((g, nystrom.solve_dense(cv, g)))
    return isl, cv, rhs


@pytest.mark.parametrize("restart", [5, 8])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("graphs", [1, 0])
def test_restarted_gmres_matches_lu(env, single, restart, prec, graphs):
    torch, lbs = env
    isl, cv, rhs = single
    sol = lbs.Solver(isl, leaf_max=16, restart=restart, graphs=graphs,
                     max_iter=2000)
    G = np.stack([g for g, _ in rhs])
    sig, A, info = sol.solve(_t(torch, G), tol=1e-12, precision=prec)
    assert info["status"] == "LBS_OK"
    # every solve needs more than one cycle of `restart` iterations
    assert info["iters"] > 2 * restart
    assert info["rel_resid"] < 1e-11 and info["true_rel_resid"] < 1e-10
    sig, A = _np(sig), _np(A)
    for r, (_, (s_ref, a_ref)) in enumerate(rhs):
        assert _rel(sig[r], s_ref) < 1e-9, r
        assert np.abs(A[r] - a_ref).max() < 1e-9 * max(1, np.abs(a_ref).max())
    sol.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_restarted_gmres_batch(env, prec):
    """A batch handle whose systems need different numbers of restart
    cycles (different geometries and data), each against its own LU."""
    torch, lbs = env
    geoms = [synth.star_islands(72, 4, (0.1, 0.25), nodes=64),
             synth.star_islands(73, 12, (0.04, 0.12), nodes=[64, 96, 128] * 4),
             synth.star_islands(74, 7, (0.08, 0.2), nodes=80)]
    sol = lbs.Solver(geoms, leaf_max=12, restart=6, max_iter=2000)
    no, io = sol.node_offsets, sol.island_offsets
    xyz = _np(sol.nodes())
    G = np.zeros((2, sol.n_nodes))
    for q, g in enumerate(geoms):
        for r in range(2):
            G[r, no[q]:no[q + 1]] = synth.exact_harmonic(
                xyz[no[q]:no[q + 1]], g.center,
                synth.random_data_coeffs(750 + 10 * q + r, g))
    sig, A, info = sol.solve(_t(torch, G), tol=1e-12, precision=prec)
    assert info["status"] == "LBS_OK" and info["iters"] > 12
    sig, A = _np(sig), _np(A)
    for q, g in enumerate(geoms):
        cv = Curves(g)
        for r in range(2):
            s_ref, a_ref = nystrom.solve_dense(cv, G[r, no[q]:no[q + 1]])
            assert _rel(sig[r, no[q]:no[q + 1]], s_ref) < 1e-9, (q, r)
            assert np.abs(A[r, io[q]:io[q + 1]] - a_ref).max() < 1e-9 * max(
                1, np.abs(a_ref).max())
    sol.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_unpreconditioned_solve_matches_lu(env, single, prec):
    """GMRES on A itself (eq. matrix_eqns) reaches the same solution as LU
    and needs more iterations than on the preconditioned system
    (Section 6, Example 1)."""
    torch, lbs = env
    isl, cv, rhs = single
    g, (s_ref, a_ref) = rhs[0]
    its = {}
    for pre in (1, 0):
        sol = lbs.Solver(isl, leaf_max=16, precond=pre, max_iter=3000)
        sig, A, info = sol.solve(_t(torch, g), tol=1e-12, precision=prec)
        assert info["status"] == "LBS_OK", info
        assert info["true_rel_resid"] < 1e-10
        if not pre:
            assert info["rel_resid"] == info["true_rel_resid"]
        assert _rel(_np(sig), s_ref) < 1e-9
        assert np.abs(_np(A) - a_ref).max() < 1e-9 * max(
            1, np.abs(a_ref).max())
        its[pre] = info["iters"]
        sol.close()
    assert its[0] > its[1]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_transposed_operator(env, prec, tol):
    """lbs_matvec(LBS_OP_IPLUSK_T) against the transpose of the oracle's
    dense Nystrom matrix, one handle (two columns) and a batch handle."""
    torch, lbs = env
    isl = synth.star_islands(75, 6, (0.08, 0.2), nodes=[80, 64, 96, 72, 64, 88])
    cv = Curves(isl)
    K = nystrom.kernel_block(cv, np.arange(cv.n))
    X = np.stack([synth.random_vector(s, cv.n) for s in (5, 6)])
    sol = lbs.Solver(isl, leaf_max=10)
    Y = _np(sol.matvec(_t(torch, X), "iplusk_t", prec))
    for r in range(2):
        assert _rel(Y[r], K.T @ X[r] + X[r]) < tol, r
    sol.close()
    geoms = [isl, synth.star_islands(76, 3, (0.1, 0.3), nodes=64)]
    sol = lbs.Solver(geoms, leaf_max=10)
    no = sol.node_offsets
    x = synth.random_vector(7, sol.n_nodes)
    y = _np(sol.matvec(_t(torch, x), "iplusk_t", prec))
    for q, gm in enumerate(geoms):
        cq = Curves(gm)
        Kq = nystrom.kernel_block(cq, np.arange(cq.n))
        xq = x[no[q]:no[q + 1]]
        assert _rel(y[no[q]:no[q + 1]], Kq.T @ xq + xq) < tol, q
    sol.close()
