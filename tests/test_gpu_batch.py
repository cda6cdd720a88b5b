"""GPU parity of batch handles (many geometries, many right-hand sides in
one handle) against the CPU oracle, geometry by geometry."""
import numpy as np
import pytest

import synth
from oracle import nystrom, evaluate
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


def _geoms():
    return [synth.star_islands(61, 5, (0.08, 0.2), nodes=64),
            synth.star_islands(62, 2, (0.1, 0.3), nodes=[96, 48]),
            synth.star_islands(63, 9, (0.05, 0.12), nodes=80)]


@pytest.fixture(scope="module")
def batch(env):
    torch, lbs = env
    geoms = _geoms()
    sol = lbs.Solver(geoms, leaf_max=12)
    cvs = [Curves(g) for g in geoms]
    return geoms, sol, cvs


def test_batch_layout(batch):
    geoms, sol, cvs = batch
    assert sol.n_geoms == 3
    assert sol.node_offsets[-1] == sum(cv.n for cv in cvs) == sol.n_nodes
    assert sol.island_offsets[-1] == sum(g.m for g in geoms)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_batch_matvec(env, batch, prec, tol):
    torch, lbs = env
    geoms, sol, cvs = batch
    no = sol.node_offsets
    X = np.stack([synth.random_vector(s, sol.n_nodes) for s in (1, 2)])
    Y = sol.matvec(_t(torch, X), "iplusk", prec).cpu().numpy()
    for q, cv in enumerate(cvs):
        for r in range(2):
            ref = nystrom.apply_iplusk(cv, X[r, no[q]:no[q + 1]])
            assert _rel(Y[r, no[q]:no[q + 1]], ref) < tol, (q, r)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_solve_matches_lu(env, batch, prec):
    torch, lbs = env
    geoms, sol, cvs = batch
    no, io = sol.node_offsets, sol.island_offsets
    xyz = sol.nodes().cpu().numpy()
    G = np.zeros((3, sol.n_nodes))
    coeffs = []
    for q, g in enumerate(geoms):
        for r in range(3):
            c = synth.random_data_coeffs(100 * q + r, g)
            coeffs.append(c)
            G[r, no[q]:no[q + 1]] = synth.exact_harmonic(
                xyz[no[q]:no[q + 1]], g.center, c)
    sig, A, info = sol.solve(_t(torch, G), tol=1e-12, precision=prec)
    assert info["rel_resid"] < 1e-11
    sig, A = sig.cpu().numpy(), A.cpu().numpy()
    for q, cv in enumerate(cvs):
        for r in range(3):
            s_ref, a_ref = nystrom.solve_dense(cv, G[r, no[q]:no[q + 1]])
            assert _rel(sig[r, no[q]:no[q + 1]], s_ref) < 1e-9, (q, r)
            assert np.abs(A[r, io[q]:io[q + 1]] - a_ref).max() < 1e-9 * max(
                1, np.abs(a_ref).max())


def test_batch_matches_single_handles(env, batch):
    torch, lbs = env
    geoms, sol, cvs = batch
    no = sol.node_offsets
    x = synth.random_vector(9, sol.n_nodes)
    yb = sol.matvec(_t(torch, x), "iplusk", "fp64").cpu().numpy()
    for q, g in enumerate(geoms):
        single = lbs.Solver(g, leaf_max=12)
        ys = single.matvec(_t(torch, x[no[q]:no[q + 1]]), "iplusk",
                           "fp64").cpu().numpy()
        assert np.abs(ys - yb[no[q]:no[q + 1]]).max() < 1e-13 * np.abs(ys).max()


def test_batch_eval(env, batch):
    torch, lbs = env
    geoms, sol, cvs = batch
    no, io = sol.node_offsets, sol.island_offsets
    sig = synth.random_vector(3, sol.n_nodes)
    A = synth.random_vector(4, sol.n_islands)
    tgs = [synth.sphere_targets(10 + q, 40 + 7 * q, g)
           for q, g in enumerate(geoms)]
    toff = np.concatenate([[0], np.cumsum([len(t) for t in tgs])])
    u = sol.eval(_t(torch, sig), _t(torch, A), _t(torch, np.concatenate(tgs)),
                 target_offsets=toff).cpu().numpy()
    for q, cv in enumerate(cvs):
        ref = evaluate.evaluate(cv, sig[no[q]:no[q + 1]], A[io[q]:io[q + 1]],
                                tgs[q])
        assert _rel(u[toff[q]:toff[q + 1]], ref) < 1e-10, q
