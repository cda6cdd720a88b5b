"""GPU parity of the full batch workload the benchmark times: 64 geometries
of 10-400 star islands (128-512 nodes per curve, 4k-100k nodes each, 2.88M
nodes in all) with 16 right-hand sides each, in one handle.

* (I + K) X for all 1024 systems, checked on 32 sampled rows of every
  geometry against the oracle's direct sum (FP64 <= 1e-10, mixed <= 1e-6);
* all 1024 systems solved together (mixed precision, tol 1e-12) from
  exactly harmonic data Re sum_k c_k / (xi - xi_k) over four random islands
  of the geometry; u at sphere targets against the exact solution for
  systems of six geometries (<= 1e-10) and every system's residual."""
import numpy as np
import pytest

import synth
from oracle import nystrom
from oracle.geometry import Curves

pytestmark = pytest.mark.gpu

N_RHS = 16


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


@pytest.fixture(scope="module")
def batch(env):
    torch, lbs = env
    geoms = synth.batch_geometries(64)
    sol = lbs.Solver(geoms)
    yield geoms, sol
    sol.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_full_batch_rows(env, batch, prec, tol):
    torch, lbs = env
    geoms, sol = batch
    no = sol.node_offsets
    assert sol.n_geoms == 64 and sol.n_nodes > 2_000_000
    X = np.random.default_rng(91).standard_normal((N_RHS, sol.n_nodes))
    Y = sol.matvec(_t(torch, X), "iplusk", prec).cpu().numpy()
    rng = np.random.default_rng(92)
    for q, gm in enumerate(geoms):
        cv = Curves(gm)
        rows = np.sort(rng.choice(cv.n, 32, replace=False))
        Xq = X[:, no[q]:no[q + 1]]
        ref = nystrom.kernel_block(cv, rows) @ Xq.T + Xq[:, rows].T
        got = Y[:, no[q]:no[q + 1]][:, rows].T
        assert _rel(got, ref) < tol, q


def test_full_batch_solve(env, batch):
    torch, lbs = env
    geoms, sol = batch
    no, io = sol.node_offsets, sol.island_offsets
    xyz = sol.nodes().cpu().numpy()
    rng = np.random.default_rng(93)
    G = np.empty((N_RHS, sol.n_nodes))
    picks = {}
    for q, gm in enumerate(geoms):
        cf = synth.random_data_coeffs(9400 + q, gm)
        for r in range(N_RHS):
            k = rng.choice(gm.m, 4, replace=False)
            picks[q, r] = (k, cf[k])
            G[r, no[q]:no[q + 1]] = synth.exact_harmonic(
                xyz[no[q]:no[q + 1]], gm.center[k], cf[k])
    sig, A, info = sol.solve(_t(torch, G), tol=1e-12, precision="mixed")
    assert info["status"] == "LBS_OK"
    assert info["rel_resid"] < 1e-11 and info["true_rel_resid"] < 1e-10
    sig, A = sig.cpu().numpy(), A.cpu().numpy()
    for q in (0, 7, 21, 40, 55, 63):
        gm = geoms[q]
        tg = synth.sphere_targets(9500 + q, 300, gm)
        for r in (0, 5, 15):
            k, c = picks[q, r]
            exact = synth.exact_harmonic(tg, gm.center[k], c)
            # batch handle: evaluate geometry q's system r through
            # lbs_eval_batch with targets only for geometry q
            toff = [0] * (q + 1) + [len(tg)] * (sol.n_geoms - q)
            u = sol.eval(_t(torch, sig[r]), _t(torch, A[r]), _t(torch, tg),
                         target_offsets=toff).cpu().numpy()
            assert _rel(u, exact) < 1e-10, (q, r)
