"""GPU parity of the full batch workload the benchmark times: 64 geometries
of 10-400 star islands (128-512 nodes per curve, 4k-100k nodes each, 2.88M
nodes in all) with 16 right-hand sides each, in one handle.

* (I + K) X for all 1024 systems, checked on 32 sampled rows of every
  geometry against the oracle's direct sum (FP64 <= 1e-10, mixed <= 1e-6);
* all 1024 systems solved together (mixed precision, tol 1e-12) from
  exactly harmonic data Re sum_k c_k / (xi - xi_k) over four random islands
  of the geometry: every system's residual; sigma and u against the
  oracle's LU solution for three systems of each of the four smallest
  geometries (<= 1e-9, <= 1e-10); u against the exact solution for
  systems of four large geometries (to the Nystrom error of 128-node
  curves)."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import nystrom, evaluate
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
    sizes = [gm.n_total for gm in geoms]
    # the four smallest geometries (5k-8k nodes): sigma and u against the
    # oracle's LU solution of the same Nystrom system
    for q in [int(v) for v in np.argsort(sizes)[:4]]:
        gm = geoms[q]
        cv = Curves(gm)
        Mx = nystrom.system_matrix(cv)
        lu = sla.lu_factor(Mx, check_finite=False)
        tg = synth.sphere_targets(9500 + q, 300, gm)
        for r in (0, 5, 15):
            rhs = np.concatenate([2.0 * G[r, no[q]:no[q + 1]], np.zeros(cv.m)])
            x = sla.lu_solve(lu, rhs, check_finite=False)
            assert _rel(sig[r, no[q]:no[q + 1]], x[:cv.n]) < 1e-9, (q, r)
            u = _eval(torch, sol, sig[r], A[r], tg, q)
            ref = evaluate.evaluate(cv, x[:cv.n], x[cv.n:], tg)
            assert _rel(u, ref) < 1e-10, (q, r)
    # large geometries: u against the exact solution, to the Nystrom error
    # of curves with 128 nodes (the oracle's own LU solution of geometry 40
    # is 6.5e-9 from the exact u for right-hand side 15)
    for q in (0, 21, 40, 63):
        gm = geoms[q]
        tg = synth.sphere_targets(9500 + q, 300, gm)
        for r in (0, 5, 15):
            k, c = picks[q, r]
            exact = synth.exact_harmonic(tg, gm.center[k], c)
            u = _eval(torch, sol, sig[r], A[r], tg, q)
            assert _rel(u, exact) < 2e-8, (q, r)


def _eval(torch, sol, sig, A, tg, q):
    """u of one column at targets of geometry q (lbs_eval_batch with no
    targets for the other geometries)."""
    toff = [0] * (q + 1) + [len(tg)] * (sol.n_geoms - q)
    return sol.eval(_t(torch, sig), _t(torch, A), _t(torch, tg),
                    target_offsets=toff).cpu().numpy()
