"""GPU parity on a geometry whose quadtree has 21-23 levels: islands from
near the north pole to within 1e-3 rad of the south pole, shrinking from
0.25 to 2e-5 rad, so that stereographic projection spreads their images
over seven orders of magnitude (the distortion of Section 6, Example 3,
where the paper's trees reach 16-22 levels).  Every row of (I + K) sigma
against the oracle's direct sum (FP64 <= 1e-10, FP32 far field <= 1e-6),
and the solve against the oracle's LU."""
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


@pytest.mark.parametrize("leaf_max", [16, 48])
def test_deep_tree_rows(env, leaf_max):
    torch, lbs = env
    isl = synth.deep_tree_islands(256)
    cv = Curves(isl)
    sol = lbs.Solver(isl, leaf_max=leaf_max)
    st = sol.tree_info()
    assert st["levels"] >= 20, st
    X = np.stack([synth.random_vector(s, cv.n) for s in (81, 82)])
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-6)):
        Y = sol.matvec(_t(torch, X), "iplusk", prec).cpu().numpy()
        for r in range(2):
            assert _rel(Y[r], nystrom.apply_iplusk(cv, X[r])) < tol, (prec, r)
    sol.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_deep_tree_solve(env, prec):
    torch, lbs = env
    isl = synth.deep_tree_islands(256)
    cv = Curves(isl)
    g = synth.exact_harmonic(cv.x, isl.center,
                             synth.random_data_coeffs(83, isl))
    s_ref, a_ref = nystrom.solve_dense(cv, g)
    sol = lbs.Solver(isl, leaf_max=16)
    sig, A, info = sol.solve(_t(torch, g), tol=1e-12, precision=prec)
    assert info["status"] == "LBS_OK" and info["true_rel_resid"] < 1e-10
    assert _rel(sig.cpu().numpy(), s_ref) < 1e-9
    assert np.abs(A.cpu().numpy() - a_ref).max() < 1e-9 * max(
        1, np.abs(a_ref).max())
    sol.close()
