"""GPU parity of the point-vortex decomposition (Section 6, Example 2):
lbs_vortex_data -> lbs_solve -> lbs_eval -> lbs_vortex_field against the
closed form for one cap and one vortex, and against the oracle (dense LU)
for star islands with 72 vortices of strengths in (-2 pi, 2 pi) and zero
coastline data, where psi must also vanish at the coastline (close
evaluation at targets 1e-9 island radii off the curves)."""
import numpy as np
import pytest

import synth
from oracle import vortex
from oracle.close import evaluate_close
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


def _psi(torch, sol, g, xyz_v, gam, tg, prec):
    gs = sol.vortex_data(_t(torch, g), _t(torch, xyz_v), _t(torch, gam))
    sig, A, info = sol.solve(gs, tol=1e-12, precision=prec)
    assert info["status"] == "LBS_OK"
    u = sol.eval(sig, A, _t(torch, tg))
    sol.vortex_field(u, _t(torch, xyz_v), _t(torch, gam), _t(torch, tg))
    return sig.cpu().numpy(), A.cpu().numpy(), u.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_cap_one_vortex_closed_form(env, prec):
    torch, lbs = env
    from test_oracle_vortex import closed_form
    isl = synth.cap_island(1.0, 0.4, 256)
    v = np.array([[np.sin(1.8) * np.cos(0.7), np.sin(1.8) * np.sin(0.7),
                   np.cos(1.8)]])
    tg = synth.sphere_targets(7, 80, isl)
    tg = tg[np.linalg.norm(tg - v[0], axis=1) > 0.05]
    sol = lbs.Solver(isl, leaf_max=32)
    _, _, u = _psi(torch, sol, np.zeros(sol.n_nodes), v, [1.7], tg, prec)
    exact = closed_form(tg, 1.0, 0.4, v[0], 1.7)
    assert _rel(u, exact) < 1e-10
    sol.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_stars_72_vortices(env, prec):
    torch, lbs = env
    isl = synth.star_islands(51, 5, (0.15, 0.3), k_range=(2, 4), nodes=384)
    cv = Curves(isl)
    xyz_v, gam = synth.point_vortices(52, 72, isl)
    gam2 = np.stack([gam, -0.5 * gam])
    sol = lbs.Solver(isl, leaf_max=32)
    tg = synth.sphere_targets(53, 200, isl)
    near, _ = synth.near_curve_targets(isl, 54, [1e-9])
    pts = np.concatenate([tg, near])
    G0 = np.zeros((2, cv.n))
    sig, A, u = _psi(torch, sol, G0, xyz_v, gam2, pts, prec)
    for r in range(2):
        s_ref, a_ref = vortex.solve(cv, G0[r], xyz_v, gam2[r])
        assert _rel(sig[r], s_ref) < 1e-9, r
        # close evaluation (the library's default) at the near targets
        ref = (evaluate_close(cv, s_ref, a_ref, pts)
               + vortex.vortex_field(pts, xyz_v, gam2[r]))
        assert _rel(u[r], ref) < 1e-10, r
    # zero data: psi vanishes at the coastline
    assert np.abs(u[0, len(tg):]).max() < 1e-8 * np.abs(u[0]).max()
    sol.close()
