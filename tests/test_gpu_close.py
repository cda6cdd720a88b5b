"""GPU parity of close evaluation (lbs_eval with close_eval = 1) against the
oracle's compensated rule (oracle/close.py) and against the exact harmonic
solution, at targets 1e-1 .. 1e-6 island radii outside the curves, mixed
with far targets and the north pole; FMM and direct far field, two columns,
a batch handle; the trapezoidal rule with close_eval = 0; and the adjoint
entry points' refusal of close targets."""
import numpy as np
import pytest

import synth
from oracle import nystrom, evaluate
from oracle.close import evaluate_close
from oracle.geometry import Curves

pytestmark = pytest.mark.gpu

DISTS = [1e-1, 1e-2, 1e-3, 1e-4, 1e-6]


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
def case():
    # 320 nodes per curve resolve the densities to ~1e-13
    isl = synth.star_islands(12, 5, (0.1, 0.25), nodes=320)
    cv = Curves(isl)
    coeffs = synth.random_data_coeffs(13, isl)
    g = synth.exact_harmonic(cv.x, isl.center, coeffs)
    s, a = nystrom.solve_dense(cv, g)
    near, _ = synth.near_curve_targets(isl, 14, DISTS)
    far = synth.sphere_targets(15, 50, isl)
    tg = np.concatenate([near, far, [[0.0, 0.0, 1.0]]])
    return isl, cv, coeffs, g, s, a, tg


@pytest.mark.parametrize("mode", ["fmm", "direct"])
def test_close_eval_matches_oracle(env, case, mode):
    torch, lbs = env
    isl, cv, coeffs, g, s, a, tg = case
    sol = lbs.Solver(isl, leaf_max=24, matvec=mode)
    S = np.stack([s, -0.5 * s + 1.0])
    AA = np.stack([a, 2.0 * a])
    u = sol.eval(_t(torch, S), _t(torch, AA), _t(torch, tg)).cpu().numpy()
    for r in range(2):
        ref = evaluate_close(cv, S[r], AA[r], tg)
        assert _rel(u[r], ref) < 1e-10, r
    # the exact solution vanishes at the pole (xi = infinity)
    exact = synth.exact_harmonic(tg[:-1], isl.center, coeffs)
    assert _rel(u[0][:-1], exact) < 1e-10 and abs(u[0][-1]) < 1e-10
    sol.close()


def test_close_eval_after_gpu_solve(env, case):
    """The whole path: GPU solve (mixed precision, tol 1e-12), then close
    evaluation at the near targets, against the exact solution."""
    torch, lbs = env
    isl, cv, coeffs, g, s, a, tg = case
    sol = lbs.Solver(isl, leaf_max=24)
    sig, A, info = sol.solve(_t(torch, g), tol=1e-12, precision="mixed")
    u = sol.eval(sig, A, _t(torch, tg)).cpu().numpy()
    exact = synth.exact_harmonic(tg[:-1], isl.center, coeffs)
    assert _rel(u[:-1], exact) < 1e-10 and abs(u[-1]) < 1e-10
    sol.close()


def test_trapezoidal_rule_when_off(env, case):
    torch, lbs = env
    isl, cv, coeffs, g, s, a, tg = case
    sol = lbs.Solver(isl, leaf_max=24, close_eval=0)
    u = sol.eval(_t(torch, s), _t(torch, a), _t(torch, tg)).cpu().numpy()
    assert _rel(u, evaluate.evaluate(cv, s, a, tg)) < 1e-10
    # the adjoint covers the trapezoidal rule: accepted here
    sol.eval_T(_t(torch, np.ones(len(tg))), _t(torch, tg))
    sol.close()


def test_adjoint_refuses_close_targets(env, case):
    torch, lbs = env
    isl, cv, coeffs, g, s, a, tg = case
    sol = lbs.Solver(isl, leaf_max=24)
    with pytest.raises(lbs.LBSError) as e:
        sol.eval_T(_t(torch, np.ones(len(tg))), _t(torch, tg))
    assert e.value.status == "LBS_ERR_UNSUPPORTED"
    sol.close()


def test_close_eval_batch(env, case):
    torch, lbs = env
    isl, cv, coeffs, g, s, a, tg = case
    other = synth.star_islands(16, 3, (0.15, 0.3), nodes=256)
    cvo = Curves(other)
    so = synth.random_vector(17, cvo.n)
    ao = synth.random_vector(18, cvo.m)
    tgo, _ = synth.near_curve_targets(other, 19, DISTS[:3])
    sol = lbs.Solver([isl, other], leaf_max=24)
    toff = [0, len(tg), len(tg) + len(tgo)]
    u = sol.eval(_t(torch, np.concatenate([s, so])),
                 _t(torch, np.concatenate([a, ao])),
                 _t(torch, np.concatenate([tg, tgo])),
                 target_offsets=toff).cpu().numpy()
    assert _rel(u[:len(tg)], evaluate_close(cv, s, a, tg)) < 1e-10
    assert _rel(u[len(tg):], evaluate_close(cvo, so, ao, tgo)) < 1e-10
    sol.close()
