"""GPU parity at the benchmark's full sizes (20,480, 256,000 and 1,024,000
nodes; default options, the launch configuration bench.py times) on
outputs the oracle computes row by row, and on properties that hold at any
size:

* sampled rows of (I + K) sigma (all rows at 20,480 nodes), FP64 FMM
  <= 1e-10, mixed <= 1e-6;
* sampled rows of the full system [(I + K) sigma + E A; F sigma + D A];
* the solved u at sphere targets against the exact harmonic solution the
  data was drawn from (the Nystrom error of these smooth curves is far
  below the solver tolerance), solve tolerance 1e-12, bound 1e-10.
"""
import numpy as np
import pytest

import synth
from oracle import nystrom
from oracle.geometry import Curves

pytestmark = pytest.mark.gpu

CONFIGS = [("stars40x512", None), ("stars1000x256", 300),
           ("stars2000x512", 120)]


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


@pytest.fixture(scope="module", params=CONFIGS, ids=[c[0] for c in CONFIGS])
def case(env, request):
    torch, lbs = env
    name, nrows = request.param
    isl = synth.config_islands(name)
    sol = lbs.Solver(isl)
    cv = Curves(isl)
    rng = np.random.default_rng(7)
    rows = (np.arange(cv.n) if nrows is None
            else np.sort(rng.choice(cv.n, nrows, replace=False)))
    yield isl, cv, sol, rows
    sol.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_iplusk_rows(env, case, prec, tol):
    torch, lbs = env
    isl, cv, sol, rows = case
    x = synth.random_vector(8, cv.n)
    y = sol.matvec(_t(torch, x), "iplusk", prec).cpu().numpy()
    ref = nystrom.apply_iplusk(cv, x, rows)
    assert _rel(y[rows], ref) < tol


def test_system_rows(env, case):
    torch, lbs = env
    isl, cv, sol, rows = case
    xs = synth.random_vector(9, cv.n)
    xa = synth.random_vector(10, cv.m)
    y = sol.matvec(_t(torch, np.concatenate([xs, xa])), "system",
                   "fp64").cpu().numpy()
    top = nystrom.apply_iplusk(cv, xs, rows) + \
        nystrom.log_source_block(cv, rows) @ xa
    assert _rel(y[rows], top) < 1e-10
    bottom = np.array([xa.sum()] + [xs[cv.island == k].sum()
                                    for k in range(1, cv.m)])
    assert np.abs(y[cv.n:] - bottom).max() < 1e-10 * np.abs(bottom).max()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_solve_against_exact_solution(env, case, prec):
    torch, lbs = env
    isl, cv, sol, rows = case
    coeffs = synth.paper_data_coeffs(cv.m)
    g = synth.exact_harmonic(cv.x, isl.center, coeffs)
    sig, A, info = sol.solve(_t(torch, g), tol=1e-12, precision=prec)
    assert info["status"] == "LBS_OK" and info["rel_resid"] < 1e-12
    tg = synth.sphere_targets(11, 2000, isl)
    u = sol.eval(sig, A, _t(torch, tg)).cpu().numpy()
    exact = synth.exact_harmonic(tg, isl.center, coeffs)
    assert _rel(u, exact) < 1e-10
