"""The GPU quadtree builder against the host builder (lbs_compare_trees):
every box field (centres, ranges, levels, parents, children, Morton cell),
the level pointers, both permutations and the U, V (with offset codes),
W and X lists must agree entry for entry.  Point sets: node images of the
workload's star islands, a clustered set whose tree is 20+ levels deep,
targets apart from the sources (forward and transposed evaluation trees),
one point, coincident points (the tree runs to its maximum depth) and
several leaf sizes.  A handle set up with the GPU builder then gives the
same matvec, bit for bit, as one set up with the host builder."""
import numpy as np
import pytest

import synth
from oracle.geometry import Curves

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1306_0612_amd import lbs
    lbs.load()
    return torch, lbs


def _t(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _stereo(x):
    d = 1.0 - x[:, 2]
    return x[:, 0] / d, x[:, 1] / d


def _cmp(env, x, y, leaf_max, tx=None, ty=None):
    torch, lbs = env
    print(f"compare_trees n={len(x)} nt={0 if tx is None else len(tx)} "
          f"leaf_max={leaf_max}", flush=True)
    bad, lev = lbs.compare_trees(
        _t(torch, x), _t(torch, y), leaf_max,
        None if tx is None else _t(torch, tx), None if ty is None else _t(torch, ty))
    assert bad == 0, (bad, lev)
    return lev


@pytest.mark.parametrize("leaf_max", [1, 16, 64])
def test_star_nodes(env, leaf_max):
    isl = synth.star_islands(40, 7, (0.05, 0.2), nodes=96)
    x, y = _stereo(Curves(isl).x)
    assert _cmp(env, x, y, leaf_max) >= 4


def test_deep_clustered(env):
    x, y = _stereo(Curves(synth.deep_tree_islands(256)).x)
    assert _cmp(env, x, y, 16) >= 20


def test_uniform_large(env):
    rng = np.random.default_rng(5)
    x = rng.uniform(-3, 3, 300_000)
    y = rng.uniform(-3, 3, 300_000)
    _cmp(env, x, y, 64)


@pytest.mark.parametrize("transposed", [False, True])
def test_targets_apart(env, transposed):
    isl = synth.star_islands(24, 11, (0.05, 0.2), nodes=128)
    sx, sy = _stereo(Curves(isl).x)
    tg = synth.sphere_targets(13, 4000, isl)
    tg = tg[tg[:, 2] < 1 - 1e-12]
    tx, ty = _stereo(tg)
    if transposed:
        sx, sy, tx, ty = tx, ty, sx, sy
    _cmp(env, sx, sy, 32, tx, ty)


def test_single_point(env):
    assert _cmp(env, np.array([0.3]), np.array([-0.2]), 1) == 1


def test_coincident_points(env):
    # three copies of one point: split to the maximum level (29)
    x = np.array([0.25, 0.25, 0.25, -0.5])
    y = np.array([0.75, 0.75, 0.75, 0.1])
    assert _cmp(env, x, y, 2) == 30
    assert _cmp(env, x[:3], y[:3], 1, np.array([0.25]), np.array([0.75])) == 30


def test_ragged_counts(env):
    rng = np.random.default_rng(9)
    for n in (2, 63, 64, 65, 4095, 4097):
        x = rng.standard_normal(n)
        y = rng.standard_normal(n)
        _cmp(env, x, y, 8)


def test_solver_same_matvec(env):
    torch, lbs = env
    isl = synth.star_islands(30, 12, (0.05, 0.15), nodes=128)
    cv = Curves(isl)
    X = _t(torch, synth.random_vector(17, cv.n)[None, :])
    out = []
    for gt in (0, 1):
        sol = lbs.Solver(isl, gpu_tree=gt, leaf_max=32)
        info = sol.tree_info()
        out.append((info, sol.matvec(X, "iplusk", "fp64").cpu().numpy(),
                    sol.matvec(X, "iplusk", "mixed").cpu().numpy()))
        sol.close()
    assert out[0][0] == out[1][0]
    assert np.array_equal(out[0][1], out[1][1])
    assert np.array_equal(out[0][2], out[1][2])


def test_solver_same_evaluations(env):
    """Evaluation plans from the GPU builder (points, maps and list tables
    formed on the device) give the same forward and transposed evaluations,
    bit for bit, as plans from the host builder."""
    torch, lbs = env
    isl = synth.star_islands(30, 12, (0.05, 0.15), nodes=128)
    cv = Curves(isl)
    tg = _t(torch, synth.sphere_targets(21, 3000, isl))
    sig = _t(torch, synth.random_vector(22, cv.n))
    A = _t(torch, synth.random_vector(23, cv.m))
    w = _t(torch, synth.random_vector(24, tg.shape[0]))
    out = []
    for gt in (0, 1):
        sol = lbs.Solver(isl, gpu_tree=gt, leaf_max=32)
        u = sol.eval(sig, A, tg).cpu().numpy()
        gs, ga = sol.eval_T(w, tg)
        out.append((u, gs.cpu().numpy(), ga.cpu().numpy()))
        sol.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
