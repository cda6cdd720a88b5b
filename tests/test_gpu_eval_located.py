"""GPU parity of the evaluation that places each target in the handle's own
quadtree (option eval_tree = 0, the default) against the oracle's direct
evaluation and against the evaluation over a quadtree of nodes and targets
(eval_tree = 1): targets away from the curves, in quadrants without nodes,
far outside the nodes' root square (near the north pole), at the pole,
exactly at nodes; several right-hand sides; batch handles; the full-size
workload at 1e5 targets.  The same for the transposed evaluation
(lbs_eval_T), where the located targets are the sources of the handle's
own FMM, against the oracle's dense transpose.

The two evaluations are different FMM approximations of the same sums, each
within the FMM's error at p64 = 30 (ratio 0.47 at worst): each is held to
1e-10 of the oracle, and to 3e-10 of each other where the oracle cannot
follow (targets at nodes, the full size).  Targets near the north pole are
held to the oracle on the located path only: a quadtree over nodes and such
targets has a root square of half-width ~2 / colatitude around nodes within
|xi| < 2, and its deep boxes' centres carry rounding errors of that root's
scale (2e-10 of the oracle at every target of a set with colatitudes down
to 1e-6), so the tree path is run on the targets away from the pole."""
import numpy as np
import pytest

import synth
from oracle import adjoint, evaluate
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


def _near_pole(count, seed):
    """Points at colatitudes 1e-6 .. 0.05 (stereographic images far outside
    the nodes' bounding square)."""
    rng = np.random.default_rng(seed)
    th = 10.0 ** rng.uniform(-6, np.log10(0.05), count)
    ph = rng.uniform(0, 2 * np.pi, count)
    return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1)


CASES = [  # (seed, islands, nodes, r0 range, leaf_max)
    (41, 7, 90, (0.08, 0.2), 6),
    (42, 25, 64, (0.03, 0.08), 16),
    (43, 2, 400, (0.2, 0.35), 40),
]


@pytest.mark.parametrize("case", CASES)
def test_located_matches_oracle_and_tree_path(env, case):
    torch, lbs = env
    seed, m, n, rr, lm = case
    isl = synth.star_islands(seed, m, rr, nodes=n)
    cv = Curves(isl)
    sig = np.stack([synth.random_vector(seed + 1, cv.n), synth.random_vector(seed + 2, cv.n),
                    synth.random_vector(seed + 3, cv.n)])
    A = np.stack([synth.random_vector(seed + 4, cv.m), synth.random_vector(seed + 5, cv.m),
                  np.zeros(cv.m)])
    tg = np.concatenate([synth.sphere_targets(seed + 6, 500, isl), _near_pole(40, seed + 7),
                         [[0.0, 0.0, 1.0]]])
    loc = lbs.Solver(isl, leaf_max=lm)
    ref_tree = lbs.Solver(isl, leaf_max=lm, eval_tree=1)
    u = _np(loc.eval(_t(torch, sig), _t(torch, A), _t(torch, tg)))
    v = _np(ref_tree.eval(_t(torch, sig), _t(torch, A), _t(torch, tg[:500])))
    for r in range(3):
        ref = evaluate.evaluate(cv, sig[r], A[r], tg)
        print(f"column {r}: located {_rel(u[r], ref):.2e}, tree {_rel(v[r], ref[:500]):.2e}")
        assert _rel(u[r], ref) < 1e-10, r
        assert _rel(v[r], ref[:500]) < 1e-10, r
        assert _rel(u[r][:500], v[r]) < 3e-10, r
    # a second target set on the same handle (the plan is rebuilt), and the
    # first one again (cached)
    tg2 = synth.sphere_targets(seed + 8, 300, isl)
    u2 = _np(loc.eval(_t(torch, sig[0]), _t(torch, A[0]), _t(torch, tg2)))
    assert _rel(u2, evaluate.evaluate(cv, sig[0], A[0], tg2)) < 1e-10
    u3 = _np(loc.eval(_t(torch, sig), _t(torch, A), _t(torch, tg)))
    assert np.array_equal(u3, u)


def test_located_at_nodes_and_in_empty_quadrants(env):
    """Targets exactly at nodes (the node's own term is left out, as in the
    operator's rows) and on a fine grid over the whole sphere cap, with the
    trapezoidal rule everywhere (close_eval = 0): both evaluations sum the
    same terms."""
    torch, lbs = env
    isl = synth.star_islands(44, 9, (0.05, 0.15), nodes=72)
    cv = Curves(isl)
    sig = synth.random_vector(45, cv.n)
    A = synth.random_vector(46, cv.m)
    g = np.linspace(-0.95, 0.95, 41)
    X, Y = np.meshgrid(g, g)
    keep = X ** 2 + Y ** 2 < 0.95
    Z = np.sqrt(1 - X[keep] ** 2 - Y[keep] ** 2)
    grid = np.stack([X[keep], Y[keep], Z], 1)
    nn = len(cv.x[::7])
    tg = np.concatenate([cv.x[::7], grid, -grid])
    loc = lbs.Solver(isl, leaf_max=8, close_eval=0)
    ref_tree = lbs.Solver(isl, leaf_max=8, close_eval=0, eval_tree=1)
    u = _np(loc.eval(_t(torch, sig), _t(torch, A), _t(torch, tg)))
    v = _np(ref_tree.eval(_t(torch, sig), _t(torch, A), _t(torch, tg)))
    assert np.isfinite(u).all()
    assert _rel(u, v) < 3e-10
    ref = evaluate.evaluate(cv, sig, A, tg[nn:])
    assert _rel(u[nn:], ref) < 1e-10


def test_located_batch(env):
    torch, lbs = env
    geoms = [synth.star_islands(50 + q, 3 + 2 * q, (0.08, 0.2), nodes=64 + 16 * q)
             for q in range(4)]
    cvs = [Curves(g) for g in geoms]
    loc = lbs.Solver(geoms, leaf_max=10)
    ref_tree = lbs.Solver(geoms, leaf_max=10, eval_tree=1)
    no, io = loc.node_offsets, loc.island_offsets
    sig = synth.random_vector(60, loc.n_nodes)
    A = synth.random_vector(61, loc.n_islands)
    tgs = [np.concatenate([synth.sphere_targets(70 + q, 60 + 9 * q, g), _near_pole(5, 80 + q)])
           for q, g in enumerate(geoms)]
    toff = np.concatenate([[0], np.cumsum([len(t) for t in tgs])])
    away = np.concatenate([np.arange(toff[q], toff[q + 1] - 5) for q in range(len(geoms))])
    aoff = toff - 5 * np.arange(len(toff))
    tall = _t(torch, np.concatenate(tgs))
    u = _np(loc.eval(_t(torch, sig), _t(torch, A), tall, target_offsets=toff))
    v = _np(ref_tree.eval(_t(torch, sig), _t(torch, A), _t(torch, np.concatenate(tgs)[away]),
                          target_offsets=aoff))
    assert _rel(u[away], v) < 3e-10
    for q, cv in enumerate(cvs):
        ref = evaluate.evaluate(cv, sig[no[q]:no[q + 1]], A[io[q]:io[q + 1]], tgs[q])
        assert _rel(u[toff[q]:toff[q + 1]], ref) < 1e-10, q


def test_located_full_size(env):
    """2000 star islands x 512 nodes, 1e5 targets: the two evaluations agree
    on every target; a second target set costs no tree."""
    torch, lbs = env
    import time
    isl = synth.config_islands("stars2000x512")
    loc = lbs.Solver(isl, leaf_max=64)
    sig = _t(torch, synth.random_vector(90, loc.n_nodes))
    A = _t(torch, synth.random_vector(91, loc.n_islands))
    tg = _t(torch, synth.sphere_targets(92, 100000, isl))
    u = loc.eval(sig, A, tg)
    tg2 = _t(torch, synth.sphere_targets(93, 100000, isl))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u2 = loc.eval(sig, A, tg2)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"eval at 1e5 new targets: {1e3 * dt:.2f} ms", flush=True)
    del loc
    ref_tree = lbs.Solver(isl, leaf_max=64, eval_tree=1)
    v = ref_tree.eval(sig, A, tg)
    v2 = ref_tree.eval(sig, A, tg2)
    assert _rel(_np(u), _np(v)) < 3e-10
    assert _rel(_np(u2), _np(v2)) < 3e-10


@pytest.mark.parametrize("case", CASES)
def test_located_transpose_matches_dense(env, case):
    torch, lbs = env
    seed, m, n, rr, lm = case
    isl = synth.star_islands(seed, m, rr, nodes=n)
    cv = Curves(isl)
    tg = np.concatenate([synth.sphere_targets(seed + 6, 400, isl), _near_pole(30, seed + 7),
                         [[0.0, 0.0, 1.0]]])
    rng = np.random.default_rng(seed + 9)
    W = rng.standard_normal((2, len(tg)))
    loc = lbs.Solver(isl, leaf_max=lm)
    ref_tree = lbs.Solver(isl, leaf_max=lm, eval_tree=1)
    gs, ga = loc.eval_T(_t(torch, W), _t(torch, tg))
    gs2, _ = ref_tree.eval_T(_t(torch, W[:, :400]), _t(torch, tg[:400]))
    for r in range(2):
        rs, ra = adjoint.eval_transpose(cv, tg, W[r])
        print(f"column {r}: located {_rel(_np(gs[r]), rs):.2e}")
        assert _rel(_np(gs[r]), rs) < 1e-10, r
        assert _rel(_np(ga[r]), ra) < 1e-12, r
        rs4, _ = adjoint.eval_transpose(cv, tg[:400], W[r, :400])
        assert _rel(_np(gs2[r]), rs4) < 1e-10, r
    # duality with the located forward evaluation: w . u(sigma, A) equals
    # (eval_T w) . (sigma, A) to the FMM's accuracy
    sig = synth.random_vector(seed + 10, cv.n)
    A = synth.random_vector(seed + 11, cv.m)
    u = _np(loc.eval(_t(torch, sig), _t(torch, A), _t(torch, tg)))
    lhs = W[0] @ u
    rhs = _np(gs[0]) @ sig + _np(ga[0]) @ A
    assert abs(lhs - rhs) < 1e-10 * np.abs(W[0]).sum() * np.abs(u).max()


def test_located_transpose_full_size(env):
    """2000 star islands x 512 nodes, 1e5 targets: the located transposed
    evaluation against the tree path on every node; timed on a second
    target set."""
    torch, lbs = env
    import time
    isl = synth.config_islands("stars2000x512")
    loc = lbs.Solver(isl, leaf_max=64)
    tg = _t(torch, synth.sphere_targets(94, 100000, isl))
    w = _t(torch, np.random.default_rng(95).standard_normal(100000))
    gs, ga = loc.eval_T(w, tg)
    tg2 = _t(torch, synth.sphere_targets(96, 100000, isl))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gs2, ga2 = loc.eval_T(w, tg2)
    torch.cuda.synchronize()
    print(f"eval_T at 1e5 new targets: {1e3 * (time.perf_counter() - t0):.2f} ms", flush=True)
    del loc
    ref_tree = lbs.Solver(isl, leaf_max=64, eval_tree=1)
    hs, ha = ref_tree.eval_T(w, tg)
    assert _rel(_np(gs), _np(hs)) < 3e-10
    assert _rel(_np(ga), _np(ha)) < 1e-12


def test_plan_lookup_sees_changed_targets(env):
    """The cached placement is found by comparing the targets themselves:
    targets changed in place in the same tensor get a new placement."""
    torch, lbs = env
    isl = synth.star_islands(47, 6, (0.08, 0.2), nodes=64)
    cv = Curves(isl)
    sig = synth.random_vector(48, cv.n)
    A = synth.random_vector(49, cv.m)
    tg1 = synth.sphere_targets(50, 200, isl)
    tg2 = synth.sphere_targets(51, 200, isl)
    sol = lbs.Solver(isl, leaf_max=8)
    t = _t(torch, tg1)
    s_, a_ = _t(torch, sig), _t(torch, A)
    u1 = _np(sol.eval(s_, a_, t))
    t.copy_(_t(torch, tg2))
    u2 = _np(sol.eval(s_, a_, t))
    assert _rel(u1, evaluate.evaluate(cv, sig, A, tg1)) < 1e-10
    assert _rel(u2, evaluate.evaluate(cv, sig, A, tg2)) < 1e-10
    w = np.random.default_rng(52).standard_normal(200)
    gs, _ = sol.eval_T(_t(torch, w), t)
    rs, _ = adjoint.eval_transpose(cv, tg2, w)
    assert _rel(_np(gs), rs) < 1e-10
