"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every declared symbol, validates its input before touching the GPU, and its
quadtree builder covers every point pair exactly once."""
import os
import re

import numpy as np
import pytest

import synth
from oracle.geometry import Curves

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lbs():
    from paper_1306_0612_amd import lbs as mod
    if not os.path.exists(mod.LIB_PATH):
        from paper_1306_0612_amd import build
        build.build()
    mod.load()
    return mod


def _declared():
    src = open(os.path.join(ROOT, "include", "lbs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbs_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(lbs):
    names = _declared()
    assert "lbs_setup" in names and "lbs_solve" in names
    lib = lbs.load()
    for n in names:
        assert hasattr(lib, n), n


def test_default_options(lbs):
    o = lbs.default_options()
    assert (o.p64, o.p32, o.restart) == (30, 16, 50)
    assert o.inner_tol == 1e-5
    assert (o.matvec, o.graphs, o.precond, o.close_eval, o.gpu_tree, o.eval_tree,
            o.m2l_groups) == (0, 1, 1, 1, 1, 0, 0)
    assert o.schur_tol == 1e-12


def test_refinement_step_rejects_non_finite_residuals(lbs):
    """The refinement step of the mixed-precision solves never takes a NaN
    or Inf residual for a converged system (it reports LBS_ERR_NOT_FINITE),
    and otherwise sets each system's inner tolerance."""
    tol, itol_frac = 1e-10, 1e-5
    bn2 = np.array([4.0, 9.0, 1.0])
    rn2 = np.array([4.0 * 1e-22, 9.0 * 1e-8, 1.0])
    itol, done = lbs.refine_tolerances(rn2, bn2, tol, itol_frac)
    assert not done
    assert itol[0] == pytest.approx(np.sqrt(rn2[0]))       # converged: kept
    assert itol[1] == pytest.approx(itol_frac * np.sqrt(rn2[1]))
    assert itol[2] == pytest.approx(itol_frac * 1.0)
    # the floor: half the outer target
    itol, _ = lbs.refine_tolerances([1e-10], [1.0], 1e-6, 1e-5)
    assert itol[0] == pytest.approx(0.5e-6)
    itol, done = lbs.refine_tolerances(rn2 * 1e-30, bn2, tol, itol_frac)
    assert done
    for bad in (np.nan, np.inf, -1.0):
        with pytest.raises(lbs.LBSError) as e:
            lbs.refine_tolerances([1e-30, bad], [1.0, 1.0], tol, itol_frac)
        assert e.value.status == "LBS_ERR_NOT_FINITE"
    with pytest.raises(lbs.LBSError) as e:
        lbs.refine_tolerances([1e-30], [np.nan], tol, itol_frac)
    assert e.value.status == "LBS_ERR_NOT_FINITE"


@pytest.mark.parametrize("case", ["uniform", "curves", "clustered", "tiny"])
def test_quadtree_covers_each_pair_once(lbs, case):
    rng = np.random.default_rng(1)
    if case == "uniform":
        x, y, lm = rng.random(1500), rng.random(1500), 12
    elif case == "curves":
        cv = Curves(synth.star_islands(11, 6, (0.1, 0.3), nodes=150))
        x, y, lm = cv.xi.real, cv.xi.imag, 16
    elif case == "clustered":
        x = np.concatenate([rng.random(300) * 1e-7, 1 + rng.random(300)])
        y = np.concatenate([rng.random(300) * 1e-7, rng.random(300)])
        lm = 5
    else:
        x, y, lm = np.array([0.0, 1.0, 0.5]), np.array([0.0, 1.0, 0.25]), 1
    bad, st = lbs.check_tree_host(x, y, lm)
    assert bad == 0, st
    assert st["leaves"] >= 1


def test_quadtree_depth_grows_with_clustering(lbs):
    """Points crowded near one spot force a deep adaptive tree, as under the
    stereographic distortion of Section 6, Example 3."""
    rng = np.random.default_rng(2)
    _, shallow = lbs.check_tree_host(rng.random(400), rng.random(400), 8)
    x = np.concatenate([rng.random(200), 0.5 + 1e-6 * rng.random(200)])
    y = np.concatenate([rng.random(200), 0.5 + 1e-6 * rng.random(200)])
    _, deep = lbs.check_tree_host(x, y, 8)
    assert deep["levels"] > shallow["levels"] + 10


def test_quadtree_with_near_coincident_clusters(lbs):
    """Clusters of points closer than 2^-22 of the domain share the leading
    Morton key bits that the radix passes sort by; the runs they form are
    ordered by the remaining bits.  Coverage of every leaf pair stays exact
    and the clusters force the deepest levels."""
    rng = np.random.default_rng(4)
    base = rng.random((300, 2))
    clusters = [base[i] + 1e-8 * rng.random((12, 2)) for i in range(0, 300, 25)]
    pts = np.concatenate([base] + clusters)
    pts = pts[rng.permutation(len(pts))]
    bad, st = lbs.check_tree_host(pts[:, 0], pts[:, 1], 8)
    assert bad == 0, st
    assert st["levels"] >= 20


def _bad_islands(kind):
    isl = synth.star_islands(3, 4, (0.1, 0.2), nodes=32)
    if kind == "overlap":
        isl.center[1] = isl.center[0]
        isl.e1[1] = isl.e1[0]
    elif kind == "pole":
        isl.center[2] = np.array([0.0, 0.0, 1.0])
        isl.e1[2] = np.array([1.0, 0.0, 0.0])
    elif kind == "nan":
        isl.r0[0] = np.nan
    elif kind == "frame":
        isl.e1[0] = isl.center[0]
    elif kind == "radius":
        isl.coef[0, :] = 0.2
    return isl


@pytest.mark.parametrize("kind", ["overlap", "pole", "nan", "frame",
                                  "radius"])
def test_setup_rejects_bad_geometry(lbs, kind):
    assert lbs.setup_status(_bad_islands(kind)) == "LBS_ERR_GEOMETRY"


def test_setup_rejects_bad_options(lbs):
    isl = synth.star_islands(3, 2, (0.1, 0.2), nodes=32)
    assert lbs.setup_status(isl, p64=31) == "LBS_ERR_UNSUPPORTED"
    assert lbs.setup_status(isl, restart=0) == "LBS_ERR_INVALID_ARG"
    assert lbs.setup_status(isl, nodes=4) == "LBS_ERR_INVALID_ARG"
    assert lbs.setup_status(isl, graphs=2) == "LBS_ERR_INVALID_ARG"
    assert lbs.setup_status(isl, eval_tree=2) == "LBS_ERR_INVALID_ARG"
    assert lbs.setup_status(isl, m2l_groups=32) == "LBS_ERR_INVALID_ARG"
    assert lbs.setup_status(isl, schur_tol=float("nan")) == "LBS_ERR_INVALID_ARG"
    assert lbs.setup_status(isl, schur_tol=0.5) == "LBS_ERR_INVALID_ARG"


def test_deep_tree_geometry_levels_and_coverage(lbs):
    """The projection-distorted geometry (islands from near the north pole
    to near the south pole) needs 20+ quadtree levels, and its lists still
    cover every point pair exactly once."""
    cv = Curves(synth.deep_tree_islands(128))
    for lm in (16, 48):
        bad, st = lbs.check_tree_host(cv.xi.real, cv.xi.imag, lm)
        assert bad == 0
        assert st["levels"] >= 21, st


@pytest.mark.parametrize("case", ["stars", "deep", "uniform", "coincident"])
def test_pass_programs_compute_every_box_once_in_order(lbs, case):
    """The upward / downward pass programs (components of at most `cap` LDS
    slots, launched round by round) run on the host with scalar stand-ins:
    every multipole ends as its box's source count, every local as its
    box's level, from inputs that were final or written by then; the
    capacities 16 .. 408 span the FP64 and FP32 kernels' (40 .. 408)."""
    if case == "stars":
        xi = Curves(synth.star_islands(40, 30, (0.05, 0.2), nodes=128)).xi
        x, y = xi.real, xi.imag
    elif case == "deep":
        xi = Curves(synth.deep_tree_islands(128)).xi
        x, y = xi.real, xi.imag
    elif case == "uniform":
        x, y = np.random.default_rng(1).uniform(-1, 1, (2, 20000))
    else:  # five coincident points: a chain of boxes to the deepest level
        x = np.array([0.25] * 5 + [-0.5])
        y = np.array([0.75] * 5 + [0.1])
    for lm in (1, 8, 64):
        for cap in (16, 40, 96, 408):
            bad, rounds = lbs.check_passes_host(x, y, lm, cap)
            assert bad == 0, (lm, cap)
            assert min(rounds) >= 1


def test_pass_programs_need_few_rounds(lbs):
    """Larger components take fewer launches: at the FP32 kernel's capacity
    a clustered star geometry needs at most two rounds each way, fewer than
    its quadtree has levels by far."""
    xi = Curves(synth.star_islands(40, 30, (0.05, 0.2), nodes=128)).xi
    _, st = lbs.check_tree_host(xi.real[:2000], xi.imag[:2000], 1)
    bad, rounds = lbs.check_passes_host(xi.real, xi.imag, 1, 408)
    assert bad == 0 and max(rounds) <= 2 and st["levels"] >= 8
