"""lbs_set_orders and the schedule autotuner (lbs_autotune)."""
import numpy as np
import pytest

import synth
from oracle import nystrom
from oracle.geometry import Curves

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1306_0612_amd import lbs
    lbs.load()
    return torch, lbs


def _t(torch, a):
    return torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda")


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(b).max()


@pytest.fixture(scope="module")
def geom():
    isl = synth.star_islands(101, 6, (0.08, 0.2), nodes=128)
    cv = Curves(isl)
    x = synth.random_vector(102, cv.n)
    return isl, cv, x, nystrom.apply_iplusk(cv, x)


def test_set_orders_matches_fresh_handle(env, geom):
    torch, lbs = env
    isl, cv, x, ref = geom
    a = lbs.Solver(isl, leaf_max=16, p64=20, p32=12)
    xd = _t(torch, x)
    a.matvec(xd, "iplusk", "mixed")                  # buffers for p32 = 12
    a.set_orders(36, 20)
    b = lbs.Solver(isl, leaf_max=16, p64=36, p32=20)
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-6)):
        ya = a.matvec(xd, "iplusk", prec)
        yb = b.matvec(xd, "iplusk", prec)
        assert torch.equal(ya, yb), prec
        assert _rel(ya.cpu().numpy(), ref) < tol, prec
    # solves after the change use the new orders
    s1, A1, _ = a.solve(xd, tol=1e-12)
    s2, A2, _ = b.solve(xd, tol=1e-12)
    assert torch.equal(s1, s2) and torch.equal(A1, A2)


def test_autotune_meets_tolerances(env, geom):
    torch, lbs = env
    isl, cv, x, ref = geom
    best, entries = lbs.autotune(isl, tol_mixed=1e-6, tol_fp64=1e-10)
    assert len(entries) == 6 * 8 + 3  # leaf sizes x orders, then M2L widths
    assert all(e["ms"] > 0 for e in entries)
    assert best.leaf_max in (24, 32, 48, 64, 96, 128)
    assert best.p32 in (12, 16, 20, 24) and best.p64 in (20, 24, 30, 36)
    assert best.m2l_groups in (512, 1024, 2048)
    widths = [e for e in entries if e["m2l_groups"]]
    assert [e["m2l_groups"] for e in widths] == [512, 1024, 2048]
    assert all(e["leaf_max"] == best.leaf_max and e["p32"] == best.p32 for e in widths)
    assert best.graphs == 1
    chosen = [e for e in entries if e["leaf_max"] == best.leaf_max and
              e["p32"] == best.p32]
    assert chosen and chosen[0]["err"] <= 1e-6
    sol = lbs.Solver(isl, options=best)
    xd = _t(torch, x)
    assert _rel(sol.matvec(xd, "iplusk", "mixed").cpu().numpy(), ref) < 1e-6
    assert _rel(sol.matvec(xd, "iplusk", "fp64").cpu().numpy(), ref) < 1e-10
    # errors fall with the order on a fixed tree
    for lm in (24, 128):
        errs = [e["err"] for e in entries if e["leaf_max"] == lm and e["p64"]]
        assert errs[-1] < errs[0]


@pytest.mark.parametrize("p64,p32", [(20, 12), (24, 16), (30, 20), (40, 24), (48, 24)])
def test_every_order_against_oracle(env, geom, p64, p32):
    """Each supported expansion order, through the P2M / P2L register
    passes it takes (FP64 orders above 16 and FP32 orders above 16 use
    several passes or wider sums), against the oracle's direct sum: a wrong
    pass would give O(1) errors; the orders the library defaults to and
    above meet the production tolerances."""
    torch, lbs = env
    isl, cv, x, ref = geom
    sol = lbs.Solver(isl, leaf_max=16, p64=p64, p32=p32)
    xd = _t(torch, x)
    e64 = _rel(sol.matvec(xd, "iplusk", "fp64").cpu().numpy(), ref)
    e32 = _rel(sol.matvec(xd, "iplusk", "mixed").cpu().numpy(), ref)
    assert e64 < (1e-10 if p64 >= 30 else 1e-5), e64
    assert e32 < (1e-6 if p32 >= 16 else 1e-4), e32


def test_m2l_width_changes_no_result(env, geom):
    """The FP32 M2L launch width only changes which wave takes which box:
    the products are bit for bit the same."""
    torch, lbs = env
    isl, cv, x, ref = geom
    xd = _t(torch, x)
    ys = [lbs.Solver(isl, leaf_max=16, m2l_groups=g).matvec(xd, "iplusk", "mixed")
          for g in (0, 64, 512, 4096)]
    for y in ys[1:]:
        assert torch.equal(y, ys[0])


def test_autotune_cache(env, geom, tmp_path):
    """A second call with the same problem reads the tuned schedule back from
    the cache file; another tolerance is another key."""
    torch, lbs = env
    isl, cv, x, ref = geom
    path = str(tmp_path / "tune.txt")
    b1, e1, hit1 = lbs.autotune(isl, tol_mixed=1e-6, tol_fp64=1e-10, cache=path)
    b2, e2, hit2 = lbs.autotune(isl, tol_mixed=1e-6, tol_fp64=1e-10, cache=path)
    assert (hit1, hit2) == (False, True)
    for f in ("leaf_max", "p32", "p64", "m2l_groups", "graphs"):
        assert getattr(b1, f) == getattr(b2, f), f
    assert e1 == e2
    _, _, hit3 = lbs.autotune(isl, tol_mixed=2e-6, tol_fp64=1e-10, cache=path)
    assert not hit3
    assert len(open(path).read().splitlines()) == 2
