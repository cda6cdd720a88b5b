"""The Schur-complement inverse of the preconditioner (eq. matrix_eqns_c),
formed at set-up by in-place blocked Gauss-Jordan elimination, in the
natural order (checked by a probe backward error) or with partial pivoting:
S (S^-1 e_j) = e_j for sampled columns at island counts that take every
panel shape of the pivoted GPU elimination (one row per thread and panels
of 32 columns up to 1024 islands; 2, 4 and 8 rows per thread with panels of
16, 8 and 4 columns above that) and ragged last panels of the natural-order
one (64 columns), and for a batch whose geometries have different island
counts.  The bound is a backward-error one: the entries of S reach
n / (2 pi) |log d^2| (hundreds), and the elimination is stable to a small
multiple of M eps in the norms of S and S^-1."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbs():
    from paper_1306_0612_amd import lbs as mod
    mod.load()
    return mod


@pytest.mark.parametrize("m,r0,seed,nodes", [
    (30, (0.05, 0.15), 3, 64),      # one panel shape: 32 columns
    (1100, (0.005, 0.01), 11, 32),  # 2 rows per thread, then 1
    (3000, (0.003, 0.006), 9, 24),  # 4, 2, 1
    (4500, (0.002, 0.004), 7, 24),  # 8, 4, 2, 1
])
@pytest.mark.parametrize("tol", [1e-12, 0.0])
def test_schur_inverse_columns(lbs, m, r0, seed, nodes, tol):
    isl = synth.star_islands(seed, m, r0, nodes=nodes)
    print(f"schur m={m} nodes={nodes} tol={tol}", flush=True)
    sol = lbs.Solver(isl, options=lbs.default_options(schur_tol=tol))
    err = sol.schur_residual(96)
    piv, om = sol.schur_info()
    sol.close()
    assert err < 1e-9, err
    if tol > 0:
        # these geometries need no interchanges: the natural order is kept
        assert piv == 0 and 0 <= om <= tol, (piv, om)
    else:
        assert piv == 1 and om == -1.0, (piv, om)


def test_schur_natural_order_matches_pivoted(lbs):
    """The two eliminations give the same S^-1 (to the backward error of
    either) on the preconditioned operator, and a tolerance no result can
    meet sends set-up through the fallback: the natural order is tried,
    rejected, and every block redone with partial pivoting from the intact
    S."""
    import torch
    isl = synth.star_islands(21, 700, (0.005, 0.012), nodes=32)
    print("schur natural vs pivoted m=700", flush=True)
    out = {}
    for name, tol in (("natural", 1e-12), ("pivoted", 0.0), ("fallback", 1e-300)):
        sol = lbs.Solver(isl, options=lbs.default_options(schur_tol=tol))
        x = synth.random_vector(5, sol.n_nodes + sol.n_islands)
        y = sol.matvec(torch.tensor(x, dtype=torch.float64, device="cuda"), "precond", "fp64")
        out[name] = (sol.schur_info(), sol.schur_residual(64), y.cpu().numpy())
        sol.close()
    assert out["natural"][0][0] == 0 and out["pivoted"][0] == (1, -1.0)
    piv, om = out["fallback"][0]
    assert piv == 1 and 0 < om <= 1e-12, (piv, om)
    for name in out:
        assert out[name][1] < 1e-9, (name, out[name][1])
    ref = out["pivoted"][2]
    for name in ("natural", "fallback"):
        d = np.abs(out[name][2] - ref).max() / np.abs(ref).max()
        assert d < 1e-11, (name, d)


@pytest.mark.parametrize("tol", [1e-12, 0.0])
def test_schur_inverse_batch(lbs, tol):
    sets = [synth.star_islands(61, 5, (0.08, 0.2), nodes=64),
            synth.star_islands(62, 1100, (0.005, 0.01), nodes=32),
            synth.star_islands(63, 37, (0.05, 0.12), nodes=48)]
    sol = lbs.Solver(sets, options=lbs.default_options(schur_tol=tol))
    err = sol.schur_residual(64)
    piv, _ = sol.schur_info()
    sol.close()
    assert err < 1e-9, err
    assert piv == (0 if tol > 0 else 1)
