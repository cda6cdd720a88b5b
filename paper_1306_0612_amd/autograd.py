"""Differentiable solve-and-evaluate: u(g, beta) at sphere targets.

Forward: set up the islands with radius coefficients beta (the handle of the
last geometry is kept and reused while the geometry and options are the
same), solve the system of eqs. matrix_eqns with data g (GMRES with the
block preconditioner; FP64 FMM, or the FP32 far and near field inside FP64
refinement with precision="mixed") and evaluate eq. eqn:u_multi at the
targets.  Backward, for
the incoming w = dL/du: the transposed evaluation T^T w, the transposed solve
A^T lambda = T^T w, then dL/dg = 2 lambda_sigma and dL/dbeta from the shape
derivatives of the operator and the evaluation.  Every step runs in liblbs
(lbs_setup, lbs_solve, lbs_eval, lbs_eval_T, lbs_solve_T, lbs_shape_vjp);
this module only moves tensors.
"""
import hashlib
import types

import numpy as np
import torch

from . import lbs


def _islands_with(islands, coef):
    c = coef.detach().to("cpu", torch.float64).numpy()
    if c.shape != (len(islands.r0), 16):
        raise ValueError("coef must have shape (M, 16)")
    return types.SimpleNamespace(center=islands.center, e1=islands.e1,
                                 r0=islands.r0, coef=c, n=islands.n)


# The handle of the last geometry, keyed by its content and the options: an
# optimization loop that changes only the data g, or calls forward again
# before moving the shape, reuses it instead of building a new one.
_LAST = {"key": None, "sol": None}


def _geometry_key(isl, options):
    h = hashlib.sha1()
    for a in (isl.center, isl.e1, isl.r0, isl.coef, isl.n):
        h.update(np.ascontiguousarray(np.asarray(a, dtype=np.float64)).tobytes())
    h.update(repr(sorted(options.items())).encode())
    return h.hexdigest()


def _solver(isl, options):
    key = _geometry_key(isl, options)
    if _LAST["key"] != key:
        # a graph of an earlier geometry still holds its own handle (freed
        # with the last reference), so the cache only lets go of it here
        _LAST["key"], _LAST["sol"] = None, None
        _LAST["sol"] = lbs.Solver(isl, **options)
        _LAST["key"] = key
    return _LAST["sol"]


class SolveEval(torch.autograd.Function):
    """u = SolveEval.apply(g, coef, islands, targets, tol, precision,
    options)."""

    @staticmethod
    def forward(ctx, g, coef, islands, targets, tol, precision, options):
        sol = _solver(_islands_with(islands, coef), options)
        sig, A, info = sol.solve(g.detach().contiguous(), tol=tol,
                                 precision=precision)
        u = sol.eval(sig, A, targets)
        ctx.sol = sol
        ctx.targets = targets
        ctx.tol = tol
        ctx.precision = precision
        ctx.coef_device = coef.device
        ctx.forward_info = info
        ctx.save_for_backward(sig, A)
        return u

    @staticmethod
    def backward(ctx, w):
        sol, targets = ctx.sol, ctx.targets
        sig, A = ctx.saved_tensors
        w = w.detach().to(torch.float64).contiguous()
        gs, ga = sol.eval_T(w, targets)
        lam_s, _, info = sol.solve_T(gs, ga, tol=ctx.tol,
                                     precision=ctx.precision)
        ctx.adjoint_info = info
        dg = 2.0 * lam_s if ctx.needs_input_grad[0] else None
        dc = None
        if ctx.needs_input_grad[1]:
            dc = sol.shape_vjp(sig, A, lam_s, w, targets).to(ctx.coef_device)
        ctx.sol = None  # the handle stays alive only in the cache
        return dg, dc, None, None, None, None, None


def solve_eval(g, coef, islands, targets, tol=1e-12, precision="fp64",
               **options):
    """u at `targets` (T x 3, float64 CUDA) for node data g (N, float64
    CUDA) on islands whose radius coefficients are `coef` (M x 16);
    `islands` supplies center, e1, r0 and n.  Differentiable in g and coef.
    precision ("fp64" or "mixed") applies to the solve and to the
    transposed solve of the backward pass."""
    return SolveEval.apply(g, coef, islands, targets, tol, precision, options)
