"""Derivatives of a linear functional of the solution at sphere targets.

J = w . u,  u = T x  (eq. eqn:u_multi, Section 4.1),
A x = [2 g; 0]       (eq. matrix_eqns, Section 5),

with x = [sigma; A].  The method's quantities are written out densely:

* T is the evaluation as a matrix, column by column from evaluate.evaluate
  (linear in sigma and A);
* the adjoint lambda solves A^T lambda = T^T w by LU of the transposed
  system matrix of nystrom.system_matrix;
* dJ/dg = 2 lambda_sigma (the right-hand side is 2 g);
* dJ/dbeta for the 16 radius coefficients of each island (Section 3's curves
  r(t) = r0 (1 + sum a_n cos nt + b_n sin nt)) two ways: by central
  differences of the whole dense pipeline (rebuild the curves, solve by LU,
  evaluate), and by the adjoint assembly
  dJ/dbeta = w . (dT/dbeta) x - lambda . (dA/dbeta) x
  with the two matrix derivatives by central differences of the assembled
  matrices (the derivative of A x = b with b fixed gives
  A dx = -(dA) x, and w . T dx = -lambda . (dA) x).  The node data g is a
  vector held fixed when the shape moves.

For a quadratic misfit L = 1/2 |u - u*|^2 the same formulas apply with
w = u - u* at the current shape.
"""
import numpy as np
import scipy.linalg as sla

from . import nystrom, evaluate
from .geometry import Curves


def eval_matrix(cv, targets):
    """Dense T (n_targets x (N + M)) with u = T [sigma; A]."""
    targets = np.asarray(targets, float)
    n, m = cv.n, cv.m
    out = np.empty((targets.shape[0], n + m))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        out[:, j] = evaluate.evaluate(cv, e, np.zeros(m), targets)
    for k in range(m):
        e = np.zeros(m)
        e[k] = 1.0
        out[:, n + k] = evaluate.evaluate(cv, np.zeros(n), e, targets)
    return out


def adjoint_solve(cv, rhs_s, rhs_a=None):
    """lambda = A^-T [rhs_s; rhs_a] by LU of the dense system matrix."""
    rhs_a = np.zeros(cv.m) if rhs_a is None else np.asarray(rhs_a, float)
    rhs = np.concatenate([np.asarray(rhs_s, float), rhs_a])
    lam = sla.lu_solve(sla.lu_factor(nystrom.system_matrix(cv).T,
                                     check_finite=False), rhs,
                       check_finite=False)
    return lam[:cv.n], lam[cv.n:]


def eval_transpose(cv, targets, w):
    """T^T w split into its node part (N) and island part (M)."""
    tw = eval_matrix(cv, targets).T @ np.asarray(w, float)
    return tw[:cv.n], tw[cv.n:]


def functional(islands, g, targets, w):
    """J = w . u for node data g on the geometry `islands` (dense)."""
    cv = Curves(islands)
    sigma, A = nystrom.solve_dense(cv, g)
    return float(np.dot(w, evaluate.evaluate(cv, sigma, A, targets)))


def grad_data(cv, targets, w):
    """dJ/dg = 2 lambda_sigma with lambda = A^-T T^T w."""
    gs, ga = eval_transpose(cv, targets, w)
    lam_s, _ = adjoint_solve(cv, gs, ga)
    return 2.0 * lam_s


def _with_coef(islands, k, q, value):
    out = islands.subset(np.arange(islands.m))
    out.coef[k, q] = value
    return out


def grad_shape_fd(islands, g, targets, w, step=1e-4, islands_idx=None):
    """dJ/dcoef (M x 16) by the fourth-order central difference
    (8 (J(+h) - J(-h)) - (J(+2h) - J(-2h))) / (12 h) per coefficient."""
    m = islands.m
    out = np.zeros((m, 16))
    ks = range(m) if islands_idx is None else islands_idx
    for k in ks:
        for q in range(16):
            b = islands.coef[k, q]
            f = {s: functional(_with_coef(islands, k, q, b + s * step), g,
                               targets, w) for s in (-2, -1, 1, 2)}
            out[k, q] = (8.0 * (f[1] - f[-1]) - (f[2] - f[-2])) / (12.0 * step)
    return out


def grad_shape_adjoint(islands, g, targets, w, step=1e-5, islands_idx=None):
    """dJ/dcoef (M x 16) by the adjoint assembly: x = [sigma; A] of the
    current shape, lambda = A^-T T^T w, and per coefficient
    w . (dT) x - lambda . (dA) x with dT, dA the central differences
    (X(+h) - X(-h)) / (2 h) of the dense evaluation and system matrices."""
    cv = Curves(islands)
    sigma, A = nystrom.solve_dense(cv, g)
    x = np.concatenate([sigma, A])
    gs, ga = eval_transpose(cv, targets, w)
    lam = np.concatenate(adjoint_solve(cv, gs, ga))
    w = np.asarray(w, float)
    m = islands.m
    out = np.zeros((m, 16))
    ks = range(m) if islands_idx is None else islands_idx
    for k in ks:
        for q in range(16):
            b = islands.coef[k, q]
            cp = Curves(_with_coef(islands, k, q, b + step))
            cm = Curves(_with_coef(islands, k, q, b - step))
            dT = (eval_matrix(cp, targets) - eval_matrix(cm, targets)) / (2.0 * step)
            dA = (nystrom.system_matrix(cp) - nystrom.system_matrix(cm)) / (2.0 * step)
            out[k, q] = w @ (dT @ x) - lam @ (dA @ x)
    return out
