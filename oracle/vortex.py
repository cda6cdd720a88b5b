"""Point vortices in the domain (Section 6, Example 2).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

With point vortices of strengths Gamma_j at sphere points v_j in the domain,
the stream function is decomposed as

    psi = psi* + sum_j Gamma_j G(x, v_j),

G the generalized fundamental solution of Section 1.1 (eq.
eqn:greens_func), and psi* solves the Laplace-Beltrami Dirichlet problem of
the paper with the data g - sum_j Gamma_j G(x, v_j) on the island curves
(so psi = g there).  psi* is solved and evaluated exactly as any other data
(nystrom.solve_dense, evaluate.evaluate); the vortex sum is direct.
"""
import numpy as np

from . import nystrom, evaluate


def vortex_field(points, xyz_v, gamma):
    """sum_j gamma_j G(x, v_j) at sphere points (n, 3)."""
    return nystrom.greens(np.asarray(points, float),
                          np.asarray(xyz_v, float)) @ np.asarray(gamma, float)


def solve(cv, g, xyz_v, gamma):
    """sigma, A of psi* for node data g and the vortices."""
    return nystrom.solve_dense(cv, np.asarray(g, float)
                               - vortex_field(cv.x, xyz_v, gamma))


def evaluate_psi(cv, sigma, A, targets, xyz_v, gamma):
    """psi = psi* + sum_j gamma_j G(x, v_j) at sphere targets."""
    return (evaluate.evaluate(cv, sigma, A, targets)
            + vortex_field(targets, xyz_v, gamma))
