"""Dense Nystrom discretization of the augmented double-layer system.

Section 5, eqs. disc_sphere, disc_constr and matrix_eqns:

    [ I + K   E ] [ sigma ]   [ 2 g ]
    [   F     D ] [   A   ] = [  0  ]

with, for a target node i and a source node j on curve m (parameter spacing
h_m, orientation sign s_m, Section 3 eq. dlpC with the correction term's
sign as obtained from differentiating eq. fundC),

    (I + K)_ij = delta_ij + 2 h_m Khat_ij,
    Khat_ij = (s_m / 2 pi) Im[ xi'_j / (xi_i - xi_j)
                               + conj(xi_j) xi'_j / (1 + |xi_j|^2) ],  i != j
    Khat_ii = (s_k / 2 pi) Im[ -xi''_i / (2 xi'_i)
                               + conj(xi_i) xi'_i / (1 + |xi_i|^2) ],

where the diagonal's first term is the exact limit of the off-diagonal
Cauchy term along the curve (the curvature term of eq. cont_kern).
E_im = 2 G(x_i, c_m) with the generalized fundamental solution
G(x, y) = -(1/2 pi) log|x - y| + (1/4 pi) log 2 (Section 1.1,
eq. eqn:greens_func), F's row k >= 1 sums island k's densities
(eq. disc_constr), and D's row 0 imposes sum(A) = 0 (eq. eqn:sum_ak).
"""
import numpy as np
import scipy.linalg as sla

from .geometry import Curves

LOG2 = np.log(2.0)


def greens(x, y):
    """G(x, y) for sphere points x (n,3), y (m,3) -> (n, m)."""
    d2 = ((x[:, None, :] - y[None, :, :]) ** 2).sum(-1)
    return -np.log(d2) / (4 * np.pi) + LOG2 / (4 * np.pi)


def kernel_block(cv, rows):
    """Rows `rows` of K = (I + K) - I as a dense (len(rows), N) block."""
    rows = np.asarray(rows)
    xi_t = cv.xi[rows]
    diff = xi_t[:, None] - cv.xi[None, :]
    same = rows[:, None] == np.arange(cv.n)[None, :]
    diff = np.where(same, 1.0, diff)
    cauchy = np.imag(cv.dxi[None, :] / diff)
    # exact self-limit of the Cauchy term along the curve
    diag = np.imag(-cv.ddxi[rows] / (2 * cv.dxi[rows]))
    cauchy = np.where(same, diag[:, None], cauchy)
    corr = np.imag(np.conj(cv.xi) * cv.dxi / (1 + np.abs(cv.xi) ** 2))
    w = cv.s * cv.h / np.pi                     # 2 h_m * s_m / (2 pi)
    return (cauchy + corr[None, :]) * w[None, :]


def log_source_block(cv, rows=None):
    """E (or its rows): E_im = 2 G(x_i, c_m)."""
    x = cv.x if rows is None else cv.x[np.asarray(rows)]
    return 2.0 * greens(x, cv.center)


def constraint_blocks(cv):
    """F (M x N) and D (M x M): row 0 is sum(A) = 0, row k >= 1 is
    sum over island k of sigma = 0."""
    m, n = cv.m, cv.n
    F = np.zeros((m, n))
    for k in range(1, m):
        F[k, cv.island == k] = 1.0
    D = np.zeros((m, m))
    D[0, :] = 1.0
    return F, D


def system_matrix(cv):
    """The full (N + M) x (N + M) matrix of eq. matrix_eqns."""
    n, m = cv.n, cv.m
    A = np.empty((n + m, n + m))
    blk = max(1, (1 << 24) // max(n, 1))
    for a in range(0, n, blk):
        rows = np.arange(a, min(n, a + blk))
        A[rows, :n] = kernel_block(cv, rows)
    A[np.arange(n), np.arange(n)] += 1.0
    A[:n, n:] = log_source_block(cv)
    F, D = constraint_blocks(cv)
    A[n:, :n] = F
    A[n:, n:] = D
    return A


def solve_dense(cv, g):
    """sigma, A from LU of the dense system with right-hand side [2g; 0]."""
    n = cv.n
    A = system_matrix(cv)
    rhs = np.concatenate([2.0 * np.asarray(g, float), np.zeros(cv.m)])
    sol = sla.lu_solve(sla.lu_factor(A, check_finite=False), rhs,
                       check_finite=False)
    return sol[:n], sol[n:]


def apply_iplusk(cv, sigma, rows=None, block_bytes=1 << 27):
    """((I + K) sigma)[rows] by the direct O(N) sum per row, in row blocks,
    never storing the matrix."""
    sigma = np.asarray(sigma, float)
    rows = np.arange(cv.n) if rows is None else np.asarray(rows)
    out = np.empty(rows.shape[0])
    blk = max(1, block_bytes // (32 * max(cv.n, 1)))
    for a in range(0, rows.shape[0], blk):
        r = rows[a:a + blk]
        out[a:a + blk] = kernel_block(cv, r) @ sigma + sigma[r]
    return out


def apply_system(cv, sigma, A):
    """[ (I+K) sigma + E A ; F sigma + D A ] by direct sums."""
    sigma = np.asarray(sigma, float)
    A = np.asarray(A, float)
    top = apply_iplusk(cv, sigma)
    blk = max(1, (1 << 24) // max(cv.m, 1))
    for a in range(0, cv.n, blk):
        r = np.arange(a, min(cv.n, a + blk))
        top[r] += log_source_block(cv, r) @ A
    bottom = np.zeros(cv.m)
    bottom[0] = A.sum()
    for k in range(1, cv.m):
        bottom[k] = sigma[cv.island == k].sum()
    return top, bottom


def sphere_kernel_block(cv, rows):
    """The same rows of K from the kernel's sphere form (Appendix A,
    eq. kern1): 2 h (1/2 pi) (x_j - x_i) . n_j / |x_i - x_j|^2 |x'_j|, with
    n_j the unit normal to the curve, tangent to the sphere, pointing into
    the island; the diagonal is its limit -(h / 2 pi) (x''_j . n_j) / |x'_j|.
    No stereographic quantity is used."""
    rows = np.asarray(rows)
    speed = np.linalg.norm(cv.xt, axis=1)
    nrm = np.cross(cv.x, cv.xt) / speed[:, None]
    # orient every normal towards its island's centre
    # the normal points into the island when it has a positive component
    # along the island centre (star-shaped curves about c)
    toward = np.einsum("ij,ij->i", nrm, cv.center[cv.island])
    isl_sg = np.array([np.sign(np.sum(np.sign(toward[cv.island == k])))
                       for k in range(cv.m)])
    nrm = nrm * isl_sg[cv.island][:, None]
    xi = cv.x[rows]
    dx = cv.x[None, :, :] - xi[:, None, :]
    d2 = (dx ** 2).sum(-1)
    same = rows[:, None] == np.arange(cv.n)[None, :]
    d2 = np.where(same, 1.0, d2)
    val = np.einsum("rjk,jk->rj", dx, nrm) / d2
    diag = -0.5 * np.einsum("jk,jk->j", cv.xtt, nrm) / speed ** 2
    val = np.where(same, diag[None, :], val)
    return val * (cv.h * speed / np.pi)[None, :]


def build(islands):
    return Curves(islands)
