"""GMRES(m) on the left-preconditioned system (Section 5, eq. matrix_eqns_c).

The preconditioner is P = [[I, E], [F, D]].  Solving P z = r uses the Schur
complement S = D - F E (factored once by Gaussian elimination):
    S z_a = r_a - F r_sigma,   z_sigma = r_sigma - E z_a.
Since the system matrix is P + diag(K, 0), the preconditioned operator is
x -> x + P^{-1} [K sigma; 0].  GMRES starts from x0 = 0 and stops when the
residual of the preconditioned system, as tracked by the Givens rotations,
falls below tol times the norm of the preconditioned right-hand side.
"""
import numpy as np
import scipy.linalg as sla

from . import nystrom


class Preconditioner:
    def __init__(self, cv):
        self.cv = cv
        self.E = nystrom.log_source_block(cv)
        F, D = nystrom.constraint_blocks(cv)
        self.F, self.D = F, D
        self.S = D - F @ self.E
        self.lu = sla.lu_factor(self.S, check_finite=False)

    def solve(self, r_sigma, r_a):
        z_a = sla.lu_solve(self.lu, r_a - self.F @ r_sigma,
                           check_finite=False)
        return r_sigma - self.E @ z_a, z_a


def gmres(apply_op, b, tol, restart=50, max_iter=1000):
    """Plain restarted GMRES with modified Gram-Schmidt and Givens rotations.
    Returns (x, iterations, residual history relative to |b|)."""
    n = b.shape[0]
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    hist = []
    if bnorm == 0:
        return x, 0, hist
    it = 0
    r = b.copy()
    while it < max_iter:
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol:
            break
        V = np.zeros((restart + 1, n))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        gvec = np.zeros(restart + 1)
        gvec[0] = beta
        V[0] = r / beta
        k_used = 0
        for k in range(restart):
            w = apply_op(V[k])
            for j in range(k + 1):
                H[j, k] = np.dot(V[j], w)
                w = w - H[j, k] * V[j]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] > 0:
                V[k + 1] = w / H[k + 1, k]
            for j in range(k):
                t = cs[j] * H[j, k] + sn[j] * H[j + 1, k]
                H[j + 1, k] = -sn[j] * H[j, k] + cs[j] * H[j + 1, k]
                H[j, k] = t
            den = np.hypot(H[k, k], H[k + 1, k])
            cs[k] = H[k, k] / den
            sn[k] = H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            gvec[k + 1] = -sn[k] * gvec[k]
            gvec[k] = cs[k] * gvec[k]
            it += 1
            k_used = k + 1
            hist.append(abs(gvec[k + 1]) / bnorm)
            if hist[-1] <= tol or it >= max_iter:
                break
        y = sla.solve_triangular(H[:k_used, :k_used], gvec[:k_used])
        x = x + V[:k_used].T @ y
        if hist and hist[-1] <= tol:
            break
        r = b - apply_op(x)
    return x, it, hist


def solve_preconditioned(cv, g, tol=1e-12, restart=50, max_iter=1000,
                         precondition=True):
    """sigma, A, iterations, history for data g.  The matvec is the direct
    O(N^2) sum (nystrom.apply_iplusk), so this suits mid-size problems."""
    n, m = cv.n, cv.m
    b_sigma = 2.0 * np.asarray(g, float)
    b_a = np.zeros(m)
    if precondition:
        P = Preconditioner(cv)

        def op(v):
            ks = nystrom.apply_iplusk(cv, v[:n]) - v[:n]
            zs, za = P.solve(ks, np.zeros(m))
            return v + np.concatenate([zs, za])

        bs, ba = P.solve(b_sigma, b_a)
        b = np.concatenate([bs, ba])
    else:
        def op(v):
            top, bottom = nystrom.apply_system(cv, v[:n], v[n:])
            return np.concatenate([top, bottom])

        b = np.concatenate([b_sigma, b_a])
    x, it, hist = gmres(op, b, tol, restart, max_iter)
    return x[:n], x[n:], it, hist
