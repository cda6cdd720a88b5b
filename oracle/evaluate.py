"""The solution at sphere targets (Section 4.1, eq. eqn:u_multi).

psi(x) = (W sigma)(x) + sum_m A_m G(x, c_m), where the double layer is
discretized by the same trapezoidal rule as the equation:
    (W sigma)(x) = sum_j h_m (s_m / 2 pi)
                   Im[ xi'_j / (xi(x) - xi_j) + conj(xi_j) xi'_j / (1 + |xi_j|^2) ] sigma_j.
At the north pole xi(x) is infinite and the Cauchy term vanishes.
"""
import numpy as np

from .nystrom import greens


def evaluate(cv, sigma, A, targets, block_bytes=1 << 27):
    targets = np.asarray(targets, float)
    sigma = np.asarray(sigma, float)
    A = np.asarray(A, float)
    den = 1.0 - targets[:, 2]
    at_pole = den <= 0.0
    xi_t = np.where(at_pole, 0.0,
                    (targets[:, 0] + 1j * targets[:, 1]) /
                    np.where(at_pole, 1.0, den))
    w = cv.s * cv.h / (2 * np.pi) * sigma
    corr = np.sum(w * np.imag(np.conj(cv.xi) * cv.dxi /
                              (1 + np.abs(cv.xi) ** 2)))
    out = np.empty(targets.shape[0])
    blk = max(1, block_bytes // (32 * max(cv.n, 1)))
    for a in range(0, targets.shape[0], blk):
        xt = xi_t[a:a + blk]
        c = np.imag(cv.dxi[None, :] / (xt[:, None] - cv.xi[None, :])) @ w
        c = np.where(at_pole[a:a + blk], 0.0, c)
        out[a:a + blk] = c + corr + greens(targets[a:a + blk], cv.center) @ A
    return out
