"""Transpose-free QMR (oracle; test infrastructure only).

The paper solves the Z0 system of every time step with Freund's TFQMR
(Sec. II, solver paragraph) to a relative tolerance of 1e-6 (Sec. V-A).
Readings where the paper is silent: start from x0 = 0, shadow vector
r~ = r0, stop when the quasi-residual bound tau*sqrt(m+1) is below
tol*||b|| AND the true residual ||b - A x|| is below tol*||b||; b = 0 gives
x = 0 after zero iterations.  Real arithmetic.

Freund's recurrences, one half step per index m (two half steps and two
products with A make one iteration):

    alpha = rho / (v . r~)                          (m even)
    u_next = u - alpha v                            (m even)
    w   <- w - alpha A u
    d   <- u + (theta^2 eta / alpha) d
    theta = ||w|| / tau,  c = 1/sqrt(1+theta^2),  tau <- tau theta c,
    eta = c^2 alpha,       x <- x + eta d
    rho' = w . r~,  beta = rho'/rho,                (m odd)
    u <- w + beta u,  v <- A u + beta (A u_prev + beta v)
"""

import numpy as np


class TfqmrResult:
    __slots__ = ("x", "iterations", "matvecs", "relres", "converged", "breakdown")

    def __init__(self, x, iterations, matvecs, relres, converged, breakdown=False):
        self.x = x
        self.iterations = iterations
        self.matvecs = matvecs
        self.relres = relres
        self.converged = converged
        self.breakdown = breakdown


def tfqmr(apply_a, b, tol=1e-6, max_iter=1000):
    """Solve A x = b; ``apply_a`` maps an FP64 array to an FP64 array."""
    b = np.asarray(b, dtype=np.float64)
    bnorm = float(np.linalg.norm(b))
    x = np.zeros_like(b)
    if bnorm == 0.0:
        return TfqmrResult(x, 0, 0, 0.0, True)
    r0 = b.copy()
    rt = r0.copy()
    w = r0.copy()
    u = r0.copy()
    au = apply_a(u)
    nmv = 1
    v = au.copy()
    d = np.zeros_like(b)
    tau = bnorm
    theta = 0.0
    eta = 0.0
    rho = float(np.vdot(rt, r0))
    it = 0
    while it < max_iter:
        it += 1
        sigma = float(np.vdot(v, rt))
        if sigma == 0.0 or rho == 0.0:
            res = float(np.linalg.norm(b - apply_a(x))) / bnorm
            return TfqmrResult(x, it, nmv + 1, res, res <= tol, True)
        alpha = rho / sigma
        u_next = u - alpha * v
        for half in range(2):
            m = 2 * (it - 1) + half
            uu, auu = (u, au) if half == 0 else (u_next, None)
            if half == 1:
                auu = apply_a(u_next)
                nmv += 1
                au_next = auu
            w = w - alpha * auu
            d = uu + (theta * theta * eta / alpha) * d
            theta = float(np.linalg.norm(w)) / tau
            c = 1.0 / np.sqrt(1.0 + theta * theta)
            tau = tau * theta * c
            eta = c * c * alpha
            x = x + eta * d
            if tau * np.sqrt(m + 2.0) <= tol * bnorm:
                res = float(np.linalg.norm(b - apply_a(x))) / bnorm
                nmv += 1
                if res <= tol:
                    return TfqmrResult(x, it, nmv, res, True)
        rho_new = float(np.vdot(w, rt))
        beta = rho_new / rho
        rho = rho_new
        u = w + beta * u_next
        au_new = apply_a(u)
        nmv += 1
        v = au_new + beta * (au_next + beta * v)
        au = au_new
    res = float(np.linalg.norm(b - apply_a(x))) / bnorm
    return TfqmrResult(x, it, nmv + 1, res, res <= tol)
