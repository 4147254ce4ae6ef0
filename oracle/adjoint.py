"""Adjoint MOT march and the gradient of a far-field energy with respect to
the permittivity (oracle; test infrastructure only).

Transposed operators.  Every G_k is a symmetric matrix: G_k(-d) = G_k(d) and
each 3x3 block is symmetric (the symmetries of the Green dyad, Sec. III), so
the transpose of Z_k = T(k) diag(eps_r) - diag(eps_r - 1) G_k (Eq. 10 form) is
    Z_k^T = T(k) diag(eps_r) - G_k diag(eps_r - 1):
the contrast acts on the input.  In particular
    Z0^T v = (eps_r/2) v - G_0 ((eps_r - 1) v).
With the regularization of ``operators`` the local weights of Z0, Z1, Z2
become (w0, w1, w2) = (1/2 + d_0, 1/2 + d_1, d_2) (diagonal, so the transpose
keeps them).

Far field (reading; the paper does not use one).  The current radiates
through the retarded vector potential of Eq. 1; far from the scatterer, with
the common factor 1/(4 pi R) and the delay R dropped (c0 = mu0 = h = 1),
    e(tau) = -(1/(4 pi)) P d/dtau sum_m J(r_m, tau + rhat . r_m),
P = I - rhat rhat^T the projection transverse to rhat, r_m the voxel centre
relative to the grid centre.  With the basis current of Sec. II,
J(r_m, t) = sum_n J_{m,n} T(t/dt - n), sampled at tau_j = j dt:
    e_j = -(1/(4 pi dt)) P sum_m sum_n J_{m,n} T'(j - n + s_m),   s_m = rhat . r_m / dt,
with T' the derivative of the spline in step units.  The energy is
W = dt sum_j |e_j|^2.

Adjoint march.  The march (Eq. 3) is the block lower-triangular Toeplitz
system sum_{k=0..ell} Z_k J_{n-k} = E_n, n = 0..Nt-1.  Its transpose,
sum_k Z_k^T lam_{n+k} = g_n with g_n = dW/dJ_n, is solved backwards in time
from n = Nt-1 (lam_{n >= Nt} = 0):
    Z0^T lam_n = g_n - (eps_r/2) lam_{n+1} + sum_{k>=1} G_k ((eps_r - 1) lam_{n+k}).
(with the regularization: w0 eps_r in Z0^T, w1 eps_r on lam_{n+1}, w2 eps_r on lam_{n+2}).

Gradient.  E_n = (eps_r - 1) d_t E^i(r_m, t_n) and the Z_k depend on eps_r, so
    dW/d eps_m = sum_n lam_n(m) . [d_t E^i(r_m, t_n) - (J_n(m) + J_{n-1}(m))/2 + u_n(m)],
(with the regularization: -w0 J_n(m) - w1 J_{n-1}(m) - w2 J_{n-2}(m) in the bracket),
    u_n = sum_{k=0..ell} G_k J_{n-k}.

Pins (tests/test_oracle_adjoint.py): the transpose against the dense Z0 and
the dot-product identity; the far field of a single voxel in closed form and
its adjoint by the dot-product identity; the adjoint march against a dense
solve of the transposed space-time system; the gradient against central
finite differences of the forward march and energy.
"""

import math

import numpy as np

from .krylov import tfqmr
from .march import Mot, dt_einc, voxel_centres
from .operators import gconv_fft, reg_weights


def z0t_apply(g0_oct, eps, v, lam=None, delta=0.0):
    """Z0^T v = w0 eps_r v - G_0 ((eps_r - 1) v); v shape (3, nz, ny, nx)."""
    return reg_weights(delta)[0] * eps[None] * v - gconv_fft(g0_oct, (eps[None] - 1.0) * v, lam=lam)


def dspline(s):
    """dT/ds of the spline of ``basis`` (step units): s+1, 1-2s, s-2 on
    [-1,0), [0,1), [1,2); 0 elsewhere."""
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros_like(s)
    m0 = (s >= -1.0) & (s < 0.0)
    m1 = (s >= 0.0) & (s < 1.0)
    m2 = (s >= 1.0) & (s < 2.0)
    out[m0] = s[m0] + 1.0
    out[m1] = 1.0 - 2.0 * s[m1]
    out[m2] = s[m2] - 2.0
    return out


def _shift(shape, rhat, dt):
    nz, ny, nx = shape
    x, y, z = voxel_centres(nx, ny, nz)
    return (rhat[0] * x + rhat[1] * y + rhat[2] * z) / dt


def _proj(rhat):
    r = np.asarray(rhat, dtype=np.float64)
    return np.eye(3) - np.outer(r, r)


def farfield(Jhist, rhat, dt, j0, nj):
    """e_j for j = j0..j0+nj-1 from the currents J_n, Jhist (Nt, 3, nz, ny, nx);
    returns (nj, 3)."""
    Jhist = np.asarray(Jhist, dtype=np.float64)
    s = _shift(Jhist.shape[2:], rhat, dt)
    P = _proj(rhat)
    e = np.zeros((nj, 3))
    for n in range(Jhist.shape[0]):
        for j in range(j0, j0 + nj):
            w = dspline(j - n + s)
            if not w.any():
                continue
            a = np.array([np.sum(Jhist[n, p] * w) for p in range(3)])
            e[j - j0] += -(1.0 / (4.0 * math.pi * dt)) * (P @ a)
    return e


def farfield_adjoint(w, rhat, dt, j0, nsteps, shape):
    """Transpose of ``farfield``: g_n(p, m) = d/dJ_{m,n,p} sum_j w_j . e_j;
    w (nj, 3); returns (nsteps, 3, nz, ny, nx)."""
    w = np.asarray(w, dtype=np.float64)
    s = _shift(shape, rhat, dt)
    P = _proj(rhat)
    g = np.zeros((nsteps, 3) + tuple(shape))
    for n in range(nsteps):
        for jj in range(w.shape[0]):
            t = dspline(j0 + jj - n + s)
            if not t.any():
                continue
            pw = P @ w[jj]
            for p in range(3):
                g[n, p] += -(1.0 / (4.0 * math.pi * dt)) * pw[p] * t
    return g


def energy(e, dt):
    """W = dt sum_j |e_j|^2."""
    return float(dt * np.sum(np.asarray(e) ** 2))


def gfield(greens, Jhist, n):
    """u_n = sum_{k=0..ell} G_k J_{n-k} (J_{<0} = 0)."""
    u = np.zeros(Jhist.shape[1:])
    for k in range(min(n, len(greens) - 1) + 1):
        u += gconv_fft(greens[k], Jhist[n - k])
    return u


def forward(eps, greens, dt, pulse, nsteps, tol=1e-12, max_iter=1000, delta=0.0):
    """The MOT march of ``march.Mot``; returns Jhist (nsteps, 3, nz, ny, nx)."""
    mot = Mot(eps, greens, dt, delta=delta)
    out = []
    for n in range(nsteps):
        J, _ = mot.step(dt_einc(pulse, mot.eps, n * dt), tol=tol, max_iter=max_iter)
        out.append(J)
    return np.array(out)


def adjoint_march(eps, greens, g, tol=1e-12, max_iter=1000, delta=0.0):
    """lam_n for n = Nt-1 .. 0 from the sources g (Nt, 3, nz, ny, nx)."""
    eps = np.asarray(eps, dtype=np.float64)
    nt = g.shape[0]
    nl = len(greens) - 1
    lam = np.zeros_like(g)
    shape = g.shape[1:]
    for n in range(nt - 1, -1, -1):
        rhs = g[n].copy()
        if n + 1 < nt:
            rhs -= reg_weights(delta)[1] * eps[None] * lam[n + 1]
        if n + 2 < nt:
            rhs -= reg_weights(delta)[2] * eps[None] * lam[n + 2]
        for k in range(1, nl + 1):
            if n + k < nt:
                rhs += gconv_fft(greens[k], (eps[None] - 1.0) * lam[n + k])
        res = tfqmr(lambda v: z0t_apply(greens[0], eps, v.reshape(shape), delta=delta).ravel(), rhs.ravel(), tol=tol,
                    max_iter=max_iter)
        lam[n] = res.x.reshape(shape)
    return lam


def incident_dt(pulse, shape, t):
    """d_t E^i at every voxel centre (the excitation without the contrast)."""
    return dt_einc(pulse, np.full(shape, 2.0), t)


def energy_of(eps, greens, dt, pulse, nsteps, rhat, j0, nj, tol=1e-12, delta=0.0):
    """W for permittivity eps (forward march, far field, energy)."""
    J = forward(eps, greens, dt, pulse, nsteps, tol=tol, delta=delta)
    return energy(farfield(J, rhat, dt, j0, nj), dt)


def gradient(eps, greens, dt, pulse, nsteps, rhat, j0, nj, tol=1e-12, delta=0.0):
    """(W, dW/d eps) by the adjoint march; dW/d eps has the shape of eps."""
    eps = np.asarray(eps, dtype=np.float64)
    J = forward(eps, greens, dt, pulse, nsteps, tol=tol, delta=delta)
    e = farfield(J, rhat, dt, j0, nj)
    W = energy(e, dt)
    g = farfield_adjoint(2.0 * dt * e, rhat, dt, j0, nsteps, eps.shape)
    lam = adjoint_march(eps, greens, g, tol=tol, delta=delta)
    grad = np.zeros(eps.shape)
    for n in range(nsteps):
        q = incident_dt(pulse, eps.shape, n * dt) + gfield(greens, J, n)
        w = reg_weights(delta)
        q -= w[0] * J[n]
        if n > 0:
            q -= w[1] * J[n - 1]
        if n > 1:
            q -= w[2] * J[n - 2]
        grad += np.sum(lam[n] * q, axis=0)
    return W, grad
