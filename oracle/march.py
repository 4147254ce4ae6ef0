"""Plane-wave excitation and the MOT recursion (oracle; test infrastructure only).

Excitation (Eq. 7, Eq. 8): a modulated Gaussian plane wave
    E^i(r, t) = amp * e_hat * exp(-tau^2 / (2 sigma^2)) cos(2 pi f0 tau),
    tau = t - t0 - k_hat . (r - r_c) / c0,
with r_c the grid centre (reading: the paper does not fix the origin of r).
``amp`` carries the 1/(sigma sqrt(2 pi)) factor of Eq. 7 when a run follows the
paper's shape; it is 1 for a peak-normalized pulse.  The tested right-hand
side of Eq. 1 at voxel m and time t_n = n dt is (eps_r(m) - 1) d_t E^i(r_m, t_n)
(eps0 = c0 = h = 1), with r_m the voxel centre.

MOT recursion (Eq. 3, Eq. 6):
    Z0 J_n = E_n - sum_{k=1..ell} Z_k J_{n-k},   J_{n<0} = 0,
    Z_k    = T(k) diag(eps_r) - diag(eps_r - 1) G_k,
so with T(1) = 1/2 and T(k >= 2) = 0 the history term is
    sum_{k>=1} Z_k J_{n-k} = (eps_r/2) J_{n-1} - (eps_r - 1) sum_{k>=1} G_k * J_{n-k}.
With the regularization of ``operators`` the local weights become
(w0, w1, w2) = (1/2 + d_0, 1/2 + d_1, d_2): w0 on J_n in Z0, and w1, w2 on
J_{n-1}, J_{n-2} in the history term.
Each Z0 system is solved by ``krylov.tfqmr``; each Green convolution uses the
FFT form of Eq. 11 (``operators``), with the spectra of past currents kept so
that each current is transformed once.
"""

import math

import numpy as np
import scipy.fft as sfft

from .krylov import tfqmr
from .operators import PAIR, embed_spectra, reg_weights


def voxel_centres(nx, ny, nz):
    """Centres r_m - r_c in units of h, each of shape (nz, ny, nx)."""
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x + 0.5 - nx / 2.0, y + 0.5 - ny / 2.0, z + 0.5 - nz / 2.0


def dt_einc(pulse, eps, t):
    """(eps_r - 1) d_t E^i at every voxel centre, time t; shape (3, nz, ny, nx).

    ``pulse`` is a dict with keys e (3,), k (3,), f0, sigma, t0, amp.
    """
    nz, ny, nx = eps.shape
    x, y, z = voxel_centres(nx, ny, nz)
    kx, ky, kz = pulse["k"]
    tau = t - pulse["t0"] - (kx * x + ky * y + kz * z)
    s = pulse["sigma"]
    w = 2.0 * math.pi * pulse["f0"]
    env = np.exp(-tau * tau / (2.0 * s * s))
    dg = env * (-(tau / (s * s)) * np.cos(w * tau) - w * np.sin(w * tau))
    amp = pulse.get("amp", 1.0)
    return np.stack([(eps - 1.0) * amp * pulse["e"][p] * dg for p in range(3)])


class Mot:
    """Plain FP64 MOT-JVIE march for one scatterer.

    ``greens`` is the list [G_0, ..., G_ell] of octant tables (``green``).
    """

    def __init__(self, eps, greens, cdt, delta=0.0):
        self.eps = np.asarray(eps, dtype=np.float64)
        self.w = reg_weights(delta)
        self.nz, self.ny, self.nx = self.eps.shape
        self.cdt = float(cdt)
        self.nl = len(greens) - 1
        self.lams = [embed_spectra(g)[0] for g in greens]
        self.P = self.lams[0].shape[1:]
        self.hist = []          # spectra of J_{n-1}, J_{n-2}, ... (newest first)
        self.jprev = np.zeros((3, self.nz, self.ny, self.nx))
        self.jprev2 = np.zeros((3, self.nz, self.ny, self.nx))
        self.n = 0

    def _spec(self, J):
        return np.stack([sfft.fftn(J[q], s=self.P, axes=(0, 1, 2)) for q in range(3)])

    def _apply_spec(self, lam, Jh):
        out = np.zeros((3,) + self.P, dtype=np.complex128)
        for p in range(3):
            for q in range(3):
                out[p] += lam[PAIR.index((min(p, q), max(p, q)))] * Jh[q]
        return out

    def _back(self, S):
        return np.stack([sfft.ifftn(S[p]).real[:self.nz, :self.ny, :self.nx] for p in range(3)])

    def z0(self, J):
        """Z0 J (Eq. 12)."""
        gj = self._back(self._apply_spec(self.lams[0], self._spec(J)))
        return self.w[0] * self.eps[None] * J - (self.eps[None] - 1.0) * gj

    def history_rhs(self):
        """-sum_{k>=1} Z_k J_{n-k} for the current n."""
        S = np.zeros((3,) + self.P, dtype=np.complex128)
        for k in range(1, self.nl + 1):
            if k - 1 < len(self.hist):
                S += self._apply_spec(self.lams[k], self.hist[k - 1])
        h = self._back(S)
        return (-self.eps[None] * (self.w[1] * self.jprev + self.w[2] * self.jprev2)
                + (self.eps[None] - 1.0) * h)

    def step(self, einc, tol=1e-6, max_iter=1000):
        """One MOT step: returns (J_n, TfqmrResult)."""
        b = einc + self.history_rhs()
        shape = b.shape
        res = tfqmr(lambda v: self.z0(v.reshape(shape)).ravel(), b.ravel(), tol=tol,
                    max_iter=max_iter)
        J = res.x.reshape(shape)
        self.hist.insert(0, self._spec(J))
        del self.hist[self.nl:]
        self.jprev2 = self.jprev
        self.jprev = J
        self.n += 1
        return J, res


def run(eps, greens, cdt, pulse, nsteps, tol=1e-6, max_iter=1000, probe=None, delta=0.0):
    """March ``nsteps`` steps; returns (J history or probe trace, iteration counts)."""
    mot = Mot(eps, greens, cdt, delta=delta)
    out, iters = [], []
    for n in range(nsteps):
        J, res = mot.step(dt_einc(pulse, mot.eps, n * cdt), tol=tol, max_iter=max_iter)
        out.append(J if probe is None else J[probe])
        iters.append(res.iterations)
    return np.array(out), iters
