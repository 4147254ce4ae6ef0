"""Z0 = D - X G and the Green convolution (oracle; test infrastructure only).

Eq. 10: Z0 = D - X G with D = diag(eps_r) T(0) = diag(eps_r)/2 and
X = diag(eps_r - 1) (reading of Eq. 1: the constitutive term eps_r J is
tested at t_n, where the spline basis gives J(t_n) = (J_n + J_{n-1})/2).

Regularization (Sec. II, the delta-notation Z^delta_n = Z_n + delta_n I of
the regularized MOT formulation the paper cites; the paper itself runs with
delta_n = 0).  Reading used here: delta_n = d_n diag(eps_r) for n = 0, 1, 2
(zero beyond), i.e. the constitutive term eps_r J is tested with the local
weights (1/2 + d_0, 1/2 + d_1, d_2) on (J_n, J_{n-1}, J_{n-2}) instead of the
spline's (1/2, 1/2, 0).  ``delta`` is either the triple (d_0, d_1, d_2) or a
number d for the first difference (d, -d, 0).  delta = 0 (the default
everywhere) is the paper's unregularized operator; D = diag(eps_r)(1/2 + d_0).

Three forms of the same product, all FP64:

* ``z0_dense``     -- the 3N x 3N matrix assembled entry by entry (tiny grids);
* ``gconv_direct`` -- the Toeplitz sum (G J)_p(m) = sum_m' sum_q G(m-m')[p,q] J_q(m');
* ``gconv_fft``    -- Eq. 11: zero-pad each component to the doubled grid,
                      3-D FFT, multiply by the spectra Lambda_pq of the
                      circulant embedding of G, inverse FFT, truncate.

Vectors are laid out [3][nz][ny][nx] (component, then z, y, x; x fastest).
"""

import numpy as np
import scipy.fft as sfft

from .green import PAIR, green_full


def reg_weights(delta):
    """Local weights (w0, w1, w2) of eps_r on (J_n, J_{n-1}, J_{n-2}) for a
    regularization ``delta`` (a number d: (d, -d, 0); or (d_0, d_1, d_2))."""
    if np.ndim(delta) == 0:
        d = (float(delta), -float(delta), 0.0)
    else:
        d = tuple(float(v) for v in delta)
        if len(d) != 3:
            raise ValueError("delta: a number or (d_0, d_1, d_2)")
    return 0.5 + d[0], 0.5 + d[1], d[2]


def z0_dense(g0_oct, eps, delta=0.0):
    """Dense Z0 for a grid with eps of shape (nz, ny, nx); row/col = p*N + m."""
    nz, ny, nx = eps.shape
    N = eps.size
    full = green_full(g0_oct)
    Z = np.zeros((3 * N, 3 * N))
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    zz, yy, xx = zz.ravel(), yy.ravel(), xx.ravel()
    e = eps.ravel()
    for m in range(N):
        dz = zz[m] - zz + nz - 1
        dy = yy[m] - yy + ny - 1
        dx = xx[m] - xx + nx - 1
        for p in range(3):
            for q in range(3):
                Z[p * N + m, q * N:(q + 1) * N] = -(e[m] - 1.0) * full[p, q, dz, dy, dx]
            Z[p * N + m, p * N + m] += e[m] * reg_weights(delta)[0]
    return Z


def gconv_direct(g_oct, J):
    """(G J) by direct summation over all offsets; J shape (3, nz, ny, nx)."""
    _, nz, ny, nx = J.shape
    full = green_full(g_oct)
    out = np.zeros_like(J, dtype=np.float64)
    for dz in range(-(nz - 1), nz):
        for dy in range(-(ny - 1), ny):
            for dx in range(-(nx - 1), nx):
                blk = full[:, :, dz + nz - 1, dy + ny - 1, dx + nx - 1]
                if not blk.any():
                    continue
                # out[m] += G(d) J[m - d]
                oz = slice(max(dz, 0), nz + min(dz, 0))
                oy = slice(max(dy, 0), ny + min(dy, 0))
                ox = slice(max(dx, 0), nx + min(dx, 0))
                iz = slice(max(-dz, 0), nz + min(-dz, 0))
                iy = slice(max(-dy, 0), ny + min(-dy, 0))
                ix = slice(max(-dx, 0), nx + min(-dx, 0))
                src = J[:, iz, iy, ix]
                for p in range(3):
                    out[p, oz, oy, ox] += np.tensordot(blk[p], src, axes=(0, 0))
    return out


def embed_spectra(g_oct):
    """Spectra Lambda of the circulant embedding of G on P = 2N per axis.

    Offset d (|d_i| <= N_i - 1) goes to index d mod P_i; index N_i (no
    offset) stays zero.  Returns (6, Pz, Py, Px) real FP64 (component order
    xx, yy, zz, xy, xz, yz) and the largest |imaginary part| found, which is
    a rounding-level number because each component is even or odd-odd along
    every axis.
    """
    _, nz, ny, nx = g_oct.shape
    full = green_full(g_oct)
    P = (2 * nz, 2 * ny, 2 * nx)
    lam = np.zeros((6,) + P)
    imag = 0.0
    iz = np.arange(-(nz - 1), nz) % P[0]
    iy = np.arange(-(ny - 1), ny) % P[1]
    ix = np.arange(-(nx - 1), nx) % P[2]
    for c, (p, q) in enumerate(PAIR):
        e = np.zeros(P)
        e[np.ix_(iz, iy, ix)] = full[p, q]
        f = sfft.fftn(e)
        imag = max(imag, float(np.abs(f.imag).max()))
        lam[c] = f.real
    return lam, imag


def gconv_fft(g_oct, J, lam=None):
    """(G J) via Eq. 11 on the doubled grid; J shape (3, nz, ny, nx)."""
    _, nz, ny, nx = J.shape
    if lam is None:
        lam, _ = embed_spectra(g_oct)
    P = lam.shape[1:]
    Jh = [sfft.fftn(J[q], s=P, axes=(0, 1, 2)) for q in range(3)]
    out = np.zeros(J.shape)
    for p in range(3):
        acc = np.zeros(P, dtype=np.complex128)
        for q in range(3):
            c = PAIR.index((min(p, q), max(p, q)))
            acc += lam[c] * Jh[q]
        out[p] = sfft.ifftn(acc).real[:nz, :ny, :nx]
    return out


def z0_apply(g0_oct, eps, J, method="fft", lam=None, delta=0.0):
    """Z0 J = D J - X (G J), Eq. 12 (D = diag(eps_r)(1/2 + d_0))."""
    if method == "fft":
        gj = gconv_fft(g0_oct, J, lam=lam)
    elif method == "direct":
        gj = gconv_direct(g0_oct, J)
    else:
        raise ValueError(method)
    return reg_weights(delta)[0] * eps[None] * J - (eps[None] - 1.0) * gj
