"""Green dyad G_k(d) of the discretized TDJVIE (oracle; test infrastructure only).

Definition.  Eq. 1 with ``nabla x nabla x = nabla nabla . - nabla^2`` and the
wave equation of the retarded potential gives, for the observation point at
the origin (centre-point testing of the piecewise-constant basis, Sec. II),
Dirac temporal testing at t_n = n dt and the spline basis T of ``basis``:

    Pi_k(d)      = int_{B(d)} T(k - R/L) / (4 pi R) dV',   R = |r'|,
    G_k(d)[p,q]  = d_p d_q Pi_k  -  delta_pq d_t^2 Pi_k  +  delta_pq T(k) [d = 0],

where d_p are derivatives in the observation coordinate and d_t^2 Pi_k is the
same box integral with T replaced by its second time derivative.  The last
term is the -nabla^2 source term of the curl-curl operator at the observation
point; it is present only for the self box.  B(d) = prod_i [d_i-1/2, d_i+1/2].
Units c0 = h = 1, L = c0 dt / h.

The interaction matrices of Eq. 3 are then
    Z_k = T(k) diag(eps_r) (x) I_3  -  diag(eps_r - 1) G_k,
i.e. Z0 = D - X G of Eq. 10 with D = diag(eps_r)/2, X = diag(eps_r - 1).

Evaluation (divergence theorem, exact identities):

  * off-diagonal  A_pq = sum_{sp,sq=+-1} sp sq int f(R) dx_r  along the four
    box edges parallel to the third axis r, with f(R) = T(k - R/L)/(4 pi R);
    on every piece of T the integral is elementary.
  * diagonal      A_pp = sum_{s=+-1} s a_s iint_{x_p = a_s} f'(R)/R du dv.
  * time term     B = -sum_faces (n . x') iint H(R)/R^3 dS',
                  H(R) = (1/(4 pi L^2)) int_0^R T''(k - r/L) r dr.
  * G_pp = A_pp + B + T(k)[d=0],  G_pq = A_pq (p != q).

Face integrals are iterated: the inner integral (along v) is taken exactly
on every piece between the knot spheres R = (k-2)L ... (k+1)L; the outer one
(along u) by Gauss-Legendre on the sub-intervals between the points where a
knot circle is tangent to the line u = const or passes through a face corner,
after the smoothing substitution u = ua + (ub-ua) t^2 (3-2t), which turns the
square-root behaviour at tangency points into a smooth one.

Component order everywhere: (xx, yy, zz, xy, xz, yz).
"""

import math

import numpy as np

from .basis import SPLINE_PIECES, spline
from .masks import mask

COMPONENTS = ("xx", "yy", "zz", "xy", "xz", "yz")
PAIR = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
FOUR_PI = 4.0 * math.pi

_A = np.array(SPLINE_PIECES)  # (3, 3): piece j -> (a0, a1, a2)


def _knots(k, L):
    """Knot radii (k-2)L, (k-1)L, kL, (k+1)L; non-positive ones -> NaN."""
    kk = np.asarray(k, dtype=np.float64)[..., None]
    r = (kk + np.array([-2.0, -1.0, 0.0, 1.0])) * L
    return np.where(r > 0, r, np.nan)


def _piece(R, k, L):
    """Spline piece j (0,1,2) holding s = k - R/L, or -1 outside [-1, 2)."""
    s = k - R / L
    j = np.floor(s).astype(np.int64) + 1
    return np.where((s >= -1) & (s < 2), j, -1)


def _poly_in_R(j, k, L):
    """T(k - R/L) = b0 + b1 R + b2 R^2 on piece j (zeros where j = -1)."""
    jj = np.where(j >= 0, j, 0)
    a0, a1, a2 = _A[jj, 0], _A[jj, 1], _A[jj, 2]
    b0 = a0 + a1 * k + a2 * k * k
    b1 = -(a1 + 2.0 * a2 * k) / L
    b2 = a2 / (L * L)
    z = j < 0
    return np.where(z, 0.0, b0), np.where(z, 0.0, b1), np.where(z, 0.0, b2)


def _h_coeffs(R, k, L):
    """H(R)/R^3 = c1/R + c3/R^3 at R (coefficients constant on each piece)."""
    j = _piece(R, k, L)
    jj = np.where(j >= 0, j, 0)
    c_here = np.where(j >= 0, 2.0 * _A[jj, 2], 0.0)
    q = np.zeros_like(R)
    for jp in range(3):
        lo = np.maximum((k - jp) * L, 0.0)
        hi = np.maximum((k - jp + 1) * L, 0.0)
        rc = np.clip(R, lo, hi)
        q = q + 2.0 * _A[jp, 2] * (rc * rc - lo * lo) / 2.0
    scale = 1.0 / (FOUR_PI * L * L)
    return c_here / 2.0 * scale, (q - c_here * R * R / 2.0) * scale


def _a_coeffs(R, k, L):
    """f'(R)/R = c1/R + c3/R^3 with f = T(k-R/L)/(4 pi R)."""
    b0, _, b2 = _poly_in_R(_piece(R, k, L), k, L)
    return b2 / FOUR_PI, -b0 / FOUR_PI


def _inner(kind, a, u, v0, v1, k, L):
    """Exact int_{v0}^{v1} (c1/R + c3/R^3) dv, R^2 = a^2+u^2+v^2, piecewise."""
    rho2 = a * a + u * u
    kn = _knots(k, L)                               # (..., 4)
    d2 = kn * kn - rho2[..., None]
    s = np.sqrt(np.where(d2 > 0, d2, np.nan))
    sp = np.concatenate([s, -s], axis=-1)
    sp = np.where(np.isnan(sp), v0[..., None], sp)
    sp = np.clip(sp, v0[..., None], v1[..., None])
    V = np.sort(np.concatenate([v0[..., None], sp, v1[..., None]], axis=-1), axis=-1)
    va, vb = V[..., :-1], V[..., 1:]
    rm = np.sqrt(rho2[..., None] + (0.5 * (va + vb)) ** 2)
    kb = np.broadcast_to(np.asarray(k, dtype=np.float64)[..., None], rm.shape)
    c1, c3 = (_a_coeffs if kind == "A" else _h_coeffs)(rm, kb, L)
    rho = np.sqrt(rho2)[..., None]
    r2 = rho2[..., None]

    def prim(v):
        return c1 * np.arcsinh(v / rho) + c3 * v / (r2 * np.sqrt(r2 + v * v))

    return (prim(vb) - prim(va)).sum(axis=-1)


def _face_integral(kind, a, u0, u1, v0, v1, k, L, nq=16, chunk=4096):
    """iint_{[u0,u1]x[v0,v1]} (c1/R + c3/R^3) du dv on the plane x_p = a."""
    a, u0, u1, v0, v1 = (np.asarray(x, dtype=np.float64) for x in (a, u0, u1, v0, v1))
    k = np.asarray(k, dtype=np.float64)
    x, w = np.polynomial.legendre.leggauss(nq)
    t = 0.5 * (x + 1.0)[None, :]
    w = 0.5 * w[None, :]
    out = np.zeros(a.shape[0])
    for c0 in range(0, a.shape[0], chunk):
        sl = slice(c0, c0 + chunk)
        A_, U0, U1, V0, V1, K = a[sl], u0[sl], u1[sl], v0[sl], v1[sl], k[sl]
        kn = _knots(K, L)
        cands, kinds = [], []
        # tangency of a knot circle with u = const (kind 1: square-root end),
        # knot circle through a face corner (kind 0: kink only)
        for kind_, ve in ((1, np.zeros_like(V0)), (0, V0), (0, V1)):
            d2 = kn * kn - (A_ * A_ + ve * ve)[:, None]
            s = np.sqrt(np.where(d2 > 0, d2, np.nan))
            cands += [s, -s]
            kinds += [np.full(s.shape, kind_)] * 2
        C = np.concatenate(cands + [np.zeros_like(U0)[:, None]], axis=1)
        T = np.concatenate(kinds + [np.zeros((C.shape[0], 1), dtype=np.int64)], axis=1)
        inside = (C > U0[:, None]) & (C < U1[:, None])
        C = np.where(inside, C, U0[:, None])
        T = np.where(inside, T, 0)
        P = np.concatenate([U0[:, None], C, U1[:, None]], axis=1)
        T = np.concatenate([np.zeros_like(T[:, :1]), T, np.zeros_like(T[:, :1])], axis=1)
        order = np.argsort(P, axis=1, kind="stable")
        P = np.take_along_axis(P, order, axis=1)
        T = np.take_along_axis(T, order, axis=1)
        ua, ub = P[:, :-1], P[:, 1:]
        ta, tb = T[:, :-1], T[:, 1:]
        keep = ub > ua
        fid = np.nonzero(keep)[0]
        ua, ub, ta, tb = ua[keep], ub[keep], ta[keep][:, None], tb[keep][:, None]
        h = (ub - ua)[:, None]
        # substitution per end: t^2 (3-2t) both ends, t^2 left, 1-(1-t)^2 right
        both = (ta == 1) & (tb == 1)
        left = (ta == 1) & (tb == 0)
        right = (ta == 0) & (tb == 1)
        phi = np.where(both, t * t * (3 - 2 * t), np.where(left, t * t, np.where(right, 1 - (1 - t) ** 2, t)))
        dphi = np.where(both, 6 * t * (1 - t), np.where(left, 2 * t, np.where(right, 2 * (1 - t), 1.0)))
        U = ua[:, None] + h * phi
        W = h * dphi * w
        val = _inner(kind, A_[fid][:, None] + 0 * U, U, V0[fid][:, None] + 0 * U,
                     V1[fid][:, None] + 0 * U, K[fid][:, None] + 0 * U, L)
        np.add.at(out[sl], fid, (W * val).sum(axis=1))
    return out


def _edge_integral(rho2, z0, z1, k, L):
    """Exact int_{z0}^{z1} T(k-R/L)/(4 pi R) dz along a line at distance sqrt(rho2)."""
    rho2, z0, z1 = (np.asarray(x, dtype=np.float64) for x in (rho2, z0, z1))
    k = np.asarray(k, dtype=np.float64)
    kn = _knots(k, L)
    d2 = kn * kn - rho2[:, None]
    s = np.sqrt(np.where(d2 > 0, d2, np.nan))
    sp = np.concatenate([s, -s], axis=1)
    sp = np.where(np.isnan(sp), z0[:, None], sp)
    sp = np.clip(sp, z0[:, None], z1[:, None])
    Z = np.sort(np.concatenate([z0[:, None], sp, z1[:, None]], axis=1), axis=1)
    za, zb = Z[:, :-1], Z[:, 1:]
    rm = np.sqrt(rho2[:, None] + (0.5 * (za + zb)) ** 2)
    kb = np.broadcast_to(k[:, None], rm.shape)
    b0, b1, b2 = _poly_in_R(_piece(rm, kb, L), kb, L)
    rho = np.sqrt(rho2)[:, None]
    r2 = rho2[:, None]

    def prim(z):
        R = np.sqrt(r2 + z * z)
        ash = np.arcsinh(z / rho)
        return b0 * ash + b1 * z + b2 * 0.5 * (z * R + r2 * ash)

    return ((prim(zb) - prim(za)).sum(axis=1)) / FOUR_PI


def dyad_at(dx, dy, dz, k, L, nq=16):
    """G_k(d) for arrays of non-negative integer offsets; returns (6, n) FP64.

    No masking is applied: entries outside the causal shell come out as
    (rounding-level) zeros of the exact formulas.
    """
    d = [np.asarray(v, dtype=np.float64).ravel() for v in (dx, dy, dz)]
    n = d[0].size
    k = np.broadcast_to(np.asarray(k, dtype=np.float64), (n,)).copy()
    G = np.zeros((6, n))
    # diagonal A and the time term B, face by face
    B = np.zeros(n)
    for p in range(3):
        q1, q2 = [i for i in range(3) if i != p]
        for sgn in (1.0, -1.0):
            a = d[p] + 0.5 * sgn
            args = (a, d[q1] - 0.5, d[q1] + 0.5, d[q2] - 0.5, d[q2] + 0.5, k, L)
            G[p] += sgn * a * _face_integral("A", *args, nq=nq)
            B -= sgn * a * _face_integral("H", *args, nq=nq)
    for p in range(3):
        G[p] += B
    selfbox = (d[0] == 0) & (d[1] == 0) & (d[2] == 0)
    tk = spline(k)
    for p in range(3):
        G[p] += np.where(selfbox, tk, 0.0)
    # off-diagonal: edge integrals
    for c in (3, 4, 5):
        p, q = PAIR[c]
        r = 3 - p - q
        acc = np.zeros(n)
        for sp_ in (1.0, -1.0):
            for sq_ in (1.0, -1.0):
                xp = d[p] + 0.5 * sp_
                xq = d[q] + 0.5 * sq_
                acc += sp_ * sq_ * _edge_integral(xp * xp + xq * xq, d[r] - 0.5, d[r] + 0.5, k, L)
        acc[(d[p] == 0) | (d[q] == 0)] = 0.0
        G[c] = acc
    return G


def green_octant(nx, ny, nz, k, alpha=None, cdt=None, nq=16):
    """G_k on the non-negative octant of offsets, shape (6, nz, ny, nx), FP64.

    Entries outside the causal mask of ``masks`` are exact zeros.
    """
    L = float(cdt) if cdt is not None else float(alpha) / math.sqrt(3.0)
    DZ, DY, DX = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    m = mask(DX, DY, DZ, k, alpha=alpha, cdt=cdt)
    out = np.zeros((6, nz, ny, nx))
    if m.any():
        vals = dyad_at(DX[m], DY[m], DZ[m], k, L, nq=nq)
        for c in range(6):
            out[c][m] = vals[c]
    return out


def green_all(nx, ny, nz, nl, alpha=None, cdt=None, nq=16):
    """[G_0, ..., G_nl] octant tables."""
    return [green_octant(nx, ny, nz, k, alpha=alpha, cdt=cdt, nq=nq) for k in range(nl + 1)]


def green_full(goct):
    """Expand an octant table to all offsets: (3, 3, 2nz-1, 2ny-1, 2nx-1).

    G(s*d)[p,q] = s_p s_q G(d)[p,q] for reflections s, and G[q,p] = G[p,q].
    Index (nz-1+dz, ny-1+dy, nx-1+dx) holds offset d.
    """
    _, nz, ny, nx = goct.shape
    iz = np.abs(np.arange(-(nz - 1), nz))
    iy = np.abs(np.arange(-(ny - 1), ny))
    ix = np.abs(np.arange(-(nx - 1), nx))
    sz = np.where(np.arange(-(nz - 1), nz) < 0, -1.0, 1.0)
    sy = np.where(np.arange(-(ny - 1), ny) < 0, -1.0, 1.0)
    sx = np.where(np.arange(-(nx - 1), nx) < 0, -1.0, 1.0)
    sgn = (sx[None, None, :], sy[None, :, None], sz[:, None, None])
    full = np.zeros((3, 3, 2 * nz - 1, 2 * ny - 1, 2 * nx - 1))
    for c, (p, q) in enumerate(PAIR):
        blk = goct[c][np.ix_(iz, iy, ix)]
        if p != q:
            blk = blk * sgn[p] * sgn[q]
        full[p, q] = blk
        full[q, p] = blk
    return full
