"""Causal regions of the interaction matrices (oracle; test infrastructure only).

Sec. III-A (Fig. 1 and its discussion): a column of Z_k is populated by the
testing voxels that the spherical wavefront of the basis voxel intersects or
encloses over the k-th time interval.  With centre-point testing and the
temporal basis of ``basis`` (support [-dt, 2dt)), Z_k couples observation and
source voxels at offset d iff the source box B(d) = prod_i [d_i-1/2, d_i+1/2]
(seen from the observation centre) meets the open shell

    (k-2) L < R < (k+1) L ,      L = c0 dt / h.

With dmin(d)^2 = sum_i max(|d_i|-1/2, 0)^2 and dmax(d)^2 = sum_i (|d_i|+1/2)^2
that is dmin < (k+1) L  and  dmax > (k-2) L.  For an integer alpha
(L = alpha/sqrt 3) both tests are exact in integers:

    3 * sum max(2|d_i|-1, 0)^2 < 4 (k+1)^2 alpha^2
    k <= 2  or  3 * sum (2|d_i|+1)^2 > 4 (k-2)^2 alpha^2 .

Table III counts the nonzeros of Z0 in MATLAB sparse storage; an offset with
0/1/2/3 nonzero components carries 3/3/5/9 nonzero dyad entries (the
off-diagonal entries G_pq with d_p = 0 or d_q = 0 vanish by symmetry).
"""

import numpy as np

DYAD_WEIGHT = np.array([3, 3, 5, 9], dtype=np.int64)


def mask(dx, dy, dz, k, alpha=None, cdt=None):
    """Boolean M_k(d) for integer offset arrays (any sign)."""
    ax, ay, az = (np.abs(np.asarray(v, dtype=np.int64)) for v in (dx, dy, dz))
    if alpha is not None and float(alpha) == int(alpha):
        a2 = int(alpha) ** 2
        lo = (3 * (np.maximum(2 * ax - 1, 0) ** 2 + np.maximum(2 * ay - 1, 0) ** 2
                   + np.maximum(2 * az - 1, 0) ** 2)) < 4 * (k + 1) ** 2 * a2
        if k <= 2:
            return lo
        hi = (3 * ((2 * ax + 1) ** 2 + (2 * ay + 1) ** 2 + (2 * az + 1) ** 2)) > 4 * (k - 2) ** 2 * a2
        return lo & hi
    L = float(cdt)
    dmin = np.sqrt(np.maximum(ax - 0.5, 0) ** 2 + np.maximum(ay - 0.5, 0) ** 2
                   + np.maximum(az - 0.5, 0) ** 2)
    dmax = np.sqrt((ax + 0.5) ** 2 + (ay + 0.5) ** 2 + (az + 0.5) ** 2)
    return (dmin < (k + 1) * L) & (dmax > (k - 2) * L)


def zk_nnz(nx, ny, nz, k=0, alpha=None, cdt=None):
    """Nonzero count of Z_k on an nx*ny*nz grid (3 unknowns per voxel).

    Sum over offsets d of mask * dyad weight * number of voxel pairs at that
    offset, prod_i (N_i - |d_i|).  Exact integer.
    """
    total = 0
    ddx = np.arange(-(nx - 1), nx, dtype=np.int64)
    ddy = np.arange(-(ny - 1), ny, dtype=np.int64)
    for dz in range(-(nz - 1), nz):
        DY, DX = np.meshgrid(ddy, ddx, indexing="ij")
        DZ = np.full_like(DX, dz)
        m = mask(DX, DY, DZ, k, alpha=alpha, cdt=cdt)
        nzc = (DX != 0).astype(np.int64) + (DY != 0) + (DZ != 0)
        pairs = (nx - np.abs(DX)) * (ny - np.abs(DY)) * (nz - abs(dz))
        total += int((m * DYAD_WEIGHT[nzc] * pairs).sum())
    return total


def lag_support(nx, ny, nz, nl, alpha=None, cdt=None):
    """List of (k, boolean octant mask [nz][ny][nx]) for k = 0..nl."""
    DZ, DY, DX = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return [(k, mask(DX, DY, DZ, k, alpha=alpha, cdt=cdt)) for k in range(nl + 1)]
