"""Gradient of a far-field energy with respect to the permittivity, through
the adjoint (transposed, time-reversed) MOT march, behind torch.autograd.

Sequencing and marshalling only: every product, solve, far-field sum and
gradient term runs in the HIP library (see include/mot_jvie.h, "Adjoint
march and permittivity gradient").

    march = FarFieldMarch(ctx, pulse, nsteps, rhat)
    W = far_field_energy(eps, march)      # eps: FP64 device tensor (N,), requires_grad
    W.backward()                          # eps.grad = dW/d eps by the adjoint march

W = dt sum_j |e_j|^2 is the energy of the far-field signature e_j (samples
tau_j = j dt) radiated in direction rhat by the current history of a march of
nsteps MOT steps (Eq. 3) driven by the plane wave `pulse` (Eq. 7, Eq. 8).
"""

import math

import torch

from . import native


def farfield_window(shape, rhat, dt, nsteps):
    """(j0, nj): far-field samples that a march of nsteps steps can reach.

    |rhat . r_m| <= (|r_x| nx + |r_y| ny + |r_z| nz)/2 for every voxel centre,
    and T'(j - n + s) vanishes outside -1 <= j - n + s < 2."""
    nx, ny, nz = shape
    r = [float(v) for v in rhat]
    nr = math.sqrt(sum(v * v for v in r))
    if not nr > 0.0:
        raise ValueError("rhat must be non-zero")
    r = [v / nr for v in r]
    S = (abs(r[0]) * nx + abs(r[1]) * ny + abs(r[2]) * nz) / (2.0 * dt)
    j0 = math.floor(-1.0 - S) - 1
    j1 = math.ceil(nsteps + 1.0 + S) + 1
    return j0, j1 - j0 + 1


class FarFieldMarch:
    """A forward march that records what the adjoint gradient needs.

    ``ctx`` is a ``native.Context`` whose Green spectra are built; its
    material is set by ``forward``.  FP64 contexts give gradients to the
    solver tolerance; the refined and FP32 modes are accepted."""

    def __init__(self, ctx, pulse, nsteps, rhat, tol=1e-10, max_iter=1000):
        self.ctx = ctx
        self.pulse = dict(pulse)
        self.nsteps = int(nsteps)
        self.rhat = [float(v) for v in rhat]
        self.tol = float(tol)
        self.max_iter = int(max_iter)
        nl = ctx.info()["nlags"]
        self.dt = float(ctx.grid.alpha) / math.sqrt(3.0) if ctx.grid.alpha else float(ctx.grid.cdt)
        self.nlags = nl
        self.j0, self.nj = farfield_window(ctx.shape, self.rhat, self.dt, self.nsteps)
        self.Jhist = None
        self.UH = None
        self.e = None
        self.eps = None
        self.generation = 0   # forward marches run so far; the recorded state is that of the last

    def forward(self, eps):
        """Run the march for permittivity eps; returns W (a Python float)."""
        c = self.ctx
        n3 = 3 * c.N
        dev = eps.device
        self.eps = eps.detach().contiguous().clone()
        self.generation += 1
        c.set_material(self.eps)
        c.set_adjoint(False)
        c.reset()
        self.Jhist = torch.empty((self.nsteps, n3), dtype=torch.float64, device=dev)
        self.UH = torch.empty((self.nsteps, n3), dtype=torch.float64, device=dev)
        einc = torch.empty(n3, dtype=torch.float64, device=dev)
        for n in range(self.nsteps):
            c.history_gfield(self.UH[n])
            c.excitation(self.pulse, n * self.dt, einc)
            c.step(einc, self.Jhist[n], tol=self.tol, max_iter=self.max_iter, stats=False)
        self.e = torch.empty((self.nj, 3), dtype=torch.float64, device=dev)
        W = torch.empty(1, dtype=torch.float64, device=dev)
        c.farfield(self.Jhist, self.rhat, self.j0, self.nj, self.e, W)
        return float(W.item())

    def gradient(self):
        """dW/d eps (FP64 device tensor of N) for the last ``forward``."""
        if self.e is None:
            raise RuntimeError("forward() must run before gradient()")
        c = self.ctx
        n3 = 3 * c.N
        dev = self.e.device
        # the adjoint operators use the material of the recorded march
        c.set_material(self.eps)
        g = torch.empty(n3, dtype=torch.float64, device=dev)
        lam = torch.empty(n3, dtype=torch.float64, device=dev)
        u0 = torch.empty(n3, dtype=torch.float64, device=dev)
        grad = torch.zeros(c.N, dtype=torch.float64, device=dev)
        c.set_adjoint(True)
        c.reset()
        try:
            for n in range(self.nsteps - 1, -1, -1):
                c.farfield_adjoint(self.e, self.j0, self.rhat, n, g, scale=2.0 * self.dt)
                c.step(g, lam, tol=self.tol, max_iter=self.max_iter, stats=False)
                c.gk_matvec(0, self.Jhist[n], u0, "f64")
                c.adjoint_gradient(self.pulse, n * self.dt, lam, self.Jhist[n],
                                   self.Jhist[n - 1] if n > 0 else None, self.UH[n], u0, grad,
                                   J_prev2=self.Jhist[n - 2] if n > 1 else None)
        finally:
            c.set_adjoint(False)
            c.reset()
        return grad


class FarFieldEnergy(torch.autograd.Function):
    """W(eps) with dW/d eps from the adjoint march."""

    @staticmethod
    def forward(fctx, eps, march):
        W = march.forward(eps)
        fctx.march = march
        fctx.generation = march.generation
        fctx.eps = march.eps
        return torch.tensor(W, dtype=torch.float64, device=eps.device)

    @staticmethod
    def backward(fctx, grad_out):
        m = fctx.march
        if m.generation != fctx.generation:
            # another forward ran on this march since this node's: the recorded
            # currents are not this node's, so march again from its permittivity
            m.forward(fctx.eps)
            fctx.generation = m.generation
        return grad_out * m.gradient(), None


def far_field_energy(eps, march):
    """W(eps) as a differentiable scalar (see FarFieldEnergy)."""
    return FarFieldEnergy.apply(eps, march)
