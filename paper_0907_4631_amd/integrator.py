"""Exponential Rosenbrock-Euler for the Allen-Cahn equation u_t = Lap u + u - u^3
on the unit square (homogeneous Dirichlet boundary), the consumer of the
reaction-diffusion call sequence: its Jacobians J(u) = Lap + diag(1 - 3 u^2)
are the operators of those calls.

One step is one solver call (the paper's motivating use, its Sect. 1):

    u_{n+1} = u_n + h phi_1(h J_n) F(u_n),   F(u) = Lap u + u - u^3,

i.e. phipm at t = h with b_0 = 0 and b_1 = F(u_n).  The solve runs in the
library's solver; F, the Jacobian's diagonal and the update u += h phi_1 F run
in its phipm_allen_cahn_update kernels.
"""
from __future__ import annotations

import numpy as np

from . import FP64, DeviceCSR, Solver, allen_cahn_update


class AllenCahnERE:
    """State u (float64 device tensor of N*N interior values) advanced with
    time step h.  proposer: device float32 weights of the learned (tau, m)
    proposer or None; warm: carry the last step's (tau, m) to the next call."""

    def __init__(self, lap, u0, h: float, tol: float = 1e-6, proposer=None,
                 warm: bool = False, device="cuda"):
        import torch
        self.torch = torch
        lap = lap.tocsr()
        lap.sort_indices()
        self.n = lap.shape[0]
        self.h = float(h)
        self.L = DeviceCSR(lap, device=device)
        self.J = DeviceCSR(lap, device=device)  # same pattern; diagonal updated per step
        rows = np.repeat(np.arange(self.n), np.diff(lap.indptr))
        diag = np.nonzero(lap.indices == rows)[0]
        if diag.size != self.n:
            raise ValueError("the Laplacian must store its full diagonal")
        self.diag = torch.as_tensor(diag.astype(np.int32), device=device)
        self.lap_diag = torch.as_tensor(np.asarray(lap.data[diag], dtype=np.float64),
                                        device=device)
        self.u = torch.as_tensor(np.asarray(u0, dtype=np.float64), device=device).clone()
        self.solver = Solver(self.J, 1, tol=tol, precision=FP64, symm=1)
        self.hist = None
        if proposer is not None:
            self.weights = proposer
            self.solver.opts.proposer = proposer.data_ptr()
        if warm:
            self.hist = torch.zeros(4, dtype=torch.float64, device=device)
            self.solver.opts.history = self.hist.data_ptr()
        self.b = torch.zeros((2, self.n), dtype=torch.float64, device=device)
        self.du = torch.empty(self.n, dtype=torch.float64, device=device)

    def rhs(self, out):
        """out <- F(u) = Lap u + u - u^3."""
        allen_cahn_update(self.L, self.u, F=out)
        return out

    def step(self, stats: bool = False):
        allen_cahn_update(self.L, self.u, diag_pos=self.diag, lap_diag=self.lap_diag,
                          J_val=self.J.val, F=self.b[1])
        st = self.solver(self.h, self.b, self.du, stats=stats)
        allen_cahn_update(self.L, self.u, du=self.du)
        return st

    def run(self, steps: int, stats: bool = False):
        return [self.step(stats) for _ in range(steps)]
