"""Differentiable upwind advection solve: u = A(theta)^{-1} b(g, theta).

`advect(g_west, g_south, theta, nx, ny)` assembles the finite-volume system on
the device (airg_fv_assemble), builds the AIRG hierarchy and solves with
FGMRES (airg_setup / airg_solve).  The backward pass solves the adjoint
system A^T lam = dL/du with a hierarchy built on the transpose
(airg_adjoint_solve) and contracts it into the gradients (airg_fv_gradients):

    dL/dg_west[j]  = vx lam[j nx]          (west inflow cells)
    dL/dg_south[i] = vy lam[i]             (south inflow cells)
    dL/dtheta      = lam^T (db/dtheta - dA/dtheta u)

This module only marshals arguments; every step runs in libairg.so.
"""
import ctypes

import torch

from . import binding
from . import Solver, _ptr, _stream_ptr


class FVSystem:
    """The assembled upwind system on the device."""

    def __init__(self, nx, ny, theta, g_west, g_south, stream=None):
        lib = binding.load()
        nnz = ctypes.c_int64()
        binding.check(lib.airg_fv_nnz(nx, ny, float(theta), ctypes.byref(nnz)), lib)
        n = nx * ny
        dev = torch.device("cuda")
        self.nx, self.ny, self.theta, self.n, self.nnz = nx, ny, float(theta), n, nnz.value
        self.rowptr = torch.empty(n + 1, dtype=torch.int32, device=dev)
        self.col = torch.empty(self.nnz, dtype=torch.int32, device=dev)
        self.val = torch.empty(self.nnz, dtype=torch.float64, device=dev)
        self.b = torch.empty(n, dtype=torch.float64, device=dev)
        self.dval = torch.empty(self.nnz, dtype=torch.float64, device=dev)
        self.db = torch.empty(n, dtype=torch.float64, device=dev)
        gw = g_west.detach().to(device=dev, dtype=torch.float64).contiguous()
        gs = g_south.detach().to(device=dev, dtype=torch.float64).contiguous()
        code = lib.airg_fv_assemble(nx, ny, self.theta, _ptr(gw), _ptr(gs), _ptr(self.rowptr),
                                    _ptr(self.col), _ptr(self.val), _ptr(self.b), _ptr(self.dval),
                                    _ptr(self.db), _stream_ptr(stream))
        binding.check(code, lib)


class _AdvectionSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, g_west, g_south, theta, nx, ny, params):
        sysm = FVSystem(nx, ny, float(theta), g_west, g_south)
        solver = Solver(sysm.rowptr, sysm.col, sysm.val, params=params)
        u, info = solver.solve(sysm.b)
        if info["converged"] != 1:
            raise binding.AirgError(1, f"forward solve did not converge: {info}")
        ctx.sysm, ctx.solver = sysm, solver
        ctx.theta_dtype = theta.dtype if isinstance(theta, torch.Tensor) else torch.float64
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        (u,) = ctx.saved_tensors
        sysm, solver = ctx.sysm, ctx.solver
        w = grad_u.detach().to(dtype=torch.float64).contiguous()
        lam, info = solver.adjoint_solve(w)
        if info["converged"] != 1:
            raise binding.AirgError(1, f"adjoint solve did not converge: {info}")
        dgw = torch.empty(sysm.ny, dtype=torch.float64, device="cuda")
        dgs = torch.empty(sysm.nx, dtype=torch.float64, device="cuda")
        dth = torch.empty(1, dtype=torch.float64, device="cuda")
        lib = binding.load()
        code = lib.airg_fv_gradients(sysm.nx, sysm.ny, sysm.theta, _ptr(sysm.rowptr), _ptr(sysm.col),
                                     _ptr(sysm.dval), _ptr(sysm.db), _ptr(u), _ptr(lam), _ptr(dgw),
                                     _ptr(dgs), _ptr(dth), _stream_ptr(None))
        binding.check(code, lib)
        solver.close()
        return dgw, dgs, dth.reshape(()).to(ctx.theta_dtype), None, None, None


def advect(g_west, g_south, theta, nx, ny=None, **overrides):
    """u (CUDA float64, length nx*ny, unknown k = j nx + i) solving the upwind
    advection system; differentiable in g_west [ny], g_south [nx] and theta
    (a 0-d tensor).  Keyword overrides set solver parameters (e.g. rtol)."""
    ny = nx if ny is None else ny
    params = binding.default_params(**overrides)
    if not isinstance(theta, torch.Tensor):
        theta = torch.tensor(float(theta), dtype=torch.float64)
    return _AdvectionSolve.apply(g_west, g_south, theta, nx, ny, params)
