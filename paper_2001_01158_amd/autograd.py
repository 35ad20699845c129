"""Differentiable local character-based solve (hand-written adjoint).

x = A(logk)^-1 b, with A the five- or seven-point log-conductivity operator
(A = I/dt + sum_f T_f (e_P - e_Q)(e_P - e_Q)^T, T_f the harmonic face mean of
exp(logk)), solved by Algorithm 1 from the warm start x0.

Backward: A is symmetric, so the adjoint lambda = A^-T g = A^-1 g is one more
local-then-global solve on the forward's local domain Omega (no re-marking),
from lambda^(0) = 0.  Then dL/db = lambda and
dL/dlogk_P = -sum_{faces (P,Q)} (dT_f/dlogk_P)(x_P - x_Q)(lambda_P - lambda_Q).
Every step runs in the HIP library; this module only orders the calls.
"""
from __future__ import annotations

import dataclasses

import torch

from . import lcs


@dataclasses.dataclass
class SolveConfig:
    kind: int                 # lcs.STENCIL5_2D or lcs.STENCIL7_3D
    nx: int
    ny: int
    nz: int
    inv_dt: float
    mode: str = "residual"
    thresh: str = "paper"
    theta: float = 1e-10
    e_max: int = 1
    opts: lcs.Options = dataclasses.field(default_factory=lcs.Options)
    adjoint_opts: lcs.Options = None   # default: opts


def _local_then_global(A, b, x, idx, opts, ctx):
    """Steps 3-11 of Algorithm 1 for a given domain: local solve, smoothing,
    then the global finish (which returns at once when x~ already meets the
    criterion)."""
    sl = lcs.solve_local(A, b, x, idx, opts, ctx=ctx)
    sg = lcs.solve_global(A, b, x, opts, ctx=ctx)
    sl.its_global = sg.its_global
    sl.relres_final = sg.relres_final
    return sl


class LocalSolve(torch.autograd.Function):
    """x = LocalSolve.apply(logk, b, x0, cfg, ctx)"""

    @staticmethod
    def forward(fctx, logk, b, x0, cfg: SolveConfig, ctx=None):
        ctx = ctx or lcs.default_context()
        fctx.logk_shape = logk.shape
        logk = logk.detach().contiguous().reshape(-1)
        b = b.detach().contiguous()
        coef = lcs.assemble_logk(cfg.kind, cfg.nx, cfg.ny, cfg.nz, cfg.inv_dt, logk, ctx=ctx)
        A = lcs.Matrix(cfg.kind, cfg.nx, cfg.ny, cfg.nz, coef)
        idx, _, _ = lcs.build_local_domain(A, b, x0.detach().contiguous(), cfg.mode, cfg.thresh,
                                           cfg.theta, cfg.e_max, ctx=ctx)
        idx = idx.clone()
        x = x0.detach().clone().contiguous()
        st = _local_then_global(A, b, x, idx, cfg.opts, ctx)
        fctx.save_for_backward(logk, x, idx, coef)
        fctx.cfg = cfg
        fctx.lcs_ctx = ctx
        fctx.stats = st
        return x

    @staticmethod
    def backward(fctx, gx):
        logk, x, idx, coef = fctx.saved_tensors
        cfg = fctx.cfg
        ctx = fctx.lcs_ctx
        A = lcs.Matrix(cfg.kind, cfg.nx, cfg.ny, cfg.nz, coef)
        g = gx.detach().contiguous().to(torch.float64)
        lam = torch.zeros_like(g)
        if torch.count_nonzero(g).item() > 0:
            _local_then_global(A, g, lam, idx, cfg.adjoint_opts or cfg.opts, ctx)
        grad_logk = lcs.grad_logk(cfg.kind, cfg.nx, cfg.ny, cfg.nz, logk, x, lam, ctx=ctx)
        return grad_logk.reshape(fctx.logk_shape), lam, None, None, None


def local_solve(logk, b, x0, cfg: SolveConfig, ctx=None):
    return LocalSolve.apply(logk, b, x0, cfg, ctx)
