"""The 2-D nonlinear heat-conduction test of Section 3.1 on the GPU.

Backward Euler in time and Picard iterations (the paper's algorithm for the
2-D heat conduction equation): at time step n, T^(n+1,0) = T^n; Picard
iteration s assembles A(k(T^(n+1,s))) and b(T^n) (lcs_assemble_heat), solves
A T^(n+1,s+1) = b from the initial iterate T^(n+1,s) with the chosen method,
and stops once ||T^(n+1,s+1) - T^(n+1,s)||_2 < 1e-8 (lcs_norm2_diff).  The
three methods compared by the paper are the global solve ("global"), the
local character-based method with the gradient domain (Algorithm 2,
alpha = 1e-4) and with the residual domain (Algorithm 3, paper threshold,
E_max = 1), each finished by the global PCG when needed (Algorithm 1).

This module only orders library calls; every arithmetic step runs in the
library's kernels.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, List

import torch

from . import lcs
from . import workloads as W

METHODS = ("global", "gradient", "residual")


@dataclasses.dataclass
class SystemRecord:
    step: int
    picard: int
    K: int
    its_local: int
    its_global: int
    ms: float            # wall time of the linear solve (the call synchronises)


def solver(method: str, opts: lcs.Options, ctx: lcs.Context = None) -> Callable:
    """The linear solve of one Picard system for the given method."""
    if method == "global":
        return lambda A, b, x: lcs.solve_global(A, b, x, opts, ctx=ctx)
    if method == "gradient":
        return lambda A, b, x: lcs.solve_local_then_global(A, b, x, "gradient", "relmax", W.HEAT_ALPHA,
                                                           0, opts, ctx=ctx)
    if method == "residual":
        return lambda A, b, x: lcs.solve_local_then_global(A, b, x, "residual", "paper", opts.eps,
                                                           W.HEAT_E_MAX, opts, ctx=ctx)
    raise ValueError(f"unknown method {method!r}")


class Heat2D:
    """One simulation of the test problem on n x n cells."""

    def __init__(self, n: int, method: str, device: str = "cuda:0", dt: float = W.HEAT_DT,
                 opts: lcs.Options = None, ctx: lcs.Context = None):
        self.n, self.N = n, n * n
        self.inv_dt = (1.0 / n) ** 2 / dt       # equations scaled by h^2
        self.ctx = ctx if ctx is not None else lcs.Context()
        self.opts = opts if opts is not None else lcs.Options(eps=1e-10)
        self.solve = solver(method, self.opts, self.ctx)
        self.T = torch.as_tensor(W.heat2d_initial(n, n)).to(device)
        self.coef = torch.empty((3, self.N), dtype=torch.float64, device=device)
        self.b = torch.empty(self.N, dtype=torch.float64, device=device)
        self.A = lcs.Matrix(lcs.STENCIL5_2D, n, n, 1, self.coef)
        self._told = torch.empty_like(self.T)
        self._ts = torch.empty_like(self.T)
        self._x = torch.empty_like(self.T)
        self.steps_done = 0

    def step(self, picard_tol: float = W.HEAT_PICARD_TOL, max_picard: int = 200) -> List[SystemRecord]:
        """Advance one time step; returns one record per Picard system."""
        n = self.n
        self._told.copy_(self.T)
        ts, x = self._ts, self._x
        ts.copy_(self.T)
        recs = []
        for s in range(max_picard):
            lcs.assemble_heat(n, n, self.inv_dt, W.HEAT_POWER, W.HEAT_T_LEFT, W.HEAT_T_RIGHT, ts,
                              self._told, self.coef, self.b, ctx=self.ctx)
            x.copy_(ts)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = self.solve(self.A, self.b, x)
            ms = (time.perf_counter() - t0) * 1e3
            recs.append(SystemRecord(self.steps_done, s, st.K, st.its_local, st.its_global, ms))
            d = lcs.norm2_diff(x, ts, ctx=self.ctx)
            ts, x = x, ts
            if d < picard_tol:
                break
        self.T.copy_(ts)
        self.steps_done += 1
        return recs
