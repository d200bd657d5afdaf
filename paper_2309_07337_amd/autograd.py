"""Differentiable halo exchange over every rank of a plan.

``HaloExchange`` binds a whole-decomposition batch (all ranks on this GPU)
to persistent buffers; ``HaloGather`` is the ``torch.autograd.Function``
whose forward runs Start/Wait of all ranks (pack, simulated transfer,
redistribution, unpack) and whose backward runs the library's fixed-order
transpose sum: for every owned row c, the gradient is the sum over the ranks
whose halo holds c, in ascending rank order, of that halo entry's gradient
(or, with ``staged_backward``, the same sum grouped by the locality plan's
stages: each forwarder's partial sum first, see ``hx.h``).
Both directions run in the library's HIP kernels.

Buffers and copies.  The library reads ``ex.x`` and writes ``ex.halo``
(forward), reads ``ex.g_halo`` and writes ``ex.g_x`` (backward), all bound
once.  ``halo_gather(x, ex)`` copies ``x`` into ``ex.x`` unless ``x`` is
``ex.x`` itself, and returns a fresh tensor (a copy of ``ex.halo``), so a
later forward on the same exchange cannot change an earlier output.  The
zero-copy path: write the input into ``ex.x`` in place, call
``halo_gather(ex.x, ex, copy_out=False)`` (the output then IS ``ex.halo``),
and give the backward its gradient in ``ex.g_halo`` (a gradient tensor that
is ``ex.g_halo`` is not copied).  An aliased output is guarded: its backward
raises if another forward ran on the exchange in between.
"""
from __future__ import annotations

import torch

from . import _lib as L


class HaloExchange:
    """Persistent exchange of ``x_global [n, ncols] -> halo_all [sum H, ncols]``.

    The buffers are allocated once (persistent semantics); ``forward()``
    overwrites ``self.halo`` and counts itself in ``self.generation``.
    """

    def __init__(self, plan: L.Plan, n: int, halo_rows: int, ncols: int, dtype=torch.float32,
                 device="cuda", sim_transfer: bool = True, sched=None, staged_backward: bool = False):
        self.x = torch.zeros(n, ncols, dtype=dtype, device=device)
        self.halo = torch.zeros(halo_rows, ncols, dtype=dtype, device=device)
        self.g_halo = torch.zeros_like(self.halo)
        self.g_x = torch.zeros_like(self.x)
        self.generation = 0
        flags = L.HX_WORLD_SIM_TRANSFER if sim_transfer else 0
        if staged_backward:   # locality plans: the backward through the plan's stages
            flags |= L.HX_WORLD_STAGED_BACKWARD
        self.batch = L.hx_batch_from_plan(plan, self.x, self.halo, flags=flags, sched=sched)
        L.hx_batch_bind_grad(self.batch, self.g_halo, self.g_x)

    def forward(self, stream=None) -> torch.Tensor:
        L.hx_batch_start(self.batch, stream)
        L.hx_batch_wait(self.batch, stream)
        self.generation += 1
        return self.halo

    def backward(self, stream=None) -> torch.Tensor:
        L.hx_batch_backward(self.batch, stream)
        return self.g_x


class HaloGather(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, ex: HaloExchange, copy_out: bool = True):
        if x.data_ptr() != ex.x.data_ptr():
            ex.x.copy_(x)
        ex.forward()
        ctx.ex = ex
        ctx.generation = ex.generation
        ctx.copy_out = copy_out
        return ex.halo.clone() if copy_out else ex.halo.detach()

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        ex: HaloExchange = ctx.ex
        if not ctx.copy_out and ex.generation != ctx.generation:
            raise RuntimeError("halo_gather: the aliased output of this forward was overwritten by a later "
                               "forward on the same exchange before its backward ran")
        if g.data_ptr() != ex.g_halo.data_ptr() or not g.is_contiguous():
            ex.g_halo.copy_(g)
        ex.backward()
        return ex.g_x.clone(), None, None


def halo_gather(x: torch.Tensor, ex: HaloExchange, copy_out: bool = True) -> torch.Tensor:
    return HaloGather.apply(x, ex, copy_out)
