"""torch.autograd.Function over the Chebyshev filter and its hand-written adjoint."""

from __future__ import annotations

import numpy as np
import torch

from .binding import Graph, cheb_filter, filter_backward


class ChebFilter(torch.autograd.Function):
    """Y = sum_j a_j T_j(L~) X on a float32 graph.

    Inputs: X (n x w float32, device), a (float64 tensor of m + 1 coefficients), edge_vals
    (float32 tensor with one value per stored entry of A, or None to use the graph's own
    values), the Graph, lmax and the checkpoint interval of the backward pass.  When
    edge_vals is given it is written into the graph before filtering, and its gradient is
    the per-entry adjoint dl/dA_e.
    """

    @staticmethod
    def forward(ctx, X, a, edge_vals, graph: Graph, lmax: float = 2.0, ckpt_every: int = 0):
        if edge_vals is not None:
            graph.set_values(edge_vals.detach())
        coeffs = a.detach().cpu().numpy().astype(np.float64)
        Y = cheb_filter(graph, coeffs, X.detach().contiguous(), lmax=lmax)
        ctx.save_for_backward(X, a)
        ctx.graph = graph
        ctx.lmax = lmax
        ctx.ckpt = ckpt_every
        ctx.has_vals = edge_vals is not None
        return Y

    @staticmethod
    def backward(ctx, G):
        X, a = ctx.saved_tensors
        coeffs = a.detach().cpu().numpy().astype(np.float64)
        dX, da, dA = filter_backward(ctx.graph, coeffs, X.detach().contiguous(),
                                     G.detach().float().contiguous(), lmax=ctx.lmax,
                                     ckpt_every=ctx.ckpt, want_dx=ctx.needs_input_grad[0],
                                     want_da=ctx.needs_input_grad[1],
                                     want_dA=ctx.has_vals and ctx.needs_input_grad[2])
        da_out = da.to(device=a.device, dtype=a.dtype) if da is not None else None
        return dX, da_out, dA, None, None, None


def cheb_filter_autograd(X, a, graph: Graph, edge_vals=None, lmax: float = 2.0, ckpt_every: int = 0):
    return ChebFilter.apply(X, a, edge_vals, graph, lmax, ckpt_every)
