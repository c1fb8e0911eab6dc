"""Differentiable GN layer: ``torch.autograd.Function`` over the library's unrolled
forward and hand-written adjoint (gn_unrolled_forward / gn_unrolled_backward).

Marshalling only: the steps and their adjoint run in HIP.  ``w`` (vertex weights)
and ``x0`` may both require gradients; the returned ``x_T`` is the state after T
WRGN steps with the given gamma schedule."""
from __future__ import annotations

import numpy as np
import torch

from . import libgn


class GNUnrolled(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w, x0, graph_handle, gammas, ckpt_every):
        gam = np.ascontiguousarray(np.asarray(gammas, dtype=np.float32))
        w = w.detach().contiguous()
        x0 = x0.detach().contiguous()
        xT = torch.empty_like(x0)
        ckpt = torch.empty(libgn.gn_unrolled_ckpt_floats(graph_handle, len(gam), ckpt_every),
                           dtype=torch.float32, device=x0.device)
        libgn.gn_unrolled_forward(graph_handle, w, gam, ckpt_every, x0, xT, ckpt)
        ctx.save_for_backward(w, ckpt)
        ctx.graph = graph_handle
        ctx.gammas = gam
        ctx.ckpt_every = ckpt_every
        return xT

    @staticmethod
    def backward(ctx, gxT):
        w, ckpt = ctx.saved_tensors
        gxT = gxT.contiguous()
        gw = torch.empty_like(w)
        gx0 = torch.empty_like(gxT)
        libgn.gn_unrolled_backward(ctx.graph, w, ctx.gammas, ctx.ckpt_every, ckpt, gxT, gw, gx0)
        return gw, gx0, None, None, None


# default memory for keeping every step's y and s (ckpt_every = 1, no recompute in
# the backward); above it the default checkpoints every ~sqrt(T) steps
KEEP_ALL_BYTES = 1 << 30


def default_ckpt_every(n: int, T: int) -> int:
    """1 (keep y and s of every step, 8 T n bytes) while that fits KEEP_ALL_BYTES,
    else ceil(sqrt(T)) (about 2 sqrt(T) n floats of checkpoints and segments)."""
    if T <= 1 or 8 * T * n <= KEEP_ALL_BYTES:
        return 1
    return int(np.ceil(np.sqrt(T)))


def gn_unrolled(w, x0, graph_handle, gammas, ckpt_every=None):
    """x_T after len(gammas) WRGN steps from x0 with weights w (differentiable in w, x0).
    ckpt_every: checkpoint interval of the backward's recompute; None picks
    default_ckpt_every.  The gradient does not depend on it."""
    if ckpt_every is None:
        ckpt_every = default_ckpt_every(int(x0.numel()), len(gammas))
    return GNUnrolled.apply(w, x0, graph_handle, gammas, ckpt_every)


class GNUnrolledBatch(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w, x0, batch_handle, gammas):
        gam = np.ascontiguousarray(np.asarray(gammas, dtype=np.float32))
        w = w.detach().contiguous()
        x0 = x0.detach().contiguous()
        xT = torch.empty_like(x0)
        store = torch.empty(libgn.gn_batch_unrolled_store_floats(batch_handle, len(gam)), dtype=torch.float32,
                            device=x0.device)
        libgn.gn_batch_unrolled_forward(batch_handle, w, gam, x0, xT, store)
        ctx.save_for_backward(w, store)
        ctx.batch = batch_handle
        ctx.gammas = gam
        return xT

    @staticmethod
    def backward(ctx, gxT):
        w, store = ctx.saved_tensors
        gxT = gxT.contiguous()
        gw = torch.empty_like(w)
        gx0 = torch.empty_like(gxT)
        libgn.gn_batch_unrolled_backward(ctx.batch, w, ctx.gammas, store, gxT, gw, gx0)
        return gw, gx0, None, None


def gn_unrolled_batch(w, x0, batch_handle, gammas):
    """The same for every graph of a batch (vertex vectors: the graphs' user
    orders back to back), one workgroup per graph: x_T and both gradients are
    bit-identical to gn_unrolled on the batch's union graph with every state
    kept."""
    return GNUnrolledBatch.apply(w, x0, batch_handle, gammas)
