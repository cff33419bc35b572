"""torch.autograd bindings of the compressed-contraction library.

Torch supplies device memory; every arithmetic step (the Ising coupling map,
the forward tree, the reverse pass and the coupling chain rule) runs in the
library's HIP kernels through the C ABI.  The library works on its own stream:
each call first waits for torch's current stream (its inputs) and the library
stream is synchronised before torch reads what it wrote.

    import torch, paper_2206_07044_amd as tn
    from paper_2206_07044_amd.autograd import IsingLogZ, TensorLogZ
    net = IsingLogZ(n, edges, pairs, chi=16, beta=0.5)            # plans once
    J = torch.ones(n_edges, dtype=torch.float64, device="cuda", requires_grad=True)
    lnz = net(J); lnz.backward()                                   # J.grad = d ln|Z| / d J

checkpoint_segments (0: every forward buffer the reverse pass reads stays resident; S >= 2:
forward segments recomputed in the reverse pass; -1: the S of smallest arena) trades device
memory for up to one more forward pass per backward.
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np
import torch

from ._capi import Context


class _LogZFromData(torch.autograd.Function):
    """ln|Z| as a function of the flattened input tensors (float64, device)."""

    @staticmethod
    def _evaluate(tnctx: Context, data: torch.Tensor) -> float:
        torch.cuda.current_stream().synchronize()
        tnctx.tn_update_values_device(data.data_ptr())
        tnctx.tn_contract_compressed()
        return tnctx.tn_result()[1]

    @staticmethod
    def forward(ctx, data: torch.Tensor, tnctx: Context):
        data = data.detach().contiguous()
        lnz = _LogZFromData._evaluate(tnctx, data)
        ctx.save_for_backward(data)
        ctx.tnctx = tnctx
        ctx.state_id = tnctx.state_id
        return torch.tensor(lnz, dtype=torch.float64, device=data.device)

    @staticmethod
    def backward(ctx, g):
        (data,) = ctx.saved_tensors
        if ctx.tnctx.state_id != ctx.state_id:
            # the context has evaluated something else since this forward pass: recompute it
            # (the reverse pass reads the forward intermediates the context holds)
            _LogZFromData._evaluate(ctx.tnctx, data)
        out = torch.empty(data.numel(), dtype=torch.float64, device=g.device)
        torch.cuda.current_stream().synchronize()
        ctx.tnctx.tn_grad_device(out.data_ptr())
        ctx.tnctx.tn_sync()
        return g * out, None


class _LogZFromCouplings(torch.autograd.Function):
    """ln|Z| of the Ising model (SI F.1) as a function of the couplings J."""

    @staticmethod
    def _evaluate(tnctx: Context, J: torch.Tensor, beta: float) -> float:
        torch.cuda.current_stream().synchronize()
        tnctx.tn_ising_values_device(beta, J.data_ptr())
        tnctx.tn_contract_compressed()
        return tnctx.tn_result()[1]

    @staticmethod
    def forward(ctx, J: torch.Tensor, tnctx: Context, beta: float, n_data: int):
        Jc = J.detach().contiguous()
        lnz = _LogZFromCouplings._evaluate(tnctx, Jc, beta)
        ctx.save_for_backward(Jc)
        ctx.tnctx, ctx.beta, ctx.n_data = tnctx, beta, n_data
        ctx.state_id = tnctx.state_id
        return torch.tensor(lnz, dtype=torch.float64, device=J.device)

    @staticmethod
    def backward(ctx, g):
        (J,) = ctx.saved_tensors
        if ctx.tnctx.state_id != ctx.state_id:
            # another evaluation ran on this context after this forward pass: recompute it
            _LogZFromCouplings._evaluate(ctx.tnctx, J, ctx.beta)
        dT = torch.empty(ctx.n_data, dtype=torch.float64, device=J.device)
        dJ = torch.empty_like(J)
        torch.cuda.current_stream().synchronize()
        ctx.tnctx.tn_grad_device(dT.data_ptr())
        ctx.tnctx.tn_ising_coupling_grad_device(ctx.beta, J.data_ptr(), dT.data_ptr(), dJ.data_ptr())
        ctx.tnctx.tn_sync()
        return g * dJ, None, None, None


class _Planned:
    def __init__(self, n: int, edges: Sequence[Tuple[int, int, int]], offsets, pairs, chi: int,
                 precision: str = "fp64", cutoff: float = 0.0, checkpoint_segments: int = 0):
        eu = np.array([e[0] for e in edges], dtype=np.int32)
        ev = np.array([e[1] for e in edges], dtype=np.int32)
        ed = np.array([e[2] for e in edges], dtype=np.int32)
        self.offsets = np.asarray(offsets, dtype=np.int64)
        self.n_data = int(self.offsets[-1])
        self.ctx = Context(torch.cuda.current_device())
        self.ctx.tn_load_graph(n, eu, ev, ed, self.offsets, np.zeros(self.n_data))
        self.ctx.tn_set_tree([a for a, _ in pairs], [b for _, b in pairs], chi, precision=precision,
                             cutoff=cutoff, grad=True, checkpoint_segments=checkpoint_segments)

    def close(self) -> None:
        self.ctx.close()


class TensorLogZ(_Planned):
    """ln|Z| of a fixed graph and tree as a differentiable function of its flattened tensor data."""

    def __call__(self, data: torch.Tensor) -> torch.Tensor:
        if data.dtype != torch.float64 or data.numel() != self.n_data or not data.is_cuda:
            raise ValueError(f"data must be a float64 device tensor of {self.n_data} entries")
        return _LogZFromData.apply(data, self.ctx)


class IsingLogZ(_Planned):
    """ln|Z| of the Ising model on a graph with dimension-2 edges, differentiable in J."""

    def __init__(self, n: int, edges, pairs, chi: int, beta: float, precision: str = "fp64", cutoff: float = 0.0,
                 checkpoint_segments: int = 0):
        deg = np.zeros(n, dtype=np.int64)
        for u, v, d in edges:
            if d != 2:
                raise ValueError("Ising edges have dimension 2")
            deg[u] += 1
            deg[v] += 1
        offsets = np.zeros(n + 1, dtype=np.int64)
        offsets[1:] = np.cumsum(2 ** deg)
        super().__init__(n, edges, offsets, pairs, chi, precision, cutoff, checkpoint_segments)
        self.beta = float(beta)
        self.n_edges = len(edges)

    def __call__(self, J: torch.Tensor) -> torch.Tensor:
        if J.dtype != torch.float64 or J.numel() != self.n_edges or not J.is_cuda:
            raise ValueError(f"J must be a float64 device tensor of {self.n_edges} couplings")
        return _LogZFromCouplings.apply(J, self.ctx, self.beta, self.n_data)
