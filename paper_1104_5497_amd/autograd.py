"""Differentiable landscape objectives of one ring.

NPHCEnergies.apply(J, gamma) returns (E_min, S_min): the energy of the global
minimum and the sum of the energies of all certified minima (real,
nondegenerate stationary points of Hessian index 0).  Their gradients with
respect to the couplings come from the adjoint kernel (nphc_adjoint): at a
nonsingular stationary point z(J) the implicit-function theorem gives
dz/dJ = -F_z^{-1} dF/dJ, so dL/dJ = dL/dJ|_z - lambda^T dF/dJ with
F_z^T lambda = dL/dz (one transposed solve per minimum, float64).

J is read as the symmetric coupling matrix (J + J^T) / 2 with its diagonal
ignored, so dL/dJ_ab = dL/dJ_ba = (1/2) dL/dc_ab for the coupling c_ab.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L
from . import pipeline


def _sym(J: torch.Tensor) -> np.ndarray:
    Jn = J.detach().to("cpu", torch.float64).numpy()
    Jn = 0.5 * (Jn + Jn.T)
    np.fill_diagonal(Jn, 0.0)
    return Jn


def minima(res: dict):
    """Items, energies and the index of the global minimum among the
    certified minima of the first ring of a pipeline result."""
    s = res["systems"][0]
    sel = (s.index == 0) & ~s.degenerate
    items = s.real_items[sel]
    V = s.V[sel]
    if items.size == 0:
        raise ValueError("no certified minimum")
    return items, V, int(np.argmin(V))


def adjoint(batch: pipeline.Batch, bufs: pipeline.Buffers, items: np.ndarray, w_V: np.ndarray,
            g_z: np.ndarray | None = None, stream=None) -> np.ndarray:
    """dL/dc (N x N, symmetric, per coupling) for L = sum_i w_V[i] V(z_i)
    + sum_i <g_z[i], z_i> over the listed stationary points (item ids)."""
    order = np.argsort(items, kind="stable")
    ids = torch.from_numpy(np.ascontiguousarray(items[order], dtype=np.int64)).to(batch.device)
    w = torch.from_numpy(np.ascontiguousarray(np.asarray(w_V, np.float64)[order])).to(batch.device)
    gz = None
    if g_z is not None:
        g = np.asarray(g_z, np.float64)[order]          # (K, n)
        gz = torch.from_numpy(np.ascontiguousarray(g.T)).to(batch.device)  # planes of stride K
    N = int(batch.N_host[0])
    out = torch.zeros(int(batch.J.numel()), dtype=torch.float64, device=batch.device)
    s = pipeline._stream(stream)
    L.check(L.lib().nphc_adjoint(ctypes.byref(batch.c), pipeline._p(ids), ids.numel(), None,
                                 pipeline._p(bufs.z), batch.num_items, pipeline._p(w),
                                 pipeline._p(gz), pipeline._p(out), s), "nphc_adjoint")
    torch.cuda.current_stream().synchronize()
    return out[: N * N].cpu().numpy().reshape(N, N)


class NPHCEnergies(torch.autograd.Function):
    @staticmethod
    def forward(ctx, J: torch.Tensor, gamma: complex, precision: str = "fp32"):
        Jn = _sym(J)
        res = pipeline.find_all_sps(Jn, gamma, precision=precision)
        items, V, arg = minima(res)
        ctx.res = res
        ctx.items, ctx.arg = items, arg
        ctx.shape, ctx.dtype, ctx.device = J.shape, J.dtype, J.device
        E = torch.tensor(float(V[arg]), dtype=J.dtype, device=J.device)
        S = torch.tensor(float(np.sum(V)), dtype=J.dtype, device=J.device)
        return E, S

    @staticmethod
    def backward(ctx, gE, gS):
        items = ctx.items
        w = np.full(items.size, float(gS) if gS is not None else 0.0)
        if gE is not None:
            w[ctx.arg] += float(gE)
        G = adjoint(ctx.res["batch"], ctx.res["buffers"], items, w)
        grad = torch.from_numpy(0.5 * G).to(ctx.device, ctx.dtype)
        return grad, None, None
