"""Autograd form of the Ozaki-II p-bit product: C = A B with a hand-written backward.

PyTorch lets only floating tensors carry gradients, so differentiable p-bit
matrices travel as float64 carriers ([rows, cols, 2 + 2 ceil(p/64)], the
encoding of oz2h_carrier_pack: slot 0 a readable double approximation, the
other slots exact integers holding sign, exponent and limbs).  Every product,
forward and backward, runs in the library's kernels:

  forward   C = A B                                   (oz2h_gemm)
  backward  dA = W B^T,  dB = A^T W   for W = dL/dC   (Ozaki-II products)

Two backward strategies:
  "reuse"      the forward runs on a plan of oz2h_plan_create_grad and its
               workspace (shared exponents e, f and the integer residue planes
               of A and B) is kept; the backward folds 2^(f_j) / 2^(e_i) into W
               and reads the saved planes transposed (oz2h_gemm_backward).
  "recompute"  only the input carriers are kept; the backward runs two plain
               products with transposed operands, W B^T and A^T W, which
               re-integerize B^T per row of B and A^T per column of A.
  "auto"       reuse when the saved workspace fits in `reuse_budget` bytes
               (default: a quarter of the free device memory), else recompute.

Carriers must reach the backward unchanged: a carrier that went through
floating-point arithmetic (for example gradient accumulation when C feeds two
consumers) is rejected with an error.
"""
from __future__ import annotations

import threading
from typing import Optional

import torch

from . import oz2h

_plans = {}
_lock = threading.Lock()


def _plan(kind: str, p: int, M: int, N: int, K: int, opts: Optional[oz2h.Opts]):
    o = opts or oz2h.default_opts()
    key = (kind, p, M if kind == "grad" else 0, N if kind == "grad" else 0, K,
           o.guard_bits, o.t_bits, o.crt_margin, o.tile, torch.cuda.current_device())
    with _lock:
        pl = _plans.get(key)
        if pl is None:
            pl = (oz2h.Plan.create_grad(p, M, N, K, o) if kind == "grad"
                  else oz2h.Plan.create(p, K, o))
            _plans[key] = pl
        return pl


def to_carrier(X) -> torch.Tensor:
    """Float64 carrier of a p-bit matrix (a DeviceMP, or host arrays such as synth.MPMatrix)."""
    if not isinstance(X, oz2h.DeviceMP):
        X = oz2h.to_device(X)
    return oz2h.carrier_pack(X)


def from_carrier(car: torch.Tensor, p: int, check: bool = True) -> oz2h.DeviceMP:
    """DeviceMP from a float64 carrier; raises if an element is not a valid encoding."""
    bad = torch.zeros(1, dtype=torch.int32, device=car.device) if check else None
    X = oz2h.carrier_unpack(car.detach(), p, bad)
    if check and int(bad.item()):
        raise ValueError("carrier holds an invalid p-bit encoding (was it changed by "
                         "floating-point arithmetic, e.g. gradient accumulation?)")
    return X


class OzMatmulFn(torch.autograd.Function):
    """C = A B on float64 carriers of p-bit matrices (A M x K, B K x N)."""

    @staticmethod
    def forward(ctx, a, b, p: int, mode: str, opts, reuse_budget):
        A = from_carrier(a, p)
        B = from_carrier(b, p)
        M, K = A.shape
        K2, N = B.shape
        if K != K2:
            raise ValueError(f"inner dimensions differ: {K} vs {K2}")
        if mode not in ("auto", "reuse", "recompute"):
            raise ValueError(f"mode must be auto, reuse or recompute, not {mode!r}")
        ctx.p, ctx.shape, ctx.opts = p, (M, N, K), opts
        if mode == "auto":
            mode = "recompute"
            if M * N * K:
                plan = _plan("grad", p, M, N, K, opts)
                budget = reuse_budget
                if budget is None:
                    budget = torch.cuda.mem_get_info(a.device)[0] // 4
                if plan.workspace_size(M, N) + plan.backward_workspace_size() <= budget:
                    mode = "reuse"
        if M * N * K == 0:
            mode = "recompute"
        ctx.mode = mode
        if mode == "reuse":
            plan = _plan("grad", p, M, N, K, opts)
            ws = oz2h.workspace(plan, M, N, device=a.device)
            C = oz2h.gemm(plan, A, B, ws=ws)
            ctx.plan, ctx.saved_ws = plan, ws
        else:
            C = oz2h.gemm(_plan("fwd", p, M, N, max(K, 1), opts), A, B)
            ctx.save_for_backward(a, b)
        return oz2h.carrier_pack(C)

    @staticmethod
    def backward(ctx, dc):
        p, (M, N, K) = ctx.p, ctx.shape
        need_a, need_b = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if dc.shape != (M, N, oz2h.carrier_width(p)):
            raise ValueError(f"upstream gradient has shape {tuple(dc.shape)}")
        W = from_carrier(dc, p)
        dA = dB = None
        if ctx.mode == "reuse":
            dA, dB = oz2h.gemm_backward(ctx.plan, ctx.saved_ws, W, need_a, need_b)
        else:
            a, b = ctx.saved_tensors
            if need_a:
                B = from_carrier(b, p, check=False)
                dA = oz2h.gemm(_plan("fwd", p, M, K, max(N, 1), ctx.opts), W, B, oz2h.OP_N,
                               oz2h.OP_T)
            if need_b:
                A = from_carrier(a, p, check=False)
                dB = oz2h.gemm(_plan("fwd", p, K, N, max(M, 1), ctx.opts), A, W, oz2h.OP_T,
                               oz2h.OP_N)
        ga = oz2h.carrier_pack(dA) if dA is not None else None
        gb = oz2h.carrier_pack(dB) if dB is not None else None
        return ga, gb, None, None, None, None


def oz_matmul(a: torch.Tensor, b: torch.Tensor, p: int, mode: str = "auto",
              opts: Optional[oz2h.Opts] = None, reuse_budget: Optional[int] = None) -> torch.Tensor:
    """Differentiable p-bit product of two float64 carriers; returns C's carrier."""
    return OzMatmulFn.apply(a, b, p, mode, opts, reuse_budget)
