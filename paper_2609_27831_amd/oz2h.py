"""Python binding of liboz2h.so (include/oz2h.h): argument marshalling only.

Every step of the product runs in the library's HIP kernels; PyTorch only
provides device memory and the current stream.  If the built library is
missing, every call raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liboz2h.so")

OK, EINVAL, ERANGE, ENOMEM, EDEVICE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
OP_N, OP_T = 0, 1


class Oz2hError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"oz2h error {code}: {msg}")
        self.code = code


TILE_AUTO, TILE_128x128, TILE_256x128, TILE_128x256 = 0, 1, 2, 3
# option flags: the matrix-core variants of stage 2 (residues) and stage 4 (CRT)
FLAG_RESIDUES_MMA, FLAG_CRT_MMA = 0x1, 0x2
FLAG_BACKEND_F64, FLAG_BACKEND_MIXED = 0x4, 0x8
TILE_SHAPES = {TILE_128x128: (128, 128), TILE_256x128: (256, 128), TILE_128x256: (128, 256)}


class Opts(ctypes.Structure):
    _fields_ = [("guard_bits", ctypes.c_int32), ("t_bits", ctypes.c_int32),
                ("crt_margin", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class CMat(ctypes.Structure):
    _fields_ = [("limbs", ctypes.c_void_p), ("exp", ctypes.c_void_p),
                ("sign", ctypes.c_void_p), ("ld", ctypes.c_int64)]


class Mat(ctypes.Structure):
    _fields_ = [("limbs", ctypes.c_void_p), ("exp", ctypes.c_void_p),
                ("sign", ctypes.c_void_p), ("ld", ctypes.c_int64)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("t", ctypes.c_int32), ("K", ctypes.c_int64),
                ("L", ctypes.c_int32), ("L1", ctypes.c_int32), ("L2", ctypes.c_int32),
                ("G", ctypes.c_int32), ("nw32", ctypes.c_int32), ("nd32", ctypes.c_int32),
                ("log2P", ctypes.c_double), ("tw_a", ctypes.c_int32), ("tw_b", ctypes.c_int32),
                ("grad_M", ctypes.c_int64), ("grad_N", ctypes.c_int64),
                ("backend", ctypes.c_int32), ("Lf", ctypes.c_int32)]


class Problem(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("N", ctypes.c_int64), ("K", ctypes.c_int64),
                ("p", ctypes.c_int32), ("opA", ctypes.c_int32), ("opB", ctypes.c_int32),
                ("A", CMat), ("B", CMat), ("C", Mat)]


# (name, restype, argtypes) of every exported symbol
_P, _I32, _I64, _SZ, _D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
SIGNATURES = {
    "oz2h_opts_default": (None, [ctypes.POINTER(Opts)]),
    "oz2h_last_error": (ctypes.c_char_p, []),
    "oz2h_plan_moduli": (ctypes.c_int, [_I32, _I64, ctypes.POINTER(Opts), _P, _P, _P, _P, _P, _P]),
    "oz2h_plan_create": (ctypes.c_int, [_I32, _I64, ctypes.POINTER(Opts), ctypes.POINTER(_P)]),
    "oz2h_plan_create_custom": (ctypes.c_int, [_I32, _I32, _I64, _I32, _P, ctypes.POINTER(_P)]),
    "oz2h_plan_set_flags": (ctypes.c_int, [_P, ctypes.c_uint32]),
    "oz2h_plan_destroy": (None, [_P]),
    "oz2h_plan_get_info": (ctypes.c_int, [_P, ctypes.POINTER(PlanInfo)]),
    "oz2h_plan_get_moduli": (ctypes.c_int, [_P, _P]),
    "oz2h_plan_get_moduli32": (ctypes.c_int, [_P, _P]),
    "oz2h_plan_moduli32": (ctypes.c_int, [_I32, _I64, ctypes.POINTER(Opts), _P, _P, _P, _P, _P, _P]),
    "oz2h_gemm_workspace_size": (_SZ, [_P, _I64, _I64]),
    "oz2h_gemm": (ctypes.c_int, [_P, _I64, _I64, _I64, ctypes.c_int, CMat, ctypes.c_int, CMat,
                                 Mat, _P, _SZ, _P]),
    "oz2h_gemm_timed": (ctypes.c_int, [_P, _I64, _I64, _I64, ctypes.c_int, CMat, ctypes.c_int, CMat,
                                       Mat, _P, _SZ, _P, _P]),
    "oz2h_gemm_integers": (ctypes.c_int, [_P, _I64, _I64, _I64, ctypes.c_int, CMat, ctypes.c_int,
                                          CMat, _P, _P, _I32, _P, _P, _P, _SZ, _P]),
    "oz2h_plan_create_grad": (ctypes.c_int, [_I32, _I64, _I64, _I64, ctypes.POINTER(Opts),
                                             ctypes.POINTER(_P)]),
    "oz2h_gemm_backward_workspace_size": (_SZ, [_P]),
    "oz2h_gemm_backward": (ctypes.c_int, [_P, _I64, _I64, _I64, _P, _SZ, CMat, ctypes.POINTER(Mat),
                                          ctypes.POINTER(Mat), _P, _SZ, _P]),
    "oz2h_carrier_pack": (ctypes.c_int, [_I64, _I64, _I32, CMat, _P, _P]),
    "oz2h_carrier_unpack": (ctypes.c_int, [_I64, _I64, _I32, _P, Mat, _P, _P]),
    "oz2h_exponents": (ctypes.c_int, [_I64, _I64, _P, _P, _I64, _I64, _P, _P]),
    "oz2h_residues": (ctypes.c_int, [_P, _I64, _I64, _P, _P, _P, _I64, _I64, _P, _I64, _I64, _P, _P]),
    "oz2h_residue_gemm": (ctypes.c_int, [_P, _I64, _I64, _I64, _P, _P, _P, _P]),
    "oz2h_i8gemm": (ctypes.c_int, [_I64, _I64, _I64, _P, _P, _P, _I32, _P]),
    "oz2h_crt": (ctypes.c_int, [_P, _I64, _I64, _P, _I64, _I64, _P, _P, _I32, _P, _SZ, _P]),
    "oz2h_crt_workspace_size": (_SZ, [_P, _I64, _I64]),
    "oz2h_residues_create": (ctypes.c_int, [_P, _I32, _I64, ctypes.c_int, CMat, _P, ctypes.POINTER(_P)]),
    "oz2h_gemm_from_residues": (ctypes.c_int, [_P, _I64, _I64, _I64, _P, ctypes.c_int, CMat, _P,
                                               ctypes.c_int, CMat, Mat, _P, _SZ, _P]),
    "oz2h_residues_destroy": (None, [_P]),
    "oz2h_zgemm_workspace_size": (_SZ, [_P, _I32, _I64, _I64]),
    "oz2h_zgemm": (ctypes.c_int, [_P, _I32, _I64, _I64, _I64, ctypes.c_int, CMat, CMat, ctypes.c_int,
                                  CMat, CMat, Mat, Mat, _P, _SZ, _P]),
    "oz2h_gemm_noalloc_max_bytes": (_SZ, []),
    "oz2h_gemm_noalloc": (ctypes.c_int, [_P, _I64, _I64, _I64, ctypes.c_int, CMat, ctypes.c_int, CMat,
                                         Mat, _P]),
    "oz2h_batched_plan_create": (ctypes.c_int, [_I32, _P, ctypes.POINTER(Opts), ctypes.POINTER(_P)]),
    "oz2h_batched_workspace_size": (_SZ, [_P]),
    "oz2h_batched_tune": (ctypes.c_int, [_P, _P, _SZ, _P]),
    "oz2h_batched_run": (ctypes.c_int, [_P, _P, _SZ, _P]),
    "oz2h_batched_run_eager": (ctypes.c_int, [_P, _P, _SZ, _P]),
    "oz2h_batched_get_config": (ctypes.c_int, [_P, _P, _P, _P]),
    "oz2h_batched_set_config": (ctypes.c_int, [_P, _I32, _I32]),
    "oz2h_batched_get_schedule": (ctypes.c_int, [_P, _P, _P]),
    "oz2h_batched_set_schedule": (ctypes.c_int, [_P, _I32, _I32]),
    "oz2h_batched_plan_destroy": (None, [_P]),
}

_lib = None


def lib():
    """Load the in-tree library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is missing: run "
                               "`python -m paper_2609_27831_amd.build` (or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code: int):
    if code != OK:
        raise Oz2hError(code, lib().oz2h_last_error().decode())


def default_opts(guard_bits: Optional[int] = None, t_bits: Optional[int] = None,
                 crt_margin: Optional[int] = None, tile: Optional[int] = None,
                 flags: Optional[int] = None) -> Opts:
    o = Opts()
    lib().oz2h_opts_default(ctypes.byref(o))
    if flags is not None:
        o.flags = flags
    if tile is not None:
        o.tile = tile
    if guard_bits is not None:
        o.guard_bits = guard_bits
    if t_bits is not None:
        o.t_bits = t_bits
    if crt_margin is not None:
        o.crt_margin = crt_margin
    return o


def plan_moduli(p: int, K: int, opts: Optional[Opts] = None):
    """Host-only moduli selection: dict(L, L1, G, t, log2P, moduli)."""
    L, L1, G, t = (ctypes.c_int32() for _ in range(4))
    lp = ctypes.c_double()
    o = opts or default_opts()
    _check(lib().oz2h_plan_moduli(p, K, ctypes.byref(o), ctypes.addressof(L), ctypes.addressof(L1),
                                  ctypes.addressof(G), ctypes.addressof(t), ctypes.addressof(lp), None))
    mods = np.zeros(L.value, np.uint16)
    _check(lib().oz2h_plan_moduli(p, K, ctypes.byref(o), None, None, None, None, None,
                                  mods.ctypes.data))
    return {"L": L.value, "L1": L1.value, "G": G.value, "t": t.value, "log2P": lp.value,
            "moduli": mods}


def plan_moduli32(p: int, K: int, opts: Optional[Opts] = None):
    """Host-only moduli selection of any backend: dict(L, L8, G, t, log2P, moduli)."""
    L, L8, G, t = (ctypes.c_int32() for _ in range(4))
    lp = ctypes.c_double()
    o = opts or default_opts()
    _check(lib().oz2h_plan_moduli32(p, K, ctypes.byref(o), ctypes.addressof(L), ctypes.addressof(L8),
                                    ctypes.addressof(G), ctypes.addressof(t), ctypes.addressof(lp), None))
    mods = np.zeros(L.value, np.uint32)
    _check(lib().oz2h_plan_moduli32(p, K, ctypes.byref(o), None, None, None, None, None,
                                    mods.ctypes.data))
    return {"L": L.value, "L8": L8.value, "G": G.value, "t": t.value, "log2P": lp.value,
            "moduli": mods}


class Plan:
    """Moduli set + device constant tables for one (p, K) on the current device."""

    def __init__(self, handle: int):
        self.handle = handle
        info = PlanInfo()
        _check(lib().oz2h_plan_get_info(handle, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in PlanInfo._fields_}
        mods = np.zeros(self.info["L"], np.uint32)
        _check(lib().oz2h_plan_get_moduli32(handle, mods.ctypes.data))
        self.moduli = mods if self.info["backend"] else mods.astype(np.uint16)

    @classmethod
    def create(cls, p: int, K: int, opts: Optional[Opts] = None) -> "Plan":
        h = ctypes.c_void_p()
        o = opts or default_opts()
        _check(lib().oz2h_plan_create(p, K, ctypes.byref(o), ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def create_grad(cls, p: int, M: int, N: int, K: int, opts: Optional[Opts] = None) -> "Plan":
        """Plan of an M x K by K x N product that also serves its backward products."""
        h = ctypes.c_void_p()
        o = opts or default_opts()
        _check(lib().oz2h_plan_create_grad(p, M, N, K, ctypes.byref(o), ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def custom(cls, p: int, t: int, K: int, moduli: Sequence[int]) -> "Plan":
        m = np.ascontiguousarray(moduli, dtype=np.uint16)
        h = ctypes.c_void_p()
        _check(lib().oz2h_plan_create_custom(p, t, K, m.size, m.ctypes.data, ctypes.byref(h)))
        return cls(h.value)

    def __getattr__(self, k):
        info = self.__dict__.get("info")
        if info is not None and k in info:
            return info[k]
        raise AttributeError(k)

    def set_flags(self, flags: int) -> "Plan":
        """Select the stage-2 / stage-4 kernel variants (FLAG_* bits)."""
        _check(lib().oz2h_plan_set_flags(self.handle, flags))
        return self

    def workspace_size(self, M: int, N: int) -> int:
        return int(lib().oz2h_gemm_workspace_size(self.handle, M, N))

    def backward_workspace_size(self) -> int:
        return int(lib().oz2h_gemm_backward_workspace_size(self.handle))

    def destroy(self):
        if self.handle:
            lib().oz2h_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


# ------------------------------------------------------------------ device data

@dataclass
class DeviceMP:
    """A p-bit matrix in device memory (torch tensors), rows x cols, row-major."""
    sign: "object"   # torch.int8 [rows, ld]
    exp: "object"    # torch.int32 [rows, ld]
    limbs: "object"  # torch.int64 [rows, ld, nl] (bit pattern of uint64)
    p: int

    @property
    def shape(self):
        return tuple(self.sign.shape)

    @property
    def ld(self) -> int:
        return int(self.sign.stride(0))

    def cmat(self) -> CMat:
        return CMat(self.limbs.data_ptr(), self.exp.data_ptr(), self.sign.data_ptr(), self.ld)

    def mat(self) -> Mat:
        return Mat(self.limbs.data_ptr(), self.exp.data_ptr(), self.sign.data_ptr(), self.ld)

    def to_host(self):
        """-> synth.MPMatrix-like numpy arrays (sign, exp, limbs as uint64)."""
        s = self.sign.cpu().numpy()
        e = self.exp.cpu().numpy()
        l = self.limbs.cpu().numpy().view(np.uint64)
        return s, e, l


def _torch():
    import torch
    return torch


def to_device(X, device="cuda") -> DeviceMP:
    """Copy a host operand (sign/exp/limbs numpy arrays, e.g. synth.MPMatrix) to the GPU."""
    torch = _torch()
    return DeviceMP(torch.from_numpy(np.ascontiguousarray(X.sign)).to(device),
                    torch.from_numpy(np.ascontiguousarray(X.exp)).to(device),
                    torch.from_numpy(np.ascontiguousarray(X.limbs).view(np.int64)).to(device),
                    X.p)


def empty_mp(rows: int, cols: int, p: int, device="cuda") -> DeviceMP:
    torch = _torch()
    nl = (p + 63) // 64
    return DeviceMP(torch.empty((rows, cols), dtype=torch.int8, device=device),
                    torch.empty((rows, cols), dtype=torch.int32, device=device),
                    torch.empty((rows, cols, nl), dtype=torch.int64, device=device), p)


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _keep_for(stream, *tensors):
    """Tensors this module allocated on the current stream but handed to a launch on
    another stream: tell the caching allocator, so that their memory is not reused
    before that stream's work is done."""
    if stream is None:
        return
    torch = _torch()
    if stream == torch.cuda.current_stream(stream.device):
        return
    for t in tensors:
        if t is not None:
            t.record_stream(stream)


def workspace(plan: Plan, M: int, N: int, device="cuda"):
    torch = _torch()
    n = plan.workspace_size(M, N)
    return torch.empty(max(n, 256), dtype=torch.uint8, device=device)


def _dims(A: DeviceMP, B: DeviceMP, opA: int, opB: int):
    M, K = A.shape if opA == OP_N else A.shape[::-1]
    K2, N = B.shape if opB == OP_N else B.shape[::-1]
    if K != K2:
        raise ValueError(f"inner dimensions differ: {K} vs {K2}")
    return M, N, K


def gemm(plan: Plan, A: DeviceMP, B: DeviceMP, opA: int = OP_N, opB: int = OP_N,
         out: Optional[DeviceMP] = None, ws=None, stream=None) -> DeviceMP:
    """C = op(A) op(B) at the plan's precision (oz2h_gemm)."""
    M, N, K = _dims(A, B, opA, opB)
    new_out, new_ws = out is None, ws is None
    if out is None:
        out = empty_mp(M, N, plan.p, device=A.sign.device)
    if ws is None:
        ws = workspace(plan, M, N, device=A.sign.device)
    _check(lib().oz2h_gemm(plan.handle, M, N, K, opA, A.cmat(), opB, B.cmat(), out.mat(),
                           ws.data_ptr(), ws.numel(), _stream_ptr(stream)))
    if new_out:
        _keep_for(stream, out.sign, out.exp, out.limbs)
    if new_ws:
        _keep_for(stream, ws)
    return out


ZGEMM_3M, ZGEMM_4M = 3, 4


def zgemm(plan: Plan, Ar: DeviceMP, Ai: DeviceMP, Br: DeviceMP, Bi: DeviceMP, scheme: int = ZGEMM_3M,
          opA: int = OP_N, opB: int = OP_N, out=None, ws=None, stream=None):
    """(Re C, Im C) of C = op(A) op(B), A = Ar + i Ai, B = Br + i Bi (oz2h_zgemm); the plan
    is built for contraction length 2K.  out: optional (Cr, Ci) pair."""
    M, N, K = _dims(Ar, Br, opA, opB)
    if _dims(Ai, Bi, opA, opB) != (M, N, K):
        raise ValueError("real and imaginary parts differ in shape")
    new_out, new_ws = out is None, ws is None
    dev = Ar.sign.device
    if out is None:
        out = (empty_mp(M, N, plan.p, device=dev), empty_mp(M, N, plan.p, device=dev))
    if ws is None:
        torch = _torch()
        n = lib().oz2h_zgemm_workspace_size(plan.handle, scheme, M, N)
        ws = torch.empty(max(n, 256), dtype=torch.uint8, device=dev)
    Cr, Ci = out
    _check(lib().oz2h_zgemm(plan.handle, scheme, M, N, K, opA, Ar.cmat(), Ai.cmat(), opB, Br.cmat(),
                            Bi.cmat(), Cr.mat(), Ci.mat(), ws.data_ptr(), ws.numel(),
                            _stream_ptr(stream)))
    if new_out:
        for C in out:
            _keep_for(stream, C.sign, C.exp, C.limbs)
    if new_ws:
        _keep_for(stream, ws)
    return Cr, Ci


SIDE_A, SIDE_B = 0, 1


class Residues:
    """Stages 1-2 of one operand kept on the device (oz2h_residues_create), for operand
    reuse: side SIDE_A (X is op(A), rows x K) or SIDE_B (X is op(B), K x rows)."""

    def __init__(self, plan: Plan, X: "DeviceMP", side: int, op: int = OP_N, stream=None):
        r, c = X.shape
        rows_first = (side == SIDE_A) == (op == OP_N)
        rows = r if rows_first else c
        h = ctypes.c_void_p()
        _check(lib().oz2h_residues_create(plan.handle, side, rows, op, X.cmat(), _stream_ptr(stream),
                                          ctypes.byref(h)))
        self.handle, self.side, self.rows = h.value, side, rows

    def destroy(self):
        if self.handle:
            lib().oz2h_residues_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _empty_cmat() -> CMat:
    return CMat(None, None, None, 1)


def gemm_from_residues(plan: Plan, A=None, B=None, ra: Optional[Residues] = None,
                       rb: Optional[Residues] = None, opA: int = OP_N, opB: int = OP_N,
                       M: Optional[int] = None, N: Optional[int] = None,
                       out: Optional["DeviceMP"] = None, ws=None, stream=None) -> "DeviceMP":
    """C = op(A) op(B) with side A from `ra` and/or side B from `rb` (oz2h_gemm_from_residues)."""
    K = plan.K
    if ra is not None:
        M = ra.rows
    elif M is None:
        M = A.shape[0] if opA == OP_N else A.shape[1]
    if rb is not None:
        N = rb.rows
    elif N is None:
        N = B.shape[1] if opB == OP_N else B.shape[0]
    dev = (A.sign.device if A is not None else B.sign.device if B is not None else "cuda")
    new_out, new_ws = out is None, ws is None
    if out is None:
        out = empty_mp(M, N, plan.p, device=dev)
    if ws is None:
        ws = workspace(plan, M, N, device=dev)
    _check(lib().oz2h_gemm_from_residues(plan.handle, M, N, K, ra.handle if ra else None, opA,
                                         A.cmat() if A is not None else _empty_cmat(),
                                         rb.handle if rb else None, opB,
                                         B.cmat() if B is not None else _empty_cmat(), out.mat(),
                                         ws.data_ptr(), ws.numel(), _stream_ptr(stream)))
    if new_out:
        _keep_for(stream, out.sign, out.exp, out.limbs)
    if new_ws:
        _keep_for(stream, ws)
    return out


def gemm_noalloc(plan: Plan, A: DeviceMP, B: DeviceMP, opA: int = OP_N, opB: int = OP_N,
                 out: DeviceMP = None, stream=None) -> DeviceMP:
    """oz2h_gemm_noalloc: the library's static per-device scratch instead of a workspace.
    `out` must be given by callers that allocate nothing themselves."""
    M, N, K = _dims(A, B, opA, opB)
    new_out = out is None
    if out is None:
        out = empty_mp(M, N, plan.p, device=A.sign.device)
    _check(lib().oz2h_gemm_noalloc(plan.handle, M, N, K, opA, A.cmat(), opB, B.cmat(), out.mat(),
                                   _stream_ptr(stream)))
    if new_out:
        _keep_for(stream, out.sign, out.exp, out.limbs)
    return out


def gemm_timed(plan: Plan, A: DeviceMP, B: DeviceMP, out: DeviceMP, ws, events_array,
               opA: int = OP_N, opB: int = OP_N, stream=None) -> DeviceMP:
    """oz2h_gemm recording five stage events (a ctypes array of hipEvent_t)."""
    M, N, K = _dims(A, B, opA, opB)
    _check(lib().oz2h_gemm_timed(plan.handle, M, N, K, opA, A.cmat(), opB, B.cmat(), out.mat(),
                                 ws.data_ptr(), ws.numel(), _stream_ptr(stream),
                                 ctypes.cast(events_array, ctypes.c_void_p)))
    return out


def gemm_integers(plan: Plan, A: DeviceMP, B: DeviceMP, opA: int = OP_N, opB: int = OP_N,
                  nlc: Optional[int] = None, ws=None, stream=None):
    """Exact c^ (sign, magnitude limbs) and shared exponents e, f (oz2h_gemm_integers)."""
    torch = _torch()
    M, N, K = _dims(A, B, opA, opB)
    dev = A.sign.device
    if nlc is None:
        nlc = (int(np.ceil(plan.log2P)) + 1 + 63) // 64
    cs = torch.empty((M, N), dtype=torch.int8, device=dev)
    cm = torch.empty((M, N, nlc), dtype=torch.int64, device=dev)
    e = torch.empty(M, dtype=torch.int32, device=dev)
    f = torch.empty(N, dtype=torch.int32, device=dev)
    new_ws = ws is None
    if ws is None:
        ws = workspace(plan, M, N, device=dev)
    _check(lib().oz2h_gemm_integers(plan.handle, M, N, K, opA, A.cmat(), opB, B.cmat(),
                                    cs.data_ptr(), cm.data_ptr(), nlc, e.data_ptr(), f.data_ptr(),
                                    ws.data_ptr(), ws.numel(), _stream_ptr(stream)))
    _keep_for(stream, cs, cm, e, f, ws if new_ws else None)
    return cs, cm, e, f


def exponents(sign, exp, rows: int, count: int, rs: int, cs: int, out=None, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty(rows, dtype=torch.int32, device=sign.device)
    _check(lib().oz2h_exponents(rows, count, sign.data_ptr(), exp.data_ptr(), rs, cs,
                                out.data_ptr(), _stream_ptr(stream)))
    return out


def residues(plan: Plan, X: DeviceMP, erow, side: str, rpad: int, kpad: int, stream=None):
    """Stage-2 planes of one side: side 'A' (rows of X own the exponent) or 'B' (columns)."""
    torch = _torch()
    r, c = X.shape
    if side == "A":
        rows, count, rs, cs = r, c, X.ld, 1
    else:
        rows, count, rs, cs = c, r, 1, X.ld
    planes = torch.empty((plan.G, rpad, kpad), dtype=torch.int8, device=X.sign.device)
    _check(lib().oz2h_residues(plan.handle, rows, count, X.limbs.data_ptr(), X.exp.data_ptr(),
                               X.sign.data_ptr(), rs, cs, erow.data_ptr(), rpad, kpad,
                               planes.data_ptr(), _stream_ptr(stream)))
    return planes


def residue_gemm(plan: Plan, a_planes, b_planes, stream=None):
    torch = _torch()
    G, mpad, kpad = a_planes.shape
    G2, npad, kpad2 = b_planes.shape
    assert G == G2 == plan.G and kpad == kpad2
    u = torch.empty((plan.L, mpad, npad), dtype=torch.int16, device=a_planes.device)
    _check(lib().oz2h_residue_gemm(plan.handle, mpad, npad, kpad, a_planes.data_ptr(),
                                   b_planes.data_ptr(), u.data_ptr(), _stream_ptr(stream)))
    return u


def i8gemm(A, B, tile: int = TILE_AUTO, stream=None):
    torch = _torch()
    M, K = A.shape
    N, K2 = B.shape
    assert K == K2
    C = torch.empty((M, N), dtype=torch.int32, device=A.device)
    _check(lib().oz2h_i8gemm(M, N, K, A.data_ptr(), B.data_ptr(), C.data_ptr(), tile,
                             _stream_ptr(stream)))
    return C


def crt(plan: Plan, u, M: int, N: int, nlc: Optional[int] = None, stream=None, ws=None):
    """u: uint16 planes as a torch int16 tensor [L, rows, ld].  ws: None (no workspace),
    "auto" (allocate oz2h_crt_workspace_size bytes), or a device uint8 tensor."""
    torch = _torch()
    L, rows, ldu = u.shape
    if nlc is None:
        nlc = (int(np.ceil(plan.log2P)) + 1 + 63) // 64
    cs = torch.empty((M, N), dtype=torch.int8, device=u.device)
    cm = torch.empty((M, N, nlc), dtype=torch.int64, device=u.device)
    if isinstance(ws, str) and ws == "auto":
        n = int(lib().oz2h_crt_workspace_size(plan.handle, M, ldu))
        ws = torch.empty(max(n, 256), dtype=torch.uint8, device=u.device) if n else None
    wp, wn = (ws.data_ptr(), ws.numel()) if ws is not None else (None, 0)
    _check(lib().oz2h_crt(plan.handle, M, N, u.data_ptr(), ldu, rows * ldu, cs.data_ptr(),
                          cm.data_ptr(), nlc, wp, wn, _stream_ptr(stream)))
    _keep_for(stream, cs, cm)
    return cs, cm


def gemm_backward(plan: Plan, saved, W: DeviceMP, want_a: bool = True, want_b: bool = True,
                  dA: Optional[DeviceMP] = None, dB: Optional[DeviceMP] = None, ws=None,
                  stream=None):
    """dA = W B^T and dB = A^T W from the forward's saved workspace (oz2h_gemm_backward).

    `saved` is the workspace tensor of a completed gemm() with this grad plan."""
    torch = _torch()
    M, N = W.shape
    K = plan.K
    dev = W.sign.device
    fresh = []
    if want_a and dA is None:
        dA = empty_mp(M, K, plan.p, device=dev)
        fresh += [dA.sign, dA.exp, dA.limbs]
    if want_b and dB is None:
        dB = empty_mp(K, N, plan.p, device=dev)
        fresh += [dB.sign, dB.exp, dB.limbs]
    if ws is None:
        ws = torch.empty(max(plan.backward_workspace_size(), 256), dtype=torch.uint8, device=dev)
        fresh.append(ws)
    ma = ctypes.byref(dA.mat()) if want_a else None
    mb = ctypes.byref(dB.mat()) if want_b else None
    _check(lib().oz2h_gemm_backward(plan.handle, M, N, K, saved.data_ptr(), saved.numel(),
                                    W.cmat(), ma, mb, ws.data_ptr(), ws.numel(),
                                    _stream_ptr(stream)))
    _keep_for(stream, *fresh)
    return (dA if want_a else None), (dB if want_b else None)


def carrier_width(p: int) -> int:
    """Doubles per element of a float64 carrier: 2 + 2 ceil(p/64)."""
    return 2 + 2 * ((p + 63) // 64)


def carrier_pack(X: DeviceMP, out=None, stream=None):
    """Float64 carrier [rows, cols, 2 + 2 nl] of a p-bit matrix (oz2h_carrier_pack)."""
    torch = _torch()
    r, c = X.shape
    if out is None:
        out = torch.empty((r, c, carrier_width(X.p)), dtype=torch.float64, device=X.sign.device)
    if out.shape != (r, c, carrier_width(X.p)) or not out.is_contiguous():
        raise ValueError("carrier must be a contiguous [rows, cols, 2 + 2 nl] float64 tensor")
    _check(lib().oz2h_carrier_pack(r, c, X.p, X.cmat(), out.data_ptr(), _stream_ptr(stream)))
    return out


def carrier_unpack(car, p: int, bad=None, stream=None) -> DeviceMP:
    """p-bit matrix from a float64 carrier (oz2h_carrier_unpack); `bad` is an optional
    device int32 tensor that receives 1 if an element is not a valid encoding."""
    if car.dim() != 3 or car.shape[2] != carrier_width(p) or car.dtype != _torch().float64:
        raise ValueError(f"not a float64 carrier of {p}-bit numbers: {tuple(car.shape)}")
    car = car.contiguous()
    r, c = car.shape[0], car.shape[1]
    X = empty_mp(r, c, p, device=car.device)
    _check(lib().oz2h_carrier_unpack(r, c, p, car.data_ptr(), X.mat(),
                                     None if bad is None else bad.data_ptr(), _stream_ptr(stream)))
    return X


def limbs_to_ints(mag: np.ndarray, sign: np.ndarray):
    """Signed Python ints from (sign, uint64 magnitude limbs) arrays of any leading shape."""
    mag = mag.view(np.uint64)
    flat = mag.reshape(-1, mag.shape[-1])
    sg = sign.reshape(-1)
    out = []
    for row, s in zip(flat, sg):
        v = 0
        for x in row[::-1]:
            v = (v << 64) | int(x)
        out.append(int(s) * v)
    return out


# ------------------------------------------------------------------ batched form

class BatchedPlan:
    """Many independent products in one grouped pass per stage (oz2h_batched_*).

    problems: list of (A, B, C, opA, opB) with DeviceMP operands; each product
    runs at its operands' precision.  The device pointers are captured by the plan.
    """

    def __init__(self, problems, opts: Optional[Opts] = None):
        arr = (Problem * len(problems))()
        self._keep = problems   # the captured tensors must outlive the plan
        for i, (A, B, C, opA, opB) in enumerate(problems):
            M, N, K = _dims(A, B, opA, opB)
            if C.shape != (M, N) or A.p != B.p or C.p != A.p:
                raise ValueError(f"problem {i}: inconsistent shapes or precisions")
            arr[i] = Problem(M, N, K, A.p, opA, opB, A.cmat(), B.cmat(), C.mat())
        h = ctypes.c_void_p()
        o = opts or default_opts()
        _check(lib().oz2h_batched_plan_create(len(problems), arr, ctypes.byref(o), ctypes.byref(h)))
        self.handle = h.value
        self.count = len(problems)

    def workspace_size(self) -> int:
        return int(lib().oz2h_batched_workspace_size(self.handle))

    def workspace(self, device="cuda"):
        torch = _torch()
        return torch.empty(max(self.workspace_size(), 256), dtype=torch.uint8, device=device)

    def tune(self, ws, stream=None):
        _check(lib().oz2h_batched_tune(self.handle, ws.data_ptr(), ws.numel(), _stream_ptr(stream)))
        return self.config()

    def run(self, ws, stream=None):
        _check(lib().oz2h_batched_run(self.handle, ws.data_ptr(), ws.numel(), _stream_ptr(stream)))

    def run_eager(self, ws, stream=None):
        _check(lib().oz2h_batched_run_eager(self.handle, ws.data_ptr(), ws.numel(), _stream_ptr(stream)))

    def config(self):
        t, bc, n = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib().oz2h_batched_get_config(self.handle, ctypes.addressof(t), ctypes.addressof(bc),
                                             ctypes.addressof(n)))
        ns, g = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().oz2h_batched_get_schedule(self.handle, ctypes.addressof(ns), ctypes.addressof(g)))
        return {"tile": t.value, "blocks_per_cu": bc.value, "gemm_items": n.value,
                "gemm_stages": ns.value, "graph": bool(g.value)}

    def set_config(self, tile: int, blocks_per_cu: int):
        _check(lib().oz2h_batched_set_config(self.handle, tile, blocks_per_cu))

    def set_schedule(self, gemm_stages: int, graph: bool):
        _check(lib().oz2h_batched_set_schedule(self.handle, gemm_stages, int(graph)))

    def destroy(self):
        if self.handle:
            lib().oz2h_batched_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
