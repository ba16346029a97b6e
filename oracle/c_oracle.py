"""ctypes front end of the plain-C oracle (oz2_oracle.c).

TEST INFRASTRUCTURE ONLY (tests, smoke(), bench.py's cpu_baseline leg).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oz2_oracle.c")
LIB = os.path.join(HERE, "liboz2oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc + OpenMP (plain C, no GPU code)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-shared", "-fPIC",
                               SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int
        L.oz2o_internal_width.argtypes = [i32, i64, i32, i32]
        L.oz2o_internal_width.restype = i32
        L.oz2o_num_threads.restype = i32
        L.oz2o_integerize.argtypes = [i64, i64, i32, i32, P, P, P, i64, i64, P, P, P, i32]
        L.oz2o_integerize.restype = i32
        L.oz2o_gemm.argtypes = [i64, i64, i64, i32, i32,
                                P, P, P, i64, i64, P, P, P, i64, i64,
                                i64, P, P, P, P, i32, P, P, P, P, P]
        L.oz2o_gemm.restype = i32
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def internal_width(p: int, K: int, guard_bits: int = 16, t_bits: int = 0) -> int:
    return lib().oz2o_internal_width(p, K, guard_bits, t_bits)


def num_threads() -> int:
    return lib().oz2o_num_threads()


def chat_limbs(t: int, K: int) -> int:
    """Limbs that always hold |c^| <= K 2^(2t) (Eq. 2 bound)."""
    return (2 * t + (K - 1).bit_length() + 1 + 63) // 64


def integerize(X, t: int, side: str = "A"):
    """Shared exponents and integer matrix of one operand (Eq. 1).

    side "A": rows of X own the exponent (X is M x K) -> (e[M], sign[M,K], mag[M,K,na]).
    side "B": columns of X own it (X is K x N)       -> (f[N], sign[N,K], mag[N,K,na]).
    """
    p = X.p
    r, c = X.sign.shape
    na = (t + 1 + 63) // 64
    if side == "A":
        rows, count, rs, cs = r, c, c, 1
    else:
        rows, count, rs, cs = c, r, 1, c
    e = np.zeros(rows, np.int32)
    sg = np.zeros((rows, count), np.int8)
    mag = np.zeros((rows, count, na), np.uint64)
    st = lib().oz2o_integerize(rows, count, p, t, _p(X.sign), _p(X.exp), _p(X.limbs),
                               rs, cs, _p(e), _p(sg), _p(mag), na)
    assert st == 0
    return e, sg, mag


def gemm(A, B, guard_bits: int = 16, t_bits: int = 0, sel=None,
         want_chat: bool = True, want_c: bool = True):
    """Reference product.  sel = (i_array, j_array) computes only those entries."""
    p = A.p
    M, K = A.sign.shape
    K2, N = B.sign.shape
    assert K == K2 and B.p == p
    t = internal_width(p, K, guard_bits, t_bits)
    nl = (p + 63) // 64
    nlc = chat_limbs(t, K)
    if sel is None:
        nout, si, sj = M * N, None, None
    else:
        si = np.ascontiguousarray(sel[0], dtype=np.int64)
        sj = np.ascontiguousarray(sel[1], dtype=np.int64)
        nout = si.size
    e = np.zeros(M, np.int32)
    f = np.zeros(N, np.int32)
    cm = np.zeros((nout, nlc), np.uint64) if want_chat else None
    cs = np.zeros(nout, np.int8) if want_chat else None
    os_ = np.zeros(nout, np.int8) if want_c else None
    oe = np.zeros(nout, np.int32) if want_c else None
    ol = np.zeros((nout, nl), np.uint64) if want_c else None
    st = lib().oz2o_gemm(M, N, K, p, t,
                         _p(A.sign), _p(A.exp), _p(A.limbs), K, 1,
                         _p(B.sign), _p(B.exp), _p(B.limbs), N, 1,
                         nout, _p(si), _p(sj), _p(e), _p(f),
                         nlc, _p(cm), _p(cs), _p(os_), _p(oe), _p(ol))
    if st != 0:
        raise RuntimeError(f"oracle failed with status {st}")
    out = {"t": t, "e": e, "f": f, "nlc": nlc}
    if want_chat:
        out["chat_mag"], out["chat_sign"] = cm, cs
    if want_c:
        out["c_sign"], out["c_exp"], out["c_limbs"] = os_, oe, ol
    if sel is None:
        for k in ("chat_mag", "chat_sign", "c_sign", "c_exp", "c_limbs"):
            if k in out:
                a = out[k]
                out[k] = a.reshape((M, N) + a.shape[1:])
    return out


def limbs_to_int(limbs) -> int:
    v = 0
    for x in reversed([int(y) for y in limbs]):
        v = (v << 64) | x
    return v
