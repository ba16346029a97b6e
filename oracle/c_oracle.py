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
        L.oz2o_gemm_scaled.argtypes = [i64, i64, i64, i32,
                                       i32, P, P, P, i64, i64, P, P,
                                       i32, P, P, P, i64, i64, P, P,
                                       i64, P, P, P, P, i32, P, P, P, P, P]
        L.oz2o_gemm_scaled.restype = i32
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


def _i32(v):
    return None if v is None else np.ascontiguousarray(v, dtype=np.int32)


def gemm_scaled(M: int, N: int, K: int, p: int, a_side, b_side, sel=None,
                want_chat: bool = True, want_c: bool = True):
    """General reference product (oz2o_gemm_scaled).

    a_side / b_side = (MPMatrix X, t, rs, cs, koff or None, efix or None): the
    logical operand's entry (r, k) (A: r = row i; B: r = column j) is stored at
    X's flat index r*rs + k*cs.  Returns the same dictionary as gemm() plus
    "scale_t" = ta + tb.
    """
    Xa, ta, a_rs, a_cs, a_koff, a_efix = a_side
    Xb, tb, b_rs, b_cs, b_koff, b_efix = b_side
    assert Xa.p == p and Xb.p == p
    a_koff, a_efix, b_koff, b_efix = _i32(a_koff), _i32(a_efix), _i32(b_koff), _i32(b_efix)
    nl = (p + 63) // 64
    nlc = (ta + tb + (K - 1).bit_length() + 1 + 63) // 64
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
    # B's strides are passed as (stride along k, stride along j)
    st = lib().oz2o_gemm_scaled(M, N, K, p,
                                ta, _p(Xa.sign), _p(Xa.exp), _p(Xa.limbs), a_rs, a_cs,
                                _p(a_koff), _p(a_efix),
                                tb, _p(Xb.sign), _p(Xb.exp), _p(Xb.limbs), b_cs, b_rs,
                                _p(b_koff), _p(b_efix),
                                nout, _p(si), _p(sj), _p(e), _p(f),
                                nlc, _p(cm), _p(cs), _p(os_), _p(oe), _p(ol))
    if st != 0:
        raise RuntimeError(f"oracle failed with status {st}")
    out = {"e": e, "f": f, "nlc": nlc, "scale_t": ta + tb}
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


def backward_widths(p: int, M: int, N: int, K: int, guard_bits: int = 16, t_bits: int = 0):
    """(t, t_wA, t_wB): the forward width (Eq. 3) and the widths of the upstream
    gradient W when it is scaled for dA = W B^T (contraction N) and for
    dB = A^T W (contraction M), by the same rule as Eq. 3."""
    t = internal_width(p, K, guard_bits, t_bits)
    return (t, p + guard_bits + (N - 1).bit_length(), p + guard_bits + (M - 1).bit_length())


def grad_reuse(A, B, W, guard_bits: int = 16, t_bits: int = 0, sel_a=None, sel_b=None,
               want_chat: bool = True):
    """Backward products of C = A B that reuse the forward's integer matrices.

    Exponent folding: dA = W B^T is formed from W'_ij = W_ij 2^(f_j) scaled per
    row i (h_i = max_j exp W_ij + f_j) and the forward's b^_kj; dB = A^T W from
    W''_ij = W_ij 2^(e_i) scaled per column j and the forward's a^_ik.
    Returns (dA dict, dB dict) as gemm_scaled() does; dA's "e" is h, dB's "f" is g.
    """
    p = A.p
    M, K = A.sign.shape
    N = B.sign.shape[1]
    assert B.sign.shape[0] == K and W.sign.shape == (M, N)
    t, twa, twb = backward_widths(p, M, N, K, guard_bits, t_bits)
    e = integerize(A, t, "A")[0]
    f = integerize(B, t, "B")[0]
    zK = np.zeros(K, np.int32)
    # dA (M x K, contraction j < N): left W rows i, right B^T: entry (k, j) = B[k, j]
    dA = gemm_scaled(M, K, N, p, (W, twa, N, 1, f, None), (B, t, N, 1, -f, zK),
                     sel=sel_a, want_chat=want_chat)
    # dB (K x N, contraction i < M): left A^T: entry (k, i) = A[i, k]; right W columns j
    dB = gemm_scaled(K, N, M, p, (A, t, 1, K, -e, zK), (W, twb, 1, N, e, None),
                     sel=sel_b, want_chat=want_chat)
    return dA, dB


def grad_recompute(A, B, W, guard_bits: int = 16, sel_a=None, sel_b=None):
    """Backward products as plain products of re-integerized operands:
    dA = W (B^T) with K' = N, dB = (A^T) W with K' = M (Eqs. 1-3 each)."""
    dA = gemm(W, B.transpose(), guard_bits, sel=sel_a)
    dB = gemm(A.transpose(), W, guard_bits, sel=sel_b)
    return dA, dB


def limbs_to_int(limbs) -> int:
    v = 0
    for x in reversed([int(y) for y in limbs]):
        v = (v << 64) | x
    return v


def _hcat(X, Y, negate_y: bool = False):
    """[X | Y] (or [X | -Y]) as one matrix of X's own type."""
    MPMatrix = type(X)
    ys = -Y.sign if negate_y else Y.sign
    return MPMatrix(np.ascontiguousarray(np.concatenate([X.sign, ys], axis=1)),
                    np.ascontiguousarray(np.concatenate([X.exp, Y.exp], axis=1)),
                    np.ascontiguousarray(np.concatenate([X.limbs, Y.limbs], axis=1)), X.p)


def _vcat(X, Y, negate_y: bool = False):
    """[X ; Y] (or [X ; -Y]) as one matrix of X's own type."""
    MPMatrix = type(X)
    ys = -Y.sign if negate_y else Y.sign
    return MPMatrix(np.ascontiguousarray(np.concatenate([X.sign, ys], axis=0)),
                    np.ascontiguousarray(np.concatenate([X.exp, Y.exp], axis=0)),
                    np.ascontiguousarray(np.concatenate([X.limbs, Y.limbs], axis=0)), X.p)


def zgemm(Ar, Ai, Br, Bi, guard_bits: int = 16, t_bits: int = 0, sel=None,
          want_chat: bool = False, want_c: bool = True):
    """Complex reference product (the definition of oz2_ref.oz2_zgemm_ref) through the
    real C oracle: with A' = [Ar | Ai] (M x 2K),
      Re C = A' [Br ; -Bi]   and   Im C = A' [Bi ; Br]
    as real products of contraction length 2K.  Row i of A' holds row i of both parts,
    so its shared exponent is the complex one; column j of either right operand holds
    column j of both parts of B (negation does not change an exponent, and the
    nearest-even rounding of Eq. 1 is odd in its argument).  Returns (re, im), each the
    dictionary of gemm()."""
    Ac = _hcat(Ar, Ai)
    re = gemm(Ac, _vcat(Br, Bi, negate_y=True), guard_bits, t_bits, sel, want_chat, want_c)
    im = gemm(Ac, _vcat(Bi, Br), guard_bits, t_bits, sel, want_chat, want_c)
    return re, im
