"""Exact reference of the Ozaki-II p-bit matrix product, in plain Python ints.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares
no code with the GPU path and uses no moduli: the method reaches, exactly,
the integer product of the shared-exponent integer matrices (Algorithm
section, "Integerization with shared exponents", Eqs. 1-2), so this oracle
is that definition written out, followed by the single final rounding.

Steps, in the paper's notation:
  t     = p + g + ceil(log2 K)                        (Eq. 3, g = 16 by default)
  e_i   = max exp(a_ik) over the nonzero a_ik          (Eq. 1; 0 for an all-zero row)
  a^_ik = round(a_ik * 2^(t - e_i)),  |a^_ik| <= 2^t   (Eq. 1, round = nearest-even)
  f_j, b^_kj likewise per column of B
  c^_ij = sum_k a^_ik b^_kj                            (Eq. 2, exact)
  c_ij  = round_p(c^_ij * 2^(e_i + f_j - 2t))          (Eq. 2 + one rounding, nearest-even)

Number format (MPFR convention, |x| < 2^exp): value = sign * mant * 2^(exp - p)
with sign in {-1, 0, +1} (0 is the number zero) and 0 <= mant < 2^p; bits of
the stored significand at or above p are ignored.  Outputs are normalised:
2^(p-1) <= mant < 2^p, or (0, 0, 0) for zero.

Backward products (autograd form; the paper has no backward, so this is a
reading): for C = A B and an upstream gradient W = dL/dC,
  dA = W B^T  and  dB = A^T W,
formed either by re-integerizing B^T and A^T as ordinary operands
(oz2_gemm_ref on the transposes), or by reusing the forward's a^, b^ with the
exponents folded into W:
  h_i    = max_j (exp W_ij + f_j),  W'_ij = round(W_ij 2^(t_wA + f_j - h_i))
  dA_ik  = round_p( (sum_j W'_ij b^_kj) 2^(h_i - t_wA - t) )
  g_j    = max_i (exp W_ij + e_i),  W''_ij = round(W_ij 2^(t_wB + e_i - g_j))
  dB_kj  = round_p( (sum_i a^_ik W''_ij) 2^(g_j - t_wB - t) )
with t_wA = p + g + ceil(log2 N) and t_wB = p + g + ceil(log2 M) (Eq. 3's rule
for the backward contraction lengths).

Readings of the paper that this file takes (listed with the others in the
design notes): round() is round-to-nearest-even on the exact dyadic value;
the final rounding is nearest-even; an all-zero row/column gets exponent 0;
ceil(log2 K) is used for non-power-of-two K.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple


def ceil_log2(K: int) -> int:
    """ceil(log2 K) for K >= 1."""
    if K < 1:
        raise ValueError("K must be >= 1")
    return (K - 1).bit_length()


def internal_width(p: int, K: int, guard_bits: int = 16, t_bits: int = 0) -> int:
    """t of Eq. 3; an explicit t_bits overrides it (the paper's t_bits option)."""
    if t_bits:
        return t_bits
    return p + guard_bits + ceil_log2(K)


def shared_exponent(entries: Sequence[Tuple[int, int, int]]) -> int:
    """max exp over the nonzero entries (Eq. 1); 0 when every entry is zero."""
    exps = [e for (s, _m, e) in entries if s != 0]
    return max(exps) if exps else 0


def round_half_even_shift(x: int, shift: int) -> int:
    """RNE(x / 2^shift) for x >= 0, shift >= 0."""
    if shift <= 0:
        return x << (-shift)
    q = x >> shift
    r = x - (q << shift)
    half = 1 << (shift - 1)
    if r > half or (r == half and (q & 1)):
        q += 1
    return q


def integerize(sign: int, mant: int, exp: int, e: int, t: int, p: int) -> int:
    """a^ = round(a * 2^(t - e)) for a = sign * mant * 2^(exp - p) (Eq. 1)."""
    if sign == 0:
        return 0
    mant &= (1 << p) - 1
    s = t - p + exp - e            # a * 2^(t-e) = sign * mant * 2^s
    mag = mant << s if s >= 0 else round_half_even_shift(mant, -s)
    return -mag if sign < 0 else mag


def round_to_precision(c: int, scale: int, p: int) -> Tuple[int, int, int]:
    """(sign, mant, exp) of RNE_p(c * 2^scale) in the MPFR convention."""
    if c == 0:
        return (0, 0, 0)
    sign = -1 if c < 0 else 1
    mag = -c if c < 0 else c
    nb = mag.bit_length()
    if nb <= p:
        mant = mag << (p - nb)
    else:
        mant = round_half_even_shift(mag, nb - p)
        if mant == (1 << p):        # rounding carried into a new bit
            mant >>= 1
            nb += 1
    return (sign, mant, nb + scale)


def scaled_matrices(A, B, t: int):
    """(A^, B^, e, f) of Eq. 1 for operand matrices A (M x K) and B (K x N)."""
    p = A.p
    M, K = A.sign.shape
    K2, N = B.sign.shape
    assert K == K2 and B.p == p
    a_rows = [[A.value_parts(i, k) for k in range(K)] for i in range(M)]
    b_cols = [[B.value_parts(k, j) for k in range(K)] for j in range(N)]
    e = [shared_exponent(r) for r in a_rows]
    f = [shared_exponent(c) for c in b_cols]
    Ah = [[integerize(s, m, x, e[i], t, p) for (s, m, x) in a_rows[i]] for i in range(M)]
    Bh = [[integerize(s, m, x, f[j], t, p) for (s, m, x) in b_cols[j]] for j in range(N)]
    return Ah, Bh, e, f   # Bh is stored per column: Bh[j][k] = b^_kj


def exact_product(Ah: List[List[int]], Bh_cols: List[List[int]]) -> List[List[int]]:
    """c^_ij = sum_k a^_ik b^_kj (Eq. 2), exact."""
    return [[sum(a * b for a, b in zip(Ah[i], Bh_cols[j])) for j in range(len(Bh_cols))]
            for i in range(len(Ah))]


def oz2_gemm_ref(A, B, guard_bits: int = 16, t_bits: int = 0):
    """Full reference: returns t, e, f, c^ (ints) and C as (sign, mant, exp) triples."""
    p = A.p
    K = A.sign.shape[1]
    t = internal_width(p, K, guard_bits, t_bits)
    Ah, Bh, e, f = scaled_matrices(A, B, t)
    chat = exact_product(Ah, Bh)
    C = [[round_to_precision(chat[i][j], e[i] + f[j] - 2 * t, p)
          for j in range(len(f))] for i in range(len(e))]
    return {"t": t, "e": e, "f": f, "Ah": Ah, "Bh": Bh, "chat": chat, "C": C}


def backward_widths(p: int, M: int, N: int, K: int, guard_bits: int = 16, t_bits: int = 0):
    """(t, t_wA, t_wB): forward width and the widths of W for dA and dB."""
    return (internal_width(p, K, guard_bits, t_bits), p + guard_bits + ceil_log2(N),
            p + guard_bits + ceil_log2(M))


def oz2_grad_ref(A, B, W, guard_bits: int = 16, t_bits: int = 0):
    """Backward products reusing the forward's integer matrices (exponent folding)."""
    p = A.p
    M, K = A.sign.shape
    N = B.sign.shape[1]
    t, twa, twb = backward_widths(p, M, N, K, guard_bits, t_bits)
    Ah, Bh, e, f = scaled_matrices(A, B, t)          # the forward's saved integers
    w = [[W.value_parts(i, j) for j in range(N)] for i in range(M)]
    # dA: W scaled per row after folding 2^(f_j) into column j
    h = [shared_exponent([(s, m, x + f[j]) for j, (s, m, x) in enumerate(w[i])]) for i in range(M)]
    Wa = [[integerize(s, m, x + f[j], h[i], twa, p) for j, (s, m, x) in enumerate(w[i])]
          for i in range(M)]
    chat_a = [[sum(Wa[i][j] * Bh[j][k] for j in range(N)) for k in range(K)] for i in range(M)]
    dA = [[round_to_precision(chat_a[i][k], h[i] - twa - t, p) for k in range(K)]
          for i in range(M)]
    # dB: W scaled per column after folding 2^(e_i) into row i
    g = [shared_exponent([(w[i][j][0], w[i][j][1], w[i][j][2] + e[i]) for i in range(M)])
         for j in range(N)]
    Wb = [[integerize(w[i][j][0], w[i][j][1], w[i][j][2] + e[i], g[j], twb, p) for i in range(M)]
          for j in range(N)]
    chat_b = [[sum(Ah[i][k] * Wb[j][i] for i in range(M)) for j in range(N)] for k in range(K)]
    dB = [[round_to_precision(chat_b[k][j], g[j] - twb - t, p) for j in range(N)]
          for k in range(K)]
    return {"t": t, "tw": (twa, twb), "e": e, "f": f, "h": h, "g": g,
            "chat_a": chat_a, "chat_b": chat_b, "dA": dA, "dB": dB}


def oz2_zgemm_ref(Ar, Ai, Br, Bi, guard_bits: int = 16, t_bits: int = 0):
    """Complex product C = A B with A = Ar + i Ai, B = Br + i Bi (Conclusions, "Complex
    matrix products": the 3M/4M schemes turn it into real products).

    Reading: the real and imaginary parts of a row of A share one exponent, and so do
    those of a column of B, so that each part of C is one exact integer of the kind
    Eq. 2 defines, rounded once:
      t      = p + g + ceil(log2 2K)        (Eq. 3 for the 2K products summed per entry)
      e_i    = max exp over the nonzero entries of row i of Ar and of Ai   (Eq. 1)
      f_j    = max exp over the nonzero entries of column j of Br and of Bi
      ar^, ai^, br^, bi^ = the entries rounded to integers at those exponents (Eq. 1)
      cr^_ij = sum_k ar^_ik br^_kj - ai^_ik bi^_kj
      ci^_ij = sum_k ar^_ik bi^_kj + ai^_ik br^_kj
      Cr_ij, Ci_ij = round_p(cr^_ij 2^(e_i + f_j - 2t)), round_p(ci^_ij 2^(...))
    The 3M and 4M forms compute these same integers; they differ only in which real
    integer products they sum.
    """
    p = Ar.p
    M, K = Ar.sign.shape
    K2, N = Br.sign.shape
    assert K == K2 and Ai.sign.shape == (M, K) and Bi.sign.shape == (K, N)
    assert Ai.p == p and Br.p == p and Bi.p == p
    t = internal_width(p, 2 * K, guard_bits, t_bits)
    ar = [[Ar.value_parts(i, k) for k in range(K)] for i in range(M)]
    ai = [[Ai.value_parts(i, k) for k in range(K)] for i in range(M)]
    br = [[Br.value_parts(k, j) for k in range(K)] for j in range(N)]
    bi = [[Bi.value_parts(k, j) for k in range(K)] for j in range(N)]
    e = [shared_exponent(ar[i] + ai[i]) for i in range(M)]
    f = [shared_exponent(br[j] + bi[j]) for j in range(N)]
    arh = [[integerize(s, m, x, e[i], t, p) for (s, m, x) in ar[i]] for i in range(M)]
    aih = [[integerize(s, m, x, e[i], t, p) for (s, m, x) in ai[i]] for i in range(M)]
    brh = [[integerize(s, m, x, f[j], t, p) for (s, m, x) in br[j]] for j in range(N)]
    bih = [[integerize(s, m, x, f[j], t, p) for (s, m, x) in bi[j]] for j in range(N)]
    cre = [[sum(arh[i][k] * brh[j][k] - aih[i][k] * bih[j][k] for k in range(K))
            for j in range(N)] for i in range(M)]
    cim = [[sum(arh[i][k] * bih[j][k] + aih[i][k] * brh[j][k] for k in range(K))
            for j in range(N)] for i in range(M)]
    Cr = [[round_to_precision(cre[i][j], e[i] + f[j] - 2 * t, p) for j in range(N)]
          for i in range(M)]
    Ci = [[round_to_precision(cim[i][j], e[i] + f[j] - 2 * t, p) for j in range(N)]
          for i in range(M)]
    return {"t": t, "e": e, "f": f, "chat_re": cre, "chat_im": cim, "Cr": Cr, "Ci": Ci}
