"""Counter-based SplitMix64 generator and p-bit operand matrices.

SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): the n-th output (n = 1, 2, ...) of a generator
seeded with s is mix(s + n * 0x9E3779B97F4A7C15) with the 64-bit finaliser
  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27; z *= 0x94D049BB133111EB;
  z ^= z >> 31.
Because the state advances by a constant, any output can be computed from
its counter, which lets numpy produce large blocks at once.

Operand format (one entry = one p-bit floating-point number, the paper's
MPFR-style convention |x| < 2^exp):
  sign  int8   +1 / -1, or 0 for the number zero
  exp   int32  value = sign * mant * 2^(exp - p)
  limbs uint64 nl = ceil(p/64) little-endian limbs of mant, 2^(p-1) <= mant < 2^p
Per entry, in row-major order, the generator consumes 2 + nl draws:
sign = bit 0 of draw 0, exp = lo + draw 1 mod (hi - lo + 1), then the nl
limb draws from low to high with the top limb masked to p bits and bit p-1
set.  This is the paper's test distribution (uniform significands, random
signs, exponents uniform in a chosen range, Experimental Setup section).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
MASK64 = (1 << 64) - 1
CONFIG_SEED_BASE = 0x0A2A0000


def limbs_for(p: int) -> int:
    return (p + 63) // 64


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs number start+1 .. start+count of SplitMix64 seeded with `seed`."""
    n = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK64) + n * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix64_at(seed: int, counters: np.ndarray) -> np.ndarray:
    """Outputs number c + 1 of SplitMix64 seeded with `seed`, for each counter c."""
    n = np.asarray(counters, dtype=np.uint64) + np.uint64(1)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK64) + n * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


@dataclass
class MPMatrix:
    """A rows x cols matrix of p-bit numbers in the operand format above."""
    sign: np.ndarray   # int8  [rows, cols]
    exp: np.ndarray    # int32 [rows, cols]
    limbs: np.ndarray  # uint64 [rows, cols, nl]
    p: int

    @property
    def shape(self):
        return self.sign.shape

    @property
    def nl(self):
        return self.limbs.shape[-1]

    def mant_int(self, i: int, j: int) -> int:
        v = 0
        for l in range(self.nl - 1, -1, -1):
            v = (v << 64) | int(self.limbs[i, j, l])
        return v

    def value_parts(self, i: int, j: int):
        """(sign, mant, exp) of one entry as Python ints."""
        return int(self.sign[i, j]), self.mant_int(i, j), int(self.exp[i, j])

    def transpose(self) -> "MPMatrix":
        return MPMatrix(np.ascontiguousarray(self.sign.T),
                        np.ascontiguousarray(self.exp.T),
                        np.ascontiguousarray(self.limbs.transpose(1, 0, 2)), self.p)

    def slice(self, rows: slice, cols: slice) -> "MPMatrix":
        return MPMatrix(np.ascontiguousarray(self.sign[rows, cols]),
                        np.ascontiguousarray(self.exp[rows, cols]),
                        np.ascontiguousarray(self.limbs[rows, cols]), self.p)


def mp_zeros(rows: int, cols: int, p: int) -> MPMatrix:
    nl = limbs_for(p)
    return MPMatrix(np.zeros((rows, cols), np.int8), np.zeros((rows, cols), np.int32),
                    np.zeros((rows, cols, nl), np.uint64), p)


def mp_random(seed: int, rows: int, cols: int, p: int, elo: int, ehi: int,
              counter: int = 0, chunk_entries: int = 1 << 20) -> MPMatrix:
    """Random p-bit matrix drawn from SplitMix64 counters starting at `counter`."""
    if p < 2:
        raise ValueError("p must be >= 2")
    nl = limbs_for(p)
    per = 2 + nl
    total = rows * cols
    sign = np.empty(total, np.int8)
    exp = np.empty(total, np.int32)
    limbs = np.empty((total, nl), np.uint64)
    top_bits = p - 64 * (nl - 1)                  # bits used in the top limb, 1..64
    top_mask = np.uint64(MASK64 >> (64 - top_bits))
    top_set = np.uint64(1 << (top_bits - 1))
    span = np.uint64(ehi - elo + 1)
    for e0 in range(0, total, chunk_entries):
        ne = min(chunk_entries, total - e0)
        d = splitmix64(seed, counter + e0 * per, ne * per).reshape(ne, per)
        sign[e0:e0 + ne] = np.where((d[:, 0] & np.uint64(1)) == 1, -1, 1).astype(np.int8)
        exp[e0:e0 + ne] = (np.int64(elo) + (d[:, 1] % span).astype(np.int64)).astype(np.int32)
        lb = d[:, 2:].copy()
        lb[:, nl - 1] = (lb[:, nl - 1] & top_mask) | top_set
        limbs[e0:e0 + ne] = lb
    return MPMatrix(sign.reshape(rows, cols), exp.reshape(rows, cols),
                    limbs.reshape(rows, cols, nl), p)


def mp_block(seed: int, rows: int, cols: int, p: int, elo: int, ehi: int, r0: int, r1: int,
             c0: int, c1: int, counter: int = 0) -> MPMatrix:
    """Block [r0:r1, c0:c1] of mp_random(seed, rows, cols, p, elo, ehi, counter), drawn
    from its counters directly (no need to draw the whole matrix)."""
    if p < 2:
        raise ValueError("p must be >= 2")
    nl = limbs_for(p)
    per = 2 + nl
    r = np.arange(r0, r1, dtype=np.uint64)[:, None]
    c = np.arange(c0, c1, dtype=np.uint64)[None, :]
    base = np.uint64(counter) + (r * np.uint64(cols) + c) * np.uint64(per)      # [nr, nc]
    d = splitmix64_at(seed, base[..., None] + np.arange(per, dtype=np.uint64))  # [nr, nc, per]
    top_bits = p - 64 * (nl - 1)
    top_mask = np.uint64(MASK64 >> (64 - top_bits))
    top_set = np.uint64(1 << (top_bits - 1))
    span = np.uint64(ehi - elo + 1)
    sign = np.where((d[..., 0] & np.uint64(1)) == 1, -1, 1).astype(np.int8)
    exp = (np.int64(elo) + (d[..., 1] % span).astype(np.int64)).astype(np.int32)
    limbs = np.ascontiguousarray(d[..., 2:])
    limbs[..., nl - 1] = (limbs[..., nl - 1] & top_mask) | top_set
    return MPMatrix(sign, exp, limbs, p)


def operand_blocks_for(seed: int, M: int, N: int, K: int, p: int, elo: int, ehi: int,
                       rows_a: range, cols_b: range):
    """Rows `rows_a` of A (all of K) and columns `cols_b` of B (all of K) of
    operands_for(seed, M, N, K, p, elo, ehi), drawn from their counters."""
    per = 2 + limbs_for(p)
    A = mp_block(seed, M, K, p, elo, ehi, rows_a.start, rows_a.stop, 0, K, counter=0)
    B = mp_block(seed, K, N, p, elo, ehi, 0, K, cols_b.start, cols_b.stop, counter=M * K * per)
    return A, B


def mp_unit_uniform(seed: int, rows: int, cols: int, p: int, counter: int = 0,
                    chunk_entries: int = 1 << 20) -> MPMatrix:
    """Random +-u 2^-p with u uniform on [0, 2^p), stored normalised (|x| < 1).

    Per entry 1 + nl draws: the sign from bit 0 of the first, u from the next nl
    (masked to p bits).  A zero u gives the number zero.
    """
    if p < 2:
        raise ValueError("p must be >= 2")
    nl = limbs_for(p)
    per = 1 + nl
    total = rows * cols
    sign = np.empty(total, np.int8)
    exp = np.empty(total, np.int32)
    limbs = np.empty((total, nl), np.uint64)
    top_bits = p - 64 * (nl - 1)
    top_mask = np.uint64(MASK64 >> (64 - top_bits))
    for e0 in range(0, total, chunk_entries):
        ne = min(chunk_entries, total - e0)
        d = splitmix64(seed, counter + e0 * per, ne * per).reshape(ne, per)
        u = d[:, 1:].copy()
        u[:, nl - 1] &= top_mask
        # bit length of u, from its highest nonzero limb
        blen = np.zeros(ne, np.int64)
        for w in range(nl):
            x = u[:, w]
            nz = x != 0
            bl = np.zeros(ne, np.int64)
            xf = x[nz]
            b = np.zeros(xf.size, np.int64)
            for sh in (32, 16, 8, 4, 2, 1):          # integer log2 by halving
                big = (xf >> np.uint64(sh)) != 0
                b[big] += sh
                xf = np.where(big, xf >> np.uint64(sh), xf)
            bl[nz] = b + 1 + 64 * w
            blen = np.where(nz, bl, blen)
        # left-align u to p bits: shift by p - blen (a multi-limb shift)
        s_all = np.where(blen > 0, p - blen, 0)
        out = np.zeros_like(u)
        for w in range(nl):
            acc = np.zeros(ne, np.uint64)
            for src in range(nl):
                off = 64 * (w - src)                  # bit offset of limb src into limb w
                sh = s_all - off                      # left shift needed for this pair
                lft = (sh >= 0) & (sh < 64)
                rgt = (sh < 0) & (sh > -64)
                acc |= np.where(lft, u[:, src] << np.clip(sh, 0, 63).astype(np.uint64), 0
                                ).astype(np.uint64)
                acc |= np.where(rgt, u[:, src] >> np.clip(-sh, 0, 63).astype(np.uint64), 0
                                ).astype(np.uint64)
            out[:, w] = acc
        out[:, nl - 1] &= top_mask
        zero = blen == 0
        sign[e0:e0 + ne] = np.where(zero, 0,
                                    np.where((d[:, 0] & np.uint64(1)) == 1, -1, 1)).astype(np.int8)
        exp[e0:e0 + ne] = np.where(zero, 0, blen - p).astype(np.int32)
        limbs[e0:e0 + ne] = out
    return MPMatrix(sign.reshape(rows, cols), exp.reshape(rows, cols),
                    limbs.reshape(rows, cols, nl), p)


def grad_operands_for(seed: int, M: int, N: int, K: int, p: int, elo: int, ehi: int):
    """A (M x K), B (K x N) as in operands_for, then the upstream gradient W (M x N)
    from mp_unit_uniform, all from one counter stream."""
    per = 2 + limbs_for(p)
    A, B = operands_for(seed, M, N, K, p, elo, ehi)
    W = mp_unit_uniform(seed, M, N, p, counter=(M * K + K * N) * per)
    return A, B, W


def operands_for(seed: int, M: int, N: int, K: int, p: int, elo: int, ehi: int):
    """A (M x K) then B (K x N) from one counter stream, in that order."""
    per = 2 + limbs_for(p)
    A = mp_random(seed, M, K, p, elo, ehi, counter=0)
    B = mp_random(seed, K, N, p, elo, ehi, counter=M * K * per)
    return A, B
