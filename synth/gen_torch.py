"""The generator of gen.py on torch tensors (any device), for large operands drawn
straight into device memory.  Same counters, same outputs bit for bit: uint64
arithmetic is emulated on int64 tensors (wrapping multiplication; logical shifts by
masking; unsigned remainders from the halved value).  No method arithmetic here.
"""
from __future__ import annotations

from .gen import CONFIG_SEED_BASE, limbs_for  # noqa: F401

_GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB


def _s64(x: int) -> int:
    """The int64 with the bit pattern of the uint64 x."""
    x &= (1 << 64) - 1
    return x - (1 << 64) if x >= 1 << 63 else x


def _lsr(z, s: int):
    """Logical right shift of int64 bit patterns."""
    return (z >> s) & ((1 << (64 - s)) - 1)


def splitmix64_torch(seed: int, counters):
    """Outputs number c + 1 of SplitMix64 for each int64 counter c (as int64 bit patterns)."""
    z = (counters + 1) * _s64(_GAMMA) + _s64(seed)
    z = (z ^ _lsr(z, 30)) * _s64(_M1)
    z = (z ^ _lsr(z, 27)) * _s64(_M2)
    return z ^ _lsr(z, 31)


def _umod(z, m: int):
    """Unsigned remainder of int64 bit patterns by a small positive m."""
    return (((_lsr(z, 1) % m) * 2) + (z & 1)) % m


def mp_random_torch(seed: int, rows: int, cols: int, p: int, elo: int, ehi: int,
                    counter: int = 0, device="cuda", chunk_entries: int = 1 << 22):
    """(sign int8, exp int32, limbs int64 [rows, cols, nl]) equal to gen.mp_random."""
    import torch
    if p < 2:
        raise ValueError("p must be >= 2")
    nl = limbs_for(p)
    per = 2 + nl
    total = rows * cols
    sign = torch.empty(total, dtype=torch.int8, device=device)
    exp = torch.empty(total, dtype=torch.int32, device=device)
    limbs = torch.empty((total, nl), dtype=torch.int64, device=device)
    top_bits = p - 64 * (nl - 1)
    top_mask = _s64((1 << top_bits) - 1)
    top_set = _s64(1 << (top_bits - 1))
    span = ehi - elo + 1
    off = torch.arange(per, dtype=torch.int64, device=device)
    for e0 in range(0, total, chunk_entries):
        ne = min(chunk_entries, total - e0)
        cnt = counter + (e0 + torch.arange(ne, dtype=torch.int64, device=device))[:, None] * per + off
        d = splitmix64_torch(seed, cnt)
        sign[e0:e0 + ne] = torch.where((d[:, 0] & 1) == 1, -1, 1).to(torch.int8)
        exp[e0:e0 + ne] = (elo + _umod(d[:, 1], span)).to(torch.int32)
        lb = d[:, 2:].clone()
        lb[:, nl - 1] = (lb[:, nl - 1] & top_mask) | top_set
        limbs[e0:e0 + ne] = lb
    return sign.reshape(rows, cols), exp.reshape(rows, cols), limbs.reshape(rows, cols, nl)


def operands_for_torch(seed: int, M: int, N: int, K: int, p: int, elo: int, ehi: int,
                       device="cuda"):
    """gen.operands_for drawn on `device`: ((sign, exp, limbs) of A, the same of B)."""
    per = 2 + limbs_for(p)
    A = mp_random_torch(seed, M, K, p, elo, ehi, counter=0, device=device)
    B = mp_random_torch(seed, K, N, p, elo, ehi, counter=M * K * per, device=device)
    return A, B
