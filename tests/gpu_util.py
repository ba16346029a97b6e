"""Helpers shared by the GPU tests (no method arithmetic of the product here)."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev_mp(X):
    from paper_2609_27831_amd import oz2h
    return oz2h.to_device(X)


def py_centered_residue(v: int, m: int) -> int:
    """Residue of v mod m in [-floor(m/2), ceil(m/2) - 1]."""
    r = v % m
    if r > (m - 1) // 2:
        r -= m
    return r


def read_worked_example():
    ex = {"ra": {}, "rb": {}, "dot": {}, "mod": {}}
    with open(os.path.join(GOLDEN, "crt_worked_example.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if not line:
                continue
            key, rest = line.split(None, 1)
            if key in ("a", "b"):
                ex[key] = [int(x) for x in rest.split()]
            elif key in ("chat", "P"):
                ex[key] = int(rest)
            elif key == "m":
                parts = [s.strip() for s in rest.split("|")]
                m = int(parts[0])
                ex["ra"][m] = [int(x) for x in parts[1].split()]
                ex["rb"][m] = [int(x) for x in parts[2].split()]
                ex["dot"][m] = int(parts[3])
                ex["mod"][m] = int(parts[4])
    return ex


def mp_to_ints(sign, limbs):
    """Signed significands as Python ints from sign/limb arrays."""
    flat = limbs.view(np.uint64).reshape(-1, limbs.shape[-1])
    out = []
    for row, s in zip(flat, sign.reshape(-1)):
        v = 0
        for x in row[::-1]:
            v = (v << 64) | int(x)
        out.append(int(s) * v)
    return out
