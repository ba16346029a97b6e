"""GPU parity of the binary64 and mixed backends against the oracle (marked gpu).

A plan of OZ2H_FLAG_BACKEND_F64 takes the binary64 moduli of Eq. fp64bound and runs
its residue products on the fp64 matrix cores; OZ2H_FLAG_BACKEND_MIXED splits the
moduli between INT8 and binary64.  The CRT reconstructs the same exact integer c^
from any sufficient moduli set, so both must reproduce the oracle's c^ and rounded
p-bit results bit for bit, like the INT8 backend.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import dev_mp, need_gpu
from tests.test_gpu_parity import _compare_full, _run_gpu, _zeros

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oz():
    need_gpu()
    from paper_2609_27831_amd import oz2h
    return oz2h


F64, MIXED = 0x4, 0x8

CASES = [
    # name, seed, M, N, K, p, elo, ehi, zero_frac, opA, opB, backend flags
    ("f64_ragged_p113", 201, 300, 200, 257, 113, -16, 16, 0.02, 0, 0, F64),
    ("f64_tiny_p53", 202, 7, 5, 3, 53, -30, 30, 0.0, 0, 0, F64),
    ("f64_p2", 203, 33, 20, 9, 2, -20, 20, 0.1, 0, 1, F64),
    ("f64_p512_TN", 204, 130, 129, 190, 512, -32, 32, 0.0, 1, 0, F64),
    ("f64_p1024_row_crt", 205, 64, 70, 33, 1024, -40, 40, 0.0, 0, 0, F64),
    ("f64_K_small_bound_cap", 206, 90, 70, 100, 64, -8, 8, 0.0, 0, 0, F64),
    ("f64_K_large", 207, 20, 24, 5000, 53, -4, 4, 0.0, 0, 0, F64),
    ("mixed_p256", 208, 260, 130, 200, 256, -32, 32, 0.05, 0, 0, MIXED),
    ("mixed_p2048", 209, 40, 36, 33, 2048, -16, 16, 0.0, 0, 1, MIXED),
    ("mixed_p53_TT", 210, 129, 257, 140, 53, -200, 200, 0.02, 1, 1, MIXED),
    ("mixed_residue_mma_variant", 211, 100, 90, 120, 384, -8, 8, 0.0, 0, 0, MIXED | 1),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_backend_matches_oracle(oz, c_oracle, case):
    name, seed, M, N, K, p, lo, hi, zf, opA, opB, flags = case
    A, B = synth.operands_for(seed, M, N, K, p, lo, hi)
    if zf:
        _zeros(A, zf, seed)
        _zeros(B, zf, seed + 1)
    if M > 3 and N > 3:
        A.sign[M // 2, :] = 0
        B.sign[:, N // 3] = 0
    print(f"backend {name}: M={M} N={N} K={K} p={p} flags={flags}", flush=True)
    plan = oz.Plan.create(p, K, oz.default_opts(flags=flags))
    assert plan.backend == (1 if flags & F64 else 2)
    assert plan.Lf > 0
    ref = c_oracle.gemm(A, B)
    got = _run_gpu(oz, plan, A, B, opA, opB)
    _compare_full(got, ref, ref["nlc"])
    plan.destroy()


def test_backends_agree_1024(oz, c_oracle):
    """1024^3 at p = 256: the three backends give identical outputs on every entry, and
    sampled entries (corner blocks and random ones) equal the oracle's."""
    import torch
    M = N = K = 1024
    p = 256
    print("backends 1024^3 p=256", flush=True)
    A, B = synth.operands_for(220, M, N, K, p, -16, 16)
    Ad, Bd = dev_mp(A), dev_mp(B)
    outs = []
    for flags in (0, F64, MIXED):
        plan = oz.Plan.create(p, K, oz.default_opts(flags=flags))
        C = oz.gemm(plan, Ad, Bd)
        torch.cuda.synchronize()
        outs.append(C.to_host())
        plan.destroy()
    for o in outs[1:]:
        for x, y in zip(o, outs[0]):
            assert np.array_equal(x, y)
    rng = np.random.default_rng(9)
    ii = np.concatenate([np.repeat(np.arange(4), 4), np.repeat(np.arange(M - 4, M), 4),
                         rng.integers(0, M, 48)])
    jj = np.concatenate([np.tile(np.arange(4), 4), np.tile(np.arange(N - 4, N), 4),
                         rng.integers(0, N, 48)])
    ref = c_oracle.gemm(A, B, sel=(ii, jj), want_chat=False)
    s, e, l = outs[1]
    assert np.array_equal(s[ii, jj], ref["c_sign"])
    assert np.array_equal(e[ii, jj], ref["c_exp"])
    assert np.array_equal(l[ii, jj], ref["c_limbs"])


def test_backend_plan_rules(oz):
    A = dev_mp(synth.mp_random(5, 8, 16, 64, -4, 4))
    plan = oz.Plan.create(64, 16, oz.default_opts(flags=F64))
    with pytest.raises(oz.Oz2hError) as ei:
        oz.Residues(plan, A, oz.SIDE_A)
    assert ei.value.code == oz.EUNSUPPORTED
    with pytest.raises(oz.Oz2hError) as ei:
        plan.set_flags(0)                  # the backend is fixed at creation
    assert ei.value.code == oz.EINVAL
    plan.set_flags(F64 | 2)                # kernel-variant bits may change
    with pytest.raises(oz.Oz2hError):
        oz.Plan.create(64, 16, oz.default_opts(flags=F64 | MIXED))
    info = oz.plan_moduli32(64, 16, oz.default_opts(flags=F64))
    assert plan.L == info["L"] and list(plan.moduli) == list(info["moduli"])
    plan.destroy()


@pytest.mark.parametrize("flags", [F64, MIXED])
def test_backend_largest_K(oz, c_oracle, flags):
    """K = 133000, the largest contraction: the binary64 moduli shrink to about 5.2e5 so that
    K ((m - 1)/2)^2 stays below 2^53; every product sum is then still exact."""
    M, N, K, p = 9, 7, 133000, 53
    print(f"backend K={K} flags={flags}", flush=True)
    A, B = synth.operands_for(230 + flags, M, N, K, p, -4, 4)
    plan = oz.Plan.create(p, K, oz.default_opts(flags=flags))
    assert all(K * ((int(m) - 1) // 2) ** 2 < 2 ** 53 for m in plan.moduli[plan.L - plan.Lf:])
    ref = c_oracle.gemm(A, B)
    _compare_full(_run_gpu(oz, plan, A, B), ref, ref["nlc"])
    plan.destroy()
