"""End-to-end GPU parity against the oracle (marked gpu).

The GPU must reproduce the oracle's reconstructed integers c^ bit for bit
(oz2h_gemm_integers) and its rounded p-bit results bit for bit (oz2h_gemm),
which is within 1 ulp of the oracle by construction.  Small and ragged cases
are compared element by element; the full-size workloads are compared on
sampled entries (four corner blocks, which catch tile-edge mistakes, plus
seeded random entries) that the oracle computes one by one.
"""
import time
from fractions import Fraction

import numpy as np
import pytest

import synth
from tests.gpu_util import dev_mp, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oz():
    need_gpu()
    from paper_2609_27831_amd import oz2h
    return oz2h


def _zeros(X, frac, seed):
    rng = np.random.default_rng(seed)
    X.sign[rng.random(X.sign.shape) < frac] = 0


def _run_gpu(oz, plan, A, B, opA=0, opB=0):
    """Upload (transposing the stored matrix for op T), run both entry points."""
    Ad = dev_mp(A.transpose() if opA else A)
    Bd = dev_mp(B.transpose() if opB else B)
    cs, cm, e, f = oz.gemm_integers(plan, Ad, Bd, opA, opB)
    C = oz.gemm(plan, Ad, Bd, opA, opB)
    import torch
    torch.cuda.synchronize()
    return (cs.cpu().numpy(), cm.cpu().numpy().view(np.uint64), e.cpu().numpy(), f.cpu().numpy(),
            C.sign.cpu().numpy(), C.exp.cpu().numpy(), C.limbs.cpu().numpy().view(np.uint64))


def _compare_full(got, ref, nlc_ref):
    cs, cm, e, f, os_, oe, ol = got
    assert np.array_equal(e, ref["e"]) and np.array_equal(f, ref["f"])
    assert np.array_equal(cs, ref["chat_sign"])
    n = min(cm.shape[-1], nlc_ref)
    assert np.array_equal(cm[..., :n], ref["chat_mag"][..., :n])
    assert not cm[..., n:].any() and not ref["chat_mag"][..., n:].any()
    assert np.array_equal(os_, ref["c_sign"])
    assert np.array_equal(oe, ref["c_exp"])
    assert np.array_equal(ol, ref["c_limbs"])


CASES = [
    # name, seed, M, N, K, p, elo, ehi, zero_frac, opA, opB
    ("cfg1_256_p128", synth.CONFIG_SEED_BASE + 1, 256, 256, 256, 128, -4, 4, 0.0, 0, 0),
    ("ragged_p256", 101, 200, 130, 77, 256, -32, 32, 0.05, 0, 0),
    ("ragged_p256_TN", 102, 131, 200, 96, 256, -32, 32, 0.0, 1, 0),
    ("ragged_p256_NT", 103, 129, 65, 200, 256, -32, 32, 0.0, 0, 1),
    ("ragged_p256_TT", 104, 67, 190, 130, 256, -8, 8, 0.1, 1, 1),
    ("wide_p53", 105, 129, 257, 300, 53, -300, 300, 0.02, 0, 0),
    ("tiny_p2", 106, 5, 3, 4, 2, -20, 20, 0.0, 0, 0),
    ("p1024_two_limb", 107, 64, 70, 33, 1024, -40, 40, 0.0, 0, 0),
    ("p2048_small", 108, 20, 30, 17, 2048, -16, 16, 0.0, 0, 0),
    ("p3250_widest", 113, 9, 12, 7, 3250, -8, 8, 0.0, 0, 1),
    ("p113_K_odd", 109, 140, 129, 1001, 113, -16, 16, 0.01, 0, 0),
    ("tile256x128_p256", 110, 300, 200, 150, 256, -32, 32, 0.02, 0, 0, 2),
    ("tile128x256_p512", 111, 130, 260, 70, 512, -32, 32, 0.0, 0, 1, 3),
    ("tile128x128_p113", 112, 260, 140, 333, 113, -16, 16, 0.0, 1, 0, 1),
    # the matrix-core CRT variant over its whole digit range: p = 384 (28 digits, 6
    # contraction steps) and p = 440 (32 digits, 7 steps, 4 row blocks), and the VALU kernel
    ("p384_mma_variants", 114, 96, 80, 256, 384, -8, 8, 0.0, 0, 0, 0, 3),
    ("p440_mma_variants", 115, 70, 130, 256, 440, -8, 8, 0.02, 0, 0, 0, 3),
    ("p440_valu", 115, 70, 130, 256, 440, -8, 8, 0.02, 0, 0, 0, 0),
    ("p384_crt_mma_only", 116, 129, 64, 200, 384, -30, 30, 0.0, 0, 1, 0, 2),
    # the matrix-core variants of stages 2 and 4 on cases above
    ("cfg1_mma_variants", synth.CONFIG_SEED_BASE + 1, 256, 256, 256, 128, -4, 4, 0.0, 0, 0, 0, 3),
    ("ragged_p256_mma_variants", 101, 200, 130, 77, 256, -32, 32, 0.05, 0, 0, 0, 3),
    ("p1024_mma_variants", 107, 64, 70, 33, 1024, -40, 40, 0.0, 0, 0, 0, 3),
    ("p2048_mma_variants", 108, 20, 30, 17, 2048, -16, 16, 0.0, 0, 0, 0, 3),
    ("p3250_residues_mma", 113, 9, 12, 7, 3250, -8, 8, 0.0, 0, 1, 0, 1),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_gemm_matches_oracle_elementwise(oz, c_oracle, case):
    name, seed, M, N, K, p, lo, hi, zf, opA, opB = case[:11]
    tile = case[11] if len(case) > 11 else 0
    flags = case[12] if len(case) > 12 else 0
    A, B = synth.operands_for(seed, M, N, K, p, lo, hi)
    if zf:
        _zeros(A, zf, seed)
        _zeros(B, zf, seed + 1)
    if M > 3 and N > 3:
        A.sign[M // 2, :] = 0       # an all-zero row of A and column of B
        B.sign[:, N // 3] = 0
    print(f"parity {name}: M={M} N={N} K={K} p={p} tile={tile} flags={flags}", flush=True)
    plan = oz.Plan.create(p, K, oz.default_opts(tile=tile, flags=flags))
    ref = c_oracle.gemm(A, B)
    got = _run_gpu(oz, plan, A, B, opA, opB)
    _compare_full(got, ref, ref["nlc"])


def test_accuracy_vs_exact_product(oz):
    """GPU outputs stay within 1 unit 2^-p of relative error of the true product."""
    p, M, N, K = 128, 128, 128, 64
    A, B = synth.operands_for(55, M, N, K, p, -4, 4)
    plan = oz.Plan.create(p, K)
    C = oz.gemm(plan, dev_mp(A), dev_mp(B))
    s, e, l = C.to_host()
    rng = np.random.default_rng(0)
    for _ in range(32):
        i, j = int(rng.integers(M)), int(rng.integers(N))
        exact = Fraction(0)
        for k in range(K):
            sa, ma, ea = A.value_parts(i, k)
            sb, mb, eb = B.value_parts(k, j)
            exact += Fraction(sa * ma * sb * mb) * Fraction(2) ** (ea + eb - 2 * p)
        mant = 0
        for x in l[i, j][::-1]:
            mant = (mant << 64) | int(x)
        y = int(s[i, j]) * Fraction(mant) * Fraction(2) ** (int(e[i, j]) - p)
        assert abs(y - exact) <= abs(exact) * Fraction(2) ** (-p)


def test_empty_and_k0(oz):
    import torch
    plan = oz.Plan.create(128, 16)
    A = dev_mp(synth.mp_random(1, 0, 16, 128, -4, 4))
    B = dev_mp(synth.mp_random(2, 16, 5, 128, -4, 4))
    C = oz.gemm(plan, A, B)
    assert C.shape == (0, 5)
    A0 = dev_mp(synth.mp_random(3, 4, 0, 128, -4, 4))
    B0 = dev_mp(synth.mp_random(4, 0, 6, 128, -4, 4))
    C0 = oz.empty_mp(4, 6, 128)
    C0.sign.fill_(7)
    C0 = oz.gemm(plan, A0, B0, out=C0)
    torch.cuda.synchronize()
    assert not C0.sign.any() and not C0.exp.any() and not C0.limbs.any()


def test_argument_errors(oz):
    plan = oz.Plan.create(64, 32)
    A = dev_mp(synth.mp_random(1, 8, 32, 64, -4, 4))
    B = dev_mp(synth.mp_random(2, 31, 8, 64, -4, 4))
    with pytest.raises(ValueError):
        oz.gemm(plan, A, B)
    B2 = dev_mp(synth.mp_random(2, 16, 8, 64, -4, 4))
    plan16 = oz.Plan.create(64, 16)
    with pytest.raises(oz.Oz2hError) as ei:
        oz.gemm(plan, dev_mp(synth.mp_random(1, 8, 16, 64, -4, 4)), B2)   # K differs from the plan's
    assert ei.value.code == oz.EINVAL
    import torch
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(oz.Oz2hError) as ei:
        oz.gemm(plan16, dev_mp(synth.mp_random(1, 8, 16, 64, -4, 4)), B2, ws=ws)
    assert ei.value.code == oz.ENOMEM
    with pytest.raises(oz.Oz2hError) as ei:
        oz.Plan.create(64, 200000)
    assert ei.value.code == oz.ERANGE


# ------------------------------------------------------------ full-size workloads

FULL = [
    # name, seed, M, N, K, p, elo, ehi
    ("cfg2_2048_p256", synth.CONFIG_SEED_BASE + 2, 2048, 2048, 2048, 256, -32, 32),
    ("cfg3b_8192_p113", synth.CONFIG_SEED_BASE + 32, 8192, 8192, 8192, 113, -16, 16),
    ("cfg3a_4096_p2048", synth.CONFIG_SEED_BASE + 31, 4096, 4096, 4096, 2048, -16, 16),
]


def sample_entries(M, N, corner, nrand, seed):
    ii, jj = [], []
    for (r0, c0) in ((0, 0), (0, N - corner), (M - corner, 0), (M - corner, N - corner)):
        for a in range(corner):
            for b in range(corner):
                ii.append(r0 + a)
                jj.append(c0 + b)
    rng = np.random.default_rng(seed)
    ii += list(rng.integers(0, M, nrand))
    jj += list(rng.integers(0, N, nrand))
    return np.array(ii, np.int64), np.array(jj, np.int64)


@pytest.mark.parametrize("case", FULL, ids=[c[0] for c in FULL])
def test_full_size_sampled(oz, c_oracle, case):
    import torch
    name, seed, M, N, K, p, lo, hi = case
    t0 = time.time()
    A, B = synth.operands_for(seed, M, N, K, p, lo, hi)
    print(f"full {name}: inputs {time.time() - t0:.1f}s", flush=True)
    plan = oz.Plan.create(p, K)
    Ad, Bd = dev_mp(A), dev_mp(B)
    corner = 32 if p <= 256 else 8
    si, sj = sample_entries(M, N, corner, 512 if p <= 256 else 96, seed)
    ws = oz.workspace(plan, M, N)
    cs, cm, e, f = oz.gemm_integers(plan, Ad, Bd, ws=ws)
    C = oz.gemm(plan, Ad, Bd, ws=ws)
    torch.cuda.synchronize()
    print(f"full {name}: gpu done {time.time() - t0:.1f}s", flush=True)
    ti, tj = torch.from_numpy(si).cuda(), torch.from_numpy(sj).cuda()
    g_cs = cs[ti, tj].cpu().numpy()
    g_cm = cm[ti, tj].cpu().numpy().view(np.uint64)
    g_os = C.sign[ti, tj].cpu().numpy()
    g_oe = C.exp[ti, tj].cpu().numpy()
    g_ol = C.limbs[ti, tj].cpu().numpy().view(np.uint64)
    e, f = e.cpu().numpy(), f.cpu().numpy()
    del Ad, Bd, ws, cs, cm, C
    torch.cuda.empty_cache()
    ref = c_oracle.gemm(A, B, sel=(si, sj))
    print(f"full {name}: oracle done {time.time() - t0:.1f}s", flush=True)
    assert np.array_equal(e[np.unique(si)], ref["e"][np.unique(si)])
    assert np.array_equal(f[np.unique(sj)], ref["f"][np.unique(sj)])
    assert np.array_equal(g_cs, ref["chat_sign"])
    n = min(g_cm.shape[-1], ref["nlc"])
    assert np.array_equal(g_cm[:, :n], ref["chat_mag"][:, :n])
    assert np.array_equal(g_os, ref["c_sign"])
    assert np.array_equal(g_oe, ref["c_exp"])
    assert np.array_equal(g_ol, ref["c_limbs"])
