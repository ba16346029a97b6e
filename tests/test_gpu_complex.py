"""GPU parity of complex products (oz2h_zgemm: the 3M and 4M schemes) against the
oracle (marked gpu).

Both parts of C must equal the oracle's rounded p-bit results bit for bit: the
oracle is the exact complex integer product of the shared-exponent integer
matrices, rounded once per part (oracle/oz2_ref.oz2_zgemm_ref, computed here
through the real C oracle on the 2K-long concatenated operands).  Small and
ragged cases are compared element by element; a 1024^2 case on sampled
entries; the exact symmetries (i A) B = i (A B) and 3M = 4M on the full output.
"""
import numpy as np
import pytest

from tests.gpu_util import dev_mp, need_gpu
from tests.test_oracle_complex_pins import neg, zoperands

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oz():
    need_gpu()
    from paper_2609_27831_amd import oz2h
    return oz2h


def _host(C):
    return (C.sign.cpu().numpy(), C.exp.cpu().numpy(), C.limbs.cpu().numpy().view(np.uint64))


def _run(oz, plan, ops, scheme, opA=0, opB=0):
    import torch
    Ar, Ai, Br, Bi = ops
    dA = [dev_mp(X.transpose() if opA else X) for X in (Ar, Ai)]
    dB = [dev_mp(X.transpose() if opB else X) for X in (Br, Bi)]
    Cr, Ci = oz.zgemm(plan, dA[0], dA[1], dB[0], dB[1], scheme=scheme, opA=opA, opB=opB)
    torch.cuda.synchronize()
    return _host(Cr), _host(Ci)


def _same(got, ref, sel=None):
    s, e, l = got
    if sel is not None:
        s, e, l = s[sel], e[sel], l[sel]
    assert np.array_equal(s, ref["c_sign"])
    assert np.array_equal(e, ref["c_exp"])
    assert np.array_equal(l, ref["c_limbs"])


CASES = [
    # name, seed, M, N, K, p, elo, ehi, zero_frac, opA, opB, flags
    ("ragged_p113", 11, 300, 200, 257, 113, -16, 16, 0.0, 0, 0, 0),
    ("two_limb_p256", 12, 260, 130, 200, 256, -32, 32, 0.05, 0, 0, 0),
    ("transposed_p64", 13, 129, 257, 130, 64, -8, 8, 0.1, 1, 1, 0),
    ("tiny_p2", 14, 7, 5, 3, 2, -30, 30, 0.2, 0, 1, 0),
    ("wide_p1024", 15, 140, 70, 64, 1024, -100, 100, 0.0, 0, 0, 0),
    ("variants_p384", 16, 200, 140, 96, 384, -20, 20, 0.05, 0, 0, 3),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_zgemm_matches_oracle(oz, c_oracle, case):
    name, seed, M, N, K, p, lo, hi, zf, opA, opB, flags = case
    print(f"zgemm {name}: M={M} N={N} K={K} p={p} flags={flags}", flush=True)
    ops = zoperands(seed, M, N, K, p, lo, hi, zf)
    plan = oz.Plan.create(p, 2 * K).set_flags(flags)
    re, im = c_oracle.zgemm(*ops)
    for scheme in (oz.ZGEMM_3M, oz.ZGEMM_4M):
        gr, gi = _run(oz, plan, ops, scheme, opA, opB)
        _same(gr, re)
        _same(gi, im)
    plan.destroy()


def test_zgemm_1024_sampled_and_symmetries(oz, c_oracle):
    """1024^2 x 1024 at p = 256 (two-limb moduli, several XCD rectangles): sampled
    entries (the four corner blocks and random ones) against the oracle; 3M = 4M and
    (i A) B = i (A B) on every entry."""
    import torch
    M = N = K = 1024
    p = 256
    print("zgemm 1024^3 p=256", flush=True)
    ops = zoperands(21, M, N, K, p, -16, 16)
    plan = oz.Plan.create(p, 2 * K)
    g3 = _run(oz, plan, ops, oz.ZGEMM_3M)
    g4 = _run(oz, plan, ops, oz.ZGEMM_4M)
    for a, b in zip(g3, g4):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    rot = _run(oz, plan, (neg(ops[1]), ops[0], ops[2], ops[3]), oz.ZGEMM_3M)
    assert np.array_equal(rot[0][0], -g3[1][0])          # Re(i A B) = -Im(A B)
    assert np.array_equal(rot[0][1], g3[1][1]) and np.array_equal(rot[0][2], g3[1][2])
    for x, y in zip(rot[1], g3[0]):                      # Im(i A B) = Re(A B)
        assert np.array_equal(x, y)
    rng = np.random.default_rng(5)
    ii = np.concatenate([np.repeat(np.arange(4), 4), np.repeat(np.arange(M - 4, M), 4),
                         rng.integers(0, M, 64)])
    jj = np.concatenate([np.tile(np.arange(4), 4), np.tile(np.arange(N - 4, N), 4),
                         rng.integers(0, N, 64)])
    re, im = c_oracle.zgemm(*ops, sel=(ii, jj))
    _same(g3[0], re, (ii, jj))
    _same(g3[1], im, (ii, jj))
    plan.destroy()
    torch.cuda.empty_cache()


def test_zgemm_edges(oz):
    import torch
    ops = zoperands(31, 6, 5, 4, 53, -4, 4)
    plan = oz.Plan.create(53, 8)
    dA = [dev_mp(X) for X in ops[:2]]
    dB = [dev_mp(X) for X in ops[2:]]
    # K = 0: both parts are zero
    z = [oz.empty_mp(6, 0, 53), oz.empty_mp(6, 0, 53)]
    zb = [oz.empty_mp(0, 5, 53), oz.empty_mp(0, 5, 53)]
    Cr, Ci = oz.zgemm(plan, z[0], z[1], zb[0], zb[1])
    torch.cuda.synchronize()
    for C in (Cr, Ci):
        assert not C.sign.any() and not C.exp.any() and not C.limbs.any()
    # a plan for K (not 2K) is rejected; so is an unknown scheme
    bad = oz.Plan.create(53, 4)
    with pytest.raises(oz.Oz2hError):
        oz.zgemm(bad, dA[0], dA[1], dB[0], dB[1])
    with pytest.raises(oz.Oz2hError):
        oz.zgemm(plan, dA[0], dA[1], dB[0], dB[1], scheme=2)
    # M = 0 is a no-op
    e0 = [oz.empty_mp(0, 4, 53), oz.empty_mp(0, 4, 53)]
    oz.zgemm(plan, e0[0], e0[1], dB[0], dB[1])
    bad.destroy()
    plan.destroy()


@pytest.mark.parametrize("scheme", [3, 4])
def test_zgemm_largest_K(oz, c_oracle, scheme):
    """K = 66500, the largest complex contraction (a plan of length 2K = 133000): each real
    residue GEMM accumulates K products of centred residues in INT32."""
    M, N, K, p = 5, 6, 66500, 64
    print(f"zgemm K={K} scheme={scheme}", flush=True)
    ops = zoperands(41 + scheme, M, N, K, p, -4, 4)
    plan = oz.Plan.create(p, 2 * K)
    re, im = c_oracle.zgemm(*ops)
    gr, gi = _run(oz, plan, ops, scheme)
    _same(gr, re)
    _same(gi, im)
    plan.destroy()
