"""GPU parity of each stage kernel through the C ABI (marked gpu).

Expected values come from plain numpy / Python-int computations on the same
inputs, or from the oracle's integerization (oracle/oz2_oracle.c).
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import dev_mp, need_gpu, py_centered_residue

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oz(request):
    need_gpu()
    from paper_2609_27831_amd import oz2h
    return oz2h


@pytest.mark.parametrize("tile", [1, 2, 3])
def test_i8gemm_exact_random(oz, tile):
    import torch
    rng = np.random.default_rng(1)
    bm, bn = oz.TILE_SHAPES[tile]
    for (M, N, K) in [(bm, bn, 128), (2 * bm, 3 * bn, 1024), (3 * bm, bn, 4224), (bm, 2 * bn, 256)]:
        A = rng.integers(-127, 128, (M, K), dtype=np.int8)
        B = rng.integers(-127, 128, (N, K), dtype=np.int8)
        print(f"i8gemm tile={tile} M={M} N={N} K={K}", flush=True)
        C = oz.i8gemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), tile).cpu().numpy()
        ref = A.astype(np.int64) @ B.astype(np.int64).T
        assert np.array_equal(C.astype(np.int64), ref)


def test_i8gemm_int32_limit(oz):
    """K*127^2 < 2^31 at the largest K the kernel takes (Step 3 of the tutorial section)."""
    import torch
    K = 132992           # largest multiple of 128 <= 133000
    A = np.full((128, K), 127, np.int8)
    B = np.full((128, K), 127, np.int8)
    B[1::2] = -127
    print("i8gemm int32 limit", flush=True)
    C = oz.i8gemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()).cpu().numpy()
    assert int(C[0, 0]) == K * 127 * 127
    assert int(C[0, 1]) == -K * 127 * 127


def test_exponent_scan_both_layouts(oz, c_oracle):
    import torch
    X = synth.mp_random(3, 300, 517, 128, -50, 50)
    X.sign[5, :] = 0
    X.sign[:, 7] = 0
    X.sign[rng_idx(300, 517, 0.3)] = 0
    t = 128 + 16 + 10
    eA, _, _ = c_oracle.integerize(X, t, "A")
    eB, _, _ = c_oracle.integerize(X, t, "B")
    sg = torch.from_numpy(X.sign).cuda()
    ex = torch.from_numpy(X.exp).cuda()
    print("exponent scan", flush=True)
    gA = oz.exponents(sg, ex, 300, 517, 517, 1).cpu().numpy()
    gB = oz.exponents(sg, ex, 517, 300, 1, 517).cpu().numpy()
    assert np.array_equal(gA, eA)
    assert np.array_equal(gB, eB)
    assert gA[5] == 0 and gB[7] == 0


def rng_idx(r, c, frac, seed=0):
    rng = np.random.default_rng(seed)
    return rng.random((r, c)) < frac


@pytest.mark.parametrize("p,lo,hi,side,flags", [
    (128, -4, 4, "A", 0), (256, -32, 32, "B", 0), (2048, -16, 16, "A", 0), (53, -300, 300, "B", 0),
    (113, -64, 64, "A", 0), (1024, -300, 300, "B", 0),
    # the row-broadcast VALU kernel (integers of 32 words or more) on both sides, and the
    # matrix-core variant
    (2048, -16, 16, "B", 0), (1536, -40, 40, "A", 0), (960, -8, 8, "A", 0), (3000, -8, 8, "B", 0),
    # 34, 37 and 38 words: a last chunk of two words, after none or one chunk of four
    (1050, -24, 24, "A", 0), (1150, -24, 24, "B", 0), (1180, -24, 24, "A", 0),
    (2048, -16, 16, "A", 1), (512, -32, 32, "B", 1)])
def test_residue_planes(oz, c_oracle, p, lo, hi, side, flags):
    """Stage 2 vs Python-int centred residues of the oracle's integers a^."""
    R, C = (70, 150) if side == "A" else (150, 70)
    X = synth.mp_random(11 + p, R, C, p, lo, hi)
    X.sign[rng_idx(R, C, 0.05, p)] = 0
    K = C if side == "A" else R
    check_residue_planes(oz, c_oracle, oz.Plan.create(p, K, oz.default_opts(flags=flags)), X, side, K,
                         f"p={p} side={side} flags={flags}")


# the lowest and highest p of every word count 1 .. 13 at K = 150 (t = p + 16 + 8): integers of
# up to 12 words keep their words in registers, one kernel per word count; 13 words take the
# kernel with LDS words
_WORD_P = [p for w in range(1, 14) for p in (max(2, 32 * w - 56), 32 * w - 25)]


@pytest.mark.parametrize("p", _WORD_P)
def test_residue_planes_every_word_count(oz, c_oracle, p):
    """Stage 2 against the oracle's integers for every word count of the narrow kernel, on
    both operand sides, with exponents spread over +-40 (shifts across word boundaries)."""
    side = "A" if (p // 32) % 2 else "B"
    R, C = (70, 150) if side == "A" else (150, 70)
    K = C if side == "A" else R
    plan = oz.Plan.create(p, K)
    assert plan.nw32 == -(-(p + 16 + 8 + 1) // 32)
    X = synth.mp_random(97 + p, R, C, p, -40, 40)
    X.sign[rng_idx(R, C, 0.07, p)] = 0
    check_residue_planes(oz, c_oracle, plan, X, side, K, f"p={p} side={side} words={plan.nw32}")


def test_residue_planes_wide_set_narrow_integers(oz, c_oracle):
    """The fp64 residue kernel with groups of 16 moduli: integers below 8 words (p = 113)
    against a 100-modulus prefix of the global list (54 one-limb, 46 two-limb), so that
    full one-limb groups, a mixed group, full two-limb groups and a partial group occur."""
    p, side, R, C = 113, "A", 70, 150
    mods = oz.Plan.create(1024, C).moduli.tolist()[:100]
    base = oz.Plan.create(p, C)
    plan = oz.Plan.custom(p, base.t, C, mods)
    assert plan.L == 100 and plan.L1 == 54 and plan.nw32 < 8   # the fp64 kernel, 16 per group
    X = synth.mp_random(23, R, C, p, -20, 20)
    X.sign[rng_idx(R, C, 0.05, 23)] = 0
    check_residue_planes(oz, c_oracle, plan, X, side, C, "wide set, p=113")


def check_residue_planes(oz, c_oracle, plan, X, side, K, label):
    import torch
    t = plan.t
    e, sg, mag = c_oracle.integerize(X, t, side)
    rows = e.size
    Xd = dev_mp(X)
    erow = torch.from_numpy(e).cuda()
    rpad, kpad = 128, 256
    print(f"residues {label}", flush=True)
    planes = oz.residues(plan, Xd, erow, side, rpad, kpad).cpu().numpy()
    assert planes.shape == (plan.G, rpad, kpad)
    # padding is zero
    assert not planes[:, rows:, :].any() and not planes[:, :, K:].any()
    ahat = np.array(oz.limbs_to_ints(mag, sg), dtype=object).reshape(rows, K)
    # any representative of a^ mod m is a valid residue for the exact GEMM, as long
    # as it fits the INT8 operands: |r| <= 127 for a one-limb modulus (<= 64 for 128),
    # and for a two-limb one |r| <= (m + 3)/2 with the balanced base-128 split
    for li, m in enumerate(plan.moduli.tolist()):
        res = np.vectorize(lambda v: py_centered_residue(v, m), otypes=[np.int64])(ahat)
        g0 = li if li < plan.L1 else plan.L1 + 3 * (li - plan.L1)
        if m <= 255:
            got = planes[g0, :rows, :K].astype(np.int64)
            assert np.array_equal(np.mod(got - res, m), np.zeros_like(res)), f"modulus {m}"
            assert np.abs(got).max() <= min(127, m // 2 + (m % 2 == 0)), f"modulus {m}"
        else:
            r0 = planes[g0, :rows, :K].astype(np.int64)
            r1 = planes[g0 + 1, :rows, :K].astype(np.int64)
            rs = planes[g0 + 2, :rows, :K].astype(np.int64)
            r = r0 + 128 * r1
            assert np.array_equal(np.mod(r - res, m), np.zeros_like(res)), f"modulus {m}"
            assert np.abs(r).max() <= (m + 3) // 2
            assert np.array_equal(rs, r0 + r1)
            assert r0.min() >= -64 and r0.max() <= 63 and np.abs(r1).max() <= 63


@pytest.mark.parametrize("mpad,npad,kpad,tile", [(256, 128, 384, 0), (512, 256, 256, 0),
                                               (128, 384, 128, 1), (256, 256, 256, 2),
                                               (128, 512, 128, 3)])
def test_residue_gemm_mod_m(oz, mpad, npad, kpad, tile):
    """Stage 3 vs int64 numpy products of the same planes, reduced mod m (Karatsuba included)
    and weighted by the direct-CRT factor (P/m)^-1 mod m."""
    import torch
    plan = oz.Plan.create(256, 320, oz.default_opts(tile=tile))   # 54 one-limb + 16 two-limb
    G, L1 = plan.G, plan.L1
    rng = np.random.default_rng(5 + mpad)
    A = np.zeros((G, mpad, kpad), np.int8)
    B = np.zeros((G, npad, kpad), np.int8)
    for li, m in enumerate(plan.moduli.tolist()):
        g0 = li if li < L1 else L1 + 3 * (li - L1)
        if m <= 255:
            h = (m - 1) // 2
            A[g0] = rng.integers(-(m // 2), h + 1, (mpad, kpad))
            B[g0] = rng.integers(-(m // 2), h + 1, (npad, kpad))
        else:
            for X, rows in ((A, mpad), (B, npad)):
                r = rng.integers(-(m - 1) // 2, (m - 1) // 2 + 1, (rows, kpad))
                r0 = ((r + 64) & 127) - 64
                r1 = (r - r0) // 128
                X[g0], X[g0 + 1], X[g0 + 2] = r0, r1, r0 + r1
    print("residue gemm", flush=True)
    v = oz.residue_gemm(plan, torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda())
    v = v.cpu().numpy().astype(np.int64)
    P = 1
    for m in plan.moduli.tolist():
        P *= m
    for li, m in enumerate(plan.moduli.tolist()):
        minv = pow((P // m) % m, -1, m)
        g0 = li if li < L1 else L1 + 3 * (li - L1)
        if m <= 255:
            prod = A[g0].astype(np.int64) @ B[g0].astype(np.int64).T
        else:
            a = A[g0].astype(np.int64) + 128 * A[g0 + 1].astype(np.int64)
            b = B[g0].astype(np.int64) + 128 * B[g0 + 1].astype(np.int64)
            prod = a @ b.T
        assert np.abs(v[li]).max() <= m // 2, f"modulus {m}: not centred"
        assert np.array_equal(np.mod(v[li], m), np.mod(np.mod(prod, m) * minv, m)), f"modulus {m}"


def test_residue_gemm_high_address(oz):
    """Stage 3 writing v at a device address whose low 32-bit word has bit 31 set (a base
    address composed from two 32-bit halves must not sign-extend the low one): same v as a
    plain allocation, and correct mod m."""
    import torch
    plan = oz.Plan.create(256, 320)
    G, L = plan.G, plan.L
    mpad = npad = kpad = 128
    rng = np.random.default_rng(11)
    A = rng.integers(-60, 61, (G, mpad, kpad)).astype(np.int8)
    B = rng.integers(-60, 61, (G, npad, kpad)).astype(np.int8)
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    ref = oz.residue_gemm(plan, Ad, Bd).cpu().numpy()
    nbytes = L * mpad * npad * 2
    buf = torch.empty(2 ** 31 + nbytes + 512, dtype=torch.uint8, device="cuda")
    base = buf.data_ptr()
    x = base if base & 0x80000000 else (base & ~0xFFFFFFFF) + 0x80000000
    x = (x + 255) & ~255
    assert x & 0x80000000 and base <= x and x + nbytes <= base + buf.numel()
    print("residue gemm at high address", hex(x), flush=True)
    oz._check(oz.lib().oz2h_residue_gemm(plan.handle, mpad, npad, kpad, Ad.data_ptr(),
                                         Bd.data_ptr(), x, oz._stream_ptr(None)))
    got = buf[x - base:x - base + nbytes].cpu().numpy().view(np.int16).reshape(L, mpad, npad)
    assert np.array_equal(got, ref)
    P = 1
    for m in plan.moduli.tolist():
        P *= m
    m = int(plan.moduli[0])   # a one-limb modulus: plane 0
    prod = A[0].astype(np.int64) @ B[0].astype(np.int64).T
    minv = pow((P // m) % m, -1, m)
    assert np.array_equal(np.mod(got[0].astype(np.int64), m), np.mod(np.mod(prod, m) * minv, m))
    del buf


def test_crt_worked_example(oz):
    """The tutorial's worked example: moduli 5, 7, 9 and residues (0, 3, 1) give 10."""
    import torch
    from tests.gpu_util import read_worked_example
    ex = read_worked_example()
    plan = oz.Plan.custom(8, 2, 3, [5, 7, 9])   # P = 315 > 2^(2t + ceil(log2 K) + 1) = 128
    assert list(plan.moduli) == [5, 7, 9]
    u = np.zeros((3, 1, 1), np.uint16)
    for li, m in enumerate([5, 7, 9]):
        u[li, 0, 0] = ex["mod"][m]
    print("crt worked example", flush=True)
    cs, cm = oz.crt(plan, torch.from_numpy(u.view(np.int16)).cuda(), 1, 1)
    val = oz.limbs_to_ints(cm.cpu().numpy(), cs.cpu().numpy())[0]
    assert val == ex["chat"] == 10
    # and the whole path on the example's vectors: residues -> GEMM -> CRT
    for li, m in enumerate([5, 7, 9]):
        ra = [py_centered_residue(v, m) for v in ex["a"]]
        rb = [py_centered_residue(v, m) for v in ex["b"]]
        assert ra == ex["ra"][m] and rb == ex["rb"][m]
        assert sum(x * y for x, y in zip(ra, rb)) == ex["dot"][m]


@pytest.mark.parametrize("t,row", [(t, False) for t in range(40, 1121, 8)] +
                         [(t, True) for t in range(480, 1121, 40)])
def test_crt_random_exact_integers(oz, t, row):
    """Direct CRT sweep over t = 40..1120 in steps of 8 (Correctness section); row: the
    row-broadcast kernels (planes padded to 128 columns, with a workspace)."""
    import torch
    plan = oz.Plan.create(max(2, t - 28), 4096, oz.default_opts(t_bits=t))
    P = 1
    for m in plan.moduli.tolist():
        P *= m
    rng = np.random.default_rng(t)
    M, N = 3, 43
    bound = (1 << (2 * t)) * 4096
    vals = []
    for k in range(M * N):
        bits = int(rng.integers(1, 2 * t + 13))
        v = int.from_bytes(rng.bytes((bits + 7) // 8), "little") % (1 << bits)
        v = min(v, bound)
        if k % 7 == 3:
            v = bound                       # the extreme |c^| = K 2^(2t)
        if k % 11 == 5:
            v = 0
        vals.append(-v if rng.integers(0, 2) else v)
    ldu = 128 if row else N
    u = np.zeros((plan.L, M, ldu), np.uint16)
    for li, m in enumerate(plan.moduli.tolist()):
        u[li, :, :N] = np.array([v % m for v in vals], np.uint16).reshape(M, N)
    print(f"crt sweep t={t} row={row}", flush=True)
    cs, cm = oz.crt(plan, torch.from_numpy(u.view(np.int16)).cuda(), M, N, ws="auto" if row else None)
    got = oz.limbs_to_ints(cm.cpu().numpy(), cs.cpu().numpy())
    assert got == vals
