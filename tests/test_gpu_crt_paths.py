"""The paper's direct-CRT sequence and the kernel variants of stages 2 and 4 (marked gpu).

"Direct CRT without multiple-precision division": S = sum_l v_l M_l, alpha from a
binary64 sum of v_l / m_l, R = S - (alpha - 1) P in [0, 3P), at most two subtractions
of P, then the symmetric lift against floor(P/2).  The kernels take the nearest-integer
quotient when sum_l v_l / m_l is farther than 2^-30 from a half-integer and the paper's
sequence otherwise, which is exactly the case |c^| / P within 2^-30 of 1/2.  These
tests feed the CRT entry point residues of integers next to +-P/2 (and everything else
in between) on custom moduli sets, through both stage-4 kernels, and run end-to-end
products whose plans have the least CRT margin, so that |c^| may come close to P/2.
"""
import random

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


def _prod(ms):
    P = 1
    for m in ms:
        P *= int(m)
    return P


def _crt_values(P, rng, n_random=40):
    """Integers in (-P/2, P/2) with the ones next to +-P/2 that take the paper's sequence."""
    h = P // 2
    top = h if P % 2 else h - 1            # largest |c^| strictly below P/2
    vals = [0, 1, -1, top, -top, top - 1, -(top - 1), top - 2, -(top - 2), P // 4, -(P // 4),
            P // 4 + 1, -(P // 4 + 1)]
    near = max(1, P >> 31)                  # |c^| / P within 2^-31 of 1/2
    for _ in range(20):
        v = top - rng.randrange(near)
        vals.append(v if rng.random() < 0.5 else -v)
    for _ in range(n_random):
        vals.append(rng.randrange(-top, top + 1))
    return vals


def _run_crt(oz, plan, vals, rng, ncols=7, row=False):
    """row: planes with a leading dimension padded to 128 and a workspace, which selects
    the row-broadcast CRT kernels for CRTs of more than 32 digits."""
    import torch
    ms = plan.moduli.tolist()
    n = len(vals)
    M = (n + ncols - 1) // ncols
    vals = vals + [0] * (M * ncols - n)
    ldu = 128 if row else ncols
    u = np.zeros((len(ms), M, ldu), np.int16)
    for li, m in enumerate(ms):
        # any representative with |u| < m: the least nonnegative one, the centred one, or u - m
        res = []
        for v in vals:
            r = v % m
            kind = rng.randrange(3)
            if kind == 1 and r > (m - 1) // 2:
                r -= m
            elif kind == 2 and r > 0:
                r -= m
            res.append(r)
        u[li, :, :ncols] = np.array(res, np.int64).reshape(M, ncols)
    cs, cm = oz.crt(plan, torch.from_numpy(u).cuda(), M, ncols, ws="auto" if row else None)
    got = oz.limbs_to_ints(cm.cpu().numpy(), cs.cpu().numpy())
    return got[:n], vals[:n]


def _custom_sets(oz):
    glob = oz.plan_moduli(2048, 4096)["moduli"].tolist()   # a 329-modulus prefix of the global list
    one = [m for m in glob if m <= 255]
    two = [m for m in glob if m > 255]
    return [
        # (label, p, t, K, moduli)
        ("worked_example_315", 8, 2, 3, [5, 7, 9]),
        ("even_P_with_128", 8, 12, 2, [128, 127, 125, 121]),
        ("one_limb_26", 53, 80, 16, one[:26]),                    # contains 128: P even
        ("two_limb_30_odd", 113, 200, 16, two[:30]),              # odd P, 16 CRT digits
        ("mixed_70", 256, 283, 2048, one + two[:16]),             # cfg 2's set
        ("mixed_96_32_digits", 440, 464, 256, one + two[:42]),    # 32 CRT digits
        ("wide_200", 1024, 1100, 64, one + two[:146]),            # wide digit columns
        ("wide_329_cfg3a", 2048, 2076, 4096, one + two),          # cfg 3a's set, 133 digits
        ("wide_33_digits", 440, 480, 256, one + two[:44]),        # just past 32 digits
    ]


@pytest.mark.parametrize("flags,row", [(0, False), (2, False), (0, True)],
                         ids=["valu_crt", "mma_crt", "row_crt"])
def test_crt_paper_sequence_near_half_P(oz, flags, row):
    """c^ = +-floor(P/2), +-(floor(P/2) - 1), values within P 2^-31 of +-P/2 and random
    values round-trip through the CRT entry point, for odd and even P, on the fp64 kernel,
    on the matrix-core variant (where its digit range applies) and on the row-broadcast
    kernels (CRTs of more than 32 digits, given a workspace)."""
    for label, p, t, K, ms in _custom_sets(oz):
        plan = oz.Plan.custom(p, t, K, ms).set_flags(flags)
        P = _prod(plan.moduli)
        rng = random.Random(hash(label) & 0xFFFF)
        vals = _crt_values(P, rng)
        print(f"crt near P/2: {label} L={plan.L} nd32={plan.nd32} flags={flags} row={row}", flush=True)
        got, want = _run_crt(oz, plan, vals, rng, row=row)
        assert got == want, label


def test_crt_brute_force_worked_example(oz):
    """Every integer of (-P/2, P/2) for the worked example's moduli (5, 7, 9), P = 315."""
    plan = oz.Plan.custom(8, 2, 3, [5, 7, 9])
    vals = list(range(-157, 158))
    got, want = _run_crt(oz, plan, vals, random.Random(315))
    assert got == want


def test_crt_even_P_half_class(oz):
    """P even (the global list holds 128): the residue class of P/2 is reconstructed as
    +P/2 (lift tie: x0 = floor(P/2) stays positive)."""
    for flags in (0, 2):
        plan = oz.Plan.custom(8, 12, 2, [128, 127, 125, 121]).set_flags(flags)
        P = _prod(plan.moduli)
        got, _ = _run_crt(oz, plan, [P // 2, -(P // 2)], random.Random(1))
        assert got == [P // 2, P // 2]


def test_custom_plan_rejects_undersized_moduli(oz):
    """P must exceed 2^(2t + ceil(log2 K) + 1) (Eq. crtcond with margin 1)."""
    with pytest.raises(oz.Oz2hError) as ei:
        oz.Plan.custom(8, 4, 3, [5, 7, 9])             # 2^11 > 315
    assert ei.value.code == oz.ERANGE
    oz.Plan.custom(8, 3, 2, [5, 7, 9])                 # 2^8 = 256 < 315: accepted


def _extreme_operands(M, N, K, p):
    """Every entry of A and B the largest p-bit significand at one exponent, so that
    every |a^| = 2^t - 2^(t-p) and every |c^| is K (2^t - 2^(t-p))^2, next to K 2^(2t);
    row 0 / column 0 of alternating sign (cancellation to 0 for even K)."""
    A = synth.mp_zeros(M, K, p)
    B = synth.mp_zeros(K, N, p)
    full = (1 << p) - 1
    for X in (A, B):
        X.sign[:] = 1
        X.exp[:] = 3
        for l in range(X.limbs.shape[-1]):
            X.limbs[..., l] = np.uint64((full >> (64 * l)) & ((1 << 64) - 1))
    A.sign[0, 1::2] = -1
    B.sign[::3, 1] = -1
    A.sign[M - 1, :] = -1
    return A, B


@pytest.mark.parametrize("p,K,flags", [(113, 256, 0), (256, 2048, 0), (256, 2048, 3),
                                       (440, 256, 3), (1024, 64, 0), (53, 4096, 0)])
def test_margin_one_end_to_end(oz, c_oracle, p, K, flags):
    """Plans with the least CRT margin (log2 P > 2t + ceil(log2 K) + 1) on operands whose
    |c^| reach K (2^t - 2^(t-p))^2, against the oracle element by element."""
    M, N = 67, 45
    A, B = _extreme_operands(M, N, K, p)
    plan = oz.Plan.create(p, K, oz.default_opts(crt_margin=1, flags=flags))
    print(f"margin 1: p={p} K={K} L={plan.L} log2P={plan.log2P:.2f} flags={flags}", flush=True)
    ref = c_oracle.gemm(A, B)
    cs, cm, e, f = oz.gemm_integers(plan, dev_mp(A), dev_mp(B))
    C = oz.gemm(plan, dev_mp(A), dev_mp(B))
    cm = cm.cpu().numpy().view(np.uint64)
    n = min(cm.shape[-1], ref["nlc"])
    assert np.array_equal(cs.cpu().numpy(), ref["chat_sign"])
    assert np.array_equal(cm[..., :n], ref["chat_mag"][..., :n])
    assert np.array_equal(C.sign.cpu().numpy(), ref["c_sign"])
    assert np.array_equal(C.exp.cpu().numpy(), ref["c_exp"])
    assert np.array_equal(C.limbs.cpu().numpy().view(np.uint64), ref["c_limbs"])
    # the bound the margin is for: |c^| < P/2
    P = _prod(plan.moduli)
    top = max(oz.limbs_to_ints(cm[..., :n], np.abs(cs.cpu().numpy())))
    assert top < P // 2


def test_residue_gemm_int32_limit_two_limb(oz):
    """Residue GEMM at kpad = 132992 (the largest multiple of 128 under the K cap) with
    every plane constant +-127: each product's int32 sum is K 127^2 = 2145027968 < 2^31,
    and v_l = (P/m_l)^-1 (c0 P0 + c2 P2 + cs Ps) mod m_l follows analytically."""
    import torch
    kpad = 132992
    plan = oz.Plan.custom(53, 8, kpad, [251, 16189, 16187])
    ms = plan.moduli.tolist()
    P = _prod(ms)
    G, mpad, npad = plan.G, 128, 128
    sa = [127, -127, 127, 127, -127, -127, 127]     # per plane: one-limb, then two triples
    sb = [-127, -127, 127, 127, 127, -127, -127]
    a = torch.empty((G, mpad, kpad), dtype=torch.int8, device="cuda")
    b = torch.empty((G, npad, kpad), dtype=torch.int8, device="cuda")
    for g in range(G):
        a[g].fill_(sa[g])
        b[g].fill_(sb[g])
    print("residue GEMM at kpad 132992", flush=True)
    u = oz.residue_gemm(plan, a, b).cpu().numpy()
    for li, m in enumerate(ms):
        minv = pow((P // m) % m, -1, m)
        if m <= 255:
            c = kpad * sa[li] * sb[li]
        else:
            g0 = 1 + 3 * (li - 1)
            P0 = kpad * sa[g0] * sb[g0]
            P2 = kpad * sa[g0 + 1] * sb[g0 + 1]
            Ps = kpad * sa[g0 + 2] * sb[g0 + 2]
            c = -127 * P0 + 16256 * P2 + 128 * Ps
        v = c * minv % m
        v_c = v - m if v > (m - 1) // 2 else v
        got = u[li].astype(np.int64)
        assert np.all(np.mod(got - v_c, m) == 0) and np.abs(got).max() <= m // 2, f"modulus {m}"


def test_tie_cases_on_gpu(oz, c_oracle):
    """The oracle's constructed ties (integerization and final rounding) through the GPU."""
    from tests.test_oracle_pins import tie_cases
    for idx, (A, B) in enumerate(tie_cases()):
        K = A.sign.shape[1]
        for flags in (0, 3):
            plan = oz.Plan.create(A.p, K, oz.default_opts(flags=flags))
            print(f"tie case {idx} p={A.p} K={K} flags={flags}", flush=True)
            ref = c_oracle.gemm(A, B)
            C = oz.gemm(plan, dev_mp(A), dev_mp(B))
            assert np.array_equal(C.sign.cpu().numpy(), ref["c_sign"])
            assert np.array_equal(C.exp.cpu().numpy(), ref["c_exp"])
            assert np.array_equal(C.limbs.cpu().numpy().view(np.uint64), ref["c_limbs"])
