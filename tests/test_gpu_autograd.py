"""GPU parity of the autograd form (marked gpu).

* float64 carriers: pack/unpack round trip bit for bit, readable slot 0, and
  rejection of encodings changed by arithmetic;
* oz2h_gemm_backward (reuse: exponent folding + saved residue planes) against
  the oracle's reuse reading, element by element, bit-exact;
* the recompute strategy against the oracle's products of the transposes;
* torch.autograd end to end (C.backward(W) fills a.grad and b.grad) in both
  modes, equal to the direct entry points;
* exact finite differences of the loss on the 64 x 64 x 64, p = 512
  subproblem: every sampled gradient entry within 1 ulp;
* the 4096^2, p = 256 workload on sampled entries.
"""
import time
from fractions import Fraction

import numpy as np
import pytest

import synth
from tests.gpu_util import dev_mp, need_gpu

pytestmark = pytest.mark.gpu

CFG5_SEED = synth.CONFIG_SEED_BASE + 5


@pytest.fixture(scope="module")
def oz():
    need_gpu()
    from paper_2609_27831_amd import oz2h
    return oz2h


@pytest.fixture(scope="module")
def ag():
    need_gpu()
    from paper_2609_27831_amd import autograd
    return autograd


def _host(X):
    import torch
    torch.cuda.synchronize()
    return X.to_host()


def _assert_equals_oracle(got, ref, sel=None):
    s, e, l = got
    if sel is not None:
        s, e, l = s[sel], e[sel], l[sel]
    assert np.array_equal(s, ref["c_sign"])
    assert np.array_equal(e, ref["c_exp"])
    assert np.array_equal(l, ref["c_limbs"])


# ---------------------------------------------------------------- carriers

@pytest.mark.parametrize("p", [2, 53, 64, 65, 256, 448, 2048, 3000, 4032, 4100])
def test_carrier_round_trip(oz, p):
    import torch
    X = synth.mp_random(300 + p, 37, 29, p, -1100, 1100)
    X.sign[3, :] = 0
    Xd = dev_mp(X)
    print(f"carrier p={p}", flush=True)
    car = oz.carrier_pack(Xd)
    assert car.shape == (37, 29, oz.carrier_width(p)) and car.dtype == torch.float64
    bad = torch.zeros(1, dtype=torch.int32, device="cuda")
    Y = oz.carrier_unpack(car, p, bad)
    s, e, l = _host(Y)
    assert int(bad.item()) == 0
    nz = X.sign != 0
    assert np.array_equal(s, X.sign)
    assert np.array_equal(e[nz], X.exp[nz]) and not e[~nz].any()
    mask = np.full(X.limbs.shape[-1], np.uint64(0xFFFFFFFFFFFFFFFF))
    top = p - 64 * (X.limbs.shape[-1] - 1)
    mask[-1] = np.uint64((1 << top) - 1)
    assert np.array_equal(l[nz], (X.limbs & mask)[nz]) and not l[~nz].any()
    # slot 0: the value truncated to 53 bits
    c0 = car[..., 0].cpu().numpy()
    for (i, j) in [(0, 0), (5, 7), (36, 28), (3, 4)]:
        sg, m, ex = X.value_parts(i, j)
        if sg == 0:
            assert c0[i, j] == 0.0
            continue
        sh = max(p - 53, 0)
        v = Fraction(sg * (m >> sh)) * Fraction(2) ** (ex - p + sh)
        want = float(v) if abs(v) < Fraction(2) ** 1024 else sg * float("inf")
        if abs(v) >= Fraction(2) ** -1022 or v == 0:
            assert c0[i, j] == want


@pytest.mark.parametrize("p", [64, 448, 2048])
def test_carrier_unpack_into_strided_output(oz, p):
    """oz2h_carrier_unpack into a matrix of row stride ld > cols (the C call; the binding
    allocates dense outputs): the columns it covers equal the dense unpack, the others are
    left untouched."""
    import torch
    X = synth.mp_random(500 + p, 37, 29, p, -50, 50)
    X.sign[2, :] = 0
    car = oz.carrier_pack(dev_mp(X))
    dense = oz.carrier_unpack(car, p)
    wide = oz.empty_mp(37, 29 + 5, p)
    wide.sign.fill_(7)
    wide.exp.fill_(-3)
    wide.limbs.fill_(-1)
    bad = torch.zeros(1, dtype=torch.int32, device="cuda")
    print(f"carrier strided unpack p={p}", flush=True)
    st = oz.lib().oz2h_carrier_unpack(37, 29, p, car.data_ptr(), wide.mat(), bad.data_ptr(), None)
    assert st == 0
    torch.cuda.synchronize()
    assert int(bad.item()) == 0
    ds, de, dl = dense.to_host()
    ws, we, wl = wide.to_host()
    assert np.array_equal(ws[:, :29], ds) and np.array_equal(we[:, :29], de)
    assert np.array_equal(wl[:, :29], dl)
    assert (ws[:, 29:] == 7).all() and (we[:, 29:] == -3).all()
    assert (wl[:, 29:] == np.uint64(0xFFFFFFFFFFFFFFFF)).all()

def test_carrier_rejects_arithmetic(oz):
    import torch
    X = synth.mp_random(7, 4, 5, 128, -8, 8)
    car = oz.carrier_pack(dev_mp(X))
    bad = torch.zeros(1, dtype=torch.int32, device="cuda")
    oz.carrier_unpack(car, 128, bad)
    assert int(bad.item()) == 0
    for (i, j, slot, delta) in [(0, 0, 1, 0.5), (1, 1, 1, 1.0), (2, 2, 2, 2.0 ** 32), (3, 3, 3, 0.25),
                                (0, 4, 5, 2.0 ** 31)]:
        c2 = car.clone()
        c2[i, j, slot] += delta
        bad.zero_()
        Y = oz.carrier_unpack(c2, 128, bad)
        assert int(bad.item()) == 1, (i, j, slot)
        assert int(Y.sign[i, j].item()) == 0
    # a sum of two carriers (what gradient accumulation would produce) is rejected
    bad.zero_()
    oz.carrier_unpack(car + car, 128, bad)
    assert int(bad.item()) == 1


# ---------------------------------------------------------------- backward products

CASES = [
    # name, seed, M, N, K, p, elo, ehi
    ("fd_64_p512", CFG5_SEED + 100, 64, 64, 64, 512, -4, 4),
    ("ragged_p256", 501, 200, 130, 77, 256, -32, 32),
    ("wide_p113", 502, 129, 257, 300, 113, -300, 300),
    ("tall_p53", 503, 300, 7, 45, 53, -20, 20),
    ("p2048_small", 504, 20, 30, 17, 2048, -16, 16),
    ("p1024_K1", 505, 33, 65, 1, 1024, -8, 8),
]


def _inputs(case):
    name, seed, M, N, K, p, lo, hi = case
    A, B, W = synth.grad_operands_for(seed, M, N, K, p, lo, hi)
    if M > 4 and N > 4:
        W.sign[M // 3, :] = 0      # a zero row and column of the upstream gradient
        W.sign[:, N // 2] = 0
        A.sign[:, 0] = 0
    return A, B, W


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_backward_reuse_matches_oracle(oz, c_oracle, case):
    name, seed, M, N, K, p = case[:6]
    A, B, W = _inputs(case)
    print(f"backward reuse {name}: M={M} N={N} K={K} p={p}", flush=True)
    plan = oz.Plan.create_grad(p, M, N, K)
    assert plan.tw_a == p + 16 + (N - 1).bit_length() and plan.tw_b == p + 16 + (M - 1).bit_length()
    ws = oz.workspace(plan, M, N)
    Ad, Bd, Wd = dev_mp(A), dev_mp(B), dev_mp(W)
    C = oz.gemm(plan, Ad, Bd, ws=ws)
    dA, dB = oz.gemm_backward(plan, ws, Wd)
    rA, rB = c_oracle.grad_reuse(A, B, W, want_chat=False)
    _assert_equals_oracle(_host(dA), rA)
    _assert_equals_oracle(_host(dB), rB)
    # the forward on the larger moduli set is still the plain product
    _assert_equals_oracle(_host(C), c_oracle.gemm(A, B, want_chat=False))
    # a second backward from the same saved forward, one side only
    dA2, none = oz.gemm_backward(plan, ws, Wd, want_b=False)
    assert none is None
    _assert_equals_oracle(_host(dA2), rA)


@pytest.mark.parametrize("case", CASES[:4], ids=[c[0] for c in CASES[:4]])
def test_backward_recompute_matches_oracle(ag, oz, c_oracle, case):
    import torch
    name, seed, M, N, K, p = case[:6]
    A, B, W = _inputs(case)
    print(f"backward recompute {name}", flush=True)
    a = ag.to_carrier(A).requires_grad_()
    b = ag.to_carrier(B).requires_grad_()
    c = ag.oz_matmul(a, b, p, mode="recompute")
    c.backward(ag.to_carrier(W))
    rA, rB = c_oracle.grad_recompute(A, B, W)
    _assert_equals_oracle(_host(ag.from_carrier(a.grad, p)), rA)
    _assert_equals_oracle(_host(ag.from_carrier(b.grad, p)), rB)
    torch.cuda.synchronize()


@pytest.mark.parametrize("mode", ["reuse", "auto"])
def test_autograd_reuse_end_to_end(ag, oz, c_oracle, mode):
    case = CASES[1]
    name, seed, M, N, K, p = case[:6]
    A, B, W = _inputs(case)
    print(f"autograd {mode}", flush=True)
    a = ag.to_carrier(A).requires_grad_()
    b = ag.to_carrier(B).requires_grad_()
    c = ag.oz_matmul(a, b, p, mode=mode)
    assert c.grad_fn is not None
    # forward value through the carrier
    _assert_equals_oracle(_host(ag.from_carrier(c.detach(), p)), c_oracle.gemm(A, B, want_chat=False))
    c.backward(ag.to_carrier(W))
    rA, rB = c_oracle.grad_reuse(A, B, W, want_chat=False)
    _assert_equals_oracle(_host(ag.from_carrier(a.grad, p)), rA)
    _assert_equals_oracle(_host(ag.from_carrier(b.grad, p)), rB)


def test_autograd_only_one_input_requires_grad(ag, c_oracle):
    case = CASES[3]
    name, seed, M, N, K, p = case[:6]
    A, B, W = _inputs(case)
    a = ag.to_carrier(A).requires_grad_()
    b = ag.to_carrier(B)
    c = ag.oz_matmul(a, b, p, mode="reuse")
    c.backward(ag.to_carrier(W))
    assert b.grad is None
    rA, _ = c_oracle.grad_reuse(A, B, W, want_chat=False)
    _assert_equals_oracle(_host(ag.from_carrier(a.grad, p)), rA)


def test_autograd_rejects_accumulated_gradient(ag):
    A, B, W = _inputs(CASES[3])
    p = 53
    a = ag.to_carrier(A).requires_grad_()
    c = ag.oz_matmul(a, ag.to_carrier(B), p, mode="recompute")
    w = ag.to_carrier(W)
    with pytest.raises(ValueError):
        c.backward(w + w)


def test_backward_errors(oz):
    import torch
    p, M, N, K = 64, 40, 30, 20
    A, B, W = synth.grad_operands_for(9, M, N, K, p, -4, 4)
    Ad, Bd, Wd = dev_mp(A), dev_mp(B), dev_mp(W)
    plain = oz.Plan.create(p, K)
    ws0 = oz.workspace(plain, M, N)
    oz.gemm(plain, Ad, Bd, ws=ws0)
    with pytest.raises(oz.Oz2hError) as ei:
        oz.gemm_backward(plain, ws0, Wd, ws=torch.empty(1 << 20, dtype=torch.uint8, device="cuda"))
    assert ei.value.code == oz.EINVAL
    plan = oz.Plan.create_grad(p, M, N, K)
    ws = oz.workspace(plan, M, N)
    oz.gemm(plan, Ad, Bd, ws=ws)
    with pytest.raises(oz.Oz2hError) as ei:      # saved workspace too small
        oz.gemm_backward(plan, ws[:1024], Wd)
    assert ei.value.code == oz.EINVAL
    with pytest.raises(oz.Oz2hError) as ei:      # backward workspace too small
        oz.gemm_backward(plan, ws, Wd, ws=torch.empty(256, dtype=torch.uint8, device="cuda"))
    assert ei.value.code == oz.ENOMEM
    W2 = dev_mp(synth.mp_random(3, M + 1, N, p, -4, 4))
    with pytest.raises(oz.Oz2hError) as ei:      # W of another shape
        oz.gemm_backward(plan, ws, W2)
    assert ei.value.code == oz.EINVAL
    with pytest.raises(oz.Oz2hError) as ei:
        oz.Plan.create_grad(p, 200000, N, K)
    assert ei.value.code == oz.ERANGE


# ---------------------------------------------------------------- finite differences

def _ints(X):
    """Entries as Python ints on a common scale: value = int * 2^scale."""
    r, c = X.sign.shape
    parts = [[X.value_parts(i, j) for j in range(c)] for i in range(r)]
    exps = [e - X.p for row in parts for (s, m, e) in row if s]
    scale = min(exps) if exps else 0
    vals = [[(s * m) << (e - X.p - scale) if s else 0 for (s, m, e) in row] for row in parts]
    return vals, scale


def _mp_value(s, e, l, p):
    if s == 0:
        return Fraction(0)
    mant = 0
    for x in l[::-1]:
        mant = (mant << 64) | int(x)
    return int(s) * Fraction(mant) * Fraction(2) ** (int(e) - p)


def test_finite_differences_p512(ag, oz):
    """Central differences of L = sum W o (A B) in exact integer arithmetic, on the
    64 x 64 x 64, p = 512 subproblem: the gradient of a bilinear loss is the
    difference quotient for any step, so each GPU entry must lie within 1 ulp of it."""
    M = N = K = 64
    p = 512
    A, B, W = synth.grad_operands_for(CFG5_SEED + 100, M, N, K, p, -4, 4)
    Ai, sa = _ints(A)
    Bi, sb = _ints(B)
    Wi, sw = _ints(W)

    def crow(arow):        # one row of C = A B, from the forward definition
        return [sum(arow[k] * Bi[k][j] for k in range(K)) for j in range(N)]

    def ccol(bcol):        # one column of C
        return [sum(Ai[i][k] * bcol[k] for k in range(K)) for i in range(M)]

    def full_loss(Am, Bm):
        return sum(Wi[i][j] * sum(Am[i][k] * Bm[k][j] for k in range(K))
                   for i in range(M) for j in range(N))

    rng = np.random.default_rng(5)
    samp_a = [(int(rng.integers(M)), int(rng.integers(K))) for _ in range(64)]
    samp_b = [(int(rng.integers(K)), int(rng.integers(N))) for _ in range(64)]
    # step h = one unit of A's (B's) integer scale; difference quotient in exact ints
    fd_a, fd_b = [], []
    for (i, k) in samp_a:
        rp = list(Ai[i]); rp[k] += 1
        rm = list(Ai[i]); rm[k] -= 1
        cp, cm = crow(rp), crow(rm)      # only row i of C changes
        diff = sum(Wi[i][j] * (cp[j] - cm[j]) for j in range(N))
        fd_a.append(Fraction(diff, 2) * Fraction(2) ** (sb + sw))
    for (k, j) in samp_b:
        bp = [Bi[kk][j] for kk in range(K)]; bp[k] += 1
        bm = [Bi[kk][j] for kk in range(K)]; bm[k] -= 1
        cp, cm = ccol(bp), ccol(bm)      # only column j of C changes
        diff = sum(Wi[i][j] * (cp[i] - cm[i]) for i in range(M))
        fd_b.append(Fraction(diff, 2) * Fraction(2) ** (sa + sw))
    # the restriction to one row / column is exact: check two samples on the full loss
    for n, (i, k) in enumerate(samp_a[:2]):
        Ap = [list(r) for r in Ai]; Ap[i][k] += 1
        Am = [list(r) for r in Ai]; Am[i][k] -= 1
        d = full_loss(Ap, Bi) - full_loss(Am, Bi)
        assert Fraction(d, 2) * Fraction(2) ** (sb + sw) == fd_a[n]
    for mode in ("reuse", "recompute"):
        print(f"finite differences p=512 mode={mode}", flush=True)
        a = ag.to_carrier(A).requires_grad_()
        b = ag.to_carrier(B).requires_grad_()
        ag.oz_matmul(a, b, p, mode=mode).backward(ag.to_carrier(W))
        ga = _host(ag.from_carrier(a.grad, p))
        gb = _host(ag.from_carrier(b.grad, p))
        for (grid, samples, fds) in ((ga, samp_a, fd_a), (gb, samp_b, fd_b)):
            s, e, l = grid
            for (r, c), g in zip(samples, fds):
                y = _mp_value(s[r, c], e[r, c], l[r, c], p)
                ulp = Fraction(2) ** (int(e[r, c]) - p) if s[r, c] else Fraction(0)
                assert abs(y - g) <= ulp, (mode, r, c)


# ---------------------------------------------------------------- full size

def test_full_size_4096_p256_sampled(oz, c_oracle):
    import torch
    M = N = K = 4096
    p = 256
    t0 = time.time()
    A, B, W = synth.grad_operands_for(CFG5_SEED, M, N, K, p, -4, 4)
    print(f"4096 p=256 backward: inputs {time.time() - t0:.1f}s", flush=True)
    plan = oz.Plan.create_grad(p, M, N, K)
    Ad, Bd, Wd = dev_mp(A), dev_mp(B), dev_mp(W)
    ws = oz.workspace(plan, M, N)
    oz.gemm(plan, Ad, Bd, ws=ws)
    dA, dB = oz.gemm_backward(plan, ws, Wd)
    torch.cuda.synchronize()
    print(f"4096 p=256 backward: gpu done {time.time() - t0:.1f}s", flush=True)
    from tests.test_gpu_parity import sample_entries
    sa = sample_entries(M, K, 16, 256, 1)
    sb = sample_entries(K, N, 16, 256, 2)
    ga = [x[torch.from_numpy(sa[0]).cuda(), torch.from_numpy(sa[1]).cuda()].cpu().numpy()
          for x in (dA.sign, dA.exp, dA.limbs)]
    gb = [x[torch.from_numpy(sb[0]).cuda(), torch.from_numpy(sb[1]).cuda()].cpu().numpy()
          for x in (dB.sign, dB.exp, dB.limbs)]
    del Ad, Bd, Wd, ws, dA, dB
    torch.cuda.empty_cache()
    rA, rB = c_oracle.grad_reuse(A, B, W, sel_a=sa, sel_b=sb, want_chat=False)
    print(f"4096 p=256 backward: oracle done {time.time() - t0:.1f}s", flush=True)
    for (g, r) in ((ga, rA), (gb, rB)):
        assert np.array_equal(g[0], r["c_sign"])
        assert np.array_equal(g[1], r["c_exp"])
        assert np.array_equal(g[2].view(np.uint64), r["c_limbs"])
