"""Pins of the oracle against facts fixed outside it (CPU only).

The oracle (oracle/oz2_ref.py, oracle/oz2_oracle.c) computes the exact integer
product of the shared-exponent integer matrices and one final rounding
(Algorithm section, Eqs. 1-3).  Nothing here re-types that code path:

* brute force with Fractions: exponents are derived from the VALUES (the
  smallest e with |x| < 2^e), integerization uses Python's round() on exact
  rationals, the final rounding uses mpmath's correctly rounded conversion;
* special cases that reduce to textbook routines: when every row/column has an
  exponent spread <= t - p the integerization is exact and the result is the
  correctly rounded exact dot product (mpmath at precision p; Python's
  float(Fraction) at p = 53); K = 1 is a correctly rounded product;
* the paper's invariants (|a^| <= 2^t, |c^| <= K 2^(2t)) and its accuracy
  claim (below one unit 2^-p of relative error, Accuracy section);
* the C oracle against the (pinned) Python oracle, element by element;
* planted mistakes in the Python oracle that these pins must catch.
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import synth
from oracle import oz2_ref as R


def val(sign, mant, exp, p):
    if sign == 0:
        return Fraction(0)
    mant &= (1 << p) - 1
    return sign * Fraction(mant) * Fraction(2) ** (exp - p)


def exp_of(x: Fraction):
    """Smallest integer e with |x| < 2^e (MPFR's exponent), from the value."""
    x = abs(x)
    e = x.numerator.bit_length() - x.denominator.bit_length()
    while x >= Fraction(2) ** e:
        e += 1
    while x < Fraction(2) ** (e - 1):
        e -= 1
    return e


def mp_round(x: Fraction, p: int) -> Fraction:
    """Correctly rounded (nearest-even) p-bit value of a dyadic rational, via mpmath."""
    if x == 0:
        return Fraction(0)
    n, d = x.numerator, x.denominator
    k = d.bit_length() - 1
    assert d == 1 << k
    s, man, ex, _bc = mpmath.libmp.from_man_exp(n, -k, p, "n")
    v = Fraction(man) * Fraction(2) ** ex
    return -v if s else v


def oracle_out_value(trip, p):
    s, m, e = trip
    if s == 0:
        assert m == 0
        return Fraction(0)
    assert (1 << (p - 1)) <= m < (1 << p), "output significand not normalised"
    return s * Fraction(m) * Fraction(2) ** (e - p)


def with_zeros(X, frac, seed):
    rng = np.random.default_rng(seed)
    z = rng.random(X.sign.shape) < frac
    X.sign[z] = 0
    return X


# ---------------------------------------------------------------- pin helpers
# Each returns a list of mismatch descriptions (empty = pinned).

def pin_bruteforce(ref, A, B, guard_bits=16):
    p = A.p
    M, K = A.sign.shape
    N = B.sign.shape[1]
    out = ref.oz2_gemm_ref(A, B, guard_bits=guard_bits)
    t = p + guard_bits + (K - 1).bit_length()
    bad = []
    if out["t"] != t:
        bad.append(("t", out["t"], t))
    av = [[val(*A.value_parts(i, k), p) for k in range(K)] for i in range(M)]
    bv = [[val(*B.value_parts(k, j), p) for j in range(N)] for k in range(K)]
    e = [max([exp_of(x) for x in row if x != 0], default=0) for row in av]
    f = [max([exp_of(bv[k][j]) for k in range(K) if bv[k][j] != 0], default=0) for j in range(N)]
    ah = [[round(av[i][k] * Fraction(2) ** (t - e[i])) for k in range(K)] for i in range(M)]
    bh = [[round(bv[k][j] * Fraction(2) ** (t - f[j])) for j in range(N)] for k in range(K)]
    for i in range(M):
        for j in range(N):
            chat = sum(ah[i][k] * bh[k][j] for k in range(K))
            if out["chat"][i][j] != chat:
                bad.append(("chat", i, j))
            want = mp_round(Fraction(chat) * Fraction(2) ** (e[i] + f[j] - 2 * t), p)
            if oracle_out_value(out["C"][i][j], p) != want:
                bad.append(("C", i, j))
    return bad


def pin_exact_dot(ref, A, B):
    """Exponent spread <= t - p: result must be RNE_p of the exact sum."""
    p = A.p
    M, K = A.sign.shape
    N = B.sign.shape[1]
    out = ref.oz2_gemm_ref(A, B)
    bad = []
    for i in range(M):
        for j in range(N):
            exact = sum(val(*A.value_parts(i, k), p) * val(*B.value_parts(k, j), p)
                        for k in range(K))
            if oracle_out_value(out["C"][i][j], p) != mp_round(exact, p):
                bad.append((i, j))
            if p == 53 and exact != 0:
                y = oracle_out_value(out["C"][i][j], p)
                if float(y) != float(exact):     # CPython rounds rationals correctly (RNE)
                    bad.append(("float", i, j))
    return bad


def pin_invariants(ref, A, B):
    out = ref.oz2_gemm_ref(A, B)
    t = out["t"]
    K = A.sign.shape[1]
    bad = []
    for row in out["Ah"]:
        bad += [("ah", a) for a in row if abs(a) > (1 << t)]
    for col in out["Bh"]:
        bad += [("bh", b) for b in col if abs(b) > (1 << t)]
    for row in out["chat"]:
        bad += [("chat", c) for c in row if abs(c) > K * (1 << (2 * t))]
    return bad


def tie_cases():
    """Constructed operands whose integerization and final rounding hit exact ties."""
    cases = []
    # p = 2: a = (3, 2) * 2^E with exponents 0 and -2, b = (3, 2): c^ = 2^34 * 10 -> tie
    A = synth.mp_zeros(1, 2, 2)
    B = synth.mp_zeros(2, 1, 2)
    A.sign[:] = 1
    B.sign[:] = 1
    A.limbs[0, 0, 0], A.exp[0, 0] = 3, 0
    A.limbs[0, 1, 0], A.exp[0, 1] = 2, -2
    B.limbs[0, 0, 0], B.exp[0, 0] = 3, 0
    B.limbs[1, 0, 0], B.exp[1, 0] = 2, 0
    cases.append((A, B))
    # integerization ties: a huge exponent gap with a 2-bit significand,
    # a = 3*2^(E-2) with E - e = -(t - p) - 1 -> a*2^(t-e) = 1.5 -> rounds to 2;
    # and E - e = -(t - p) - 2 -> 0.75 -> 1; -(t-p) - 3 -> 0.375 -> 0
    for gap in (1, 2, 3):
        A = synth.mp_zeros(1, 2, 2)
        B = synth.mp_zeros(2, 1, 2)
        A.sign[:] = 1
        B.sign[:] = 1
        t = 2 + 16 + 1
        A.limbs[0, 0, 0], A.exp[0, 0] = 2, 0
        A.limbs[0, 1, 0], A.exp[0, 1] = 3, -(t - 2) - gap
        B.limbs[0, 0, 0], B.exp[0, 0] = 2, 0
        B.limbs[1, 0, 0], B.exp[1, 0] = 2, 0
        cases.append((A, B))
    # 2.5 -> 2 and 3.5 -> 4: significands 5 and 7 (p = 3) shifted right by one bit
    for mant in (5, 7):
        A = synth.mp_zeros(1, 2, 3)
        B = synth.mp_zeros(2, 1, 3)
        A.sign[:] = 1
        B.sign[:] = 1
        t = 3 + 16 + 1
        A.limbs[0, 0, 0], A.exp[0, 0] = 4, 0
        A.limbs[0, 1, 0], A.exp[0, 1] = mant, -(t - 3) - 1
        B.limbs[0, 0, 0], B.exp[0, 0] = 4, 0
        B.limbs[1, 0, 0], B.exp[1, 0] = 4, 0
        cases.append((A, B))
    return cases


# ---------------------------------------------------------------- the pins

@pytest.mark.parametrize("p", [2, 3, 8, 16, 53])
@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 4), (4, 4, 3), (3, 2, 5)])
def test_bruteforce_tiny(p, shape):
    M, N, K = shape
    seed = 1000 + 17 * p + 7 * M + 3 * N + K
    A, B = synth.operands_for(seed, M, N, K, p, -40, 40)
    with_zeros(A, 0.2, seed)
    with_zeros(B, 0.2, seed + 1)
    assert pin_bruteforce(R, A, B) == []
    assert pin_bruteforce(R, A, B, guard_bits=0) == []


def test_constructed_ties():
    for A, B in tie_cases():
        assert pin_bruteforce(R, A, B) == []


@pytest.mark.parametrize("p", [53, 64, 113, 128, 200])
def test_exact_dot_special_case(p):
    # exponents in [-4, 4]: spread 8 <= t - p, so Eq. 1 rounds nothing
    A, B = synth.operands_for(77 + p, 3, 4, 9, p, -4, 4)
    with_zeros(A, 0.1, p)
    assert pin_exact_dot(R, A, B) == []


def test_k1_is_correctly_rounded_product():
    for p in (2, 7, 53, 113, 256):
        A, B = synth.operands_for(5 + p, 3, 3, 1, p, -100, 100)
        assert pin_exact_dot(R, A, B) == []


def test_invariants_and_zero_rows():
    A, B = synth.operands_for(9, 5, 4, 8, 64, -70, 70)
    A.sign[2, :] = 0           # an all-zero row of A
    B.sign[:, 1] = 0           # an all-zero column of B
    assert pin_invariants(R, A, B) == []
    out = R.oz2_gemm_ref(A, B)
    assert out["e"][2] == 0 and out["f"][1] == 0
    assert all(out["C"][2][j] == (0, 0, 0) for j in range(4))
    assert all(out["C"][i][1] == (0, 0, 0) for i in range(5))


@pytest.mark.parametrize("p", [53, 113, 212])
def test_accuracy_within_one_unit(p):
    """Accuracy section, table of maximum relative errors: below 1 unit of 2^-p."""
    A, B = synth.operands_for(31 + p, 6, 6, 32, p, -8, 8)
    out = R.oz2_gemm_ref(A, B)
    worst = Fraction(0)
    for i in range(6):
        for j in range(6):
            exact = sum(val(*A.value_parts(i, k), p) * val(*B.value_parts(k, j), p)
                        for k in range(32))
            y = oracle_out_value(out["C"][i][j], p)
            rel = abs(y - exact) / abs(exact) * Fraction(2) ** p
            worst = max(worst, rel)
    assert worst < 1


# ---------------------------------------------------------------- C oracle

CASES = [
    # (seed, M, N, K, p, elo, ehi, zero_frac)
    (1, 7, 5, 9, 128, -4, 4, 0.0),
    (2, 6, 9, 33, 256, -32, 32, 0.05),
    (3, 4, 4, 17, 2, -30, 30, 0.1),
    (4, 5, 3, 12, 53, -200, 200, 0.1),
    (5, 3, 6, 64, 65, -16, 16, 0.0),
    (6, 4, 5, 10, 300, -500, 500, 0.2),
    (7, 2, 3, 5, 1024, -3000, 3000, 0.0),
]


@pytest.mark.parametrize("case", CASES)
def test_c_oracle_matches_python(c_oracle, case):
    seed, M, N, K, p, lo, hi, zf = case
    A, B = synth.operands_for(seed, M, N, K, p, lo, hi)
    with_zeros(A, zf, seed)
    with_zeros(B, zf, seed + 9)
    o = c_oracle.gemm(A, B)
    r = R.oz2_gemm_ref(A, B)
    assert o["t"] == r["t"]
    assert list(o["e"]) == r["e"] and list(o["f"]) == r["f"]
    for i in range(M):
        for j in range(N):
            c = c_oracle.limbs_to_int(o["chat_mag"][i, j]) * int(o["chat_sign"][i, j])
            assert c == r["chat"][i][j]
            got = (int(o["c_sign"][i, j]), c_oracle.limbs_to_int(o["c_limbs"][i, j]),
                   int(o["c_exp"][i, j]))
            assert got == r["C"][i][j]


def test_c_oracle_ties_and_bits_above_p(c_oracle):
    for A, B in tie_cases():
        o = c_oracle.gemm(A, B)
        r = R.oz2_gemm_ref(A, B)
        assert (int(o["c_sign"][0, 0]), c_oracle.limbs_to_int(o["c_limbs"][0, 0]),
                int(o["c_exp"][0, 0])) == r["C"][0][0]
    # garbage above bit p-1 must be ignored by both
    A, B = synth.operands_for(12, 3, 3, 4, 70, -5, 5)
    A.limbs[:, :, 1] |= np.uint64(0xFFFF0000000000C0)
    o = c_oracle.gemm(A, B)
    r = R.oz2_gemm_ref(A, B)
    for i in range(3):
        for j in range(3):
            assert c_oracle.limbs_to_int(o["chat_mag"][i, j]) * int(o["chat_sign"][i, j]) == r["chat"][i][j]


def test_c_oracle_sampled_equals_full(c_oracle):
    A, B = synth.operands_for(21, 40, 33, 50, 192, -20, 20)
    full = c_oracle.gemm(A, B)
    rng = np.random.default_rng(0)
    si = rng.integers(0, 40, 60)
    sj = rng.integers(0, 33, 60)
    part = c_oracle.gemm(A, B, sel=(si, sj))
    assert np.array_equal(part["chat_mag"], full["chat_mag"][si, sj])
    assert np.array_equal(part["c_limbs"], full["c_limbs"][si, sj])
    assert np.array_equal(part["c_exp"], full["c_exp"][si, sj])
    assert np.array_equal(part["c_sign"], full["c_sign"][si, sj])


def test_c_oracle_int32_edge_K(c_oracle):
    """Large K with a single row/column: exercises the accumulator width."""
    A, B = synth.operands_for(44, 1, 1, 5000, 53, -3, 3)
    o = c_oracle.gemm(A, B)
    exact = sum(val(*A.value_parts(0, k), 53) * val(*B.value_parts(k, 0), 53) for k in range(5000))
    y = Fraction(int(o["c_sign"][0, 0])) * c_oracle.limbs_to_int(o["c_limbs"][0, 0]) * \
        Fraction(2) ** (int(o["c_exp"][0, 0]) - 53)
    assert y == mp_round(exact, 53)


# ---------------------------------------------------------------- planted mistakes

def _mutants():
    import types

    def half_up(x, shift):
        if shift <= 0:
            return x << (-shift)
        return (x + (1 << (shift - 1))) >> shift

    def truncate(x, shift):
        return x >> shift if shift > 0 else x << (-shift)

    def width_no_log(p, K, guard_bits=16, t_bits=0):
        return p + guard_bits

    def bad_int_sign(sign, mant, exp, e, t, p):
        v = R.integerize(sign, mant, exp, e, t, p)
        return abs(v)

    def bad_scale_round(c, scale, p):
        s, m, e = R.round_to_precision(c, scale, p)
        return (s, m, e + 1) if s else (s, m, e)

    def bad_exp_min(entries):
        exps = [e for (s, _m, e) in entries if s != 0]
        return min(exps) if exps else 0

    muts = {
        "round_half_up": {"round_half_even_shift": half_up},
        "truncate": {"round_half_even_shift": truncate},
        "t_without_log2K": {"internal_width": width_no_log},
        "sign_dropped": {"integerize": bad_int_sign},
        "exp_off_by_one": {"round_to_precision": bad_scale_round},
        "shared_exp_min": {"shared_exponent": bad_exp_min},
    }
    out = {}
    for name, patch in muts.items():
        mod = types.ModuleType("mut_" + name)
        mod.__dict__.update({k: v for k, v in R.__dict__.items() if not k.startswith("__")})
        mod.__dict__.update(patch)
        # rebind module-level functions so that they see the patched globals
        for k, v in list(mod.__dict__.items()):
            if isinstance(v, types.FunctionType) and v.__module__ == R.__name__ and k not in patch:
                mod.__dict__[k] = types.FunctionType(v.__code__, mod.__dict__, k,
                                                     v.__defaults__, v.__closure__)
        out[name] = mod
    return out


def _pins_fail(mod):
    fails = 0
    for A, B in tie_cases():
        fails += len(pin_bruteforce(mod, A, B))
    for p in (2, 8, 53):
        A, B = synth.operands_for(5000 + p, 3, 3, 4, p, -40, 40)
        fails += len(pin_bruteforce(mod, A, B))
    A, B = synth.operands_for(6000, 3, 3, 5, 113, -4, 4)
    fails += len(pin_exact_dot(mod, A, B))
    return fails


def test_pins_catch_planted_mistakes():
    assert _pins_fail(R) == 0
    for name, mod in _mutants().items():
        assert _pins_fail(mod) > 0, f"pins missed the planted mistake {name}"


def _brute_integerize(X, t, side):
    """Shared exponents and integers of one operand from the VALUES: e = the largest
    exponent (smallest e with |x| < 2^e) over the nonzero entries of a row of A or a
    column of B, 0 when there is none, and a^ = Python round() (ties to even) of the
    exact rational x 2^(t - e) (Eq. 1)."""
    p = X.p
    R_, C_ = X.sign.shape
    lines = range(R_) if side == "A" else range(C_)
    es, ints = [], []
    for r in lines:
        idx = [(r, k) for k in range(C_)] if side == "A" else [(k, r) for k in range(R_)]
        vals = [val(*X.value_parts(i, j), p) for (i, j) in idx]
        nz = [exp_of(v) for v in vals if v != 0]
        e = max(nz) if nz else 0
        es.append(e)
        ints.append([round(v * Fraction(2) ** (t - e)) for v in vals])
    return es, ints


@pytest.mark.parametrize("side", ["A", "B"])
@pytest.mark.parametrize("p,lo,hi,shape", [(2, -30, 30, (5, 7)), (53, -200, 200, (6, 9)),
                                           (130, -4, 4, (4, 5)), (64, -80, 80, (7, 3))])
def test_c_integerize_against_values(c_oracle, side, p, lo, hi, shape):
    """The C oracle's integerization (the checker of the stage-1/2 GPU tests) against
    Fractions, on both sides (row exponents of A, column exponents of B and its strided
    layout), with wide exponent spreads (many entries round to 0 or to ties), an all-zero
    line and bits above p set in the stored significands."""
    rows, cols = shape
    X = synth.mp_random(7 * p + rows, rows, cols, p, lo, hi)
    X.sign[1, :] = 0                      # an all-zero row (a zero line of side A)
    X.sign[:, 2] = 0                      # an all-zero column (side B)
    nl = X.limbs.shape[-1]
    top = p - 64 * (nl - 1)
    if top < 64:                          # garbage above bit p - 1 is ignored
        X.limbs[0, 0, nl - 1] |= np.uint64(1) << np.uint64(top)
    t = R.internal_width(p, cols if side == "A" else rows)
    e, sg, mag = c_oracle.integerize(X, t, side)
    be, bints = _brute_integerize(X, t, side)
    assert e.tolist() == be
    got = [[int(s) * int(sum(int(x) << (64 * l) for l, x in enumerate(m))) for s, m in zip(srow, mrow)]
           for srow, mrow in zip(sg, mag)]
    assert got == bints
    # the invariant of Eq. 1
    assert all(abs(v) <= 1 << t for row in got for v in row)


def test_c_integerize_ties():
    """Constructed ties of the integerization (2.5 -> 2, 3.5 -> 4, 1.5 -> 2, 0.5 -> 0)
    through the C oracle, both sides, against Python's round()."""
    from oracle import c_oracle
    cases = tie_cases()
    for (A, B) in cases:
        p = A.p
        K = A.sign.shape[1]
        t = R.internal_width(p, K)
        for X, side in ((A, "A"), (B, "B")):
            e, sg, mag = c_oracle.integerize(X, t, side)
            be, bints = _brute_integerize(X, t, side)
            got = [[int(s) * int(sum(int(x) << (64 * l) for l, x in enumerate(m)))
                    for s, m in zip(srow, mrow)] for srow, mrow in zip(sg, mag)]
            assert e.tolist() == be and got == bints
