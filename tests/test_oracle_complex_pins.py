"""Pins of the complex-product oracle against facts fixed outside it (CPU only).

The oracle (oz2_ref.oz2_zgemm_ref; c_oracle.zgemm through the real C oracle) computes
the exact integers Re and Im of the shared-exponent integer matrices' complex product
and rounds each once (Conclusions, "Complex matrix products", with Eqs. 1-3).  The pins:

* brute force with Fractions: exponents derived from the VALUES of both parts,
  integers by Python's round() on exact rationals, final rounding by mpmath;
* the special case with no integerization error: each part is the correctly rounded
  real or imaginary part of the exact complex dot product;
* exact symmetries of the definition: (i A) B = i (A B), conj(A) conj(B) = conj(A B),
  (A B)^T = B^T A^T, and a purely real product equals the real oracle at the same t;
* the C route (two real products of length 2K) against the Python definition;
* planted mistakes in the Python oracle that these pins must catch.
"""
import inspect
import types
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import oz2_ref as R
from tests.test_oracle_pins import exp_of, mp_round, oracle_out_value, val, with_zeros


def zoperands(seed, M, N, K, p, lo, hi, zf=0.0):
    Ar, Br = synth.operands_for(seed, M, N, K, p, lo, hi)
    Ai, Bi = synth.operands_for(seed + 7919, M, N, K, p, lo, hi)
    if zf:
        for n, X in enumerate((Ar, Ai, Br, Bi)):
            with_zeros(X, zf, seed + n)
    return Ar, Ai, Br, Bi


def neg(X):
    return synth.MPMatrix(-X.sign, X.exp.copy(), X.limbs.copy(), X.p)


def pin_zbrute(ref, Ar, Ai, Br, Bi, guard_bits=16):
    p = Ar.p
    M, K = Ar.sign.shape
    N = Br.sign.shape[1]
    out = ref.oz2_zgemm_ref(Ar, Ai, Br, Bi, guard_bits=guard_bits)
    t = p + guard_bits + (2 * K - 1).bit_length()
    bad = []
    if out["t"] != t:
        bad.append(("t", out["t"], t))
    ar = [[val(*Ar.value_parts(i, k), p) for k in range(K)] for i in range(M)]
    ai = [[val(*Ai.value_parts(i, k), p) for k in range(K)] for i in range(M)]
    br = [[val(*Br.value_parts(k, j), p) for j in range(N)] for k in range(K)]
    bi = [[val(*Bi.value_parts(k, j), p) for j in range(N)] for k in range(K)]
    e = [max([exp_of(x) for x in ar[i] + ai[i] if x != 0], default=0) for i in range(M)]
    f = [max([exp_of(X[k][j]) for X in (br, bi) for k in range(K) if X[k][j] != 0], default=0)
         for j in range(N)]
    sa = [Fraction(2) ** (t - e[i]) for i in range(M)]
    sb = [Fraction(2) ** (t - f[j]) for j in range(N)]
    for i in range(M):
        for j in range(N):
            cre = sum(round(ar[i][k] * sa[i]) * round(br[k][j] * sb[j]) -
                      round(ai[i][k] * sa[i]) * round(bi[k][j] * sb[j]) for k in range(K))
            cim = sum(round(ar[i][k] * sa[i]) * round(bi[k][j] * sb[j]) +
                      round(ai[i][k] * sa[i]) * round(br[k][j] * sb[j]) for k in range(K))
            if out["chat_re"][i][j] != cre:
                bad.append(("chat_re", i, j))
            if out["chat_im"][i][j] != cim:
                bad.append(("chat_im", i, j))
            sc = Fraction(2) ** (e[i] + f[j] - 2 * t)
            if oracle_out_value(out["Cr"][i][j], p) != mp_round(cre * sc, p):
                bad.append(("Cr", i, j))
            if oracle_out_value(out["Ci"][i][j], p) != mp_round(cim * sc, p):
                bad.append(("Ci", i, j))
    return bad


def pin_zexact(ref, Ar, Ai, Br, Bi):
    """Exponent spread <= t - p: each part is RNE_p of the exact complex dot product."""
    p = Ar.p
    M, K = Ar.sign.shape
    N = Br.sign.shape[1]
    out = ref.oz2_zgemm_ref(Ar, Ai, Br, Bi)
    bad = []
    for i in range(M):
        for j in range(N):
            z = sum(complex_fr(Ar, Ai, i, k, p) * complex_fr(Br, Bi, k, j, p)
                    for k in range(K))
            if oracle_out_value(out["Cr"][i][j], p) != mp_round(z.re, p):
                bad.append(("Cr", i, j))
            if oracle_out_value(out["Ci"][i][j], p) != mp_round(z.im, p):
                bad.append(("Ci", i, j))
    return bad


class ZF:
    """An exact complex number with Fraction parts (textbook multiplication)."""

    def __init__(self, re, im):
        self.re, self.im = Fraction(re), Fraction(im)

    def __mul__(self, o):
        return ZF(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    def __add__(self, o):
        return ZF(self.re + o.re, self.im + o.im)

    def __radd__(self, o):
        return self if o == 0 else self + o


def complex_fr(Xr, Xi, r, c, p):
    return ZF(val(*Xr.value_parts(r, c), p), val(*Xi.value_parts(r, c), p))


def negate_trip(tr):
    s, m, e = tr
    return (-s, m, e)


def pin_zsymmetries(ref, Ar, Ai, Br, Bi):
    """Exact identities of the definition (any mistake in an index, a sign or the
    exponent sharing breaks one of them)."""
    M, K = Ar.sign.shape
    N = Br.sign.shape[1]
    base = ref.oz2_zgemm_ref(Ar, Ai, Br, Bi)
    bad = []
    # (i A) B = i (A B): i A = -Ai + i Ar
    rot = ref.oz2_zgemm_ref(neg(Ai), Ar, Br, Bi)
    # conj(A) conj(B) = conj(A B)
    cj = ref.oz2_zgemm_ref(Ar, neg(Ai), Br, neg(Bi))
    # (A B)^T = B^T A^T
    tr = ref.oz2_zgemm_ref(Br.transpose(), Bi.transpose(), Ar.transpose(), Ai.transpose())
    for i in range(M):
        for j in range(N):
            if rot["Cr"][i][j] != negate_trip(base["Ci"][i][j]) or rot["Ci"][i][j] != base["Cr"][i][j]:
                bad.append(("i*A", i, j))
            if cj["Cr"][i][j] != base["Cr"][i][j] or cj["Ci"][i][j] != negate_trip(base["Ci"][i][j]):
                bad.append(("conj", i, j))
            if tr["Cr"][j][i] != base["Cr"][i][j] or tr["Ci"][j][i] != base["Ci"][i][j]:
                bad.append(("transpose", i, j))
    # a real product: Im = 0 and Re = the real oracle at the complex product's t
    zr = ref.oz2_zgemm_ref(Ar, synth.mp_zeros(M, K, Ar.p), Br, synth.mp_zeros(K, N, Ar.p))
    real = R.oz2_gemm_ref(Ar, Br, t_bits=zr["t"])
    for i in range(M):
        for j in range(N):
            if zr["Ci"][i][j] != (0, 0, 0):
                bad.append(("real-im", i, j))
            if zr["Cr"][i][j] != real["C"][i][j]:
                bad.append(("real-re", i, j))
    return bad


# ---------------------------------------------------------------- the pins

@pytest.mark.parametrize("p", [2, 5, 53, 70])
@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 4), (3, 2, 5)])
def test_zbruteforce_tiny(p, shape):
    M, N, K = shape
    ops = zoperands(300 + 13 * p + 5 * M + N + K, M, N, K, p, -40, 40, zf=0.2)
    assert pin_zbrute(R, *ops) == []
    assert pin_zbrute(R, *ops, guard_bits=0) == []


@pytest.mark.parametrize("p", [53, 113, 200])
def test_zexact_special_case(p):
    ops = zoperands(90 + p, 3, 3, 7, p, -4, 4)
    assert pin_zexact(R, *ops) == []


@pytest.mark.parametrize("p,lo,hi", [(8, -30, 30), (64, -200, 200), (128, -6, 6)])
def test_zsymmetries(p, lo, hi):
    ops = zoperands(500 + p, 3, 4, 5, p, lo, hi, zf=0.1)
    assert pin_zsymmetries(R, *ops) == []


def test_zero_rows_and_parts():
    Ar, Ai, Br, Bi = zoperands(71, 4, 3, 6, 96, -50, 50)
    Ar.sign[1, :] = 0
    Ai.sign[1, :] = 0          # an all-zero row of A
    Ai.sign[2, :] = 0          # a purely real row: its exponent comes from Ar alone
    Br.sign[:, 0] = 0          # a purely imaginary column of B
    out = R.oz2_zgemm_ref(Ar, Ai, Br, Bi)
    assert out["e"][1] == 0
    assert out["e"][2] == max(int(x) for x in Ar.exp[2])
    assert out["f"][0] == max(int(x) for x in Bi.exp[:, 0])
    assert all(out["Cr"][1][j] == (0, 0, 0) and out["Ci"][1][j] == (0, 0, 0) for j in range(3))
    assert pin_zbrute(R, Ar, Ai, Br, Bi) == []


@pytest.mark.parametrize("p", [53, 113, 212])
def test_zaccuracy(p):
    """Each part within one unit 2^-p of relative error of the exact part (the
    Accuracy section's claim, for the sums of 2K products the parts are)."""
    Ar, Ai, Br, Bi = zoperands(41 + p, 4, 4, 16, p, -8, 8)
    out = R.oz2_zgemm_ref(Ar, Ai, Br, Bi)
    worst = Fraction(0)
    for i in range(4):
        for j in range(4):
            z = sum(complex_fr(Ar, Ai, i, k, p) * complex_fr(Br, Bi, k, j, p) for k in range(16))
            for got, ex in ((out["Cr"][i][j], z.re), (out["Ci"][i][j], z.im)):
                y = oracle_out_value(got, p)
                worst = max(worst, abs(y - ex) / abs(ex) * Fraction(2) ** p)
    assert worst < 1


ZCASES = [
    # (seed, M, N, K, p, elo, ehi, zero_frac)
    (1, 5, 4, 9, 113, -4, 4, 0.0),
    (2, 4, 6, 17, 256, -32, 32, 0.05),
    (3, 3, 3, 8, 2, -30, 30, 0.1),
    (4, 4, 2, 12, 53, -200, 200, 0.1),
    (5, 2, 5, 5, 700, -900, 900, 0.0),
]


@pytest.mark.parametrize("case", ZCASES)
def test_c_zgemm_matches_python(c_oracle, case):
    seed, M, N, K, p, lo, hi, zf = case
    ops = zoperands(seed, M, N, K, p, lo, hi, zf)
    re, im = c_oracle.zgemm(*ops, want_chat=True)
    r = R.oz2_zgemm_ref(*ops)
    assert re["t"] == r["t"] and im["t"] == r["t"]
    assert list(re["e"]) == r["e"] and list(re["f"]) == r["f"]
    assert list(im["e"]) == r["e"] and list(im["f"]) == r["f"]
    for o, ck, Ck in ((re, "chat_re", "Cr"), (im, "chat_im", "Ci")):
        for i in range(M):
            for j in range(N):
                c = c_oracle.limbs_to_int(o["chat_mag"][i, j]) * int(o["chat_sign"][i, j])
                assert c == r[ck][i][j]
                got = (int(o["c_sign"][i, j]), c_oracle.limbs_to_int(o["c_limbs"][i, j]),
                       int(o["c_exp"][i, j]))
                assert got == r[Ck][i][j]


def test_c_zgemm_sampled_equals_full(c_oracle):
    ops = zoperands(23, 30, 20, 40, 160, -20, 20)
    full = c_oracle.zgemm(*ops)
    rng = np.random.default_rng(3)
    si, sj = rng.integers(0, 30, 50), rng.integers(0, 20, 50)
    part = c_oracle.zgemm(*ops, sel=(si, sj))
    for f, q in zip(full, part):
        for k in ("c_sign", "c_exp", "c_limbs"):
            assert np.array_equal(q[k], f[k][si, sj])


# ---------------------------------------------------------------- planted mistakes

def _zmutants():
    src = inspect.getsource(R.oz2_zgemm_ref)
    edits = {
        "im_bi_sign_flip": ("sum(arh[i][k] * brh[j][k] - aih[i][k] * bih[j][k]",
                            "sum(arh[i][k] * brh[j][k] + aih[i][k] * bih[j][k]"),
        "exponent_from_real_part": ("shared_exponent(ar[i] + ai[i])", "shared_exponent(ar[i])"),
        "column_exponent_from_real_part": ("shared_exponent(br[j] + bi[j])", "shared_exponent(br[j])"),
        "t_from_K": ("internal_width(p, 2 * K,", "internal_width(p, K,"),
        "im_wrong_operand": ("aih[i][k] * brh[j][k] for k", "aih[i][k] * bih[j][k] for k"),
        "b_transposed_index": ("brh = [[integerize(s, m, x, f[j], t, p) for (s, m, x) in br[j]]",
                               "brh = [[integerize(s, m, x, f[j], t, p) for (s, m, x) in br[j][::-1]]"),
    }
    out = {}
    for name, (old, new) in edits.items():
        assert src.count(old) == 1, f"mutant {name}: pattern not found once"
        mod = types.ModuleType("zmut_" + name)
        mod.__dict__.update({k: v for k, v in R.__dict__.items() if not k.startswith("__")})
        exec(compile(src.replace(old, new), "<" + name + ">", "exec"), mod.__dict__)
        out[name] = mod
    return out


def _zpins_fail(mod):
    fails = 0
    for p in (5, 53):
        fails += len(pin_zbrute(mod, *zoperands(7000 + p, 2, 3, 4, p, -40, 40)))
    fails += len(pin_zexact(mod, *zoperands(7100, 2, 2, 5, 113, -4, 4)))
    try:
        fails += len(pin_zsymmetries(mod, *zoperands(7200, 3, 2, 4, 64, -30, 30)))
    except Exception:   # a mutant that breaks a shape counts as caught
        fails += 1
    return fails


def test_zpins_catch_planted_mistakes():
    assert _zpins_fail(R) == 0
    for name, mod in _zmutants().items():
        assert _zpins_fail(mod) > 0, f"pins missed the planted mistake {name}"
