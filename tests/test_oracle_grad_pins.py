"""Pins of the backward-product oracle (autograd form) against facts fixed outside it.

For L(A, B) = sum_ij W_ij (A B)_ij the gradients are dL/dA = W B^T and
dL/dB = A^T W.  L is bilinear, so a central difference evaluated in exact
rational arithmetic equals the gradient exactly for any step h; the pins below
take that difference of the loss (computed from the forward definition, never
from a gradient formula) as the truth:

* when every integerization is exact (small exponent spreads), both backward
  readings (reuse with exponent folding, and recompute) must equal the
  correctly rounded finite difference, element by element;
* with wide spreads the reuse reading must stay within its derived error bound;
* the C oracle must equal the Python oracle element by element (both readings);
* planted mistakes in the Python backward oracle must be caught.
"""
import inspect
import types
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import oz2_ref as R
from tests.test_oracle_pins import mp_round, oracle_out_value, val


def values(X):
    r, c = X.sign.shape
    return [[val(*X.value_parts(i, j), X.p) for j in range(c)] for i in range(r)]


def loss(av, bv, wv):
    """sum_ij W_ij (A B)_ij, exactly, from the forward definition."""
    M, K, N = len(av), len(bv), len(bv[0])
    return sum(wv[i][j] * sum(av[i][k] * bv[k][j] for k in range(K))
               for i in range(M) for j in range(N))


def fd_gradients(A, B, W, h=Fraction(3, 7)):
    """Central differences of the exact loss in every entry of A and of B."""
    av, bv, wv = values(A), values(B), values(W)
    M, K, N = len(av), len(bv), len(bv[0])
    gA = [[None] * K for _ in range(M)]
    gB = [[None] * N for _ in range(K)]
    for i in range(M):
        for k in range(K):
            ap = [row[:] for row in av]
            am = [row[:] for row in av]
            ap[i][k] += h
            am[i][k] -= h
            gA[i][k] = (loss(ap, bv, wv) - loss(am, bv, wv)) / (2 * h)
    for k in range(K):
        for j in range(N):
            bp = [row[:] for row in bv]
            bm = [row[:] for row in bv]
            bp[k][j] += h
            bm[k][j] -= h
            gB[k][j] = (loss(av, bp, wv) - loss(av, bm, wv)) / (2 * h)
    return gA, gB


def grad_inputs(seed, M, N, K, p, elo, ehi, welo=-3, wehi=0):
    A, B = synth.operands_for(seed, M, N, K, p, elo, ehi)
    W = synth.mp_random(seed + 7, M, N, p, welo, wehi, counter=0)
    return A, B, W


def pin_grad_exact(ref, A, B, W):
    """Exact integerization: dA, dB must be RNE_p of the finite-difference gradient."""
    p = A.p
    out = ref.oz2_grad_ref(A, B, W)
    gA, gB = fd_gradients(A, B, W)
    bad = []
    for i, row in enumerate(gA):
        for k, g in enumerate(row):
            if oracle_out_value(out["dA"][i][k], p) != mp_round(g, p):
                bad.append(("dA", i, k))
    for k, row in enumerate(gB):
        for j, g in enumerate(row):
            if oracle_out_value(out["dB"][k][j], p) != mp_round(g, p):
                bad.append(("dB", k, j))
    return bad


def pin_recompute_exact(A, B, W):
    """The recompute reading is the plain product of the transposes."""
    p = A.p
    gA, gB = fd_gradients(A, B, W)
    oa = R.oz2_gemm_ref(W, B.transpose())
    ob = R.oz2_gemm_ref(A.transpose(), W)
    bad = [("dA", i, k) for i, row in enumerate(gA) for k, g in enumerate(row)
           if oracle_out_value(oa["C"][i][k], p) != mp_round(g, p)]
    bad += [("dB", k, j) for k, row in enumerate(gB) for j, g in enumerate(row)
            if oracle_out_value(ob["C"][k][j], p) != mp_round(g, p)]
    return bad


@pytest.mark.parametrize("p", [8, 53, 113, 512])
@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 5, 4), (4, 2, 3), (5, 3, 2)])
def test_grad_exact_integerization(p, shape):
    M, N, K = shape
    A, B, W = grad_inputs(900 + p + 10 * M + N, M, N, K, p, -4, 4)
    assert pin_grad_exact(R, A, B, W) == []
    assert pin_recompute_exact(A, B, W) == []


def test_grad_zero_rows_and_columns():
    A, B, W = grad_inputs(77, 4, 5, 3, 53, -4, 4)
    W.sign[1, :] = 0          # a zero row of W: dA row 1 is zero
    W.sign[:, 2] = 0          # a zero column of W: dB column 2 is zero
    A.sign[:, 0] = 0
    assert pin_grad_exact(R, A, B, W) == []
    out = R.oz2_grad_ref(A, B, W)
    assert all(s == 0 for (s, _m, _e) in out["dA"][1])
    assert all(out["dB"][k][2][0] == 0 for k in range(3))
    assert out["h"][1] == 0 and out["g"][2] == 0


@pytest.mark.parametrize("p", [16, 53])
def test_grad_reuse_error_bound_wide_spread(p):
    """Wide exponent spreads make the integerizations inexact; the reuse reading stays
    within N 2^h_i (2^-t_wA + 2^-t) + ulp_p (and the same for dB), derived from
    |W'^ 2^(h-t_w) - W 2^f| <= 2^(h-t_w-1) and |b^ 2^-t - b 2^-f| <= 2^(-t-1)."""
    M, N, K = 4, 6, 5
    A, B, W = grad_inputs(31 + p, M, N, K, p, -40, 40, -60, 10)
    out = R.oz2_grad_ref(A, B, W)
    t, twa, twb = out["t"], out["tw"][0], out["tw"][1]
    gA, gB = fd_gradients(A, B, W)
    for i in range(M):
        for k in range(K):
            y = oracle_out_value(out["dA"][i][k], p)
            ulp = Fraction(2) ** (out["dA"][i][k][2] - p) if y else 0
            bound = N * Fraction(2) ** out["h"][i] * (Fraction(2) ** -twa + Fraction(2) ** -t) + ulp
            assert abs(y - gA[i][k]) <= bound
    for k in range(K):
        for j in range(N):
            y = oracle_out_value(out["dB"][k][j], p)
            ulp = Fraction(2) ** (out["dB"][k][j][2] - p) if y else 0
            bound = M * Fraction(2) ** out["g"][j] * (Fraction(2) ** -twb + Fraction(2) ** -t) + ulp
            assert abs(y - gB[k][j]) <= bound


def _c_result_equals(res, trips, p):
    for idx in np.ndindex(res["c_sign"].shape):
        s, m, e = trips[idx[0]][idx[1]]
        if int(res["c_sign"][idx]) != s:
            return False
        if s and (int(res["c_exp"][idx]) != e or
                  R_limbs(res["c_limbs"][idx]) != m):
            return False
    return True


def R_limbs(limbs):
    v = 0
    for x in reversed([int(y) for y in limbs]):
        v = (v << 64) | x
    return v


@pytest.mark.parametrize("case", [(5, 7, 6, 113, -4, 4, -3, 0), (9, 4, 11, 256, -30, 30, -50, 5),
                                  (6, 6, 6, 53, -200, 200, -9, 9), (3, 8, 2, 1024, -8, 8, -4, 0)])
def test_c_grad_oracle_matches_python(c_oracle, case):
    M, N, K, p, lo, hi, wlo, whi = case
    A, B, W = grad_inputs(4000 + p, M, N, K, p, lo, hi, wlo, whi)
    W.sign[0, 1] = 0
    ref = R.oz2_grad_ref(A, B, W)
    dA, dB = c_oracle.grad_reuse(A, B, W)
    assert list(dA["e"]) == ref["h"] and list(dB["f"]) == ref["g"]
    assert _c_result_equals(dA, ref["dA"], p)
    assert _c_result_equals(dB, ref["dB"], p)
    for (res, chat) in ((dA, ref["chat_a"]), (dB, ref["chat_b"])):
        for idx in np.ndindex(res["chat_sign"].shape):
            v = int(res["chat_sign"][idx]) * R_limbs(res["chat_mag"][idx])
            assert v == chat[idx[0]][idx[1]]
    # recompute reading = plain products of the transposes
    rA, rB = c_oracle.grad_recompute(A, B, W)
    assert _c_result_equals(rA, R.oz2_gemm_ref(W, B.transpose())["C"], p)
    assert _c_result_equals(rB, R.oz2_gemm_ref(A.transpose(), W)["C"], p)


def test_c_grad_sampled_equals_full(c_oracle):
    A, B, W = grad_inputs(55, 20, 17, 13, 128, -16, 16, -8, 0)
    fa, fb = c_oracle.grad_reuse(A, B, W)
    si = np.array([0, 19, 7, 3]), np.array([0, 12, 5, 12])
    sj = np.array([12, 0, 4]), np.array([16, 3, 9])
    sa, sb = c_oracle.grad_reuse(A, B, W, sel_a=si, sel_b=sj)
    for (full, samp, sel) in ((fa, sa, si), (fb, sb, sj)):
        for key in ("c_sign", "c_exp", "c_limbs", "chat_sign", "chat_mag"):
            assert np.array_equal(full[key][sel[0], sel[1]], samp[key])


# ---------------------------------------------------------------- planted mistakes

GRAD_MUTANTS = {
    "fold_sign_flipped": ("x + f[j]", "x - f[j]"),
    "fold_dropped": ("x + f[j], h[i]", "x, h[i]"),
    "dA_scale_without_t": ("h[i] - twa - t", "h[i] - twa"),
    "dB_width_swapped": ("g[j] - twb - t", "g[j] - twa - t"),
    "dB_fold_from_f": ("w[i][j][2] + e[i], g[j]", "w[i][j][2] + f[j % K], g[j]"),
}


def _grad_mutant(old, new):
    src = inspect.getsource(R.oz2_grad_ref)
    assert old in src
    ns = dict(R.__dict__)
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    mod = types.SimpleNamespace(oz2_grad_ref=ns["oz2_grad_ref"])
    return mod


def _grad_pins_fail(mod):
    fails = 0
    for (seed, M, N, K, p) in ((1, 3, 5, 4, 53), (2, 4, 2, 3, 16), (3, 2, 3, 5, 113)):
        A, B, W = grad_inputs(seed, M, N, K, p, -4, 4)
        fails += len(pin_grad_exact(mod, A, B, W))
    return fails


def test_grad_pins_catch_planted_mistakes():
    assert _grad_pins_fail(R) == 0
    for name, (old, new) in GRAD_MUTANTS.items():
        assert _grad_pins_fail(_grad_mutant(old, new)) > 0, f"pins missed {name}"
