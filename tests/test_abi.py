"""Host-only checks of the C ABI (no GPU needed, no compute calls).

* the built library exports every function include/oz2h.h declares, and the
  Python binding declares a signature for each of them;
* moduli selection (host only) reproduces the paper's Table "Moduli
  configuration" and the text constants of its subsection "(a) AMX-INT8
  backend" (tests/golden/tab_moduli.txt);
* the selection's argument errors.
"""
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "oz2h.h")
GOLDEN = os.path.join(ROOT, "tests", "golden", "tab_moduli.txt")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \t\*]*?\b(oz2h_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def oz():
    from paper_2609_27831_amd import oz2h
    if not os.path.exists(oz2h.LIB_PATH):
        from paper_2609_27831_amd import build
        build.build()
    return oz2h


def test_header_declares_the_api():
    names = declared_functions()
    for n in ("oz2h_gemm", "oz2h_plan_create", "oz2h_batched_run", "oz2h_gemm_backward",
              "oz2h_carrier_pack", "oz2h_crt"):
        assert n in names
    assert len(names) >= 30


def test_library_exports_every_declared_symbol(oz):
    import ctypes
    L = ctypes.CDLL(oz.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert missing == []
    assert sorted(oz.SIGNATURES) == declared_functions()
    oz.lib()   # every signature binds


def _golden():
    rows, consts = [], {}
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if not line:
            continue
        if line.startswith("const"):
            _, k, v = line.split()
            consts[k] = float(v)
        else:
            rows.append(tuple(int(x) for x in line.split()))
    return rows, consts


def test_plan_moduli_reproduces_the_moduli_table(oz):
    rows, _ = _golden()
    assert len(rows) == 8
    for (p, t, L, G, log2p_up) in rows:
        r = oz.plan_moduli(p, 4096)
        assert (r["t"], r["L"], r["G"]) == (t, L, G), p
        assert math.ceil(r["log2P"]) == log2p_up, p


def test_moduli_list_text_constants(oz):
    _, c = _golden()
    mods = [int(m) for m in oz.plan_moduli(2048, 4096)["moduli"]]
    one = [m for m in mods if m <= 255]
    two = [m for m in mods if m > 255]
    assert len(one) == c["n_one_limb"]
    assert round(sum(math.log2(m) for m in one), 1) == c["log2_prod_one_limb"]
    assert round(math.log2(one[0]), 2) == c["top_bits"]
    assert round(sum(math.log2(m) for m in one) / len(one), 2) == c["mean_bits"]
    assert round(math.log2(two[0]), 2) == c["two_limb_bits"]
    # one-limb: the largest power of every prime <= 255, decreasing
    assert one == sorted(one, reverse=True) and two == sorted(two, reverse=True)
    for m in one:
        q = min(d for d in range(2, m + 1) if m % d == 0)
        x = q
        while x * q <= 255:
            x *= q
        assert x == m
    for i, a in enumerate(mods):
        for b in mods[:i]:
            assert math.gcd(a, b) == 1


def test_plan_moduli_errors(oz):
    with pytest.raises(oz.Oz2hError) as ei:
        oz.plan_moduli(1, 16)
    assert ei.value.code == oz.EINVAL
    with pytest.raises(oz.Oz2hError) as ei:
        oz.plan_moduli(64, 200000)
    assert ei.value.code == oz.ERANGE
    with pytest.raises(oz.Oz2hError) as ei:
        oz.plan_moduli(4000, 4096)        # beyond 512 moduli
    assert ei.value.code == oz.ERANGE
    with pytest.raises(oz.Oz2hError) as ei:
        oz.plan_moduli(64, 16, oz.default_opts(crt_margin=0))
    assert ei.value.code == oz.EINVAL


# ---------------------------------------------------------------- binary64 and mixed backends

GOLDEN_F64 = os.path.join(ROOT, "tests", "golden", "tab_moduli_binary64.txt")


def _is_prime(n):
    if n < 2:
        return False
    f = 2
    while f * f <= n:
        if n % f == 0:
            return False
        f += 1
    return True


def test_plan_moduli_reproduces_the_binary64_half(oz):
    """Table "Moduli configuration", binary64 columns: L, DGEMMs and log2 P (rounded up)
    at K = 4096, with the moduli bounded by Eq. fp64bound."""
    rows = [tuple(int(x) for x in l.split("#")[0].split())
            for l in open(GOLDEN_F64) if l.split("#")[0].strip()]
    assert len(rows) == 8
    o = oz.default_opts(flags=oz.FLAG_BACKEND_F64)
    for (p, t, L, G, log2p_up) in rows:
        r = oz.plan_moduli32(p, 4096, o)
        assert (r["t"], r["L"], r["G"], r["L8"]) == (t, L, G, 0), p
        assert math.ceil(r["log2P"]) == log2p_up, p
    mods = [int(m) for m in oz.plan_moduli32(2048, 4096, o)["moduli"]]
    # Eq. fp64bound: m <= sqrt(2^55 / K) = 2965821 (text of the same subsection)
    assert mods[0] <= 2965821 and mods == sorted(mods, reverse=True)
    assert all(_is_prime(m) for m in mods[:12])
    assert all(4096 * ((m - 1) // 2) ** 2 < 2 ** 53 for m in mods)
    assert len(set(mods)) == len(mods)


def test_binary64_bound_follows_K(oz):
    o = oz.default_opts(flags=oz.FLAG_BACKEND_F64)
    for K in (1, 1000, 2048, 4096, 65536, 133000):
        m = int(oz.plan_moduli32(53, K, o)["moduli"][0])
        assert K * ((m - 1) // 2) ** 2 < 2 ** 53
        assert m < 2 ** 22                    # two 11-bit CRT terms per residue
        # the largest prime under the bound (and under 2^22)
        bound = min(math.isqrt(2 ** 55 // K), 2 ** 22 - 1)
        while not _is_prime(bound):
            bound -= 1
        assert m == bound, K


def test_mixed_moduli(oz):
    o = oz.default_opts(flags=oz.FLAG_BACKEND_MIXED)
    for p in (53, 256, 2048):
        r = oz.plan_moduli32(p, 4096, o)
        mods = [int(m) for m in r["moduli"]]
        m8, m64 = mods[:r["L8"]], mods[r["L8"]:]
        need = 2 * r["t"] + 12 + 2
        assert m8 and m64 and all(m <= 255 for m in m8) and all(m > 16191 for m in m64)
        assert sum(math.log2(m) for m in m8) <= need / 2
        assert r["log2P"] > need and r["G"] == len(m8) + len(m64)
        for i, a in enumerate(mods):
            for b in mods[:i]:
                assert math.gcd(a, b) == 1
    with pytest.raises(oz.Oz2hError):
        oz.plan_moduli32(53, 4096, oz.default_opts(flags=oz.FLAG_BACKEND_F64 | oz.FLAG_BACKEND_MIXED))
    with pytest.raises(oz.Oz2hError) as ei:
        oz.plan_moduli(53, 4096, oz.default_opts(flags=oz.FLAG_BACKEND_F64))
    assert ei.value.code == oz.EUNSUPPORTED


def test_backend_flags_rejected_where_unsupported(oz):
    """Backward and batched plans are built on the INT8 residue planes: the backend flags
    are refused before any device work (host-side check)."""
    for flags in (oz.FLAG_BACKEND_F64, oz.FLAG_BACKEND_MIXED):
        with pytest.raises(oz.Oz2hError) as ei:
            oz.Plan.create_grad(64, 8, 8, 8, oz.default_opts(flags=flags))
        assert ei.value.code == oz.EUNSUPPORTED


def test_batched_schedule_calls_reject_null_plans(oz):
    """The batched schedule calls check their arguments on the host before any device work."""
    import ctypes
    L = oz.lib()
    a, b = ctypes.c_int32(), ctypes.c_int32()
    assert L.oz2h_batched_get_schedule(None, ctypes.addressof(a), ctypes.addressof(b)) == oz.EINVAL
    assert L.oz2h_batched_set_schedule(None, 2, 1) == oz.EINVAL
    assert L.oz2h_batched_get_config(None, None, None, None) == oz.EINVAL
    assert L.oz2h_batched_set_config(None, 0, 0) == oz.EINVAL
