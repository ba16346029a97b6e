#!/usr/bin/env python3
"""Benchmark of the Ozaki-II p-bit matrix product on one MI355X.

One step = one full pass of the hot path (shared exponents, residues, INT8
MFMA residue GEMMs with the fused reduction, direct CRT + lift + rounding)
over one synthetic input already resident in HBM.

The default line headlines the high-precision workload, M = N = K = 4096 at
p = 2048 bits (exponents uniform in [-16, 16]), and carries as extra keys:
  - the large-GEMM workload, M = N = K = 8192 at p = 113 bits;
  - the matrix-core variants of stages 2 and 4 timed beside the default
    MFMA-free kernels (same inputs, bit-identical outputs);
  - the batched form (64 uneven products, one graph) against the loop of plain
    calls ("speedup_vs_loop"), and the autograd form's residue reuse against
    recomputation ("reuse_vs_recompute");
  - complex products at M = N = K = 4096, p = 256: the 3M scheme against 4M
    ("complex");
  - the binary64 and mixed backends against INT8 at M = N = K = 4096, p = 113
    ("backends");
  - operand reuse: one A (4096^2, p = 2048) against 8 right-hand sides of 4096 x 256,
    residue handle against plain calls ("operand_reuse");
  - the oracle on the host cores over a bounded block of outputs, which also
    checks the timed GPU output on that block bit for bit.

  python bench.py [--steps K] [--warmup W] [--config cfg3|cfg1|cfg2|cfg3a|cfg3b|cfg4|cfg5|complex|backends|gemm_context]
                  [--cpu-seconds S] [--no-cpu-baseline] [--no-extras]

Per-stage times come from HIP events that the library records on the launch
stream between stages (oz2h_gemm_timed); the end-to-end time is wall clock
over exactly K steps bracketed by torch.cuda.synchronize().
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import platform
import struct
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "effective p-bit GEMM GFlop/s (2MNK/s) at ≤1 ulp; INT8 MFMA % of peak"

# name: (workload, M, N, K, p, elo, ehi, seed offset)
CONFIGS = {
    "cfg1": ("plain Ozaki-II, M=N=K=256, p=128, exponents U[-4,4]", 256, 256, 256, 128, -4, 4, 1),
    "cfg2": ("plain Ozaki-II, M=N=K=2048, p=256, exponents U[-32,32]", 2048, 2048, 2048, 256, -32, 32, 2),
    "cfg3a": ("plain Ozaki-II, M=N=K=4096, p=2048, exponents U[-16,16]", 4096, 4096, 4096, 2048, -16, 16, 31),
    "cfg3b": ("plain Ozaki-II, M=N=K=8192, p=113, exponents U[-16,16]", 8192, 8192, 8192, 113, -16, 16, 32),
}

# MI355X published peaks
PEAK_INT8_TOPS = 5000.0      # dense INT8 MFMA, TOP/s
PEAK_HBM_GBS = 8000.0        # HBM3E, GB/s
PEAK_FP64_TFLOPS = 78.6      # FP64 vector, TFLOP/s (FMA = 2 flops)

PHASES = ["exponents", "residues", "gemm", "crt"]


class Hip:
    """The few HIP runtime calls the bench needs for events."""

    def __init__(self):
        self.h = ctypes.CDLL("libamdhip64.so")
        self.h.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.h.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.h.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                               ctypes.c_void_p]
        self.h.hipEventSynchronize.argtypes = [ctypes.c_void_p]

    def events(self, n):
        arr = (ctypes.c_void_p * n)()
        for i in range(n):
            ev = ctypes.c_void_p()
            assert self.h.hipEventCreate(ctypes.byref(ev)) == 0
            arr[i] = ev
        return arr

    def elapsed_ms(self, a, b) -> float:
        assert self.h.hipEventSynchronize(b) == 0
        ms = ctypes.c_float()
        assert self.h.hipEventElapsedTime(ctypes.byref(ms), a, b) == 0
        return ms.value

    def destroy(self, arr):
        for ev in arr:
            self.h.hipEventDestroy(ev)


LIBOZ2H = os.path.join(ROOT, "paper_2609_27831_amd", "liboz2h.so")


def _gfx950_code_object(path: str):
    """The gfx950 code object of a library built here (clang offload bundle: magic,
    entry count, then (offset, size, triple length, triple) per entry)."""
    with open(path, "rb") as fh:
        d = fh.read()
    i = d.find(b"__CLANG_OFFLOAD_BUNDLE__")
    if i < 0:
        return None
    n = struct.unpack_from("<Q", d, i + 24)[0]
    o = i + 32
    for _ in range(n):
        off, size, tl = struct.unpack_from("<QQQ", d, o)
        o += 24
        triple = d[o:o + tl].decode(errors="replace")
        o += tl
        if triple.endswith("gfx950") and size:
            return d[i + off:i + off + size]
    return None


def _elf_function_bytes(co: bytes, names):
    """{symbol: bytes} of the named symbols (kernel code and kernel descriptor) of an
    ELF64 code object."""
    shoff = struct.unpack_from("<Q", co, 0x28)[0]
    shentsize, shnum = struct.unpack_from("<HH", co, 0x3A)
    secs = [struct.unpack_from("<IIQQQQIIQQ", co, shoff + k * shentsize) for k in range(shnum)]
    out = {}
    for sec in secs:
        if sec[1] != 2:   # SHT_SYMTAB
            continue
        stroff = secs[sec[6]][4]
        for k in range(sec[5] // 24):
            st_name, _info, _other, shndx, value, size = struct.unpack_from(
                "<IBBHQQ", co, sec[4] + 24 * k)
            end = co.index(b"\0", stroff + st_name)
            name = co[stroff + st_name:end].decode(errors="replace")
            if name in names and 0 < shndx < shnum:
                host = secs[shndx]
                fo = host[4] + (value - host[3])
                out[name] = co[fo:fo + size]
    return out


def kernel_code_digest(symbol: str):
    """sha256 of one kernel's gfx950 machine code and kernel descriptor in the built
    library (the descriptor's code-entry offset masked: it moves with the layout of
    the code object, not with the kernel), or None: a counter record is valid only for
    the code it was taken on."""
    try:
        co = _gfx950_code_object(LIBOZ2H)
        if co is None:
            return None
        got = _elf_function_bytes(co, {symbol, symbol + ".kd"})
    except (OSError, struct.error, ValueError):
        return None
    if symbol not in got or symbol + ".kd" not in got:
        return None
    kd = bytearray(got[symbol + ".kd"])
    kd[16:24] = bytes(8)   # kernel_code_entry_byte_offset: relative to where the linker put it
    h = hashlib.sha256()
    h.update(got[symbol])
    h.update(bytes(kd))
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, config: str, field: str = "hbm_bytes_per_launch"):
    """HBM bytes (FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel of known size) from a
    committed rocprofv3 PMC summary, if every kernel it covers still has the machine
    code the counters were taken on.  field: "hbm_bytes_per_launch" (the named kernel)
    or "phase_hbm_bytes_per_step" (every kernel of its stage, one step)."""
    rec = measured_record(kernel, config)
    return rec.get(field) if rec else None


def measured_record(kernel: str, config: str):
    """The committed counter record of a kernel at a workload, or None when it is absent
    or was taken on other machine code."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{config}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    digests = rec.get("code_digests") or {}
    if not digests or any(kernel_code_digest(sym) != d for sym, d in digests.items()):
        return None
    return rec


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def device_operands(cfg, seed):
    """The workload's A and B drawn straight into device memory (same counters and
    values as synth.operands_for)."""
    import torch

    from paper_2609_27831_amd import oz2h
    from synth.gen_torch import operands_for_torch
    _, M, N, K, p, elo, ehi, _ = cfg
    (sa, ea, la), (sb, eb, lb) = operands_for_torch(seed, M, N, K, p, elo, ehi, device="cuda")
    torch.cuda.synchronize()
    return oz2h.DeviceMP(sa, ea, la, p), oz2h.DeviceMP(sb, eb, lb, p)


def kernel_names(plan, flags):
    """The stage-2 / stage-4 kernels a plain call of this plan launches (the dominant one
    where a stage has two)."""
    from paper_2609_27831_amd import oz2h
    if (flags & oz2h.FLAG_RESIDUES_MMA) and plan.nw32 >= 8:
        res = "k_residues_mma"
    else:
        res = "k_residues_row" if plan.nw32 >= 32 else "k_residues"
    if (flags & oz2h.FLAG_CRT_MMA) and 16 <= plan.nd32 <= 32 and plan.L <= 127:
        crt = "k_crt_mma"
    else:
        crt = "k_crt_row_sums" if plan.nd32 > 32 else "k_crt"
    return res, crt


def time_plain(name, Ad, Bd, steps, warmup, flags=0):
    """Time `steps` plain products; per-stage event times and derived rates."""
    import numpy as np
    import torch

    from paper_2609_27831_amd import oz2h
    workload, M, N, K, p, elo, ehi, _ = CONFIGS[name]
    plan = oz2h.Plan.create(p, K, oz2h.default_opts(flags=flags))
    ws = oz2h.workspace(plan, M, N)
    out = oz2h.empty_mp(M, N, p)
    hip = Hip()
    stream = torch.cuda.current_stream()
    evs = [hip.events(5) for _ in range(steps)]
    wev = hip.events(5)
    for _ in range(warmup):
        oz2h.gemm_timed(plan, Ad, Bd, out, ws, wev, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        oz2h.gemm_timed(plan, Ad, Bd, out, ws, evs[s], stream=stream)
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / steps
    phase_ms = {n: float(np.mean([hip.elapsed_ms(e[k], e[k + 1]) for e in evs]))
                for k, n in enumerate(PHASES)}
    for e in evs + [wev]:
        hip.destroy(e)
    del ws

    flops = 2.0 * M * N * K
    nl = (p + 63) // 64
    L, G, nd32, nw32 = plan.L, plan.G, plan.nd32, plan.nw32
    res_k, crt_k = kernel_names(plan, flags)
    # algorithmic work per stage (per launch = per step)
    res_bytes = (M * K + K * N) * (8 * nl + 5) + (M * K + K * N) * G
    res_fma = (M * K + K * N) * L * nw32          # word x weight multiply-adds
    gemm_ops = G * 2.0 * M * N * K
    gemm_bytes = G * (M * K + K * N) + L * M * N * 2
    crt_bytes = L * M * N * 2 + M * N * (8 * nl + 5)
    crt_fma = M * N * L * nd32                     # weight x digit multiply-adds
    phases = {n: {"ms": round(phase_ms[n], 4),
                  "effective_gflops": round(flops / (phase_ms[n] * 1e-3) / 1e9, 2)}
              for n in PHASES}
    sec = {n: phase_ms[n] * 1e-3 for n in PHASES}
    gemm_tops = gemm_ops / sec["gemm"] / 1e12
    phases["residues"].update({
        "kernel": res_k, "hbm_gbs": round(res_bytes / sec["residues"] / 1e9, 1),
        "fp64_tflops": round(2.0 * res_fma / sec["residues"] / 1e12, 2) if not res_k.endswith("_mma") else None,
        "counter_hbm_gbs": None})
    phases["gemm"].update({"kernel": "k_resgemm", "int8_tops": round(gemm_tops, 1),
                           "int8_mfma_pct_of_peak": round(100.0 * gemm_tops / PEAK_INT8_TOPS, 2)})
    phases["crt"].update({
        "kernel": crt_k, "hbm_gbs": round(crt_bytes / sec["crt"] / 1e9, 1),
        "fp64_tflops": round(2.0 * crt_fma / sec["crt"] / 1e12, 2) if not crt_k.endswith("_mma") else None,
        "counter_hbm_gbs": None})
    for ph, kern in (("residues", res_k), ("crt", crt_k)):
        tb = measured_traffic(kern, name, "phase_hbm_bytes_per_step")
        if tb:
            phases[ph]["counter_hbm_gbs"] = round(tb / sec[ph] / 1e9, 1)

    def roof(ph):
        if ph == "gemm":
            r = {"kernel": "k_resgemm", "bound": "mfma", "achieved": round(gemm_tops, 2),
                 "peak": PEAK_INT8_TOPS, "unit": "TOP/s", "frac": round(gemm_tops / PEAK_INT8_TOPS, 4),
                 "algorithmic_bytes": gemm_bytes}
            kern = "k_resgemm"
        else:
            kern = phases[ph]["kernel"]
            fma = res_fma if ph == "residues" else crt_fma
            a = 2.0 * fma / sec[ph] / 1e12
            r = {"kernel": kern, "bound": "alu", "achieved": round(a, 3), "peak": PEAK_FP64_TFLOPS,
                 "unit": "TFLOP/s", "frac": round(a / PEAK_FP64_TFLOPS, 4),
                 "algorithmic_bytes": res_bytes if ph == "residues" else crt_bytes}
            if kern.endswith("_mma"):   # a matrix-core variant: no fp64 work to rate
                r = {"kernel": kern, "bound": "alu", "achieved": None, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": None}
        # counter bytes over the same span as `achieved`: the GEMM's one launch per step,
        # the other stages' launches of one step
        r["traffic"] = measured_traffic(kern, name, "hbm_bytes_per_launch" if ph == "gemm"
                                        else "phase_hbm_bytes_per_step")
        rec = measured_record(kern, name)
        if rec and "sq" in rec:
            r["counters"] = {k: rec["sq"][k] for k in ("mfma_busy_pct", "wait_pct", "clock_ghz")}
        return r

    dominant = max(("residues", "gemm", "crt"), key=lambda n: phase_ms[n])
    res = {
        "workload": workload, "M": M, "N": N, "K": K, "p": p, "t": plan.t, "moduli": L,
        "int8_gemms": G, "exponent_range": [elo, ehi], "flags": flags,
        "ms_per_step": round(ms_per_step, 4),
        "value": round(flops / (ms_per_step * 1e-3) / 1e9, 3),
        "int8_mfma_pct_of_peak": round(100.0 * gemm_tops / PEAK_INT8_TOPS, 2),
        "phases": phases, "roofline": roof(dominant),
        "rooflines": {ph: roof(ph) for ph in ("residues", "gemm", "crt")},
    }
    return res, out


def cpu_baseline_and_check(name, out, seconds: float):
    """The oracle on the host cores over a bounded block of C (rows 0..r-1, columns
    0..c-1, drawn from the generator's counters) and a bit-for-bit check of the GPU's
    timed output on that block."""
    import numpy as np

    import synth
    from oracle import c_oracle
    _, M, N, K, p, elo, ehi, soff = CONFIGS[name]
    seed = synth.CONFIG_SEED_BASE + soff

    def run(r, c):
        A, B = synth.operand_blocks_for(seed, M, N, K, p, elo, ehi, range(0, r), range(0, c))
        t0 = time.perf_counter()
        ref = c_oracle.gemm(A, B, want_chat=False)
        return time.perf_counter() - t0, ref

    r = c = 1
    t, ref = run(r, c)
    while t < seconds / 8 and (r < M or c < N):
        r, c = min(M, r * 2), min(N, c * 2)
        t, ref = run(r, c)
    if t < seconds / 2:
        f = (seconds / max(t, 1e-3)) ** 0.5
        r, c = min(M, max(r + 1, int(r * f))), min(N, max(c + 1, int(c * f)))
        t, ref = run(r, c)
    gs = out.sign[:r, :c].cpu().numpy()
    ge = out.exp[:r, :c].cpu().numpy()
    gl = out.limbs[:r, :c].cpu().numpy().view(np.uint64)
    same = (np.array_equal(gs, ref["c_sign"]) and np.array_equal(ge, ref["c_exp"])
            and np.array_equal(gl, ref["c_limbs"]))
    ent = r * c
    base = {"value": round(2.0 * ent * K / t / 1e9, 4), "unit": "GFlop/s",
            "cores": c_oracle.num_threads(), "kind": "oracle",
            "sample": f"block C[0:{r}, 0:{c}] ({ent} entries, K={K}): exact bignum c^ of the "
                      f"shared-exponent integers plus one nearest-even rounding, including the "
                      f"integerization of those rows of A and columns of B; {t:.1f} s; the rate "
                      f"extrapolates to the whole product (full-matrix time = {t * M * N / ent:.0f} s)",
            "extrapolated": True, "host_cpu": cpu_model(), "nproc": os.cpu_count()}
    return base, {"entries": ent, "bit_identical": bool(same)}


def batched_problems(seed: int, count: int = 64, lo: int = 128, hi: int = 4096,
                     ps=(53, 113, 256, 512)):
    """The batched workload: M, N, K log-uniform in [lo, hi], p drawn from ps, exponents U[-4,4]."""
    import numpy as np

    import synth
    u = synth.splitmix64(seed, 0, 4 * count).reshape(count, 4)
    out = []
    for i in range(count):
        f = (u[i, :3] >> np.uint64(11)).astype(np.float64) / float(1 << 53)
        M, N, K = (int(round(lo * (hi / lo) ** x)) for x in f)
        p = ps[int(u[i, 3] % np.uint64(len(ps)))]
        out.append((M, N, K, p, seed * 1000 + i))
    return out


def measure_batched(steps, warmup):
    """Batched form: 64 products through oz2h_batched_run (tuned: GEMM tile, schedule, LDS
    stages, graph replay or direct launches) vs the same products as a loop of plain calls."""
    import torch

    import synth
    from paper_2609_27831_amd import oz2h
    from synth.gen_torch import operands_for_torch
    spec = batched_problems(synth.CONFIG_SEED_BASE + 4)
    probs, plans = [], []
    flops = 0.0
    for (M, N, K, p, sd) in spec:
        (sa, ea, la), (sb, eb, lb) = operands_for_torch(sd, M, N, K, p, -4, 4, device="cuda")
        probs.append((oz2h.DeviceMP(sa, ea, la, p), oz2h.DeviceMP(sb, eb, lb, p),
                      oz2h.empty_mp(M, N, p), 0, 0))
        flops += 2.0 * M * N * K
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    for (Ad, Bd, C, _, _) in probs:
        plans.append(oz2h.Plan.create(Ad.p, Ad.shape[1]))
    wsz = max(pl.workspace_size(Ad.shape[0], Bd.shape[1]) for pl, (Ad, Bd, _, _, _) in zip(plans, probs))
    ws1 = torch.empty(wsz, dtype=torch.uint8, device="cuda")

    def loop():
        for pl, (Ad, Bd, C, _, _) in zip(plans, probs):
            oz2h.gemm(pl, Ad, Bd, out=C, ws=ws1, stream=stream)
    ms_loop = timed(loop, steps)
    ref = [tuple(x.clone() for x in (C.sign, C.exp, C.limbs)) for (_, _, C, _, _) in probs]
    del ws1
    bp = oz2h.BatchedPlan(probs)
    ws = bp.workspace()
    cfg = bp.tune(ws)
    # oz2h_batched_run in the tuned mode; then the two modes forced
    ms_run = timed(lambda: bp.run(ws, stream=stream), steps)
    same = all(torch.equal(a, C.sign) and torch.equal(b, C.exp) and torch.equal(c, C.limbs)
               for (a, b, c), (_, _, C, _, _) in zip(ref, probs))
    ms_eager = timed(lambda: bp.run_eager(ws, stream=stream), steps)
    bp.set_schedule(cfg["gemm_stages"], True)
    ms_graph = timed(lambda: bp.run(ws, stream=stream), steps)
    bp.destroy()
    return {"workload": "64 products, M, N, K log-uniform in [128, 4096], p in {53, 113, 256, 512}, "
                        "exponents U[-4,4]",
            "sum_2MNK": flops, "tuned": cfg, "run_ms": round(ms_run, 4),
            "graph_replay_ms": round(ms_graph, 4), "direct_launch_ms": round(ms_eager, 4),
            "loop_of_plain_calls_ms": round(ms_loop, 4),
            "value": round(flops / (ms_run * 1e-3) / 1e9, 3),
            "speedup_vs_loop": round(ms_loop / ms_run, 3), "bit_identical_to_loop": bool(same)}


def measure_autograd(steps, warmup):
    """Autograd form: forward C = A B plus both backward products (dA = W B^T, dB = A^T W)
    at 4096^2, p = 256, through torch.autograd (float64 carriers), reuse vs recompute; and the
    same at 2048^2, p = 1024."""
    import torch

    import synth
    from paper_2609_27831_amd import autograd as ag
    from paper_2609_27831_amd import oz2h
    M = N = K = 4096
    p = 256
    A, B, W = synth.grad_operands_for(synth.CONFIG_SEED_BASE + 5, M, N, K, p, -4, 4)
    flops = 3 * 2.0 * M * N * K

    def modes(A, B, W, p):
        a0, b0, w = ag.to_carrier(A), ag.to_carrier(B), ag.to_carrier(W)
        res = {}
        for mode in ("reuse", "recompute"):
            def step():
                a = a0.detach().requires_grad_()
                b = b0.detach().requires_grad_()
                c = ag.oz_matmul(a, b, p, mode=mode)
                c.backward(w)
                return a.grad, b.grad
            for _ in range(warmup):
                step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                step()
            torch.cuda.synchronize()
            res[mode] = (time.perf_counter() - t0) * 1e3 / steps
        return res

    out = modes(A, B, W, p)
    # a higher precision, where a residue pass is a larger share of a product
    M2, p2 = 2048, 1024
    A2, B2, W2 = synth.grad_operands_for(synth.CONFIG_SEED_BASE + 6, M2, M2, M2, p2, -4, 4)
    out2 = modes(A2, B2, W2, p2)
    del A2, B2, W2
    plan = oz2h.Plan.create_grad(p, M, N, K)
    Ad, Bd, Wd = oz2h.to_device(A), oz2h.to_device(B), oz2h.to_device(W)
    ws = oz2h.workspace(plan, M, N)
    bws = torch.empty(plan.backward_workspace_size(), dtype=torch.uint8, device="cuda")
    dA, dB = oz2h.empty_mp(M, K, p), oz2h.empty_mp(K, N, p)
    oz2h.gemm(plan, Ad, Bd, ws=ws)
    for _ in range(warmup):
        oz2h.gemm_backward(plan, ws, Wd, dA=dA, dB=dB, ws=bws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        oz2h.gemm_backward(plan, ws, Wd, dA=dA, dB=dB, ws=bws)
    torch.cuda.synchronize()
    ms_bwd = (time.perf_counter() - t0) * 1e3 / steps
    return {"workload": "C = A B and its backward, M=N=K=4096, p=256, A and B exponents U[-4,4], "
                        "upstream gradient +-u 2^-p",
            "reuse_ms_per_step": round(out["reuse"], 4),
            "recompute_ms_per_step": round(out["recompute"], 4),
            "reuse_vs_recompute": round(out["recompute"] / out["reuse"], 3),
            "value": round(flops / (out["reuse"] * 1e-3) / 1e9, 3),
            "backward_entry_point_ms": round(ms_bwd, 4),
            "at_2048_p1024": {"reuse_ms_per_step": round(out2["reuse"], 4),
                              "recompute_ms_per_step": round(out2["recompute"], 4),
                              "reuse_vs_recompute": round(out2["recompute"] / out2["reuse"], 3)}}


def measure_complex(steps, warmup):
    """Complex products C = A B (A = Ar + i Ai, B = Br + i Bi) at M = N = K = 4096, p = 256
    through oz2h_zgemm: the 3M scheme (three residue GEMMs per modulus) against 4M (four),
    with the two outputs checked bit for bit against each other."""
    import torch

    import synth
    from paper_2609_27831_amd import oz2h
    M = N = K = 4096
    p = 256
    cfg = ("", M, N, K, p, -16, 16, 0)
    Ar, Br = device_operands(cfg, synth.CONFIG_SEED_BASE + 61)
    Ai, Bi = device_operands(cfg, synth.CONFIG_SEED_BASE + 62)
    plan = oz2h.Plan.create(p, 2 * K)
    flops = 8.0 * M * N * K      # real flops of a complex product
    out, res = {}, {}
    for scheme, name in ((oz2h.ZGEMM_3M, "3M"), (oz2h.ZGEMM_4M, "4M")):
        n = oz2h.lib().oz2h_zgemm_workspace_size(plan.handle, scheme, M, N)
        ws = torch.empty(n, dtype=torch.uint8, device="cuda")
        C = (oz2h.empty_mp(M, N, p), oz2h.empty_mp(M, N, p))
        for _ in range(warmup):
            oz2h.zgemm(plan, Ar, Ai, Br, Bi, scheme=scheme, out=C, ws=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            oz2h.zgemm(plan, Ar, Ai, Br, Bi, scheme=scheme, out=C, ws=ws)
        torch.cuda.synchronize()
        out[name] = (time.perf_counter() - t0) * 1e3 / steps
        res[name] = C
        del ws
        torch.cuda.empty_cache()
    same = all(bool(torch.equal(getattr(x, f), getattr(y, f)))
               for x, y in zip(res["3M"], res["4M"]) for f in ("sign", "exp", "limbs"))
    plan.destroy()
    return {"workload": "complex Ozaki-II, M=N=K=4096, p=256, exponents U[-16,16]",
            "ms_3m": round(out["3M"], 4), "ms_4m": round(out["4M"], 4),
            "speedup_3m_vs_4m": round(out["4M"] / out["3M"], 3),
            "value_3m": round(flops / (out["3M"] * 1e-3) / 1e9, 3),
            "unit": "GFlop/s (8MNK/s)", "bit_identical_3m_4m": same}


def measure_backends(steps, warmup):
    """The INT8, binary64 and mixed backends on one product, M = N = K = 4096 at p = 113
    (Table "Moduli configuration": 42 INT8 GEMMs against 14 binary64 GEMMs): time per
    product, per-stage times, the fp64 matrix-core rate of the binary64 residue GEMMs,
    and a bit-for-bit check that the three outputs agree."""
    import numpy as np
    import torch

    import synth
    from paper_2609_27831_amd import oz2h
    M = N = K = 4096
    p = 113
    Ad, Bd = device_operands(("", M, N, K, p, -16, 16, 0), synth.CONFIG_SEED_BASE + 71)
    hip = Hip()
    stream = torch.cuda.current_stream()
    out, res = {}, {}
    for name, flags in (("int8", 0), ("binary64", oz2h.FLAG_BACKEND_F64),
                        ("mixed", oz2h.FLAG_BACKEND_MIXED)):
        plan = oz2h.Plan.create(p, K, oz2h.default_opts(flags=flags))
        ws = oz2h.workspace(plan, M, N)
        C = oz2h.empty_mp(M, N, p)
        evs = [hip.events(5) for _ in range(steps)]
        for _ in range(warmup):
            oz2h.gemm(plan, Ad, Bd, out=C, ws=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            oz2h.gemm_timed(plan, Ad, Bd, C, ws, evs[s], stream=stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        ph = {n: round(float(np.mean([hip.elapsed_ms(e[k], e[k + 1]) for e in evs])), 4)
              for k, n in enumerate(PHASES)}
        for e in evs:
            hip.destroy(e)
        r = {"ms_per_step": round(ms, 4), "moduli": plan.L, "gemms": plan.G,
             "binary64_moduli": plan.Lf, "log2P": round(plan.log2P, 1), "phases_ms": ph}
        if flags == oz2h.FLAG_BACKEND_F64:
            kpad = (K + 127) // 128 * 128
            tf = 2.0 * plan.Lf * M * N * kpad / (ph["gemm"] * 1e-3) / 1e12
            r["fp64_mfma_tflops"] = round(tf, 2)
            r["fp64_pct_of_peak"] = round(100.0 * tf / PEAK_FP64_TFLOPS, 1)
        out[name] = r
        res[name] = C
        del ws
        plan.destroy()
        torch.cuda.empty_cache()
    same = all(bool(torch.equal(getattr(res[n], f), getattr(res["int8"], f)))
               for n in ("binary64", "mixed") for f in ("sign", "exp", "limbs"))
    return {"workload": "plain Ozaki-II on three backends, M=N=K=4096, p=113, exponents U[-16,16]",
            **out, "bit_identical": same}


def measure_operand_reuse(steps, warmup):
    """Operand reuse (residue handles): one A of 4096 x 4096 at p = 2048 against 8 right-hand
    sides of 4096 x 256, as 8 plain calls against one residue handle for A plus 8 products
    from it (its creation inside the timed region); outputs checked bit for bit."""
    import torch

    import synth
    from paper_2609_27831_amd import oz2h
    M = K = 4096
    N, p, nrhs = 256, 2048, 8
    cfg = ("", M, N, K, p, -16, 16, 0)
    from synth.gen_torch import mp_random_torch
    A, B0 = device_operands(cfg, synth.CONFIG_SEED_BASE + 81)
    Bs = [B0] + [oz2h.DeviceMP(*mp_random_torch(synth.CONFIG_SEED_BASE + 82 + r, K, N, p, -16, 16), p)
                 for r in range(nrhs - 1)]
    plan = oz2h.Plan.create(p, K)
    ws = oz2h.workspace(plan, M, N)
    Cp = [oz2h.empty_mp(M, N, p) for _ in range(nrhs)]
    Cr = [oz2h.empty_mp(M, N, p) for _ in range(nrhs)]

    def plain():
        for b, c in zip(Bs, Cp):
            oz2h.gemm(plan, A, b, out=c, ws=ws)

    def reuse():
        ra = oz2h.Residues(plan, A, oz2h.SIDE_A)
        for b, c in zip(Bs, Cr):
            oz2h.gemm_from_residues(plan, B=b, ra=ra, out=c, ws=ws)
        torch.cuda.synchronize()   # the handle's planes are read until here
        ra.destroy()

    out = {}
    for name, fn in (("plain", plain), ("reuse", reuse)):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        out[name] = (time.perf_counter() - t0) * 1e3 / steps
    same = all(bool(torch.equal(getattr(x, f), getattr(y, f)))
               for x, y in zip(Cp, Cr) for f in ("sign", "exp", "limbs"))
    plan.destroy()
    return {"workload": "A 4096 x 4096 at p = 2048 against 8 right-hand sides of 4096 x 256, "
                        "exponents U[-16,16]",
            "plain_ms": round(out["plain"], 4), "reuse_ms": round(out["reuse"], 4),
            "reuse_vs_plain": round(out["plain"] / out["reuse"], 3),
            "ms_per_product_amortized": round(out["reuse"] / nrhs, 4), "bit_identical": same}


def measure_int8_gemm_context(steps, warmup):
    """Context for the residue-GEMM roofline: the raw INT8 core (oz2h_i8gemm, int8 A [M][K] and
    B [N][K], exact int32 C) against the vendor library's int8 GEMM (torch._int_mm, which
    dispatches to hipBLASLt) on the same 8192^3 operands in the same k-contiguous layout."""
    import torch

    from paper_2609_27831_amd import oz2h
    n = 8192
    g = torch.Generator(device="cuda").manual_seed(20260901)
    A = torch.randint(-127, 128, (n, n), dtype=torch.int8, device="cuda", generator=g)
    Bt = torch.randint(-127, 128, (n, n), dtype=torch.int8, device="cuda", generator=g)   # [N][K]

    def timed(fn):
        for _ in range(max(warmup, 1)):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    tile = oz2h.TILE_256x128   # the residue GEMMs' block tile at these sizes
    ms_core = timed(lambda: oz2h.i8gemm(A, Bt, tile))
    ms_lib = timed(lambda: torch._int_mm(A, Bt.t()))
    same = bool(torch.equal(oz2h.i8gemm(A, Bt, tile), torch._int_mm(A, Bt.t())))
    ops = 2.0 * n ** 3
    return {"workload": "int8 C = A B^T, M=N=K=8192, exact int32 results, B k-contiguous; "
                        "the core with the 256 x 128 block tile",
            "oz2h_i8gemm_ms": round(ms_core, 4), "oz2h_i8gemm_tops": round(ops / ms_core / 1e9, 1),
            "library_int_mm_ms": round(ms_lib, 4), "library_int_mm_tops": round(ops / ms_lib / 1e9, 1),
            "same_results": same}


def copy_calibration():
    """A plain device copy of known size, for the HBM-counter scale factors."""
    import torch
    n = 1 << 30
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": n, "launches": 3}), flush=True)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="cfg3",
                    choices=sorted(CONFIGS) + ["cfg3", "cfg4", "cfg5", "complex", "backends", "gemm_context"])
    ap.add_argument("--flags", type=int, default=0,
                    help="OZ2H_FLAG_* bits of the timed plain products (default 0: MFMA-free "
                         "stages 2 and 4)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline workload (no variant, batched or autograd keys)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device to device three times (the reference "
                         "kernel for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: measures one MI355X only; --gpus N > 1 is not supported "
              "(the multi-GPU sharding is a design only)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        return copy_calibration()

    import torch

    import synth
    torch.cuda.set_device(0)
    base = {"metric": METRIC, "unit": "GFlop/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "i8", "data": "synthetic"}

    if args.config == "gemm_context":
        r = measure_int8_gemm_context(args.steps, args.warmup)
        line = dict(base, value=r["oz2h_i8gemm_tops"], unit="TOP/s", ms_per_step=r["oz2h_i8gemm_ms"],
                    config={"workload": r.pop("workload")}, **r)
        print(json.dumps(line), flush=True)
        return

    if args.config in ("cfg4", "cfg5", "complex", "backends"):
        log(f"{args.config}")
        fn = {"cfg4": measure_batched, "cfg5": measure_autograd, "complex": measure_complex,
              "backends": measure_backends}[args.config]
        r = fn(args.steps, args.warmup)
        if args.config == "complex":
            r["value"] = r["value_3m"]
        if args.config == "backends":
            r["value"] = round(2.0 * 4096 ** 3 / (r["binary64"]["ms_per_step"] * 1e-3) / 1e9, 3)
        ms = r.get("run_ms", r.get("reuse_ms_per_step", r.get("ms_3m")))
        if args.config == "backends":
            ms = r["binary64"]["ms_per_step"]
        line = dict(base, value=r.pop("value"), ms_per_step=ms,
                    config={"workload": r.pop("workload")}, **r)
        print(json.dumps(line), flush=True)
        return

    head = "cfg3a" if args.config == "cfg3" else args.config
    cfg = CONFIGS[head]
    log(f"{head}: drawing inputs on the GPU")
    Ad, Bd = device_operands(cfg, synth.CONFIG_SEED_BASE + cfg[7])
    log(f"{head}: timing")
    r, out = time_plain(head, Ad, Bd, args.steps, args.warmup, args.flags)
    line = dict(base, value=r["value"], ms_per_step=r["ms_per_step"],
                config={"workload": r["workload"], "M": r["M"], "N": r["N"], "K": r["K"],
                        "p": r["p"], "t": r["t"], "moduli": r["moduli"], "int8_gemms": r["int8_gemms"],
                        "exponent_range": r["exponent_range"], "flags": r["flags"]},
                int8_mfma_pct_of_peak=r["int8_mfma_pct_of_peak"], phases=r["phases"],
                roofline=r["roofline"], rooflines=r["rooflines"])
    if not args.no_cpu_baseline:
        log(f"{head}: oracle on the host cores")
        cb, chk = cpu_baseline_and_check(head, out, args.cpu_seconds)
        line["cpu_baseline"] = cb
        line["output_check_vs_oracle"] = chk
    del out
    if not args.no_extras:
        variants = {}
        log(f"{head}: matrix-core variants of stages 2 and 4")
        rv, _ = time_plain(head, Ad, Bd, max(2, args.steps // 2), 1, args.flags ^ 3)
        variants[head] = {"flags": rv["flags"], "ms_per_step": rv["ms_per_step"],
                          "residues": {k: rv["phases"]["residues"][k] for k in ("ms", "kernel")},
                          "crt": {k: rv["phases"]["crt"][k] for k in ("ms", "kernel")}}
        del Ad, Bd
        torch.cuda.empty_cache()
        if args.config == "cfg3":
            log("cfg3b: drawing inputs on the GPU")
            c3b = CONFIGS["cfg3b"]
            Ad, Bd = device_operands(c3b, synth.CONFIG_SEED_BASE + c3b[7])
            log("cfg3b: timing")
            rb, outb = time_plain("cfg3b", Ad, Bd, args.steps, args.warmup, args.flags)
            del outb
            rb.pop("rooflines")
            line["cfg3b"] = rb
            del Ad, Bd
            torch.cuda.empty_cache()
        line["stage_variants"] = variants
        log("cfg4: batched form vs loop of plain calls")
        line["batched"] = measure_batched(max(2, args.steps // 2), 1)
        line["speedup_vs_loop"] = line["batched"]["speedup_vs_loop"]
        torch.cuda.empty_cache()
        log("cfg5: autograd reuse vs recompute")
        line["autograd"] = measure_autograd(max(2, args.steps // 2), 1)
        line["reuse_vs_recompute"] = line["autograd"]["reuse_vs_recompute"]
        torch.cuda.empty_cache()
        log("complex products: 3M vs 4M")
        line["complex"] = measure_complex(max(2, args.steps // 2), 1)
        torch.cuda.empty_cache()
        log("backends: INT8, binary64, mixed")
        line["backends"] = measure_backends(max(2, args.steps // 2), 1)
        torch.cuda.empty_cache()
        log("operand reuse: residue handles against plain calls")
        line["operand_reuse"] = measure_operand_reuse(max(2, args.steps // 2), 1)
        torch.cuda.empty_cache()
        log("int8 GEMM context: raw core against the library")
        line["int8_gemm_context"] = measure_int8_gemm_context(args.steps, 2)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
