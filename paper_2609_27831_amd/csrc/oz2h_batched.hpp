// oz2h_batched.hpp -- grouped kernels of the batched form: many independent
// Ozaki-II products of uneven M, N, K and p in one pass per stage.
//
// Every product keeps its own moduli set (a prefix of the global list) and
// constant tables; the stages walk segment tables (one segment per product
// and operand side) and the residue GEMMs run as ONE persistent grouped launch
// over a cost-sorted list of (product, modulus, output tile) work items.
#pragma once

#include "oz2h_kernels.hpp"

namespace oz2h {

// per-product descriptor in device memory; workspace regions are byte offsets
// from the workspace base passed to every grouped kernel
struct ProbDev {
    const uint64_t *limbs[2];   // side 0: A (rows = M), side 1: B (rows = N)
    const int32_t *exps[2];
    const int8_t *signs[2];
    int64_t rs[2], cs[2], rows[2], rpad[2];
    uint64_t erow_off[2], planes_off[2], v_off;
    uint64_t dig_off;     // CRT digit columns in global memory (classes with large nd32)
    int64_t dig_stride;   // entries per digit row there
    int64_t K, kpad;
    int32_t p, nl, t, nw32, L, lgroups, G;
    int32_t nd32, crt_dc, crt_nc, crt_ndpad;
    const ModInfo *mi;
    const double *resid, *crt;
    const ResGroup *rgrp;
    const uint32_t *pd, *phd;
    uint64_t *climbs;
    int32_t *cexp;
    int8_t *csign;
    int64_t ldc;
    const int8_t *crt_afr;   // matrix-core CRT tables (plan fields of the same names)
    int32_t crt_nbk, crt_kq, crt_nt;
    double crt_inv_ptop;
};

struct Seg {
    int64_t first;   // first block of the segment
    int32_t prod, side;
    int64_t nbx;     // blocks along the fast grid dimension of the segment
};

// largest i with segs[i].first <= b
__device__ __forceinline__ int find_seg(const Seg *__restrict__ segs, int nseg, int64_t b) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].first <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// stage 1, grouped, in three passes like the plain scan: fill every output row with
// INT_MIN, combine partial maxima with atomicMax, then give all-zero rows exponent 0.
// Fill / fix: segment (prod, side) is a 1-D grid of blocks of 256 rows.
__global__ __launch_bounds__(256) void k_exp_fill_grouped(const ProbDev *__restrict__ probs,
                                                          const Seg *__restrict__ segs, int nseg,
                                                          char *ws, int fix) {
    const int si = find_seg(segs, nseg, blockIdx.x);
    const Seg sg = segs[si];
    const ProbDev &P = probs[sg.prod];
    const int64_t r = ((int64_t)blockIdx.x - sg.first) * 256 + threadIdx.x;
    if (r >= P.rows[sg.side]) return;
    int32_t *out = (int32_t *)(ws + P.erow_off[sg.side]) + r;
    if (!fix) *out = INT_MIN;
    else if (*out == INT_MIN) *out = 0;
}

// Scan: segment (prod, side) is an nbx x (k chunks) grid of blocks, row blocks fastest.  A
// side whose contraction is contiguous (cs == 1) gets one wave per row (4 rows per block)
// over kExpChunk entries; any other side one thread per row (256 rows per block) over
// kExpRowsK entries, loads unrolled so that they are in flight together.
__global__ __launch_bounds__(256) void k_exp_scan_grouped(const ProbDev *__restrict__ probs,
                                                          const Seg *__restrict__ segs, int nseg,
                                                          char *ws) {
    const int si = find_seg(segs, nseg, blockIdx.x);
    const Seg sg = segs[si];
    const ProbDev &P = probs[sg.prod];
    const int side = sg.side;
    const int64_t lb = (int64_t)blockIdx.x - sg.first;
    const int64_t rb = lb % sg.nbx, kb = lb / sg.nbx;
    const int8_t *__restrict__ sign = P.signs[side];
    const int32_t *__restrict__ exps = P.exps[side];
    const int64_t rows = P.rows[side], K = P.K, rs = P.rs[side], cs = P.cs[side];
    int32_t *out = (int32_t *)(ws + P.erow_off[side]);
    int m = INT_MIN;
    if (cs == 1) {
        const int lane = threadIdx.x & 63;
        const int64_t r = rb * 4 + (threadIdx.x >> 6);
        if (r >= rows) return;   // whole wave
        const int64_t k0 = kb * kExpChunk;
        m = exp_max_wave(sign, exps, nullptr, r * rs, k0, min(K, k0 + kExpChunk), lane);
        if (lane == 0 && m != INT_MIN) atomicMax(out + r, m);
    } else {
        const int64_t r = rb * 256 + threadIdx.x;
        if (r >= rows) return;
        m = exp_max_thread(sign, exps, nullptr, r * rs, cs, kb * kExpRowsK, K);
        if (m != INT_MIN) atomicMax(out + r, m);
    }
}

__device__ __forceinline__ ResArgs res_args(const ProbDev &P, int side, char *ws) {
    return ResArgs{P.limbs[side], P.exps[side], P.signs[side], P.rs[side], P.cs[side],
                   P.rows[side], P.K, P.kpad, P.rpad[side] * P.kpad,
                   (const int32_t *)(ws + P.erow_off[side]), P.p, P.nl, P.t, P.nw32, P.resid,
                   P.rgrp, P.L, P.lgroups, (int8_t *)(ws + P.planes_off[side]), nullptr};
}

// stage 2, grouped: segment (prod, side) is a (kpad / (64 KW)) x (rpad / (RB / KW)) grid of
// blocks, KW = res_waves_k(RB); one launch per moduli group width KG (the plans' kg)
template <int RB, int KG, int NW = 0>
__global__ __launch_bounds__(64 * RB) void k_residues_grouped(const ProbDev *__restrict__ probs,
                                                              const Seg *__restrict__ segs,
                                                              int nseg, char *ws) {
    extern __shared__ uint32_t words[];
    const int si = find_seg(segs, nseg, blockIdx.x);
    const Seg sg = segs[si];
    const int64_t lb = (int64_t)blockIdx.x - sg.first;
    const ResArgs a = res_args(probs[sg.prod], sg.side, ws);
    residue_block<RB, KG, 1, NW>(a, lb % sg.nbx, lb / sg.nbx, words);
}

// one work item of the grouped GEMM: output tile (mt, nt) of modulus l of product prod
// (prod = kSkipItem: a placeholder that keeps the item list's XCD alignment)
struct GemmItem {
    uint16_t prod, l, mt, nt;
};
constexpr uint16_t kSkipItem = 0xFFFF;

// stage 3, persistent grouped launch: a grid of a few blocks per compute unit
// walks the cost-sorted item list with a grid stride
template <int WM, int WN, int NS = 3>
__global__ __launch_bounds__(256) void k_resgemm_grouped(const ProbDev *__restrict__ probs,
                                                         const GemmItem *__restrict__ items,
                                                         int nitems, char *ws) {
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const GemmItem it = items[i];
        if (it.prod == kSkipItem) continue;   // uniform over the block
        const ProbDev &P = probs[it.prod];
        const GemmArgs g{(const int8_t *)(ws + P.planes_off[0]), (const int8_t *)(ws + P.planes_off[1]),
                         P.kpad, P.rpad[0] * P.kpad, P.rpad[1] * P.kpad, P.mi,
                         (int16_t *)(ws + P.v_off), P.rpad[0] * P.rpad[1], P.rpad[1], nullptr};
        __syncthreads();   // the previous item's LDS tiles are no longer read
        gemm_tile<WM, WN, false, NS>(g, it.mt, it.nt, it.l);
    }
}

// stages 4-5, grouped: segment prod is a 1-D grid of CRT blocks
template <int DC, int EPT, bool GDIG>
__global__ __launch_bounds__(256) void k_crt_grouped(const ProbDev *__restrict__ probs,
                                                     const Seg *__restrict__ segs, int nseg,
                                                     char *ws, int LB) {
    extern __shared__ __attribute__((aligned(16))) uint32_t sdig[];
    const int si = find_seg(segs, nseg, blockIdx.x);
    const Seg sg = segs[si];
    const ProbDev &P = probs[sg.prod];
    const CrtArgs a{(const int16_t *)(ws + P.v_off), P.rpad[0] * P.rpad[1], P.rpad[1], P.rows[0],
                    P.rows[1], P.mi, P.L, P.crt, P.crt_ndpad, P.crt_nc, P.nd32, P.pd, P.phd,
                    (const int32_t *)(ws + P.erow_off[0]), (const int32_t *)(ws + P.erow_off[1]),
                    2 * P.t, P.p, P.csign, P.cexp, P.climbs, P.ldc, nullptr, 0, LB,
                    GDIG ? (uint32_t *)(ws + P.dig_off) : nullptr, P.dig_stride};
    crt_block<DC, EPT, true, false, GDIG>(a, (int64_t)blockIdx.x - sg.first, sdig);
}

// stages 4-5, grouped, on the matrix cores (products whose plan has the tables)
template <int KQ>
__global__ __launch_bounds__(256) void k_crt_mma_grouped(const ProbDev *__restrict__ probs,
                                                         const Seg *__restrict__ segs, int nseg,
                                                         char *ws) {
    extern __shared__ __attribute__((aligned(16))) uint32_t sdig[];
    const int si = find_seg(segs, nseg, blockIdx.x);
    const Seg sg = segs[si];
    const ProbDev &P = probs[sg.prod];
    const CrtArgs a{(const int16_t *)(ws + P.v_off), P.rpad[0] * P.rpad[1], P.rpad[1], P.rows[0],
                    P.rows[1], P.mi, P.L, P.crt, P.crt_ndpad, P.crt_nc, P.nd32, P.pd, P.phd,
                    (const int32_t *)(ws + P.erow_off[0]), (const int32_t *)(ws + P.erow_off[1]),
                    2 * P.t, P.p, P.csign, P.cexp, P.climbs, P.ldc, nullptr, 0, 0, nullptr, 0,
                    P.crt_afr, P.crt_nbk, P.crt_kq, P.crt_nt, P.crt_inv_ptop};
    crt_mma_block<KQ, true>(a, (int64_t)blockIdx.x - sg.first, sdig);
}

}  // namespace oz2h
