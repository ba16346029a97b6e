// oz2h_kernels.hpp -- gfx950 kernels of the Ozaki-II pipeline (device code).
//
//   k_exp_*      stage 1: shared exponents e_i / f_j (Eq. 1)
//   k_residues   stage 2: integerization (Eq. 1) + centred residues per modulus,
//                balanced base-128 halves for two-limb moduli (VALU, fp64-exact sums)
//   k_resgemm    stage 3: INT8 MFMA residue GEMMs (LDS-staged tiles) with the
//                mod-m_l reduction and Karatsuba recombination fused in the epilogue
//   k_crt        stage 4+5: direct CRT, symmetric lift, rescale and one RNE rounding
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <type_traits>

#ifndef OZ2H_GEMM_SCHED
#define OZ2H_GEMM_SCHED 1
#endif

#include "oz2h_plan.hpp"

namespace oz2h {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------- stage 1

constexpr int kExpChunk = 1024;   // contraction entries per wave (contiguous rows)
constexpr int kExpRowsK = 16;     // contraction entries per thread (other layouts)

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Largest exponent of the nonzero entries of one contiguous stretch [k0, k1) of a row (base
// offset rb), over a wave: lane reads k0 + lane + 64 u.  Every load is issued before any is
// used: entries past k1 read entry k0 (always in range) and are ignored, and the exponent is
// read whatever the sign.  INT_MIN when the stretch has no nonzero entry.
__device__ __forceinline__ int exp_max_wave(const int8_t *__restrict__ sign, const int32_t *__restrict__ exps,
                                            const int32_t *__restrict__ koff, int64_t rb, int64_t k0,
                                            int64_t k1, int lane) {
    constexpr int U = kExpChunk / 64;
    int sg[U], ex[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t k = k0 + lane + 64 * u;
        const int64_t kk = k < k1 ? k : k0;
        sg[u] = k < k1 ? sign[rb + kk] : 0;
        ex[u] = exps[rb + kk] + (koff ? koff[kk] : 0);
    }
    int m = INT_MIN;
#pragma unroll
    for (int u = 0; u < U; ++u) m = sg[u] ? max(m, ex[u]) : m;
    for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off));
    return m;
}

// The same for one thread over kExpRowsK entries k0 .. of a row with entry stride cs.
__device__ __forceinline__ int exp_max_thread(const int8_t *__restrict__ sign, const int32_t *__restrict__ exps,
                                              const int32_t *__restrict__ koff, int64_t rb, int64_t cs,
                                              int64_t k0, int64_t count) {
    int sg[kExpRowsK], ex[kExpRowsK];
#pragma unroll
    for (int u = 0; u < kExpRowsK; ++u) {
        const int64_t k = k0 + u;
        const int64_t kk = k < count ? k : k0;
        sg[u] = k < count ? sign[rb + kk * cs] : 0;
        ex[u] = exps[rb + kk * cs] + (koff ? koff[kk] : 0);
    }
    int m = INT_MIN;
#pragma unroll
    for (int u = 0; u < kExpRowsK; ++u) m = sg[u] ? max(m, ex[u]) : m;
    return m;
}

// rows whose entries are contiguous along the contraction (cs == 1): one wave
// per (row, kExpChunk-entry chunk), lanes stride 1, partial maxima combined by atomicMax
// koff (nullable): a per-contraction-index exponent offset added before the max
// (the exponent folding of the backward products)
__global__ __launch_bounds__(256) void k_exp_kcontig(const int8_t *__restrict__ sign,
                                                     const int32_t *__restrict__ exps,
                                                     int64_t rows, int64_t count, int64_t rs,
                                                     const int32_t *__restrict__ koff,
                                                     int32_t *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= rows) return;
    const int64_t k0 = (int64_t)blockIdx.y * kExpChunk;
    int m = exp_max_wave(sign, exps, koff, r * rs, k0, min(count, k0 + kExpChunk), lane);
    if (lane == 0 && m != INT_MIN) atomicMax(out + r, m);
}

// any other layout: one thread per row, kExpRowsK entries of the contraction per block
// row (loads unrolled, so that they are all in flight at once)
__global__ __launch_bounds__(256) void k_exp_generic(const int8_t *__restrict__ sign,
                                                     const int32_t *__restrict__ exps,
                                                     int64_t rows, int64_t count, int64_t rs,
                                                     int64_t cs, const int32_t *__restrict__ koff,
                                                     int32_t *__restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= rows) return;
    const int m = exp_max_thread(sign, exps, koff, r * rs, cs, (int64_t)blockIdx.y * kExpRowsK, count);
    if (m != INT_MIN) atomicMax(out + r, m);
}

// all-zero rows get exponent 0
__global__ void k_exp_fix(int32_t *__restrict__ p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && p[i] == INT_MIN) p[i] = 0;
}

// ---------------------------------------------------------------- stage 2

// global-memory views of pointers (pointers read from a descriptor are generic;
// the casts let the compiler use global and scalar loads)
#define OZ2H_G(T) const __attribute__((address_space(1))) T
typedef __attribute__((address_space(1))) int8_t g_i8;
typedef __attribute__((address_space(1))) uint32_t g_u32;
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) v4u g_v4u;

// a ModInfo record read through a global-memory pointer (field by field: the
// implicit copy constructor does not bind to an address-space-qualified object)
__device__ __forceinline__ ModInfo load_info(OZ2H_G(ModInfo) *p) {
    ModInfo r;
    r.m = p->m;
    r.g0 = p->g0;
    r.nprod = p->nprod;
    r.minv = p->minv;
    r.inv_m = p->inv_m;
    r.kc[0] = p->kc[0];
    r.kc[1] = p->kc[1];
    r.kc[2] = p->kc[2];
    r.pad = 0;
    return r;
}

// The (t+1)-bit integer a^ = RNE(mant * 2^sh) of one entry as nw 32-bit words
// col[w * st] (zero above the value); returns the sign after rounding (0 if a^ = 0).
// sh = t - p + exp - e <= t - p (Eq. 1); mant is p bits in 64-bit limbs (bits at or
// above p ignored).  One pass over the significand's 32-bit words: with sh = 32 q + r,
// r in [1, 32], word j lands in output word q + j as the funnel shift
// alignbit(m_j, m_{j-1}, 32 - r); for sh < 0 the same pass collects the round bit
// (position -sh - 1) and the sticky bits below it, and a round-up carries through the
// words.  A shift below -(32 nd + 2) drops every bit, the round bit included (a^ = 0).
// The limbs stream through a ring of two registers, loaded two limbs ahead with clamped
// unconditional loads, so that the loads of one entry overlap.
__device__ __forceinline__ int build_words(OZ2H_G(uint64_t) *__restrict__ sl, int s, int64_t sh,
                                           int p, int nw, uint32_t *col, int st) {
    for (int w = 0; w < nw; ++w) col[w * st] = 0u;
    if (s == 0) return 0;
    const int nlimb = (p + 63) >> 6;
    const int nd = (p + 31) >> 5;
    const uint64_t topm = (p & 63) ? (1ull << (p & 63)) - 1ull : ~0ull;
    const int shc = (int)max(sh, (int64_t)-(32 * nd + 2));
    const int q = (shc - 1) >> 5;        // floor((sh - 1) / 32)
    const int sa = 32 * (q + 1) - shc;   // 32 - r, in [0, 31]
    const int rp = -shc - 1;             // round bit position (sh < 0)
    uint32_t prev = 0u, nz = 0u;
    bool rbit = false, sticky = false;
    auto word = [&](int j, uint32_t cur) {   // word j of the significand (0 above it)
        const int w = q + j;
        if (w >= 0 && w < nw) {
            const uint32_t v = __builtin_amdgcn_alignbit(cur, prev, sa);
            col[w * st] = v;
            nz |= v;
        }
        if (shc < 0) {
            const int b = rp - 32 * j;   // the round bit's position within word j
            if (b >= 32) {
                sticky |= cur != 0u;
            } else if (b >= 0) {
                rbit = (cur >> b) & 1u;
                sticky |= (cur & ((1u << b) - 1u)) != 0u;
            }
        }
        prev = cur;
    };
    auto ld = [&](int l) { return sl[min(l, nlimb - 1)]; };
    uint64_t r0 = ld(0), r1 = ld(1);
    auto limb = [&](int l, uint64_t &r) {
        uint64_t x = l < nlimb ? r : 0ull;
        if (l == nlimb - 1) x &= topm;
        r = ld(l + 2);
        word(2 * l, (uint32_t)x);
        word(2 * l + 1, (uint32_t)(x >> 32));
    };
    // limbs 0 .. nlimb - 1, then one more word of zeros for the carry-out of the shift
    for (int l = 0; l < nlimb; l += 2) {
        limb(l, r0);
        limb(l + 1, r1);
    }
    word(2 * ((nlimb + 1) & ~1), 0u);
    if (rbit && (sticky || (col[0] & 1u))) {   // round half to even: add one
        for (int w = 0; w < nw; ++w) {
            const uint32_t v = col[w * st] + 1u;
            col[w * st] = v;
            if (v) break;
        }
        nz = 1u;
    }
    return nz ? s : 0;
}

// Residues of a^ (stage 2).  One thread per entry (r, k) of a rows x count
// operand side; a block covers 64 consecutive k of RB rows, so a wave stores
// 64 contiguous int8 per plane.  The integer a^ of the entry is built once into
// an LDS column of 32-bit words; the moduli are then swept in groups of 8 with
// fp64 FMAs against centred 2^(32 w) mod m weights (every partial sum is an
// exact integer below 2^53), read with wave-uniform scalar loads.  Reduction:
// r = a - rint(a/m) m.  The quotient is exact for the odd one-limb moduli (a is
// below 2^51, so a/m stays 1/(2m) away from a half-integer, farther than the
// rounding error) and at worst off by one for a two-limb modulus, so |r| <= 127
// for every one-limb modulus (|r| <= 64 for m = 128, ties included) and
// |r| <= (m + 3)/2 for a two-limb one, whose balanced base-128 split
// r = r0 + 128 r1 then has |r0|, |r1|, |r0 + r1| <= 127.  Any representative
// of a^ mod m within these bounds gives the same exact GEMM result mod m.
struct ResArgs {
    const uint64_t *limbs;
    const int32_t *exps;
    const int8_t *signs;
    int64_t rs, cs, rows, count, kpad, plane_stride;
    const int32_t *erow;
    int p, nl, t, nw32;
    const double *tab;
    const ResGroup *rgrp;
    int L, lgroups;
    int8_t *planes;
    const int32_t *koff;   // nullable per-contraction exponent offsets (exponent folding)
};

// a wave-uniform plane pointer held in scalar registers, so that a store through it with a
// 32-bit lane offset takes the scalar-base form
__device__ __forceinline__ g_i8 *uniform_ptr(g_i8 *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (g_i8 *)(((uint64_t)hi << 32) | lo);
}

// Low bytes of four ints in one dword, byte i from b[i].
__device__ __forceinline__ uint32_t pack_bytes(int b0, int b1, int b2, int b3) {
    const uint32_t lo = __builtin_amdgcn_perm((uint32_t)b1, (uint32_t)b0, 0x0c0c0400u);
    const uint32_t hi = __builtin_amdgcn_perm((uint32_t)b3, (uint32_t)b2, 0x0c0c0400u);
    return __builtin_amdgcn_perm(hi, lo, 0x05040100u);
}

// 4 x 4 byte transpose within each quad of lanes: lane 4 a + q enters holding byte i of
// row q and leaves holding byte q of rows 0..3 (byte j from row j).  Two exchanges (with
// lane ^ 2, then lane ^ 1) of DPP quad permutes, each followed by a byte select whose
// selector depends on the lane's place in the quad (v_perm_b32: selector values 0-3 take
// the bytes of the second operand, 4-7 those of the first).
struct QuadSel {
    uint32_t a, b;
};
__device__ __forceinline__ QuadSel quad_sel(int lane) {
    const int q = lane & 3;
    return QuadSel{q < 2 ? 0x05040100u : 0x03020706u, (q & 1) ? 0x03070105u : 0x06020400u};
}
__device__ __forceinline__ uint32_t quad_transpose_bytes(uint32_t w, QuadSel sel) {
    const uint32_t p2 = (uint32_t)__builtin_amdgcn_mov_dpp((int)w, 0x4E, 0xF, 0xF, false);
    w = __builtin_amdgcn_perm(p2, w, sel.a);
    const uint32_t p1 = (uint32_t)__builtin_amdgcn_mov_dpp((int)w, 0xB1, 0xF, 0xF, false);
    return __builtin_amdgcn_perm(p1, w, sel.b);
}

// Waves of a residue block along k: two when the block has at least two, so that a block
// covers 128 consecutive entries of RB / 2 rows.  Blocks are dealt to the XCDs round-robin,
// so with one wave per row the two 64-byte halves of a plane line would be written from two
// different L2s.  Grids: (kpad / (64 KW)) x (rpad / (RB / KW)) blocks, launched as a 1-D grid
// with the k blocks fastest (no 65535 limit on the rows).
__host__ __device__ constexpr int res_waves_k(int rb) { return rb >= 2 ? 2 : 1; }
// The VALU kernel with EPT entries per thread: a wave covers 64 EPT consecutive k of one
// row (EPT = 2: a whole 128-byte plane line, one wave per row).
__host__ __device__ constexpr int res_kw(int rb, int ept) { return ept >= 2 ? 1 : res_waves_k(rb); }
// k entries a block covers
__host__ __device__ constexpr int res_block_k(int rb, int ept) { return 64 * ept * res_kw(rb, ept); }

// The pointers are passed as __restrict__ parameters (kept as scoped no-alias
// information when inlined), so the compiler knows that the plane stores do
// not clobber the constant tables and reads those with scalar loads.
// EPT entries per thread share every constant the thread reads: entry e of a lane is
// k = kbase + 64 e + lane, its words in the LDS column words + e BD + tid (stride EPT BD).
// NW > 0 (integers of exactly NW words): the words are read from LDS once, as doubles with
// the entry's sign applied, and stay in registers for every group of moduli.
template <int RB, int KG, int EPT = 1, int NW = 0>
__device__ __forceinline__ void residue_block_r(
    const uint64_t *__restrict__ limbs, const int32_t *__restrict__ exps,
    const int8_t *__restrict__ signs, const int32_t *__restrict__ erow,
    const int32_t *__restrict__ koff, const double *__restrict__ tab,
    const ResGroup *__restrict__ rgrp, int8_t *__restrict__ planes, int64_t rs, int64_t cs,
    int64_t rows, int64_t count, int64_t kpad, int64_t plane_stride, int p, int nl, int t,
    int nw32, int L, int lgroups, int64_t bx, int64_t by, uint32_t *words) {
    constexpr int BD = 64 * RB;
    constexpr int ST = BD * EPT;   // word stride of an LDS column
    const int tid = threadIdx.x;
    constexpr int KW = res_kw(RB, EPT);
    const int lane = tid & 63;
    const int64_t kbase = (bx * KW + (tid >> 6) % KW) * 64 * EPT;
    const int64_t r = by * (RB / KW) + (tid >> 6) / KW;

    OZ2H_G(int8_t) *gsigns = (OZ2H_G(int8_t) *)signs;
    OZ2H_G(int32_t) *gexps = (OZ2H_G(int32_t) *)exps;
    OZ2H_G(int32_t) *gerow = (OZ2H_G(int32_t) *)erow;
    OZ2H_G(int32_t) *gkoff = (OZ2H_G(int32_t) *)koff;
    double sgn[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int64_t k = kbase + 64 * e + lane;
        int s = 0;
        int64_t sh = 0, idx = 0;
        if (r < rows && k < count) {
            idx = r * rs + k * cs;
            s = gsigns[idx];
            sh = (int64_t)t - p + gexps[idx] + (koff ? gkoff[k] : 0) - gerow[r];
        }
        s = build_words((OZ2H_G(uint64_t) *)limbs + idx * nl, s, sh, p, nw32, words + e * BD + tid, ST);
        sgn[e] = s < 0 ? -1.0 : 1.0;
    }

    // the tables live in global memory: say so, so that pointers read from a
    // descriptor (the grouped kernels) still qualify for scalar loads
    typedef const __attribute__((address_space(1))) double gdouble;
    gdouble *gtab = (gdouble *)tab;
    OZ2H_G(ResGroup) *grec = (OZ2H_G(ResGroup) *)rgrp;
    // per-plane base of this block's region (uniform, 64-bit) + a 32-bit lane offset within
    // it (below (RB / KW) kpad + 128 < 2^32 whatever the plane size): scalar-base stores, no
    // per-lane 64-bit address arithmetic
    const int64_t r0b = by * (RB / KW), k0b = bx * res_block_k(RB, EPT);
    planes += r0b * kpad + k0b;
    const uint32_t loff = (uint32_t)((r - r0b) * kpad + (kbase + lane - k0b));   // entry 0
    // packed stores: lane 4 a + q writes entries 4 a .. 4 a + 3 of plane q of four
    const QuadSel qsel = quad_sel(lane);
    const int64_t qoff = (int64_t)(lane & 3) * plane_stride + (int64_t)(loff & ~3u);
    const uint32_t *col = words + tid;
    double xw[NW > 0 ? NW : 1][EPT];
    if constexpr (NW > 0) {
#pragma unroll
        for (int w = 0; w < NW; ++w)
#pragma unroll
            for (int e = 0; e < EPT; ++e) xw[w][e] = (double)col[e * BD + w * ST] * sgn[e];
    }
    // the signed integer's multiply-add sum for modulus g of the group
    auto sacc = [&](const double (&acc)[EPT][KG], int e, int g) { return NW > 0 ? acc[e][g] : acc[e][g] * sgn[e]; };
    for (int grp = 0; grp < lgroups; ++grp) {
        double acc[EPT][KG];
#pragma unroll
        for (int e = 0; e < EPT; ++e)
#pragma unroll
            for (int g = 0; g < KG; ++g) acc[e][g] = 0.0;
        gdouble *c = gtab + (size_t)grp * nw32 * KG;   // uniform: scalar loads
        if constexpr (NW > 0) {
#pragma unroll
            for (int w = 0; w < NW; ++w)
#pragma unroll
                for (int g = 0; g < KG; ++g) {
                    const double cg = c[w * KG + g];
#pragma unroll
                    for (int e = 0; e < EPT; ++e) acc[e][g] = fma(xw[w][e], cg, acc[e][g]);
                }
        } else {
            for (int w = 0; w < nw32; ++w) {
                double x[EPT];
#pragma unroll
                for (int e = 0; e < EPT; ++e) x[e] = (double)col[e * BD + w * ST];
#pragma unroll
                for (int g = 0; g < KG; ++g) {
                    const double cg = c[w * KG + g];
#pragma unroll
                    for (int e = 0; e < EPT; ++e) acc[e][g] = fma(x[e], cg, acc[e][g]);
                }
            }
        }
        OZ2H_G(ResGroup) *R = grec + grp;
        const uint32_t two = R->two;
        // a full group of one kind owns consecutive planes from that of its first modulus:
        // dword stores after a quad byte transpose, four planes per store
        if ((grp + 1) * KG <= L && (two == 0u || two == (1u << KG) - 1u)) {
            const uint32_t gb = R->g0[0];
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                int ri[KG];
#pragma unroll
                for (int g = 0; g < KG; ++g) {
                    const double a = sacc(acc, e, g);
                    ri[g] = (int)fma(-rint(a * R->inv_m[g]), R->md[g], a);
                }
                auto store4 = [&](uint32_t gp, int b0, int b1, int b2, int b3) {
                    g_i8 *pb = uniform_ptr((g_i8 *)planes + (int64_t)gp * plane_stride);
                    *(g_u32 *)(pb + qoff + 64 * e) = quad_transpose_bytes(pack_bytes(b0, b1, b2, b3), qsel);
                };
                if (two == 0u) {
#pragma unroll
                    for (int g = 0; g < KG; g += 4) store4(gb + g, ri[g], ri[g + 1], ri[g + 2], ri[g + 3]);
                } else {
                    int pl[3 * KG];   // (r0, r1, r0 + r1) of each modulus, in plane order
#pragma unroll
                    for (int g = 0; g < KG; ++g) {
                        const int r0 = ((ri[g] + 64) & 127) - 64;   // balanced base-128 split
                        const int r1 = (ri[g] - r0) >> 7;
                        pl[3 * g] = r0;
                        pl[3 * g + 1] = r1;
                        pl[3 * g + 2] = r0 + r1;
                    }
#pragma unroll
                    for (int j = 0; j < 3 * KG; j += 4) store4(gb + j, pl[j], pl[j + 1], pl[j + 2], pl[j + 3]);
                }
            }
            continue;
        }
#pragma unroll
        for (int g = 0; g < KG; ++g) {
            if (grp * KG + g >= L) break;
            g_i8 *pb = (g_i8 *)planes + (int64_t)R->g0[g] * plane_stride;
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const double a = sacc(acc, e, g);
                const int ri = (int)fma(-rint(a * R->inv_m[g]), R->md[g], a);
                const uint32_t lo = loff + 64 * e;
                if (!((two >> g) & 1u)) {
                    pb[lo] = (int8_t)ri;
                } else {
                    const int r0 = ((ri + 64) & 127) - 64;   // balanced base-128 split
                    const int r1 = (ri - r0) >> 7;
                    pb[lo] = (int8_t)r0;
                    pb[plane_stride + lo] = (int8_t)r1;
                    pb[2 * plane_stride + lo] = (int8_t)(r0 + r1);
                }
            }
        }
    }
}

template <int RB, int KG, int EPT = 1, int NW = 0>
__device__ __forceinline__ void residue_block(const ResArgs &a, int64_t bx, int64_t by,
                                              uint32_t *words) {
    residue_block_r<RB, KG, EPT, NW>(a.limbs, a.exps, a.signs, a.erow, a.koff, a.tab, a.rgrp, a.planes,
                                 a.rs, a.cs, a.rows, a.count, a.kpad, a.plane_stride, a.p, a.nl, a.t,
                                 a.nw32, a.L, a.lgroups, bx, by, words);
}

template <int RB, int KG, int EPT, int NW = 0>
__global__ __launch_bounds__(64 * RB) void k_residues(ResArgs a) {
    extern __shared__ uint32_t words[];
    const int64_t nbx = a.kpad / res_block_k(RB, EPT);
    residue_block<RB, KG, EPT, NW>(a, (int64_t)blockIdx.x % nbx, (int64_t)blockIdx.x / nbx, words);
}

// lanes of one wave hand data over through LDS: keep the compiler from moving LDS
// accesses across this point (LDS itself serves a wave's instructions in order)
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Residues of a^ on the vector ALUs with row broadcasts (stage 2, no MFMA).  The residue
// of a^ = sum_w x_w 2^(32 w) modulo m is sum_w x_w c_w with the centred c_w = 2^(32 w) mod m
// (an exact fp64 integer, |sum| < 2^53), then a^ - rint(a^/m) m.  Each lane of a 16-lane row
// owns one modulus of a group of 16 and keeps that modulus's weights c_w in registers; the
// row works on one entry at a time, its 32-bit words spread over the row's lanes (lane j
// holds word 16 c + j of chunk c), and each multiply-add takes the word from lane w % 16 by
// a DPP row broadcast (v_fmac_f64 with row_newbcast): no constant loads in the inner loop.
// A block of four waves covers 128 consecutive k of one row of the operand side:
//   phase 1: threads 0-127 build their entry's words into LDS (word w of entry e at
//            words[w * kResRowS + e]: a row of 16 lanes reading 16 words of one entry, and
//            the four rows four entries 16 apart, hit 64 different banks);
//   phase 2: wave v takes entry half h = v & 1 (entries 64 h ..) and the moduli groups
//            g = v >> 1, v >> 1 + 2, ..; row q of the wave takes entries 64 h + 16 q + i,
//            i < 16, four at a time (four independent accumulators per lane);
//   stores:  a lane holds its modulus's residues of 16 consecutive entries, packs their bytes
//            in registers and stores 16 bytes per plane.
constexpr int kResRowS = 129;   // LDS word stride of the row-broadcast residue kernel

// v_fmac_f64 with its first source broadcast from lane LANE of each row of 16 lanes (DPP
// row_newbcast).  The DPP source must not be written by a VALU instruction in the two
// instructions before; the words come from asm blocks that end with s_nop 1.
template <int LANE>
__device__ __forceinline__ void fmac_rowbcast(double &acc, double x, double c) {
    asm volatile("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                 : "+v"(acc)
                 : "v"(x), "v"(c), "n"(LANE));
}

// four words as doubles, followed by the two wait states a DPP read of them needs
__device__ __forceinline__ void cvt4_words(uint32_t a, uint32_t b, uint32_t c, uint32_t d, double &x0,
                                           double &x1, double &x2, double &x3) {
    asm volatile(
        "v_cvt_f64_u32 %0, %4\n\t"
        "v_cvt_f64_u32 %1, %5\n\t"
        "v_cvt_f64_u32 %2, %6\n\t"
        "v_cvt_f64_u32 %3, %7\n\t"
        "s_nop 1"
        : "=&v"(x0), "=&v"(x1), "=&v"(x2), "=&v"(x3)
        : "v"(a), "v"(b), "v"(c), "v"(d));
}

// an NC-word chunk (NC = 16, 4 or 2) into NE accumulators: lane j's weights c[i] are word
// w0 + i's; word w0 + i of entry u comes from lane i of the row.  For each broadcast lane the
// NE entries follow each other, so that consecutive multiply-adds are independent.
template <int NC, int NE, int I = 0>
__device__ __forceinline__ void row_fmas(double (&a)[NE], const double (&x)[NE], const double *c) {
    if constexpr (I < NC) {
#pragma unroll
        for (int u = 0; u < NE; ++u) fmac_rowbcast<I>(a[u], x[u], c[I]);
        row_fmas<NC, NE, I + 1>(a, x, c);
    }
}

struct ResRowArgs {
    const uint64_t *limbs;
    const int32_t *exps;
    const int8_t *signs;
    int64_t rs, cs, rows, count, kpad, plane_stride;
    const int32_t *erow;
    const int32_t *koff;   // nullable per-contraction exponent offsets (exponent folding)
    int p, nl, t, nw32, nwp, L, rg16;
    const double *tab;     // [rg16][16][nwp]
    const ModInfo *mi;
    int8_t *planes;
};

__host__ __device__ constexpr size_t res_row_lds(int nwp) {
    return (size_t)nwp * kResRowS * 4 + 128 * 8;
}

// EPR entries per row of a wave and group (16: wave v takes the entry half v & 1 and the
// groups v >> 1, v >> 1 + 2, ..; 32: wave v takes all 128 entries and the groups v, v + 4,
// .., so that every weight it loads serves twice the multiply-adds).  Row q's entries are
// 64 s + 16 q + i (i < 16) for its half(s) s.  (Measured at 4096^2: EPR 32 is 4 % faster
// than 16 at p = 2048; loading the next chunk's weights ahead was slower, and spilled.)
template <int EPR>
__device__ __forceinline__ void residues_row_block(const ResRowArgs &a, uint32_t *smem) {
    constexpr int NH = EPR / 16;   // entry halves per wave
    uint32_t *words = smem;
    double *sgn = (double *)(smem + (size_t)a.nwp * kResRowS);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t nbx = a.kpad / 128;
    const int64_t bx = (int64_t)blockIdx.x % nbx, r = (int64_t)blockIdx.x / nbx;
    const int64_t k0 = bx * 128;

    // phase 1: the words of the block's 128 entries
    if (tid < 128) {
        OZ2H_G(int8_t) *gsigns = (OZ2H_G(int8_t) *)a.signs;
        OZ2H_G(int32_t) *gexps = (OZ2H_G(int32_t) *)a.exps;
        const int64_t k = k0 + tid;
        int s = 0;
        int64_t sh = 0, idx = 0;
        if (r < a.rows && k < a.count) {
            idx = r * a.rs + k * a.cs;
            s = gsigns[idx];
            sh = (int64_t)a.t - a.p + gexps[idx] + (a.koff ? a.koff[k] : 0) - a.erow[r];
        }
        s = build_words((OZ2H_G(uint64_t) *)a.limbs + idx * a.nl, s, sh, a.p, a.nwp, words + tid,
                        kResRowS);
        sgn[tid] = s < 0 ? -1.0 : 1.0;
    }
    __syncthreads();

    // phase 2
    const int j = lane & 15, q = lane >> 4;
    const int h0 = NH == 2 ? 0 : (wv & 1);        // first entry half of this wave
    const int g0w = NH == 2 ? wv : (wv >> 1), gstep = NH == 2 ? 4 : 2;
    // words past the full 16-word chunks: chunks of 4, and a last chunk of 2 when at most two
    // words remain (the words past nw32 are zero in LDS)
    const int nfull = a.nw32 >> 4, nrem = a.nw32 & 15;
    const int ntail = (nrem & 3) == 3 ? (nrem >> 2) + 1 : nrem >> 2;
    const bool tail2 = (nrem & 3) == 1 || (nrem & 3) == 2;
    int8_t *prow = a.planes + r * a.kpad + k0;   // the block's segment of plane 0
    for (int g = g0w; g < a.rg16; g += gstep) {
        const int l = 16 * g + j;
        const bool live = l < a.L;
        const ModInfo mi = live ? load_info((OZ2H_G(ModInfo) *)a.mi + l) : ModInfo{};
        const double *crow = a.tab + ((size_t)g * 16 + j) * a.nwp;
        double acc[EPR];
#pragma unroll
        for (int i = 0; i < EPR; ++i) acc[i] = 0.0;
        // one NC-word chunk (NC = 16, 4 or 2) from word w0 with the weights c
        auto chunk = [&](auto nc_, int w0, const double *c) {
            constexpr int NC = decltype(nc_)::value;
            const uint32_t *wr = words + (size_t)(w0 + (j & (NC - 1))) * kResRowS + 16 * q;
#pragma unroll
            for (int eb = 0; eb < EPR / 8; ++eb) {
                const int e = 64 * (h0 + eb / 2) + 8 * (eb % 2);   // + 16 q, entries e .. e + 7
                double x[8], a8[8];
                cvt4_words(wr[e], wr[e + 1], wr[e + 2], wr[e + 3], x[0], x[1], x[2], x[3]);
                cvt4_words(wr[e + 4], wr[e + 5], wr[e + 6], wr[e + 7], x[4], x[5], x[6], x[7]);
#pragma unroll
                for (int u = 0; u < 8; ++u) a8[u] = acc[8 * eb + u];
                row_fmas<NC, 8>(a8, x, c);
#pragma unroll
                for (int u = 0; u < 8; ++u) acc[8 * eb + u] = a8[u];
            }
        };
        for (int c = 0; c < nfull; ++c) {
            double cc[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) cc[i] = crow[16 * c + i];
            chunk(std::integral_constant<int, 16>{}, 16 * c, cc);
        }
        for (int c = 0; c < ntail; ++c) {
            double c4[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) c4[i] = crow[16 * nfull + 4 * c + i];
            chunk(std::integral_constant<int, 4>{}, 16 * nfull + 4 * c, c4);
        }
        if (tail2) {
            double c2[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) c2[i] = crow[16 * nfull + 4 * ntail + i];
            chunk(std::integral_constant<int, 2>{}, 16 * nfull + 4 * ntail, c2);
        }

        // per entry half: lane (q, j) holds the residues of its modulus for the 16 consecutive
        // entries 64 hs + 16 q + i; their bytes are packed in registers and leave as one
        // 16-byte store per plane (the four rows of a wave write 64 contiguous bytes of each
        // of its planes)
#pragma unroll
        for (int hh = 0; hh < NH; ++hh) {
            const int hs = h0 + hh;
            if (live) {
                const double md = (double)mi.m;
                const double *sg = sgn + 64 * hs + 16 * q;
                g_i8 *dst = (g_i8 *)prow + (int64_t)mi.g0 * a.plane_stride + 64 * hs + 16 * q;
                auto resid = [&](int i) {
                    const double x = acc[16 * hh + i] * sg[i];
                    return (int)fma(-rint(x * mi.inv_m), md, x);
                };
                v4u b0;
                if (mi.nprod == 1) {
#pragma unroll
                    for (int i4 = 0; i4 < 4; ++i4)
                        b0[i4] = pack_bytes(resid(4 * i4), resid(4 * i4 + 1), resid(4 * i4 + 2),
                                            resid(4 * i4 + 3));
                    *(g_v4u *)dst = b0;
                } else {
                    v4u b1, b2;
#pragma unroll
                    for (int i4 = 0; i4 < 4; ++i4) {
                        int r0[4], r1[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int ri = resid(4 * i4 + u);
                            r0[u] = ((ri + 64) & 127) - 64;   // balanced base-128 split
                            r1[u] = (ri - r0[u]) >> 7;
                        }
                        b0[i4] = pack_bytes(r0[0], r0[1], r0[2], r0[3]);
                        b1[i4] = pack_bytes(r1[0], r1[1], r1[2], r1[3]);
                        b2[i4] = pack_bytes(r0[0] + r1[0], r0[1] + r1[1], r0[2] + r1[2], r0[3] + r1[3]);
                    }
                    *(g_v4u *)dst = b0;
                    *(g_v4u *)(dst + a.plane_stride) = b1;
                    *(g_v4u *)(dst + 2 * a.plane_stride) = b2;
                }
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_residues_row(ResRowArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint32_t smem_rr[];
    residues_row_block<32>(a, smem_rr);
}

// Residues of a^ on the matrix cores (stage 2).  For every modulus the residue of an
// entry is a dot product of its magnitude's bytes with the weights 256^j mod m, so a
// wave computes a (weight rows) x (64 entries) int8 product with
// v_mfma_i32_32x32x32_i8 and then reduces each exact int32 sum x to the centred
// x - rint(x/m) m (exact in fp64, |x| < 2^31): no per-modulus pass over the words.
// The weight rows, the correction bytes that carry the sign, and the row layout are
// described with build_residue_mma_tables.  One wave per (row r, 64 consecutive k):
//   phase 0: lane k writes its entry's bytes to LDS (entry-major, stride es words),
//            complemented if negative, already offset by -128 (xor 0x80);
//   phase 1: per block of 32 weight rows, rnq k-steps of two MFMAs (entries 0-31 and
//            32-63) with A = weight fragments (global), B = entry bytes (read from LDS
//            into registers once);
//   phase 2: the 32 x 64 sums go through an LDS scratch (entry-major, 144-byte rows) so
//            that lane k reduces its own entry for every modulus of the block with
//            wave-uniform modulus data, and stores 64 contiguous bytes per plane.
// Bank layout: es = 4 (2 i + 1) words and the 144-byte scratch rows put the 16 lanes a
// 16-byte LDS access serves per cycle on 16 different bank groups.
struct ResMmaArgs {
    const uint64_t *limbs;
    const int32_t *exps;
    const int8_t *signs;
    int64_t rs, cs, rows, count, kpad, plane_stride;
    const int32_t *erow;
    const int32_t *koff;
    int p, nl, t, nw32, nq, nrb, es;
    const int8_t *wfrag;
    const ResRowBlock *rblk;
    int8_t *planes;
};

static_assert(offsetof(ResRowBlock, md) == 256 && offsetof(ResRowBlock, g0) == 512 &&
                  offsetof(ResRowBlock, n1) == 640 && offsetof(ResRowBlock, p0) == 644 &&
                  offsetof(ResRowBlock, n2) == 648,
              "byte offsets the MFMA residue kernel reads the row block record at");
constexpr int kResScratchRow = 144;   // bytes per entry in the sums scratch (32 rows + 16)
constexpr int kResMmaMaxQ = 16;       // k-steps of the widest integer (t < 3400 bits: 14)
constexpr int kResMmaPfQ = 8;         // up to this many k-steps the next weights are prefetched

__host__ __device__ constexpr int res_mma_es(int nq) { return 8 * nq + 4; }
// LDS per wave: the entry bytes, later reused by the sums scratch
__host__ __device__ constexpr int res_mma_wave_lds(int nq) {
    return 64 * res_mma_es(nq) * 4 > 64 * kResScratchRow ? 64 * res_mma_es(nq) * 4 : 64 * kResScratchRow;
}


// At most NQ k-steps: entry and weight fragments live in registers (up to kResMmaPfQ
// k-steps the weights of the next block of rows are prefetched while one block is
// reduced), and the sums scratch reuses the entry bytes' LDS.
template <int RB, int NQ>
__device__ __forceinline__ void residue_block_mma_r(
    const uint64_t *__restrict__ limbs, const int32_t *__restrict__ exps,
    const int8_t *__restrict__ signs, const int32_t *__restrict__ erow,
    const int32_t *__restrict__ koff, const int8_t *__restrict__ wfrag,
    const ResRowBlock *__restrict__ rblk, int8_t *__restrict__ planes, int64_t rs, int64_t cs,
    int64_t rows, int64_t count, int64_t kpad, int64_t plane_stride, int p, int nl, int t,
    int nw32, int nq, int nrb, int64_t bx, int64_t by, uint32_t *smem) {
    static_assert(NQ >= 1 && NQ <= kResMmaMaxQ, "k-steps");
    constexpr bool PF = NQ <= kResMmaPfQ;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int es = res_mma_es(nq);
    uint32_t *ent = smem + (size_t)wv * (res_mma_wave_lds(nq) / 4);
    uint8_t *scr = (uint8_t *)ent;
    constexpr int KW = res_waves_k(RB);   // waves side by side along k, as in residue_block_r
    const int64_t k = (bx * KW + wv % KW) * 64 + lane;
    const int64_t r = by * (RB / KW) + wv / KW;

    typedef const __attribute__((address_space(1))) v4i gv4i;
    gv4i *wf = (gv4i *)wfrag + lane;
    v4i wa[NQ], wn[PF ? NQ : 1];
#pragma unroll
    for (int q = 0; q < NQ; ++q)   // the first block's weights load while the entry is built
        if (q < nq) wa[q] = wf[q * 64];

    // phase 0: this lane's entry, bytes offset by -128
    OZ2H_G(int8_t) *gsigns = (OZ2H_G(int8_t) *)signs;
    OZ2H_G(int32_t) *gexps = (OZ2H_G(int32_t) *)exps;
    OZ2H_G(int32_t) *gerow = (OZ2H_G(int32_t) *)erow;
    OZ2H_G(int32_t) *gkoff = (OZ2H_G(int32_t) *)koff;
    int s = 0;
    int64_t sh = 0, idx = 0;
    if (r < rows && k < count) {
        idx = r * rs + k * cs;
        s = gsigns[idx];
        sh = (int64_t)t - p + gexps[idx] + (koff ? gkoff[k] : 0) - gerow[r];
    }
    uint32_t *ew = ent + lane * es;
    s = build_words((OZ2H_G(uint64_t) *)limbs + idx * nl, s, sh, p, nw32, ew, 1);
    const uint32_t cmask = s < 0 ? 0xFFFFFFFFu : 0u;
    for (int w = 0; w < nw32; ++w) ew[w] = (s == 0 ? 0u : ew[w] ^ cmask) ^ 0x80808080u;
    ew[nw32] = (s < 0 ? 0x100u : 0u) ^ 0x80808080u;   // correction bytes nb, nb + 1
    for (int w = nw32 + 1; w < 8 * nq; ++w) ew[w] = 0x80808080u;

    // read-only for the whole launch: the constant address space keeps these wave-uniform
    // reads on the scalar unit across the LDS hand-over fences
    typedef const __attribute__((address_space(4))) ResRowBlock crb_t;
    crb_t *grb = (crb_t *)rblk;
    const int h = lane >> 5, c = lane & 31;
    const v4i *b0p = (const v4i *)(ent + c * es + 4 * h);          // entries 0-31
    const v4i *b1p = (const v4i *)(ent + (32 + c) * es + 4 * h);   // entries 32-63
    v4i bf0[NQ], bf1[NQ];
    wave_lds_sync();   // entry bytes written
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        if (q < nq) {
            bf0[q] = b0p[2 * q];
            bf1[q] = b1p[2 * q];
        }
    // the block's region of every plane (uniform 64-bit base) and a 32-bit lane offset in it
    const int64_t r0b = by * (RB / KW), k0b = bx * KW * 64;
    planes += r0b * kpad + k0b;
    const uint32_t loff = (uint32_t)((r - r0b) * kpad + (k - k0b));
    // stores: after a quad byte transpose, lane 4 a + q writes entries 4 a .. 4 a + 3 of
    // plane q of a group of four (a dword at the quad's first entry)
    const QuadSel qsel = quad_sel(lane);
    const int64_t qoff = (int64_t)(lane & 3) * plane_stride + (int64_t)(loff & ~3u);
    const uint32_t *xrow = (const uint32_t *)(scr + lane * kResScratchRow);
    for (int rb = 0; rb < nrb; ++rb) {
        wave_lds_sync();   // entry bytes read; the previous block's sums read
        v16i acc0 = v16i{}, acc1 = v16i{};
        if constexpr (PF) {
            if (rb + 1 < nrb) {
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    if (q < nq) wn[q] = wf[((size_t)(rb + 1) * nq + q) * 64];
            }
        } else if (rb > 0) {
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                if (q < nq) wa[q] = wf[((size_t)rb * nq + q) * 64];
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (q < nq) {
                acc0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(wa[q], bf0[q], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(wa[q], bf1[q], acc1, 0, 0, 0);
            }
        // sums element e: row 8 (e / 4) + 4 h + e % 4, entry c (acc0) or 32 + c (acc1)
#pragma unroll
        for (int a4 = 0; a4 < 4; ++a4) {
            const int ro = (8 * a4 + 4 * h) * 4;
            *(v4i *)(scr + c * kResScratchRow + ro) =
                v4i{acc0[4 * a4], acc0[4 * a4 + 1], acc0[4 * a4 + 2], acc0[4 * a4 + 3]};
            *(v4i *)(scr + (32 + c) * kResScratchRow + ro) =
                v4i{acc1[4 * a4], acc1[4 * a4 + 1], acc1[4 * a4 + 2], acc1[4 * a4 + 3]};
        }
        wave_lds_sync();   // sums written
        // lane k reduces its own entry: four rows per 16-byte read (two-limb pairs start
        // on a multiple of 4), the modulus data of four rows per scalar load, every row of
        // the four computed (rows past the moduli hold zeros).  The sums and modulus data of
        // the next four rows load while four rows are reduced (scheduling fences keep those
        // loads behind the first use of the current ones, whose wait covers every scalar and
        // LDS load in flight); reads up to row 35 stay inside the block record and the
        // scratch row.  Only the last group of a kind guards its stores.
        typedef double d4 __attribute__((ext_vector_type(4)));
        typedef const __attribute__((address_space(4))) d4 cd4;
        typedef const __attribute__((address_space(4))) char cch;
        typedef const __attribute__((address_space(4))) uint32_t cu32;
        cch *B = (cch *)(grb + rb);
        const int n1 = (int)((cu32 *)(B + 640))[0], p0 = (int)((cu32 *)(B + 640))[1],
                  n2 = (int)((cu32 *)(B + 640))[2];
        // row data of rows i .. i + 3: fl(1/m) at byte 8 i, m at 256 + 8 i
        v4i xn;
        d4 imn, mmn;
        auto fetch = [&](uint32_t i) {
            xn = *(const v4i *)(xrow + i);
            imn = *(cd4 *)(B + 8u * i);
            mmn = *(cd4 *)(B + (256u + 8u * i));
        };
        // first planes (byte 512 + 4 i): the one-limb rows of a block own consecutive planes
        // from that of row 0, and its two-limb pairs consecutive triples from that of row p0
        const uint32_t g1 = *(cu32 *)(B + 512);
        int i4 = 0;
        fetch(0);
        auto group1 = [&](auto full_) {   // one-limb rows i4 .. i4 + 3
            constexpr bool FULL = decltype(full_)::value;
            const d4 mm = mmn;
            double x[4], q[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                x[e] = (double)xn[e];
                q[e] = rint(x[e] * imn[e]);
            }
            __builtin_amdgcn_sched_barrier(0);
            fetch(i4 + 4);
            __builtin_amdgcn_sched_barrier(0);
            g_i8 *pb = uniform_ptr((g_i8 *)planes + (int64_t)(g1 + i4) * plane_stride);
            int ri[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) ri[e] = (int)fma(-q[e], mm[e], x[e]);
            const uint32_t w = quad_transpose_bytes(pack_bytes(ri[0], ri[1], ri[2], ri[3]), qsel);
            if (FULL || (lane & 3) < n1 - i4) *(g_u32 *)(pb + qoff) = w;
        };
        for (; i4 + 4 <= n1; i4 += 4) group1(std::true_type{});
        if (i4 < n1) group1(std::false_type{});
        if (n2 > 0) {
            const uint32_t g2 = *(cu32 *)(B + (512u + 4u * (uint32_t)p0));
            // only the first row of a pair holds modulus data: load those two of four rows
            // (loading all four would leave half of the destination registers dead, free for
            // reuse while the load is still in flight)
            typedef const __attribute__((address_space(4))) double cdbl;
            double im0, im2, mm0, mm2;
            auto fetch2 = [&](uint32_t i) {
                xn = *(const v4i *)(xrow + i);
                im0 = *(cdbl *)(B + 8u * i);
                im2 = *(cdbl *)(B + (16u + 8u * i));
                mm0 = *(cdbl *)(B + (256u + 8u * i));
                mm2 = *(cdbl *)(B + (272u + 8u * i));
            };
            int j2 = 0;
            fetch2((uint32_t)p0);
            auto group2 = [&](auto full_) {   // two-limb pairs j2, j2 + 1 (rows p0 + 2 j2 ..)
                constexpr bool FULL = decltype(full_)::value;
                const uint32_t i4 = (uint32_t)(p0 + 2 * j2);
                const double mm[2] = {mm0, mm2};
                double x[2], q[2];
#pragma unroll
                for (int e = 0; e < 2; ++e) x[e] = (double)(xn[2 * e] + 128 * xn[2 * e + 1]);
                q[0] = rint(x[0] * im0);
                q[1] = rint(x[1] * im2);
                __builtin_amdgcn_sched_barrier(0);
                fetch2(i4 + 4);
                __builtin_amdgcn_sched_barrier(0);
                g_i8 *pb = uniform_ptr((g_i8 *)planes + (int64_t)(g2 + 3u * (uint32_t)j2) * plane_stride);
                int r0[2], r1[2];
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int ri = (int)fma(-q[e], mm[e], x[e]);
                    r0[e] = ((ri + 64) & 127) - 64;   // balanced base-128 split
                    r1[e] = (ri - r0[e]) >> 7;
                }
                // planes 0-5 of the two pairs: (r0, r1, r0 + r1) of the first, then the second
                const uint32_t wa = quad_transpose_bytes(pack_bytes(r0[0], r1[0], r0[0] + r1[0], r0[1]), qsel);
                const uint32_t wb = quad_transpose_bytes(pack_bytes(r1[1], r0[1] + r1[1], 0, 0), qsel);
                const int nv = FULL ? 6 : 3 * (n2 - j2);   // planes to write
                if ((lane & 3) < nv) *(g_u32 *)(pb + qoff) = wa;
                if ((lane & 3) + 4 < nv) *(g_u32 *)(pb + 4 * plane_stride + qoff) = wb;
            };
            for (; j2 + 2 <= n2; j2 += 2) group2(std::true_type{});
            if (j2 < n2) group2(std::false_type{});
        }
        if constexpr (PF) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) wa[q] = wn[q];
        }
    }
}

template <int RB, int NQ>
__global__ __launch_bounds__(64 * RB) void k_residues_mma(ResMmaArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint32_t smem_res[];
    const int64_t nbx = a.kpad / (64 * res_waves_k(RB));
    residue_block_mma_r<RB, NQ>(a.limbs, a.exps, a.signs, a.erow, a.koff, a.wfrag, a.rblk, a.planes,
                            a.rs, a.cs, a.rows, a.count, a.kpad, a.plane_stride, a.p, a.nl, a.t,
                            a.nw32, a.nq, a.nrb, (int64_t)blockIdx.x % nbx, (int64_t)blockIdx.x / nbx,
                            smem_res);
}

// ---------------------------------------------------------------- stage 3

constexpr int GBK = 128;   // k padding granule of the residue planes = the GEMM k-tile
constexpr int TBK = 128;   // k-tile of the GEMM kernel: one 128-byte LDS row per output row

// centred residue x - rint(x/m) m of an exact fp64 integer x (|x| < 2^52)
__device__ __forceinline__ int32_t centred_mod(double x, double md, double inv_m) {
    return (int32_t)fma(-rint(x * inv_m), md, x);
}

// chunk swizzle of LDS tile row r: distinct over the rows of equal parity among any 16
// aligned rows, and over any 8 aligned rows
__device__ __forceinline__ int lds_swz(int r) { return (r & 7) ^ ((r >> 3) & 1); }

// One (2 WM) x (2 WN) output tile of one modulus per block; four waves in 2x2,
// each a WM x WN sub-tile of v_mfma_i32_32x32x32_i8 blocks (exact int32 sums,
// K * 127^2 < 2^31).  k-tiles of 128 bytes move global -> LDS by direct loads
// (global_load_lds_dwordx4: no register staging, no LDS store instructions) into a
// three-stage LDS ring, two tiles ahead of the multiplies.  A tile row is 128 bytes
// = eight 16-byte chunks, chunk c of row r stored at c ^ lds_swz(r): the 16 rows a
// ds_read_b128 serves per LDS cycle (64 banks of 4 bytes, two 128-byte rows per bank
// period) then hit 16 different 16-byte bank groups, and so do any 8 consecutive rows.
// The lane order of a direct load fixes the LDS side (16 bytes per lane, consecutive),
// so the swizzle is applied to the global addresses: load i of wave w fills LDS rows
// 32 i + 8 w .. + 7, lane -> row 32 i + 8 w + lane / 8, physical chunk lane % 8, which
// holds logical chunk (lane % 8) ^ lds_swz(row).
// The output is v_l = c_l (P/m_l)^-1 mod m_l as a centred int16: the reduction
// mod m_l and the first step of the direct CRT are fused here.
// A two-limb modulus runs its three Karatsuba products (planes r0, r1, r0 + r1:
// P0, P2, Ps) as one continuous k-loop into the SAME accumulators: we want
// c0 P0 + c2 P2 + cs Ps mod m with the weighted coefficients
// (c0, c2, cs) = (-127, 16256, 128) (P/m)^-1, and fold in place at the end of
// each product with w0 = c2^-1 c0, w1 = cs^-1 c2, w2 = cs (m is prime, so the
// inverses exist): acc = P0 w0 -> + P2 -> * w1 -> + Ps -> * w2.  Between the
// products |acc| <= m/2, so acc + K 127^2 < 2^31 stays exact.
// Blocks run the two-limb moduli first (they are three times longer).
// RAW = true: plain int32 output of a single plane (exactness tests).
struct GemmArgs {
    const int8_t *A, *B;
    int64_t kpad, a_ps, b_ps;
    const ModInfo *mi;
    int16_t *V;
    int64_t v_ps, ldv;
    int32_t *Craw;
};

// LDS stage S of the direct-load GEMM: one object per stage, so that the compiler can
// tell a read of one stage from a load still filling another
template <int WM, int WN, int S>
__device__ __forceinline__ int8_t *gemm_stage() {
    __shared__ __attribute__((aligned(1024))) int8_t st[(2 * WM + 2 * WN) * TBK];
    return st;
}

// s_waitcnt immediate: wait until at most `vm` vector-memory loads are outstanding
// (LDS/scalar and export counters left at their maximum)
constexpr int vmcnt_imm(int vm) { return (vm & 0xF) | (((vm >> 4) & 3) << 14) | (0x7 << 4) | (0xF << 8); }

// Arguments of the products that combine into an existing output (complex products):
// V2 is a second output set with the same strides as V.
struct GemmArgsZ : GemmArgs {
    int16_t *V2;
};

// output combination of a complex product's residue GEMMs (x = this product's weighted
// residue, all values centred mod m_l):
//   ZSTORE  V = x;   ZADD  V = V + x;   ZSUB  V = V - x;
//   ZGAUSS  (t1, t2) = (V, V2);  V = t1 - t2;  V2 = x - t1 - t2   (3M's last product)
enum GemmMode { ZSTORE = 0, ZADD = 1, ZSUB = 2, ZGAUSS = 3 };

// one output tile (mt, nt) of modulus l with an NS-stage LDS ring, NS - 1 tiles ahead
template <int WM, int WN, bool RAW, int NS = 3, int MODE = ZSTORE, class Args = GemmArgs>
__device__ __forceinline__ void gemm_tile(const Args &args, int64_t mt, int64_t nt, int l) {
    static_assert(NS == 2 || NS == 3, "two or three LDS stages");
    constexpr int BM = 2 * WM, BN = 2 * WN, FM = WM / 32, FN = WN / 32;
    constexpr int NLA = BM / 32, NL = (BM + BN) / 32;   // direct loads per wave per k-tile
    const int8_t *__restrict__ A = args.A;
    const int8_t *__restrict__ B = args.B;
    const int64_t kpad = args.kpad, a_ps = args.a_ps, b_ps = args.b_ps, ldv = args.ldv;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave >> 1, wc = wave & 1;
    const int64_t m0 = mt * BM, n0 = nt * BN;

    uint32_t g0 = 0, nprod = 1;
    double md = 1.0, inv_m = 1.0;
    int32_t kc[3] = {1, 1, 1};
    if (!RAW) {
        const ModInfo info = args.mi[l];
        g0 = info.g0;
        nprod = info.nprod;
        md = (double)info.m;
        inv_m = info.inv_m;
        kc[0] = info.kc[0];
        kc[1] = info.kc[1];
        kc[2] = info.kc[2];
    }
    const int nk = (int)(kpad / TBK);   // kpad is a multiple of 128
    const int ntile = (int)nprod * nk;

    uint32_t goff[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int R = 32 * i + 8 * wave + (lane >> 3);
        const int rl = i < NLA ? R : R - BM;
        goff[i] = (uint32_t)(rl * kpad) + ((((lane & 7) ^ lds_swz(R))) << 4);
    }
    const int8_t *Ab = A + m0 * kpad, *Bb = B + n0 * kpad;
    auto issue = [&](auto s_, int prod, int kt) {
        int8_t *dst = gemm_stage<WM, WN, decltype(s_)::value>();
        const int64_t ko = (int64_t)kt * TBK;
        const int8_t *a = Ab + (int64_t)(g0 + prod) * a_ps + ko;
        const int8_t *b = Bb + (int64_t)(g0 + prod) * b_ps + ko;
#pragma unroll
        for (int i = 0; i < NL; ++i)
            __builtin_amdgcn_global_load_lds((const void *)((i < NLA ? a : b) + goff[i]),
                                             (__attribute__((address_space(3))) void *)(dst + (4 * i + wave) * 1024),
                                             16, 0, 0);
    };

    v16i acc[FM][FN];
#pragma unroll
    for (int x = 0; x < FM; ++x)
#pragma unroll
        for (int y = 0; y < FN; ++y) acc[x][y] = v16i{};

    const int frow = lane & 31;
    v4i fa[2][FM], fb[2][FN];
    auto fload = [&](int set, int ks, const int8_t *cA, const int8_t *cB) {
        const int fo = frow * TBK + (((2 * ks + (lane >> 5)) ^ lds_swz(frow)) << 4);
#pragma unroll
        for (int x = 0; x < FM; ++x) fa[set][x] = *(const v4i *)(cA + (wr * WM + x * 32) * TBK + fo);
#pragma unroll
        for (int y = 0; y < FN; ++y) fb[set][y] = *(const v4i *)(cB + (wc * WN + y * 32) * TBK + fo);
    };
    auto fold = [&](int prod) {
        const double w = (double)(prod == 0 ? kc[0] : prod == 1 ? kc[1] : kc[2]);
#pragma unroll
        for (int x = 0; x < FM; ++x)
#pragma unroll
            for (int y = 0; y < FN; ++y)
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    acc[x][y][e] = centred_mod((double)acc[x][y][e] * w, md, inv_m);
    };

    // (cp, ck): product and k-tile of tile T; (lp, lk): of the tile loaded next, clamped to
    // the last one.  Every k-tile issues one tile (the last one again near the end), so the
    // number of loads in flight behind a tile does not depend on the path taken.
    int cp = 0, ck = 0, lp = 0, lk = 0;
    auto advance = [&](int &pp, int &kk) {
        if (++kk == nk) {
            kk = 0;
            ++pp;
        }
    };
    auto advance_clamped = [&](int &pp, int &kk) {   // branch-free: selects only
        const bool more = pp * nk + kk < ntile - 1, wrap = kk + 1 == nk;
        pp = more && wrap ? pp + 1 : pp;
        kk = more ? (wrap ? 0 : kk + 1) : kk;
    };
    auto mfma = [&](int set) {
#pragma unroll
        for (int x = 0; x < FM; ++x)
#pragma unroll
            for (int y = 0; y < FN; ++y)
                acc[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[set][x], fb[set][y], acc[x][y], 0, 0, 0);
    };
    issue(std::integral_constant<int, 0>{}, lp, lk);
    advance_clamped(lp, lk);
    if constexpr (NS == 3) {
        issue(std::integral_constant<int, 1>{}, lp, lk);
        advance_clamped(lp, lk);
    }
    // one k-tile from stage S; the tile NS - 1 ahead goes into stage (S + NS - 1) % NS,
    // which every wave finished reading before the barrier
    auto body = [&](auto s_) {
        constexpr int S = decltype(s_)::value, SN = (S + NS - 1) % NS;
        __builtin_amdgcn_s_waitcnt(vmcnt_imm((NS - 2) * NL));   // own loads of tile T landed
        __builtin_amdgcn_s_barrier();                            // everyone's did
        issue(std::integral_constant<int, SN>{}, lp, lk);
        advance_clamped(lp, lk);
        const int8_t *cA = gemm_stage<WM, WN, S>(), *cB = cA + BM * TBK;
        fload(0, 0, cA, cB);
        auto kstep = [&](auto kc_) {
            constexpr int ks = decltype(kc_)::value;
            if constexpr (ks + 1 < 4) fload((ks + 1) & 1, ks + 1, cA, cB);
            mfma(ks & 1);
#if OZ2H_GEMM_SCHED
            if constexpr (ks + 1 < 4) __builtin_amdgcn_sched_group_barrier(0x100, FM + FN, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, FM * FN, 0);
#endif
        };
        kstep(std::integral_constant<int, 0>{});
        kstep(std::integral_constant<int, 1>{});
        kstep(std::integral_constant<int, 2>{});
        kstep(std::integral_constant<int, 3>{});
        if (!RAW && ck == nk - 1) fold(cp);
        advance(cp, ck);
    };
    int t0 = 0;
    for (; t0 + NS <= ntile; t0 += NS) {
        body(std::integral_constant<int, 0>{});
        body(std::integral_constant<int, 1>{});
        if constexpr (NS == 3) body(std::integral_constant<int, 2>{});
    }
    if (t0 < ntile) {
        body(std::integral_constant<int, 0>{});
        if (NS == 3 && t0 + 1 < ntile) body(std::integral_constant<int, 1>{});
    }
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));   // no load still writing LDS past the block's end

    const int64_t lane_off = (m0 + wr * WM + 4 * (lane >> 5)) * ldv + n0 + wc * WN + (lane & 31);
    if (RAW) {
        int32_t *base = args.Craw + lane_off;
#pragma unroll
        for (int x = 0; x < FM; ++x)
#pragma unroll
            for (int y = 0; y < FN; ++y)
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    base[(int64_t)(x * 32 + 8 * (e >> 2) + (e & 3)) * ldv + y * 32] = acc[x][y][e];
        return;
    }
    int16_t *base = args.V + (int64_t)l * args.v_ps + lane_off;
    if constexpr (MODE == ZSTORE) {
#pragma unroll
        for (int x = 0; x < FM; ++x)
#pragma unroll
            for (int y = 0; y < FN; ++y)
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    base[(int64_t)(x * 32 + 8 * (e >> 2) + (e & 3)) * ldv + y * 32] = (int16_t)acc[x][y][e];
    } else {
        int16_t *base2 = nullptr;
        if constexpr (MODE == ZGAUSS) base2 = args.V2 + (int64_t)l * args.v_ps + lane_off;
        // per row group x: every old value is loaded before the first store, so the group
        // waits once (stores count against the same counter as loads: interleaved, each
        // load would wait for the stores before it)
#pragma unroll
        for (int x = 0; x < FM; ++x) {
            int32_t t1[FN][16], t2[FN][16];
#pragma unroll
            for (int y = 0; y < FN; ++y)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int64_t o = (int64_t)(x * 32 + 8 * (e >> 2) + (e & 3)) * ldv + y * 32;
                    t1[y][e] = base[o];
                    if constexpr (MODE == ZGAUSS) t2[y][e] = base2[o];
                }
#pragma unroll
            for (int y = 0; y < FN; ++y)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int64_t o = (int64_t)(x * 32 + 8 * (e >> 2) + (e & 3)) * ldv + y * 32;
                    const int32_t v = acc[x][y][e];
                    if constexpr (MODE == ZADD) {
                        base[o] = (int16_t)centred_mod((double)(t1[y][e] + v), md, inv_m);
                    } else if constexpr (MODE == ZSUB) {
                        base[o] = (int16_t)centred_mod((double)(t1[y][e] - v), md, inv_m);
                    } else {
                        base[o] = (int16_t)centred_mod((double)(t1[y][e] - t2[y][e]), md, inv_m);
                        base2[o] = (int16_t)centred_mod((double)(v - t1[y][e] - t2[y][e]), md, inv_m);
                    }
                }
        }
    }
}

// XCD-aware block order of the plain launch.  Blocks are dealt to the 8 XCDs round-robin
// (block b runs on XCD b % 8, as its (b / 8)-th block there), and each XCD has its own L2.
// With `on`, XCD x covers one rectangle of h x w tiles (rectangle row x / rx, column x % rx)
// of every modulus, moduli in launch order: all XCDs still share each modulus's work
// evenly, but an XCD reads h tile rows of A and w tile columns of B instead of all of A.
struct XcdMap {
    uint32_t on, rx, h, w;   // h * w tiles per XCD and modulus
};

// plain launch: two-limb moduli (listed last) first; grid (N tiles, M tiles, moduli), or
// with an XCD map a 1-D grid of the same blocks
template <int WM, int WN, bool RAW>
__global__ __launch_bounds__(256) void k_resgemm(GemmArgs args, int L, XcdMap xm) {
    uint32_t mt = blockIdx.y, nt = blockIdx.x, zi = blockIdx.z;
    if (xm.on) {
        const uint32_t b = blockIdx.x, x = b & 7u, s = b >> 3, t8 = xm.h * xm.w;
        zi = s / t8;
        const uint32_t u = s - zi * t8;
        mt = (x / xm.rx) * xm.h + u / xm.w;
        nt = (x % xm.rx) * xm.w + u % xm.w;
    }
    const int l = RAW ? 0 : L - 1 - (int)zi;
    gemm_tile<WM, WN, RAW>(args, mt, nt, l);
}

// one residue GEMM of a complex product (the 3M / 4M schemes): the plain launch's block
// order and tiles, the output combined into V (and V2) by MODE
template <int WM, int WN, int MODE>
__global__ __launch_bounds__(256) void k_resgemm_z(GemmArgsZ args, int L, XcdMap xm) {
    uint32_t mt = blockIdx.y, nt = blockIdx.x, zi = blockIdx.z;
    if (xm.on) {
        const uint32_t b = blockIdx.x, x = b & 7u, s = b >> 3, t8 = xm.h * xm.w;
        zi = s / t8;
        const uint32_t u = s - zi * t8;
        mt = (x / xm.rx) * xm.h + u / xm.w;
        nt = (x % xm.rx) * xm.w + u % xm.w;
    }
    gemm_tile<WM, WN, false, 3, MODE, GemmArgsZ>(args, mt, nt, L - 1 - (int)zi);
}

// Residue planes of a sum of two operands (3M: Ar + Ai, Br + Bi) from the planes of
// each: per modulus l, s = x + y reduced to the centred residue s - rint(s/m) m (the
// quotient in fp32 is exact: |s| <= m + 3 < 2^15 and s/m is at least 1/(2m) from a
// half-integer for odd m; for the even one-limb modulus 128 either tie is a valid
// representative with |r| <= 64), then split like the residue kernels (one byte, or
// the balanced base-128 limbs (r0, r1, r0 + r1)).  One thread per 16 bytes of a plane;
// grid (ps / 4096 blocks of 256 threads, L).  ps is a multiple of 4096.
__global__ __launch_bounds__(256) void k_plane_sum(const int8_t *__restrict__ X,
                                                   const int8_t *__restrict__ Y,
                                                   int8_t *__restrict__ S, int64_t ps,
                                                   const ModInfo *__restrict__ mi) {
    const ModInfo info = load_info((OZ2H_G(ModInfo) *)(mi + blockIdx.y));
    const int64_t o = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 16;
    if (o >= ps) return;
    const float inv_m = (float)info.inv_m;
    const int64_t b0 = (int64_t)info.g0 * ps + o;
    auto reduce = [&](int sv) { return sv - (int)rintf((float)sv * inv_m) * (int)info.m; };
    if (info.nprod == 1) {
        const int4 xa = *(const int4 *)(X + b0), ya = *(const int4 *)(Y + b0);
        const int8_t *xb = (const int8_t *)&xa, *yb = (const int8_t *)&ya;
        int4 out;
        int8_t *ob = (int8_t *)&out;
#pragma unroll
        for (int i = 0; i < 16; ++i) ob[i] = (int8_t)reduce((int)xb[i] + (int)yb[i]);
        *(int4 *)(S + b0) = out;
        return;
    }
    const int4 x0 = *(const int4 *)(X + b0), x1 = *(const int4 *)(X + b0 + ps);
    const int4 y0 = *(const int4 *)(Y + b0), y1 = *(const int4 *)(Y + b0 + ps);
    const int8_t *x0b = (const int8_t *)&x0, *x1b = (const int8_t *)&x1;
    const int8_t *y0b = (const int8_t *)&y0, *y1b = (const int8_t *)&y1;
    int4 o0, o1, o2;
    int8_t *o0b = (int8_t *)&o0, *o1b = (int8_t *)&o1, *o2b = (int8_t *)&o2;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int r = reduce((int)x0b[i] + 128 * (int)x1b[i] + (int)y0b[i] + 128 * (int)y1b[i]);
        const int r0 = ((r + 64) & 127) - 64;   // balanced base-128 split
        const int r1 = (r - r0) >> 7;
        o0b[i] = (int8_t)r0;
        o1b[i] = (int8_t)r1;
        o2b[i] = (int8_t)(r0 + r1);
    }
    *(int4 *)(S + b0) = o0;
    *(int4 *)(S + b0 + ps) = o1;
    *(int4 *)(S + b0 + 2 * ps) = o2;
}

// ---------------------------------------------------------------- stage 4 + 5

// multi-digit helpers on an LDS digit column (stride `st` words between digits)
__device__ __forceinline__ bool dig_ge(const uint32_t *sd, int64_t st, const uint32_t *__restrict__ Q,
                                       int nd) {   // column >= Q ?
    int64_t br = 0;
    for (int k = 0; k < nd; ++k) br = ((int64_t)sd[k * st] - (int64_t)Q[k] - br) < 0;
    return br == 0;
}
__device__ __forceinline__ void dig_sub(uint32_t *sd, int64_t st, const uint32_t *__restrict__ Q,
                                        int nd) {   // column -= Q
    int64_t br = 0;
    for (int k = 0; k < nd; ++k) {
        const int64_t d = (int64_t)sd[k * st] - (int64_t)Q[k] - br;
        sd[k * st] = (uint32_t)d;
        br = d < 0;
    }
}
__device__ __forceinline__ void dig_rsub(uint32_t *sd, int64_t st, const uint32_t *__restrict__ Q,
                                         int nd) {   // column = Q - column
    int64_t br = 0;
    for (int k = 0; k < nd; ++k) {
        const int64_t d = (int64_t)Q[k] - (int64_t)sd[k * st] - br;
        sd[k * st] = (uint32_t)d;
        br = d < 0;
    }
}
__device__ __forceinline__ void dig_add(uint32_t *sd, int64_t st, const uint32_t *__restrict__ Q,
                                        int nd) {   // column += Q (mod 2^(32 nd))
    uint64_t cy = 0;
    for (int k = 0; k < nd; ++k) {
        const uint64_t d = (uint64_t)sd[k * st] + Q[k] + cy;
        sd[k * st] = (uint32_t)d;
        cy = d >> 32;
    }
}
// The magnitude digits of c^ read from its digit column.  On the fast path the
// column holds c^ in two's complement; for c^ < 0, |c^| = ~X + 1, so with z the
// lowest nonzero digit of X: digit k of |c^| is ~X_k above z, -X_z at z and 0
// below (no negation pass over the column).  Digits outside [0, nd) read as 0.
struct MagView {
    const uint32_t *sd;
    int64_t st;
    int nd, z;
    bool inv;
    __device__ __forceinline__ uint32_t operator()(int64_t k) const {
        if (k < 0 || k >= nd) return 0u;
        const uint32_t x = sd[k * st];
        if (!inv) return x;
        return k > z ? ~x : (k == z ? 0u - x : 0u);
    }
    // bits [pos, pos + 32)
    __device__ __forceinline__ uint32_t bits32(int64_t pos) const {
        const int64_t q = pos >> 5;
        const int r = (int)(pos & 31);
        const uint64_t lo = (*this)(q), hi = (*this)(q + 1);
        return (uint32_t)(((hi << 32) | lo) >> r);
    }
    // any nonzero bit below position pos
    __device__ __forceinline__ bool any_below(int64_t pos) const {
        const int64_t full = pos >> 5;
        const int rr = (int)(pos & 31);
        if (rr && ((*this)(full) & ((1u << rr) - 1)) != 0) return true;
        if (inv) return z < full;   // digit z is nonzero, everything below it is zero
        for (int64_t k = min(full, (int64_t)nd) - 1; k >= 0; --k)
            if (sd[k * st] != 0) return true;
        return false;
    }
};

// Direct CRT (subsection "Direct CRT without multiple-precision division").
// Each thread reconstructs EPT output entries (entries tid + q*blockDim of the
// block's range, so every load is coalesced).  Pass c accumulates digits
// [c*DC, (c+1)*DC) of S = sum_l v_l M_l over all moduli: v_l centred, M_l in
// balanced base-2^32 digits, so each column sum is an exact fp64 integer and
// the DC digit constants of modulus l are shared by the EPT entries.  Pass 0
// also forms sum_l v_l / m_l in binary64, an estimate of S/P = n + c^/P.
// Since |c^| < P/2, the nearest integer beta of that estimate is n unless the
// estimate lies within 2^-30 of a half-integer (never, when the CRT margin is
// at least 2, because then |c^| < P/4); in that case c^ = S - beta P comes out
// of one signed carry pass, already lifted.  Otherwise the paper's sequence is
// used: R = S - (alpha - 1) P with alpha = floor(estimate), R in [0, 3P), at
// most two subtractions of P, and the symmetric lift against floor(P/2).
// The magnitude digits sit in an LDS column; (ROUND) they are rounded once,
// nearest-even, to p bits with the scale 2^(e_i + f_j - 2t).
// The planes hold v_l = u_l (P/m_l)^-1 mod m_l as centred int16 (the residue
// GEMM applies the weight); WEIGHT = true takes plain residues u_l instead.
// The digit constants (and 1/m_l) are wave-uniform: scalar loads (SGPR operands of the
// FMAs) with LDS digit columns, LDS-staged slices of LB moduli with global ones.
struct CrtArgs {
    const int16_t *V;
    int64_t v_ps, ldv, M, N;
    const ModInfo *mi;
    int L;
    const double *dig;
    int ndpad, nc, nd32;
    const uint32_t *Pd, *Phd;
    const int32_t *erow, *fcol;   // nullable (0)
    int tsum, p;                  // value = c^ 2^(erow + fcol - tsum); tsum = 2t in the forward
    int8_t *osign;
    int32_t *oexp;
    uint64_t *olimbs;
    int64_t ldc;
    uint64_t *chat_mag;
    int nlc, LB;
    uint32_t *gdig;    // GDIG: digit columns in global memory, digit k of entry e at
    int64_t gstride;   // gdig[k * gstride + e] (gstride >= all entries the grid covers)
    // matrix-core CRT (k_crt_mma): A fragments, row blocks, contraction steps, top digits
    const int8_t *afr;
    int nbk, kq, nt;
    double inv_ptop;
};

// Lift and (ROUND) rounding of one output entry e from its digit column sd (stride
// cst): on the fast path the column holds c^ in two's complement over nd32 digits
// (sign = carry < 0); on the slow path it holds R = S - (alpha - 1) P in [0, 3P).
template <bool ROUND>
__device__ __forceinline__ void crt_finish(const CrtArgs &a, int64_t e, uint32_t *sd, int64_t cst,
                                           bool slow, int64_t carry) {
    const int nd32 = a.nd32, p = a.p;
    const int64_t N = a.N;
    const uint32_t *__restrict__ Phd = a.Phd;
    const int nl = (p + 63) / 64;
    bool neg;
    MagView mag{sd, cst, nd32, 0, false};
    if (!slow) {
        neg = carry < 0;   // two's complement c^ over nd32 digits
        if (neg) {
            int z = 0;
            while (z < nd32 - 1 && sd[z * cst] == 0) ++z;
            mag.z = z;
            mag.inv = true;
        }
    } else {
        // R in [0, 3P): at most two subtractions of P, then the symmetric lift
        if (dig_ge(sd, cst, a.Pd, nd32)) dig_sub(sd, cst, a.Pd, nd32);
        if (dig_ge(sd, cst, a.Pd, nd32)) dig_sub(sd, cst, a.Pd, nd32);
        neg = !dig_ge(sd, cst, Phd, nd32) ? false : true;   // x0 >= floor(P/2) ...
        if (neg) {                                          // ... and x0 != floor(P/2)
            dig_sub(sd, cst, Phd, nd32);
            bool eq = true;
            for (int k = 0; k < nd32 && eq; ++k) eq = sd[k * cst] == 0;
            dig_add(sd, cst, Phd, nd32);
            neg = !eq;
        }
        if (neg) dig_rsub(sd, cst, a.Pd, nd32);   // |c^| = P - x0
    }
    int top = nd32 - 1;
    while (top >= 0 && mag(top) == 0) --top;
    const int64_t i = e / N, j = e - i * N;

    if (!ROUND) {
        __attribute__((address_space(1))) uint64_t *o =
            (__attribute__((address_space(1))) uint64_t *)a.chat_mag + e * a.nlc;
        for (int w = 0; w < a.nlc; ++w)
            o[w] = (uint64_t)mag(2 * w) | ((uint64_t)mag(2 * w + 1) << 32);
        a.osign[e] = top < 0 ? 0 : (neg ? -1 : 1);
        return;
    }
    const int64_t oi = i * a.ldc + j;
    __attribute__((address_space(1))) uint64_t *o =
        (__attribute__((address_space(1))) uint64_t *)a.olimbs + oi * nl;
    if (top < 0) {
        for (int w = 0; w < nl; ++w) o[w] = 0;
        a.osign[oi] = 0;
        a.oexp[oi] = 0;
        return;
    }
    int64_t nb = 32 * (int64_t)top + (32 - __builtin_clz(mag(top)));
    const int64_t sh = nb - p;   // mant = RNE(mag / 2^sh)
    bool inc = false;
    if (sh > 0) {
        const int64_t rpos = sh - 1;
        if ((mag.bits32(rpos) & 1u) != 0)   // round bit set: up unless an exact tie to even
            inc = mag.any_below(rpos) || (mag.bits32(sh) & 1u);
    }
    // mant = mag / 2^sh (+ 1): limb w is bits [sh + 64 w, sh + 64 w + 64) of mag, formed from
    // three consecutive digits by funnel shifts, one pass from the bottom
    const int64_t q0 = sh >> 5;   // floor: sh < 0 reads zero digits below the column
    const int rsh = (int)(sh & 31);
    uint32_t prev = mag(q0);
    bool cy = inc;
    uint64_t last = 0;
    for (int w = 0; w < nl; ++w) {
        const uint32_t d1 = mag(q0 + 2 * w + 1), d2 = mag(q0 + 2 * w + 2);
        const uint64_t v = ((uint64_t)__builtin_amdgcn_alignbit(d2, d1, rsh) << 32) |
                           __builtin_amdgcn_alignbit(d1, prev, rsh);
        last = v + (cy ? 1u : 0u);
        cy = cy && last == 0;
        o[w] = last;
        prev = d2;
    }
    const int pb = p - 64 * (nl - 1);   // bits of the top limb
    if (pb < 64 ? (last >> pb) != 0 : cy) {   // mant = 2^p - 1 rounded up to 2^p: renormalise
        for (int w = 0; w < nl; ++w) o[w] = 0;
        o[(p - 1) >> 6] = 1ull << ((p - 1) & 63);
        nb += 1;
    }
    a.osign[oi] = neg ? -1 : 1;
    a.oexp[oi] = (int32_t)(nb + (int64_t)(a.erow ? a.erow[i] : 0) + (a.fcol ? a.fcol[j] : 0) -
                           (int64_t)a.tsum);
}

// LDS of a CRT block: bd * EPT digit columns of nd32 words (GDIG = false), or the
// LB x (DC + 1) doubles of a constant slice (GDIG = true: the digit columns of large
// nd32 sit in global memory).
template <int DC, int EPT, bool ROUND, bool WEIGHT, bool GDIG = false>
__device__ __forceinline__ void crt_block(const CrtArgs &a, int64_t blk, uint32_t *sdig) {
    const int tid = threadIdx.x, bd = blockDim.x, st = bd * EPT;
    const int64_t cst = GDIG ? a.gstride : (int64_t)st;   // digit stride of a column
    const int nd32 = a.nd32, L = a.L, LB = a.LB, ndpad = a.ndpad, p = a.p;
    const int64_t N = a.N, v_ps = a.v_ps;
    // global-memory views (pointers from a descriptor are generic otherwise)
    OZ2H_G(uint32_t) *Pd = (OZ2H_G(uint32_t) *)a.Pd;
    const uint32_t *__restrict__ Phd = a.Phd;
    OZ2H_G(ModInfo) *mi = (OZ2H_G(ModInfo) *)a.mi;
    // digit constants and 1/m: read-only for the launch and wave-uniform.  With LDS digit
    // columns (two entries per thread) the constant address space puts them on the scalar
    // unit (SGPR operands of the FMAs); with global columns (GDIG) a slice of LB moduli is
    // staged in LDS and read as broadcasts, two constants per ds_read_b128.
    typedef const __attribute__((address_space(4))) double cdouble;
    typedef const __attribute__((address_space(4))) ModInfo cmodinfo;
    cdouble *cdig = (cdouble *)a.dig;
    cmodinfo *cmi = (cmodinfo *)a.mi;
    double *stab = (double *)sdig;               // GDIG: LB x DC digits
    double *sinv = stab + (size_t)LB * DC;       // GDIG: LB x 1/m
    const int64_t MN = a.M * N;
    int64_t idx[EPT];
    OZ2H_G(int16_t) *vp[EPT];
    bool live[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        idx[q] = blk * st + q * bd + tid;
        live[q] = idx[q] < MN;
        // a dead lane reads entry 0 (always valid) and writes nothing: no branch around loads
        const int64_t ii = live[q] ? idx[q] / N : 0, jj = live[q] ? idx[q] - ii * N : 0;
        vp[q] = (OZ2H_G(int16_t) *)a.V + ii * a.ldv + jj;
    }
    auto col = [&](int q) -> uint32_t * { return GDIG ? a.gdig + idx[q] : sdig + q * bd + tid; };

    int64_t beta[EPT], carry[EPT];
    bool slow[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        beta[q] = 0;
        carry[q] = 0;
        slow[q] = false;
    }
    for (int c = 0; c < a.nc; ++c) {
        double acc[EPT][DC], asum[EPT];
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            asum[q] = 0.0;
#pragma unroll
            for (int d = 0; d < DC; ++d) acc[q][d] = 0.0;
        }
        for (int l0 = 0; l0 < L; l0 += LB) {
            const int nlb = min(LB, L - l0);
            if constexpr (GDIG) {
                OZ2H_G(double) *dc = (OZ2H_G(double) *)a.dig + c * DC;
                __syncthreads();   // the previous slice has been consumed by every thread
                for (int e = tid; e < nlb * DC; e += bd) {
                    const int ll = e / DC, d = e - ll * DC;
                    stab[e] = dc[(size_t)(l0 + ll) * ndpad + d];
                }
                for (int e = tid; e < nlb; e += bd) sinv[e] = mi[l0 + e].inv_m;
                __syncthreads();
            }
            // v_l of the next PF moduli are loaded ahead (unconditional, clamped at the end)
            constexpr int PF = 4;
            int ring[PF][EPT];
#pragma unroll
            for (int f = 0; f < PF; ++f)
#pragma unroll
                for (int q = 0; q < EPT; ++q) ring[f][q] = vp[q][(int64_t)(l0 + min(f, nlb - 1)) * v_ps];
            // one modulus: its v values (one per entry of the thread) into the digit sums
            auto inv_of = [&](int ll) { return GDIG ? sinv[ll] : cmi[l0 + ll].inv_m; };
            auto modulus = [&](int ll, const int *cur, double inv_m) {
                const int l = l0 + ll;
                double vd[EPT];
#pragma unroll
                for (int q = 0; q < EPT; ++q) {
                    const int raw = cur[q];
                    if (WEIGHT) {
                        const ModInfo info = load_info(mi + l);
                        vd[q] = (double)centred_mod((double)raw * (double)info.minv, (double)info.m, inv_m);
                    } else {
                        vd[q] = (double)raw;
                    }
                    if (c == 0) asum[q] = fma(vd[q], inv_m, asum[q]);
                }
                if constexpr (GDIG) {
                    const double *dl = stab + (size_t)ll * DC;
#pragma unroll
                    for (int d = 0; d < DC; d += 2) {
                        const double2 w = *(const double2 *)(dl + d);
#pragma unroll
                        for (int q = 0; q < EPT; ++q) {
                            acc[q][d] = fma(vd[q], w.x, acc[q][d]);
                            acc[q][d + 1] = fma(vd[q], w.y, acc[q][d + 1]);
                        }
                    }
                } else {
                    cdouble *dl = cdig + (size_t)l * ndpad + c * DC;
#pragma unroll
                    for (int d = 0; d < DC; ++d) {
                        const double w = dl[d];
#pragma unroll
                        for (int q = 0; q < EPT; ++q) acc[q][d] = fma(vd[q], w, acc[q][d]);
                    }
                }
            };
            // full groups of PF moduli: straight-line code, so that the scalar constants of a
            // modulus can load while the previous one multiplies (measured faster from 16
            // digits per pass on with LDS columns; narrower passes and global columns, whose
            // constants come from the LDS slice, keep one guarded loop, which measured 2x
            // faster there at 4096^3 and p = 2048); the v ring runs PF moduli ahead
            constexpr bool SL = DC >= 16 && !GDIG;
            const int nfull = SL ? nlb - nlb % PF : 0;
            for (int lb = 0; lb < nfull; lb += PF) {
#pragma unroll
                for (int f = 0; f < PF; ++f) {
                    const int ll = lb + f;
                    int cur[EPT];
#pragma unroll
                    for (int q = 0; q < EPT; ++q) {
                        cur[q] = ring[f][q];
                        ring[f][q] = vp[q][(int64_t)(l0 + min(ll + PF, nlb - 1)) * v_ps];
                    }
                    modulus(ll, cur, inv_of(ll));
                }
            }
            if constexpr (SL) {
                for (int ll = nfull; ll < nlb; ++ll) {   // the last nlb % PF moduli
                    int cur[EPT];
#pragma unroll
                    for (int q = 0; q < EPT; ++q) cur[q] = vp[q][(int64_t)(l0 + ll) * v_ps];
                    modulus(ll, cur, inv_of(ll));
                }
            } else {
                for (int lb = 0; lb < nlb; lb += PF) {
#pragma unroll
                    for (int f = 0; f < PF; ++f) {
                        const int ll = lb + f;
                        if (ll >= nlb) break;
                        // 1/m is read before the next v load is issued: with global columns
                        // (1/m from LDS) the other order measured 1.4x slower at p = 2048
                        const double inv_m = inv_of(ll);
                        int cur[EPT];
#pragma unroll
                        for (int q = 0; q < EPT; ++q) {
                            cur[q] = ring[f][q];
                            ring[f][q] = vp[q][(int64_t)(l0 + min(ll + PF, nlb - 1)) * v_ps];
                        }
                        modulus(ll, cur, inv_m);
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            if (c == 0) {
                const double r = rint(asum[q]);
                slow[q] = fabs(asum[q] - r) > 0.5 - 0x1p-30;
                beta[q] = slow[q] ? (int64_t)floor(asum[q]) - 1 : (int64_t)r;   // alpha - 1 when slow
            }
            // digit k of S - beta P in binary64, exact: |acc| <= L 8095 2^31 < 2^53 - 2^46 for
            // L <= 512, |beta P_k| < 2^42 and the carry is below 2^22
            uint32_t *sd = col(q);
            double cy = (double)carry[q];
            const double bq = (double)beta[q];
#pragma unroll
            for (int d = 0; d < DC; ++d) {
                const int k = c * DC + d;
                if (k < nd32) {
                    const double x = fma(-bq, (double)Pd[k], acc[q][d] + cy);
                    const double hi = floor(x * 0x1p-32);
                    sd[k * cst] = (uint32_t)fma(-hi, 0x1p32, x);
                    cy = hi;
                }
            }
            carry[q] = (int64_t)cy;
        }
    }

#pragma unroll
    for (int q = 0; q < EPT; ++q)
        if (live[q]) crt_finish<ROUND>(a, idx[q], col(q), cst, slow[q], carry[q]);
}

template <int DC, int EPT, bool ROUND, bool WEIGHT, bool GDIG>
__global__ __launch_bounds__(256) void k_crt(CrtArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint32_t sdig[];
    crt_block<DC, EPT, ROUND, WEIGHT, GDIG>(a, blockIdx.x, sdig);
}

// Direct CRT on the matrix cores (digit columns in LDS: nd32 <= 32, L <= 127).  The
// digit sums S = sum_l v_l M_l are formed as the int8 product (byte rows of S) x
// (entries) of the tables of build_crt_mma_tables with each v_l's two bytes; one wave
// covers 64 consecutive entries as two 32-entry column blocks.
//   B fragments: lane (h, c) holds, per 32-byte step q, the words of moduli
//     16 q + 8 h .. + 7 of entries c and 32 + c, each xor 0x0080 (low byte - 128).
//   Output element 4 a + i of a 32 x 32 block is byte row 8 a + 4 h + i, i.e. byte i of
//     digit 2 a + h: a lane assembles four digit partials per block; one ds_bpermute
//     hand-over then gives lane (0, c) all digits of entry c and lane (1, c) all digits of
//     entry 32 + c, which it carries into its LDS column.
//   S / P is estimated from the top nt digits (error below 2^-40); the nearest integer
//   beta is exact unless the estimate lies within 2^-30 of a half-integer, else the
//   paper's alpha - 1 (at most two subtractions of P follow in crt_finish).  Then the
//   column receives S - beta P and crt_finish lifts and rounds as in k_crt.
constexpr int kCrtMmaMaxQ = 8;   // contraction steps of the matrix-core CRT (2 L + 1 <= 256)
// below this many digits (p <~ 180) the fp64 CRT is faster: the matrix-core kernel's
// per-entry carry and subtraction passes outweigh its L x nd32 multiply-adds
constexpr int kCrtMmaMinDigits = 16;

// WEIGHT = true: the planes hold plain residues u_l (any representative, |u_l| < m_l),
// weighted here to v_l = u_l (P/m_l)^-1 mod m_l (the stage-4 parity entry point).
template <int KQ, bool ROUND, bool WEIGHT = false>
__device__ __forceinline__ void crt_mma_block(const CrtArgs &a, int64_t blk, uint32_t *sdig) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int h = lane >> 5, c = lane & 31;
    const int nd32 = a.nd32, L = a.L, kq = a.kq, nbk = a.nbk;
    const int64_t N = a.N, MN = a.M * N, v_ps = a.v_ps;
    const int64_t e0 = blk * 256 + wv * 64;
    typedef const __attribute__((address_space(1))) uint16_t gu16;
    typedef const __attribute__((address_space(1))) v4i gv4i;
    typedef const __attribute__((address_space(4))) uint32_t cu32;

    // B fragments (a dead entry reads entry 0, always valid, and writes nothing).  Steps
    // with all 16 moduli present load unguarded (a lane base plus a wave-uniform offset);
    // the last step clamps the modulus and feeds 0 past L.
    v4i bf0[KQ], bf1[KQ];
    {
        gu16 *vb[2];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int64_t e = e0 + 32 * b + c, ee = e < MN ? e : 0;
            const int64_t i = ee / N, j = ee - i * N;
            vb[b] = (gu16 *)a.V + i * a.ldv + j + (int64_t)(8 * h) * v_ps;
        }
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
            if (q < kq) {
                const bool full = 16 * q + 16 <= L;   // wave-uniform
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    uint32_t w[8];
                    if (full) {
#pragma unroll
                        for (int t = 0; t < 8; ++t) w[t] = vb[b][(int64_t)(16 * q + t) * v_ps];
                    } else {
#pragma unroll
                        for (int t = 0; t < 8; ++t) {
                            const int l = 16 * q + 8 * h + t;
                            const int lc = min(l, L - 1) - 8 * h;   // relative to the lane base
                            const uint32_t x = vb[b][(int64_t)lc * v_ps];
                            w[t] = l < L ? x : 0u;
                        }
                    }
                    if constexpr (WEIGHT) {
#pragma unroll
                        for (int t = 0; t < 8; ++t) {
                            const int l = 16 * q + 8 * h + t;
                            if (l < L) {
                                const ModInfo info = load_info((OZ2H_G(ModInfo) *)a.mi + l);
                                const int32_t v = centred_mod((double)(int16_t)w[t] * (double)info.minv,
                                                              (double)info.m, info.inv_m);
                                w[t] = (uint32_t)(uint16_t)(int16_t)v;
                            }
                        }
                    }
                    const v4i f = v4i{(int)((w[0] | (w[1] << 16)) ^ 0x00800080u),
                                      (int)((w[2] | (w[3] << 16)) ^ 0x00800080u),
                                      (int)((w[4] | (w[5] << 16)) ^ 0x00800080u),
                                      (int)((w[6] | (w[7] << 16)) ^ 0x00800080u)};
                    if (b == 0) bf0[q] = f;
                    else bf1[q] = f;
                }
            }
        }
    }

    // S: eight digits per block of 32 byte rows, carried into this lane's LDS column
    gv4i *af = (gv4i *)a.afr + lane;
    uint32_t *col = sdig + tid;   // digit k at col[256 k]
    int64_t carry = 0;
    for (int nb = 0; nb < nbk; ++nb) {
        v16i acc0 = v16i{}, acc1 = v16i{};
#pragma unroll
        for (int q = 0; q < KQ; ++q)
            if (q < kq) {
                const v4i f = af[((size_t)nb * kq + q) * 64];
                acc0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(f, bf0[q], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(f, bf1[q], acc1, 0, 0, 0);
            }
        int64_t mine[4], got[4];
#pragma unroll
        for (int a4 = 0; a4 < 4; ++a4) {
            const int64_t d0 = (int64_t)acc0[4 * a4] + (int64_t)acc0[4 * a4 + 1] * 256 +
                               (int64_t)acc0[4 * a4 + 2] * 65536 + (int64_t)acc0[4 * a4 + 3] * 16777216;
            const int64_t d1 = (int64_t)acc1[4 * a4] + (int64_t)acc1[4 * a4 + 1] * 256 +
                               (int64_t)acc1[4 * a4 + 2] * 65536 + (int64_t)acc1[4 * a4 + 3] * 16777216;
            const int64_t send = h ? d0 : d1;   // the partner's entry
            mine[a4] = h ? d1 : d0;
            const int plo = __builtin_amdgcn_ds_bpermute((lane ^ 32) << 2, (int)(uint32_t)send);
            const int phi = __builtin_amdgcn_ds_bpermute((lane ^ 32) << 2, (int)(send >> 32));
            got[a4] = (int64_t)(((uint64_t)(uint32_t)phi << 32) | (uint32_t)plo);
        }
#pragma unroll
        for (int dk = 0; dk < 8; ++dk) {
            const int k = 8 * nb + dk;
            const int64_t D = (dk & 1) == h ? mine[dk >> 1] : got[dk >> 1];
            if (k < nd32) {
                const int64_t x = D + carry;
                col[256 * k] = (uint32_t)x;
                carry = x >> 32;
            }
        }
    }

    // beta from S / P, then S - beta P into the column
    double val = (double)(int32_t)col[256 * (nd32 - 1)];
    for (int k = nd32 - 2; k >= nd32 - a.nt; --k) val = val * 4294967296.0 + (double)col[256 * k];
    const double est = val * a.inv_ptop, r = rint(est);
    const bool slow = fabs(est - r) > 0.5 - 0x1p-30;
    const int64_t beta = slow ? (int64_t)floor(est) - 1 : (int64_t)r;
    cu32 *Pd = (cu32 *)a.Pd;
    int64_t cy = 0;
    for (int k = 0; k < nd32; ++k) {
        const int64_t x = (int64_t)col[256 * k] - beta * (int64_t)Pd[k] + cy;
        col[256 * k] = (uint32_t)x;
        cy = x >> 32;
    }
    const int64_t e = e0 + lane;
    if (e < MN) crt_finish<ROUND>(a, e, col, 256, slow, cy + carry);
}

template <int KQ, bool ROUND, bool WEIGHT>
__global__ __launch_bounds__(256) void k_crt_mma(CrtArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint32_t sdig[];
    crt_mma_block<KQ, ROUND, WEIGHT>(a, blockIdx.x, sdig);
}

// Direct CRT for wide moduli sets on the vector ALUs with row broadcasts (no MFMA), in two
// kernels.  S = sum_l v_l M_l, M_l = P / m_l in balanced base-2^32 digits D[d][l]: each digit
// sum S_d = sum_l v_l D[d][l] is an exact fp64 integer (|S_d| < L 2^44 < 2^53).
//   k_crt_row_sums: a wave takes 64 consecutive entries and one group of 16 digits.  Lane j
//     of row q owns digit 16 dg + j of the row's entries 16 q + i (i < 16) and keeps, per
//     chunk of 16 moduli, their 16 digit constants in registers; lane m of the row loads v of
//     modulus 16 c + m for the row's 16 entries, and each multiply-add takes v from lane m by
//     a DPP row broadcast.  The 16 sums of an entry then go through LDS to one lane, which
//     carries them into 16 digits in [0, 2^32) and a carry-out (digit-major in the
//     workspace: digit k of entry e at dig[k * estride + e]).  Blocks are one wave; the
//     digit groups of a tile run on one XCD (block b goes to XCD b mod 8), so that the tile's
//     v planes are read from HBM once and then from that XCD's L2.
//   k_crt_row_finish: one entry per thread: the groups' carry-outs are added in, S's nd32
//     digits land in an LDS column, and from there as in the matrix-core CRT: beta from the
//     top digits (the paper's alpha - 1 when the estimate is within 2^-30 of a half-integer),
//     S - beta P, and crt_finish (symmetric lift, one rounding).
struct CrtRowArgs {
    const int16_t *V;
    int64_t v_ps;       // plane stride of v; entry e' = i * ldv + j of a plane is at V + e'
    int64_t nent;       // entries e' covered: M * ldv
    int64_t ldv;
    int L, lpad, ndg, nd32;
    const double *drow;   // [16 ndg][lpad]
    const ModInfo *mi;    // WEIGHT: plain residues u_l, weighted here
    uint32_t *dig;        // [16 ndg][estride]
    int32_t *cout;        // [ndg][estride]
    int64_t estride;      // >= 64 * ntiles
    int ntiles;           // tiles of 64 entries (a multiple of 32: four per block, one block
                          // per XCD)
};

// 16 values as doubles, followed by the two wait states a DPP read of them needs
__device__ __forceinline__ void dpp_ready16(double (&x)[16]) {
    asm volatile("s_nop 1"
                 : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]),
                   "+v"(x[6]), "+v"(x[7]), "+v"(x[8]), "+v"(x[9]), "+v"(x[10]), "+v"(x[11]),
                   "+v"(x[12]), "+v"(x[13]), "+v"(x[14]), "+v"(x[15]));
}

// 16 x 16 multiply-adds: for each broadcast lane m (modulus 16 c + m), the 16 entries'
// accumulators in turn, so that consecutive multiply-adds are independent
template <int M = 0>
__device__ __forceinline__ void crt_row_fmas(double (&acc)[16], const double (&x)[16], const double (&c)[16]) {
    if constexpr (M < 16) {
#pragma unroll
        for (int i = 0; i < 16; ++i) fmac_rowbcast<M>(acc[i], x[i], c[M]);
        crt_row_fmas<M + 1>(acc, x, c);
    }
}

// The digit constants of the block's digit group are staged in LDS kCrtRowStage moduli at a
// time (row jj = digit 16 dg + jj), with a row stride = 2 mod 32 doubles, so that the 16 rows
// a ds_read_b128 of 16 lanes touches start on 16 different 4-bank groups.
constexpr int kCrtRowStage = 192;
constexpr int kCrtRowDStride = kCrtRowStage + 2;
constexpr int kCrtRowPairs = kCrtRowStage / 32;   // 16-byte pairs per thread and stage
static_assert(kCrtRowStage % 32 == 0 && kCrtRowDStride % 2 == 0, "stage rows of whole pairs");
constexpr size_t kCrtRowSumsLds = (size_t)16 * kCrtRowDStride * 8 + (size_t)4 * 32 * 17 * 8;

// blocks of four waves: four consecutive tiles of 64 entries, one digit group; block b runs
// on XCD b mod 8 and the digit groups of a tile quad go to one XCD.  Every wave takes part
// in the staging barriers; a wave past the last tile computes on tile 0 and stores nothing.
template <bool WEIGHT>
__global__ __launch_bounds__(256) void k_crt_row_sums(CrtRowArgs a) {
    extern __shared__ __attribute__((aligned(16))) double smem_crs[];
    double *Dl = smem_crs;   // [16][kCrtRowDStride]
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double *T = smem_crs + (size_t)16 * kCrtRowDStride + (size_t)wv * 32 * 17;   // transpose
    const uint32_t b = blockIdx.x, x8 = b & 7u, s = b >> 3;
    const int dg = (int)(s % (uint32_t)a.ndg);
    const int64_t tile0 = ((int64_t)(s / (uint32_t)a.ndg) * 8 + x8) * 4 + wv;
    const bool live = tile0 * 64 < a.nent;
    const int64_t tile = live ? tile0 : 0;
    const int q = lane >> 4, j = lane & 15;
    const int64_t e_row = tile * 64 + 16 * q;   // this row's entries e_row + i
    typedef const __attribute__((address_space(1))) v4i gv4i;
    typedef double d2 __attribute__((ext_vector_type(2)));
    const double *gsrc = a.drow + (size_t)16 * dg * a.lpad;
    double acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0;
    const int nch = a.lpad >> 4;
    // chunk c of 16 moduli: v of modulus min(16 c + j, L - 1) for the row's 16 entries (32
    // bytes; nent is a multiple of 64 and the launch checks that every plane holds nent
    // entries), loaded one chunk ahead; the 16 digit constants of this lane's digit from LDS
    // (zero past L)
    // plane addresses: the chunk's offset 16 c v_ps is wave-uniform (scalar arithmetic); a lane
    // past the last modulus reads the last plane
    const int16_t *vj = a.V + (int64_t)j * a.v_ps + e_row;
    const int16_t *vlast = a.V + (int64_t)(a.L - 1) * a.v_ps + e_row;
    auto loadv = [&](int c, v4i &w0, v4i &w1) {
        gv4i *src = (gv4i *)(16 * c + j < a.L ? vj + (int64_t)(16 * c) * a.v_ps : vlast);
        w0 = src[0];
        w1 = src[1];
    };
    auto mult = [&](int c, int l0, const v4i &w0, const v4i &w1) {
        const double *drow = Dl + j * kCrtRowDStride + (16 * c - l0);
        double dc[16];
#pragma unroll
        for (int m = 0; m < 16; m += 2) {
            const d2 t = *(const d2 *)(drow + m);
            dc[m] = t.x;
            dc[m + 1] = t.y;
        }
        double vd[16];
        const int raw[8] = {w0[0], w0[1], w0[2], w0[3], w1[0], w1[1], w1[2], w1[3]};
        ModInfo mi{};
        if constexpr (WEIGHT) mi = load_info((OZ2H_G(ModInfo) *)a.mi + min(16 * c + j, a.L - 1));
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int lo = (raw[t] << 16) >> 16, hi = raw[t] >> 16;
            if constexpr (WEIGHT) {
                vd[2 * t] = (double)centred_mod((double)lo * (double)mi.minv, (double)mi.m, mi.inv_m);
                vd[2 * t + 1] = (double)centred_mod((double)hi * (double)mi.minv, (double)mi.m, mi.inv_m);
            } else {
                vd[2 * t] = (double)lo;
                vd[2 * t + 1] = (double)hi;
            }
        }
        dpp_ready16(vd);
        crt_row_fmas(acc, vd, dc);
    };
    // a stage's constants: thread t moves pairs (t & 15) + 16 i of row t >> 4 (lpad and the
    // stage are multiples of 16, so a row of a stage is a whole number of 16-byte pairs); the
    // next stage's pairs load into registers while the current stage is multiplied
    const int srow = threadIdx.x >> 4, spair = threadIdx.x & 15;
    d2 pre[kCrtRowPairs];
    auto stage_load = [&](int l0) {
        const int nl = min(kCrtRowStage, a.lpad - l0);
        const double *src = gsrc + (size_t)srow * a.lpad + l0;
#pragma unroll
        for (int i = 0; i < kCrtRowPairs; ++i) {
            const int l = 2 * (spair + 16 * i);
            if (l < nl) pre[i] = *(const d2 *)(src + l);
        }
    };
    auto stage_store = [&](int l0) {
        const int nl = min(kCrtRowStage, a.lpad - l0);
        double *dst = Dl + srow * kCrtRowDStride;
#pragma unroll
        for (int i = 0; i < kCrtRowPairs; ++i) {
            const int l = 2 * (spair + 16 * i);
            if (l < nl) *(d2 *)(dst + l) = pre[i];
        }
    };
    v4i aw0, aw1, bw0, bw1;
    stage_load(0);
    loadv(0, aw0, aw1);
    for (int l0 = 0; l0 < a.lpad; l0 += kCrtRowStage) {
        const int nl = min(kCrtRowStage, a.lpad - l0);
        __syncthreads();   // the previous stage has been read by every wave
        stage_store(l0);
        if (l0 + kCrtRowStage < a.lpad) stage_load(l0 + kCrtRowStage);
        __syncthreads();
        const int c1 = (l0 + nl) >> 4;
        int c = l0 >> 4;
        for (; c + 2 <= c1; c += 2) {
            loadv(min(c + 1, nch - 1), bw0, bw1);
            mult(c, l0, aw0, aw1);
            loadv(min(c + 2, nch - 1), aw0, aw1);
            mult(c + 1, l0, bw0, bw1);
        }
        if (c < c1) {
            mult(c, l0, aw0, aw1);
            loadv(min(c + 1, nch - 1), aw0, aw1);
        }
    }
    // two halves of 32 entries: entry 16 q + i of the half's rows gets digit sum j at
    // T[(16 (q & 1) + i) * 17 + j]; lane 32 h + e then carries entry 32 h + e's 16 sums into
    // digits in [0, 2^32) and a carry-out
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        wave_lds_sync();
        if ((q >> 1) == h) {
#pragma unroll
            for (int i = 0; i < 16; ++i) T[(16 * (q & 1) + i) * 17 + j] = acc[i];
        }
        wave_lds_sync();
        if ((lane >> 5) == h) {
            const int el = lane & 31;
            const int64_t e = tile * 64 + lane;
            double cy = 0.0;
            uint32_t dv[16];
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) {
                const double xv = T[el * 17 + jj] + cy;
                cy = floor(xv * 0x1p-32);
                dv[jj] = (uint32_t)(xv - cy * 0x1p32);
            }
            if (live) {
#pragma unroll
                for (int jj = 0; jj < 16; ++jj) a.dig[(int64_t)(16 * dg + jj) * a.estride + e] = dv[jj];
                a.cout[(int64_t)dg * a.estride + e] = (int32_t)cy;
            }
        }
    }
}

// N columns of valid entries per row of ldv: entry e' = i * ldv + j, output (i, j) if j < N.
// beta comes first, from S's top digits: an exact carry pass over the top two digit groups
// (their digit sums and carry-outs) leaves out only the carry into them from the groups
// below, at most one unit at a digit 12 or more places below the top nt, far inside the
// 2^-30 margin of the half-integer test.  One carry pass from the bottom then forms
// c^ = S - beta P digit by digit in binary64 (every term an integer below 2^43: exact) and
// keeps its low nd32 digits in an LDS column, c^ in two's complement (|c^| < P/2, so the
// top digit is sign extension); on the paper's alpha - 1 path the column holds R in [0, 3P).
template <bool ROUND>
__global__ __launch_bounds__(64) void k_crt_row_finish(CrtArgs a, CrtRowArgs r) {
    extern __shared__ __attribute__((aligned(16))) uint32_t sdig[];
    const int tid = threadIdx.x;
    const int64_t ep = (int64_t)blockIdx.x * 64 + tid;
    const int64_t i = ep / r.ldv, jj = ep - i * r.ldv;
    if (ep >= r.nent || jj >= a.N) return;
    const int nd32 = a.nd32, nt = a.nt;
    uint32_t *col = sdig + tid;   // digit k at col[64 k]
    // groups holding digits below nd32 (at least three: this kernel runs for nd32 > 32)
    const int ng = min(r.ndg, (nd32 + 15) / 16);
    auto ldg = [&](int g, uint32_t (&dv)[16], int32_t &co) {
        const int gc = min(g, ng - 1);
#pragma unroll
        for (int u = 0; u < 16; ++u) dv[u] = r.dig[(int64_t)(16 * gc + u) * r.estride + ep];
        co = gc > 0 ? r.cout[(int64_t)(gc - 1) * r.estride + ep] : 0;
    };
    uint32_t da[16], db[16];
    int32_t ca, cb;

    // S's top nt digits (the highest as a signed digit) as one binary64 value
    ldg(ng - 2, da, ca);
    ldg(ng - 1, db, cb);
    double val = 0.0;
    {
        const int base = 16 * (ng - 2), kb = nd32 - nt;
        uint32_t top[32];
        int64_t cy = ca;
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            const int64_t x = (int64_t)(u < 16 ? da[u] : db[u - 16]) + (u == 16 ? (int64_t)cb : 0) + cy;
            top[u] = (uint32_t)x;
            cy = x >> 32;
        }
        // Horner from the signed top digit down: the sign-extension digits cancel exactly
#pragma unroll
        for (int u = 31; u >= 0; --u) {
            const int k = base + u;
            if (k == nd32 - 1) val = (double)(int32_t)top[u];
            else if (k >= kb && k < nd32) val = fma(val, 0x1p32, (double)top[u]);
        }
    }
    const double est = val * a.inv_ptop, rr = rint(est);
    const bool slow = fabs(est - rr) > 0.5 - 0x1p-30;
    const double beta = slow ? floor(est) - 1.0 : rr;   // |beta| <= L + 2

    // c^ = S - beta P from the bottom, the next group's digits loading during a group
    typedef const __attribute__((address_space(4))) uint32_t cu32;
    cu32 *Pd = (cu32 *)a.Pd;
    double cy = 0.0;
    auto digit = [&](int k, uint32_t d, double add, uint32_t pk) {
        const double x = fma(-beta, (double)pk, (double)d + add + cy);
        const double hi = floor(x * 0x1p-32);
        col[64 * k] = (uint32_t)fma(-hi, 0x1p32, x);
        cy = hi;
    };
    auto pass = [&](int g, const uint32_t (&dv)[16], int32_t co) {
        if (16 * g + 16 <= nd32) {   // a whole group: its 16 digits of P in one scalar load
            uint32_t pk[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) pk[u] = Pd[16 * g + u];
#pragma unroll
            for (int u = 0; u < 16; ++u) digit(16 * g + u, dv[u], u == 0 ? (double)co : 0.0, pk[u]);
        } else {
            for (int u = 0; u < 16 && 16 * g + u < nd32; ++u)
                digit(16 * g + u, dv[u], u == 0 ? (double)co : 0.0, Pd[16 * g + u]);
        }
    };
    ldg(0, da, ca);
    int g = 0;
    for (; g + 2 <= ng; g += 2) {
        ldg(g + 1, db, cb);
        pass(g, da, ca);
        ldg(g + 2, da, ca);
        pass(g + 1, db, cb);
    }
    if (g < ng) pass(g, da, ca);
    const int64_t sgn = !slow && (int32_t)col[64 * (nd32 - 1)] < 0 ? -1 : 0;
    crt_finish<ROUND>(a, i * a.N + jj, col, 64, slow, sgn);
}

// planes [G][R][C] (int8, row stride ldi) -> [G][Co][Ro] (row stride Ro), zero where
// the source row is out of range.  A block moves a 128 x 128 byte tile.  Thread t loads the
// 16-byte column chunk t % 8 of source rows 4 (t / 8) .. + 3 (four loads in flight), turns
// each 4 x 4 byte block into four dwords (one source column, four source rows each) and
// writes them to an LDS tile of output rows; the 16-byte chunks of an output row are stored
// XOR-swizzled by its column chunk, so that a dword write instruction touches 32 banks
// rather than 8.  Then 8 consecutive threads read one output row's eight chunks and store
// them as one 128-byte segment.  Requires ldi to be a multiple of 16 with C <= ldi (a chunk
// that starts below C stays in its row; its bytes past C, the planes' zero padding, land in
// output rows >= C) and Ro, Co multiples of 128 (the residue planes are padded to 128 and
// the GEMM tiles to 128 or 256).
__global__ __launch_bounds__(256) void k_plane_transpose(const int8_t *__restrict__ in, int64_t R,
                                                         int64_t C, int64_t ldi, int64_t ips,
                                                         int8_t *__restrict__ out, int64_t Ro,
                                                         int64_t Co, int64_t ops) {
    __shared__ __attribute__((aligned(16))) uint32_t tile[128 * 32];   // [output row][32 dwords]
    const int64_t g = blockIdx.z;
    const int64_t c0 = (int64_t)blockIdx.x * 128, r0 = (int64_t)blockIdx.y * 128;   // source tile
    const int t = threadIdx.x;
    {
        const int cc = t & 7, rg = t >> 3;   // column chunk, group of four source rows
        const int64_t c = c0 + 16 * cc;
        v4i x[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t r = r0 + 4 * rg + i;
            x[i] = v4i{0, 0, 0, 0};
            if (r < R && c < C) x[i] = *(const v4i *)(in + g * ips + r * ldi + c);
        }
        // dword of output row o = 16 cc + 4 q + j: byte j of each of the four rows' word q
        const int pc = 4 * ((rg >> 2) ^ cc) + (rg & 3);   // swizzled dword position in the row
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t d = (((uint32_t)x[0][q] >> (8 * j)) & 0xFFu) |
                                   ((((uint32_t)x[1][q] >> (8 * j)) & 0xFFu) << 8) |
                                   ((((uint32_t)x[2][q] >> (8 * j)) & 0xFFu) << 16) |
                                   ((((uint32_t)x[3][q] >> (8 * j)) & 0xFFu) << 24);
                tile[(16 * cc + 4 * q + j) * 32 + pc] = d;
            }
    }
    __syncthreads();
    const int qc = t & 7;   // logical chunk: output columns r0 + 16 qc .. + 15
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int o = (t >> 3) + 32 * i;   // output row c0 + o
        const v4i v = *(const v4i *)&tile[o * 32 + 4 * (qc ^ ((o >> 4) & 7))];
        *(v4i *)(out + g * ops + (c0 + o) * Ro + r0 + 16 * qc) = v;
    }
}

// zero output for K = 0
__global__ void k_zero_out(int8_t *__restrict__ s, int32_t *__restrict__ e,
                           uint64_t *__restrict__ limbs, int64_t M, int64_t N, int64_t ld, int nl) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * N) return;
    const int64_t i = idx / N, j = idx - i * N;
    const int64_t o = i * ld + j;
    s[o] = 0;
    e[o] = 0;
    for (int l = 0; l < nl; ++l) limbs[o * nl + l] = 0;
}

// ---------------------------------------------------------------- float64 carriers
// Element (r, c) of a carrier is CW = 2 + 2 nl doubles: [0] the value truncated
// to 53 bits, [1] 4 exp + sign + 1, [2 + 2l], [3 + 2l] the 32-bit halves of limb l.
// Every slot but [0] is an exactly representable integer, so the encoding
// survives any copy, view or device move of a floating tensor.

// the CW slots of element src of X into o
__device__ __forceinline__ void carrier_encode(int p, int nl, const int8_t *__restrict__ sign,
                                               const int32_t *__restrict__ exps,
                                               const uint64_t *__restrict__ limbs, int64_t src,
                                               double *o) {
    const int s = sign[src];
    const int e = s ? exps[src] : 0;
    const int top = p - 64 * (nl - 1);   // bits of the top limb, 1..64
    uint64_t hi = 0;                     // the 64 (or p, if fewer) leading bits of mant
    for (int l = 0; l < nl; ++l) {
        uint64_t x = s ? limbs[src * nl + l] : 0;
        if (l == nl - 1 && top < 64) x &= (~0ull) >> (64 - top);
        o[2 + 2 * l] = (double)(uint32_t)x;
        o[3 + 2 * l] = (double)(uint32_t)(x >> 32);
        if (l == nl - 1) {
            if (top == 64 || nl == 1) hi = x;
            else hi = (x << (64 - top)) | (limbs[src * nl + l - 1] >> top);
        }
    }
    const int hb = p < 64 ? p : 64;      // bits held in `hi`
    double approx = 0.0;
    if (s) {
        const uint64_t m53 = hb > 53 ? hi >> (hb - 53) : hi;
        const int mb = hb > 53 ? 53 : hb;
        approx = ldexp((double)m53, e - mb);
        if (s < 0) approx = -approx;
    }
    o[0] = approx;
    o[1] = 4.0 * (double)e + (double)(s + 1);
}

// STAGED: a block's elements are consecutive, so its part of the carrier is one contiguous
// run of blockDim.x * CW doubles; each thread writes its CW slots into LDS and the block then
// copies the run out with consecutive lanes on consecutive doubles (one thread per element
// writing its own slots directly puts lanes CW * 8 bytes apart).  Dynamic LDS:
// blockDim.x * CW doubles.
template <bool STAGED>
__global__ __launch_bounds__(256) void k_carrier_pack(int64_t rows, int64_t cols, int p, int nl,
                                                      const int8_t *__restrict__ sign,
                                                      const int32_t *__restrict__ exps,
                                                      const uint64_t *__restrict__ limbs,
                                                      int64_t ld, double *__restrict__ car) {
    extern __shared__ __attribute__((aligned(16))) double cstage[];
    const int64_t n = rows * cols, e0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t idx = e0 + threadIdx.x;
    const int cw = 2 + 2 * nl;
    if (idx < n) {
        const int64_t r = idx / cols, c = idx - r * cols;
        carrier_encode(p, nl, sign, exps, limbs, r * ld + c,
                       STAGED ? cstage + (size_t)threadIdx.x * cw : car + idx * cw);
    }
    if constexpr (STAGED) {
        __syncthreads();
        const int64_t total = (n - e0 < (int64_t)blockDim.x ? n - e0 : (int64_t)blockDim.x) * cw;
        double *dst = car + e0 * cw;
        for (int64_t i = threadIdx.x; i < total; i += blockDim.x) dst[i] = cstage[i];
    }
}

// bad (nullable) gets a 1 if any element is not a valid encoding; such an
// element is written as zero
// STAGED: the block first copies its contiguous run of the carrier into LDS (consecutive
// lanes on consecutive doubles), then each thread decodes its element from there.
template <bool STAGED>
__global__ __launch_bounds__(256) void k_carrier_unpack(int64_t rows, int64_t cols, int p, int nl,
                                                        const double *__restrict__ car,
                                                        int8_t *__restrict__ sign,
                                                        int32_t *__restrict__ exps,
                                                        uint64_t *__restrict__ limbs, int64_t ld,
                                                        int32_t *bad) {
    extern __shared__ __attribute__((aligned(16))) double cstage[];
    const int64_t n = rows * cols, e0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t idx = e0 + threadIdx.x;
    const int cw = 2 + 2 * nl;
    if constexpr (STAGED) {
        const int64_t total = (n - e0 < (int64_t)blockDim.x ? n - e0 : (int64_t)blockDim.x) * cw;
        const double *src = car + e0 * cw;
        for (int64_t i = threadIdx.x; i < total; i += blockDim.x) cstage[i] = src[i];
        __syncthreads();
    }
    // STAGED with ld == cols: the block's limbs are one contiguous run too; each thread puts
    // its limbs over its own (already read) LDS slots and the block stores the run together
    const bool dense = STAGED && ld == cols;
    if (!dense && idx >= n) return;
    if (idx < n) {
        const int64_t r = idx / cols, c = idx - r * cols, dst = r * ld + c;
        double *in = STAGED ? cstage + (size_t)threadIdx.x * cw : const_cast<double *>(car) + idx * cw;
        const double code = in[1];
        bool ok = code == rint(code) && fabs(code) < 0x1p33;
        const double q = floor(code * 0.25);
        const int s = ok ? (int)(code - 4.0 * q) - 1 : 0;
        const int64_t e = (int64_t)q;
        ok = ok && s <= 1 && e >= INT_MIN && e <= INT_MAX;
        const int top = p - 64 * (nl - 1);
        for (int l = 0; l < nl; ++l) {
            const double lo = in[2 + 2 * l], hi = in[3 + 2 * l];
            ok = ok && lo == rint(lo) && hi == rint(hi) && lo >= 0.0 && hi >= 0.0 &&
                 lo < 0x1p32 && hi < 0x1p32;
        }
        uint64_t topl = 0, any = 0;
        // dense: limb l goes over LDS slot l, kept as a double bit pattern (slot l was read
        // before: limb l reads slots 2 + 2l and 3 + 2l)
        auto put = [&](int l, uint64_t v) {
            if (dense) in[l] = __builtin_bit_cast(double, v);
            else limbs[dst * nl + l] = v;
        };
        for (int l = 0; l < nl; ++l) {
            const uint64_t x = ok ? ((uint64_t)(uint32_t)in[2 + 2 * l] |
                                     ((uint64_t)(uint32_t)in[3 + 2 * l] << 32)) : 0;
            if (l == nl - 1) topl = x;
            any |= x;
            put(l, s && ok ? x : 0);
        }
        // a nonzero value must be normalised (bit p - 1 set, nothing above it), a
        // zero must have zero limbs
        if (ok) ok = s ? (topl >> (top - 1)) == 1 : any == 0;
        if (!ok) {
            for (int l = 0; l < nl; ++l) put(l, 0);
            if (bad) *bad = 1;
        }
        sign[dst] = ok ? (int8_t)s : 0;
        exps[dst] = ok && s ? (int32_t)e : 0;
    }
    if (dense) {
        __syncthreads();
        const int64_t cnt = n - e0 < (int64_t)blockDim.x ? n - e0 : (int64_t)blockDim.x;
        uint64_t *out = limbs + e0 * nl;
        const int bd = blockDim.x, dt = bd / nl, dw = bd % nl;   // flat f = t nl + l advances by bd
        int t = (int)threadIdx.x / nl, l = (int)threadIdx.x - t * nl;
        for (int64_t f = threadIdx.x; f < cnt * nl; f += bd) {
            out[f] = __builtin_bit_cast(uint64_t, cstage[(size_t)t * cw + l]);
            t += dt;
            l += dw;
            if (l >= nl) {
                l -= nl;
                ++t;
            }
        }
    }
}

}  // namespace oz2h
