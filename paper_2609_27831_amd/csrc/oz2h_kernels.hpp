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

#include "oz2h_plan.hpp"

namespace oz2h {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------- stage 1

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// rows whose entries are contiguous along the contraction (cs == 1): one wave
// per (row, 4096-entry chunk), lanes stride 1, partial maxima combined by atomicMax
__global__ __launch_bounds__(256) void k_exp_kcontig(const int8_t *__restrict__ sign,
                                                     const int32_t *__restrict__ exps,
                                                     int64_t rows, int64_t count, int64_t rs,
                                                     int32_t *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= rows) return;
    const int64_t k0 = (int64_t)blockIdx.y * 4096;
    const int64_t k1 = min(count, k0 + 4096);
    int m = INT_MIN;
    for (int64_t k = k0 + lane; k < k1; k += 64) {
        const int64_t idx = r * rs + k;
        if (sign[idx]) m = max(m, exps[idx]);
    }
    for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off));
    if (lane == 0 && m != INT_MIN) atomicMax(out + r, m);
}

// any other layout: one thread per row, 64 entries of the contraction per block row
__global__ __launch_bounds__(256) void k_exp_generic(const int8_t *__restrict__ sign,
                                                     const int32_t *__restrict__ exps,
                                                     int64_t rows, int64_t count, int64_t rs,
                                                     int64_t cs, int32_t *__restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= rows) return;
    const int64_t k0 = (int64_t)blockIdx.y * 64;
    const int64_t k1 = min(count, k0 + 64);
    int m = INT_MIN;
    for (int64_t k = k0; k < k1; ++k) {
        const int64_t idx = r * rs + k * cs;
        if (sign[idx]) m = max(m, exps[idx]);
    }
    if (m != INT_MIN) atomicMax(out + r, m);
}

// all-zero rows get exponent 0
__global__ void k_exp_fix(int32_t *__restrict__ p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && p[i] == INT_MIN) p[i] = 0;
}

// ---------------------------------------------------------------- stage 2

__device__ __forceinline__ uint64_t mant_limb(const uint64_t *__restrict__ base, int nl,
                                              uint64_t topmask, int64_t i) {
    if (i < 0 || i >= nl) return 0;
    const uint64_t v = base[i];
    return i == nl - 1 ? (v & topmask) : v;
}

// bits [off, off + 32) of the significand (bits outside [0, p) read as 0)
__device__ __forceinline__ uint32_t mant_bits32(const uint64_t *__restrict__ base, int nl,
                                                uint64_t topmask, int64_t off) {
    const int64_t q = off >> 6;
    const int r = (int)(off & 63);
    const uint64_t lo = mant_limb(base, nl, topmask, q);
    const uint64_t hi = mant_limb(base, nl, topmask, q + 1);
    return (uint32_t)(r ? ((lo >> r) | (hi << (64 - r))) : lo);
}

__device__ __forceinline__ int mant_bit(const uint64_t *__restrict__ base, int nl,
                                        uint64_t topmask, int64_t pos) {
    if (pos < 0) return 0;
    return (int)((mant_limb(base, nl, topmask, pos >> 6) >> (pos & 63)) & 1u);
}

// any bit set in [0, pos)
__device__ __forceinline__ int mant_any_below(const uint64_t *__restrict__ base, int nl,
                                              uint64_t topmask, int64_t pos) {
    if (pos <= 0) return 0;
    const int64_t full = pos >> 6;
    const int r = (int)(pos & 63);
    for (int64_t i = 0; i < full && i < nl; ++i)
        if (mant_limb(base, nl, topmask, i)) return 1;
    if (r && full < nl && (mant_limb(base, nl, topmask, full) & ((1ull << r) - 1))) return 1;
    return 0;
}

// One thread per entry (r, k) of a rows x count operand side; a block covers 64
// consecutive k of RB rows, so the int8 plane stores of a wave are 64
// contiguous bytes.  The (t+1)-bit integer a^ is built once per entry into a
// per-thread LDS column of 32-bit words; the moduli are then swept in groups
// of 8 with fp64 FMAs against centred 2^(32w) mod m weights (exact: every
// partial sum stays below 2^53), one rint-based reduction per modulus.
template <int RB>
__global__ __launch_bounds__(64 * RB) void k_residues(
    const uint64_t *__restrict__ limbs, const int32_t *__restrict__ exps,
    const int8_t *__restrict__ signs, int64_t rs, int64_t cs, int64_t rows, int64_t count,
    int64_t kpad, int64_t plane_stride, const int32_t *__restrict__ erow, int p, int nl, int t,
    int nw32, const double *__restrict__ tab, const ModInfo *__restrict__ mi, int L,
    int lgroups, int8_t *__restrict__ planes) {
    extern __shared__ uint32_t words[];
    constexpr int BD = 64 * RB;
    const int tid = threadIdx.x;
    const int64_t k = (int64_t)blockIdx.x * 64 + (tid & 63);
    const int64_t r = (int64_t)blockIdx.y * RB + (tid >> 6);

    int s = 0;
    if (r < rows && k < count) {
        const int64_t idx = r * rs + k * cs;
        s = signs[idx];
        if (s != 0) {
            const uint64_t *base = limbs + idx * nl;
            const int topbits = p - 64 * (nl - 1);
            const uint64_t topmask = topbits >= 64 ? ~0ull : ((1ull << topbits) - 1);
            // a * 2^(t - e) = sign * mant * 2^sh, sh <= t - p  (Eq. 1)
            const int64_t sh = (int64_t)t - p + exps[idx] - erow[r];
            if (sh >= 0) {
                for (int w = 0; w < nw32; ++w)
                    words[w * BD + tid] = mant_bits32(base, nl, topmask, 32 * (int64_t)w - sh);
            } else {
                const int64_t rsh = -sh;   // round to nearest even on the dropped bits
                uint32_t nz = 0;
                for (int w = 0; w < nw32; ++w) {
                    const uint32_t v = mant_bits32(base, nl, topmask, 32 * (int64_t)w + rsh);
                    words[w * BD + tid] = v;
                    nz |= v;
                }
                const int rb = mant_bit(base, nl, topmask, rsh - 1);
                if (rb) {
                    const int st = mant_any_below(base, nl, topmask, rsh - 1);
                    if (st || (words[tid] & 1u)) {
                        for (int w = 0; w < nw32; ++w) {
                            const uint32_t v = words[w * BD + tid] + 1u;
                            words[w * BD + tid] = v;
                            if (v) break;
                        }
                        nz = 1;
                    }
                }
                if (!nz) s = 0;
            }
        }
    }
    if (s == 0)
        for (int w = 0; w < nw32; ++w) words[w * BD + tid] = 0;

    int8_t *out = planes + r * kpad + k;
    for (int grp = 0; grp < lgroups; ++grp) {
        double acc[kModGroup];
#pragma unroll
        for (int g = 0; g < kModGroup; ++g) acc[g] = 0.0;
        const double *c = tab + (size_t)grp * nw32 * kModGroup;
        for (int w = 0; w < nw32; ++w) {
            const double x = (double)words[w * BD + tid];
#pragma unroll
            for (int g = 0; g < kModGroup; ++g) acc[g] = fma(x, c[w * kModGroup + g], acc[g]);
        }
#pragma unroll
        for (int g = 0; g < kModGroup; ++g) {
            const int l = grp * kModGroup + g;
            if (l >= L) break;
            const ModInfo info = mi[l];
            const double a = s < 0 ? -acc[g] : acc[g];
            const double md = (double)info.m;
            const double q = rint(a * info.inv_m);
            int ri = (int)fma(-q, md, a);
            const int hi = (int)((info.m - 1) >> 1), lo = -(int)(info.m >> 1);
            if (ri > hi) ri -= (int)info.m;
            else if (ri < lo) ri += (int)info.m;
            int8_t *o = out + (int64_t)info.g0 * plane_stride;
            if (info.nprod == 1) {
                o[0] = (int8_t)ri;
            } else {
                const int r0 = ((ri + 64) & 127) - 64;   // balanced base-128 split
                const int r1 = (ri - r0) >> 7;
                o[0] = (int8_t)r0;
                o[plane_stride] = (int8_t)r1;
                o[2 * plane_stride] = (int8_t)(r0 + r1);
            }
        }
    }
}

// ---------------------------------------------------------------- stage 3

constexpr int GBM = 128, GBN = 128, GBK = 64, GLDS = 80;   // 80-byte LDS rows: conflict-free b128 reads

// u = (coef * acc + part) mod m in [0, m); |coef * acc + part| < 2^45 is exact in fp64
__device__ __forceinline__ int32_t fold_mod(int32_t acc, double coef, int32_t part, double md,
                                            double inv_m) {
    const double y = fma(coef, (double)acc, (double)part);
    const double q = floor(y * inv_m);
    int32_t r = (int32_t)fma(-q, md, y);
    const int32_t m = (int32_t)md;
    if (r < 0) r += m;
    else if (r >= m) r -= m;
    return r;
}

// One 128x128 output tile of one modulus per block; four waves in 2x2, each
// a 64x64 sub-tile of 2x2 v_mfma_i32_32x32x32_i8 blocks.  A/B k-tiles of 64
// bytes are staged through double-buffered LDS.  For a two-limb modulus the
// three Karatsuba products run one after another and are folded into a
// per-element residue: sum r_a r_b = -127 P0 + 128 Ps + 16256 P2.
// RAW = true: plain int32 output of a single plane (exactness tests).
template <bool RAW>
__global__ __launch_bounds__(256) void k_resgemm(const int8_t *__restrict__ A,
                                                 const int8_t *__restrict__ B, int64_t kpad,
                                                 int64_t a_ps, int64_t b_ps,
                                                 const ModInfo *__restrict__ mi,
                                                 uint16_t *__restrict__ U, int64_t u_ps,
                                                 int64_t ldu, int32_t *__restrict__ Craw) {
    __shared__ __attribute__((aligned(16))) int8_t sA[2][GBM * GLDS];
    __shared__ __attribute__((aligned(16))) int8_t sB[2][GBN * GLDS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int64_t m0 = (int64_t)blockIdx.y * GBM, n0 = (int64_t)blockIdx.x * GBN;

    uint32_t g0 = 0, nprod = 1;
    double md = 1.0, inv_m = 1.0;
    if (!RAW) {
        const ModInfo info = mi[blockIdx.z];
        g0 = info.g0;
        nprod = info.nprod;
        md = (double)info.m;
        inv_m = info.inv_m;
    }

    int32_t part[2][2][16];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 16; ++e) part[a][b][e] = 0;

    const int ldrow = tid >> 2, ldchunk = (tid & 3) * 16;   // global->LDS: 4 lanes per 64-byte row
    const int nk = (int)(kpad / GBK);

    for (uint32_t prod = 0; prod < nprod; ++prod) {
        const int8_t *Ag = A + (int64_t)(g0 + prod) * a_ps + m0 * kpad;
        const int8_t *Bg = B + (int64_t)(g0 + prod) * b_ps + n0 * kpad;
        v16i acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = v16i{};

        v4i ga0, ga1, gb0, gb1;
        auto gload = [&](int kt) {
            const int64_t ko = (int64_t)kt * GBK + ldchunk;
            ga0 = *(const v4i *)(Ag + (int64_t)ldrow * kpad + ko);
            ga1 = *(const v4i *)(Ag + (int64_t)(ldrow + 64) * kpad + ko);
            gb0 = *(const v4i *)(Bg + (int64_t)ldrow * kpad + ko);
            gb1 = *(const v4i *)(Bg + (int64_t)(ldrow + 64) * kpad + ko);
        };
        auto sstore = [&](int buf) {
            *(v4i *)(&sA[buf][ldrow * GLDS + ldchunk]) = ga0;
            *(v4i *)(&sA[buf][(ldrow + 64) * GLDS + ldchunk]) = ga1;
            *(v4i *)(&sB[buf][ldrow * GLDS + ldchunk]) = gb0;
            *(v4i *)(&sB[buf][(ldrow + 64) * GLDS + ldchunk]) = gb1;
        };

        gload(0);
        sstore(0);
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            const int cur = kt & 1;
            if (kt + 1 < nk) gload(kt + 1);
#pragma unroll
            for (int kh = 0; kh < 2; ++kh) {
                v4i fa[2], fb[2];
                const int koff = kh * 32 + (lane >> 5) * 16;
#pragma unroll
                for (int x = 0; x < 2; ++x) {
                    fa[x] = *(const v4i *)(&sA[cur][(wr * 64 + x * 32 + (lane & 31)) * GLDS + koff]);
                    fb[x] = *(const v4i *)(&sB[cur][(wc * 64 + x * 32 + (lane & 31)) * GLDS + koff]);
                }
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a], fb[b], acc[a][b],
                                                                          0, 0, 0);
            }
            if (kt + 1 < nk) sstore(cur ^ 1);
            __syncthreads();
        }

        if (RAW) {
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        const int64_t row =
                            m0 + wr * 64 + a * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                        const int64_t col = n0 + wc * 64 + b * 32 + (lane & 31);
                        Craw[row * ldu + col] = acc[a][b][e];
                    }
            return;
        }
        // planes are (r0, r1, r0 + r1): products P0, P2, Ps in that order
        const double coef = nprod == 1 ? 1.0 : (prod == 0 ? -127.0 : (prod == 1 ? 16256.0 : 128.0));
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    part[a][b][e] = fold_mod(acc[a][b][e], coef, part[a][b][e], md, inv_m);
    }

    uint16_t *Ul = U + (int64_t)blockIdx.z * u_ps;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int64_t row = m0 + wr * 64 + a * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                const int64_t col = n0 + wc * 64 + b * 32 + (lane & 31);
                Ul[row * ldu + col] = (uint16_t)part[a][b][e];
            }
}

// ---------------------------------------------------------------- stage 4 + 5

// bits [pos, pos + 32) of a digit column in LDS (bits outside [0, 32 nd) read as 0)
__device__ __forceinline__ uint32_t dig_bits32(const uint32_t *__restrict__ sd, int bd, int nd,
                                               int64_t pos) {
    const int64_t q = pos >> 5;
    const int r = (int)(pos & 31);
    const uint64_t lo = (q >= 0 && q < nd) ? sd[q * bd] : 0u;
    const uint64_t hi = (q + 1 >= 0 && q + 1 < nd) ? sd[(q + 1) * bd] : 0u;
    return (uint32_t)(((hi << 32) | lo) >> r);
}

// One thread per output entry.  Pass c accumulates digits [c*DC, (c+1)*DC) of
// S = sum_l v_l M_l over all moduli (centred v_l, balanced digits of M_l, so
// each column sum is an exact fp64 integer), pass 0 also forms alpha =
// floor(sum v_l / m_l) in binary64; R = S - (alpha - 1) P is carried into
// 32-bit digits in an LDS column.  Then at most two subtractions of P give x0,
// the lift compares with floor(P/2), and (ROUND) the magnitude is rounded once
// to p bits with its scale 2^(e_i + f_j - 2t).
template <int DC, bool ROUND>
__global__ void k_crt(const uint16_t *__restrict__ U, int64_t u_ps, int64_t ldu, int64_t M,
                      int64_t N, const ModInfo *__restrict__ mi, int L,
                      const double *__restrict__ dig, int ndpad, int nc, int nd32,
                      const uint32_t *__restrict__ Pd, const uint32_t *__restrict__ Phd,
                      const int32_t *__restrict__ erow, const int32_t *__restrict__ fcol, int t,
                      int p, int8_t *__restrict__ osign, int32_t *__restrict__ oexp,
                      uint64_t *__restrict__ olimbs, int64_t ldc, uint64_t *__restrict__ chat_mag,
                      int nlc) {
    extern __shared__ uint32_t sdig[];
    const int tid = threadIdx.x, bd = blockDim.x;
    const int64_t idx = (int64_t)blockIdx.x * bd + tid;
    if (idx >= M * N) return;
    const int64_t i = idx / N, j = idx - i * N;
    const uint16_t *up = U + i * ldu + j;
    uint32_t *sd = sdig + tid;

    int64_t beta = 0, carry = 0;
    for (int c = 0; c < nc; ++c) {
        double acc[DC];
#pragma unroll
        for (int d = 0; d < DC; ++d) acc[d] = 0.0;
        double asum = 0.0;
        const double *dc = dig + c * DC;
        for (int l = 0; l < L; ++l) {
            const ModInfo info = mi[l];
            const uint32_t x = (uint32_t)up[(int64_t)l * u_ps] * info.minv;   // < 2^28
            const double xd = (double)x, md = (double)info.m;
            const double q = floor(xd * info.inv_m);
            int v = (int)fma(-q, md, xd);
            if (v < 0) v += (int)info.m;
            else if (v >= (int)info.m) v -= (int)info.m;
            if (v > (int)((info.m - 1) >> 1)) v -= (int)info.m;   // centred v_l
            const double vd = (double)v;
            if (c == 0) asum = fma(vd, info.inv_m, asum);
            const double *dl = dc + (size_t)l * ndpad;
#pragma unroll
            for (int d = 0; d < DC; ++d) acc[d] = fma(vd, dl[d], acc[d]);
        }
        if (c == 0) beta = (int64_t)floor(asum) - 1;   // alpha - 1
#pragma unroll
        for (int d = 0; d < DC; ++d) {
            const int k = c * DC + d;
            if (k < nd32) {
                const int64_t x = (int64_t)acc[d] - beta * (int64_t)Pd[k] + carry;
                sd[k * bd] = (uint32_t)x;
                carry = x >> 32;
            }
        }
    }

    // R in [0, 3P): at most two subtractions of P
    for (int rep = 0; rep < 2; ++rep) {
        int64_t br = 0;
        for (int k = 0; k < nd32; ++k) {
            const int64_t d = (int64_t)sd[k * bd] - (int64_t)Pd[k] - br;
            br = d < 0;
        }
        if (br) break;
        br = 0;
        for (int k = 0; k < nd32; ++k) {
            const int64_t d = (int64_t)sd[k * bd] - (int64_t)Pd[k] - br;
            sd[k * bd] = (uint32_t)d;
            br = d < 0;
        }
    }
    // symmetric lift: x0 > floor(P/2) means c^ = x0 - P < 0
    int64_t br = 0;
    for (int k = 0; k < nd32; ++k) {
        const int64_t d = (int64_t)Phd[k] - (int64_t)sd[k * bd] - br;
        br = d < 0;
    }
    const bool neg = br != 0;
    if (neg) {
        br = 0;
        for (int k = 0; k < nd32; ++k) {
            const int64_t d = (int64_t)Pd[k] - (int64_t)sd[k * bd] - br;
            sd[k * bd] = (uint32_t)d;
            br = d < 0;
        }
    }
    int top = nd32 - 1;
    while (top >= 0 && sd[top * bd] == 0) --top;

    if (!ROUND) {
        uint64_t *o = chat_mag + idx * nlc;
        for (int l = 0; l < nlc; ++l) {
            const uint64_t lo = (2 * l < nd32) ? sd[2 * l * bd] : 0u;
            const uint64_t hi = (2 * l + 1 < nd32) ? sd[(2 * l + 1) * bd] : 0u;
            o[l] = lo | (hi << 32);
        }
        osign[idx] = top < 0 ? 0 : (neg ? -1 : 1);
        return;
    }

    const int nl = (p + 63) / 64;
    const int64_t oi = i * ldc + j;
    uint64_t *o = olimbs + oi * nl;
    if (top < 0) {
        for (int l = 0; l < nl; ++l) o[l] = 0;
        osign[oi] = 0;
        oexp[oi] = 0;
        return;
    }
    int64_t nb = 32 * (int64_t)top + (32 - __builtin_clz(sd[top * bd]));
    const int64_t sh = nb - p;   // mant = RNE(mag / 2^sh)
    bool inc = false;
    if (sh > 0) {
        const int64_t rpos = sh - 1;
        const int rb = (int)((sd[(rpos >> 5) * bd] >> (rpos & 31)) & 1u);
        if (rb) {
            bool st = false;
            const int64_t full = rpos >> 5;
            for (int64_t k = 0; k < full && !st; ++k) st = sd[k * bd] != 0;
            const int rr = (int)(rpos & 31);
            if (!st && rr) st = (sd[full * bd] & ((1u << rr) - 1)) != 0;
            const uint32_t lsb = dig_bits32(sd, bd, nd32, sh) & 1u;
            inc = st || lsb;
        }
    }
    bool allones = inc;
    if (inc) {   // mant = 2^p - 1 rounds up to 2^p: renormalise
        for (int l = 0; l < nl && allones; ++l) {
            const uint64_t v = (uint64_t)dig_bits32(sd, bd, nd32, 64 * (int64_t)l + sh) |
                               ((uint64_t)dig_bits32(sd, bd, nd32, 64 * (int64_t)l + 32 + sh) << 32);
            const int bits = (l == nl - 1) ? p - 64 * (nl - 1) : 64;
            const uint64_t mask = bits >= 64 ? ~0ull : ((1ull << bits) - 1);
            allones = v == mask;
        }
    }
    if (allones) {
        for (int l = 0; l < nl; ++l) o[l] = 0;
        o[(p - 1) >> 6] = 1ull << ((p - 1) & 63);
        nb += 1;
    } else {
        bool cy = inc;
        for (int l = 0; l < nl; ++l) {
            uint64_t v = (uint64_t)dig_bits32(sd, bd, nd32, 64 * (int64_t)l + sh) |
                         ((uint64_t)dig_bits32(sd, bd, nd32, 64 * (int64_t)l + 32 + sh) << 32);
            if (cy) {
                v += 1;
                cy = v == 0;
            }
            o[l] = v;
        }
    }
    osign[oi] = neg ? -1 : 1;
    oexp[oi] = (int32_t)(nb + (int64_t)erow[i] + fcol[j] - 2 * (int64_t)t);
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

}  // namespace oz2h
