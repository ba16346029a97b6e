// oz2h_f64.hpp -- kernels of the binary64 backend (the paper's subsection "(b) binary64
// backend", Eq. fp64bound): residues of the integerized operands as exact binary64
// values, and their products on the fp64 matrix cores, which stay exact because every
// partial sum is an integer below 2^53.  The direct CRT and the rounding are the INT8
// backend's kernels, over CRT terms (two per binary64 modulus).
#pragma once

#include "oz2h_kernels.hpp"

namespace oz2h {

// ---------------------------------------------------------------- stage 2 (binary64)

// Residues of a^ for binary64 moduli.  One thread per entry (r, k); a block covers 128
// consecutive k of one row.  The (t+1)-bit integer is built once into an LDS column of
// 32-bit words (stride 128); the residue of its magnitude is then the sum over its 16-bit
// halves h_j of h_j c_j with c_j the centred 2^(16 j) mod m (|c_j| < 2^21, so each product
// is below 2^37 and the sum of at most 512 of them below 2^46: exact), reduced to
// |r| <= (m - 1)/2 by r = x - rint(x/m) m and one correction (the quotient may be off by
// one within 2^-26 of a half-integer).  Four moduli per pass share each word read.
// Output: planes [Lf][rpad][kpad] of doubles, sign applied; entries outside the operand 0.
struct ResF64Args {
    const uint64_t *limbs;
    const int32_t *exps;
    const int8_t *signs;
    int64_t rs, cs, rows, count, kpad, plane_stride;
    const int32_t *erow;
    int p, nl, t, nw32, Lf, fnh;
    const double *rw;       // [Lf][fnh]
    const F64Mod *mods;     // [Lf]
    double *planes;
};

constexpr int kResF64Block = 128;

__global__ __launch_bounds__(kResF64Block) void k_residues_f64(ResF64Args a) {
    extern __shared__ uint32_t fwords[];
    const int tid = threadIdx.x;
    const int64_t nkb = a.kpad / kResF64Block;
    const int64_t r = (int64_t)blockIdx.x / nkb;
    const int64_t k = ((int64_t)blockIdx.x - r * nkb) * kResF64Block + tid;
    int s = 0;
    int64_t sh = 0, idx = 0;
    if (r < a.rows && k < a.count) {
        idx = r * a.rs + k * a.cs;
        s = a.signs[idx];
        sh = (int64_t)a.t - a.p + a.exps[idx] - a.erow[r];
    }
    s = build_words((OZ2H_G(uint64_t) *)a.limbs + idx * a.nl, s, sh, a.p, a.nw32, fwords + tid,
                    kResF64Block);
    const double sg = s < 0 ? -1.0 : 1.0;
    typedef const __attribute__((address_space(1))) double gdouble;
    gdouble *rw = (gdouble *)a.rw;
    OZ2H_G(F64Mod) *mods = (OZ2H_G(F64Mod) *)a.mods;
    double *out = a.planes + r * a.kpad + k;
    for (int j0 = 0; j0 < a.Lf; j0 += 4) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        const int nj = min(4, a.Lf - j0);
        for (int q = 0; q < a.nw32; ++q) {
            const uint32_t x = fwords[q * kResF64Block + tid];
            const double lo = (double)(x & 0xFFFFu), hi = (double)(x >> 16);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (u < nj) {
                    gdouble *c = rw + (int64_t)(j0 + u) * a.fnh + 2 * q;
                    acc[u] = fma(lo, c[0], acc[u]);
                    acc[u] = fma(hi, c[1], acc[u]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (u < nj) {
                const double m = mods[j0 + u].m, im = mods[j0 + u].inv_m;
                double rr = fma(-rint(acc[u] * im), m, acc[u]);
                if (rr > 0.5 * m) rr -= m;
                else if (rr < -0.5 * m) rr += m;
                out[(int64_t)(j0 + u) * a.plane_stride] = sg * rr;
            }
        }
    }
}

// ---------------------------------------------------------------- stage 3 (binary64)

// The binary64 residue GEMMs C^(j) = A^(j) B^(j)^T (planes [Lf][rows][kpad], k contiguous)
// on v_mfma_f64_16x16x4f64: exact, since |sum_k a b| <= K ((m - 1)/2)^2 < 2^53 bounds every
// partial sum too.  A block computes a 128 x 128 tile of one modulus; four waves in 2 x 2,
// each 64 x 64 as 4 x 4 MFMA tiles.  k-tiles of 16 doubles go global -> registers -> LDS
// (two stages, the next tile's loads in flight during the current tile's MFMAs).  LDS rows
// are 18 doubles apart (16-byte aligned stores; a fragment read of 16 rows at one k hits 16
// distinct bank pairs).
// Epilogue: u = c mod m in [0, m), v = u (P/m)^-1 mod m (products below 2^44: exact), stored
// as the two CRT terms v mod 2^11 and floor(v / 2^11) (int16 planes t0 + 2 j, t0 + 2 j + 1).
// MFMA lane layout (16 x 16 x 4, measured): A row lane % 16 at k = lane / 16; B column
// lane % 16 at k = lane / 16; result column lane % 16, row 4 i + lane / 16 in register i.
// Two waves per SIMD (at most 256 registers; left free the compiler takes 300, one wave):
// 44.7 against 30.2 TFLOP/s at 4096^3.
struct DgemmArgs {
    const double *A, *B;
    int64_t kpad, a_ps, b_ps;
    const F64Mod *mods;
    int16_t *V;
    int64_t v_ps, ldv;
    int t0;
};

constexpr int kDgemmBK = 16;    // k-tile (doubles)
constexpr int kDgemmLdsPitch = kDgemmBK + 2;

typedef double v4d __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_dgemm_res(DgemmArgs a) {
    __shared__ __attribute__((aligned(16))) double sA[2][128 * kDgemmLdsPitch];
    __shared__ __attribute__((aligned(16))) double sB[2][128 * kDgemmLdsPitch];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave >> 1, wc = wave & 1;
    const int j = blockIdx.z;
    const int64_t m0 = (int64_t)blockIdx.y * 128, n0 = (int64_t)blockIdx.x * 128;
    const double *A = a.A + (int64_t)j * a.a_ps + m0 * a.kpad;
    const double *B = a.B + (int64_t)j * a.b_ps + n0 * a.kpad;
    const int nk = (int)(a.kpad / kDgemmBK);

    // this thread's share of a k-tile: row tid / 2, doubles 8 (tid % 2) .. + 7, of A and of B
    const int lrow = tid >> 1, lcol = 8 * (tid & 1);
    const double *ga = A + (int64_t)lrow * a.kpad + lcol;
    const double *gb = B + (int64_t)lrow * a.kpad + lcol;
    double2 ra[4], rb[4];
    auto gload = [&](int kt) {
        const int64_t o = (int64_t)kt * kDgemmBK;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            ra[i] = *(const double2 *)(ga + o + 2 * i);
            rb[i] = *(const double2 *)(gb + o + 2 * i);
        }
    };
    auto lstore = [&](int st) {
        double *da = sA[st] + lrow * kDgemmLdsPitch + lcol;
        double *db = sB[st] + lrow * kDgemmLdsPitch + lcol;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            *(double2 *)(da + 2 * i) = ra[i];
            *(double2 *)(db + 2 * i) = rb[i];
        }
    };

    v4d acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = v4d{0.0, 0.0, 0.0, 0.0};

    const int fr = lane & 15, fk = lane >> 4;
    gload(0);
    lstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int st = kt & 1;
        if (kt + 1 < nk) gload(kt + 1);
        const double *cA = sA[st] + (wr * 64 + fr) * kDgemmLdsPitch + fk;
        const double *cB = sB[st] + (wc * 64 + fr) * kDgemmLdsPitch + fk;
#pragma unroll
        for (int ks = 0; ks < kDgemmBK / 4; ++ks) {
            double fa[4], fb[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) fa[x] = cA[x * 16 * kDgemmLdsPitch + 4 * ks];
#pragma unroll
            for (int y = 0; y < 4; ++y) fb[y] = cB[y * 16 * kDgemmLdsPitch + 4 * ks];
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[x], fb[y], acc[x][y], 0, 0, 0);
        }
        if (kt + 1 < nk) lstore(st ^ 1);
        __syncthreads();
    }

    const F64Mod fm = a.mods[j];
    const double m = fm.m, im = fm.inv_m, minv = fm.minv;
    int16_t *vlo = a.V + (int64_t)(a.t0 + 2 * j) * a.v_ps;
    int16_t *vhi = vlo + a.v_ps;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const double c = acc[x][y][i];
                double u = fma(-rint(c * im), m, c);   // exact: the result is a small integer
                if (u < 0.0) u += m;
                if (u < 0.0) u += m;
                if (u >= m) u -= m;
                double v = u * minv;                   // < 2^44
                v = fma(-rint(v * im), m, v);
                if (v < 0.0) v += m;
                if (v >= m) v -= m;
                const int iv = (int)v;
                const int64_t o = (m0 + wr * 64 + x * 16 + 4 * i + fk) * a.ldv + n0 + wc * 64 + y * 16 + fr;
                vlo[o] = (int16_t)(iv & ((1 << kF64Split) - 1));
                vhi[o] = (int16_t)(iv >> kF64Split);
            }
}

}  // namespace oz2h
