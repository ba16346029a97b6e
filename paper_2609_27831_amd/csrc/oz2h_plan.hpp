// oz2h_plan.hpp -- host-side plan of the Ozaki-II pipeline: the moduli set and
// every constant table the kernels read.  Pure host C++ (no HIP calls).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace oz2h {

constexpr int kModGroup = 8;          // moduli per group in the residue kernel (small L)
constexpr int kModGroupWide = 16;     // ... and for wide moduli sets (L >= kWideL)
constexpr int kWideL = 96;
constexpr int kResMmaMinWords = 8;    // with the matrix-core residue variant selected, integers
                                      // of >= this many 32-bit words (t >= 224) take it, narrower
                                      // ones the fp64 kernel
constexpr int kResRowMinWords = 32;  // VALU residues: integers of >= this many words (t >= 992)
constexpr int kResRegWords = 12;     // VALU residues: integers of <= this many words stay in registers
                                      // take the row-broadcast kernel (faster from about there
                                      // on at 4096^2), narrower ones the entry-per-thread kernel
constexpr int kCrtRowMinDigits = 32;  // CRTs of more digits take the row-broadcast kernels
constexpr int kMaxModuli = 512;       // fp64-exact CRT digit sums need L * 2^44 < 2^53
constexpr int kMaxWords = 256;        // fp64-exact residue sums need nw32 * 2^45 < 2^53
constexpr int64_t kMaxK = 133000;     // K * 127^2 < 2^31, the cap the paper's implementation uses
constexpr uint32_t kOneLimbMax = 255;    // centred residue fits int8
constexpr uint32_t kTwoLimbMax = 16191;  // balanced base-128 halves fit int8 (and their sum)

// Per-modulus record read by the kernels (40 bytes, 8-byte aligned).
struct ModInfo {
    uint32_t m;      // the modulus
    uint32_t g0;     // its first INT8 plane
    uint32_t nprod;  // 1 for a one-limb modulus, 3 for a two-limb modulus (Karatsuba)
    uint32_t minv;   // (P / m)^-1 mod m, the direct-CRT weight
    double inv_m;    // fl(1/m)
    int32_t kc[3];   // centred in-place fold factors of the GEMM accumulator after
                     // each product: minv (one-limb), or w0, w1, w2 (two-limb, k_resgemm)
    int32_t pad;
};

// One group of up to kModGroupWide moduli as the residue kernel reads it
// (wave-uniform scalar loads, 384 bytes).
struct ResGroup {
    double inv_m[kModGroupWide];   // fl(1/m)
    double md[kModGroupWide];      // m as a double
    uint32_t g0[kModGroupWide];    // first INT8 plane of the modulus
    uint32_t two;                  // bit g: modulus g is two-limb (three planes)
    uint32_t pad[15];
};
static_assert(sizeof(ResGroup) == 384, "ResGroup layout");

// One block of 32 weight rows of the MFMA residue kernel as it reads it (wave-uniform
// scalar loads, 768 bytes).  Rows [0, n1) are one-limb moduli; rows p0 + 2 j and
// p0 + 2 j + 1 (j < n2) hold the low and high balanced base-128 halves of a two-limb
// modulus's weights.  A modulus's data sit at its first row.  Planes follow the moduli
// order (one plane per one-limb modulus, three per two-limb one), so consecutive one-limb
// rows own consecutive planes and consecutive pairs consecutive triples.
struct ResRowBlock {
    double inv_m[32];   // fl(1/m)
    double md[32];      // m as a double
    uint32_t g0[32];    // first INT8 plane of the modulus
    uint32_t n1, p0, n2;
    uint32_t pad[29];
};
static_assert(sizeof(ResRowBlock) == 768, "ResRowBlock layout");

// One modulus of the binary64 backend as its kernels read it (32 bytes).
struct F64Mod {
    double m;       // the modulus (a prime below 2^22 with K ((m - 1)/2)^2 <= 2^53)
    double inv_m;   // fl(1/m)
    double minv;    // (P / m)^-1 mod m, the direct-CRT weight
    double pad;
};
static_assert(sizeof(F64Mod) == 32, "F64Mod layout");

constexpr int kF64Split = 11;               // CRT terms of a binary64 modulus: v = lo + 2^11 hi
constexpr uint32_t kF64MaxModulus = (1u << 22) - 1;   // so that hi < 2^11 as well

// Backends of a plan: INT8 residue GEMMs (the default), binary64 residue GEMMs (the paper's
// "(b) binary64 backend"), or both over one moduli set (its "Mixed backends").
enum PlanBackend { kBackendInt8 = 0, kBackendF64 = 1, kBackendMixed = 2 };

struct PlanHost {
    int backend = kBackendInt8;
    int Lf = 0;            // binary64 moduli (kBackendF64 / kBackendMixed)
    int L8 = 0;            // ... INT8 moduli ahead of them (kBackendMixed); their CRT terms
                           // come first, then two per binary64 modulus (low, high 11 bits)
    std::vector<uint32_t> f64_moduli;   // Lf
    std::vector<F64Mod> f64;            // Lf
    int fnh = 0;                        // 16-bit halves of an integer significand (2 nw32)
    std::vector<double> f64_rw;         // [Lf][fnh]: centred 2^(16 h) mod m
    int p = 0, t = 0;
    int tile = 0;          // oz2h_tile hint of the residue GEMMs (0 = automatic)
    uint32_t flags = 0;    // OZ2H_FLAG_* bits: matrix-core variants of stages 2 and 4
    int64_t K = 0;
    int L = 0, L1 = 0, L2 = 0, G = 0;
    int nw32 = 0;          // 32-bit words of the widest integer significand (t+1 bits, or
                           // t_w+1 for the backward's upstream gradient)
    bool grad = false;     // also covers the backward products of an M x K by K x N product
    int64_t gM = 0, gN = 0;
    int tw[2] = {0, 0};    // widths of the upstream gradient W for dA = W B^T and dB = A^T W
    int nd32 = 0;          // 32-bit digits of the CRT accumulator
    int kg = kModGroup;    // moduli per residue group: kModGroup, or kModGroupWide for L >= kWideL
    int lgroups = 0;       // ceil(L / kg)
    int crt_dc = 0;        // CRT digit chunk (digits accumulated per pass)
    int crt_nc = 0;        // CRT passes
    int crt_ndpad = 0;     // crt_dc * crt_nc
    double log2P = 0;
    int pbits = 0;         // bit length of P
    std::vector<uint32_t> moduli;    // L, one-limb first
    std::vector<ModInfo> info;       // L
    std::vector<double> resid_tab;   // [lgroups][nw32][kg]: centred 2^(32w) mod m
    int rnwp = 0;          // VALU residues: words per integer padded to a multiple of 4
    int rg16 = 0;          // ... groups of 16 moduli
    std::vector<double> resid_row;   // [rg16][16 moduli][rnwp words]: centred 2^(32w) mod m
                                     // (0 past L and past nw32)
    std::vector<ResGroup> resgrp;    // [lgroups]
    int rnb = 0;           // MFMA residues: magnitude bytes (4 nw32), then two correction bytes
    int rnq = 0;           // ... 32-byte k-steps covering rnb + 2 bytes
    int rnrb = 0;          // ... blocks of 32 weight rows
    std::vector<int8_t> rmma_w;          // [rnrb][rnq][64 lanes][16]: MFMA A fragments
    std::vector<ResRowBlock> rmma_rb;    // [rnrb]
    std::vector<double> crt_digits;  // [L][crt_ndpad]: balanced base-2^32 digits of P/m
    int crt_ndg = 0;       // row-broadcast CRT: groups of 16 digits
    int crt_lpad = 0;      // ... moduli padded to a multiple of 16
    std::vector<double> crt_row;     // [16 crt_ndg][crt_lpad]: digit d of P/m_l at [d][l]
    bool crt_mma = false;  // matrix-core CRT tables built (nd32 <= 32, L <= 127)
    int crt_nbk = 0;       // ... blocks of 32 byte rows of S
    int crt_kq = 0;        // ... 32-byte contraction steps (2 L + 1 bytes)
    int crt_nt = 0;        // top digits of S that estimate S / P (every CRT kernel)
    double crt_inv_ptop = 0;           // 1 / P_top, P_top = P / 2^(32 (nd32 - crt_nt))
    std::vector<int8_t> crt_afr;       // [crt_nbk][crt_kq][64 lanes][16]: MFMA A fragments
    std::vector<uint32_t> p_digits;  // [nd32] digits of P
    std::vector<uint32_t> ph_digits; // [nd32] digits of floor(P/2)
};

int ceil_log2(int64_t K);

// The paper's hybrid INT8 moduli list: the 54 prime powers <= 255 in
// decreasing order, then the primes 255 < m <= 16191 in decreasing order.
const std::vector<uint32_t> &global_moduli();

// Greedy prefix of the global list until log2 P > 2t + ceil(log2 K) + margin.
// Returns 0, or a negative oz2h_status with `err` set.
int select_moduli(int p, int64_t K, int guard_bits, int t_bits, int margin,
                  std::vector<uint32_t> &mods, int &t, double &log2P, std::string &err);

// Greedy prefix of the global list until log2 P > need.
int select_moduli_bits(double need, std::vector<uint32_t> &mods, double &log2P, std::string &err);

// Fill every table for the given moduli (one-limb moduli must come first);
// integer significands are up to max(t, wmax) + 1 bits wide.  extra (nullable): further
// moduli of the same CRT (a mixed plan's binary64 moduli), whose product enters the
// direct-CRT weights (P / m_l)^-1 mod m_l.
int build_plan(int p, int t, int64_t K, const std::vector<uint32_t> &mods, PlanHost &out,
               std::string &err, int wmax = 0, bool allow_wide = true,
               const std::vector<uint32_t> *extra = nullptr);

// Largest binary64 modulus for contraction length K (Eq. fp64bound, capped so that a
// residue splits into two 11-bit CRT terms).
uint32_t f64_modulus_bound(int64_t K);

// Moduli of a binary64 plan (mixed = false: primes below f64_modulus_bound in decreasing
// order) or of a mixed plan (one-limb INT8 moduli, largest first, up to half the needed
// bits, then those primes), greedy until log2 P > 2t + ceil(log2 K) + margin.
int select_moduli_f64(int p, int64_t K, int guard_bits, int t_bits, int margin, bool mixed,
                      std::vector<uint32_t> &m8, std::vector<uint32_t> &m64, int &t,
                      double &log2P, std::string &err);

// The CRT plan of a binary64 or mixed moduli set: CRT terms (one per INT8 modulus, two per
// binary64 modulus) with their digit tables, and the binary64 moduli's tables.  With INT8
// moduli, h8 receives their plan (residue and GEMM tables, weights against the whole P).
int build_plan_f64(int p, int t, int64_t K, const std::vector<uint32_t> &m8,
                   const std::vector<uint32_t> &m64, PlanHost &h, PlanHost *h8, std::string &err);

}  // namespace oz2h
