// oz2h_plan.cpp -- moduli selection and constant tables of the Ozaki-II pipeline.
//
// Moduli: subsection "(a) AMX-INT8 backend" and Table "Moduli configuration".
// CRT constants: subsection "Direct CRT without multiple-precision division".
// Residue constants: subsection "Residue generation and packing" (the residue
// of a multi-digit integer is the sum of its digits times 2^(digit weight) mod m).
#include "oz2h_plan.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace oz2h {

namespace {

// little-endian base-2^32 natural numbers, just what the plan needs
using Nat = std::vector<uint32_t>;

void nat_trim(Nat &a) {
    while (!a.empty() && a.back() == 0) a.pop_back();
}

void nat_mul_small(Nat &a, uint32_t m) {
    uint64_t carry = 0;
    for (auto &d : a) {
        uint64_t x = (uint64_t)d * m + carry;
        d = (uint32_t)x;
        carry = x >> 32;
    }
    if (carry) a.push_back((uint32_t)carry);
}

// a / m, requiring the division to be exact; returns the quotient
Nat nat_divexact_small(const Nat &a, uint32_t m) {
    Nat q(a.size());
    uint64_t rem = 0;
    for (size_t i = a.size(); i-- > 0;) {
        uint64_t x = (rem << 32) | a[i];
        q[i] = (uint32_t)(x / m);
        rem = x % m;
    }
    nat_trim(q);
    return q;
}

uint32_t nat_mod_small(const Nat &a, uint32_t m) {
    uint64_t rem = 0;
    for (size_t i = a.size(); i-- > 0;) rem = ((rem << 32) | a[i]) % m;
    return (uint32_t)rem;
}

void nat_add(Nat &a, const Nat &b) {   // a += b
    if (a.size() < b.size()) a.resize(b.size(), 0u);
    uint64_t carry = 0;
    for (size_t i = 0; i < a.size(); ++i) {
        const uint64_t x = (uint64_t)a[i] + (i < b.size() ? b[i] : 0u) + carry;
        a[i] = (uint32_t)x;
        carry = x >> 32;
    }
    if (carry) a.push_back((uint32_t)carry);
}

bool nat_ge(const Nat &a, const Nat &b) {
    const size_t n = std::max(a.size(), b.size());
    for (size_t i = n; i-- > 0;) {
        const uint32_t x = i < a.size() ? a[i] : 0u, y = i < b.size() ? b[i] : 0u;
        if (x != y) return x > y;
    }
    return true;
}

void nat_sub(Nat &a, const Nat &b) {   // a -= b, a >= b
    int64_t borrow = 0;
    for (size_t i = 0; i < a.size(); ++i) {
        const int64_t x = (int64_t)a[i] - (i < b.size() ? b[i] : 0u) - borrow;
        a[i] = (uint32_t)x;
        borrow = x < 0;
    }
    nat_trim(a);
}

// balanced base-256 digits of a (each in [-128, 127]) at n positions
std::vector<int> nat_balanced_bytes(const Nat &a, int n) {
    std::vector<int> d(n, 0);
    int carry = 0;
    for (int j = 0; j < n; ++j) {
        const size_t w = (size_t)j / 4;
        int x = (w < a.size() ? (int)((a[w] >> (8 * (j % 4))) & 255u) : 0) + carry;
        carry = x >= 128;
        d[j] = carry ? x - 256 : x;
    }
    return d;
}

int nat_bitlen(const Nat &a) {
    for (size_t i = a.size(); i-- > 0;)
        if (a[i]) return (int)(32 * i + (32 - __builtin_clz(a[i])));
    return 0;
}

// x^-1 mod m for gcd(x, m) = 1
uint32_t inv_mod(uint32_t x, uint32_t m) {
    int64_t r0 = m, r1 = x % m, s0 = 0, s1 = 1;
    while (r1) {
        int64_t q = r0 / r1;
        int64_t r2 = r0 - q * r1;
        r0 = r1;
        r1 = r2;
        int64_t s2 = s0 - q * s1;
        s0 = s1;
        s1 = s2;
    }
    if (r0 != 1) return 0;
    int64_t v = s0 % (int64_t)m;
    if (v < 0) v += m;
    return (uint32_t)v;
}

std::vector<uint32_t> primes_upto(uint32_t n) {
    std::vector<char> sieve(n + 1, 1);
    sieve[0] = 0;
    if (n >= 1) sieve[1] = 0;
    for (uint32_t i = 2; (uint64_t)i * i <= n; ++i)
        if (sieve[i])
            for (uint32_t j = i * i; j <= n; j += i) sieve[j] = 0;
    std::vector<uint32_t> out;
    for (uint32_t i = 2; i <= n; ++i)
        if (sieve[i]) out.push_back(i);
    return out;
}

}  // namespace

int ceil_log2(int64_t K) {
    int b = 0;
    int64_t v = K - 1;
    while (v > 0) {
        ++b;
        v >>= 1;
    }
    return b;
}

const std::vector<uint32_t> &global_moduli() {
    static const std::vector<uint32_t> list = [] {
        std::vector<uint32_t> one, two;
        for (uint32_t q : primes_upto(kTwoLimbMax)) {
            if (q <= kOneLimbMax) {
                uint32_t x = q;
                while (x * q <= kOneLimbMax) x *= q;   // largest power of q that fits
                one.push_back(x);
            } else {
                two.push_back(q);
            }
        }
        std::sort(one.rbegin(), one.rend());
        std::sort(two.rbegin(), two.rend());
        one.insert(one.end(), two.begin(), two.end());
        return one;
    }();
    return list;
}

int select_moduli(int p, int64_t K, int guard_bits, int t_bits, int margin,
                  std::vector<uint32_t> &mods, int &t, double &log2P, std::string &err) {
    if (p < 2) {
        err = "p must be >= 2";
        return -1;
    }
    if (K < 1 || K > kMaxK) {
        err = "K must be in [1, 133000] (INT32 exactness of the residue GEMMs)";
        return K < 1 ? -1 : -2;
    }
    if (guard_bits < 0 || t_bits < 0 || margin < 1) {
        err = "guard_bits and t_bits must be >= 0 and crt_margin >= 1";
        return -1;
    }
    t = t_bits ? t_bits : p + guard_bits + ceil_log2(K);
    if (t < 1) {
        err = "internal width t must be >= 1";
        return -1;
    }
    return select_moduli_bits(2.0 * t + ceil_log2(K) + margin, mods, log2P, err);   // Eq. crtcond
}

int select_moduli_bits(double need, std::vector<uint32_t> &mods, double &log2P, std::string &err) {
    mods.clear();
    log2P = 0;
    for (uint32_t m : global_moduli()) {
        if (log2P > need) break;
        mods.push_back(m);
        log2P += std::log2((double)m);
    }
    if (!(log2P > need) || (int)mods.size() > kMaxModuli) {
        err = "precision too large for the supported moduli set (at most 512 moduli)";
        return -2;
    }
    return 0;
}

// Tables of the matrix-core CRT (digit columns in LDS, nd32 <= 32, L <= 127).  The digit
// sums S = sum_l v_l M_l (M_l = P/m_l) are an int8 product: v_l = Lo + 256 Hi with Lo its
// low byte (fed as Lo - 128) and Hi its signed high byte, so with b_{l,j} the balanced
// base-256 digits of M_l the byte column j of S is
//   sum_l (Lo_l - 128) b_{l,j} + Hi_l b_{l,j-1},
// contraction index 2 l (the Lo byte) and 2 l + 1 (the Hi byte).  Contraction index 2 L
// is fed the byte -128 against the digits of (-sum_l M_l mod P), which adds back
// 128 sum_l M_l modulo P.  Column sums stay below 128 * 128 * (2 L + 1) < 2^23.
void build_crt_mma_tables(PlanHost &h, const std::vector<uint32_t> &mods, const Nat &P) {
    h.crt_mma = false;
    h.crt_afr.clear();
    if (h.nd32 > 32 || h.L > 127) return;
    const int nb = 4 * h.nd32;                // byte rows of S
    h.crt_nbk = (nb + 31) / 32;               // blocks of 32 byte rows (8 digits)
    h.crt_kq = (2 * h.L + 1 + 31) / 32;       // 32-byte contraction steps
    const int rows = 32 * h.crt_nbk, kk = 32 * h.crt_kq;
    std::vector<int8_t> T((size_t)rows * kk, 0);
    Nat sum;
    for (int l = 0; l < h.L; ++l) {
        const Nat Ml = nat_divexact_small(P, mods[l]);
        nat_add(sum, Ml);
        const std::vector<int> b = nat_balanced_bytes(Ml, rows);
        for (int j = 0; j < rows; ++j) {
            T[(size_t)j * kk + 2 * l] = (int8_t)b[j];
            T[(size_t)j * kk + 2 * l + 1] = (int8_t)(j ? b[j - 1] : 0);
        }
    }
    while (nat_ge(sum, P) && !sum.empty()) nat_sub(sum, P);   // sum_l M_l mod P
    Nat corr = P;
    if (sum.empty()) corr.clear();
    else nat_sub(corr, sum);                                     // -sum_l M_l mod P
    const std::vector<int> bc = nat_balanced_bytes(corr, rows);
    for (int j = 0; j < rows; ++j) T[(size_t)j * kk + 2 * h.L] = (int8_t)bc[j];
    // MFMA A fragments: lane l of step q of row block r holds row 32 r + l % 32,
    // contraction bytes 32 q + 16 (l / 32) ..
    h.crt_afr.assign((size_t)h.crt_nbk * h.crt_kq * 64 * 16, 0);
    for (int r = 0; r < h.crt_nbk; ++r)
        for (int q = 0; q < h.crt_kq; ++q)
            for (int lane = 0; lane < 64; ++lane)
                for (int e = 0; e < 16; ++e)
                    h.crt_afr[(((size_t)r * h.crt_kq + q) * 64 + lane) * 16 + e] =
                        T[(size_t)(32 * r + lane % 32) * kk + 32 * q + 16 * (lane / 32) + e];
    h.crt_mma = true;
}

// Digit tables of the direct CRT over h.L terms: S = sum_l v_l coef_l with coef_l = P / m_l
// (or a multiple of it), as balanced base-2^32 digits (|d| <= 2^31), plus P's digits and
// the top-digit estimate of S / P.
int crt_tables(PlanHost &h, const Nat &P, const std::vector<Nat> &coef, std::string &err) {
    h.pbits = nat_bitlen(P);
    h.nd32 = (h.pbits + 31) / 32 + 2;   // two digits of headroom (subsection on the batched CRT)
    h.crt_nc = (h.nd32 + 31) / 32;
    int per = (h.nd32 + h.crt_nc - 1) / h.crt_nc;
    h.crt_dc = ((per + 3) / 4) * 4;   // a multiple of 4 (two digits per LDS read, little padding)
    h.crt_ndpad = h.crt_dc * h.crt_nc;
    h.crt_digits.assign((size_t)h.L * h.crt_ndpad, 0.0);
    for (int l = 0; l < h.L; ++l) {
        const Nat &Ml = coef[l];
        int64_t carry = 0;
        for (int k = 0; k < h.crt_ndpad; ++k) {
            int64_t x = (k < (int)Ml.size() ? (int64_t)Ml[k] : 0) + carry;
            if (x >= (int64_t)1 << 31) {
                x -= (int64_t)1 << 32;
                carry = 1;
            } else {
                carry = 0;
            }
            h.crt_digits[(size_t)l * h.crt_ndpad + k] = (double)x;
        }
        if (carry || (int)Ml.size() > h.crt_ndpad) {
            err = "internal error: CRT digit table too short";
            return -1;
        }
    }
    // S/P from the top crt_nt digits of S: S_top / P_top with X_top = X / 2^(32 (nd32 - nt))
    // (P's digits below the top nt are dropped: P_top keeps at least 64 of P's bits)
    h.crt_nt = std::min(h.nd32, 5);
    {
        double ptop = 0.0;
        for (int k = h.nd32 - 1; k >= h.nd32 - h.crt_nt; --k)
            ptop = ptop * 4294967296.0 + (double)(k < (int)P.size() ? P[k] : 0u);
        h.crt_inv_ptop = 1.0 / ptop;
    }
    // the row-broadcast CRT's table: digit d of coef_l at [d][l], 16 digits per lane row group
    h.crt_ndg = (h.nd32 + 15) / 16;
    h.crt_lpad = (h.L + 15) / 16 * 16;
    h.crt_row.assign((size_t)16 * h.crt_ndg * h.crt_lpad, 0.0);
    for (int l = 0; l < h.L; ++l)
        for (int d = 0; d < h.nd32 && d < h.crt_ndpad; ++d)
            h.crt_row[(size_t)d * h.crt_lpad + l] = h.crt_digits[(size_t)l * h.crt_ndpad + d];
    h.p_digits.assign(h.nd32, 0);
    h.ph_digits.assign(h.nd32, 0);
    for (int k = 0; k < h.nd32 && k < (int)P.size(); ++k) h.p_digits[k] = P[k];
    for (int k = 0; k < h.nd32; ++k) {
        uint32_t lo = h.p_digits[k] >> 1;
        uint32_t hi = (k + 1 < h.nd32) ? (h.p_digits[k + 1] & 1u) << 31 : 0;
        h.ph_digits[k] = lo | hi;
    }
    return 0;
}

// Tables of the MFMA residue kernel.  The residue of a magnitude |a| = sum_j b_j 256^j
// (bytes b_j, j < nb) is sum_j b_j w_j mod m with w_j the centred 256^j mod m: an int8
// product of the byte string and a weight row (two rows of balanced base-128 halves for
// a two-limb modulus).  The kernel feeds the bytes as b_j - 128 (int8 range) and a
// negative entry as its complement 255 - b_j; two correction bytes at nb (always 0) and
// nb + 1 (1 for a negative entry) with weights C1 = 254 S and C2 = -255 S, S = sum_j w_j,
// make the product congruent to the signed entry:
//   positive: sum (b_j - 128) w_j - 128 C1 - 128 C2 = |a| + (-128 - 128*254 + 128*255) S = |a|
//   negative: sum (127 - b_j) w_j - 128 C1 - 127 C2 = -|a| + (127 - 128*254 + 127*255) S = -|a|
// (mod m).  Every weight row has |w| <= 127, so |product| <= 128 * 127 * (nb + 2) < 2^31.
void build_residue_mma_tables(PlanHost &h, const std::vector<uint32_t> &mods) {
    h.rnb = 4 * h.nw32;
    const int nbk = (h.rnb + 2 + 31) / 32 * 32;
    h.rnq = nbk / 32;
    const int r0 = (h.L1 + 3) / 4 * 4;   // two-limb pairs start on a multiple of 4
    const int ml = r0 + 2 * (h.L - h.L1);
    h.rnrb = (ml + 31) / 32;
    std::vector<int8_t> W((size_t)h.rnrb * 32 * nbk, 0);
    for (int l = 0; l < h.L; ++l) {
        const int64_t m = mods[l];
        auto centred = [m](int64_t x) { return x > (m - 1) / 2 ? x - m : x; };
        std::vector<int64_t> v(nbk, 0);
        int64_t x = 1 % m, S = 0;
        for (int j = 0; j < h.rnb; ++j) {
            v[j] = centred(x);
            S = (S + x) % m;
            x = x * 256 % m;
        }
        v[h.rnb] = centred(254 * S % m);
        v[h.rnb + 1] = centred((m - 255 * S % m) % m);
        if (l < h.L1) {
            for (int j = 0; j < nbk; ++j) W[(size_t)l * nbk + j] = (int8_t)v[j];
        } else {
            const size_t R = (size_t)(r0 + 2 * (l - h.L1));
            for (int j = 0; j < nbk; ++j) {
                const int64_t lo = ((v[j] + 64) & 127) - 64;
                W[R * nbk + j] = (int8_t)lo;
                W[(R + 1) * nbk + j] = (int8_t)((v[j] - lo) / 128);
            }
        }
    }
    // MFMA A fragments: lane l of k-step q holds row l % 32, bytes 32 q + 16 (l / 32) ..
    h.rmma_w.assign((size_t)h.rnrb * h.rnq * 64 * 16, 0);
    for (int rb = 0; rb < h.rnrb; ++rb)
        for (int q = 0; q < h.rnq; ++q)
            for (int lane = 0; lane < 64; ++lane)
                for (int e = 0; e < 16; ++e)
                    h.rmma_w[(((size_t)rb * h.rnq + q) * 64 + lane) * 16 + e] =
                        W[(size_t)(rb * 32 + lane % 32) * nbk + 32 * q + 16 * (lane / 32) + e];
    h.rmma_rb.assign(h.rnrb, ResRowBlock{});
    for (int rb = 0; rb < h.rnrb; ++rb) {
        ResRowBlock &B = h.rmma_rb[rb];
        const int lo = rb * 32, hi = lo + 32;
        B.n1 = (uint32_t)std::max(0, std::min(32, h.L1 - lo));
        const int pa = std::max(r0, lo), pb = std::min(ml, hi);
        B.p0 = (uint32_t)(pa - lo);
        B.n2 = pb > pa ? (uint32_t)((pb - pa) / 2) : 0u;
        for (int l = 0; l < h.L; ++l) {
            const int R = l < h.L1 ? l : r0 + 2 * (l - h.L1);
            if (R < lo || R >= hi) continue;
            B.inv_m[R - lo] = h.info[l].inv_m;
            B.md[R - lo] = (double)h.info[l].m;
            B.g0[R - lo] = h.info[l].g0;
        }
    }
}

int build_plan(int p, int t, int64_t K, const std::vector<uint32_t> &mods_in, PlanHost &h,
               std::string &err, int wmax, bool allow_wide, const std::vector<uint32_t> *extra) {
    if (mods_in.empty() || (int)mods_in.size() > kMaxModuli) {
        err = "need 1..512 moduli";
        return -1;
    }
    std::vector<uint32_t> mods;
    for (uint32_t m : mods_in)
        if (m <= kOneLimbMax) mods.push_back(m);
    for (uint32_t m : mods_in)
        if (m > kOneLimbMax) mods.push_back(m);
    for (size_t a = 0; a < mods.size(); ++a) {
        if (mods[a] < 2 || mods[a] > kTwoLimbMax) {
            err = "moduli must lie in [2, 16191]";
            return -1;
        }
        for (size_t b = 0; b < a; ++b)
            if (std::gcd(mods[a], mods[b]) != 1) {
                err = "moduli must be pairwise coprime";
                return -1;
            }
    }
    h = PlanHost{};
    h.p = p;
    h.t = t;
    h.K = K;
    h.L = (int)mods.size();
    h.moduli = mods;
    h.nw32 = (std::max(t, wmax) + 1 + 31) / 32;
    if (h.nw32 > kMaxWords) {
        err = "internal width t too large for the residue kernel";
        return -2;
    }

    // P and the one-limb / two-limb split; plane numbering
    Nat P{1};
    h.log2P = 0;
    uint32_t g = 0;
    for (uint32_t m : mods) {
        nat_mul_small(P, m);
        h.log2P += std::log2((double)m);
        ModInfo mi{};
        mi.m = m;
        mi.g0 = g;
        mi.nprod = m <= kOneLimbMax ? 1u : 3u;
        mi.inv_m = 1.0 / (double)m;
        g += mi.nprod;
        h.info.push_back(mi);
        if (mi.nprod == 1) ++h.L1;
        else ++h.L2;
    }
    h.G = (int)g;

    // direct-CRT weights: M_l = P_all / m_l, minv = M_l^-1 mod m_l, with P_all the product of
    // every modulus of the CRT (times the extra moduli of a mixed plan)
    Nat Pw = P;
    if (extra)
        for (uint32_t m : *extra) nat_mul_small(Pw, m);
    std::vector<Nat> coef(h.L);
    for (int l = 0; l < h.L; ++l) {
        const uint32_t m = mods[l];
        const Nat Ml = nat_divexact_small(Pw, m);
        uint32_t minv = inv_mod(nat_mod_small(Ml, m), m);
        if (!minv && m != 1) {
            err = "internal error: M_l not invertible";
            return -1;
        }
        h.info[l].minv = minv;
        auto centred = [m](int64_t x) {
            int64_t r = x % (int64_t)m;
            if (r < 0) r += m;
            if (r > (int64_t)((m - 1) / 2)) r -= m;
            return (int32_t)r;
        };
        if (h.info[l].nprod == 1) {
            h.info[l].kc[0] = centred(minv);
            h.info[l].kc[1] = h.info[l].kc[2] = 0;
        } else {
            // sum r_a r_b = -127 P0 + 16256 P2 + 128 Ps (Karatsuba on balanced base-128
            // halves); weighted by minv, folded after each product (see k_resgemm)
            const int64_t c0 = (-127 * (int64_t)minv) % m, c2 = (16256 * (int64_t)minv) % m,
                          cs = (128 * (int64_t)minv) % m;
            const uint32_t c2i = inv_mod((uint32_t)((c2 + m) % m), m);
            const uint32_t csi = inv_mod((uint32_t)((cs + m) % m), m);
            if (!c2i || !csi) {
                err = "two-limb moduli must be odd primes";
                return -1;
            }
            h.info[l].kc[0] = centred(((c0 + m) % m) * (int64_t)c2i);
            h.info[l].kc[1] = centred(((c2 + m) % m) * (int64_t)csi);
            h.info[l].kc[2] = centred(cs);
        }
        coef[l] = nat_divexact_small(P, m);
    }
    const int cst = crt_tables(h, P, coef, err);
    if (cst) return cst;
    build_crt_mma_tables(h, mods, P);

    // residue weights: centred 2^(32 w) mod m, grouped by kg moduli (16 for wide sets:
    // each word read then feeds twice the FMAs)
    h.kg = allow_wide && h.L >= kWideL ? kModGroupWide : kModGroup;
    const int kg = h.kg;
    h.lgroups = (h.L + kg - 1) / kg;
    h.resgrp.assign(h.lgroups, ResGroup{});
    for (int l = 0; l < h.L; ++l) {
        ResGroup &R = h.resgrp[l / kg];
        const int g = l % kg;
        R.inv_m[g] = h.info[l].inv_m;
        R.md[g] = (double)h.info[l].m;
        R.g0[g] = h.info[l].g0;
        if (h.info[l].nprod == 3) R.two |= 1u << g;
    }
    h.resid_tab.assign((size_t)h.lgroups * h.nw32 * kg, 0.0);
    for (int l = 0; l < h.L; ++l) {
        const uint64_t m = mods[l];
        uint64_t x = 1 % m;
        for (int w = 0; w < h.nw32; ++w) {
            int64_t c = (int64_t)x;
            if (c > (int64_t)((m - 1) / 2)) c -= (int64_t)m;
            h.resid_tab[((size_t)(l / kg) * h.nw32 + w) * kg + (l % kg)] =
                (double)c;
            x = ((x << 32) % m);
        }
    }
    // the VALU kernel's table: per group of 16 moduli, one row of rnwp words per modulus,
    // which the lane of that modulus reads in 16-word chunks
    h.rnwp = (h.nw32 + 3) / 4 * 4;
    h.rg16 = (h.L + 15) / 16;
    h.resid_row.assign((size_t)h.rg16 * 16 * h.rnwp, 0.0);
    for (int l = 0; l < h.L; ++l) {
        const uint64_t m = mods[l];
        uint64_t x = 1 % m;
        for (int w = 0; w < h.nw32; ++w) {
            int64_t c = (int64_t)x;
            if (c > (int64_t)((m - 1) / 2)) c -= (int64_t)m;
            h.resid_row[(size_t)l * h.rnwp + w] = (double)c;
            x = (x << 32) % m;
        }
    }
    build_residue_mma_tables(h, mods);
    return 0;
}

uint32_t f64_modulus_bound(int64_t K) {
    // m <= sqrt(2^55 / K) (Eq. fp64bound): then K ((m - 1)/2)^2 < 2^53, so every residue
    // product sum of a binary64 GEMM is an exact integer
    const long double b = std::sqrt((long double)36028797018963968.0L / (long double)K);
    uint64_t m = (uint64_t)b;
    while ((long double)(m + 1) * (m + 1) * K <= 36028797018963968.0L) ++m;
    while (m > 0 && (long double)m * m * K > 36028797018963968.0L) --m;
    return (uint32_t)std::min<uint64_t>(m, kF64MaxModulus);
}

namespace {
bool is_prime(uint32_t x) {
    if (x < 2) return false;
    if (x % 2 == 0) return x == 2;
    for (uint32_t f = 3; (uint64_t)f * f <= x; f += 2)
        if (x % f == 0) return false;
    return true;
}
}  // namespace

int select_moduli_f64(int p, int64_t K, int guard_bits, int t_bits, int margin, bool mixed,
                      std::vector<uint32_t> &m8, std::vector<uint32_t> &m64, int &t,
                      double &log2P, std::string &err) {
    if (p < 2) {
        err = "p must be >= 2";
        return -1;
    }
    if (K < 1 || K > kMaxK) {
        err = "K must be in [1, 133000]";
        return K < 1 ? -1 : -2;
    }
    if (guard_bits < 0 || t_bits < 0 || margin < 1) {
        err = "guard_bits and t_bits must be >= 0 and crt_margin >= 1";
        return -1;
    }
    t = t_bits ? t_bits : p + guard_bits + ceil_log2(K);
    if (t < 1) {
        err = "internal width t must be >= 1";
        return -1;
    }
    const double need = 2.0 * t + ceil_log2(K) + margin;   // Eq. crtcond
    m8.clear();
    m64.clear();
    log2P = 0;
    if (mixed) {
        // INT8 takes the one-limb prime powers (the most bits per GEMM) up to half the bits
        // needed, binary64 moduli the rest, so that both backends always take part
        for (uint32_t m : global_moduli()) {
            if (m > kOneLimbMax || log2P + std::log2((double)m) > 0.5 * need) break;
            m8.push_back(m);
            log2P += std::log2((double)m);
        }
    }
    for (uint32_t m = f64_modulus_bound(K); m > kTwoLimbMax && !(log2P > need); --m) {
        if (!is_prime(m)) continue;
        if ((int)(m8.size() + 2 * (m64.size() + 1)) > kMaxModuli) break;
        m64.push_back(m);
        log2P += std::log2((double)m);
    }
    if (!(log2P > need)) {
        err = "precision too large for the binary64 moduli set (at most 512 CRT terms)";
        return -2;
    }
    return 0;
}

int build_plan_f64(int p, int t, int64_t K, const std::vector<uint32_t> &m8,
                   const std::vector<uint32_t> &m64, PlanHost &h, PlanHost *h8, std::string &err) {
    const int terms = (int)(m8.size() + 2 * m64.size());
    if (m64.empty() || terms > kMaxModuli) {
        err = "need 1 to 256 binary64 moduli (at most 512 CRT terms)";
        return -1;
    }
    const uint32_t bound = f64_modulus_bound(K);
    std::vector<uint32_t> all(m8);
    all.insert(all.end(), m64.begin(), m64.end());
    for (size_t a = 0; a < all.size(); ++a) {
        const bool f = a >= m8.size();
        if (all[a] < 2 || (f && all[a] > bound) || (!f && all[a] > kTwoLimbMax)) {
            err = "binary64 moduli must lie in [2, sqrt(2^55 / K)] (and below 2^22)";
            return -1;
        }
        for (size_t b = 0; b < a; ++b)
            if (std::gcd(all[a], all[b]) != 1) {
                err = "moduli must be pairwise coprime";
                return -1;
            }
    }
    if (!m8.empty()) {
        const int st = build_plan(p, t, K, m8, *h8, err, 0, true, &m64);
        if (st) return st;
    }
    h = PlanHost{};
    h.backend = m8.empty() ? kBackendF64 : kBackendMixed;
    h.p = p;
    h.t = t;
    h.K = K;
    h.L8 = (int)m8.size();
    h.Lf = (int)m64.size();
    h.L = terms;
    h.moduli = all;
    h.f64_moduli = m64;
    h.nw32 = (t + 1 + 31) / 32;
    if (h.nw32 > kMaxWords) {
        err = "internal width t too large for the residue kernel";
        return -2;
    }
    Nat P{1};
    for (uint32_t m : all) {
        nat_mul_small(P, m);
        h.log2P += std::log2((double)m);
    }
    // CRT terms: v_l M_l for an INT8 modulus; v = lo + 2^11 hi, lo, hi < 2^11, as the two
    // terms lo M_l and hi (2^11 M_l) for a binary64 modulus (so that every term's digit
    // products stay below 2^42, as with the INT8 moduli's int16 residues)
    std::vector<Nat> coef;
    for (uint32_t m : all) {
        const Nat Ml = nat_divexact_small(P, m);
        const uint32_t minv = inv_mod(nat_mod_small(Ml, m), m);
        ModInfo mi{};
        mi.m = m;
        mi.nprod = 0;
        mi.minv = minv;
        mi.inv_m = 1.0 / (double)m;
        h.info.push_back(mi);
        coef.push_back(Ml);
        if (m > kTwoLimbMax || std::find(m64.begin(), m64.end(), m) != m64.end()) {
            Nat hi = Ml;
            nat_mul_small(hi, 1u << kF64Split);
            mi.inv_m = (double)(1u << kF64Split) * (1.0 / (double)m);
            h.info.push_back(mi);
            coef.push_back(hi);
            F64Mod fm{};
            fm.m = (double)m;
            fm.inv_m = 1.0 / (double)m;
            fm.minv = (double)minv;
            h.f64.push_back(fm);
        }
    }
    const int cst = crt_tables(h, P, coef, err);
    if (cst) return cst;
    // binary64 residues: the magnitude's 16-bit halves times centred 2^(16 j) mod m
    h.fnh = 2 * h.nw32;
    h.f64_rw.assign((size_t)h.Lf * h.fnh, 0.0);
    for (int j = 0; j < h.Lf; ++j) {
        const uint64_t m = m64[j];
        uint64_t x = 1 % m;
        for (int w = 0; w < h.fnh; ++w) {
            int64_t c = (int64_t)x;
            if (c > (int64_t)((m - 1) / 2)) c -= (int64_t)m;
            h.f64_rw[(size_t)j * h.fnh + w] = (double)c;
            x = (x << 16) % m;
        }
    }
    return 0;
}

}  // namespace oz2h
