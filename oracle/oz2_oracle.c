/*
 * oz2_oracle.c -- exact CPU reference of the Ozaki-II p-bit matrix product.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  It shares no code,
 * header, table or helper with the GPU path, and it uses no moduli at all:
 * the method reaches, exactly, the integer product of the shared-exponent
 * integer matrices (Algorithm section, Eqs. 1-2), so the oracle computes that
 * product directly with its own fixed-width bignums (64-bit limbs,
 * unsigned __int128 schoolbook), then applies the single final rounding.
 *
 *   t     = p + g + ceil(log2 K)                          (Eq. 3)
 *   e_i   = max exp(a_ik) over nonzero entries, 0 if none (Eq. 1)
 *   a^_ik = RNE(a_ik * 2^(t - e_i)),  |a^_ik| <= 2^t        (Eq. 1)
 *   c^_ij = sum_k a^_ik b^_kj                              (Eq. 2, exact)
 *   c_ij  = RNE_p(c^_ij * 2^(e_i + f_j - 2t))              (Eq. 2, one rounding)
 *
 * The general entry point oz2o_gemm_scaled gives each operand side its own
 * width t, an optional exponent offset per contraction index and optionally
 * given (instead of computed) row exponents.  This is how the backward
 * products of C = A B are integerized when they reuse the forward's integer
 * matrices (exponent folding, a reading the paper does not state):
 *   dA = W B^T:  W'_ij = W_ij 2^(f_j), scaled per row with t_w;  B^ as saved,
 *                i.e. offset -f_j per contraction index j and row exponent 0
 *   dB = A^T W:  W''_ij = W_ij 2^(e_i), scaled per column with t_w;  A^ as saved
 *
 * Number format: value = sign * mant * 2^(exp - p), sign in {-1,0,+1} (0 is
 * zero), mant stored as nl = ceil(p/64) little-endian uint64 limbs; bits at
 * or above p are ignored.  Outputs have 2^(p-1) <= mant < 2^p, or are zero.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC oz2_oracle.c -o liboz2oracle.so
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

typedef struct {
    const int8_t *sign;
    const int32_t *exp;
    const uint64_t *limbs;
    int64_t rs, cs;   /* element strides of logical rows / columns */
    int nl;
} opnd;

static int ceil_log2_i64(int64_t K) {
    int b = 0;
    int64_t v = K - 1;
    while (v > 0) { b++; v >>= 1; }
    return b;
}

int oz2o_internal_width(int p, int64_t K, int g, int t_bits) {
    return t_bits ? t_bits : p + g + ceil_log2_i64(K);
}

int oz2o_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---- small fixed-width unsigned bignum helpers (n limbs, little-endian) ---- */

static int bn_bitlen(const uint64_t *x, int n) {
    for (int i = n - 1; i >= 0; i--)
        if (x[i]) return 64 * i + (64 - __builtin_clzll(x[i]));
    return 0;
}

static int bn_bit(const uint64_t *x, int n, int64_t pos) {
    if (pos < 0 || pos >= 64 * (int64_t)n) return 0;
    return (int)((x[pos / 64] >> (pos % 64)) & 1u);
}

/* nonzero if any bit strictly below pos is set */
static int bn_any_below(const uint64_t *x, int n, int64_t pos) {
    if (pos <= 0) return 0;
    int64_t full = pos / 64;
    for (int64_t i = 0; i < full && i < n; i++)
        if (x[i]) return 1;
    int r = (int)(pos % 64);
    if (r && full < n && (x[full] & ((1ull << r) - 1))) return 1;
    return 0;
}

/* out (m limbs) = x (n limbs) >> sh, sh >= 0 */
static void bn_shr(const uint64_t *x, int n, int64_t sh, uint64_t *out, int m) {
    int64_t q = sh / 64;
    int r = (int)(sh % 64);
    for (int i = 0; i < m; i++) {
        int64_t s = i + q;
        uint64_t lo = (s < n) ? x[s] : 0;
        uint64_t hi = (s + 1 < n) ? x[s + 1] : 0;
        out[i] = r ? ((lo >> r) | (hi << (64 - r))) : lo;
    }
}

/* out (m limbs) = x (n limbs) << sh, sh >= 0, truncated to m limbs */
static void bn_shl(const uint64_t *x, int n, int64_t sh, uint64_t *out, int m) {
    int64_t q = sh / 64;
    int r = (int)(sh % 64);
    for (int i = 0; i < m; i++) {
        int64_t s = i - q;
        uint64_t cur = (s >= 0 && s < n) ? x[s] : 0;
        uint64_t low = (s - 1 >= 0 && s - 1 < n) ? x[s - 1] : 0;
        out[i] = r ? ((cur << r) | (low >> (64 - r))) : cur;
    }
}

/* x += 1 (n limbs); returns carry out */
static int bn_inc(uint64_t *x, int n) {
    for (int i = 0; i < n; i++)
        if (++x[i] != 0) return 0;
    return 1;
}

/* RNE(x / 2^sh) into out (m limbs), x has n limbs, sh >= 1 */
static void bn_shr_rne(const uint64_t *x, int n, int64_t sh, uint64_t *out, int m) {
    bn_shr(x, n, sh, out, m);
    int rb = bn_bit(x, n, sh - 1);
    int st = bn_any_below(x, n, sh - 1);
    if (rb && (st || (out[0] & 1u))) bn_inc(out, m);
}

static int bn_cmp(const uint64_t *a, const uint64_t *b, int n) {
    for (int i = n - 1; i >= 0; i--) {
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    }
    return 0;
}

/* r = a - b (n limbs), requires a >= b */
static void bn_sub(const uint64_t *a, const uint64_t *b, uint64_t *r, int n) {
    uint64_t br = 0;
    for (int i = 0; i < n; i++) {
        u128 d = (u128)a[i] - b[i] - br;
        r[i] = (uint64_t)d;
        br = (uint64_t)(d >> 64) ? 1 : 0;
    }
}

/* acc (nacc limbs) += a (na) * b (na) */
static void bn_addmul(uint64_t *acc, int nacc, const uint64_t *a, const uint64_t *b, int na) {
    for (int x = 0; x < na; x++) {
        uint64_t ax = a[x];
        if (!ax) continue;
        u128 carry = 0;
        for (int y = 0; y < na; y++) {
            u128 t = (u128)ax * b[y] + acc[x + y] + carry;
            acc[x + y] = (uint64_t)t;
            carry = t >> 64;
        }
        for (int z = x + na; carry && z < nacc; z++) {
            u128 t = (u128)acc[z] + carry;
            acc[z] = (uint64_t)t;
            carry = t >> 64;
        }
    }
}

/* ---- the method's steps ---- */

/* e = max exp (+ koff[k]) over the nonzero entries of one logical row (step 1, Eq. 1) */
static int32_t shared_exponent(const opnd *X, int64_t base, int64_t step, int64_t count,
                               const int32_t *koff) {
    int have = 0;
    int32_t e = 0;
    for (int64_t k = 0; k < count; k++) {
        int64_t idx = base + k * step;
        if (X->sign[idx] == 0) continue;
        int32_t x = X->exp[idx] + (koff ? koff[k] : 0);
        if (!have || x > e) e = x;
        have = 1;
    }
    return have ? e : 0;
}

/* a^ = RNE(a * 2^(t + off - e)) as sign + na-limb magnitude (Eq. 1); returns sign */
static int integerize_entry(const opnd *X, int64_t idx, int p, int t, int32_t off, int32_t e,
                            uint64_t *mag, int na) {
    memset(mag, 0, sizeof(uint64_t) * na);
    int s = X->sign[idx];
    if (s == 0) return 0;
    uint64_t mant[X->nl > 0 ? X->nl : 1];
    memcpy(mant, X->limbs + idx * X->nl, sizeof(uint64_t) * X->nl);
    int topbits = p - 64 * (X->nl - 1);
    if (topbits < 64) mant[X->nl - 1] &= (1ull << topbits) - 1;
    int64_t sh = (int64_t)t - p + X->exp[idx] + off - e;
    if (sh >= 0) bn_shl(mant, X->nl, sh, mag, na);
    else bn_shr_rne(mant, X->nl, -sh, mag, na);
    if (bn_bitlen(mag, na) == 0) return 0;
    return s > 0 ? 1 : -1;
}

/*
 * Integerize every entry of a rows x count operand side.  The "row" index is
 * the one that owns the shared exponent (rows of A, columns of B); entry
 * (r, k) lives at r*X->rs + k*X->cs.  Outputs: e[rows], sign[rows*count],
 * mag[rows*count*na].
 */
int oz2o_integerize(int64_t rows, int64_t count, int p, int t,
                    const int8_t *sign, const int32_t *exp, const uint64_t *limbs,
                    int64_t rs, int64_t cs, int32_t *e_out,
                    int8_t *sign_out, uint64_t *mag_out, int na) {
    opnd X = {sign, exp, limbs, rs, cs, (p + 63) / 64};
    if (na * 64 < t + 1) return -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < rows; r++) {
        int32_t e = shared_exponent(&X, r * rs, cs, count, NULL);
        e_out[r] = e;
        for (int64_t k = 0; k < count; k++) {
            int64_t idx = r * rs + k * cs;
            sign_out[r * count + k] =
                (int8_t)integerize_entry(&X, idx, p, t, 0, e, mag_out + (r * count + k) * na, na);
        }
    }
    return 0;
}

/* RNE_p of mag * 2^scale (sign given) into (sign, exp, nl limbs); returns 0 or -1 on exp overflow */
static int round_out(int sgn, const uint64_t *mag, int n, int64_t scale, int p,
                     int8_t *osign, int32_t *oexp, uint64_t *olimbs) {
    int nl = (p + 63) / 64;
    memset(olimbs, 0, sizeof(uint64_t) * nl);
    int64_t nb = bn_bitlen(mag, n);
    if (nb == 0 || sgn == 0) { *osign = 0; *oexp = 0; return 0; }
    uint64_t tmp[nl + 1];
    if (nb <= p) {
        bn_shl(mag, n, p - nb, tmp, nl + 1);
    } else {
        bn_shr_rne(mag, n, nb - p, tmp, nl + 1);
        if (bn_bit(tmp, nl + 1, p)) {           /* carried to 2^p */
            bn_shr(tmp, nl + 1, 1, tmp, nl + 1);
            nb += 1;
        }
    }
    memcpy(olimbs, tmp, sizeof(uint64_t) * nl);
    int64_t ex = nb + scale;
    if (ex > INT32_MAX || ex < INT32_MIN) return -1;
    *osign = (int8_t)sgn;
    *oexp = (int32_t)ex;
    return 0;
}

/*
 * The whole reference, general form.  A is M x K, B is K x N, given as
 * (sign, exp, limbs) with element strides (a_rs, a_cs), (b_rs, b_cs).  Side A
 * is integerized with width ta: a^_ik = RNE(a_ik 2^(ta + a_koff[k] - e_i)) with
 * e_i = a_efix[i] if a_efix is given, else max(exp a_ik + a_koff[k]) over the
 * nonzero a_ik (0 if none); side B likewise per column with tb, b_koff, b_efix.
 * Every integer must satisfy |x^| <= 2^t of its side (true whenever the row
 * exponent is the max; checked otherwise).  c_ij = RNE_p(c^_ij 2^(e_i + f_j -
 * ta - tb)).  If sel_i is NULL every entry of C is computed (row-major, index
 * i*N + j); else the nsel entries (sel_i[s], sel_j[s]) are computed into slot
 * s.  Optional outputs (NULL to skip): e[M], f[N]; c^ as sign + nlc-limb
 * magnitude; C as sign/exp/nl limbs.  Returns 0, -1 for a too-small nlc, -2
 * for an exponent overflow, -3 for an integer wider than its t.
 */
int oz2o_gemm_scaled(int64_t M, int64_t N, int64_t K, int p,
                     int ta, const int8_t *As, const int32_t *Ae, const uint64_t *Al,
                     int64_t a_rs, int64_t a_cs, const int32_t *a_koff, const int32_t *a_efix,
                     int tb, const int8_t *Bs, const int32_t *Be, const uint64_t *Bl,
                     int64_t b_rs, int64_t b_cs, const int32_t *b_koff, const int32_t *b_efix,
                     int64_t nsel, const int64_t *sel_i, const int64_t *sel_j,
                     int32_t *e_out, int32_t *f_out,
                     int nlc, uint64_t *chat_mag, int8_t *chat_sign,
                     int8_t *c_sign, int32_t *c_exp, uint64_t *c_limbs) {
    opnd A = {As, Ae, Al, a_rs, a_cs, (p + 63) / 64};
    opnd B = {Bs, Be, Bl, b_rs, b_cs, (p + 63) / 64};
    int tmax = ta > tb ? ta : tb;
    int na = (tmax + 1 + 63) / 64 + 1;   /* one spare limb to detect a too-wide integer */
    int nacc = (ta + tb + ceil_log2_i64(K) + 2 + 63) / 64 + 1;
    int nl = (p + 63) / 64;
    int64_t nout = sel_i ? nsel : M * N;

    /* which rows of A / columns of B are needed */
    int64_t *rmap = malloc(sizeof(int64_t) * (M > 0 ? M : 1));
    int64_t *cmap = malloc(sizeof(int64_t) * (N > 0 ? N : 1));
    for (int64_t i = 0; i < M; i++) rmap[i] = sel_i ? -1 : i;
    for (int64_t j = 0; j < N; j++) cmap[j] = sel_i ? -1 : j;
    int64_t nr = sel_i ? 0 : M, nc = sel_i ? 0 : N;
    if (sel_i) {
        for (int64_t s = 0; s < nsel; s++) {
            if (rmap[sel_i[s]] < 0) rmap[sel_i[s]] = nr++;
            if (cmap[sel_j[s]] < 0) cmap[sel_j[s]] = nc++;
        }
    }
    int64_t *rlist = malloc(sizeof(int64_t) * (nr > 0 ? nr : 1));
    int64_t *clist = malloc(sizeof(int64_t) * (nc > 0 ? nc : 1));
    for (int64_t i = 0; i < M; i++) if (rmap[i] >= 0) rlist[rmap[i]] = i;
    for (int64_t j = 0; j < N; j++) if (cmap[j] >= 0) clist[cmap[j]] = j;

    int32_t *er = malloc(sizeof(int32_t) * (nr > 0 ? nr : 1));
    int32_t *fc = malloc(sizeof(int32_t) * (nc > 0 ? nc : 1));
    int8_t *ras = malloc((size_t)(nr * K > 0 ? nr * K : 1));
    int8_t *cbs = malloc((size_t)(nc * K > 0 ? nc * K : 1));
    uint64_t *ram = malloc(sizeof(uint64_t) * (size_t)(nr * K * na > 0 ? nr * K * na : 1));
    uint64_t *cbm = malloc(sizeof(uint64_t) * (size_t)(nc * K * na > 0 ? nc * K * na : 1));
    int status = 0;

    /* steps 1-2: shared exponents and integer matrices (Eq. 1) */
#pragma omp parallel for schedule(dynamic, 1) reduction(min : status)
    for (int64_t r = 0; r < nr; r++) {
        int64_t i = rlist[r];
        er[r] = a_efix ? a_efix[i] : shared_exponent(&A, i * a_rs, a_cs, K, a_koff);
        for (int64_t k = 0; k < K; k++) {
            uint64_t *m = ram + (r * K + k) * na;
            ras[r * K + k] = (int8_t)integerize_entry(&A, i * a_rs + k * a_cs, p, ta,
                                                      a_koff ? a_koff[k] : 0, er[r], m, na);
            if (bn_bitlen(m, na) > ta + 1) status = -3;
        }
    }
#pragma omp parallel for schedule(dynamic, 1) reduction(min : status)
    for (int64_t c = 0; c < nc; c++) {
        int64_t j = clist[c];
        fc[c] = b_efix ? b_efix[j] : shared_exponent(&B, j * b_cs, b_rs, K, b_koff);
        for (int64_t k = 0; k < K; k++) {
            uint64_t *m = cbm + (c * K + k) * na;
            cbs[c * K + k] = (int8_t)integerize_entry(&B, k * b_rs + j * b_cs, p, tb,
                                                      b_koff ? b_koff[k] : 0, fc[c], m, na);
            if (bn_bitlen(m, na) > tb + 1) status = -3;
        }
    }
    if (e_out) for (int64_t i = 0; i < M; i++) if (rmap[i] >= 0) e_out[i] = er[rmap[i]];
    if (f_out) for (int64_t j = 0; j < N; j++) if (cmap[j] >= 0) f_out[j] = fc[cmap[j]];

    /* steps 3-4: exact c^ and the final rounding (Eq. 2) */
#pragma omp parallel for schedule(dynamic, 16) reduction(min : status)
    for (int64_t s = 0; s < nout; s++) {
        int64_t i = sel_i ? sel_i[s] : s / N;
        int64_t j = sel_i ? sel_j[s] : s % N;
        int64_t r = rmap[i], c = cmap[j];
        uint64_t pos[nacc], neg[nacc], mag[nacc];
        memset(pos, 0, sizeof pos);
        memset(neg, 0, sizeof neg);
        for (int64_t k = 0; k < K; k++) {
            int sa = ras[r * K + k], sb = cbs[c * K + k];
            if (!sa || !sb) continue;
            bn_addmul(sa * sb > 0 ? pos : neg, nacc, ram + (r * K + k) * na,
                      cbm + (c * K + k) * na, na);
        }
        int sgn;
        if (bn_cmp(pos, neg, nacc) >= 0) { bn_sub(pos, neg, mag, nacc); sgn = 1; }
        else { bn_sub(neg, pos, mag, nacc); sgn = -1; }
        int nb = bn_bitlen(mag, nacc);
        if (nb == 0) sgn = 0;
        if (chat_mag) {
            if (nb > 64 * nlc) { status = -1; }
            else {
                for (int l = 0; l < nlc; l++) chat_mag[s * nlc + l] = l < nacc ? mag[l] : 0;
                chat_sign[s] = (int8_t)sgn;
            }
        }
        if (c_limbs) {
            int64_t scale = (int64_t)er[r] + fc[c] - (int64_t)ta - tb;
            if (round_out(sgn, mag, nacc, scale, p, c_sign + s, c_exp + s, c_limbs + s * nl))
                if (status > -2) status = -2;
        }
    }
    free(rmap); free(cmap); free(rlist); free(clist); free(er); free(fc);
    free(ras); free(cbs); free(ram); free(cbm);
    return status;
}

/* The forward product: both sides at width t, exponents computed (Eqs. 1-3). */
int oz2o_gemm(int64_t M, int64_t N, int64_t K, int p, int t,
              const int8_t *As, const int32_t *Ae, const uint64_t *Al, int64_t a_rs, int64_t a_cs,
              const int8_t *Bs, const int32_t *Be, const uint64_t *Bl, int64_t b_rs, int64_t b_cs,
              int64_t nsel, const int64_t *sel_i, const int64_t *sel_j,
              int32_t *e_out, int32_t *f_out,
              int nlc, uint64_t *chat_mag, int8_t *chat_sign,
              int8_t *c_sign, int32_t *c_exp, uint64_t *c_limbs) {
    return oz2o_gemm_scaled(M, N, K, p, t, As, Ae, Al, a_rs, a_cs, NULL, NULL,
                            t, Bs, Be, Bl, b_rs, b_cs, NULL, NULL, nsel, sel_i, sel_j,
                            e_out, f_out, nlc, chat_mag, chat_sign, c_sign, c_exp, c_limbs);
}
