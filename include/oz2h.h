/*
 * oz2h.h -- C ABI of the MI355X (gfx950) Ozaki scheme II p-bit matrix product.
 *
 * C = A * B for p-bit floating-point matrices (p = 2 .. about 3300), computed
 * as in the paper's Algorithm section ("Overall flow"):
 *   (1) shared-exponent integer significands (Eqs. 1-3),
 *   (2) centred residues modulo pairwise-coprime moduli m_l <= 16191, balanced
 *       base-128 halves for moduli above 255 (subsection "(a) AMX-INT8 backend",
 *       the Karatsuba identity there),
 *   (3) exact INT8 x INT8 -> INT32 products, one per modulus (three for a
 *       two-limb modulus), reduced to u_l = c^ mod m_l,
 *   (4) direct CRT without multiple-precision division and the symmetric lift
 *       ("Direct CRT without multiple-precision division" subsection),
 *   (5) rescaling by 2^(e_i + f_j - 2t) and one round-to-nearest-even to p bits.
 * Every stage runs in HIP kernels on the GPU; nothing falls back to the CPU.
 *
 * Number format (the MPFR convention the paper uses, |x| < 2^exp):
 *   value = sign * mant * 2^(exp - p),  sign in {-1, 0, +1}  (0 means the number 0),
 *   mant = nl = ceil(p/64) little-endian uint64 limbs per element, mant < 2^p;
 *   bits at or above p in the top limb are ignored on input.  Results are
 *   normalised: 2^(p-1) <= mant < 2^p, or sign = 0, exp = 0, mant = 0.
 * Matrices are row-major with a leading dimension `ld` (in elements) shared by
 * the sign, exp and limb arrays: element (r, c) is at index r*ld + c, its limbs
 * at limbs[(r*ld + c)*nl ...].  OZ2H_OP_T means the stored matrix is op(X)^T.
 *
 * Conventions for every call:
 *   - Pointers to matrices, workspaces and outputs are DEVICE pointers owned by
 *     the caller; the library never frees them.  Plan and batched-plan handles
 *     are owned by the library and released by their destroy calls.
 *   - Argument checks happen on the host, synchronously, before anything is
 *     launched; a failed check returns a negative oz2h_status, launches
 *     nothing and sets the message returned by oz2h_last_error().  No C++
 *     exception crosses the ABI.
 *   - Compute calls are asynchronous on `stream` (0 = the null stream) and do
 *     not synchronise; a launch failure returns OZ2H_EDEVICE.
 *   - M or N equal to 0 is a successful no-op; oz2h_gemm with K = 0 writes the
 *     zero matrix, oz2h_gemm_integers rejects K = 0 (its plan has K >= 1).
 *   - Inputs must be normalised or zero in the sense above; exponents must lie
 *     in [-2^29, 2^29] so that no intermediate exponent overflows.
 */
#ifndef OZ2H_H
#define OZ2H_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OZ2H_OK = 0,
    OZ2H_EINVAL = -1,       /* bad argument (null pointer, bad shape, bad option)   */
    OZ2H_ERANGE = -2,       /* K > 133000, or p / t beyond the supported moduli set */
    OZ2H_ENOMEM = -3,       /* workspace too small, or plan tables not allocatable  */
    OZ2H_EDEVICE = -4,      /* a HIP call or kernel launch failed                   */
    OZ2H_EUNSUPPORTED = -5  /* the current device is not gfx950                     */
} oz2h_status;

typedef enum { OZ2H_OP_N = 0, OZ2H_OP_T = 1 } oz2h_op;

/* Block tile of the INT8 residue GEMMs (output rows x columns per block). */
typedef enum {
    OZ2H_TILE_AUTO = 0,     /* chosen from M and N (padding, occupancy)                 */
    OZ2H_TILE_128x128 = 1,  /* four waves of 64 x 64                                    */
    OZ2H_TILE_256x128 = 2,  /* four waves of 128 x 64                                   */
    OZ2H_TILE_128x256 = 3   /* four waves of 64 x 128                                   */
} oz2h_tile;

/* Options, the paper's oz2_opts (Implementation section, "Structure"). */
typedef struct {
    int32_t guard_bits;  /* g in t = p + g + ceil(log2 K) (Eq. 3); default 16          */
    int32_t t_bits;      /* 0: t from Eq. 3; otherwise the internal width t itself    */
    int32_t crt_margin;  /* moduli satisfy log2 P > 2t + ceil(log2 K) + margin; the
                            paper's implementation uses 2 (after Eq. crtcond)        */
    int32_t tile;        /* oz2h_tile of the residue GEMMs; default OZ2H_TILE_AUTO    */
    uint32_t flags;      /* OZ2H_FLAG_* bits below; default 0                        */
} oz2h_opts;

/*
 * Option flags.  By default stage 2 (residues) and stage 4 (direct CRT) run as
 * MFMA-free multi-limb integer kernels on the vector ALUs: exact fp64
 * multiply-adds of 32-bit words against 2^(32 w) mod m (residues), and of the
 * moduli weights v_l against balanced base-2^32 digits of P/m_l (CRT); only the
 * residue GEMMs use the INT8 matrix cores.  The two flags select, per plan, the
 * compared variants that cast these stages as INT8 contractions on the matrix
 * cores as well (the paper's "Faster residue conversion" direction):
 *   OZ2H_FLAG_RESIDUES_MMA  residues as (bytes of a^) x (256^j mod m) INT8
 *                           products; taken for integers of 8 or more 32-bit
 *                           words (t >= 224), the VALU kernel below that;
 *   OZ2H_FLAG_CRT_MMA       CRT digit sums as (bytes of v_l) x (bytes of P/m_l)
 *                           INT8 products; taken when the CRT has 16..32 digits
 *                           and L <= 127, the VALU kernel otherwise.
 * Both variants give bit-identical results.
 *
 * Backend flags (read when the plan is created; oz2h_plan_set_flags cannot change
 * them), following the paper's subsection "(b) binary64 backend" and its Future
 * Work item "Mixed backends":
 *   OZ2H_FLAG_BACKEND_F64    binary64 backend: moduli are the primes below
 *                            sqrt(2^55 / K) (Eq. fp64bound; also below 2^22) in
 *                            decreasing order, taken until Eq. crtcond holds; the
 *                            residues are exact binary64 values and each
 *                            modulus's product runs on the fp64 matrix cores
 *                            (exact: every partial sum is an integer below 2^53).
 *   OZ2H_FLAG_BACKEND_MIXED  INT8 one-limb moduli (largest first) for up to half
 *                            the bits Eq. crtcond needs, binary64 moduli for the
 *                            rest; one direct CRT over both.
 * The two exclude each other.  Since the CRT reconstructs the same exact integer
 * c^ from any moduli set with P large enough, every backend gives bit-identical
 * results.  Plans of these backends serve oz2h_gemm, oz2h_gemm_timed and
 * oz2h_gemm_integers; the other entry points need an INT8-backend plan
 * (OZ2H_EUNSUPPORTED otherwise).  Any other bit is rejected.
 */
#define OZ2H_FLAG_RESIDUES_MMA 0x1u
#define OZ2H_FLAG_CRT_MMA 0x2u
#define OZ2H_FLAG_BACKEND_F64 0x4u
#define OZ2H_FLAG_BACKEND_MIXED 0x8u

/* Input matrix (device pointers). */
typedef struct {
    const uint64_t *limbs;
    const int32_t *exp;
    const int8_t *sign;
    int64_t ld;
} oz2h_cmat;

/* Output matrix (device pointers). */
typedef struct {
    uint64_t *limbs;
    int32_t *exp;
    int8_t *sign;
    int64_t ld;
} oz2h_mat;

typedef struct oz2h_plan oz2h_plan;

typedef struct {
    int32_t p;          /* significand bits                                          */
    int32_t t;          /* internal width, Eq. 3                                     */
    int64_t K;          /* contraction length the moduli were chosen for            */
    int32_t L;          /* number of moduli (of both parts of a mixed plan)          */
    int32_t L1;         /* one-limb INT8 moduli (m <= 255), listed first             */
    int32_t L2;         /* two-limb INT8 moduli (255 < m <= 16191)                   */
    int32_t G;          /* GEMMs: INT8 GEMMs L1 + 3*L2, plus one per binary64 modulus */
    int32_t nw32;       /* 32-bit words of an integer significand (t+1 bits)         */
    int32_t nd32;       /* 32-bit digits of the CRT accumulator: ceil(log2 P/32) + 2 */
    double log2P;       /* log2 of the moduli product P                              */
    int32_t tw_a, tw_b; /* plans of oz2h_plan_create_grad: widths of the upstream
                           gradient for dA and dB (0 otherwise)                      */
    int64_t grad_M, grad_N; /* and the forward's M and N (0 otherwise)              */
    int32_t backend;    /* 0 INT8, 1 binary64, 2 mixed                               */
    int32_t Lf;         /* binary64 moduli (listed after the INT8 ones)              */
} oz2h_plan_info;

/* Default options: guard_bits 16, t_bits 0, crt_margin 2, tile AUTO, flags 0
   (MFMA-free residue and CRT stages). */
void oz2h_opts_default(oz2h_opts *o);

/* Message for the last failed call on this thread ("" if none). */
const char *oz2h_last_error(void);

/*
 * Moduli selection, host only (no device needed).  The set follows the
 * subsection "(a) AMX-INT8 backend" and Table "Moduli configuration": all 54
 * prime powers <= 255 (largest power of each prime), in decreasing order, then
 * the primes 255 < m <= 16191 in decreasing order, taken until
 * log2 P > 2t + ceil(log2 K) + crt_margin.  Writes L, L1, G, t and log2 P;
 * if `moduli` is non-null it must hold L entries (call once with NULL to size).
 * Returns OZ2H_ERANGE if K > 133000 (INT32 exactness, K*127^2 < 2^31) or the
 * required width exceeds what this library supports (at most 512 moduli).
 */
int oz2h_plan_moduli(int32_t p, int64_t K, const oz2h_opts *o, int32_t *L, int32_t *L1,
                     int32_t *G, int32_t *t, double *log2P, uint16_t *moduli);

/*
 * The same for every backend (o->flags may hold a backend flag; binary64 moduli
 * need 32 bits): writes L (all moduli), L8 (the INT8 moduli, listed first), G
 * (INT8 GEMMs plus one GEMM per binary64 modulus), t and log2 P, and the moduli
 * if `moduli` is non-null.  Errors as oz2h_plan_moduli.
 */
int oz2h_plan_moduli32(int32_t p, int64_t K, const oz2h_opts *o, int32_t *L, int32_t *L8,
                       int32_t *G, int32_t *t, double *log2P, uint32_t *moduli);

/*
 * Build the constant tables for precision p and contraction length K and
 * upload them to the CURRENT device (synchronous hipMalloc + hipMemcpy; the
 * only allocations the library itself makes).  The plan is then valid for
 * products with exactly that K on that device.  o may be NULL (defaults).
 */
int oz2h_plan_create(int32_t p, int64_t K, const oz2h_opts *o, oz2h_plan **out);

/*
 * Test/expert variant: explicit internal width t and an explicit list of L
 * pairwise-coprime moduli 2 <= m <= 16191 (e.g. the worked example's 5, 7, 9).
 * Moduli <= 255 are one-limb, larger ones two-limb; they are reordered so that
 * the one-limb moduli come first (oz2h_plan_get_moduli returns that order).
 * K is the contraction length the plan accepts.  The moduli must satisfy
 * Eq. crtcond with the least margin, P > 2^(2t + ceil(log2 K) + 1), so that
 * every |c^| <= K 2^(2t) is below P/2; otherwise OZ2H_ERANGE.  Options are the
 * defaults (flags 0); see oz2h_plan_set_flags.
 */
int oz2h_plan_create_custom(int32_t p, int32_t t, int64_t K, int32_t L, const uint16_t *moduli,
                            oz2h_plan **out);

/*
 * Replace the OZ2H_FLAG_* bits of a plan (the stage-2 / stage-4 kernel variants;
 * results are identical).  Host only; must not race with calls that launch with
 * the plan.  OZ2H_EINVAL for unknown bits.
 */
int oz2h_plan_set_flags(oz2h_plan *plan, uint32_t flags);

void oz2h_plan_destroy(oz2h_plan *plan);
int oz2h_plan_get_info(const oz2h_plan *plan, oz2h_plan_info *info);
/* The plan's moduli in the order the library uses (L entries); OZ2H_EUNSUPPORTED
   for a plan with binary64 moduli, whose moduli oz2h_plan_get_moduli32 returns. */
int oz2h_plan_get_moduli(const oz2h_plan *plan, uint16_t *moduli);
int oz2h_plan_get_moduli32(const oz2h_plan *plan, uint32_t *moduli);

/* Bytes of device workspace oz2h_gemm / oz2h_gemm_integers need for M x N. */
size_t oz2h_gemm_workspace_size(const oz2h_plan *plan, int64_t M, int64_t N);

/*
 * C = op(A) * op(B), op(A) M x K, op(B) K x N, p-bit in and out (the plan's p),
 * K must equal the plan's K.  Workspace: at least oz2h_gemm_workspace_size
 * bytes of device memory, 256-byte aligned; its contents are scratch.
 * C may not alias A or B.
 */
int oz2h_gemm(const oz2h_plan *plan, int64_t M, int64_t N, int64_t K,
              oz2h_op opA, oz2h_cmat A, oz2h_op opB, oz2h_cmat B, oz2h_mat C,
              void *workspace, size_t ws_bytes, hipStream_t stream);

/*
 * oz2h_gemm that also records five caller-created HIP events on `stream`:
 * events[0] before stage 1 (shared exponents), [1] before stage 2 (residues),
 * [2] before stage 3 (residue GEMMs), [3] before stages 4-5 (CRT and
 * rounding), [4] after the last kernel.  For per-stage timing; the events
 * must have been created on the current device and stay owned by the caller.
 * For M or N = 0 or K = 0 no event is recorded.
 */
int oz2h_gemm_timed(const oz2h_plan *plan, int64_t M, int64_t N, int64_t K,
                    oz2h_op opA, oz2h_cmat A, oz2h_op opB, oz2h_cmat B, oz2h_mat C,
                    void *workspace, size_t ws_bytes, hipStream_t stream, hipEvent_t *events);

/*
 * Parity entry point: the same pipeline, stopping after the CRT and lift
 * (stage 4).  Writes the exact integers c^_ij as chat_sign[i*N + j] in
 * {-1, 0, +1} and magnitude limbs chat_mag[(i*N + j)*nlc + l] (nlc limbs,
 * little-endian; nlc*64 must be >= log2 P), and the shared exponents
 * e[M], f[N] (0 for an all-zero row / column).  The output value is
 * c^_ij * 2^(e_i + f_j - 2t).
 */
int oz2h_gemm_integers(const oz2h_plan *plan, int64_t M, int64_t N, int64_t K,
                       oz2h_op opA, oz2h_cmat A, oz2h_op opB, oz2h_cmat B,
                       int8_t *chat_sign, uint64_t *chat_mag, int32_t nlc,
                       int32_t *e, int32_t *f,
                       void *workspace, size_t ws_bytes, hipStream_t stream);

/* ---------------- complex products ---------------- */

/*
 * Complex product C = op(A) op(B) with A = Ar + i Ai, B = Br + i Bi, each part a
 * p-bit matrix in the operand format (the paper's Conclusions and Future Work,
 * "Complex matrix products": the 3M/4M schemes reduce it to real products).
 * op is the plain transpose (no conjugation: to conjugate, negate the signs of
 * the imaginary part).
 *
 * Row i of op(A) owns one exponent over its real AND imaginary entries, column j
 * of op(B) likewise (Eq. 1), so that Re C_ij and Im C_ij are the exact integers
 *   sum_k ar^ br^ - ai^ bi^   and   sum_k ar^ bi^ + ai^ br^
 * each rounded once to p bits at the scale 2^(e_i + f_j - 2t): every entry is the
 * real Ozaki-II product of contraction length 2K of [Ar | Ai] with [Br ; -Bi] and
 * with [Bi ; Br].  The plan is therefore a plan for contraction length 2K
 * (oz2h_plan_create(p, 2K, ...), so t and the moduli follow Eqs. 3 and crtcond
 * for 2K products; K <= 66500).
 *
 * scheme 4 (4M): four residue GEMMs per modulus (Ar Br, Ai Bi, Ar Bi, Ai Br)
 * combined mod m_l in their epilogues.  scheme 3 (3M, Gauss): the residue planes
 * of Ar + Ai and Br + Bi are formed mod m_l from those of the parts, and three
 * GEMMs T1 = Ar Br, T2 = Ai Bi, T3 = (Ar + Ai)(Br + Bi) give Re = T1 - T2 and
 * Im = T3 - T1 - T2 mod m_l (a quarter fewer MFMA operations).  Both schemes give
 * bit-identical results: the combinations are exact in residue space.
 *
 * Cr and Ci are p-bit outputs (ld >= N) and may not alias any input or each
 * other.  Workspace: oz2h_zgemm_workspace_size(plan, scheme, M, N) bytes of device
 * memory, 256-byte aligned (about (2 or 3) G (M + N) K + 4 L M N bytes).  K = 0
 * writes zeros; M = 0 or N = 0 is a no-op.  Errors: OZ2H_EINVAL (scheme not 3 or
 * 4, a NULL pointer, ld too small, K not half the plan's K), OZ2H_ENOMEM (workspace
 * too small).  Asynchronous on `stream`.
 */
size_t oz2h_zgemm_workspace_size(const oz2h_plan *plan, int32_t scheme, int64_t M, int64_t N);
int oz2h_zgemm(const oz2h_plan *plan, int32_t scheme, int64_t M, int64_t N, int64_t K,
               oz2h_op opA, oz2h_cmat Ar, oz2h_cmat Ai, oz2h_op opB, oz2h_cmat Br, oz2h_cmat Bi,
               oz2h_mat Cr, oz2h_mat Ci, void *workspace, size_t ws_bytes, hipStream_t stream);

/* ---------------- operand reuse: residue handles ---------------- */

/*
 * Operand reuse (the paper's Conclusions and Future Work, "Operand reuse"): stages
 * 1-2 of one operand -- its shared exponents (Eq. 1) and its G INT8 residue planes
 * -- computed once and kept in a library-owned handle, so that products with many
 * right-hand sides (or left-hand sides) skip them.  Side A: X is op(A), rows x K,
 * each row owns an exponent; side B: X is op(B), K x rows, each column owns one.
 * The planes are bit-identical to those a plain call writes, so every product
 * from residues equals oz2h_gemm on the same operands bit for bit.
 */
typedef enum { OZ2H_SIDE_A = 0, OZ2H_SIDE_B = 1 } oz2h_side;
typedef struct oz2h_saved_residues oz2h_saved_residues;

/*
 * Computes the residues of X (stored as the op says: side A, op N: rows x K; side
 * B, op N: K x rows; OZ2H_OP_T the transposes) with the plan's moduli, into device
 * memory the handle owns (one hipMalloc of about G * round_up(rows, 256) *
 * round_up(K, 128) bytes).  The kernels run asynchronously on `stream`; the
 * handle is ready for launches ordered after them.  X is not read afterwards.
 */
int oz2h_residues_create(const oz2h_plan *plan, int32_t side, int64_t rows, oz2h_op op, oz2h_cmat X,
                         hipStream_t stream, oz2h_saved_residues **out);

/*
 * C = op(A) op(B) as oz2h_gemm, with side A taken from `ra` and/or side B from `rb`
 * (either may be NULL, not both; the operand of a side given by a handle is not
 * read and may be empty).  Each handle must come from a plan with the same p, t,
 * K and moduli on the same device, of side A with M rows / side B with N rows.
 * Workspace: oz2h_gemm_workspace_size(plan, M, N) bytes.
 */
int oz2h_gemm_from_residues(const oz2h_plan *plan, int64_t M, int64_t N, int64_t K,
                            const oz2h_saved_residues *ra, oz2h_op opA, oz2h_cmat A,
                            const oz2h_saved_residues *rb, oz2h_op opB, oz2h_cmat B, oz2h_mat C,
                            void *workspace, size_t ws_bytes, hipStream_t stream);

/* Frees the handle's memory; no launch that reads it may still be pending. */
void oz2h_residues_destroy(oz2h_saved_residues *r);

/* ---------------- without allocations ---------------- */

/*
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): oz2h_gemm without a
 * workspace argument.  Its scratch is a file-scope device array of
 * oz2h_gemm_noalloc_max_bytes() bytes (128 MiB) that every GPU the library runs on
 * holds until the process ends; the call itself allocates nothing (no hipMalloc,
 * hipFree or allocating library routine).  Products whose workspace
 * (oz2h_gemm_workspace_size) exceeds that size return OZ2H_ERANGE.  Every call on
 * one GPU shares that GPU's scratch: calls that overlap on one GPU (other streams,
 * other threads) race, so callers serialise them.  Nothing in the scratch needs to
 * start at zero (every stage writes what the next one reads).
 */
size_t oz2h_gemm_noalloc_max_bytes(void);
int oz2h_gemm_noalloc(const oz2h_plan *plan, int64_t M, int64_t N, int64_t K,
                      oz2h_op opA, oz2h_cmat A, oz2h_op opB, oz2h_cmat B, oz2h_mat C,
                      hipStream_t stream);

/* ---------------- autograd form: backward products ---------------- */

/*
 * Plan for a forward product C = A B (op(A) M x K, op(B) K x N) AND its two
 * backward products for an upstream gradient W = dL/dC (M x N, p bits):
 *   dA = W B^T (M x K)  and  dB = A^T W (K x N).
 * The paper defines no backward pass; the backward reuses the forward's
 * integer matrices (Eq. 1) by folding their scale factors into W:
 *   dA: h_i = max_j (exp W_ij + f_j), W'_ij = RNE(W_ij 2^(t_wA + f_j - h_i)),
 *       dA_ik = RNE_p( (sum_j W'_ij b^_kj) 2^(h_i - t_wA - t) );
 *   dB: g_j = max_i (exp W_ij + e_i), W''_ij = RNE(W_ij 2^(t_wB + e_i - g_j)),
 *       dB_kj = RNE_p( (sum_i a^_ik W''_ij) 2^(g_j - t_wB - t) ),
 * where a^, b^, e, f, t are the forward's and t_wA = p + g + ceil(log2 N),
 * t_wB = p + g + ceil(log2 M) (Eq. 3's rule for the backward contraction
 * lengths).  The moduli are the prefix of the oz2h_plan_moduli list with
 *   log2 P > max(2t + ceil(log2 K), t + t_wA + ceil(log2 N), t + t_wB + ceil(log2 M))
 *            + crt_margin,
 * so every |c^| < P/2 (Eq. crtcond for each product).  The plan also serves
 * oz2h_gemm / oz2h_gemm_integers with this K.  M, N <= 133000 (INT32
 * exactness of the backward GEMMs).
 */
int oz2h_plan_create_grad(int32_t p, int64_t M, int64_t N, int64_t K, const oz2h_opts *o,
                          oz2h_plan **out);

/* Bytes of device workspace oz2h_gemm_backward needs (0 for a plan of another kind). */
size_t oz2h_gemm_backward_workspace_size(const oz2h_plan *plan);

/*
 * Backward products from the saved forward.  `saved` is the workspace of a
 * completed oz2h_gemm or oz2h_gemm_integers call with this plan and these M, N
 * (earlier on `stream`, or synchronised); its exponents e, f and integer
 * residue planes are read, not written, so one forward serves any number of
 * backward calls.  W is M x N, not transposed.  dA (M x K) and dB (K x N) are
 * outputs; either pointer may be NULL to skip that product.  The residue
 * planes of the saved forward are re-laid out for the backward contractions
 * (over j for dA, over i for dB) by a transpose kernel into the workspace.
 */
int oz2h_gemm_backward(const oz2h_plan *plan, int64_t M, int64_t N, int64_t K,
                       const void *saved, size_t saved_bytes, oz2h_cmat W,
                       const oz2h_mat *dA, const oz2h_mat *dB,
                       void *workspace, size_t ws_bytes, hipStream_t stream);

/*
 * Float64 carriers of p-bit matrices, for frameworks whose differentiable
 * tensors must be floating point.  A carrier of a rows x cols matrix is a dense
 * rows x cols x (2 + 2 nl) array of doubles (nl = ceil(p/64)); element (r, c)
 * starts at carrier[(r*cols + c)*(2 + 2 nl)]:
 *   [0]           the value truncated to 53 bits (readable; +-inf or 0 outside
 *                 the double range), ignored by unpack;
 *   [1]           4 exp + sign + 1, an exact integer;
 *   [2+2l, 3+2l]  the low and high 32-bit halves of limb l, exact integers.
 * Every slot unpack reads is an exactly representable integer, so a carrier
 * survives any copy, view or device move bit for bit (but not arithmetic).
 * pack reads X (rows x cols, leading dimension X.ld); unpack writes X.  If
 * `bad` (a device int32, nullable) is given, unpack stores 1 there when an
 * element is not a valid encoding of a normalised p-bit number or zero; such
 * elements are written as zero.  It never clears `bad`.
 */
int oz2h_carrier_pack(int64_t rows, int64_t cols, int32_t p, oz2h_cmat X, double *carrier,
                      hipStream_t stream);
int oz2h_carrier_unpack(int64_t rows, int64_t cols, int32_t p, const double *carrier,
                        oz2h_mat X, int32_t *bad, hipStream_t stream);

/* ---------------- stage entry points (parity tests of single kernels) ---------------- */

/*
 * Stage 1, shared exponents (Eq. 1): out[r] = max exp(x) over the nonzero
 * entries of logical row r, 0 if the row is all zero.  Entry (r, k) of the
 * rows x count operand is at index r*rs + k*cs of sign/exp.
 */
int oz2h_exponents(int64_t rows, int64_t count, const int8_t *sign, const int32_t *exp,
                   int64_t rs, int64_t cs, int32_t *out, hipStream_t stream);

/*
 * Stage 2, residues (Eq. 1 integerization + centred residues + balanced
 * base-128 split).  For the logical rows x count operand (entry (r, k) at
 * index r*rs + k*cs of sign/exp, limbs at that index * nl) and its shared
 * exponents erow[rows], writes the plan's G int8 planes, plane g at
 * planes[g*rpad*kpad + r*kpad + k]; rows >= `rows` and columns >= `count`
 * are written as 0.  Plane order follows the moduli: one plane per one-limb
 * modulus (the centred residue), then three per two-limb modulus (r0, r1,
 * r0 + r1 with r = r0 + 128 r1, -64 <= r0 <= 63).  rpad must be a multiple of
 * 128 and >= rows, kpad a multiple of 128 and >= count.
 */
int oz2h_residues(const oz2h_plan *plan, int64_t rows, int64_t count,
                  const uint64_t *limbs, const int32_t *exp, const int8_t *sign,
                  int64_t rs, int64_t cs, const int32_t *erow,
                  int64_t rpad, int64_t kpad, int8_t *planes, hipStream_t stream);

/*
 * Stage 3, residue GEMMs, the fused reduction and the first step of the direct
 * CRT: for every modulus l, with c_l = sum_k A_l[i][k] B_l[j][k] (and, for a
 * two-limb modulus, the Karatsuba recombination P0 + 128 (Ps - P0 - P2) +
 * 16384 P2 of its three planes r0, r1, r0 + r1), writes
 *   v_l = c_l * (P/m_l)^-1 mod m_l   as a centred int16, |v_l| <= m_l / 2,
 * at v[l*mpad*npad + i*npad + j].  A planes are laid out as oz2h_residues
 * writes them (G x mpad x kpad), B planes as G x npad x kpad (K-contiguous,
 * i.e. B transposed).  mpad, npad multiples of the plan's tile (128 for
 * OZ2H_TILE_AUTO, which then picks a tile dividing them), kpad of 128.
 */
int oz2h_residue_gemm(const oz2h_plan *plan, int64_t mpad, int64_t npad, int64_t kpad,
                      const int8_t *a_planes, const int8_t *b_planes, int16_t *v,
                      hipStream_t stream);

/*
 * The bare exact INT8 GEMM (Step 3 of the tutorial section): C[i][j] =
 * sum_k A[i][k] B[j][k] in int32, A M x K and B N x K K-contiguous int8 with
 * leading dimension K; M, N multiples of the block tile (OZ2H_TILE_AUTO: 128),
 * K a multiple of 128, K <= 133000.
 */
int oz2h_i8gemm(int64_t M, int64_t N, int64_t K, const int8_t *A, const int8_t *B, int32_t *C,
                int32_t tile, hipStream_t stream);

/*
 * Stage 4, direct CRT + symmetric lift from plain residues ("Direct CRT without
 * multiple-precision division"): from u_l = c^ mod m_l (int16, any
 * representative with |u_l| < m_l, plane l at u[l*plane_stride + i*ldu + j])
 * reconstructs c^ with |c^| < P/2 as chat_sign[i*N + j] and nlc magnitude limbs
 * chat_mag[(i*N + j)*nlc + l].  Every c^ in (-P/2, P/2) is reconstructed, those
 * next to +-P/2 through the paper's alpha - 1 sequence; for even P the class of
 * P/2 comes back as +P/2.
 * Kernel: the plan's stage-4 variant (the matrix-core one under OZ2H_FLAG_CRT_MMA
 * where it applies).  For CRTs of more than 32 digits, a device workspace of
 * oz2h_crt_workspace_size(plan, M, ldu) bytes (256-byte aligned; scratch) selects
 * the row-broadcast VALU kernels, which need ldu % 16 == 0, plane_stride >=
 * M*ldu, plane_stride % 16 == 0 and u 32-byte aligned, and read all M*ldu
 * entries of every plane; workspace = NULL (or a layout outside these
 * conditions) takes the entry-per-thread VALU kernel.  A non-NULL workspace below
 * the size is OZ2H_ENOMEM.
 */
size_t oz2h_crt_workspace_size(const oz2h_plan *plan, int64_t M, int64_t ldu);
int oz2h_crt(const oz2h_plan *plan, int64_t M, int64_t N, const int16_t *u, int64_t ldu,
             int64_t plane_stride, int8_t *chat_sign, uint64_t *chat_mag, int32_t nlc,
             void *workspace, size_t ws_bytes, hipStream_t stream);

/* ---------------- batched form ---------------- */

/* One product of a batch: C = op(A) op(B) at precision p (device pointers). */
typedef struct {
    int64_t M, N, K;   /* op(A) is M x K, op(B) K x N; all >= 1, K <= 133000 */
    int32_t p;         /* significand bits of this product's A, B and C */
    int32_t opA, opB;  /* oz2h_op */
    oz2h_cmat A, B;
    oz2h_mat C;
} oz2h_problem;

typedef struct oz2h_batched_plan oz2h_batched_plan;

/*
 * Plan for `count` independent products (1 <= count <= 65535) of uneven
 * M, N, K and p.  Each product gets its own moduli set (the prefix of the list
 * of oz2h_plan_moduli that its p and K need) and constant tables, uploaded to
 * the current device now.  The pointers in `probs` are captured: the plan
 * always reads those inputs and writes those outputs.  A run executes, for all
 * products at once, one grouped launch per stage (shared exponents, residues,
 * and the CRT/rounding, the latter one launch per digit-chunk class) and the
 * residue GEMMs of all products and moduli as ONE persistent grouped launch
 * over a cost-sorted list of (product, modulus, output tile) work items (one
 * launch per block tile in use), ordered so that each XCD works on one rectangle
 * of every large (product, modulus) tile grid.  o->tile fixes the block tile of
 * every product; OZ2H_TILE_AUTO takes a previously tuned configuration for the
 * same shapes if the process has one (see oz2h_batched_tune), else the tile a
 * plain call would choose for each product, one block per work item.
 */
int oz2h_batched_plan_create(int32_t count, const oz2h_problem *probs, const oz2h_opts *o,
                             oz2h_batched_plan **out);
/* Device workspace bytes a run needs (256-byte aligned, contents scratch). */
size_t oz2h_batched_workspace_size(const oz2h_batched_plan *plan);
/*
 * Autotuner: times whole runs for every block tile setting of the grouped GEMM
 * (per product as plain calls choose, or 128x128, 256x128, 128x256 for all),
 * every persistent schedule (1, 2 or 4 resident blocks per compute unit, or one
 * block per work item) and both GEMM LDS depths (three stages, or two, which
 * leave room on a compute unit for the other chunk's residue and CRT blocks),
 * keeps the fastest, then times it replayed as a HIP graph against the same
 * launches issued directly and keeps the faster mode for oz2h_batched_run.  The
 * result goes to an in-process cache keyed by the batch's shapes (and, if the
 * environment variable OZ2H_TUNE_CACHE names a file, is appended there, one line
 * "signature tile blocks_per_cu stages graph"; plans created later with
 * OZ2H_TILE_AUTO pick it up, the file being read once per process; a later line for
 * the same signature wins, and lines that do not parse or hold values outside the
 * ranges of oz2h_batched_set_config and oz2h_batched_set_schedule are skipped).
 * Synchronizes `stream`; the runs write the outputs
 * C (with the product's results).
 */
int oz2h_batched_tune(oz2h_batched_plan *plan, void *workspace, size_t ws_bytes,
                      hipStream_t stream);
/*
 * Runs the whole batch.  In graph mode (the default, and the tuner's choice when it
 * measured replay faster) the launch sequence is captured on a private stream at
 * the first call (and again whenever the workspace pointer or the configuration
 * changes) and replayed on `stream`; otherwise the launches are issued directly on
 * `stream` (and on a second stream for the second chunk, joined by events), as
 * oz2h_batched_run_eager does.  Asynchronous.  Runs of one plan must not overlap
 * (they share the workspace and outputs).
 */
int oz2h_batched_run(oz2h_batched_plan *plan, void *workspace, size_t ws_bytes,
                     hipStream_t stream);
/* The same launches issued directly on `stream` (no graph). */
int oz2h_batched_run_eager(oz2h_batched_plan *plan, void *workspace, size_t ws_bytes,
                           hipStream_t stream);
/* Current block tile setting (oz2h_tile; OZ2H_TILE_AUTO: per product), resident blocks
   per compute unit (0: one block per work item instead of a persistent grid), GEMM work
   items (placeholders that keep the XCD alignment included). */
int oz2h_batched_get_config(const oz2h_batched_plan *plan, int32_t *tile, int32_t *blocks_per_cu,
                            int64_t *gemm_items);
/* Sets the tile setting (0..3) and blocks per compute unit (0..16) by hand. */
int oz2h_batched_set_config(oz2h_batched_plan *plan, int32_t tile, int32_t blocks_per_cu);
/* LDS stages of the grouped GEMM (2 or 3) and the mode of oz2h_batched_run (1: graph
   replay, 0: direct launches); the setter takes the same values, OZ2H_EINVAL otherwise. */
int oz2h_batched_get_schedule(const oz2h_batched_plan *plan, int32_t *gemm_stages, int32_t *graph);
int oz2h_batched_set_schedule(oz2h_batched_plan *plan, int32_t gemm_stages, int32_t graph);
void oz2h_batched_plan_destroy(oz2h_batched_plan *plan);

#ifdef __cplusplus
}
#endif

#endif /* OZ2H_H */
