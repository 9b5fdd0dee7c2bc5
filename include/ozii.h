/*
 * ozii -- Ozaki-scheme-II multiple-precision LU for AMD MI355X (gfx950).
 *
 * C ABI of the library libozii.so.  Every matrix is column-major and every
 * element is a non-overlapping expansion of nc binary64 components (nc = 2:
 * double-double, 3: triple-double, 4: quad-double; Sec. 2 of Kouya,
 * "Accelerating Multiple-Precision LU Decomposition with Ozaki Scheme II"):
 * component c of element (i, j) of a matrix X with leading dimension ld sits
 * at X[(i + j*ld)*nc + c].  All matrix, pivot and info pointers are DEVICE
 * pointers owned by the caller; the library never frees caller memory.  The
 * handle owns its plan tables and workspace.
 *
 * Asynchrony: every call is enqueued on the handle's HIP stream and returns
 * without waiting.  Host-detectable problems (bad sizes, null pointers, plans
 * that do not fit) are reported synchronously before anything is enqueued.
 * Data-dependent conditions (an exactly zero pivot) are reported through the
 * device `info` word, LAPACK style.
 *
 * Threads: one handle per host thread.
 */
#ifndef OZII_H
#define OZII_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  OZII_OK = 0,
  OZII_EINVAL = 1,       /* bad argument (size, pointer, leading dimension) */
  OZII_ECAPACITY = 2,    /* the requested plan exceeds the CRT capacity      */
  OZII_EOVERFLOW = 3,    /* a forced plan breaks an accumulator bound        */
  OZII_ENOMEM = 4,       /* workspace allocation failed                      */
  OZII_EHIP = 5,         /* a HIP runtime call failed                        */
  OZII_EUNSUPPORTED = 6, /* format or option not built into this library     */
  OZII_EDEVICE = 7       /* a kernel reported an internal error (see text)   */
} ozII_status;

/* Back-ends of (S3)/(S4).  All three give bit-identical products at equal
 * (S, w): the digit-group sums are exact integers either way.
 *   INT8:  the 54 largest prime powers <= 256 (Sec. 3.2), int8 residues,
 *          exact int32 MFMA accumulation (K S 128^2 < 2^31);
 *   FP8:   the same moduli, every residue split into balanced base-17 digits
 *          (Eq. fp8digits) stored as E4M3, four sub-products per pair with
 *          exact FP32 accumulation;
 *   F64:   the 20 largest primes m with K S m^2 < 2^53 (Eq. fp64mod),
 *          residues in binary64, exact FP64 MFMA accumulation;
 *   FP16:  the INT8 moduli and residue planes, one product per modulus on
 *          the FP16 engine (Sec. 4.1.3): residues converted to f16 in
 *          registers, FP32 partial sums of at most 1024 products (exact,
 *          Eq. fp16cond per chunk) folded into int32.
 * AUTO currently means INT8. */
typedef enum {
  OZII_BE_AUTO = 0,
  OZII_BE_INT8 = 1,
  OZII_BE_FP8_B17 = 2,
  OZII_BE_F64MOD = 3,
  OZII_BE_FP16 = 4
} ozII_backend;

typedef enum {
  OZII_METHOD_OZAKI = 0, /* Schur update by the Ozaki-II product              */
  OZII_METHOD_NAIVE = 1  /* Schur update by expansion multiply-subtracts       */
} ozII_method;

typedef enum {
  OZII_TILE_AUTO = 0,    /* 256x128 when it gives 2 workgroups per CU, else 128x128 */
  OZII_TILE_128x128 = 1, /* 4 wavefronts of 64x64, operands straight from L2  */
  OZII_TILE_256x128 = 2, /* 4 wavefronts of 128x64, operands staged in LDS    */
  OZII_TILE_256x256 = 3  /* 8 wavefronts of 128x64, operands staged in LDS    */
} ozII_gemm_tile;

/* Options.  A null pointer means all defaults (zero). */
typedef struct {
  int32_t backend;      /* ozII_backend                                        */
  int32_t nslice;       /* force the slice count S; 0 = plan rule (Sec. 3.2)   */
  int32_t extra_groups; /* keep this many digit groups below S-1 (Sec. 3.2)    */
  int32_t guard_ex;     /* extra guard bits g_ex added to the slack (Sec. 3.2) */
  int32_t block;        /* getrf panel width b; 0 = 256                        */
  int32_t method;       /* getrf Schur update: ozII_method                     */
  int32_t flags;        /* OZII_F_* bits below; 0 = defaults                   */
  int32_t gemm_tile;    /* (S4) workgroup tile: ozII_gemm_tile; the residue   */
                        /* planes are padded to it.  Results do not depend on */
                        /* it (exact integer products).                       */
  int32_t qbits;        /* > 0: the unsliced product of Sec. 3.1 at a stated  */
                        /* scaling, |a_bar|, |b_bar| < 2^qbits (S = 1, Q =    */
                        /* qbits + 1) with N_mod the fewest moduli covering   */
                        /* the CRT range 2 K 2^(2 qbits); 0 = plan rule.      */
                        /* Needs nslice <= 1 and no extra groups (EINVAL).    */
  int32_t panel_leaf;   /* ozII_getrf_limbs: > 0 = recursive panel and U12    */
                        /* solve down to this many columns / rows, their      */
                        /* inner updates by the Schur update's method (the    */
                        /* Ozaki-II panel of Sec. 5.2); 0 = unblocked panel   */
                        /* and row-by-row solve.                              */
} ozII_opts;

/* ozII_opts.flags.  OZII_F_NO_LOOKAHEAD: getrf runs each Schur update as
 * one product after its panel, instead of updating the next panel's columns
 * first and the rest on a side stream while the next panel is factored
 * (the default).  The results are the same bit for bit. */
#define OZII_F_NO_LOOKAHEAD 1
/* OZII_F_FUSED: on the INT8 back-end, run (S4)-(S6) of each product as one
 * kernel per 32 x 32 output tile that keeps the tile's t-values (Eq. crt)
 * in LDS, instead of a batched GEMM writing t-planes to HBM and a separate
 * consumer.  Plans of more than 120 (group, modulus) products, and the stage
 * hooks, use the unfused kernels.  The results are the same bit for bit. */
#define OZII_F_FUSED 2

typedef struct ozII_ctx *ozII_handle;

/* Create a handle on HIP device `device`, enqueueing on `stream` (a
 * hipStream_t; null = the default stream). */
ozII_status ozII_create(ozII_handle *h, int device, void *stream);
ozII_status ozII_destroy(ozII_handle h);
ozII_status ozII_set_stream(ozII_handle h, void *stream);

/* Plan of Sec. 3.2 ("Determining w and N") for precision p bits and inner
 * dimension K: slice count S, slice width w, fixed-point width Q = w S,
 * number of moduli nmod and the moduli themselves (up to 64 entries written).
 * Host only; returns OZII_ECAPACITY when no slice count fits. */
ozII_status ozII_plan_query(int32_t p, int64_t K, const ozII_opts *o, int32_t *S, int32_t *w,
                            int32_t *Q, int32_t *nmod, int32_t *moduli);

/* Grow the workspace so that products up to M x N x K and LUs up to order n
 * (panel width b) run without allocation (needed before graph capture). */
ozII_status ozII_reserve(ozII_handle h, int32_t nc, int64_t M, int64_t N, int64_t K, int64_t n,
                         const ozII_opts *o);

/* Ozaki-II product, steps (S1)-(S6) of Sec. 3.1 with the slices of Sec. 3.2:
 *   mode 0: C = A B,   mode 1: C = C - A B,
 * A is M x K (lda >= M), B is K x N (ldb >= K), C is M x N (ldc >= M).  The
 * product is rounded once (greedy round-to-nearest expansion of the exact
 * integer result); mode 1 then subtracts with expansion addition. */
ozII_status ozII_gemm(ozII_handle h, int32_t mode, int32_t nc, int64_t M, int64_t N, int64_t K,
                      const double *A, int64_t lda, const double *B, int64_t ldb, double *C,
                      int64_t ldc, const ozII_opts *o);

/* ozII_gemm for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid allocation).
 * Same arguments, operations and results as ozII_gemm (bit for bit), but
 * the plan tables and the workspace live in a static device array that the
 * library reserves once per GPU it runs on and holds until the process ends
 * (64 MiB: eight plan slots of 32 KiB, the rest workspace); the call makes
 * no hipMalloc or hipFree and creates no event (profiling records nothing
 * for it).  The first use of a plan (p, K, options) copies its tables into
 * a slot on the handle's stream; a ninth distinct plan evicts the oldest.
 * Limit: the product's workspace -- about 4 (M + N) + S N_mod b_r (Mp + Np)
 * Kp + ng N_mod b_t Mp Np bytes, Mp, Np rounded up to 128 or 256, Kp to 64
 * or 128, b_r / b_t the residue / t-value bytes of the back-end -- must fit
 * ozII_gemm_noalloc_capacity() bytes (e.g. QD with M = N = K = 512, or
 * M = N = 1024 with K = 64); larger products return OZII_EINVAL before
 * anything is enqueued.  All calls on one GPU share its array, which keeps
 * the last call's contents: calls that overlap on one GPU (other streams,
 * other handles, other host threads) race and give undefined results.
 * Errors: those of ozII_gemm; OZII_EINVAL for a product beyond the
 * capacity; OZII_EHIP if the array could not be mapped on this device. */
ozII_status ozII_gemm_noalloc(ozII_handle h, int32_t mode, int32_t nc, int64_t M, int64_t N,
                              int64_t K, const double *A, int64_t lda, const double *B,
                              int64_t ldb, double *C, int64_t ldc, const ozII_opts *o);
/* Workspace bytes available to ozII_gemm_noalloc (host only). */
ozII_status ozII_gemm_noalloc_capacity(int64_t *bytes);

/* Arbitrary-precision limb matrices (the MPFR-like input of Sec. 3.3 and
 * the p-bit results of (S6)), p = 64 nlimb bits, 1 <= nlimb <= 64 for the
 * LU, its solve and the element arithmetic, up to OZII_GEMM_LIMBS_MAX for
 * the product (p <= 16384, the range of Sec. 4.1.6's back-end comparison):
 *   x = (-1)^sign * (sum_q limb_q 2^(64 q)) * 2^(exp - p),
 * mantissa normalised (bit 63 of limb nlimb-1 set, i.e. x = 0.m 2^exp as
 * mpfr_get_exp reports it); zero has every limb 0 (on input exp and sign are
 * then ignored; outputs write exp = INT32_MIN, sign = 0).  Non-zero
 * exponents must lie in [-2^30, 2^30] (MPFR's default range); inputs that
 * are not normalised give undefined results.  All arrays are device memory
 * owned by the caller; element (i, j) of an M-row matrix:
 *   limb q at limb[q * plane + i + j * ld]   (one plane per limb: SoA)
 *   exp[i + j * ld], sign[i + j * ld] (0 positive, 1 negative),
 * with ld >= rows and plane >= ld * cols. */
typedef struct {
  uint64_t *limb;
  int32_t *exp;
  uint8_t *sign;
  int64_t ld;
  int64_t plane;
} ozII_limbs;
#define OZII_GEMM_LIMBS_MAX 256

/* Ozaki-II product on limb matrices, steps (S1)-(S6) of Sec. 3.1 with the
 * slices of Sec. 3.2, on the INT8 back-end (default) or the binary64 moduli
 * (o->backend = OZII_BE_F64MOD; Sec. 4.1.6 compares the two over p):
 *   mode 0: C = RN_p(A B),   mode 1: C = RN_p(C - RN_p(A B)),
 * RN_p: round to nearest, ties to even (MPFR's RNDN), applied once to the
 * exact integer result of (S5) and once to the update.  (S2) truncates:
 * X = sgn(x) trunc(|x| 2^mu) (mpfr_mul_2si then mpfr_get_z toward zero).
 * A is M x K, B is K x N, C is M x N; C must not overlap A or B.
 * Errors: OZII_EINVAL (bad sizes, null pointers, nlimb outside
 * 1..OZII_GEMM_LIMBS_MAX, ld or plane too small), OZII_EUNSUPPORTED (a
 * back-end other than INT8 or binary64 moduli, or a plan beyond the compiled
 * sizes), OZII_ENOMEM.  Uses handle workspace of about (M + N) K S N_mod e +
 * M N (ng N_mod t + 4 * words) bytes (e = 1, t = 1 on INT8; e = 8, t = 4 on
 * the binary64 moduli). */
ozII_status ozII_gemm_limbs(ozII_handle h, int32_t mode, int32_t nlimb, int64_t M, int64_t N,
                            int64_t K, const ozII_limbs *A, const ozII_limbs *B, ozII_limbs *C,
                            const ozII_opts *o);

/* ozII_gemm_limbs with the group sums of (S5) copied out (parity hook):
 * sbar (device, may be null) receives, per retained digit group gi and
 * element (i, j), Sbar_(g0+gi) of Eq. (crt) as nlimb_out (1..6) 64-bit
 * two's-complement limbs, layout [ng][N][M][nlimb_out], computed by the CRT
 * routine the limb consumer itself runs.  Errors: those of
 * ozII_gemm_limbs; OZII_EINVAL for nlimb_out outside 1..6. */
ozII_status ozII_gemm_limbs_stages(ozII_handle h, int32_t mode, int32_t nlimb, int64_t M,
                                   int64_t N, int64_t K, const ozII_limbs *A,
                                   const ozII_limbs *B, ozII_limbs *C, const ozII_opts *o,
                                   uint64_t *sbar, int32_t nlimb_out);

/* Blocked right-looking LU with partial pivoting (Sec. 3.4) on an n x n limb
 * matrix (the layout above), in place.  Per panel of b = o->block columns
 * (0 = 256): the unblocked panel -- pivot = the entry of largest exact
 * magnitude at or below the diagonal, ties to the lowest row; rows
 * interchanged across the panel; l = RN_p(a / pivot); a = RN_p(a -
 * RN_p(l u)) on the panel's remaining columns --, the panel's interchanges
 * on the other columns, U12 = L11^-1 U12 by the same multiply-subtracts,
 * then the Schur update A22 = RN_p(A22 - RN_p(L21 U12)) by the Ozaki-II
 * product of ozII_gemm_limbs (o->method = OZII_METHOD_OZAKI, plan for
 * K = b) or by multiply-subtracts RN_p(a - RN_p(l_ik u_kj)), k ascending
 * (OZII_METHOD_NAIVE, which gives the unblocked LU bit for bit for any b).
 * RN_p rounds to nearest, ties to even, like MPFR's RNDN (the number type
 * of Sec. 2).  ipiv (device int64, n entries, 0-based, LAPACK semantics)
 * and *info (device int32, first j+1 with an exactly zero pivot, else 0);
 * a zero pivot skips its column's division and update.  Errors:
 * OZII_EINVAL (bad sizes, null pointers, bad descriptor, nlimb outside
 * 1..64, unknown method), OZII_EUNSUPPORTED (a back-end other than INT8,
 * or a plan beyond the compiled sizes), OZII_ENOMEM, OZII_EHIP. */
ozII_status ozII_getrf_limbs(ozII_handle h, int32_t nlimb, int64_t n, ozII_limbs *A,
                             int64_t *ipiv, int32_t *info, const ozII_opts *o);

/* Solve A X = B from ozII_getrf_limbs's factors by forward and backward
 * substitution (Sec. 4.3): the interchanges ipiv[0..n) applied to B in
 * order, then element i takes RN_p(x_i - RN_p(l_ik x_k)) for k ascending,
 * and RN_p(x_i - RN_p(u_ik x_k)) for k descending with x_k = RN_p(x_k /
 * u_kk) once its updates are in (an exactly zero u_kk gives x_k = 0).  LU
 * is the n x n factor matrix, B an n x nrhs limb matrix (element (i, r) at
 * index i + r ld), overwritten by X; device memory owned by the caller.
 * Errors: OZII_EINVAL (bad sizes, null pointers, bad descriptors,
 * nlimb outside 1..64), OZII_EHIP. */
ozII_status ozII_getrs_limbs(ozII_handle h, int32_t nlimb, int64_t n, int64_t nrhs,
                             const ozII_limbs *LU, const int64_t *ipiv, ozII_limbs *B);

/* The p-bit arithmetic of the limb LU element by element (parity hook; the
 * correctly rounded operations of the number type of Sec. 2): C_t =
 * RN_p(A_t op B_t) for t < count, op 0 add, 1 subtract, 2 multiply,
 * 3 divide (a zero divisor gives 0).  A, B, C are vectors: element t at
 * index t of every plane.  Errors: OZII_EINVAL (bad op, sizes or
 * descriptors), OZII_EHIP. */
ozII_status ozII_limbs_arith(ozII_handle h, int32_t op, int32_t nlimb, int64_t count,
                             const ozII_limbs *A, const ozII_limbs *B, ozII_limbs *C);

/* Same product with the intermediate stages copied out (parity hooks); any
 * output pointer may be null.  Sizes follow ozII_gemm_stage_dims:
 *   ea[M], eb[N]     (S1) row / column exponents (INT32_MIN for zero);
 *   planesA          (S3) residue planes of Mp x Kp elements, planesB of
 *                    Np x Kp, in MFMA fragment order: 1 KiB blocks of 16 rows
 *                    (lane l of a block holds row l%16), blocks ordered
 *                    (row block, k block).  Per back-end:
 *                      INT8: S*nmod planes of int8 residues, a block spans
 *                            64 k (lane l: k 16(l/16) .. +16);
 *                      FP8:  2*S*nmod planes (digit d0, then d1, of Eq.
 *                            fp8digits, per slice and modulus) of OCP E4M3
 *                            bytes, blocks as INT8;
 *                      F64:  S*nmod planes of residues as doubles, a block
 *                            spans 8 k (lane l: k l/16 and 4 + l/16);
 *   tpl              (S4) t-planes [ng][nmod][Np][Mp], uint8 (INT8, FP8) or
 *                    uint32 (F64);
 *   sbar             (S5) group sums, nlimb (1..6) 64-bit two's-complement
 *                    limbs per element, layout [ng][N][M][nlimb], computed by
 *                    the CRT routine of the consumer that reads these
 *                    t-planes (the byte-column CRT with its column sums on
 *                    the matrix cores for INT8, FP8 and FP16, the binary64
 *                    CRT for binary64 moduli). */
ozII_status ozII_gemm_stages(ozII_handle h, int32_t mode, int32_t nc, int64_t M, int64_t N,
                             int64_t K, const double *A, int64_t lda, const double *B,
                             int64_t ldb, double *C, int64_t ldc, const ozII_opts *o,
                             int32_t *ea, int32_t *eb, void *planesA, void *planesB,
                             void *tpl, uint64_t *sbar, int32_t nlimb);
ozII_status ozII_gemm_stage_dims(int32_t nc, int64_t M, int64_t N, int64_t K, const ozII_opts *o,
                                 int64_t *Mp, int64_t *Np, int64_t *Kp, int32_t *S,
                                 int32_t *nmod, int32_t *ng);

/* Blocked right-looking LU with partial pivoting (Sec. 3.4), in place on the
 * n x n matrix A.  ipiv[j] (0-based, device int64) = row interchanged with row
 * j (LAPACK semantics); *info (device int32) = first j+1 with an exactly zero
 * pivot, else 0.  o->method selects the Schur update (Ozaki-II or native). */
ozII_status ozII_getrf(ozII_handle h, int32_t nc, int64_t n, double *A, int64_t lda,
                       int64_t *ipiv, int32_t *info, const ozII_opts *o);

/* Solve A X = B from getrf's factors by forward and backward substitution
 * (Sec. 4.3, the solve of the Lotkin experiment; P A = L U of Sec. 3.4):
 * the interchanges ipiv[0..n) applied to B in order (LAPACK's laswp), then
 * forward substitution with the unit lower factor (element i takes
 * x_i (+) -(l_ik (x) x_k) for k ascending) and backward substitution with the
 * upper factor (element i takes x_i (+) -(u_ik (x) x_k) for k descending;
 * x_k is divided by u_kk with the expansion division once all of its
 * updates are in).  LU is the n x n output of ozII_getrf (lda >= n), ipiv
 * its pivot vector (device int64, n entries, 0-based), B is n x nrhs
 * (ldb >= n), overwritten by X; all device memory owned by the caller.  An
 * exactly zero u_kk (info > 0 from getrf) gives non-finite components, as
 * the division of the specification does.  Errors: OZII_EINVAL (null
 * pointers, negative sizes, leading dimensions below n), OZII_EUNSUPPORTED
 * (nc outside 2..4); OZII_EDEVICE is reported by ozII_sync_check if a
 * bounded wait of the pipelined one-column solve timed out. */
ozII_status ozII_getrs(ozII_handle h, int32_t nc, int64_t n, int64_t nrhs, const double *LU,
                       int64_t lda, const int64_t *ipiv, double *B, int64_t ldb);

/* Batched LU + solve of many independent small systems in one persistent
 * launch: per system the LU with partial pivoting of Sec. 3.4 and the solve
 * by forward and backward substitution of Sec. 4.3.  Each item is an n x n
 * matrix of nc-component expansions (column-major, lda = n, device memory,
 * factored in place), an optional right-hand side b of n expansions
 * (device; overwritten by the solution), ipiv (device, n entries, 0-based
 * LAPACK semantics) and info (device, one int32).  Items may mix DD / TD /
 * QD and orders.  Every item is factored by one workgroup with the
 * unblocked right-looking LU (partial pivoting) and the native expansion
 * update -- per element the operations of ozII_getrf with block = 1,
 * method = native -- then solved as ozII_getrs does.
 *
 * ozII_batch_prepare (host, synchronous) validates the items, orders them by
 * decreasing cost nc n^3 (longest first) and uploads the table into
 * handle-owned device memory, replacing any previous batch; ozII_batch_run
 * enqueues the queue reset and the persistent kernel on the handle's stream,
 * allocates nothing and may be captured in a hipGraph.  times (device, may be
 * null) receives 2 per item in the caller's item order: the 100 MHz
 * real-time counter when its workgroup started and when it finished.
 * The caller's buffers must stay allocated while the batch is in use.
 * Errors: OZII_EINVAL for a bad item (nc outside 2..4, n < 1 or > 4096, null
 * A/ipiv/info); OZII_ENOMEM when the table cannot be allocated. */
typedef struct {
  int32_t nc;
  int32_t reserved;
  int64_t n;
  double *A;
  double *b;
  int64_t *ipiv;
  int32_t *info;
} ozII_batch_item;

ozII_status ozII_batch_prepare(ozII_handle h, int32_t count, const ozII_batch_item *items);

/* ozII_batch_prepare with options.  o == NULL or o->method ==
 * OZII_METHOD_NAIVE: as ozII_batch_prepare.  o->method == OZII_METHOD_OZAKI:
 * every item is factored by one workgroup with the blocked LU of ozII_getrf
 * (panel width b = o->block, default 32, at most 256) whose Schur updates run
 * the Ozaki-II product of Sec. 3.1-3.3 inside the workgroup on the INT8
 * back-end (plans at K = b, honouring o->nslice / extra_groups / guard_ex):
 * per element the operations of ozII_getrf with the same o, so factors,
 * pivots and info agree with it bit for bit; then the solve as above.  The
 * handle allocates one scratch slot per workgroup here (exponents, residue
 * planes of L21 and U12, t-planes: about ng nmod (n - b)^2 bytes for the
 * largest item), so ozII_batch_run still allocates nothing.
 * Errors: those of ozII_batch_prepare; OZII_EUNSUPPORTED for b > 256, an item
 * of order above 1024, a back-end other than INT8 / AUTO, or a plan beyond
 * the compiled word sizes; OZII_ENOMEM when the scratch cannot be allocated. */
ozII_status ozII_batch_prepare_ex(ozII_handle h, int32_t count, const ozII_batch_item *items,
                                  const ozII_opts *o);
ozII_status ozII_batch_run(ozII_handle h, uint64_t *times);

/* Autotuner (the tuning step of Sec. 4.1, "only timing at the actual size is
 * trustworthy"), for nc-component expansions and order n.  Stage 1 times the
 * panel width b (64, 128, 256, 512 below n) x the Schur update -- one of the
 * three back-ends or the native expansion update -- x the schedule (with or
 * without OZII_F_NO_LOOKAHEAD); stage 2 times the winner (if Ozaki-II) with
 * the slice count S one above the plan rule's minimum (Eq. Lhint trades
 * slices against conversion cost) and, on the INT8 back-end, with each GEMM
 * tile and with OZII_F_FUSED (taken only when at least 3 % faster than the
 * best unfused candidate).  Candidates are ordered by a cost model (engine throughput x bits
 * per modulus, plane and t-plane traffic, panel cost) and every one is timed
 * with HIP events around ozII_getrf of a synthetic diagonally dominant n x n
 * matrix on the handle's stream; the fastest is returned in *best (block,
 * backend, method, nslice, gemm_tile, flags; other fields 0).  Candidates
 * the library cannot run at this size (OZII_EUNSUPPORTED: a panel that does
 * not fit in LDS, a plan beyond the compiled word sizes) are skipped; the
 * report lists the timed ones.
 * With a cache path (host file, JSON array with one object per line, keyed by
 * the device's architecture name, nc and n) a cached choice is returned
 * without timing unless OZII_TUNE_RETUNE is set, and a new choice is stored.
 * Allocates a scratch matrix of n*n*nc doubles for the duration of the call
 * and synchronises the stream; rep may be null. */
#define OZII_TUNE_RETUNE 1
#define OZII_TUNE_MAXCAND 40
typedef struct {
  int32_t ncand;                         /* candidates timed (1 when cached)     */
  int32_t best;                          /* index of the choice                  */
  int32_t from_cache;                    /* 1: taken from the cache file          */
  int32_t reserved;
  ozII_opts cand[OZII_TUNE_MAXCAND];     /* the candidates, in model order       */
  double ms[OZII_TUNE_MAXCAND];          /* measured getrf time [ms]             */
  double model_ms[OZII_TUNE_MAXCAND];    /* the model's estimate [ms]            */
} ozII_tune_report;

ozII_status ozII_tune(ozII_handle h, int32_t nc, int64_t n, const char *cache_path,
                      int32_t flags, ozII_opts *best, ozII_tune_report *rep);

/* Autotuner of ozII_getrf_limbs (Sec. 4.1's timing at the actual size; the
 * tuning of the limb format that Sec. 5.2 asks for) for nlimb-limb numbers
 * and order n.  Stage 1 times the panel width b (64, 128, 256, 512 below n)
 * x the panel leaf (0 = unblocked panel, 16, 32, 64 below b) with the
 * Ozaki-II update, and the native update (unblocked panel) at each b while
 * n <= 512; stage 2 times the winner with each GEMM tile and with S one
 * above the plan rule's.  Each candidate is timed with HIP events around
 * ozII_getrf_limbs of a synthetic random n x n limb matrix on the handle's
 * stream (a warm-up run first); *best receives block, backend, method,
 * panel_leaf, nslice and gemm_tile.  Cache and report as ozII_tune (key:
 * architecture, nlimb, n).  Allocates n*n*(8 nlimb + 5) bytes for the
 * duration of the call and synchronises the stream.  Errors: OZII_EINVAL
 * (nlimb outside 1..64, n outside 2..32768, unknown flags),
 * OZII_ENOMEM, OZII_EHIP, OZII_EUNSUPPORTED (no candidate runs). */
ozII_status ozII_tune_limbs(ozII_handle h, int32_t nlimb, int64_t n, const char *cache_path,
                            int32_t flags, ozII_opts *best, ozII_tune_report *rep);

/* The HIP stream the handle enqueues on (as a void*). */
ozII_status ozII_stream_of(ozII_handle h, void **stream);

/* Wait for the handle's stream and report a device-side error flag raised by
 * a kernel (a grid barrier that did not complete). */
ozII_status ozII_sync_check(ozII_handle h);

/* Per-stage timing.  When on, every kernel launch of the library is
 * bracketed by HIP events recorded on the handle's stream; ozII_profile_read
 * waits for the stream and returns, per stage, the summed event time [ms],
 * the number of launches, and the algorithmic bytes and operations of those
 * launches (what the method itself must move / compute), then clears the
 * record.  Stages: 0 exponents, 1 residue producer, 2 modular GEMM,
 * 3 CRT + rounding + update, 4 panel, 5 row interchanges, 6 U12 solve,
 * 7 native expansion update, 8 getrs.  Arrays have nstages entries (any may
 * be null). */
ozII_status ozII_set_profiling(ozII_handle h, int32_t on);
ozII_status ozII_profile_read(ozII_handle h, int32_t nstages, double *ms, int64_t *launches,
                              double *bytes, double *ops);

const char *ozII_status_string(ozII_status s);
const char *ozII_last_error(ozII_handle h);

#ifdef __cplusplus
}
#endif

#endif /* OZII_H */
