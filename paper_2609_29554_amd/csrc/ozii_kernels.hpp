// Host-side launchers of the HIP kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/ozii.h"

namespace ozk {
struct DevPlan;
}

namespace ozl {
using ozk::DevPlan;

// (S4) GEMM workgroup tiles (values of ozII_opts.gemm_tile)
enum { GEMM_TILE_AUTO = 0, GEMM_TILE_128x128 = 1, GEMM_TILE_256x128 = 2, GEMM_TILE_256x256 = 3 };

inline bool gemm_tile_fits(int tile, int64_t Mp, int64_t Np) {
  switch (tile) {
    case GEMM_TILE_128x128: return Mp % 128 == 0 && Np % 128 == 0;
    case GEMM_TILE_256x128: return Mp % 256 == 0 && Np % 128 == 0;
    case GEMM_TILE_256x256: return Mp % 256 == 0 && Np % 256 == 0;
    default: return false;
  }
}

// The 256x128 tile (three 24 KiB stages: two workgroups per CU overlap each
// other's barriers) when it still gives every CU two workgroups (prods =
// batched (group, modulus) products), else 128x128.  Measured on MI355X it
// beats the 256x256 tile (one workgroup per CU) on both the TD 4096^3
// product and the p = 4096 limb updates; 256x256 stays selectable.
inline int gemm_tile_auto(int64_t prods, int64_t Mp, int64_t Np) {
  if (gemm_tile_fits(GEMM_TILE_256x128, Mp, Np) && prods * (Mp / 256) * (Np / 128) >= 512)
    return GEMM_TILE_256x128;
  return GEMM_TILE_128x128;
}

// C = 0 (M x N expansions of nc components, leading dimension ldc)
hipError_t launch_zero_expansions(int nc, double *C, int64_t ldc, int64_t M, int64_t N,
                                  hipStream_t s);
// Ozaki-II product stages
hipError_t launch_exponents(int nc, const double *X, int64_t ld, int64_t rows, int64_t cols,
                            int rowwise, int32_t *e, hipStream_t s);
// plane encodings of the producer (one per back-end)
enum { PLANES_I8 = 0, PLANES_F8 = 1, PLANES_F64 = 2 };
hipError_t launch_producer(int nc, int nwx, int nh, int nwt, const double *X, int64_t ld, int rowwise,
                           int64_t nout, int64_t noutp, int64_t K, int64_t Kp,
                           const int32_t *exps, const DevPlan *pl, int nmod, int planes_kind,
                           void *planes, int64_t plane_elems, hipStream_t s);
hipError_t launch_gemm_i8(const int8_t *pa, const int8_t *pb, uint8_t *tpl, const DevPlan *pl,
                          int ng, int nmod, int64_t Mp, int64_t Np, int64_t Kp, int64_t planeA,
                          int64_t planeB, int tile, hipStream_t s);
hipError_t launch_gemm_f8(const uint8_t *pa, const uint8_t *pb, uint8_t *tpl, const DevPlan *pl,
                          int ng, int nmod, int64_t Mp, int64_t Np, int64_t Kp, int64_t planeA,
                          int64_t planeB, hipStream_t s);
// (S4) on the FP16 engine from the INT8 residue planes (Mp, Np multiples of 128)
hipError_t launch_gemm_f16(const int8_t *pa, const int8_t *pb, uint8_t *tpl, const DevPlan *pl,
                           int ng, int nmod, int64_t Mp, int64_t Np, int64_t Kp, int64_t planeA,
                           int64_t planeB, hipStream_t s);
// fused (S4)+(S5)+(S6), INT8 planes: t-values of a 32 x 32 tile kept in LDS
// (at most fused_max_products() (group, modulus) products)
int fused_max_products();
hipError_t launch_fused_b(int nc, int nwc, int nd, const int8_t *pa, const int8_t *pb,
                          const DevPlan *pl, int ng, int nmod, int64_t Kp, int64_t planeA,
                          int64_t planeB, double *C, int64_t ldc, int64_t M, int64_t N,
                          const int32_t *ea, const int32_t *eb, int mode, hipStream_t s);
hipError_t launch_gemm_f64(const double *pa, const double *pb, uint32_t *tpl, const DevPlan *pl,
                           int ng, int nmod, int64_t Mp, int64_t Np, int64_t Kp, int64_t planeA,
                           int64_t planeB, hipStream_t s);
hipError_t launch_consumer(int nc, int nwc, int nd, const void *tpl, int tbytes, int64_t Mp,
                           int64_t Np, double *C, int64_t ldc, int64_t M, int64_t N,
                           const int32_t *ea, const int32_t *eb, const DevPlan *pl, int mode,
                           hipStream_t s);
// group sums exported by the CRT routine of the consumer that reads these
// t-planes (byte back-ends: mx = 1 the matrix-core route of the expansion
// consumer, mx = 0 crt_group_bytes of the limb consumer, with the consumer's
// byte-column count for nd digits; binary64 moduli: crt_digits)
hipError_t launch_crt_export(const void *tpl, int tbytes, int nd, int64_t Mp, int64_t Np,
                             int64_t M, int64_t N, const DevPlan *pl, uint64_t *out, int nlimb,
                             int mx, hipStream_t s);

// LU pieces
size_t panel_lds_bytes(int nc, int kb, int R, int64_t nr);
hipError_t panel_max_blocks(int nc, int kb, int R, int64_t nr, int *maxblocks);
// lines: 2 * G candidate lines of 128 bytes (zeroed before each panel);
// crow: 2 * G rows of kb expansions
hipError_t launch_panel(int nc, double *A, int64_t lda, int64_t n, int64_t k, int kb, int R, int G,
                        int64_t *ipiv, int32_t *info, uint32_t *lines, int *err, double *crow,
                        int *perm, int *moved, int *nmoved, hipStream_t s);
hipError_t launch_laswp(int nc, double *A, int64_t lda, int64_t k, int64_t c0, int64_t c1,
                        const int *perm, const int *moved, const int *nmoved, hipStream_t s);
hipError_t launch_trsm_lower_unit(int nc, const double *L, int64_t lda, double *X, int64_t ldx,
                                  int kb, int64_t ncols, hipStream_t s);
hipError_t launch_trsm_upper(int nc, const double *U, int64_t lda, double *X, int64_t ldx, int kb,
                             int64_t ncols, hipStream_t s);
hipError_t launch_naive_gemm(int nc, const double *A, int64_t lda, const double *B, int64_t ldb,
                             double *C, int64_t ldc, int64_t M, int64_t N, int64_t K, int desc,
                             hipStream_t s);
hipError_t launch_apply_ipiv(int nc, double *B, int64_t ldb, int64_t n, int64_t nrhs,
                             const int64_t *ipiv, hipStream_t s);
hipError_t launch_fill_int(int *p, int v, int64_t cnt, hipStream_t s);

// limb format (k_limbs.hip): exponents, producer (INT8 or binary64 planes), consumer
// (exact group sums as nwords-word columns, word k of element i + j M at
// cw[k M N + i + j M]), the rounding of those sums into a limb matrix, the
// update C = RN_p(C - T) (T: M x N limb matrix with ld M, plane M N; dw:
// 2 nlimb + 2 words per element of scratch) and a zero fill
hipError_t launch_limb_exponents(const uint64_t *limb, const int32_t *lexp, int64_t ld,
                                 int64_t plane, int nlimb, int64_t rows, int64_t cols,
                                 int rowwise, int32_t *e, hipStream_t s);
// kind: PLANES_I8 (byte residues) or PLANES_F64 (binary64 moduli);
// tbytes: 1 (byte t-planes) or 4 (binary64 moduli)
hipError_t launch_producer_limbs(const uint64_t *limb, const int32_t *lexp, const uint8_t *lsign,
                                 int64_t ld, int64_t plane, int nlimb, int rowwise, int64_t nout,
                                 int64_t noutp, int64_t K, int64_t Kp, const int32_t *exps,
                                 const DevPlan *pl, int nmod, int nwt, int kind, void *planes,
                                 int64_t plane_elems, hipStream_t s);
hipError_t launch_consumer_limbs(const void *tpl, int tbytes, int64_t Mp, int64_t Np, int64_t M,
                                 int64_t N, const DevPlan *pl, int nd, int nvw, uint32_t *cw,
                                 hipStream_t s);
hipError_t launch_limb_round(const uint32_t *cw, int nwords, int64_t M, int64_t N,
                             const int32_t *ea, const int32_t *eb, int w, int g0, int Q, int nlimb,
                             uint64_t *olimb, int32_t *oexp, uint8_t *osign, int64_t ldo,
                             int64_t planeo, hipStream_t s);
hipError_t launch_limb_sub(uint64_t *climb, int32_t *cexp, uint8_t *csign, int64_t ldc,
                           int64_t planec, const uint64_t *tlimb, const int32_t *texp,
                           const uint8_t *tsign, int nlimb, int64_t M, int64_t N, uint32_t *dw,
                           hipStream_t s);
hipError_t launch_limb_zero(uint64_t *limb, int32_t *lexp, uint8_t *lsign, int64_t ld,
                            int64_t plane, int nlimb, int64_t M, int64_t N, hipStream_t s);
// pipelined triangular solve of one right-hand side (fwd: unit lower,
// ascending; else upper, descending, dividing by the diagonal); sync: two
// device words owned by the caller (finished-position counter and row-block
// ticket), reset by the launcher
hipError_t launch_trsv(int nc, int fwd, const double *LU, int64_t lda, double *x, int64_t n,
                       uint32_t *sync, int *err, hipStream_t s);

// batched LU + solve (k_batch.hip); items in processing order, each with its
// caller-order index in `reserved`
hipError_t launch_batch(const ozII_batch_item *items, int count, int *queue, uint64_t *times,
                        int grid, hipStream_t s);
// the same with the blocked LU and the in-workgroup Ozaki-II update (panel
// width b <= 256); plans at K = b for nc = 2, 3, 4 (null for absent formats),
// scratch of `slot` bytes per workgroup
hipError_t launch_batch_oz(const ozII_batch_item *items, int count, int *queue, uint64_t *times,
                           int grid, const ozk::DevPlan *pl2, const ozk::DevPlan *pl3,
                           const ozk::DevPlan *pl4, uint8_t *ws, int64_t slot, int b,
                           hipStream_t s);

// LU on limb matrices outside the Ozaki-II product (k_limb_lu.hip): limb q
// of element (i, j) at limb[q plane + i + j ld]
struct LimbMat {
  uint64_t *limb;
  int32_t *exp;
  uint8_t *sign;
  int64_t ld, plane;
};
// pivot-candidate workgroups per panel column (the size of `cand`)
constexpr int LPIV_MAXGRID = 64;
// one panel column j: pivot search over rows [j, n), ipiv[j], info, the
// interchange on columns [s0, s1), division, rank-1 update of columns
// (j, c1); zflag: one word
hipError_t launch_lpanel_column(LimbMat A, int nl, int64_t j, int64_t n, int64_t s0, int64_t s1,
                                int64_t c1, int64_t *cand, int64_t *ipiv, int32_t *info,
                                int32_t *zflag, hipStream_t s);
// interchanges ipiv[k0 .. k0+kb) on columns [ca0, ca1) and [cb0, cb1)
hipError_t launch_llaswp(LimbMat A, int nl, const int64_t *ipiv, int64_t k0, int64_t kb,
                         int64_t ca0, int64_t ca1, int64_t cb0, int64_t cb1, hipStream_t s);
// A[r0:r0+h, b0:b1] <- L^-1 A[r0:r0+h, b0:b1], L unit lower at (r0, r0)
hipError_t launch_ltrsm(LimbMat A, int nl, int64_t r0, int64_t h, int64_t b0, int64_t b1,
                        hipStream_t s);
// A[i0:i1, c0:c1] -= A[i0:i1, k0:k0+K] A[k0:k0+K, c0:c1] by multiply-subtracts
hipError_t launch_lschur_naive(LimbMat A, int nl, int64_t i0, int64_t i1, int64_t c0, int64_t c1,
                               int64_t k0, int64_t K, hipStream_t s);
hipError_t launch_lgetrs(LimbMat LU, int nl, int64_t n, const int64_t *ipiv, LimbMat X,
                         int64_t nrhs, hipStream_t s);
hipError_t launch_larith(int op, int nl, int64_t cnt, LimbMat A, LimbMat B, LimbMat C,
                         hipStream_t s);
hipError_t launch_lfill_i32(int32_t *p, int32_t v, int count, hipStream_t s);

}  // namespace ozl
