// Internal interface between the engine (host scheduling) and the HIP
// kernels.  Not part of the public C ABI (include/thck.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <cstdio>

namespace thck {

// One compression job: construct a bond-2D MPS from one or two inputs, then
// compress it.  kind 0 = layer  sum_j y_j a_j (dag 0) or a+_j (dag 1) applied
// to in_a, site 0 scaled by ca; kind 1 = direct sum ca*in_a + cb*in_b.
struct CJob {
  const double *in_a;
  const double *in_b;
  const double *y;
  double ca, cb;
  double *out;
  int kind;
  int dag;
};

constexpr int RITZ_MAX = 32;

int lq_t_stride(int k);

void launch_construct(hipStream_t st, const CJob *jobs, int nb, int site, int n_sites, int64_t in_off_a,
                      int64_t in_off_b, int la, int ra, int lb, int rb, double *out, int64_t out_stride, int lo,
                      int ro);
// GEMM modes (bits): B given transposed, A given transposed; with UPPER only
// the output tiles that reach the diagonal or above it are computed (the
// upper triangle of a symmetric product; entries below it are not written).
constexpr int GEMM_TB = 1, GEMM_TA = 2, GEMM_UPPER = 4;
// contraction precision of a GEMM (operands and result are FP64 in memory)
constexpr int GEMM_F64 = 0, GEMM_F32 = 1, GEMM_BF16X3 = 2;
// C = alpha op(A) op(B) + beta C (beta = 0: C is not read).  With only (one
// int per job), jobs whose entry is 0 are skipped (their C is untouched);
// the same holds for the other kernels that take an only array.
void launch_gemm(hipStream_t st, int nb, int mode, const double *A, int64_t sA, int lda, const double *B,
                 int64_t sB, int ldb, double *C, int64_t sC, int ldc, int M, int N, int K, double alpha = 1.0,
                 double beta = 0.0, int prec = GEMM_F64, const int *only = nullptr);
// One FP64 job (mode 0 or GEMM_TA) with the default 64 x 64 tiles: never
// consults or updates the tile autotuner, so it creates no event, never
// synchronises and shares no host state between threads.
void launch_gemm_f64_fixed(hipStream_t st, int mode, const double *A, int lda, const double *B, int ldb, double *C,
                           int ldc, int M, int N, int K);
void launch_transpose(hipStream_t st, int nb, const double *src, int64_t ss, int r, int c, double *dst, int64_t sd);
// LQ of X (m x n), k = min(m, n): L (m x k, row stride ldl), Q (k x n, row
// stride ldq).  With tr, X is given transposed (n x m row-major) and Q is
// returned transposed (n x k, row stride ldq); L keeps its layout.  ldl /
// ldq <= 0 select the dense strides.  With only (one int per job), a job
// whose entry is 0 is skipped and its L, Q are left as they are.
int launch_lq(hipStream_t st, int nb, double *X, int64_t sX, int m, int n, double *L, int64_t sL, double *Q,
              int64_t sQ, double *Tw, int64_t sT, bool tr = false, int ldl = 0, int ldq = 0,
              const int *only = nullptr);
int launch_jacobi(hipStream_t st, int nb, double *Y, int64_t sY, int m, int n, double *s, int64_t ss, int *sweeps,
                  int max_sweeps, const int *only = nullptr);
void launch_svd_select(hipStream_t st, int nb, const double *Y, int64_t sY, int m, int n, const double *s,
                       int64_t ss, int kk, double cutoff, double *W, int64_t sW, int *rank, double *disc,
                       double *sv_out, int64_t ssv, const int *only = nullptr);
void launch_svd_finish(hipStream_t st, int nb, const double *Q, int64_t sQ, int m, int kk, const int *rank,
                       double *U, int64_t sU, double *C, int64_t sC, int n, const int *only = nullptr);
// Structured LQ sweep for right-canonical inputs (see kernels.hip).
void launch_canon_pack(hipStream_t st, int nb, const CJob *jobs, int64_t in_off, int lc, int ra, int c1, double *Qt,
                       int64_t sQ, int ldq);
void launch_rest_post(hipStream_t st, int nb, const CJob *jobs, int site, int64_t in_off, int lr, int ra, int c1,
                      double *RT, int64_t sR);
void launch_site0(hipStream_t st, int nb, const CJob *jobs, int64_t in_off, int ra, int c1, double *M, int64_t sM);
void launch_fill(hipStream_t st, int nb, double *p, int64_t stride, int64_t count, double v);
void launch_copy(hipStream_t st, int nb, const double *src, int64_t ssrc, double *dst, int64_t sdst, int64_t count,
                 const int *only = nullptr);
// which: 0 = in_a, 1 = in_b, 2 = out
void launch_gather(hipStream_t st, int nb, const CJob *jobs, int which, int64_t off, double *dst, int64_t sdst,
                   int64_t count);
void launch_scatter(hipStream_t st, int nb, const CJob *jobs, int64_t off, const double *src, int64_t ssrc,
                    int64_t count);
void launch_scale(hipStream_t st, double *p, int64_t count, double c);
void launch_repack(hipStream_t st, int gx, const double *src, int64_t soff, int ks_l, int ks_r, double *dst,
                   int64_t doff, int rl, int rr);
int launch_sytrd(hipStream_t st, int nb, double *A, int64_t sA, int m, double *d, double *e, double *tau, int64_t sv,
                 const int *only = nullptr);
// Top-kk eigenpairs of tridiagonals.  With needs_lq (one int per job): 1
// where the returned vectors need not be orthonormal (completions of
// eigenvalues below the noise floor, a cluster split at the member cap),
// else 0.
int launch_tri_eig(hipStream_t st, int nb, const double *d, const double *e, int64_t sv, int m, int kk, double *Z,
                   int64_t sZ, double *lam, int64_t sl, double *scr, int64_t sscr, int *needs_lq = nullptr,
                   const int *only = nullptr);
// U = Q_H Z; written as rows of Ut (kk x m), or with zout as Z itself (m x kk).
// Tf: workspace for the blocks' compact-WY factors, ormtr_tf_stride(m) per job.
int64_t ormtr_tf_stride(int m);
// off: row offset of the reflectors (1 after sytrd, 16 after sy2sb).
int launch_ormtr(hipStream_t st, int nb, const double *A, int64_t sA, int m, const double *tau, int64_t sv, double *Z,
                 int64_t sZ, int kk, double *Ut, int64_t sU, bool zout, double *Tf, int64_t sTf,
                 const int *only = nullptr, int off = 1);
// Two-stage tridiagonalisation (band.hip), m <= 512.  sy2sb: A (upper
// triangle) to half-bandwidth 16, reflectors for ormtr with off = 16 (tau
// needs m entries).  sb2st: the band to d, e; the chase's reflectors into V2
// (sb2st_v2_stride(m) doubles per job).  q2apply: Z (m x kk) <- Q2 Z.
int launch_sy2sb(hipStream_t st, int nb, double *A, int64_t sA, int m, double *tau, int64_t sv,
                 const int *only = nullptr);
int64_t sb2st_v2_stride(int m);
int launch_sb2st(hipStream_t st, int nb, const double *A, int64_t sA, int m, double *d, double *e, int64_t sv,
                 double *V2, int64_t sV2, const int *only = nullptr);
int launch_q2apply(hipStream_t st, int nb, const double *V2, int64_t sV2, int m, double *Z, int64_t sZ, int kk,
                   const int *only = nullptr);
// Per-job flags of the Gram SVD step (see kernels.hip): jac = redo by Jacobi,
// nl |= Householder re-orthonormalisation needed.
void launch_svd_flags(hipStream_t st, int nb, const double *lam, int64_t sl, int kk, double tau, const double *Lz,
                      int64_t sLz, int *nl, int *jac);
// qt: Q given as its transpose (m x kk) instead of kk x m.
void launch_svd_finish2(hipStream_t st, int nb, const double *Q, int64_t sQ, int m, int kk, double *C, int64_t sC,
                        int n, double cutoff, const double *d, int64_t sv, double *U, int64_t sU, int *rank,
                        double *disc, bool qt = false, const int *only = nullptr);
// Second level of the Gram route (see kernels.hip).
void launch_deflate_prep(hipStream_t st, int nb, const double *lam, int64_t sl, int kk, double tau, const double *Q,
                         int64_t sQ, int m, double *Q1, int64_t sQ1, int *r1, const int *jac, int *flag);
void launch_merge_basis(hipStream_t st, int nb, const double *Q1, int64_t sQ1, const double *Z2, int64_t sZ, int m,
                        int kk, const int *r1, const int *jac, double *out, int64_t sO);
int64_t tri_eig_scratch(int m, int kk);
void launch_ritz(hipStream_t st, const double *Mm, const double *S, int m, int ld, const double *alpha,
                 const double *beta, double *out_gen, double *out_tri, int *info);

// Coefficients of the a-th Ritz vector over v_0..v_{m-1} (device x, m).
void launch_ritz_vector(hipStream_t st, const double *Mm, const double *S, int m, int ld, int a, double *x,
                        int *info);
// Krylov time step: out[0..2m) = scale * (Re a, Im a) of exp(-i delta H~) e_0
// from complex M, S given as real/imaginary parts (row stride ld); m <= 16.
void launch_evolve_coeffs(hipStream_t st, const double *Mr, const double *Mi, const double *Sr, const double *Si,
                          int m, int ld, double delta, double scale, double *out, int *info);

// Energy gradient (see kernels.hip): closing dot products of the transition
// one-body matrices, the Z-signed bra site, and the final contraction into
// out = [E, dchi (L x N), dzeta (N x N)].
void launch_rdm_close(hipStream_t st, int nblk, int nket, const double *F, int64_t sF_ket, int64_t sF_blk,
                      const double *W, int64_t sW, int lb, int rk, double *g, int n, int j, int mode);
void launch_negate_odd(hipStream_t st, const double *src, double *dst, int l, int r);
void launch_grad_final(hipStream_t st, const double *g, int n, int L, int N, const double *chi, const double *zeta,
                       const double *lam, const double *ovl, double *Gw, double *out);

// GEMM tile autotuner: decisions so far (printed with THCK_KSTATS=1) and
// how many shape classes have been tuned.
void gemm_tuning_report(FILE *f);
int gemm_tuned_classes();

}  // namespace thck
