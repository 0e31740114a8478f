/*
 * thck.h - C ABI of the MI355X THC-MPO H|psi> library (libthck.so).
 *
 * Method: Sun/Mendl et al., THC-MPO Krylov (arXiv 2409.12708).  The library
 * applies the THC-factorised molecular Hamiltonian H = T + V of eq. (1),
 * with V written as the sum of G terms of eq. (G_mu_nu_def) (Sec. 3.1), to a
 * real matrix-product state, layer by layer with compression (Fig. 4 and
 * Algorithm 1, Sec. 3.2), sums the compressed terms by a pairwise reduction
 * tree (Sec. 4.5, Fig. 11) and uses the result in a global Lanczos step
 * (Sec. 2.2).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Sites: n = 2L spin-orbital sites, site j = 2p + s (s = 0 spin up,
 *   s = 1 spin down), local dimension d = 2, local basis (empty, occupied).
 *   Jordan-Wigner: a_j = Z_0 ... Z_{j-1} c_j with c = [[0,1],[0,0]] and
 *   Z = diag(1,-1) (Sec. 3.1 and App. C).
 * - MPS data: float64 site tensors, site j shaped (bonds[j], 2, bonds[j+1])
 *   and stored row-major (left index slowest) at data + offsets[j].
 *   bonds[0] = bonds[n] = 1.  Device pointers are HIP device memory; the
 *   caller owns them (the library never frees or reallocates them).
 * - Streams: every call enqueues its work on the given hipStream_t (passed
 *   as void*, NULL = the null stream) and returns without waiting, except
 *   where a call states that it synchronises.
 * - Errors: no exception crosses the ABI.  A non-zero thc_status is returned
 *   and thc_last_error() gives a thread-local message.  On error the output
 *   MPS contents are unspecified and its bonds/offsets arrays are unchanged.
 * - Threading: a context is not re-entrant; use one context per host thread.
 */
#ifndef THCK_H
#define THCK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  THC_OK = 0,
  THC_EINVAL = -1,     /* bad argument: shape, symmetry, NULL pointer */
  THC_ENOMEM = -2,     /* device allocation failed */
  THC_EDEVICE = -3,    /* HIP runtime error */
  THC_ENONFINITE = -4, /* NaN or Inf in an input */
  THC_ENOCONV = -5,    /* Jacobi sweep limit reached before convergence */
  THC_ECAPACITY = -6   /* output buffer too small */
} thc_status;

/* Contraction precision of the compression's absorb products: a factor
 * absorbed into a site (B_j L_{j+1} of the canonicalisation sweep, the rest
 * rows' source times L', (S V^T) Q_{j+1} of the truncation sweep, and the
 * re-canonicalisation's U_j L_{j+1}).  Data stays FP64 in memory; the
 * product rounds its operands.  The QR and SVD factorisations (with the
 * Gram matrix and the projections of the structured sweep), overlaps and
 * Lanczos eigensolves are always FP64.  Expected accuracy of an untruncated
 * H|psi>: ~1e-12 relative (F64), ~1e-6 (F32), ~1e-5 (BF16X3). */
typedef enum {
  THC_PREC_F64 = 0,
  THC_PREC_F32 = 1,    /* operands rounded to FP32, FP32 MFMA, FP32 accumulation */
  THC_PREC_BF16X3 = 2  /* FP32 operands split into bf16 hi + lo, a_hi b_hi + a_hi b_lo + a_lo b_hi on BF16 MFMA,
                          FP32 accumulation */
} thc_prec;

/* Caller-owned MPS view.  On input, bonds/offsets describe the data.  On
 * output, the library writes bonds[0..n] and offsets[0..n-1] (packed, in
 * elements) and fills data; capacity (elements) must be at least
 * thc_mps_capacity(n_sites, D).
 *
 * canonical: on input, nonzero declares that sites 1..n-1 are
 * right-canonical (for every site j >= 1 the rows a of A_j[a][s][b] are
 * orthonormal over (s, b); the norm sits at site 0).  The library then
 * keeps those rows as they are in the right-to-left orthogonalisation of
 * the compression (Sec. 3.1) and factorises only the rest.  It is not
 * checked: a wrong declaration gives wrong results.  Zero is always safe.
 * On output the library writes 1: every MPS it returns is in that form. */
typedef struct {
  int32_t n_sites;
  int32_t d;          /* must be 2 */
  int32_t *bonds;     /* host, n_sites + 1 entries */
  int64_t *offsets;   /* host, n_sites entries (elements) */
  double *data;       /* device */
  int64_t capacity;   /* elements available at data */
  int32_t canonical;  /* see above */
  int32_t reserved;   /* set to 0 */
} thc_mps;

typedef struct {
  int32_t D_max;       /* MPS bond dimension after every compression */
  int32_t D_sum;       /* bond kept at the inner nodes of the reduction tree (0 = D_max) */
  double rel_cutoff;   /* drop singular values <= rel_cutoff * s_1 (default 1e-14) */
  int32_t prec;        /* thc_prec */
  int32_t batch;       /* max compressions per batched launch (0 = automatic) */
  int32_t max_sweeps;  /* Jacobi sweep limit per SVD (0 = 40) */
  int32_t include_T;   /* 1: H = T + V, 0: V only */
  int32_t include_V;   /* 1: include V, 0: T only */
  uint64_t flags;      /* THC_FLAG_* bits, 0 = defaults */
} thc_opts;

/* opts.flags: SVD method of the truncation step.  Default: eigenpairs of the
 * Gram matrix Y Y^T (Householder tridiagonalisation, bisection, inverse
 * iteration), about 5x fewer flops than a bidiagonal SVD.  An eigenvalue
 * of the m x m Gram matrix is only resolved to ~m eps lambda_1, so every
 * job whose kept eigenvalues reach 32 m eps lambda_1 (rank-deficient sums,
 * exact zeros in the Schmidt spectrum) gets a second Gram level: the
 * eigenvectors of (Y - Q1 Q1^T Y)(...)^T, with Q1 the resolved ones, fill
 * the rest of the kept basis; the count is thc_stats.svd_fallbacks.  THC_FLAG_SVD_JACOBI: one-sided block Jacobi on
 * Y for every job (high relative accuracy, slower). */
#define THC_FLAG_SVD_JACOBI 1ull

/* opts.flags: record a pair of HIP events (on the call's stream) around each
 * launch of the compression kernels and return, per kernel class, the summed
 * device time, the launch count and the algorithmic flops of those launches
 * (LAPACK operation counts: LQ with thin Q 4nk^2 - 4k^3/3 for an m x n matrix,
 * k = min(m, n), n >= m; tridiagonalisation 4m^3/3; back-transformation
 * 2m^2 k; GEMM 2MNK) and their algorithmic device-memory bytes in
 * thc_stats.kernel_*.  Bytes are the doubles each kernel's algorithm must
 * move: LQ reads X and writes L and Q; GEMM reads A and B, reads C when
 * beta != 0 and writes C (the upper half with upper-triangle tiles);
 * back-transformation reads the reflectors (m^2/2) and Z and writes U;
 * bisection/inverse iteration reads d, e and writes the k vectors;
 * tridiagonalisation reads the upper triangle once and writes the
 * reflectors over it and d, e, tau (m^2 + 3m doubles; the kernels of this
 * library re-read the trailing triangle, once per column in one stage,
 * three times per 16 columns in two, which only the measured traffic
 * shows).  The band chase of the two-stage route counts ~3072 flops and 16
 * doubles of reflector per chase step (sweep j of an m x m band takes
 * (m-3-j)/16 + 1 steps) plus its band in and d, e out; the application of
 * its reflectors to k vectors 64 k flops per step, reading them and
 * reading and writing the vectors.  A launch that skips some of its jobs (the
 * LQ re-orthonormalisation of the truncation step, run only where the
 * eigensolver's vectors need it) is counted as if every job ran; the
 * second Gram level's launches are timed in their own class with no flops or
 * bytes.  Off by default. */
#define THC_FLAG_TIME_KERNELS 2ull

/* opts.flags: capture the launch sequence of a compression batch into a HIP
 * graph the second time a batch of the same signature (plan, batch size,
 * options) runs, and launch the graph from then on (graphs are kept by the
 * context, dropped when its workspace is reallocated).  Ignored with
 * THC_FLAG_TIME_KERNELS.  Results are the same as without it. */
#define THC_FLAG_GRAPHS 4ull

/* opts.flags: tridiagonalise the Gram matrices of the SVD step in one stage
 * (Householder, one column at a time) instead of the default two stages
 * (blocked reduction to a band of half-bandwidth 16, then Householder bulge
 * chasing of the band, with the chase's reflectors applied to the
 * eigenvectors before those of the band reduction).  Both give the same
 * eigenpairs to rounding. */
#define THC_FLAG_SYTRD_ONE_STAGE 8ull

/* opts.flags: mps_apply_thc_H (and the H applications of krylov_step and
 * krylov_evolve) splits the V terms by nu into [0, N/2) and [N/2, N), the
 * kinetic terms going with the second half, and sums each half by its own
 * pairwise tree in its own engine, on its own stream and host thread (a
 * second context on the same factors, created on first use and freed with
 * the context), so that the kernels of the two halves overlap on the GPU;
 * the two partial sums are then added and compressed.  Each half's batches
 * take half of the workspace budget.  The summation order differs from the
 * single tree (the same terms, a different tree), so truncated results
 * differ from the single-stream ones within the truncation error;
 * untruncated results agree to rounding.  Ignored when either half has no
 * V term. */
#define THC_FLAG_TWO_STREAMS 16ull

enum {
  THC_K_LQ = 0,      /* Householder LQ with Q formation (canonical sweep and re-orthonormalisation) */
  THC_K_SYTRD = 1,   /* tridiagonalisation of the Gram matrix (two-stage route: its band reduction) */
  THC_K_TRI_EIG = 2, /* bisection + inverse iteration */
  THC_K_ORMTR = 3,   /* back-transformation of the eigenvectors */
  THC_K_GEMM = 4,    /* batched GEMMs of the compression */
  THC_K_SVD_FALLBACK = 5, /* second Gram level of the jobs at the noise floor (time only; flops not counted) */
  THC_K_SB2ST = 6,   /* two-stage route: bulge chasing of the band to tridiagonal form */
  THC_K_Q2 = 7,      /* two-stage route: the chase's reflectors applied to the eigenvectors */
  THC_NK = 8
};

typedef struct {
  double discarded_weight_max; /* max over compressions and bonds of sum_{i>k} s_i^2 */
  double flops_model;          /* flops of the operations the call runs: LAPACK counts of its factorisations
                                  (LQ 4nk^2 - 4k^3/3, tridiagonalisation 4m^3/3, back-transformation 2m^2 k)
                                  and 2MNK per product, for the Gram SVD route (Gram matrix, Newton-Schulz
                                  step, C = Q^T Y); second Gram levels and flagged re-orthonormalisations are
                                  not counted */
  int64_t n_compressions;      /* number of MPS compressions performed */
  int64_t n_launches;          /* kernel launches issued */
  int32_t max_bond;            /* largest bond kept (after the cutoff) */
  int32_t jacobi_sweeps_max;   /* most Jacobi sweeps any SVD needed */
  int32_t nonconverged;        /* SVDs that hit the sweep limit */
  int32_t svd_fallbacks;       /* SVDs redone by the second Gram level (kept eigenvalues at the noise floor) */
  double kernel_ms[THC_NK];        /* THC_FLAG_TIME_KERNELS: summed device time per kernel class */
  double kernel_flops[THC_NK];     /* algorithmic flops of those launches */
  int64_t kernel_launches[THC_NK];
  double kernel_bytes[THC_NK];     /* algorithmic device-memory bytes of those launches */
  int64_t graph_captures;          /* THC_FLAG_GRAPHS: compression batches captured into a HIP graph */
  int64_t graph_replays;           /* THC_FLAG_GRAPHS: compression batches launched from a captured graph */
} thc_stats;

typedef struct thc_ctx thc_ctx;
typedef struct thc_krylov thc_krylov;

/* Fill *o with defaults (D_max = D, D_sum = 0, cutoff 1e-14, FP64, T and V). */
void thc_default_opts(thc_opts *o, int32_t D);

/* Elements needed to hold any n-site MPS of bond <= D in the packed layout
 * (bond profile min(2^j, 2^(n-j), D)). */
int64_t thc_mps_capacity(int32_t n_sites, int32_t D);

/* Load the THC factors (eq. thc, Sec. 2.3) and the one-body integrals t of
 * eq. (1).  Host arrays, row-major float64, read during the call only:
 *   t    L x L, symmetric (App. D splits it as t = U diag(lambda) U^T);
 *   chi  L x N, chi[p * N + mu] = chi_p^mu;
 *   zeta N x N, symmetric.
 * Validates finiteness (THC_ENONFINITE) and symmetry of t and zeta to 1e-12
 * relative (THC_EINVAL), diagonalises t in FP64 on the host, builds the
 * 4N^2 + 2L term table (readings of Algorithm 1's loop order: nu outer,
 * sigma', mu, sigma; T terms after V) and uploads it.  *ctx receives a new
 * context owning its device copies and workspace; release it with
 * thc_destroy. */
thc_status thc_load_factors(thc_ctx **ctx, int32_t L, int32_t N, const double *t,
                            const double *chi, const double *zeta, uint64_t flags,
                            void *hip_stream);

thc_status thc_destroy(thc_ctx *ctx);

/* out <- compressed H|psi> (Algorithm 1 terms with the reuse of
 * G_{nu sigma'}|psi>, Sec. 3.2; kinetic part by App. D; summed by the
 * pairwise tree of Sec. 4.5).  psi->n_sites must equal 2L.  psi and out
 * must not alias.  st may be NULL.  Synchronises the stream after each
 * batch of compressions (the kept bond dimensions decide how later jobs
 * are grouped and how the output is packed) and at the end. */
thc_status mps_apply_thc_H(thc_ctx *ctx, const thc_mps *psi, thc_mps *out, const thc_opts *o,
                           thc_stats *st, void *hip_stream);

/* out <- compressed sum_i coeffs[i] |terms[i]> (the addition-compression of
 * Algorithm 1).  k >= 1; for k > 1 the terms are summed by the pairwise
 * tree (pair 2i with 2i+1, an odd last term carries up), every node
 * compressed to D_sum (0 = D_max) and the root to D_max.  coeffs is host.
 * All terms must have the same n_sites.  Synchronises after each batch of
 * compressions and at the end. */
thc_status mps_sum_compress(thc_ctx *ctx, int32_t k, const double *coeffs, const thc_mps *const *terms,
                            thc_mps *out, const thc_opts *o, thc_stats *st, void *hip_stream);

/* *result <- <a|b> (host double), by the transfer-matrix chain, FP64.
 * Synchronises the stream. */
thc_status mps_overlap(thc_ctx *ctx, const thc_mps *a, const thc_mps *b, double *result,
                       void *hip_stream);

/* Allocation-free <a|b>, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same transfer-matrix chain as mps_overlap, FP64; writes the
 * value to *result_dev (device memory) on the given stream and returns
 * without synchronising.  Needs no context.  The transfer matrices live in a
 * file-scope device array of 4 * 512^2 + 64 doubles (8 MiB) per GPU, which
 * the library holds until the process ends: bonds above 512 return
 * THC_ECAPACITY with nothing launched.  All calls on one GPU share that
 * array, so calls that overlap on one GPU (other streams, other threads)
 * race; a later call simply overwrites it. */
thc_status mps_overlap_noalloc(const thc_mps *a, const thc_mps *b, double *result_dev, void *hip_stream);

/* Lanczos state (Sec. 2.2): Krylov vectors v_0..v_K, the H images w_i,
 * M_ij = <v_i|w_j> and S_ij = <v_i|v_j>, all in device memory owned by the
 * state.  krylov_create copies psi0 and normalises it. */
thc_status krylov_create(thc_ctx *ctx, const thc_mps *psi0, int32_t K, const thc_opts *o,
                         thc_krylov **state, void *hip_stream);
thc_status krylov_destroy(thc_krylov *state);

/* One global Lanczos step i -> i+1 (Sec. 2.2 with the re-orthogonalised
 * effective Hamiltonian of eq. eff_H):
 *   w_i = compressed H|v_i>;  h_ji = <v_j|w_i> (j <= i);
 *   r = compressed (w_i - sum_j h_ji v_j) (one mps_sum_compress);
 *   beta_i = ||r||, v_{i+1} = r / beta_i;  S and M extended;
 * then the (i+1) x (i+1) eigenproblems are solved on the device in FP64:
 *   ritz_gen[0..i]  eigenvalues of H_sym = (M + M^T)/2 in the basis
 *                   psi_a = sum_i C_ai v_i with C S C^T = I (Cholesky;
 *                   canonical orthogonalisation if S is singular);
 *   ritz_tri[0..i]  eigenvalues of the tridiagonal (alpha_i = h_ii, beta).
 * ritz_gen, ritz_tri (nullable) and beta are host arrays / scalars written
 * before return.  The call synchronises the stream: once per compression
 * batch inside its H application and sum-compression (to read back the
 * kept bond dimensions), after every overlap, and at the end.  When S has
 * an eigenvalue at or below 1e-10, ritz_gen holds the values of the
 * canonically orthogonalised basis first and NaN in the remaining entries.
 * Returns THC_EINVAL once K steps have been taken. */
thc_status krylov_step(thc_krylov *state, double *ritz_gen, double *ritz_tri, double *beta,
                       thc_stats *st, void *hip_stream);

/* out <- the a-th Ritz vector (a = 0: lowest Ritz value) of the steps taken:
 * psi = sum_i x_i v_i over v_0..v_{m-1}, m = steps taken, with x = C^T y_a
 * from the generalised problem of krylov_step (eq. reortho, eq. eff_H;
 * y_a the a-th eigenvector of C H_sym C^T), summed and compressed by
 * mps_sum_compress with the state's options.  out follows mps_sum_compress's
 * rules (capacity, no aliasing).  THC_EINVAL when no step has been taken or
 * a is not below the number of kept basis directions.  Synchronises. */
thc_status krylov_ritz_vector(thc_krylov *state, int32_t a, thc_mps *out, void *hip_stream);

/* Restart (Sec. 2.2: restarting recovers convergence lost to truncation):
 * v_0 <- the a-th Ritz vector, normalised; the basis, M, S, alpha and beta
 * are cleared, so the next krylov_step starts a new Krylov space of up to K
 * vectors from it.  For an excited state, start krylov_create from a vector
 * orthogonal to the lower eigenstates (Sec. 2.2; the paper uses a
 * Hartree-Fock single excitation) and restart from a = 0 of that run.
 * Synchronises. */
thc_status krylov_restart(thc_krylov *state, int32_t a, void *hip_stream);

/* Copy Krylov vector v_i (i <= steps taken) into a caller MPS. */
thc_status krylov_get_vector(thc_krylov *state, int32_t i, thc_mps *out, void *hip_stream);

/* Copy the (m x m) leading blocks of M and S (host, row-major), m = steps taken. */
thc_status krylov_get_matrices(thc_krylov *state, double *Mm, double *S, int32_t *m);

/* Krylov time evolution (Sec. 2.2: psi(t + delta) = sum_i a_i v_i with
 * a(delta) = exp(-i delta H~) a(0); error bounds in App. A) of complex states
 * under the real H of each instance's context, n_steps steps of size delta,
 * for n_inst independent instances (their own contexts, so L and N may
 * differ, and their own opts, so D may differ), all on one stream, one
 * time step of each instance in turn.
 *
 * A complex state is a pair of real MPS, psi = re + i im.  Because H is
 * real, H acts on the two parts separately; each part is compressed on its
 * own to opts[q].D_max by the rules of mps_sum_compress.  Per step, with
 * v_0 = psi / ||psi||: w_i = compressed H v_i, M_ji = <v_j|w_i> (complex,
 * j <= i); unless i = K-1, v_{i+1} = r / ||r|| for r = compressed
 * (w_i - sum_j M_ji v_j), with S and M extended.  The basis stops early
 * (m < K) when ||r|| <= 1e-10 sqrt(sum_j |M_ji|^2 + ||r||^2): the Krylov space
 * is invariant and the step exact.  The coefficients a over v_0..v_{m-1}
 * follow from the effective Hamiltonian of eq. eff_H (H_sym = (M + M^H)/2
 * in a basis orthonormal in the metric S, over the eigen-directions of S
 * above 1e-10, eq. reortho), computed on the device in FP64, and
 * psi(t + delta) = ||psi|| sum_i a_i v_i.  A complex combination
 * sum_j c_j x_j is two sum-compressions: the real part over the terms
 * (Re c_j, x_j,re), (-Im c_j, x_j,im), the imaginary part over
 * (Re c_j, x_j,im), (Im c_j, x_j,re), j ascending, dropping absent parts
 * and exactly zero coefficients (a part with no term left is zero).
 *
 *   ctxs[q]       context of instance q (n = 2L sites).
 *   psi_re[q]     real part (device MPS; NULL = zero).
 *   psi_im        NULL (every imaginary part zero) or n_inst entries, each
 *                 NULL (zero) or a device MPS.  A part whose norm is zero
 *                 is treated as absent.  Not both parts zero.
 *   opts[q]       options of instance q (D_max, precision of the absorb
 *                 contractions: FP32 / BF16x3 parts are the complex64 form).
 *   K             Krylov vectors per step, 1..16.
 *   out_re[q], out_im[q]  caller MPS for the final parts, capacity at least
 *                 thc_mps_capacity(n, D_max) (and the input's size); a zero
 *                 part is written as the bond-1 MPS of zeros, canonical = 0.
 *                 Inputs are copied before any output is written, so outputs
 *                 may alias inputs.
 *   krylov_dims   host n_inst x n_steps (nullable): basis size m of each step.
 *   st            accumulated statistics of every compression (nullable).
 * Synchronises (after every compression batch, every overlap and at the
 * end).  Returns THC_EINVAL for zero-norm states or bad shapes,
 * THC_ENONFINITE for non-finite inputs or coefficients, THC_ECAPACITY for
 * small outputs; outputs are unspecified on error. */
thc_status krylov_evolve(int32_t n_inst, thc_ctx *const *ctxs, const thc_mps *const *psi_re,
                         const thc_mps *const *psi_im, const thc_opts *opts, int32_t K, double delta,
                         int32_t n_steps, thc_mps *const *out_re, thc_mps *const *out_im, int32_t *krylov_dims,
                         thc_stats *st, void *hip_stream);

/* Complex states as pairs of real MPS (the representation krylov_evolve
 * uses): out <- compressed sum_i c_i |term_i> with complex c_i
 * (coeffs[2i] = Re c_i, coeffs[2i+1] = Im c_i, host) and complex terms
 * term_i = terms_re[i] + i terms_im[i] (device MPS; a NULL entry, or a NULL
 * array, is a zero part).  The real part is one mps_sum_compress over the
 * terms (Re c_i, re_i), (-Im c_i, im_i), the imaginary part one over
 * (Re c_i, im_i), (Im c_i, re_i), i ascending, leaving out NULL parts and
 * exactly zero coefficients; a part with no term left is written as the
 * bond-1 MPS of zeros (canonical = 0).  out_re and out_im follow
 * mps_sum_compress's rules (capacity, no aliasing of any input) and must be
 * distinct.  Synchronises. */
thc_status mps_sum_compress_complex(thc_ctx *ctx, int32_t k, const double *coeffs, const thc_mps *const *terms_re,
                                    const thc_mps *const *terms_im, thc_mps *out_re, thc_mps *out_im,
                                    const thc_opts *o, thc_stats *st, void *hip_stream);

/* result[0] + i result[1] <- <a|b> for complex states given as pairs of
 * real MPS (NULL = zero part): <a_re|b_re> + <a_im|b_im>
 * + i (<a_re|b_im> - <a_im|b_re>), each by mps_overlap.  result is host.
 * Synchronises. */
thc_status mps_overlap_complex(thc_ctx *ctx, const thc_mps *a_re, const thc_mps *a_im, const thc_mps *b_re,
                               const thc_mps *b_im, double *result, void *hip_stream);

/* Compress one MPS to D (QR sweep then SVD truncation sweep, Fig. 3). */
thc_status mps_compress(thc_ctx *ctx, const thc_mps *in, thc_mps *out, const thc_opts *o,
                        thc_stats *st, void *hip_stream);

/* Apply one elementary layer sum_j y_j a_j (dag = 0) or sum_j y_j a+_j
 * (dag = 1) of eq. (elementary_MPO) to psi and compress (one arrow of Fig. 4).
 * y is a host array of n_sites spin-orbital coefficients. */
thc_status mps_apply_layer(thc_ctx *ctx, const thc_mps *psi, const double *y, int32_t dag,
                           thc_mps *out, const thc_opts *o, thc_stats *st, void *hip_stream);

/* Energy E = <psi|H|psi> of a real MPS and its gradient with respect to the
 * context's THC factors, for THC-factor fitting (Sec. 2.3) and orbital
 * gradients.  With N_nu = sum_s a+(chi^nu)_s a(chi^nu)_s (the G terms of
 * eq. G_mu_nu_def summed over the spins, Sec. 3.1), V = 1/2 sum zeta_{mu nu}
 * N_mu N_nu and, for fixed psi,
 *   dzeta[mu * N + nu] = dE/dzeta_{mu nu} = 1/2 <psi|N_mu N_nu|psi>
 *     (every entry independent, zeta not symmetrised),
 *   dchi[p * N + k]    = dE/dchi_p^k
 *     = 1/2 sum_nu (zeta_{k nu} + zeta_{nu k}) <psi|dN_k/dchi_p^k N_nu|psi>.
 * H|psi> is applied without truncation: each n_{nu s}|psi> is formed
 * exactly by two layer MPOs (bond 4 b_j) and the transition one-body
 * matrices <psi|a+_i a_j n_{nu s}|psi> are contracted by transfer-matrix
 * chains on the device.  prec: THC_PREC_F64 or THC_PREC_F32 (the
 * contraction precision of those chains; FP32 operands, FP32 accumulation).
 * energy, dchi (L x N), dzeta (N x N) are host outputs; any may be NULL, not
 * all.  psi->n_sites must equal 2L.  Device memory grows with the bonds
 * (~(2N + 2L) kets of bond 4 b_j, processed in chunks within ~48 GiB).
 * Synchronises. */
thc_status thc_energy_gradient(thc_ctx *ctx, const thc_mps *psi, int32_t prec, double *energy, double *dchi,
                               double *dzeta, void *hip_stream);

/* Thread-local description of the last non-OK status. */
const char *thc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* THCK_H */
