// Device kernels of the THC-MPO H|psi> path for gfx950 (MI355X).
//
// Every kernel is batched over independent compression jobs: blockIdx.y (or
// blockIdx.x for one-workgroup-per-matrix kernels) selects the job, and job
// b's operands sit at base + b * stride.  All jobs of a launch share the
// same static shapes; rank-deficient jobs carry exact zeros in the padding.
//
// Steps of one MPS compression (Fig. 3 caption):
//   construct   B_j = W_j (x) A_j of the layer MPO (eq. elementary_MPO in
//               JW form, App. C), or the direct sum of two MPS (Alg. 1 add)
//   gemm        absorb the L factor / the carried S V^T into the next site
//   lq          Householder LQ of a site matrix (right-canonical sweep)
//   jacobi      one-sided block Jacobi on the rows of a site matrix; with
//   svd_*       the top-k rows selected, U recovered by a second LQ
//   overlap     transfer-matrix chain <a|b>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace thck {

static constexpr int WAVE = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// Round-robin (circle method) schedule over P players (P even): in round r
// the players are listed as [0, 1 + (r mod (P-1)), 1 + (r+1 mod (P-1)), ...]
// and pair k joins list entries k and P-1-k.  Over P-1 rounds every pair of
// players meets exactly once and each round's pairs are disjoint.
__device__ __forceinline__ int rr_player(int idx, int r, int P) { return idx == 0 ? 0 : 1 + ((idx - 1 + r) % (P - 1)); }
__device__ __forceinline__ void rr_pair(int k, int r, int P, int &p, int &q) {
  p = rr_player(k, r, P);
  q = rr_player(P - 1 - k, r, P);
  if (p > q) { int t = p; p = q; q = t; }
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, WAVE));
  return v;
}

// ---------------------------------------------------------------------------
// construct: layer MPO applied to one site, or direct sum of two MPS.
// Layer: W_j = [[Z, y_j o], [0, I]], o = c (annihilation) or c^T (creation).
// Output bond index (alpha, a) -> alpha * la + a; site 0 keeps alpha = 0,
// site n-1 keeps beta = 1.  The job scale multiplies the last site.
// ---------------------------------------------------------------------------
__global__ void k_construct(const CJob *__restrict__ jobs, int site, int n_sites, int64_t in_off_a,
                            int64_t in_off_b, int la, int ra, int lb, int rb, double *__restrict__ out,
                            int64_t out_stride, int lo, int ro) {
  const CJob jb = jobs[blockIdx.y];
  double *dst = out + (int64_t)blockIdx.y * out_stride;
  const int64_t total = (int64_t)lo * 2 * ro;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int B_ = (int)(e % ro);
    const int m = (int)((e / ro) % 2);
    const int A_ = (int)(e / (2 * (int64_t)ro));
    double val = 0.0;
    if (jb.kind == 0) {
      const double *A = jb.in_a + in_off_a;
      int alpha, a, beta, b;
      if (site == 0) { alpha = 0; a = A_; } else { alpha = A_ / la; a = A_ % la; }
      if (site == n_sites - 1) { beta = 1; b = B_; } else { beta = B_ / ra; b = B_ % ra; }
      const int64_t base = (int64_t)a * 2 * ra + b;
      if (alpha == 0 && beta == 0) {
        val = (m == 0 ? 1.0 : -1.0) * A[base + (int64_t)m * ra];
      } else if (alpha == 0 && beta == 1) {
        const double y = jb.y[site];
        if (jb.dag == 0) val = (m == 0) ? y * A[base + ra] : 0.0;   // c: |1> -> |0>
        else             val = (m == 1) ? y * A[base] : 0.0;        // c^T: |0> -> |1>
      } else if (alpha == 1 && beta == 1) {
        val = A[base + (int64_t)m * ra];
      }
      if (site == n_sites - 1) val *= jb.ca;
    } else {
      // direct sum: A (la,2,ra), B (lb,2,rb)
      const double *A = jb.in_a + in_off_a;
      const double *Bm = jb.in_b + in_off_b;
      if (site == 0) {  // (1, 2, ra + rb)
        if (B_ < ra) val = jb.ca * A[(int64_t)m * ra + B_];
        else val = jb.cb * Bm[(int64_t)m * rb + (B_ - ra)];
      } else if (site == n_sites - 1) {  // (la + lb, 2, 1)
        if (A_ < la) val = A[(int64_t)A_ * 2 + m];
        else val = Bm[(int64_t)(A_ - la) * 2 + m];
      } else {
        if (A_ < la && B_ < ra) val = A[((int64_t)A_ * 2 + m) * ra + B_];
        else if (A_ >= la && B_ >= ra) val = Bm[((int64_t)(A_ - la) * 2 + m) * rb + (B_ - ra)];
      }
    }
    dst[e] = val;
  }
}

// ---------------------------------------------------------------------------
// gemm: C = op(A) * op(B), row-major, FP64, batched by blockIdx.z.
// 64x64 output tile, BK = 16, 256 threads, 4x4 outputs per thread.
// transB: B is given as N x K (row-major) and used transposed.
// ---------------------------------------------------------------------------
template <bool TRANS_B>
__global__ __launch_bounds__(256) void k_gemm_f64(const double *__restrict__ A, int64_t sA, int lda,
                                                  const double *__restrict__ B, int64_t sB, int ldb,
                                                  double *__restrict__ C, int64_t sC, int ldc, int M,
                                                  int N, int K) {
  constexpr int TM = 64, TN = 64, TK = 16;
  __shared__ double As[TK][TM + 1];
  __shared__ double Bs[TK][TN + 1];
  A += (int64_t)blockIdx.z * sA;
  B += (int64_t)blockIdx.z * sB;
  C += (int64_t)blockIdx.z * sC;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int tid = threadIdx.x;
  const int tr = tid / 16, tc = tid % 16;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += TK) {
    for (int e = tid; e < TM * TK; e += 256) {
      int mm = e / TK, kk = e % TK;
      int gm = m0 + mm, gk = k0 + kk;
      As[kk][mm] = (gm < M && gk < K) ? A[(int64_t)gm * lda + gk] : 0.0;
    }
    for (int e = tid; e < TN * TK; e += 256) {
      if (TRANS_B) {
        int nn = e / TK, kk = e % TK;
        int gn = n0 + nn, gk = k0 + kk;
        Bs[kk][nn] = (gn < N && gk < K) ? B[(int64_t)gn * ldb + gk] : 0.0;
      } else {
        int kk = e / TN, nn = e % TN;
        int gn = n0 + nn, gk = k0 + kk;
        Bs[kk][nn] = (gn < N && gk < K) ? B[(int64_t)gk * ldb + gn] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][tr * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tc * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int gm = m0 + tr * 4 + i;
    if (gm >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int gn = n0 + tc * 4 + j;
      if (gn < N) C[(int64_t)gm * ldc + gn] = acc[i][j];
    }
  }
}

// ---------------------------------------------------------------------------
// lq: X (m x n, row-major, in place) = L Q by Householder reflections acting
// on rows (LAPACK dgelqf/dorglq style, blocked with panels of NB rows and
// the compact WY form H_i ... H_{i+nb-1} = I - V T V^T).  One workgroup
// (256 threads) per matrix.  Outputs: L (m x k, row-major), Q (k x n,
// row-major), k = min(m, n).  X keeps the reflectors afterwards.
// LDS: the panel rows (NB x n) and T (NB x NB).
// ---------------------------------------------------------------------------
template <int NB, int NMAX>
__global__ __launch_bounds__(256) void k_lq(double *__restrict__ Xb, int64_t sX, int m, int n,
                                            double *__restrict__ Lb, int64_t sL, double *__restrict__ Qb,
                                            int64_t sQ, double *__restrict__ Tb, int64_t sT) {
  extern __shared__ double lds[];
  double *P = lds;                // NB x NMAX panel (reflectors v, unit diagonal implicit)
  double *T = P + NB * NMAX;      // NB x NB
  double *tau = T + NB * NB;      // NB
  double *X = Xb + (int64_t)blockIdx.x * sX;
  double *Lo = Lb + (int64_t)blockIdx.x * sL;
  double *Qo = Qb + (int64_t)blockIdx.x * sQ;
  double *Ts = Tb + (int64_t)blockIdx.x * sT;  // all panels' T factors and taus
  const int tid = threadIdx.x, lane = tid % WAVE, wid = tid / WAVE, nw = blockDim.x / WAVE;
  const int k = m < n ? m : n;

  for (int i0 = 0; i0 < k; i0 += NB) {
    const int pb = (k - i0) < NB ? (k - i0) : NB;
    const int w = n - i0;  // panel width
    // load panel rows i0..i0+pb-1, columns i0..n-1
    for (int e = tid; e < pb * w; e += blockDim.x) {
      int p = e / w, c = e % w;
      P[p * NMAX + c] = X[(int64_t)(i0 + p) * n + i0 + c];
    }
    __syncthreads();
    if (wid == 0) {
      for (int p = 0; p < pb; ++p) {
        double *row = P + p * NMAX;
        for (int q = 0; q < p; ++q) {  // apply H_q (q < p) to row p
          const double *v = P + q * NMAX;
          double s = 0.0;
          for (int c = q + lane; c < w; c += WAVE) s += row[c] * (c == q ? 1.0 : v[c]);
          s = wave_sum(s) * tau[q];
          for (int c = q + lane; c < w; c += WAVE) row[c] -= s * (c == q ? 1.0 : v[c]);
        }
        // Householder vector for row p on columns p..w-1
        double ss = 0.0;
        for (int c = p + 1 + lane; c < w; c += WAVE) ss += row[c] * row[c];
        ss = wave_sum(ss);
        const double alpha = row[p];
        double tp, beta;
        if (ss == 0.0) {
          tp = 0.0;
          beta = alpha;
        } else {
          beta = -copysign(sqrt(alpha * alpha + ss), alpha);
          tp = (beta - alpha) / beta;
          const double sc = 1.0 / (alpha - beta);
          for (int c = p + 1 + lane; c < w; c += WAVE) row[c] *= sc;
        }
        if (lane == 0) {
          row[p] = beta;
          tau[p] = tp;
        }
      }
      // T factor (forward, columnwise): T[p][p] = tau_p,
      // T[0:p, p] = -tau_p T[0:p, 0:p] (V[:, 0:p]^T v_p)
      for (int p = 0; p < pb; ++p) {
        for (int q = 0; q < p; ++q) {
          const double *vq = P + q * NMAX, *vp = P + p * NMAX;
          double s = 0.0;
          for (int c = p + lane; c < w; c += WAVE) s += (c == q ? 1.0 : vq[c]) * (c == p ? 1.0 : vp[c]);
          s = wave_sum(s);
          if (lane == 0) T[q * NB + p] = s;  // temporarily V^T v_p
        }
        if (lane == 0) {
          // y = V^T v_p (stored in column p rows 0..p-1); T[0:p,p] = -tau_p * T[0:p,0:p] y
          double y[NB];
          for (int q = 0; q < p; ++q) y[q] = T[q * NB + p];
          for (int q = 0; q < p; ++q) {
            double acc = 0.0;
            for (int r = q; r < p; ++r) acc += T[q * NB + r] * y[r];
            T[q * NB + p] = -tau[p] * acc;
          }
          T[p * NB + p] = tau[p];
          for (int q = p + 1; q < NB; ++q) T[q * NB + p] = 0.0;
        }
      }
    }
    __syncthreads();
    // store the panel back (L part and reflectors) and T/tau for the Q pass
    for (int e = tid; e < pb * w; e += blockDim.x) {
      int p = e / w, c = e % w;
      X[(int64_t)(i0 + p) * n + i0 + c] = P[p * NMAX + c];
    }
    for (int e = tid; e < NB * NB; e += blockDim.x) Ts[(int64_t)(i0 / NB) * (NB * NB + NB) + e] = T[e];
    for (int e = tid; e < NB; e += blockDim.x) Ts[(int64_t)(i0 / NB) * (NB * NB + NB) + NB * NB + e] = (e < pb) ? tau[e] : 0.0;
    // trailing rows: X_r <- X_r - (X_r V) T V^T, columns i0..n-1
    for (int r = i0 + pb + wid; r < m; r += nw) {
      double *xr = X + (int64_t)r * n + i0;
      double wv[NB];
#pragma unroll
      for (int p = 0; p < NB; ++p) wv[p] = 0.0;
      for (int c = lane; c < w; c += WAVE) {
        const double x = xr[c];
#pragma unroll
        for (int p = 0; p < NB; ++p)
          if (p < pb) wv[p] += x * (c == p ? 1.0 : (c > p ? P[p * NMAX + c] : 0.0));
      }
#pragma unroll
      for (int p = 0; p < NB; ++p) wv[p] = wave_sum(wv[p]);
      double u[NB];
#pragma unroll
      for (int p = 0; p < NB; ++p) {
        double a = 0.0;
        for (int q = 0; q <= p && q < pb; ++q) a += wv[q] * T[q * NB + p];
        u[p] = (p < pb) ? a : 0.0;
      }
      for (int c = lane; c < w; c += WAVE) {
        double d = 0.0;
#pragma unroll
        for (int p = 0; p < NB; ++p)
          if (p < pb) d += u[p] * (c == p ? 1.0 : (c > p ? P[p * NMAX + c] : 0.0));
        xr[c] -= d;
      }
    }
    __syncthreads();
  }

  // L (m x k): lower-triangular part of X
  for (int64_t e = tid; e < (int64_t)m * k; e += blockDim.x) {
    int r = (int)(e / k), c = (int)(e % k);
    Lo[e] = (c <= r) ? X[(int64_t)r * n + c] : 0.0;
  }
  // Q = [I_k 0] H_{k-1} ... H_0, panels applied last-to-first:
  // rows i0..k-1: Q_r <- Q_r - (Q_r V) T^T V^T
  for (int64_t e = tid; e < (int64_t)k * n; e += blockDim.x) {
    int r = (int)(e / n), c = (int)(e % n);
    Qo[e] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int npanel = (k + NB - 1) / NB;
  for (int pi = npanel - 1; pi >= 0; --pi) {
    const int i0 = pi * NB;
    const int pb = (k - i0) < NB ? (k - i0) : NB;
    const int w = n - i0;
    for (int e = tid; e < pb * w; e += blockDim.x) {
      int p = e / w, c = e % w;
      P[p * NMAX + c] = X[(int64_t)(i0 + p) * n + i0 + c];
    }
    for (int e = tid; e < NB * NB; e += blockDim.x) T[e] = Ts[(int64_t)pi * (NB * NB + NB) + e];
    __syncthreads();
    for (int r = i0 + wid; r < k; r += nw) {
      double *qr = Qo + (int64_t)r * n + i0;
      double wv[NB];
#pragma unroll
      for (int p = 0; p < NB; ++p) wv[p] = 0.0;
      for (int c = lane; c < w; c += WAVE) {
        const double x = qr[c];
#pragma unroll
        for (int p = 0; p < NB; ++p)
          if (p < pb) wv[p] += x * (c == p ? 1.0 : (c > p ? P[p * NMAX + c] : 0.0));
      }
#pragma unroll
      for (int p = 0; p < NB; ++p) wv[p] = wave_sum(wv[p]);
      double u[NB];
#pragma unroll
      for (int p = 0; p < NB; ++p) {  // u = w T^T : u_p = sum_q w_q T[p][q]
        double a = 0.0;
        for (int q = p; q < pb; ++q) a += wv[q] * T[p * NB + q];
        u[p] = (p < pb) ? a : 0.0;
      }
      for (int c = lane; c < w; c += WAVE) {
        double d = 0.0;
#pragma unroll
        for (int p = 0; p < NB; ++p)
          if (p < pb) d += u[p] * (c == p ? 1.0 : (c > p ? P[p * NMAX + c] : 0.0));
        qr[c] -= d;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// jacobi: one-sided block Jacobi on the rows of Y (m x n, row-major, in
// place) until the rows are mutually orthogonal.  Rows are split in blocks
// of BS; every pair of blocks (round-robin order) is staged in LDS, its
// Gram matrix G (2BS x 2BS) is diagonalised by cyclic two-sided Jacobi
// (R^T G R diagonal) and the rows are replaced by R^T rows.  A pair counts
// as converged when |G_ab| <= TOL_REL sqrt(G_aa G_bb) + TOL_ABS * Gmax for
// all a != b, Gmax the largest squared row norm.  Output: row norms s (m),
// the sweep count.
// ---------------------------------------------------------------------------
static constexpr double JAC_TOL_REL = 1e-12;
static constexpr double JAC_TOL_ABS = 1e-15;

template <int BS, int NMAX>
__global__ __launch_bounds__(256) void k_jacobi_rows(double *__restrict__ Yb, int64_t sY, int m, int n,
                                                     double *__restrict__ sb, int64_t ss,
                                                     int *__restrict__ sweeps_out, int max_sweeps) {
  constexpr int P2 = 2 * BS;
  extern __shared__ double lds[];
  double *R = lds;                 // P2 x P2 rotation
  double *G = R + P2 * P2;         // P2 x P2 Gram
  double *cs = G + P2 * P2;        // 2 * BS (c, s) of the current round
  double *scratch = cs + 2 * BS;   // 8
  double *rows = scratch + 8;      // P2 x NMAX
  double *Y = Yb + (int64_t)blockIdx.x * sY;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nblk0 = (m + BS - 1) / BS;
  const int nblk = nblk0 + (nblk0 & 1);  // even number of players (one may be empty)
  __shared__ int s_flag;
  __shared__ double s_gmax;

  // Gmax: largest squared row norm (fixed during the iteration up to rounding;
  // recomputed at each sweep)
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) { s_flag = 0; s_gmax = 0.0; }
    __syncthreads();
    {
      double gm = 0.0;
      for (int r = tid; r < m; r += nt) {
        double a = 0.0;
        for (int c = 0; c < n; ++c) a += Y[(int64_t)r * n + c] * Y[(int64_t)r * n + c];
        gm = fmax(gm, a);
      }
      gm = wave_max(gm);
      if (tid % WAVE == 0) atomicMax((unsigned long long *)&s_gmax, __double_as_longlong(gm));
    }
    __syncthreads();
    const double gmax = s_gmax;
    if (gmax == 0.0) break;
    for (int round = 0; round < nblk - 1; ++round) {
      for (int pr = 0; pr < nblk / 2; ++pr) {
        int a, b;
        rr_pair(pr, round, nblk, a, b);
        const int ra0 = a * BS, rb0 = b * BS;
        const int na = (ra0 < m) ? ((m - ra0) < BS ? (m - ra0) : BS) : 0;
        const int nbk = (rb0 < m) ? ((m - rb0) < BS ? (m - rb0) : BS) : 0;
        const int np = na + nbk;
        if (np < 2) continue;
        // stage rows: local index l < na -> row ra0 + l, else rb0 + l - na
        for (int e = tid; e < np * n; e += nt) {
          int l = e / n, c = e % n;
          int gr = (l < na) ? ra0 + l : rb0 + l - na;
          rows[l * NMAX + c] = Y[(int64_t)gr * n + c];
        }
        __syncthreads();
        // Gram (np x np): thread per (i,j), j >= i
        for (int e = tid; e < np * np; e += nt) {
          int i = e / np, j = e % np;
          if (j < i) continue;
          double acc = 0.0;
          const double *ri = rows + i * NMAX, *rj = rows + j * NMAX;
          for (int c = 0; c < n; ++c) acc = fma(ri[c], rj[c], acc);
          G[i * P2 + j] = acc;
          G[j * P2 + i] = acc;
        }
        __syncthreads();
        // convergence test on this pair
        if (tid == 0) {
          int need = 0;
          for (int i = 0; i < np && !need; ++i)
            for (int j = i + 1; j < np; ++j) {
              double g = fabs(G[i * P2 + j]);
              if (g > JAC_TOL_REL * sqrt(G[i * P2 + i] * G[j * P2 + j]) + JAC_TOL_ABS * gmax) {
                need = 1;
                break;
              }
            }
          scratch[0] = need;
        }
        __syncthreads();
        if (scratch[0] == 0.0) continue;
        if (tid == 0) s_flag = 1;
        // R = I
        for (int e = tid; e < P2 * P2; e += nt) R[e] = ((e / P2) == (e % P2)) ? 1.0 : 0.0;
        __syncthreads();
        // cyclic two-sided Jacobi on G (np x np), parallel rounds
        const int npl = np + (np & 1);
        for (int isw = 0; isw < 30; ++isw) {
          // off-diagonal check
          if (tid == 0) {
            int need = 0;
            for (int i = 0; i < np && !need; ++i)
              for (int j = i + 1; j < np; ++j) {
                double g = fabs(G[i * P2 + j]);
                if (g > 1e-15 * sqrt(G[i * P2 + i] * G[j * P2 + j]) + 1e-300) { need = 1; break; }
              }
            scratch[1] = need;
          }
          __syncthreads();
          if (scratch[1] == 0.0) break;
          for (int rd = 0; rd < npl - 1; ++rd) {
            // pairs of this inner round (circle method over npl players)
            if (tid < npl / 2) {
              int pr = tid, p, q;
              rr_pair(pr, rd, npl, p, q);
              double c = 1.0, s = 0.0;
              if (q < np) {
                const double gpq = G[p * P2 + q];
                if (gpq != 0.0) {
                  const double th = (G[q * P2 + q] - G[p * P2 + p]) / (2.0 * gpq);
                  const double t = copysign(1.0, th) / (fabs(th) + sqrt(1.0 + th * th));
                  c = 1.0 / sqrt(1.0 + t * t);
                  s = t * c;
                }
              }
              cs[2 * pr] = c;
              cs[2 * pr + 1] = s;
              // record pair indices in scratch-free way: recompute below
            }
            __syncthreads();
            // rows of G: G <- J^T G (each pair updates rows p, q)
            for (int e = tid; e < (npl / 2) * np; e += nt) {
              int pr = e / np, col = e % np, p, q;
              rr_pair(pr, rd, npl, p, q);
              if (q >= np) continue;
              const double c = cs[2 * pr], s = cs[2 * pr + 1];
              const double gp = G[p * P2 + col], gq = G[q * P2 + col];
              G[p * P2 + col] = c * gp - s * gq;
              G[q * P2 + col] = s * gp + c * gq;
            }
            __syncthreads();
            // columns of G and R: X <- X J
            for (int e = tid; e < (npl / 2) * np * 2; e += nt) {
              int which = e / ((npl / 2) * np);
              int e2 = e % ((npl / 2) * np);
              int pr = e2 / np, rr = e2 % np, p, q;
              rr_pair(pr, rd, npl, p, q);
              if (q >= np) continue;
              const double c = cs[2 * pr], s = cs[2 * pr + 1];
              double *X = which == 0 ? G : R;
              const double xp = X[rr * P2 + p], xq = X[rr * P2 + q];
              X[rr * P2 + p] = c * xp - s * xq;
              X[rr * P2 + q] = s * xp + c * xq;
            }
            __syncthreads();
          }
        }
        // rows <- R^T rows, column by column
        for (int c = tid; c < n; c += nt) {
          double v[P2];
#pragma unroll
          for (int l = 0; l < P2; ++l) v[l] = (l < np) ? rows[l * NMAX + c] : 0.0;
          for (int l = 0; l < np; ++l) {
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < P2; ++q)
              if (q < np) acc = fma(R[q * P2 + l], v[q], acc);
            rows[l * NMAX + c] = acc;
          }
        }
        __syncthreads();
        for (int e = tid; e < np * n; e += nt) {
          int l = e / n, c = e % n;
          int gr = (l < na) ? ra0 + l : rb0 + l - na;
          Y[(int64_t)gr * n + c] = rows[l * NMAX + c];
        }
        __syncthreads();
      }
    }
    __syncthreads();
    if (s_flag == 0) break;
    __syncthreads();
  }
  // row norms
  double *s = sb + (int64_t)blockIdx.x * ss;
  for (int r = tid; r < m; r += nt) {
    double a = 0.0;
    for (int c = 0; c < n; ++c) a += Y[(int64_t)r * n + c] * Y[(int64_t)r * n + c];
    s[r] = sqrt(a);
  }
  if (tid == 0) sweeps_out[blockIdx.x] = sweep + 1;
}

// ---------------------------------------------------------------------------
// svd_select: sort the row norms s (descending, ties by index), keep
// kk rows; rank = max(1, min(kk, #{s > cutoff * s_max})).  Writes the
// selected rows scaled by 1/s into W (kk x n, zero rows beyond rank), the
// rank and the discarded weight sum_{t >= rank} s_t^2.
// One workgroup per job; m <= 2048.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_svd_select(const double *__restrict__ Yb, int64_t sY, int m, int n,
                                                    const double *__restrict__ sb, int64_t ss, int kk,
                                                    double cutoff, double *__restrict__ Wb, int64_t sW,
                                                    int *__restrict__ rank_out, double *__restrict__ disc_out,
                                                    double *__restrict__ sv_out, int64_t ssv) {
  __shared__ double sv[2048];
  __shared__ int id[2048];
  __shared__ int s_rank;
  const double *Y = Yb + (int64_t)blockIdx.x * sY;
  const double *s = sb + (int64_t)blockIdx.x * ss;
  double *W = Wb + (int64_t)blockIdx.x * sW;
  const int tid = threadIdx.x;
  int P = 1;
  while (P < m) P <<= 1;
  for (int i = tid; i < P; i += blockDim.x) {
    sv[i] = (i < m) ? s[i] : -1.0;
    id[i] = i;
  }
  __syncthreads();
  // bitonic sort, descending by value, ascending by index on ties
  for (int k2 = 2; k2 <= P; k2 <<= 1) {
    for (int j = k2 >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < P; i += blockDim.x) {
        int ixj = i ^ j;
        if (ixj > i) {
          bool desc = ((i & k2) == 0);
          double a = sv[i], b = sv[ixj];
          bool a_first = (a > b) || (a == b && id[i] < id[ixj]);
          bool swap = desc ? !a_first : a_first;
          if (swap) {
            sv[i] = b; sv[ixj] = a;
            int t = id[i]; id[i] = id[ixj]; id[ixj] = t;
          }
        }
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    const double smax = sv[0];
    int r = 0;
    if (smax > 0.0) {
      for (int t = 0; t < m; ++t) if (sv[t] > cutoff * smax) ++r;
    }
    if (r < 1) r = 1;
    if (r > kk) r = kk;
    s_rank = r;
    double d = 0.0;
    for (int t = r; t < m; ++t) d += sv[t] * sv[t];
    rank_out[blockIdx.x] = r;
    disc_out[blockIdx.x] = d;
  }
  __syncthreads();
  const int r = s_rank;
  if (sv_out) {
    for (int t = tid; t < m; t += blockDim.x) sv_out[(int64_t)blockIdx.x * ssv + t] = sv[t];
  }
  for (int64_t e = tid; e < (int64_t)kk * n; e += blockDim.x) {
    int t = (int)(e / n), c = (int)(e % n);
    double v = 0.0;
    if (t < r && sv[t] > 0.0) v = Y[(int64_t)id[t] * n + c] / sv[t];
    W[e] = v;
  }
}

// ---------------------------------------------------------------------------
// svd_finish: site tensor U = Q^T (m x kk) and carried C = Q Y (computed by
// gemm beforehand into Cb); columns / rows t >= rank zeroed.
// ---------------------------------------------------------------------------
__global__ void k_svd_finish(const double *__restrict__ Qb, int64_t sQ, int m, int kk,
                             const int *__restrict__ rank, double *__restrict__ Ub, int64_t sU,
                             double *__restrict__ Cb, int64_t sC, int n) {
  const int job = blockIdx.y;
  const double *Q = Qb + (int64_t)job * sQ;
  double *U = Ub + (int64_t)job * sU;
  double *Cc = Cb + (int64_t)job * sC;
  const int r = rank[job];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)m * kk;
       e += (int64_t)gridDim.x * blockDim.x) {
    int row = (int)(e / kk), t = (int)(e % kk);
    U[e] = (t < r) ? Q[(int64_t)t * m + row] : 0.0;
  }
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)kk * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    int t = (int)(e / n);
    if (t >= r) Cc[e] = 0.0;
  }
}

// plain batched copy with strides
__global__ void k_copy(const double *__restrict__ src, int64_t ssrc, double *__restrict__ dst, int64_t sdst,
                       int64_t count) {
  const double *s = src + (int64_t)blockIdx.y * ssrc;
  double *d = dst + (int64_t)blockIdx.y * sdst;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
    d[e] = s[e];
}

// gather copy: dst[job] = src_ptrs[job] + off (count elements)
__global__ void k_gather(const CJob *__restrict__ jobs, int which, int64_t off, double *__restrict__ dst,
                         int64_t sdst, int64_t count) {
  const CJob jb = jobs[blockIdx.y];
  const double *s = (which == 0 ? jb.in_a : jb.in_b) + off;
  double *d = dst + (int64_t)blockIdx.y * sdst;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
    d[e] = s[e];
}

// scatter copy: jobs[job].out + off <- src[job]
__global__ void k_scatter(const CJob *__restrict__ jobs, int64_t off, const double *__restrict__ src,
                          int64_t ssrc, int64_t count) {
  const CJob jb = jobs[blockIdx.y];
  const double *s = src + (int64_t)blockIdx.y * ssrc;
  double *d = jb.out + off;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
    d[e] = s[e];
}

// ---------------------------------------------------------------------------
// overlap: E_j = sum_n A_j^{nT} E_{j-1} B_j^n for a batch of MPS pairs, one
// workgroup per pair, E held in global scratch (ping-pong).  FP64.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_overlap(const OJob *__restrict__ jobs, int n_sites,
                                                 const int *__restrict__ bonds_a, const int64_t *__restrict__ off_a,
                                                 const int *__restrict__ bonds_b, const int64_t *__restrict__ off_b,
                                                 double *__restrict__ scratch, int64_t s_scr, double *__restrict__ out) {
  const OJob jb = jobs[blockIdx.x];
  double *E0 = scratch + (int64_t)blockIdx.x * s_scr;
  double *F = E0 + s_scr / 3;        // F = E A^n stage  (la x? ) sized by caller
  double *E1 = E0 + 2 * (s_scr / 3);
  const int tid = threadIdx.x;
  if (tid == 0) E0[0] = 1.0;
  __syncthreads();
  double *Ecur = E0, *Enext = E1;
  for (int j = 0; j < n_sites; ++j) {
    const int la = bonds_a[j], ra = bonds_a[j + 1], lb = bonds_b[j], rb = bonds_b[j + 1];
    const double *A = jb.a + off_a[j];
    const double *B = jb.b + off_b[j];
    // Enext[c][d] = sum_n sum_a (sum_b E[a][b] B[b][n][d]) A[a][n][c]
    for (int e = tid; e < ra * rb; e += blockDim.x) Enext[e] = 0.0;
    __syncthreads();
    for (int nn = 0; nn < 2; ++nn) {
      // F[a][d] = sum_b E[a][b] B[b][nn][d]
      for (int e = tid; e < la * rb; e += blockDim.x) {
        int a = e / rb, d = e % rb;
        double acc = 0.0;
        for (int b = 0; b < lb; ++b) acc = fma(Ecur[a * lb + b], B[((int64_t)b * 2 + nn) * rb + d], acc);
        F[e] = acc;
      }
      __syncthreads();
      for (int e = tid; e < ra * rb; e += blockDim.x) {
        int c = e / rb, d = e % rb;
        double acc = 0.0;
        for (int a = 0; a < la; ++a) acc = fma(A[((int64_t)a * 2 + nn) * ra + c], F[a * rb + d], acc);
        Enext[e] += acc;
      }
      __syncthreads();
    }
    double *t = Ecur; Ecur = Enext; Enext = t;
  }
  if (tid == 0) out[blockIdx.x] = Ecur[0];
}

// repack: dst (bonds rl x 2 x rr, packed at doff) <- leading block of src
// stored with static bonds (ks_l x 2 x ks_r) at soff.
__global__ void k_repack(const double *__restrict__ src, int64_t soff, int ks_l, int ks_r, double *__restrict__ dst,
                         int64_t doff, int rl, int rr) {
  const int64_t total = (int64_t)rl * 2 * rr;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int b = (int)(e % rr), m = (int)((e / rr) % 2), a = (int)(e / (2 * (int64_t)rr));
    dst[doff + e] = src[soff + ((int64_t)a * 2 + m) * ks_r + b];
  }
  (void)ks_l;
}

__global__ void k_scale_range(double *__restrict__ p, int64_t count, double c) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
    p[e] *= c;
}

// ---------------------------------------------------------------------------
// small dense symmetric eigensolver (cyclic Jacobi), one workgroup, m <= 64.
// Computes the Ritz values of the Lanczos step:
//   mode 0: eigenvalues of the tridiagonal (alpha, beta);
//   mode 1: eigenvalues of C H_sym C^T with C S C^T = I (Cholesky of S), or
//           of X^T H_sym X with X = U_k s_k^{-1/2} when S is not positive
//           definite enough (canonical orthogonalisation, s > 1e-10).
// ---------------------------------------------------------------------------
__device__ void jacobi_eig_small(double *A, int m, int lda, double *w) {
  // serial cyclic Jacobi (m tiny), run by one thread
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        tot += A[i * lda + j] * A[i * lda + j];
        if (i != j) off += A[i * lda + j] * A[i * lda + j];
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) {
        const double apq = A[p * lda + q];
        if (apq == 0.0) continue;
        const double th = (A[q * lda + q] - A[p * lda + p]) / (2.0 * apq);
        const double t = copysign(1.0, th) / (fabs(th) + sqrt(1.0 + th * th));
        const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < m; ++k) {
          const double ap = A[p * lda + k], aq = A[q * lda + k];
          A[p * lda + k] = c * ap - s * aq;
          A[q * lda + k] = s * ap + c * aq;
        }
        for (int k = 0; k < m; ++k) {
          const double ap = A[k * lda + p], aq = A[k * lda + q];
          A[k * lda + p] = c * ap - s * aq;
          A[k * lda + q] = s * ap + c * aq;
        }
      }
  }
  for (int i = 0; i < m; ++i) w[i] = A[i * lda + i];
  // ascending insertion sort
  for (int i = 1; i < m; ++i) {
    double v = w[i];
    int j = i - 1;
    while (j >= 0 && w[j] > v) { w[j + 1] = w[j]; --j; }
    w[j + 1] = v;
  }
}

__global__ void k_ritz(const double *__restrict__ Mm, const double *__restrict__ S, int m, int ld,
                       const double *__restrict__ alpha, const double *__restrict__ beta,
                       double *__restrict__ out_gen, double *__restrict__ out_tri, int *__restrict__ info) {
  constexpr int LD = RITZ_MAX;
  __shared__ double H[LD * LD], Sc[LD * LD], C[LD * LD], T1[LD * LD], wv[LD];
  if (threadIdx.x != 0) return;
  // tridiagonal
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) T1[i * LD + j] = 0.0;
  for (int i = 0; i < m; ++i) T1[i * LD + i] = alpha[i];
  for (int i = 0; i + 1 < m; ++i) { T1[i * LD + i + 1] = beta[i]; T1[(i + 1) * LD + i] = beta[i]; }
  jacobi_eig_small(T1, m, LD, wv);
  for (int i = 0; i < m; ++i) out_tri[i] = wv[i];
  // generalised
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      H[i * LD + j] = 0.5 * (Mm[i * ld + j] + Mm[j * ld + i]);
      Sc[i * LD + j] = S[i * ld + j];
    }
  // Cholesky S = L L^T (in Sc, lower)
  bool ok = true;
  for (int j = 0; j < m && ok; ++j) {
    double d = Sc[j * LD + j];
    for (int k = 0; k < j; ++k) d -= Sc[j * LD + k] * Sc[j * LD + k];
    if (!(d > 1e-10)) { ok = false; break; }
    d = sqrt(d);
    Sc[j * LD + j] = d;
    for (int i = j + 1; i < m; ++i) {
      double v = Sc[i * LD + j];
      for (int k = 0; k < j; ++k) v -= Sc[i * LD + k] * Sc[j * LD + k];
      Sc[i * LD + j] = v / d;
    }
  }
  int mk = m;
  if (ok) {
    // C = L^{-1} (lower), by forward substitution on the identity
    for (int col = 0; col < m; ++col)
      for (int i = 0; i < m; ++i) {
        double v = (i == col) ? 1.0 : 0.0;
        for (int k = 0; k < i; ++k) v -= Sc[i * LD + k] * C[k * LD + col];
        C[i * LD + col] = (i < col) ? 0.0 : v / Sc[i * LD + i];
      }
  } else {
    // canonical orthogonalisation: S = U diag(s) U^T, keep s > 1e-10,
    // C = diag(s_k^{-1/2}) U_k^T  (rows)
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) { T1[i * LD + j] = S[i * ld + j]; C[i * LD + j] = (i == j) ? 1.0 : 0.0; }
    // Jacobi with eigenvectors
    for (int sweep = 0; sweep < 100; ++sweep) {
      double off = 0.0, tot = 0.0;
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) { tot += T1[i * LD + j] * T1[i * LD + j]; if (i != j) off += T1[i * LD + j] * T1[i * LD + j]; }
      if (off <= 1e-30 * tot || off == 0.0) break;
      for (int p = 0; p < m; ++p)
        for (int q = p + 1; q < m; ++q) {
          const double apq = T1[p * LD + q];
          if (apq == 0.0) continue;
          const double th = (T1[q * LD + q] - T1[p * LD + p]) / (2.0 * apq);
          const double t = copysign(1.0, th) / (fabs(th) + sqrt(1.0 + th * th));
          const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
          for (int k = 0; k < m; ++k) {
            const double ap = T1[p * LD + k], aq = T1[q * LD + k];
            T1[p * LD + k] = c * ap - s * aq; T1[q * LD + k] = s * ap + c * aq;
          }
          for (int k = 0; k < m; ++k) {
            const double ap = T1[k * LD + p], aq = T1[k * LD + q];
            T1[k * LD + p] = c * ap - s * aq; T1[k * LD + q] = s * ap + c * aq;
          }
          for (int k = 0; k < m; ++k) {  // eigenvector columns in C (C <- C J)
            const double ap = C[k * LD + p], aq = C[k * LD + q];
            C[k * LD + p] = c * ap - s * aq; C[k * LD + q] = s * ap + c * aq;
          }
        }
    }
    // rows of the transform: X^T rows = u_k^T / sqrt(s_k) for s_k > 1e-10
    mk = 0;
    for (int k = 0; k < m; ++k) {
      const double sk = T1[k * LD + k];
      if (sk > 1e-10) {
        for (int i = 0; i < m; ++i) Sc[mk * LD + i] = C[i * LD + k] / sqrt(sk);
        ++mk;
      }
    }
    for (int r = 0; r < mk; ++r)
      for (int i = 0; i < m; ++i) C[r * LD + i] = Sc[r * LD + i];
  }
  // T1 = C H C^T (mk x mk)
  for (int i = 0; i < mk; ++i)
    for (int j = 0; j < m; ++j) {
      double v = 0.0;
      for (int k = 0; k < m; ++k) v += C[i * LD + k] * H[k * LD + j];
      Sc[i * LD + j] = v;
    }
  for (int i = 0; i < mk; ++i)
    for (int j = 0; j < mk; ++j) {
      double v = 0.0;
      for (int k = 0; k < m; ++k) v += Sc[i * LD + k] * C[j * LD + k];
      T1[i * LD + j] = v;
    }
  jacobi_eig_small(T1, mk, LD, wv);
  for (int i = 0; i < m; ++i) out_gen[i] = (i < mk) ? wv[i] : 0.0;
  info[0] = ok ? 0 : 1;
  info[1] = mk;
}

// ---------------------------------------------------------------------------
// host launch wrappers
// ---------------------------------------------------------------------------
static inline int cdiv64(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

void launch_construct(hipStream_t st, const CJob *jobs, int nb, int site, int n_sites, int64_t in_off_a,
                      int64_t in_off_b, int la, int ra, int lb, int rb, double *out, int64_t out_stride, int lo,
                      int ro) {
  int64_t total = (int64_t)lo * 2 * ro;
  int gx = cdiv64(total, 256);
  if (gx > 4096) gx = 4096;
  hipLaunchKernelGGL(k_construct, dim3(gx, nb), dim3(256), 0, st, jobs, site, n_sites, in_off_a, in_off_b, la,
                     ra, lb, rb, out, out_stride, lo, ro);
}

void launch_gemm(hipStream_t st, int nb, bool transB, const double *A, int64_t sA, int lda, const double *B,
                 int64_t sB, int ldb, double *C, int64_t sC, int ldc, int M, int N, int K) {
  dim3 grid(cdiv64(N, 64), cdiv64(M, 64), nb);
  if (transB)
    hipLaunchKernelGGL(k_gemm_f64<true>, grid, dim3(256), 0, st, A, sA, lda, B, sB, ldb, C, sC, ldc, M, N, K);
  else
    hipLaunchKernelGGL(k_gemm_f64<false>, grid, dim3(256), 0, st, A, sA, lda, B, sB, ldb, C, sC, ldc, M, N, K);
}

int lq_t_stride(int k) {
  const int NB = 16;
  return ((k + NB - 1) / NB) * (NB * NB + NB);
}

int launch_lq(hipStream_t st, int nb, double *X, int64_t sX, int m, int n, double *L, int64_t sL, double *Q,
              int64_t sQ, double *Tw, int64_t sT) {
  constexpr int NB = 16;
  if (n <= 1024) {
    constexpr int NMAX = 1024;
    size_t lds = (NB * NMAX + NB * NB + NB + 4) * sizeof(double);
    static bool attr = false;
    if (!attr) {
      (void)hipFuncSetAttribute((const void *)k_lq<NB, NMAX>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      attr = true;
    }
    hipLaunchKernelGGL((k_lq<NB, NMAX>), dim3(nb), dim3(256), lds, st, X, sX, m, n, L, sL, Q, sQ, Tw, sT);
    return 0;
  }
  return -1;
}

int launch_jacobi(hipStream_t st, int nb, double *Y, int64_t sY, int m, int n, double *s, int64_t ss,
                  int *sweeps, int max_sweeps) {
  if (n <= 512) {
    constexpr int BS = 16, NMAX = 512;
    size_t lds = (2 * (2 * BS) * (2 * BS) + 2 * BS + 8 + 2 * BS * NMAX) * sizeof(double);
    static bool attr = false;
    if (!attr) {
      (void)hipFuncSetAttribute((const void *)k_jacobi_rows<BS, NMAX>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
      attr = true;
    }
    hipLaunchKernelGGL((k_jacobi_rows<BS, NMAX>), dim3(nb), dim3(256), lds, st, Y, sY, m, n, s, ss, sweeps,
                       max_sweeps);
    return 0;
  }
  if (n <= 1024) {
    constexpr int BS = 8, NMAX = 1024;
    size_t lds = (2 * (2 * BS) * (2 * BS) + 2 * BS + 8 + 2 * BS * NMAX) * sizeof(double);
    static bool attr = false;
    if (!attr) {
      (void)hipFuncSetAttribute((const void *)k_jacobi_rows<BS, NMAX>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
      attr = true;
    }
    hipLaunchKernelGGL((k_jacobi_rows<BS, NMAX>), dim3(nb), dim3(256), lds, st, Y, sY, m, n, s, ss, sweeps,
                       max_sweeps);
    return 0;
  }
  return -1;
}

void launch_svd_select(hipStream_t st, int nb, const double *Y, int64_t sY, int m, int n, const double *s,
                       int64_t ss, int kk, double cutoff, double *W, int64_t sW, int *rank, double *disc,
                       double *sv_out, int64_t ssv) {
  hipLaunchKernelGGL(k_svd_select, dim3(nb), dim3(256), 0, st, Y, sY, m, n, s, ss, kk, cutoff, W, sW, rank, disc,
                     sv_out, ssv);
}

void launch_svd_finish(hipStream_t st, int nb, const double *Q, int64_t sQ, int m, int kk, const int *rank,
                       double *U, int64_t sU, double *C, int64_t sC, int n) {
  int gx = cdiv64((int64_t)m * kk > (int64_t)kk * n ? (int64_t)m * kk : (int64_t)kk * n, 256);
  if (gx > 2048) gx = 2048;
  hipLaunchKernelGGL(k_svd_finish, dim3(gx, nb), dim3(256), 0, st, Q, sQ, m, kk, rank, U, sU, C, sC, n);
}

void launch_copy(hipStream_t st, int nb, const double *src, int64_t ssrc, double *dst, int64_t sdst, int64_t count) {
  int gx = cdiv64(count, 256);
  if (gx > 2048) gx = 2048;
  if (gx < 1) gx = 1;
  hipLaunchKernelGGL(k_copy, dim3(gx, nb), dim3(256), 0, st, src, ssrc, dst, sdst, count);
}

void launch_gather(hipStream_t st, int nb, const CJob *jobs, int which, int64_t off, double *dst, int64_t sdst,
                   int64_t count) {
  int gx = cdiv64(count, 256);
  if (gx > 2048) gx = 2048;
  if (gx < 1) gx = 1;
  hipLaunchKernelGGL(k_gather, dim3(gx, nb), dim3(256), 0, st, jobs, which, off, dst, sdst, count);
}

void launch_scatter(hipStream_t st, int nb, const CJob *jobs, int64_t off, const double *src, int64_t ssrc,
                    int64_t count) {
  int gx = cdiv64(count, 256);
  if (gx > 2048) gx = 2048;
  if (gx < 1) gx = 1;
  hipLaunchKernelGGL(k_scatter, dim3(gx, nb), dim3(256), 0, st, jobs, off, src, ssrc, count);
}

void launch_overlap(hipStream_t st, int nb, const OJob *jobs, int n_sites, const int *bonds_a, const int64_t *off_a,
                    const int *bonds_b, const int64_t *off_b, double *scratch, int64_t s_scr, double *out) {
  hipLaunchKernelGGL(k_overlap, dim3(nb), dim3(256), 0, st, jobs, n_sites, bonds_a, off_a, bonds_b, off_b, scratch,
                     s_scr, out);
}

void launch_repack(hipStream_t st, int gx, const double *src, int64_t soff, int ks_l, int ks_r, double *dst,
                   int64_t doff, int rl, int rr) {
  hipLaunchKernelGGL(k_repack, dim3(gx), dim3(256), 0, st, src, soff, ks_l, ks_r, dst, doff, rl, rr);
}

void launch_scale(hipStream_t st, double *p, int64_t count, double c) {
  int gx = cdiv64(count, 256);
  if (gx > 2048) gx = 2048;
  if (gx < 1) gx = 1;
  hipLaunchKernelGGL(k_scale_range, dim3(gx), dim3(256), 0, st, p, count, c);
}

void launch_ritz(hipStream_t st, const double *Mm, const double *S, int m, int ld, const double *alpha,
                 const double *beta, double *out_gen, double *out_tri, int *info) {
  hipLaunchKernelGGL(k_ritz, dim3(1), dim3(64), 0, st, Mm, S, m, ld, alpha, beta, out_gen, out_tri, info);
}

}  // namespace thck
