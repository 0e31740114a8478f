// Two-stage tridiagonalisation of the symmetric Gram matrices of the SVD step
// (the eigen route to the truncated SVD of Fig. 3), m <= 512, one matrix per
// workgroup:
//   sy2sb     dense -> band of half-bandwidth BW = 16 by blocked Householder
//             panels; the trailing matrix is touched three times per panel of
//             16 columns (update, panel read, product) instead of once per
//             column as in the one-stage reduction.
//   sb2st     band -> tridiagonal by Householder bulge chasing with the band
//             resident in LDS; up to eight sweeps run at once, one per wave.
//   q2apply   eigenvectors of the tridiagonal -> eigenvectors of the band
//             (the chase's reflectors, last sweep first).
// The panel reflectors of sy2sb are stored like those of the one-stage
// reduction, shifted by BW rows, and are applied afterwards by ormtr with a
// row offset of BW.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "device_util.h"
#include "kernels.h"

namespace thck {

namespace {
constexpr int BW = 16;          // half-bandwidth of the intermediate band
constexpr int VLD = 17;         // row stride of the n x 16 panel arrays in LDS
constexpr int R_ROWS = 512 - 16; // rows of the panel arrays (m <= 512)
constexpr int NT = 512;         // threads per workgroup
constexpr int NW = NT / WAVE;   // waves per workgroup

// 1/b from the hardware estimate and two Newton steps, for normal |b|
__device__ __forceinline__ double rcp2(double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(r, fma(-b, r, 1.0), r);
  return fma(r, fma(-b, r, 1.0), r);
}

// Householder reflector H = I - tau v v^T, v[0] = 1, H x = beta e_0, from
// alpha = x[0], amx = max |x[1:]|, s2 = |x[1:]|^2.  Returns false when the
// squares are out of range and the caller must supply the scaled sum s3 of
// (x[1:] / max(amx, |alpha|))^2 to house_scaled.
__device__ __forceinline__ bool house_direct(double alpha, double amx, double s2, double &tau, double &sc,
                                             double &beta) {
  if (!(amx > 1e-290)) {  // nothing below the first entry but denormal dust: no reflection
    tau = 0.0;
    sc = 0.0;
    beta = alpha;
    return true;
  }
  if (s2 > 1e-280 && s2 < 1e280 && fabs(alpha) < 1e140) {
    const double bs = -copysign(sqrt(alpha * alpha + s2), alpha);
    // |bs| >= amx > 1e-290 and |alpha - bs| >= |bs|: reciprocal estimates
    // refined by two Newton steps (a few ulps) instead of full divisions
    tau = (bs - alpha) * rcp2(bs);
    sc = rcp2(alpha - bs);
    beta = bs;
    return true;
  }
  return false;
}
__device__ __forceinline__ void house_scaled(double alpha, double scl, double s3, double &tau, double &sc,
                                             double &beta) {
  const double inv = 1.0 / scl, as = alpha * inv;
  const double bs = -copysign(sqrt(as * as + s3), as);
  tau = (bs - as) / bs;
  sc = inv / (as - bs);
  beta = bs * scl;
}

// The 16 x 16 tile (row0, col0) of a symmetric matrix stored as its upper
// triangle (row-major, m x m), in the MFMA accumulator layout: register r of
// lane (li, lk) holds element (lk + 4r, li).  On a diagonal tile the lower
// elements are read from their mirror; past m the tile reads 0.
__device__ __forceinline__ d4_t load_sym_tile(const double *A, int m, int row0, int col0, int li, int lk) {
  d4_t t;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int a = lk + 4 * r, b = li;
    if (row0 == col0 && a > b) {
      const int s = a;
      a = b;
      b = s;
    }
    const int gr = row0 + a, gc = col0 + b;
    t[r] = (gr < m && gc < m) ? A[(int64_t)gr * m + gc] : 0.0;
  }
  return t;
}
__device__ __forceinline__ void store_sym_tile(double *A, int m, int row0, int col0, int li, int lk, d4_t t) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int a = lk + 4 * r, b = li;
    const int gr = row0 + a, gc = col0 + b;
    if (gr < m && gc < m && (row0 != col0 || a <= b)) A[(int64_t)gr * m + gc] = t[r];
  }
}

// Upper-triangle tile t (row-major over the nt x nt tile grid) -> (I, J).
__device__ __forceinline__ void tile_ij(int t, int nt, int &I, int &J) {
  I = 0;
  while (t >= nt - I) {
    t -= nt - I;
    ++I;
  }
  J = I + t;
}

// A[base:, base:] -= V Y^T + Y V^T on the upper triangle, V and Y (rows
// relative to base, 16 columns) in LDS.  Each wave takes every NW-th tile and
// keeps the next PD - 1 of its tiles in flight while it updates one.
__device__ void band_update(double *A, int m, int base, const double *Vs, const double *Ys, int wvs, int li,
                            int lk) {
  constexpr int PD = 6;
  const int nn = m - base, nt = (nn + 15) / 16, ntiles = nt * (nt + 1) / 2;
  const int count = wvs < ntiles ? (ntiles - wvs + NW - 1) / NW : 0;
  d4_t buf[PD];
  auto load = [&](int i) {
    int I, J;
    tile_ij(wvs + NW * i, nt, I, J);
    return load_sym_tile(A, m, base + 16 * I, base + 16 * J, li, lk);
  };
#pragma unroll
  for (int u = 0; u < PD - 1; ++u)
    if (u < count) buf[u] = load(u);
  for (int i0 = 0; i0 < count; i0 += PD) {
#pragma unroll
    for (int u = 0; u < PD; ++u) {
      const int i = i0 + u;
      if (i < count) {
        if (i + PD - 1 < count) buf[(u + PD - 1) % PD] = load(i + PD - 1);
        int I, J;
        tile_ij(wvs + NW * i, nt, I, J);
        d4_t acc = buf[u];
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
          const int k = 4 * kc + lk;
          acc = mfma16(-Vs[(16 * I + li) * VLD + k], Ys[(16 * J + li) * VLD + k], acc);
          acc = mfma16(-Ys[(16 * I + li) * VLD + k], Vs[(16 * J + li) * VLD + k], acc);
        }
        store_sym_tile(A, m, base + 16 * I, base + 16 * J, li, lk, acc);
      }
    }
  }
}

// Ys += A[base:, base:] V for the symmetric A (upper triangle read once), V in
// Vs.  Tile (I, J), I < J, adds A_IJ V_J to block row I and A_IJ^T V_I to
// block row J, so two waves must not hold tiles that share a block row: the
// tiles are dealt in rounds of a round-robin over the block rows (odd count
// P; in round rr, blocks i and j with i + j = 2 rr mod P meet and block rr
// takes its diagonal tile), and each round's tiles touch disjoint block rows.
// A wave holds at most two tiles per round (P <= 31) and loads the next
// round's while it multiplies; the transposed product reads the tile through
// the wave's LDS scratch.
__device__ __forceinline__ bool round_tile(int rr, int s, int P, int nt, int &I, int &J) {
  int i = rr, j = rr;
  if (s > 0) {
    i = (rr + s) % P;
    j = (rr - s + P) % P;
  }
  I = i < j ? i : j;
  J = i < j ? j : i;
  return s <= P / 2 && i < nt && j < nt;
}

__device__ void band_product(const double *A, int m, int base, const double *Vs, double *Ys, double *scw, int wvs,
                             int li, int lk) {
  const int nn = m - base, nt = (nn + 15) / 16, P = nt | 1;
  d4_t cur[2], nxt[2];
  bool cv[2], nv[2];
  int cI[2], cJ[2], nI[2], nJ[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    cv[u] = round_tile(0, wvs + NW * u, P, nt, cI[u], cJ[u]);
    if (cv[u]) cur[u] = load_sym_tile(A, m, base + 16 * cI[u], base + 16 * cJ[u], li, lk);
  }
  for (int rr = 0; rr < P; ++rr) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      nv[u] = rr + 1 < P && round_tile(rr + 1, wvs + NW * u, P, nt, nI[u], nJ[u]);
      if (nv[u]) nxt[u] = load_sym_tile(A, m, base + 16 * nI[u], base + 16 * nJ[u], li, lk);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (cv[u]) {
        const int I = cI[u], J = cJ[u];
        const d4_t t = cur[u];
        // block row J: (V_I^T A_IJ)^T, register r <-> (column li of block J, reflector lk + 4r)
        d4_t x1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) x1 = mfma16(Vs[(16 * I + 4 * kc + lk) * VLD + li], t[kc], x1);
#pragma unroll
        for (int r = 0; r < 4; ++r) Ys[(16 * J + li) * VLD + lk + 4 * r] += x1[r];
        if (I != J) {
          // block row I: (V_J^T A_IJ^T)^T with A_IJ^T read from the scratch
#pragma unroll
          for (int r = 0; r < 4; ++r) scw[(lk + 4 * r) * VLD + li] = t[r];
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
          d4_t x2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int kc = 0; kc < 4; ++kc)
            x2 = mfma16(Vs[(16 * J + 4 * kc + lk) * VLD + li], scw[li * VLD + 4 * kc + lk], x2);
#pragma unroll
          for (int r = 0; r < 4; ++r) Ys[(16 * I + li) * VLD + lk + 4 * r] += x2[r];
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
        }
      }
    }
    lds_barrier();  // the next round's tiles stay in flight
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      cur[u] = nxt[u];
      cv[u] = nv[u];
      cI[u] = nI[u];
      cJ[u] = nJ[u];
    }
  }
}

// out[a][b] (16 x 16, row stride 16) = sum over rows of X[row][a] Y[row][b]
// for the R-row LDS arrays X, Y: each wave multiplies its 64 rows on MFMA,
// the partials meet in the scratch.  Ends with the result in out; the
// caller's barrier must follow before out is read by other threads.
__device__ void gram16(const double *X, const double *Y, int R, double *sc, double *out, int tid, int wvs, int li,
                       int lk) {
  d4_t g = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int c4 = 0; c4 < 16; ++c4) {
    const int row = 64 * wvs + 4 * c4 + lk;
    const double a = row < R ? X[row * VLD + li] : 0.0;
    const double b = row < R ? Y[row * VLD + li] : 0.0;
    g = mfma16(a, b, g);
  }
  double *sw = sc + wvs * 16 * VLD;
#pragma unroll
  for (int r = 0; r < 4; ++r) sw[(lk + 4 * r) * VLD + li] = g[r];
  lds_barrier();
  if (tid < 256) {
    const int a = tid / 16, b = tid % 16;
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += sc[w * 16 * VLD + a * VLD + b];
    out[tid] = s;
  }
}
}  // namespace

// Householder QR of the n x 16 panel P = A^T[r0:, c0:c0+16] (column q of P is
// row c0 + q of the stored upper triangle, from column r0 on), by columns:
// wave w holds columns w and w + 8 in registers (rows l + 64 i in lane l).
// Column q's owner applies the earlier reflectors to it (as every wave does
// to its columns), forms reflector q, writes v to V (rows of stride VLD) and
// tau to tl; after the barrier every wave applies it to its columns after q.
// At the end each wave stores its columns (R above the diagonal, beta on
// it, the reflector tail below) back to A.
__device__ void panel_qr_cols(double *A, int m, int c0, int r0, int n, double *V, double *tl, int wvs, int lane) {
  constexpr int RPL = 8;  // rows per lane (n <= 512)
  double col[2][RPL];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int q = wvs + NW * h;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int t = lane + WAVE * i;
      col[h][i] = (t < n) ? A[(int64_t)(c0 + q) * m + r0 + t] : 0.0;
    }
  }
#pragma unroll
  for (int h2 = 0; h2 < 2; ++h2) {
#pragma unroll 1
    for (int qq = 0; qq < NW; ++qq) {
      const int q = qq + NW * h2;
      if (wvs == qq) {  // the owner of column q (its register slot h2)
        double x[RPL];
        double am = 0.0, ss = 0.0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int t = lane + WAVE * i;
          x[i] = (t > q && t < n) ? col[h2][i] : 0.0;
          am = fmax(am, fabs(x[i]));
          ss = fma(x[i], x[i], ss);
        }
        const double amx = wave_max(am), s2 = wave_sum(ss);
        const double alpha = read_lane(col[h2][0], q);  // row q < 16: lane q, i = 0
        double tp, scv, ei;
        if (!house_direct(alpha, amx, s2, tp, scv, ei)) {
          const double scl = fmax(amx, fabs(alpha)), inv = 1.0 / scl;
          double s3 = 0.0;
#pragma unroll
          for (int i = 0; i < RPL; ++i) s3 = fma(x[i] * inv, x[i] * inv, s3);
          house_scaled(alpha, scl, wave_sum(s3), tp, scv, ei);
        }
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int t = lane + WAVE * i;
          const double v = (t == q) ? ((q < n) ? 1.0 : 0.0) : x[i] * scv;
          if (t < R_ROWS) V[t * VLD + q] = (t < n) ? v : 0.0;
          if (t == q) col[h2][i] = ei;
          else if (t > q) col[h2][i] = v;
        }
        if (lane == 0) tl[q] = tp;
      }
      lds_barrier();
      // H_q on this wave's columns after q: c -= tau (v . c) v (rows >= q)
      const double tp = tl[q];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int c = wvs + NW * h;
        if (c > q) {
          double vv[RPL], acc = 0.0;
#pragma unroll
          for (int i = 0; i < RPL; ++i) {
            const int t = lane + WAVE * i;
            vv[i] = (t >= q && t < n) ? V[t * VLD + q] : 0.0;
            acc = fma(vv[i], col[h][i], acc);
          }
          const double f = tp * wave_sum(acc);
#pragma unroll
          for (int i = 0; i < RPL; ++i) col[h][i] -= f * vv[i];
        }
      }
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int q = wvs + NW * h;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int t = lane + WAVE * i;
      if (t < n) A[(int64_t)(c0 + q) * m + r0 + t] = col[h][i];
    }
  }
  lds_barrier();  // V and tl complete for every wave
}

// ---------------------------------------------------------------------------
// sy2sb: Q1^T A Q1 = B with B of half-bandwidth 16, for the symmetric A given
// by its upper triangle (row-major, row stride m, m <= 512).  Panel p (columns
// c0 = 16p .. c0+15, rows r0 = c0+16 .. m-1):
//   * the previous panel's two-sided update A[c0:, c0:] -= V Y^T + Y V^T;
//   * Householder QR of the panel (thread t holds panel row t in registers),
//     R into the band, the reflector tails after it: reflector i = c0 + q has
//     v[i+16] = 1 and v[r] = A[i][r] for r > i+16, tau[i];
//   * compact-WY T of the panel (V^T V on MFMA);
//   * X = A22 V (A22 = A[r0:, r0:], upper triangle read once, MFMA tiles),
//     then Y = X T - V (T^T V^T X T) / 2, so that Q^T A22 Q = A22 - V Y^T - Y V^T.
// The band is left in the upper triangle (A[c][c..c+16]).
// ---------------------------------------------------------------------------
template <int MMAX>
__global__ __launch_bounds__(512) void k_sy2sb(double *__restrict__ Ab, int64_t sA, int m, double *__restrict__ taub,
                                                int64_t sv, const int *__restrict__ only) {
  if (only != nullptr && only[blockIdx.x] == 0) return;  // job not selected
  constexpr int R = MMAX - BW;
  extern __shared__ double lds[];
  double *Vs = lds;                 // R x VLD: panel reflectors, rows relative to r0
  double *Ys = Vs + R * VLD;        // R x VLD: X, then Y
  double *sc = Ys + R * VLD;        // NW x 16 x VLD: per-wave 16 x 16 scratch
  double *Tm = sc + NW * 16 * VLD;  // 16 x 16 (upper triangular T)
  double *Gq = Tm + 256;            // 16 x 16
  double *red = Gq + 256;           // 4 NW + 1 + NW * 16
  double *tl = red + 4 * NW + 1 + NW * BW;  // 16
  double *A = Ab + (int64_t)blockIdx.x * sA;
  double *tau = taub + (int64_t)blockIdx.x * sv;
  const int tid = threadIdx.x, lane = tid % WAVE, wid = tid / WAVE;
  const int wvs = __builtin_amdgcn_readfirstlane(wid);
  const int li = lane & 15, lk = lane >> 4;
  double *scw = sc + wvs * 16 * VLD;

  for (int e = tid; e < 2 * R * VLD; e += NT) Vs[e] = 0.0;  // Vs and Ys
  lds_barrier();

  for (int c0 = 0;; c0 += BW) {
    if (c0 > 0) {
      band_update(A, m, c0, Vs, Ys, wvs, li, lk);
      __syncthreads();  // the panel load below reads what other waves stored
    }
    const int r0 = c0 + BW, n = m - r0;
    if (n < 2) break;
    // ---- panel QR: wave w owns panel columns w and w + 8 (rows l + 64 i in
    //      lane l); column q's owner forms its reflector (wave reductions)
    //      and writes v to Vs, then every wave applies it to its later
    //      columns: one barrier per column ----
    for (int e = n + tid; e < R; e += NT)
      for (int q = 0; q < BW; ++q) Vs[e * VLD + q] = 0.0;  // rows past the panel: V = 0
    panel_qr_cols(A, m, c0, r0, n, Vs, tl, wvs, lane);
    if (tid < BW) tau[c0 + tid] = tl[tid];
    // ---- T: G = V^T V, T[0:p, p] = -tau_p T[0:p, 0:p] G[0:p, p] ----
    gram16(Vs, Vs, R, sc, Gq, tid, wvs, li, lk);
    lds_barrier();
    if (tid < BW) {
      const int q = tid;  // this thread's row of T
      for (int p = 0; p < BW; ++p) {
        double x = 0.0;
        if (q < p) {
          double acc = 0.0;
          for (int r = q; r < p; ++r) acc += Tm[q * 16 + r] * Gq[r * 16 + p];
          x = -tl[p] * acc;
        } else if (q == p) {
          x = tl[p];
        }
        Tm[q * 16 + p] = x;
      }
    }
    // ---- X = A22 V ----
    for (int e = tid; e < R * VLD; e += NT) Ys[e] = 0.0;
    lds_barrier();
    band_product(A, m, r0, Vs, Ys, scw, wvs, li, lk);
    // ---- Y = X T - V (T^T V^T X T) / 2, on MFMA tiles of 16 rows ----
    const int ntr = (n + 15) / 16;
    for (int I = wvs; I < ntr; I += NW) {  // Y <- X T
      double xa[4], tb[4];
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        xa[kc] = Ys[(16 * I + li) * VLD + 4 * kc + lk];
        tb[kc] = Tm[(4 * kc + lk) * 16 + li];
      }
      d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) acc = mfma16(xa[kc], tb[kc], acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) Ys[(16 * I + lk + 4 * r) * VLD + li] = acc[r];
    }
    lds_barrier();
    gram16(Vs, Ys, R, sc, Gq, tid, wvs, li, lk);  // Gq = V^T X T
    lds_barrier();
    if (wvs == 0) {  // Gq <- -(T^T Gq) / 2
      double ta[4], wb[4];
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        ta[kc] = Tm[(4 * kc + lk) * 16 + li];
        wb[kc] = Gq[(4 * kc + lk) * 16 + li];
      }
      d4_t z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) z = mfma16(ta[kc], wb[kc], z);
#pragma unroll
      for (int r = 0; r < 4; ++r) Gq[(lk + 4 * r) * 16 + li] = -0.5 * z[r];
    }
    lds_barrier();
    for (int I = wvs; I < ntr; I += NW) {  // Y += V Gq
      d4_t acc;
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = Ys[(16 * I + lk + 4 * r) * VLD + li];
#pragma unroll
      for (int kc = 0; kc < 4; ++kc)
        acc = mfma16(Vs[(16 * I + li) * VLD + 4 * kc + lk], Gq[(4 * kc + lk) * 16 + li], acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) Ys[(16 * I + lk + 4 * r) * VLD + li] = acc[r];
    }
    lds_barrier();
  }
}

// ---------------------------------------------------------------------------
// sb2st: the band (half-bandwidth 16, upper triangle of A as left by sy2sb)
// to tridiagonal form, Q2^T B Q2 = T, outputs d (m) and e (m-1).  The band
// sits in LDS as its lower part, column by column: S[c 32 + d] = B[c+d][c]
// for d < 32 (the chase fills up to 31 below the diagonal).  Sweep j annihilates column j below the
// subdiagonal with one reflector on rows j+1 .. j+16; its right application
// fills the next 16 rows, whose first column the next reflector annihilates,
// and so on down the band (the rest of each bulge is removed by the later
// sweeps).  Step k of sweep j works on rows/columns [j+1+16(k-1), j+16(k+2)]
// only, so step k' of sweep j+1 may run once step k'+3 of sweep j is done:
// sweep j starts at phase 4j, at most 8 sweeps are active in any phase, wave
// j mod 8 runs sweep j, and a barrier closes each phase.
// Reflector (j, k): v[0] = 1, tau in V2[(j NS + k) 16], v[1..n-1] after it
// (rows r0 = j + 1 + 16k ...), NS = (m-3)/16 + 1.
// ---------------------------------------------------------------------------
namespace {
// Row-of-16 reductions by DPP (row_shr 1, 2, 4, 8): lane 15 of each row of 16
// lanes ends with the row's total (sum) or maximum.
__device__ __forceinline__ double row_sum16(double v) {
  v += dpp_shift<0x111>(v, 0.0);
  v += dpp_shift<0x112>(v, 0.0);
  v += dpp_shift<0x114>(v, 0.0);
  v += dpp_shift<0x118>(v, 0.0);
  return v;
}
__device__ __forceinline__ double row_max16(double v) {
  v = fmax(v, dpp_shift<0x111>(v, v));
  v = fmax(v, dpp_shift<0x112>(v, v));
  v = fmax(v, dpp_shift<0x114>(v, v));
  v = fmax(v, dpp_shift<0x118>(v, v));
  return v;
}

// One chase step, run by one wave.  Rows of 16 lanes split the work: row 0
// owns the columns col+1 .. r0-1 of the left application (lane = column),
// row 1 the rows of the two-sided block (lane = row), row 2 the rows below
// it for the right application (lane = row); row 3 only pads.  Every lane
// loads its 16 entries (and lanes of rows 0 and 1 the entry x of the column
// being annihilated) at once; lanes without work read a slot that holds zero
// and write zero back to it.  v and w reach every lane through
// the wave's 32-double LDS scratch (uniform-address reads).  Band entry
// (i, c), i >= c, sits at S[c CW + i - c]: lanes along a row step by
// CW - 1 = 31 doubles, lanes along a column by 1, both free of bank
// conflicts.
template <int CW>
__device__ __forceinline__ void chase_step(double *S, int m, int j, int k, int NS, double *V2, int lane, int qmax,
                                           int zpad, int padbase, double *wsc) {
  constexpr int CS = CW - 1;  // band entry (i, c) at S[CS c + i]
  const int r0 = j + 1 + k * BW;
  const int r1 = min(r0 + BW - 1, m - 1);
  const int n = r1 - r0 + 1;  // 2 .. 16
  const int col = (k == 0) ? j : r0 - BW;
  const int nc = r0 - col - 1;              // 0 (first step) or 15
  const int nr = min(r1 + BW, m - 1) - r1;  // rows below the block
  const int li = lane & 15, part = lane >> 4;
  // entry q of the lane sits at a0 + a1 q for q <= li and b0 + b1 q above
  // (the two differ only in the two-sided block, whose upper half is read
  // from the mirror):
  //   row 0: (r0 + q, col + 1 + li);  row 1: (r0 + max, r0 + min) of (li, q);
  //   row 2: (r1 + 1 + li, r0 + q)
  int a0 = CS * (col + 1 + li) + r0, a1 = 1;
  bool lok = li < nc;
  if (part == 1) {
    a0 = CW * r0 + li;
    a1 = CS;
    lok = li < n;
  } else if (part >= 2) {
    a0 = CS * r0 + r1 + 1 + li;
    a1 = CS;
    lok = part == 2 && li < nr;
  }
  int b0 = (part == 1) ? CW * r0 + CS * li : a0, b1 = (part == 1) ? 1 : a1;
  // Masks are per lane, not per entry: a lane without work reads its zero
  // slot for every q and writes back the zero its update leaves there (its
  // a, v and w are zero; the slots are per lane, so that these writes do
  // not collide).  Slots are shared by the waves, which all write zero.  Entries q >= n of a working lane (the last step
  // of a sweep, r1 = m - 1) are rows >= m: band slots of columns < m that
  // hold zero and get zero written back (v_q = w_q = 0).  In the two-sided
  // block the entries above the diagonal (q > li) are read from the mirror
  // and written to the lane's pad, their owner writing the lower copy; the
  // other rows write all q (qmax = 15).
  if (!lok) {
    a0 = b0 = zpad + lane;
    a1 = b1 = 0;
  }
  // (byte offsets, stepped from entry to entry: a1 up to qmax, b1 after it)
  const int sa = 8 * a1, sb = 8 * b1, pado = 8 * (padbase + lane);
  char *Sb = reinterpret_cast<char *>(S);
  int off = 8 * a0;
  int ad[BW];
  double a[BW];
#pragma unroll
  for (int q = 0; q < BW; ++q) {
    if (q > 0) off += (q <= qmax) ? sa : sb;
    a[q] = *reinterpret_cast<const double *>(Sb + off);
    ad[q] = (q <= qmax) ? off : pado;
  }
  const bool xin = part <= 1 && li < n;
  const int xad = CS * col + r0 + li;  // (r0 + li, col)
  const double xl = S[xin ? xad : zpad + lane];
  // (a) reflector of column col over rows r0..r1 (row 0 holds x_i in lane i)
  const double xb = (part == 0 && li >= 1) ? xl : 0.0;
  const double amx = read_lane(row_max16(fabs(xb)), 15);
  const double s2 = read_lane(row_sum16(xb * xb), 15);
  const double alpha = read_lane(xl, 0);
  double tp, sc, ei;
  if (!house_direct(alpha, amx, s2, tp, sc, ei)) {
    const double scl = fmax(amx, fabs(alpha)), inv = 1.0 / scl;
    house_scaled(alpha, scl, read_lane(row_sum16((xb * inv) * (xb * inv)), 15), tp, sc, ei);
  }
  const double vi = (li == 0) ? 1.0 : xl * sc;  // the lane's own v (rows 0, 1; 0 past n)
  if (part == 0) {
    wsc[li] = vi;
    // all 16 entries: v is zero past the block, which lets the back
    // transformation read whole blocks without bounds
    V2[((int64_t)j * NS + k) * BW + li] = (li == 0) ? tp : vi;
    if (li < n) S[xad] = (li == 0) ? ei : 0.0;  // the annihilated column: beta, then zeros
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  double vs[BW];
#pragma unroll
  for (int q = 0; q < BW; ++q) vs[q] = wsc[q];
  double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
#pragma unroll
  for (int q = 0; q < BW; q += 4) {
    d0 = fma(vs[q], a[q], d0);
    d1 = fma(vs[q + 1], a[q + 1], d1);
    d2 = fma(vs[q + 2], a[q + 2], d2);
    d3 = fma(vs[q + 3], a[q + 3], d3);
  }
  const double dot = (d0 + d1) + (d2 + d3);
  // rows 0, 2: a -= tau (v.a) v; row 1: p = tau A v, w = p - tau (p.v) v / 2,
  // A -= v w^T + w v^T (lower triangle, q <= li)
  const double p = tp * dot;
  const double pv = read_lane(row_sum16(part == 1 ? p * vi : 0.0), 31);
  const double w = p - 0.5 * tp * pv * vi;
  if (part == 1) wsc[BW + li] = w;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const double al = (part == 1) ? vi : 0.0;
  const double be = (part == 1) ? w : p;
  double ws[BW];
#pragma unroll
  for (int q = 0; q < BW; ++q) ws[q] = wsc[BW + q];  // all read before the band stores (same LDS array)
#pragma unroll
  for (int q = 0; q < BW; ++q) *reinterpret_cast<double *>(Sb + ad[q]) = fma(-be, vs[q], fma(-al, ws[q], a[q]));
}
}  // namespace

// CNT threads (CNT / 64 waves), sweeps CLAG phases apart: the active sweeps
// of a phase are those with 0 <= P - CLAG j < (m-3-j)/16 + 1 <= 32, at most
// ceil(32 / CLAG), each run by wave j mod (CNT / 64).  CLAG = 3 gives the
// same result as CLAG = 4 bit for bit (a step of sweep j+1 three phases
// behind sweep j touches only entries the latter no longer does).
template <int MMAX, int CNT, int CLAG>
__global__ __launch_bounds__(CNT) void k_sb2st(const double *__restrict__ Ab, int64_t sA, int m,
                                                double *__restrict__ db, double *__restrict__ eb, int64_t sv,
                                                double *__restrict__ V2b, int64_t sV2,
                                                const int *__restrict__ only) {
  if (only != nullptr && only[blockIdx.x] == 0) return;  // job not selected
  constexpr int CW = 2 * BW;     // entries kept per band column
  constexpr int CNW = CNT / WAVE;
  static_assert((MMAX - 3) / BW + 1 <= CLAG * CNW, "more sweeps in flight than waves");
  // MMAX x CW band, then WAVE pad entries (writes of the two-sided block
  // above its diagonal), WAVE zero slots (lanes without work), CNW x 32
  // scratch (each wave's v and w broadcasts)
  extern __shared__ double S[];
  constexpr int PADB = MMAX * CW, ZPAD = PADB + WAVE, WSC = ZPAD + WAVE;
  const double *A = Ab + (int64_t)blockIdx.x * sA;
  double *d = db + (int64_t)blockIdx.x * sv;
  double *e = eb + (int64_t)blockIdx.x * sv;
  double *V2 = V2b + (int64_t)blockIdx.x * sV2;
  const int tid = threadIdx.x, lane = tid % WAVE;
  const int wvs = __builtin_amdgcn_readfirstlane(tid / WAVE);
  for (int i = tid; i < WSC; i += CNT) S[i] = 0.0;
  lds_barrier();
  for (int c = tid; c < m; c += CNT) {
    double bnd[BW + 1];  // the band's column c, loads in flight together
#pragma unroll
    for (int dd = 0; dd <= BW; ++dd) bnd[dd] = (c + dd < m) ? A[(int64_t)c * m + c + dd] : 0.0;
#pragma unroll
    for (int dd = 0; dd <= BW; ++dd) S[c * CW + dd] = bnd[dd];
  }
  __syncthreads();
  if (m >= 3) {
    const int NS = (m - 3) / BW + 1;
    const int nph = CLAG * (m - 3) + 1;
    // the last entry a lane writes back (the two-sided block's rows stop at
    // their diagonal)
    const int qmax = ((lane >> 4) == 1) ? (lane & 15) : BW - 1;
    for (int P = 0; P < nph; ++P) {
      const int jhi = min(P / CLAG, m - 3);
      const int j = jhi - (((jhi - wvs) % CNW) + CNW) % CNW;  // largest j <= jhi run by this wave
      if (j >= 0) {
        const int k = P - CLAG * j;
        if (k < (m - 3 - j) / BW + 1) chase_step<CW>(S, m, j, k, NS, V2, lane, qmax, ZPAD, PADB, S + WSC + 2 * BW * wvs);
      }
      lds_barrier();
    }
  }
  for (int c = tid; c < m; c += CNT) {
    d[c] = S[c * CW];
    if (c + 1 < m) e[c] = S[c * CW + 1];
  }
}

// ---------------------------------------------------------------------------
// q2apply: Z <- Q2 Z in place for the eigenvectors Z (m x kk, row-major) of
// the tridiagonal, with the chase's reflectors applied last sweep first.
// One workgroup per (job, slab of 16 columns); thread (kq, c) keeps a window
// of 16 consecutive rows of column c0 + c in registers: during sweep j the
// rows j+1+16kq .. j+16+16kq, exactly those of reflector (j, kq).  Between
// sweeps every window moves up one row: its bottom row passes to thread
// (kq+1, c) through LDS and its new top row comes from thread (kq-1, c), or
// for kq = 0 from Z itself (row j has not been touched yet).  The windows
// are rotating register buffers (the loop is unrolled by 16, so every slot
// index is a constant); a few leading sweeps without reflectors make the
// number of moves a multiple of 16, so that at the end slot q holds window
// row q.  After sweep 0 the windows hold rows 1..m-1 (row 0 never changes)
// and are stored.  A sweep's reflectors are one contiguous block of NS x 16
// doubles: the workgroup loads it with one coalesced load per thread, 8
// sweeps ahead, and stages it through a two-slot LDS ring.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_q2apply(const double *__restrict__ V2b, int64_t sV2, int m,
                                                 double *__restrict__ Zb, int64_t sZ, int kk, int nslab,
                                                 const int *__restrict__ only) {
  // (integer division runs on the vector unit: take the uniform result back
  // to a scalar register, so that the job's pointers stay scalar)
  const int job = __builtin_amdgcn_readfirstlane(blockIdx.x / nslab), slab = blockIdx.x - job * nslab;
  if (only != nullptr && only[job] == 0) return;  // job not selected
  if (m < 3) return;                              // no reflectors
  constexpr int RB = 32 * BW;                     // largest reflector block (NS <= 32)
  __shared__ double ring[2 * RB];
  __shared__ double xfer[2 * NT];
  const double *V2 = V2b + (int64_t)job * sV2;
  double *Z = Zb + (int64_t)job * sZ;
  const int tid = threadIdx.x, c = tid & 15, kq = tid >> 4;
  const int col = slab * 16 + c;
  const bool cok = col < kk;
  const int NS = (m - 3) / BW + 1, nsw = m - 2, blk = NS * BW;
  const int pad = (16 - (nsw - 1) % 16) % 16;  // leading sweeps without reflectors
  const int nv = pad + nsw;                    // nv - 1 moves, a multiple of 16
  auto zrow = [&](int r) -> double { return (cok && r >= 0 && r < m) ? Z[(int64_t)r * kk + col] : 0.0; };
  // block of real sweep i (i = 0: sweep j = m-3), entry tid
  auto ldblk = [&](int i) -> double {
    return (i >= 0 && i < nsw && tid < blk) ? V2[(int64_t)(m - 3 - i) * blk + tid] : 0.0;
  };
  // The prefetched loads are unconditional (clamped into the arrays) and
  // their masks are applied where the values are used: a load under a
  // branch makes every later wait count wait for all loads in flight,
  // the prefetch included.
  auto zrow_raw = [&](int r) -> double {
    return Z[(int64_t)min(max(r, 0), m - 1) * kk + min(col, kk - 1)];
  };
  auto zrow_ok = [&](int r) { return cok && r >= 0 && r < m; };
  auto ldblk_raw = [&](int i) -> double {
    return V2[(int64_t)(m - 3 - min(max(i, 0), nsw - 1)) * blk + min(tid, blk - 1)];
  };
  // virtual sweep v covers rows j_v + 1 + 16 kq + q, j_v = m - 3 + pad - v
  constexpr int PF = 8;  // sweeps of prefetch (reflector blocks, thread 0's rows of Z)
  double w[16], stg[PF], zin[PF];
  {
    const int j0 = m - 3 + pad;
#pragma unroll
    for (int q = 0; q < 16; ++q) w[q] = zrow(j0 + 1 + 16 * kq + q);
  }
  // stg[v mod PF]: block of real sweep v - pad + 1 for the move after sweep v;
  // zin[v mod PF]: row j_v of Z for thread 0's move after sweep v
#pragma unroll
  for (int u = 0; u < PF; ++u) {
    stg[u] = ldblk_raw(u - pad + 1);
    zin[u] = zrow_raw(m - 3 + pad - u);
  }
  if (tid < RB) ring[tid] = ldblk(0);  // real sweep 0
  lds_barrier();
  auto sweep = [&](int v, auto U) {
    constexpr int u = decltype(U)::value;
    const int i = v - pad;
    if (i < 0) return;
    const int j = m - 3 - i;
    if (kq >= (m - 3 - j) / BW + 1) return;
    const double *vp = ring + (i & 1) * RB + kq * BW;
    double vr[16];  // zero past row m - 1 (so rows past m - 1 stay zero)
    vr[0] = 1.0;
#pragma unroll
    for (int q = 1; q < 16; ++q) vr[q] = vp[q];
    double dot = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) dot = fma(vr[q], w[(q - u + 16) & 15], dot);
    dot *= vp[0];
#pragma unroll
    for (int q = 0; q < 16; ++q) w[(q - u + 16) & 15] -= vr[q] * dot;
  };
  auto move = [&](int v, auto U) {
    constexpr int u = decltype(U)::value;
    constexpr int bot = (15 - u + 16) & 15;  // slot of window row 15 (becomes row 0)
    const int i1 = v - pad + 1;               // real sweep that comes next
    constexpr int sl = u % PF;
    if (i1 >= 0 && i1 < nsw && tid < RB) ring[(i1 & 1) * RB + tid] = (tid < blk) ? stg[sl] : 0.0;
    stg[sl] = ldblk_raw(i1 + PF);
    xfer[(u & 1) * NT + tid] = w[bot];
    lds_barrier();
    const int rz = m - 3 + pad - v;  // the row zin[sl] holds
    const double in = (kq == 0) ? (zrow_ok(rz) ? zin[sl] : 0.0) : xfer[(u & 1) * NT + tid - 16];
    zin[sl] = zrow_raw(rz - PF);
    w[bot] = in;
  };
  for (int v0 = 0; v0 + 1 < nv; v0 += 16) {
#define Q2_STEP(U)                                  \
  sweep(v0 + U, std::integral_constant<int, U>{}); \
  move(v0 + U, std::integral_constant<int, U>{});
    Q2_STEP(0) Q2_STEP(1) Q2_STEP(2) Q2_STEP(3) Q2_STEP(4) Q2_STEP(5) Q2_STEP(6) Q2_STEP(7)
    Q2_STEP(8) Q2_STEP(9) Q2_STEP(10) Q2_STEP(11) Q2_STEP(12) Q2_STEP(13) Q2_STEP(14) Q2_STEP(15)
#undef Q2_STEP
  }
  sweep(nv - 1, std::integral_constant<int, 0>{});
  if (cok) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int r = 1 + 16 * kq + q;
      if (r < m) Z[(int64_t)r * kk + col] = w[q];
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <class K>
static void set_lds_band(K kern, size_t lds) {
  (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

int64_t sb2st_v2_stride(int m) {
  if (m < 3) return 0;
  const int NS = (m - 3) / BW + 1;
  return (int64_t)(m - 2) * NS * BW;
}

int launch_sy2sb(hipStream_t st, int nb, double *A, int64_t sA, int m, double *tau, int64_t sv, const int *only) {
  constexpr int MMAX = 512;
  if (m > MMAX) return -1;
  if (nb <= 0 || m < BW + 2) return 0;  // already within the band
  constexpr int R = MMAX - BW;
  const size_t lds = (size_t)(2 * R * VLD + NW * 16 * VLD + 256 + 256 + 4 * NW + 1 + NW * BW + BW) * sizeof(double);
  // kernel attributes set once per process (thread-safe static initialisation)
  static const bool attr = [&] {
    set_lds_band(k_sy2sb<MMAX>, lds);
    return true;
  }();
  (void)attr;
  hipLaunchKernelGGL(k_sy2sb<MMAX>, dim3(nb), dim3(NT), lds, st, A, sA, m, tau, sv, only);
  return 0;
}

int launch_sb2st(hipStream_t st, int nb, const double *A, int64_t sA, int m, double *d, double *e, int64_t sv,
                 double *V2, int64_t sV2, const int *only) {
  constexpr int MMAX = 512;
  if (m > MMAX) return -1;
  if (nb <= 0) return 0;
  constexpr int CNT = 768, CLAG = 3;  // 12 waves, sweeps 3 phases apart
  const size_t lds = ((size_t)MMAX * 2 * BW + 2 * WAVE + (CNT / WAVE) * 2 * BW) * sizeof(double);  // band, pads, zeros, scratch
  // kernel attributes set once per process (thread-safe static initialisation)
  static const bool attr = [&] {
    set_lds_band(k_sb2st<MMAX, CNT, CLAG>, lds);
    return true;
  }();
  (void)attr;
  hipLaunchKernelGGL((k_sb2st<MMAX, CNT, CLAG>), dim3(nb), dim3(CNT), lds, st, A, sA, m, d, e, sv, V2, sV2, only);
  return 0;
}

int launch_q2apply(hipStream_t st, int nb, const double *V2, int64_t sV2, int m, double *Z, int64_t sZ, int kk,
                   const int *only) {
  if (m > 512) return -1;
  const int nslab = (kk + 15) / 16;
  if (nb <= 0 || nslab == 0 || m < 3) return 0;
  hipLaunchKernelGGL(k_q2apply, dim3(nb * nslab), dim3(NT), 0, st, V2, sV2, m, Z, sZ, kk, nslab, only);
  return 0;
}

}  // namespace thck
