// Host engine and C ABI of libthck: schedules the batched compression jobs
// of H|psi> (Algorithm 1 with prefix reuse, Sec. 3.2; kinetic terms, App. D;
// pairwise reduction tree, Sec. 4.5) and of the Lanczos step (Sec. 2.2).
//
// Memory: every MPS produced on the device lives in a "slot" of
// thc_mps_capacity(n, D) doubles from a per-context pool; a slot records its
// static bond profile (the shape it is stored with).  Bond dimensions past
// the numerical rank hold exact zeros.  All work of a call is enqueued on
// one stream, so a slot can be recycled as soon as the job that reads it
// has been enqueued.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <chrono>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/thck.h"
#include "kernels.h"

using namespace thck;

namespace {

thread_local std::string g_err;

thc_status fail(thc_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

struct HipError {
  hipError_t e;
  std::string where;
};

#define HIPCHK(x)                                                         \
  do {                                                                    \
    hipError_t e_ = (x);                                                  \
    if (e_ != hipSuccess) throw HipError{e_, std::string(#x)};            \
  } while (0)

struct StatusError {
  thc_status s;
  std::string msg;
};

[[noreturn]] void raise(thc_status s, const std::string &m) { throw StatusError{s, m}; }

// ---------------------------------------------------------------------------
// bond profiles
// ---------------------------------------------------------------------------
struct Profile {
  std::vector<int> b;        // b[0..n]
  std::vector<int64_t> off;  // packed offsets, n entries
  int64_t size = 0;
  int n() const { return (int)b.size() - 1; }
  void pack() {
    int n_ = n();
    off.assign(n_, 0);
    int64_t o = 0;
    for (int j = 0; j < n_; ++j) {
      off[j] = o;
      o += (int64_t)b[j] * 2 * b[j + 1];
    }
    size = o;
  }
  bool operator<(const Profile &o) const { return b < o.b; }
  bool operator==(const Profile &o) const { return b == o.b; }
};

Profile capacity_profile(int n, int D) {
  Profile p;
  p.b.resize(n + 1);
  for (int j = 0; j <= n; ++j) {
    int64_t x = std::min<int64_t>(D, std::min<int64_t>(j >= 62 ? (1LL << 62) : (1LL << j),
                                                        (n - j) >= 62 ? (1LL << 62) : (1LL << (n - j))));
    p.b[j] = (int)x;
  }
  p.pack();
  return p;
}

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  void ensure(size_t need) {
    if (need <= bytes) return;
    if (p) {
      HIPCHK(hipDeviceSynchronize());
      HIPCHK(hipFree(p));
      p = nullptr;
      bytes = 0;
    }
    hipError_t e = hipMalloc(&p, need);
    if (e != hipSuccess) raise(THC_ENOMEM, "hipMalloc of " + std::to_string(need) + " bytes failed");
    bytes = need;
  }
  template <class T>
  T *as() const {
    return (T *)p;
  }
};

struct PinnedBuf {
  void *p = nullptr;
  size_t bytes = 0;
  ~PinnedBuf() {
    if (p) (void)hipHostFree(p);
  }
  void ensure(size_t need) {
    if (need <= bytes) return;
    if (p) {
      HIPCHK(hipDeviceSynchronize());
      HIPCHK(hipHostFree(p));
      p = nullptr;
    }
    HIPCHK(hipHostMalloc(&p, need, hipHostMallocDefault));
    bytes = need;
  }
};

// One MPS in device memory owned by the pool.
struct Slot {
  double *data = nullptr;
  Profile prof;  // static storage profile
  int id = -1;
};

}  // namespace

struct thc_ctx {
  int L = 0, N = 0, n = 0;
  std::vector<double> t, chi, zeta, lam, u;  // host copies (u column-major per eigvec: u[p*L+i])
  // device layer coefficients: rows [2*mu + s] (chi), then [2N + 2*i + s] (u)
  DevBuf coef;
  // pool
  int64_t slot_elems = 0;
  int slot_D = 0;
  std::vector<double *> free_slots;
  std::vector<std::unique_ptr<DevBuf>> slot_store;
  // batch workspace
  DevBuf ws, jobs_dev, small_dev;
  DevBuf ovl;  // transfer matrices of mps_overlap
  PinnedBuf jobs_host;
  size_t jobs_host_used = 0;
  // statistics accumulated on the host from device readbacks
  int64_t n_compressions = 0, n_launches = 0;
  double flops = 0.0;
  // device stats per call: ranks/disc/sweeps arrays are read back at the end of a call
  DevBuf stat_dev;
  std::vector<int> stat_rank_host;
  int batch_default = 0;
  // per-batch device arrays (rank, discarded weight, sweep count per job and
  // bond; the re-orthonormalisation and Jacobi flags per job), sized once for
  // the largest batch so that captured graphs can keep their addresses
  DevBuf rk, dw, sw, nl, jf, r1, gjobs;
  int batch_cap = 0;
  // captured compression batches (THC_FLAG_GRAPHS)
  struct GraphRec {
    hipGraphExec_t exec;
    int64_t launches;
  };
  std::map<std::string, GraphRec> graphs;
  std::map<std::string, int> graph_seen;
  int64_t graph_captures = 0, graph_replays = 0;

  double *coef_ptr(int row) const { return coef.as<double>() + (size_t)row * n; }
  void drop_graphs() {
    for (auto &g : graphs) (void)hipGraphExecDestroy(g.second.exec);
    graphs.clear();
    graph_seen.clear();
  }
  void ensure_batch_arrays(int nb) {
    if (nb <= batch_cap) return;
    drop_graphs();
    rk.ensure((size_t)nb * n * sizeof(int));
    dw.ensure((size_t)nb * n * sizeof(double));
    sw.ensure((size_t)nb * n * sizeof(int) + sizeof(double));  // cleared as whole doubles
    nl.ensure((size_t)nb * sizeof(int));
    jf.ensure((size_t)nb * sizeof(int));
    r1.ensure((size_t)nb * sizeof(int));
    gjobs.ensure((size_t)nb * sizeof(CJob));
    batch_cap = nb;
  }
  hipStream_t cap_stream = nullptr;  // stream the graphs are captured on
  // THC_FLAG_TWO_STREAMS: a second context on the same factors (its own
  // workspace and slot pool) and its own stream, created on first use
  std::unique_ptr<thc_ctx> twin;
  hipStream_t twin_stream = nullptr;
  ~thc_ctx() {
    drop_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (twin_stream) (void)hipStreamDestroy(twin_stream);
  }
};

namespace {

// ---------------------------------------------------------------------------
// slot pool
// ---------------------------------------------------------------------------
double *slot_alloc(thc_ctx *c, int D) {
  int64_t need = thc_mps_capacity(c->n, D);
  if (need > c->slot_elems) {
    // grow: previous slots stay valid (different allocations); new ones use the larger size
    c->slot_elems = need;
    c->free_slots.clear();
  }
  if (!c->free_slots.empty()) {
    double *p = c->free_slots.back();
    c->free_slots.pop_back();
    return p;
  }
  auto b = std::make_unique<DevBuf>();
  b->ensure((size_t)c->slot_elems * sizeof(double));
  double *p = b->as<double>();
  c->slot_store.push_back(std::move(b));
  return p;
}

void slot_free(thc_ctx *c, double *p) {
  // only recycle slots of the current size
  for (auto &b : c->slot_store)
    if (b->as<double>() == p && b->bytes >= (size_t)c->slot_elems * sizeof(double)) {
      c->free_slots.push_back(p);
      return;
    }
}

// Noise floor of the Gram route, per row of the m x m Gram matrix G = Y Y^T:
// Householder tridiagonalisation perturbs G by ~m eps ||G||, so a kept
// eigenvalue below GRAM_NOISE_PER_ROW * m * eps * lambda_1 cannot be told
// from an exact zero (a singular value near sqrt(m eps) s_1) and its vector
// mixes with the noise directions.  Jobs whose kept set reaches that floor
// (rank-deficient sums, states with exact zeros in their Schmidt spectra)
// get a second Gram level on the deflated matrix (gram_level2).
constexpr double GRAM_NOISE_PER_ROW = 32.0;
inline double gram_floor(int m) { return GRAM_NOISE_PER_ROW * m * 2.220446049250313e-16; }

// ---------------------------------------------------------------------------
// compression plan
// ---------------------------------------------------------------------------
struct Plan {
  int n = 0;
  int kind = 0;
  // mode 1: inputs right-canonical, structured LQ sweep (canonical rows kept,
  // only the rest rows factorised); mode 0: the plain LQ sweep
  int mode = 0;
  std::vector<int> lc, lr, c0;  // per site: canonical rows, rest rows, new Q rows
  int64_t oLt = 0, sLt = 0;     // two L' blocks (ping-pong), each sLt elements
  Profile pa, pb;            // input profiles
  std::vector<int> bo;       // constructed bonds (2D)
  std::vector<int> c;        // right-canonical bonds
  std::vector<int> k;        // output bonds (static)
  Profile out;
  // per-job workspace layout (elements)
  int64_t oB = 0, oT = 0, oL = 0, oQs = 0, oM = 0, oY = 0, oW = 0, oZ = 0, oC = 0, oLz = 0, oQz = 0, oTf = 0,
          oS = 0, oU = 0, oG = 0, oDet = 0, oDet2 = 0, oZm = 0, oLam = 0, oScr = 0, oTo = 0, oV2 = 0;
  int64_t sv = 0;  // stride of the d / e / tau vectors inside oDet
  std::vector<int64_t> qs_off;  // offset of Q_j inside Qs
  int64_t per_job = 0;
  double flops_per_job = 0.0;
  double flops_two_stage_per_job = 0.0;  // the band chase and its back-transformation (two-stage route only)
};

double lq_flops(double m, double n) {  // LQ of m x n (m rows): R + thin Q, LAPACK counts, FMA = 2
  double k = std::min(m, n), M = std::max(m, n);
  return 2.0 * (2.0 * M * k * k - 2.0 * k * k * k / 3.0);
}
// Device-memory bytes the tridiagonalisation of an m x m symmetric matrix
// must move: its upper triangle read once, the reflectors written over it,
// d, e and tau written.  (The one-stage kernel re-reads the trailing
// triangle once per column; that excess shows in the measured traffic.)
double sytrd_bytes(int m) { return 8.0 * ((double)m * m + 3.0 * m); }

// Two-stage route: reflectors of the band chase (sweep j has (m-3-j)/16 + 1
// of at most 16 entries), each applied two-sided to its 16 x 16 blocks
// (~3072 flops) and, in the back-transformation, to kk vectors (4 x 16 kk).
double chase_steps(int m) {
  double s = 0.0;
  for (int x = 0; x <= m - 3; ++x) s += x / 16 + 1;
  return s;
}
double sb2st_flops(int m) { return 3072.0 * chase_steps(m); }
double sb2st_bytes(int m) { return 8.0 * (19.0 * m + 16.0 * chase_steps(m)); }
double q2_flops(int m, int kk) { return 64.0 * kk * chase_steps(m); }
double q2_bytes(int m, int kk) { return 8.0 * (2.0 * m * (double)kk + 16.0 * chase_steps(m)); }

Plan make_plan(int kind, const Profile &pa, const Profile *pb, int D, bool rc_in = false) {
  Plan P;
  P.kind = kind;
  P.n = pa.n();
  const int n = P.n;
  P.pa = pa;
  if (pb) P.pb = *pb;
  P.bo.assign(n + 1, 1);
  for (int j = 1; j < n; ++j) P.bo[j] = (kind == 0) ? 2 * pa.b[j] : pa.b[j] + pb->b[j];
  P.c.assign(n + 1, 1);
  for (int j = n - 1; j >= 1; --j) P.c[j] = std::min(P.bo[j], 2 * P.c[j + 1]);
  P.k.assign(n + 1, 1);
  for (int j = 0; j + 1 < n; ++j) P.k[j + 1] = std::min(std::min(2 * P.k[j], P.c[j + 1]), D);
  // structured sweep: rows [A_j | 0] (orthonormal for a right-canonical
  // input) are kept as the first lc_j rows of Q_j; the lr_j rest rows are
  // projected on their complement and factorised, giving c0_j more rows.
  // Usable when every c0_j is 0 or lr_j (then c_j = lc_j + c0_j equals the
  // plain sweep's c_j).
  if (rc_in && n >= 2) {
    P.lc.assign(n + 1, 0);
    P.lr.assign(n + 1, 0);
    P.c0.assign(n + 1, 0);
    P.lc[n] = 1;
    P.lr[n] = (kind == 0) ? 0 : 1;
    bool ok = true;
    for (int j = n - 1; j >= 1 && ok; --j) {
      P.lc[j] = pa.b[j];
      P.lr[j] = (kind == 0) ? pa.b[j] : pb->b[j];
      const int room = 2 * P.c[j + 1] - P.lc[j];
      if (room < 0) { ok = false; break; }
      P.c0[j] = std::min(P.lr[j], room);
      if (P.c0[j] != 0 && P.c0[j] != P.lr[j]) ok = false;
      if (P.lc[j] + P.c0[j] != P.c[j]) ok = false;
      if (j + 1 < n && pa.b[j + 1] != P.lc[j + 1]) ok = false;
      if (j + 1 < n && ((kind == 0) ? pa.b[j + 1] : pb->b[j + 1]) != P.lr[j + 1]) ok = false;
    }
    if (ok) P.mode = 1;
  }
  P.out.b = P.k;
  P.out.pack();
  int64_t mB = 0, mT = 0, mL = 0, mM = 0, mW = 0, mZ = 0, mQz = 0, mLz = 0, mS = 0, mTf = 0, mU = 0, mG = 0,
          mZm = 0, mScr = 0, mTo = 0, mV2 = 0;
  P.qs_off.assign(n, 0);
  int64_t qs = 0;
  double fl = 0.0;
  for (int j = 0; j < n; ++j) {
    mB = std::max(mB, (int64_t)P.bo[j] * 2 * P.bo[j + 1]);
    mT = std::max(mT, (int64_t)P.bo[j] * 2 * P.c[j + 1]);
    mL = std::max(mL, (int64_t)P.bo[j] * P.c[j]);
    if (j >= 1) {
      P.qs_off[j] = qs;
      qs += (int64_t)P.c[j] * 2 * P.c[j + 1];
      if (P.mode == 1) {
        const double c1 = P.c[j + 1], lcj = P.lc[j], lrj = P.lr[j];
        fl += 2.0 * (2.0 * c1) * lrj * P.lr[j + 1];  // rest rows: source x L'
        fl += 2.0 * 2.0 * (2.0 * c1) * lrj * lcj;    // projection on the canonical rows
        if (P.c0[j] > 0) fl += lq_flops(lrj, 2.0 * c1);
      } else {
        fl += lq_flops(P.bo[j], 2.0 * P.c[j + 1]);
        if (j + 1 < n) fl += 2.0 * (2.0 * P.bo[j - 1]) * P.bo[j] * P.c[j];  // absorb L into site j-1
      }
      // right-canonical output: LQ of U_j L_{j+1} (k_j x 2 k_{j+1})
      fl += lq_flops(P.k[j], 2.0 * P.k[j + 1]);
      fl += 2.0 * (2.0 * P.k[j - 1]) * P.k[j] * P.k[j];
    }
    if (P.mode == 1 && j >= 1) P.sLt = std::max(P.sLt, (int64_t)P.lr[j] * P.c[j]);
    if (j + 1 < n) {
      const int m = 2 * P.k[j], nc = P.c[j + 1], kk = P.k[j + 1];
      mM = std::max(mM, (int64_t)m * nc);
      mW = std::max(mW, std::max((int64_t)kk * nc, (int64_t)m * kk));
      mZ = std::max(mZ, (int64_t)kk * m);
      mQz = std::max(mQz, (int64_t)kk * m);
      mLz = std::max(mLz, (int64_t)kk * kk);
      mS = std::max(mS, (int64_t)m);
      mU = std::max(mU, (int64_t)m * kk);
      mTf = std::max(mTf, (int64_t)lq_t_stride(std::max(kk, 1)));
      mG = std::max(mG, (int64_t)m * m);
      mZm = std::max(mZm, (int64_t)m * kk);
      mScr = std::max(mScr, tri_eig_scratch(m, kk));
      mTo = std::max(mTo, ormtr_tf_stride(m));
      mV2 = std::max(mV2, sb2st_v2_stride(m));
      P.flops_two_stage_per_job += sb2st_flops(m) + q2_flops(m, kk);
      // the Gram route of the SVD as it runs: G = Y Y^T (upper half),
      // tridiagonalisation, back-transformation of kk vectors, one
      // Newton-Schulz step (Z^T Z and Z (Z^T Z)), C = Q^T Y
      fl += (double)m * m * nc + 4.0 / 3.0 * m * (double)m * m + 2.0 * m * (double)m * kk +
            4.0 * m * (double)kk * kk + 2.0 * kk * (double)m * nc;
      fl += 2.0 * kk * nc * 2.0 * P.c[j + 2];  // absorb S V^T into site j+1
    }
    mTf = std::max(mTf, (int64_t)lq_t_stride(std::max(P.c[j], 1)));
  }
  mM = std::max(mM, (int64_t)2 * P.c[1]);
  int64_t o = 0;
  auto take = [&](int64_t sz) {
    int64_t r = o;
    o += (sz + 31) / 32 * 32;
    return r;
  };
  P.oB = take(mB);
  P.oT = take(mT);
  P.oL = take(mL);
  P.oQs = take(qs);
  P.oM = take(mM);
  P.oY = take(mM);
  P.oW = take(mW);
  P.oZ = take(mZ);
  P.oC = take(mW);
  P.oLz = take(mLz);
  P.oQz = take(mQz);
  P.oTf = take(mTf);
  P.oS = take(std::max<int64_t>(mS, 1));
  P.oU = take(std::max<int64_t>(mU, 1));
  P.oG = take(std::max<int64_t>(mG, 1));
  P.sv = (std::max<int64_t>(mS, 1) + 31) / 32 * 32;
  P.oDet = take(3 * P.sv);
  P.oDet2 = take(3 * P.sv);
  P.oZm = take(std::max<int64_t>(mZm, 1));
  P.oLam = take(std::max<int64_t>(mS, 1));
  P.oScr = take(std::max<int64_t>(mScr, 1));
  P.oTo = take(std::max<int64_t>(mTo, 1));
  P.oV2 = take(std::max<int64_t>(mV2, 1));
  if (P.mode == 1) {
    P.sLt = std::max<int64_t>(P.sLt, 1);
    P.oLt = take(2 * ((P.sLt + 31) / 32 * 32));
  }
  P.per_job = o;
  P.flops_per_job = fl;
  return P;
}

// per-call device statistics: for each compression job and bond, rank and
// discarded weight, and per SVD the Jacobi sweep count.
struct CallStats {
  double disc_max = 0.0;
  int max_bond = 0;
  int sweeps_max = 0;
  int nonconv = 0;
  int fallbacks = 0;
  int64_t graph_captures = 0, graph_replays = 0;
  int64_t compressions = 0;
  int64_t launches = 0;
  double flops = 0.0;
  double kms[THC_NK] = {};
  double kflops[THC_NK] = {};
  double kbytes[THC_NK] = {};
  int64_t kn[THC_NK] = {};
};

// Per-shape totals of the timed kernels, printed on stderr at process exit
// when THCK_KSTATS=1 (a tuning aid; THC_FLAG_TIME_KERNELS must be set).
struct ShapeKey {
  int cls, nb, m, n, k, mode;
  bool operator<(const ShapeKey &o) const {
    return std::tie(cls, nb, m, n, k, mode) < std::tie(o.cls, o.nb, o.m, o.n, o.k, o.mode);
  }
};
struct ShapeStat {
  int64_t calls = 0;
  double ms = 0.0, flops = 0.0;
};
std::map<ShapeKey, ShapeStat> &shape_stats() {
  // never destroyed: the exit handler below reads it after static destructors may have run
  static auto *m = new std::map<ShapeKey, ShapeStat>();
  return *m;
}
void print_shape_stats() {
  static const char *names[THC_NK] = {"lq", "sytrd", "tri_eig", "ormtr", "gemm", "svd_fallback"};
  gemm_tuning_report(stderr);
  std::vector<std::pair<ShapeKey, ShapeStat>> v(shape_stats().begin(), shape_stats().end());
  std::sort(v.begin(), v.end(), [](const auto &a, const auto &b) { return a.second.ms > b.second.ms; });
  double tot = 0.0;
  for (auto &e : v) tot += e.second.ms;
  fprintf(stderr, "[thck] timed kernels by shape (total %.2f s)\n", tot / 1e3);
  for (size_t i = 0; i < v.size() && i < 40; ++i) {
    const ShapeKey &k = v[i].first;
    const ShapeStat &s = v[i].second;
    fprintf(stderr, "[thck] %-7s nb %4d  %4d x %4d x %4d  mode %d  calls %7lld  %8.2f s (%4.1f%%)  avg %7.3f ms  %6.2f TF/s\n",
            names[k.cls], k.nb, k.m, k.n, k.k, k.mode, (long long)s.calls, s.ms / 1e3, 100.0 * s.ms / tot,
            s.ms / s.calls, s.ms > 0 ? s.flops / (s.ms * 1e-3) / 1e12 : 0.0);
  }
}
bool shape_stats_on() {
  static const bool on = [] {
    const char *e = getenv("THCK_KSTATS");
    const bool v = e && e[0] == '1';
    if (v) {
      (void)shape_stats();
      atexit(print_shape_stats);
    }
    return v;
  }();
  return on;
}

// Event pairs around kernel launches (THC_FLAG_TIME_KERNELS): recorded on
// the compression stream, resolved after the batch's synchronisation.
struct KernelTimer {
  struct Rec {
    hipEvent_t a, b;
    int cls;
    double flops, bytes;
    ShapeKey key;
  };
  std::vector<hipEvent_t> pool;
  std::vector<Rec> pending;
  size_t used = 0;
  ~KernelTimer() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      pool.push_back(e);
    }
    return pool[used++];
  }
  template <class F>
  void run(hipStream_t st, int cls, double flops, double bytes, const ShapeKey &key, F &&launch) {
    Rec r{get(), get(), cls, flops, bytes, key};
    HIPCHK(hipEventRecord(r.a, st));
    launch();
    HIPCHK(hipEventRecord(r.b, st));
    pending.push_back(r);
  }
  // call after the stream has been synchronised
  void resolve(CallStats &cs) {
    for (const Rec &r : pending) {
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
      cs.kms[r.cls] += ms;
      cs.kflops[r.cls] += r.flops;
      cs.kbytes[r.cls] += r.bytes;
      cs.kn[r.cls] += 1;
      if (shape_stats_on()) {
        static std::mutex mu;  // engines on several host threads share the table
        std::lock_guard<std::mutex> lock(mu);
        ShapeStat &s = shape_stats()[r.key];
        s.calls += 1;
        s.ms += ms;
        s.flops += r.flops;
      }
    }
    pending.clear();
    used = 0;
  }
};

struct Engine {
  thc_ctx *c;
  hipStream_t st;
  const thc_opts &o;
  CallStats cs;
  // device arrays for rank / disc / sweeps of the current batch (per job x site)
  std::vector<int> h_rank;
  std::vector<double> h_disc;
  std::vector<int> h_sw;
  // pending stats readbacks are done synchronously per batch only in debug
  KernelTimer kt;
  bool timing = false;
  // precision of the contractions that absorb a factor into a site (the
  // factorisations, their projections, Gram matrices and overlaps are FP64)
  int cprec = GEMM_F64;
  // share of the ~96 GiB batch-workspace budget (two engines at once each take half)
  double budget_scale = 1.0;
  Engine(thc_ctx *c_, hipStream_t s_, const thc_opts &o_)
      : c(c_), st(s_), o(o_), timing((o_.flags & THC_FLAG_TIME_KERNELS) != 0),
        cprec(o_.prec == THC_PREC_F32 ? GEMM_F32 : (o_.prec == THC_PREC_BF16X3 ? GEMM_BF16X3 : GEMM_F64)) {}
  // launch through the timer when kernel timing is on
  template <class F>
  void timed(int cls, double flops, double bytes, const ShapeKey &key, F &&launch) {
    if (timing) kt.run(st, cls, flops, bytes, key, launch);
    else launch();
  }
  // launchers of the timed kernel classes, with their algorithmic flops and bytes
  void gemm(int nb, int mode, const double *A, int64_t sA, int lda, const double *B, int64_t sB, int ldb, double *C,
            int64_t sC, int ldc, int M, int N, int K, double alpha = 1.0, double beta = 0.0, int prec = GEMM_F64) {
    // flops of the upper-triangle mode: the tiles on or above the diagonal
    // (64 x 64 tiles for FP64, the only precision that mode runs in)
    double fl = 2.0 * M * N * (double)K * nb;
    if (mode & GEMM_UPPER) {
      const double tm = std::ceil(M / 64.0), tn = std::ceil(N / 64.0);
      double run = 0.0;
      for (int a = 0; a < (int)tm; ++a)
        for (int b = 0; b < (int)tn; ++b) run += (a * 64 < b * 64 + 64) ? 1.0 : 0.0;
      fl *= run / (tm * tn);
    }
    const double cbytes = (mode & GEMM_UPPER) ? 0.5 * M * (double)N : (double)M * N;
    timed(THC_K_GEMM, fl,
          8.0 * nb * ((double)M * K + (double)K * N + cbytes * (beta != 0.0 ? 2.0 : 1.0)), ShapeKey{THC_K_GEMM, nb, M, N, K, mode + (beta != 0.0 ? 16 : 0) + 32 * prec},
          [&] { launch_gemm(st, nb, mode, A, sA, lda, B, sB, ldb, C, sC, ldc, M, N, K, alpha, beta, prec); });
  }
  int lq(int nb, double *X, int64_t sX, int m, int n, double *L, int64_t sL, double *Q, int64_t sQ, double *T,
         int64_t sT, bool tr = false, int ldl = 0, int ldq = 0, const int *only = nullptr) {
    int rc = 0;
    const double k = std::min(m, n);
    timed(THC_K_LQ, lq_flops(m, n) * nb, 8.0 * nb * ((double)m * n + m * k + k * n), ShapeKey{THC_K_LQ, nb, m, n, 0, tr ? 1 : 0},
          [&] { rc = launch_lq(st, nb, X, sX, m, n, L, sL, Q, sQ, T, sT, tr, ldl, ldq, only); });
    return rc;
  }
  int sytrd(int nb, double *A, int64_t sA, int m, double *d, double *e, double *tau, int64_t sv) {
    int rc = 0;
    timed(THC_K_SYTRD, 4.0 / 3.0 * m * (double)m * m * nb, sytrd_bytes(m) * nb, ShapeKey{THC_K_SYTRD, nb, m, m, 0, 0}, [&] { rc = launch_sytrd(st, nb, A, sA, m, d, e, tau, sv); });
    return rc;
  }
  // the two-stage route (default): sy2sb timed as the tridiagonalisation
  // (its flops and bytes), then the band chase
  bool two_stage() const { return (o.flags & THC_FLAG_SYTRD_ONE_STAGE) == 0; }
  int tridiag2(int nb, double *A, int64_t sA, int m, double *d, double *e, double *tau, int64_t sv, double *V2,
               int64_t sV2) {
    int rc = 0;
    timed(THC_K_SYTRD, 4.0 / 3.0 * m * (double)m * m * nb, sytrd_bytes(m) * nb, ShapeKey{THC_K_SYTRD, nb, m, m, 0, 1},
          [&] { rc = launch_sy2sb(st, nb, A, sA, m, tau, sv); });
    if (rc != 0) return rc;
    timed(THC_K_SB2ST, sb2st_flops(m) * nb, sb2st_bytes(m) * nb, ShapeKey{THC_K_SB2ST, nb, m, m, 0, 0},
          [&] { rc = launch_sb2st(st, nb, A, sA, m, d, e, sv, V2, sV2); });
    return rc;
  }
  int q2(int nb, const double *V2, int64_t sV2, int m, double *Z, int64_t sZ, int kk) {
    int rc = 0;
    timed(THC_K_Q2, q2_flops(m, kk) * nb, q2_bytes(m, kk) * nb, ShapeKey{THC_K_Q2, nb, m, kk, 0, 0},
          [&] { rc = launch_q2apply(st, nb, V2, sV2, m, Z, sZ, kk); });
    return rc;
  }
  int tri_eig(int nb, const double *d, const double *e, int64_t sv, int m, int kk, double *Z, int64_t sZ, double *lam,
              int64_t sl, double *scr, int64_t sscr, int *needs_lq = nullptr) {
    int rc = 0;
    timed(THC_K_TRI_EIG, 0.0, 8.0 * nb * (2.0 * m + (double)m * kk + kk), ShapeKey{THC_K_TRI_EIG, nb, m, kk, 0, 0}, [&] { rc = launch_tri_eig(st, nb, d, e, sv, m, kk, Z, sZ, lam, sl, scr, sscr, needs_lq); });
    return rc;
  }
  int ormtr(int nb, const double *A, int64_t sA, int m, const double *tau, int64_t sv, double *Z, int64_t sZ, int kk,
            double *Ut, int64_t sU, bool zout, double *Tf, int64_t sTf, int off = 1) {
    int rc = 0;
    timed(THC_K_ORMTR, 2.0 * m * (double)m * kk * nb, 8.0 * nb * (0.5 * m * (double)m + 2.0 * m * (double)kk), ShapeKey{THC_K_ORMTR, nb, m, kk, off, zout ? 1 : 0},
          [&] { rc = launch_ormtr(st, nb, A, sA, m, tau, sv, Z, sZ, kk, Ut, sU, zout, Tf, sTf, nullptr, off); });
    return rc;
  }

  int max_sweeps() const { return o.max_sweeps > 0 ? o.max_sweeps : 40; }
  double cutoff() const { return o.rel_cutoff > 0 ? o.rel_cutoff : 0.0; }

  // Upload job descriptors; returns device pointer.
  CJob *upload_jobs(const std::vector<CJob> &jobs) {
    size_t bytes = jobs.size() * sizeof(CJob);
    // bump allocator inside the call's pinned + device arenas
    size_t need = c->jobs_host_used + bytes;
    if (need > c->jobs_host.bytes || need > c->jobs_dev.bytes) {
      // arenas too small: synchronise, then grow (rare: sized per call up front)
      HIPCHK(hipStreamSynchronize(st));
      size_t nb = std::max(need * 2, (size_t)1 << 20);
      c->jobs_host.ensure(nb);
      c->jobs_dev.ensure(nb);
      c->jobs_host_used = 0;
      need = bytes;
    }
    char *h = (char *)c->jobs_host.p + c->jobs_host_used;
    char *d = (char *)c->jobs_dev.p + c->jobs_host_used;
    memcpy(h, jobs.data(), bytes);
    HIPCHK(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, st));
    c->jobs_host_used += (bytes + 255) / 256 * 256;
    return (CJob *)d;
  }

  // Structured R->L sweep for right-canonical inputs: Q_j = [[A_j | 0] ; Q0_j]
  // with Q0_j from the LQ of the rest rows projected on the complement of
  // [A_j | 0]; L'_j = [P_j | L0_j] carries the rest rows to site j-1.  Q_j
  // is stored transposed, as in the plain sweep.
  int64_t structured_sweep(const Plan &P, CJob *dj, int nb) {
    const int n = P.n;
    const int64_t S = P.per_job;
    double *W = c->ws.as<double>();
    double *Bb = W + P.oB, *Tb = W + P.oT, *Qs = W + P.oQs, *Mb = W + P.oM, *Tf = W + P.oTf;
    const int64_t slt = (P.sLt + 31) / 32 * 32;
    double *Lt[2] = {W + P.oLt, W + P.oLt + slt};
    int cur = 0;  // Lt[cur]: L' of site j+1
    int64_t launches = 0;
    // right boundary: no rest part for a layer, the shared boundary state for a sum
    if (P.lr[n] > 0) {
      launch_fill(st, nb, Lt[cur], S, 1, 1.0);
      ++launches;
    }
    const int srcw = (P.kind == 0) ? 0 : 1;  // input holding the rest rows' source
    for (int j = n - 1; j >= 1; --j) {
      const int lc = P.lc[j], lr = P.lr[j], c1 = P.c[j + 1], cj = P.c[j], lr1 = P.lr[j + 1];
      const int ra = P.pa.b[j + 1];
      const int rsrc = (P.kind == 0) ? P.pa.b[j + 1] : P.pb.b[j + 1];
      const int64_t off_src = (P.kind == 0) ? P.pa.off[j] : P.pb.off[j];
      double *Qt = Qs + P.qs_off[j];
      double *Lnew = Lt[1 - cur];
      // canonical rows [A_j | 0] -> columns 0..lc-1 of Q_j^T
      launch_canon_pack(st, nb, dj, P.pa.off[j], lc, ra, c1, Qt, S, cj);
      // rest rows, transposed: RT = (src L')^T (2 c1 x lr), one GEMM per physical index
      launch_gather(st, nb, dj, srcw, off_src, Bb, S, (int64_t)lr * 2 * rsrc);
      for (int sg = 0; sg < 2; ++sg)
        gemm(nb, GEMM_TA | GEMM_TB, Lt[cur], S, c1, Bb + sg * rsrc, S, 2 * rsrc, Tb + (int64_t)sg * c1 * lr, S, lr,
             c1, lr, lr1, 1.0, 0.0, cprec);
      if (P.kind == 0) launch_rest_post(st, nb, dj, j, P.pa.off[j], lr, ra, c1, Tb, S);
      // P_j = X_rest X_canon^T (lr x lc) -> columns 0..lc-1 of L'_j
      gemm(nb, GEMM_TA, Tb, S, lr, Qt, S, cj, Lnew, S, cj, lr, lc, 2 * c1);
      // X_rest -= P_j X_canon (transposed: RT -= X_canon^T P_j^T)
      gemm(nb, GEMM_TB, Qt, S, cj, Lnew, S, cj, Tb, S, lr, 2 * c1, lr, lc, -1.0, 1.0);
      // LQ of the remainder: Q0_j -> columns lc.. of Q_j^T, L0_j -> columns lc.. of L'_j
      if (P.c0[j] > 0) {
        if (lq(nb, Tb, S, lr, 2 * c1, Lnew + lc, S, Qt + lc, S, Tf, S, true, cj, cj) != 0)
          raise(THC_EINVAL, "site matrix too wide for the LQ kernel (2*bond > 1024)");
      }
      launches += 8;
      cur = 1 - cur;
    }
    // site 0: M_0 (2 x c_1)
    {
      const int lr1 = P.lr[1], c1 = P.c[1];
      const int rsrc = (P.kind == 0) ? P.pa.b[1] : P.pb.b[1];
      const int64_t off_src = (P.kind == 0) ? P.pa.off[0] : P.pb.off[0];
      launch_gather(st, nb, dj, srcw, off_src, Bb, S, (int64_t)2 * rsrc);
      gemm(nb, 0, Bb, S, rsrc, Lt[cur], S, c1, Mb, S, c1, 2, c1, lr1, 1.0, 0.0, cprec);
      launch_site0(st, nb, dj, P.pa.off[0], P.pa.b[1], c1, Mb, S);
      launches += 3;
    }
    return launches;
  }

  // Right-canonical form of the compressed outputs (in their slots): R->L
  // LQ sweep X_j = U_j L_{j+1} = L_j Q_j, site 0 absorbs L_1 and carries the
  // norm.  The state is unchanged (a change of gauge).
  int64_t recanon(const Plan &P, CJob *dj, int nb) {
    const int n = P.n;
    if (n < 2) return 0;
    const int64_t S = P.per_job;
    double *W = c->ws.as<double>();
    double *Bb = W + P.oB, *Tb = W + P.oT, *Lb = W + P.oL, *Yb = W + P.oY, *Tf = W + P.oTf;
    int64_t launches = 0;
    for (int j = n - 1; j >= 1; --j) {
      const int kj = P.k[j], kj1 = P.k[j + 1];
      if (j == n - 1) {
        launch_gather(st, nb, dj, 2, P.out.off[j], Tb, S, (int64_t)kj * 2 * kj1);
      } else {
        launch_gather(st, nb, dj, 2, P.out.off[j], Bb, S, (int64_t)kj * 2 * kj1);
        gemm(nb, 0, Bb, S, kj1, Lb, S, kj1, Tb, S, kj1, 2 * kj, kj1, kj1, 1.0, 0.0, cprec);
      }
      if (lq(nb, Tb, S, kj, 2 * kj1, Lb, S, Yb, S, Tf, S) != 0)
        raise(THC_EINVAL, "site matrix too wide for the LQ kernel (2*bond > 1024)");
      launch_scatter(st, nb, dj, P.out.off[j], Yb, S, (int64_t)kj * 2 * kj1);
      launches += 4;
    }
    launch_gather(st, nb, dj, 2, P.out.off[0], Bb, S, (int64_t)2 * P.k[1]);
    gemm(nb, 0, Bb, S, P.k[1], Lb, S, P.k[1], Yb, S, P.k[1], 2, P.k[1], P.k[1], 1.0, 0.0, cprec);
    launch_scatter(st, nb, dj, P.out.off[0], Yb, S, (int64_t)2 * P.k[1]);
    return launches + 3;
  }

  // Run the compression of nb jobs (same plan).  Output slots in jobs[].out.
  // nrc: the first nrc jobs get right-canonical outputs (all when negative)
  // Second level of the Gram route for the jobs selected by jac, whose kept
  // eigenvalues reached the noise floor gram_floor(m) * lambda_1 (exact or
  // near-zero singular values that the first level cannot tell apart).
  // Q1 = the r1 resolved eigenvectors (before re-orthonormalisation), then
  // Y2 = Y - Q1 Q1^T Y carries the unresolved part at its own scale: the
  // eigenvectors of G2 = Y2 Y2^T resolve singular values down to
  // ~sqrt(m eps) ||Y2|| (about (m eps) s_1 in all), and the kept basis is
  // [Q1 | leading kk - r1 eigenvectors of G2], orthonormalised by the
  // Householder LQ; C = Q^T Y and the cutoff as on the first level.  The
  // job's flag is recorded in flag[job] (the sweep-count array).
  void gram_level2(const Plan &P, int j, int m, int nc, int kk, const int *jac, int *flag, int nb) {
    double *W = c->ws.as<double>();
    const int64_t S = P.per_job;
    double *Mb = W + P.oM, *Yb = W + P.oY, *Wb = W + P.oW, *Zb = W + P.oZ, *Cb = W + P.oC, *Lz = W + P.oLz,
           *Qz = W + P.oQz, *Tf = W + P.oTf, *Ub = W + P.oU, *Gb = W + P.oG, *Db = W + P.oDet, *Zm = W + P.oZm,
           *Lam = W + P.oLam, *Scr = W + P.oScr, *To = W + P.oTo;
    double *D2 = W + P.oDet2, *E2 = D2 + P.sv, *T2 = D2 + 2 * P.sv;
    int *r1 = c->r1.as<int>();
    int *rk_d = c->rk.as<int>();
    double *dw_d = c->dw.as<double>();
    const ShapeKey key{THC_K_SVD_FALLBACK, nb, m, nc, kk, 1};
    auto step = [&](auto &&f) { timed(THC_K_SVD_FALLBACK, 0.0, 0.0, key, f); };
    int rc = 0;
    step([&] { launch_deflate_prep(st, nb, Lam, S, kk, gram_floor(m), Zb, S, m, Wb, S, r1, jac, flag); });
    // Tm = Q1^T Y (kk x nc); Y2 = Y - Q1 Tm
    step([&] { launch_gemm(st, nb, GEMM_TA, Wb, S, kk, Mb, S, nc, Cb, S, nc, kk, nc, m, 1.0, 0.0, GEMM_F64, jac); });
    step([&] { launch_copy(st, nb, Mb, S, Yb, S, (int64_t)m * nc, jac); });
    step([&] { launch_gemm(st, nb, 0, Wb, S, kk, Cb, S, nc, Yb, S, nc, m, nc, kk, -1.0, 1.0, GEMM_F64, jac); });
    // eigenpairs of G2 = Y2 Y2^T
    step([&] { launch_gemm(st, nb, GEMM_TB | GEMM_UPPER, Yb, S, nc, Yb, S, nc, Gb, S, m, m, m, nc, 1.0, 0.0, GEMM_F64, jac); });
    step([&] { rc = launch_sytrd(st, nb, Gb, S, m, D2, E2, T2, S, jac); });
    if (rc != 0) raise(THC_EINVAL, "site matrix too tall for sytrd");
    step([&] { rc = launch_tri_eig(st, nb, D2, E2, S, m, kk, Zm, S, Lam, S, Scr, S, nullptr, jac); });
    if (rc != 0) raise(THC_EINVAL, "site matrix too tall for the tridiagonal eigensolver");
    step([&] { rc = launch_ormtr(st, nb, Gb, S, m, T2, S, Zm, S, kk, Zb, S, true, To, S, jac); });
    if (rc != 0) raise(THC_EINVAL, "ormtr size");
    // basis [Q1 | Z2], orthonormalised; C = Q^T Y; cutoff, U
    step([&] { launch_merge_basis(st, nb, Wb, S, Zb, S, m, kk, r1, jac, Zm, S); });
    step([&] { rc = launch_lq(st, nb, Zm, S, kk, m, Lz, S, Qz, S, Tf, S, true, 0, 0, jac); });
    if (rc != 0) raise(THC_EINVAL, "site matrix too wide for the LQ kernel");
    step([&] { launch_gemm(st, nb, GEMM_TA, Qz, S, kk, Mb, S, nc, Cb, S, nc, kk, nc, m, 1.0, 0.0, GEMM_F64, jac); });
    step([&] {
      launch_svd_finish2(st, nb, Qz, S, m, kk, Cb, S, nc, cutoff(), Db, S, Ub, S, rk_d + (size_t)j * nb,
                         dw_d + (size_t)j * nb, true, jac);
    });
  }

  // Enqueue every launch of one compression batch (nb jobs of plan P, the
  // first nr of which get right-canonical outputs); returns the launch count.
  int64_t enqueue_batch(const Plan &P, CJob *dj, int nb, int nr) {
    const int n = P.n;
    double *W = c->ws.as<double>();
    const int64_t S = P.per_job;
    int *rk_d = c->rk.as<int>();
    double *dw_d = c->dw.as<double>();
    int *sw_d = c->sw.as<int>();
    int *jf_d = c->jf.as<int>();
    int *nl_d = c->nl.as<int>();
    double *Bb = W + P.oB, *Tb = W + P.oT, *Lb = W + P.oL, *Qs = W + P.oQs, *Mb = W + P.oM, *Yb = W + P.oY,
           *Wb = W + P.oW, *Zb = W + P.oZ, *Cb = W + P.oC, *Lz = W + P.oLz, *Qz = W + P.oQz, *Tf = W + P.oTf,
           *Sb = W + P.oS, *Ub = W + P.oU;
    int64_t launches = 0;
    if (P.mode == 1) {
      launches += structured_sweep(P, dj, nb);
    } else {
      // ---- right -> left LQ sweep ----
      for (int j = n - 1; j >= 1; --j) {
        const int la = P.pa.b[j], ra = P.pa.b[j + 1];
        const int lb = P.kind ? P.pb.b[j] : 0, rb = P.kind ? P.pb.b[j + 1] : 0;
        launch_construct(st, dj, nb, j, n, P.pa.off[j], P.kind ? P.pb.off[j] : 0, la, ra, lb, rb, Bb, S, P.bo[j],
                         P.bo[j + 1]);
        ++launches;
        // X_j = B_j L_{j+1} (bo_j x 2 c_{j+1}) is handed to the LQ kernel
        // transposed; the kernel returns Q_j transposed (2 c_{j+1} x c_j)
        if (j == n - 1) {
          launch_transpose(st, nb, Bb, S, P.bo[j], 2, Tb, S);
        } else {
          // X_j^T = [(B_j^0 L)^T ; (B_j^1 L)^T], B_j^s = B_j[:, s, :]: one GEMM per
          // physical index with both operands read transposed
          for (int sg = 0; sg < 2; ++sg)
            gemm(nb, GEMM_TA | GEMM_TB, Lb, S, P.c[j + 1], Bb + sg * P.bo[j + 1], S, 2 * P.bo[j + 1],
                 Tb + (int64_t)sg * P.c[j + 1] * P.bo[j], S, P.bo[j], P.c[j + 1], P.bo[j], P.bo[j + 1], 1.0, 0.0,
                 cprec);
        }
        ++launches;
        if (lq(nb, Tb, S, P.bo[j], 2 * P.c[j + 1], Lb, S, Qs + P.qs_off[j], S, Tf, S, true) != 0)
          raise(THC_EINVAL, "site matrix too wide for the LQ kernel (2*bond > 1024)");
      }
      // site 0: M_0 = B_0 * L_1 (1, 2, c_1)
      {
        const int la = P.pa.b[0], ra = P.pa.b[1];
        const int lb = P.kind ? P.pb.b[0] : 0, rb = P.kind ? P.pb.b[1] : 0;
        launch_construct(st, dj, nb, 0, n, P.pa.off[0], P.kind ? P.pb.off[0] : 0, la, ra, lb, rb, Bb, S, P.bo[0],
                         P.bo[1]);
        if (n > 1)
          gemm(nb, 0, Bb, S, P.bo[1], Lb, S, P.c[1], Mb, S, P.c[1], 2, P.c[1], P.bo[1], 1.0, 0.0, cprec);
        else
          launch_copy(st, nb, Bb, S, Mb, S, 2);
        launches += 2;
      }
    }
    // ---- left -> right SVD sweep ----
    double *Gb = W + P.oG, *Db = W + P.oDet, *Eb = Db + P.sv, *Taub = Db + 2 * P.sv, *Zm = W + P.oZm,
           *Lam = W + P.oLam, *Scr = W + P.oScr, *V2b = W + P.oV2;
    const bool jacobi = (o.flags & THC_FLAG_SVD_JACOBI) != 0;
    const bool ts = two_stage();
    // sweep counts start at zero: the Gram route leaves them there except
    // for the jobs it hands to Jacobi (a fill kernel, not a memset node,
    // should the caller capture the stream into a graph)
    launch_fill(st, 1, reinterpret_cast<double *>(sw_d), 0, ((int64_t)nb * n + 1) / 2, 0.0);
    // One-sided Jacobi SVD of Y = M_j (m x nc) for the jobs selected by only
    // (all when NULL): rows of Y rotated until orthogonal, the kk largest row
    // norms kept (cutoff applied), right factor W (kk x nc), Q from the LQ
    // of Z = W M^T, C = Q M.  Writes U (m x kk), C, rank, discarded weight.
    auto jacobi_svd = [&](int j, int m, int nc, int kk, const int *only) {
      const int cls = only ? THC_K_SVD_FALLBACK : -1;
      auto step = [&](int c, double fl, double by, const ShapeKey &key, auto &&f) {
        if (c >= 0) timed(c, fl, by, key, f);
        else f();
      };
      const ShapeKey key{THC_K_SVD_FALLBACK, nb, m, nc, kk, 0};
      step(cls, 0.0, 0.0, key, [&] { launch_copy(st, nb, Mb, S, Yb, S, (int64_t)m * nc, only); });
      int rc = 0;
      step(cls, 0.0, 0.0, key, [&] { rc = launch_jacobi(st, nb, Yb, S, m, nc, Sb, S, sw_d + (size_t)j * nb, max_sweeps(), only); });
      if (rc != 0) raise(THC_EINVAL, "site matrix too wide for the Jacobi kernel (bond > 1024)");
      step(cls, 0.0, 0.0, key, [&] {
        launch_svd_select(st, nb, Yb, S, m, nc, Sb, S, kk, cutoff(), Wb, S, rk_d + (size_t)j * nb, dw_d + (size_t)j * nb,
                          nullptr, 0, only);
      });
      // Z = W (kk x nc) * M^T (nc x m)
      if (only) step(cls, 0.0, 0.0, key, [&] { launch_gemm(st, nb, GEMM_TB, Wb, S, nc, Mb, S, nc, Zb, S, m, kk, m, nc, 1.0, 0.0, GEMM_F64, only); });
      else gemm(nb, GEMM_TB, Wb, S, nc, Mb, S, nc, Zb, S, m, kk, m, nc);
      if (only) {
        step(cls, 0.0, 0.0, key, [&] { rc = launch_lq(st, nb, Zb, S, kk, m, Lz, S, Qz, S, Tf, S, false, 0, 0, only); });
      } else {
        rc = lq(nb, Zb, S, kk, m, Lz, S, Qz, S, Tf, S);
      }
      if (rc != 0) raise(THC_EINVAL, "site matrix too wide for the LQ kernel");
      // C = Qz (kk x m) * M (m x nc)
      if (only) step(cls, 0.0, 0.0, key, [&] { launch_gemm(st, nb, 0, Qz, S, m, Mb, S, nc, Cb, S, nc, kk, nc, m, 1.0, 0.0, GEMM_F64, only); });
      else gemm(nb, 0, Qz, S, m, Mb, S, nc, Cb, S, nc, kk, nc, m);
      step(cls, 0.0, 0.0, key, [&] { launch_svd_finish(st, nb, Qz, S, m, kk, rk_d + (size_t)j * nb, Ub, S, Cb, S, nc, only); });
    };
    for (int j = 0; j + 1 < n; ++j) {
      const int m = 2 * P.k[j], nc = P.c[j + 1], kk = P.k[j + 1];
      if (jacobi) {
        jacobi_svd(j, m, nc, kk, nullptr);
        launches += 7;
      } else {
        // Gram G = Y Y^T, Y = M_j (m x nc)
        // (the tridiagonalisation reads the upper triangle only)
        gemm(nb, GEMM_TB | GEMM_UPPER, Mb, S, nc, Mb, S, nc, Gb, S, m, m, m, nc);
        // (two-stage: G -> band -> tridiagonal; else one stage)
        if ((ts ? tridiag2(nb, Gb, S, m, Db, Eb, Taub, S, V2b, S) : sytrd(nb, Gb, S, m, Db, Eb, Taub, S)) != 0)
          raise(THC_EINVAL, "site matrix too tall for the tridiagonalisation");
        if (tri_eig(nb, Db, Eb, S, m, kk, Zm, S, Lam, S, Scr, S, nl_d) != 0)
          raise(THC_EINVAL, "site matrix too tall for the tridiagonal eigensolver");
        // eigenvectors as the columns of Z (m x kk): the chase's reflectors,
        // then those of the band reduction (or of the one-stage reduction)
        if (ts && q2(nb, V2b, S, m, Zm, S, kk) != 0) raise(THC_EINVAL, "site matrix too tall for the band chase");
        if (ormtr(nb, Gb, S, m, Taub, S, Zm, S, kk, Zb, S, true, W + P.oTo, S, ts ? 16 : 1) != 0)
          raise(THC_EINVAL, "ormtr size");
        // orthonormal columns spanning the top-kk eigenvectors, Qz (m x kk).
        // Inverse iteration returns them orthonormal to rounding except where
        // the eigensolver flags the job (completions below its noise floor, a
        // cluster split at its member cap) or Z^T Z is off the identity by
        // more than one Newton-Schulz step repairs: every job takes one step
        // Qz = Z (3I - Z^T Z) / 2 (Z^T Z in Lz), the flagged jobs the
        // Householder LQ of Z^T (given transposed; Qz holds Q^T).  Jobs whose
        // kept eigenvalues reach the noise floor gram_floor(m) * lambda_1 are
        // redone by the second Gram level below.
        launch_copy(st, nb, Zb, S, Qz, S, (int64_t)m * kk);
        gemm(nb, GEMM_TA, Zb, S, kk, Zb, S, kk, Lz, S, kk, kk, kk, m);
        launch_svd_flags(st, nb, Lam, S, kk, gram_floor(m), Lz, S, nl_d, jf_d);
        gemm(nb, 0, Zb, S, kk, Lz, S, kk, Qz, S, kk, m, kk, kk, -0.5, 1.5);
        if (lq(nb, Zb, S, kk, m, Lz, S, Qz, S, Tf, S, true, 0, 0, nl_d) != 0)
          raise(THC_EINVAL, "site matrix too wide for the LQ kernel");
        // C = Q (kk x m) * M (m x nc)
        gemm(nb, GEMM_TA, Qz, S, kk, Mb, S, nc, Cb, S, nc, kk, nc, m);
        launch_svd_finish2(st, nb, Qz, S, m, kk, Cb, S, nc, cutoff(), Db, S, Ub, S, rk_d + (size_t)j * nb,
                           dw_d + (size_t)j * nb, true);
        // the flagged jobs: a second Gram level on the deflated matrix
        // (overwrites their U, C, rank, weight)
        gram_level2(P, j, m, nc, kk, jf_d, sw_d + (size_t)j * nb, nb);
        launches += 30;
      }
      launch_scatter(st, nb, dj, P.out.off[j], Ub, S, (int64_t)m * kk);
      // M_{j+1} = C (kk x c_{j+1}) * Q_{j+1} (Q_{j+1} stored transposed)
      gemm(nb, GEMM_TB, Cb, S, nc, Qs + P.qs_off[j + 1], S, nc, Mb, S, 2 * P.c[j + 2], kk, 2 * P.c[j + 2], nc, 1.0,
           0.0, cprec);
      launches += 2;
    }
    // last site
    launch_scatter(st, nb, dj, P.out.off[n - 1], Mb, S, (int64_t)P.k[n - 1] * 2);
    ++launches;
    // outputs in right-canonical form (inputs of later structured sweeps)
    if (nr > 0) launches += recanon(P, dj, nr);
    return launches;
  }

  // Graph of a batch: plan signature, batch size, canonical-output count and
  // the options that change the launch sequence.
  std::string graph_key(const Plan &P, int nb, int nr) const {
    std::string k;
    auto put = [&](int64_t v) { k += std::to_string(v); k += ','; };
    put(P.kind); put(P.mode); put(nb); put(nr); put(cprec); put((int64_t)(o.flags & THC_FLAG_SVD_JACOBI));
    put(o.max_sweeps);
    k += std::to_string(cutoff());
    k += '|';
    for (int v : P.pa.b) put(v);
    for (int64_t v : P.pa.off) put(v);
    k += '|';
    for (int v : P.pb.b) put(v);
    for (int64_t v : P.pb.off) put(v);
    k += '|';
    for (int v : P.k) put(v);
    return k;
  }

  // Run the compression of nb jobs (same plan).  Output slots in jobs[].out.
  // nrc: the first nrc jobs get right-canonical outputs (all when negative).
  // With THC_FLAG_GRAPHS (and kernel timing off) the launch sequence of a
  // batch is captured into a HIP graph the second time its signature
  // occurs and replayed from then on; the jobs then travel through a
  // fixed device buffer, copied before each launch.
  void compress(const Plan &P, const std::vector<CJob> &hjobs, int D, int nrc = -1) {
    const int nb = (int)hjobs.size();
    if (nb == 0) return;
    const int n = P.n;
    static const char *trace_path = getenv("THCK_TRACE");
    const void *ws_before = c->ws.p;
    c->ws.ensure((size_t)P.per_job * nb * sizeof(double));
    if (c->ws.p != ws_before) c->drop_graphs();  // captured graphs point into the old workspace
    c->ensure_batch_arrays(std::max(nb, 512));
    const int nr = (nrc < 0 || nrc > nb) ? nb : nrc;
    const bool graphs = (o.flags & THC_FLAG_GRAPHS) != 0 && !timing && nb <= 512;
    int64_t launches = 0;
    if (!graphs) {
      CJob *dj = upload_jobs(hjobs);
      launches = enqueue_batch(P, dj, nb, nr);
    } else {
      CJob *dj = c->gjobs.as<CJob>();
      HIPCHK(hipMemcpyAsync(dj, hjobs.data(), nb * sizeof(CJob), hipMemcpyHostToDevice, st));
      const std::string key = graph_key(P, nb, nr);
      auto it = c->graphs.find(key);
      if (it != c->graphs.end()) {
        HIPCHK(hipGraphLaunch(it->second.exec, st));
        launches = it->second.launches;
        ++c->graph_replays;
        ++cs.graph_replays;
      } else if (c->graph_seen[key]++ == 0) {
        launches = enqueue_batch(P, dj, nb, nr);  // first time: eager (tunes tiles, sets kernel attributes)
      } else {
        // capture on the context's own non-blocking stream (the caller's
        // may be the null stream, which cannot be captured); the graph then
        // runs on the caller's stream, in order with its other work
        if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        const hipStream_t caller = st;
        st = c->cap_stream;
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        hipGraph_t g = nullptr;
        try {
          launches = enqueue_batch(P, dj, nb, nr);
        } catch (...) {
          (void)hipStreamEndCapture(st, &g);
          if (g) (void)hipGraphDestroy(g);
          st = caller;
          throw;
        }
        const hipError_t ec = hipStreamEndCapture(st, &g);
        st = caller;
        if (ec != hipSuccess) throw HipError{ec, "hipStreamEndCapture"};
        hipGraphExec_t ex = nullptr;
        hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) throw HipError{e, "hipGraphInstantiate"};
        c->graphs[key] = thc_ctx::GraphRec{ex, launches};
        HIPCHK(hipGraphLaunch(ex, st));
        ++c->graph_captures;
        ++cs.graph_captures;
      }
    }
    int *rk_d = c->rk.as<int>();
    double *dw_d = c->dw.as<double>();
    int *sw_d = c->sw.as<int>();
    HIPCHK(hipGetLastError());
    // statistics: read back ranks/disc/sweeps of this batch (async into host arrays after sync at end)
    h_rank.resize((size_t)nb * n);
    h_disc.resize((size_t)nb * n);
    h_sw.resize((size_t)nb * n);
    HIPCHK(hipMemcpyAsync(h_rank.data(), rk_d, (size_t)nb * (n - 1) * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h_disc.data(), dw_d, (size_t)nb * (n - 1) * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h_sw.data(), sw_d, (size_t)nb * (n - 1) * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (timing) kt.resolve(cs);
    report_progress(nb);
    const bool jac_all = (o.flags & THC_FLAG_SVD_JACOBI) != 0;
    for (size_t i = 0; i < (size_t)nb * (n - 1); ++i) {
      cs.disc_max = std::max(cs.disc_max, h_disc[i]);
      cs.max_bond = std::max(cs.max_bond, h_rank[i]);
      cs.sweeps_max = std::max(cs.sweeps_max, h_sw[i]);
      if (h_sw[i] > max_sweeps()) cs.nonconv++;
      if (!jac_all && h_sw[i] > 0) cs.fallbacks++;  // SVD redone by the second Gram level
    }
    if (trace_path) trace_batch(trace_path, P, hjobs);
    last_ranks.assign(h_rank.begin(), h_rank.begin() + (size_t)nb * (n - 1));
    last_nb = nb;
    ++batch_counter;
    cs.compressions += nb;
    cs.launches += launches;
    cs.flops += (P.flops_per_job + (two_stage() ? P.flops_two_stage_per_job : 0.0)) * nb;
  }
  // THCK_PROGRESS=1: a line on stderr after a compression batch, at most
  // every 30 s, so that long calls show that they advance
  void report_progress(int nb) {
    static const bool on = [] {
      const char *e = getenv("THCK_PROGRESS");
      return e && *e && *e != '0';
    }();
    if (!on) return;
    using clk = std::chrono::steady_clock;
    static std::mutex mu;  // engines on several host threads report here
    std::lock_guard<std::mutex> lock(mu);
    static clk::time_point t0 = clk::now(), last = t0;
    static int64_t done = 0;
    done += nb;
    const clk::time_point now = clk::now();
    if (std::chrono::duration<double>(now - last).count() >= 30.0) {
      last = now;
      fprintf(stderr, "[thck] %lld compressions done, %.0f s since the first\n", (long long)done,
              std::chrono::duration<double>(now - t0).count());
      fflush(stderr);
    }
  }
  // debugging aid: append every job of the batch (inputs, metadata, output) to a file
  void trace_batch(const char *path, const Plan &P, const std::vector<CJob> &hj) {
    FILE *f = fopen(path, "ab");
    if (!f) return;
    const int n = P.n;
    auto dump = [&](const double *dev, const Profile &pr) {
      std::vector<double> h(std::max<int64_t>(pr.size, 1));
      HIPCHK(hipMemcpy(h.data(), dev, pr.size * sizeof(double), hipMemcpyDeviceToHost));
      fwrite(pr.b.data(), sizeof(int), n + 1, f);
      fwrite(pr.off.data(), sizeof(int64_t), n, f);
      int64_t sz = pr.size;
      fwrite(&sz, sizeof(int64_t), 1, f);
      fwrite(h.data(), sizeof(double), pr.size, f);
    };
    for (const CJob &j : hj) {
      int hdr[3] = {j.kind, j.dag, n};
      fwrite(hdr, sizeof(int), 3, f);
      double co[2] = {j.ca, j.cb};
      fwrite(co, sizeof(double), 2, f);
      std::vector<double> y(n, 0.0);
      if (j.kind == 0) HIPCHK(hipMemcpy(y.data(), j.y, n * sizeof(double), hipMemcpyDeviceToHost));
      fwrite(y.data(), sizeof(double), n, f);
      Profile pa = P.pa;
      pa.size = 0;
      for (int q = 0; q < n; ++q) pa.size = std::max(pa.size, pa.off[q] + (int64_t)pa.b[q] * 2 * pa.b[q + 1]);
      dump(j.in_a, pa);
      if (j.kind == 1) {
        Profile pb = P.pb;
        pb.size = 0;
        for (int q = 0; q < n; ++q) pb.size = std::max(pb.size, pb.off[q] + (int64_t)pb.b[q] * 2 * pb.b[q + 1]);
        dump(j.in_b, pb);
      }
      dump(j.out, P.out);
    }
    fclose(f);
  }
  std::vector<int> last_ranks;  // [site j][job] rank at bond j+1
  int last_nb = 0;
  int batch_counter = 0;

  int batch_limit(const Plan &P) {
    if (o.batch > 0) return o.batch;
    // keep the batch workspace under ~96 GiB; the big kernels run one
    // workgroup per job on one CU each, so a batch of 256 or 512 fills the
    // 256 CUs evenly, while e.g. 300 would leave a nearly empty second round
    const double budget = 96.0 * (1ull << 30) * budget_scale;
    int b = (int)std::max(1.0, std::min(512.0 * budget_scale, budget / (P.per_job * 8.0)));
    if (b >= 256) b = b / 256 * 256;
    return b;
  }
};

// A node of work: an MPS held in a slot, with its static profile and a
// pending scalar coefficient (applied when it enters a sum or the root).
struct Node {
  double *data = nullptr;
  Profile prof;
  double coef = 1.0;
  bool owned = true;       // slot from the pool (vs caller memory)
  bool rc = false;         // sites 1..n-1 right-canonical
  std::vector<int> ranks;  // numerical ranks at bonds 1..n-1 (empty: unknown)
};

void check_mps(const thc_mps *m, int n_expected) {
  if (!m) raise(THC_EINVAL, "NULL MPS");
  if (m->d != 2) raise(THC_EINVAL, "local dimension must be 2");
  if (n_expected > 0 && m->n_sites != n_expected) raise(THC_EINVAL, "n_sites must equal 2L");
  if (m->n_sites < 2) raise(THC_EINVAL, "need at least 2 sites");
  if (!m->bonds || !m->offsets || !m->data) raise(THC_EINVAL, "NULL bonds/offsets/data");
  if (m->bonds[0] != 1 || m->bonds[m->n_sites] != 1) raise(THC_EINVAL, "boundary bonds must be 1");
  for (int j = 0; j < m->n_sites; ++j) {
    if (m->bonds[j + 1] < 1) raise(THC_EINVAL, "bond < 1");
    int64_t end = m->offsets[j] + (int64_t)m->bonds[j] * 2 * m->bonds[j + 1];
    if (m->offsets[j] < 0 || end > m->capacity) raise(THC_EINVAL, "site tensor outside the buffer capacity");
  }
}

Profile profile_of(const thc_mps *m) {
  Profile p;
  p.b.assign(m->bonds, m->bonds + m->n_sites + 1);
  p.off.assign(m->offsets, m->offsets + m->n_sites);
  p.size = 0;
  for (int j = 0; j < m->n_sites; ++j)
    p.size = std::max(p.size, m->offsets[j] + (int64_t)m->bonds[j] * 2 * m->bonds[j + 1]);
  return p;
}

bool packed(const Profile &p) {
  Profile q = p;
  q.pack();
  return q.off == p.off;
}


}  // namespace

namespace {

void repack(hipStream_t st, const double *src, const Profile &ps, double *dst, const std::vector<int> &r,
            std::vector<int64_t> &doff) {
  int n = ps.n();
  doff.assign(n, 0);
  int64_t o = 0;
  for (int j = 0; j < n; ++j) {
    doff[j] = o;
    int64_t tot = (int64_t)r[j] * 2 * r[j + 1];
    int gx = (int)std::min<int64_t>(2048, std::max<int64_t>(1, (tot + 255) / 256));
    launch_repack(st, gx, src, ps.off[j], ps.b[j], ps.b[j + 1], dst, o, r[j], r[j + 1]);
    o += tot;
  }
}

// Compress groups of jobs that share a plan signature.
struct JobSpec {
  int kind;
  const Node *a;
  const Node *b;
  const double *y;
  int dag;
  double scale;  // for layer jobs (multiplies site 0)
  // the output must be right-canonical (it will be the first input of a
  // structured compression); otherwise the re-canonicalisation is skipped
  // and the output is left in the truncation sweep's (left-canonical) form
  bool rc_out = true;
};

// Run a list of job specs (any mix of signatures); returns output nodes in order.
std::vector<Node> run_jobs(Engine &E, const std::vector<JobSpec> &specs, int D) {
  thc_ctx *c = E.c;
  std::vector<Node> out(specs.size());
  // a sum is symmetric: put a right-canonical term first, where the
  // structured sweep can use it
  std::vector<JobSpec> sp = specs;
  for (JobSpec &s : sp)
    if (s.kind == 1 && !s.a->rc && s.b->rc) std::swap(s.a, s.b);
  // group by signature (kind, bonds, canonical form of the first input)
  std::map<std::pair<int, std::pair<std::vector<int>, std::vector<int>>>, std::vector<size_t>> groups;
  for (size_t i = 0; i < sp.size(); ++i) {
    const JobSpec &s = sp[i];
    const int kk = s.kind + (s.a->rc ? 2 : 0);
    auto key = std::make_pair(kk, std::make_pair(s.a->prof.b, s.kind ? s.b->prof.b : std::vector<int>()));
    groups[key].push_back(i);
  }
  for (auto &g : groups) {
    const JobSpec &s0 = sp[g.second[0]];
    // all members share offsets too? profiles with equal bonds in slots are packed the same way;
    // caller-owned inputs may have other offsets, so split by offsets as well
    std::map<std::pair<std::vector<int64_t>, std::vector<int64_t>>, std::vector<size_t>> sub;
    for (size_t i : g.second) {
      const JobSpec &s = sp[i];
      sub[{s.a->prof.off, s.kind ? s.b->prof.off : std::vector<int64_t>()}].push_back(i);
    }
    for (auto &sg : sub) {
      const JobSpec &sf = sp[sg.second[0]];
      Plan P = make_plan(sf.kind, sf.a->prof, sf.kind ? &sf.b->prof : nullptr, D, sf.a->rc);
      int B = E.batch_limit(P);
      // jobs whose output must be right-canonical first: the
      // re-canonicalisation then runs on a leading part of each batch
      std::stable_partition(sg.second.begin(), sg.second.end(), [&](size_t i) { return sp[i].rc_out; });
      for (size_t i0 = 0; i0 < sg.second.size(); i0 += B) {
        size_t i1 = std::min(sg.second.size(), i0 + B);
        std::vector<CJob> hj;
        int nrc = 0;
        for (size_t t = i0; t < i1; ++t) {
          size_t i = sg.second[t];
          if (sp[i].rc_out) ++nrc;
          const JobSpec &s = sp[i];
          CJob j{};
          j.kind = s.kind;
          j.in_a = s.a->data;
          j.in_b = s.kind ? s.b->data : nullptr;
          j.y = s.y;
          j.dag = s.dag;
          if (s.kind == 0) {
            j.ca = s.scale * s.a->coef;
            j.cb = 0.0;
          } else {
            j.ca = s.a->coef;
            j.cb = s.b->coef;
          }
          out[i].data = slot_alloc(c, D);
          out[i].prof = P.out;
          out[i].coef = 1.0;
          out[i].owned = true;
          out[i].rc = s.rc_out;
          j.out = out[i].data;
          hj.push_back(j);
        }
        E.compress(P, hj, D, nrc);
        const int nbt = (int)hj.size();
        for (size_t t = i0; t < i1; ++t) {
          Node &nd = out[sg.second[t]];
          nd.ranks.resize(P.n - 1);
          for (int jj = 0; jj + 1 < P.n; ++jj) nd.ranks[jj] = E.last_ranks[(size_t)jj * nbt + (t - i0)];
        }
      }
    }
    (void)s0;
  }
  return out;
}

void release(thc_ctx *c, Node &nd) {
  if (nd.owned && nd.data) slot_free(c, nd.data);
  nd.data = nullptr;
}

// Streaming pairwise reduction tree (Sec. 4.5, Fig. 11).  Level l keeps its
// nodes in order; the first two nodes of a level always form the next pair,
// which is the pairing (2k, 2k+1) of the level-by-level tree.  At the end an
// odd last node of level l is appended to level l+1, as the tree carries it.
// Pairs that are ready at any level are compressed together in one batch.
struct Reducer {
  Engine &E;
  int D;
  std::vector<std::vector<Node>> levels;
  // nodes ever appended to each level: a node's position there decides its
  // role, first (even) or second (odd) member of its pair
  std::vector<size_t> pushed;
  Reducer(Engine &e, int D_) : E(e), D(D_) {}

  void append(size_t l, const Node &nd) {
    if (levels.size() < l + 1) levels.resize(l + 1);
    if (pushed.size() < l + 1) pushed.resize(l + 1, 0);
    levels[l].push_back(nd);
    ++pushed[l];
  }
  void push(const Node &leaf) { append(0, leaf); }
  // only the first member of a pair has to be right-canonical (a sum puts a
  // canonical term first); an odd node carried up is the last, even-placed
  // one of its level
  static bool needs_rc(size_t position) { return position % 2 == 0; }
  size_t ready_pairs() const {
    size_t r = 0;
    for (auto &q : levels) r += q.size() / 2;
    return r;
  }
  size_t queued() const {
    size_t r = 0;
    for (auto &q : levels) r += q.size();
    return r;
  }
  // one batch: the ready pairs, lowest level first, at most max_pairs
  void step(size_t max_pairs = SIZE_MAX) {
    std::vector<JobSpec> specs;
    std::vector<std::pair<size_t, size_t>> where;  // (level, pair index)
    std::vector<std::vector<Node>> taken(levels.size());
    size_t budget = max_pairs;
    for (size_t l = 0; l < levels.size(); ++l) {
      size_t np = std::min(levels[l].size() / 2, budget);
      budget -= np;
      taken[l].assign(levels[l].begin(), levels[l].begin() + 2 * np);
      levels[l].erase(levels[l].begin(), levels[l].begin() + 2 * np);
    }
    std::vector<size_t> next(taken.size() + 1, 0);  // positions the results will take
    for (size_t l = 0; l < taken.size(); ++l) next[l + 1] = (l + 1 < pushed.size()) ? pushed[l + 1] : 0;
    for (size_t l = 0; l < taken.size(); ++l)
      for (size_t p = 0; p + 1 < taken[l].size(); p += 2) {
        JobSpec js{1, &taken[l][p], &taken[l][p + 1], nullptr, 0, 1.0};
        js.rc_out = needs_rc(next[l + 1]++);
        specs.push_back(js);
        where.push_back({l, p / 2});
      }
    if (specs.empty()) return;
    std::vector<Node> res = run_jobs(E, specs, D);
    for (auto &t : taken)
      for (auto &nd : t) release(E.c, nd);
    // results go to the next level in pair order (levels before higher ones)
    for (size_t i = 0; i < res.size(); ++i) append(where[i].first + 1, res[i]);
  }
  void flush(size_t min_pairs) {
    const size_t b = std::max<size_t>(1, min_pairs);
    while (ready_pairs() >= b) step(b);
  }
  Node finish() {
    for (;;) {
      while (ready_pairs() > 0) step();
      // carry the lowest odd node up one level
      size_t nonempty = 0, top = 0;
      for (size_t l = 0; l < levels.size(); ++l)
        if (!levels[l].empty()) {
          ++nonempty;
          top = l;
        }
      if (nonempty <= 1) return nonempty ? levels[top][0] : Node{};
      for (size_t l = 0; l < levels.size(); ++l)
        if (levels[l].size() == 1 && l < top) {
          const Node nd = levels[l][0];
          levels[l].clear();
          append(l + 1, nd);
          break;
        }
    }
  }
};

// Write node -> caller MPS (compacting to the numerical ranks of the last
// compression when the node came from one), and set bonds/offsets.
void emit(Engine &E, const Node &nd, thc_mps *out) {
  const int n = nd.prof.n();
  std::vector<int> r = nd.prof.b;
  if ((int)nd.ranks.size() == n - 1) {
    for (int j = 1; j < n; ++j) r[j] = std::max(1, std::min(r[j], nd.ranks[j - 1]));
  }
  int64_t need = 0;
  for (int j = 0; j < n; ++j) need += (int64_t)r[j] * 2 * r[j + 1];
  if (need > out->capacity) raise(THC_ECAPACITY, "output capacity too small");
  std::vector<int64_t> doff;
  repack(E.st, nd.data, nd.prof, out->data, r, doff);
  if (nd.coef != 1.0) {
    // apply a pending coefficient to site 0 (keeps sites 1..n-1 as they are)
    int64_t cnt = (int64_t)r[0] * 2 * r[1];
    launch_scale(E.st, out->data + doff[0], cnt, nd.coef);
  }
  HIPCHK(hipGetLastError());
  for (int j = 0; j <= n; ++j) out->bonds[j] = r[j];
  for (int j = 0; j < n; ++j) out->offsets[j] = doff[j];
  out->canonical = nd.rc ? 1 : 0;
  out->reserved = 0;
}

Node caller_node(const thc_mps *m) {
  Node nd;
  nd.data = m->data;
  nd.prof = profile_of(m);
  nd.coef = 1.0;
  nd.owned = false;
  nd.rc = m->canonical != 0;
  return nd;
}

void fill_stats(thc_stats *st, const CallStats &cs) {
  if (!st) return;
  st->discarded_weight_max = cs.disc_max;
  st->flops_model = cs.flops;
  st->n_compressions = cs.compressions;
  st->n_launches = cs.launches;
  st->max_bond = cs.max_bond;
  st->jacobi_sweeps_max = cs.sweeps_max;
  st->nonconverged = cs.nonconv;
  st->svd_fallbacks = cs.fallbacks;
  st->graph_captures = cs.graph_captures;
  st->graph_replays = cs.graph_replays;
  for (int k = 0; k < THC_NK; ++k) {
    st->kernel_ms[k] = cs.kms[k];
    st->kernel_flops[k] = cs.kflops[k];
    st->kernel_launches[k] = cs.kn[k];
    st->kernel_bytes[k] = cs.kbytes[k];
  }
}

thc_opts norm_opts(const thc_opts *o, int *D) {
  thc_opts r;
  if (o) r = *o;
  else thc_default_opts(&r, 64);
  if (r.D_max < 1) raise(THC_EINVAL, "D_max must be >= 1");
  if (r.D_max > 256) raise(THC_EINVAL, "D_max > 256 is not supported by the kernels of this build");
  if (r.D_sum <= 0) r.D_sum = r.D_max;
  if (r.D_sum > 256) raise(THC_EINVAL, "D_sum > 256 is not supported");
  if (r.rel_cutoff < 0) raise(THC_EINVAL, "negative cutoff");
  if (r.prec != THC_PREC_F64 && r.prec != THC_PREC_F32 && r.prec != THC_PREC_BF16X3)
    raise(THC_EINVAL, "unknown precision");
  *D = r.D_max;
  return r;
}

template <class F>
thc_status run_guarded(F &&f) {
  try {
    f();
    return THC_OK;
  } catch (const StatusError &e) {
    return fail(e.s, e.msg);
  } catch (const HipError &e) {
    return fail(THC_EDEVICE, e.where + ": " + hipGetErrorString(e.e));
  } catch (const std::bad_alloc &) {
    return fail(THC_ENOMEM, "host allocation failed");
  }
}

// compress(coef * x) alone: the direct sum of x with a zero-weight copy of
// itself has the same state, so the sum job compresses it exactly as the
// QR + SVD sweep of Fig. 3 would (the zero half adds only exact zeros).
Node compress_node(Engine &E, Node x, int D) {
  Node zero = x;
  zero.coef = 0.0;
  std::vector<JobSpec> sp{JobSpec{1, &x, &zero, nullptr, 0, 1.0}};
  std::vector<Node> r = run_jobs(E, sp, D);
  release(E.c, x);
  return r[0];
}

// H|psi> (Algorithm 1 terms with prefix reuse + T terms, reduced by the tree)
// The terms with nu in [nu0, nu1) (and the kinetic terms when with_T),
// summed by one pairwise tree; the whole H is nu0 = 0, nu1 = N, with_T.
Node apply_H_nodes(Engine &E, const Node &psi, int D, int D_sum, int nu0 = 0, int nu1 = -1, bool with_T = true) {
  thc_ctx *c = E.c;
  const int N = c->N, L = c->L;
  if (nu1 < 0) nu1 = N;
  const thc_opts &o = E.o;
  Reducer red(E, D_sum);
  // leaves in order: V (nu, s', mu, s) then T (i, s)
  // prefix states (prefix[2 (nu - nu0) + s'])
  std::vector<Node> prefix;
  if (o.include_V && nu1 > nu0) {
    std::vector<JobSpec> s1;
    for (int nu = nu0; nu < nu1; ++nu)
      for (int sp = 0; sp < 2; ++sp) s1.push_back(JobSpec{0, &psi, nullptr, c->coef_ptr(2 * nu + sp), 0, 1.0});
    std::vector<Node> a1 = run_jobs(E, s1, D);
    std::vector<JobSpec> s2;
    for (size_t i = 0; i < a1.size(); ++i) {
      int nu = nu0 + (int)i / 2, sp = (int)i % 2;
      s2.push_back(JobSpec{0, &a1[i], nullptr, c->coef_ptr(2 * nu + sp), 1, 1.0});
    }
    prefix = run_jobs(E, s2, D);
    for (auto &nd : a1) release(c, nd);
  }
  struct Leaf {
    const Node *src;
    const double *y;
    double scale;
  };
  std::vector<Leaf> leaves;
  if (o.include_V) {
    for (int nu = nu0; nu < nu1; ++nu)
      for (int sp = 0; sp < 2; ++sp)
        for (int mu = 0; mu < N; ++mu)
          for (int s = 0; s < 2; ++s) {
            double z = 0.5 * c->zeta[(size_t)mu * N + nu];
            if (z == 0.0) continue;
            leaves.push_back(Leaf{&prefix[2 * (nu - nu0) + sp], c->coef_ptr(2 * mu + s), z});
          }
  }
  if (o.include_T && with_T) {
    for (int i = 0; i < L; ++i) {
      if (c->lam[i] == 0.0) continue;
      for (int s = 0; s < 2; ++s) leaves.push_back(Leaf{&psi, c->coef_ptr(2 * N + 2 * i + s), c->lam[i]});
    }
  }
  if (leaves.empty()) raise(THC_EINVAL, "H has no terms (all coefficients zero or both parts disabled)");
  // chunked leaf production
  Plan probe = make_plan(0, leaves[0].src->prof, nullptr, D);
  int B = E.batch_limit(probe);
  for (size_t i0 = 0; i0 < leaves.size(); i0 += B) {
    size_t i1 = std::min(leaves.size(), i0 + B);
    std::vector<JobSpec> s1;
    for (size_t i = i0; i < i1; ++i) s1.push_back(JobSpec{0, leaves[i].src, nullptr, leaves[i].y, 0, leaves[i].scale});
    std::vector<Node> a1 = run_jobs(E, s1, D);
    std::vector<JobSpec> s2;
    for (size_t i = i0; i < i1; ++i) {
      JobSpec js{0, &a1[i - i0], nullptr, leaves[i].y, 1, 1.0};
      js.rc_out = Reducer::needs_rc(i);  // leaf i is node i of the tree's first level
      s2.push_back(js);
    }
    std::vector<Node> a2 = run_jobs(E, s2, D);
    for (auto &nd : a1) release(c, nd);
    for (auto &nd : a2) red.push(nd);
    // batch the ready sums once a full batch of pairs is available
    red.flush(std::max<size_t>(1, (size_t)B));
  }
  Node root = red.finish();
  for (auto &nd : prefix) release(c, nd);
  return root;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void thc_default_opts(thc_opts *o, int32_t D) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->D_max = D;
  o->D_sum = 0;
  o->rel_cutoff = 1e-14;
  o->prec = THC_PREC_F64;
  o->batch = 0;
  o->max_sweeps = 40;
  o->include_T = 1;
  o->include_V = 1;
  o->flags = 0;
}

int64_t thc_mps_capacity(int32_t n_sites, int32_t D) {
  if (n_sites < 1 || D < 1) return 0;
  Profile p = capacity_profile(n_sites, D);
  return p.size;
}

const char *thc_last_error(void) { return g_err.c_str(); }

thc_status thc_load_factors(thc_ctx **ctx, int32_t L, int32_t N, const double *t, const double *chi,
                            const double *zeta, uint64_t flags, void *hip_stream) {
  (void)flags;
  if (!ctx) return fail(THC_EINVAL, "ctx is NULL");
  *ctx = nullptr;
  if (L < 1 || N < 0) return fail(THC_EINVAL, "need L >= 1 and N >= 0");
  if (!t || (N > 0 && (!chi || !zeta))) return fail(THC_EINVAL, "NULL factor array");
  for (int i = 0; i < L * L; ++i)
    if (!std::isfinite(t[i])) return fail(THC_ENONFINITE, "t has a non-finite entry");
  for (int i = 0; i < L * N; ++i)
    if (!std::isfinite(chi[i])) return fail(THC_ENONFINITE, "chi has a non-finite entry");
  for (int i = 0; i < N * N; ++i)
    if (!std::isfinite(zeta[i])) return fail(THC_ENONFINITE, "zeta has a non-finite entry");
  auto sym_ok = [](const double *a, int m) {
    double mx = 0.0, asym = 0.0;
    for (int i = 0; i < m * m; ++i) mx = std::max(mx, std::fabs(a[i]));
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) asym = std::max(asym, std::fabs(a[i * m + j] - a[j * m + i]));
    return asym <= 1e-12 * std::max(mx, 1e-300);
  };
  if (!sym_ok(t, L)) return fail(THC_EINVAL, "t is not symmetric");
  if (N > 0 && !sym_ok(zeta, N)) return fail(THC_EINVAL, "zeta is not symmetric");
  auto c = std::make_unique<thc_ctx>();
  c->L = L;
  c->N = N;
  c->n = 2 * L;
  c->t.assign(t, t + L * L);
  c->chi.assign(chi, chi + (size_t)L * N);
  c->zeta.assign(zeta, zeta + (size_t)N * N);
  // t = U diag(lam) U^T (App. D), FP64 cyclic Jacobi on the host; ascending lam
  {
    std::vector<double> A(c->t), V((size_t)L * L, 0.0);
    for (int i = 0; i < L; ++i) V[(size_t)i * L + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
      double off = 0.0, tot = 0.0;
      for (int i = 0; i < L; ++i)
        for (int j = 0; j < L; ++j) {
          tot += A[i * L + j] * A[i * L + j];
          if (i != j) off += A[i * L + j] * A[i * L + j];
        }
      if (off <= 1e-32 * tot || off == 0.0) break;
      for (int p = 0; p < L; ++p)
        for (int q = p + 1; q < L; ++q) {
          double apq = A[p * L + q];
          if (apq == 0.0) continue;
          double th = (A[q * L + q] - A[p * L + p]) / (2.0 * apq);
          double tt = std::copysign(1.0, th) / (std::fabs(th) + std::sqrt(1.0 + th * th));
          double cc = 1.0 / std::sqrt(1.0 + tt * tt), ss = tt * cc;
          for (int k = 0; k < L; ++k) {
            double ap = A[p * L + k], aq = A[q * L + k];
            A[p * L + k] = cc * ap - ss * aq;
            A[q * L + k] = ss * ap + cc * aq;
          }
          for (int k = 0; k < L; ++k) {
            double ap = A[k * L + p], aq = A[k * L + q];
            A[k * L + p] = cc * ap - ss * aq;
            A[k * L + q] = ss * ap + cc * aq;
          }
          for (int k = 0; k < L; ++k) {
            double vp = V[k * L + p], vq = V[k * L + q];
            V[k * L + p] = cc * vp - ss * vq;
            V[k * L + q] = ss * vp + cc * vq;
          }
        }
    }
    std::vector<int> idx(L);
    for (int i = 0; i < L; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return A[a * L + a] < A[b * L + b]; });
    c->lam.resize(L);
    c->u.assign((size_t)L * L, 0.0);
    for (int i = 0; i < L; ++i) {
      c->lam[i] = A[idx[i] * L + idx[i]];
      for (int p = 0; p < L; ++p) c->u[(size_t)p * L + i] = V[(size_t)p * L + idx[i]];
    }
  }
  // coefficient rows: y_j = x_p at j = 2p + s
  const int n = 2 * L;
  std::vector<double> rows((size_t)(2 * N + 2 * L) * n, 0.0);
  for (int mu = 0; mu < N; ++mu)
    for (int s = 0; s < 2; ++s)
      for (int p = 0; p < L; ++p) rows[(size_t)(2 * mu + s) * n + 2 * p + s] = chi[(size_t)p * N + mu];
  for (int i = 0; i < L; ++i)
    for (int s = 0; s < 2; ++s)
      for (int p = 0; p < L; ++p) rows[(size_t)(2 * N + 2 * i + s) * n + 2 * p + s] = c->u[(size_t)p * L + i];
  thc_ctx *raw = c.get();
  thc_status stt = run_guarded([&] {
    raw->coef.ensure(rows.size() * sizeof(double));
    HIPCHK(hipMemcpyAsync(raw->coef.p, rows.data(), rows.size() * sizeof(double), hipMemcpyHostToDevice,
                          (hipStream_t)hip_stream));
    HIPCHK(hipStreamSynchronize((hipStream_t)hip_stream));
  });
  if (stt != THC_OK) return stt;
  *ctx = c.release();
  return THC_OK;
}

thc_status thc_destroy(thc_ctx *ctx) {
  if (!ctx) return THC_OK;
  (void)hipDeviceSynchronize();
  delete ctx;
  return THC_OK;
}

namespace {

// both halves of the nu split hold at least one V term (zeta not all zero there)
bool two_halves_have_terms(const thc_ctx *c) {
  const int N = c->N, N0 = N / 2;
  bool a = false, b = false;
  for (int nu = 0; nu < N; ++nu)
    for (int mu = 0; mu < N; ++mu)
      if (c->zeta[(size_t)mu * N + nu] != 0.0) (nu < N0 ? a : b) = true;
  return a && b;
}

void add_call_stats(CallStats &a, const CallStats &b) {
  a.disc_max = std::max(a.disc_max, b.disc_max);
  a.max_bond = std::max(a.max_bond, b.max_bond);
  a.sweeps_max = std::max(a.sweeps_max, b.sweeps_max);
  a.nonconv += b.nonconv;
  a.fallbacks += b.fallbacks;
  a.graph_captures += b.graph_captures;
  a.graph_replays += b.graph_replays;
  a.compressions += b.compressions;
  a.launches += b.launches;
  a.flops += b.flops;
  for (int q = 0; q < THC_NK; ++q) {
    a.kms[q] += b.kms[q];
    a.kflops[q] += b.kflops[q];
    a.kbytes[q] += b.kbytes[q];
    a.kn[q] += b.kn[q];
  }
}

// the second context of THC_FLAG_TWO_STREAMS: same factors, own workspace,
// own non-blocking stream (default priority)
thc_ctx *ensure_twin(thc_ctx *c, hipStream_t st) {
  if (c->twin) return c->twin.get();
  // the stream first: a twin is only kept together with its stream
  if (!c->twin_stream) HIPCHK(hipStreamCreateWithFlags(&c->twin_stream, hipStreamNonBlocking));
  thc_ctx *tw = nullptr;
  thc_status r = thc_load_factors(&tw, c->L, c->N, c->t.data(), c->chi.data(), c->zeta.data(), 0, st);
  if (r != THC_OK) raise(r, thc_last_error());
  c->twin.reset(tw);
  return tw;
}

// H|psi> with the V terms split by nu into [0, N/2) and [N/2, N) (the
// kinetic terms with the second half), each half summed by its own tree in
// its own engine, context and stream, the second on a host thread of its
// own, so that the kernels of the two halves overlap on the GPU; the two
// roots are then added and compressed.  Returns the root (context c).
Node apply_H_two_streams(thc_ctx *c, hipStream_t s, const thc_opts &oo, const Node &in, int D, CallStats &cs) {
  thc_ctx *tw = ensure_twin(c, s);
  hipStream_t s1 = c->twin_stream;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  // the second stream starts after the caller's stream has produced psi
  hipEvent_t ev;
  HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  HIPCHK(hipEventRecord(ev, s));
  HIPCHK(hipStreamWaitEvent(s1, ev, 0));
  HIPCHK(hipEventDestroy(ev));
  const int N0 = c->N / 2;
  Engine E0(c, s, oo), E1(tw, s1, oo);
  E0.budget_scale = E1.budget_scale = 0.5;
  c->jobs_host_used = 0;
  tw->jobs_host_used = 0;
  Node r0, r1;
  thc_status st1 = THC_OK;
  std::string msg1;
  std::thread worker([&] {
    (void)hipSetDevice(dev);
    st1 = run_guarded([&] {
      r1 = apply_H_nodes(E1, in, D, oo.D_sum, N0, c->N, true);
      HIPCHK(hipStreamSynchronize(s1));
    });
    if (st1 != THC_OK) msg1 = thc_last_error();
  });
  thc_status st0 = run_guarded([&] { r0 = apply_H_nodes(E0, in, D, oo.D_sum, 0, N0, false); });
  std::string msg0 = st0 != THC_OK ? std::string(thc_last_error()) : std::string();
  worker.join();
  if (st0 != THC_OK || st1 != THC_OK) {
    if (st0 == THC_OK) release(c, r0);
    if (st1 == THC_OK) release(tw, r1);
    raise(st0 != THC_OK ? st0 : st1, st0 != THC_OK ? msg0 : msg1);
  }
  std::vector<JobSpec> sp{JobSpec{1, &r0, &r1, nullptr, 0, 1.0}};
  Node root = run_jobs(E0, sp, oo.D_sum)[0];
  HIPCHK(hipStreamSynchronize(s));
  release(c, r0);
  release(tw, r1);
  cs = E0.cs;
  add_call_stats(cs, E1.cs);
  return root;
}

}  // namespace

thc_status mps_apply_thc_H(thc_ctx *ctx, const thc_mps *psi, thc_mps *out, const thc_opts *o, thc_stats *st,
                           void *hip_stream) {
  if (!ctx) return fail(THC_EINVAL, "ctx is NULL");
  return run_guarded([&] {
    int D;
    thc_opts oo = norm_opts(o, &D);
    check_mps(psi, ctx->n);
    if (!out || !out->bonds || !out->offsets || !out->data) raise(THC_EINVAL, "bad output MPS");
    if (out->n_sites != ctx->n) raise(THC_EINVAL, "output n_sites must equal 2L");
    if (out->data == psi->data) raise(THC_EINVAL, "psi and out alias");
    if (out->capacity < thc_mps_capacity(ctx->n, D)) raise(THC_ECAPACITY, "output capacity below thc_mps_capacity");
    hipStream_t s = (hipStream_t)hip_stream;
    if ((oo.flags & THC_FLAG_TWO_STREAMS) && oo.include_V && ctx->N >= 2 && two_halves_have_terms(ctx)) {
      CallStats cs;
      Node root = apply_H_two_streams(ctx, s, oo, caller_node(psi), D, cs);
      Engine E(ctx, s, oo);
      ctx->jobs_host_used = 0;
      if (oo.D_sum != D) root = compress_node(E, root, D);
      emit(E, root, out);
      HIPCHK(hipStreamSynchronize(s));
      release(ctx, root);
      add_call_stats(cs, E.cs);
      fill_stats(st, cs);
      return;
    }
    Engine E(ctx, s, oo);
    ctx->jobs_host_used = 0;
    Node in = caller_node(psi);
    Node root = apply_H_nodes(E, in, D, oo.D_sum);
    if (oo.D_sum != D) root = compress_node(E, root, D);
    emit(E, root, out);
    HIPCHK(hipStreamSynchronize(s));
    release(ctx, root);
    fill_stats(st, E.cs);
  });
}

thc_status mps_sum_compress(thc_ctx *ctx, int32_t k, const double *coeffs, const thc_mps *const *terms,
                            thc_mps *out, const thc_opts *o, thc_stats *st, void *hip_stream) {
  if (!ctx) return fail(THC_EINVAL, "ctx is NULL");
  return run_guarded([&] {
    int D;
    thc_opts oo = norm_opts(o, &D);
    if (k < 1 || !coeffs || !terms) raise(THC_EINVAL, "need k >= 1 terms");
    const int n = terms[0] ? terms[0]->n_sites : 0;
    for (int i = 0; i < k; ++i) {
      check_mps(terms[i], n);
      if (!std::isfinite(coeffs[i])) raise(THC_ENONFINITE, "non-finite coefficient");
    }
    if (!out || out->n_sites != n) raise(THC_EINVAL, "bad output MPS");
    if (out->capacity < thc_mps_capacity(n, D)) raise(THC_ECAPACITY, "output capacity below thc_mps_capacity");
    for (int i = 0; i < k; ++i)
      if (terms[i]->data == out->data) raise(THC_EINVAL, "output aliases an input");
    hipStream_t s = (hipStream_t)hip_stream;
    Engine E(ctx, s, oo);
    ctx->jobs_host_used = 0;
    if (ctx->n != n) raise(THC_EINVAL, "n_sites differs from the context's 2L");
    std::vector<Node> leaves(k);
    for (int i = 0; i < k; ++i) {
      leaves[i] = caller_node(terms[i]);
      leaves[i].coef = coeffs[i];
    }
    Node root;
    if (k == 1) {
      root = compress_node(E, leaves[0], D);
    } else {
      Reducer red(E, oo.D_sum);
      for (int i = 0; i < k; ++i) red.push(leaves[i]);
      root = red.finish();
      if (oo.D_sum != D) root = compress_node(E, root, D);
    }
    emit(E, root, out);
    HIPCHK(hipStreamSynchronize(s));
    release(ctx, root);
    fill_stats(st, E.cs);
  });
}

thc_status mps_compress(thc_ctx *ctx, const thc_mps *in, thc_mps *out, const thc_opts *o, thc_stats *st,
                        void *hip_stream) {
  double one = 1.0;
  const thc_mps *t[1] = {in};
  return mps_sum_compress(ctx, 1, &one, t, out, o, st, hip_stream);
}

thc_status mps_apply_layer(thc_ctx *ctx, const thc_mps *psi, const double *y, int32_t dag, thc_mps *out,
                           const thc_opts *o, thc_stats *st, void *hip_stream) {
  if (!ctx) return fail(THC_EINVAL, "ctx is NULL");
  return run_guarded([&] {
    int D;
    thc_opts oo = norm_opts(o, &D);
    check_mps(psi, 0);
    const int n = psi->n_sites;
    if (!y) raise(THC_EINVAL, "y is NULL");
    for (int j = 0; j < n; ++j)
      if (!std::isfinite(y[j])) raise(THC_ENONFINITE, "non-finite coefficient");
    if (!out || out->n_sites != n) raise(THC_EINVAL, "bad output MPS");
    if (out->capacity < thc_mps_capacity(n, D)) raise(THC_ECAPACITY, "output capacity below thc_mps_capacity");
    hipStream_t s = (hipStream_t)hip_stream;
    Engine E(ctx, s, oo);
    ctx->jobs_host_used = 0;
    DevBuf yd;
    yd.ensure(n * sizeof(double));
    HIPCHK(hipMemcpyAsync(yd.p, y, n * sizeof(double), hipMemcpyHostToDevice, s));
    Node in = caller_node(psi);
    std::vector<JobSpec> sp{JobSpec{0, &in, nullptr, yd.as<double>(), dag ? 1 : 0, 1.0}};
    std::vector<Node> r = run_jobs(E, sp, D);
    emit(E, r[0], out);
    HIPCHK(hipStreamSynchronize(s));
    release(ctx, r[0]);
    fill_stats(st, E.cs);
  });
}

thc_status mps_overlap(thc_ctx *ctx, const thc_mps *a, const thc_mps *b, double *result, void *hip_stream) {
  if (!ctx) return fail(THC_EINVAL, "ctx is NULL");
  return run_guarded([&] {
    check_mps(a, 0);
    check_mps(b, a->n_sites);
    if (!result) raise(THC_EINVAL, "result is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    const int n = a->n_sites;
    int maxb = 1;
    for (int j = 0; j <= n; ++j) maxb = std::max(maxb, std::max(a->bonds[j], b->bonds[j]));
    // transfer-matrix chain E_{j+1} = sum_s A_j^{sT} E_j B_j^s as two GEMMs
    // per site: F = E B_j ((la) x (2 rb)), viewed as ((la 2) x rb), then
    // E' = A_j^T F with A_j viewed as ((la 2) x ra)
    const int64_t sz = (int64_t)maxb * maxb;
    DevBuf &w = ctx->ovl;
    w.ensure((size_t)(4 * sz + 32) * sizeof(double));
    double *E = w.as<double>(), *E2 = E + sz, *F = E + 2 * sz;
    static const double one = 1.0;
    HIPCHK(hipMemcpyAsync(E, &one, sizeof(double), hipMemcpyHostToDevice, s));
    for (int j = 0; j < n; ++j) {
      const int la = a->bonds[j], ra = a->bonds[j + 1], lb = b->bonds[j], rb = b->bonds[j + 1];
      const double *Aj = a->data + a->offsets[j], *Bj = b->data + b->offsets[j];
      launch_gemm(s, 1, 0, E, 0, lb, Bj, 0, 2 * rb, F, 0, 2 * rb, la, 2 * rb, lb);
      launch_gemm(s, 1, GEMM_TA, Aj, 0, ra, F, 0, rb, E2, 0, rb, ra, rb, 2 * la);
      std::swap(E, E2);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(result, E, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  });
}

}  // extern "C"

// ===========================================================================
// Allocation-free overlap: the transfer matrices of the chain live in a
// file-scope device array (one copy per GPU), found through
// hipGetSymbolAddress once per device.
// ===========================================================================
namespace {
constexpr int NOALLOC_MAX_BOND = 512;
// E, E' (b x b) and F (b x 2b) of the chain, plus padding
constexpr int64_t NOALLOC_SCRATCH_ELEMS = (int64_t)4 * NOALLOC_MAX_BOND * NOALLOC_MAX_BOND + 64;
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_ELEMS];

// Device address of this GPU's scratch (the array's name is a host-side
// stand-in in host code and must not be passed to a kernel).
double *scratch_ptr() {
  constexpr int MAX_DEV = 64;
  static std::mutex mu;
  static double *ptrs[MAX_DEV] = {};
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEV) raise(THC_EDEVICE, "device index out of range for the scratch table");
  std::lock_guard<std::mutex> lock(mu);
  if (!ptrs[dev]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) throw HipError{e, "hipGetSymbolAddress(scratch)"};
    ptrs[dev] = static_cast<double *>(p);
  }
  return ptrs[dev];
}
}  // namespace

extern "C" {

thc_status mps_overlap_noalloc(const thc_mps *a, const thc_mps *b, double *result_dev, void *hip_stream) {
  return run_guarded([&] {
    check_mps(a, 0);
    check_mps(b, a->n_sites);
    if (!result_dev) raise(THC_EINVAL, "result_dev is NULL");
    const int n = a->n_sites;
    int maxb = 1;
    for (int j = 0; j <= n; ++j) maxb = std::max(maxb, std::max(a->bonds[j], b->bonds[j]));
    if (maxb > NOALLOC_MAX_BOND) raise(THC_ECAPACITY, "bond dimension above 512, the limit of the allocation-free overlap's scratch");
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t sz = (int64_t)maxb * maxb;
    double *W = scratch_ptr();
    double *E = W, *E2 = W + sz, *F = W + 2 * sz;
    launch_fill(s, 1, E, 0, 1, 1.0);  // E_0 = [1]; nothing else is read before it is written
    for (int j = 0; j < n; ++j) {
      const int la = a->bonds[j], ra = a->bonds[j + 1], lb = b->bonds[j], rb = b->bonds[j + 1];
      const double *Aj = a->data + a->offsets[j], *Bj = b->data + b->offsets[j];
      launch_gemm_f64_fixed(s, 0, E, lb, Bj, 2 * rb, F, 2 * rb, la, 2 * rb, lb);
      launch_gemm_f64_fixed(s, GEMM_TA, Aj, ra, F, rb, E2, rb, ra, rb, 2 * la);
      std::swap(E, E2);
    }
    launch_copy(s, 1, E, 0, result_dev, 0, 1);
    HIPCHK(hipGetLastError());
  });
}

}  // extern "C"

// ===========================================================================
// Lanczos (Sec. 2.2)
// ===========================================================================
struct thc_krylov {
  thc_ctx *ctx = nullptr;
  thc_opts o{};
  int K = 0, i = 0, n = 0, D = 0;
  int64_t cap = 0;
  std::vector<std::unique_ptr<DevBuf>> vbuf, wbuf;
  std::vector<std::vector<int>> vb, wb;          // bonds
  std::vector<std::vector<int64_t>> vo, wo;      // offsets
  std::vector<int> vc, wc;                       // right-canonical flags
  std::vector<double> Mm, S, alpha, beta;        // host mirrors, (K+1)^2
  DevBuf dM, dS, dA, dB, dOutG, dOutT, dInfo, dX;
};

namespace {
thc_mps view(thc_krylov *k, bool isw, int i) {
  thc_mps m{};
  m.n_sites = k->n;
  m.d = 2;
  auto &b = isw ? k->wb[i] : k->vb[i];
  auto &o = isw ? k->wo[i] : k->vo[i];
  m.bonds = b.data();
  m.offsets = o.data();
  m.data = (isw ? k->wbuf[i] : k->vbuf[i])->as<double>();
  m.capacity = k->cap;
  m.canonical = isw ? k->wc[i] : k->vc[i];
  return m;
}
}  // namespace

extern "C" {

thc_status krylov_create(thc_ctx *ctx, const thc_mps *psi0, int32_t K, const thc_opts *o, thc_krylov **state,
                         void *hip_stream) {
  if (!ctx || !state) return fail(THC_EINVAL, "NULL argument");
  *state = nullptr;
  if (K < 1 || K + 1 > RITZ_MAX) return fail(THC_EINVAL, "K must be in [1, 31]");
  auto k = std::make_unique<thc_krylov>();
  thc_status s = run_guarded([&] {
    int D;
    k->o = norm_opts(o, &D);
    check_mps(psi0, ctx->n);
    k->ctx = ctx;
    k->K = K;
    k->n = ctx->n;
    k->D = D;
    k->cap = std::max<int64_t>(thc_mps_capacity(ctx->n, D), 0);
    int64_t in_size = 0;
    for (int j = 0; j < psi0->n_sites; ++j)
      in_size = std::max(in_size, psi0->offsets[j] + (int64_t)psi0->bonds[j] * 2 * psi0->bonds[j + 1]);
    k->cap = std::max(k->cap, in_size);
    for (int i = 0; i <= K; ++i) {
      k->vbuf.push_back(std::make_unique<DevBuf>());
      k->vbuf.back()->ensure((size_t)k->cap * sizeof(double));
      k->vb.push_back(std::vector<int>(k->n + 1, 1));
      k->vo.push_back(std::vector<int64_t>(k->n, 0));
      k->vc.push_back(0);
    }
    for (int i = 0; i < K; ++i) {
      k->wbuf.push_back(std::make_unique<DevBuf>());
      k->wbuf.back()->ensure((size_t)k->cap * sizeof(double));
      k->wb.push_back(std::vector<int>(k->n + 1, 1));
      k->wo.push_back(std::vector<int64_t>(k->n, 0));
      k->wc.push_back(0);
    }
    hipStream_t st = (hipStream_t)hip_stream;
    // v_0 = psi0 / ||psi0|| (copied as given, then scaled on site 0)
    k->vb[0].assign(psi0->bonds, psi0->bonds + k->n + 1);
    k->vo[0].assign(psi0->offsets, psi0->offsets + k->n);
    k->vc[0] = psi0->canonical != 0;
    HIPCHK(hipMemcpyAsync(k->vbuf[0]->p, psi0->data, (size_t)in_size * sizeof(double), hipMemcpyDeviceToDevice, st));
    thc_mps v0 = view(k.get(), false, 0);
    double nn = 0.0;
    thc_status r = mps_overlap(ctx, &v0, &v0, &nn, hip_stream);
    if (r != THC_OK) raise(r, thc_last_error());
    if (!(nn > 0.0) || !std::isfinite(nn)) raise(THC_EINVAL, "start vector has zero or non-finite norm");
    launch_scale(st, k->vbuf[0]->as<double>() + k->vo[0][0], (int64_t)k->vb[0][0] * 2 * k->vb[0][1],
                 1.0 / std::sqrt(nn));
    int R = K + 1;
    k->Mm.assign(R * R, 0.0);
    k->S.assign(R * R, 0.0);
    thc_mps v0b = view(k.get(), false, 0);
    double s00 = 0.0;
    r = mps_overlap(ctx, &v0b, &v0b, &s00, hip_stream);
    if (r != THC_OK) raise(r, thc_last_error());
    k->S[0] = s00;
    k->dM.ensure(R * R * sizeof(double));
    k->dS.ensure(R * R * sizeof(double));
    k->dA.ensure(R * sizeof(double));
    k->dB.ensure(R * sizeof(double));
    k->dOutG.ensure(R * sizeof(double));
    k->dOutT.ensure(R * sizeof(double));
    k->dInfo.ensure(4 * sizeof(int));
  });
  if (s != THC_OK) return s;
  *state = k.release();
  return THC_OK;
}

thc_status krylov_destroy(thc_krylov *state) {
  if (!state) return THC_OK;
  (void)hipDeviceSynchronize();
  delete state;
  return THC_OK;
}

thc_status krylov_step(thc_krylov *k, double *ritz_gen, double *ritz_tri, double *beta, thc_stats *st,
                       void *hip_stream) {
  if (!k) return fail(THC_EINVAL, "state is NULL");
  if (k->i >= k->K) return fail(THC_EINVAL, "all K Krylov steps have been taken");
  return run_guarded([&] {
    thc_ctx *ctx = k->ctx;
    const int i = k->i, R = k->K + 1;
    thc_stats s1{}, s2{};
    // w_i = H v_i
    thc_mps vi = view(k, false, i);
    thc_mps wi = view(k, true, i);
    thc_status r = mps_apply_thc_H(ctx, &vi, &wi, &k->o, &s1, hip_stream);
    if (r != THC_OK) raise(r, thc_last_error());
    k->wc[i] = wi.canonical;
    // h_ji = <v_j|w_i>
    for (int j = 0; j <= i; ++j) {
      thc_mps vj = view(k, false, j);
      double h = 0.0;
      r = mps_overlap(ctx, &vj, &wi, &h, hip_stream);
      if (r != THC_OK) raise(r, thc_last_error());
      k->Mm[j * R + i] = h;
    }
    k->alpha.push_back(k->Mm[i * R + i]);
    // r = compress(w_i - sum_j h_ji v_j)
    std::vector<double> co{1.0};
    std::vector<thc_mps> views{wi};
    for (int j = 0; j <= i; ++j) {
      co.push_back(-k->Mm[j * R + i]);
      views.push_back(view(k, false, j));
    }
    std::vector<const thc_mps *> ptrs;
    for (auto &v : views) ptrs.push_back(&v);
    thc_mps vn = view(k, false, i + 1);
    r = mps_sum_compress(ctx, (int)co.size(), co.data(), ptrs.data(), &vn, &k->o, &s2, hip_stream);
    if (r != THC_OK) raise(r, thc_last_error());
    k->vc[i + 1] = vn.canonical;
    double rr = 0.0;
    r = mps_overlap(ctx, &vn, &vn, &rr, hip_stream);
    if (r != THC_OK) raise(r, thc_last_error());
    double b = std::sqrt(std::max(rr, 0.0));
    k->beta.push_back(b);
    hipStream_t st_ = (hipStream_t)hip_stream;
    if (b > 0.0) {
      launch_scale(st_, k->vbuf[i + 1]->as<double>() + k->vo[i + 1][0],
                   (int64_t)k->vb[i + 1][0] * 2 * k->vb[i + 1][1], 1.0 / b);
      HIPCHK(hipGetLastError());
      for (int j = 0; j <= i + 1; ++j) {
        thc_mps a = view(k, false, i + 1), bj = view(k, false, j);
        double sv = 0.0;
        r = mps_overlap(ctx, &a, &bj, &sv, hip_stream);
        if (r != THC_OK) raise(r, thc_last_error());
        k->S[(i + 1) * R + j] = k->S[j * R + (i + 1)] = sv;
      }
      for (int l = 0; l <= i; ++l) {
        thc_mps a = view(k, false, i + 1), wl = view(k, true, l);
        double mv = 0.0;
        r = mps_overlap(ctx, &a, &wl, &mv, hip_stream);
        if (r != THC_OK) raise(r, thc_last_error());
        k->Mm[(i + 1) * R + l] = mv;
      }
    }
    // Ritz values on the device (FP64)
    const int m = i + 1;
    HIPCHK(hipMemcpyAsync(k->dM.p, k->Mm.data(), R * R * sizeof(double), hipMemcpyHostToDevice, st_));
    HIPCHK(hipMemcpyAsync(k->dS.p, k->S.data(), R * R * sizeof(double), hipMemcpyHostToDevice, st_));
    HIPCHK(hipMemcpyAsync(k->dA.p, k->alpha.data(), m * sizeof(double), hipMemcpyHostToDevice, st_));
    if (m > 1)
      HIPCHK(hipMemcpyAsync(k->dB.p, k->beta.data(), (m - 1) * sizeof(double), hipMemcpyHostToDevice, st_));
    launch_ritz(st_, k->dM.as<double>(), k->dS.as<double>(), m, R, k->dA.as<double>(), k->dB.as<double>(),
                k->dOutG.as<double>(), k->dOutT.as<double>(), k->dInfo.as<int>());
    HIPCHK(hipGetLastError());
    std::vector<double> g(m), t(m);
    HIPCHK(hipMemcpyAsync(g.data(), k->dOutG.p, m * sizeof(double), hipMemcpyDeviceToHost, st_));
    HIPCHK(hipMemcpyAsync(t.data(), k->dOutT.p, m * sizeof(double), hipMemcpyDeviceToHost, st_));
    HIPCHK(hipStreamSynchronize(st_));
    if (ritz_gen) memcpy(ritz_gen, g.data(), m * sizeof(double));
    if (ritz_tri) memcpy(ritz_tri, t.data(), m * sizeof(double));
    if (beta) *beta = b;
    k->i = i + 1;
    if (st) {
      st->discarded_weight_max = std::max(s1.discarded_weight_max, s2.discarded_weight_max);
      st->flops_model = s1.flops_model + s2.flops_model;
      st->n_compressions = s1.n_compressions + s2.n_compressions;
      st->n_launches = s1.n_launches + s2.n_launches;
      st->max_bond = std::max(s1.max_bond, s2.max_bond);
      st->jacobi_sweeps_max = std::max(s1.jacobi_sweeps_max, s2.jacobi_sweeps_max);
      st->nonconverged = s1.nonconverged + s2.nonconverged;
      st->svd_fallbacks = s1.svd_fallbacks + s2.svd_fallbacks;
      st->graph_captures = s1.graph_captures + s2.graph_captures;
      st->graph_replays = s1.graph_replays + s2.graph_replays;
      for (int q = 0; q < THC_NK; ++q) {
        st->kernel_ms[q] = s1.kernel_ms[q] + s2.kernel_ms[q];
        st->kernel_flops[q] = s1.kernel_flops[q] + s2.kernel_flops[q];
        st->kernel_launches[q] = s1.kernel_launches[q] + s2.kernel_launches[q];
        st->kernel_bytes[q] = s1.kernel_bytes[q] + s2.kernel_bytes[q];
      }
    }
  });
}

}  // extern "C"

// Coefficients x (host, m = steps taken) of the a-th Ritz vector over
// v_0..v_{m-1}, computed on the device from the M and S mirrors.
namespace {
std::vector<double> ritz_coefficients(thc_krylov *k, int a, hipStream_t st) {
  const int m = k->i, R = k->K + 1;
  if (m < 1) raise(THC_EINVAL, "no Krylov step taken yet");
  if (a < 0 || a >= m) raise(THC_EINVAL, "Ritz index out of range");
  k->dX.ensure(R * sizeof(double));
  HIPCHK(hipMemcpyAsync(k->dM.p, k->Mm.data(), R * R * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(k->dS.p, k->S.data(), R * R * sizeof(double), hipMemcpyHostToDevice, st));
  launch_ritz_vector(st, k->dM.as<double>(), k->dS.as<double>(), m, R, a, k->dX.as<double>(), k->dInfo.as<int>());
  HIPCHK(hipGetLastError());
  std::vector<double> x(m);
  int info = 0;
  HIPCHK(hipMemcpyAsync(x.data(), k->dX.p, m * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&info, k->dInfo.p, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (info != 0) raise(THC_EINVAL, "Ritz index beyond the basis directions kept by the canonical orthogonalisation");
  for (double v : x)
    if (!std::isfinite(v)) raise(THC_ENONFINITE, "non-finite Ritz vector coefficient");
  return x;
}
}  // namespace

extern "C" {

thc_status krylov_ritz_vector(thc_krylov *k, int32_t a, thc_mps *out, void *hip_stream) {
  if (!k || !out) return fail(THC_EINVAL, "NULL argument");
  return run_guarded([&] {
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<double> x = ritz_coefficients(k, a, st);
    std::vector<thc_mps> views;
    for (int i = 0; i < k->i; ++i) views.push_back(view(k, false, i));
    std::vector<const thc_mps *> ptrs;
    for (auto &v : views) ptrs.push_back(&v);
    thc_status r = mps_sum_compress(k->ctx, (int)x.size(), x.data(), ptrs.data(), out, &k->o, nullptr, hip_stream);
    if (r != THC_OK) raise(r, thc_last_error());
  });
}

thc_status krylov_restart(thc_krylov *k, int32_t a, void *hip_stream) {
  if (!k) return fail(THC_EINVAL, "state is NULL");
  return run_guarded([&] {
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<double> x = ritz_coefficients(k, a, st);
    // the Ritz vector goes to slot K, which is never one of the terms (m <= K)
    const int m = k->i, K = k->K;
    std::vector<thc_mps> views;
    for (int i = 0; i < m; ++i) views.push_back(view(k, false, i));
    std::vector<const thc_mps *> ptrs;
    for (auto &v : views) ptrs.push_back(&v);
    thc_mps tmp = view(k, false, K);
    thc_status r = mps_sum_compress(k->ctx, m, x.data(), ptrs.data(), &tmp, &k->o, nullptr, hip_stream);
    if (r != THC_OK) raise(r, thc_last_error());
    k->vc[K] = tmp.canonical;
    int64_t used = 0;
    for (int j = 0; j < k->n; ++j) used = std::max(used, k->vo[K][j] + (int64_t)k->vb[K][j] * 2 * k->vb[K][j + 1]);
    HIPCHK(hipMemcpyAsync(k->vbuf[0]->p, k->vbuf[K]->p, (size_t)used * sizeof(double), hipMemcpyDeviceToDevice, st));
    k->vb[0] = k->vb[K];
    k->vo[0] = k->vo[K];
    k->vc[0] = k->vc[K];
    // normalise (site 0 carries the norm) and reset the basis and matrices
    thc_mps v0 = view(k, false, 0);
    double nn = 0.0;
    r = mps_overlap(k->ctx, &v0, &v0, &nn, hip_stream);
    if (r != THC_OK) raise(r, thc_last_error());
    if (!(nn > 0.0) || !std::isfinite(nn)) raise(THC_EINVAL, "Ritz vector has zero or non-finite norm");
    launch_scale(st, k->vbuf[0]->as<double>() + k->vo[0][0], (int64_t)k->vb[0][0] * 2 * k->vb[0][1],
                 1.0 / std::sqrt(nn));
    HIPCHK(hipGetLastError());
    const int R = K + 1;
    std::fill(k->Mm.begin(), k->Mm.end(), 0.0);
    std::fill(k->S.begin(), k->S.end(), 0.0);
    k->alpha.clear();
    k->beta.clear();
    k->i = 0;
    double s00 = 0.0;
    v0 = view(k, false, 0);
    r = mps_overlap(k->ctx, &v0, &v0, &s00, hip_stream);
    if (r != THC_OK) raise(r, thc_last_error());
    k->S[0] = s00;
    (void)R;
  });
}

thc_status krylov_get_vector(thc_krylov *k, int32_t i, thc_mps *out, void *hip_stream) {
  if (!k || !out) return fail(THC_EINVAL, "NULL argument");
  if (i < 0 || i > k->i) return fail(THC_EINVAL, "vector index out of range");
  return run_guarded([&] {
    int64_t need = 0;
    for (int j = 0; j < k->n; ++j) need = std::max(need, k->vo[i][j] + (int64_t)k->vb[i][j] * 2 * k->vb[i][j + 1]);
    if (out->capacity < need || out->n_sites != k->n) raise(THC_ECAPACITY, "output too small");
    HIPCHK(hipMemcpyAsync(out->data, k->vbuf[i]->p, need * sizeof(double), hipMemcpyDeviceToDevice,
                          (hipStream_t)hip_stream));
    for (int j = 0; j <= k->n; ++j) out->bonds[j] = k->vb[i][j];
    for (int j = 0; j < k->n; ++j) out->offsets[j] = k->vo[i][j];
    out->canonical = k->vc[i];
    out->reserved = 0;
    HIPCHK(hipStreamSynchronize((hipStream_t)hip_stream));
  });
}

thc_status krylov_get_matrices(thc_krylov *k, double *Mm, double *S, int32_t *m) {
  if (!k) return fail(THC_EINVAL, "NULL state");
  const int R = k->K + 1, mm = k->i;
  if (m) *m = mm;
  for (int a = 0; a < mm; ++a)
    for (int b = 0; b < mm; ++b) {
      if (Mm) Mm[a * mm + b] = k->Mm[a * R + b];
      if (S) S[a * mm + b] = k->S[a * R + b];
    }
  return THC_OK;
}

}  // extern "C"

// ===========================================================================
// Krylov time evolution (Sec. 2.2: psi(t + delta) = sum_i a_i v_i with
// a(delta) = exp(-i delta H~) a(0); error bounds in App. A).  H is real, so a
// complex state is held as a pair of real MPS, its real and imaginary part,
// either of which may be the zero MPS (not stored); H acts on each part
// alone, overlaps combine four real ones, and a complex combination
// sum_j c_j x_j is two real sum-compressions: the real part over the terms
// (Re c_j, x_j,re), (-Im c_j, x_j,im), the imaginary part over
// (Re c_j, x_j,im), (Im c_j, x_j,re), j ascending, leaving out absent parts
// and exactly zero coefficients.
// ===========================================================================
namespace {

using cplx = std::complex<double>;
constexpr double EVOLVE_BREAKDOWN = 1e-10;

struct RPart {
  std::unique_ptr<DevBuf> buf = std::make_unique<DevBuf>();
  std::vector<int> b;
  std::vector<int64_t> off;
  int canon = 0;
  bool zero = true;
};

struct CState {
  RPart re, im;
};

struct EvolveWork {
  int n = 0;
  int64_t cap = 0;
  std::vector<CState> v, w;
  std::vector<double> hM, hS;  // host staging: Mr, Mi, Sr, Si (K x K each)
  DevBuf dMS, dA, dInfo;
};

void part_init(RPart &p, int n, int64_t cap) {
  p.buf->ensure((size_t)std::max<int64_t>(cap, 1) * sizeof(double));
  p.b.assign(n + 1, 1);
  p.off.assign(n, 0);
  p.canon = 0;
  p.zero = true;
}

thc_mps part_view(RPart &p, int n) {
  thc_mps m{};
  m.n_sites = n;
  m.d = 2;
  m.bonds = p.b.data();
  m.offsets = p.off.data();
  m.data = p.buf->as<double>();
  m.capacity = (int64_t)(p.buf->bytes / sizeof(double));
  m.canonical = p.canon;
  return m;
}

int64_t used_elems(const std::vector<int> &b, const std::vector<int64_t> &off) {
  int64_t u = 0;
  for (size_t j = 0; j < off.size(); ++j) u = std::max(u, off[j] + (int64_t)b[j] * 2 * b[j + 1]);
  return u;
}

void add_stats(thc_stats &a, const thc_stats &s) {
  a.discarded_weight_max = std::max(a.discarded_weight_max, s.discarded_weight_max);
  a.flops_model += s.flops_model;
  a.n_compressions += s.n_compressions;
  a.n_launches += s.n_launches;
  a.max_bond = std::max(a.max_bond, s.max_bond);
  a.jacobi_sweeps_max = std::max(a.jacobi_sweeps_max, s.jacobi_sweeps_max);
  a.nonconverged += s.nonconverged;
  a.svd_fallbacks += s.svd_fallbacks;
  a.graph_captures += s.graph_captures;
  a.graph_replays += s.graph_replays;
  for (int q = 0; q < THC_NK; ++q) {
    a.kernel_ms[q] += s.kernel_ms[q];
    a.kernel_flops[q] += s.kernel_flops[q];
    a.kernel_launches[q] += s.kernel_launches[q];
    a.kernel_bytes[q] += s.kernel_bytes[q];
  }
}

void check(thc_status r) {
  if (r != THC_OK) raise(r, thc_last_error());
}

double rov(thc_ctx *ctx, RPart &a, RPart &b, int n, hipStream_t st) {
  if (a.zero || b.zero) return 0.0;
  thc_mps x = part_view(a, n), y = part_view(b, n);
  double r = 0.0;
  check(mps_overlap(ctx, &x, &y, &r, st));
  return r;
}

// <a|b> = <a_r|b_r> + <a_i|b_i> + i (<a_r|b_i> - <a_i|b_r>)
cplx cov(thc_ctx *ctx, CState &a, CState &b, int n, hipStream_t st) {
  return cplx(rov(ctx, a.re, b.re, n, st) + rov(ctx, a.im, b.im, n, st),
              rov(ctx, a.re, b.im, n, st) - rov(ctx, a.im, b.re, n, st));
}

void part_copy(RPart &src, RPart &dst, int n, hipStream_t st) {
  dst.zero = src.zero;
  if (src.zero) return;
  const int64_t u = used_elems(src.b, src.off);
  dst.buf->ensure((size_t)std::max<int64_t>(u, 1) * sizeof(double));
  HIPCHK(hipMemcpyAsync(dst.buf->p, src.buf->p, (size_t)u * sizeof(double), hipMemcpyDeviceToDevice, st));
  dst.b = src.b;
  dst.off = src.off;
  dst.canon = src.canon;
  (void)n;
}

void cscale(CState &x, double c, hipStream_t st) {
  for (RPart *p : {&x.re, &x.im})
    if (!p->zero) launch_scale(st, p->buf->as<double>() + p->off[0], (int64_t)p->b[0] * 2 * p->b[1], c);
  HIPCHK(hipGetLastError());
}

// out <- compressed sum_j c_j x_j (out must not be one of the x_j)
void ccombine(thc_ctx *ctx, const thc_opts &o, const std::vector<cplx> &c, const std::vector<CState *> &x,
              CState &out, int n, thc_stats &acc, hipStream_t st) {
  for (int part = 0; part < 2; ++part) {
    std::vector<double> co;
    std::vector<thc_mps> views;
    for (size_t j = 0; j < x.size(); ++j) {
      const double first = c[j].real(), second = part == 0 ? -c[j].imag() : c[j].imag();
      RPart &same = part == 0 ? x[j]->re : x[j]->im, &other = part == 0 ? x[j]->im : x[j]->re;
      if (!same.zero && first != 0.0) { co.push_back(first); views.push_back(part_view(same, n)); }
      if (!other.zero && second != 0.0) { co.push_back(second); views.push_back(part_view(other, n)); }
    }
    RPart &dst = part == 0 ? out.re : out.im;
    if (co.empty()) { dst.zero = true; continue; }
    std::vector<const thc_mps *> ptrs;
    for (auto &v : views) ptrs.push_back(&v);
    thc_mps ov = part_view(dst, n);
    thc_stats s{};
    check(mps_sum_compress(ctx, (int)co.size(), co.data(), ptrs.data(), &ov, &o, &s, st));
    add_stats(acc, s);
    dst.canon = ov.canonical;
    dst.zero = false;
  }
}

void capply(thc_ctx *ctx, const thc_opts &o, CState &x, CState &out, int n, thc_stats &acc, hipStream_t st) {
  for (int part = 0; part < 2; ++part) {
    RPart &src = part == 0 ? x.re : x.im, &dst = part == 0 ? out.re : out.im;
    dst.zero = src.zero;
    if (src.zero) continue;
    thc_mps iv = part_view(src, n), ov = part_view(dst, n);
    thc_stats s{};
    check(mps_apply_thc_H(ctx, &iv, &ov, &o, &s, st));
    add_stats(acc, s);
    dst.canon = ov.canonical;
  }
}

// One time step psi(t) -> psi(t + delta) with at most K Krylov vectors;
// returns the basis size used (smaller than K when the space is invariant).
int evolve_step(thc_ctx *ctx, const thc_opts &o, EvolveWork &W, CState &psi, int K, double delta, thc_stats &acc,
                hipStream_t st) {
  const int n = W.n;
  const double nn = cov(ctx, psi, psi, n, st).real();
  if (!(nn > 0.0) || !std::isfinite(nn)) raise(THC_EINVAL, "state has zero or non-finite norm");
  const double nrm = std::sqrt(nn);
  part_copy(psi.re, W.v[0].re, n, st);
  part_copy(psi.im, W.v[0].im, n, st);
  cscale(W.v[0], 1.0 / nrm, st);
  std::vector<cplx> Mm(K * K), S(K * K);
  S[0] = cov(ctx, W.v[0], W.v[0], n, st);
  int m = K;
  for (int i = 0; i < K; ++i) {
    capply(ctx, o, W.v[i], W.w[i], n, acc, st);
    for (int j = 0; j <= i; ++j) Mm[j * K + i] = cov(ctx, W.v[j], W.w[i], n, st);
    if (i == K - 1) break;
    std::vector<cplx> c{1.0};
    std::vector<CState *> x{&W.w[i]};
    for (int j = 0; j <= i; ++j) {
      c.push_back(-Mm[j * K + i]);
      x.push_back(&W.v[j]);
    }
    ccombine(ctx, o, c, x, W.v[i + 1], n, acc, st);
    const double rr = cov(ctx, W.v[i + 1], W.v[i + 1], n, st).real();
    if (!std::isfinite(rr)) raise(THC_ENONFINITE, "non-finite Krylov residual");
    const double b = std::sqrt(std::max(rr, 0.0));
    double hn = b * b;
    for (int j = 0; j <= i; ++j) hn += std::norm(Mm[j * K + i]);
    if (!(b > EVOLVE_BREAKDOWN * std::sqrt(hn))) {
      m = i + 1;
      break;
    }
    cscale(W.v[i + 1], 1.0 / b, st);
    for (int j = 0; j <= i + 1; ++j) {
      S[(i + 1) * K + j] = cov(ctx, W.v[i + 1], W.v[j], n, st);
      S[j * K + i + 1] = std::conj(S[(i + 1) * K + j]);
    }
    for (int l = 0; l <= i; ++l) Mm[(i + 1) * K + l] = cov(ctx, W.v[i + 1], W.w[l], n, st);
  }
  // a(delta) on the device
  W.hM.assign(4 * K * K, 0.0);
  for (int q = 0; q < K * K; ++q) {
    W.hM[q] = Mm[q].real();
    W.hM[K * K + q] = Mm[q].imag();
    W.hM[2 * K * K + q] = S[q].real();
    W.hM[3 * K * K + q] = S[q].imag();
  }
  W.dMS.ensure(4 * K * K * sizeof(double));
  W.dA.ensure(2 * K * sizeof(double));
  W.dInfo.ensure(4 * sizeof(int));
  double *d = W.dMS.as<double>();
  HIPCHK(hipMemcpyAsync(d, W.hM.data(), 4 * K * K * sizeof(double), hipMemcpyHostToDevice, st));
  launch_evolve_coeffs(st, d, d + K * K, d + 2 * K * K, d + 3 * K * K, m, K, delta, nrm, W.dA.as<double>(),
                       W.dInfo.as<int>());
  HIPCHK(hipGetLastError());
  std::vector<double> a(2 * m);
  HIPCHK(hipMemcpyAsync(a.data(), W.dA.p, 2 * m * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::vector<cplx> c(m);
  std::vector<CState *> x(m);
  for (int i = 0; i < m; ++i) {
    if (!std::isfinite(a[i]) || !std::isfinite(a[m + i])) raise(THC_ENONFINITE, "non-finite evolution coefficient");
    c[i] = cplx(a[i], a[m + i]);
    x[i] = &W.v[i];
  }
  ccombine(ctx, o, c, x, psi, n, acc, st);
  return m;
}

// caller MPS -> owned part (NULL or zero norm -> the zero part)
void load_part(thc_ctx *ctx, const thc_mps *src, RPart &p, int n, int64_t cap, hipStream_t st) {
  p.zero = true;
  p.b.assign(n + 1, 1);
  p.off.assign(n, 0);
  int64_t u = 0;
  if (src) {
    check_mps(src, n);
    u = used_elems(std::vector<int>(src->bonds, src->bonds + n + 1),
                   std::vector<int64_t>(src->offsets, src->offsets + n));
  }
  // sized once (a later growth would drop the contents)
  p.buf->ensure((size_t)std::max<int64_t>(std::max(u, cap), 1) * sizeof(double));
  if (!src) return;
  HIPCHK(hipMemcpyAsync(p.buf->p, src->data, (size_t)u * sizeof(double), hipMemcpyDeviceToDevice, st));
  p.b.assign(src->bonds, src->bonds + n + 1);
  p.off.assign(src->offsets, src->offsets + n);
  p.canon = src->canonical != 0;
  p.zero = false;
  const double nn = rov(ctx, p, p, n, st);
  if (!std::isfinite(nn)) raise(THC_ENONFINITE, "non-finite input state");
  if (nn == 0.0) p.zero = true;
}

// owned part -> caller MPS (the zero part as a bond-1 MPS of zeros)
void store_part(RPart &p, thc_mps *dst, int n, hipStream_t st) {
  if (!dst || dst->n_sites != n || dst->d != 2 || !dst->bonds || !dst->offsets || !dst->data)
    raise(THC_EINVAL, "bad output MPS");
  if (p.zero) {
    if (dst->capacity < 2 * (int64_t)n) raise(THC_ECAPACITY, "output capacity below 2 n");
    HIPCHK(hipMemsetAsync(dst->data, 0, 2 * (size_t)n * sizeof(double), st));
    for (int j = 0; j <= n; ++j) dst->bonds[j] = 1;
    for (int j = 0; j < n; ++j) dst->offsets[j] = 2 * j;
    dst->canonical = 0;
    return;
  }
  const int64_t u = used_elems(p.b, p.off);
  if (dst->capacity < u) raise(THC_ECAPACITY, "output capacity below the evolved state's size");
  HIPCHK(hipMemcpyAsync(dst->data, p.buf->p, (size_t)u * sizeof(double), hipMemcpyDeviceToDevice, st));
  for (int j = 0; j <= n; ++j) dst->bonds[j] = p.b[j];
  for (int j = 0; j < n; ++j) dst->offsets[j] = p.off[j];
  dst->canonical = p.canon;
}

}  // namespace

extern "C" {

thc_status krylov_evolve(int32_t n_inst, thc_ctx *const *ctxs, const thc_mps *const *psi_re,
                         const thc_mps *const *psi_im, const thc_opts *opts, int32_t K, double delta,
                         int32_t n_steps, thc_mps *const *out_re, thc_mps *const *out_im, int32_t *krylov_dims,
                         thc_stats *st, void *hip_stream) {
  if (n_inst < 1 || !ctxs || !psi_re || !opts || !out_re || !out_im) return fail(THC_EINVAL, "NULL argument");
  if (K < 1 || 2 * K > RITZ_MAX) return fail(THC_EINVAL, "K must be in [1, 16]");
  if (n_steps < 0) return fail(THC_EINVAL, "n_steps must be >= 0");
  if (!std::isfinite(delta)) return fail(THC_ENONFINITE, "non-finite time step");
  return run_guarded([&] {
    hipStream_t s = (hipStream_t)hip_stream;
    std::vector<thc_opts> oo(n_inst);
    std::vector<CState> state(n_inst);
    int64_t cap = 0;
    int nmax = 0;
    for (int q = 0; q < n_inst; ++q) {
      if (!ctxs[q]) raise(THC_EINVAL, "NULL context");
      int D;
      oo[q] = norm_opts(&opts[q], &D);
      const int n = ctxs[q]->n;
      cap = std::max(cap, thc_mps_capacity(n, D));
      nmax = std::max(nmax, n);
      for (thc_mps *o : {out_re[q], out_im[q]})
        if (!o || o->n_sites != n) raise(THC_EINVAL, "bad output MPS");
    }
    // inputs are copied before any output is written, so outputs may alias them
    for (int q = 0; q < n_inst; ++q) {
      const int n = ctxs[q]->n;
      load_part(ctxs[q], psi_re[q], state[q].re, n, cap, s);
      load_part(ctxs[q], psi_im ? psi_im[q] : nullptr, state[q].im, n, cap, s);
      if (state[q].re.zero && state[q].im.zero) raise(THC_EINVAL, "state has zero norm");
    }
    // one Krylov workspace, sized for the largest instance, used by each in turn
    EvolveWork W;
    W.cap = cap;
    W.v.resize(K);
    W.w.resize(K);
    for (auto *vec : {&W.v, &W.w})
      for (CState &c : *vec) {
        part_init(c.re, nmax, cap);
        part_init(c.im, nmax, cap);
      }
    thc_stats acc{};
    for (int step = 0; step < n_steps; ++step)
      for (int q = 0; q < n_inst; ++q) {
        W.n = ctxs[q]->n;
        for (auto *vec : {&W.v, &W.w})
          for (CState &c : *vec) {
            c.re.b.assign(W.n + 1, 1); c.re.off.assign(W.n, 0);
            c.im.b.assign(W.n + 1, 1); c.im.off.assign(W.n, 0);
          }
        const int m = evolve_step(ctxs[q], oo[q], W, state[q], K, delta, acc, s);
        if (krylov_dims) krylov_dims[q * n_steps + step] = m;
      }
    for (int q = 0; q < n_inst; ++q) {
      const int n = ctxs[q]->n;
      store_part(state[q].re, out_re[q], n, s);
      store_part(state[q].im, out_im[q], n, s);
    }
    HIPCHK(hipStreamSynchronize(s));
    if (st) *st = acc;
  });
}

thc_status mps_sum_compress_complex(thc_ctx *ctx, int32_t k, const double *coeffs, const thc_mps *const *terms_re,
                                    const thc_mps *const *terms_im, thc_mps *out_re, thc_mps *out_im,
                                    const thc_opts *o, thc_stats *st, void *hip_stream) {
  if (!ctx) return fail(THC_EINVAL, "ctx is NULL");
  if (k < 1 || !coeffs || (!terms_re && !terms_im)) return fail(THC_EINVAL, "need k >= 1 terms");
  if (!out_re || !out_im || out_re == out_im || out_re->data == out_im->data)
    return fail(THC_EINVAL, "need two distinct outputs");
  return run_guarded([&] {
    const int n = ctx->n;
    for (int i = 0; i < 2 * k; ++i)
      if (!std::isfinite(coeffs[i])) raise(THC_ENONFINITE, "non-finite coefficient");
    // the two term lists, in the order of krylov_evolve's combinations
    std::vector<double> co[2];
    std::vector<const thc_mps *> tm[2];
    for (int i = 0; i < k; ++i) {
      const double cr = coeffs[2 * i], ci = coeffs[2 * i + 1];
      const thc_mps *xr = terms_re ? terms_re[i] : nullptr, *xi = terms_im ? terms_im[i] : nullptr;
      for (const thc_mps *x : {xr, xi})
        if (x) {
          check_mps(x, n);
          if (x->data == out_re->data || x->data == out_im->data) raise(THC_EINVAL, "output aliases an input");
        }
      const double c[2][2] = {{cr, -ci}, {cr, ci}};
      const thc_mps *x[2][2] = {{xr, xi}, {xi, xr}};
      for (int part = 0; part < 2; ++part)
        for (int h = 0; h < 2; ++h)
          if (x[part][h] && c[part][h] != 0.0) {
            co[part].push_back(c[part][h]);
            tm[part].push_back(x[part][h]);
          }
    }
    hipStream_t s = (hipStream_t)hip_stream;
    thc_stats acc{};
    for (int part = 0; part < 2; ++part) {
      thc_mps *dst = part == 0 ? out_re : out_im;
      if (co[part].empty()) {
        RPart zero;
        store_part(zero, dst, n, s);
        continue;
      }
      thc_stats s1{};
      check(mps_sum_compress(ctx, (int)co[part].size(), co[part].data(), tm[part].data(), dst, o, &s1, s));
      add_stats(acc, s1);
    }
    HIPCHK(hipStreamSynchronize(s));
    if (st) *st = acc;
  });
}

thc_status mps_overlap_complex(thc_ctx *ctx, const thc_mps *a_re, const thc_mps *a_im, const thc_mps *b_re,
                               const thc_mps *b_im, double *result, void *hip_stream) {
  if (!ctx || !result) return fail(THC_EINVAL, "NULL argument");
  return run_guarded([&] {
    auto ov = [&](const thc_mps *x, const thc_mps *y) {
      if (!x || !y) return 0.0;
      double r = 0.0;
      check(mps_overlap(ctx, x, y, &r, hip_stream));
      return r;
    };
    const double re = ov(a_re, b_re) + ov(a_im, b_im);
    const double im = ov(a_re, b_im) - ov(a_im, b_re);
    result[0] = re;
    result[1] = im;
  });
}

}  // extern "C"

// ===========================================================================
// Energy and gradient w.r.t. the THC factors (THC-factor fitting, Sec. 2.3;
// the G-term structure of Sec. 3.1).  With E_pq = sum_s a+_{ps} a_{qs} and
// N_nu = sum_s a+(chi^nu)_s a(chi^nu)_s, everything follows from the
// transition one-body matrices G^nu_pq = <psi|E_pq N_nu|psi>:
//   <psi|N_mu N_nu|psi> = chi^mu^T G^nu chi^mu,  dE/dzeta = that / 2,
//   dE/dchi_p^k = ((M_k + M_k^T) chi^k)_p,  M_k = sum_nu sym(zeta)_{k nu} G^nu.
// Kets: n_{nu s'}|psi> = a+(chi^nu)_s' a(chi^nu)_s' |psi> for the 2N pairs
// (nu, s'), formed exactly by two layer constructions (bond 4 b_j, no
// compression), and n_{u_i s}|psi> for the 2L kinetic pairs (App. D), of
// which only the overlap <psi|n|psi> is needed.  g_ij = <psi|a+_i a_j|ket>
// comes from transfer-matrix chains with the Jordan-Wigner string of
// a+_i a_j (c+_i Z...Z c_j for i < j, c_j Z...Z c+_i for i > j): a stack
// of environments opened at every site i is carried to the right through Z
// and closed at every later site, all kets of a chunk batched per GEMM.
// ===========================================================================
namespace {

struct GradPlan {
  int n = 0;
  std::vector<int> b, B1, B4;         // bra, first-layer and ket bonds
  std::vector<int64_t> o1, o4, oR;    // site offsets (per ket) of the layer states and right environments
  int64_t S1 = 0, S4 = 0, SR = 0;     // per-ket strides
  int64_t blkO = 0, blkF = 0;         // largest environment block (b x B) and F block (b x 2B)
};

GradPlan make_grad_plan(const thc_mps *psi) {
  GradPlan G;
  const int n = psi->n_sites;
  G.n = n;
  G.b.assign(psi->bonds, psi->bonds + n + 1);
  G.B1.assign(n + 1, 1);
  G.B4.assign(n + 1, 1);
  for (int j = 1; j < n; ++j) {
    G.B1[j] = 2 * G.b[j];
    G.B4[j] = 4 * G.b[j];
  }
  G.o1.assign(n, 0);
  G.o4.assign(n, 0);
  G.oR.assign(n + 1, 0);
  for (int j = 0; j < n; ++j) {
    G.o1[j] = G.S1;
    G.S1 += (int64_t)G.B1[j] * 2 * G.B1[j + 1];
    G.o4[j] = G.S4;
    G.S4 += (int64_t)G.B4[j] * 2 * G.B4[j + 1];
  }
  for (int j = 0; j <= n; ++j) {
    G.oR[j] = G.SR;
    G.SR += (int64_t)G.b[j] * G.B4[j];
    G.blkO = std::max(G.blkO, (int64_t)G.b[j] * G.B4[j]);
    if (j < n) G.blkF = std::max(G.blkF, (int64_t)G.b[j] * 2 * G.B4[j + 1]);
  }
  return G;
}

}  // namespace

extern "C" {

thc_status thc_energy_gradient(thc_ctx *ctx, const thc_mps *psi, int32_t prec, double *energy, double *dchi,
                               double *dzeta, void *hip_stream) {
  if (!ctx) return fail(THC_EINVAL, "ctx is NULL");
  return run_guarded([&] {
    check_mps(psi, ctx->n);
    if (prec != THC_PREC_F64 && prec != THC_PREC_F32) raise(THC_EINVAL, "gradient precision must be F64 or F32");
    if (!energy && !dchi && !dzeta) raise(THC_EINVAL, "no output requested");
    const int gp = (prec == THC_PREC_F32) ? GEMM_F32 : GEMM_F64;
    hipStream_t st = (hipStream_t)hip_stream;
    const int L = ctx->L, N = ctx->N, n = ctx->n;
    const GradPlan P = make_grad_plan(psi);
    const int nkx = 2 * N, nkt = 2 * L, nk = nkx + nkt;
    // per-ket device memory: layer states, right environments, E and F_E,
    // W, two stacks of open environments and the stack product
    const int64_t per_ket = P.S1 + P.S4 + P.SR + 2 * P.blkO + 2 * P.blkF + 2 * (2 * n) * P.blkO + (2 * n) * P.blkF;
    const double budget = 48.0 * (1ull << 30);
    int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(nk, (int64_t)(budget / (8.0 * per_ket))));
    DevBuf ws, jobs_d, gbuf, ovl, fin, lamd, chid, zetad;
    ws.ensure((size_t)per_ket * chunk * sizeof(double));
    gbuf.ensure((size_t)std::max(nkx, 1) * n * n * sizeof(double));
    ovl.ensure((size_t)nk * sizeof(double));
    launch_fill(st, 1, gbuf.as<double>(), 0, (int64_t)std::max(nkx, 1) * n * n, 0.0);
    double *W0 = ws.as<double>();
    double *Phi1 = W0, *Phi4 = Phi1 + P.S1 * chunk, *Renv = Phi4 + P.S4 * chunk, *Eb = Renv + P.SR * chunk,
           *E2 = Eb + P.blkO * chunk, *FE = E2 + P.blkO * chunk, *Wb = FE + P.blkF * chunk,
           *Ost = Wb + P.blkF * chunk, *Ost2 = Ost + (2 * n) * P.blkO * chunk, *Fst = Ost2 + (2 * n) * P.blkO * chunk;
    const int64_t sO = (2 * n) * P.blkO, sF = (2 * n) * P.blkF;
    DevBuf AZ;
    int64_t maxA = 1;
    for (int j = 0; j < n; ++j) maxA = std::max(maxA, (int64_t)P.b[j] * 2 * P.b[j + 1]);
    AZ.ensure((size_t)maxA * sizeof(double));
    jobs_d.ensure((size_t)chunk * sizeof(CJob));
    std::vector<CJob> hj(chunk);
    for (int k0 = 0; k0 < nk; k0 += chunk) {
      const int nc = std::min(chunk, nk - k0);
      // ---- kets: two layer constructions per ket ----
      for (int layer = 0; layer < 2; ++layer) {
        for (int q = 0; q < nc; ++q) {
          const int k = k0 + q;
          const int row = (k < nkx) ? k : 2 * N + (k - nkx);  // coefficient rows: 2 nu + s', then 2N + 2i + s
          CJob jb{};
          jb.kind = 0;
          jb.in_a = (layer == 0) ? psi->data : Phi1 + (int64_t)q * P.S1;
          jb.y = ctx->coef_ptr(row);
          jb.dag = layer;
          jb.ca = 1.0;
          hj[q] = jb;
        }
        HIPCHK(hipMemcpyAsync(jobs_d.p, hj.data(), nc * sizeof(CJob), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));  // the host job array is reused by the next layer
        for (int j = 0; j < n; ++j) {
          if (layer == 0)
            launch_construct(st, jobs_d.as<CJob>(), nc, j, n, psi->offsets[j], 0, P.b[j], P.b[j + 1], 0, 0,
                             Phi1 + P.o1[j], P.S1, P.B1[j], P.B1[j + 1]);
          else
            launch_construct(st, jobs_d.as<CJob>(), nc, j, n, P.o1[j], 0, P.B1[j], P.B1[j + 1], 0, 0,
                             Phi4 + P.o4[j], P.S4, P.B4[j], P.B4[j + 1]);
        }
      }
      // ---- right environments R_j (b_j x B_j), R_n = [1] ----
      launch_fill(st, nc, Renv + P.oR[n], P.SR, 1, 1.0);
      for (int j = n - 1; j >= 1; --j) {
        const double *Aj = psi->data + psi->offsets[j];
        // W = A_j (2 b_j x b_{j+1}) R_{j+1} (b_{j+1} x B_{j+1})
        launch_gemm(st, nc, 0, Aj, 0, P.b[j + 1], Renv + P.oR[j + 1], P.SR, P.B4[j + 1], Wb, P.blkF, P.B4[j + 1],
                    2 * P.b[j], P.B4[j + 1], P.b[j + 1], 1.0, 0.0, gp);
        // R_j = W (b_j x 2 B_{j+1}) B_j^T (ket site j viewed B_j x 2 B_{j+1})
        launch_gemm(st, nc, GEMM_TB, Wb, P.blkF, 2 * P.B4[j + 1], Phi4 + P.o4[j], P.S4, 2 * P.B4[j + 1],
                    Renv + P.oR[j], P.SR, P.B4[j], P.b[j], P.B4[j], 2 * P.B4[j + 1], 1.0, 0.0, gp);
      }
      // ---- left sweep: plain environment, open stack, closings ----
      const int nx = std::max(0, std::min(nc, nkx - k0));  // kets of this chunk that need g
      launch_fill(st, nc, Eb, P.blkO, 1, 1.0);
      double *Ocur = Ost, *Onext = Ost2;
      for (int j = 0; j < n; ++j) {
        const int bl = P.b[j], br = P.b[j + 1], Bl = P.B4[j], Br = P.B4[j + 1];
        const double *Aj = psi->data + psi->offsets[j];
        const double *Kj = Phi4 + P.o4[j];
        // F_E = E_j (bl x Bl) B_j (Bl x 2 Br)
        launch_gemm(st, nc, 0, Eb, P.blkO, Bl, Kj, P.S4, 2 * Br, FE, P.blkF, 2 * Br, bl, 2 * Br, Bl, 1.0, 0.0, gp);
        if (nx > 0) {
          // W = A_j (2 bl x br) R_{j+1} (br x Br)
          launch_gemm(st, nx, 0, Aj, 0, br, Renv + P.oR[j + 1], P.SR, Br, Wb, P.blkF, Br, 2 * bl, Br, br, 1.0, 0.0,
                      gp);
          launch_rdm_close(st, 1, nx, FE, P.blkF, 0, Wb, P.blkF, bl, Br, gbuf.as<double>() + (int64_t)k0 * n * n, n, j,
                           1);
          if (j > 0) {
            // stack of 2j open environments (bl x Bl each) times the ket site
            launch_gemm(st, nx, 0, Ocur, sO, Bl, Kj, P.S4, 2 * Br, Fst, sF, 2 * Br, 2 * j * bl, 2 * Br, Bl, 1.0, 0.0,
                        gp);
            launch_rdm_close(st, 2 * j, nx, Fst, sF, (int64_t)bl * 2 * Br, Wb, P.blkF, bl, Br,
                             gbuf.as<double>() + (int64_t)k0 * n * n, n, j, 0);
          }
          if (j + 1 < n) {
            // carry the open environments through Z: O' = A^Z^T F_r
            launch_negate_odd(st, Aj, AZ.as<double>(), bl, br);
            for (int r = 0; r < 2 * j; ++r)
              launch_gemm(st, nx, GEMM_TA, AZ.as<double>(), 0, br, Fst + (int64_t)r * bl * 2 * Br, sF, Br,
                          Onext + (int64_t)r * br * Br, sO, Br, br, Br, 2 * bl, 1.0, 0.0, gp);
            // open two more at site j: c+ (bra 1, ket 0) and c (bra 0, ket 1)
            launch_gemm(st, nx, GEMM_TA, Aj + br, 0, 2 * br, FE, P.blkF, 2 * Br, Onext + (int64_t)(2 * j) * br * Br,
                        sO, Br, br, Br, bl, 1.0, 0.0, gp);
            launch_gemm(st, nx, GEMM_TA, Aj, 0, 2 * br, FE + Br, P.blkF, 2 * Br, Onext + (int64_t)(2 * j + 1) * br * Br,
                        sO, Br, br, Br, bl, 1.0, 0.0, gp);
            std::swap(Ocur, Onext);
          }
        }
        // E_{j+1} = A_j^T (br x 2 bl) F_E (2 bl x Br)
        launch_gemm(st, nc, GEMM_TA, Aj, 0, br, FE, P.blkF, Br, E2, P.blkO, Br, br, Br, 2 * bl, 1.0, 0.0, gp);
        launch_copy(st, nc, E2, P.blkO, Eb, P.blkO, (int64_t)br * Br);
      }
      // E_n is 1 x 1: the overlap <psi|ket>
      launch_copy(st, nc, Eb, P.blkO, ovl.as<double>() + k0, 1, 1);
      HIPCHK(hipGetLastError());
    }
    // ---- final contraction on the device ----
    std::vector<double> lam(ctx->lam);
    lamd.ensure((size_t)L * sizeof(double));
    chid.ensure((size_t)std::max(1, L * N) * sizeof(double));
    zetad.ensure((size_t)std::max(1, N * N) * sizeof(double));
    fin.ensure((size_t)(1 + L * N + N * N + N * L * L + L * L + 1) * sizeof(double));
    HIPCHK(hipMemcpyAsync(lamd.p, lam.data(), L * sizeof(double), hipMemcpyHostToDevice, st));
    if (N > 0) {
      HIPCHK(hipMemcpyAsync(chid.p, ctx->chi.data(), (size_t)L * N * sizeof(double), hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(zetad.p, ctx->zeta.data(), (size_t)N * N * sizeof(double), hipMemcpyHostToDevice, st));
    }
    double *out_d = fin.as<double>();
    double *Gw = out_d + 1 + L * N + N * N;
    launch_grad_final(st, gbuf.as<double>(), n, L, N, chid.as<double>(), zetad.as<double>(), lamd.as<double>(),
                      ovl.as<double>(), Gw, out_d);
    HIPCHK(hipGetLastError());
    std::vector<double> host(1 + L * N + N * N);
    HIPCHK(hipMemcpyAsync(host.data(), out_d, host.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (energy) *energy = host[0];
    if (dchi) memcpy(dchi, host.data() + 1, (size_t)L * N * sizeof(double));
    if (dzeta) memcpy(dzeta, host.data() + 1 + L * N, (size_t)N * N * sizeof(double));
  });
}

}  // extern "C"
