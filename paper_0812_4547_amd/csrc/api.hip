// extern "C" entry points of librnnls.so (declared and documented in rnnls.h).
#include <math.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "common.h"

namespace rnnls {

int device_cus() {
  static std::mutex mu;
  static std::vector<int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RNNLS_E_HIP;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
  if (cache[dev] == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return RNNLS_E_HIP;
    cache[dev] = cus > 0 ? cus : 1;
  }
  return cache[dev];
}

namespace {

struct Opts {
  int sample_mode = RNNLS_SAMPLE_EXACT;
  int precision = RNNLS_PREC_FP32;
  int max_iter = 0;
  int r_cap = 0;
  double tol = 0.0;
};

Opts read_opts(const rnnls_opts* o) {
  Opts r;
  if (o) {
    r.sample_mode = o->sample_mode;
    r.precision = o->precision;
    r.max_iter = o->max_iter;
    r.r_cap = o->r_cap;
    r.tol = o->tol;
  }
  return r;
}

bool opts_valid(const Opts& o) {
  return (o.sample_mode == RNNLS_SAMPLE_EXACT || o.sample_mode == RNNLS_SAMPLE_BERNOULLI) &&
         (o.precision == RNNLS_PREC_FP32 || o.precision == RNNLS_PREC_SPLIT_BF16);
}

// Rows the sketch buffers hold.
// Rows the sketch buffers hold.  A Bernoulli sample never keeps more than
// n' rows, so the capacity is clamped to n' (beyond it a tile could not hold
// the kept rows of one column).
int row_capacity(int r, const Opts& o, int64_t n_pad) {
  if (o.sample_mode == RNNLS_SAMPLE_EXACT) return r;
  const int64_t want = o.r_cap > 0 ? o.r_cap : r + 8 * (int64_t)ceil(sqrt((double)r)) + 64;
  return (int)(want < n_pad ? want : n_pad);
}

// Workspace layout; every region 256-byte aligned.
struct Layout {
  size_t rows = 0, count = 0, status = 0, signs = 0, bern = 0, partials = 0, sa = 0, sb = 0,
         mom = 0, G = 0, q = 0, cc = 0, colabs = 0, tab = 0, total = 0;
};

size_t put(size_t& off, size_t bytes) {
  const size_t at = off;
  off += align256(bytes);
  return at;
}

struct Sizes {
  int64_t n = 0, n_pad = 0;
  int d = 0, r = 0, r_cap = 0, m = 0;
  SrhtPlan sp{};
  MomentsPlan mp{};
};

Layout layout_sketch(const Sizes& z, const Opts& o, bool with_solve, bool with_b) {
  Layout L;
  size_t off = 0;
  L.rows = put(off, sizeof(int32_t) * z.r_cap);
  L.count = put(off, sizeof(int32_t));
  L.status = put(off, sizeof(int32_t));
  L.signs = put(off, sizeof(uint32_t) * (size_t)((z.n_pad + 31) / 32));
  L.bern = put(off, sizeof(uint32_t) * streams_scratch_words(z.n_pad));
  L.partials = put(off, srht_partials_bytes(z.sp));
  L.sa = put(off, sizeof(float) * (size_t)z.d * z.r_cap);
  L.sb = put(off, sizeof(float) * (size_t)(with_b ? z.r_cap : 0));
  if (with_solve) {
    L.mom = put(off, moments_scratch_bytes(z.mp));
    L.G = put(off, sizeof(double) * (size_t)z.d * z.d);
    L.q = put(off, sizeof(double) * (size_t)z.d);
    L.cc = put(off, sizeof(double));
    L.colabs = put(off, sizeof(double) * (size_t)z.d);
    L.tab = put(off, lh_large_tableau_bytes(z.d));
  }
  L.total = off;
  return L;
}

// many right-hand sides: sb holds r_cap x k, q holds d x k, cc holds k
Layout layout_multi(const Sizes& z, int k) {
  Layout L;
  size_t off = 0;
  L.rows = put(off, sizeof(int32_t) * z.r_cap);
  L.count = put(off, sizeof(int32_t));
  L.status = put(off, sizeof(int32_t));
  L.signs = put(off, sizeof(uint32_t) * (size_t)((z.n_pad + 31) / 32));
  L.bern = put(off, sizeof(uint32_t) * streams_scratch_words(z.n_pad));
  L.partials = put(off, srht_partials_bytes(z.sp));
  L.sa = put(off, sizeof(float) * (size_t)z.d * z.r_cap);
  L.sb = put(off, sizeof(float) * (size_t)k * z.r_cap);
  L.mom = put(off, moments_scratch_bytes(z.mp));
  L.G = put(off, sizeof(double) * (size_t)z.d * z.d);
  L.q = put(off, sizeof(double) * (size_t)z.d * k);
  L.cc = put(off, sizeof(double) * (size_t)k);
  L.colabs = put(off, sizeof(double) * (size_t)z.d);
  L.total = off;
  return L;
}

Layout layout_solve(const Sizes& z) {
  Layout L;
  size_t off = 0;
  L.mom = put(off, moments_scratch_bytes(z.mp));
  L.G = put(off, sizeof(double) * (size_t)z.d * z.d);
  L.q = put(off, sizeof(double) * (size_t)z.d);
  L.cc = put(off, sizeof(double));
  L.colabs = put(off, sizeof(double) * (size_t)z.d);
  L.tab = put(off, lh_large_tableau_bytes(z.d));
  L.total = off;
  return L;
}

// Validate sketch sizes; returns 0 or -(argument position).
int check_sketch_sizes(int64_t n, int32_t d, int32_t r, const Opts& o, int pos_n, int pos_d,
                       int pos_r, int pos_opts, Sizes* z, int max_d = RNNLS_MAX_D) {
  if (n < 2 || n > (1ll << 30)) return -pos_n;
  if (d < 1 || d > max_d) return -pos_d;
  const int64_t n_pad = (int64_t)next_pow2((uint64_t)n);
  if (r < 1 || (int64_t)r >= n_pad || r > RNNLS_MAX_R) return -pos_r;
  if (!opts_valid(o)) return -pos_opts;
  const int r_cap = row_capacity(r, o, n_pad);
  if (r_cap < 1 || r_cap > RNNLS_MAX_R) return -pos_opts;
  z->n = n;
  z->n_pad = n_pad;
  z->d = d;
  z->r = r;
  z->r_cap = r_cap;
  return 0;
}

// The sketch plan for the requested precision.  Split-BF16 needs n' >= 2^14
// (smaller problems run the FP32 transform, which is at least as accurate)
// and at most 32 kept rows per thread of its 256-thread workgroups.
SrhtPlan plan_for(int64_t n, int ncols, int r_cap, int cus, const Opts& o) {
  if (o.precision == RNNLS_PREC_SPLIT_BF16 && next_pow2((uint64_t)n) >= (1ull << 14))
    return srht_plan_split_bf16(n, ncols, r_cap, cus);
  return srht_plan(n, ncols, r_cap, cus);
}

int sketch_core(const Sizes& z, const Opts& o, uint64_t seed, const float* A, int64_t lda,
                const float* b, float* SA, int64_t ldsa, float* Sb, int32_t* rows,
                int32_t* count, uint32_t* signs, uint32_t* sign_export, int32_t* status,
                uint32_t* stream_scratch, float* partials, hipStream_t s) {
  if (z.sp.log_t < 0) return RNNLS_E_UNSUPPORTED;  // nothing is launched
  StreamJob sj{};
  sj.seed = seed;
  sj.m = ilog2_exact((uint64_t)z.n_pad);
  sj.r = z.r;
  sj.r_cap = z.r_cap;
  sj.mode = o.sample_mode;
  sj.sign_log_t = z.sp.mfma ? 0 : z.sp.log_t;
  sj.sign_words = signs;
  sj.sign_export = sign_export;
  sj.scratch = stream_scratch;
  sj.rows = rows;
  sj.count = count;
  sj.status = status;
  int rc = launch_streams(sj, s);
  if (rc) return rc;
  SketchJob kj{};
  kj.A = A;
  kj.lda = lda;
  kj.B = b;
  kj.ldb = z.n;
  kj.d = z.d;
  kj.sign_words = signs;
  kj.rows = rows;
  kj.count = count;
  kj.partials = partials;
  kj.SA = SA;
  kj.ldsa = ldsa;
  kj.SB = Sb;
  kj.ldsb = z.r_cap;
  kj.inv_sqrt_r = 1.0 / sqrt((double)z.r);
  return launch_srht(z.sp, kj, s);
}

MomentJob moment_job(const MomentsPlan& mp, const float* M, int64_t ldm, const float* F,
                     int64_t ldf, const int32_t* m_dev, double* scratch, double* G, double* Q,
                     int64_t ldq, double* c, double* colabs) {
  MomentJob j{};
  j.M = M;
  j.ldm = ldm;
  j.F = F;
  j.ldf = ldf;
  j.m_dev = m_dev;
  j.part = scratch;
  j.part_abs = moments_abs_scratch(mp, scratch);
  j.G = G;
  j.Q = Q;
  j.ldq = ldq;
  j.c = c;
  j.colabs = colabs;
  return j;
}

LhJob lh_job(int d, int64_t m, const int32_t* m_dev, const Opts& o, const double* G,
             const double* q, const double* c, const double* colabs, const int32_t* pre_status,
             double* x, double* w, double* rnorm, int32_t* iters, int32_t* status) {
  LhJob j{};
  j.d = d;
  j.max_iter = o.max_iter > 0 ? o.max_iter : 3 * d;
  j.m = m;
  j.tol = o.tol;
  j.G = G;
  j.q = q;
  j.q_stride = d;
  j.c = c;
  j.c_stride = 1;
  j.colabs = colabs;
  j.m_dev = m_dev;
  j.pre_status = pre_status;
  j.x = x;
  j.x_stride = d;
  j.w = w;
  j.w_stride = d;
  j.rnorm = rnorm;
  j.iters = iters;
  j.status = status;
  return j;
}

bool ws_ok(void* ws, size_t ws_bytes, size_t need) {
  return need == 0 || (ws != nullptr && ((uintptr_t)ws % 256) == 0 && ws_bytes >= need);
}

// A sketch workspace serves calls with and without b.
size_t sketch_ws_need(Sizes z, const Opts& o, int64_t n, int cus) {
  z.sp = plan_for(n, z.d + 1, z.r_cap, cus, o);
  const size_t with_b = layout_sketch(z, o, false, true).total;
  z.sp = plan_for(n, z.d, z.r_cap, cus, o);
  const size_t without_b = layout_sketch(z, o, false, false).total;
  return with_b > without_b ? with_b : without_b;
}

template <class T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(ws) + off);
}

}  // namespace
}  // namespace rnnls

using namespace rnnls;

extern "C" {

int rnnls_version(void) { return 10000; }

int rnnls_device_cus(void) { return device_cus(); }

int rnnls_set_tuning(const rnnls_tuning* tuning) { return set_tuning(tuning); }

int rnnls_get_tuning(rnnls_tuning* tuning) { return get_tuning(tuning); }

size_t rnnls_workspace_bytes(int32_t op, int64_t n, int32_t d, int32_t r,
                             const rnnls_opts* opts) {
  const Opts o = read_opts(opts);
  Sizes z;
  const int cus = device_cus();
  if (cus < 0) return 0;
  if (op == RNNLS_OP_SOLVE) {
    if (n < 1 || d < 1 || d > RNNLS_MAX_D_SOLVE) return 0;
    z.d = d;
    z.mp = moments_plan(n, d, 1, cus);
    return layout_solve(z).total;
  }
  if (op != RNNLS_OP_SKETCH && op != RNNLS_OP_RAND_NNLS) return 0;
  if (check_sketch_sizes(n, d, r, o, 1, 2, 3, 4, &z, RNNLS_MAX_D_SOLVE)) return 0;
  z.mp = moments_plan(z.r_cap, d, 1, cus);
  if (op == RNNLS_OP_RAND_NNLS) {
    z.sp = plan_for(n, d + 1, z.r_cap, cus, o);
    return layout_sketch(z, o, true, true).total;
  }
  return sketch_ws_need(z, o, n, cus);
}

int rnnls_srht_sketch(int64_t n, int32_t d, int32_t r, uint64_t seed, const float* A,
                      int64_t lda, const float* b, float* SA, int64_t ldsa, float* Sb,
                      int32_t* rows, int32_t* r_out, uint32_t* sign_bits, int32_t* status,
                      const rnnls_opts* opts, void* ws, size_t ws_bytes, void* stream) {
  const Opts o = read_opts(opts);
  Sizes z;
  int rc = check_sketch_sizes(n, d, r, o, 1, 2, 3, 15, &z, RNNLS_MAX_D_SOLVE);
  if (rc) return rc;
  if (!A) return -5;
  if (lda < n) return -6;
  if (!SA) return -8;
  if (ldsa < z.r_cap) return -9;
  if (b && !Sb) return -10;
  const int cus = device_cus();
  if (cus < 0) return cus;
  if (!ws_ok(ws, ws_bytes, sketch_ws_need(z, o, n, cus))) return RNNLS_E_WORKSPACE;
  z.sp = plan_for(n, d + (b ? 1 : 0), z.r_cap, cus, o);
  const Layout L = layout_sketch(z, o, false, b != nullptr);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return sketch_core(z, o, seed, A, lda, b, SA, ldsa, Sb,
                     rows ? rows : at<int32_t>(ws, L.rows),
                     r_out ? r_out : at<int32_t>(ws, L.count),
                     at<uint32_t>(ws, L.signs), sign_bits,
                     status ? status : at<int32_t>(ws, L.status), at<uint32_t>(ws, L.bern),
                     at<float>(ws, L.partials), s);
}

int rnnls_nnls_solve(int64_t m, int32_t d, const float* M, int64_t ldm, const float* f,
                     const int32_t* m_dev, double* x, double* w, double* rnorm, int32_t* iters,
                     int32_t* status, const rnnls_opts* opts, void* ws, size_t ws_bytes,
                     void* stream) {
  const Opts o = read_opts(opts);
  if (m < 1) return -1;
  if (d < 1 || d > RNNLS_MAX_D_SOLVE) return -2;
  if (!M) return -3;
  if (ldm < m) return -4;
  if (!f) return -5;
  if (!x) return -7;
  if (!opts_valid(o)) return -12;
  const int cus = device_cus();
  if (cus < 0) return cus;
  Sizes z;
  z.d = d;
  z.mp = moments_plan(m, d, 1, cus);
  const Layout L = layout_solve(z);
  if (!ws_ok(ws, ws_bytes, L.total)) return RNNLS_E_WORKSPACE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  double* G = at<double>(ws, L.G);
  double* q = at<double>(ws, L.q);
  double* cc = at<double>(ws, L.cc);
  double* colabs = at<double>(ws, L.colabs);
  int rc = launch_moments(
      z.mp, moment_job(z.mp, M, ldm, f, m, m_dev, at<double>(ws, L.mom), G, q, d, cc, colabs), s);
  if (rc) return rc;
  LhJob lj = lh_job(d, m, m_dev, o, G, q, cc, colabs, nullptr, x, w, rnorm, iters, status);
  lj.tab = at<double>(ws, L.tab);
  return launch_lawson_hanson(lj, 1, s);
}

int rnnls_rand_nnls(int64_t n, int32_t d, int32_t r, uint64_t seed, const float* A, int64_t lda,
                    const float* b, double* x, double* rnorm, int32_t* iters, int32_t* status,
                    float* SA, int64_t ldsa, float* Sb, int32_t* rows, int32_t* r_out,
                    const rnnls_opts* opts, void* ws, size_t ws_bytes, void* stream) {
  const Opts o = read_opts(opts);
  Sizes z;
  int rc = check_sketch_sizes(n, d, r, o, 1, 2, 3, 17, &z, RNNLS_MAX_D_SOLVE);
  if (rc) return rc;
  if (!A) return -5;
  if (lda < n) return -6;
  if (!b) return -7;
  if (!x) return -8;
  if (SA && ldsa < z.r_cap) return -13;
  const int cus = device_cus();
  if (cus < 0) return cus;
  z.sp = plan_for(n, d + 1, z.r_cap, cus, o);
  z.mp = moments_plan(z.r_cap, d, 1, cus);
  const Layout L = layout_sketch(z, o, true, true);
  if (!ws_ok(ws, ws_bytes, L.total)) return RNNLS_E_WORKSPACE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  float* sa = SA ? SA : at<float>(ws, L.sa);
  const int64_t ld = SA ? ldsa : z.r_cap;
  float* sb = Sb ? Sb : at<float>(ws, L.sb);
  int32_t* cnt = r_out ? r_out : at<int32_t>(ws, L.count);
  int32_t* st = status ? status : at<int32_t>(ws, L.status);
  rc = sketch_core(z, o, seed, A, lda, b, sa, ld, sb, rows ? rows : at<int32_t>(ws, L.rows), cnt,
                   at<uint32_t>(ws, L.signs), nullptr, st, at<uint32_t>(ws, L.bern),
                   at<float>(ws, L.partials), s);
  if (rc) return rc;
  double* G = at<double>(ws, L.G);
  double* q = at<double>(ws, L.q);
  double* cc = at<double>(ws, L.cc);
  double* colabs = at<double>(ws, L.colabs);
  rc = launch_moments(
      z.mp, moment_job(z.mp, sa, ld, sb, z.r_cap, cnt, at<double>(ws, L.mom), G, q, d, cc, colabs),
      s);
  if (rc) return rc;
  LhJob lj = lh_job(d, z.r_cap, cnt, o, G, q, cc, colabs, st, x, nullptr, rnorm, iters, status);
  lj.tab = at<double>(ws, L.tab);
  return launch_lawson_hanson(lj, 1, s);
}

int rnnls_rand_box(int64_t n, int32_t d, int32_t r, uint64_t seed, const float* A,
                   int64_t lda, const float* b, const double* lo, const double* hi,
                   double* x, double* rnorm, int32_t* iters, int32_t* status,
                   const rnnls_opts* opts, void* ws, size_t ws_bytes, void* stream) {
  const Opts o = read_opts(opts);
  Sizes z;
  int rc = check_sketch_sizes(n, d, r, o, 1, 2, 3, 14, &z);
  if (rc) return rc;
  if (d > RNNLS_MAX_BOX_D) return -2;
  if (!A) return -5;
  if (lda < n) return -6;
  if (!b) return -7;
  if (!lo) return -8;
  if (!hi) return -9;
  if (!x) return -10;
  const int cus = device_cus();
  if (cus < 0) return cus;
  z.sp = plan_for(n, d + 1, z.r_cap, cus, o);
  z.mp = moments_plan(z.r_cap, d, 1, cus);
  const Layout L = layout_sketch(z, o, true, true);
  if (!ws_ok(ws, ws_bytes, L.total)) return RNNLS_E_WORKSPACE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  float* sa = at<float>(ws, L.sa);
  float* sb = at<float>(ws, L.sb);
  int32_t* cnt = at<int32_t>(ws, L.count);
  int32_t* st = at<int32_t>(ws, L.status);
  rc = sketch_core(z, o, seed, A, lda, b, sa, z.r_cap, sb, at<int32_t>(ws, L.rows), cnt,
                   at<uint32_t>(ws, L.signs), nullptr, st, at<uint32_t>(ws, L.bern),
                   at<float>(ws, L.partials), s);
  if (rc) return rc;
  double* G = at<double>(ws, L.G);
  double* q = at<double>(ws, L.q);
  double* cc = at<double>(ws, L.cc);
  double* colabs = at<double>(ws, L.colabs);
  rc = launch_moments(
      z.mp, moment_job(z.mp, sa, z.r_cap, sb, z.r_cap, cnt, at<double>(ws, L.mom), G, q, d, cc,
                       colabs),
      s);
  if (rc) return rc;
  BoxJob bj{};
  bj.d = d;
  bj.max_iter = o.max_iter > 0 ? o.max_iter : 3 * d;
  bj.m = z.r_cap;
  bj.tol = o.tol;
  bj.G = G;
  bj.q = q;
  bj.c = cc;
  bj.colabs = colabs;
  bj.lo = lo;
  bj.hi = hi;
  bj.m_dev = cnt;
  bj.pre_status = st;
  bj.x = x;
  bj.rnorm = rnorm;
  bj.iters = iters;
  bj.status = status;
  return launch_bvls(bj, s);
}

}  // extern "C"

namespace {

// Repetition workspace: one rand_nnls workspace (the k runs reuse it in
// stream order), then the k candidates, their statuses and the residual
// partials.
struct BoostLayout {
  size_t rand = 0, X = 0, st = 0, part = 0, total = 0;
  int grid = 0;
};

int boost_layout(int64_t n, int32_t d, int32_t r, int32_t k, const Opts& o, BoostLayout* B) {
  Sizes z;
  int rc = check_sketch_sizes(n, d, r, o, 1, 2, 3, 13, &z);
  if (rc) return rc;
  if (k < 1 || k > RNNLS_MAX_BOOST) return -4;
  const int cus = device_cus();
  if (cus < 0) return cus;
  z.sp = plan_for(n, d + 1, z.r_cap, cus, o);
  z.mp = moments_plan(z.r_cap, d, 1, cus);
  size_t off = 0;
  B->rand = put(off, layout_sketch(z, o, true, true).total);
  B->X = put(off, sizeof(double) * (size_t)k * d);
  B->st = put(off, sizeof(int32_t) * (size_t)k);
  B->grid = boost_residual_grid(n, cus);
  B->part = put(off, sizeof(double) * (size_t)B->grid * boost_slots(k));
  B->total = off;
  return 0;
}

}  // namespace

extern "C" {

size_t rnnls_boost_workspace_bytes(int64_t n, int32_t d, int32_t r, int32_t k,
                                   const rnnls_opts* opts) {
  BoostLayout B;
  return boost_layout(n, d, r, k, read_opts(opts), &B) ? 0 : B.total;
}

int rnnls_rand_nnls_boost(int64_t n, int32_t d, int32_t r, int32_t k, uint64_t seed,
                          const float* A, int64_t lda, const float* b, double* x,
                          double* resid, int32_t* best, int32_t* status,
                          const rnnls_opts* opts, void* ws, size_t ws_bytes, void* stream) {
  const Opts o = read_opts(opts);
  Sizes z;
  int rc = check_sketch_sizes(n, d, r, o, 1, 2, 3, 13, &z);
  if (rc) return rc;
  if (k < 1 || k > RNNLS_MAX_BOOST) return -4;
  if (!A) return -6;
  if (lda < n) return -7;
  if (!b) return -8;
  if (!x) return -9;
  BoostLayout B;
  rc = boost_layout(n, d, r, k, o, &B);
  if (rc) return rc;
  if (!ws_ok(ws, ws_bytes, B.total)) return RNNLS_E_WORKSPACE;
  double* X = at<double>(ws, B.X);
  int32_t* st = at<int32_t>(ws, B.st);
  const size_t rand_bytes = B.X - B.rand;
  for (int i = 0; i < k; ++i) {
    rc = rnnls_rand_nnls(n, d, r, seed + (uint64_t)i, A, lda, b, X + (size_t)i * d, nullptr,
                         nullptr, st + i, nullptr, 0, nullptr, nullptr, nullptr, opts,
                         at<void>(ws, B.rand), rand_bytes, stream);
    if (rc) return rc;
  }
  return launch_boost_select(n, d, k, A, lda, b, X, st, at<double>(ws, B.part), B.grid, x, resid,
                             best, status, reinterpret_cast<hipStream_t>(stream));
}

size_t rnnls_multi_workspace_bytes(int64_t n, int32_t d, int32_t k, int32_t r,
                                   const rnnls_opts* opts) {
  const Opts o = read_opts(opts);
  Sizes z;
  const int cus = device_cus();
  if (cus < 0 || k < 1 || k > RNNLS_MAX_K) return 0;
  if (check_sketch_sizes(n, d, r, o, 1, 2, 4, 15, &z)) return 0;
  z.sp = plan_for(n, d + k, z.r_cap, cus, o);
  z.mp = moments_plan(z.r_cap, d, k, cus);
  return layout_multi(z, k).total;
}

int rnnls_rand_nnls_multi(int64_t n, int32_t d, int32_t k, int32_t r, uint64_t seed,
                          const float* A, int64_t lda, const float* B, int64_t ldb, double* X,
                          int64_t ldx, double* rnorm, int32_t* iters, int32_t* status,
                          const rnnls_opts* opts, void* ws, size_t ws_bytes, void* stream) {
  const Opts o = read_opts(opts);
  Sizes z;
  if (k < 1 || k > RNNLS_MAX_K) return -3;
  int rc = check_sketch_sizes(n, d, r, o, 1, 2, 4, 15, &z);
  if (rc) return rc;
  if (!A) return -6;
  if (lda < n) return -7;
  if (!B) return -8;
  if (ldb < n) return -9;
  if (!X) return -10;
  if (ldx < d) return -11;
  const int cus = device_cus();
  if (cus < 0) return cus;
  z.sp = plan_for(n, d + k, z.r_cap, cus, o);
  z.mp = moments_plan(z.r_cap, d, k, cus);
  if (z.sp.log_t < 0) return RNNLS_E_UNSUPPORTED;
  const Layout L = layout_multi(z, k);
  if (!ws_ok(ws, ws_bytes, L.total)) return RNNLS_E_WORKSPACE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  float* sa = at<float>(ws, L.sa);
  float* sb = at<float>(ws, L.sb);
  int32_t* cnt = at<int32_t>(ws, L.count);
  int32_t* st = at<int32_t>(ws, L.status);
  int32_t* rows = at<int32_t>(ws, L.rows);
  uint32_t* signs = at<uint32_t>(ws, L.signs);
  StreamJob sj{};
  sj.seed = seed;
  sj.m = ilog2_exact((uint64_t)z.n_pad);
  sj.r = z.r;
  sj.r_cap = z.r_cap;
  sj.mode = o.sample_mode;
  sj.sign_log_t = z.sp.mfma ? 0 : z.sp.log_t;
  sj.sign_words = signs;
  sj.scratch = at<uint32_t>(ws, L.bern);
  sj.rows = rows;
  sj.count = cnt;
  sj.status = st;
  rc = launch_streams(sj, s);
  if (rc) return rc;
  SketchJob kj{};
  kj.A = A;
  kj.lda = lda;
  kj.B = B;
  kj.ldb = ldb;
  kj.d = d;
  kj.sign_words = signs;
  kj.rows = rows;
  kj.count = cnt;
  kj.partials = at<float>(ws, L.partials);
  kj.SA = sa;
  kj.ldsa = z.r_cap;
  kj.SB = sb;
  kj.ldsb = z.r_cap;
  kj.inv_sqrt_r = 1.0 / sqrt((double)z.r);
  rc = launch_srht(z.sp, kj, s);
  if (rc) return rc;
  double* G = at<double>(ws, L.G);
  double* Q = at<double>(ws, L.q);
  double* cc = at<double>(ws, L.cc);
  double* colabs = at<double>(ws, L.colabs);
  rc = launch_moments(z.mp,
                      moment_job(z.mp, sa, z.r_cap, sb, z.r_cap, cnt, at<double>(ws, L.mom), G,
                                 Q, d, cc, colabs),
                      s);
  if (rc) return rc;
  LhJob lj = lh_job(d, z.r_cap, cnt, o, G, Q, cc, colabs, st, X, nullptr, rnorm, iters, status);
  lj.G_stride = 0;        // one G for all right-hand sides
  lj.colabs_stride = 0;
  lj.m_dev_stride = 0;
  lj.pre_stride = 0;
  lj.q_stride = d;
  lj.x_stride = ldx;
  return launch_lawson_hanson(lj, k, s);
}

}  // extern "C"
