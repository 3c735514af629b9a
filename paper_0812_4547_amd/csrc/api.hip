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
int row_capacity(int r, const Opts& o) {
  if (o.sample_mode == RNNLS_SAMPLE_EXACT) return r;
  if (o.r_cap > 0) return o.r_cap;
  return r + 8 * (int)ceil(sqrt((double)r)) + 64;
}

// Workspace layout; every region 256-byte aligned.
struct Layout {
  size_t rows = 0, count = 0, status = 0, signs = 0, bern = 0, partials = 0, sa = 0, sb = 0,
         mom = 0, G = 0, q = 0, cc = 0, colabs = 0, lh = 0, total = 0;
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
    L.lh = put(off, lh_global_scratch_bytes(z.d, 1));
  }
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
  L.lh = put(off, lh_global_scratch_bytes(z.d, 1));
  L.total = off;
  return L;
}

// Validate sketch sizes; returns 0 or -(argument position).
int check_sketch_sizes(int64_t n, int32_t d, int32_t r, const Opts& o, int pos_n, int pos_d,
                       int pos_r, int pos_opts, Sizes* z) {
  if (n < 2 || n > (1ll << 30)) return -pos_n;
  if (d < 1 || d > RNNLS_MAX_D) return -pos_d;
  const int64_t n_pad = (int64_t)next_pow2((uint64_t)n);
  if (r < 1 || (int64_t)r >= n_pad || r > RNNLS_MAX_R) return -pos_r;
  if (!opts_valid(o)) return -pos_opts;
  const int r_cap = row_capacity(r, o);
  if (r_cap < 1 || r_cap > RNNLS_MAX_R) return -pos_opts;
  z->n = n;
  z->n_pad = n_pad;
  z->d = d;
  z->r = r;
  z->r_cap = r_cap;
  return 0;
}

int sketch_core(const Sizes& z, const Opts& o, uint64_t seed, const float* A, int64_t lda,
                const float* b, float* SA, int64_t ldsa, float* Sb, int32_t* rows,
                int32_t* count, uint32_t* signs, uint32_t* sign_export, int32_t* status,
                uint32_t* stream_scratch,
                float* partials, hipStream_t s) {
  const int m = ilog2_exact((uint64_t)z.n_pad);
  int rc = launch_streams(seed, m, z.r, z.r_cap, o.sample_mode, z.sp.log_t, signs, sign_export,
                          rows, count, status, stream_scratch, s);
  if (rc) return rc;
  const double inv_sqrt_r = 1.0 / sqrt((double)z.r);
  return launch_srht(z.sp, A, lda, b, signs, rows, count, 0.0f, partials, SA, ldsa, Sb, z.d,
                     inv_sqrt_r, s);
}

bool ws_ok(void* ws, size_t ws_bytes, size_t need) {
  return need == 0 || (ws != nullptr && ((uintptr_t)ws % 256) == 0 && ws_bytes >= need);
}

// A sketch workspace serves calls with and without b.
size_t sketch_ws_need(Sizes z, const Opts& o, int64_t n, int cus) {
  z.sp = srht_plan(n, z.d + 1, z.r_cap, cus);
  const size_t with_b = layout_sketch(z, o, false, true).total;
  z.sp = srht_plan(n, z.d, z.r_cap, cus);
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
    if (n < 1 || d < 1 || d > RNNLS_MAX_D) return 0;
    z.d = d;
    z.mp = moments_plan(n, d, cus);
    return layout_solve(z).total;
  }
  if (op != RNNLS_OP_SKETCH && op != RNNLS_OP_RAND_NNLS) return 0;
  if (check_sketch_sizes(n, d, r, o, 1, 2, 3, 4, &z)) return 0;
  z.mp = moments_plan(z.r_cap, d, cus);
  if (op == RNNLS_OP_RAND_NNLS) {
    z.sp = srht_plan(n, d + 1, z.r_cap, cus);
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
  int rc = check_sketch_sizes(n, d, r, o, 1, 2, 3, 15, &z);
  if (rc) return rc;
  if (o.precision != RNNLS_PREC_FP32) return RNNLS_E_UNSUPPORTED;
  if (!A) return -5;
  if (lda < n) return -6;
  if (!SA) return -8;
  if (ldsa < z.r_cap) return -9;
  if (b && !Sb) return -10;
  const int cus = device_cus();
  if (cus < 0) return cus;
  if (!ws_ok(ws, ws_bytes, sketch_ws_need(z, o, n, cus))) return RNNLS_E_WORKSPACE;
  z.sp = srht_plan(n, d + (b ? 1 : 0), z.r_cap, cus);
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
  if (d < 1 || d > RNNLS_MAX_D) return -2;
  if (!M) return -3;
  if (ldm < m) return -4;
  if (!f) return -5;
  if (!x) return -7;
  if (!opts_valid(o)) return -12;
  const int cus = device_cus();
  if (cus < 0) return cus;
  Sizes z;
  z.d = d;
  z.mp = moments_plan(m, d, cus);
  const Layout L = layout_solve(z);
  if (!ws_ok(ws, ws_bytes, L.total)) return RNNLS_E_WORKSPACE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  double* G = at<double>(ws, L.G);
  double* q = at<double>(ws, L.q);
  double* cc = at<double>(ws, L.cc);
  double* colabs = at<double>(ws, L.colabs);
  int rc = launch_moments(z.mp, M, ldm, f, m_dev, at<double>(ws, L.mom), G, q, cc, colabs, s);
  if (rc) return rc;
  const int max_iter = o.max_iter > 0 ? o.max_iter : 3 * d;
  return launch_lawson_hanson(d, G, q, cc, colabs, m, m_dev, o.tol, max_iter, x, w, rnorm, iters,
                              status, nullptr, 1, at<double>(ws, L.lh), s);
}

int rnnls_rand_nnls(int64_t n, int32_t d, int32_t r, uint64_t seed, const float* A, int64_t lda,
                    const float* b, double* x, double* rnorm, int32_t* iters, int32_t* status,
                    float* SA, int64_t ldsa, float* Sb, int32_t* rows, int32_t* r_out,
                    const rnnls_opts* opts, void* ws, size_t ws_bytes, void* stream) {
  const Opts o = read_opts(opts);
  Sizes z;
  int rc = check_sketch_sizes(n, d, r, o, 1, 2, 3, 17, &z);
  if (rc) return rc;
  if (o.precision != RNNLS_PREC_FP32) return RNNLS_E_UNSUPPORTED;
  if (!A) return -5;
  if (lda < n) return -6;
  if (!b) return -7;
  if (!x) return -8;
  if (SA && ldsa < z.r_cap) return -13;
  const int cus = device_cus();
  if (cus < 0) return cus;
  z.sp = srht_plan(n, d + 1, z.r_cap, cus);
  z.mp = moments_plan(z.r_cap, d, cus);
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
  rc = launch_moments(z.mp, sa, ld, sb, cnt, at<double>(ws, L.mom), G, q, cc, colabs, s);
  if (rc) return rc;
  const int max_iter = o.max_iter > 0 ? o.max_iter : 3 * d;
  return launch_lawson_hanson(d, G, q, cc, colabs, z.r_cap, cnt, o.tol, max_iter, x, nullptr, rnorm,
                              iters, status, st, 1, at<double>(ws, L.lh), s);
}

}  // extern "C"
