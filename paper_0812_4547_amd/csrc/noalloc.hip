// rnnls_rand_nnls_noalloc: Algorithm 1 (as rnnls_rand_nnls) for callers that
// cannot allocate device memory.  Its scratch -- the random streams' words,
// the kept rows, the sketch partials and the sketch itself, the moments
// scratch and G, q, c -- lives in one fixed array in the library's device
// memory instead of a caller workspace.
//
// Host code never passes the array's name to a kernel or a copy: on the host
// the name is only a stand-in for the symbol.  Its device address is read
// once per device with hipGetSymbolAddress (each device holds its own copy of
// the array at its own address) on the first call made with that device
// current, and every later call on that device passes that address down as
// the workspace pointer, exactly as a caller's workspace is passed.
//
// Nothing in the array has to start at zero: every region a call reads is
// written earlier in the same call (as with a caller's uninitialised
// workspace).  Calls that overlap on one device race on the array.
#include <mutex>

#include "common.h"

static __device__ __align__(256) unsigned char scratch[RNNLS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (read once per device).
int scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return RNNLS_E_HIP;
  if (dev < 0 || dev >= kMaxDevices) return RNNLS_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RNNLS_E_HIP;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return RNNLS_OK;
}

}  // namespace

extern "C" int rnnls_rand_nnls_noalloc(int64_t n, int32_t d, int32_t r, uint64_t seed,
                                       const float* A, int64_t lda, const float* b, double* x,
                                       double* rnorm, int32_t* iters, int32_t* status,
                                       float* SA, int64_t ldsa, float* Sb, int32_t* rows,
                                       int32_t* r_out, const rnnls_opts* opts, void* stream) {
  // invalid sizes (need == 0) fall through: rnnls_rand_nnls names the argument
  const size_t need = rnnls_workspace_bytes(RNNLS_OP_RAND_NNLS, n, d, r, opts);
  if (need > (size_t)RNNLS_NOALLOC_SCRATCH_BYTES) return RNNLS_E_WORKSPACE;
  void* ws = nullptr;
  const int rc = scratch_address(&ws);
  if (rc) return rc;
  return rnnls_rand_nnls(n, d, r, seed, A, lda, b, x, rnorm, iters, status, SA, ldsa, Sb, rows,
                         r_out, opts, ws, (size_t)RNNLS_NOALLOC_SCRATCH_BYTES, stream);
}
