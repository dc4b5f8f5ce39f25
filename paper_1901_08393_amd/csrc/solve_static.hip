// bc_solve_static: bc_solve with the solver workspace in a device array of
// the library, for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The array is a file-scope __device__ variable: each GPU the library runs
// on holds its own copy, at its own address, until the process ends.  Its
// device address is looked up once per device (hipGetSymbolAddress, with
// that device current) on the first call there and kept; host code uses
// only that address, never the symbol itself, which on the host is a
// stand-in and not a device address.  Every call on one GPU shares the
// array: calls that overlap on one GPU (different streams, or a batched
// solve still running) race and must be serialised by the caller.  Nothing
// in the array needs to start at zero: k_solve_init resets the control
// block, barrier slots and release records of every call, the state
// machine's first phase writes every vector it later reads (padding
// included), and the symmetric product writes its partial sums before its
// gather reads them.
#include <mutex>

#include "bc_internal.h"

namespace bc {

// 96 MiB: the solver workspace of any N up to 32000 (both precisions), which
// covers the serving workload's largest meshes (N <= 30000).
constexpr size_t kStaticBytes = size_t(96) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of this device's copy of `scratch`, looked up on the first
// call on the device.
static int scratch_address(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return BC_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) return BC_EDEVICE;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return BC_OK;
}

}  // namespace bc

using namespace bc;

extern "C" {

int32_t bc_solve_static(const void *d_V, int64_t N, int32_t precision, const void *d_pattern, int64_t nnz,
                        const double *d_area, double *d_sigma, const bc_solve_opts *opts, bc_result *d_result,
                        bc_stream stream) {
  if (precision != BC_FP64 && precision != BC_MIXED) return BC_EINVAL;
  if (N < 1 || N > ((int64_t)1 << 20)) return BC_EINVAL;
  if (SolveLayout(N, precision).total > kStaticBytes) return BC_ENOMEM;  // beyond the array: use bc_solve
  void *ws = nullptr;
  const int st = scratch_address(&ws);
  if (st != BC_OK) return st;
  return solve_one(d_V, N, precision, d_pattern, nnz, d_area, d_sigma, opts, ws, kStaticBytes, d_result,
                   static_cast<hipStream_t>(stream));
}

}  // extern "C"
