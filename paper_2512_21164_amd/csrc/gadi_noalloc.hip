// Allocation-free solve: the workspace of the solve is a static device array
// inside the library instead of caller-provided memory, for callers that
// cannot allocate device memory.
//
// The array `scratch` has one instance per GPU, created when the library's
// code object is loaded on that GPU and held until the process ends.  Its
// name is a device symbol: in host code it stands for a host-side shadow, not
// a device address, so the device address is looked up once per GPU (with
// that GPU current) through hipGetSymbolAddress and only that address is
// used afterwards.  All calls on one GPU share the array: overlapping calls
// race.  Each call clears the part it uses with a fill kernel before the
// solve, so a call never sees the previous call's counters or padding.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/gadi.h"
#include "gadi_internal.h"

namespace gadi {
int32_t solve_in_place(const gadi_stencil* st, const gadi_params* p, void* hip_stream, void* ws, size_t ws_cap,
                       hipError_t (*zero_fill)(void*, size_t, hipStream_t), const void* d_b, void* d_x,
                       gadi_report* out, double* h_history);
}

namespace {

static __device__ __align__(256) unsigned char scratch[GADI_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices];          // device address of `scratch` on each GPU (null: not looked up yet)

// Zero `bytes` (a multiple of 16) at p with 16-byte vector stores.
__global__ __launch_bounds__(256) void zero_fill_kernel(uint4* p, size_t n16) {
  const uint4 z = make_uint4(0u, 0u, 0u, 0u);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
    p[i] = z;
}

hipError_t zero_fill(void* p, size_t bytes, hipStream_t st) {
  if (bytes % 16 != 0) return hipErrorInvalidValue;
  const size_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  const size_t want = (n16 + 255) / 256;
  const unsigned grid = (unsigned)(want < 4096 ? want : 4096);
  zero_fill_kernel<<<grid, 256, 0, st>>>(static_cast<uint4*>(p), n16);
  return hipGetLastError();
}

// Device address of this GPU's scratch array (looked up on the first call on the GPU).
int32_t scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return gadi::set_error(GADI_ERR_HIP, "allocation-free solve: no current device");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return gadi::set_error(GADI_ERR_HIP, "allocation-free solve: hipGetSymbolAddress of the scratch array failed");
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return GADI_OK;
}

}  // namespace

extern "C" gadi_status gadi_solve_noalloc(const gadi_stencil* st, const gadi_params* p, void* hip_stream,
                                          const void* d_b, void* d_x, gadi_report* out, double* h_history) {
  void* ws = nullptr;
  const int32_t s = scratch_address(&ws);
  if (s != GADI_OK) return s;
  return gadi::solve_in_place(st, p, hip_stream, ws, GADI_NOALLOC_SCRATCH_BYTES, zero_fill, d_b, d_x, out,
                              h_history);
}
