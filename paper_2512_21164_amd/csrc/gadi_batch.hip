// Batch bookkeeping on the device: gather the control blocks of all members
// of a batch into one contiguous array, so that a poll reads every member's
// state machine with one kernel and one copy instead of one copy per member.
#include <hip/hip_runtime.h>

#include "gadi_internal.h"

namespace gadi {

namespace {

constexpr int kCtlWords = (int)(sizeof(GadiCtl) / sizeof(uint32_t));
static_assert(sizeof(GadiCtl) % sizeof(uint32_t) == 0, "control block is a whole number of words");

// One block per slot: copy slot i's control block (src[i], null for a free
// slot) to dst[i]; a free slot gets phase PH_IDLE and zeros.
__global__ __launch_bounds__(64) void gather_ctl_kernel(const GadiCtl* const* src, GadiCtl* dst, int n) {
  const int i = blockIdx.x;
  if (i >= n) return;
  const uint32_t* s = reinterpret_cast<const uint32_t*>(src[i]);
  uint32_t* d = reinterpret_cast<uint32_t*>(dst + i);
  for (int w = threadIdx.x; w < kCtlWords; w += blockDim.x) d[w] = s ? s[w] : 0u;
}

}  // namespace

hipError_t launch_gather_ctl(const GadiCtl* const* src, GadiCtl* dst, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  gather_ctl_kernel<<<n, 64, 0, st>>>(src, dst, n);
  return hipGetLastError();
}

}  // namespace gadi
