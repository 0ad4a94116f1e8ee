// Allocation-free fraction to the boundary (the IPM's min-reduction of
// Sec. 2.1), for callers that cannot allocate device memory or create a
// handle: code under stream capture, tight serving loops.
//
// The partial records of the reduction live in a file-scope device array
// (`scratch`, kNoAllocWords doubles, held by every GPU the library runs on
// until the process ends).  Host code never passes the array's name to a
// kernel: the name is a host-side stand-in, not a device address.  The first
// call on a device looks up that device's copy with hipGetSymbolAddress and
// keeps the address per device; every launch takes that address.
//
// Every record the reduction reads is written earlier in the same call, so
// nothing has to start at zero.  Calls on one GPU share its array: calls
// that overlap on that GPU (two streams, or two host threads) race.
#include <mutex>

#include "internal.hpp"
#include "ipm.hpp"
#include "mdsipm.h"

namespace mds {
namespace {

// kRedBlocks records of 8 doubles, then the 8-double final record
constexpr size_t kNoAllocWords = (size_t)kRedBlocks * 8 + 8;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kNoAllocWords];

std::mutex g_mu;
double *g_ptr[kMaxDevices] = {};

// Device address of the current device's `scratch`, looked up once per device.
int scratch_ptr(double **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MDS_EHIP;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return MDS_EHIP;
    }
    g_ptr[dev] = static_cast<double *>(p);
  }
  *out = g_ptr[dev];
  return MDS_OK;
}

}  // namespace
}  // namespace mds

extern "C" {

size_t mds_ftb_noalloc_scratch_bytes(void) { return sizeof(double) * mds::kNoAllocWords; }

int mds_ftb_noalloc(int64_t n, const double *v, const double *dv, double tau, double *alpha,
                    void *stream) {
  using namespace mds;
  if (!alpha) return MDS_ENULL;
  if (n < 0) return MDS_EDIMS;
  if (n > 0 && (!v || !dv)) return MDS_ENULL;
  if (!(tau > 0.0 && tau <= 1.0)) return MDS_EINVAL;
  // the reduction uses at most kRedBlocks partial records for any n (its
  // grid is capped there), which is what the array holds
  static_assert(kNoAllocWords >= (size_t)kRedBlocks * 8 + 8, "scratch size");
  double *sp = nullptr;
  const int rc = scratch_ptr(&sp);
  if (rc != MDS_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  ipm_ftb1_to_device(s, n, v, dv, tau, sp, sp + (size_t)kRedBlocks * 8, alpha);
  if (hipGetLastError() != hipSuccess) return MDS_EHIP;
  return MDS_OK;
}

}  // extern "C"
