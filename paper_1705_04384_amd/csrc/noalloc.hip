// P^{-1} (eq. 4.7 / 4.9) for callers that cannot allocate device memory: the same
// passes as fdg_apply_prec, with the intermediates between the passes carved out of a
// file-scope device array instead of the context's own workspace.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "common.h"
#include "context.h"

using namespace fdg;

namespace {

// Each device that loads the library holds its own copy of this array until the
// process ends.  Host code never passes the array's name to a kernel: it uses the
// device address that hipGetSymbolAddress returned for the current device.
__device__ __align__(256) unsigned char scratch[FDG_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
bool g_scratch_done[kMaxDevices] = {};
void *g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// Bytes one intermediate of `count` elements of `elem` bytes takes, 256-byte aligned,
// with the 256 bytes of slack the context's own workspace buffers also carry.
size_t carve_bytes(size_t count, size_t elem) { return ((count * elem + 256) + 255) / 256 * 256; }

}  // namespace

namespace fdg {

// Looks the array up on device dev (which must be current); once per device.
int scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return set_error(FDG_EINVAL, "device %d beyond the supported %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_done[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_err[dev] = e;
    g_scratch_ptr[dev] = e == hipSuccess ? p : nullptr;
    g_scratch_done[dev] = true;
  }
  return hip_check(g_scratch_err[dev], "hipGetSymbolAddress(scratch)");
}

}  // namespace fdg

extern "C" int fdg_apply_prec_noalloc(fdg_ctx *c, const double *b, double *s) {
  clear_error();
  if (!c || !b || !s) return set_error(FDG_EINVAL, "apply_prec_noalloc: NULL argument");
  if (b == s) return set_error(FDG_EINVAL, "apply_prec_noalloc: input and output alias");
  int st = ctx_ready_prec(c);
  if (st != FDG_OK) return st;
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (c->device < 0 || c->device >= kMaxDevices || !g_scratch_done[c->device])
      return set_error(FDG_EHIP, "apply_prec_noalloc: scratch of device %d not set up", c->device);
    if (g_scratch_err[c->device] != hipSuccess)
      return hip_check(g_scratch_err[c->device], "hipGetSymbolAddress(scratch)");
    base = g_scratch_ptr[c->device];
  }
  const size_t count = (size_t)c->N * (size_t)c->batch;
  // FP64 intermediates (and every pencil with complex pairs, which runs in FP64); the
  // reduced-precision passes keep theirs in FP32
  const bool wide = c->prec == FDG_PREC_FP64 || ctx_has_pairs(c);
  const size_t one = carve_bytes(count, wide ? sizeof(double) : sizeof(float));
  if (2 * one > (size_t)FDG_NOALLOC_SCRATCH_BYTES)
    return set_error(FDG_EINVAL,
                     "apply_prec_noalloc: batch * N = %zu needs %zu scratch bytes, above the %zu available", count,
                     2 * one, (size_t)FDG_NOALLOC_SCRATCH_BYTES);
  unsigned char *p0 = static_cast<unsigned char *>(base), *p1 = p0 + one;
  const Exec ex{c->stream, false};
  if (wide)
    return apply_entries(c, ex, cstrided(b, c->N), mstrided(s, c->N), c->batch, mstrided((double *)p0, c->N),
                         mstrided((double *)p1, c->N), nullptr, nullptr, false);
  return apply_entries(c, ex, cstrided(b, c->N), mstrided(s, c->N), c->batch, mstrided((double *)nullptr, c->N),
                       mstrided((double *)nullptr, c->N), p0, p1, false);
}
