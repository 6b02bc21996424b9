// qdwf_dot_noalloc: the FP64-accumulated inner products of qdwf_dot without a
// caller workspace, for callers that cannot allocate device memory. Its
// per-block partial sums and its results live in one file-scope device array,
// `scratch`, of a fixed size; each GPU the library runs on holds its own copy
// until the process ends. The kernels are qdwf_dot's own (same reduction tree),
// so the two entry points return bitwise equal results.
//
// Host code never hands the array's name to a kernel or a copy: it stands for
// a host-side shadow, not a device address. The device address is looked up
// once per device with hipGetSymbolAddress (with that device current) and kept
// in g_scratch_ptr; every launch takes that pointer.
#include <mutex>

#include "common.h"
#include "solver.h"

static __device__ __align__(256) double scratch[QDWF_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace qdwf {
namespace {

constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
void* g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];

// Device address of `scratch` on `device`, which must be current.
int scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices)
    return fail(QDWF_EINVAL, "device %d beyond the %d devices this entry point serves", device,
                kMaxDevices);
  std::call_once(g_scratch_once[device], [device] {
    void* p = nullptr;
    g_scratch_err[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_ptr[device] = p;
  });
  if (g_scratch_err[device] != hipSuccess || !g_scratch_ptr[device])
    return fail(QDWF_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", device,
                hipGetErrorString(g_scratch_err[device]));
  *out = g_scratch_ptr[device];
  return QDWF_OK;
}

}  // namespace
}  // namespace qdwf

using namespace qdwf;

extern "C" int qdwf_dot_noalloc(qdwf_ctx* ctx, double* out, const void* x, const void* y,
                                int subset, int prec, int layout, int nrhs, void* stream) {
  if (!ctx) return fail(QDWF_EINVAL, "null context");
  if (!out || !x || !y) return fail(QDWF_EINVAL, "out, x and y must not be NULL");
  if (prec < QDWF_F64 || prec > QDWF_BF16) return fail(QDWF_EINVAL, "unknown precision %d", prec);
  if (layout != QDWF_RRII && layout != QDWF_RIRI) return fail(QDWF_EINVAL, "unknown layout %d", layout);
  if (subset != QDWF_EVEN && subset != QDWF_ODD && subset != QDWF_FULL)
    return fail(QDWF_EINVAL, "unknown subset %d", subset);
  if (nrhs < 1 || nrhs > 4096) return fail(QDWF_EINVAL, "nrhs %d out of range [1, 4096]", nrhs);
  const long n = (long)(subset == QDWF_FULL ? 2 : 1) * ctx->g.n5h * 24;
  const size_t need = dot_ws_bytes(n, nrhs);
  if (need > (size_t)QDWF_NOALLOC_SCRATCH_BYTES)
    return fail(QDWF_EINVAL,
                "%d right-hand sides of this field need %zu bytes of scratch; the static "
                "scratch holds %zu (use qdwf_dot with a workspace)",
                nrhs, need, (size_t)QDWF_NOALLOC_SCRATCH_BYTES);
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(ctx->device) != hipSuccess)
    return fail(QDWF_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
  void* ws = nullptr;
  int rc = scratch_address(ctx->device, &ws);
  if (rc == QDWF_OK)
    rc = dot_re_im(ctx, out, x, y, n, prec, layout, nrhs, ws, reinterpret_cast<hipStream_t>(stream));
  (void)hipSetDevice(prev);
  return rc;
}
