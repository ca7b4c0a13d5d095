// hl_lambda_min_noalloc: the eigen-step of hl_lambda_min (Sections 4.2 and
// 4.5) for callers that cannot allocate device memory.  Its scratch (the status
// word and the eigen-step's work area) is a file-scope device array of
// kNoAllocBytes, one copy per GPU for the life of the process, instead of a
// region of the caller's workspace.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "hl_host.hpp"
#include "hl_kernels.hpp"

namespace hl {

// 64 MiB: the eigen work area of k <= 16 at every precision, of k = 24 up to
// P = 36224 bits and of k = 32 up to P = 20608 (larger shapes are refused)
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
constexpr size_t kNoAllocStatus = 256;  // DevStatus at offset 0, the eigen work area after it
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// device address of `scratch` on each device, looked up once with that device
// current (the array's host-side name is not a device address)
static void* g_scratch[kMaxDevices];
static std::mutex g_scratch_mu;

hipError_t noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return hipSuccess;
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != device) {
    const hipError_t e2 = hipSetDevice(cur);
    if (e == hipSuccess) e = e2;
  }
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch[device] = p;
  return hipSuccess;
}

static void* noalloc_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch[device];
}

}  // namespace hl

using namespace hl;

#define NACHK(x)                                                                   \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess) return fail(HL_EHIP, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

extern "C" hl_status hl_lambda_min_noalloc(hl_ctx* ctx, const hl_shape* sh, const uint32_t* blk,
                                           const int64_t* blk_exp, uint32_t* lam_mant, uint32_t* lam_mant_km1,
                                           hl_lambda_t* out, void* stream) {
  if (!ctx) return fail(HL_EINVAL, "null ctx");
  Dims dm;
  hl_status s = make_dims(sh, &dm);
  if (s != HL_OK) return s;
  if (!blk || !blk_exp || !out) return fail(HL_EINVAL, "null argument");
  const size_t need = kNoAllocStatus + eig_ws_bytes(dm);
  if (need > kNoAllocBytes)
    return fail(HL_EINVAL, "k=%d, P=%d: the eigen-step needs %zu bytes of scratch, more than the %zu of "
                "hl_lambda_min_noalloc (use hl_lambda_min with a workspace)", dm.k, dm.P, need, kNoAllocBytes);
  int dev = 0;
  NACHK(hipGetDevice(&dev));
  char* base = (char*)noalloc_ptr(dev);
  if (!base) {
    NACHK(noalloc_init(dev));
    base = (char*)noalloc_ptr(dev);
  }
  hipStream_t st = (hipStream_t)stream;
  DevStatus* dst = (DevStatus*)base;
  void* ews = base + kNoAllocStatus;
  // the array keeps the last call's contents: clear the status word and the
  // whole work area first (a fill kernel, no memset node)
  NACHK(launch_fill((u32*)base, need / 4, 0u, st));
  NACHK(launch_eig_host(blk, dm, ews, dst, st, nullptr, ctx_eig_maxit(ctx)));
  NACHK(hipStreamSynchronize(st));
  unsigned long long v = 0;
  NACHK(hipMemcpy(&v, dst, 8, hipMemcpyDeviceToHost));
  if (v) return fail((hl_status)(v >> 32), "device status %d at index %d", (int)(v >> 32), (int)(v & 0xffffffffu));
  int64_t bexp = 0;
  NACHK(hipMemcpy(&bexp, blk_exp, 8, hipMemcpyDeviceToHost));
  return read_lambda(dm, ews, bexp, lam_mant, lam_mant_km1, out);
}
