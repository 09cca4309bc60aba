// fsc_cluster_noalloc: fsc_cluster on a fixed device scratch array instead of
// the context's workspace, for callers that cannot allocate device memory
// (graph capture, tight serving loops).  The array lives in this file; its
// device address is looked up once per device when a context is created.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>

#include "fsc_internal.hpp"

namespace fsc {

constexpr size_t kScratchBytes = size_t(64) << 20;  // FSC_NOALLOC_MAX_BYTES
constexpr int kMaxDevices = 64;

static_assert(kScratchBytes == FSC_NOALLOC_MAX_BYTES, "scratch size and its public constant differ");

// Each GPU the library runs on holds its own copy until the process ends.
static __device__ __align__(256) char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static char* g_scratch_ptr[kMaxDevices] = {};

// Resolves this device's address of `scratch`; `device` must be current.
int noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(FSC_E_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return FSC_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return fail(FSC_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  }
  g_scratch_ptr[device] = static_cast<char*>(p);
  return FSC_OK;
}

int cluster_noalloc_run(Context* ctx, const fsc_csr* g, int k, int l, int t, uint64_t seed, const fsc_opts& o,
                        int32_t* labels, void* emb, float* centres, hipStream_t s) {
  char* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (ctx->device >= 0 && ctx->device < kMaxDevices) base = g_scratch_ptr[ctx->device];
  }
  int rc;
  if (!base) {  // the context's creation could not resolve it: try once more
    if ((rc = noalloc_setup(ctx->device))) return rc;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    base = g_scratch_ptr[ctx->device];
  }
  const size_t need = cluster_workspace_bytes(ctx, g, l, o);
  if (need > kScratchBytes)
    return fail(FSC_E_NOMEM, "fsc_cluster_noalloc: this graph needs " + std::to_string(need) +
                                 " bytes of workspace, more than the " + std::to_string(kScratchBytes) +
                                 " bytes of the no-allocation scratch array (use fsc_cluster)");
  Arena a;
  a.base = base;
  a.size = kScratchBytes;
  a.used = 0;
  // timing events may be created on first use: none in this entry point
  const bool timing = ctx->timing;
  ctx->timing = false;
  rc = cluster_run(ctx, g, k, l, t, seed, o, labels, emb, centres, s, &a);
  ctx->timing = timing;
  return rc;
}

}  // namespace fsc
