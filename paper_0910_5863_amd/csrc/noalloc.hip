// bddc_apply_noalloc: the preconditioner application of bddc_apply without
// any device allocation.  Its work vectors (local stacks, coarse vector,
// front updates of the interior solves, triangular-solve counters) are laid
// out in one static device array instead of the context's buffers; the
// kernels are bddc_apply's own.
//
// The array is a file-scope __device__ object: every device the library runs
// on holds its own copy, from the module's load until the process ends.  Host
// code never passes the array's name to a kernel (in host code it only stands
// for the symbol): on the first call on a device, with that device current,
// hipGetSymbolAddress gives the device address, which is kept per device and
// is the only address used afterwards.  All calls on one device share the
// array, so calls that overlap on one device race; each call clears the part
// it uses with a fill kernel before its first launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "ctx.h"

using namespace bddc;

namespace {

constexpr size_t kNoallocScratchBytes = size_t(64) << 20;  // 64 MiB per device

__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;  // device address of `scratch`, per device ordinal

// device address of the static array on `dev` (the current device)
void *scratch_address(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) throw DeviceError("hipGetSymbolAddress(scratch) returned a null address");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

__global__ void clear_words_kernel(uint64_t *p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

}  // namespace

extern "C" {

bddc_status bddc_apply_noalloc(bddc_ctx *c, int nrhs, const double *r, int64_t ldr, double *z,
                               int64_t ldz) {
  if (!c) return BDDC_ERR_ARG;
  if (c->state < 2) return fail(c, BDDC_ERR_STATE, "bddc_apply_noalloc before bddc_factor");
  if (nrhs < 0 || (nrhs > 0 && (!r || !z))) return fail(c, BDDC_ERR_ARG, "bad vectors");
  if (ldr < c->P.n_glob || ldz < c->P.n_glob) return fail(c, BDDC_ERR_ARG, "leading dimension < n_glob");
  return guarded(c, [&] {
    check_hip(hipSetDevice(c->opt.device), "hipSetDevice");
    const size_t need = c->S->work_bytes();
    if (need > kNoallocScratchBytes)
      throw ArgError("bddc_apply_noalloc: this problem's work vectors need " + std::to_string(need) +
                     " bytes; the static work array holds " +
                     std::to_string(kNoallocScratchBytes) + " (use bddc_apply)");
    void *base = scratch_address(c->opt.device);
    const ApplyWork w = c->S->carve_work(base);
    const size_t words = (need + 7) / 8;
    for (int q = 0; q < nrhs; ++q) {
      clear_words_kernel<<<(unsigned)std::min<size_t>((words + 255) / 256, 4096), 256, 0, c->stream>>>(
          (uint64_t *)base, words);
      check_hip(hipGetLastError(), "clear_words_kernel");
      c->S->apply_global(r + q * ldr, z + q * ldz, w);
    }
  });
}

}  // extern "C"
