// Allocation-free rotation: the key switch's workspace is a fixed device array of this
// library instead of a caller buffer, for callers that cannot allocate device memory.
#include <algorithm>
#include <cstdio>
#include <mutex>
#include <string>

#include "ctx.h"
#include "ops.h"

namespace {

// One rotation of one ciphertext at N = 2^16 with 24 ciphertext limbs and 7 special primes
// needs 310 rows of N words (155 MiB); batches are rotated in chunks that fit.
constexpr size_t kScratchBytes = (size_t)HEQG_SCRATCH_MIB << 20;
constexpr int kMaxDevices = 64;

// Each device holds its own copy once the code object is loaded there, until the process
// ends.  Host code never passes `scratch` itself (on the host it only names the symbol):
// it uses the address hipGetSymbolAddress returns for the current device.
__device__ __align__(256) uint64_t scratch[kScratchBytes / 8];

std::mutex g_mu;
uint64_t* g_scratch[kMaxDevices];

int scratch_of_current_device(uint64_t** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    set_err(std::string("rotate_noalloc: no current HIP device (") + hipGetErrorString(e) + ")");
    return HEQG_ERR_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_err(std::string("rotate_noalloc: hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
      return HEQG_ERR_DEVICE;
    }
    g_scratch[dev] = static_cast<uint64_t*>(p);
  }
  *out = g_scratch[dev];
  return HEQG_OK;
}

}  // namespace

// Set-up, from heqg_ctx_create on the context's device: looks the array up there (which also
// loads the code object holding it), so that the entry point's first call allocates nothing.
// A failure is not reported here; the entry point repeats the lookup and reports it.
void noalloc_setup_current_device() {
  uint64_t* p = nullptr;
  (void)scratch_of_current_device(&p);
}

extern "C" int heqg_rotate_noalloc(heqg_ctx* c, const heqg_keys* k, const heqg_ct_batch* in, int step,
                                   heqg_ct_batch* out, hipStream_t s) {
  if (!c || !k || !in || !out) {
    set_err("rotate_noalloc: null argument");
    return HEQG_ERR_ARG;
  }
  const int64_t words = 2 * (int64_t)(in->level + 1) * c->g.N;
  if (in->count < 1 || in->level < 0 || in->level >= c->g.n_q || out->count != in->count ||
      (in->count > 1 && (in->stride < words || out->stride < words))) {
    set_err("rotate_noalloc: bad ciphertext batch");
    return HEQG_ERR_ARG;
  }
  const size_t per_ct = 8 * ops::rot_ws_words(c, 1, in->level);
  if (per_ct > kScratchBytes) {
    char msg[200];
    std::snprintf(msg, sizeof msg,
                  "rotate_noalloc: one ciphertext at level %d needs %zu bytes of scratch, more than the %zu the "
                  "library holds",
                  in->level, per_ct, kScratchBytes);
    set_err(msg);
    return HEQG_ERR_UNSUPPORTED;
  }
  uint64_t* ws = nullptr;
  int rc = scratch_of_current_device(&ws);
  if (rc) return rc;
  // chunks of whole ciphertexts; each is checked by heqg_rotate before anything is enqueued, and
  // every chunk has the first one's shape, so an argument error leaves the output untouched
  const int64_t per = (int64_t)(kScratchBytes / per_ct);
  for (int64_t i0 = 0; i0 < in->count; i0 += per) {
    const int64_t n = std::min(per, in->count - i0);
    heqg_ct_batch a = *in, o = *out;
    a.data = in->data + i0 * in->stride;
    o.data = out->data + i0 * out->stride;
    a.count = o.count = n;
    rc = heqg_rotate(c, k, &a, step, &o, ws, kScratchBytes, s);
    if (rc) return rc;
    out->scale = o.scale;
  }
  return HEQG_OK;
}
