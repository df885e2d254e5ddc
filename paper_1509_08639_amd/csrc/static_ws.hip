// Allocation-free form of the device entry point: ym_mine_device_static.
//
// Its workspace is a file-scope device array rather than a caller buffer, so
// a call makes no device or pinned-host allocation at all (the score table and
// the plan staging buffer are set up by ym_create).  Each device holds its own
// copy of the array at its own address, looked up once per device with that
// device current; host code only ever passes that looked-up address on.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/ymine.h"
#include "ym_internal.h"
#include "ym_runtime.h"

using namespace ym;

namespace {

constexpr size_t kScratchBytes = (size_t)YM_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};  // device address of `scratch` on each device (nullptr: not looked up)

void *scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  return device >= 0 && device < kMaxDevices ? g_scratch[device] : nullptr;
}

}  // namespace

namespace ym {

ym_status static_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(YM_EINVAL, "device %d: static scratch supports devices 0..%d", device, kMaxDevices - 1);
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return YM_OK;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return e != hipSuccess ? hip_fail(e, "hipGetSymbolAddress(scratch)")
                           : fail(YM_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
  }
  g_scratch[device] = p;
  return YM_OK;
}

}  // namespace ym

extern "C" {

ym_status ym_mine_device_static(ym_ctx *c, const ym_lexicon *L, const ym_device_batch *b, const ym_params *prm,
                                const ym_device_out *out, void *stream) {
  if (!c || !b) return fail(YM_EINVAL, "NULL argument");
  if (b->n_pairs < 0) return fail(YM_EINVAL, "n_pairs < 0");
  if (b->n_src_tok < 0 || b->n_tgt_tok < 0) return fail(YM_EINVAL, "negative token count");
  ym_status s;
  if ((s = check_doc_off(b->src_doc_off, b->n_pairs, "src_doc_off"))) return s;
  if ((s = check_doc_off(b->tgt_doc_off, b->n_pairs, "tgt_doc_off"))) return s;
  const size_t need = ym_mine_device_workspace_min(b->src_doc_off, b->tgt_doc_off, b->n_pairs, b->n_src_tok);
  if (need > kScratchBytes)
    return fail(YM_ENOMEM, "batch needs %zu bytes of workspace (token translations and its largest pair); the static "
                "scratch holds %zu", need, kScratchBytes);
  hipSetDevice(c->device);
  void *ws = scratch_of(c->device);
  if (!ws) return fail(YM_EDEVICE, "static scratch of device %d was not set up", c->device);
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->stage.buf.cap < kStagingBytes) return fail(YM_EDEVICE, "plan staging buffer was not set up");
  return mine_device(c, L, b, prm, ws, kScratchBytes, out, stream, c->stage.buf.cap);
}

}  // extern "C"
