// scratch.hip -- aln_execute_noalloc: aln_execute with the workspace taken
// from a fixed device array instead of a caller allocation, for callers that
// cannot allocate device memory.
//
// The array lives in this file's code object; each GPU the library runs on
// holds its own copy from the first aln_create on that GPU until the process
// ends.  In host code `scratch` names a host-side stand-in, not device memory,
// so its device address is looked up once per device (with that device
// current) and only that address is ever passed to kernels.
#include <mutex>

#include "runtime.h"

namespace {

static __device__ __align__(256) uint8_t scratch[ALN_NOALLOC_WORKSPACE_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};

} // namespace

// Called by aln_create with ctx->device current.
aln_status alnrt::scratch_init(aln_ctx *ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return fail(ctx, ALN_E_DEVICE, "device %d beyond the scratch table", ctx->device);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_addr[ctx->device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(ctx, ALN_E_DEVICE, "scratch address on device %d: %s", ctx->device,
                  hipGetErrorString(e));
    g_addr[ctx->device] = p;
  }
  ctx->scratch = g_addr[ctx->device];
  return ALN_OK;
}

extern "C" aln_status aln_execute_noalloc(aln_ctx *ctx, aln_plan *plan, const aln_batch *batch,
                                          aln_result *d_res, uint32_t *d_cigar,
                                          uint64_t cigar_words, void *stream) {
  if (!ctx || !plan || !batch || plan->ctx != ctx)
    return alnrt::fail(ctx, ALN_E_INVAL, "bad context or plan");
  if (!ctx->scratch) return alnrt::fail(ctx, ALN_E_DEVICE, "no scratch workspace on this device");
  if (plan->ws_bytes > ALN_NOALLOC_WORKSPACE_BYTES)
    return alnrt::fail(ctx, ALN_E_CAPACITY,
                       "plan needs %llu workspace bytes, the fixed workspace holds %llu",
                       (unsigned long long)plan->ws_bytes,
                       (unsigned long long)ALN_NOALLOC_WORKSPACE_BYTES);
  // kernel timing would create HIP events: not on this path
  if (ctx->profiling) return alnrt::fail(ctx, ALN_E_INVAL, "kernel timing is on");
  aln_status st = alnrt::exec_check(ctx, plan, batch, ctx->scratch, ALN_NOALLOC_WORKSPACE_BYTES,
                                    d_res, d_cigar, cigar_words);
  if (st != ALN_OK) return st;
  return alnrt::plan_run(ctx, plan, batch, ctx->scratch, d_res, d_cigar, (hipStream_t)stream,
                         false);
}
