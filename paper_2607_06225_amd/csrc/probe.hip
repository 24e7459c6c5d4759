// probe.hip -- VALU issue-rate and shader-clock probe (a measurement tool).
//
// One kernel per instruction class keeps every SIMD busy with that
// instruction only: each wave runs `iters` iterations of 32 instructions,
// spread over 8 independent register chains (or 1 chain, to time the
// latency of dependent instructions).  Each wave records how many shader
// clock cycles (s_memtime) and how many ticks of the constant 100 MHz clock
// (s_memrealtime) its loop took.  From these, aln_valu_probe reports issue
// rates (wave instructions per SIMD per cycle) and the clock under load,
// which the roofline of the alignment kernels is priced against.
#include "runtime.h"

namespace alnk {

enum ProbeOp {
  P_ADD = 0,      // v_add_u32
  P_MAX,          // v_max_i32
  P_MAX3,         // v_max3_i32
  P_CMP,          // v_cmp_gt_i32 (writes an SGPR pair)
  P_CNDMASK,      // v_cndmask_b32 (SGPR-pair condition)
  P_PK_MAX,       // v_pk_max_i16
  P_PK_ADD,       // v_pk_add_u16
  P_LSHL_OR,      // v_lshl_or_b32
  P_ADD3,         // v_add3_u32
  P_DPP_MOV,      // v_mov_b32 with DPP row_shr:1
  P_DPP_MAX,      // v_max_i32 with DPP row_shr:1 on its first source
  P_SDWA_ADD,     // v_add_u32 with SDWA sign-extended byte operand
  P_PERM,         // v_perm_b32
  P_ALIGNBYTE,    // v_alignbyte_b32
  P_BFE,          // v_bfe_u32
  P_ADDC,         // v_addc_co_u32 (carry in and out in SGPR pairs)
  P_NUM
};

template <int OP>
__device__ __forceinline__ void probe_op(uint32_t &a, uint32_t b, uint32_t c, uint64_t &s) {
  if constexpr (OP == P_ADD) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a) : "v"(b));
  if constexpr (OP == P_MAX) asm volatile("v_max_i32 %0, %0, %1" : "+v"(a) : "v"(b));
  if constexpr (OP == P_MAX3) asm volatile("v_max3_i32 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
  if constexpr (OP == P_CMP) asm volatile("v_cmp_gt_i32_e64 %0, %1, %2" : "=s"(s) : "v"(a), "v"(b));
  if constexpr (OP == P_CNDMASK)
    asm volatile("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(a) : "v"(b), "s"(s));
  if constexpr (OP == P_PK_MAX) asm volatile("v_pk_max_i16 %0, %0, %1" : "+v"(a) : "v"(b));
  if constexpr (OP == P_PK_ADD) asm volatile("v_pk_add_u16 %0, %0, %1" : "+v"(a) : "v"(b));
  if constexpr (OP == P_LSHL_OR) asm volatile("v_lshl_or_b32 %0, %0, 6, %1" : "+v"(a) : "v"(b));
  if constexpr (OP == P_ADD3) asm volatile("v_add3_u32 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
  if constexpr (OP == P_DPP_MOV)
    asm volatile("v_mov_b32_dpp %0, %0 row_shr:1 row_mask:0xf bank_mask:0xf" : "+v"(a));
  if constexpr (OP == P_DPP_MAX)
    asm volatile("v_max_i32_dpp %0, %0, %1 row_shr:1 row_mask:0xf bank_mask:0xf" : "+v"(a) : "v"(b));
  if constexpr (OP == P_SDWA_ADD)
    asm volatile("v_add_u32_sdwa %0, %0, sext(%1) dst_sel:DWORD dst_unused:UNUSED_PAD "
                 "src0_sel:DWORD src1_sel:BYTE_1"
                 : "+v"(a)
                 : "v"(b));
  if constexpr (OP == P_PERM) asm volatile("v_perm_b32 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
  if constexpr (OP == P_ALIGNBYTE)
    asm volatile("v_alignbyte_b32 %0, %0, %1, 3" : "+v"(a) : "v"(b));
  if constexpr (OP == P_BFE) asm volatile("v_bfe_u32 %0, %0, 3, 8" : "+v"(a));
  if constexpr (OP == P_ADDC)
    asm volatile("v_addc_co_u32_e64 %0, %1, %0, %0, %1" : "+v"(a), "+s"(s));
}

// out[2*wave] = shader cycles of the loop, out[2*wave+1] = 100 MHz ticks
template <int OP, int CHAINS>
__global__ __launch_bounds__(256) void valu_probe_kernel(uint64_t *out, int iters, uint32_t seed) {
  uint32_t a[8], s0 = seed ^ threadIdx.x;
  uint64_t sg[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    a[c] = s0 * (2 * c + 1);
    sg[c] = 0x5555555555555555ull << (c & 1);
  }
  const uint32_t b = s0 | 1u, cc = s0 >> 3;
  const uint64_t t0 = __builtin_readcyclecounter();
  const uint64_t r0 = __builtin_amdgcn_s_memrealtime();
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 32 / CHAINS; ++u) {
#pragma unroll
      for (int c = 0; c < CHAINS; ++c) probe_op<OP>(a[c], b, cc, sg[c]);
    }
  }
  const uint64_t t1 = __builtin_readcyclecounter();
  const uint64_t r1 = __builtin_amdgcn_s_memrealtime();
  uint32_t sink = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) sink ^= a[c] ^ (uint32_t)sg[c];
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if ((threadIdx.x & 63) == 0) {
    out[2 * wave] = (t1 - t0) + (sink == 0x9e3779b9u ? 1 : 0);
    out[2 * wave + 1] = r1 - r0;
  }
}

template <int OP>
static hipError_t launch_probe_op(bool dep, int blocks, uint64_t *out, int iters, hipStream_t s) {
  if (dep)
    hipLaunchKernelGGL((valu_probe_kernel<OP, 1>), dim3(blocks), dim3(256), 0, s, out, iters, 12345u);
  else
    hipLaunchKernelGGL((valu_probe_kernel<OP, 8>), dim3(blocks), dim3(256), 0, s, out, iters, 12345u);
  return hipGetLastError();
}

template <int OP = 0>
static hipError_t launch_probe(int op, bool dep, int blocks, uint64_t *out, int iters, hipStream_t s) {
  if constexpr (OP >= P_NUM) {
    return hipErrorInvalidValue;
  } else {
    if (op == OP) return launch_probe_op<OP>(dep, blocks, out, iters, s);
    return launch_probe<OP + 1>(op, dep, blocks, out, iters, s);
  }
}

} // namespace alnk

extern "C" aln_status aln_valu_probe(aln_ctx *ctx, int32_t op, int32_t dependent,
                                     int32_t waves_per_simd, int32_t iters, double *out) {
  if (!ctx || !out || op < 0 || op >= alnk::P_NUM || waves_per_simd < 1 || waves_per_simd > 8 ||
      iters < 1)
    return alnrt::fail(ctx, ALN_E_INVAL, "bad probe arguments");
  if (hipSetDevice(ctx->device) != hipSuccess) return alnrt::fail(ctx, ALN_E_DEVICE, "set device");
  const int blocks = ctx->cus * waves_per_simd; // four waves per block, one per SIMD
  const int waves = blocks * 4;
  uint64_t *d = nullptr;
  if (hipMalloc(&d, sizeof(uint64_t) * 2 * (size_t)waves) != hipSuccess)
    return alnrt::fail(ctx, ALN_E_NOMEM, "probe buffer");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  aln_status st = ALN_OK;
  std::vector<uint64_t> h((size_t)2 * waves);
  float ms = 0.f;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
      alnk::launch_probe(op, dependent != 0, blocks, d, 1, nullptr) != hipSuccess || // warm-up
      hipEventRecord(e0, nullptr) != hipSuccess ||
      alnk::launch_probe(op, dependent != 0, blocks, d, iters, nullptr) != hipSuccess ||
      hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
      hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
      hipMemcpy(h.data(), d, sizeof(uint64_t) * h.size(), hipMemcpyDeviceToHost) != hipSuccess)
    st = alnrt::fail(ctx, ALN_E_DEVICE, "probe launch failed");
  double cyc = 0, ticks = 0;
  for (int w = 0; w < waves; ++w) {
    cyc += (double)h[2 * w];
    ticks += (double)h[2 * w + 1];
  }
  out[0] = ms;                        // wall time of the launch
  out[1] = cyc / waves;               // mean shader cycles per wave loop
  out[2] = ticks / waves;             // mean 100 MHz ticks per wave loop
  out[3] = (double)waves;
  out[4] = 32.0 * (double)iters;      // wave instructions per wave
  out[5] = (double)ctx->cus * 4;      // SIMDs
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(d);
  return st;
}
