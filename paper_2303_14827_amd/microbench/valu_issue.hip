// valu_issue.hip -- issue cost of the VALU instruction forms the marchers use, on gfx950.
//
// Each kernel runs a fixed-count loop whose body is one inline-asm block of 8 instructions
// of one form (optionally interleaved with 8 independent v_fmac_f32), with 4 waves per SIMD
// (4 blocks of 256 threads per CU). Every wave records the 100 MHz constant clock at the
// start and end of its loop; the span over all waves gives the time per instruction per
// SIMD. A second set runs one wave per SIMD over a single dependent chain to give latency.
// Registers only: the one store per wave goes to its own slot of `out`. The control-flow
// forms restore exec inside their own block and branch only to the next instruction.
//
// Build and run:  hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
//                   -o valu_issue valu_issue.hip && ./valu_issue
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <vector>

#define ITERS 4096

#define R8(I) I(0) I(1) I(2) I(3) I(4) I(5) I(6) I(7)
// operands: %0..%7 = a0..a7 (state), %8 = x, %9 = y, %10..%13 = b0..b3 (scratch)
#define FMAC_VV(i) "v_fmac_f32 %" #i ", %8, %9\n\t"
#define FMA_VVV(i) "v_fma_f32 %" #i ", %8, %9, %" #i "\n\t"
#define FMA_VVS(i) "v_fma_f32 %" #i ", %8, %" #i ", s98\n\t"
#define FMAC_SV(i) "v_fmac_f32 %" #i ", s98, %9\n\t"
#define FMAC_LIT(i) "v_fmac_f32 %" #i ", 0x3f800001, %9\n\t"
#define ADD_SV(i) "v_add_f32 %" #i ", s98, %" #i "\n\t"
#define PK_FMA(i) "v_pk_fma_f16 %" #i ", %" #i ", %8, %9\n\t"
#define PK_FMAC(i) "v_pk_fmac_f16 %" #i ", %8, %9\n\t"
#define PK_ADD(i) "v_pk_add_f16 %" #i ", %" #i ", %8\n\t"
#define DOT2C(i) "v_dot2c_f32_f16 %" #i ", %8, %9\n\t"
#define MOV_VV "v_mov_b32 %10, %11\n\tv_mov_b32 %11, %12\n\tv_mov_b32 %12, %13\n\tv_mov_b32 %13, %10\n\t"
#define MOV_SV "v_mov_b32 %10, s98\n\tv_mov_b32 %11, s99\n\tv_mov_b32 %12, s98\n\tv_mov_b32 %13, s99\n\t"
#define CMP_VV "v_cmp_gt_f32 vcc, %10, %11\n\tv_cmp_gt_f32 vcc, %11, %12\n\tv_cmp_gt_f32 vcc, %12, %13\n\tv_cmp_gt_f32 vcc, %13, %10\n\t"
#define CND_V "v_cndmask_b32 %10, %10, %11, vcc\n\tv_cndmask_b32 %11, %11, %12, vcc\n\tv_cndmask_b32 %12, %12, %13, vcc\n\tv_cndmask_b32 %13, %13, %10, vcc\n\t"
#define SDWA4 "v_min_f16_sdwa %10, %10, %11 dst_sel:WORD_0 dst_unused:UNUSED_PAD src0_sel:WORD_0 src1_sel:WORD_1\n\t" \
              "v_min_f16_sdwa %11, %11, %12 dst_sel:WORD_0 dst_unused:UNUSED_PAD src0_sel:WORD_0 src1_sel:WORD_1\n\t" \
              "v_min_f16_sdwa %12, %12, %13 dst_sel:WORD_0 dst_unused:UNUSED_PAD src0_sel:WORD_0 src1_sel:WORD_1\n\t" \
              "v_min_f16_sdwa %13, %13, %10 dst_sel:WORD_0 dst_unused:UNUSED_PAD src0_sel:WORD_0 src1_sel:WORD_1\n\t"
#define MIX4 "v_fma_mixlo_f16 %10, %0, %8, %9\n\tv_fma_mixhi_f16 %10, %1, %8, %9\n\t" \
             "v_fma_mixlo_f16 %11, %2, %8, %9\n\tv_fma_mixhi_f16 %11, %3, %8, %9\n\t"
#define LOG4 "v_log_f32 %10, %10\n\tv_log_f32 %11, %11\n\tv_log_f32 %12, %12\n\tv_log_f32 %13, %13\n\t"
#define EXP4 "v_exp_f32 %10, %10\n\tv_exp_f32 %11, %11\n\tv_exp_f32 %12, %12\n\tv_exp_f32 %13, %13\n\t"
#define RSQ4 "v_rsq_f32 %10, %10\n\tv_rsq_f32 %11, %11\n\tv_rsq_f32 %12, %12\n\tv_rsq_f32 %13, %13\n\t"
// a uniform conditional branch (never taken) and an exec-masked region around nothing:
// the cost of the control flow the state machines compile to
#define BR1 "s_cmp_eq_u32 s98, s99\n\ts_cbranch_scc1 1f\n1:\n\t"
// (EXEC0: the compare is false on every lane, so the region is skipped by a taken branch;
// EXEC1: true on every lane, branch not taken)
#define EXEC0 "v_cmp_gt_f32 vcc, %10, %11\n\ts_and_saveexec_b64 s[98:99], vcc\n\t" \
              "s_cbranch_execz 1f\n1:\n\ts_or_b64 exec, exec, s[98:99]\n\t"
#define EXEC1 "v_cmp_gt_f32 vcc, %8, %9\n\ts_and_saveexec_b64 s[98:99], vcc\n\t" \
              "s_cbranch_execz 1f\n1:\n\ts_or_b64 exec, exec, s[98:99]\n\t"
#define MOV64_4 "v_mov_b64 v[100:101], s[98:99]\n\tv_mov_b64 v[102:103], s[98:99]\n\t" \
                "v_mov_b64 v[100:101], s[98:99]\n\tv_mov_b64 v[102:103], s[98:99]\n\t"

#define KERNEL(NAME, BODY)                                                                       \
  __global__ void NAME(unsigned long long *out, float xf, float yf) {                           \
    float a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5,     \
          a6 = a0 + 6, a7 = a0 + 7, x = xf, y = yf, b0 = 1, b1 = 2, b2 = 3, b3 = 4;              \
    unsigned long long r0, r1;                                                                   \
    asm volatile("s_memrealtime %0\n\ts_waitcnt lgkmcnt(0)" : "=s"(r0));                       \
    for (int it = 0; it < ITERS; ++it) {                                                         \
      asm volatile(BODY : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6),  \
                   "+v"(a7), "+v"(x), "+v"(y), "+v"(b0), "+v"(b1), "+v"(b2), "+v"(b3)            \
                   :                                                                             \
                   : "vcc", "scc", "s98", "s99", "v100", "v101", "v102", "v103");                     \
    }                                                                                            \
    asm volatile("s_memrealtime %0\n\ts_waitcnt lgkmcnt(0)" : "=s"(r1) : "v"(a0), "v"(a7), "v"(b0)); \
    const int w = (blockIdx.x * blockDim.x + threadIdx.x) / 64;                                  \
    if ((threadIdx.x & 63) == 0) {                                                               \
      out[2 * w] = r0;                                                                           \
      out[2 * w + 1] = r1;                                                                       \
    }                                                                                            \
  }

KERNEL(k_fmac_vv, R8(FMAC_VV))
KERNEL(k_fma_vvv, R8(FMA_VVV))
KERNEL(k_fma_vvs, R8(FMA_VVS))
KERNEL(k_fmac_sv, R8(FMAC_SV))
KERNEL(k_fmac_lit, R8(FMAC_LIT))
KERNEL(k_add_sv, R8(ADD_SV))
KERNEL(k_pk_fma, R8(PK_FMA))
KERNEL(k_pk_fmac, R8(PK_FMAC))
KERNEL(k_pk_add, R8(PK_ADD))
KERNEL(k_dot2c, R8(DOT2C))
KERNEL(k_fmac_mov_vv, R8(FMAC_VV) MOV_VV MOV_VV)
KERNEL(k_fmac_mov_sv, R8(FMAC_VV) MOV_SV MOV_SV)
KERNEL(k_fmac_cmp, R8(FMAC_VV) CMP_VV CMP_VV)
KERNEL(k_fmac_cnd, R8(FMAC_VV) CND_V CND_V)
KERNEL(k_fmac_sdwa, R8(FMAC_VV) SDWA4 SDWA4)
KERNEL(k_fmac_mix, R8(FMAC_VV) MIX4 MIX4)
KERNEL(k_fmac_mov64, R8(FMAC_VV) MOV64_4 MOV64_4)
KERNEL(k_fmac_log, R8(FMAC_VV) LOG4 LOG4)
KERNEL(k_fmac_exp, R8(FMAC_VV) EXP4 EXP4)
KERNEL(k_fmac_rsq, R8(FMAC_VV) RSQ4 RSQ4)
KERNEL(k_fmac_br, R8(FMAC_VV) BR1 BR1 BR1 BR1 BR1 BR1 BR1 BR1)
KERNEL(k_fmac_exec0, R8(FMAC_VV) EXEC0 EXEC0 EXEC0 EXEC0 EXEC0 EXEC0 EXEC0 EXEC0)
KERNEL(k_fmac_exec1, R8(FMAC_VV) EXEC1 EXEC1 EXEC1 EXEC1 EXEC1 EXEC1 EXEC1 EXEC1)

// One dependent chain per wave, one wave per SIMD: latency of dependent FP32 FMA and packed FP16 FMA.
#define CHAIN_F32 "v_fmac_f32 %0, %8, %9\n\t"
#define CHAIN_F16 "v_pk_fma_f16 %0, %0, %8, %9\n\t"
KERNEL(k_chain_f32, CHAIN_F32 CHAIN_F32 CHAIN_F32 CHAIN_F32 CHAIN_F32 CHAIN_F32 CHAIN_F32 CHAIN_F32)
KERNEL(k_chain_f16, CHAIN_F16 "s_nop 1\n\t" CHAIN_F16 "s_nop 1\n\t" CHAIN_F16 "s_nop 1\n\t" CHAIN_F16 "s_nop 1\n\t"
                    CHAIN_F16 "s_nop 1\n\t" CHAIN_F16 "s_nop 1\n\t" CHAIN_F16 "s_nop 1\n\t" CHAIN_F16 "s_nop 1\n\t")

typedef void (*Kern)(unsigned long long *, float, float);

static double span_ns(Kern k, int blocks_per_cu, int threads, int cus, unsigned long long *d) {
  const int blocks = cus * blocks_per_cu, waves = blocks * threads / 64;
  for (int rep = 0; rep < 2; ++rep)
    hipLaunchKernelGGL(k, dim3(blocks), dim3(threads), 0, 0, d, 0.999f, 0.001f);
  if (hipDeviceSynchronize() != hipSuccess) return -1;
  std::vector<unsigned long long> h(2 * waves);
  if (hipMemcpy(h.data(), d, 16 * (size_t)waves, hipMemcpyDeviceToHost) != hipSuccess) return -1;
  unsigned long long t0 = ~0ull, t1 = 0;
  for (int w = 0; w < waves; ++w) {
    t0 = std::min(t0, h[2 * w]);
    t1 = std::max(t1, h[2 * w + 1]);
  }
  return (t1 - t0) * 10.0;   // 100 MHz ticks
}

int main() {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, 0) != hipSuccess) return 1;
  const int cus = p.multiProcessorCount;
  unsigned long long *d = nullptr;
  if (hipMalloc(&d, sizeof(unsigned long long) * 2 * cus * 16) != hipSuccess) return 1;
  const double ghz = p.clockRate / 1e6;
  printf("device %s, %d CUs, clock %.2f GHz (cycles below use this clock)\n", p.gcnArchName, cus, ghz);
  struct T { const char *name; Kern k; int n_form; bool with_fmac; };
  const T tests[] = {
      {"v_fmac_f32 (VGPR operands)", k_fmac_vv, 8, false},
      {"v_fma_f32 (3 VGPR operands)", k_fma_vvv, 8, false},
      {"v_fma_f32 (one SGPR operand)", k_fma_vvs, 8, false},
      {"v_fmac_f32 (SGPR src0)", k_fmac_sv, 8, false},
      {"v_fmac_f32 (literal)", k_fmac_lit, 8, false},
      {"v_add_f32 (SGPR src0)", k_add_sv, 8, false},
      {"v_pk_fma_f16", k_pk_fma, 8, false},
      {"v_pk_fmac_f16", k_pk_fmac, 8, false},
      {"v_pk_add_f16", k_pk_add, 8, false},
      {"v_dot2c_f32_f16", k_dot2c, 8, false},
      {"v_mov_b32 (VGPR)", k_fmac_mov_vv, 8, true},
      {"v_mov_b32 (from SGPR)", k_fmac_mov_sv, 8, true},
      {"v_cmp_gt_f32 (to vcc)", k_fmac_cmp, 8, true},
      {"v_cndmask_b32", k_fmac_cnd, 8, true},
      {"v_min_f16_sdwa", k_fmac_sdwa, 8, true},
      {"v_fma_mix{lo,hi}_f16", k_fmac_mix, 8, true},
      {"v_mov_b64 (from SGPR pair)", k_fmac_mov64, 8, true},
      {"v_log_f32", k_fmac_log, 8, true},
      {"v_exp_f32", k_fmac_exp, 8, true},
      {"v_rsq_f32", k_fmac_rsq, 8, true},
      {"s_cmp + s_cbranch_scc1 (not taken)", k_fmac_br, 8, true},
      {"masked region, skipped (branch taken)", k_fmac_exec0, 8, true},
      {"masked region, entered (not taken)", k_fmac_exec1, 8, true},
  };
  // 4 waves per SIMD: 4 blocks of 256 threads per CU
  const double base = span_ns(k_fmac_vv, 4, 256, cus, d) / (4.0 * ITERS * 8);
  printf("%-34s %12s\n", "form", "clk/instr/SIMD");
  for (const T &t : tests) {
    const double ns = span_ns(t.k, 4, 256, cus, d);
    if (ns < 0) return 1;
    const double total = 4.0 * ITERS * (t.n_form + (t.with_fmac ? 8 : 0));
    double per = ns / total;
    if (t.with_fmac) per = (ns - base * 4.0 * ITERS * 8) / (4.0 * ITERS * t.n_form);   // subtract the FMAs
    printf("%-34s %12.2f%s\n", t.name, per * ghz, t.with_fmac ? "   (interleaved with v_fmac_f32)" : "");
  }
  // latency: one wave per SIMD (1 block of 256 threads per CU), one chain
  const double l32 = span_ns(k_chain_f32, 1, 256, cus, d) / (ITERS * 8.0);
  const double l16 = span_ns(k_chain_f16, 1, 256, cus, d) / (ITERS * 8.0);
  printf("dependent v_fmac_f32 chain, 1 wave/SIMD:   %.2f clk per instruction\n", l32 * ghz);
  printf("dependent v_pk_fma_f16 chain (+s_nop 1):   %.2f clk per instruction\n", l16 * ghz);
  printf("status %s\n", hipGetErrorString(hipDeviceSynchronize()));
  return 0;
}
