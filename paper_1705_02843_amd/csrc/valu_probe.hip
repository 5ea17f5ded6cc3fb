// valu_probe.hip -- measures the integer VALU issue ceiling of the device
// the batched search is measured against: every lane of many waves runs
// independent chains of 32-bit integer adds, and the rate of wave64 VALU
// instructions per second is timed with device events.  Not part of the
// search; the benchmark uses it to state the roofline peak it divides by.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 8;   // independent dependency chains per lane
constexpr int kUnroll = 16;  // adds per chain per loop trip

// KIND 0: v_add_u32 (a two-operand add of vector registers: the simple
// integer class, add/sub/and/or/xor/right shift, which gfx950 issues at up
// to twice the base rate); KIND 1: v_bfe_u32 (a three-operand bit-field
// extract: the class of everything else the search round executes, 64-bit
// shifts and adds, multiplies, mbcnt, compares, selects, which issues at one
// wave64 instruction per compute unit per clock).
template <int KIND>
__global__ __launch_bounds__(256) void valu_kernel(uint32_t* out, int trips, uint32_t seed) {
  uint32_t v[kChains];
  for (int c = 0; c < kChains; ++c) v[c] = seed + threadIdx.x * 7u + (uint32_t)c;
  const uint32_t k = seed | 1u;
  for (int t = 0; t < trips; ++t) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) {
        if constexpr (KIND == 0) asm volatile("v_add_u32 %0, %0, %1" : "+v"(v[c]) : "v"(k));
        else asm volatile("v_bfe_u32 %0, %0, %1, 7" : "+v"(v[c]) : "v"(k));
      }
    }
  }
  uint32_t r = 0;
  for (int c = 0; c < kChains; ++c) r ^= v[c];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = r;
}

}  // namespace

// Runs `blocks` workgroups of 256 threads, `trips` loop trips each, of the
// instruction class `kind` (0 or 1, above) on the current device; returns 0
// and the measured wave64 VALU instructions per second (the timed class
// only; the loop's own counter is scalar) and the elapsed milliseconds, or a
// nonzero HIP error code.
extern "C" int bpida_valu_probe(int kind, int blocks, int trips, double* insts_per_s, double* ms_out) {
  if (blocks <= 0 || trips <= 0 || !insts_per_s || !ms_out || kind < 0 || kind > 1)
    return (int)hipErrorInvalidValue;
  void (*kern)(uint32_t*, int, uint32_t) = kind == 0 ? valu_kernel<0> : valu_kernel<1>;
  uint32_t* d = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&d, sizeof(uint32_t) * (size_t)blocks * 256);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) {
    // one untimed launch, then the timed one
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, nullptr, d, trips, 12345u);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, nullptr, d, trips, 54321u);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e == hipSuccess) {
    const double waves = (double)blocks * 4.0;
    const double insts = waves * (double)trips * kUnroll * kChains;
    *insts_per_s = insts / (ms * 1e-3);
    *ms_out = ms;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (d) (void)hipFree(d);
  return (int)e;
}
