// valu_probe.hip -- issue-rate probes for the integer VALU roof of the sweep
// kernels on gfx950.  Not part of the method: bench.py (--form probe) times
// these loops to measure, on the running part, how fast the instruction mix
// the sweep kernels are built from issues when nothing else limits it.
//
// Each thread runs kChains independent dependency chains (so that a wave
// always has an instruction ready), kIters iterations each, and writes one
// word per thread so that nothing is optimised away.  Instructions per chain
// iteration, by kind:
//   0  v_mad_u64_u32 + v_bitop3_b32 (xor3): the Philox round pair     2
//   1  v_bitop3_b32 alone                                             1
//   2  v_add_u32 alone (the plainest full-rate operation)             1
//   3  one Philox4x32-10 block (scalar key words), 4 words per block  37 + 4
//      (37 for the block and one compare per word, as in the kernels)
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 8;

__device__ __forceinline__ uint32_t x3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// The three single-instruction probes are written in inline assembly so that
// each chain iteration is exactly the instructions named above (the compiler
// would otherwise fold or rearrange them); none of them touches memory.
__global__ void k_mad_xor(uint32_t *out, uint32_t iters, uint32_t k) {
  uint64_t p[kChains];
  uint32_t a[kChains];
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    a[c] = t * 2654435761u + c;
    p[c] = ((uint64_t)(t ^ (c * 40503u)) << 32) | c;
  }
  const uint32_t M = 0xD2511F53u;
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      uint64_t carry;
      asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(p[c]), "=s"(carry) : "v"(a[c]), "s"(M));
      asm volatile("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96"
                   : "=v"(a[c]) : "v"((uint32_t)p[c]), "v"((uint32_t)(p[c] >> 32)), "s"(k));
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s ^= a[c] + (uint32_t)p[c];
  out[t] = s;
}

__global__ void k_xor3(uint32_t *out, uint32_t iters, uint32_t k) {
  uint32_t a[kChains], b[kChains];
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    a[c] = t * 2654435761u + c;
    b[c] = t ^ (c * 40503u);
  }
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c)
      asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(a[c]) : "v"(b[c]), "s"(k));
  }
  uint32_t s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s ^= a[c];
  out[t] = s;
}

__global__ void k_add(uint32_t *out, uint32_t iters, uint32_t k) {
  uint32_t a[kChains], b[kChains];
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    a[c] = t * 2654435761u + c;
    b[c] = t ^ (c * 40503u) ^ k;
  }
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[c]) : "v"(b[c]));
  }
  uint32_t s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s ^= a[c];
  out[t] = s;
}

// Philox4x32-10 blocks whose counter word 0 varies per lane and iteration
// while words 1-3 and the key are uniform, as in the sweep kernels (group,
// sweep, slot, colour); each word is compared with a threshold and the
// outcomes counted.
__global__ void k_philox(uint32_t *out, uint32_t iters, uint32_t k) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t n = 0;
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      uint32_t c0 = (t * 2654435761u) ^ (c ? 0x6A09E667u : 0u) ^ (i << 12), c1 = i, c2 = k,
               c3 = 1u << 8, k0 = k, k1 = k ^ 0x5A5A5A5Au;
#pragma unroll
      for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = x3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = x3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
      }
      n += (c0 <= 0x80000000u) + (c1 <= 0x80000000u) + (c2 <= 0x80000000u) + (c3 <= 0x80000000u);
    }
  }
  out[t] = n;
}

}  // namespace

extern "C" {

// Run probe `kind` (0..3, see above) with blocks x threads threads and iters
// iterations on `stream`; out must hold blocks * threads uint32 words (device).
// *ms receives the kernel time from HIP events.  Returns a hipError_t value.
int ptprobe_run(int kind, uint32_t blocks, uint32_t threads, uint32_t iters, void *out,
                size_t out_words, void *stream, float *ms) {
  if (kind < 0 || kind > 3 || !out || !ms || threads == 0 || threads > 1024 || threads % 64 ||
      (size_t)blocks * threads > out_words)
    return (int)hipErrorInvalidValue;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t a, b;
  hipError_t e = hipEventCreate(&a);
  if (e != hipSuccess) return (int)e;
  if ((e = hipEventCreate(&b)) != hipSuccess) {
    (void)hipEventDestroy(a);
    return (int)e;
  }
  uint32_t *o = (uint32_t *)out;
  e = hipEventRecord(a, s);
  if (e == hipSuccess) {
    if (kind == 0) hipLaunchKernelGGL(k_mad_xor, dim3(blocks), dim3(threads), 0, s, o, iters, 12345u);
    else if (kind == 1) hipLaunchKernelGGL(k_xor3, dim3(blocks), dim3(threads), 0, s, o, iters, 12345u);
    else if (kind == 2) hipLaunchKernelGGL(k_add, dim3(blocks), dim3(threads), 0, s, o, iters, 12345u);
    else hipLaunchKernelGGL(k_philox, dim3(blocks), dim3(threads), 0, s, o, iters, 12345u);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(b, s);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return (int)e;
}

}  // extern "C"
