// Arithmetic-rate probe for the benchmark (not part of the libsym ABI; built into its own
// libsymprobe.so): the vector FMA throughput that roofline fractions are quoted against,
// measured on the device instead of taken from the data sheet. Each thread runs kChains
// independent FMA chains of `iters` steps (no loads inside the loop), so the issue rate
// of v_fma (v_fmac) alone sets the time.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 8;
constexpr int kBlocks = 4096;
constexpr int kThreads = 256;

template <typename T>
__global__ __launch_bounds__(kThreads) void fma_probe_kernel(T* __restrict__ out, int iters, T a, T b) {
  T x[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) x[k] = T(threadIdx.x + k);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = fma(x[k], a, b);
  }
  T s = T(0);
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += x[k];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

extern "C" {

/*
 * One launch of 4096 workgroups x 256 threads, each thread running 8 independent
 * chains of `iters` fused multiply-adds (2 x 8 x iters x 4096 x 256 flop) in float
 * (prec 1) or double (prec 2). out: device buffer of 4096 x 256 elements of that type,
 * 16-byte aligned (one value per thread is written). Returns 0, -1 for a bad prec, iters
 * outside [1, 2^20] or a misaligned out, -2 for out == NULL, -4 if the launch fails.
 * The caller times the call (e.g. with events on `stream`).
 */
int probe_fma(int prec, int32_t iters, void* out, hipStream_t stream) {
  if (prec != 1 && prec != 2) return -1;
  if (out == nullptr) return -2;
  if (((uintptr_t)out & 15u) != 0 || iters < 1 || iters > (1 << 20)) return -1;
  // a, b keep every chain bounded (|a| < 1) so no value overflows
  if (prec == 1)
    fma_probe_kernel<float><<<kBlocks, kThreads, 0, stream>>>(static_cast<float*>(out), iters, 0.999f, 0.001f);
  else
    fma_probe_kernel<double><<<kBlocks, kThreads, 0, stream>>>(static_cast<double*>(out), iters, 0.999, 0.001);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // extern "C"
