// Arithmetic-rate probe: the vector FMA throughput the roofline fractions are quoted
// against, measured on the device instead of taken from the data sheet. Each thread
// runs kChains independent FMA chains of `iters` steps (no loads inside the loop), so
// the issue rate of v_fma (v_fmac) alone sets the time.
#include "kernels.hpp"

namespace sym {
namespace {

constexpr int kChains = 8;

template <typename T>
__global__ __launch_bounds__(256) void fma_probe_kernel(T* __restrict__ out, int iters, T a, T b) {
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

template <typename T>
hipError_t launch_fma_probe(T* out, int iters, hipStream_t s) {
  // a, b keep every chain bounded (|a| < 1) so no value overflows
  fma_probe_kernel<T><<<kProbeBlocks, 256, 0, s>>>(out, iters, T(0.999), T(0.001));
  return hipGetLastError();
}

template hipError_t launch_fma_probe<float>(float*, int, hipStream_t);
template hipError_t launch_fma_probe<double>(double*, int, hipStream_t);

}  // namespace sym
