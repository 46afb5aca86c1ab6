// Conversion between the canonical array-of-structures lexicographic link layout,
// complex (Lt, Lz, Ly, Lx, 4, 3, 3), and the even-odd structure-of-arrays layout of
// lattice.hpp. One thread per (site, direction); reads (pack) or writes (unpack) of
// the 9 complex elements of a link are contiguous across consecutive threads.
#include "kernels.hpp"

namespace sym {
namespace {

__device__ __forceinline__ void lex_to_cb(const Geom& g, int s, int& p, int& cb) {
  int r = s;
  const int x = r % g.L[0];
  r /= g.L[0];
  const int y = r % g.L[1];
  r /= g.L[1];
  const int z = r % g.L[2];
  const int t = r / g.L[2];
  p = (x + y + z + t) & 1;
  cb = s >> 1;
}

template <typename T, bool PACK>
__global__ __launch_bounds__(kBlock) void layout_kernel(Geom g, const T* __restrict__ src, T* __restrict__ dst) {
  const long long idx = (long long)blockIdx.x * kBlock + threadIdx.x;  // site * 4 + mu
  if (idx >= 4ll * 2 * g.Vh) return;
  const int site = (int)(idx >> 2), mu = (int)(idx & 3);
  int p, cb;
  lex_to_cb(g, site, p, cb);
  const cx<T>* s = reinterpret_cast<const cx<T>*>(src);
  cx<T>* d = reinterpret_cast<cx<T>*>(dst);
  const size_t blk = (size_t)((mu * 2 + p) * 9) * (size_t)g.Vh;
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    const size_t soa = blk + (size_t)c * g.Vh + cb;
    const size_t aos = (size_t)idx * 9 + c;
    if constexpr (PACK)
      d[soa] = s[aos];
    else
      d[aos] = s[soa];
  }
}

}  // namespace

template <typename T>
hipError_t launch_pack(const Geom& g, const T* aos, T* soa, hipStream_t s) {
  const long long n = 8ll * g.Vh;
  layout_kernel<T, true><<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(g, aos, soa);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_unpack(const Geom& g, const T* soa, T* aos, hipStream_t s) {
  const long long n = 8ll * g.Vh;
  layout_kernel<T, false><<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(g, soa, aos);
  return hipGetLastError();
}

template hipError_t launch_pack<float>(const Geom&, const float*, float*, hipStream_t);
template hipError_t launch_pack<double>(const Geom&, const double*, double*, hipStream_t);
template hipError_t launch_unpack<float>(const Geom&, const float*, float*, hipStream_t);
template hipError_t launch_unpack<double>(const Geom&, const double*, double*, hipStream_t);

}  // namespace sym
