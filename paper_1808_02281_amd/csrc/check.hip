// Link-field check for callers of the factored force path, which reads links as their
// first two rows and rebuilds the third, so it assumes special-unitary links: per link
// the unitarity defect ||U^dagger U - 1||_F and |det U - 1| in double, and whether any
// element is not finite. Per-workgroup maxima (order-independent, hence deterministic)
// and counts, then one finishing block. And the repair: every link projected onto SU(3).
#include "project.hpp"

namespace sym {
namespace {

using cd = cx<double>;

__device__ __forceinline__ cd cm(cd a, cd b) { return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

__device__ __forceinline__ double block_max(double v) {
  __shared__ double red[kBlock / 64];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double m = red[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, red[w]);
  __syncthreads();
  return m;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void check_links_kernel(Geom g, const T* __restrict__ U,
                                                             double* __restrict__ partials, int ntiles) {
  const LinkTile lt = link_tile(g, blockIdx.x, ntiles);
  const int cb = lt.chunk * kBlock + threadIdx.x;
  double unit = 0.0, det = 0.0, bad = 0.0;
  if (cb < g.Vh) {
    const su3<T> u = load_link(block_ptr(U, lt.mu, lt.p, g.Vh), g.Vh, cb);
    su3<double> d;
    bool finite = true;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      d.e[i] = cd{double(u.e[i].re), double(u.e[i].im)};
      finite = finite && isfinite(d.e[i].re) && isfinite(d.e[i].im);
    }
    if (finite) {
      const su3<double> h = mul<true, false>(d, d);  // U^dagger U
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const double re = h.e[i].re - ((i % 4 == 0) ? 1.0 : 0.0);
        s += re * re + h.e[i].im * h.e[i].im;
      }
      unit = sqrt(s);
      const cd m0 = cd{cm(d.e[4], d.e[8]).re - cm(d.e[5], d.e[7]).re, cm(d.e[4], d.e[8]).im - cm(d.e[5], d.e[7]).im};
      const cd m1 = cd{cm(d.e[3], d.e[8]).re - cm(d.e[5], d.e[6]).re, cm(d.e[3], d.e[8]).im - cm(d.e[5], d.e[6]).im};
      const cd m2 = cd{cm(d.e[3], d.e[7]).re - cm(d.e[4], d.e[6]).re, cm(d.e[3], d.e[7]).im - cm(d.e[4], d.e[6]).im};
      const cd a = cm(d.e[0], m0), b = cm(d.e[1], m1), c = cm(d.e[2], m2);
      const double dre = a.re - b.re + c.re - 1.0, dim = a.im - b.im + c.im;
      det = sqrt(dre * dre + dim * dim);
    } else {
      bad = 1.0;
    }
  }
  unit = block_max(unit);
  det = block_max(det);
  double cnt[1] = {bad};
  block_sum<1>(cnt);
  if (threadIdx.x == 0) {
    double* o = partials + 3 * (size_t)blockIdx.x;
    o[0] = unit;
    o[1] = det;
    o[2] = cnt[0];
  }
}

__global__ __launch_bounds__(kBlock) void check_finish_kernel(const double* __restrict__ partials, int n,
                                                              double* __restrict__ out) {
  double unit = 0.0, det = 0.0;
  double cnt[1] = {0.0};
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    unit = fmax(unit, partials[3 * (size_t)i]);
    det = fmax(det, partials[3 * (size_t)i + 1]);
    cnt[0] += partials[3 * (size_t)i + 2];
  }
  unit = block_max(unit);
  det = block_max(det);
  block_sum<1>(cnt);
  if (threadIdx.x == 0) {
    out[0] = unit;
    out[1] = det;
    out[2] = cnt[0];
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void reunitarise_kernel(Geom g, T* __restrict__ U, int ntiles) {
  const LinkTile lt = link_tile(g, blockIdx.x, ntiles);
  const int cb = lt.chunk * kBlock + threadIdx.x;
  if (cb >= g.Vh) return;
  cx<T>* blk = block_ptr(U, lt.mu, lt.p, g.Vh);
  const su3<T> u = load_link(static_cast<const cx<T>*>(blk), g.Vh, cb);
  su3<double> d;
#pragma unroll
  for (int i = 0; i < 9; ++i) d.e[i] = cd{double(u.e[i].re), double(u.e[i].im)};
  proj::project_su3(d);
  su3<T> out;
#pragma unroll
  for (int i = 0; i < 9; ++i) out.e[i] = cx<T>{T(d.e[i].re), T(d.e[i].im)};
  store_link(blk, g.Vh, cb, out);
}

}  // namespace

template <typename T>
hipError_t launch_reunitarise(const Geom& g, T* U, hipStream_t s) {
  const int nt = link_tiles(g);
  reunitarise_kernel<T><<<nt, kBlock, 0, s>>>(g, U, nt);
  return hipGetLastError();
}

template hipError_t launch_reunitarise<float>(const Geom&, float*, hipStream_t);
template hipError_t launch_reunitarise<double>(const Geom&, double*, hipStream_t);

template <typename T>
hipError_t launch_check_links(const Geom& g, const T* U, double* partials, double* out, hipStream_t s) {
  const int nt = link_tiles(g);
  check_links_kernel<T><<<nt, kBlock, 0, s>>>(g, U, partials, nt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  check_finish_kernel<<<1, kBlock, 0, s>>>(partials, nt, out);
  return hipGetLastError();
}

template hipError_t launch_check_links<float>(const Geom&, const float*, double*, double*, hipStream_t);
template hipError_t launch_check_links<double>(const Geom&, const double*, double*, double*, hipStream_t);

}  // namespace sym
