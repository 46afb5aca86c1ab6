// Factored gauge force, single lattice: pass 1 (plaquette staples) and pass 2 (force)
// kernels over one lattice; the per-link device code is in factored.hpp.
#include "factored.hpp"

namespace sym {
namespace {

using factored::factored_link;
using factored::staples_site;

template <typename T>
__global__ __launch_bounds__(kBlock) void staples_kernel(Geom g, const T* __restrict__ U, T* __restrict__ S8,
                                                         int ntiles) {
  const SiteTile st = site_tile(g, blockIdx.x, ntiles);
  const int cb = st.chunk * kBlock + threadIdx.x;
  if (cb < g.Vh) staples_site(g, U, S8, st.p, cb);
}

template <typename T, ForceOut MODE>
__global__ __launch_bounds__(factored_links<T>()) void force_factored_kernel(Geom g, const T* __restrict__ U,
                                                                             const T* __restrict__ S8,
                                                                             T* __restrict__ out, double kick,
                                                                             double* __restrict__ partials, Coeffs cf,
                                                                             int ntiles) {
  constexpr int N = factored_links<T>();
  const LinkTile lt = link_tile(g, blockIdx.x, ntiles, kBlock / N);
  const int cb = lt.chunk * N + threadIdx.x;
  double a[3] = {0.0, 0.0, 0.0};
  if (cb < g.Vh) factored_link<T, MODE>(g, U, S8, out, kick, cf, lt.mu, lt.p, cb, a);
  if (partials != nullptr) block_sum_store<3>(a, partials + 3 * (size_t)blockIdx.x);
}

}  // namespace

template <typename T>
hipError_t launch_staples(const Geom& g, const T* U, T* S8, hipStream_t s) {
  const int nt = site_tiles(g);
  staples_kernel<T><<<nt, kBlock, 0, s>>>(g, U, S8, nt);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_force_factored(const Geom& g, const T* U, const T* S8, T* out, double kick, double* partials,
                                 const Coeffs& c, ForceOut mode, hipStream_t s) {
  const int nt = factored_tiles<T>(g);
  constexpr int N = factored_links<T>();
  // one or two waves per SIMD by registers (FP64, FP32); no LDS reservation: with
  // workgroups of one or two waves it would only take waves away
  if (mode == ForceOut::Store)
    force_factored_kernel<T, ForceOut::Store><<<nt, N, 0, s>>>(g, U, S8, out, kick, partials, c, nt);
  else if (mode == ForceOut::Kick)
    force_factored_kernel<T, ForceOut::Kick><<<nt, N, 0, s>>>(g, U, S8, out, kick, partials, c, nt);
  else
    force_factored_kernel<T, ForceOut::Grad><<<nt, N, 0, s>>>(g, U, S8, out, kick, partials, c, nt);
  return hipGetLastError();
}

#ifndef SYM_ONLY_F64
template hipError_t launch_staples<float>(const Geom&, const float*, float*, hipStream_t);
#endif
#ifndef SYM_ONLY_F32
template hipError_t launch_staples<double>(const Geom&, const double*, double*, hipStream_t);
#endif
#ifndef SYM_ONLY_F64
template hipError_t launch_force_factored<float>(const Geom&, const float*, const float*, float*, double, double*,
                                                 const Coeffs&, ForceOut, hipStream_t);
#endif
#ifndef SYM_ONLY_F32
template hipError_t launch_force_factored<double>(const Geom&, const double*, const double*, double*, double, double*,
                                                  const Coeffs&, ForceOut, hipStream_t);
#endif

}  // namespace sym
