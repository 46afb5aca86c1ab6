// Batched factored force: many independent lattices (uneven sizes) in one launch per
// pass. Workgroups walk the concatenated tiles of all lattices with a static schedule
// (one tile each when the grid covers every tile, else a persistent loop; no atomics:
// the result, including the action partials, does not depend on timing) and run the
// same per-link code as the single-lattice kernels (factored.hpp), so every link's
// force is bitwise the single-lattice one.
#include "factored.hpp"

namespace sym {
namespace {

using factored::factored_link;
using factored::staples_site;

// k-th tile of workgroup blk among `total` tiles, or -1 when the workgroup has no more
// work (-2: none this round, continue).
__device__ __forceinline__ int batch_tile(const BatchTable& b, int total, int blk, int grid, int k) {
  if (b.order == 0) {
    const int t = blk + k * grid;
    return t < total ? t : -1;
  }
  const int gx = grid >> 3;                      // workgroups per XCD
  const int per = (total + 7) >> 3;              // tiles per XCD
  const int r = (blk >> 3) + k * gx;
  if (r >= per) return -1;
  const int t = (blk & 7) * per + r;
  return t < total ? t : -2;
}

// Lattice of a link tile (SITES = false) or of a site tile (SITES = true).
template <bool SITES>
__device__ __forceinline__ int find_lattice(const BatchTable& b, int tile) {
  int l = 0;
  for (int k = 1; k < b.n; ++k) l = tile >= (SITES ? b.e[k].site_tile_begin : b.e[k].tile_begin) ? k : l;
  return l;
}

__device__ __forceinline__ Geom geom_of(const BatchEntry& e) {
  Geom g;
  for (int a = 0; a < 4; ++a) g.L[a] = e.L[a];
  g.Vh = e.Vh;
  g.Lxh = e.L[0] / 2;
  g.tslab = 0;
  g.cps = 0;
  return g;
}

// Pass 1 over the site tiles of all lattices (two per 256-site chunk: the parities).
template <typename T>
__global__ __launch_bounds__(kBlock) void staples_batch_kernel(const BatchTable b) {
  for (int k = 0;; ++k) {
    const int tile = batch_tile(b, b.total_site_tiles, blockIdx.x, gridDim.x, k);
    if (tile == -1) break;
    if (tile < 0) continue;
    const BatchEntry& e = b.e[find_lattice<true>(b, tile)];
    const Geom g = geom_of(e);
    const int local = tile - e.site_tile_begin;
    const int cb = (local >> 1) * kBlock + threadIdx.x;
    if (cb < g.Vh) staples_site(g, static_cast<const T*>(e.U), static_cast<T*>(e.S8), local & 1, cb);
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void force_batch_kernel(const BatchTable b, double* __restrict__ partials,
                                                             Coeffs cf) {
  for (int k = 0;; ++k) {
    const int tile = batch_tile(b, b.total_tiles, blockIdx.x, gridDim.x, k);
    if (tile == -1) break;
    if (tile < 0) continue;
    const BatchEntry& e = b.e[find_lattice<false>(b, tile)];
    const Geom g = geom_of(e);
    const int local = tile - e.tile_begin;
    const int cb = (local >> 3) * (int)blockDim.x + threadIdx.x;  // blockDim.x links per tile
    double a[3] = {0.0, 0.0, 0.0};
    if (cb < g.Vh)
      factored_link<T, ForceOut::Store>(g, static_cast<const T*>(e.U), static_cast<const T*>(e.S8),
                                        static_cast<T*>(e.F), 0.0, cf, local & 3, (local >> 2) & 1, cb, a);
    block_sum_store<3>(a, partials + 3 * (size_t)tile);
  }
}

// Block l: S and W of lattice l from its tiles' partials (same formulas as the kind-2
// finish in action.hip).
__global__ __launch_bounds__(256) void finish_batch_kernel(const BatchTable b, const double* __restrict__ partials,
                                                           Coeffs c, double* __restrict__ out) {
  const int l = blockIdx.x;
  const int t0 = b.e[l].tile_begin;
  const int t1 = l + 1 < b.n ? b.e[l + 1].tile_begin : b.total_tiles;
  double v[3] = {0.0, 0.0, 0.0};
#pragma unroll 8
  for (int t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
    v[0] += partials[3 * (size_t)t + 0];
    v[1] += partials[3 * (size_t)t + 1];
    v[2] += partials[3 * (size_t)t + 2];
  }
  block_sum<3>(v);
  if (threadIdx.x == 0) {
    const double V = 2.0 * b.e[l].Vh;
    const double wP = v[0] / 4.0, wR = v[1] / 4.0;
    const double cwC = (v[2] - 0.5 * c.c[1] * v[1]) / 6.0;
    const double wC = c.c[2] != 0.0 ? cwC / c.c[2] : __builtin_nan("");
    out[4 * l + 0] = c.beta / 3.0 * (c.c[0] * wP + c.c[1] * wR + cwC);
    out[4 * l + 1] = 18.0 * V - wP;
    out[4 * l + 2] = 36.0 * V - wR;
    out[4 * l + 3] = 48.0 * V - wC;
  }
}

}  // namespace

template <typename T>
hipError_t launch_staples_batch(const BatchTable& b, int grid, hipStream_t s) {
  // the persistent grid of the force pass covers every site tile; one workgroup per site
  // tile otherwise
  const int g = grid > 0 ? grid : (b.order == 1 ? (b.total_site_tiles + 7) / 8 * 8 : b.total_site_tiles);
  staples_batch_kernel<T><<<g, kBlock, 0, s>>>(b);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_force_batch(const BatchTable& b, int grid, int links, int lds_kib, double* partials,
                              const Coeffs& c, hipStream_t s) {
  const size_t lds = lds_kib < 0 ? factored_lds_reservation<T>() : (size_t)lds_kib * 1024;
  force_batch_kernel<T><<<grid, links, lds, s>>>(b, partials, c);
  return hipGetLastError();
}

#ifndef SYM_ONLY_F64
template hipError_t launch_staples_batch<float>(const BatchTable&, int, hipStream_t);
template hipError_t launch_force_batch<float>(const BatchTable&, int, int, int, double*, const Coeffs&, hipStream_t);
#endif
#ifndef SYM_ONLY_F32
template hipError_t launch_staples_batch<double>(const BatchTable&, int, hipStream_t);
template hipError_t launch_force_batch<double>(const BatchTable&, int, int, int, double*, const Coeffs&,
                                               hipStream_t);
// the finish kernel is precision independent; it lives in the FP64 object
hipError_t launch_finish_batch(const BatchTable& b, const double* partials, const Coeffs& c, double* out,
                               hipStream_t s) {
  finish_batch_kernel<<<b.n, 256, 0, s>>>(b, partials, c, out);
  return hipGetLastError();
}
#endif

}  // namespace sym
