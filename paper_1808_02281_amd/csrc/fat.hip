// Fat-link smearing (asqtad / HISQ) and its path force: kernels and launchers.
// The per-link device code and the derivation are in fat.hpp.
#include "fat.hpp"

namespace sym {

using fat::Ctx;
using fat::FatCoeffs;
using fat::Fields;

namespace {

template <typename T>
__global__ __launch_bounds__(kBlock) void fat_fk1_kernel(Geom g, const T* __restrict__ U, Fields<T> w, FatCoeffs cf,
                                                          int ntiles) {
  const LinkTile lt = link_tile(g, blockIdx.x, ntiles);
  const int cb = lt.chunk * kBlock + threadIdx.x;
  if (cb >= g.Vh) return;
  Ctx<T> c;
  fat::make_ctx(g, U, lt.mu, lt.p, cb, c);
  fat::fk1_step<1>(c, w, T(cf.c[2]), T(cf.c[3]), cb);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void fat_fk2_kernel(Geom g, const T* __restrict__ U, Fields<T> w, FatCoeffs cf,
                                                          int ntiles) {
  const LinkTile lt = link_tile(g, blockIdx.x, ntiles);
  const int cb = lt.chunk * kBlock + threadIdx.x;
  if (cb >= g.Vh) return;
  Ctx<T> c;
  fat::make_ctx(g, U, lt.mu, lt.p, cb, c);
  // transport direction outermost (two_out), both precisions; FP64 holds the three
  // accumulators in VGPRs and AGPRs at one wave per SIMD (6.05 -> 4.71 ms at 32^3 x 64
  // against one M at a time)
  su3<T> acc[3];
  const su3<T> u = c.template u<0, 0, 0, 0, 0>();
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    acc[k] = u;
    fat::scale(acc[k], T(cf.c[1]));
  }
  SYM_FAT_FENCE();
  fat::two_out<1, false>(acc, c, static_cast<const T*>(w.inner));
  fat::launder(c);
  SYM_FAT_FENCE();
  fat::store_m<1>(acc[0], c, w, T(cf.c[4]), cb);
  SYM_FAT_FENCE();
  fat::store_m<2>(acc[1], c, w, T(cf.c[4]), cb);
  SYM_FAT_FENCE();
  fat::store_m<3>(acc[2], c, w, T(cf.c[4]), cb);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void fat_fk3_kernel(Geom g, const T* __restrict__ U, Fields<T> w,
                                                          T* __restrict__ V, T* __restrict__ W, FatCoeffs cf,
                                                          int ntiles) {
  const LinkTile lt = link_tile(g, blockIdx.x, ntiles);
  const int cb = lt.chunk * kBlock + threadIdx.x;
  if (cb >= g.Vh) return;
  Ctx<T> c;
  fat::make_ctx(g, U, lt.mu, lt.p, cb, c);
  su3<T> acc = c.template u<0, 0, 0, 0, 0>();
  fat::scale(acc, T(cf.c[0]));
  fat::fk3_step<1>(acc, c, w);
  store_link(block_ptr(V, lt.mu, lt.p, g.Vh), g.Vh, cb, acc);
  if (W != nullptr) {
    fat::launder(c);
    su3<T> nk = mul<false, false>(c.template u<0, 0, 0, 0, 0>(), c.template u<1, 0, 0, 0, 0>());
    nk = mul<false, false>(nk, c.template u<2, 0, 0, 0, 0>());
    fat::scale(nk, T(cf.c[5]));
    store_link(block_ptr(W, lt.mu, lt.p, g.Vh), g.Vh, cb, nk);
  }
}

// FP32: six waves per SIMD (80 VGPRs, no spills): 1.26 -> 1.16 ms at 32^3 x 64
template <typename T>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 1))) void fat_bk3_kernel(Geom g, const T* __restrict__ U, const T* __restrict__ GV,
                                                          Fields<T> w, int ntiles) {
  const LinkTile lt = link_tile(g, blockIdx.x, ntiles);
  const int cb = lt.chunk * kBlock + threadIdx.x;
  if (cb >= g.Vh) return;
  Ctx<T> c;
  fat::make_ctx(g, U, lt.mu, lt.p, cb, c);
  fat::bk3_step<1>(c, GV, w, cb);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void fat_bk2_kernel(Geom g, const T* __restrict__ U, const T* __restrict__ GV,
                                                          Fields<T> w, FatCoeffs cf, int ntiles) {
  const LinkTile lt = link_tile(g, blockIdx.x, ntiles);
  const int cb = lt.chunk * kBlock + threadIdx.x;
  if (cb >= g.Vh) return;
  Ctx<T> c;
  fat::make_ctx(g, U, lt.mu, lt.p, cb, c);
  // D = c1 GV + c3 sum_k gmid_k + c5 sum_m g_inner_m
  su3<T> dsum = c.template f<0, 0, 0, 0, 0>(GV, 1, 0);
  fat::scale(dsum, T(cf.c[0]));
  for (int k = 0; k < 3; ++k) axpy(dsum, T(cf.c[1]), c.template f<0, 0, 0, 0, 0>(w.gmid, 3, k));
  SYM_FAT_FENCE();
  // transport direction outermost, both precisions (FP64: 6.78 -> 5.50 ms at 32^3 x 64)
  su3<T> gi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) set_zero(gi[k]);
  fat::two_out<1, true>(gi, c, static_cast<const T*>(w.gmid));
  fat::launder(c);
  const T c5 = T(cf.c[2]), c7 = T(cf.c[3]), cL = T(cf.c[4]);
  SYM_FAT_FENCE();
  fat::store_gt<1>(gi[0], c, GV, w, c7, cL, cb);
  SYM_FAT_FENCE();
  fat::store_gt<2>(gi[1], c, GV, w, c7, cL, cb);
  SYM_FAT_FENCE();
  fat::store_gt<3>(gi[2], c, GV, w, c7, cL, cb);
#pragma unroll
  for (int m = 0; m < 3; ++m) axpy(dsum, c5, gi[m]);
  fat::store_slot(w.D, 1, 0, lt.mu, lt.p, g.Vh, cb, dsum);
}

// Gradient (or force) of the thin link (y, nu): the direct terms D, the transports of
// U_nu's own chain, the Naik terms, and the deposits of the transports along nu of the
// other chains.
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void fat_gk_kernel(Geom g, const T* __restrict__ U, const T* __restrict__ GV,
                                                         const T* __restrict__ GW, Fields<T> w, T* __restrict__ out,
                                                         FatCoeffs cf, int ntiles) {
  const LinkTile lt = link_tile(g, blockIdx.x, ntiles);
  const int cb = lt.chunk * kBlock + threadIdx.x;
  if (cb >= g.Vh) return;
  Ctx<T> c;
  fat::make_ctx(g, U, lt.mu, lt.p, cb, c);

  su3<T> acc = c.template f<0, 0, 0, 0, 0>(w.D, 1, 0);
  SYM_FAT_FENCE();
  fat::gk_pull<1>(acc, c, w);

  if (GW != nullptr) {
    // W_{y-k nu} = cN U_{y-k nu,nu} U_{y-(k-1)nu,nu} U_{y-(k-2)nu,nu} for k = 0, 1, 2
    Ctx<T> cc = c;
    fat::launder(cc);
    const su3<T> u1 = cc.template u<1, 0, 0, 0, 0>(), u2 = cc.template u<2, 0, 0, 0, 0>();
    su3<T> t = mul<false, true>(cc.template f<0, 0, 0, 0, 0>(GW, 1, 0), u2);
    su3<T> nk = mul<false, true>(t, u1);
    const su3<T> um1 = cc.template u<-1, 0, 0, 0, 0>();
    t = mul<true, false>(um1, cc.template f<-1, 0, 0, 0, 0>(GW, 1, 0));
    mac<false, true>(nk, t, u1);
    t = mul<true, true>(um1, cc.template u<-2, 0, 0, 0, 0>());
    mac<false, false>(nk, t, cc.template f<-2, 0, 0, 0, 0>(GW, 1, 0));
    axpy(acc, T(cf.c[5]), nk);
    SYM_FAT_FENCE();
  }

  if constexpr (sizeof(T) == 4)
    fat::gk_factor_pipe<1>(acc, c, GV, w);
  else
    fat::gk_factor_links_once<1>(acc, c, GV, w);

  fat::launder(c);
  cx<T>* dst = block_ptr(out, lt.mu, lt.p, g.Vh);
  if constexpr (MODE == 0) {
    store_link(dst, g.Vh, cb, acc);
  } else {
    // G = -(1/2)(U grad^dagger)_TA, the force in the convention of the gauge force
    const su3<T> b = mul<false, true>(c.template u<0, 0, 0, 0, 0>(), acc);
    store_link(dst, g.Vh, cb, ta_scaled(b, T(-0.5)));
  }
}

}  // namespace

template <typename T>
hipError_t launch_fat_fk3(const Geom& g, const T* U, T* V, T* W, const FatCoeffs& c, const Fields<T>& w,
                          hipStream_t s) {
  const int nt = link_tiles(g);
  fat_fk3_kernel<T><<<nt, kBlock, 0, s>>>(g, U, w, V, W, c, nt);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fat_stage(int stage, const Geom& g, const T* U, const T* GV, const T* GW, T* out, int mode,
                            const FatCoeffs& c, const Fields<T>& w, hipStream_t s) {
  const int nt = link_tiles(g);
  switch (stage) {
    case 0:
      fat_fk1_kernel<T><<<nt, kBlock, 0, s>>>(g, U, w, c, nt);
      break;
    case 1:
      fat_fk2_kernel<T><<<nt, kBlock, 0, s>>>(g, U, w, c, nt);
      break;
    case 2:
      fat_bk3_kernel<T><<<nt, kBlock, 0, s>>>(g, U, GV, w, nt);
      break;
    case 3:
      fat_bk2_kernel<T><<<nt, kBlock, 0, s>>>(g, U, GV, w, c, nt);
      break;
    default: {
      // two workgroups per CU (56 KiB LDS reservation, no LDS used): fewer links in
      // flight keep more of the gathered neighbour matrices in L2 (FP32 at 32^3 x 64:
      // 8.97 -> 8.54 ms; FP64 is at two per CU by registers anyway)
      const size_t lds = 56 * 1024;
      if (mode == 0)
        fat_gk_kernel<T, 0><<<nt, kBlock, lds, s>>>(g, U, GV, GW, w, out, c, nt);
      else
        fat_gk_kernel<T, 1><<<nt, kBlock, lds, s>>>(g, U, GV, GW, w, out, c, nt);
      break;
    }
  }
  return hipGetLastError();
}

#ifndef SYM_ONLY_F64
template hipError_t launch_fat_fk3<float>(const Geom&, const float*, float*, float*, const FatCoeffs&,
                                            const Fields<float>&, hipStream_t);
template hipError_t launch_fat_stage<float>(int, const Geom&, const float*, const float*, const float*, float*, int,
                                            const FatCoeffs&, const Fields<float>&, hipStream_t);
#endif
#ifndef SYM_ONLY_F32
template hipError_t launch_fat_fk3<double>(const Geom&, const double*, double*, double*, const FatCoeffs&,
                                             const Fields<double>&, hipStream_t);
template hipError_t launch_fat_stage<double>(int, const Geom&, const double*, const double*, const double*, double*,
                                             int, const FatCoeffs&, const Fields<double>&, hipStream_t);
#endif

}  // namespace sym
