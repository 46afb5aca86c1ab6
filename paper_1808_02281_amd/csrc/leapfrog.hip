// Molecular-dynamics pieces for md_leapfrog: kinetic energy partials and the link
// drift U <- exp(dt Pi) U. Links are written U = exp(i omega.T) with dU/domega = iTU
// (arXiv:1808.02281 Sec. II, eqs. 18_1_29_3 and 18_7_26_1), so momenta are
// antihermitian Pi = i p_a T_a, the equation of motion of U is U-dot = Pi U, and the
// kinetic energy is -tr(Pi^2) = (1/2) sum_a p_a^2 per link. All of it in double; in
// the FP32 layout the updated link is projected onto SU(3) and rounded to float on store.
#include "project.hpp"

namespace sym {
namespace {

using cd = cx<double>;

__device__ __forceinline__ cd cadd(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd cmul(cd a, cd b) { return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cd cscale(cd a, double s) { return cd{a.re * s, a.im * s}; }

// exp(X) of a 3x3 complex matrix with small trace (antihermitian momenta times dt).
// X = tau I + Z with tau = tr(X)/3 and Z traceless, exp(X) = e^tau exp(Z). Z satisfies
// Cayley-Hamilton Z^3 = c1 Z + c0 I (c1 = tr(Z^2)/2, c0 = det Z), so every power of
// Y = Z/2^s is a_k I + b_k Y + g_k Y^2 with a scalar recurrence; the Taylor series of
// exp(Y) reduces to three scalar series (each term divided by k! on the fly). With
// ||Y||_F <= 1/2 twenty terms leave a remainder below 1e-21; s squarings undo the
// scaling.
__device__ su3<double> su3_exp(const su3<double>& X) {
  const cd tau = cscale(cadd(cadd(X.e[0], X.e[4]), X.e[8]), 1.0 / 3.0);
  su3<double> Z = X;
  Z.e[0].re -= tau.re; Z.e[0].im -= tau.im;
  Z.e[4].re -= tau.re; Z.e[4].im -= tau.im;
  Z.e[8].re -= tau.re; Z.e[8].im -= tau.im;

  double nrm2 = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) nrm2 += Z.e[i].re * Z.e[i].re + Z.e[i].im * Z.e[i].im;
  int s = 0;
  double nrm = sqrt(nrm2);
  while (nrm > 0.5 && s < 64) {
    nrm *= 0.5;
    ++s;
  }
  const double sc = ldexp(1.0, -s);
#pragma unroll
  for (int i = 0; i < 9; ++i) Z.e[i] = cscale(Z.e[i], sc);

  const su3<double> Z2 = mul<false, false>(Z, Z);
  const cd c1 = cscale(cadd(cadd(Z2.e[0], Z2.e[4]), Z2.e[8]), 0.5);
  // det Z by cofactors along the first row
  const cd m0 = cadd(cmul(Z.e[4], Z.e[8]), cscale(cmul(Z.e[5], Z.e[7]), -1.0));
  const cd m1 = cadd(cmul(Z.e[3], Z.e[8]), cscale(cmul(Z.e[5], Z.e[6]), -1.0));
  const cd m2 = cadd(cmul(Z.e[3], Z.e[7]), cscale(cmul(Z.e[4], Z.e[6]), -1.0));
  const cd c0 = cadd(cadd(cmul(Z.e[0], m0), cscale(cmul(Z.e[1], m1), -1.0)), cmul(Z.e[2], m2));

  cd A{1.0, 0.0}, B{0.0, 0.0}, G{0.0, 0.0};
  cd f0 = A, f1 = B, f2 = G;
#pragma unroll
  for (int k = 1; k <= 20; ++k) {
    const double inv = 1.0 / k;
    const cd An = cscale(cmul(G, c0), inv);
    const cd Bn = cscale(cadd(A, cmul(G, c1)), inv);
    const cd Gn = cscale(B, inv);
    A = An;
    B = Bn;
    G = Gn;
    f0 = cadd(f0, A);
    f1 = cadd(f1, B);
    f2 = cadd(f2, G);
  }
  su3<double> E;
#pragma unroll
  for (int i = 0; i < 9; ++i) E.e[i] = cadd(cmul(f1, Z.e[i]), cmul(f2, Z2.e[i]));
  E.e[0] = cadd(E.e[0], f0);
  E.e[4] = cadd(E.e[4], f0);
  E.e[8] = cadd(E.e[8], f0);
  for (int i = 0; i < s; ++i) E = mul<false, false>(E, E);

  const double mag = exp(tau.re);
  const cd phase{mag * cos(tau.im), mag * sin(tau.im)};
#pragma unroll
  for (int i = 0; i < 9; ++i) E.e[i] = cmul(E.e[i], phase);
  return E;
}

template <typename T>
__device__ __forceinline__ su3<double> to_double(const su3<T>& a) {
  su3<double> r;
#pragma unroll
  for (int i = 0; i < 9; ++i) r.e[i] = cd{double(a.e[i].re), double(a.e[i].im)};
  return r;
}

// U <- exp(dt Pi) U in double. In the FP32 layout the product is projected back onto
// SU(3) before it is rounded to float: rounding leaves a unitarity defect of a few
// 1e-8 per step, which would otherwise accumulate over a trajectory, while the force
// kernels that read links as two rows assume special-unitary links. The projection
// moves a link by the size of that defect, so each step starts again from a link that
// is special unitary to float rounding. FP64 links are stored as computed.
template <typename T>
__global__ __launch_bounds__(kBlock) void drift_kernel(Geom g, T* __restrict__ U, const T* __restrict__ P, double dt,
                                                       int ntiles) {
  const LinkTile lt = link_tile(g, blockIdx.x, ntiles);
  const int mu = lt.mu, p = lt.p, chunk = lt.chunk;
  const int cb = chunk * kBlock + threadIdx.x;
  if (cb >= g.Vh) return;
  su3<double> X = to_double(load_link(block_ptr(P, mu, p, g.Vh), g.Vh, cb));
#pragma unroll
  for (int i = 0; i < 9; ++i) X.e[i] = cscale(X.e[i], dt);
  const su3<double> E = su3_exp(X);
  cx<T>* ub = block_ptr(U, mu, p, g.Vh);
  const su3<double> u = to_double(load_link(static_cast<const cx<T>*>(ub), g.Vh, cb));
  su3<double> un = mul<false, false>(E, u);
  if constexpr (sizeof(T) == 4) proj::project_su3(un);
  su3<T> out;
#pragma unroll
  for (int i = 0; i < 9; ++i) out.e[i] = cx<T>{T(un.e[i].re), T(un.e[i].im)};
  store_link(ub, g.Vh, cb, out);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void kinetic_kernel(Geom g, const T* __restrict__ P, double* __restrict__ partials,
                                                         int ntiles) {
  const LinkTile lt = link_tile(g, blockIdx.x, ntiles);
  const int mu = lt.mu, p = lt.p, chunk = lt.chunk;
  const int cb = chunk * kBlock + threadIdx.x;
  double v[1] = {0.0};
  if (cb < g.Vh) {
    const su3<double> q = to_double(load_link(block_ptr(P, mu, p, g.Vh), g.Vh, cb));
    double s = 0.0;  // -Re tr(Pi^2) = -sum_ij Re(Pi_ij Pi_ji)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) s -= q.e[3 * i + j].re * q.e[3 * j + i].re - q.e[3 * i + j].im * q.e[3 * j + i].im;
    v[0] = s;
  }
  block_sum_store<1>(v, partials + blockIdx.x);
}

}  // namespace

template <typename T>
hipError_t launch_kinetic(const Geom& g, const T* P, double* partials, hipStream_t s) {
  const int nt = link_tiles(g);
  kinetic_kernel<T><<<nt, kBlock, 0, s>>>(g, P, partials, nt);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_drift(const Geom& g, T* U, const T* P, double dt, hipStream_t s) {
  const int nt = link_tiles(g);
  drift_kernel<T><<<nt, kBlock, 0, s>>>(g, U, P, dt, nt);
  return hipGetLastError();
}

template hipError_t launch_kinetic<float>(const Geom&, const float*, double*, hipStream_t);
template hipError_t launch_kinetic<double>(const Geom&, const double*, double*, hipStream_t);
template hipError_t launch_drift<float>(const Geom&, float*, const float*, double, hipStream_t);
template hipError_t launch_drift<double>(const Geom&, double*, const double*, double, hipStream_t);

}  // namespace sym
