// Wilson fermion force with clover term for given vectors X, Y: spinor layout
// kernels, clover insertion kernel and the per-link force kernel.
//
// arXiv:1808.02281, Sec. "Wilson fermion action with clover term". With
// D = A - kappa Dh (eq. 18_7_17_2), hopping part of eq. 18_7_17_4 and clover diagonal
// A_n = 1 - c_sw kappa/16 sum_{mu != nu} [g_mu, g_nu] Q_{n;mu nu} (eq. 18_7_18_0; kappa =
// 1/(2(m+4))), the kernels differentiate Psi(U) = Y^+ D X + c.c. (eq. 18_6_24_0) along
// U_{k,rho} -> exp(i omega.T) U_{k,rho} and store G = -(1/2) M_TA with
// dPsi/domega^a = Re tr(i T_a M) = -2i tr(T_a G).
//
// Hopping (eqs. 18_1_29_20_1..3): with B' = sum_a ((1 - g_rho) X_{k+rho})_a (x) Y_{k,a}^+
// and C' = sum_a X_{k,a} (x) ((1 + g_rho) Y_{k+rho})_a^+ (colour outer products summed
// over spin a), B = U B' and C = C' U^+, and M_hop = -2 kappa (B - C).
//
// Clover: Y_n^+ G P X_n = tr(P S_n) for a colour matrix P with
// S_n = sum_a (G X_n)_a (x) Y_{n,a}^+, so the clover part of Psi is
// -(c_sw kappa / 8) Re sum_n sum_{mu<nu} tr(Q_{n;mu nu} K_n^{mu nu}), K = S - S^+ with
// G = [g_mu, g_nu]. Pass 1 (wilson_clover_kernel) stores the six K per site. The leaves
// through link (k, rho) lie in the plaquettes k -> k+rho -> k+rho+nu_s -> k+nu_s -> k
// (nu_s = +-nu), each a leaf of Q at its four corners c0..c3; splitting each leaf at
// U_{k,rho} (eqs. 18_7_26_9, 18_7_26_10, in matrix form) gives
//   M_clov = -(c_sw kappa / 8) U sum_{nu, s} sigma (abd K_c0 + K_c1 abd + a K_c2 bd + ab K_c3 d),
// with a = U_{k+rho,nu_s}, b = U_{k+rho+nu_s,-rho}, d = U_{k+nu_s,-nu_s}, and
// sigma = +-1 as the plaquette's sense rho -> nu_s agrees with the leaf sense min -> max.
// The last two terms share their outer factors, a (K_c2 b + b K_c3) d: 8 products per
// plaquette, 50 per link with U B' and C' U^+.
//
// Spinor layout: field[p][3*spin + colour][V/2] complex (parity p, checkerboard cb).
// Clover insertions, pair = (0,1),(0,2),(0,3),(1,2),(1,3),(2,3): K is anti-Hermitian,
// so each is stored in 9 reals, block K[p][pair] of 9 V/2 reals = complex planes
// K01, K02, K12, (Im K00, Im K11), then a real plane Im K22; half the bytes of a full
// matrix on both sides (the force kernel reads 24 of them per link). Links are read as
// their first two rows, the third rebuilt (special unitary).
// Gamma matrices: Hermitian, DeGrand-Rossi basis, g_1..g_4 along x, y, z, t.
#include "kernels.hpp"

namespace sym {

namespace {

template <typename T>
struct spinor {
  cx<T> s[4][3];
};

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return cx<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> times_i(cx<T> a, int sgn) {  // sgn * i * a
  return sgn > 0 ? cx<T>{-a.im, a.re} : cx<T>{a.im, -a.re};
}
template <typename T>
__device__ __forceinline__ cx<T> neg(cx<T> a) {
  return cx<T>{-a.re, -a.im};
}

// gamma_mu x (spin rows, per colour)
template <typename T>
__device__ __forceinline__ spinor<T> gamma_apply(int mu, const spinor<T>& x) {
  spinor<T> r;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (mu == 0) {
      r.s[0][c] = times_i(x.s[3][c], 1);
      r.s[1][c] = times_i(x.s[2][c], 1);
      r.s[2][c] = times_i(x.s[1][c], -1);
      r.s[3][c] = times_i(x.s[0][c], -1);
    } else if (mu == 1) {
      r.s[0][c] = neg(x.s[3][c]);
      r.s[1][c] = x.s[2][c];
      r.s[2][c] = x.s[1][c];
      r.s[3][c] = neg(x.s[0][c]);
    } else if (mu == 2) {
      r.s[0][c] = times_i(x.s[2][c], 1);
      r.s[1][c] = times_i(x.s[3][c], -1);
      r.s[2][c] = times_i(x.s[0][c], -1);
      r.s[3][c] = times_i(x.s[1][c], 1);
    } else {
      r.s[0][c] = x.s[2][c];
      r.s[1][c] = x.s[3][c];
      r.s[2][c] = x.s[0][c];
      r.s[3][c] = x.s[1][c];
    }
  }
  return r;
}

// (1 + sgn gamma_mu) x
template <typename T>
__device__ __forceinline__ spinor<T> project(int mu, int sgn, const spinor<T>& x) {
  const spinor<T> g = gamma_apply(mu, x);
  spinor<T> r;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      r.s[a][c] = sgn > 0 ? cx<T>{x.s[a][c].re + g.s[a][c].re, x.s[a][c].im + g.s[a][c].im}
                          : cx<T>{x.s[a][c].re - g.s[a][c].re, x.s[a][c].im - g.s[a][c].im};
  return r;
}

// sum over spin of the colour outer product: out_{ba} = sum_alpha p_{alpha b} conj(q_{alpha a})
template <typename T>
__device__ __forceinline__ su3<T> outer(const spinor<T>& p, const spinor<T>& q) {
  su3<T> r;
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      T re = T(0), im = T(0);
#pragma unroll
      for (int al = 0; al < 4; ++al) {
        const cx<T> x = p.s[al][b], y = q.s[al][a];
        re = fma(x.re, y.re, re);
        re = fma(x.im, y.im, re);
        im = fma(x.im, y.re, im);
        im = fma(-x.re, y.im, im);
      }
      r.e[3 * b + a] = cx<T>{re, im};
    }
  return r;
}

template <typename T>
__device__ __forceinline__ spinor<T> load_spinor(const T* F, int p, int Vh, int cb) {
  const cx<T>* blk = reinterpret_cast<const cx<T>*>(F) + (size_t)p * 12 * (size_t)Vh;
  const unsigned bytes = 12u * (unsigned)Vh * (unsigned)sizeof(cx<T>);
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(const_cast<cx<T>*>(blk), (short)0, (int)bytes,
                                                                     kBufferWord3);
  const int voff = cb * (int)sizeof(cx<T>);
  spinor<T> s;
#pragma unroll
  for (int e = 0; e < 12; ++e) {
    const int soff = (int)((unsigned)e * (unsigned)Vh * (unsigned)sizeof(cx<T>));
    if constexpr (sizeof(T) == 4)
      s.s[e / 3][e % 3] = __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    else
      s.s[e / 3][e % 3] = __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  }
  return s;
}

constexpr int pair_index(int lo, int hi) { return lo == 0 ? hi - 1 : (lo == 1 ? hi + 1 : 5); }

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t antiherm_rsrc(const T* blk, int Vh) {
  const unsigned bytes = 9u * (unsigned)Vh * (unsigned)sizeof(T);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(blk), (short)0, (int)bytes, kBufferWord3);
}

// the anti-Hermitian k into its 9-real block (layout above)
template <typename T>
__device__ __forceinline__ void store_antiherm(T* blk, int Vh, int cb, const su3<T>& k) {
  const __amdgpu_buffer_rsrc_t r = antiherm_rsrc(static_cast<const T*>(blk), Vh);
  const cx<T> v[4] = {k.e[1], k.e[2], k.e[5], cx<T>{k.e[0].im, k.e[4].im}};
  const int voff = cb * (int)sizeof(cx<T>);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int soff = (int)((unsigned)c * (unsigned)Vh * (unsigned)sizeof(cx<T>));
    if constexpr (sizeof(T) == 4)
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v[c]),
                                            r, voff, soff, kStoreNT);
    else
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, v[c]),
                                             r, voff, soff, kStoreNT);
  }
  const int voff1 = cb * (int)sizeof(T), soff1 = (int)(8u * (unsigned)Vh * (unsigned)sizeof(T));
  if constexpr (sizeof(T) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, k.e[8].im), r, voff1, soff1, kStoreNT);
  else
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, k.e[8].im),
                                          r, voff1, soff1, kStoreNT);
}

template <typename T>
__device__ __forceinline__ su3<T> load_antiherm(const T* blk, int Vh, int cb) {
  const __amdgpu_buffer_rsrc_t r = antiherm_rsrc(blk, Vh);
  const int voff = cb * (int)sizeof(cx<T>);
  cx<T> v[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int soff = (int)((unsigned)c * (unsigned)Vh * (unsigned)sizeof(cx<T>));
    if constexpr (sizeof(T) == 4)
      v[c] = __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    else
      v[c] = __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  }
  const int voff1 = cb * (int)sizeof(T), soff1 = (int)(8u * (unsigned)Vh * (unsigned)sizeof(T));
  T d2;
  if constexpr (sizeof(T) == 4)
    d2 = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff1, soff1, 0));
  else
    d2 = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff1, soff1, 0));
  su3<T> k;
  k.e[0] = cx<T>{T(0), v[3].re};
  k.e[1] = v[0];
  k.e[2] = v[1];
  k.e[3] = cx<T>{-v[0].re, v[0].im};
  k.e[4] = cx<T>{T(0), v[3].im};
  k.e[5] = v[2];
  k.e[6] = cx<T>{-v[1].re, v[1].im};
  k.e[7] = cx<T>{-v[2].re, v[2].im};
  k.e[8] = cx<T>{T(0), d2};
  return k;
}

// pass 1: K^{mu nu} = S - S^+, S = sum_a ([g_mu, g_nu] X)_a (x) Y_a^+, for every site
template <typename T>
__global__ __launch_bounds__(kBlock) void wilson_clover_kernel(Geom g, const T* __restrict__ X,
                                                                const T* __restrict__ Y, T* __restrict__ K) {
  const long long idx = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= 2ll * g.Vh) return;
  const int p = (int)(idx / g.Vh), cb = (int)(idx - (long long)p * g.Vh);
  const spinor<T> x = load_spinor(X, p, g.Vh, cb);
  const spinor<T> y = load_spinor(Y, p, g.Vh, cb);
  spinor<T> gx[4];
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) gx[mu] = gamma_apply(mu, x);
#pragma unroll
  for (int mu = 0; mu < 4; ++mu)
#pragma unroll
    for (int nu = mu + 1; nu < 4; ++nu) {
      const spinor<T> a = gamma_apply(mu, gx[nu]), b = gamma_apply(nu, gx[mu]);
      spinor<T> cm;
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) cm.s[s][c] = cx<T>{a.s[s][c].re - b.s[s][c].re, a.s[s][c].im - b.s[s][c].im};
      const su3<T> S = outer(cm, y);
      su3<T> k;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const cx<T> sij = S.e[3 * i + j], sji = S.e[3 * j + i];
          k.e[3 * i + j] = cx<T>{sij.re - sji.re, sij.im + sji.im};
        }
      store_antiherm(K + (size_t)((p * 6 + pair_index(mu, nu)) * 9) * (size_t)g.Vh, g.Vh, cb, k);
    }
}

template <typename T>
struct WCtx {
  const T* U;
  const T* K;
  int Vh;
  int p;
  int ax[4];
  Nbr nb;

  template <int D0, int D1, int D2, int D3, int A>
  __device__ __forceinline__ su3<T> u() const {
    constexpr int dp = offset_parity<D0, D1, D2, D3>();
    return load_su3_rows(block_ptr(U, ax[A], p ^ dp, Vh), Vh, nbr_cb<D0, D1, D2, D3>(nb));
  }
  template <int D0, int D1, int D2, int D3>
  __device__ __forceinline__ su3<T> k(int pair) const {
    constexpr int dp = offset_parity<D0, D1, D2, D3>();
    return load_antiherm(K + (size_t)((((p ^ dp) * 6) + pair) * 9) * (size_t)Vh, Vh, nbr_cb<D0, D1, D2, D3>(nb));
  }
};

template <typename T>
__device__ __forceinline__ su3<T> dagger(const su3<T>& a) {
  su3<T> r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.e[3 * i + j] = cx<T>{a.e[3 * j + i].re, -a.e[3 * j + i].im};
  return r;
}

// acc += sigma (abd K0 + K1 abd + a K2 bd + ab K3 d) for the plaquette k, k+rho, k+rho+nu_s, k+nu_s
// with nu = ax[J], s = S
template <int J, int S, typename T>
__device__ __forceinline__ void clover_plaquette(su3<T>& acc, const WCtx<T>& c0) {
  WCtx<T> c = c0;
  asm volatile("" : "+s"(c.U), "+s"(c.K));
  constexpr int e1 = J == 1 ? 1 : 0, e2 = J == 2 ? 1 : 0, e3 = J == 3 ? 1 : 0;
  constexpr int f1 = S * e1, f2 = S * e2, f3 = S * e3;
  const int rho = c.ax[0], nu = c.ax[J];
  const int pair = rho < nu ? pair_index(rho, nu) : pair_index(nu, rho);
  const T sigma = T(S * (rho < nu ? 1 : -1));
  su3<T> a, d;
  if constexpr (S > 0) {
    a = c.template u<1, 0, 0, 0, J>();
    d = dagger(c.template u<0, 0, 0, 0, J>());
  } else {
    a = dagger(c.template u<1, -e1, -e2, -e3, J>());
    d = c.template u<0, -e1, -e2, -e3, J>();
  }
  const su3<T> b = dagger(c.template u<0, f1, f2, f3, 0>());
  const su3<T> abd = mul<false, false>(mul<false, false>(a, b), d);
  su3<T> t = mul<false, false>(abd, c.template k<0, 0, 0, 0>(pair));
  mac<false, false>(t, c.template k<1, 0, 0, 0>(pair), abd);
  // a K2 b d + a b K3 d = a (K2 b + b K3) d
  su3<T> x = mul<false, false>(c.template k<1, f1, f2, f3>(pair), b);
  mac<false, false>(x, b, c.template k<0, f1, f2, f3>(pair));
  mac<false, false>(t, mul<false, false>(a, x), d);
  axpy(acc, sigma, t);
}

// FP32: three waves per SIMD (168 VGPRs, 32 bytes of spills) instead of two at 175:
// 1.78 -> 1.70 ms at 32^3 x 64. FP64 keeps one wave (256 VGPRs and 93 AGPRs; two waves
// would spill 360 bytes).
template <typename T>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 1))) void wilson_force_kernel(Geom g, const T* __restrict__ U,
                                                               const T* __restrict__ X, const T* __restrict__ Y,
                                                               const T* __restrict__ K, T* __restrict__ out,
                                                               double kappa, double csw, int ntiles) {
  const LinkTile lt = link_tile(g, blockIdx.x, ntiles);
  const int cb = lt.chunk * kBlock + threadIdx.x;
  if (cb >= g.Vh) return;
  WCtx<T> c;
  {
    int x[4];
    cb_coords(g, lt.p, cb, x);
    c.U = U;
    c.K = K;
    c.Vh = g.Vh;
    c.p = lt.p;
    const int mu = lt.mu;
    c.ax[0] = mu;
    c.ax[1] = mu == 0 ? 1 : 0;
    c.ax[2] = mu <= 1 ? 2 : 1;
    c.ax[3] = mu <= 2 ? 3 : 2;
    Nbr full;
    make_nbr(g, x, full);
#pragma unroll
    for (int fa = 0; fa < 4; ++fa) {
      const int a = c.ax[fa];
#pragma unroll
      for (int dd = 0; dd < 5; ++dd)
        c.nb.o[fa][dd] = a == 0 ? full.o[0][dd] : a == 1 ? full.o[1][dd] : a == 2 ? full.o[2][dd] : full.o[3][dd];
    }
  }
  const int rho = lt.mu;

  // clover leaves through the link
  su3<T> acc;
  set_zero(acc);
  if (csw != 0.0) {
    clover_plaquette<1, 1>(acc, c);
    __builtin_amdgcn_sched_barrier(0);
    clover_plaquette<1, -1>(acc, c);
    __builtin_amdgcn_sched_barrier(0);
    clover_plaquette<2, 1>(acc, c);
    __builtin_amdgcn_sched_barrier(0);
    clover_plaquette<2, -1>(acc, c);
    __builtin_amdgcn_sched_barrier(0);
    clover_plaquette<3, 1>(acc, c);
    __builtin_amdgcn_sched_barrier(0);
    clover_plaquette<3, -1>(acc, c);
    __builtin_amdgcn_sched_barrier(0);
  }
  // M = U (-2 kappa B' + w acc) + 2 kappa C' U^+, w = -c_sw kappa / 8
  const int pr = lt.p ^ 1;
  const int cbr = nbr_cb<1, 0, 0, 0>(c.nb);
  const spinor<T> xk = load_spinor(X, lt.p, g.Vh, cb), yk = load_spinor(Y, lt.p, g.Vh, cb);
  const spinor<T> xr = load_spinor(X, pr, g.Vh, cbr), yr = load_spinor(Y, pr, g.Vh, cbr);
  const su3<T> Bp = outer(project(rho, -1, xr), yk);
  const su3<T> Cp = outer(xk, project(rho, 1, yr));
  const T w = T(-csw * kappa / 8.0), mk = T(-2.0 * kappa);
  su3<T> inner;
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    inner.e[e].re = fma(mk, Bp.e[e].re, w * acc.e[e].re);
    inner.e[e].im = fma(mk, Bp.e[e].im, w * acc.e[e].im);
  }
  const su3<T> u = c.template u<0, 0, 0, 0, 0>();
  su3<T> M = mul<false, false>(u, inner);
  su3<T> cu = mul<false, true>(Cp, u);
  axpy(M, T(2.0 * kappa), cu);
  store_link(block_ptr(out, rho, lt.p, g.Vh), g.Vh, cb, ta_scaled(M, T(-0.5)));
}

// canonical (Lt,Lz,Ly,Lx,4,3) complex <-> field[p][12][V/2]
template <typename T, bool PACK>
__global__ __launch_bounds__(kBlock) void spinor_layout_kernel(Geom g, const T* __restrict__ src,
                                                                T* __restrict__ dst) {
  const long long s = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (s >= 2ll * g.Vh) return;
  int r = (int)s;
  const int x = r % g.L[0];
  r /= g.L[0];
  const int y = r % g.L[1];
  r /= g.L[1];
  const int z = r % g.L[2];
  const int t = r / g.L[2];
  const int p = (x + y + z + t) & 1, cb = (int)(s >> 1);
  const cx<T>* a = reinterpret_cast<const cx<T>*>(src);
  cx<T>* b = reinterpret_cast<cx<T>*>(dst);
#pragma unroll
  for (int e = 0; e < 12; ++e) {
    const size_t soa = (size_t)(p * 12 + e) * (size_t)g.Vh + cb;
    const size_t aos = (size_t)s * 12 + e;
    if constexpr (PACK)
      b[soa] = a[aos];
    else
      b[aos] = a[soa];
  }
}

}  // namespace

template <typename T>
hipError_t launch_wilson_clover(const Geom& g, const T* X, const T* Y, T* K, hipStream_t s) {
  const long long n = 2ll * g.Vh;
  wilson_clover_kernel<T><<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(g, X, Y, K);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_wilson_force(const Geom& g, const T* U, const T* X, const T* Y, const T* K, T* out, double kappa,
                               double csw, hipStream_t s) {
  const int nt = link_tiles(g);
  wilson_force_kernel<T><<<nt, kBlock, 0, s>>>(g, U, X, Y, K, out, kappa, csw, nt);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_spinor_layout(const Geom& g, const T* src, T* dst, bool pack, hipStream_t s) {
  const long long n = 2ll * g.Vh;
  const unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
  if (pack)
    spinor_layout_kernel<T, true><<<blocks, kBlock, 0, s>>>(g, src, dst);
  else
    spinor_layout_kernel<T, false><<<blocks, kBlock, 0, s>>>(g, src, dst);
  return hipGetLastError();
}

#ifndef SYM_ONLY_F64
template hipError_t launch_wilson_clover<float>(const Geom&, const float*, const float*, float*, hipStream_t);
template hipError_t launch_wilson_force<float>(const Geom&, const float*, const float*, const float*, const float*,
                                               float*, double, double, hipStream_t);
template hipError_t launch_spinor_layout<float>(const Geom&, const float*, float*, bool, hipStream_t);
#endif
#ifndef SYM_ONLY_F32
template hipError_t launch_wilson_clover<double>(const Geom&, const double*, const double*, double*, hipStream_t);
template hipError_t launch_wilson_force<double>(const Geom&, const double*, const double*, const double*,
                                                const double*, double*, double, double, hipStream_t);
template hipError_t launch_spinor_layout<double>(const Geom&, const double*, double*, bool, hipStream_t);
#endif

}  // namespace sym
