// Fat-link smearing of the asqtad / HISQ actions and its path force: device code.
//
// arXiv:1808.02281, Sec. "Asqtad fermion" (fat link V of eq. 18_6_6_7_2 with the
// Lepage term of eq. 18_6_6_7, Naik term eq. 18_6_6_3) and Sec. "HISQ fermion"
// (the pull-back F~ of eq. 18_7_24_7 and B = U F~^T of eq. 18_7_24_6).
//
// The 85 smearing paths from x to x+mu are not multiplied out one by one. With the
// staple transport along a direction nu perpendicular to mu, for a matrix field A
// living on the mu links,
//   St+_nu(A)_x = U_{x,nu} A_{x+nu} U_{x+mu,nu}^dagger,
//   St-_nu(A)_x = U_{x-nu,nu}^dagger A_{x-nu} U_{x-nu+mu,nu},
// every path class is a nested transport of U_mu:
//   three-staple St_nu(U), five-staple St_nu(St_rho(U)), seven-staple
//   St_nu(St_rho(St_sigma(U))) (nu, rho, sigma distinct), Lepage St+-_nu(St+-_nu(U))
//   (same sign twice). Summing inside out,
//   V_mu = c1 U_mu + sum_{nu, s} Sts_nu( midc_nu + cL T1_{nu,s} ),
//   midc_nu = c3 U_mu + sum_{rho != nu} sum_s Sts_rho( c5 U_mu + c7 (T1_{sigma,+} + T1_{sigma,-}) ),
//   T1_{sigma,s} = Sts_sigma(U_mu),   sigma the axis other than mu, nu, rho.
// Pass FK1 writes T1 (6 per link), FK2 midc (3 per link), FK3 V and the Naik link
// W = cN U_{x,mu} U_{x+mu,mu} U_{x+2mu,mu}: 12 + 24 + 14 products per link, against
// 505 link positions over the 86 paths.
//
// Reverse pass for Phi = Re sum tr(GV^dagger V) + Re sum tr(GW^dagger W), gradients
// in the convention dPhi = Re sum tr(grad^dagger dU):
//   the gradient of the transported field is the opposite transport of the output
//   gradient, grad(A) += St-s_nu(Gamma) for every St s_nu(A) (BK3: gM = St-s_nu(GV);
//   BK2: g_inner_sigma = sum St_rho(gmid_nu)); each transport also deposits on its two
//   outer links (s = +: U_{x,nu}, U_{x+mu,nu}; s = -: U_{x-nu,nu}, U_{x-nu+mu,nu})
//     s = +:  Gamma_y U_{y+mu,nu} A_{y+nu}^dagger + Gamma_{y-mu}^dagger U_{y-mu,nu} A_{y-mu+nu}
//     s = -:  A_y U_{y+mu,nu} Gamma_{y+nu}^dagger + A_{y-mu}^dagger U_{y-mu,nu} Gamma_{y-mu+nu}
//   gathered per receiving link (y, nu) in GK together with the direct terms of U_nu.
// Everything is a gather: each thread owns its output, no atomics.
//
// Intermediate fields (workspace), per direction mu and parity, "slot fields"
//   X[mu][p][slot][9][V/2] complex:  T1 6 slots (slot 2k + (s<0), k = index of sigma
//   among the axes other than mu, ascending), midc 3, gM 6, g_inner 3.
#pragma once

#include "kernels.hpp"

namespace sym {
namespace fat {

#define SYM_FAT_FENCE() __builtin_amdgcn_sched_barrier(0)

constexpr int comp(int fa, int which) { return fa == which ? 1 : 0; }

template <typename T>
struct Ctx {
  const T* U;
  int Vh;
  int p;
  int ax[4];  // ax[0]: the thread's direction; ax[1..3]: the other axes ascending
  Nbr nb;     // neighbour offsets, rows in frame order

  // U_{x+D, ax[A]}
  template <int D0, int D1, int D2, int D3, int A>
  __device__ __forceinline__ su3<T> u() const {
    constexpr int dp = offset_parity<D0, D1, D2, D3>();
    return load_link(block_ptr(U, ax[A], p ^ dp, Vh), Vh, nbr_cb<D0, D1, D2, D3>(nb));
  }

  // slot `slot` of a field with `nslot` matrices per link, direction ax[A], at x+D
  template <int D0, int D1, int D2, int D3, int A>
  __device__ __forceinline__ su3<T> f(const T* F, int nslot, int slot) const {
    constexpr int dp = offset_parity<D0, D1, D2, D3>();
    const cx<T>* blk =
        reinterpret_cast<const cx<T>*>(F) + (size_t)((((ax[A] * 2) + (p ^ dp)) * nslot + slot) * 9) * (size_t)Vh;
    return load_link(blk, Vh, nbr_cb<D0, D1, D2, D3>(nb));
  }
};

template <typename T>
__device__ __forceinline__ void make_ctx(const Geom& g, const T* U, int mu, int p, int cb, Ctx<T>& c) {
  int x[4];
  cb_coords(g, p, cb, x);
  c.U = U;
  c.Vh = g.Vh;
  c.p = p;
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
    for (int d = 0; d < 5; ++d)
      c.nb.o[fa][d] = a == 0 ? full.o[0][d] : a == 1 ? full.o[1][d] : a == 2 ? full.o[2][d] : full.o[3][d];
  }
}

template <typename T>
__device__ __forceinline__ void launder(Ctx<T>& c) {
  asm volatile("" : "+s"(c.U));
}

// Linear combination [wu U] + sum_j w_j F_j[slot_j] of matrices living on the links of
// direction ax[A] (n <= 3 fields; all weights and slots wave-uniform). Whether the U
// term is present is a compile-time property (HU), so that no branch separates the
// loads from the arithmetic.
template <typename T, bool HU>
struct Comb {
  const T* F[3];
  int nslot[3];
  int slot[3];
  T w[3];
  int n;
  T wu;

  template <int D0, int D1, int D2, int D3, int A>
  __device__ __forceinline__ su3<T> at(const Ctx<T>& c) const {
    su3<T> r;
    if constexpr (HU) {
      r = c.template u<D0, D1, D2, D3, A>();
#pragma unroll
      for (int e = 0; e < 9; ++e) {
        r.e[e].re *= wu;
        r.e[e].im *= wu;
      }
    } else {
      set_zero(r);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (j < n) axpy(r, w[j], c.template f<D0, D1, D2, D3, A>(F[j], nslot[j], slot[j]));
    return r;
  }
};

template <typename T, bool HU>
__device__ __forceinline__ Comb<T, HU> make_comb(T wu) {
  Comb<T, HU> k;
  k.n = 0;
  k.wu = wu;
  for (int j = 0; j < 3; ++j) {
    k.F[j] = nullptr;
    k.nslot[j] = 1;
    k.slot[j] = 0;
    k.w[j] = T(0);
  }
  return k;
}

// U alone / U times wu plus fields / fields only
template <typename T>
__device__ __forceinline__ Comb<T, true> comb_u(T wu) { return make_comb<T, true>(wu); }
template <typename T>
__device__ __forceinline__ Comb<T, false> comb_f() { return make_comb<T, false>(T(0)); }

// Opaque copies of the field pointers: keeps the compiler from merging (and keeping
// alive) loads of the same matrices made in different transports.
template <typename C>
__device__ __forceinline__ C fresh(const C& k) {
  C r = k;
  asm volatile("" : "+s"(r.F[0]), "+s"(r.F[1]), "+s"(r.F[2]));
  return r;
}

template <typename C, typename T>
__device__ __forceinline__ void comb_add(C& k, const T* F, int nslot, int slot, T w) {
  k.F[k.n] = F;
  k.nslot[k.n] = nslot;
  k.slot[k.n] = slot;
  k.w[k.n] = w;
  ++k.n;
}

// acc += St^S_{ax[K]}(A)_x for A on the links of direction ax[0]
template <int K, int S, typename T, typename C>
__device__ __forceinline__ void st_acc(su3<T>& acc, const Ctx<T>& c, const C& A0) {
  constexpr int e1 = comp(1, K), e2 = comp(2, K), e3 = comp(3, K);
  const C A = fresh(A0);
  if constexpr (S > 0) {
    const su3<T> m = mul<false, false>(c.template u<0, 0, 0, 0, K>(), A.template at<0, e1, e2, e3, 0>(c));
    mac<false, true>(acc, m, c.template u<1, 0, 0, 0, K>());
  } else {
    const su3<T> m = mul<true, false>(c.template u<0, -e1, -e2, -e3, K>(), A.template at<0, -e1, -e2, -e3, 0>(c));
    mac<false, false>(acc, m, c.template u<1, -e1, -e2, -e3, K>());
  }
}

// acc += the two outer-link deposits on U_{y, ax[0]} of St^S_{ax[0]}(A) on the links of
// direction ax[I] with output gradient G (both fields of direction ax[I]).
template <int I, int S, typename T, typename CG, typename CA>
__device__ __forceinline__ void factor_acc(su3<T>& acc, const Ctx<T>& c, const CG& G0, const CA& A0) {
  constexpr int e1 = comp(1, I), e2 = comp(2, I), e3 = comp(3, I);
  const CG G = fresh(G0);
  const CA A = fresh(A0);
  if constexpr (S > 0) {
    // G_y U_{y+mu,nu} A_{y+nu}^dagger + G_{y-mu}^dagger U_{y-mu,nu} A_{y-mu+nu}
    const su3<T> m1 = mul<false, false>(G.template at<0, 0, 0, 0, I>(c), c.template u<0, e1, e2, e3, 0>());
    mac<false, true>(acc, m1, A.template at<1, 0, 0, 0, I>(c));
    const su3<T> m2 = mul<true, false>(G.template at<0, -e1, -e2, -e3, I>(c), c.template u<0, -e1, -e2, -e3, 0>());
    mac<false, false>(acc, m2, A.template at<1, -e1, -e2, -e3, I>(c));
  } else {
    // A_y U_{y+mu,nu} G_{y+nu}^dagger + A_{y-mu}^dagger U_{y-mu,nu} G_{y-mu+nu}
    const su3<T> m1 = mul<false, false>(A.template at<0, 0, 0, 0, I>(c), c.template u<0, e1, e2, e3, 0>());
    mac<false, true>(acc, m1, G.template at<1, 0, 0, 0, I>(c));
    const su3<T> m2 = mul<true, false>(A.template at<0, -e1, -e2, -e3, I>(c), c.template u<0, -e1, -e2, -e3, 0>());
    mac<false, false>(acc, m2, G.template at<1, -e1, -e2, -e3, I>(c));
  }
}

// Workspace fields of one lattice (slot fields, see the header comment).
template <typename T>
struct Fields {
  T* T1;     // 6 slots
  T* midc;   // 3 slots
  T* gM;     // 6 slots
  T* ginner; // 3 slots
};

struct FatCoeffs {
  double c[6];  // c1, c3, c5, c7, cL, cN
};

template <typename T>
__device__ __forceinline__ void store_slot(T* F, int nslot, int slot, int dir, int p, int Vh, int cb, const su3<T>& m) {
  cx<T>* blk = reinterpret_cast<cx<T>*>(F) + (size_t)((((dir * 2) + p) * nslot + slot) * 9) * (size_t)Vh;
  store_link(blk, Vh, cb, m);
}

// ------------------------------------------------------------------ forward

// FK1: T1[mu][2(K-1) + (S<0)] = St^S_{ax[K]}(U_mu)
template <int K, typename T>
__device__ __forceinline__ void fk1_step(const Ctx<T>& c0, T* T1, int cb) {
  if constexpr (K <= 3) {
    Ctx<T> c = c0;
    launder(c);
    const auto A = comb_u<T>(T(1));
    su3<T> r;
    set_zero(r);
    st_acc<K, 1>(r, c, A);
    store_slot(T1, 6, 2 * (K - 1), c.ax[0], c.p, c.Vh, cb, r);
    SYM_FAT_FENCE();
    set_zero(r);
    st_acc<K, -1>(r, c, A);
    store_slot(T1, 6, 2 * (K - 1) + 1, c.ax[0], c.p, c.Vh, cb, r);
    SYM_FAT_FENCE();
    fk1_step<K + 1>(c0, T1, cb);
  }
}

// FK2, one output: midc[mu][K-1] = c3 U_mu + sum_{J != K} sum_s Sts_{ax[J]}(c5 U_mu + c7 (T1_{M,+} + T1_{M,-}))
template <int K, int J, typename T>
__device__ __forceinline__ void fk2_inner(su3<T>& acc, const Ctx<T>& c0, const T* T1, T c5, T c7) {
  if constexpr (J <= 3) {
    if constexpr (J != K) {
      Ctx<T> c = c0;
      launder(c);
      constexpr int M = 6 - K - J;
      auto A = comb_u<T>(c5);
      comb_add(A, T1, 6, 2 * (M - 1), c7);
      comb_add(A, T1, 6, 2 * (M - 1) + 1, c7);
      st_acc<J, 1>(acc, c, A);
      SYM_FAT_FENCE();
      st_acc<J, -1>(acc, c, A);
      SYM_FAT_FENCE();
    }
    fk2_inner<K, J + 1>(acc, c0, T1, c5, c7);
  }
}

template <int K, typename T>
__device__ __forceinline__ void fk2_step(const Ctx<T>& c0, const T* T1, T* midc, const FatCoeffs& cf, int cb) {
  if constexpr (K <= 3) {
    su3<T> acc = c0.template u<0, 0, 0, 0, 0>();
    const T c3 = T(cf.c[1]);
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      acc.e[e].re *= c3;
      acc.e[e].im *= c3;
    }
    fk2_inner<K, 1>(acc, c0, T1, T(cf.c[2]), T(cf.c[3]));
    store_slot(midc, 3, K - 1, c0.ax[0], c0.p, c0.Vh, cb, acc);
    fk2_step<K + 1>(c0, T1, midc, cf, cb);
  }
}

// FK3: V_mu = c1 U_mu + sum_{K,s} Sts_{ax[K]}(midc_K + cL T1_{K,s})
template <int K, typename T>
__device__ __forceinline__ void fk3_step(su3<T>& acc, const Ctx<T>& c0, const T* T1, const T* midc, T cL) {
  if constexpr (K <= 3) {
    Ctx<T> c = c0;
    launder(c);
    auto Ap = comb_f<T>();
    comb_add(Ap, midc, 3, K - 1, T(1));
    comb_add(Ap, T1, 6, 2 * (K - 1), cL);
    st_acc<K, 1>(acc, c, Ap);
    SYM_FAT_FENCE();
    auto Am = comb_f<T>();
    comb_add(Am, midc, 3, K - 1, T(1));
    comb_add(Am, T1, 6, 2 * (K - 1) + 1, cL);
    st_acc<K, -1>(acc, c, Am);
    SYM_FAT_FENCE();
    fk3_step<K + 1>(acc, c0, T1, midc, cL);
  }
}

// ------------------------------------------------------------------ reverse

// BK3: gM[mu][2(K-1) + (S<0)] = St^{-S}_{ax[K]}(GV_mu)
template <int K, typename T>
__device__ __forceinline__ void bk3_step(const Ctx<T>& c0, const T* GV, T* gM, int cb) {
  if constexpr (K <= 3) {
    Ctx<T> c = c0;
    launder(c);
    auto G = comb_f<T>();
    comb_add(G, GV, 1, 0, T(1));
    su3<T> r;
    set_zero(r);
    st_acc<K, -1>(r, c, G);
    store_slot(gM, 6, 2 * (K - 1), c.ax[0], c.p, c.Vh, cb, r);
    SYM_FAT_FENCE();
    set_zero(r);
    st_acc<K, 1>(r, c, G);
    store_slot(gM, 6, 2 * (K - 1) + 1, c.ax[0], c.p, c.Vh, cb, r);
    SYM_FAT_FENCE();
    bk3_step<K + 1>(c0, GV, gM, cb);
  }
}

// BK2: g_inner[mu][M-1] = sum_{(K,J): {K,J,M} = {1,2,3}} sum_s Sts_{ax[J]}(gM_{K,+} + gM_{K,-})
template <int M, int K, typename T>
__device__ __forceinline__ void bk2_inner(su3<T>& acc, const Ctx<T>& c0, const T* gM) {
  if constexpr (K <= 3) {
    if constexpr (K != M) {
      constexpr int J = 6 - K - M;
      Ctx<T> c = c0;
      launder(c);
      auto G = comb_f<T>();
      comb_add(G, gM, 6, 2 * (K - 1), T(1));
      comb_add(G, gM, 6, 2 * (K - 1) + 1, T(1));
      st_acc<J, 1>(acc, c, G);
      SYM_FAT_FENCE();
      st_acc<J, -1>(acc, c, G);
      SYM_FAT_FENCE();
    }
    bk2_inner<M, K + 1>(acc, c0, gM);
  }
}

template <int M, typename T>
__device__ __forceinline__ void bk2_step(const Ctx<T>& c0, const T* gM, T* ginner, int cb) {
  if constexpr (M <= 3) {
    su3<T> acc;
    set_zero(acc);
    bk2_inner<M, 1>(acc, c0, gM);
    store_slot(ginner, 3, M - 1, c0.ax[0], c0.p, c0.Vh, cb, acc);
    bk2_step<M + 1>(c0, gM, ginner, cb);
  }
}

// GK, transports into U_nu (nu = ax[0]) as the transported field: St^{-S}_{ax[M]}(gT1_{M,S})
// with gT1_{M,S} = c7 g_inner_M + cL gM_{M,S}
template <int M, typename T>
__device__ __forceinline__ void gk_pull(su3<T>& acc, const Ctx<T>& c0, const Fields<T>& w, T c7, T cL) {
  if constexpr (M <= 3) {
    Ctx<T> c = c0;
    launder(c);
    auto Gp = comb_f<T>();
    comb_add(Gp, w.ginner, 3, M - 1, c7);
    comb_add(Gp, w.gM, 6, 2 * (M - 1), cL);
    st_acc<M, -1>(acc, c, Gp);
    SYM_FAT_FENCE();
    auto Gm = comb_f<T>();
    comb_add(Gm, w.ginner, 3, M - 1, c7);
    comb_add(Gm, w.gM, 6, 2 * (M - 1) + 1, cL);
    st_acc<M, 1>(acc, c, Gm);
    SYM_FAT_FENCE();
    gk_pull<M + 1>(acc, c0, w, c7, cL);
  }
}

// GK, deposits on U_{y,nu} from the transports along nu in the chains of mu = ax[I].
template <int I, typename T>
__device__ __forceinline__ void gk_factor(su3<T>& acc, const Ctx<T>& c0, const T* GV, const Fields<T>& w,
                                          const FatCoeffs& cf) {
  if constexpr (I <= 3) {
    const int mu = c0.ax[I], nu = c0.ax[0];
    const int kn = nu < mu ? nu : nu - 1;  // index of nu among the axes other than mu
    const T c5 = T(cf.c[2]), c7 = T(cf.c[3]), cL = T(cf.c[4]);
    {
      // V_mu = ... + Sts_nu(midc_nu + cL T1_{nu,s}) with gradient GV_mu
      Ctx<T> c = c0;
      launder(c);
      auto G = comb_f<T>();
      comb_add(G, GV, 1, 0, T(1));
      auto Ap = comb_f<T>();
      comb_add(Ap, w.midc, 3, kn, T(1));
      comb_add(Ap, w.T1, 6, 2 * kn, cL);
      factor_acc<I, 1>(acc, c, G, Ap);
      SYM_FAT_FENCE();
      auto Am = comb_f<T>();
      comb_add(Am, w.midc, 3, kn, T(1));
      comb_add(Am, w.T1, 6, 2 * kn + 1, cL);
      factor_acc<I, -1>(acc, c, G, Am);
      SYM_FAT_FENCE();
    }
    for (int k = 0; k < 3; ++k) {
      if (k == kn) continue;
      // midc_k = ... + Sts_nu(c5 U_mu + c7 (T1_{m,+} + T1_{m,-})) with gradient gmid_k
      const int m = 3 - k - kn;
      Ctx<T> c = c0;
      launder(c);
      auto G = comb_f<T>();
      comb_add(G, w.gM, 6, 2 * k, T(1));
      comb_add(G, w.gM, 6, 2 * k + 1, T(1));
      auto A = comb_u<T>(c5);
      comb_add(A, w.T1, 6, 2 * m, c7);
      comb_add(A, w.T1, 6, 2 * m + 1, c7);
      factor_acc<I, 1>(acc, c, G, A);
      SYM_FAT_FENCE();
      factor_acc<I, -1>(acc, c, G, A);
      SYM_FAT_FENCE();
    }
    {
      // T1_{nu,s} = Sts_nu(U_mu) with gradient gT1_{nu,s} = c7 g_inner_nu + cL gM_{nu,s}
      Ctx<T> c = c0;
      launder(c);
      const auto A = comb_u<T>(T(1));
      auto Gp = comb_f<T>();
      comb_add(Gp, w.ginner, 3, kn, c7);
      comb_add(Gp, w.gM, 6, 2 * kn, cL);
      factor_acc<I, 1>(acc, c, Gp, A);
      SYM_FAT_FENCE();
      auto Gm = comb_f<T>();
      comb_add(Gm, w.ginner, 3, kn, c7);
      comb_add(Gm, w.gM, 6, 2 * kn + 1, cL);
      factor_acc<I, -1>(acc, c, Gm, A);
      SYM_FAT_FENCE();
    }
    gk_factor<I + 1>(acc, c0, GV, w, cf);
  }
}

}  // namespace fat
}  // namespace sym

namespace sym {

// Last pass of the fat links: V and Naik links W (W may be null) from T1 and midc
// (stages 0 and 1 below).
template <typename T>
hipError_t launch_fat_fk3(const Geom& g, const T* U, T* V, T* W, const fat::FatCoeffs& c, const fat::Fields<T>& w,
                            hipStream_t s);
// One pass of the path force: 0 FK1 (T1), 1 FK2 (midc), 2 BK3 (gM), 3 BK2 (g_inner),
// 4 GK (out: gradient for mode 0, force for mode 1). GW may be null (no Naik term).
template <typename T>
hipError_t launch_fat_stage(int stage, const Geom& g, const T* U, const T* GV, const T* GW, T* out, int mode,
                            const fat::FatCoeffs& c, const fat::Fields<T>& w, hipStream_t s);

}  // namespace sym
