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
// Pass FK1 writes T1 and the combinations inner = c5 U + c7 (T1_+ + T1_-), FK2 writes
// M_{nu,s} = midc_nu + cL T1_{nu,s}, FK3 V and the Naik link
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
//   X[mu][p][slot][9][V/2] complex: see struct Fields. Every linear combination a later
//   pass reads at several neighbours is stored once, so each transport loads one matrix
//   besides its two links.
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

// One matrix field (slot `slot` of a field with `nslot` matrices per link) on the links
// of direction ax[A]; the U field itself.
template <typename T>
struct One {
  const T* F[3];  // F[0] used; the array keeps the interface of Comb for fresh()
  int nslot;
  int slot;

  template <int D0, int D1, int D2, int D3, int A>
  __device__ __forceinline__ su3<T> at(const Ctx<T>& c) const {
    return c.template f<D0, D1, D2, D3, A>(F[0], nslot, slot);
  }
};

template <typename T>
__device__ __forceinline__ One<T> one(const T* F, int nslot, int slot) {
  One<T> o;
  o.F[0] = F;
  o.F[1] = nullptr;
  o.F[2] = nullptr;
  o.nslot = nslot;
  o.slot = slot;
  return o;
}

template <typename T>
struct UOnly {
  const T* F[3];  // unused

  template <int D0, int D1, int D2, int D3, int A>
  __device__ __forceinline__ su3<T> at(const Ctx<T>& c) const {
    return c.template u<D0, D1, D2, D3, A>();
  }
};

template <typename T>
__device__ __forceinline__ UOnly<T> u_only() {
  UOnly<T> o;
  o.F[0] = o.F[1] = o.F[2] = nullptr;
  return o;
}

// Workspace fields of one lattice (slot fields X[mu][p][slot][9][V/2]), with
// T1[2k + (s<0)] = Sts_{a_k}(U_mu) and gM[2k + (s<0)] = St-s_{a_k}(GV_mu) (a_k the k-th
// axis other than mu, ascending), which are not stored: the passes that need them at
// their own site multiply them out again (two products each).
//   inner[m] = c5 U_mu + c7 (T1[2m] + T1[2m+1])             (3 slots, FK1)
//   M[2k + (s<0)] = midc_k + cL T1[2k + (s<0)]              (6 slots, FK2)
//   gmid[k] = gM[2k] + gM[2k+1]                             (3 slots, BK3)
//   gT1[2m + (s<0)] = c7 g_inner_m + cL gM[2m + (s<0)]      (6 slots, BK2)
//   D = c1 GV + c3 sum_k gmid_k + c5 sum_m g_inner_m        (1 slot,  BK2)
// 19 matrices per link.
template <typename T>
struct Fields {
  T* inner;
  T* M;
  T* gmid;
  T* gT1;
  T* D;
};
constexpr int kFatFields = 19;

struct FatCoeffs {
  double c[6];  // c1, c3, c5, c7, cL, cN
};

template <typename T>
__device__ __forceinline__ void store_slot(T* F, int nslot, int slot, int dir, int p, int Vh, int cb, const su3<T>& m) {
  cx<T>* blk = reinterpret_cast<cx<T>*>(F) + (size_t)((((dir * 2) + p) * nslot + slot) * 9) * (size_t)Vh;
  store_link(blk, Vh, cb, m);
}

template <typename T>
__device__ __forceinline__ void scale(su3<T>& a, T s) {
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    a.e[e].re *= s;
    a.e[e].im *= s;
  }
}

// ------------------------------------------------------------------ forward

// FK1: inner[K-1] = c5 U + c7 (T1_{K,+} + T1_{K,-}) with T1_{K,s} = Sts_{ax[K]}(U_mu)
template <int K, typename T>
__device__ __forceinline__ void fk1_step(const Ctx<T>& c0, const Fields<T>& w, T c5, T c7, int cb) {
  if constexpr (K <= 3) {
    Ctx<T> c = c0;
    launder(c);
    const auto A = u_only<T>();
    su3<T> r;
    set_zero(r);
    st_acc<K, 1>(r, c, A);
    su3<T> in = c.template u<0, 0, 0, 0, 0>();
    scale(in, c5);
    axpy(in, c7, r);
    SYM_FAT_FENCE();
    set_zero(r);
    st_acc<K, -1>(r, c, A);
    axpy(in, c7, r);
    store_slot(w.inner, 3, K - 1, c.ax[0], c.p, c.Vh, cb, in);
    SYM_FAT_FENCE();
    fk1_step<K + 1>(c0, w, c5, c7, cb);
  }
}

// M[K, s] = midc_K + cL T1_{K,s}, with T1_{K,s} = Sts_{ax[K]}(U_mu) multiplied out again
// here (two products) rather than stored by FK1 and read back
template <int K, typename T>
__device__ __forceinline__ void store_m(const su3<T>& midc, const Ctx<T>& c0, const Fields<T>& w, T cL, int cb) {
  Ctx<T> c = c0;
  launder(c);
  const auto A = u_only<T>();
  su3<T> t;
  set_zero(t);
  st_acc<K, 1>(t, c, A);
  su3<T> m = midc;
  axpy(m, cL, t);
  store_slot(w.M, 6, 2 * (K - 1), c.ax[0], c.p, c.Vh, cb, m);
  SYM_FAT_FENCE();
  set_zero(t);
  st_acc<K, -1>(t, c, A);
  m = midc;
  axpy(m, cL, t);
  store_slot(w.M, 6, 2 * (K - 1) + 1, c.ax[0], c.p, c.Vh, cb, m);
}

// gT1[M, s] = c7 g_inner_M + cL gM[M, s], with gM[M, s] = St-s_{ax[M]}(GV_mu) multiplied
// out again here rather than stored by BK3 and read back
template <int M, typename T>
__device__ __forceinline__ void store_gt(const su3<T>& gi, const Ctx<T>& c0, const T* GV, const Fields<T>& w, T c7,
                                         T cL, int cb) {
  Ctx<T> c = c0;
  launder(c);
  const auto G = one(GV, 1, 0);
  su3<T> t;
  set_zero(t);
  st_acc<M, -1>(t, c, G);
  scale(t, cL);
  axpy(t, c7, gi);
  store_slot(w.gT1, 6, 2 * (M - 1), c.ax[0], c.p, c.Vh, cb, t);
  SYM_FAT_FENCE();
  set_zero(t);
  st_acc<M, 1>(t, c, G);
  scale(t, cL);
  axpy(t, c7, gi);
  store_slot(w.gT1, 6, 2 * (M - 1) + 1, c.ax[0], c.p, c.Vh, cb, t);
}

// FK3: V_mu = c1 U_mu + sum_{K,s} Sts_{ax[K]}(M[K, s])
template <int K, typename T>
__device__ __forceinline__ void fk3_step(su3<T>& acc, const Ctx<T>& c0, const Fields<T>& w) {
  if constexpr (K <= 3) {
    Ctx<T> c = c0;
    launder(c);
    st_acc<K, 1>(acc, c, one(static_cast<const T*>(w.M), 6, 2 * (K - 1)));
    SYM_FAT_FENCE();
    st_acc<K, -1>(acc, c, one(static_cast<const T*>(w.M), 6, 2 * (K - 1) + 1));
    SYM_FAT_FENCE();
    fk3_step<K + 1>(acc, c0, w);
  }
}

// ------------------------------------------------------------------ reverse

// BK3: gmid[K-1] = gM[K, +] + gM[K, -] with gM[K, S] = St-S_{ax[K]}(GV_mu)
template <int K, typename T>
__device__ __forceinline__ void bk3_step(const Ctx<T>& c0, const T* GV, const Fields<T>& w, int cb) {
  if constexpr (K <= 3) {
    Ctx<T> c = c0;
    launder(c);
    const auto G = one(GV, 1, 0);
    su3<T> r, gm;
    set_zero(r);
    st_acc<K, -1>(r, c, G);
    gm = r;
    SYM_FAT_FENCE();
    set_zero(r);
    st_acc<K, 1>(r, c, G);
    add(gm, r);
    store_slot(w.gmid, 3, K - 1, c.ax[0], c.p, c.Vh, cb, gm);
    SYM_FAT_FENCE();
    bk3_step<K + 1>(c0, GV, w, cb);
  }
}

// FK2: midc_K = c3 U_mu + sum_{J != K} sum_s Sts_{ax[J]}(inner[M]), M the third axis,
// stores M[K, s] = midc_K + cL T1[K, s] (store_m). BK2: g_inner_M = sum over (K, J)
// with {K, J, M} = {1, 2, 3} of sum_s Sts_{ax[J]}(gmid_K), stores gT1 (store_gt) and
// adds c5 g_inner_M into D.
// Both with the transport direction J outermost: each transport along
// ax[J] serves two outputs, so its four links (U_{x,J}, U_{x+mu,J}, U_{x-J,J},
// U_{x-J+mu,J}) are loaded once for both; the three accumulators stay in registers.
// acc[K-1] += sum_s Sts_{ax[J]}(F[slot(K)]) for the two K != J, where (K, J, M) is a
// permutation of (1, 2, 3) and the transported field is inner[M-1] (FK2: outputs
// midc_K) or gmid[K-1] into output g_inner_M (BK2, with the roles of K and M swapped).
template <int J, int K, bool BACK, typename T>
__device__ __forceinline__ void two_out_step(su3<T> (&acc)[3], const Ctx<T>& c, const T* F, const su3<T>& u0,
                                             const su3<T>& u1, const su3<T>& v0, const su3<T>& v1) {
  if constexpr (K <= 3) {
    if constexpr (K != J) {
      constexpr int M = 6 - K - J;
      constexpr int e1 = comp(1, J), e2 = comp(2, J), e3 = comp(3, J);
      // FK2: output midc_K from inner_M; BK2: output g_inner_M from gmid_K
      constexpr int out = BACK ? M - 1 : K - 1;
      constexpr int src = BACK ? K - 1 : M - 1;
      const su3<T> ap = c.template f<0, e1, e2, e3, 0>(F, 3, src);
      mac<false, true>(acc[out], mul<false, false>(u0, ap), u1);
      const su3<T> am = c.template f<0, -e1, -e2, -e3, 0>(F, 3, src);
      mac<false, false>(acc[out], mul<true, false>(v0, am), v1);
      SYM_FAT_FENCE();
    }
    two_out_step<J, K + 1, BACK>(acc, c, F, u0, u1, v0, v1);
  }
}

template <int J, bool BACK, typename T>
__device__ __forceinline__ void two_out(su3<T> (&acc)[3], const Ctx<T>& c0, const T* F) {
  if constexpr (J <= 3) {
    constexpr int e1 = comp(1, J), e2 = comp(2, J), e3 = comp(3, J);
    Ctx<T> c = c0;
    launder(c);
    asm volatile("" : "+s"(F));
    const su3<T> u0 = c.template u<0, 0, 0, 0, J>();              // U_{x,J}
    const su3<T> u1 = c.template u<1, 0, 0, 0, J>();              // U_{x+mu,J}
    const su3<T> v0 = c.template u<0, -e1, -e2, -e3, J>();        // U_{x-J,J}
    const su3<T> v1 = c.template u<1, -e1, -e2, -e3, J>();        // U_{x-J+mu,J}
    two_out_step<J, 1, BACK>(acc, c, F, u0, u1, v0, v1);
    two_out<J + 1, BACK>(acc, c0, F);
  }
}

// GK, transports of U_nu's own chain: St-S_{ax[M]}(gT1[M, S])
template <int M, typename T>
__device__ __forceinline__ void gk_pull(su3<T>& acc, const Ctx<T>& c0, const Fields<T>& w) {
  if constexpr (M <= 3) {
    Ctx<T> c = c0;
    launder(c);
    st_acc<M, -1>(acc, c, one(static_cast<const T*>(w.gT1), 6, 2 * (M - 1)));
    SYM_FAT_FENCE();
    st_acc<M, 1>(acc, c, one(static_cast<const T*>(w.gT1), 6, 2 * (M - 1) + 1));
    SYM_FAT_FENCE();
    gk_pull<M + 1>(acc, c0, w);
  }
}


// GK deposits on U_{y,nu} (nu = ax[0]) from the transports along nu in the chains of
// mu = ax[I]. A transport Sts_nu(A) with output gradient G deposits on its two outer
// links (derivation in the header comment)
//   s = +:  G_y U_{y+mu,nu} A_{y+nu}^dag + G_{y-mu}^dag U_{y-mu,nu} A_{y-mu+nu}
//   s = -:  A_y U_{y+mu,nu} G_{y+nu}^dag + A_{y-mu}^dag U_{y-mu,nu} G_{y-mu+nu}
// i.e. acc += X0 U_{y+mu,nu} Y0^dag + X1^dag U_{y-mu,nu} Y1 with (X0, X1, Y0, Y1) as
// above. Eight transports per mu: (GV, M[nu,s]) from V, (gmid_k, inner_m) from midc for
// the two k other than nu, (gT1[nu,s], U_mu) from T1. The two links are loaded once per
// mu; in FP32 the four matrices of the next transport are requested before the current
// one is multiplied out (FP64 keeps one transport at a time: with the look-ahead its
// operands overflow VGPRs and AGPRs, spill 48 bytes and measured 14.8 against 14.5 ms;
// loading the links once took its gather from 19.5 to 14.4 ms at 32^3 x 64, and FP32
// went from 8.5 to 7.0 ms).
template <typename T>
struct Dep {
  su3<T> x0, x1, y0, y1;
};

template <int I, int K, typename T>
__device__ __forceinline__ Dep<T> load_dep(const Ctx<T>& c0, const T* GV, const Fields<T>& w, int kn) {
  constexpr int e1 = comp(1, I), e2 = comp(2, I), e3 = comp(3, I);
  constexpr bool plus = (K % 2) == 0;
  Ctx<T> c = c0;
  launder(c);
  // fields of the K-th transport: K = 0,1: (GV, M[nu,s]); 2..5: (gmid[k], inner[m]);
  // 6,7: (gT1[nu,s], U_mu)
  const T* gf;
  int gn, gs;
  const T* af = nullptr;
  int an = 1, as = 0;
  if constexpr (K < 2) {
    gf = GV;
    gn = 1;
    gs = 0;
    af = w.M;
    an = 6;
    as = 2 * kn + (K & 1);
  } else if constexpr (K < 6) {
    const int j = (K - 2) / 2;  // j-th of the two axes other than mu and nu
    const int k = (j == 0) ? (kn == 0 ? 1 : 0) : (kn == 2 ? 1 : 2);
    gf = w.gmid;
    gn = 3;
    gs = k;
    af = w.inner;
    an = 3;
    as = 3 - k - kn;
  } else {
    gf = w.gT1;
    gn = 6;
    gs = 2 * kn + (K & 1);
  }
  asm volatile("" : "+s"(gf), "+s"(af));
  Dep<T> d;
  if constexpr (plus) {
    d.x0 = c.template f<0, 0, 0, 0, I>(gf, gn, gs);
    d.x1 = c.template f<0, -e1, -e2, -e3, I>(gf, gn, gs);
    if constexpr (K < 6) {
      d.y0 = c.template f<1, 0, 0, 0, I>(af, an, as);
      d.y1 = c.template f<1, -e1, -e2, -e3, I>(af, an, as);
    } else {
      d.y0 = c.template u<1, 0, 0, 0, I>();
      d.y1 = c.template u<1, -e1, -e2, -e3, I>();
    }
  } else {
    if constexpr (K < 6) {
      d.x0 = c.template f<0, 0, 0, 0, I>(af, an, as);
      d.x1 = c.template f<0, -e1, -e2, -e3, I>(af, an, as);
    } else {
      d.x0 = c.template u<0, 0, 0, 0, I>();
      d.x1 = c.template u<0, -e1, -e2, -e3, I>();
    }
    d.y0 = c.template f<1, 0, 0, 0, I>(gf, gn, gs);
    d.y1 = c.template f<1, -e1, -e2, -e3, I>(gf, gn, gs);
  }
  return d;
}

template <typename T>
__device__ __forceinline__ void use_dep(su3<T>& acc, const Dep<T>& d, const su3<T>& up, const su3<T>& um) {
  mac<false, true>(acc, mul<false, false>(d.x0, up), d.y0);
  mac<false, false>(acc, mul<true, false>(d.x1, um), d.y1);
}

template <int I, int K, typename T>
__device__ __forceinline__ void dep_pipe(su3<T>& acc, const Ctx<T>& c, const T* GV, const Fields<T>& w, int kn,
                                         const su3<T>& up, const su3<T>& um, const Dep<T>& d) {
  if constexpr (K < 7) {
    const Dep<T> dn = load_dep<I, K + 1>(c, GV, w, kn);
    SYM_FAT_FENCE();
    use_dep(acc, d, up, um);
    SYM_FAT_FENCE();
    dep_pipe<I, K + 1>(acc, c, GV, w, kn, up, um, dn);
  } else {
    use_dep(acc, d, up, um);
    SYM_FAT_FENCE();
  }
}

template <int I, int K, typename T>
__device__ __forceinline__ void dep_serial(su3<T>& acc, const Ctx<T>& c, const T* GV, const Fields<T>& w, int kn,
                                           const su3<T>& up, const su3<T>& um) {
  if constexpr (K < 8) {
    const Dep<T> d = load_dep<I, K>(c, GV, w, kn);
    use_dep(acc, d, up, um);
    SYM_FAT_FENCE();
    dep_serial<I, K + 1>(acc, c, GV, w, kn, up, um);
  }
}

// The same deposits without the look-ahead (FP64: no registers for two transports).
template <int I, typename T>
__device__ __forceinline__ void gk_factor_links_once(su3<T>& acc, const Ctx<T>& c0, const T* GV,
                                                     const Fields<T>& w) {
  if constexpr (I <= 3) {
    constexpr int e1 = comp(1, I), e2 = comp(2, I), e3 = comp(3, I);
    const int mu = c0.ax[I], nu = c0.ax[0];
    const int kn = nu < mu ? nu : nu - 1;
    Ctx<T> c = c0;
    launder(c);
    const su3<T> up = c.template u<0, e1, e2, e3, 0>();
    const su3<T> um = c.template u<0, -e1, -e2, -e3, 0>();
    SYM_FAT_FENCE();
    dep_serial<I, 0>(acc, c, GV, w, kn, up, um);
    gk_factor_links_once<I + 1>(acc, c0, GV, w);
  }
}

template <int I, typename T>
__device__ __forceinline__ void gk_factor_pipe(su3<T>& acc, const Ctx<T>& c0, const T* GV, const Fields<T>& w) {
  if constexpr (I <= 3) {
    constexpr int e1 = comp(1, I), e2 = comp(2, I), e3 = comp(3, I);
    const int mu = c0.ax[I], nu = c0.ax[0];
    const int kn = nu < mu ? nu : nu - 1;
    Ctx<T> c = c0;
    launder(c);
    const su3<T> up = c.template u<0, e1, e2, e3, 0>();     // U_{y+mu,nu}
    const su3<T> um = c.template u<0, -e1, -e2, -e3, 0>();  // U_{y-mu,nu}
    const Dep<T> d0 = load_dep<I, 0>(c, GV, w, kn);
    SYM_FAT_FENCE();
    dep_pipe<I, 0>(acc, c, GV, w, kn, up, um, d0);
    gk_factor_pipe<I + 1>(acc, c0, GV, w);
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
