// Factored gauge force: device code shared by the single-lattice kernels
// (force_factored.hip) and the batched kernels (force_batch.hip).
//
// Same result as the direct form (every staple of arXiv:1808.02281 Sec. II,
// eq. 18_7_25_2), with rectangle and cube staples assembled from plaquette staples
// instead of multiplied out link by link.
//
// Notation: U_{y,d} for a signed direction d is the link matrix of the step y -> y+d
// (U_{y,-nu} = U_{y-nu,nu}^dagger). For the link at y in signed direction d and a
// signed direction e perpendicular to it,
//   S(y, d, e) = U_{y+d, e} U_{y+d+e, -d} U_{y+e, -e}
// is the plaquette staple (path e, -d, -e from y+d back to y); S(y, -nu, e) =
// S(y-nu, nu, e)^dagger. Inserting U^dagger U = 1 along the paths gives, for the 42
// five-link staples of link (x, mu):
//   rectangles, link first on the long side:  U_{x+mu,mu} S(x+mu,mu,e) S(x,mu,e)
//   rectangles, link second on the long side: S(x,mu,e) S(x-mu,mu,e) U_{x-mu,mu}
//   rectangles with the link as short side:   U_{x+mu,f} S(x+f,mu,f) U_{x+f,-f}
//   cube loop (mu, e, f, -mu, -e, -f), two ways:
//     A: U_{x+mu,e} S(x+e,mu,f) S(x,e,f)
//     B: S(x+mu,f,e)^dagger S(x+f,mu,e) U_{x+f,-f}
// Forms A of cube (f, e) and B of cube (e, f) share the middle staple S(x+f, mu, e).
// Pass 2 takes, for every f (6 signed directions) and the two e along the next frame
// axis (cyclically), cube (f, e) in form A and cube (e, f) in form B; this covers each
// of the 24 cube loops once (every unordered pair {e, f} once) and loads 36 staples for
// them instead of 48, at the price of a second outer product per f:
//   t += U_{x+mu,f} [c_R S(x+f,mu,f) U_{x+f,-f} + c_C QA_f] + c_C QB_f U_{x+f,-f},
//   QA_f = sum_e S(x+f,mu,e) S(x,f,e),   QB_f = sum_e S(x+mu,f,e)^dagger S(x+f,mu,e).
// The pass is bound by the bytes its loads move through the caches (its vector memory
// unit is busier than its ALUs), so trading six products per link for twelve staple
// loads makes it faster: 2.79 -> 2.48 ms (FP32) and 6.55 -> 5.53 ms (FP64) on the
// 32^3 x 64 workload.
//
// Pass 1 (staples_site) writes the 24 staples S(x, mu, e) of the four links of every
// site, one thread per site: the two staples S(x,mu,+a) = m U_{x,a}^dagger and
// S(x,a,+mu) = m^dagger U_{x,mu}^dagger of the plaquette at x in the plane (mu, a)
// share m = U_{x+mu,a} U_{x+a,mu}^dagger, and the links at x and x-a serve several
// staples, so a site loads 44 links instead of 72 (one thread per link) and forms the
// staples with 42 products instead of 48. Each thread writes only its own site.
// Pass 2 (factored_link) reads them and forms
//   t = c_P sum_e S + c_R (long-side rect sums) + (c_R short-side rect + c_C cube sums).
//
// Action: per link the kernel emits three deficit sums
//   a1 = 18 - Re tr(U t_P), a2 = 36 - Re tr(U t_RA+RB), a3 = 18 c_R + 72 c_C - Re tr(U t_mix)
// (t_mix = short-side rectangles weighted c_R plus cubes weighted c_C). Every
// rectangle is seen from its 4 long-side links in a2 and from its 2 short-side links
// in a3, every cube loop from its 6 links, every plaquette from its 4: see the final
// reduction (kind 2) in action.hip.
//
// Staple storage: S8[mu][p][slot][6][V/2 + pad] complex, slot = 2*axis(e) + (e < 0);
// the two slots with axis(e) = mu are never touched. In FP32 the six element planes of
// a block are stored as three planes of element pairs (e[2q], e[2q+1]), 16 bytes per
// site, so that a staple is three 16-byte loads per lane instead of six 8-byte ones.
// A staple is a product of three SU(3) links, hence itself in SU(3): only its first two
// rows are stored and the third is rebuilt on load (lattice.hpp), which cuts the staple
// traffic by a third. This relies on the links being special unitary to working
// precision.
#pragma once

#include "kernels.hpp"

namespace sym {
namespace factored {

// Scheduling fence between the groups of loads and products below: keeps the
// scheduler from hoisting every load of the kernel to the top (which costs occupancy).
#define SYM_FENCE() __builtin_amdgcn_sched_barrier(0)

// Frame: axis[0] = mu (the link's direction), axis[1..3] = the other axes ascending.
__device__ __forceinline__ void make_frame(const Geom& g, int mu, const int x[4], int axis[4], Nbr& nb) {
  axis[0] = mu;
  axis[1] = mu == 0 ? 1 : 0;
  axis[2] = mu <= 1 ? 2 : 1;
  axis[3] = mu <= 2 ? 3 : 2;
  Nbr full;
  make_nbr(g, x, full);
#pragma unroll
  for (int fa = 0; fa < 4; ++fa) {
    const int a = axis[fa];
#pragma unroll
    for (int d = 0; d < 5; ++d)
      nb.o[fa][d] = a == 0 ? full.o[0][d] : a == 1 ? full.o[1][d] : a == 2 ? full.o[2][d] : full.o[3][d];
  }
}

// Signed direction e_J, J = 0..5: frame axis 1 + J/2, sign + for even J.
constexpr int e_axis(int J) { return 1 + J / 2; }
constexpr int e_sign(int J) { return (J & 1) ? -1 : 1; }
constexpr int comp(int fa, int which) { return fa == which ? 1 : 0; }

// First two rows of a special-unitary matrix (see load_su3_rows); full() rebuilds it.
template <typename T>
struct Rows2 {
  cx<T> e[6];
};

template <typename T>
__device__ __forceinline__ su3<T> full(const Rows2<T>& r) {
  su3<T> u;
#pragma unroll
  for (int c = 0; c < 6; ++c) u.e[c] = r.e[c];
  complete_third_row(u);
  return u;
}

// Two adjacent complex elements: the unit of the FP32 staple loads and stores. Whole
// 16-byte buffer-load results are bit-cast into it: indexing the builtin's vector
// result element by element was compiled into a single dword load whose value stood
// for all four elements.
template <typename T>
struct CxPair {
  cx<T> a, b;
};
using U32x4 = __attribute__((ext_vector_type(4))) unsigned;

template <typename T>
struct FCtx {
  const T* U;
  const T* S8;
  int Vh;
  int Ss;  // plane stride of S8 (complex elements)
  int p;
  int axis[4];
  Nbr nb;

  // the first two rows of U_{x+d, axis[AX]} (a third less link traffic than all nine
  // elements), loaded only: full() rebuilds the third where the link is used, so that the
  // loads can be issued ahead of their use like the staples'
  template <int D0, int D1, int D2, int D3, int AX>
  __device__ __forceinline__ Rows2<T> link_rows() const {
    constexpr int dp = offset_parity<D0, D1, D2, D3>();
    const cx<T>* blk = block_ptr(U, axis[AX], p ^ dp, Vh);
    const unsigned bytes = 6u * (unsigned)Vh * (unsigned)sizeof(cx<T>);
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<cx<T>*>(blk), (short)0, (int)bytes, kBufferWord3);
    const int voff = nbr_cb<D0, D1, D2, D3>(nb) * (int)sizeof(cx<T>);
    Rows2<T> u;
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const int soff = (int)((unsigned)e * (unsigned)Vh * (unsigned)sizeof(cx<T>));
      if constexpr (sizeof(T) == 4)
        u.e[e] = __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
      else
        u.e[e] = __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    }
    return u;
  }

  // the first two rows of S(x+d, axis[AX], e), e = sign ES along frame axis EAX, loaded
  // only (the third row is rebuilt where the matrix is used, so that the loads can be
  // issued well ahead of their use)
  template <int D0, int D1, int D2, int D3, int AX, int EAX, int ES>
  __device__ __forceinline__ Rows2<T> stap_rows() const {
    constexpr int dp = offset_parity<D0, D1, D2, D3>();
    const int slot = 2 * axis[EAX] + (ES < 0 ? 1 : 0);
    const cx<T>* blk = reinterpret_cast<const cx<T>*>(S8) +
                       (size_t)((((axis[AX] * 2) + (p ^ dp)) * 8 + slot) * 6) * (size_t)Ss;
    const unsigned bytes = 6u * (unsigned)Ss * (unsigned)sizeof(cx<T>);
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<cx<T>*>(blk), (short)0, (int)bytes, kBufferWord3);
    Rows2<T> u;
    if constexpr (sizeof(T) == 4) {
      // element pairs (e[2q], e[2q+1]): three 16-byte loads per lane
      const int voff = nbr_cb<D0, D1, D2, D3>(nb) * (int)(2 * sizeof(cx<T>));
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int soff = (int)((unsigned)q * (unsigned)Ss * (unsigned)(2 * sizeof(cx<T>)));
        const CxPair<T> v = __builtin_bit_cast(CxPair<T>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
        u.e[2 * q] = v.a;
        u.e[2 * q + 1] = v.b;
      }
    } else {
      const int voff = nbr_cb<D0, D1, D2, D3>(nb) * (int)sizeof(cx<T>);
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const int soff = (int)((unsigned)c * (unsigned)Ss * (unsigned)sizeof(cx<T>));
        u.e[c] = __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
      }
    }
    return u;
  }
};

template <typename T>
__device__ __forceinline__ void launder(FCtx<T>& c) {
  asm volatile("" : "+s"(c.U));
  asm volatile("" : "+s"(c.S8));
}

// ---------------------------------------------------------------- pass 1

// Staple store: FP32 as three planes of 16-byte element pairs, FP64 as six planes.
template <typename T, int POL = kStoreNT>
__device__ __forceinline__ void store_staple(T* S8, int Ss, int mu, int p, int slot, int cb, const Rows2<T>& s) {
  cx<T>* dst = reinterpret_cast<cx<T>*>(S8) + (size_t)(((mu * 2 + p) * 8 + slot) * 6) * (size_t)Ss;
  const unsigned bytes = 6u * (unsigned)Ss * (unsigned)sizeof(cx<T>);
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(dst, (short)0, (int)bytes, kBufferWord3);
  if constexpr (sizeof(T) == 4) {
    const int voff = cb * (int)(2 * sizeof(cx<T>));
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int soff = (int)((unsigned)q * (unsigned)Ss * (unsigned)(2 * sizeof(cx<T>)));
      const CxPair<T> v{s.e[2 * q], s.e[2 * q + 1]};
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U32x4, v), r, voff, soff, POL);
    }
  } else {
    const int voff = cb * (int)sizeof(cx<T>);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const int soff = (int)((unsigned)c * (unsigned)Ss * (unsigned)sizeof(cx<T>));
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, s.e[c]),
                                             r, voff, soff, POL);
    }
  }
}

// Rows 0, 1 of a^{DA} b^{DB} for a, b given in full.
template <bool DA, bool DB, typename T>
__device__ __forceinline__ Rows2<T> rows_mul2(const su3<T>& a, const su3<T>& b) {
  Rows2<T> P;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      T re = T(0), im = T(0);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const cx<T> x = elem<DA>(a, i, k);
        const cx<T> y = elem<DB>(b, k, j);
        re = fma(x.re, y.re, re);
        im = fma(x.re, y.im, im);
        re = fma(-x.im, y.im, re);
        im = fma(x.im, y.re, im);
      }
      P.e[3 * i + j] = cx<T>{re, im};
    }
  }
  return P;
}

// The first two rows of l r^{DB} for l given by its two stored rows and r in full; the
// product of two special-unitary matrices is special unitary, so full() of the result
// rebuilds its third row.
template <bool DB, typename T>
__device__ __forceinline__ Rows2<T> rows_mul(const Rows2<T>& l, const su3<T>& r) {
  Rows2<T> P;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      T re = T(0), im = T(0);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const cx<T> x = l.e[3 * i + k];
        const cx<T> y = elem<DB>(r, k, j);
        re = fma(x.re, y.re, re);
        im = fma(x.re, y.im, im);
        re = fma(-x.im, y.im, re);
        im = fma(x.im, y.re, im);
      }
      P.e[3 * i + j] = cx<T>{re, im};
    }
  }
  return P;
}

// One thread per site: absolute directions, links of the site's neighbourhood.
template <typename T>
struct SCtx {
  const T* U;
  T* S8;
  int Vh;
  int Ss;
  int p;
  int cb;
  Nbr nb;

  // the first two rows of U_{x+d, MU} (loaded only; full() rebuilds the third row)
  template <int MU, int D0, int D1, int D2, int D3>
  __device__ __forceinline__ Rows2<T> link() const {
    constexpr int dp = offset_parity<D0, D1, D2, D3>();
    const cx<T>* blk = block_ptr(U, MU, p ^ dp, Vh);
    const __amdgpu_buffer_rsrc_t r = block_rsrc(blk, Vh);
    const int voff = nbr_cb<D0, D1, D2, D3>(nb) * (int)sizeof(cx<T>);
    Rows2<T> u;
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const int soff = (int)((unsigned)e * (unsigned)Vh * (unsigned)sizeof(cx<T>));
      if constexpr (sizeof(T) == 4)
        u.e[e] = __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
      else
        u.e[e] = __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    }
    return u;
  }
};

template <typename T>
__device__ __forceinline__ void launder(SCtx<T>& c) {
  asm volatile("" : "+s"(c.U));
  asm volatile("" : "+s"(c.S8));
}

constexpr int unit(int axis, int a) { return axis == a ? 1 : 0; }

// The staples of a site in 18 steps, each needing two links besides the site's own
// links u_a = U_{x,a} and w_a = U_{x-a,a}:
//   K = 0..5, plane (MU, A), MU < A: m = U_{x+MU,A} U_{x+A,MU}^dagger gives
//     S(x,MU,+A) = m u_A^dagger and S(x,A,+MU) = m^dagger u_MU^dagger;
//   K = 6 + 3A + J, MU the J-th direction other than A:
//     S(x,MU,-A) = U_{x+MU-A,A}^dagger U_{x-A,MU}^dagger w_A.
template <int K>
struct StapleStep {
  static constexpr bool fwd = K < 6;
  static constexpr int A = fwd ? (K < 3 ? K + 1 : (K < 5 ? K - 1 : 3)) : (K - 6) / 3;
  static constexpr int J = fwd ? 0 : (K - 6) % 3;
  static constexpr int MU = fwd ? (K < 3 ? 0 : (K < 5 ? 1 : 2)) : (J < A ? J : J + 1);
};
constexpr int kStapleSteps = 18;

// What one step loads: the two links besides the site's own, and, with the first step
// of a backward group (J = 0), w_A = U_{x-A,A}. The site's own u_a stay in registers
// through the forward steps only, and one w_A at a time through its group (FP64, one
// step ahead: 269 registers instead of 380), which leaves room to run the loads three
// steps ahead at one wave per SIMD (424 registers; FP32 192, two waves).
template <typename T>
struct StepData {
  Rows2<T> a, b, w;
};

template <int K, typename T>
__device__ __forceinline__ StepData<T> load_step(const SCtx<T>& c0) {
  SCtx<T> c = c0;
  launder(c);
  using St = StapleStep<K>;
  constexpr int MU = St::MU, A = St::A;
  StepData<T> d;
  if constexpr (St::fwd) {
    d.a = c.template link<A, unit(0, MU), unit(1, MU), unit(2, MU), unit(3, MU)>();  // U_{x+MU,A}
    d.b = c.template link<MU, unit(0, A), unit(1, A), unit(2, A), unit(3, A)>();     // U_{x+A,MU}
  } else {
    d.a = c.template link<A, unit(0, MU) - unit(0, A), unit(1, MU) - unit(1, A), unit(2, MU) - unit(2, A),
                          unit(3, MU) - unit(3, A)>();                               // U_{x+MU-A,A}
    d.b = c.template link<MU, -unit(0, A), -unit(1, A), -unit(2, A), -unit(3, A)>();  // U_{x-A,MU}
    if constexpr (St::J == 0)
      d.w = c.template link<A, -unit(0, A), -unit(1, A), -unit(2, A), -unit(3, A)>();  // U_{x-A,A}
  }
  return d;
}

template <int K, int POL, typename T>
__device__ __forceinline__ void use_step(const SCtx<T>& c, const Rows2<T> (&u)[4], const Rows2<T>& wA,
                                         const StepData<T>& d) {
  using St = StapleStep<K>;
  constexpr int MU = St::MU, A = St::A;
  if constexpr (St::fwd) {
    const su3<T> m = full(rows_mul<true>(d.a, full(d.b)));  // special unitary
    store_staple<T, POL>(c.S8, c.Ss, MU, c.p, 2 * A, c.cb, rows_mul2<false, true>(m, full(u[A])));
    store_staple<T, POL>(c.S8, c.Ss, A, c.p, 2 * MU, c.cb, rows_mul2<true, true>(m, full(u[MU])));
  } else {
    const su3<T> n = full(rows_mul2<true, true>(full(d.a), full(d.b)));
    Rows2<T> nr;
#pragma unroll
    for (int i = 0; i < 6; ++i) nr.e[i] = n.e[i];
    store_staple<T, POL>(c.S8, c.Ss, MU, c.p, 2 * A + 1, c.cb, rows_mul<false>(nr, full(wA)));
  }
}

// Software-pipelined: the links of step K+3 are requested before the staples of step K
// are formed and stored (vector memory operations complete in issue order, so a load
// issued after a store would wait for it). On the 32^3 x 64 workload: one step ahead
// 0.82 -> 0.79 ms FP32, 1.46 -> 1.42 ms FP64; three steps ahead with the lean register
// set 1.44 -> 1.41 ms FP64 (FP32 unchanged). n1, n2 hold the two steps already loaded.
constexpr int kStapleAhead = 3;

template <int K, int POL, typename T>
__device__ __forceinline__ void staple_pipe(const SCtx<T>& c, const Rows2<T> (&u)[4], const Rows2<T>& wprev,
                                            const StepData<T>& cur, const StepData<T>& n1, const StepData<T>& n2) {
  using St = StapleStep<K>;
  const Rows2<T>& wA = (!St::fwd && St::J == 0) ? cur.w : wprev;
  if constexpr (K + kStapleAhead < kStapleSteps) {
    const StepData<T> n3 = load_step<K + kStapleAhead>(c);
    SYM_FENCE();
    use_step<K, POL>(c, u, wA, cur);
    SYM_FENCE();
    staple_pipe<K + 1, POL>(c, u, wA, n1, n2, n3);
  } else {
    use_step<K, POL>(c, u, wA, cur);
    SYM_FENCE();
    if constexpr (K + 1 < kStapleSteps) staple_pipe<K + 1, POL>(c, u, wA, n1, n2, n2);  // last argument unused
  }
}

// Pass 1 for site (p, cb) of lattice g: the 24 staples of its four links into S8
// (POL: cache policy of the stores).
template <typename T, int POL = kStoreNT>
__device__ __forceinline__ void staples_site(const Geom& g, const T* U, T* S8, int p, int cb) {
  int x[4];
  cb_coords(g, p, cb, x);
  SCtx<T> c;
  c.U = U;
  c.S8 = S8;
  c.Vh = g.Vh;
  c.Ss = s8_stride(g);
  c.p = p;
  c.cb = cb;
  make_nbr(g, x, c.nb);
  Rows2<T> u[4];
  u[0] = c.template link<0, 0, 0, 0, 0>();
  u[1] = c.template link<1, 0, 0, 0, 0>();
  u[2] = c.template link<2, 0, 0, 0, 0>();
  u[3] = c.template link<3, 0, 0, 0, 0>();
  const StepData<T> d0 = load_step<0>(c);
  const StepData<T> d1 = load_step<1>(c);
  const StepData<T> d2 = load_step<2>(c);
  SYM_FENCE();
  staple_pipe<0, POL>(c, u, d0.w, d0, d1, d2);  // d0.w unused: step 0 is a forward step
}


// ---------------------------------------------------------------- pass 2

// Pass 2 runs as one software pipeline of kSteps steps; the loads of step S+1 are
// issued before step S is multiplied out (vector memory operations complete in issue
// order, so the loads of the next step never wait for the stores or products of this
// one). Every matrix is loaded as its first two rows and rebuilt where it is used.
//   S = 0..5   long side, e = e_S: tP += S(x,mu,e), RA += S(x+mu,mu,e) S(x,mu,e),
//              RB += S(x,mu,e) S(x-mu,mu,e);
//   S = 6      U_{x,mu}, U_{x+-mu,mu}: plaquette and long-side rectangle parts of t and
//              their deficit partials;
//   S = 7..24  items K = S - 7 = 3F + k, f = e_F: k = 0, 1 the triple (S(x+f,mu,e),
//              S(x,f,e), S(x+mu,f,e)) for e = +-(next frame axis) into QA_f, QB_f;
//              k = 2 the short side (S(x+f,mu,f), U_{x+f,-f}, U_{x+mu,f}) and the outer
//              products of f (mixed factorisation, see the top of the file);
//   S = 25     U_{x,mu} again: B = U t, the force epilogue and the last partial.
// One pipeline across the phases, with the short-side links rebuilt at use rather than
// on load, took the pass from 2.43 to 2.38 ms (FP32) and 5.27 to 5.12 ms (FP64) on the
// 32^3 x 64 workload; loading two or three steps ahead was not faster.
constexpr int next_axis(int a) { return a == 3 ? 1 : a + 1; }
constexpr int kSteps = 26;

template <typename T>
struct LongSide {
  Rows2<T> sx, sp, sm;  // S(x,mu,e), S(x+mu,mu,e), S(x-mu,mu,e)
};
template <typename T>
struct Middle {
  Rows2<T> u, up, um;   // U_{x,mu}, U_{x+mu,mu}, U_{x-mu,mu}
};
template <typename T>
struct Triple {
  Rows2<T> m, a, b;  // S(x+f,mu,e); S(x,f,e) (or its dagger's storage); S(x+mu,f,e) (likewise)
};
template <typename T>
struct Short {
  Rows2<T> see;       // S(x+f,mu,f)
  Rows2<T> lnk, uxm;  // U_{x,a} or U_{x-a,a}; U_{x+mu,a} or U_{x+mu-a,a}  (f = +-a)
};
template <typename T>
struct Last {
  Rows2<T> u;  // U_{x,mu}
};

// Per-link state of the pipeline.
template <typename T>
struct FState {
  su3<T> tP, RA, RB, t, QA, QB;
  double part;  // Re tr(U t) before the short-side rectangles and cubes are added
  double a[3];
  T cP, cR, cC;
  double beta, kick;
  T* out;
  int Vh, mu, p, cb;
};

template <int S, typename T>
__device__ __forceinline__ auto load_fstep(const FCtx<T>& c0) {
  FCtx<T> c = c0;
  launder(c);
  if constexpr (S < 6) {
    constexpr int a = e_axis(S), s = e_sign(S);
    LongSide<T> d;
    d.sx = c.template stap_rows<0, 0, 0, 0, 0, a, s>();
    d.sp = c.template stap_rows<1, 0, 0, 0, 0, a, s>();
    d.sm = c.template stap_rows<-1, 0, 0, 0, 0, a, s>();
    return d;
  } else if constexpr (S == 6) {
    Middle<T> d;
    d.u = c.template link_rows<0, 0, 0, 0, 0>();
    d.up = c.template link_rows<1, 0, 0, 0, 0>();
    d.um = c.template link_rows<-1, 0, 0, 0, 0>();
    return d;
  } else if constexpr (S < kSteps - 1) {
    constexpr int K = S - 7, F = K / 3, k = K % 3;
    constexpr int fa = e_axis(F), fs = e_sign(F);
    constexpr int f1 = fs * comp(1, fa), f2 = fs * comp(2, fa), f3 = fs * comp(3, fa);
    if constexpr (k < 2) {
      constexpr int ea = next_axis(fa), es = k == 0 ? 1 : -1;
      Triple<T> d;
      d.m = c.template stap_rows<0, f1, f2, f3, 0, ea, es>();  // S(x+f, mu, e)
      // S(x, f, e) and S(x+mu, f, e): for f = -a stored as S(x-a, a, e)^dagger and
      // S(x+mu-a, a, e)^dagger
      d.a = c.template stap_rows<0, (fs < 0 ? f1 : 0), (fs < 0 ? f2 : 0), (fs < 0 ? f3 : 0), fa, ea, es>();
      d.b = c.template stap_rows<1, (fs < 0 ? f1 : 0), (fs < 0 ? f2 : 0), (fs < 0 ? f3 : 0), fa, ea, es>();
      return d;
    } else {
      Short<T> d;
      d.see = c.template stap_rows<0, f1, f2, f3, 0, fa, fs>();
      if constexpr (fs > 0) {
        d.lnk = c.template link_rows<0, 0, 0, 0, fa>();
        d.uxm = c.template link_rows<1, 0, 0, 0, fa>();
      } else {
        d.lnk = c.template link_rows<0, f1, f2, f3, fa>();
        d.uxm = c.template link_rows<1, f1, f2, f3, fa>();
      }
      return d;
    }
  } else {
    Last<T> d;
    d.u = c.template link_rows<0, 0, 0, 0, 0>();
    return d;
  }
}

template <int S, ForceOut MODE, typename T, typename D>
__device__ __forceinline__ void use_fstep(FState<T>& st, const D& d) {
  if constexpr (S < 6) {
    const su3<T> sx = full(d.sx);
    add(st.tP, sx);
    add(st.RA, full(rows_mul<false>(d.sp, sx)));
    mac<false, false>(st.RB, sx, full(d.sm));
  } else if constexpr (S == 6) {
    const su3<T> u = full(d.u);
    su3<T> WR = mul<false, false>(full(d.up), st.RA);  // U_{x+mu,mu} RA
    mac<false, false>(WR, st.RB, full(d.um));          // + RB U_{x-mu,mu}
    st.a[0] = 18.0 - re_tr_mul(u, st.tP);
    st.a[1] = 36.0 - re_tr_mul(u, WR);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      st.t.e[i].re = fma(st.cP, st.tP.e[i].re, st.cR * WR.e[i].re);
      st.t.e[i].im = fma(st.cP, st.tP.e[i].im, st.cR * WR.e[i].im);
    }
    st.part = double(st.cP) * (18.0 - st.a[0]) + double(st.cR) * (36.0 - st.a[1]);
  } else if constexpr (S < kSteps - 1) {
    constexpr int K = S - 7, F = K / 3, k = K % 3;
    constexpr int fs = e_sign(F);
    if constexpr (k < 2) {
      if constexpr (k == 0) {
        set_zero(st.QA);
        set_zero(st.QB);
      }
      // every factor is special unitary, so is every product: two rows are multiplied
      // out and the third rebuilt
      const su3<T> m = full(d.m);
      if constexpr (fs > 0) {
        add(st.QA, full(rows_mul<false>(d.m, full(d.a))));      // S(x+f,mu,e) S(x,a,e)
        add(st.QB, full(rows_mul2<true, false>(full(d.b), m)));  // S(x+mu,a,e)^dagger S(x+f,mu,e)
      } else {
        add(st.QA, full(rows_mul<true>(d.m, full(d.a))));  // S(x+f,mu,e) S(x-a,a,e)^dagger
        add(st.QB, full(rows_mul<false>(d.b, m)));         // S(x+mu-a,a,e) S(x+f,mu,e)
      }
    } else {
      const su3<T> lnk = full(d.lnk), uxm = full(d.uxm);
      su3<T> R = full(rows_mul<(fs > 0)>(d.see, lnk));  // S(x+f,mu,f) U_{x+f,-f}
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        R.e[i].re = fma(st.cC, st.QA.e[i].re, st.cR * R.e[i].re);
        R.e[i].im = fma(st.cC, st.QA.e[i].im, st.cR * R.e[i].im);
        st.QB.e[i].re *= st.cC;
        st.QB.e[i].im *= st.cC;
      }
      if constexpr (fs > 0) {
        mac<false, false>(st.t, uxm, R);
        mac<false, true>(st.t, st.QB, lnk);
      } else {
        mac<true, false>(st.t, uxm, R);
        mac<false, false>(st.t, st.QB, lnk);
      }
    }
  } else {
    const su3<T> u = full(d.u);
    const su3<T> B = mul<false, false>(u, st.t);
    st.a[2] = 18.0 * double(st.cR) + 72.0 * double(st.cC) - (re_tr(B) - st.part);
    const su3<T> G = ta_scaled(B, T(st.beta / 6.0));
    cx<T>* dst = block_ptr(st.out, st.mu, st.p, st.Vh);
    if constexpr (MODE == ForceOut::Store) {
      store_link(dst, st.Vh, st.cb, G);
    } else if constexpr (MODE == ForceOut::Grad) {
      su3<T> gr = mul<false, false>(G, u);
#pragma unroll
      for (int e = 0; e < 9; ++e) {
        gr.e[e].re *= T(2);
        gr.e[e].im *= T(2);
      }
      store_link(dst, st.Vh, st.cb, gr);
    } else {
      su3<T> q = load_link(static_cast<const cx<T>*>(dst), st.Vh, st.cb);
#pragma unroll
      for (int e = 0; e < 9; ++e) {
        q.e[e].re = T(double(q.e[e].re) - st.kick * double(G.e[e].re));
        q.e[e].im = T(double(q.e[e].im) - st.kick * double(G.e[e].im));
      }
      store_link(dst, st.Vh, st.cb, q);
    }
  }
}

template <int S, ForceOut MODE, typename T, typename D>
__device__ __forceinline__ void force_pipe(const FCtx<T>& c, FState<T>& st, const D& cur) {
  if constexpr (S + 1 < kSteps) {
    const auto nxt = load_fstep<S + 1>(c);
    SYM_FENCE();
    use_fstep<S, MODE>(st, cur);
    SYM_FENCE();
    force_pipe<S + 1, MODE>(c, st, nxt);
  } else {
    use_fstep<S, MODE>(st, cur);
  }
}

// Pass 2 for link (mu, p, cb): force epilogue per MODE, deficit partials into a[3].
template <typename T, ForceOut MODE>
__device__ __forceinline__ void factored_link(const Geom& g, const T* U, const T* S8, T* out, double kick,
                                              const Coeffs& cf, int mu, int p, int cb, double a[3]) {
  int x[4];
  cb_coords(g, p, cb, x);
  FCtx<T> c;
  c.U = U;
  c.S8 = S8;
  c.Vh = g.Vh;
  c.Ss = s8_stride(g);
  c.p = p;
  make_frame(g, mu, x, c.axis, c.nb);
  FState<T> st;
  st.cP = T(cf.c[0]);
  st.cR = T(cf.c[1]);
  st.cC = T(cf.c[2]);
  st.beta = cf.beta;
  st.kick = kick;
  st.out = out;
  st.Vh = g.Vh;
  st.mu = mu;
  st.p = p;
  st.cb = cb;
  set_zero(st.tP);
  set_zero(st.RA);
  set_zero(st.RB);
  const auto d0 = load_fstep<0>(c);
  SYM_FENCE();
  force_pipe<0, MODE>(c, st, d0);
  a[0] = st.a[0];
  a[1] = st.a[1];
  a[2] = st.a[2];
}

}  // namespace factored
}  // namespace sym
