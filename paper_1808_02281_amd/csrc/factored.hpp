// Factored gauge force: per-link device code shared by the single-lattice kernels
// (force_factored.hip) and the batched persistent kernels (force_batch.hip).
//
// Factored gauge force. Same result as the direct form (every staple of
// arXiv:1808.02281 Sec. II, eq. 18_7_25_2), with rectangle and cube staples assembled
// from plaquette staples instead of multiplied out link by link.
//
// Notation: for link (x, mu) and a signed direction e perpendicular to mu,
//   S(x, mu, e) = U_{x+mu, e} U_{x+e, mu}^dagger U_{x, e}^dagger
// is the plaquette staple (path e, -mu, -e from x+mu back to x), with
// U_{y,-nu} = U_{y-nu,nu}^dagger. Inserting U^dagger U = 1 along the paths gives,
// for the 42 five-link staples of link (x, mu):
//   rectangles, link first on the long side:  U_{x+mu,mu} S(x+mu,mu,e) S(x,mu,e)
//   rectangles, link second on the long side: S(x,mu,e) S(x-mu,mu,e) U_{x-mu,mu}
//   rectangles with the link as short side:   U_{x+mu,e} S(x+e,mu,e) U_{x,e}^dagger
//   cube loops (e, f, -mu, -e, -f):           U_{x+mu,e} S(x+e,mu,f) S'(x,e,f)
// where f is perpendicular to mu and to e, and S'(x,e,f) is the path f, -e, -f from
// x+e to x: S(x,nu,f) for e = +nu, S(x-nu,nu,f)^dagger for e = -nu. Sums over e and f
// are taken before the shared outer factors are applied.
//
// Pass 1 (staples_kernel) writes the six S(x,mu,e) of every link to the workspace:
// 12 SU(3) products per link, each link read as its first two rows (the third rebuilt),
// which cuts the pass from 1.05 to 0.88 ms (FP32) and 1.93 to 1.55 ms (FP64) on the
// 32^3 x 64 workload; the links of the short-side and cube terms of pass 2 are read
// the same way (3.02 -> 2.92 ms FP32). Pass 2 (force_factored_kernel) reads them and forms
//   t = c_P sum_e S + c_R (rect sums) + (c_R short-side rect + c_C cube sums):
// 6+1 and 6+1 products for the long-side rectangles, 6 x (1 + 4 + 1) for the rest,
// plus U t: 51 products. 63 products per link in all, against 181 for the direct form.
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

  // U_{x+d, axis[AX]} (forward link)
  template <int D0, int D1, int D2, int D3, int AX>
  __device__ __forceinline__ su3<T> link() const {
    constexpr int dp = offset_parity<D0, D1, D2, D3>();
    return load_link(block_ptr(U, axis[AX], p ^ dp, Vh), Vh, nbr_cb<D0, D1, D2, D3>(nb));
  }

  // U_{x+d, axis[AX]} from its first two rows, the third rebuilt (special unitary):
  // a third less link traffic than load_link
  template <int D0, int D1, int D2, int D3, int AX>
  __device__ __forceinline__ su3<T> link_rows() const {
    constexpr int dp = offset_parity<D0, D1, D2, D3>();
    return load_su3_rows(block_ptr(U, axis[AX], p ^ dp, Vh), Vh, nbr_cb<D0, D1, D2, D3>(nb));
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

  // S(x+d, axis[AX], e) for e = sign ES along frame axis EAX
  template <int D0, int D1, int D2, int D3, int AX, int EAX, int ES>
  __device__ __forceinline__ su3<T> stap() const {
    return full(stap_rows<D0, D1, D2, D3, AX, EAX, ES>());
  }
};

template <typename T>
__device__ __forceinline__ void launder(FCtx<T>& c) {
  asm volatile("" : "+s"(c.U));
  asm volatile("" : "+s"(c.S8));
}

// ---------------------------------------------------------------- pass 1

template <typename T, int J>
__device__ __forceinline__ su3<T> plaquette_staple(const FCtx<T>& c) {
  constexpr int a = e_axis(J);
  constexpr int a1 = comp(1, a), a2 = comp(2, a), a3 = comp(3, a);
  if constexpr (e_sign(J) > 0) {
    // U_{x+mu,a} U_{x+a,mu}^dag U_{x,a}^dag
    const su3<T> m = mul<false, true>(c.template link_rows<1, 0, 0, 0, a>(), c.template link_rows<0, a1, a2, a3, 0>());
    return mul<false, true>(m, c.template link_rows<0, 0, 0, 0, a>());
  } else {
    // U_{x+mu-a,a}^dag U_{x-a,mu}^dag U_{x-a,a}
    const su3<T> m = mul<true, true>(c.template link_rows<1, -a1, -a2, -a3, a>(), c.template link_rows<0, -a1, -a2, -a3, 0>());
    return mul<false, false>(m, c.template link_rows<0, -a1, -a2, -a3, a>());
  }
}

template <typename T, int J>
__device__ __forceinline__ void write_staples(const FCtx<T>& c, T* S8, int cb) {
  if constexpr (J < 6) {
    FCtx<T> lc = c;
    launder(lc);
    const su3<T> s = plaquette_staple<T, J>(lc);
    const int slot = 2 * c.axis[e_axis(J)] + (e_sign(J) < 0 ? 1 : 0);
    cx<T>* dst = reinterpret_cast<cx<T>*>(S8) + (size_t)(((c.axis[0] * 2 + c.p) * 8 + slot) * 6) * (size_t)c.Ss;
    if constexpr (sizeof(T) == 4) {
      const unsigned bytes = 6u * (unsigned)c.Ss * (unsigned)sizeof(cx<T>);
      const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(dst, (short)0, (int)bytes, kBufferWord3);
      const int voff = cb * (int)(2 * sizeof(cx<T>));
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int soff = (int)((unsigned)q * (unsigned)c.Ss * (unsigned)(2 * sizeof(cx<T>)));
        const CxPair<T> v{s.e[2 * q], s.e[2 * q + 1]};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U32x4, v), r, voff, soff, kStoreNT);
      }
    } else {
      store_su3_rows(dst, c.Ss, cb, s);
    }
    SYM_FENCE();
    write_staples<T, J + 1>(c, S8, cb);
  }
}


// ---------------------------------------------------------------- pass 2

// Short-side rectangles and cube loops, software-pipelined. For e = e_J (J = 0..5) and
// the four f perpendicular to mu and e (cube_f(J, i)):
//   t += U_{x+mu,e} [ c_R S(x+e,mu,e) U_{x,e}^dag + c_C sum_f S(x+e,mu,f) S'(x,e,f) ].
// The loads of each e are split in two halves, A (two cube terms) and B (two cube terms,
// the short-side staple and the two links); the loads of the next half are issued
// before the current half is multiplied out, so that their latency is covered by
// arithmetic instead of by other waves alone (FP32, 32^3 x 64 force pass: 3.26 ms in
// plain order, 3.11 ms with the cube loop pipelined, 3.08 ms with the long-side sums
// pipelined too, 223 VGPRs; issuing the first cube loads during the long-side epilogue
// as well reached 256 VGPRs and was slower). FP64 takes the same form: its operands
// need about 420 registers, so one wave per SIMD holds them in VGPRs and AGPRs
// (6.72 ms in plain order, 6.50 ms pipelined).
constexpr int cube_f(int J, int i) {
  int n = 0;
  for (int K = 0; K < 6; ++K) {
    if (e_axis(K) != e_axis(J)) {
      if (n == i) return K;
      ++n;
    }
  }
  return -1;
}

template <typename T>
struct CubeA {
  Rows2<T> l0, r0, l1, r1;
};
template <typename T>
struct CubeB {
  Rows2<T> l2, r2, l3, r3, see;
  su3<T> lnk, uxm;
};

// S(x+e,mu,f) and S'(x,e,f) for the i-th f of e_J
template <int J, int I, typename T>
__device__ __forceinline__ void cube_pair(const FCtx<T>& c, Rows2<T>& l, Rows2<T>& r) {
  constexpr int a = e_axis(J), s = e_sign(J), K = cube_f(J, I), fa = e_axis(K), fs = e_sign(K);
  constexpr int e1 = s * comp(1, a), e2 = s * comp(2, a), e3 = s * comp(3, a);
  l = c.template stap_rows<0, e1, e2, e3, 0, fa, fs>();
  if constexpr (s > 0)
    r = c.template stap_rows<0, 0, 0, 0, a, fa, fs>();
  else
    r = c.template stap_rows<0, e1, e2, e3, a, fa, fs>();
}

template <int J, typename T>
__device__ __forceinline__ CubeA<T> load_cube_a(const FCtx<T>& c0) {
  FCtx<T> c = c0;
  launder(c);
  CubeA<T> d;
  cube_pair<J, 0>(c, d.l0, d.r0);
  cube_pair<J, 1>(c, d.l1, d.r1);
  return d;
}

template <int J, typename T>
__device__ __forceinline__ CubeB<T> load_cube_b(const FCtx<T>& c0) {
  FCtx<T> c = c0;
  launder(c);
  constexpr int a = e_axis(J), s = e_sign(J);
  constexpr int e1 = s * comp(1, a), e2 = s * comp(2, a), e3 = s * comp(3, a);
  CubeB<T> d;
  cube_pair<J, 2>(c, d.l2, d.r2);
  cube_pair<J, 3>(c, d.l3, d.r3);
  d.see = c.template stap_rows<0, e1, e2, e3, 0, a, s>();
  if constexpr (s > 0) {
    d.lnk = c.template link_rows<0, 0, 0, 0, a>();
    d.uxm = c.template link_rows<1, 0, 0, 0, a>();
  } else {
    d.lnk = c.template link_rows<0, e1, e2, e3, a>();
    d.uxm = c.template link_rows<1, e1, e2, e3, a>();
  }
  return d;
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

// Q += l r (e > 0) or l r^dagger (e < 0) for staples l, r in SU(3) given by their first
// two rows. The product is special unitary too, so only its first two rows are
// multiplied out (from the two stored rows of l) and its third row is rebuilt from
// them: 18 complex multiply-adds and one rebuild instead of 27 and two.
template <int J, typename T>
__device__ __forceinline__ void cube_mac(su3<T>& Q, const Rows2<T>& l, const Rows2<T>& r) {
  add(Q, full(rows_mul<(e_sign(J) < 0)>(l, full(r))));
}

template <int J, typename T>
__device__ __forceinline__ void use_cube_b(su3<T>& t, su3<T>& Q, const CubeB<T>& d, T cR, T cC) {
  cube_mac<J>(Q, d.l2, d.r2);
  cube_mac<J>(Q, d.l3, d.r3);
  su3<T> R = full(rows_mul<(e_sign(J) > 0)>(d.see, d.lnk));  // S(x+e,mu,e) U_{x,e}^dag (special unitary)
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    R.e[i].re = fma(cC, Q.e[i].re, cR * R.e[i].re);
    R.e[i].im = fma(cC, Q.e[i].im, cR * R.e[i].im);
  }
  if constexpr (e_sign(J) > 0)
    mac<false, false>(t, d.uxm, R);
  else
    mac<true, false>(t, d.uxm, R);
}

template <int J, typename T>
__device__ __forceinline__ void cubes_pipe(const FCtx<T>& c, su3<T>& t, const CubeA<T>& a, const CubeB<T>& b, T cR,
                                           T cC) {
  su3<T> Q;
  set_zero(Q);
  cube_mac<J>(Q, a.l0, a.r0);
  cube_mac<J>(Q, a.l1, a.r1);
  SYM_FENCE();
  if constexpr (J < 5) {
    const CubeA<T> an = load_cube_a<J + 1>(c);
    SYM_FENCE();
    use_cube_b<J>(t, Q, b, cR, cC);
    SYM_FENCE();
    const CubeB<T> bn = load_cube_b<J + 1>(c);
    SYM_FENCE();
    cubes_pipe<J + 1>(c, t, an, bn, cR, cC);
  } else {
    use_cube_b<J>(t, Q, b, cR, cC);
    SYM_FENCE();
  }
}


// Long-side rectangles, RA += S(x+mu,mu,e) S(x,mu,e), RB += S(x,mu,e) S(x-mu,mu,e),
// tP += S(x,mu,e), software-pipelined: the three staples of e_{J+1} are requested
// before those of e_J are multiplied out.
template <typename T>
struct LongSide {
  Rows2<T> sx, sp, sm;  // S(x,mu,e), S(x+mu,mu,e), S(x-mu,mu,e)
};
template <int J, typename T>
__device__ __forceinline__ LongSide<T> load_long(const FCtx<T>& c0) {
  FCtx<T> c = c0;
  launder(c);
  constexpr int a = e_axis(J), s = e_sign(J);
  LongSide<T> d;
  d.sx = c.template stap_rows<0, 0, 0, 0, 0, a, s>();
  d.sp = c.template stap_rows<1, 0, 0, 0, 0, a, s>();
  d.sm = c.template stap_rows<-1, 0, 0, 0, 0, a, s>();
  return d;
}
template <int J, typename T>
__device__ __forceinline__ void long_pipe(const FCtx<T>& c, su3<T>& tP, su3<T>& RA, su3<T>& RB, const LongSide<T>& d) {
  if constexpr (J < 5) {
    const LongSide<T> dn = load_long<J + 1>(c);
    SYM_FENCE();
    const su3<T> sx = full(d.sx);
    add(tP, sx);
    add(RA, full(rows_mul<false>(d.sp, sx)));
    mac<false, false>(RB, sx, full(d.sm));
    SYM_FENCE();
    long_pipe<J + 1>(c, tP, RA, RB, dn);
  } else {
    const su3<T> sx = full(d.sx);
    add(tP, sx);
    add(RA, full(rows_mul<false>(d.sp, sx)));
    mac<false, false>(RB, sx, full(d.sm));
  }
}

// Pass 1 for link (mu, p, cb) of lattice g: its six plaquette staples into S8.
template <typename T>
__device__ __forceinline__ void staples_link(const Geom& g, const T* U, T* S8, int mu, int p, int cb) {
  int x[4];
  cb_coords(g, p, cb, x);
  FCtx<T> c;
  c.U = U;
  c.S8 = S8;
  c.Vh = g.Vh;
  c.Ss = s8_stride(g);
  c.p = p;
  make_frame(g, mu, x, c.axis, c.nb);
  write_staples<T, 0>(c, S8, cb);
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
  const T cP = T(cf.c[0]), cR = T(cf.c[1]), cC = T(cf.c[2]);

  su3<T> t;
  double part;  // Re tr(U t) before the short-side rectangles and cubes are added
  {
    su3<T> tP, RA, RB;
    set_zero(tP);
    set_zero(RA);
    set_zero(RB);
    const LongSide<T> d0 = load_long<0>(c);
    SYM_FENCE();
    long_pipe<0>(c, tP, RA, RB, d0);
    SYM_FENCE();
    FCtx<T> lc = c;
    launder(lc);
    const su3<T> u = lc.template link<0, 0, 0, 0, 0>();
    su3<T> WR = mul<false, false>(lc.template link<1, 0, 0, 0, 0>(), RA);  // U_{x+mu,mu} RA
    mac<false, false>(WR, RB, lc.template link<-1, 0, 0, 0, 0>());         // + RB U_{x-mu,mu}
    a[0] = 18.0 - re_tr_mul(u, tP);
    a[1] = 36.0 - re_tr_mul(u, WR);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      t.e[i].re = fma(cP, tP.e[i].re, cR * WR.e[i].re);
      t.e[i].im = fma(cP, tP.e[i].im, cR * WR.e[i].im);
    }
    part = re_tr_mul(u, t);
  }
  SYM_FENCE();
  {
    // software-pipelined short-side rectangles and cube loops
    const CubeA<T> a0 = load_cube_a<0>(c);
    const CubeB<T> b0 = load_cube_b<0>(c);
    SYM_FENCE();
    cubes_pipe<0>(c, t, a0, b0, cR, cC);
  }

  FCtx<T> lc = c;
  launder(lc);
  const su3<T> u = lc.template link<0, 0, 0, 0, 0>();
  const su3<T> B = mul<false, false>(u, t);
  a[2] = 18.0 * cf.c[1] + 72.0 * cf.c[2] - (re_tr(B) - part);
  const su3<T> G = ta_scaled(B, T(cf.beta / 6.0));
  cx<T>* dst = block_ptr(out, mu, p, g.Vh);
  if constexpr (MODE == ForceOut::Store) {
    store_link(dst, g.Vh, cb, G);
  } else if constexpr (MODE == ForceOut::Grad) {
    su3<T> gr = mul<false, false>(G, u);
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      gr.e[e].re *= T(2);
      gr.e[e].im *= T(2);
    }
    store_link(dst, g.Vh, cb, gr);
  } else {
    su3<T> q = load_link(static_cast<const cx<T>*>(dst), g.Vh, cb);
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      q.e[e].re = T(double(q.e[e].re) - kick * double(G.e[e].re));
      q.e[e].im = T(double(q.e[e].im) - kick * double(G.e[e].im));
    }
    store_link(dst, g.Vh, cb, q);
  }
}

}  // namespace factored
}  // namespace sym
