// Direct gauge force: one thread per link, every staple of the generated table
// multiplied out link by link (arXiv:1808.02281 Sec. II, force algorithm after
// eq. 18_6_6_13, with the loop over sites k made the thread index).
//
// For link (k, rho) the thread sums the 48 staples class by class, takes
// G = (beta/6) (U_{k,rho} t)_TA with t = c_P t_P + c_R t_R + c_C t_C, and also emits
// Re tr(U t_X) per class, from which the action follows (each loop of class X is seen
// once from each of its L_X links; the per-link partial is sum over the class's
// staples of (3 - Re tr(U staple)), in double). 181 SU(3) products per link.
//
// The staple table is written for rho = x; the other directions use it in a rotated
// frame (frame axis 0 is rho, frame axes 1..3 are the other axes in increasing order),
// which is exact because the set of staples is symmetric under axis permutations.
#include "kernels.hpp"
#include "path_table.hpp"

namespace sym {
namespace {

struct LinkRef {
  int off[4];  // site offset from k, in frame axes
  int ax;      // frame axis of the link
  bool dag;    // traversed backwards
};

struct StapleRefs {
  int n;
  LinkRef r[5];
};

// Links visited by staple s of the frame table, starting at k + rho-hat.
constexpr StapleRefs staple_refs(int s) {
  StapleRefs out{};
  const table::StapleDef& d = table::kStaple[0][s];
  int p[4] = {1, 0, 0, 0};
  out.n = d.len;
  for (int j = 0; j < d.len; ++j) {
    const int a = (d.dir[j] > 0 ? d.dir[j] : -d.dir[j]) - 1;
    if (d.dir[j] > 0) {
      out.r[j] = LinkRef{{p[0], p[1], p[2], p[3]}, a, false};
      p[a] += 1;
    } else {
      p[a] -= 1;
      out.r[j] = LinkRef{{p[0], p[1], p[2], p[3]}, a, true};
    }
  }
  return out;
}

template <typename T>
struct Ctx {
  const T* U;
  int Vh;
  int p;          // parity of k
  int axis[4];    // frame axis -> lattice axis (uniform)
  Nbr nb;         // indexed by frame axis

  template <int D0, int D1, int D2, int D3, int AX>
  __device__ __forceinline__ su3<T> link() const {
    constexpr int dp = offset_parity<D0, D1, D2, D3>();
    const cx<T>* blk = block_ptr(U, axis[AX], p ^ dp, Vh);
    return load_link(blk, Vh, nbr_cb<D0, D1, D2, D3>(nb));
  }
};

#define SYM_LINK(ctx, R) (ctx).template link<(R).off[0], (R).off[1], (R).off[2], (R).off[3], (R).ax>()

template <typename T, int S>
__device__ __forceinline__ void add_staple(const Ctx<T>& ctx, su3<T>& acc) {
  constexpr StapleRefs R = staple_refs(S);
  constexpr LinkRef a = R.r[0], b = R.r[1], c = R.r[2];
  su3<T> m = mul<a.dag, b.dag>(SYM_LINK(ctx, a), SYM_LINK(ctx, b));
  if constexpr (R.n == 3) {
    mac<false, c.dag>(acc, m, SYM_LINK(ctx, c));
  } else {
    constexpr LinkRef d = R.r[3], e = R.r[4];
    m = mul<false, c.dag>(m, SYM_LINK(ctx, c));
    m = mul<false, d.dag>(m, SYM_LINK(ctx, d));
    mac<false, e.dag>(acc, m, SYM_LINK(ctx, e));
  }
}

template <typename T, int S, int E>
__device__ __forceinline__ void add_staples(const Ctx<T>& ctx, su3<T>& acc) {
  if constexpr (S < E) {
    // Each staple reloads its links (they hit in L1/L2). Without hiding the field
    // pointer, common-subexpression elimination keeps every link shared by two
    // staples alive in registers across the whole kernel, and the kernel spills.
    Ctx<T> local = ctx;
    asm volatile("" : "+s"(local.U));
    add_staple<T, S>(local, acc);
    __builtin_amdgcn_sched_barrier(0);
    add_staples<T, S + 1, E>(ctx, acc);
  }
}

// Frame: axis[0] = rho, axis[1..3] = the other axes ascending; build the neighbour
// offsets per frame axis.
__device__ __forceinline__ void make_frame(const Geom& g, int rho, const int x[4], int axis[4], Nbr& nb) {
  axis[0] = rho;
  axis[1] = rho == 0 ? 1 : 0;
  axis[2] = rho <= 1 ? 2 : 1;
  axis[3] = rho <= 2 ? 3 : 2;
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

template <typename T, ForceOut MODE>
__global__ __launch_bounds__(kBlock) void force_direct_kernel(Geom g, const T* __restrict__ U, T* __restrict__ out,
                                                              double kick, double* __restrict__ partials, Coeffs c,
                                                              int ntiles) {
  const LinkTile lt = link_tile(g, blockIdx.x, ntiles);
  const int rho = lt.mu, p = lt.p, chunk = lt.chunk;
  const int cb = chunk * kBlock + threadIdx.x;
  double tr[3] = {0.0, 0.0, 0.0};
  if (cb < g.Vh) {
    int x[4];
    cb_coords(g, p, cb, x);
    Ctx<T> ctx;
    ctx.U = U;
    ctx.Vh = g.Vh;
    ctx.p = p;
    make_frame(g, rho, x, ctx.axis, ctx.nb);

    const su3<T> u = load_link(block_ptr(U, rho, p, g.Vh), g.Vh, cb);
    su3<T> t, acc;
    set_zero(t);
    set_zero(acc);
    add_staples<T, table::kClassBegin[0], table::kClassBegin[1]>(ctx, acc);
    tr[0] = 18.0 - re_tr_mul(u, acc);  // 6 plaquette staples: sum of (3 - Re tr loop)
    axpy(t, T(c.c[0]), acc);
    set_zero(acc);
    add_staples<T, table::kClassBegin[1], table::kClassBegin[2]>(ctx, acc);
    tr[1] = 54.0 - re_tr_mul(u, acc);  // 18 rectangle staples
    axpy(t, T(c.c[1]), acc);
    set_zero(acc);
    add_staples<T, table::kClassBegin[2], table::kClassBegin[3]>(ctx, acc);
    tr[2] = 72.0 - re_tr_mul(u, acc);  // 24 cube staples
    axpy(t, T(c.c[2]), acc);

    const su3<T> G = ta_scaled(mul<false, false>(u, t), T(c.beta / 6.0));
    cx<T>* dst = block_ptr(out, rho, p, g.Vh);
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
  if (partials != nullptr) block_sum_store<3>(tr, partials + 3 * (size_t)blockIdx.x);
}

}  // namespace

template <typename T>
hipError_t launch_force_direct(const Geom& g, const T* U, T* out, double kick, double* partials, const Coeffs& c,
                               ForceOut mode, hipStream_t s) {
  const int nt = link_tiles(g);
  if (mode == ForceOut::Store)
    force_direct_kernel<T, ForceOut::Store><<<nt, kBlock, 0, s>>>(g, U, out, kick, partials, c, nt);
  else if (mode == ForceOut::Kick)
    force_direct_kernel<T, ForceOut::Kick><<<nt, kBlock, 0, s>>>(g, U, out, kick, partials, c, nt);
  else
    force_direct_kernel<T, ForceOut::Grad><<<nt, kBlock, 0, s>>>(g, U, out, kick, partials, c, nt);
  return hipGetLastError();
}

#ifndef SYM_ONLY_F64
template hipError_t launch_force_direct<float>(const Geom&, const float*, float*, double, double*, const Coeffs&,
                                               ForceOut, hipStream_t);
#endif
#ifndef SYM_ONLY_F32
template hipError_t launch_force_direct<double>(const Geom&, const double*, double*, double, double*,
                                                const Coeffs&, ForceOut, hipStream_t);
#endif

}  // namespace sym
