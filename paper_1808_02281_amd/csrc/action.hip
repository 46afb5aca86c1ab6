// Symanzik action S_G (arXiv:1808.02281 Sec. II, eq. 18_6_4_1) and the final
// deterministic reductions shared by the action, the fused force action and the
// leapfrog Hamiltonian.
//
// Action kernel: one thread per site computes the 34 loop products of eq. (18_6_6_3_0)
// at its site and accumulates w_X = sum (3 - Re tr P_n) per class X in double. The last
// product of every loop is replaced by its trace (124 products + 34 traces per site).
#include "kernels.hpp"
#include "path_table.hpp"

namespace sym {
namespace {

struct LinkRef {
  int off[4];
  int ax;
  bool dag;
};

struct LoopRefs {
  int n;
  int cls;
  LinkRef r[6];
};

constexpr LoopRefs loop_refs(int l) {
  LoopRefs out{};
  const table::LoopDef& d = table::kLoop[l];
  int p[4] = {0, 0, 0, 0};
  out.n = d.len;
  out.cls = d.cls;
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
struct SiteCtx {
  const T* U;
  int Vh;
  int p;
  Nbr nb;

  template <int D0, int D1, int D2, int D3, int AX>
  __device__ __forceinline__ su3<T> link() const {
    constexpr int dp = offset_parity<D0, D1, D2, D3>();
    return load_link(block_ptr(U, AX, p ^ dp, Vh), Vh, nbr_cb<D0, D1, D2, D3>(nb));
  }
};

#define SYM_LINK(ctx, R) (ctx).template link<(R).off[0], (R).off[1], (R).off[2], (R).off[3], (R).ax>()

template <typename T, int LP>
__device__ __forceinline__ void add_loop(const SiteCtx<T>& ctx, double w[3]) {
  constexpr LoopRefs R = loop_refs(LP);
  constexpr LinkRef a = R.r[0], b = R.r[1], c = R.r[2], d = R.r[3];
  su3<T> m = mul<a.dag, b.dag>(SYM_LINK(ctx, a), SYM_LINK(ctx, b));
  m = mul<false, c.dag>(m, SYM_LINK(ctx, c));
  double rt;
  if constexpr (R.n == 4) {
    rt = re_tr_mul<d.dag>(m, SYM_LINK(ctx, d));
  } else {
    constexpr LinkRef e = R.r[4], f = R.r[5];
    m = mul<false, d.dag>(m, SYM_LINK(ctx, d));
    m = mul<false, e.dag>(m, SYM_LINK(ctx, e));
    rt = re_tr_mul<f.dag>(m, SYM_LINK(ctx, f));
  }
  w[R.cls] += 3.0 - rt;
}

template <typename T, int LP>
__device__ __forceinline__ void add_loops(const SiteCtx<T>& ctx, double w[3]) {
  if constexpr (LP < table::kLoops) {
    // Reload links per loop (they hit in cache) rather than keep shared ones live.
    SiteCtx<T> local = ctx;
    asm volatile("" : "+s"(local.U));
    add_loop<T, LP>(local, w);
    __builtin_amdgcn_sched_barrier(0);
    add_loops<T, LP + 1>(ctx, w);
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void action_kernel(Geom g, const T* __restrict__ U, double* __restrict__ partials,
                                                        int ntiles) {
  const int tile = xcd_tile(blockIdx.x, ntiles);
  const int site = tile * kBlock + threadIdx.x;  // both parities: [0, Vh) even, [Vh, 2Vh) odd
  double w[3] = {0.0, 0.0, 0.0};
  if (site < 2 * g.Vh) {
    const int p = site >= g.Vh ? 1 : 0;
    const int cb = site - p * g.Vh;
    int x[4];
    cb_coords(g, p, cb, x);
    SiteCtx<T> ctx;
    ctx.U = U;
    ctx.Vh = g.Vh;
    ctx.p = p;
    make_nbr(g, x, ctx.nb);
    add_loops<T, 0>(ctx, w);
  }
  block_sum_store<3>(w, partials + 3 * (size_t)blockIdx.x);
}

// Deterministic two-stage reduction of the per-workgroup partials: stage 1 (kFinishGroups
// blocks) sums contiguous groups of partials, stage 2 (one block) sums the group sums,
// both in a fixed order. One block summing all 65,536 partials of the 32^3 x 64 force
// took 25 us, alone on the GPU; the two stages take about a third of that.
constexpr int kFinishGroups = 64;

__global__ __launch_bounds__(256) void finish_stage1(const double* __restrict__ act, int nact,
                                                     const double* __restrict__ kin, int nkin,
                                                     double* __restrict__ stage) {
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const int ga = (nact + kFinishGroups - 1) / kFinishGroups, gk = (nkin + kFinishGroups - 1) / kFinishGroups;
  const int a0 = blockIdx.x * ga, a1 = min(nact, a0 + ga);
  const int k0 = blockIdx.x * gk, k1 = min(nkin, k0 + gk);
  for (int i = a0 + (int)threadIdx.x; i < a1; i += blockDim.x) {
    v[0] += act[3 * (size_t)i + 0];
    v[1] += act[3 * (size_t)i + 1];
    v[2] += act[3 * (size_t)i + 2];
  }
  for (int i = k0 + (int)threadIdx.x; i < k1; i += blockDim.x) v[3] += kin[i];
  block_sum_store<4>(v, stage + 4 * (size_t)blockIdx.x);
}

// Stage 2 (one block): with deficit sums w_X = sum over class-X loops of (3 - Re tr P),
//   S = beta/3 (c_P w_P + c_R w_R + c_C w_C),  W_X = 3 n_X V - w_X  (n = 6, 12, 16).
// mode 0 writes out[0..3] = S, W_P, W_R, W_C; mode 1 adds the kinetic partials and
// writes out[0] = S + K.
__global__ __launch_bounds__(64) void finish_stage2(const double* __restrict__ stage, int kind, Coeffs c, double V,
                                                    int mode, double* __restrict__ out) {
  double v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = stage[4 * (size_t)threadIdx.x + k];
  block_sum<4>(v);
  if (threadIdx.x == 0) {
    double wP, wR, wC, cwC;
    if (kind == 0) {  // direct force: each loop seen from 4 / 6 / 6 links
      wP = v[0] / 4.0;
      wR = v[1] / 6.0;
      wC = v[2] / 6.0;
      cwC = c.c[2] * wC;
    } else if (kind == 1) {  // action kernel: per-loop sums
      wP = v[0];
      wR = v[1];
      wC = v[2];
      cwC = c.c[2] * wC;
    } else {  // factored force: long sides see a rectangle 4 times, the mixed sum holds
              // c_R x (2 views of every rectangle) + c_C x (6 views of every cube loop);
              // W_C needs c_C != 0 (the library runs the action kernel otherwise)
      wP = v[0] / 4.0;
      wR = v[1] / 4.0;
      cwC = (v[2] - 0.5 * c.c[1] * v[1]) / 6.0;
      wC = c.c[2] != 0.0 ? cwC / c.c[2] : __builtin_nan("");
    }
    const double S = c.beta / 3.0 * (c.c[0] * wP + c.c[1] * wR + cwC);
    if (mode == 0) {
      out[0] = S;
      out[1] = 18.0 * V - wP;
      out[2] = 36.0 * V - wR;
      out[3] = 48.0 * V - wC;
    } else {
      out[0] = S + v[3];
    }
  }
}

}  // namespace

int action_tiles(const Geom& g) {
  const int n = (2 * g.Vh + kBlock - 1) / kBlock;
  return (n + 7) & ~7;
}

template <typename T>
hipError_t launch_action(const Geom& g, const T* U, double* partials, hipStream_t s) {
  const int nt = action_tiles(g);
  action_kernel<T><<<nt, kBlock, 0, s>>>(g, U, partials, nt);
  return hipGetLastError();
}

template hipError_t launch_action<float>(const Geom&, const float*, double*, hipStream_t);
template hipError_t launch_action<double>(const Geom&, const double*, double*, hipStream_t);

hipError_t launch_finish_action(const double* partials, int nparts, int kind, const Geom& g, const Coeffs& c,
                                double* stage, double* out, hipStream_t s) {
  finish_stage1<<<kFinishGroups, 256, 0, s>>>(partials, nparts, nullptr, 0, stage);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  finish_stage2<<<1, kFinishGroups, 0, s>>>(stage, kind, c, 2.0 * g.Vh, 0, out);
  return hipGetLastError();
}

hipError_t launch_finish_hamiltonian(const double* act_parts, int nact, int act_kind, const double* kin_parts,
                                     int nkin, const Geom& g, const Coeffs& c, double* stage, double* out,
                                     hipStream_t s) {
  finish_stage1<<<kFinishGroups, 256, 0, s>>>(act_parts, nact, kin_parts, nkin, stage);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  finish_stage2<<<1, kFinishGroups, 0, s>>>(stage, act_kind, c, 2.0 * g.Vh, 1, out);
  return hipGetLastError();
}

}  // namespace sym
