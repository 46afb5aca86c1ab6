// Host side of the C ABI in include/sym.h: validation, coefficients, workspace
// carving and kernel sequencing. Nothing here allocates device memory or
// synchronises; every launch goes on the caller's stream.
#include <math.h>
#include <stdint.h>

#include <atomic>
#include <initializer_list>
#include <map>
#include <mutex>
#include <string.h>
#include <vector>

#include "../../include/sym.h"
#include "fat.hpp"
#include "project.hpp"
#include "kernels.hpp"

namespace {

using sym::Coeffs;
using sym::ForceOut;
using sym::Geom;

std::mutex g_override_mu;
bool g_override_on = false;
double g_override[3] = {1.0, 0.0, 0.0};
std::atomic<int> g_algorithm{SYM_ALG_AUTO};

constexpr long long kMaxVh = 1ll << 24;  // keeps every (mu, parity) block below 4 GiB

int make_geom(const int32_t* L, Geom* g) {
  if (L == nullptr) return SYM_ENULL;
  long long V = 1;
  for (int a = 0; a < 4; ++a) {
    if (L[a] < 4 || (L[a] & 1)) return SYM_EINVAL;
    V *= L[a];
    if (V > 2 * kMaxVh) return SYM_EINVAL;
  }
  for (int a = 0; a < 4; ++a) g->L[a] = L[a];
  g->Vh = (int)(V / 2);
  g->Lxh = L[0] / 2;
  // t-fastest tile order of the per-link kernels (see link_tile in lattice.hpp)
  const long long per_slice = V / 2 / L[3];
  g->tslab = 0;
  g->cps = 0;
  if (L[3] % 8 == 0 && per_slice % sym::kBlock == 0) {
    g->tslab = L[3] / 8;
    g->cps = (int)(per_slice / sym::kBlock);
  }
  return SYM_OK;
}

int check_prec(int prec) { return (prec == SYM_F32 || prec == SYM_F64) ? SYM_OK : SYM_EINVAL; }

int check_ptr(const void* p) {
  if (p == nullptr) return SYM_ENULL;
  return ((uintptr_t)p & 15u) ? SYM_EINVAL : SYM_OK;
}

int make_coeffs(double u0, double beta, Coeffs* c) {
  if (!(u0 > 0.0) || !isfinite(u0) || !isfinite(beta)) return SYM_EINVAL;
  double a;
  sym_coeffs(u0, c->c, &a);
  {
    std::lock_guard<std::mutex> lk(g_override_mu);
    if (g_override_on)
      for (int k = 0; k < 3; ++k) c->c[k] = g_override[k];
  }
  c->beta = beta;
  return SYM_OK;
}

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// Workspace regions: [A: per-workgroup action partials, 3 doubles each]
// [B: per-workgroup kinetic partials, then the stage of the final reduction]
// [C: plaquette staples, 8 slots of two rows per link].
struct Workspace {
  double* act;
  double* kin;
  double* stage;
  void* staples;
};

size_t region_a(const Geom& g) {
  const int n = sym::max_force_tiles(g) > sym::action_tiles(g) ? sym::max_force_tiles(g) : sym::action_tiles(g);
  return align256(sizeof(double) * 3 * (size_t)n);
}
size_t region_b(const Geom& g) {
  return align256(sizeof(double) * ((size_t)sym::link_tiles(g) + sym::kFinishStage));
}
size_t region_c(const Geom& g, int prec) {
  const size_t real = prec == SYM_F64 ? sizeof(double) : sizeof(float);
  return align256((size_t)8 * sym::s8_stride(g) * 8 * 12 * real);  // 8 staple slots of 2 rows per link
}

size_t ws_bytes_for(const Geom& g, int prec) { return region_a(g) + region_b(g) + region_c(g, prec); }

Workspace carve(void* ws, const Geom& g) {
  char* p = static_cast<char*>(ws);
  Workspace w;
  w.act = reinterpret_cast<double*>(p);
  w.kin = reinterpret_cast<double*>(p + region_a(g));
  w.stage = w.kin + sym::link_tiles(g);
  w.staples = p + region_a(g) + region_b(g);
  return w;
}

int check_ws(void* ws, size_t ws_bytes, const Geom& g, int prec) {
  int rc = check_ptr(ws);
  if (rc != SYM_OK) return rc;
  return ws_bytes >= ws_bytes_for(g, prec) ? SYM_OK : SYM_EWORKSPACE;
}

int hip_status(hipError_t e) { return e == hipSuccess ? SYM_OK : SYM_EHIP; }

// ------------------------------------------------------ static scratch memory
// Workspace of sym_force_static, for callers that cannot allocate device memory: a
// fixed array in the library's device image, one copy per GPU, held until the process
// ends. In host code `scratch` only names the symbol; its device address on the current
// GPU comes from hipGetSymbolAddress, taken once per device on the first call there
// and kept. Every call on one GPU shares that GPU's copy.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int static_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SYM_EHIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return SYM_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SYM_OK;
}

size_t link_field_bytes(const Geom& g, int prec) {
  const size_t real = prec == SYM_F64 ? sizeof(double) : sizeof(float);
  return (size_t)8 * 9 * 2 * real * (size_t)g.Vh;  // 4 directions x 2 parities x 9 complex
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  if (a == nullptr || b == nullptr) return false;
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

// A device region an entry point reads or writes.
struct Region {
  const void* p;
  size_t n;
};

// The kernels read neighbouring links (and workspace intermediates) while writing their
// outputs, so no two regions of one call may overlap (NULL regions are skipped).
int check_disjoint(std::initializer_list<Region> rs) {
  for (auto a = rs.begin(); a != rs.end(); ++a)
    for (auto b = a + 1; b != rs.end(); ++b)
      if (overlap(a->p, a->n, b->p, b->n)) return SYM_EINVAL;
  return SYM_OK;
}

// ------------------------------------------------------------ kernel timing
struct TimedLaunch {
  const char* name;
  hipEvent_t start, stop;
};
std::mutex g_prof_mu;
std::atomic<bool> g_prof_on{false};
std::vector<TimedLaunch> g_prof_pending;
std::vector<hipEvent_t> g_prof_pool;

hipEvent_t prof_event() {
  if (!g_prof_pool.empty()) {
    hipEvent_t e = g_prof_pool.back();
    g_prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Run `launch` (which enqueues one kernel on s); bracket it with events when profiling.
template <class F>
hipError_t timed(const char* name, hipStream_t s, F&& launch) {
  if (!g_prof_on.load()) return launch();
  std::lock_guard<std::mutex> lk(g_prof_mu);
  hipEvent_t a = prof_event(), b = prof_event();
  bool ok = a != nullptr && b != nullptr && hipEventRecord(a, s) == hipSuccess;
  const hipError_t e = launch();
  ok = ok && hipEventRecord(b, s) == hipSuccess;
  if (ok) {
    g_prof_pending.push_back(TimedLaunch{name, a, b});
  } else {
    if (a) g_prof_pool.push_back(a);
    if (b) g_prof_pool.push_back(b);
  }
  return e;
}

// The force algorithm is read once per ABI call and passed down, so that the launch and
// the finish of one call always agree even if another thread switches the algorithm.
bool use_factored() {
  const int a = g_algorithm.load();
  return a == SYM_ALG_FACTORED || a == SYM_ALG_AUTO;
}

// One force evaluation; G goes to `out` (Store) or is subtracted, times `kick`, from the
// momenta in `out` (Kick). With act != nullptr the per-workgroup staple partials go there.
template <typename T>
hipError_t force_into(bool factored, const Geom& g, const T* U, T* out, double kick, double* act, const Coeffs& c,
                      ForceOut mode, const Workspace& w, hipStream_t s) {
  if (factored) {
    T* S8 = static_cast<T*>(w.staples);
    hipError_t e = timed("staples", s, [&] { return sym::launch_staples<T>(g, U, S8, s); });
    if (e != hipSuccess) return e;
    return timed("force_factored", s,
                 [&] { return sym::launch_force_factored<T>(g, U, S8, out, kick, act, c, mode, s); });
  }
  return timed("force_direct", s, [&] { return sym::launch_force_direct<T>(g, U, out, kick, act, c, mode, s); });
}

template <typename T>
int force_tiles(bool factored, const Geom& g) {
  return factored ? sym::factored_tiles<T>(g) : sym::link_tiles(g);
}
int force_kind(bool factored) { return factored ? 2 : 0; }

// The factored kernels fold the short-side rectangles and the cube loops into one
// c-weighted partial; W_C is recovered from it by dividing by c_C, which is impossible
// when c_C = 0 (u0 = 1, or an override). The action kernel then supplies S and W.
bool fused_action_ok(bool factored, const Coeffs& c) { return !factored || c.c[2] != 0.0; }

template <typename T>
hipError_t action_into(const Geom& g, const Coeffs& c, const T* U, double* S_dev, const Workspace& w, hipStream_t s) {
  hipError_t e = timed("action", s, [&] { return sym::launch_action<T>(g, U, w.act, s); });
  if (e == hipSuccess)
    e = timed("finish", s, [&] { return sym::launch_finish_action(w.act, sym::action_tiles(g), 1, g, c, w.stage, S_dev, s); });
  return e;
}

// Force (Store) or gradient (Grad) of one lattice, with the action from the fused
// partials of the same pass when they determine it, else from the action kernel.
template <typename T>
int do_force(bool factored, const Geom& g, const Coeffs& c, const void* Uv, void* out, double* S_dev, ForceOut mode,
             const Workspace& w, hipStream_t s) {
  const T* U = static_cast<const T*>(Uv);
  const bool fused = S_dev != nullptr && fused_action_ok(factored, c);
  hipError_t e = force_into<T>(factored, g, U, static_cast<T*>(out), 0.0, fused ? w.act : nullptr, c, mode, w, s);
  if (e == hipSuccess && fused)
    e = timed("finish", s, [&] {
      return sym::launch_finish_action(w.act, force_tiles<T>(factored, g), force_kind(factored), g, c, w.stage, S_dev,
                                       s);
    });
  else if (e == hipSuccess && S_dev)
    e = action_into<T>(g, c, U, S_dev, w, s);
  return hip_status(e);
}

template <typename T>
int do_action(const Geom& g, const Coeffs& c, const void* U, double* S_dev, const Workspace& w, hipStream_t s) {
  return hip_status(action_into<T>(g, c, static_cast<const T*>(U), S_dev, w, s));
}

template <typename T>
hipError_t hamiltonian(const Geom& g, const Coeffs& c, const T* U, const T* P, double* out, const Workspace& w,
                       hipStream_t s) {
  hipError_t e = timed("action", s, [&] { return sym::launch_action<T>(g, U, w.act, s); });
  if (e == hipSuccess) e = timed("kinetic", s, [&] { return sym::launch_kinetic<T>(g, P, w.kin, s); });
  if (e == hipSuccess)
    e = timed("finish", s, [&] {
      return sym::launch_finish_hamiltonian(w.act, sym::action_tiles(g), 1, w.kin, sym::link_tiles(g), g, c, w.stage,
                                            out, s);
    });
  return e;
}

template <typename T>
int do_leapfrog(bool factored, const Geom& g, const Coeffs& c, void* Uv, void* Pv, double dt, int nsteps,
                double* H_dev, const Workspace& w, hipStream_t s) {
  T* U = static_cast<T*>(Uv);
  T* P = static_cast<T*>(Pv);
  hipError_t e = hipSuccess;
  if (nsteps == 0) {
    if (H_dev) e = hamiltonian<T>(g, c, U, P, H_dev, w, s);
    if (H_dev && e == hipSuccess) e = hamiltonian<T>(g, c, U, P, H_dev + 1, w, s);
    return hip_status(e);
  }
  // The first force pass sees U at the start and the last one U at the end: their
  // fused action partials give S for H, with the kinetic energy of P taken before the
  // first kick and after the last.
  auto finish_h = [&](double* out) {
    return timed("finish", s, [&] {
      return sym::launch_finish_hamiltonian(w.act, force_tiles<T>(factored, g), force_kind(factored), w.kin,
                                            sym::link_tiles(g), g, c, w.stage, out, s);
    });
  };
  double* act = H_dev ? w.act : nullptr;
  if (H_dev) e = timed("kinetic", s, [&] { return sym::launch_kinetic<T>(g, P, w.kin, s); });
  if (e == hipSuccess) e = force_into<T>(factored, g, U, P, 0.5 * dt, act, c, ForceOut::Kick, w, s);
  if (H_dev && e == hipSuccess) e = finish_h(H_dev);
  for (int it = 0; it < nsteps && e == hipSuccess; ++it) {
    e = timed("drift", s, [&] { return sym::launch_drift<T>(g, U, P, dt, s); });
    if (e == hipSuccess) {
      const bool last = it + 1 == nsteps;
      e = force_into<T>(factored, g, U, P, last ? 0.5 * dt : dt, last ? act : nullptr, c, ForceOut::Kick, w, s);
    }
  }
  if (H_dev && e == hipSuccess) e = timed("kinetic", s, [&] { return sym::launch_kinetic<T>(g, P, w.kin, s); });
  if (H_dev && e == hipSuccess) e = finish_h(H_dev + 1);
  return hip_status(e);
}

// ------------------------------------------------------------ batched force
// Workspace: [partials: 3 doubles per tile of the largest launch chunk, counted with the
//             smallest workgroup any schedule uses]
//            [per lattice: plaquette-staple buffer, 256-byte aligned]
constexpr int kMinBatchLinks = 128;
struct BatchPlan {
  std::vector<Geom> g;
  std::vector<size_t> s8_off;
  size_t part_bytes = 0;
  size_t stage_off = 0;  // doubles from the start of the partials region
  size_t total = 0;
};

int batch_plan(int n, const int32_t* L, int prec, BatchPlan* plan) {
  if (n < 1) return SYM_EINVAL;
  if (L == nullptr) return SYM_ENULL;
  int rc = check_prec(prec);
  if (rc != SYM_OK) return rc;
  plan->g.resize(n);
  plan->s8_off.resize(n);
  long long max_chunk_tiles = 0;
  for (int c0 = 0; c0 < n; c0 += sym::kMaxBatch) {
    long long tiles = 0;
    for (int i = c0; i < n && i < c0 + sym::kMaxBatch; ++i) {
      if ((rc = make_geom(L + 4 * i, &plan->g[i])) != SYM_OK) return rc;
      tiles += sym::link_tiles(plan->g[i], kMinBatchLinks);  // the most tiles any schedule uses
    }
    if (tiles > (1ll << 30)) return SYM_EINVAL;
    max_chunk_tiles = tiles > max_chunk_tiles ? tiles : max_chunk_tiles;
  }
  // per-tile partials, then the stage of the final reduction (c_C = 0 only)
  plan->stage_off = 3 * (size_t)max_chunk_tiles;
  plan->part_bytes = align256(sizeof(double) * (3 * (size_t)max_chunk_tiles + sym::kFinishStage));
  size_t off = plan->part_bytes;
  for (int i = 0; i < n; ++i) {
    plan->s8_off[i] = off;
    off += region_c(plan->g[i], prec);
  }
  plan->total = off;
  return SYM_OK;
}

// Schedule of the batched force pass.
//   grid: number of persistent workgroups, or 0 for one workgroup per tile (the launch
//         covers every tile of its lattices and the hardware dispatcher balances them);
//   order: tile order (0 strided, 1 XCD-contiguous, see BatchTable);
//   links: links (threads) per workgroup, 256 or 128;
//   lds_kib: dynamic LDS reserved per workgroup, capping the workgroups per CU (160 KiB
//            of LDS) and hence the waves per SIMD; -1 = the single-lattice default.
struct Schedule {
  int grid;
  int order;
  int links;
  int lds_kib;
};
std::mutex g_tune_mu;
std::map<std::vector<int>, Schedule> g_tune;

std::vector<int> tune_key(int n, const int32_t* L, int prec) {
  std::vector<int> k{prec, n};
  for (int i = 0; i < 4 * n; ++i) k.push_back(L[i]);
  return k;
}

Schedule default_schedule(int) {
  // one workgroup of 256 links per tile, XCD-contiguous, the single-lattice occupancy:
  // on 64 lattices from {8^4, 12^4, 16^3x32} (FP32) 4.43 ms, against 5.41 ms for 64
  // single-lattice calls
  return Schedule{0, 1, 256, -1};
}

template <typename T>
hipError_t force_batch_run(int n, const BatchPlan& plan, const Coeffs& c, const void* const* U, void* const* F,
                           double* S_dev, void* ws, const Schedule& sch, hipStream_t s) {
  char* base = static_cast<char*>(ws);
  double* parts = reinterpret_cast<double*>(base);
  hipError_t e = hipSuccess;
  for (int c0 = 0; c0 < n && e == hipSuccess; c0 += sym::kMaxBatch) {
    sym::BatchTable b;
    memset(&b, 0, sizeof b);
    b.n = (n - c0) < sym::kMaxBatch ? (n - c0) : sym::kMaxBatch;
    b.order = sch.order;
    int tiles = 0, site_tiles = 0;
    for (int k = 0; k < b.n; ++k) {
      const int i = c0 + k;
      sym::BatchEntry& en = b.e[k];
      en.U = U[i];
      en.F = F[i];
      en.S8 = base + plan.s8_off[i];
      for (int a = 0; a < 4; ++a) en.L[a] = plan.g[i].L[a];
      en.Vh = plan.g[i].Vh;
      en.tile_begin = tiles;
      en.site_tile_begin = site_tiles;
      tiles += sym::link_tiles(plan.g[i], sch.links);
      site_tiles += sym::site_tiles(plan.g[i]);
    }
    b.total_tiles = tiles;
    b.total_site_tiles = site_tiles;
    const int grid = sch.grid > 0 ? sch.grid : (sch.order == 1 ? (tiles + 7) / 8 * 8 : tiles);
    e = timed("staples_batch", s, [&] { return sym::launch_staples_batch<T>(b, sch.grid, s); });
    if (e == hipSuccess)
      e = timed("force_batch", s,
                [&] { return sym::launch_force_batch<T>(b, grid, sch.links, sch.lds_kib, parts, c, s); });
    if (e == hipSuccess && S_dev && c.c[2] != 0.0)
      e = timed("finish_batch", s, [&] { return sym::launch_finish_batch(b, parts, c, S_dev + 4 * c0, s); });
  }
  // c_C = 0: the fused partials do not determine W_C (see fused_action_ok); the action
  // kernel of each lattice supplies S and W, its partials in the batch partials region
  // (a lattice has fewer action tiles than link tiles)
  for (int i = 0; i < n && e == hipSuccess && S_dev && c.c[2] == 0.0; ++i) {
    Workspace w{parts, nullptr, parts + plan.stage_off, nullptr};
    e = action_into<T>(plan.g[i], c, static_cast<const T*>(U[i]), S_dev + 4 * i, w, s);
  }
  return e;
}

int check_batch_ptrs(int n, const void* const* U, void* const* F) {
  if (U == nullptr || F == nullptr) return SYM_ENULL;
  int rc;
  for (int i = 0; i < n; ++i)
    if ((rc = check_ptr(U[i])) || (rc = check_ptr(F[i]))) return rc;
  return SYM_OK;
}

// Every output field of a batch is disjoint from every field, from the scalars and from
// the workspace (input fields may be shared between lattices).
int check_batch_disjoint(int n, const BatchPlan& plan, int prec, const void* const* U, void* const* F,
                         const double* S_dev, const void* ws) {
  int rc;
  for (int i = 0; i < n; ++i) {
    const size_t ni = link_field_bytes(plan.g[i], prec);
    if ((rc = check_disjoint({{F[i], ni}, {S_dev, 32 * (size_t)n}, {ws, plan.total}}))) return rc;
    if ((rc = check_disjoint({{U[i], ni}, {ws, plan.total}}))) return rc;
    for (int j = 0; j < n; ++j) {
      const size_t nj = link_field_bytes(plan.g[j], prec);
      if ((rc = check_disjoint({{F[i], ni}, {U[j], nj}}))) return rc;
      if (j > i && (rc = check_disjoint({{F[i], ni}, {F[j], nj}}))) return rc;
    }
  }
  return SYM_OK;
}

}  // namespace

// ------------------------------------------------------------ fat links

namespace {

size_t fat_ws_bytes(const Geom& g, int prec) { return sym::fat::kFatFields * align256(link_field_bytes(g, prec)); }

template <typename T>
sym::fat::Fields<T> fat_carve(void* ws, const Geom& g, int prec) {
  const size_t one = align256(link_field_bytes(g, prec));
  char* p = static_cast<char*>(ws);
  sym::fat::Fields<T> w;
  w.inner = reinterpret_cast<T*>(p);
  w.M = reinterpret_cast<T*>(p + 3 * one);
  w.gmid = reinterpret_cast<T*>(p + 9 * one);
  w.gT1 = reinterpret_cast<T*>(p + 12 * one);
  w.D = reinterpret_cast<T*>(p + 18 * one);
  return w;
}

int fat_coeffs(const double* c, sym::fat::FatCoeffs* out) {
  if (c == nullptr) return SYM_ENULL;
  for (int k = 0; k < 6; ++k) {
    if (!isfinite(c[k])) return SYM_EINVAL;
    out->c[k] = c[k];
  }
  return SYM_OK;
}

template <typename T>
int do_fat_links(const Geom& g, const sym::fat::FatCoeffs& c, const void* U, void* V, void* W,
                 const sym::fat::Fields<T>& w, hipStream_t s) {
  const T* u = static_cast<const T*>(U);
  hipError_t e = timed("fat_fk1", s, [&] { return sym::launch_fat_stage<T>(0, g, u, nullptr, nullptr, nullptr, 0, c, w, s); });
  if (e == hipSuccess)
    e = timed("fat_fk2", s, [&] { return sym::launch_fat_stage<T>(1, g, u, nullptr, nullptr, nullptr, 0, c, w, s); });
  if (e == hipSuccess)
    e = timed("fat_fk3", s, [&] {
      return sym::launch_fat_fk3<T>(g, u, static_cast<T*>(V), static_cast<T*>(W), c, w, s);
    });
  return hip_status(e);
}

template <typename T>
int do_fat_force(const Geom& g, const sym::fat::FatCoeffs& c, const void* U, const void* GV, const void* GW,
                 void* out, int mode, const sym::fat::Fields<T>& w, hipStream_t s) {
  const T* u = static_cast<const T*>(U);
  const T* gv = static_cast<const T*>(GV);
  const T* gw = static_cast<const T*>(GW);
  T* o = static_cast<T*>(out);
  static const char* names[5] = {"fat_fk1", "fat_fk2", "fat_bk3", "fat_bk2", "fat_gk"};
  hipError_t e = hipSuccess;
  // with SYM_FAT_REUSE_LINKS the workspace already holds what FK1 and FK2 write
  const int first = (mode & SYM_FAT_REUSE_LINKS) ? 2 : 0, out_mode = mode & SYM_FAT_FORCE;
  for (int stage = first; stage < 5 && e == hipSuccess; ++stage)
    e = timed(names[stage], s, [&] { return sym::launch_fat_stage<T>(stage, g, u, gv, gw, o, out_mode, c, w, s); });
  return hip_status(e);
}

size_t wilson_ws(const Geom& g, int prec) {
  const size_t rb = prec == SYM_F64 ? sizeof(double) : sizeof(float);
  return align256((size_t)2 * 6 * 9 * rb * (size_t)g.Vh);  // six anti-Hermitian matrices per site
}

}  // namespace

extern "C" {

size_t sym_batch_workspace_bytes(int n, const int32_t* L, int prec) {
  BatchPlan plan;
  return batch_plan(n, L, prec, &plan) == SYM_OK ? plan.total : 0;
}

int sym_force_batch(int n, const int32_t* L, double u0, double beta, int prec, const void* const* U, void* const* F,
                    double* S_dev, void* ws, size_t ws_bytes, sym_stream_t stream) {
  BatchPlan plan;
  Coeffs c;
  int rc;
  if ((rc = batch_plan(n, L, prec, &plan)) || (rc = make_coeffs(u0, beta, &c)) || (rc = check_batch_ptrs(n, U, F)) ||
      (S_dev && (rc = check_ptr(S_dev))) || (rc = check_ptr(ws)))
    return rc;
  if (ws_bytes < plan.total) return SYM_EWORKSPACE;
  if ((rc = check_batch_disjoint(n, plan, prec, U, F, S_dev, ws))) return rc;
  Schedule sch = default_schedule(prec);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(tune_key(n, L, prec));
    if (it != g_tune.end()) sch = it->second;
  }
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const hipError_t e = prec == SYM_F64 ? force_batch_run<double>(n, plan, c, U, F, S_dev, ws, sch, s)
                                       : force_batch_run<float>(n, plan, c, U, F, S_dev, ws, sch, s);
  return hip_status(e);
}

int sym_batch_autotune(int n, const int32_t* L, double u0, double beta, int prec, const void* const* U, void* const* F,
                       void* ws, size_t ws_bytes, sym_stream_t stream, int32_t* schedule_out, int32_t max_log,
                       int32_t* log_schedules, float* log_ms, int32_t* n_log_out) {
  BatchPlan plan;
  Coeffs c;
  int rc;
  if ((rc = batch_plan(n, L, prec, &plan)) || (rc = make_coeffs(u0, beta, &c)) || (rc = check_batch_ptrs(n, U, F)) ||
      (rc = check_ptr(ws)))
    return rc;
  if (max_log < 0) return SYM_EINVAL;
  if (ws_bytes < plan.total) return SYM_EWORKSPACE;
  if ((rc = check_batch_disjoint(n, plan, prec, U, F, nullptr, ws))) return rc;
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    return SYM_EHIP;
  }
  Schedule best = default_schedule(prec);
  float best_ms = -1.0f;
  int nlog = 0;
  // links per workgroup x occupancy cap (LDS KiB per workgroup: none, the default, one
  // workgroup per CU) x grid (one workgroup per tile, or persistent) x tile order; the
  // last candidate timed is 512 persistent workgroups of 128 links in XCD-contiguous order
  // with one workgroup per CU
  const int linkss[] = {256, 128};
  const int ldss[] = {0, -1, 96};
  const int grids[] = {0, 2048, 1024, 512};
  hipError_t e = hipSuccess;
  for (int li = 0; li < 2 && e == hipSuccess; ++li)
    for (int lds : ldss)
      for (int grid : grids)
        for (int order = 0; order < 2 && e == hipSuccess; ++order) {
          const Schedule sch{grid, order, linkss[li], lds};
          auto run = [&] {
            return prec == SYM_F64 ? force_batch_run<double>(n, plan, c, U, F, nullptr, ws, sch, s)
                                   : force_batch_run<float>(n, plan, c, U, F, nullptr, ws, sch, s);
          };
          if ((e = run()) != hipSuccess) break;  // warm-up
          if ((e = hipEventRecord(a, s)) != hipSuccess) break;
          for (int r = 0; r < 3 && e == hipSuccess; ++r) e = run();
          if (e == hipSuccess) e = hipEventRecord(b, s);
          if (e == hipSuccess) e = hipEventSynchronize(b);
          float ms = 0.0f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
          if (e != hipSuccess) break;
          ms /= 3.0f;
          if (nlog < max_log) {
            if (log_schedules) {
              log_schedules[4 * nlog + 0] = sch.grid;
              log_schedules[4 * nlog + 1] = sch.order;
              log_schedules[4 * nlog + 2] = sch.links;
              log_schedules[4 * nlog + 3] = sch.lds_kib;
            }
            if (log_ms) log_ms[nlog] = ms;
            ++nlog;
          }
          if (best_ms < 0.0f || ms < best_ms) {
            best_ms = ms;
            best = sch;
          }
        }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return SYM_EHIP;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[tune_key(n, L, prec)] = best;
  }
  if (schedule_out) {
    schedule_out[0] = best.grid;
    schedule_out[1] = best.order;
    schedule_out[2] = best.links;
    schedule_out[3] = best.lds_kib;
  }
  if (n_log_out) *n_log_out = nlog;
  return SYM_OK;
}


int sym_coeffs(double u0, double c_out[3], double* alpha_s_out) {
  if (c_out == nullptr) return SYM_ENULL;
  if (!(u0 > 0.0) || !isfinite(u0)) return SYM_EINVAL;
  const double as = -4.0 * log(u0) / 3.06839;
  c_out[0] = 1.0;
  c_out[1] = -(1.0 + 0.4805 * as) / (20.0 * u0 * u0);
  c_out[2] = -2.0 * 0.03325 * as / (u0 * u0);
  if (alpha_s_out) *alpha_s_out = as;
  return SYM_OK;
}

size_t sym_workspace_bytes(const int32_t L[4], int prec) {
  Geom g;
  if (make_geom(L, &g) != SYM_OK || check_prec(prec) != SYM_OK) return 0;
  return ws_bytes_for(g, prec);
}

int sym_action(const int32_t L[4], double u0, double beta, int prec, const void* U, double* S_dev, void* ws,
               size_t ws_bytes, sym_stream_t stream) {
  Geom g;
  Coeffs c;
  int rc;
  if ((rc = make_geom(L, &g)) || (rc = check_prec(prec)) || (rc = make_coeffs(u0, beta, &c)) || (rc = check_ptr(U)) ||
      (rc = check_ptr(S_dev)) || (rc = check_ws(ws, ws_bytes, g, prec)) ||
      (rc = check_disjoint({{U, link_field_bytes(g, prec)}, {S_dev, 32}, {ws, ws_bytes_for(g, prec)}})))
    return rc;
  const Workspace w = carve(ws, g);
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return prec == SYM_F64 ? do_action<double>(g, c, U, S_dev, w, s) : do_action<float>(g, c, U, S_dev, w, s);
}

int sym_force(const int32_t L[4], double u0, double beta, int prec, const void* U, void* F, double* S_dev, void* ws,
              size_t ws_bytes, sym_stream_t stream) {
  Geom g;
  Coeffs c;
  int rc;
  if ((rc = make_geom(L, &g)) || (rc = check_prec(prec)) || (rc = make_coeffs(u0, beta, &c)) || (rc = check_ptr(U)) ||
      (rc = check_ptr(F)) || (S_dev && (rc = check_ptr(S_dev))) || (rc = check_ws(ws, ws_bytes, g, prec)) ||
      (rc = check_disjoint({{U, link_field_bytes(g, prec)}, {F, link_field_bytes(g, prec)}, {S_dev, 32},
                            {ws, ws_bytes_for(g, prec)}})))
    return rc;
  const Workspace w = carve(ws, g);
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool fac = use_factored();
  return prec == SYM_F64 ? do_force<double>(fac, g, c, U, F, S_dev, ForceOut::Store, w, s)
                         : do_force<float>(fac, g, c, U, F, S_dev, ForceOut::Store, w, s);
}

int sym_force_static(const int32_t L[4], double u0, double beta, int prec, const void* U, void* F, double* S_dev,
                     sym_stream_t stream) {
  Geom g;
  Coeffs c;
  int rc;
  if ((rc = make_geom(L, &g)) || (rc = check_prec(prec)) || (rc = make_coeffs(u0, beta, &c)) || (rc = check_ptr(U)) ||
      (rc = check_ptr(F)) || (S_dev && (rc = check_ptr(S_dev))))
    return rc;
  if (ws_bytes_for(g, prec) > kStaticScratchBytes) return SYM_EWORKSPACE;
  void* ws = nullptr;
  if ((rc = static_scratch(&ws))) return rc;
  if ((rc = check_disjoint({{U, link_field_bytes(g, prec)}, {F, link_field_bytes(g, prec)}, {S_dev, 32},
                            {ws, ws_bytes_for(g, prec)}})))
    return rc;
  const Workspace w = carve(ws, g);
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool fac = use_factored();
  return prec == SYM_F64 ? do_force<double>(fac, g, c, U, F, S_dev, ForceOut::Store, w, s)
                         : do_force<float>(fac, g, c, U, F, S_dev, ForceOut::Store, w, s);
}

int sym_action_grad(const int32_t L[4], double u0, double beta, int prec, const void* U, void* grad, double* S_dev,
                    void* ws, size_t ws_bytes, sym_stream_t stream) {
  Geom g;
  Coeffs c;
  int rc;
  if ((rc = make_geom(L, &g)) || (rc = check_prec(prec)) || (rc = make_coeffs(u0, beta, &c)) || (rc = check_ptr(U)) ||
      (rc = check_ptr(grad)) || (S_dev && (rc = check_ptr(S_dev))) || (rc = check_ws(ws, ws_bytes, g, prec)) ||
      (rc = check_disjoint({{U, link_field_bytes(g, prec)}, {grad, link_field_bytes(g, prec)}, {S_dev, 32},
                            {ws, ws_bytes_for(g, prec)}})))
    return rc;
  const Workspace w = carve(ws, g);
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool fac = use_factored();
  return prec == SYM_F64 ? do_force<double>(fac, g, c, U, grad, S_dev, ForceOut::Grad, w, s)
                         : do_force<float>(fac, g, c, U, grad, S_dev, ForceOut::Grad, w, s);
}

int md_leapfrog(const int32_t L[4], double u0, double beta, int prec, void* U, void* P, double dt, int32_t nsteps,
                double* H_dev, void* ws, size_t ws_bytes, sym_stream_t stream) {
  Geom g;
  Coeffs c;
  int rc;
  if ((rc = make_geom(L, &g)) || (rc = check_prec(prec)) || (rc = make_coeffs(u0, beta, &c)) || (rc = check_ptr(U)) ||
      (rc = check_ptr(P)) || (H_dev && (rc = check_ptr(H_dev))) || (rc = check_ws(ws, ws_bytes, g, prec)))
    return rc;
  if (!isfinite(dt) || nsteps < 0) return SYM_EINVAL;
  if ((rc = check_disjoint({{U, link_field_bytes(g, prec)}, {P, link_field_bytes(g, prec)}, {H_dev, 16},
                            {ws, ws_bytes_for(g, prec)}})))
    return rc;
  const Workspace w = carve(ws, g);
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool fac = use_factored();
  return prec == SYM_F64 ? do_leapfrog<double>(fac, g, c, U, P, dt, nsteps, H_dev, w, s)
                         : do_leapfrog<float>(fac, g, c, U, P, dt, nsteps, H_dev, w, s);
}

int sym_check_links(const int32_t L[4], int prec, const void* U, double* out_dev, void* ws, size_t ws_bytes,
                    sym_stream_t stream) {
  Geom g;
  int rc;
  if ((rc = make_geom(L, &g)) || (rc = check_prec(prec)) || (rc = check_ptr(U)) || (rc = check_ptr(out_dev)) ||
      (rc = check_ws(ws, ws_bytes, g, prec)) ||
      (rc = check_disjoint({{U, link_field_bytes(g, prec)}, {out_dev, 24}, {ws, ws_bytes_for(g, prec)}})))
    return rc;
  const Workspace w = carve(ws, g);
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const hipError_t e = timed("check_links", s, [&] {
    return prec == SYM_F64 ? sym::launch_check_links<double>(g, static_cast<const double*>(U), w.act, out_dev, s)
                           : sym::launch_check_links<float>(g, static_cast<const float*>(U), w.act, out_dev, s);
  });
  return hip_status(e);
}

int sym_reunitarise(const int32_t L[4], int prec, void* U, sym_stream_t stream) {
  Geom g;
  int rc;
  if ((rc = make_geom(L, &g)) || (rc = check_prec(prec)) || (rc = check_ptr(U))) return rc;
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const hipError_t e = timed("reunitarise", s, [&] {
    return prec == SYM_F64 ? sym::launch_reunitarise<double>(g, static_cast<double*>(U), s)
                           : sym::launch_reunitarise<float>(g, static_cast<float*>(U), s);
  });
  return hip_status(e);
}

int sym_pack(const int32_t L[4], int prec, const void* aos_lex, void* soa, sym_stream_t stream) {
  Geom g;
  int rc;
  if ((rc = make_geom(L, &g)) || (rc = check_prec(prec)) || (rc = check_ptr(aos_lex)) || (rc = check_ptr(soa)))
    return rc;
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = timed("pack", s, [&] {
    return prec == SYM_F64
               ? sym::launch_pack<double>(g, static_cast<const double*>(aos_lex), static_cast<double*>(soa), s)
               : sym::launch_pack<float>(g, static_cast<const float*>(aos_lex), static_cast<float*>(soa), s);
  });
  return hip_status(e);
}

int sym_unpack(const int32_t L[4], int prec, const void* soa, void* aos_lex, sym_stream_t stream) {
  Geom g;
  int rc;
  if ((rc = make_geom(L, &g)) || (rc = check_prec(prec)) || (rc = check_ptr(soa)) || (rc = check_ptr(aos_lex)))
    return rc;
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = timed("unpack", s, [&] {
    return prec == SYM_F64
               ? sym::launch_unpack<double>(g, static_cast<const double*>(soa), static_cast<double*>(aos_lex), s)
               : sym::launch_unpack<float>(g, static_cast<const float*>(soa), static_cast<float*>(aos_lex), s);
  });
  return hip_status(e);
}

size_t sym_fat_workspace_bytes(const int32_t L[4], int prec) {
  Geom g;
  if (make_geom(L, &g) != SYM_OK || check_prec(prec) != SYM_OK) return 0;
  return fat_ws_bytes(g, prec);
}

int sym_fat_links(const int32_t L[4], int prec, const double c[6], const void* U, void* V, void* W, void* ws,
                  size_t ws_bytes, sym_stream_t stream) {
  Geom g;
  sym::fat::FatCoeffs cf;
  int rc;
  if ((rc = make_geom(L, &g)) || (rc = check_prec(prec)) || (rc = fat_coeffs(c, &cf)) || (rc = check_ptr(U)) ||
      (rc = check_ptr(V)) || (W && (rc = check_ptr(W))) || (rc = check_ptr(ws)))
    return rc;
  if (ws_bytes < fat_ws_bytes(g, prec)) return SYM_EWORKSPACE;
  const size_t nf = link_field_bytes(g, prec);
  if ((rc = check_disjoint({{U, nf}, {V, nf}, {W, nf}, {ws, fat_ws_bytes(g, prec)}}))) return rc;
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return prec == SYM_F64 ? do_fat_links<double>(g, cf, U, V, W, fat_carve<double>(ws, g, prec), s)
                         : do_fat_links<float>(g, cf, U, V, W, fat_carve<float>(ws, g, prec), s);
}

int sym_fat_force(const int32_t L[4], int prec, const double c[6], const void* U, const void* GV, const void* GW,
                  void* out, int mode, void* ws, size_t ws_bytes, sym_stream_t stream) {
  Geom g;
  sym::fat::FatCoeffs cf;
  int rc;
  if ((rc = make_geom(L, &g)) || (rc = check_prec(prec)) || (rc = fat_coeffs(c, &cf)) || (rc = check_ptr(U)) ||
      (rc = check_ptr(GV)) || (GW && (rc = check_ptr(GW))) || (rc = check_ptr(out)) || (rc = check_ptr(ws)))
    return rc;
  if ((mode & ~(SYM_FAT_FORCE | SYM_FAT_REUSE_LINKS)) != 0) return SYM_EINVAL;
  if (ws_bytes < fat_ws_bytes(g, prec)) return SYM_EWORKSPACE;
  const size_t nf = link_field_bytes(g, prec);
  // U, GV and GW are only read and may coincide; the output and the workspace may not
  // overlap any of them
  if ((rc = check_disjoint({{U, nf}, {out, nf}, {ws, fat_ws_bytes(g, prec)}})) ||
      (rc = check_disjoint({{GV, nf}, {out, nf}, {ws, fat_ws_bytes(g, prec)}})) ||
      (rc = check_disjoint({{GW, nf}, {out, nf}})))
    return rc;
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return prec == SYM_F64 ? do_fat_force<double>(g, cf, U, GV, GW, out, mode, fat_carve<double>(ws, g, prec), s)
                         : do_fat_force<float>(g, cf, U, GV, GW, out, mode, fat_carve<float>(ws, g, prec), s);
}

size_t sym_wilson_workspace_bytes(const int32_t L[4], int prec) {
  Geom g;
  if (make_geom(L, &g) != SYM_OK || check_prec(prec) != SYM_OK) return 0;
  return wilson_ws(g, prec);
}

int sym_wilson_force(const int32_t L[4], int prec, double kappa, double csw, const void* U, const void* X,
                     const void* Y, void* G, void* ws, size_t ws_bytes, sym_stream_t stream) {
  Geom g;
  int rc;
  if ((rc = make_geom(L, &g)) || (rc = check_prec(prec)) || (rc = check_ptr(U)) || (rc = check_ptr(X)) ||
      (rc = check_ptr(Y)) || (rc = check_ptr(G)) || (rc = check_ptr(ws)))
    return rc;
  if (!isfinite(kappa) || !isfinite(csw)) return SYM_EINVAL;
  if (ws_bytes < wilson_ws(g, prec)) return SYM_EWORKSPACE;
  {
    // U, X and Y are only read and may coincide; G and the workspace may not overlap them
    const size_t nf = link_field_bytes(g, prec), nsp = nf / 3, nw = wilson_ws(g, prec);
    if ((rc = check_disjoint({{U, nf}, {G, nf}, {ws, nw}})) || (rc = check_disjoint({{X, nsp}, {G, nf}, {ws, nw}})) ||
        (rc = check_disjoint({{Y, nsp}, {G, nf}, {ws, nw}})))
      return rc;
  }
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e;
  if (prec == SYM_F64) {
    double* K = static_cast<double*>(ws);
    e = timed("wilson_clover", s, [&] {
      return sym::launch_wilson_clover<double>(g, static_cast<const double*>(X), static_cast<const double*>(Y), K, s);
    });
    if (e == hipSuccess)
      e = timed("wilson_force", s, [&] {
        return sym::launch_wilson_force<double>(g, static_cast<const double*>(U), static_cast<const double*>(X),
                                                static_cast<const double*>(Y), K, static_cast<double*>(G), kappa, csw,
                                                s);
      });
  } else {
    float* K = static_cast<float*>(ws);
    e = timed("wilson_clover", s, [&] {
      return sym::launch_wilson_clover<float>(g, static_cast<const float*>(X), static_cast<const float*>(Y), K, s);
    });
    if (e == hipSuccess)
      e = timed("wilson_force", s, [&] {
        return sym::launch_wilson_force<float>(g, static_cast<const float*>(U), static_cast<const float*>(X),
                                               static_cast<const float*>(Y), K, static_cast<float*>(G), kappa, csw, s);
      });
  }
  return hip_status(e);
}

int sym_pack_spinor(const int32_t L[4], int prec, const void* aos_lex, void* soa, sym_stream_t stream) {
  Geom g;
  int rc;
  if ((rc = make_geom(L, &g)) || (rc = check_prec(prec)) || (rc = check_ptr(aos_lex)) || (rc = check_ptr(soa)))
    return rc;
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const hipError_t e =
      prec == SYM_F64
          ? sym::launch_spinor_layout<double>(g, static_cast<const double*>(aos_lex), static_cast<double*>(soa), true, s)
          : sym::launch_spinor_layout<float>(g, static_cast<const float*>(aos_lex), static_cast<float*>(soa), true, s);
  return hip_status(e);
}

int sym_unpack_spinor(const int32_t L[4], int prec, const void* soa, void* aos_lex, sym_stream_t stream) {
  Geom g;
  int rc;
  if ((rc = make_geom(L, &g)) || (rc = check_prec(prec)) || (rc = check_ptr(soa)) || (rc = check_ptr(aos_lex)))
    return rc;
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const hipError_t e =
      prec == SYM_F64
          ? sym::launch_spinor_layout<double>(g, static_cast<const double*>(soa), static_cast<double*>(aos_lex), false, s)
          : sym::launch_spinor_layout<float>(g, static_cast<const float*>(soa), static_cast<float*>(aos_lex), false, s);
  return hip_status(e);
}

int sym_set_coeffs_override(const double c[3]) {
  std::lock_guard<std::mutex> lk(g_override_mu);
  if (c == nullptr) {
    g_override_on = false;
    return SYM_OK;
  }
  for (int k = 0; k < 3; ++k)
    if (!isfinite(c[k])) return SYM_EINVAL;
  for (int k = 0; k < 3; ++k) g_override[k] = c[k];
  g_override_on = true;
  return SYM_OK;
}

int sym_set_force_algorithm(int algorithm) {
  if (algorithm != SYM_ALG_AUTO && algorithm != SYM_ALG_DIRECT && algorithm != SYM_ALG_FACTORED) return SYM_EINVAL;
  g_algorithm.store(algorithm);
  return SYM_OK;
}

int sym_profile_enable(int on) {
  g_prof_on.store(on != 0);
  return SYM_OK;
}

int sym_profile_collect(int max_kinds, char* names, double* total_ms, int32_t* launches) {
  if (max_kinds < 0) return SYM_EINVAL;
  if (max_kinds > 0 && (names == nullptr || total_ms == nullptr || launches == nullptr)) return SYM_ENULL;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  int n = 0;
  int status = SYM_OK;
  for (const TimedLaunch& r : g_prof_pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(r.stop) != hipSuccess || hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess)
      status = SYM_EHIP;
    int k = 0;
    while (k < n && strncmp(names + 32 * k, r.name, 31) != 0) ++k;
    if (k == n) {
      if (n == max_kinds) continue;
      strncpy(names + 32 * k, r.name, 31);
      names[32 * k + 31] = 0;
      total_ms[k] = 0.0;
      launches[k] = 0;
      ++n;
    }
    total_ms[k] += ms;
    launches[k] += 1;
  }
  for (const TimedLaunch& r : g_prof_pending) {
    g_prof_pool.push_back(r.start);
    g_prof_pool.push_back(r.stop);
  }
  g_prof_pending.clear();
  return status == SYM_OK ? n : status;
}

const char* sym_strerror(int status) {
  switch (status) {
    case SYM_OK: return "success";
    case SYM_EINVAL: return "invalid argument (dimension, precision, scalar, algorithm or alignment)";
    case SYM_ENULL: return "required pointer is NULL";
    case SYM_EWORKSPACE: return "workspace smaller than sym_workspace_bytes()";
    case SYM_EHIP: return "HIP launch failed";
    case SYM_EUNSUPPORTED: return "not supported by this library";
    default: return "unknown status";
  }
}

}  // extern "C"
