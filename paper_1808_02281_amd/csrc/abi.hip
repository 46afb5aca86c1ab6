// Host side of the C ABI in include/sym.h: validation, coefficients, workspace
// carving and kernel sequencing. Nothing here allocates device memory or
// synchronises; every launch goes on the caller's stream.
#include <math.h>
#include <stdint.h>

#include <atomic>
#include <mutex>
#include <string.h>
#include <vector>

#include "../../include/sym.h"
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
// [B: per-workgroup kinetic partials] [C: plaquette staples, 8 slots of two rows per link].
struct Workspace {
  double* act;
  double* kin;
  void* staples;
};

size_t region_a(const Geom& g) {
  const int n = sym::link_tiles(g) > sym::action_tiles(g) ? sym::link_tiles(g) : sym::action_tiles(g);
  return align256(sizeof(double) * 3 * (size_t)n);
}
size_t region_b(const Geom& g) { return align256(sizeof(double) * (size_t)sym::link_tiles(g)); }
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
  w.staples = p + region_a(g) + region_b(g);
  return w;
}

int check_ws(void* ws, size_t ws_bytes, const Geom& g, int prec) {
  int rc = check_ptr(ws);
  if (rc != SYM_OK) return rc;
  return ws_bytes >= ws_bytes_for(g, prec) ? SYM_OK : SYM_EWORKSPACE;
}

int hip_status(hipError_t e) { return e == hipSuccess ? SYM_OK : SYM_EHIP; }

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

bool use_factored() {
  const int a = g_algorithm.load();
  return a == SYM_ALG_FACTORED || a == SYM_ALG_AUTO;
}

// One force evaluation; G goes to `out` (Store) or is subtracted, times `kick`, from the
// momenta in `out` (Kick). With act != nullptr the per-workgroup staple partials go there.
template <typename T>
hipError_t force_into(const Geom& g, const T* U, T* out, double kick, double* act, const Coeffs& c, ForceOut mode,
                      const Workspace& w, hipStream_t s) {
  if (use_factored()) {
    T* S8 = static_cast<T*>(w.staples);
    hipError_t e = timed("staples", s, [&] { return sym::launch_staples<T>(g, U, S8, s); });
    if (e != hipSuccess) return e;
    return timed("force_factored", s,
                 [&] { return sym::launch_force_factored<T>(g, U, S8, out, kick, act, c, mode, s); });
  }
  return timed("force_direct", s, [&] { return sym::launch_force_direct<T>(g, U, out, kick, act, c, mode, s); });
}

int force_tiles(const Geom& g) { return use_factored() ? sym::factored_tiles(g) : sym::link_tiles(g); }
int force_kind() { return use_factored() ? 2 : 0; }

template <typename T>
int do_force(const Geom& g, const Coeffs& c, const void* U, void* F, double* S_dev, const Workspace& w,
             hipStream_t s) {
  hipError_t e = force_into<T>(g, static_cast<const T*>(U), static_cast<T*>(F), 0.0, S_dev ? w.act : nullptr, c,
                               ForceOut::Store, w, s);
  if (e == hipSuccess && S_dev)
    e = timed("finish", s, [&] { return sym::launch_finish_action(w.act, force_tiles(g), force_kind(), g, c, S_dev, s); });
  return hip_status(e);
}

template <typename T>
int do_action_grad(const Geom& g, const Coeffs& c, const void* U, void* grad, double* S_dev, const Workspace& w,
                   hipStream_t s) {
  hipError_t e = force_into<T>(g, static_cast<const T*>(U), static_cast<T*>(grad), 0.0, S_dev ? w.act : nullptr, c,
                               ForceOut::Grad, w, s);
  if (e == hipSuccess && S_dev)
    e = timed("finish", s, [&] { return sym::launch_finish_action(w.act, force_tiles(g), force_kind(), g, c, S_dev, s); });
  return hip_status(e);
}

template <typename T>
int do_action(const Geom& g, const Coeffs& c, const void* U, double* S_dev, const Workspace& w, hipStream_t s) {
  hipError_t e = timed("action", s, [&] { return sym::launch_action<T>(g, static_cast<const T*>(U), w.act, s); });
  if (e == hipSuccess)
    e = timed("finish", s, [&] { return sym::launch_finish_action(w.act, sym::action_tiles(g), 1, g, c, S_dev, s); });
  return hip_status(e);
}

template <typename T>
hipError_t hamiltonian(const Geom& g, const Coeffs& c, const T* U, const T* P, double* out, const Workspace& w,
                       hipStream_t s) {
  hipError_t e = timed("action", s, [&] { return sym::launch_action<T>(g, U, w.act, s); });
  if (e == hipSuccess) e = timed("kinetic", s, [&] { return sym::launch_kinetic<T>(g, P, w.kin, s); });
  if (e == hipSuccess)
    e = timed("finish", s, [&] {
      return sym::launch_finish_hamiltonian(w.act, sym::action_tiles(g), 1, w.kin, sym::link_tiles(g), g, c, out, s);
    });
  return e;
}

template <typename T>
int do_leapfrog(const Geom& g, const Coeffs& c, void* Uv, void* Pv, double dt, int nsteps, double* H_dev,
                const Workspace& w, hipStream_t s) {
  T* U = static_cast<T*>(Uv);
  T* P = static_cast<T*>(Pv);
  hipError_t e = hipSuccess;
  if (H_dev) e = hamiltonian<T>(g, c, U, P, H_dev, w, s);
  if (nsteps > 0 && e == hipSuccess) e = force_into<T>(g, U, P, 0.5 * dt, nullptr, c, ForceOut::Kick, w, s);
  for (int it = 0; it < nsteps && e == hipSuccess; ++it) {
    e = timed("drift", s, [&] { return sym::launch_drift<T>(g, U, P, dt, s); });
    if (e == hipSuccess) {
      const double kick = (it + 1 == nsteps) ? 0.5 * dt : dt;
      e = force_into<T>(g, U, P, kick, nullptr, c, ForceOut::Kick, w, s);
    }
  }
  if (H_dev && e == hipSuccess) e = hamiltonian<T>(g, c, U, P, H_dev + 1, w, s);
  return hip_status(e);
}

}  // namespace

extern "C" {

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
      (rc = check_ptr(S_dev)) || (rc = check_ws(ws, ws_bytes, g, prec)))
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
      (rc = check_ptr(F)) || (S_dev && (rc = check_ptr(S_dev))) || (rc = check_ws(ws, ws_bytes, g, prec)))
    return rc;
  const Workspace w = carve(ws, g);
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return prec == SYM_F64 ? do_force<double>(g, c, U, F, S_dev, w, s) : do_force<float>(g, c, U, F, S_dev, w, s);
}

int sym_action_grad(const int32_t L[4], double u0, double beta, int prec, const void* U, void* grad, double* S_dev,
                    void* ws, size_t ws_bytes, sym_stream_t stream) {
  Geom g;
  Coeffs c;
  int rc;
  if ((rc = make_geom(L, &g)) || (rc = check_prec(prec)) || (rc = make_coeffs(u0, beta, &c)) || (rc = check_ptr(U)) ||
      (rc = check_ptr(grad)) || (S_dev && (rc = check_ptr(S_dev))) || (rc = check_ws(ws, ws_bytes, g, prec)))
    return rc;
  const Workspace w = carve(ws, g);
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return prec == SYM_F64 ? do_action_grad<double>(g, c, U, grad, S_dev, w, s)
                         : do_action_grad<float>(g, c, U, grad, S_dev, w, s);
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
  const Workspace w = carve(ws, g);
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return prec == SYM_F64 ? do_leapfrog<double>(g, c, U, P, dt, nsteps, H_dev, w, s)
                         : do_leapfrog<float>(g, c, U, P, dt, nsteps, H_dev, w, s);
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
    case SYM_EUNSUPPORTED: return "not supported by this build";
    default: return "unknown status";
  }
}

}  // extern "C"
