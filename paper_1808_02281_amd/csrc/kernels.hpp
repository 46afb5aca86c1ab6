// Internal launch interface between the C ABI (sym_abi.cpp) and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "lattice.hpp"

namespace sym {

constexpr int kBlock = 256;  // threads per workgroup for the per-link kernels

// Coefficients of the three loop classes and beta (eq. 18_3_27_30, eq. 18_6_4_1).
struct Coeffs {
  double c[3];  // plaquette, rectangle, cube
  double beta;
};

// What a force kernel does with G = (beta/6)(U t)_TA: store it, subtract kick * G from
// the momenta in `out`, or store the gradient of S_G with respect to U projected on the
// tangent space of SU(3) at U, 2 G U (see sym_action_grad).
enum class ForceOut { Store = 0, Kick = 1, Grad = 2 };

// Number of workgroups of a per-link launch (a multiple of 8: 4 directions x 2 parities)
// with `links` links (threads) per workgroup.
inline int link_tiles(const Geom& g, int links = kBlock) { return ((g.Vh + links - 1) / links) * 8; }
// Number of workgroups of a per-site launch (2 parities per chunk, rounded up to a
// multiple of 8 for the XCD-contiguous order).
inline int site_tiles(const Geom& g) { return (((g.Vh + kBlock - 1) / kBlock) * 2 + 7) & ~7; }

// Each per-link force launch writes 3 doubles per workgroup: sum of Re tr(U t_X).
// The action kernel writes 3 per workgroup too (W_X partials).

// Direct force: every staple of the generated table multiplied out (Sec. II algorithm).
template <typename T>
hipError_t launch_force_direct(const Geom& g, const T* U, T* out, double kick, double* partials,
                               const Coeffs& c, ForceOut mode, hipStream_t s);

// Factored force: plaquette staples first (one pass, one thread per site), then
// rectangles and cube loops assembled from them (second pass, one thread per link).
// Staple buffer: 8 slots of 6 complex (two rows) per link (two slots unused), see
// factored.hpp. Each element plane holds V/2 + kS8Pad complex numbers (no padding at
// present; the constant is kept so that the plane stride has one definition).
constexpr int kS8Pad = 0;
__host__ __device__ inline int s8_stride(const Geom& g) { return g.Vh + kS8Pad; }
// Links per workgroup of the factored force pass: 128 (FP32) and 64 (FP64). At one or two
// waves per SIMD, small workgroups let each SIMD take new work as soon as its own wave
// finishes instead of waiting for the workgroup's other waves: 2.46 -> 2.42 ms (FP32) and
// 5.49 -> 5.20 ms (FP64) on the 32^3 x 64 workload, against 256 links per workgroup.
template <typename T>
constexpr int factored_links() {
  return sizeof(T) == 4 ? 128 : 64;
}
template <typename T>
inline int factored_tiles(const Geom& g) {
  return link_tiles(g, factored_links<T>());
}
// The most per-workgroup partials any force launch writes (workspace sizing).
inline int max_force_tiles(const Geom& g) { return link_tiles(g, 64); }
// Dynamic LDS reserved by the batched force launch (default schedule) to cap resident
// workgroups of 256 links per CU (160 KiB of LDS per CU): 56 KiB -> 2 (FP32), 96 KiB -> 1
// (FP64), which is where the registers put them anyway.
template <typename T>
constexpr size_t factored_lds_reservation() {
  return sizeof(T) == 4 ? 56 * 1024 : 96 * 1024;
}
template <typename T>
hipError_t launch_staples(const Geom& g, const T* U, T* S8, hipStream_t s);
template <typename T>
hipError_t launch_force_factored(const Geom& g, const T* U, const T* S8, T* out, double kick,
                                 double* partials, const Coeffs& c, ForceOut mode, hipStream_t s);

// Batched factored force over many independent lattices (force_batch.hip). The work
// table travels by value in the kernel arguments, so a captured launch holds no host
// pointers. Tiles of all lattices are concatenated (tile_begin / site_tile_begin
// ascending); persistent workgroups walk them with a static schedule:
//   order 0: tile = blockIdx + k * grid;
//   order 1: XCD x (= blockIdx % 8) owns the x-th eighth of the tiles, walked in order.
// launch_staples_batch: grid 0 means one workgroup per site tile.
constexpr int kMaxBatch = 64;
struct BatchEntry {
  const void* U;
  void* F;
  void* S8;
  int L[4];
  int Vh;
  int tile_begin;       // first link tile of the lattice (force pass)
  int site_tile_begin;  // first site tile of the lattice (staple pass)
  int pad;
};
struct BatchTable {
  int n;
  int total_tiles;       // link tiles of all lattices
  int total_site_tiles;  // site tiles of all lattices
  int order;
  BatchEntry e[kMaxBatch];
};
template <typename T>
hipError_t launch_staples_batch(const BatchTable& b, int grid, hipStream_t s);
template <typename T>
// links: threads (links) per workgroup of the force pass, 256 or 128 (the table's link
// tiles must have been counted with it); lds_kib: dynamic LDS reserved per workgroup, which
// caps the resident workgroups per CU (negative: the single-lattice default).
hipError_t launch_force_batch(const BatchTable& b, int grid, int links, int lds_kib, double* partials,
                              const Coeffs& c, hipStream_t s);
// One block per lattice: per-lattice action from the pass-2 partials (kind 2).
hipError_t launch_finish_batch(const BatchTable& b, const double* partials, const Coeffs& c, double* out,
                               hipStream_t s);

// Action: loop products per site; W partials per workgroup.
int action_tiles(const Geom& g);
template <typename T>
hipError_t launch_action(const Geom& g, const T* U, double* partials, hipStream_t s);

// Final deterministic reduction of per-workgroup partials. All partials are "deficit"
// sums of (3 - Re tr loop), three per workgroup:
//   kind 0 (direct force): per-link sums over each class's staples (divide by 4, 6, 6);
//   kind 1 (action kernel): per-site sums over each class's loops;
//   kind 2 (factored force): plaquette / long-side rectangle / (c_R short-side
//          rectangle + c_C cube) sums, see force_factored.hip.
// launch_finish_action writes out[0..3] = S, W_P, W_R, W_C; launch_finish_hamiltonian
// adds the kinetic partials and writes out[0] = S + kinetic. Both reduce in two fixed-
// order stages through `stage` (kFinishStage doubles of workspace).
constexpr int kFinishStage = 4 * 64;
hipError_t launch_finish_action(const double* partials, int nparts, int kind, const Geom& g,
                                const Coeffs& c, double* stage, double* out, hipStream_t s);

// Leapfrog pieces.
template <typename T>
hipError_t launch_kinetic(const Geom& g, const T* P, double* partials, hipStream_t s);
hipError_t launch_finish_hamiltonian(const double* act_parts, int nact, int act_kind,
                                     const double* kin_parts, int nkin, const Geom& g,
                                     const Coeffs& c, double* stage, double* out, hipStream_t s);
template <typename T>
hipError_t launch_drift(const Geom& g, T* U, const T* P, double dt, hipStream_t s);

// Link check: max over links of ||U^dagger U - 1||_F and |det U - 1| (double), and the
// number of links with a non-finite element, into out[0..2]; partials: 3 doubles per
// link tile.
template <typename T>
hipError_t launch_check_links(const Geom& g, const T* U, double* partials, double* out, hipStream_t s);

// Layout conversion between array-of-structures lexicographic complex
// (Lt,Lz,Ly,Lx,4,3,3) and the even-odd structure-of-arrays layout.
template <typename T>
hipError_t launch_pack(const Geom& g, const T* aos, T* soa, hipStream_t s);
template <typename T>
hipError_t launch_unpack(const Geom& g, const T* soa, T* aos, hipStream_t s);

// Wilson fermion force with clover term (wilson.hip): clover insertions K (6 colour
// matrices per site) from X, Y; per-link force; spinor layout conversion.
template <typename T>
hipError_t launch_wilson_clover(const Geom& g, const T* X, const T* Y, T* K, hipStream_t s);
template <typename T>
hipError_t launch_wilson_force(const Geom& g, const T* U, const T* X, const T* Y, const T* K, T* out, double kappa,
                               double csw, hipStream_t s);
template <typename T>
hipError_t launch_spinor_layout(const Geom& g, const T* src, T* dst, bool pack, hipStream_t s);

}  // namespace sym
