// Lattice geometry and the even-odd structure-of-arrays link layout.
//
// Sites n = (x, y, z, t), x fastest, periodic in all four directions; dims even.
// Parity p = (x+y+z+t) & 1; within a parity, site n has checkerboard index
// cb = lex(n) >> 1 with lex = ((t*Lz + z)*Ly + y)*Lx + x.
//
// A link field (U, force F, momentum P) is stored as
//     field[mu][p][c][cb]  of complex T (re, im adjacent),  c = 3*row + col,
// so a wavefront reading one matrix element for 64 consecutive cb indices touches
// one contiguous 512 B (float) / 1 KiB (double) span. Element (mu, p, c, cb) is at
// complex offset ((mu*2 + p)*9 + c) * Vh + cb with Vh = V/2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "su3.hpp"

namespace sym {

struct Geom {
  int L[4];   // Lx, Ly, Lz, Lt
  int Vh;     // V / 2 sites per parity
  int Lxh;    // Lx / 2
};

// Coordinates of checkerboard index cb in parity p.
__device__ __forceinline__ void cb_coords(const Geom& g, int p, int cb, int x[4]) {
  int r = cb;
  const int xh = r % g.Lxh;
  r /= g.Lxh;
  x[1] = r % g.L[1];
  r /= g.L[1];
  x[2] = r % g.L[2];
  x[3] = r / g.L[2];
  x[0] = 2 * xh + ((p + x[1] + x[2] + x[3]) & 1);
}

// Lexicographic index contributions of the wrapped coordinates x_a + d, d = -2..2.
// lex(n + delta) = ox[dx+2] + oy[dy+2] + oz[dz+2] + ot[dt+2].
struct Nbr {
  int o[4][5];
};

__device__ __forceinline__ void make_nbr(const Geom& g, const int x[4], Nbr& nb) {
  int stride = 1;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int d = -2; d <= 2; ++d) {
      int w = x[a] + d;
      w = (w < 0) ? w + g.L[a] : w;
      w = (w >= g.L[a]) ? w - g.L[a] : w;
      nb.o[a][d + 2] = w * stride;
    }
    stride *= g.L[a];
  }
}

template <int DX, int DY, int DZ, int DT>
__device__ __forceinline__ int nbr_cb(const Nbr& nb) {
  static_assert(DX >= -2 && DX <= 2 && DY >= -2 && DY <= 2 && DZ >= -2 && DZ <= 2 && DT >= -2 && DT <= 2,
                "neighbour offsets are limited to radius 2");
  return (nb.o[0][DX + 2] + nb.o[1][DY + 2] + nb.o[2][DZ + 2] + nb.o[3][DT + 2]) >> 1;
}

template <int DX, int DY, int DZ, int DT>
constexpr int offset_parity() {
  return ((DX < 0 ? -DX : DX) + (DY < 0 ? -DY : DY) + (DZ < 0 ? -DZ : DZ) + (DT < 0 ? -DT : DT)) & 1;
}

// Base of the (mu, p) block of a link field, as complex elements.
template <typename T>
__device__ __forceinline__ const cx<T>* block_ptr(const T* field, int mu, int p, int Vh) {
  return reinterpret_cast<const cx<T>*>(field) + (size_t)((mu * 2 + p) * 9) * (size_t)Vh;
}

template <typename T>
__device__ __forceinline__ cx<T>* block_ptr(T* field, int mu, int p, int Vh) {
  return reinterpret_cast<cx<T>*>(field) + (size_t)((mu * 2 + p) * 9) * (size_t)Vh;
}

// Loads take a wave-uniform base per matrix element (scalar registers) plus one
// per-lane 32-bit byte offset shared by the nine elements.
template <typename T>
__device__ __forceinline__ su3<T> load_link(const cx<T>* __restrict__ blk, int Vh, int cb) {
  su3<T> u;
  const unsigned off = (unsigned)cb * (unsigned)sizeof(cx<T>);
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    const char* base = reinterpret_cast<const char*>(blk + (size_t)c * (size_t)Vh);
    u.e[c] = *reinterpret_cast<const cx<T>*>(base + off);
  }
  return u;
}

template <typename T>
__device__ __forceinline__ void store_link(cx<T>* __restrict__ blk, int Vh, int cb, const su3<T>& u) {
#pragma unroll
  for (int c = 0; c < 9; ++c) blk[(unsigned)(c * Vh + cb)] = u.e[c];
}

// XCD-aware tile order. The dispatcher hands consecutive workgroups to the 8 XCDs in
// turn; this permutation gives XCD k the contiguous logical tiles
// [k*n/8, (k+1)*n/8), so neighbouring tiles (which read the same neighbour links)
// share one L2. n must be a multiple of 8.
__device__ __forceinline__ int xcd_tile(int linear, int ntiles) {
  const int per = ntiles >> 3;
  return (linear & 7) * per + (linear >> 3);
}

// ------------------------------------------------------------ FP64 reductions
// Fixed-order (deterministic) sums: wavefront butterfly, then the block's waves in
// order. No atomics.

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum N doubles per thread over a block of blockDim.x (multiple of 64, <= 1024)
// threads. The block's sums end up in thread 0's v (other threads' v are partial).
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N]) {
  __shared__ double red[16][N];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) red[wave][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double s = red[0][k];
      for (int w = 1; w < nw; ++w) s += red[w][k];
      v[k] = s;
    }
  }
}

// block_sum, then thread 0 writes the N sums to out[0..N).
template <int N>
__device__ __forceinline__ void block_sum_store(double (&v)[N], double* __restrict__ out) {
  block_sum<N>(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) out[k] = v[k];
  }
}

}  // namespace sym
