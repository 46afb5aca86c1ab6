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
  int tslab;  // t-slices per XCD in the t-fastest tile order (0: plain order)
  int cps;    // 256-site chunks per t-slice and parity (with tslab > 0)
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

// Link loads and stores are raw buffer operations: one resource descriptor per
// (mu, p) block (scalar registers), a per-lane 32-bit byte offset shared by the nine
// matrix elements, and a wave-uniform scalar offset per element. Accesses outside the
// block return zero (loads) or are dropped (stores) instead of faulting. Blocks stay
// below 4 GiB because V/2 <= 2^24.
constexpr int kBufferWord3 = 0x00020000;  // descriptor dword 3 for raw access on gfx9-family GPUs
// Cache policy of link stores: non-temporal. Every field a kernel writes (staples,
// forces, updated links) is far larger than L2 and is read by a later kernel, so it
// should not evict the neighbour links the running kernel is re-reading.
constexpr int kStoreNT = 2;

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t block_rsrc(const cx<T>* blk, int Vh) {
  const unsigned bytes = 9u * (unsigned)Vh * (unsigned)sizeof(cx<T>);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<cx<T>*>(blk), (short)0, (int)bytes, kBufferWord3);
}

template <typename T>
__device__ __forceinline__ su3<T> load_link(const cx<T>* blk, int Vh, int cb) {
  const __amdgpu_buffer_rsrc_t r = block_rsrc(blk, Vh);
  const int voff = cb * (int)sizeof(cx<T>);
  su3<T> u;
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    const int soff = (int)((unsigned)c * (unsigned)Vh * (unsigned)sizeof(cx<T>));
    if constexpr (sizeof(T) == 4)
      u.e[c] = __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    else
      u.e[c] = __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  }
  return u;
}

template <typename T>
__device__ __forceinline__ void store_link(cx<T>* blk, int Vh, int cb, const su3<T>& u) {
  const __amdgpu_buffer_rsrc_t r = block_rsrc(static_cast<const cx<T>*>(blk), Vh);
  const int voff = cb * (int)sizeof(cx<T>);
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    const int soff = (int)((unsigned)c * (unsigned)Vh * (unsigned)sizeof(cx<T>));
    if constexpr (sizeof(T) == 4)
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, u.e[c]),
                                            r, voff, soff, kStoreNT);
    else
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, u.e[c]),
                                             r, voff, soff, kStoreNT);
  }
}

// Special-unitary matrices stored as their first two rows (6 complex numbers): for
// U in SU(3) the third row is the complex conjugate of the cross product of the first
// two. Used for intermediate staples, which are products of SU(3) links.
template <typename T>
__device__ __forceinline__ cx<T> cross_conj(const cx<T>& a, const cx<T>& b, const cx<T>& c, const cx<T>& d) {
  // conj(a b - c d)
  T re = a.re * b.re;
  re = fma(-a.im, b.im, re);
  re = fma(-c.re, d.re, re);
  re = fma(c.im, d.im, re);
  T im = a.re * b.im;
  im = fma(a.im, b.re, im);
  im = fma(-c.re, d.im, im);
  im = fma(-c.im, d.re, im);
  return cx<T>{re, -im};
}

template <typename T>
__device__ __forceinline__ void complete_third_row(su3<T>& u) {
  u.e[6] = cross_conj(u.e[1], u.e[5], u.e[2], u.e[4]);
  u.e[7] = cross_conj(u.e[2], u.e[3], u.e[0], u.e[5]);
  u.e[8] = cross_conj(u.e[0], u.e[4], u.e[1], u.e[3]);
}

// Two-row blocks: 6 element planes of `stride` complex numbers each.
template <typename T>
__device__ __forceinline__ su3<T> load_su3_rows(const cx<T>* blk, int stride, int cb) {
  const unsigned bytes = 6u * (unsigned)stride * (unsigned)sizeof(cx<T>);
  const __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<cx<T>*>(blk), (short)0, (int)bytes, kBufferWord3);
  const int voff = cb * (int)sizeof(cx<T>);
  su3<T> u;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const int soff = (int)((unsigned)c * (unsigned)stride * (unsigned)sizeof(cx<T>));
    if constexpr (sizeof(T) == 4)
      u.e[c] = __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    else
      u.e[c] = __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  }
  complete_third_row(u);
  return u;
}

template <typename T>
__device__ __forceinline__ void store_su3_rows(cx<T>* blk, int stride, int cb, const su3<T>& u) {
  const unsigned bytes = 6u * (unsigned)stride * (unsigned)sizeof(cx<T>);
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(blk, (short)0, (int)bytes, kBufferWord3);
  const int voff = cb * (int)sizeof(cx<T>);
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const int soff = (int)((unsigned)c * (unsigned)stride * (unsigned)sizeof(cx<T>));
    if constexpr (sizeof(T) == 4)
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, u.e[c]),
                                            r, voff, soff, kStoreNT);
    else
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, u.e[c]),
                                             r, voff, soff, kStoreNT);
  }
}

// XCD-aware tile order. The dispatcher hands consecutive workgroups to the 8 XCDs in
// turn; this permutation gives XCD k the contiguous logical tiles
// [k*n/8, (k+1)*n/8), so neighbouring tiles (which read the same neighbour links)
// share one L2. n must be a multiple of 8.
__device__ __forceinline__ int xcd_tile(int linear, int ntiles) {
  const int per = ntiles >> 3;
  return (linear & 7) * per + (linear >> 3);
}

// Per-link kernels: workgroup -> (direction, parity, 256-site chunk). The 8
// (direction, parity) tiles of a chunk are adjacent. When the lattice allows it
// (Lt divisible by 8, whole chunks per t-slice) XCD k owns the t-slab
// [k Lt/8, (k+1) Lt/8) and walks it t-fastest, so that the t-neighbours of the sites
// in flight were read moments earlier and are still in that XCD's L2.
struct LinkTile {
  int mu, p, chunk;
};

// split: the number of chunks of the launch's workgroup size per 256-site chunk (1, 2 or
// 4 for 256, 128 or 64 links per workgroup); g.cps counts 256-site chunks.
__device__ __forceinline__ LinkTile link_tile(const Geom& g, int linear, int ntiles, int split = 1) {
  const int tile = xcd_tile(linear, ntiles);
  LinkTile r;
  r.mu = tile & 3;
  r.p = (tile >> 2) & 1;
  int chunk = tile >> 3;
  if (g.tslab > 0) {
    const int per = ntiles >> 6;  // chunks per XCD = tslab * cps * split
    const int xcd = chunk / per, j = chunk - xcd * per;
    chunk = (xcd * g.tslab + j % g.tslab) * (g.cps * split) + j / g.tslab;
  }
  r.chunk = chunk;
  return r;
}

// Per-site kernels (one thread per site of one parity): workgroup -> (parity,
// 256-site chunk), the two parities of a chunk adjacent, with the same XCD slabs and
// t-fastest walk as link_tile. ntiles is a multiple of 8; tiles past the lattice give
// chunks whose sites lie beyond V/2 (the kernels skip them).
struct SiteTile {
  int p, chunk;
};

__device__ __forceinline__ SiteTile site_tile(const Geom& g, int linear, int ntiles) {
  const int tile = xcd_tile(linear, ntiles);
  SiteTile r;
  r.p = tile & 1;
  int chunk = tile >> 1;
  if (g.tslab > 0) {
    const int per = ntiles >> 4;  // chunks per XCD = tslab * cps
    const int xcd = chunk / per, j = chunk - xcd * per;
    chunk = (xcd * g.tslab + j % g.tslab) * g.cps + j / g.tslab;
  }
  r.chunk = chunk;
  return r;
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
  __syncthreads();  // red[] may be reused by the next call in the same block
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
