// su(3) algebra for the gauge-force kernels: 3x3 complex matrices held in registers.
//
// Real type T is float or double. Products take compile-time dagger flags so that a
// link traversed backwards (U_{n,-mu} = U^dagger_{n-mu,mu}, arXiv:1808.02281 Sec. II)
// costs nothing: conjugation and transposition fold into the operand order and the
// signs of the fused multiply-adds. One product is 27 complex multiply-adds, i.e.
// 108 FMA/MUL instructions (198 flop; 216 when accumulated into an existing matrix).
#pragma once

#include <hip/hip_runtime.h>

namespace sym {

template <typename T>
struct cx {
  T re, im;
};

template <typename T>
struct su3 {
  cx<T> e[9];  // row-major: e[3*row + col]
};

template <typename T>
__device__ __forceinline__ void set_zero(su3<T>& a) {
#pragma unroll
  for (int i = 0; i < 9; ++i) a.e[i] = cx<T>{T(0), T(0)};
}

// Element (i,k) of A or of A^dagger.
template <bool D, typename T>
__device__ __forceinline__ cx<T> elem(const su3<T>& a, int i, int k) {
  if constexpr (D) {
    return cx<T>{a.e[3 * k + i].re, -a.e[3 * k + i].im};
  } else {
    return a.e[3 * i + k];
  }
}

// C = A^{DA} B^{DB}
template <bool DA, bool DB, typename T>
__device__ __forceinline__ su3<T> mul(const su3<T>& a, const su3<T>& b) {
  su3<T> c;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cx<T> x = elem<DA>(a, i, 0), y = elem<DB>(b, 0, j);
      T re = x.re * y.re;
      T im = x.re * y.im;
      re = fma(-x.im, y.im, re);
      im = fma(x.im, y.re, im);
#pragma unroll
      for (int k = 1; k < 3; ++k) {
        x = elem<DA>(a, i, k);
        y = elem<DB>(b, k, j);
        re = fma(x.re, y.re, re);
        im = fma(x.re, y.im, im);
        re = fma(-x.im, y.im, re);
        im = fma(x.im, y.re, im);
      }
      c.e[3 * i + j] = cx<T>{re, im};
    }
  }
  return c;
}

// C += A^{DA} B^{DB}
template <bool DA, bool DB, typename T>
__device__ __forceinline__ void mac(su3<T>& c, const su3<T>& a, const su3<T>& b) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      T re = c.e[3 * i + j].re, im = c.e[3 * i + j].im;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const cx<T> x = elem<DA>(a, i, k), y = elem<DB>(b, k, j);
        re = fma(x.re, y.re, re);
        im = fma(x.re, y.im, im);
        re = fma(-x.im, y.im, re);
        im = fma(x.im, y.re, im);
      }
      c.e[3 * i + j] = cx<T>{re, im};
    }
  }
}

// C += s * A
template <typename T>
__device__ __forceinline__ void axpy(su3<T>& c, T s, const su3<T>& a) {
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    c.e[i].re = fma(s, a.e[i].re, c.e[i].re);
    c.e[i].im = fma(s, a.e[i].im, c.e[i].im);
  }
}

template <typename T>
__device__ __forceinline__ void add(su3<T>& c, const su3<T>& a) {
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    c.e[i].re += a.e[i].re;
    c.e[i].im += a.e[i].im;
  }
}

// Re tr(A B^{DB}) in T, returned as double.
template <bool DB = false, typename T>
__device__ __forceinline__ double re_tr_mul(const su3<T>& a, const su3<T>& b) {
  T s = T(0);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const cx<T> y = elem<DB>(b, k, i);
      s = fma(a.e[3 * i + k].re, y.re, s);
      s = fma(-a.e[3 * i + k].im, y.im, s);
    }
  }
  return double(s);
}

template <typename T>
__device__ __forceinline__ double re_tr(const su3<T>& a) {
  return double(a.e[0].re) + double(a.e[4].re) + double(a.e[8].re);
}

// scale * B_TA with B_TA = (B - B^dagger)/2 - tr(B - B^dagger)/6 * I (eq. 18_6_6_11).
template <typename T>
__device__ __forceinline__ su3<T> ta_scaled(const su3<T>& b, T scale) {
  su3<T> g;
  const T h = T(0.5) * scale;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = i + 1; j < 3; ++j) {
      const cx<T> bij = b.e[3 * i + j], bji = b.e[3 * j + i];
      const T re = h * (bij.re - bji.re);
      const T im = h * (bij.im + bji.im);
      g.e[3 * i + j] = cx<T>{re, im};
      g.e[3 * j + i] = cx<T>{-re, im};
    }
  }
  const T tr3 = (b.e[0].im + b.e[4].im + b.e[8].im) * T(1.0 / 3.0);
#pragma unroll
  for (int i = 0; i < 3; ++i) g.e[4 * i] = cx<T>{T(0), scale * (b.e[4 * i].im - tr3)};
  return g;
}

}  // namespace sym
