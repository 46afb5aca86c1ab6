// Projection of a 3x3 complex matrix onto SU(3) by rows, shared by the FP32 drift of the
// leapfrog (leapfrog.hip) and the field repair entry point (check.hip).
#pragma once

#include "kernels.hpp"

namespace sym {
namespace proj {

// Normalise the first row, orthogonalise the second against it (Gram-Schmidt) and
// normalise it, and set the third row to the complex conjugate of the cross product of
// the first two (det = 1). For a matrix within rounding of SU(3) it moves each element by
// the size of its unitarity defect. A row of zero norm or a non-finite element gives
// non-finite output.
__device__ __forceinline__ void project_su3(su3<double>& u) {
  using cd = cx<double>;
  double n0 = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) n0 += u.e[j].re * u.e[j].re + u.e[j].im * u.e[j].im;
  const double r0 = 1.0 / sqrt(n0);
#pragma unroll
  for (int j = 0; j < 3; ++j) u.e[j] = cd{u.e[j].re * r0, u.e[j].im * r0};
  cd ov{0.0, 0.0};  // <row0, row1> = sum conj(row0_j) row1_j
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    ov.re += u.e[j].re * u.e[3 + j].re + u.e[j].im * u.e[3 + j].im;
    ov.im += u.e[j].re * u.e[3 + j].im - u.e[j].im * u.e[3 + j].re;
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const cd t{ov.re * u.e[j].re - ov.im * u.e[j].im, ov.re * u.e[j].im + ov.im * u.e[j].re};
    u.e[3 + j] = cd{u.e[3 + j].re - t.re, u.e[3 + j].im - t.im};
  }
  double n1 = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) n1 += u.e[3 + j].re * u.e[3 + j].re + u.e[3 + j].im * u.e[3 + j].im;
  const double r1 = 1.0 / sqrt(n1);
#pragma unroll
  for (int j = 0; j < 3; ++j) u.e[3 + j] = cd{u.e[3 + j].re * r1, u.e[3 + j].im * r1};
  complete_third_row(u);
}

}  // namespace proj

// Every link of U (in place) replaced by its projection, computed in double.
template <typename T>
hipError_t launch_reunitarise(const Geom& g, T* U, hipStream_t s);

}  // namespace sym
