// Real spherical harmonics up to degree 3 (colour of the SH sweeping planes, Fig. 6).
//
// Index j = l^2 + l + m.  Condon-Shortley phase, in the sign convention of 3D Gaussian
// splatting: Y_l0 = Y_l^0, Y_lm = sqrt(2) Re Y_l^m (m > 0), sqrt(2) Im Y_l^|m| (m < 0),
// as polynomials of the unit direction (x, y, z).  The constants are the normalisations
// sqrt((2l + 1) / (4 pi) (l - |m|)! / (l + |m|)!) times sqrt(2) for m != 0, folded into
// the factors of each polynomial.
#pragma once

#include <hip/hip_runtime.h>

namespace lf {

constexpr int kMaxShDegree = 3;

// Floats per SH-plane texel: q_0 (r, g, b), A, q_1 .. q_{n-1} (r, g, b), padded to 4.
__host__ __device__ constexpr int sh_texel_floats(int n_coef) { return (3 * n_coef + 1 + 3) / 4 * 4; }

template <int NC>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
  Y[0] = 0.28209479177387814f;                           // 1 / (2 sqrt(pi))
  if constexpr (NC > 1) {
    constexpr float c1 = 0.48860251190291992f;           // sqrt(3 / (4 pi))
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
  }
  if constexpr (NC > 4) {
    constexpr float a = 1.0925484305920792f;             // sqrt(15 / pi) / 2
    constexpr float b = 0.31539156525252005f;            // sqrt(5 / pi) / 4
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = a * x * y;
    Y[5] = -a * y * z;
    Y[6] = b * (2.0f * zz - xx - yy);
    Y[7] = -a * x * z;
    Y[8] = 0.5f * a * (xx - yy);
  }
  if constexpr (NC > 9) {
    constexpr float e = 0.59004358992664352f;            // sqrt(35 / (2 pi)) / 4
    constexpr float f = 2.8906114426405538f;             // sqrt(105 / pi) / 2
    constexpr float g = 0.45704579946446572f;            // sqrt(21 / (2 pi)) / 4
    constexpr float h = 0.37317633259011540f;            // sqrt(7 / pi) / 4
    const float xx = x * x, yy = y * y, zz = z * z;
    const float w = 4.0f * zz - xx - yy;
    Y[9] = -e * y * (3.0f * xx - yy);
    Y[10] = f * x * y * z;
    Y[11] = -g * y * w;
    Y[12] = h * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    Y[13] = -g * x * w;
    Y[14] = 0.5f * f * z * (xx - yy);
    Y[15] = -e * x * (xx - 3.0f * yy);
  }
}

}  // namespace lf
