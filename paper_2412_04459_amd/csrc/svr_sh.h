// Real spherical-harmonic basis up to degree 3 in Cartesian form, for the
// per-voxel view-dependent colour of Sec. 3.1.1 eq. vox_color.
//
// Basis index b = l*l + l + m (m = -l..l).  Each function is
//   Y_lm = N_lm P_l^|m|(z) {cos(m phi) for m > 0, 1 for m = 0, sin(|m| phi) for m < 0}
// with N_lm = sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) times sqrt 2 for m != 0 and
// no Condon-Shortley phase, written out as polynomials in the unit direction
// (x, y, z).  The constants below are those closed forms evaluated:
//   c0  = 1/(2 sqrt(pi))          c1  = sqrt(3/(4 pi))
//   c2a = sqrt(15/pi)/2           c2b = sqrt(5/pi)/4        c2c = sqrt(15/pi)/4
//   c3a = sqrt(35/(2 pi))/4       c3b = sqrt(105/pi)/2      c3c = sqrt(21/(2 pi))/4
//   c3d = sqrt(7/pi)/4            c3e = sqrt(105/pi)/4
#pragma once

namespace svr {

constexpr float kShC0 = 0.28209479177387814f;
constexpr float kShC1 = 0.4886025119029199f;
constexpr float kShC2a = 1.0925484305920792f;
constexpr float kShC2b = 0.31539156525252005f;
constexpr float kShC2c = 0.5462742152960396f;
constexpr float kShC3a = 0.5900435899266435f;
constexpr float kShC3b = 2.890611442640554f;
constexpr float kShC3c = 0.4570457994644658f;
constexpr float kShC3d = 0.3731763325901154f;
constexpr float kShC3e = 1.445305721320277f;

// Y[0 .. (D+1)^2) for a unit direction.
template <int D>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
  Y[0] = kShC0;
  if (D >= 1) {
    Y[1] = kShC1 * y;
    Y[2] = kShC1 * z;
    Y[3] = kShC1 * x;
  }
  if (D >= 2) {
    float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kShC2a * x * y;
    Y[5] = kShC2a * y * z;
    Y[6] = kShC2b * (3.f * zz - 1.f);
    Y[7] = kShC2a * x * z;
    Y[8] = kShC2c * (xx - yy);
    if (D >= 3) {
      Y[9] = kShC3a * y * (3.f * xx - yy);
      Y[10] = kShC3b * x * y * z;
      Y[11] = kShC3c * y * (5.f * zz - 1.f);
      Y[12] = kShC3d * z * (5.f * zz - 3.f);
      Y[13] = kShC3c * x * (5.f * zz - 1.f);
      Y[14] = kShC3e * z * (xx - yy);
      Y[15] = kShC3a * x * (xx - 3.f * yy);
    }
  }
}

}  // namespace svr
