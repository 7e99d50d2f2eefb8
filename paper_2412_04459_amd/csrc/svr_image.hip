// Anti-aliased downsampling of a supersampled render and background
// compositing (Sec. 3.1.2 "Anti-aliasing": render ss times larger, then
// downsample with an anti-aliasing filter; the supplementary implementation
// details composite a background colour, the average frame colour, behind
// the remaining transmittance), and the adjoint.
//
// Filter: per axis, output pixel i of n_out takes input pixels j of n_in with
// the tent weight w(i, j) = max(0, 1 - |j - c_i| / s), s = n_in / n_out,
// c_i = (i + 1/2) s - 1/2, normalised over the in-image taps.  In integers,
// |j - c_i| / s = |(2j+1) n_out - (2i+1) n_in| / (2 n_in), so weights are
// exact to one rounding at any image size.  Then rgb += (1 - A) bg.
// One thread per output pixel (forward) or input pixel (adjoint, a gather
// over the <= 3 output pixels per axis whose taps reach it).
#include "svr_internal.h"

namespace svr {

__device__ __forceinline__ float tent_w(int i, int j, int n_in, int n_out) {
  const int64_t num = (int64_t)(2 * j + 1) * n_out - (int64_t)(2 * i + 1) * n_in;
  const float t = 1.f - (float)(num < 0 ? -num : num) / (float)(2 * (int64_t)n_in);
  return t > 0.f ? t : 0.f;
}

// first and last input index that can have a non-zero weight for output i
__device__ __forceinline__ void tent_taps(int i, int n_in, int n_out, int& lo, int& hi) {
  // |(2j+1) n_out - (2i+1) n_in| < 2 n_in  <=>  j in ((2i-1) n_in / n_out - 1, (2i+3) n_in / n_out - 1) / 2
  lo = (int)(((int64_t)(2 * i - 1) * n_in) / (2 * (int64_t)n_out)) - 1;
  hi = (int)(((int64_t)(2 * i + 3) * n_in) / (2 * (int64_t)n_out)) + 1;
  lo = max(lo, 0);
  hi = min(hi, n_in - 1);
}

__device__ __forceinline__ float tent_norm(int i, int n_in, int n_out) {
  int lo, hi;
  tent_taps(i, n_in, n_out, lo, hi);
  float t = 0.f;
  for (int j = lo; j <= hi; ++j) t += tent_w(i, j, n_in, n_out);
  return t;
}

__global__ __launch_bounds__(kBlock) void k_downsample(const float4* __restrict__ in, int w_in,
                                                       int h_in, float4* __restrict__ out,
                                                       int w_out, int h_out, float bg0, float bg1,
                                                       float bg2) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= (int64_t)w_out * h_out) return;
  const int x = (int)(p % w_out), y = (int)(p / w_out);
  int x0, x1, y0, y1;
  tent_taps(x, w_in, w_out, x0, x1);
  tent_taps(y, h_in, h_out, y0, y1);
  const float nx = 1.f / tent_norm(x, w_in, w_out), ny = 1.f / tent_norm(y, h_in, h_out);
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int j = y0; j <= y1; ++j) {
    const float wy = tent_w(y, j, h_in, h_out) * ny;
    if (wy == 0.f) continue;
    for (int k = x0; k <= x1; ++k) {
      const float w = wy * tent_w(x, k, w_in, w_out) * nx;
      const float4 v = in[(int64_t)j * w_in + k];
      acc.x = __fmaf_rn(w, v.x, acc.x);
      acc.y = __fmaf_rn(w, v.y, acc.y);
      acc.z = __fmaf_rn(w, v.z, acc.z);
      acc.w = __fmaf_rn(w, v.w, acc.w);
    }
  }
  const float T = 1.f - acc.w;
  acc.x = __fmaf_rn(T, bg0, acc.x);
  acc.y = __fmaf_rn(T, bg1, acc.y);
  acc.z = __fmaf_rn(T, bg2, acc.z);
  out[p] = acc;
}

// adjoint: grad_in[j] = sum_i w(i, j) / norm(i) * g'(i), with
// g' = (g_r, g_g, g_b, g_A - <g_rgb, bg>) (the background term of out rgb)
__global__ __launch_bounds__(kBlock) void k_downsample_bwd(const float4* __restrict__ gout,
                                                           int w_out, int h_out,
                                                           float4* __restrict__ gin, int w_in,
                                                           int h_in, float bg0, float bg1,
                                                           float bg2) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= (int64_t)w_in * h_in) return;
  const int k = (int)(p % w_in), j = (int)(p / w_in);
  // output pixels whose taps reach input k: |(2k+1) n_out - (2i+1) n_in| < 2 n_in
  const int ix0 = max(0, (int)(((int64_t)(2 * k + 1) * w_out - 2 * (int64_t)w_in) / (2 * (int64_t)w_in)) - 1);
  const int ix1 = min(w_out - 1, (int)(((int64_t)(2 * k + 1) * w_out + 2 * (int64_t)w_in) / (2 * (int64_t)w_in)) + 1);
  const int iy0 = max(0, (int)(((int64_t)(2 * j + 1) * h_out - 2 * (int64_t)h_in) / (2 * (int64_t)h_in)) - 1);
  const int iy1 = min(h_out - 1, (int)(((int64_t)(2 * j + 1) * h_out + 2 * (int64_t)h_in) / (2 * (int64_t)h_in)) + 1);
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int iy = iy0; iy <= iy1; ++iy) {
    const float wy = tent_w(iy, j, h_in, h_out);
    if (wy == 0.f) continue;
    const float wyn = wy / tent_norm(iy, h_in, h_out);
    for (int ix = ix0; ix <= ix1; ++ix) {
      const float wx = tent_w(ix, k, w_in, w_out);
      if (wx == 0.f) continue;
      const float w = wyn * wx / tent_norm(ix, w_in, w_out);
      const float4 g = gout[(int64_t)iy * w_out + ix];
      const float ga = g.w - (g.x * bg0 + g.y * bg1 + g.z * bg2);
      acc.x = __fmaf_rn(w, g.x, acc.x);
      acc.y = __fmaf_rn(w, g.y, acc.y);
      acc.z = __fmaf_rn(w, g.z, acc.z);
      acc.w = __fmaf_rn(w, ga, acc.w);
    }
  }
  gin[p] = acc;
}

hipError_t launch_downsample(const float* in, int w_in, int h_in, float* out, int w_out,
                             int h_out, const float bg[3], hipStream_t s) {
  const int64_t n = (int64_t)w_out * h_out;
  if (n == 0) return hipSuccess;
  SVR_LAUNCH("downsample", k_downsample, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
             0, s, reinterpret_cast<const float4*>(in), w_in, h_in, reinterpret_cast<float4*>(out),
             w_out, h_out, bg[0], bg[1], bg[2]);
  return hipGetLastError();
}

hipError_t launch_downsample_bwd(const float* gout, int w_out, int h_out, float* gin, int w_in,
                                 int h_in, const float bg[3], hipStream_t s) {
  const int64_t n = (int64_t)w_in * h_in;
  if (n == 0) return hipSuccess;
  SVR_LAUNCH("downsample_bwd", k_downsample_bwd, dim3((unsigned)((n + kBlock - 1) / kBlock)),
             dim3(kBlock), 0, s, reinterpret_cast<const float4*>(gout), w_out, h_out,
             reinterpret_cast<float4*>(gin), w_in, h_in, bg[0], bg[1], bg[2]);
  return hipGetLastError();
}

}  // namespace svr
