// Display path for gfx950: the running mean of the FP64 per-pixel sums,
// tone mapped with Khronos PBR Neutral, sRGB-encoded and quantised to
// 8 bits per channel (the paper shows the tone-mapped running mean after
// every sampling iteration, Sec. 5.1.4).
//
// The arithmetic is FP64 end to end: the sums are FP64 already, the kernel
// is bound by HBM (24 bytes read and 4 written per pixel), and the 8-bit code
// is an integer decided by floating point, so it is decided in the precision
// of the sums.  Multiply-adds are not contracted.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pt_internal.h"

namespace pt {

#pragma clang fp contract(off)

// PBR Neutral (Khronos, 2024) of one linear colour, in place.
__device__ inline void pbr_neutral(double& r, double& g, double& b) {
  const double start = 0.8 - 0.04, desat = 0.15;
  const double x = fmin(r, fmin(g, b));
  const double offset = x < 0.08 ? x - 6.25 * x * x : 0.04;
  r -= offset;
  g -= offset;
  b -= offset;
  const double peak = fmax(r, fmax(g, b));
  if (peak < start) return;
  const double d = 1.0 - start;
  const double q = 1.0 - d * d / (peak + d - start);
  const double k = q / peak;
  r *= k;
  g *= k;
  b *= k;
  const double m = 1.0 - 1.0 / (desat * (peak - q) + 1.0);
  r = r * (1.0 - m) + q * m;
  g = g * (1.0 - m) + q * m;
  b = b * (1.0 - m) + q * m;
}

// sRGB transfer function (IEC 61966-2-1) on [0, 1]; NaN and v <= 0 give 0.
__device__ inline double srgb_encode(double v) {
  if (!(v > 0.0)) return 0.0;
  if (v >= 1.0) return 1.0;
  return v <= 0.0031308 ? 12.92 * v : 1.055 * pow(v, 1.0 / 2.4) - 0.055;
}

__device__ inline uint32_t code8(double e) { return (uint32_t)floor(255.0 * e + 0.5); }

// One pixel per lane: sums [n][3] -> rgba8 [n] (R in the low byte, alpha 255)
// and, optionally, the encoded values [n][3] as float.
__global__ __launch_bounds__(256) void k_display(const double* __restrict__ sum, int64_t n, double inv_samples,
                                                 double exposure, uint32_t* __restrict__ rgba8,
                                                 float* __restrict__ encoded) {
  for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double r = sum[3 * i + 0] * inv_samples * exposure;
    double g = sum[3 * i + 1] * inv_samples * exposure;
    double b = sum[3 * i + 2] * inv_samples * exposure;
    pbr_neutral(r, g, b);
    const double er = srgb_encode(r), eg = srgb_encode(g), eb = srgb_encode(b);
    if (rgba8) rgba8[i] = code8(er) | (code8(eg) << 8) | (code8(eb) << 16) | 0xFF000000u;
    if (encoded) {
      encoded[3 * i + 0] = (float)er;
      encoded[3 * i + 1] = (float)eg;
      encoded[3 * i + 2] = (float)eb;
    }
  }
}

hipError_t launch_display(const double* sum, int64_t n_pixels, double inv_samples, double exposure, uint32_t* rgba8,
                          float* encoded, hipStream_t st) {
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n_pixels + 255) / 256, 8192));
  hipLaunchKernelGGL(k_display, dim3((unsigned)blocks), dim3(256), 0, st, sum, n_pixels, inv_samples, exposure, rgba8,
                     encoded);
  return hipGetLastError();
}

}  // namespace pt
