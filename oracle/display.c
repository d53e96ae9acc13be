/*
 * Oracle of the display path (test infrastructure only), FP64.
 *
 * The paper shows the running mean after every sampling iteration
 * (progressive rendering) and tone maps it with the Khronos PBR Neutral
 * tone mapper before it reaches the canvas (Sec. 5.1.4).  Steps per pixel,
 * in this order:
 *
 * 1. mean radiance c = sum / samples, times an exposure factor;
 * 2. PBR Neutral (Khronos, 2024): with x = min(c), an offset
 *    x - 6.25 x^2 when x < 0.08, else 0.04, is subtracted from every
 *    channel; if the new peak p = max(c) is below the start of compression
 *    s = 0.8 - 0.04 the colour is final; otherwise, with d = 1 - s, the peak
 *    is compressed to q = 1 - d^2 / (p + d - s), the colour scaled by q / p,
 *    and mixed towards the grey q by g = 1 - 1 / (0.15 (p - q) + 1);
 * 3. the sRGB transfer function (IEC 61966-2-1): 12.92 v for v <= 0.0031308,
 *    else 1.055 v^(1/2.4) - 0.055, with v clamped to [0, 1];
 * 4. 8-bit code round(255 e) (halves round up).
 */
#include <math.h>
#include <stdint.h>

#include "oracle_internal.h"

void oracle_pbr_neutral(const double in[3], double out[3]) {
  const double start = 0.8 - 0.04, desat = 0.15;
  double c[3] = {in[0], in[1], in[2]};
  double x = fmin(c[0], fmin(c[1], c[2]));
  double offset = x < 0.08 ? x - 6.25 * x * x : 0.04;
  for (int k = 0; k < 3; ++k) c[k] -= offset;
  double p = fmax(c[0], fmax(c[1], c[2]));
  if (p < start) {
    for (int k = 0; k < 3; ++k) out[k] = c[k];
    return;
  }
  double d = 1.0 - start;
  double q = 1.0 - d * d / (p + d - start);
  for (int k = 0; k < 3; ++k) c[k] *= q / p;
  double g = 1.0 - 1.0 / (desat * (p - q) + 1.0);
  for (int k = 0; k < 3; ++k) out[k] = c[k] * (1.0 - g) + q * g;
}

double oracle_srgb_encode(double v) {
  if (!(v > 0.0)) return 0.0;  /* also maps NaN to 0 */
  if (v >= 1.0) return 1.0;
  return v <= 0.0031308 ? 12.92 * v : 1.055 * pow(v, 1.0 / 2.4) - 0.055;
}

/* Display image of FP64 sums [h][w][3]: encoded values [h][w][3] in [0, 1]
 * (before quantisation) and 8-bit codes [h][w][4] (alpha 255). */
void oracle_display(const double* sum, int64_t n_pixels, double inv_samples, double exposure, double* encoded,
                    uint8_t* rgba8) {
  for (int64_t i = 0; i < n_pixels; ++i) {
    double c[3], t[3];
    for (int k = 0; k < 3; ++k) c[k] = sum[3 * i + k] * inv_samples * exposure;
    oracle_pbr_neutral(c, t);
    for (int k = 0; k < 3; ++k) {
      double e = oracle_srgb_encode(t[k]);
      if (encoded) encoded[3 * i + k] = e;
      if (rgba8) rgba8[4 * i + k] = (uint8_t)floor(255.0 * e + 0.5);
    }
    if (rgba8) rgba8[4 * i + 3] = 255;
  }
}
