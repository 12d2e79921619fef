// Device helpers shared by the step kernel and the surrogate's kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace npx {

constexpr double kInvTwoPi = 0.15915494309189533577;

// sin and cos of r + q pi/2 for |r| <= pi/4: the minimax polynomials of the
// Cephes library (S. L. Moshier) on the reduced range, then the quadrant.
__device__ __forceinline__ void sin_cos_quadrant(float r, int q, float* s, float* c) {
  const float r2 = r * r;
  const float sr = fmaf(r * r2, fmaf(r2, fmaf(r2, -1.9515295891e-4f, 8.3321608736e-3f),
                                     -1.6666654611e-1f), r);
  const float cr = fmaf(r2 * r2, fmaf(r2, fmaf(r2, 2.443315711809948e-5f, -1.388731625493765e-3f),
                                      4.166664568298827e-2f), fmaf(-0.5f, r2, 1.f));
  const float ss = (q & 1) ? cr : sr;
  const float cc = (q & 1) ? sr : cr;
  *s = (q & 2) ? -ss : ss;
  *c = ((q + 1) & 2) ? -cc : cc;
}

// sin and cos of one angle. Quadrant reduction x = k pi/2 + r, |r| <= pi/4, with
// pi/2 split in two parts and fused multiply-adds (Cody & Waite), then the
// polynomials above. About 1 ulp for |x| < 1e4 rad; every angle of the step is
// far below.
__device__ __forceinline__ void sin_cos(float x, float* s, float* c) {
  const float k = rintf(x * 0.636619772367581343f);
  float r = fmaf(-k, 1.57079637050628662109375f, x);
  r = fmaf(-k, -4.37113900018624283e-8f, r);
  sin_cos_quadrant(r, (int)k, s, c);
}

// sin of 2 pi t for a phase t given in turns (double): the quarter-turn count
// and the remainder are taken in double, so only the remainder, at most pi/4,
// is rounded to float32 (about 4e-8 rad) before the polynomials.
__device__ __forceinline__ float sin_turns(double t) {
  const double x = 4.0 * (t - floor(t));
  const double k = rint(x);
  const float r = (float)((x - k) * 1.5707963267948966192);
  float s, c;
  sin_cos_quadrant(r, (int)k, &s, &c);
  return s;
}

// Every sum is an explicit fused multiply-add on a lone product, so no two
// inlined copies can contract differently: the matrix of a quaternion has
// the same bits wherever it is computed.
__device__ __forceinline__ void quat_to_mat(float w, float x, float y, float z, float R[9]) {
  const float yy_zz = fmaf(y, y, z * z), xx_zz = fmaf(x, x, z * z), xx_yy = fmaf(x, x, y * y);
  R[0] = fmaf(-2.f, yy_zz, 1.f);
  R[1] = 2.f * fmaf(x, y, -(w * z));
  R[2] = 2.f * fmaf(x, z, w * y);
  R[3] = 2.f * fmaf(x, y, w * z);
  R[4] = fmaf(-2.f, xx_zz, 1.f);
  R[5] = 2.f * fmaf(y, z, -(w * x));
  R[6] = 2.f * fmaf(x, z, -(w * y));
  R[7] = 2.f * fmaf(y, z, w * x);
  R[8] = fmaf(-2.f, xx_yy, 1.f);
}

// Cell index of a coordinate on the height-map table (Sec. III-A): floor of
// s (x - x0), clamped onto the table. It is an integer decided by arithmetic,
// so it is taken in double from the float32 coordinate: the index is then the
// exact floor for the point's own position, where float32 rounding of
// s (x - x0) would move points lying within ~1e-6 m of a cell edge across it.
// The coordinate is first held in [lo, hi] (float32 bounds chosen on the host
// half a cell outside the first and last cell edges) by one median-of-three
// (which takes a NaN coordinate to the smaller bound, lo),
// so the scaled value u = s x - s x0 (one FMA against the host's double
// -s x0) lies in about [-1/2, n - 1/2] and its truncation towards zero is the
// clamped floor.
struct HfAxis {
  double s;      // cells per metre
  double ms0;    // -s x0
  float lo, hi;  // clamp range of the coordinate, as above
};

__device__ __forceinline__ int hf_index(float x, const HfAxis& ax) {
  const float xc = __builtin_amdgcn_fmed3f(x, ax.lo, ax.hi);
  return (int)fma((double)xc, ax.s, ax.ms0);
}

// Height-map look-up (Sec. III-A): the stored height of the point's cell.
__device__ __forceinline__ float hf_lookup(const float* hf, int nx, const HfAxis& ax,
                                           const HfAxis& ay, float x, float y) {
  return hf[hf_index(y, ay) * nx + hf_index(x, ax)];
}

// Bilinear reading of the same table (the smoother-ground option): entry (i, j)
// is the height at the centre of cell (i, j); between the four surrounding
// centres the height is interpolated, beyond the outer centres it is held.
__device__ __forceinline__ float hf_bilinear(const float* hf, int nx, int ny, float x0, float y0,
                                             float s, float x, float y) {
  float u = fminf(fmaxf((x - x0) * s - 0.5f, 0.f), (float)(nx - 1));
  float w = fminf(fmaxf((y - y0) * s - 0.5f, 0.f), (float)(ny - 1));
  const int i0 = min((int)u, max(nx - 2, 0)), j0 = min((int)w, max(ny - 2, 0));
  const int i1 = min(i0 + 1, nx - 1), j1 = min(j0 + 1, ny - 1);
  const float fu = u - (float)i0, fw = w - (float)j0;
  const float h0 = hf[j0 * nx + i0] + fu * (hf[j0 * nx + i1] - hf[j0 * nx + i0]);
  const float h1 = hf[j1 * nx + i0] + fu * (hf[j1 * nx + i1] - hf[j1 * nx + i0]);
  return h0 + fw * (h1 - h0);
}

}  // namespace npx
