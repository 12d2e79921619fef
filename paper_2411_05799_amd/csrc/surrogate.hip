// The simulator side of the learned surrogate: state rows, network inputs,
// 10-frame state deltas, the rollout update and the quasi-static joint-torque
// proxy of the controller-search fitness, for every instance of a world.
//
// State row of an instance (width 13 + 2 J, J = the world's joint stride):
//   c (3, world CoG), Q (4, w x y z), v (3), omega (3), q (J), q_prev (J).
// Heading frame: psi is the heading of the torso x axis on the ground plane;
// vectors are turned by -psi about z, and the orientation is left-multiplied by
// the yaw quaternion of -psi, its sign chosen so that the w component is >= 0.
// Inputs and targets are expressed in the heading frame at the current frame,
// which makes the map independent of where the robot faces.
// Network input (width 13 + 12 J + 64):
//   [0, 13)          0, 0, c_z - h(c_x, c_y), Q_h, v_h, omega_h  (position made
//                    translation-invariant: only the height above the ground)
//   [13, 13+J)       q
//   [13+J, 13+2J)    (q - q_prev) / dt
//   [13+2J, 13+12J)  the clamped commanded angles the next 10 frames apply,
//                    frame n+k for k = 0..9, k-major
//   [13+12J, +64)    8 x 8 height-map patch at 0.08 m spacing, centred on the
//                    CoG and turned with the torso heading, relative to h(c);
//                    index 8 a + b with a along the heading, b to its left
// Joints past an instance's own count read 0.  Frame n of the controller is
// the frame about to be stepped (the world's step counter).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "npx.h"
#include "npx_device.h"
#include "npx_internal.h"
#include "npx_sur_internal.h"

using npx::fail;

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(NPX_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));            \
  } while (0)

namespace {

using npx::LINK_F;
using npx::WorldView;

constexpr int HORIZON = 10;        // frames per surrogate call
constexpr int PATCH = 8;           // patch edge (cells)
constexpr float PATCH_STEP = 0.08f;  // m between patch samples
constexpr float LOW_BAND = 0.002f;   // m: a point this close to the ground carries load

__host__ __device__ inline int state_width(int J) { return 13 + 2 * J; }
__host__ __device__ inline int feature_width(int J) { return 13 + 12 * J + PATCH * PATCH; }

// Reads row r of instance i from a row-major state (s != null) or the world's
// struct-of-arrays state.
__device__ __forceinline__ float srow(const WorldView& v, const float* s, int64_t lds, int i, int r) {
  return s ? s[(int64_t)i * lds + r] : v.a.st[(int64_t)r * v.a.n_inst + i];
}

// Commanded angle of joint j (link j + 1 of the morphology at lk_off) at frame
// n, clamped to its limits: the step kernel's own phase and sine.
__device__ __forceinline__ float command(const WorldView& v, int i, int lk_off, int j, int64_t n) {
  const float* cp = v.a.ctrl + ((int64_t)i * v.a.j_max + j) * 3;
  const float* lk = v.a.links + (int64_t)(lk_off + j + 1) * LINK_F;
  const double t = (double)n * v.a.dt_d;
  const float sq = npx::sin_turns((double)cp[1] * t + (double)cp[2] * npx::kInvTwoPi);
  return fminf(fmaxf(cp[0] * sq, lk[6]), lk[7]);
}

__device__ __forceinline__ float hf(const WorldView& v, float x, float y) {
  if (v.a.hf_bilinear)
    return npx::hf_bilinear(v.a.hf, v.a.hf_nx, v.a.hf_ny, v.a.hf_x0, v.a.hf_y0, v.a.hf_s, x, y);
  return npx::hf_lookup(v.a.hf, v.a.hf_nx, v.a.hf_ax, v.a.hf_ay, x, y);
}

// ---- heading frame -------------------------------------------------------------
struct Heading {
  float ch, sh;  // cos, sin of the heading
  float hw, hz;  // yaw quaternion of -psi: (hw, 0, 0, hz)
  float sgn;     // +-1: makes the w component of the turned orientation >= 0
};

__device__ __forceinline__ Heading heading_of(float qw, float qx, float qy, float qz) {
  float R[9];
  npx::quat_to_mat(qw, qx, qy, qz, R);
  const float hn = sqrtf(R[0] * R[0] + R[3] * R[3]);
  Heading h;
  h.ch = hn > 1e-6f ? R[0] / hn : 1.f;
  h.sh = hn > 1e-6f ? R[3] / hn : 0.f;
  const float c2 = sqrtf(fmaxf(0.f, 0.5f * (1.f + h.ch)));
  const float s2 = copysignf(sqrtf(fmaxf(0.f, 0.5f * (1.f - h.ch))), h.sh);
  h.hw = c2;
  h.hz = -s2;
  h.sgn = h.hw * qw - h.hz * qz >= 0.f ? 1.f : -1.f;
  return h;
}

// world -> heading frame of a vector's x, y (z is unchanged)
__device__ __forceinline__ void to_heading(const Heading& h, float x, float y, float* ox, float* oy) {
  *ox = h.ch * x + h.sh * y;
  *oy = -h.sh * x + h.ch * y;
}
__device__ __forceinline__ void from_heading(const Heading& h, float x, float y, float* ox, float* oy) {
  *ox = h.ch * x - h.sh * y;
  *oy = h.sh * x + h.ch * y;
}
// sgn * q_z(-psi) (x) b  and its inverse  sgn * q_z(psi) (x) b
__device__ __forceinline__ void quat_to_heading(const Heading& h, const float b[4], float o[4]) {
  o[0] = h.sgn * (h.hw * b[0] - h.hz * b[3]);
  o[1] = h.sgn * (h.hw * b[1] - h.hz * b[2]);
  o[2] = h.sgn * (h.hw * b[2] + h.hz * b[1]);
  o[3] = h.sgn * (h.hw * b[3] + h.hz * b[0]);
}
__device__ __forceinline__ void quat_from_heading(const Heading& h, const float b[4], float o[4]) {
  o[0] = h.sgn * (h.hw * b[0] + h.hz * b[3]);
  o[1] = h.sgn * (h.hw * b[1] + h.hz * b[2]);
  o[2] = h.sgn * (h.hw * b[2] - h.hz * b[1]);
  o[3] = h.sgn * (h.hw * b[3] - h.hz * b[0]);
}

// The 13 body entries of a world-frame vector (a state or a state change)
// expressed in the heading frame h, or back (inverse = true).
template <bool INVERSE>
__device__ __forceinline__ void body_frame(const Heading& h, const float in[13], float out[13]) {
  auto vec = [&](int k) __attribute__((always_inline)) {
    if (INVERSE) from_heading(h, in[k], in[k + 1], &out[k], &out[k + 1]);
    else to_heading(h, in[k], in[k + 1], &out[k], &out[k + 1]);
    out[k + 2] = in[k + 2];
  };
  vec(0);
  if (INVERSE) quat_from_heading(h, in + 3, out + 3);
  else quat_to_heading(h, in + 3, out + 3);
  vec(7);
  vec(10);
}

// ---- state rows --------------------------------------------------------------
__global__ void rows_kernel(WorldView v, float* s, int64_t lds, int width) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int I = v.a.n_inst;
  if (e >= (int64_t)I * width) return;
  const int r = (int)(e / I), i = (int)(e % I);
  s[(int64_t)i * lds + r] = v.a.st[(int64_t)r * I + i];
}

// world state of i = s[i] (the inverse of rows_kernel)
__global__ void set_rows_kernel(WorldView v, const float* s, int64_t lds, int width) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int I = v.a.n_inst;
  if (e >= (int64_t)I * width) return;
  const int r = (int)(e / I), i = (int)(e % I);
  v.a.st[(int64_t)r * I + i] = s[(int64_t)i * lds + r];
}

// y[i] = (world state of i) - s0[i], the body entries in the heading frame of
// s0[i].  One wave per instance, lanes over the columns.
__global__ __launch_bounds__(256) void delta_kernel(WorldView v, const float* s0, int64_t lds,
                                                    float* y, int64_t ldy, int width) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int I = v.a.n_inst;
  if (i >= I) return;
  const float* r0 = s0 + (int64_t)i * lds;
  float d[13], b[13];
  for (int k = 0; k < 13; ++k) d[k] = v.a.st[(int64_t)k * I + i] - r0[k];
  const Heading h = heading_of(r0[3], r0[4], r0[5], r0[6]);
  body_frame<false>(h, d, b);
  for (int c = lane; c < width; c += 64) {
    float val = 0.f;
    if (c < 13) {
#pragma unroll
      for (int k = 0; k < 13; ++k) val = c == k ? b[k] : val;
    } else {
      val = v.a.st[(int64_t)c * I + i] - r0[c];
    }
    y[(int64_t)i * ldy + c] = val;
  }
}

// ---- network inputs: a segment of lanes per instance, lanes over the features
// Values shared by the instance's features (heading, body entries in the
// heading frame, ground height under the CoG) are computed once per wave;
// each lane then writes its columns. STD: write the standardised value
// (x - mean) * inv_std as OUT (the network's own input rows), zero in the
// padding columns [nf, width) and in whole rows of instances past n_inst
// below `rows`; otherwise the raw feature as float.
// 16 lanes per instance (four per wave), for the same reason as the rollout
// update below: the per-instance values are computed once per segment, so
// narrow segments share each wave's instruction stream among more instances.
constexpr int FEAT_G = 16, FEAT_IPB = 256 / FEAT_G;
template <class OUT, bool STD>
__global__ __launch_bounds__(256) void features_kernel(WorldView v, const float* s, int64_t lds,
                                                       int64_t frame, OUT* x, int64_t ldx,
                                                       int width, int rows, const float* mean,
                                                       const float* inv_std) {
  const int lane = threadIdx.x & (FEAT_G - 1);
  const int i = blockIdx.x * FEAT_IPB + threadIdx.x / FEAT_G;
  const int J = v.a.j_max;
  const int nf = feature_width(J);
  if (i >= v.a.n_inst) {
    if (STD && i < rows)
      for (int f = lane; f < width; f += FEAT_G) x[(int64_t)i * ldx + f] = static_cast<OUT>(0.f);
    return;
  }
  const int4 mi = v.a.morph_info[v.a.inst_morph[i]];
  const int Ji = mi.w - 1;
  const int64_t n = frame >= 0 ? frame : (int64_t)v.a.step[i];
  float in[13], body[13];
#pragma unroll
  for (int k = 0; k < 13; ++k) in[k] = srow(v, s, lds, i, k);
  const Heading hd = heading_of(in[3], in[4], in[5], in[6]);
  body_frame<false>(hd, in, body);
  const float cx = in[0], cy = in[1];
  const float h0 = hf(v, cx, cy);
  body[0] = 0.f;
  body[1] = 0.f;
  body[2] = in[2] - h0;
  OUT* xr = x + (int64_t)i * ldx;
  auto put = [&](int f, float val) __attribute__((always_inline)) {
    if (STD) val = f < nf ? (val - mean[f]) * inv_std[f] : 0.f;
    xr[f] = static_cast<OUT>(val);
  };
  // The three kinds of columns go in separate passes so that the lanes of a
  // pass do the same work: body, joint angles and rates; the commanded
  // targets of frames n .. n+9 (joint j of frame n + k at 13 + 2J + kJ + j);
  // the height patch and the padding.
  const int c_cmd = 13 + 2 * J, c_patch = 13 + 12 * J;
  for (int f = lane; f < c_cmd; f += FEAT_G) {
    float val = 0.f;
    if (f < 13) {
#pragma unroll
      for (int k = 0; k < 13; ++k) val = f == k ? body[k] : val;
    } else if (f < 13 + J) {
      const int j = f - 13;
      if (j < Ji) val = srow(v, s, lds, i, 13 + j);
    } else {
      const int j = f - 13 - J;
      if (j < Ji) val = (srow(v, s, lds, i, 13 + j) - srow(v, s, lds, i, 13 + J + j)) * v.a.inv_dt;
    }
    put(f, val);
  }
  {
    // (k, j) of column c_cmd + lane, then stepped by FEAT_G columns per pass
    // without a division in the loop
    int k = lane / J, j = lane - (lane / J) * J;
    const int dk = FEAT_G / J, dj = FEAT_G - (FEAT_G / J) * J;
    for (int f = c_cmd + lane; f < c_patch; f += FEAT_G) {
      put(f, j < Ji ? command(v, i, mi.z, j, n + k) : 0.f);
      k += dk;
      j += dj;
      if (j >= J) {
        j -= J;
        k += 1;
      }
    }
  }
  for (int f = c_patch + lane; f < width; f += FEAT_G) {
    float val = 0.f;
    if (f < nf) {
      const int idx = f - c_patch;
      const int a = idx / PATCH, b = idx % PATCH;
      const float u = ((float)a - 0.5f * (PATCH - 1)) * PATCH_STEP;
      const float w = ((float)b - 0.5f * (PATCH - 1)) * PATCH_STEP;
      const float px = cx + (hd.ch * u - hd.sh * w), py = cy + (hd.sh * u + hd.ch * w);
      val = hf(v, px, py) - h0;
    }
    put(f, val);
  }
}

// ---- rollout update: a segment of lanes per instance, lanes over the columns
// The body rows gain dy turned back from the heading frame of s (Q renormalised);
// q and q_prev become what the step sets after frames n .. n+9 with joints
// re-determined every frame.
// 16 lanes per instance (four per wave): the per-instance body update is the
// same few hundred instructions whatever the segment width, so narrow
// segments share each wave's instruction stream among four instances.
constexpr int ADV_G = 16;
__global__ __launch_bounds__(256) void advance_kernel(WorldView v, float* s, int64_t lds,
                                                      const float* dy, int64_t lddy,
                                                      int64_t frame) {
  const int lane = threadIdx.x & (ADV_G - 1);
  const int i = blockIdx.x * (256 / ADV_G) + threadIdx.x / ADV_G;
  if (i >= v.a.n_inst) return;
  float* r = s + (int64_t)i * lds;
  const float* d = dy + (int64_t)i * lddy;
  float cur[13], dh[13], dw[13];
  for (int k = 0; k < 13; ++k) {
    cur[k] = r[k];
    dh[k] = d[k];
  }
  body_frame<true>(heading_of(cur[3], cur[4], cur[5], cur[6]), dh, dw);
  for (int k = 0; k < 13; ++k) cur[k] += dw[k];
  const float qn = sqrtf(cur[3] * cur[3] + cur[4] * cur[4] + cur[5] * cur[5] + cur[6] * cur[6]);
  if (qn > 0.f)
    for (int k = 3; k < 7; ++k) cur[k] /= qn;
  const int J = v.a.j_max;
  const int4 mi = v.a.morph_info[v.a.inst_morph[i]];
  const int Ji = mi.w - 1;
  for (int c = lane; c < 13 + 2 * J; c += ADV_G) {
    float val = 0.f;
    if (c < 13) {
#pragma unroll
      for (int k = 0; k < 13; ++k) val = c == k ? cur[k] : val;
    } else if (c < 13 + J) {
      const int j = c - 13;
      val = j < Ji ? command(v, i, mi.z, j, frame + HORIZON - 1) : 0.f;
    } else {
      const int j = c - 13 - J;
      val = j < Ji ? command(v, i, mi.z, j, frame + HORIZON - 2) : 0.f;
    }
    r[c] = val;
  }
}

// ---- torque proxy: one wave per instance -------------------------------------
// Sum over a segment of G lanes (32 or 64), the same bits in every lane of
// it: DPP adds with the quad partners, the mirrored half-row and row, then
// the other row and (G = 64) the other half-wave through permlane swaps.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}
template <int G>
__device__ __forceinline__ float seg_sum(float x) {
  static_assert(G == 32 || G == 64, "segment of 32 or 64 lanes");
  x += dpp_f<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp_f<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp_f<0x141>(x);  // row_half_mirror
  x += dpp_f<0x140>(x);  // row_mirror
  auto r16 = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, x),
                                              __builtin_bit_cast(unsigned, x), false, false);
  x = __builtin_bit_cast(float, (unsigned)r16[0]) + __builtin_bit_cast(float, (unsigned)r16[1]);
  if constexpr (G == 64) {
    auto r32 = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, x),
                                                __builtin_bit_cast(unsigned, x), false, false);
    x = __builtin_bit_cast(float, (unsigned)r32[0]) + __builtin_bit_cast(float, (unsigned)r32[1]);
  }
  return x;
}

// Quasi-static joint torque: every point carries its weight m_k g, and the
// points within LOW_BAND of the ground share the robot's weight as an upward
// load; joint j transmits the moment of the loads on all points distal to it
// about its anchor, projected on its axis.  Writes (or adds) the mean of |tau_j|
// over the instance's joints.
//
// The loads are linear, so a link's sums split into its weight (from the link
// mass and CoG: no per-point work) plus f_up times the count and the summed
// arms of its points in the band.  Those per-point sums are 64-bit fixed-point
// integers (2^-30 m) added with LDS atomics, which makes them exact and
// independent of timing.
constexpr double FIX = 1073741824.0;

// One robot per segment of G lanes (32 when every robot has at most 32 links:
// two robots per wave), lane l of the segment owning link l. A segment past
// the last instance takes part in the barriers with no links and no points.
template <int G>
__global__ __launch_bounds__(64) void torque_kernel(WorldView v, const float* s, int64_t lds,
                                                    float* acc, int accumulate) {
  constexpr int IPW = 64 / G;
  __shared__ float Tsh[IPW][G][12];  // link transforms in the construction frame: R, t
  __shared__ float Ssh[IPW][G][6];   // per-link load sums: force, moment about the CoG
  __shared__ int low_nsh[IPW][G];
  __shared__ int nearsh[IPW][G];     // links whose box of points may reach the load band
  __shared__ unsigned long long low_xsh[IPW][G], low_ysh[IPW][G];
  const int seg = threadIdx.x / G;
  const int l = threadIdx.x - seg * G;
  float (*T)[12] = Tsh[seg];
  float (*S)[6] = Ssh[seg];
  int* low_n = low_nsh[seg];
  int* near = nearsh[seg];
  unsigned long long* low_x = low_xsh[seg];
  unsigned long long* low_y = low_ysh[seg];
  const int I = v.a.n_inst;
  const bool live = blockIdx.x * IPW + seg < I;
  const int i = live ? blockIdx.x * IPW + seg : 0;
  const int4 mi = v.a.morph_info[v.a.inst_morph[i]];
  const int N = live ? mi.y : 0, L = live ? mi.w : 0, pt0 = mi.x, lk0 = mi.z;
  const bool own = l < L;
  const float* lk = v.a.links + (int64_t)(lk0 + (own ? l : 0)) * LINK_F;
  low_n[l] = 0;
  low_x[l] = 0ull;
  low_y[l] = 0ull;

  // joint rotation about the hinge: R_j = I + sin q [a]x + (1 - cos q) [a]x^2
  float Rj[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, tj[3] = {0, 0, 0};
  float an[3] = {0, 0, 0};
  if (own && l > 0) {
    const float o[3] = {lk[0], lk[1], lk[2]};
    const float ax = lk[3], ay = lk[4], az = lk[5];
    const float inv = 1.f / sqrtf(ax * ax + ay * ay + az * az);
    an[0] = ax * inv;
    an[1] = ay * inv;
    an[2] = az * inv;
    const float q = s ? s[(int64_t)i * lds + 13 + (l - 1)] : v.a.st[(int64_t)(13 + l - 1) * I + i];
    float sq, cq;
    npx::sin_cos(q, &sq, &cq);
    const float C = 1.f - cq;
    const float x = an[0], y = an[1], z = an[2];
    Rj[0] = cq + C * x * x;     Rj[1] = C * x * y - sq * z; Rj[2] = C * x * z + sq * y;
    Rj[3] = C * x * y + sq * z; Rj[4] = cq + C * y * y;     Rj[5] = C * y * z - sq * x;
    Rj[6] = C * x * z - sq * y; Rj[7] = C * y * z + sq * x; Rj[8] = cq + C * z * z;
    for (int r = 0; r < 3; ++r) tj[r] = o[r] - (Rj[3 * r] * o[0] + Rj[3 * r + 1] * o[1] + Rj[3 * r + 2] * o[2]);
  }
  // Each link's transform: its joint transform left-multiplied by its
  // ancestors' joint transforms, nearest first (the root's is the identity).
  // Only joint transforms are read, so one barrier separates the two phases.
  const int parent = own && l > 0 ? v.a.link_parent[lk0 + l] : 0;
  if (own) {
    for (int k = 0; k < 9; ++k) T[l][k] = Rj[k];
    for (int k = 0; k < 3; ++k) T[l][9 + k] = tj[k];
  }
  __syncthreads();
  float Rc[9], tc[3];
  for (int k = 0; k < 9; ++k) Rc[k] = Rj[k];
  for (int k = 0; k < 3; ++k) tc[k] = tj[k];
  for (int anc = parent, it = 0; anc >= 1 && it < v.a.max_depth;
       anc = v.a.link_parent[lk0 + anc], ++it) {
    float Ra[9], ta[3], Rn[9], tn[3];
    for (int k = 0; k < 9; ++k) Ra[k] = T[anc][k];
    for (int k = 0; k < 3; ++k) ta[k] = T[anc][9 + k];
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c)
        Rn[3 * r + c] = Ra[3 * r] * Rc[c] + Ra[3 * r + 1] * Rc[3 + c] + Ra[3 * r + 2] * Rc[6 + c];
      tn[r] = Ra[3 * r] * tc[0] + Ra[3 * r + 1] * tc[1] + Ra[3 * r + 2] * tc[2] + ta[r];
    }
    for (int k = 0; k < 9; ++k) Rc[k] = Rn[k];
    for (int k = 0; k < 3; ++k) tc[k] = tn[k];
  }
  __syncthreads();
  if (own) {
    for (int k = 0; k < 9; ++k) T[l][k] = Rc[k];
    for (int k = 0; k < 3; ++k) T[l][9 + k] = tc[k];
  }
  __syncthreads();

  // body CoG in the construction frame from the link masses and link CoGs
  const float ml = own ? lk[npx::LK_MASS] : 0.f;
  float yc[3] = {0, 0, 0};  // this link's CoG at the current joint angles
  if (own) {
    const float* cg = lk + npx::LK_COG;
    for (int r = 0; r < 3; ++r)
      yc[r] = T[l][3 * r] * cg[0] + T[l][3 * r + 1] * cg[1] + T[l][3 * r + 2] * cg[2] + T[l][9 + r];
  }
  const float M = v.a.morph_mass[v.a.inst_morph[i]];
  float gb[3];
  for (int r = 0; r < 3; ++r) gb[r] = seg_sum<G>(ml * yc[r]) / M;
  float c[3], R[9];
  for (int r = 0; r < 3; ++r) c[r] = s ? s[(int64_t)i * lds + r] : v.a.st[(int64_t)r * I + i];
  {
    float q4[4];
    for (int r = 0; r < 4; ++r) q4[r] = s ? s[(int64_t)i * lds + 3 + r] : v.a.st[(int64_t)(3 + r) * I + i];
    npx::quat_to_mat(q4[0], q4[1], q4[2], q4[3], R);
  }
  // arm about the CoG (world axes) of a construction-frame point p on link k
  auto arm = [&](float px, float py, float pz, int k, float out[3]) __attribute__((always_inline)) {
    float y[3];
    for (int r = 0; r < 3; ++r)
      y[r] = T[k][3 * r] * px + T[k][3 * r + 1] * py + T[k][3 * r + 2] * pz + T[k][9 + r] - gb[r];
    for (int r = 0; r < 3; ++r) out[r] = R[3 * r] * y[0] + R[3 * r + 1] * y[1] + R[3 * r + 2] * y[2];
  };

  // A link whose box of points lies wholly above the highest entry of the
  // height map plus the band has no point in it; its points are not tested
  // (the box's lowest world height: its centre's minus sum_j |w_j| e_j, w = the
  // world z row of the link's axes). The tables list the leaf links' points
  // first, so whole passes of the loop below are skipped.
  if (own) {
    const float* bx = lk + npx::LK_BOX;
    float yb[3];
    arm(bx[0], bx[1], bx[2], l, yb);
    float ez = 0.f;
    for (int j = 0; j < 3; ++j) {
      const float wz = R[6] * T[l][j] + R[7] * T[l][3 + j] + R[8] * T[l][6 + j];
      ez += fabsf(wz) * bx[3 + j];
    }
    near[l] = c[2] + yb[2] - ez <= v.a.hf_max + LOW_BAND + 1e-3f ? 1 : 0;
  }
  __syncthreads();

  // points in the load band: count and summed horizontal arms per link
#pragma unroll 2
  for (int k = l; k < N; k += G) {
    const int kl = v.a.pt_link[pt0 + k];  // link index local to the morphology
    if (!near[kl]) continue;
    const float4 p = v.a.pts[pt0 + k];
    float a[3];
    arm(p.x, p.y, p.z, kl, a);
    if (c[2] + a[2] - hf(v, c[0] + a[0], c[1] + a[1]) < LOW_BAND) {
      atomicAdd(&low_n[kl], 1);
      atomicAdd(&low_x[kl], (unsigned long long)__double2ll_rn((double)a[0] * FIX));
      atomicAdd(&low_y[kl], (unsigned long long)__double2ll_rn((double)a[1] * FIX));
    }
  }
  __syncthreads();
  const float nlow = seg_sum<G>(own ? (float)low_n[l] : 0.f);
  const float f_up = nlow > 0.f ? -M * v.a.gz / nlow : 0.f;

  // this link's load sums: weight m_l g at its CoG, plus f_up on each band point
  if (own) {
    const float y[3] = {yc[0] - gb[0], yc[1] - gb[1], yc[2] - gb[2]};
    float ac[3], F[3], Mo[3];
    for (int r = 0; r < 3; ++r) ac[r] = R[3 * r] * y[0] + R[3 * r + 1] * y[1] + R[3 * r + 2] * y[2];
    F[0] = ml * v.a.gx;
    F[1] = ml * v.a.gy;
    F[2] = ml * v.a.gz;
    Mo[0] = ac[1] * F[2] - ac[2] * F[1];
    Mo[1] = ac[2] * F[0] - ac[0] * F[2];
    Mo[2] = ac[0] * F[1] - ac[1] * F[0];
    // f_up z at arms a: force f_up n, moment f_up (sum a_y, -sum a_x, 0)
    const float sx = (float)((double)(long long)low_x[l] / FIX);
    const float sy = (float)((double)(long long)low_y[l] / FIX);
    F[2] += f_up * (float)low_n[l];
    Mo[0] += f_up * sy;
    Mo[1] -= f_up * sx;
    for (int r = 0; r < 3; ++r) {
      S[l][r] = F[r];
      S[l][3 + r] = Mo[r];
    }
  }
  __syncthreads();
  float tau = 0.f;
  if (own && l > 0) {
    // sums over the subtree, in link order
    const unsigned long long sub = v.sub_mask[lk0 + l];
    float St[6] = {0, 0, 0, 0, 0, 0};
    for (unsigned long long m = sub; m != 0ull; m &= m - 1ull) {
      const int k = __builtin_ctzll(m);
      for (int r = 0; r < 6; ++r) St[r] += S[k][r];
    }
    // the hinge anchor moves with the link (the joint rotation fixes it)
    float ao[3], ab[3], aw[3];
    arm(lk[0], lk[1], lk[2], l, ao);
    for (int r = 0; r < 3; ++r) ab[r] = T[l][3 * r] * an[0] + T[l][3 * r + 1] * an[1] + T[l][3 * r + 2] * an[2];
    for (int r = 0; r < 3; ++r) aw[r] = R[3 * r] * ab[0] + R[3 * r + 1] * ab[1] + R[3 * r + 2] * ab[2];
    const float m0 = St[3] - (ao[1] * St[2] - ao[2] * St[1]);
    const float m1 = St[4] - (ao[2] * St[0] - ao[0] * St[2]);
    const float m2 = St[5] - (ao[0] * St[1] - ao[1] * St[0]);
    tau = fabsf(aw[0] * m0 + aw[1] * m1 + aw[2] * m2);
  }
  tau = seg_sum<G>(tau);
  if (l == 0 && live) {
    const float mean = L > 1 ? tau / (float)(L - 1) : 0.f;
    acc[i] = accumulate ? acc[i] + mean : mean;
  }
}

npx_status check_world(const npx_world* w) {
  if (!w) return fail(NPX_EINVAL, "null world");
  return NPX_OK;
}

}  // namespace

extern "C" {

npx_status npx_sur_widths(const npx_world* w, int32_t* state_w, int32_t* feature_w) {
  npx_status r = check_world(w);
  if (r != NPX_OK) return r;
  const WorldView v = npx::world_view(w);
  if (state_w) *state_w = state_width(v.a.j_max);
  if (feature_w) *feature_w = feature_width(v.a.j_max);
  return NPX_OK;
}

npx_status npx_world_rows(npx_world* w, float* s, int64_t lds, void* stream) {
  npx_status r = check_world(w);
  if (r != NPX_OK) return r;
  const WorldView v = npx::world_view(w);
  const int width = state_width(v.a.j_max);
  if (!s || lds < width) return fail(NPX_EINVAL, "bad state buffer or stride");
  const int64_t n = (int64_t)v.a.n_inst * width;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(rows_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, v, s, lds,
                     width);
  HIP_TRY(hipGetLastError());
  npx::note_stream(w, st);
  return NPX_OK;
}

npx_status npx_world_set_rows(npx_world* w, const float* s, int64_t lds, void* stream) {
  npx_status r = check_world(w);
  if (r != NPX_OK) return r;
  const WorldView v = npx::world_view(w);
  const int width = state_width(v.a.j_max);
  if (!s || lds < width) return fail(NPX_EINVAL, "bad state buffer or stride");
  const int64_t n = (int64_t)v.a.n_inst * width;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(set_rows_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, v, s,
                     lds, width);
  HIP_TRY(hipGetLastError());
  npx::note_stream(w, st);
  return NPX_OK;
}

npx_status npx_sur_features(npx_world* w, const float* s, int64_t lds, int64_t frame, float* x,
                            int64_t ldx, void* stream) {
  npx_status r = check_world(w);
  if (r != NPX_OK) return r;
  const WorldView v = npx::world_view(w);
  if (!x || ldx < feature_width(v.a.j_max)) return fail(NPX_EINVAL, "bad input buffer or stride");
  if (s && lds < state_width(v.a.j_max)) return fail(NPX_EINVAL, "state stride too small");
  if (s && frame < 0) return fail(NPX_EINVAL, "state rows need a frame >= 0");
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL((features_kernel<float, false>),
                     dim3((unsigned)((v.a.n_inst + FEAT_IPB - 1) / FEAT_IPB)),
                     dim3(256), 0, st, v, s, lds, s ? frame : (int64_t)-1, x, ldx,
                     feature_width(v.a.j_max), 0, nullptr, nullptr);
  HIP_TRY(hipGetLastError());
  npx::note_stream(w, st);
  return NPX_OK;
}

npx_status npx_sur_delta(npx_world* w, const float* s0, int64_t lds, float* y, int64_t ldy,
                         void* stream) {
  npx_status r = check_world(w);
  if (r != NPX_OK) return r;
  const WorldView v = npx::world_view(w);
  const int width = state_width(v.a.j_max);
  if (!s0 || !y || lds < width || ldy < width) return fail(NPX_EINVAL, "bad buffers or strides");
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(delta_kernel, dim3((unsigned)((v.a.n_inst + 3) / 4)), dim3(256), 0, st, v, s0,
                     lds, y, ldy, width);
  HIP_TRY(hipGetLastError());
  npx::note_stream(w, st);
  return NPX_OK;
}

npx_status npx_sur_advance(npx_world* w, float* s, int64_t lds, const float* dy, int64_t lddy,
                           int64_t frame, void* stream) {
  npx_status r = check_world(w);
  if (r != NPX_OK) return r;
  const WorldView v = npx::world_view(w);
  const int width = state_width(v.a.j_max);
  if (!s || !dy || lds < width || lddy < width || frame < 0)
    return fail(NPX_EINVAL, "bad buffers, strides or frame");
  if (v.a.K != 1) return fail(NPX_EUNSUPPORTED, "the rollout update assumes joints set every frame");
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(advance_kernel, dim3((unsigned)((v.a.n_inst + 256 / ADV_G - 1) / (256 / ADV_G))),
                     dim3(256), 0, st, v, s, lds, dy, lddy, frame);
  HIP_TRY(hipGetLastError());
  npx::note_stream(w, st);
  return NPX_OK;
}

npx_status npx_sur_torque(npx_world* w, const float* s, int64_t lds, float* acc, int accumulate,
                          void* stream) {
  npx_status r = check_world(w);
  if (r != NPX_OK) return r;
  const WorldView v = npx::world_view(w);
  if (!acc) return fail(NPX_EINVAL, "null output");
  if (s && lds < state_width(v.a.j_max)) return fail(NPX_EINVAL, "state stride too small");
  if (v.l_max > 64) return fail(NPX_EUNSUPPORTED, "more than 64 links");
  hipStream_t st = (hipStream_t)stream;
  if (v.l_max <= 32)
    hipLaunchKernelGGL(torque_kernel<32>, dim3((unsigned)((v.a.n_inst + 1) / 2)), dim3(64), 0, st,
                       v, s, lds, acc, accumulate);
  else
    hipLaunchKernelGGL(torque_kernel<64>, dim3((unsigned)v.a.n_inst), dim3(64), 0, st, v, s, lds,
                       acc, accumulate);
  HIP_TRY(hipGetLastError());
  npx::note_stream(w, st);
  return NPX_OK;
}

npx_status npx_sur_rollout(npx_sur* net, npx_world* w, float* s, int64_t lds, int64_t frame0,
                           int32_t n_calls, float* x_work, int64_t ldx, float* y_work,
                           int64_t ldy, float* tau_acc, void* stream) {
  npx_status r = check_world(w);
  if (r != NPX_OK) return r;
  if (!net) return fail(NPX_EINVAL, "null surrogate");
  const WorldView v = npx::world_view(w);
  int n_in = 0, n_out = 0, max_batch = 0;
  npx::sur_dims(net, &n_in, &n_out, &max_batch);
  if (n_in != feature_width(v.a.j_max) || n_out != state_width(v.a.j_max))
    return fail(NPX_EINVAL, "network shape %d -> %d does not fit this world (%d -> %d)", n_in,
                n_out, feature_width(v.a.j_max), state_width(v.a.j_max));
  if (max_batch < v.a.n_inst)
    return fail(NPX_EINVAL, "network batch limit %d < %d instances", max_batch, v.a.n_inst);
  if (n_calls < 0 || frame0 < 0) return fail(NPX_EINVAL, "negative call count or frame");
  if (!y_work || ldy < n_out) return fail(NPX_EINVAL, "bad output workspace");
  if (!s || lds < n_out) return fail(NPX_EINVAL, "bad state buffer or stride");
  if (!x_work || ldx < n_in) return fail(NPX_EINVAL, "bad feature workspace");
  // The features go straight into the network's own standardised input rows
  // (what npx_sur_forward would make of x_work), so x_work is left unused.
  if (n_calls == 0 || v.a.n_inst == 0) return NPX_OK;
  npx::SurInput in{};
  if ((r = npx::sur_input(net, v.a.n_inst, &in)) != NPX_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  const unsigned blocks = (unsigned)((in.rows + FEAT_IPB - 1) / FEAT_IPB);
  for (int c = 0; c < n_calls; ++c) {
    const int64_t frame = frame0 + (int64_t)c * HORIZON;
    if (in.bf16)
      hipLaunchKernelGGL((features_kernel<__bf16, true>), dim3(blocks), dim3(256), 0, st, v, s,
                         lds, frame, static_cast<__bf16*>(in.x), in.ld, in.width, in.rows,
                         in.mean, in.inv_std);
    else
      hipLaunchKernelGGL((features_kernel<float, true>), dim3(blocks), dim3(256), 0, st, v, s,
                         lds, frame, static_cast<float*>(in.x), in.ld, in.width, in.rows,
                         in.mean, in.inv_std);
    HIP_TRY(hipGetLastError());
    if ((r = npx::sur_forward_input(net, v.a.n_inst, y_work, ldy, st)) != NPX_OK) return r;
    if ((r = npx_sur_advance(w, s, lds, y_work, ldy, frame, stream)) != NPX_OK) return r;
    if (tau_acc && (r = npx_sur_torque(w, s, lds, tau_acc, 1, stream)) != NPX_OK) return r;
  }
  return NPX_OK;
}

}  // extern "C"
