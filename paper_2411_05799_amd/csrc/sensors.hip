// Range sensors: the rays of the construction API (Sec. IV, createRay) read
// against the height map.
//
// A ray rides on a link like a massless point: its ends p (construction frame)
// are at c + R(Q)(T_link p - g_b) in the world, the transform the step applies
// to the mass points (Sec. III-A, III-B). Its range is the distance from the
// start to the first point of the segment that lies at or below the ground,
// the ground being the step's look-up table (Sec. III-A): the height of the
// cell named by a point's floor indices, clamped to the map. Over one cell the
// ground is flat and the segment's height linear, so the segment is walked
// cell by cell in the order it crosses them (each crossing time computed
// directly from its grid line, no accumulation) and the first cell where it
// is at or below that cell's height gives the hit: at the entry if it enters
// below, else where its height meets the cell's.
#include "npx_device.h"
#include "npx_sensor_internal.h"

namespace npx {
namespace {

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

__device__ float ray_range(const StepArgs& a, const float A[3], const float B[3]) {
  const float dx = B[0] - A[0], dy = B[1] - A[1], dz = B[2] - A[2];
  if (!(isfinite(A[0]) && isfinite(A[1]) && isfinite(A[2]) && isfinite(dx) && isfinite(dy) &&
        isfinite(dz)))
    return __builtin_nanf("");
  const float len = sqrtf(dx * dx + dy * dy + dz * dz);
  // grid coordinates: cell (ix, iy) covers [ix, ix + 1) x [iy, iy + 1)
  const float u = fminf(fmaxf(a.hf_s * (A[0] - a.hf_x0), -1e9f), 1e9f);
  const float w = fminf(fmaxf(a.hf_s * (A[1] - a.hf_y0), -1e9f), 1e9f);
  const float du = a.hf_s * dx, dw = a.hf_s * dy;
  int ix = (int)floorf(u), iy = (int)floorf(w);
  const int sx = du > 0.f ? 1 : -1, sy = dw > 0.f ? 1 : -1;
  const float inf = __builtin_inff();
  const float inv_du = du != 0.f ? 1.f / du : 0.f, inv_dw = dw != 0.f ? 1.f / dw : 0.f;
  int nbx = du > 0.f ? ix + 1 : ix, nby = dw > 0.f ? iy + 1 : iy;  // next grid lines
  float tmx = du != 0.f ? ((float)nbx - u) * inv_du : inf;
  float tmy = dw != 0.f ? ((float)nby - w) * inv_dw : inf;
  const int n_cells = min(RAY_MAX_CELLS, (int)(fabsf(du) + fabsf(dw)) + 3);
  float t = 0.f;
  for (int c = 0; c < n_cells; ++c) {
    const int cx = min(max(ix, 0), a.hf_nx - 1), cy = min(max(iy, 0), a.hf_ny - 1);
    const float h = a.hf[(int64_t)cy * a.hf_nx + cx];
    const float te = fminf(fminf(tmx, tmy), 1.f);
    if (A[2] + t * dz <= h) return t * len;
    if (A[2] + te * dz <= h) {  // enters above, leaves at or below: dz < 0
      const float th = fminf(fmaxf((h - A[2]) / dz, t), te);
      return th * len;
    }
    if (te >= 1.f) break;
    const float tx = tmx, ty = tmy;
    if (tx <= ty) {
      ix += sx;
      nbx += sx;
      tmx = ((float)nbx - u) * inv_du;
    }
    if (ty <= tx) {
      iy += sy;
      nby += sy;
      tmy = ((float)nby - w) * inv_dw;
    }
    t = te;
  }
  return len;
}

// One robot per block of one wave: lane l owns link l for the transforms and
// rays l, l + 64, ... for the march.
__global__ __launch_bounds__(64) void ray_kernel(WorldView v, RayTables r, float* dst,
                                                 int64_t ld) {
  __shared__ float T[64][12];  // link transforms in the construction frame: R, t
  const int i = blockIdx.x, l = threadIdx.x;
  const int I = v.a.n_inst;
  const int mo = v.a.inst_morph[i];
  const int2 ri = r.ray_info[mo];
  if (ri.y == 0) return;  // the whole block leaves together
  const int4 mi = v.a.morph_info[mo];
  const int L = mi.w, lk0 = mi.z;
  const bool own = l < L;
  const float* lk = v.a.links + (int64_t)(lk0 + (own ? l : 0)) * LINK_F;

  // hinge rotation R_j = I + sin q [a]x + (1 - cos q) [a]x^2 about the anchor o
  float Rj[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, tj[3] = {0, 0, 0};
  if (own && l > 0) {
    const float o[3] = {lk[0], lk[1], lk[2]};
    const float inv = 1.f / sqrtf(lk[3] * lk[3] + lk[4] * lk[4] + lk[5] * lk[5]);
    const float x = lk[3] * inv, y = lk[4] * inv, z = lk[5] * inv;
    const float q = v.a.st[(int64_t)(BODY_ROWS + l - 1) * I + i];
    float sq, cq;
    sin_cos(q, &sq, &cq);
    const float C = 1.f - cq;
    Rj[0] = cq + C * x * x;     Rj[1] = C * x * y - sq * z; Rj[2] = C * x * z + sq * y;
    Rj[3] = C * x * y + sq * z; Rj[4] = cq + C * y * y;     Rj[5] = C * y * z - sq * x;
    Rj[6] = C * x * z - sq * y; Rj[7] = C * y * z + sq * x; Rj[8] = cq + C * z * z;
    for (int k = 0; k < 3; ++k)
      tj[k] = o[k] - (Rj[3 * k] * o[0] + Rj[3 * k + 1] * o[1] + Rj[3 * k + 2] * o[2]);
  }
  if (own) {
    for (int k = 0; k < 9; ++k) T[l][k] = Rj[k];
    for (int k = 0; k < 3; ++k) T[l][9 + k] = tj[k];
  }
  __syncthreads();
  // a link's transform: its hinge's, left-multiplied by its ancestors' hinges
  float Rc[9], tc[3];
  for (int k = 0; k < 9; ++k) Rc[k] = Rj[k];
  for (int k = 0; k < 3; ++k) tc[k] = tj[k];
  const int parent = own && l > 0 ? v.a.link_parent[lk0 + l] : 0;
  for (int anc = parent, it = 0; anc >= 1 && it < v.a.max_depth;
       anc = v.a.link_parent[lk0 + anc], ++it) {
    float Rn[9], tn[3];
    for (int rr = 0; rr < 3; ++rr) {
      for (int cc = 0; cc < 3; ++cc)
        Rn[3 * rr + cc] = T[anc][3 * rr] * Rc[cc] + T[anc][3 * rr + 1] * Rc[3 + cc] +
                          T[anc][3 * rr + 2] * Rc[6 + cc];
      tn[rr] = T[anc][3 * rr] * tc[0] + T[anc][3 * rr + 1] * tc[1] + T[anc][3 * rr + 2] * tc[2] +
               T[anc][9 + rr];
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

  // body CoG g_b in the construction frame, from the link masses and CoGs
  float mc[3] = {0.f, 0.f, 0.f};
  if (own) {
    const float ml = lk[LK_MASS];
    const float* cg = lk + LK_COG;
    for (int rr = 0; rr < 3; ++rr)
      mc[rr] = ml * (Rc[3 * rr] * cg[0] + Rc[3 * rr + 1] * cg[1] + Rc[3 * rr + 2] * cg[2] + tc[rr]);
  }
  const float M = v.a.morph_mass[mo];
  float gb[3];
  for (int rr = 0; rr < 3; ++rr) gb[rr] = wave_sum(mc[rr]) / M;
  float c[3], R[9];
  for (int rr = 0; rr < 3; ++rr) c[rr] = v.a.st[(int64_t)rr * I + i];
  quat_to_mat(v.a.st[(int64_t)3 * I + i], v.a.st[(int64_t)4 * I + i], v.a.st[(int64_t)5 * I + i],
              v.a.st[(int64_t)6 * I + i], R);

  for (int k = l; k < ri.y; k += 64) {
    const float* ry = r.rays + (int64_t)(ri.x + k) * 6;
    const int kl = r.ray_link[ri.x + k];
    float P[2][3];
    for (int e = 0; e < 2; ++e) {
      const float* p = ry + 3 * e;
      float y[3];
      for (int rr = 0; rr < 3; ++rr)
        y[rr] = T[kl][3 * rr] * p[0] + T[kl][3 * rr + 1] * p[1] + T[kl][3 * rr + 2] * p[2] +
                T[kl][9 + rr] - gb[rr];
      for (int rr = 0; rr < 3; ++rr)
        P[e][rr] = c[rr] + (R[3 * rr] * y[0] + R[3 * rr + 1] * y[1] + R[3 * rr + 2] * y[2]);
    }
    dst[(int64_t)i * ld + k] = ray_range(v.a, P[0], P[1]);
  }
}

}  // namespace

hipError_t launch_ray_ranges(const WorldView& v, const RayTables& r, float* dst, int64_t ld,
                             hipStream_t stream) {
  if (v.a.n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(ray_kernel, dim3((unsigned)v.a.n_inst), dim3(64), 0, stream, v, r, dst, ld);
  return hipGetLastError();
}

}  // namespace npx
