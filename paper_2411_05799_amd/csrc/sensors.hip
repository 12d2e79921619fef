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

// The robot's frame at the current state, computed by the block's 64 lanes
// together (every lane must call it): T[l] = link l's transform in the
// construction frame (its hinge's, left-multiplied by its ancestors' hinges;
// lane l owns link l), g_b = the body CoG in that frame, c and R = the world
// CoG and the torso rotation. An end or point p of link l is then at
// c + R (T[l] p - g_b), the mass points' transform.
__device__ void robot_frame(const WorldView& v, int i, int mo, float (*T)[12], float gb[3],
                            float c[3], float R[9]) {
  const int l = threadIdx.x;
  const int I = v.a.n_inst;
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
  for (int rr = 0; rr < 3; ++rr) gb[rr] = wave_sum(mc[rr]) / M;
  for (int rr = 0; rr < 3; ++rr) c[rr] = v.a.st[(int64_t)rr * I + i];
  quat_to_mat(v.a.st[(int64_t)3 * I + i], v.a.st[(int64_t)4 * I + i], v.a.st[(int64_t)5 * I + i],
              v.a.st[(int64_t)6 * I + i], R);
}

__device__ __forceinline__ void to_world(const float (*T)[12], int k, const float p[3],
                                         const float gb[3], const float c[3], const float R[9],
                                         float P[3]) {
  float y[3];
  for (int rr = 0; rr < 3; ++rr)
    y[rr] = T[k][3 * rr] * p[0] + T[k][3 * rr + 1] * p[1] + T[k][3 * rr + 2] * p[2] + T[k][9 + rr] -
            gb[rr];
  for (int rr = 0; rr < 3; ++rr)
    P[rr] = c[rr] + (R[3 * rr] * y[0] + R[3 * rr + 1] * y[1] + R[3 * rr + 2] * y[2]);
}

// One robot per block of one wave: the robot's frame, then lanes 0..n-1 take
// rays l, l + 64, ... for the march.
__global__ __launch_bounds__(64) void ray_kernel(WorldView v, RayTables r, float* dst,
                                                 int64_t ld) {
  __shared__ float T[64][12];
  const int i = blockIdx.x, l = threadIdx.x;
  const int mo = v.a.inst_morph[i];
  const int2 ri = r.ray_info[mo];
  if (ri.y == 0) return;  // the whole block leaves together
  float gb[3], c[3], R[9];
  robot_frame(v, i, mo, T, gb, c, R);
  for (int k = l; k < ri.y; k += 64) {
    const float* ry = r.rays + (int64_t)(ri.x + k) * 6;
    const int kl = r.ray_link[ri.x + k];
    float P[2][3];
    to_world(T, kl, ry, gb, c, R, P[0]);
    to_world(T, kl, ry + 3, gb, c, R, P[1]);
    dst[(int64_t)i * ld + k] = ray_range(v.a, P[0], P[1]);
  }
}

// The machine-code controller of one robot per block (one wave): foot sensors
// from the current state, then the program's next instructions on one lane
// (the interpreter is serial), then the targets as the step's commands.
__global__ __launch_bounds__(64) void gp_kernel(WorldView v, GpArgs g) {
  __shared__ float T[64][12];
  __shared__ float tgt[64], lo[64], hi[64];
  const int i = blockIdx.x, l = threadIdx.x;
  const int mo = v.a.inst_morph[i];
  const int4 mi = v.a.morph_info[mo];
  const int L = mi.w, lk0 = mi.z, J = L - 1;
  float gb[3], c[3], R[9];
  robot_frame(v, i, mo, T, gb, c, R);

  // sensor s: any point of its foot link strictly below its cell. The lanes
  // take the morphology's (sensor, point) pairs, 64 at a time, and OR their
  // sensors' bits together.
  const int4 fi = g.foot_info[mo];
  unsigned bits = 0u;
  for (int q = l; q < fi.y; q += 64) {
    const int4 pr = g.foot_pairs[fi.x + q];
    const float4 rho = v.a.pts[pr.y];
    const float pp[3] = {rho.x, rho.y, rho.z};
    float P[3];
    to_world(T, pr.z, pp, gb, c, R, P);
    const float h = v.a.hf_bilinear
                        ? hf_bilinear(v.a.hf, v.a.hf_nx, v.a.hf_ny, v.a.hf_x0, v.a.hf_y0, v.a.hf_s,
                                      P[0], P[1])
                        : hf_lookup(v.a.hf, v.a.hf_nx, v.a.hf_ax, v.a.hf_ay, P[0], P[1]);
    if (h - P[2] > 0.f) bits |= 1u << pr.x;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) bits |= (unsigned)__shfl_xor((int)bits, o);
  const unsigned long long sense = bits;

  // the program, targets and limits staged in LDS: the serial interpreter
  // below then waits on no global load
  __shared__ unsigned char prog[GP_BYTES];
  if (l < GP_BYTES) prog[l] = g.prog[(int64_t)i * GP_BYTES + l];
  if (l < J) {
    tgt[l] = g.targets[(int64_t)i * g.ld_targets + l];
    const float* lk = v.a.links + (int64_t)(lk0 + l + 1) * LINK_F;
    lo[l] = lk[6];
    hi[l] = lk[7];
  }
  __syncthreads();
  if (l == 0) {
    int pc = g.vm[2 * (int64_t)i] & (GP_BYTES - 1);
    unsigned acc = (unsigned)g.vm[2 * (int64_t)i + 1] & 0xFFu;
    for (int e = 0; e < g.n_instr; ++e) {
      const unsigned b = prog[pc];
      const unsigned op = b >> 5, arg = b & 31u;
      int nxt = (pc + 1) & (GP_BYTES - 1);
      switch (op) {
        case 0:  // move motor left
        case 1:  // move motor right
          if ((int)arg < J) {
            const float t = op == 0 ? tgt[arg] - g.step : tgt[arg] + g.step;
            tgt[arg] = fminf(fmaxf(t, lo[arg]), hi[arg]);
          }
          break;
        case 2:  // read sensor
          acc = (int)arg < fi.z ? (unsigned)((sense >> arg) & 1ull) : 0u;
          break;
        case 3:  // load
          acc = arg;
          break;
        case 4:  // jump if true
          if (acc != 0u) nxt = (int)arg;
          break;
        case 5:  // not
          acc = ~acc & 0xFFu;
          break;
        case 6:  // inc
          acc = (acc + 1u) & 0xFFu;
          break;
        default:  // dec
          acc = (acc - 1u) & 0xFFu;
          break;
      }
      pc = nxt;
    }
    g.vm[2 * (int64_t)i] = pc;
    g.vm[2 * (int64_t)i + 1] = (int)acc;
  }
  __syncthreads();
  if (l < J) {
    g.targets[(int64_t)i * g.ld_targets + l] = tgt[l];
    float* cr = g.ctrl + ((int64_t)i * v.a.j_max + l) * 3;
    cr[0] = tgt[l];
    cr[1] = 0.f;
    cr[2] = HALF_PI_F;  // a constant command A sin(pi/2) = A
  }
}

__global__ void targets_kernel(const float* t, float* ctrl, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  ctrl[3 * k] = t[k];
  ctrl[3 * k + 1] = 0.f;
  ctrl[3 * k + 2] = HALF_PI_F;
}

}  // namespace

hipError_t launch_targets(const float* targets, float* ctrl, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(targets_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                     targets, ctrl, n);
  return hipGetLastError();
}

hipError_t launch_ray_ranges(const WorldView& v, const RayTables& r, float* dst, int64_t ld,
                             hipStream_t stream) {
  if (v.a.n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(ray_kernel, dim3((unsigned)v.a.n_inst), dim3(64), 0, stream, v, r, dst, ld);
  return hipGetLastError();
}

hipError_t launch_gp(const WorldView& v, const GpArgs& g, hipStream_t stream) {
  if (v.a.n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(gp_kernel, dim3((unsigned)v.a.n_inst), dim3(64), 0, stream, v, g);
  return hipGetLastError();
}

}  // namespace npx
