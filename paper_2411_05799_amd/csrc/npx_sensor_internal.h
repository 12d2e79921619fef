// Internal interface of the range sensors (rays riding on links).
#pragma once

#include "npx_internal.h"

namespace npx {

constexpr int RAY_MAX = 64;            // rays per morphology
constexpr int RAY_MAX_CELLS = 65536;   // cells one ray may cross

struct RayTables {
  const float* rays;     // [total rays][6] start, end (construction frame)
  const int* ray_link;   // [total rays] link of each ray within its morphology
  const int2* ray_info;  // [n_morphs] first ray, ray count
};

// dst[i * ld + k] = range of ray k of instance i (see npx_world_ray_ranges).
hipError_t launch_ray_ranges(const WorldView& v, const RayTables& r, float* dst, int64_t ld,
                             hipStream_t stream);

constexpr int GP_BYTES = 32;  // program length (jumps name one of 32 addresses)
constexpr int FOOT_MAX = 32;  // sensors per morphology (5-bit sensor numbers)

struct GpArgs {
  const uint8_t* prog;    // [n_inst][GP_BYTES]
  int* vm;                // [n_inst][2] program counter, accumulator
  float* targets;         // [n_inst][ld_targets] joint targets
  int64_t ld_targets;
  const int4* foot_pairs; // [total pairs] sensor, point (global index), link in its morphology
  const int4* foot_info;  // [n_morphs] first pair, pair count, sensor count
  int n_instr;            // instructions per joint update
  float step;             // motor step, rad
  float* ctrl;            // the world's controller [n_inst][j_max][3]
};

// One joint update of the machine-code controller of every instance.
hipError_t launch_gp(const WorldView& v, const GpArgs& g, hipStream_t stream);

// A joint target as a sinusoid row: A = target, f = 0, phi = pi/2 (the step's
// command A sin(2 pi f t + phi) is then the target itself).
constexpr float HALF_PI_F = 1.57079637f;
// ctrl[3k..3k+2] = (targets[k], 0, pi/2) for k < n.
hipError_t launch_targets(const float* targets, float* ctrl, int64_t n, hipStream_t stream);

}  // namespace npx
