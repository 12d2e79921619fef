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

}  // namespace npx
