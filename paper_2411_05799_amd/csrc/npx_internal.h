// Internal interface between the host runtime and the step kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "npx.h"
#include "npx_device.h"

namespace npx {

// Records the message returned by npx_last_error and returns s.
npx_status fail(npx_status s, const char* fmt, ...);

// Link table row (LINK_F floats): hinge anchor [0..2], axis [3..5], lower and
// upper limit [6..7], link mass [8], link CoG in the construction frame
// [9..11], inertia about the link CoG in construction axes [12..17]
// (xx yy zz xy xz yz), the box holding all the link's points in the
// construction frame [18..23] (centre, half extents along x y z).
constexpr int LINK_F = 24;
constexpr int LK_MASS = 8, LK_COG = 9, LK_INERTIA = 12, LK_BOX = 18;
constexpr int TELE_N = 4;
constexpr int BODY_ROWS = 13;  // c(3) Q(4) v(3) w(3)

inline int state_rows(int j_max) { return BODY_ROWS + 2 * j_max; }

struct StepArgs {
  int n_inst;             // instances in the world (SoA stride)
  int n_tasks;            // instances stepped by this launch
  int n_blocks;           // ceil(n_tasks / instances per wave)
  const int4* task_info;  // [n_tasks][2] (instance, morphology, point offset, link offset),
                          //   (points, links, mass bits, 0) of each task, costlier
                          //   robots first
  int j_max;              // joint stride of ctrl and q
  int max_depth;          // deepest link over all morphologies
  const int* inst_morph;  // [n_inst]
  const int4* morph_info; // [n_morphs] point offset, points, link offset, links
  const float* morph_mass;
  const float4* pts;      // [total points] x y z m (construction frame)
  const int* pt_link;     // [total points]
  const int* pt_orig;     // [total points] index in the morphology's own point order
  const float* links;     // [total links][LINK_F]
  const int* link_parent; // [total links]
  const int* fk_task;     // chain-composition passes (row | link << 2 | parent << 9, -1 idle)
  const int2* fk_info;    // [morphs][3] first entry and pass count for G = 16, 32, 64
  const float* ctrl;      // [n_inst][j_max][3] A f phi
  float dt, inv_dt;
  double dt_d;
  int K;
  float rate_step;        // > 0: largest joint change per update (rate K dt)
  float gx, gy, gz;
  float mu;
  int mu_inf;
  float kn, zeta, eps;
  int fric_w;             // friction fit weighted by each point's normal force
  int fric6;              // six-degree friction fit (rotation in 3-D, vertical displacement)
  const float* hf;
  int hf_nx, hf_ny;
  float hf_s, hf_x0, hf_y0;
  HfAxis hf_ax, hf_ay;    // cell index along x and y (see hf_index)
  float hf_max;           // highest entry of the height map
  int hf_bilinear;        // 1: read the table bilinearly between cell centres
  float* st;              // [state_rows(j_max)][n_inst]
  int* step;              // [n_inst]
  int* flags;             // [n_inst]
  double* tele;           // [TELE_N][n_inst]
  int n_steps;            // frames advanced by this launch
  int* queue;             // persistent mode: task-block counter (zeroed before launch)
  float* points_out;      // with n_steps == 0: [n_inst][n_max][3] world points
  int n_max;
  int place;              // with n_steps == 0: set q = q_cmd(t_n) and turn the
                          // torso-origin position held in the CoG rows into the CoG
};

// Kernel shape: lanes per instance G, points per lane PPL, links per lane LPL.
struct Shape {
  int G, PPL, LPL;
};

// Smallest built shape for a given G that holds n_max points and l_max links;
// returns false when none does.
bool pick_shape(int G, int n_max, int l_max, Shape* out);
hipError_t launch_step(const StepArgs& a, const Shape& s, int grid, hipStream_t stream);
hipError_t launch_zero(int* p, hipStream_t stream);
// Clears n ints on the stream with a fill kernel (graph-capturable).
hipError_t launch_zero_n(int* p, int n, hipStream_t stream);
// Max resident blocks of one wave per CU for a shape (occupancy query).
int resident_blocks_per_cu(const Shape& s);

// What the surrogate's kernels read of a world: the step arguments (tables,
// state, height map, controller) and the points of each link grouped together.
struct WorldView {
  StepArgs a;
  const int* lp_off;  // [total links + 1]
  const int* lp_idx;  // [total points]
  const unsigned long long* sub_mask;  // [total links] bit k: link k is in the subtree
  int n_max, l_max;
};
WorldView world_view(const npx_world* w);
// Records the stream of work that touched the world's state (read_state waits on it).
void note_stream(npx_world* w, hipStream_t s);

// Shape of a surrogate network (defined with the network).
void sur_dims(const npx_sur* s, int* n_in, int* n_out, int* max_batch);

}  // namespace npx
