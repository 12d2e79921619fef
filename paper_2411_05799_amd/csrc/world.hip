// Host runtime of the C ABI in include/npx.h: world creation (morphology
// tables to device CSR arrays), struct-of-arrays state, chunked launches of
// the step kernel replayed from cached hipGraphs, persistent mode, the launch
// autotuner and state I/O.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "npx.h"
#include "npx_internal.h"
#include "npx_sensor_internal.h"

namespace {
thread_local std::string g_err;
}  // namespace

namespace npx {
npx_status fail(npx_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}
}  // namespace npx

namespace {
using npx::fail;

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(NPX_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));            \
  } while (0)

template <class T>
hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void**)p, count * sizeof(T));
}

}  // namespace

struct npx_world {
  int device = 0;
  int n_inst = 0, j_max = 0, n_max = 0, l_max = 0, n_morphs = 0, max_depth = 0;
  std::vector<int> morph_points, morph_links;  // per morph
  std::vector<int> inst_morph;
  double dt = 0, mu = 0;
  int K = 1;

  // device buffers (st, step, flags, tele may be the caller's: ext_state)
  bool ext_state[4] = {false, false, false, false};
  float* st = nullptr;
  int* step = nullptr;
  int* flags = nullptr;
  double* tele = nullptr;
  int* inst_morph_d = nullptr;
  int4* morph_info = nullptr;
  float* morph_mass = nullptr;
  float4* pts = nullptr;
  int* pt_link = nullptr;
  int* pt_orig = nullptr;  // [total points] index of each point in its morphology's own order
  float* links = nullptr;
  int* link_parent = nullptr;
  int* fk_task = nullptr;   // row-composition schedule of the step kernel (see fk_schedule)
  int2* fk_info = nullptr;  // [morphs][3] (first entry, passes) for segments of 16, 32, 64 lanes
  float* ctrl = nullptr;
  float* hf = nullptr;
  int4* task_info = nullptr;  // [I][2], see StepArgs::task_info
  int* queue = nullptr;
  int* lp_off = nullptr;   // [total links + 1] point range of each link in lp_idx
  int* lp_idx = nullptr;   // [total points] point indices grouped by link
  unsigned long long* sub_mask = nullptr;  // [total links] links of each link's subtree
  // range sensors: per morphology host copies, and their device tables
  std::vector<std::vector<float>> ray_host;
  std::vector<std::vector<int>> ray_link_host;
  float* rays = nullptr;
  int* ray_link = nullptr;
  int2* ray_info = nullptr;
  int ray_max = 0;
  // foot contact sensors of the machine-code controller, per morphology
  std::vector<std::vector<int>> foot_host;
  std::vector<int> lp_off_host, lp_idx_host;  // host copies of lp_off / lp_idx
  int4* foot_pairs = nullptr;  // (sensor, point, link, 0) of every sensed point
  int4* foot_info = nullptr;   // per morphology: first pair, pair count, sensor count


  npx::StepArgs args{};
  npx_launch launch{64, 0, 100, 1, 8};
  npx::Shape shape{64, 2, 1};
  hipStream_t last_stream = nullptr;
  bool has_last_stream = false;
  hipStream_t capture_stream = nullptr;
  std::map<int, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
  // a block of controller updates (controller kernel + K frames, repeated),
  // captured once for one set of controller arguments
  hipGraph_t gp_graph = nullptr;
  hipGraphExec_t gp_exec = nullptr;
  npx::GpArgs gp_key{};
  int cu_count = 256;

  void drop_graphs() {
    for (auto& kv : graphs) {
      (void)hipGraphExecDestroy(kv.second.second);
      (void)hipGraphDestroy(kv.second.first);
    }
    graphs.clear();
    if (gp_exec) (void)hipGraphExecDestroy(gp_exec);
    if (gp_graph) (void)hipGraphDestroy(gp_graph);
    gp_exec = nullptr;
    gp_graph = nullptr;
  }
};

namespace {

// One axis of the height-map cell index (npx::hf_index): the scale, -s x0 in
// double, and a float32 range [lo, hi] half a cell beyond the table's first and
// last cell edges (rounded outwards), so that s (lo - x0) is about -1/2 and
// s (hi - x0) about n - 1/2: every clamped coordinate truncates to the cell
// floor(s (x - x0)) clamped onto [0, n - 1].
npx::HfAxis hf_axis(double x0, double s, int n) {
  npx::HfAxis a;
  a.s = s;
  a.ms0 = -s * x0;
  const double lo = x0 - 0.5 / s, hi = x0 + ((double)n - 0.5) / s;
  a.lo = (float)lo;
  if ((double)a.lo > lo) a.lo = std::nextafter(a.lo, -INFINITY);
  a.hi = (float)hi;
  if ((double)a.hi < hi) a.hi = std::nextafter(a.hi, INFINITY);
  return a;
}

size_t field_bytes(const npx_world* w, int field, size_t* row0, size_t* rows, int* kind) {
  // kind 0 float rows of st, 1 step, 2 flags, 3 tele
  const size_t I = (size_t)w->n_inst;
  *kind = 0;
  switch (field) {
    case NPX_F_COG: *row0 = 0; *rows = 3; break;
    case NPX_F_QUAT: *row0 = 3; *rows = 4; break;
    case NPX_F_VEL: *row0 = 7; *rows = 3; break;
    case NPX_F_OMEGA: *row0 = 10; *rows = 3; break;
    case NPX_F_JOINT: *row0 = npx::BODY_ROWS; *rows = (size_t)w->j_max; break;
    case NPX_F_JOINT_PREV: *row0 = npx::BODY_ROWS + w->j_max; *rows = (size_t)w->j_max; break;
    case NPX_F_BODY: *row0 = 0; *rows = npx::BODY_ROWS; break;
    case NPX_F_STEP: *kind = 1; return I * sizeof(int);
    case NPX_F_FLAGS: *kind = 2; return I * sizeof(int);
    case NPX_F_TELE: *kind = 3; return I * npx::TELE_N * sizeof(double);
    default: return 0;
  }
  return *rows * I * sizeof(float);
}

npx_status sync_last(npx_world* w) {
  if (w->has_last_stream) HIP_TRY(hipStreamSynchronize(w->last_stream));
  return NPX_OK;
}

// Launches `steps` frames (state stays in registers) as one kernel, plus the
// queue reset in persistent mode.
// One launch of `steps` frames. In persistent mode the task-queue counter is
// the world's own, cleared before the launch, or `cleared_queue`, a counter the
// caller has already cleared on the stream.
hipError_t enqueue_chunk(npx_world* w, int steps, hipStream_t s, int* cleared_queue = nullptr) {
  npx::StepArgs a = w->args;
  a.n_steps = steps;
  const int ipw = 64 / w->shape.G;
  a.n_blocks = (a.n_tasks + ipw - 1) / ipw;
  int grid = a.n_blocks;
  if (w->launch.persistent) {
    int per_cu = std::max(1, std::min(w->launch.waves_per_cu, npx::resident_blocks_per_cu(w->shape)));
    grid = std::min(a.n_blocks, per_cu * w->cu_count);
    if (cleared_queue) {
      a.queue = cleared_queue;
    } else {
      a.queue = w->queue;
      hipError_t e = npx::launch_zero(w->queue, s);
      if (e != hipSuccess) return e;
    }
  } else {
    a.queue = nullptr;
  }
  if (grid <= 0) return hipSuccess;
  return npx::launch_step(a, w->shape, grid, s);
}

npx_status run_steps(npx_world* w, int64_t n, hipStream_t s) {
  const int chunk = std::max(1, w->launch.chunk_steps);
  int64_t left = n;
  while (left > 0) {
    const int c = (int)std::min<int64_t>(left, chunk);
    // A persistent chunk is two launches (queue reset, step) and is replayed
    // from a cached graph; a chunk of one kernel is launched directly: as a
    // one-node graph it took about 10 us more per launch.
    if (w->launch.use_graph && w->launch.persistent) {
      auto it = w->graphs.find(c);
      if (it == w->graphs.end()) {
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        HIP_TRY(hipStreamBeginCapture(w->capture_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue_chunk(w, c, w->capture_stream);
        hipError_t e2 = hipStreamEndCapture(w->capture_stream, &g);
        if (e != hipSuccess) return fail(NPX_EHIP, "capture of step chunk: %s", hipGetErrorString(e));
        if (e2 != hipSuccess) return fail(NPX_EHIP, "end capture: %s", hipGetErrorString(e2));
        HIP_TRY(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        it = w->graphs.emplace(c, std::make_pair(g, ge)).first;
      }
      HIP_TRY(hipGraphLaunch(it->second.second, s));
    } else {
      hipError_t e = enqueue_chunk(w, c, s);
      if (e != hipSuccess) return fail(NPX_EHIP, "step launch: %s", hipGetErrorString(e));
    }
    left -= c;
  }
  w->last_stream = s;
  w->has_last_stream = true;
  return NPX_OK;
}

bool shape_for(const npx_world* w, int G, npx::Shape* s) {
  return npx::pick_shape(G, w->n_max, w->l_max, s);
}

// Task order: costlier robots first (longest-processing-time order), so the
// tail of an uneven batch is made of the cheap ones.
std::vector<int> task_order(const npx_world* w) {
  std::vector<int> ord(w->n_inst);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    int ma = w->inst_morph[a], mb = w->inst_morph[b];
    long ca = (long)w->morph_points[ma] * 4 + w->morph_links[ma] * 16;
    long cb = (long)w->morph_points[mb] * 4 + w->morph_links[mb] * 16;
    return ca > cb;
  });
  return ord;
}

// Schedule of the step kernel's chain composition for one morphology: links
// of depth >= 2 take their final transform as parent's final transform times
// their own joint transform, one matrix row per lane, level by level (a level
// needs its parents' level done). For each segment width G in {16, 32, 64}
// a level's links fill passes of G lanes, at most G / 3 links (three rows
// each) per pass: the rows of one link share a pass, since each row's lane
// reads the whole joint transform that the link's lanes then overwrite. An
// entry is row | link << 2 | parent << 9, or -1 for an idle lane. fki gets
// (first entry, pass count) per width.
void fk_schedule(const npx_morph_tables& m, const std::vector<int>& depth, std::vector<int>& fkt,
                 std::vector<int2>& fki) {
  int dmax = 0;
  for (int l = 0; l < m.n_links; ++l) dmax = std::max(dmax, depth[l]);
  for (int G : {16, 32, 64}) {
    const int first = (int)fkt.size();
    int passes = 0;
    for (int d = 2; d <= dmax; ++d) {
      std::vector<int> lv;
      for (int l = 1; l < m.n_links; ++l)
        if (depth[l] == d) lv.push_back(l);
      const size_t per = G / 3;
      for (size_t l0 = 0; l0 < lv.size(); l0 += per, ++passes)
        for (int k = 0; k < G; ++k) {
          const size_t t = l0 + k / 3;
          fkt.push_back(k / 3 < (int)per && t < lv.size()
                            ? (k % 3) | (lv[t] << 2) | (m.parent[lv[t]] << 9)
                            : -1);
        }
    }
    fki.push_back(make_int2(first, passes));
  }
}

npx_status check_tables(const npx_morph_tables& m, int idx) {
  if (m.n_points <= 0 || m.n_points > NPX_MAX_POINTS)
    return fail(NPX_EINVAL, "morph %d: n_points %d out of [1, %d]", idx, m.n_points, NPX_MAX_POINTS);
  if (m.n_links <= 0 || m.n_links > NPX_MAX_JOINTS + 1)
    return fail(NPX_EINVAL, "morph %d: n_links %d out of [1, %d]", idx, m.n_links, NPX_MAX_JOINTS + 1);
  if (!m.points || !m.pt_link || !m.parent || !m.joint)
    return fail(NPX_EINVAL, "morph %d: null table", idx);
  if (m.parent[0] != -1) return fail(NPX_EINVAL, "morph %d: parent[0] must be -1", idx);
  for (int l = 1; l < m.n_links; ++l)
    if (m.parent[l] < 0 || m.parent[l] >= l)
      return fail(NPX_EINVAL, "morph %d: parent[%d] = %d must be in [0, %d)", idx, l, m.parent[l], l);
  double M = 0;
  for (int k = 0; k < m.n_points; ++k) {
    if (m.pt_link[k] < 0 || m.pt_link[k] >= m.n_links)
      return fail(NPX_EINVAL, "morph %d: pt_link[%d] = %d out of range", idx, k, m.pt_link[k]);
    const float* p = m.points + 4 * k;
    if (!std::isfinite(p[0]) || !std::isfinite(p[1]) || !std::isfinite(p[2]) ||
        !std::isfinite(p[3]) || p[3] < 0)
      return fail(NPX_EINVAL, "morph %d: point %d not finite or negative mass", idx, k);
    M += p[3];
  }
  if (!(M > 0)) return fail(NPX_EINVAL, "morph %d: total mass must be > 0", idx);
  for (int l = 1; l < m.n_links; ++l) {
    const float* j = m.joint + 8 * l;
    double n2 = (double)j[3] * j[3] + (double)j[4] * j[4] + (double)j[5] * j[5];
    if (!(n2 > 0) || !std::isfinite(n2)) return fail(NPX_EINVAL, "morph %d: joint %d axis is zero", idx, l - 1);
    if (!(j[6] <= j[7])) return fail(NPX_EINVAL, "morph %d: joint %d limits lo > hi", idx, l - 1);
  }
  return NPX_OK;
}

}  // namespace

namespace npx {
WorldView world_view(const npx_world* w) {
  WorldView v;
  v.a = w->args;
  v.lp_off = w->lp_off;
  v.lp_idx = w->lp_idx;
  v.sub_mask = w->sub_mask;
  v.n_max = w->n_max;
  v.l_max = w->l_max;
  return v;
}

void note_stream(npx_world* w, hipStream_t s) {
  w->last_stream = s;
  w->has_last_stream = true;
}
}  // namespace npx

extern "C" {

const char* npx_last_error(void) { return g_err.c_str(); }
int npx_version(void) { return 1; }

npx_status npx_create_world(const npx_world_desc* d, npx_world** out) {
  if (!d || !out) return fail(NPX_EINVAL, "null argument");
  *out = nullptr;
  if (!(d->dt > 0) || d->joint_interval < 1) return fail(NPX_EINVAL, "dt must be > 0 and K >= 1");
  if (!(d->max_joint_rate >= 0)) return fail(NPX_EINVAL, "max_joint_rate must be >= 0");
  if (d->n_instances <= 0 || d->n_instances > (1 << 26))
    return fail(NPX_EINVAL, "n_instances %lld out of range", (long long)d->n_instances);
  if (d->n_morphs <= 0 || !d->morphs || !d->instance_morph || !d->init_pose)
    return fail(NPX_EINVAL, "missing morphologies, instance map or poses");
  if (d->hf_nx <= 0 || d->hf_ny <= 0 || !d->hf_heights || !(d->hf_s > 0))
    return fail(NPX_EINVAL, "bad height map");
  if (!(d->mu >= 0) || !(d->k_n >= 0) || !(d->zeta >= 0) || !(d->eps_lsq >= 0))
    return fail(NPX_EINVAL, "mu, k_n, zeta, eps must be >= 0");
  if (d->friction_weighting != 0 && d->friction_weighting != 1)
    return fail(NPX_EINVAL, "friction_weighting must be 0 or 1");
  if (d->hf_bilinear != 0 && d->hf_bilinear != 1)
    return fail(NPX_EINVAL, "hf_bilinear must be 0 or 1");
  if (d->friction_6dof != 0 && d->friction_6dof != 1)
    return fail(NPX_EINVAL, "friction_6dof must be 0 or 1");
  if (d->friction_6dof && d->friction_weighting)
    return fail(NPX_EINVAL, "friction_6dof with friction_weighting is not supported: with the "
                "weight on a set along one line, a point of near-zero force decides the roll "
                "about that line");
  for (int i = 0; i < d->n_morphs; ++i) {
    npx_status s = check_tables(d->morphs[i], i);
    if (s != NPX_OK) return s;
  }
  for (int64_t i = 0; i < d->n_instances; ++i)
    if (d->instance_morph[i] < 0 || d->instance_morph[i] >= d->n_morphs)
      return fail(NPX_EINVAL, "instance_morph[%lld] out of range", (long long)i);

  npx_world* w = new npx_world();
  HIP_TRY(hipGetDevice(&w->device));
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, w->device) == hipSuccess && cus > 0)
      w->cu_count = cus;
  }
  w->n_inst = (int)d->n_instances;
  w->n_morphs = d->n_morphs;
  w->dt = d->dt;
  w->K = d->joint_interval;
  w->mu = d->mu;
  w->inst_morph.assign(d->instance_morph, d->instance_morph + d->n_instances);

  // morphology CSR + per-link mass properties (double on the host, stored float)
  std::vector<int4> info(d->n_morphs);
  std::vector<float> mass(d->n_morphs);
  std::vector<float4> pts;
  std::vector<int> ptl, pto, par, fkt;
  std::vector<int2> fki;
  std::vector<std::vector<int>> slot_of(d->n_morphs);  // position of each point in pts
  std::vector<float> lk;
  for (int mi = 0; mi < d->n_morphs; ++mi) {
    const npx_morph_tables& m = d->morphs[mi];
    info[mi] = make_int4((int)pts.size(), m.n_points, (int)par.size(), m.n_links);
    w->morph_points.push_back(m.n_points);
    w->morph_links.push_back(m.n_links);
    w->n_max = std::max(w->n_max, m.n_points);
    w->l_max = std::max(w->l_max, m.n_links);
    std::vector<double> lm(m.n_links, 0.0), lc(3 * m.n_links, 0.0), lI(6 * m.n_links, 0.0);
    std::vector<int> depth(m.n_links, 0), children(m.n_links, 0);
    for (int l = 1; l < m.n_links; ++l) {
      depth[l] = depth[m.parent[l]] + 1;
      children[m.parent[l]] += 1;
    }
    // Point order in the tables: points of leaf links (the feet, usually the
    // only links near the ground) first, then the deeper links before the
    // shallower, each link's points in their own order. The step kernel puts
    // point k on lane k mod G, register slot k / G, and skips a slot when no
    // lane's point belongs to a link that may reach the ground, so this order
    // packs the points that get tested into the fewest slots.
    std::vector<int> order(m.n_points);
    for (int k = 0; k < m.n_points; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      const int lx = m.pt_link[x], ly = m.pt_link[y];
      const int kx = children[lx] == 0 ? 0 : 1, ky = children[ly] == 0 ? 0 : 1;
      if (kx != ky) return kx < ky;
      if (depth[lx] != depth[ly]) return depth[lx] > depth[ly];
      return lx < ly;
    });
    slot_of[mi].assign(m.n_points, 0);
    for (int k = 0; k < m.n_points; ++k) {
      const int o = order[k];
      const float* p = m.points + 4 * o;
      slot_of[mi][o] = k;
      pts.push_back(make_float4(p[0], p[1], p[2], p[3]));
      ptl.push_back(m.pt_link[o]);
      pto.push_back(o);
    }
    double M = 0;
    for (int k = 0; k < m.n_points; ++k) {
      const float* p = m.points + 4 * k;
      int l = m.pt_link[k];
      lm[l] += p[3];
      for (int i = 0; i < 3; ++i) lc[3 * l + i] += (double)p[3] * p[i];
      M += p[3];
    }
    for (int l = 0; l < m.n_links; ++l)
      for (int i = 0; i < 3; ++i) lc[3 * l + i] = lm[l] > 0 ? lc[3 * l + i] / lm[l] : 0.0;
    for (int k = 0; k < m.n_points; ++k) {
      const float* p = m.points + 4 * k;
      int l = m.pt_link[k];
      double r[3] = {p[0] - lc[3 * l], p[1] - lc[3 * l + 1], p[2] - lc[3 * l + 2]};
      double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
      double mk = p[3];
      lI[6 * l + 0] += mk * (rr - r[0] * r[0]);
      lI[6 * l + 1] += mk * (rr - r[1] * r[1]);
      lI[6 * l + 2] += mk * (rr - r[2] * r[2]);
      lI[6 * l + 3] -= mk * r[0] * r[1];
      lI[6 * l + 4] -= mk * r[0] * r[2];
      lI[6 * l + 5] -= mk * r[1] * r[2];
    }
    mass[mi] = (float)M;
    for (int l = 0; l < m.n_links; ++l) {
      w->max_depth = std::max(w->max_depth, depth[l]);
      par.push_back(m.parent[l]);
      const float* j = m.joint + 8 * l;
      float row[npx::LINK_F];
      for (int i = 0; i < 8; ++i) row[i] = l == 0 ? 0.f : j[i];
      if (l == 0) { row[6] = -1e30f; row[7] = 1e30f; }
      row[npx::LK_MASS] = (float)lm[l];
      for (int i = 0; i < 3; ++i) row[npx::LK_COG + i] = (float)lc[3 * l + i];
      for (int i = 0; i < 6; ++i) row[npx::LK_INERTIA + i] = (float)lI[6 * l + i];
      // box holding the link's points in the construction frame (rounded outward)
      {
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int k = 0; k < m.n_points; ++k)
          if (m.pt_link[k] == l)
            for (int i = 0; i < 3; ++i) {
              lo[i] = std::min(lo[i], (double)m.points[4 * k + i]);
              hi[i] = std::max(hi[i], (double)m.points[4 * k + i]);
            }
        for (int i = 0; i < 3; ++i) {
          if (!(lo[i] <= hi[i])) lo[i] = hi[i] = 0.0;  // a link without points
          row[npx::LK_BOX + i] = (float)(0.5 * (lo[i] + hi[i]));
          row[npx::LK_BOX + 3 + i] = (float)(0.5 * (hi[i] - lo[i]) * (1.0 + 1e-6) + 1e-6);
        }
      }
      lk.insert(lk.end(), row, row + npx::LINK_F);
    }
    fk_schedule(m, depth, fkt, fki);
  }
  w->j_max = std::max(1, w->l_max - 1);
  // points grouped by link (stable), for per-link sums outside the step kernel
  std::vector<int> lpo(1, 0), lpi;
  for (int mi = 0; mi < d->n_morphs; ++mi) {
    const npx_morph_tables& m = d->morphs[mi];
    const int p0 = info[mi].x;
    for (int l = 0; l < m.n_links; ++l) {
      for (int k = 0; k < m.n_points; ++k)
        if (m.pt_link[k] == l) lpi.push_back(p0 + slot_of[mi][k]);
      lpo.push_back((int)lpi.size());
    }
  }
  // subtree of every link as a bit mask over the morphology's links (<= 64)
  std::vector<unsigned long long> subm;
  for (int mi = 0; mi < d->n_morphs; ++mi) {
    const npx_morph_tables& m = d->morphs[mi];
    std::vector<unsigned long long> mk(m.n_links, 0ull);
    for (int l = m.n_links - 1; l >= 0; --l) {
      if (l < 64) mk[l] |= 1ull << l;
      if (l > 0) mk[m.parent[l]] |= mk[l];
    }
    subm.insert(subm.end(), mk.begin(), mk.end());
  }
  if (!shape_for(w, 64, &w->shape)) {
    delete w;
    return fail(NPX_EUNSUPPORTED, "no kernel shape for %d points / %d links", w->n_max, w->l_max);
  }

  const size_t I = (size_t)w->n_inst;
  const size_t rows = (size_t)npx::state_rows(w->j_max);
  auto cleanup_fail = [&](npx_status s) {
    npx_destroy_world(w);
    return s;
  };
#define ALLOC(p, n)                                                                    \
  if (dalloc(&(p), (n)) != hipSuccess)                                                 \
    return cleanup_fail(fail(NPX_ENOMEM, "device allocation of %s failed", #p));
  // the state buffers: the caller's device memory where given, else the world's
  {
    const size_t need[4] = {rows * I * sizeof(float), I * sizeof(int), I * sizeof(int),
                            I * npx::TELE_N * sizeof(double)};
    void** dst[4] = {reinterpret_cast<void**>(&w->st), reinterpret_cast<void**>(&w->step),
                     reinterpret_cast<void**>(&w->flags), reinterpret_cast<void**>(&w->tele)};
    for (int k = 0; k < 4; ++k) {
      void* p = d->ext_device_buffers[k];
      if (!p) continue;
      hipPointerAttribute_t at{};
      void* base = nullptr;
      size_t size = 0;
      if ((reinterpret_cast<uintptr_t>(p) & 15u) != 0 ||
          hipPointerGetAttributes(&at, p) != hipSuccess || at.type != hipMemoryTypeDevice ||
          at.device != w->device || hipMemGetAddressRange(&base, &size, p) != hipSuccess ||
          static_cast<char*>(p) + need[k] > static_cast<char*>(base) + size) {
        (void)hipGetLastError();
        return cleanup_fail(fail(NPX_EINVAL,
                                 "ext_device_buffers[%d]: not 16-byte aligned device memory of "
                                 "this device holding %zu bytes",
                                 k, need[k]));
      }
      *dst[k] = p;
      w->ext_state[k] = true;
    }
  }
  if (!w->ext_state[0]) ALLOC(w->st, rows * I);
  if (!w->ext_state[1]) ALLOC(w->step, I);
  if (!w->ext_state[2]) ALLOC(w->flags, I);
  if (!w->ext_state[3]) ALLOC(w->tele, I * npx::TELE_N);
  ALLOC(w->inst_morph_d, I);
  ALLOC(w->morph_info, info.size());
  ALLOC(w->morph_mass, mass.size());
  ALLOC(w->pts, pts.size());
  ALLOC(w->pt_link, ptl.size());
  ALLOC(w->pt_orig, pto.size());
  ALLOC(w->links, lk.size());
  ALLOC(w->link_parent, par.size());
  if (fkt.empty()) fkt.push_back(-1);  // no link deeper than 1: no passes, one unread entry
  ALLOC(w->fk_task, fkt.size());
  ALLOC(w->fk_info, fki.size());
  ALLOC(w->ctrl, I * w->j_max * 3);
  ALLOC(w->hf, (size_t)d->hf_nx * d->hf_ny);
  ALLOC(w->task_info, 2 * I);
  ALLOC(w->queue, 1);
  ALLOC(w->lp_off, lpo.size());
  ALLOC(w->lp_idx, lpi.size());
  ALLOC(w->sub_mask, subm.size());
#undef ALLOC

  auto h2d = [&](void* dst, const void* src, size_t bytes) {
    return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
  };
#define H2D(dst, src, bytes)                                                           \
  if (h2d((dst), (src), (bytes)) != hipSuccess)                                        \
    return cleanup_fail(fail(NPX_EHIP, "copy of %s failed", #dst));
  H2D(w->inst_morph_d, d->instance_morph, I * sizeof(int));
  H2D(w->morph_info, info.data(), info.size() * sizeof(int4));
  H2D(w->morph_mass, mass.data(), mass.size() * sizeof(float));
  H2D(w->pts, pts.data(), pts.size() * sizeof(float4));
  H2D(w->pt_link, ptl.data(), ptl.size() * sizeof(int));
  H2D(w->pt_orig, pto.data(), pto.size() * sizeof(int));
  H2D(w->links, lk.data(), lk.size() * sizeof(float));
  H2D(w->link_parent, par.data(), par.size() * sizeof(int));
  H2D(w->fk_task, fkt.data(), fkt.size() * sizeof(int));
  H2D(w->fk_info, fki.data(), fki.size() * sizeof(int2));
  H2D(w->lp_off, lpo.data(), lpo.size() * sizeof(int));
  H2D(w->lp_idx, lpi.data(), lpi.size() * sizeof(int));
  w->lp_off_host = lpo;
  w->lp_idx_host = lpi;
  H2D(w->sub_mask, subm.data(), subm.size() * sizeof(unsigned long long));
  H2D(w->hf, d->hf_heights, (size_t)d->hf_nx * d->hf_ny * sizeof(float));
  std::vector<int> ord = task_order(w);
  {
    // what the step kernel needs of a task at the start of a launch, in one
    // place: the instance, its morphology's table offsets and sizes, its mass
    std::vector<int4> ti(2 * I);
    for (size_t t = 0; t < I; ++t) {
      const int inst = ord[t], mi = d->instance_morph[inst];
      float m = mass[mi];
      int mb;
      std::memcpy(&mb, &m, sizeof(int));
      ti[2 * t] = make_int4(inst, mi, info[mi].x, info[mi].z);
      ti[2 * t + 1] = make_int4(info[mi].y, info[mi].w, mb, 0);
    }
    H2D(w->task_info, ti.data(), ti.size() * sizeof(int4));
  }
  {
    std::vector<float> zero(I * w->j_max * 3, 0.f);
    H2D(w->ctrl, d->ctrl ? d->ctrl : zero.data(), zero.size() * sizeof(float));
    std::vector<int> zi(I, 0);
    H2D(w->step, zi.data(), I * sizeof(int));
    H2D(w->flags, zi.data(), I * sizeof(int));
    std::vector<double> zt(I * npx::TELE_N, 0.0);
    H2D(w->tele, zt.data(), zt.size() * sizeof(double));
  }
#undef H2D

  npx::StepArgs& a = w->args;
  a.n_inst = w->n_inst;
  a.n_tasks = w->n_inst;
  a.task_info = w->task_info;
  a.j_max = w->j_max;
  a.max_depth = w->max_depth;
  a.inst_morph = w->inst_morph_d;
  a.morph_info = w->morph_info;
  a.morph_mass = w->morph_mass;
  a.pts = w->pts;
  a.pt_link = w->pt_link;
  a.pt_orig = w->pt_orig;
  a.links = w->links;
  a.link_parent = w->link_parent;
  a.fk_task = w->fk_task;
  a.fk_info = w->fk_info;
  a.ctrl = w->ctrl;
  a.dt = (float)d->dt;
  a.inv_dt = (float)(1.0 / d->dt);
  a.dt_d = d->dt;
  a.K = d->joint_interval;
  a.rate_step = (d->max_joint_rate > 0 && !std::isinf(d->max_joint_rate))
                    ? (float)(d->max_joint_rate * d->joint_interval * d->dt)
                    : 0.f;
  a.gx = (float)d->g[0];
  a.gy = (float)d->g[1];
  a.gz = (float)d->g[2];
  a.mu_inf = std::isinf(d->mu) ? 1 : 0;
  a.mu = a.mu_inf ? 0.f : (float)d->mu;
  a.kn = (float)d->k_n;
  a.zeta = (float)d->zeta;
  a.eps = (float)d->eps_lsq;
  a.fric_w = d->friction_weighting;
  a.fric6 = d->friction_6dof;
  a.hf_bilinear = d->hf_bilinear;
  a.hf = w->hf;
  a.hf_nx = d->hf_nx;
  a.hf_ny = d->hf_ny;
  a.hf_s = (float)d->hf_s;
  a.hf_x0 = (float)d->hf_x0;
  a.hf_ax = hf_axis(d->hf_x0, d->hf_s, d->hf_nx);
  a.hf_ay = hf_axis(d->hf_y0, d->hf_s, d->hf_ny);
  a.hf_y0 = (float)d->hf_y0;
  a.hf_max = -INFINITY;
  for (size_t k = 0; k < (size_t)d->hf_nx * d->hf_ny; ++k) a.hf_max = std::max(a.hf_max, d->hf_heights[k]);
  a.st = w->st;
  a.step = w->step;
  a.flags = w->flags;
  a.tele = w->tele;
  a.n_max = w->n_max;

  if (hipStreamCreateWithFlags(&w->capture_stream, hipStreamNonBlocking) != hipSuccess)
    return cleanup_fail(fail(NPX_EHIP, "stream creation failed"));

  // initial state: at rest, q = q_cmd(0) = 0 for the zero controller; the CoG
  // follows from the pose through the kernel's own mass properties
  {
    std::vector<float> host(rows * I, 0.f);
    for (size_t i = 0; i < I; ++i) {
      const float* p = d->init_pose + 7 * i;
      double qn = std::sqrt((double)p[3] * p[3] + (double)p[4] * p[4] + (double)p[5] * p[5] + (double)p[6] * p[6]);
      if (!(qn > 0) || !std::isfinite(qn)) return cleanup_fail(fail(NPX_EINVAL, "pose %zu: bad quaternion", i));
      for (int k = 0; k < 3; ++k) host[k * I + i] = p[k];
      for (int k = 0; k < 4; ++k) host[(3 + k) * I + i] = (float)(p[3 + k] / qn);
    }
    if (h2d(w->st, host.data(), host.size() * sizeof(float)) != hipSuccess)
      return cleanup_fail(fail(NPX_EHIP, "state upload failed"));
  }
  // q = q_cmd(0) and the torso-origin pose turned into the CoG, by the step
  // kernel's own joint and mass-property path
  {
    npx::StepArgs pa = w->args;
    pa.n_steps = 0;
    pa.place = 1;
    pa.queue = nullptr;
    const int ipw = 64 / w->shape.G;
    pa.n_blocks = (pa.n_tasks + ipw - 1) / ipw;
    hipError_t e = npx::launch_step(pa, w->shape, pa.n_blocks, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return cleanup_fail(fail(NPX_EHIP, "placement kernel: %s", hipGetErrorString(e)));
  }
  *out = w;
  return NPX_OK;
}

void npx_destroy_world(npx_world* w) {
  if (!w) return;
  if (w->has_last_stream) (void)hipStreamSynchronize(w->last_stream);
  w->drop_graphs();
  if (w->capture_stream) (void)hipStreamDestroy(w->capture_stream);
  if (w->ext_state[0]) w->st = nullptr;  // the caller's memory
  if (w->ext_state[1]) w->step = nullptr;
  if (w->ext_state[2]) w->flags = nullptr;
  if (w->ext_state[3]) w->tele = nullptr;
  void* bufs[] = {w->st, w->step, w->flags, w->tele, w->inst_morph_d, w->morph_info,
                  w->morph_mass, w->pts, w->pt_link, w->pt_orig, w->links, w->link_parent,
                  w->fk_task, w->fk_info, w->ctrl, w->hf, w->task_info, w->queue,
                  w->lp_off,
                  w->lp_idx, w->sub_mask, w->rays, w->ray_link, w->ray_info,
                  w->foot_pairs, w->foot_info};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  delete w;
}

npx_status npx_world_dims(const npx_world* w, int64_t* n_instances, int32_t* j_max, int32_t* n_max) {
  if (!w) return fail(NPX_EINVAL, "null world");
  if (n_instances) *n_instances = w->n_inst;
  if (j_max) *j_max = w->j_max;
  if (n_max) *n_max = w->n_max;
  return NPX_OK;
}

npx_status npx_set_controller(npx_world* w, int kind, const float* params, size_t n_floats,
                              int on_device) {
  if (!w || !params) return fail(NPX_EINVAL, "null argument");
  if (kind == NPX_CTRL_TARGETS) {
    const size_t nt = (size_t)w->n_inst * w->j_max;
    if (n_floats != nt) return fail(NPX_EINVAL, "targets need %zu floats, got %zu", nt, n_floats);
    npx_status s = sync_last(w);
    if (s != NPX_OK) return s;
    if (on_device) {
      HIP_TRY(npx::launch_targets(params, w->ctrl, (int64_t)nt, nullptr));
      HIP_TRY(hipDeviceSynchronize());
    } else {
      std::vector<float> rows(3 * nt);
      for (size_t k = 0; k < nt; ++k) {
        rows[3 * k] = params[k];
        rows[3 * k + 1] = 0.f;
        rows[3 * k + 2] = npx::HALF_PI_F;
      }
      HIP_TRY(hipMemcpy(w->ctrl, rows.data(), rows.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    return NPX_OK;
  }
  if (kind != NPX_CTRL_SINUSOID) return fail(NPX_EUNSUPPORTED, "controller kind %d", kind);
  const size_t need = (size_t)w->n_inst * w->j_max * 3;
  if (n_floats != need) return fail(NPX_EINVAL, "controller needs %zu floats, got %zu", need, n_floats);
  npx_status s = sync_last(w);
  if (s != NPX_OK) return s;
  HIP_TRY(hipMemcpy(w->ctrl, params, need * sizeof(float),
                    on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
  return NPX_OK;
}

npx_status npx_step_n(npx_world* w, int64_t n, void* hip_stream) {
  if (!w) return fail(NPX_EINVAL, "null world");
  if (n < 0) return fail(NPX_EINVAL, "n must be >= 0");
  if (n == 0) return NPX_OK;
  return run_steps(w, n, (hipStream_t)hip_stream);
}

// ---- stepping without allocation ---------------------------------------------
//
// The persistent-queue counters of npx_step_n_noalloc, one per chunk launch of
// a call, live in this file-scope device array: every GPU the library runs on
// holds its own copy until the process ends. Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the symbol):
// the per-device address comes from hipGetSymbolAddress, taken once per device
// with that device current.
static __device__ __align__(256) int scratch[NPX_NOALLOC_MAX_CHUNKS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int* g_scratch[kMaxDevices] = {};

npx_status scratch_counters(int device, int** out) {
  if (device < 0 || device >= kMaxDevices) return fail(NPX_EINVAL, "device %d out of range", device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != device) HIP_TRY(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
      return fail(NPX_EHIP, "hipGetSymbolAddress of the step counters: %s", hipGetErrorString(e));
    g_scratch[device] = (int*)p;
  }
  *out = g_scratch[device];
  return NPX_OK;
}
}  // namespace

npx_status npx_step_n_noalloc(npx_world* w, int64_t n, void* hip_stream) {
  if (!w) return fail(NPX_EINVAL, "null world");
  if (n < 0) return fail(NPX_EINVAL, "n must be >= 0");
  if (n == 0) return NPX_OK;
  const int chunk = std::max(1, w->launch.chunk_steps);
  const int64_t n_chunks = (n + chunk - 1) / chunk;
  if (n_chunks > NPX_NOALLOC_MAX_CHUNKS)
    return fail(NPX_EINVAL,
                "npx_step_n_noalloc: %lld frames in chunks of %d need %lld launches; its static "
                "counters hold %d (split the call or raise chunk_steps)",
                (long long)n, chunk, (long long)n_chunks, NPX_NOALLOC_MAX_CHUNKS);
  hipStream_t s = (hipStream_t)hip_stream;
  int* q = nullptr;
  if (w->launch.persistent) {
    const npx_status rc = scratch_counters(w->device, &q);
    if (rc != NPX_OK) return rc;
    HIP_TRY(npx::launch_zero_n(q, (int)n_chunks, s));
  }
  int64_t left = n;
  for (int64_t k = 0; left > 0; ++k) {
    const int c = (int)std::min<int64_t>(left, chunk);
    const hipError_t e = enqueue_chunk(w, c, s, q ? q + k : nullptr);
    if (e != hipSuccess) return fail(NPX_EHIP, "step launch: %s", hipGetErrorString(e));
    left -= c;
  }
  w->last_stream = s;
  w->has_last_stream = true;
  return NPX_OK;
}

npx_status npx_read_state(npx_world* w, int field, void* dst, size_t bytes, int on_device) {
  if (!w || !dst) return fail(NPX_EINVAL, "null argument");
  size_t row0 = 0, rows = 0;
  int kind = 0;
  size_t need = field_bytes(w, field, &row0, &rows, &kind);
  if (need == 0) return fail(NPX_EINVAL, "unknown field %d", field);
  if (bytes != need) return fail(NPX_EINVAL, "field %d needs %zu bytes, got %zu", field, need, bytes);
  npx_status s = sync_last(w);
  if (s != NPX_OK) return s;
  const void* src = kind == 0 ? (const void*)(w->st + row0 * w->n_inst)
                  : kind == 1 ? (const void*)w->step
                  : kind == 2 ? (const void*)w->flags : (const void*)w->tele;
  HIP_TRY(hipMemcpy(dst, src, need, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
  return NPX_OK;
}

npx_status npx_write_state(npx_world* w, int field, const void* src, size_t bytes, int on_device) {
  if (!w || !src) return fail(NPX_EINVAL, "null argument");
  size_t row0 = 0, rows = 0;
  int kind = 0;
  size_t need = field_bytes(w, field, &row0, &rows, &kind);
  if (need == 0) return fail(NPX_EINVAL, "unknown field %d", field);
  if (bytes != need) return fail(NPX_EINVAL, "field %d needs %zu bytes, got %zu", field, need, bytes);
  npx_status s = sync_last(w);
  if (s != NPX_OK) return s;
  void* dst = kind == 0 ? (void*)(w->st + row0 * w->n_inst)
            : kind == 1 ? (void*)w->step
            : kind == 2 ? (void*)w->flags : (void*)w->tele;
  HIP_TRY(hipMemcpy(dst, src, need, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
  return NPX_OK;
}

npx_status npx_read_points(npx_world* w, float* dst, size_t bytes, int on_device) {
  if (!w || !dst) return fail(NPX_EINVAL, "null argument");
  const size_t need = (size_t)w->n_inst * w->n_max * 3 * sizeof(float);
  if (bytes != need) return fail(NPX_EINVAL, "points need %zu bytes, got %zu", need, bytes);
  npx_status s = sync_last(w);
  if (s != NPX_OK) return s;
  float* buf = nullptr;
  if (on_device) {
    buf = dst;
  } else if (hipMalloc((void**)&buf, need) != hipSuccess) {
    return fail(NPX_ENOMEM, "points buffer");
  }
  npx_status rc = NPX_OK;
  do {
    if (hipMemset(buf, 0, need) != hipSuccess) { rc = fail(NPX_EHIP, "memset"); break; }
    npx::StepArgs a = w->args;
    a.n_steps = 0;
    a.queue = nullptr;
    a.points_out = buf;
    const int ipw = 64 / w->shape.G;
    a.n_blocks = (a.n_tasks + ipw - 1) / ipw;
    hipError_t e = npx::launch_step(a, w->shape, a.n_blocks, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) { rc = fail(NPX_EHIP, "points kernel: %s", hipGetErrorString(e)); break; }
    if (!on_device && hipMemcpy(dst, buf, need, hipMemcpyDeviceToHost) != hipSuccess) {
      rc = fail(NPX_EHIP, "points copy");
      break;
    }
  } while (0);
  if (!on_device) (void)hipFree(buf);
  return rc;
}

npx_status npx_world_set_rays(npx_world* w, int32_t morph, int32_t n_rays, const float* rays,
                              const int32_t* ray_link) {
  if (!w) return fail(NPX_EINVAL, "null world");
  if (morph < 0 || morph >= w->n_morphs) return fail(NPX_EINVAL, "morph %d out of range", morph);
  if (n_rays < 0 || n_rays > npx::RAY_MAX)
    return fail(NPX_EINVAL, "n_rays %d out of [0, %d]", n_rays, npx::RAY_MAX);
  if (n_rays > 0 && (!rays || !ray_link)) return fail(NPX_EINVAL, "null ray table");
  const int L = w->morph_links[morph];
  for (int k = 0; k < n_rays; ++k) {
    if (ray_link[k] < 0 || ray_link[k] >= L)
      return fail(NPX_EINVAL, "ray %d: link %d out of [0, %d)", k, ray_link[k], L);
    const float* r = rays + 6 * k;
    for (int e = 0; e < 6; ++e)
      if (!std::isfinite(r[e])) return fail(NPX_EINVAL, "ray %d: non-finite coordinate", k);
    // a rigid ray keeps its length; the cells it crosses are at most
    // s (|dx| + |dy|) + 3 <= s sqrt(2) length + 3
    const double len = std::sqrt((double)(r[3] - r[0]) * (r[3] - r[0]) +
                                 (double)(r[4] - r[1]) * (r[4] - r[1]) +
                                 (double)(r[5] - r[2]) * (r[5] - r[2]));
    if (w->args.hf_s * std::sqrt(2.0) * len + 4.0 > npx::RAY_MAX_CELLS)
      return fail(NPX_EINVAL, "ray %d crosses more than %d cells", k, npx::RAY_MAX_CELLS);
  }
  npx_status st = sync_last(w);
  if (st != NPX_OK) return st;
  w->ray_host.resize(w->n_morphs);
  w->ray_link_host.resize(w->n_morphs);
  w->ray_host[morph].assign(rays, rays + 6 * (size_t)n_rays);
  w->ray_link_host[morph].assign(ray_link, ray_link + n_rays);
  std::vector<float> all;
  std::vector<int> links;
  std::vector<int2> info(w->n_morphs);
  int rmax = 0;
  for (int m = 0; m < w->n_morphs; ++m) {
    const int n = (int)w->ray_link_host[m].size();
    info[m] = make_int2((int)links.size(), n);
    all.insert(all.end(), w->ray_host[m].begin(), w->ray_host[m].end());
    links.insert(links.end(), w->ray_link_host[m].begin(), w->ray_link_host[m].end());
    rmax = std::max(rmax, n);
  }
  HIP_TRY(hipDeviceSynchronize());
  void* old[] = {w->rays, w->ray_link, w->ray_info};
  for (void* b : old)
    if (b) (void)hipFree(b);
  w->rays = nullptr;
  w->ray_link = nullptr;
  w->ray_info = nullptr;
  w->ray_max = 0;
  const size_t nr = std::max<size_t>(links.size(), 1);
  if (hipMalloc((void**)&w->rays, nr * 6 * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&w->ray_link, nr * sizeof(int)) != hipSuccess ||
      hipMalloc((void**)&w->ray_info, info.size() * sizeof(int2)) != hipSuccess)
    return fail(NPX_ENOMEM, "ray tables");
  if (!links.empty()) {
    HIP_TRY(hipMemcpy(w->rays, all.data(), all.size() * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(w->ray_link, links.data(), links.size() * sizeof(int),
                      hipMemcpyHostToDevice));
  }
  HIP_TRY(hipMemcpy(w->ray_info, info.data(), info.size() * sizeof(int2), hipMemcpyHostToDevice));
  w->ray_max = rmax;
  return NPX_OK;
}

namespace {

// Rebuilds the device tables of the foot sensors from the host lists: every
// (sensor, point) pair of a morphology, so that the lanes of the controller
// kernel take the sensed points in parallel.
npx_status upload_feet(npx_world* w) {
  w->foot_host.resize(w->n_morphs);
  std::vector<int4> pairs;
  std::vector<int4> info(w->n_morphs);
  int lk0 = 0;
  for (int m = 0; m < w->n_morphs; ++m) {
    const int first = (int)pairs.size();
    const std::vector<int>& feet = w->foot_host[m];
    for (int sidx = 0; sidx < (int)feet.size(); ++sidx) {
      const int gl = lk0 + feet[sidx];
      for (int p = w->lp_off_host[gl]; p < w->lp_off_host[gl + 1]; ++p)
        pairs.push_back(make_int4(sidx, w->lp_idx_host[p], feet[sidx], 0));
    }
    info[m] = make_int4(first, (int)pairs.size() - first, (int)feet.size(), 0);
    lk0 += w->morph_links[m];
  }
  HIP_TRY(hipDeviceSynchronize());
  w->drop_graphs();  // captured controller launches hold the old table pointers
  if (w->foot_pairs) (void)hipFree(w->foot_pairs);
  if (w->foot_info) (void)hipFree(w->foot_info);
  w->foot_pairs = nullptr;
  w->foot_info = nullptr;
  if (hipMalloc((void**)&w->foot_pairs, std::max<size_t>(pairs.size(), 1) * sizeof(int4)) !=
          hipSuccess ||
      hipMalloc((void**)&w->foot_info, info.size() * sizeof(int4)) != hipSuccess)
    return fail(NPX_ENOMEM, "sensor tables");
  if (!pairs.empty())
    HIP_TRY(hipMemcpy(w->foot_pairs, pairs.data(), pairs.size() * sizeof(int4),
                      hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w->foot_info, info.data(), info.size() * sizeof(int4), hipMemcpyHostToDevice));
  return NPX_OK;
}

}  // namespace

npx_status npx_world_set_sensors(npx_world* w, int32_t morph, int32_t n, const int32_t* links) {
  if (!w) return fail(NPX_EINVAL, "null world");
  if (morph < 0 || morph >= w->n_morphs) return fail(NPX_EINVAL, "morph %d out of range", morph);
  if (n < 0 || n > npx::FOOT_MAX) return fail(NPX_EINVAL, "n %d out of [0, %d]", n, npx::FOOT_MAX);
  if (n > 0 && !links) return fail(NPX_EINVAL, "null sensor list");
  for (int k = 0; k < n; ++k)
    if (links[k] < 0 || links[k] >= w->morph_links[morph])
      return fail(NPX_EINVAL, "sensor %d: link %d out of [0, %d)", k, links[k],
                  w->morph_links[morph]);
  npx_status st = sync_last(w);
  if (st != NPX_OK) return st;
  w->foot_host.resize(w->n_morphs);
  w->foot_host[morph].assign(links, links + n);
  return upload_feet(w);
}

npx_status npx_gp_run(npx_world* w, const uint8_t* programs, int32_t* vm, float* targets,
                      int64_t ld_targets, int32_t n_updates, int32_t n_instr, float motor_step,
                      void* hip_stream) {
  if (!w || !programs || !vm || !targets) return fail(NPX_EINVAL, "null argument");
  if (ld_targets < w->j_max)
    return fail(NPX_EINVAL, "ld_targets %lld below J_max %d", (long long)ld_targets, w->j_max);
  if (n_updates < 0 || n_instr < 0 || n_instr > 4096)
    return fail(NPX_EINVAL, "n_updates must be >= 0 and n_instr in [0, 4096]");
  if (!(motor_step >= 0.f) || std::isinf(motor_step))
    return fail(NPX_EINVAL, "motor_step must be finite and >= 0");
  if (!w->foot_info) {
    npx_status st = upload_feet(w);
    if (st != NPX_OK) return st;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  const npx::GpArgs g{programs, vm, targets, ld_targets, w->foot_pairs, w->foot_info, n_instr,
                      motor_step, w->ctrl};
  // Whole blocks of updates replay one captured graph (the launches of a
  // block, back to back, without a host round per launch); the rest, and
  // every update when graphs are off, are launched one by one.
  constexpr int GP_BLOCK = 25;
  int u = 0;
  if (w->launch.use_graph && n_updates >= GP_BLOCK) {
    const npx::GpArgs& k = w->gp_key;
    const bool same = w->gp_exec && k.prog == g.prog && k.vm == g.vm && k.targets == g.targets &&
                      k.ld_targets == g.ld_targets && k.foot_pairs == g.foot_pairs &&
                      k.foot_info == g.foot_info && k.n_instr == g.n_instr &&
                      k.step == g.step && k.ctrl == g.ctrl;
    if (!same) {
      if (w->gp_exec) (void)hipGraphExecDestroy(w->gp_exec);
      if (w->gp_graph) (void)hipGraphDestroy(w->gp_graph);
      w->gp_exec = nullptr;
      w->gp_graph = nullptr;
      HIP_TRY(hipStreamBeginCapture(w->capture_stream, hipStreamCaptureModeThreadLocal));
      hipError_t e = hipSuccess;
      const npx::WorldView v = npx::world_view(w);
      const int chunk = std::max(1, w->launch.chunk_steps);
      for (int b = 0; b < GP_BLOCK && e == hipSuccess; ++b) {
        e = npx::launch_gp(v, g, w->capture_stream);
        for (int left = w->K; left > 0 && e == hipSuccess; left -= chunk)
          e = enqueue_chunk(w, std::min(left, chunk), w->capture_stream);
      }
      hipGraph_t gr = nullptr;
      hipError_t e2 = hipStreamEndCapture(w->capture_stream, &gr);
      if (e != hipSuccess) return fail(NPX_EHIP, "capture of controller updates: %s", hipGetErrorString(e));
      if (e2 != hipSuccess) return fail(NPX_EHIP, "end capture: %s", hipGetErrorString(e2));
      hipGraphExec_t ge = nullptr;
      if (hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(gr);
        return fail(NPX_EHIP, "instantiating the controller updates failed");
      }
      w->gp_graph = gr;
      w->gp_exec = ge;
      w->gp_key = g;
    }
    for (; u + GP_BLOCK <= n_updates; u += GP_BLOCK) HIP_TRY(hipGraphLaunch(w->gp_exec, st));
  }
  for (; u < n_updates; ++u) {
    HIP_TRY(npx::launch_gp(npx::world_view(w), g, st));
    npx_status r = run_steps(w, w->K, st);
    if (r != NPX_OK) return r;
  }
  w->last_stream = st;
  w->has_last_stream = true;
  npx::note_stream(w, st);
  return NPX_OK;
}

npx_status npx_world_ray_ranges(npx_world* w, float* dst, int64_t ld, void* hip_stream) {
  if (!w || !dst) return fail(NPX_EINVAL, "null argument");
  if (w->args.hf_bilinear)
    return fail(NPX_EINVAL, "ray ranges read the height map as its look-up table; this world "
                            "reads it bilinearly");
  if (ld < std::max(w->ray_max, 1))
    return fail(NPX_EINVAL, "ld %lld below the largest ray count %d", (long long)ld, w->ray_max);
  if (w->ray_max == 0) return NPX_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  const npx::RayTables r{w->rays, w->ray_link, w->ray_info};
  HIP_TRY(npx::launch_ray_ranges(npx::world_view(w), r, dst, ld, st));
  npx::note_stream(w, st);
  return NPX_OK;
}

npx_status npx_get_launch(const npx_world* w, npx_launch* out) {
  if (!w || !out) return fail(NPX_EINVAL, "null argument");
  *out = w->launch;
  return NPX_OK;
}

npx_status npx_set_launch(npx_world* w, const npx_launch* cfg) {
  if (!w || !cfg) return fail(NPX_EINVAL, "null argument");
  npx::Shape s;
  if (!shape_for(w, cfg->lanes_per_instance, &s))
    return fail(NPX_EUNSUPPORTED, "no kernel with %d lanes per instance for %d points / %d links",
                cfg->lanes_per_instance, w->n_max, w->l_max);
  if (cfg->chunk_steps < 1 || cfg->chunk_steps > 100000)
    return fail(NPX_EINVAL, "chunk_steps %d out of [1, 100000]", cfg->chunk_steps);
  if (cfg->persistent && (cfg->waves_per_cu < 1 || cfg->waves_per_cu > 32))
    return fail(NPX_EINVAL, "waves_per_cu %d out of [1, 32]", cfg->waves_per_cu);
  npx_status st = sync_last(w);
  if (st != NPX_OK) return st;
  w->drop_graphs();
  w->launch = *cfg;
  w->shape = s;
  return NPX_OK;
}

npx_status npx_autotune(npx_world* w, int32_t steps, void* hip_stream, npx_launch* best,
                        npx_launch* tried, float* times_ms, int32_t max_results, int32_t* n_tried) {
  if (!w || steps < 1) return fail(NPX_EINVAL, "bad autotune arguments");
  hipStream_t s = (hipStream_t)hip_stream;
  npx_status rc = sync_last(w);
  if (rc != NPX_OK) return rc;
  // scratch copies of the mutable state so the world's state is untouched
  const size_t I = (size_t)w->n_inst;
  const size_t rows = (size_t)npx::state_rows(w->j_max);
  float* st2 = nullptr;
  int *step2 = nullptr, *flags2 = nullptr;
  double* tele2 = nullptr;
  if (dalloc(&st2, rows * I) != hipSuccess || dalloc(&step2, I) != hipSuccess ||
      dalloc(&flags2, I) != hipSuccess || dalloc(&tele2, I * npx::TELE_N) != hipSuccess) {
    (void)hipFree(st2); (void)hipFree(step2); (void)hipFree(flags2); (void)hipFree(tele2);
    return fail(NPX_ENOMEM, "autotune scratch");
  }
  npx::StepArgs saved = w->args;
  npx_launch saved_launch = w->launch;
  npx::Shape saved_shape = w->shape;
  w->args.st = st2;
  w->args.step = step2;
  w->args.flags = flags2;
  w->args.tele = tele2;
  std::vector<npx_launch> cands;
  const int chunk = std::max(1, std::min(steps, saved_launch.chunk_steps));
  for (int G : {64, 32, 16}) {
    npx::Shape sh;
    if (!shape_for(w, G, &sh)) continue;
    cands.push_back(npx_launch{G, 0, chunk, 0, 8});
    for (int wpc : {4, 8, 16}) cands.push_back(npx_launch{G, 1, chunk, 0, wpc});
  }
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  // A persistent shape is taken only when it beats the others by more than
  // kPersistentMargin: a direct launch deals contiguous shares of the robots
  // to the XCDs and needs no queue reset, and near-ties measured over one
  // chunk here flip between runs, while the direct launch keeps its edge in
  // short timed launches.
  constexpr float kPersistentMargin = 1.03f;
  float best_ms = 1e30f;
  npx_launch best_cfg = saved_launch;
  int count = 0;
  rc = NPX_OK;
  for (const npx_launch& c : cands) {
    w->drop_graphs();
    w->launch = c;
    shape_for(w, c.lanes_per_instance, &w->shape);
    hipError_t e = hipMemcpyAsync(st2, w->st, rows * I * sizeof(float), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(step2, w->step, I * sizeof(int), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(flags2, w->flags, I * sizeof(int), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) { rc = fail(NPX_EHIP, "autotune copy"); break; }
    // warm-up (also builds nothing: graphs are off while tuning)
    if ((rc = run_steps(w, std::min(steps, chunk), s)) != NPX_OK) break;
    (void)hipEventRecord(e0, s);
    if ((rc = run_steps(w, steps, s)) != NPX_OK) break;
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) { rc = fail(NPX_EHIP, "autotune sync"); break; }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (tried && times_ms && count < max_results) {
      tried[count] = c;
      times_ms[count] = ms;
    }
    ++count;
    const float score = c.persistent ? ms * kPersistentMargin : ms;
    if (score < best_ms) {
      best_ms = score;
      best_cfg = c;
    }
  }
  (void)hipStreamSynchronize(s);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  w->drop_graphs();
  w->args = saved;
  w->launch = saved_launch;
  w->shape = saved_shape;
  (void)hipFree(st2);
  (void)hipFree(step2);
  (void)hipFree(flags2);
  (void)hipFree(tele2);
  if (n_tried) *n_tried = count;
  if (rc != NPX_OK) return rc;
  best_cfg.chunk_steps = saved_launch.chunk_steps;
  best_cfg.use_graph = saved_launch.use_graph;
  if (best) *best = best_cfg;
  return npx_set_launch(w, &best_cfg);
}

npx_status npx_flops_per_step(const npx_world* w, int64_t i, double* flops) {
  if (!w || !flops || i < 0 || i >= w->n_inst) return fail(NPX_EINVAL, "bad arguments");
  const int mi = w->inst_morph[i];
  const double N = w->morph_points[mi], L = w->morph_links[mi], K = w->K;
  // per point every frame: two body-to-world transforms (15 + 3 each) and two
  // table look-ups (4 + 1 each); per point every K frames: y = T rho - g_b (21);
  // per link every K frames: controller 6, hinge rotation 35 + 18, tree
  // composition 63, mass properties 131; per robot every frame: ~400
  // (integration, inertia inverse, quaternion exponential, closed-form fit,
  // cap, correction, telemetry). Contact-dependent force and moment terms
  // (~30 per contact point) are not counted.
  *flops = 46.0 * N + (21.0 * N + 253.0 * L) / K + 400.0;
  return NPX_OK;
}

}  // extern "C"
