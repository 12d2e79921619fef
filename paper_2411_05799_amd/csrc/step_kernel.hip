// The NeoPhysIx frame for many robots at once, FP32, gfx950.
//
// Layout of the work: a wave of 64 lanes holds 64/G robots; each robot owns a
// segment of G consecutive lanes. A segment's lanes share the robot's mass
// points (point k lives on lane k mod G, register slot k / G) and its links
// (link l on lane l mod G, slot l / G). Per-robot scalars (CoG, orientation,
// velocities, forces, the friction fit) are kept redundantly in every lane of
// the segment, so the per-point phases need no broadcast. Segment-wide sums
// (contact force and torque, link mass properties, the friction moments) are
// all-reductions made of DPP adds inside 16-lane rows and permlane swaps
// across rows; every lane ends with the same bits and the order is fixed, so
// a robot's trajectory does not depend on which segment or wave runs it. Link
// transforms pass from link lanes to point lanes through LDS. The state stays
// in registers for a whole launch of n_steps frames and touches HBM once at
// each end.
//
// The frame (Sec. III; readings as in the oracle):
//   S1 detection of every point against the height-map table (Sec. III-A)
//   S2 normal penalty forces along +z, summed to force and torque about the CoG
//   S3 joint-angle determination every K frames (Sec. III-B): new joint angles,
//      new body points about the unchanged world CoG
//   S4 trial semi-implicit Euler step to the predicted points P*
//   S5 friction set: in contact at P^n and at P* (eq. 3)
//   S6 the normal equations (4)-(6) solved in closed form
//   S7 cap by the maximum static friction mu F_N (Sec. III-C)
//   S8 move back by the capped fit, remove the matching velocity, commit
//
// Precision of the friction fit. The fit works on the slip delta = P* - P^n
// of each contact point, typically 1e-5..1e-3 m, while body points sit 0.1 m
// or more from the CoG. Taking delta as the difference of two independently
// rounded float32 positions would leave ~4e-8 m of incoherent noise per point,
// and with two or three contact points that noise dominates the fitted
// rotation. The slip is therefore built from increments that float32 holds
// accurately: the joint-angle increment is pushed down the link tree as a
// transform increment dT (forward kinematics of the change; the CoG's own move
// in the body frame, one offset shared by every point, is the difference of
// the two CoGs), and the body rotation increment comes straight from the
// rotation quaternion:
//   delta = (R1 - R) r_old + R1 dr + (c1 - c),  R1 - R = (R(dq) - I) R.
#include "npx_device.h"
#include "npx_internal.h"

namespace npx {

namespace {

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}

// The value of the lane 16 apart within the 32-lane half (LDS crossbar, no
// VALU move): swizzle with and-mask 31, xor-mask 16.
__device__ __forceinline__ float xor16(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, x), 0x401F));
}

__device__ __forceinline__ float swap_sum32(float x) {
  auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, x),
                                            __builtin_bit_cast(unsigned, x), false, false);
  return __builtin_bit_cast(float, (unsigned)r[0]) + __builtin_bit_cast(float, (unsigned)r[1]);
}

// Sums over the G-lane segment of N values at once, results in every lane of
// it: lanes exchange with quad partners, then the mirrored half-row and row
// (DPP), then the other row (swizzle) and the other half-wave (permlane32
// swap). Each step adds two operands in an order every lane shares, and takes
// all N values before the next step, so no add waits on the one before.
template <int G, int N>
__device__ __forceinline__ void seg_sum_n(float (&x)[N]) {
  static_assert(G == 16 || G == 32 || G == 64, "segment of 16, 32 or 64 lanes");
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] += dpp<0xB1>(x[i]);   // quad_perm [1,0,3,2]
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] += dpp<0x4E>(x[i]);   // quad_perm [2,3,0,1]
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] += dpp<0x141>(x[i]);  // row_half_mirror
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] += dpp<0x140>(x[i]);  // row_mirror
  if constexpr (G >= 32) {
    float o[N];
#pragma unroll
    for (int i = 0; i < N; ++i) o[i] = xor16(x[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] += o[i];
  }
  if constexpr (G >= 64) {
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = swap_sum32(x[i]);
  }
}

// The same sums for doubles: each exchange moves the two 32-bit halves.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const unsigned long long v = __builtin_bit_cast(unsigned long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)v, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double xor16_d(double x) {
  const unsigned long long v = __builtin_bit_cast(unsigned long long, x);
  const int lo = __builtin_amdgcn_ds_swizzle((int)(unsigned)v, 0x401F);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(unsigned)(v >> 32), 0x401F);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double swap_sum32_d(double x) {
  const unsigned long long v = __builtin_bit_cast(unsigned long long, x);
  auto lo = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
  auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(v >> 32), (unsigned)(v >> 32), false, false);
  const double a = __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi[0] << 32) | (unsigned)lo[0]);
  const double b = __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi[1] << 32) | (unsigned)lo[1]);
  return a + b;
}

template <int G, int N>
__device__ __forceinline__ void seg_sum_nd(double (&x)[N]) {
  static_assert(G == 16 || G == 32 || G == 64, "segment of 16, 32 or 64 lanes");
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] += dpp_d<0xB1>(x[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] += dpp_d<0x4E>(x[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] += dpp_d<0x141>(x[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] += dpp_d<0x140>(x[i]);
  if constexpr (G >= 32) {
    double o[N];
#pragma unroll
    for (int i = 0; i < N; ++i) o[i] = xor16_d(x[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] += o[i];
  }
  if constexpr (G >= 64) {
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = swap_sum32_d(x[i]);
  }
}

template <int G>
__device__ __forceinline__ float seg_sum(float x) {
  float v[1] = {x};
  seg_sum_n<G>(v);
  return v[0];
}

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Points are processed in groups of kGroup per lane; the scheduler may overlap
// the loads of one group with the arithmetic of the next but not hoist every
// point's loads to the top of a loop, which would cost a register set per point.
constexpr int kGroup = 2;
__device__ __forceinline__ void group_fence(int p) {
  if ((p + 1) % kGroup == 0) __builtin_amdgcn_sched_barrier(0);
}

// Height-map look-up (Sec. III-A) of the world's table, or (BIL, a kernel
// built for worlds that ask for it) its bilinear reading.
template <bool BIL>
__device__ __forceinline__ float hf_at(const StepArgs& a, float x, float y) {
  if constexpr (BIL) return hf_bilinear(a.hf, a.hf_nx, a.hf_ny, a.hf_x0, a.hf_y0, a.hf_s, x, y);
  return hf_lookup(a.hf, a.hf_nx, a.hf_ax, a.hf_ay, x, y);
}

// The bits of a wave-wide lane mask that belong to segment `seg` (G lanes),
// shifted down to bit 0.
template <int G>
__device__ __forceinline__ unsigned long long seg_bits(unsigned long long m, int seg) {
  if constexpr (G == 64) {
    (void)seg;
    return m;
  } else {
    return (m >> (seg * G)) & ((1ull << G) - 1ull);
  }
}

enum Mode { kStep = 0, kPlace = 1, kPoints = 2 };

// The six-degree friction fit takes a 3-D rotation only when the contact set's
// thinnest spread is at least this fraction of the trace of its spread tensor.
constexpr float kSixDofCond = 1e-3f;

// XCDs of the MI355X (eight, 32 compute units each).
constexpr unsigned kXcds = 8;

// LDS rows of one link: [R row 0 | t0], [R row 1 | t1], [R row 2 | t2].
using LinkT = float4[3];

// A link's constants for one launch (LDS). With a the unit hinge axis, o the
// anchor and K = [a]x (so K^2 = a a^T - 1): a and the upper limit; u = K o and
// the lower limit; w = K^2 o and the controller's amplitude; a_x a_y, a_x a_z,
// a_y a_z and its frequency; the diagonal of K^2 (a_i^2 - 1) and the link's
// mass; the CoG; the inertia about the CoG (xx yy zz xy, then xz yz) with the
// last two half extents of the box of the link's points; the box centre and
// first half extent; the controller's phase in turns.
struct LinkConst {
  float4 ax_hi, u_lo, w_A, aa_f, kd_m, cog, I0, I1_box, box0;
  double ph;
};

template <int G, int PPL, int LPL, int MODE, bool BIL, bool SIX>
__device__ __forceinline__ void run_block(const StepArgs& a, LinkT* T, LinkT* dT, int* cand,
                                          LinkConst* LK, int tb, int seg,
                                          int sl) {
  constexpr int IPW = 64 / G;
  const int I = a.n_inst;
  const int task = tb * IPW + seg;
  const bool valid = task < a.n_tasks;
  // the task's instance, morphology offsets, sizes and mass in one load pair
  // (a past-the-end task reads task 0's and steps nothing)
  const int4 ta = a.task_info[2 * (valid ? task : 0)];
  const int4 tc = a.task_info[2 * (valid ? task : 0) + 1];
  const int inst = valid ? ta.x : 0;
  const int mi = ta.y;
  const int N = valid ? tc.x : 0;
  const int L = valid ? tc.y : 1;
  const int pt_off = ta.z, lk_off = ta.w;
  const float M = __int_as_float(tc.z);
  const float invM = rcp(M);
  const float* st = a.st;

  // ---- per-robot state (same value in every lane of the segment), loaded
  // first: these loads depend on nothing but the instance, so they are in
  // flight while the link tables below are read
  float c[3], Q[4], v[3], w[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    c[i] = st[(size_t)i * I + inst];
    v[i] = st[(size_t)(7 + i) * I + inst];
    w[i] = st[(size_t)(10 + i) * I + inst];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) Q[i] = st[(size_t)(3 + i) * I + inst];
  int n = a.step[inst];
  int fl = a.flags[inst];
  double tele[TELE_N];
#pragma unroll
  for (int i = 0; i < TELE_N; ++i) tele[i] = a.tele[(size_t)i * I + inst];

  // ---- links of this lane: table row and joint angles (the rest of the link
  // data is read from the cache-resident tables where it is used)
  int lrow[LPL];
  bool lv[LPL], lj[LPL];
  float q[LPL], qp[LPL];
#pragma unroll
  for (int l = 0; l < LPL; ++l) {
    const int li = sl + l * G;
    lv[l] = li < L;
    lj[l] = lv[l] && li >= 1;
    lrow[l] = lk_off + (lv[l] ? li : 0);
    const int j = lj[l] ? li - 1 : 0;  // (row 0 of the joints when this lane has none)
    const float qv = st[(size_t)(BODY_ROWS + j) * I + inst];
    const float qpv = st[(size_t)(BODY_ROWS + a.j_max + j) * I + inst];
    q[l] = lj[l] ? qv : 0.f;
    qp[l] = lj[l] ? qpv : 0.f;
  }

  // ---- this lane's link constants, staged in LDS once per launch (each lane
  // writes and reads only its own links' entries, so no barrier is needed);
  // held in registers they would be spilled under the 256-register cap
#pragma unroll
  for (int l = 0; l < LPL; ++l) {
    const int li = sl + l * G;
    const float* lk = a.links + (size_t)lrow[l] * LINK_F;
    const float n2 = lk[3] * lk[3] + lk[4] * lk[4] + lk[5] * lk[5];
    const float inv = n2 > 0.f ? __builtin_amdgcn_rsqf(n2) : 0.f;
    const float x = lk[3] * inv, y = lk[4] * inv, z = lk[5] * inv;
    const float o[3] = {lk[0], lk[1], lk[2]};
    const float ao = x * o[0] + y * o[1] + z * o[2];
    const float* cp = a.ctrl + ((size_t)inst * a.j_max + (lj[l] ? li - 1 : 0)) * 3;
    LinkConst k;
    k.ax_hi = make_float4(x, y, z, lk[7]);
    k.u_lo = make_float4(y * o[2] - z * o[1], z * o[0] - x * o[2], x * o[1] - y * o[0], lk[6]);
    k.w_A = make_float4(x * ao - o[0], y * ao - o[1], z * ao - o[2], cp[0]);
    k.aa_f = make_float4(x * y, x * z, y * z, cp[1]);
    k.kd_m = make_float4(x * x - 1.f, y * y - 1.f, z * z - 1.f, lk[LK_MASS]);
    k.cog = make_float4(lk[LK_COG], lk[LK_COG + 1], lk[LK_COG + 2], 0.f);
    k.I0 = make_float4(lk[LK_INERTIA], lk[LK_INERTIA + 1], lk[LK_INERTIA + 2], lk[LK_INERTIA + 3]);
    k.I1_box = make_float4(lk[LK_INERTIA + 4], lk[LK_INERTIA + 5], lk[LK_BOX + 4], lk[LK_BOX + 5]);
    k.box0 = make_float4(lk[LK_BOX], lk[LK_BOX + 1], lk[LK_BOX + 2], lk[LK_BOX + 3]);
    k.ph = (double)cp[2] * kInvTwoPi;
    LK[li] = k;
  }
  // chain-composition passes of this robot's morphology for G-lane segments
  const int2 fki = a.fk_info[mi * 3 + (G == 16 ? 0 : (G == 32 ? 1 : 2))];
  const int fk_np = valid ? fki.y : 0;
  const int* fk_t = a.fk_task + fki.x + sl;
  // the first pass's task of this lane, held for the launch (the later
  // passes' are loaded one pass ahead)
  const int fk_r0 = fk_np > 0 ? fk_t[0] : -1;

  // ---- the link of each of this lane's points (6 bits per slot, five slots
  // per register), read once per launch. Every slot's load is issued (a slot
  // past the robot's points reads its first point's entry, which every
  // morphology has, and keeps 0), so the loads travel together instead of
  // one guarded round trip per slot.
  constexpr int PACKW = (PPL + 4) / 5;
  unsigned plk[PACKW];
#pragma unroll
  for (int w = 0; w < PACKW; ++w) plk[w] = 0u;
  unsigned lkp[PPL];
#pragma unroll
  for (int p = 0; p < PPL; ++p) {
    const int k = sl + p * G;
    lkp[p] = (unsigned)a.pt_link[pt_off + (k < N ? k : 0)];
  }
#pragma unroll
  for (int p = 0; p < PPL; ++p) {
    const unsigned lk = sl + p * G < N ? lkp[p] : 0u;
    plk[p / 5] |= (lk & 63u) << (6 * (p % 5));
  }
  // Which of the slots past the first NRC hold points of which links, for
  // the detection's skip test. First, per link (gathered in the candidate
  // list's LDS, which no frame has used yet), the slots that hold one of its
  // points in some lane of the segment; then, transposed by one ballot per
  // slot, lanes p and 32 + p of the wave hold in smask[l] the low and high
  // halves of the link lanes (bit layout of the broad phase's ballot
  // tmask[l]) whose links have points in slot p. A frame's broad-phase
  // verdicts then decide every slot at once: slot p is tested when a half of
  // its mask meets the links that may touch.
  constexpr int NRC = PPL < 3 ? PPL : 3;
  static_assert(PPL <= 32, "slot masks take lanes p and 32 + p");
  const bool hi_half = threadIdx.x >= 32;
  unsigned smask[LPL];
  if constexpr (MODE == kStep) {
    unsigned* ls = reinterpret_cast<unsigned*>(cand);
#pragma unroll
    for (int l = 0; l < LPL; ++l) ls[sl + l * G] = 0u;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int p = NRC; p < PPL; ++p)
      if (sl + p * G < N) atomicOr(&ls[lkp[p]], 1u << p);
    __builtin_amdgcn_wave_barrier();
    unsigned lsl[LPL];
#pragma unroll
    for (int l = 0; l < LPL; ++l) lsl[l] = ls[sl + l * G];
    __builtin_amdgcn_wave_barrier();
    const int slot = (int)(threadIdx.x & 31u);
#pragma unroll
    for (int l = 0; l < LPL; ++l) {
      smask[l] = 0u;
#pragma unroll
      for (int p = NRC; p < PPL; ++p) {
        const unsigned long long b = __ballot((lsl[l] >> p) & 1u);
        smask[l] = slot == p ? (unsigned)(hi_half ? b >> 32 : b) : smask[l];
      }
    }
  }
  float rc[NRC][3];
#pragma unroll
  for (int p = 0; p < NRC; ++p) {
    const int k = sl + p * G;
    const float4 r4 = a.pts[pt_off + (k < N ? k : 0)];
    rc[p][0] = r4.x;
    rc[p][1] = r4.y;
    rc[p][2] = r4.z;
  }

  // ---- mass properties and their increments; body points about the CoG are
  // not kept: a point is rebuilt from its construction-frame position and its
  // link's transform in LDS where it is needed, which keeps the registers of a
  // lane independent of its point count
  float gb[3] = {0.f, 0.f, 0.f}, dgb[3], Ib[6], Iinv[6];

  // Forward kinematics at angles q, with the increment from angles q - dql
  // (dql = 0: no joint moved). Writes T, dT for every link of the segment.
  auto forward_kinematics = [&](const float* dql) __attribute__((always_inline)) {
    // Each joint's own transform about its hinge and its increment go into the
    // link's LDS rows: with K = [a]x, the rotation is Rj = 1 + s K + (1 - c) K^2
    // (Rodrigues) and its translation o - Rj o = -(s u + (1 - c) w). The
    // increment over the last joint step, Rj(q) - Rj(q - dq) = -Rj(q) E with
    // E = sin t K + (1 - cos t) K^2 at t = -dq, reduces by K^3 = -K to
    // -(alpha K + beta K^2), alpha = sin t c - (1 - cos t) s,
    // beta = sin t s + (1 - cos t) c, and moves the origin by alpha u + beta w.
#pragma unroll
    for (int l = 0; l < LPL; ++l) {
      const int li = sl + l * G;
      const float4 k0 = LK[li].ax_hi, k1 = LK[li].u_lo, k2 = LK[li].w_A;
      const float4 k3 = LK[li].aa_f, k4 = LK[li].kd_m;
      const float x = k0.x, y = k0.y, z = k0.z;
      const float xy = k3.x, xz = k3.y, yz = k3.z;
      float s, co;
      sin_cos(q[l], &s, &co);
      const float C1 = 1.f - co;
      const float sx = s * x, sy = s * y, sz = s * z;
      // the joint increment is a fraction of a degree per frame: below 0.1 rad
      // sin t = t (1 - t^2/6 (1 - t^2/20)) and 1 - cos t = t^2/2 (1 - t^2/12
      // (1 - t^2/30)) to float32 precision (the next terms are 1e-10 relative);
      // 1 - cos t = 2 sin^2(t/2) above keeps it exact for larger steps
      float se, ve;
      const float tq = -dql[l];
      if (!__any(!(fabsf(tq) < 0.1f))) {
        const float t2 = tq * tq;
        se = tq * (1.f - t2 * (1.f / 6.f) * (1.f - t2 * (1.f / 20.f)));
        ve = 0.5f * t2 * (1.f - t2 * (1.f / 12.f) * (1.f - t2 * (1.f / 30.f)));
      } else {
        float ce, sh, ch;
        sin_cos(tq, &se, &ce);
        sin_cos(0.5f * tq, &sh, &ch);
        ve = 2.f * sh * sh;
      }
      const float al = se * co - ve * s, be = se * s + ve * co;
      const float ax_ = al * x, ay_ = al * y, az_ = al * z;
      if (lj[l]) {
        T[li][0] = make_float4(fmaf(C1, k4.x, 1.f), fmaf(C1, xy, -sz), fmaf(C1, xz, sy),
                               -(s * k1.x + C1 * k2.x));
        T[li][1] = make_float4(fmaf(C1, xy, sz), fmaf(C1, k4.y, 1.f), fmaf(C1, yz, -sx),
                               -(s * k1.y + C1 * k2.y));
        T[li][2] = make_float4(fmaf(C1, xz, -sy), fmaf(C1, yz, sx), fmaf(C1, k4.z, 1.f),
                               -(s * k1.z + C1 * k2.z));
        dT[li][0] = make_float4(-be * k4.x, fmaf(-be, xy, az_), fmaf(-be, xz, -ay_),
                                al * k1.x + be * k2.x);
        dT[li][1] = make_float4(fmaf(-be, xy, -az_), -be * k4.y, fmaf(-be, yz, ax_),
                                al * k1.y + be * k2.y);
        dT[li][2] = make_float4(fmaf(-be, xz, ay_), fmaf(-be, yz, -ax_), -be * k4.z,
                                al * k1.z + be * k2.z);
      }
    }
    if (sl == 0) {
      T[0][0] = make_float4(1.f, 0.f, 0.f, 0.f);
      T[0][1] = make_float4(0.f, 1.f, 0.f, 0.f);
      T[0][2] = make_float4(0.f, 0.f, 1.f, 0.f);
      dT[0][0] = dT[0][1] = dT[0][2] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    // Links of depth 1 hang from the torso (identity): their joint transform
    // is final. Deeper links, level by level, one matrix row per lane: row i of
    // the link's transform and increment from row i of the parent's final ones
    // (P, dP) and the link's joint transform (J, dJ):
    //   T_i = P_i J,  dT_i = dP_i J + (P_i - dP_i) dJ   (3x4 rows, affine).
    // A lane reads the whole J before any lane of the wave writes a row of it,
    // and the next pass reads what this one wrote, so program order within the
    // wave is the only ordering needed.
    __builtin_amdgcn_wave_barrier();
    int fk_next = fk_r0;
    for (int p = 0; __any(p < fk_np); ++p) {
      const int task = fk_next;
      fk_next = p + 1 < fk_np ? fk_t[(p + 1) * G] : -1;
      if (task >= 0) {
        const int i = task & 3, lk = (task >> 2) & 127, pa = task >> 9;
        const float4 P = T[pa][i], dP = dT[pa][i];
        const float4 j0 = T[lk][0], j1 = T[lk][1], j2 = T[lk][2];
        const float4 e0 = dT[lk][0], e1 = dT[lk][1], e2 = dT[lk][2];
        const float ox = P.x - dP.x, oy = P.y - dP.y, oz = P.z - dP.z;
        const float4 r = make_float4(P.x * j0.x + P.y * j1.x + P.z * j2.x,
                                     P.x * j0.y + P.y * j1.y + P.z * j2.y,
                                     P.x * j0.z + P.y * j1.z + P.z * j2.z,
                                     P.x * j0.w + P.y * j1.w + P.z * j2.w + P.w);
        const float4 d = make_float4(
            dP.x * j0.x + dP.y * j1.x + dP.z * j2.x + ox * e0.x + oy * e1.x + oz * e2.x,
            dP.x * j0.y + dP.y * j1.y + dP.z * j2.y + ox * e0.y + oy * e1.y + oz * e2.y,
            dP.x * j0.z + dP.y * j1.z + dP.z * j2.z + ox * e0.z + oy * e1.z + oz * e2.z,
            dP.x * j0.w + dP.y * j1.w + dP.z * j2.w + ox * e0.w + oy * e1.w + oz * e2.w + dP.w);
        T[lk][i] = r;
        dT[lk][i] = d;
      }
      __builtin_amdgcn_wave_barrier();
    }
    // mass properties: over links, m p and R I R^T + m (|p|^2 1 - p p^T)
    float acc[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) acc[i] = 0.f;
#pragma unroll
    for (int l = 0; l < LPL; ++l) {
      if (lv[l]) {
        const int li = sl + l * G;
        const float4 r0 = T[li][0], r1 = T[li][1], r2 = T[li][2];
        const float R[9] = {r0.x, r0.y, r0.z, r1.x, r1.y, r1.z, r2.x, r2.y, r2.z};
        const float4 cm = LK[li].cog, i0 = LK[li].I0, i1 = LK[li].I1_box;
        const float lc[3] = {cm.x, cm.y, cm.z};
        const float m = LK[li].kd_m.w;
        float p[3];
        p[0] = R[0] * lc[0] + R[1] * lc[1] + R[2] * lc[2] + r0.w;
        p[1] = R[3] * lc[0] + R[4] * lc[1] + R[5] * lc[2] + r1.w;
        p[2] = R[6] * lc[0] + R[7] * lc[1] + R[8] * lc[2] + r2.w;
        acc[0] += m * p[0];
        acc[1] += m * p[1];
        acc[2] += m * p[2];
        // A = R I (I symmetric: xx yy zz xy xz yz)
        const float S[6] = {i0.x, i0.y, i0.z, i0.w, i1.x, i1.y};
        const float Ifull[9] = {S[0], S[3], S[4], S[3], S[1], S[5], S[4], S[5], S[2]};
        float A[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int k = 0; k < 3; ++k)
            A[3 * i + k] = R[3 * i] * Ifull[k] + R[3 * i + 1] * Ifull[3 + k] +
                           R[3 * i + 2] * Ifull[6 + k];
        const float pp = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
        // (A R^T)_ik = sum_j A_ij R_kj
        acc[3] += A[0] * R[0] + A[1] * R[1] + A[2] * R[2] + m * (pp - p[0] * p[0]);
        acc[4] += A[3] * R[3] + A[4] * R[4] + A[5] * R[5] + m * (pp - p[1] * p[1]);
        acc[5] += A[6] * R[6] + A[7] * R[7] + A[8] * R[8] + m * (pp - p[2] * p[2]);
        acc[6] += A[0] * R[3] + A[1] * R[4] + A[2] * R[5] - m * p[0] * p[1];
        acc[7] += A[0] * R[6] + A[1] * R[7] + A[2] * R[8] - m * p[0] * p[2];
        acc[8] += A[3] * R[6] + A[4] * R[7] + A[5] * R[8] - m * p[1] * p[2];
      }
    }
    seg_sum_n<G>(acc);
    // the CoG's move in the body frame over the joint step, from the CoG
    // before it: both are rounded sums of a few centimetres (a few 1e-9 m),
    // the same offset for every point of the friction set
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const float g = acc[i] * invM;
      dgb[i] = g - gb[i];
      gb[i] = g;
    }
    const float gg = gb[0] * gb[0] + gb[1] * gb[1] + gb[2] * gb[2];
    Ib[0] = acc[3] - M * (gg - gb[0] * gb[0]);
    Ib[1] = acc[4] - M * (gg - gb[1] * gb[1]);
    Ib[2] = acc[5] - M * (gg - gb[2] * gb[2]);
    Ib[3] = acc[6] + M * gb[0] * gb[1];
    Ib[4] = acc[7] + M * gb[0] * gb[2];
    Ib[5] = acc[8] + M * gb[1] * gb[2];
    {
      const float xx = Ib[0], yy = Ib[1], zz = Ib[2], xy = Ib[3], xz = Ib[4], yz = Ib[5];
      const float c00 = yy * zz - yz * yz, c11 = xx * zz - xz * xz, c22 = xx * yy - xy * xy;
      const float c01 = xz * yz - xy * zz, c02 = xy * yz - xz * yy, c12 = xy * xz - xx * yz;
      const float det = xx * c00 + xy * c01 + xz * c02;
      const float tr = (xx + yy + zz) * (1.f / 3.f);
      const bool reg = tr > 0.f && det > 1e-9f * tr * tr * tr;
      const float id = reg ? rcp(det) : 0.f;
      Iinv[0] = c00 * id; Iinv[1] = c11 * id; Iinv[2] = c22 * id;
      Iinv[3] = c01 * id; Iinv[4] = c02 * id; Iinv[5] = c12 * id;
    }
  };

  // Body point k of this robot about the CoG (construction axes) from the link
  // transforms in T; returns false past the robot's point count.
  auto body_point = [&](int k, float* r) __attribute__((always_inline)) {
    const bool ok = k < N;
    const int kk = pt_off + (ok ? k : 0);
    const float4 rho = a.pts[kk];
    const int lk = ok ? a.pt_link[kk] : 0;
    const float4 r0 = T[lk][0], r1 = T[lk][1], r2 = T[lk][2];
    r[0] = r0.x * rho.x + r0.y * rho.y + r0.z * rho.z + r0.w - gb[0];
    r[1] = r1.x * rho.x + r1.y * rho.y + r1.z * rho.z + r1.w - gb[1];
    r[2] = r2.x * rho.x + r2.y * rho.y + r2.z * rho.z + r2.w - gb[2];
    return ok;
  };

  // S0: commanded angle of this lane's joints at frame n, clamped to the limits
  auto command = [&](int l) __attribute__((always_inline)) {
    const double t = (double)n * a.dt_d;
    const int li = sl + l * G;
    const float qh = LK[li].w_A.w * sin_turns((double)LK[li].aa_f.w * t + LK[li].ph);
    return lj[l] ? fminf(fmaxf(qh, LK[li].u_lo.w), LK[li].ax_hi.w) : 0.f;
  };

  float dql[LPL];
#pragma unroll
  for (int l = 0; l < LPL; ++l) dql[l] = 0.f;
  if (MODE == kPlace) {
#pragma unroll
    for (int l = 0; l < LPL; ++l) {
      q[l] = command(l);
      qp[l] = q[l];
    }
  }

  const float dt = a.dt, inv_dt = a.inv_dt;
  // The frame loop is rotated so that the forward kinematics has one call site:
  // each pass runs the pending kinematics (the launch's first, or the joint
  // update of the frame before), then the rest of that frame (S4-S9), then the
  // start of the next (S1-S3). A second inlined copy of the kinematics could
  // round differently and make a trajectory depend on where launches begin.
  bool fk_pending = true, fk_now = false;
  // the torso rotation of Q, kept beside it: set from the same conversion of
  // the same quaternion wherever Q changes, so it is bitwise quat_to_mat(Q)
  float Rq[9];
  quat_to_mat(Q[0], Q[1], Q[2], Q[3], Rq);
  unsigned kap = 0u;
  unsigned kap_slots = 0u;  // slots with a contact point in some lane of the wave
  float F = 0.f, tx = 0.f, ty = 0.f, nc = 0.f;
  for (int s = 0;; ++s) {
    if (fk_pending) forward_kinematics(dql);
    fk_pending = false;
    if (MODE == kStep && s > 0) {
      const bool active = valid && fl == 0;
      const float* R = Rq;
      // S4: trial step. Body-frame Euler equation: I_b dw_b = tau_b - w_b x I_b w_b
      float v1[3], w1[3], c1[3], Q1[4], dq[4];
      v1[0] = v[0] + dt * a.gx;
      v1[1] = v[1] + dt * a.gy;
      v1[2] = v[2] + dt * (a.gz + F * invM);
      {
        const float wb[3] = {R[0] * w[0] + R[3] * w[1] + R[6] * w[2],
                             R[1] * w[0] + R[4] * w[1] + R[7] * w[2],
                             R[2] * w[0] + R[5] * w[1] + R[8] * w[2]};
        const float tb_[3] = {R[0] * tx + R[3] * ty, R[1] * tx + R[4] * ty, R[2] * tx + R[5] * ty};
        const float Lb[3] = {Ib[0] * wb[0] + Ib[3] * wb[1] + Ib[4] * wb[2],
                             Ib[3] * wb[0] + Ib[1] * wb[1] + Ib[5] * wb[2],
                             Ib[4] * wb[0] + Ib[5] * wb[1] + Ib[2] * wb[2]};
        const float rb[3] = {tb_[0] - (wb[1] * Lb[2] - wb[2] * Lb[1]),
                             tb_[1] - (wb[2] * Lb[0] - wb[0] * Lb[2]),
                             tb_[2] - (wb[0] * Lb[1] - wb[1] * Lb[0])};
        const float ab[3] = {Iinv[0] * rb[0] + Iinv[3] * rb[1] + Iinv[4] * rb[2],
                             Iinv[3] * rb[0] + Iinv[1] * rb[1] + Iinv[5] * rb[2],
                             Iinv[4] * rb[0] + Iinv[5] * rb[1] + Iinv[2] * rb[2]};
  #pragma unroll
        for (int i = 0; i < 3; ++i)
          w1[i] = w[i] + dt * (R[3 * i] * ab[0] + R[3 * i + 1] * ab[1] + R[3 * i + 2] * ab[2]);
      }
  #pragma unroll
      for (int i = 0; i < 3; ++i) c1[i] = c[i] + dt * v1[i];
      {
        const float th0 = dt * w1[0], th1 = dt * w1[1], th2 = dt * w1[2];
        const float ang2 = th0 * th0 + th1 * th1 + th2 * th2;
        if (!__any(!(ang2 < 0.01f))) {
          // half angle h below 0.05 rad: cos h and sin(h) / |theta| = sin(h) / (2h)
          // from their series in h^2 to float32 precision (next terms < 1e-12)
          const float h2 = 0.25f * ang2;
          const float k = 0.5f - h2 * (1.f / 12.f) * (1.f - h2 * (1.f / 20.f));
          dq[0] = 1.f - 0.5f * h2 * (1.f - h2 * (1.f / 12.f) * (1.f - h2 * (1.f / 30.f)));
          dq[1] = k * th0; dq[2] = k * th1; dq[3] = k * th2;
        } else if (ang2 < 1e-24f) {
          dq[0] = 1.f; dq[1] = 0.5f * th0; dq[2] = 0.5f * th1; dq[3] = 0.5f * th2;
        } else {
          const float ang = __builtin_amdgcn_sqrtf(ang2);
          float sh, ch;
          sin_cos(0.5f * ang, &sh, &ch);
          const float k = sh * rcp(ang);
          dq[0] = ch; dq[1] = k * th0; dq[2] = k * th1; dq[3] = k * th2;
        }
        Q1[0] = dq[0] * Q[0] - dq[1] * Q[1] - dq[2] * Q[2] - dq[3] * Q[3];
        Q1[1] = dq[0] * Q[1] + dq[1] * Q[0] + dq[2] * Q[3] - dq[3] * Q[2];
        Q1[2] = dq[0] * Q[2] - dq[1] * Q[3] + dq[2] * Q[0] + dq[3] * Q[1];
        Q1[3] = dq[0] * Q[3] + dq[1] * Q[2] - dq[2] * Q[1] + dq[3] * Q[0];
        const float inv = __builtin_amdgcn_rsqf(Q1[0] * Q1[0] + Q1[1] * Q1[1] + Q1[2] * Q1[2] +
                                                Q1[3] * Q1[3]);
  #pragma unroll
        for (int i = 0; i < 4; ++i) Q1[i] *= inv;
      }
      float R1[9];
      quat_to_mat(Q1[0], Q1[1], Q1[2], Q1[3], R1);
      // R(dq) - 1 = 2 w [v]x + 2 [v]x^2 for the unit increment dq = (w, v)
      float Eb[9];
      {
        const float w0 = dq[0], x = dq[1], y = dq[2], z = dq[3];
        Eb[0] = -2.f * (y * y + z * z); Eb[1] = 2.f * (x * y - w0 * z); Eb[2] = 2.f * (x * z + w0 * y);
        Eb[3] = 2.f * (x * y + w0 * z); Eb[4] = -2.f * (x * x + z * z); Eb[5] = 2.f * (y * z - w0 * x);
        Eb[6] = 2.f * (x * z - w0 * y); Eb[7] = 2.f * (y * z + w0 * x); Eb[8] = -2.f * (x * x + y * y);
      }

      // S5 + S6 moments over the friction set in the ground plane: source
      // xi = P^n - c1 = R r_old - (c1 - c), slip delta = P* - P^n. The normal
      // equations (4)-(6) need n, sum xi, sum |xi|^2, sum delta and
      // sum xi x delta. The sums over xi are taken about one point of the set
      // itself (the first one found; eta = xi - o = U - U_o with U = R r_old):
      // about the CoG, or about any point far from the set, a foot-sized set
      // 0.3 m away leaves D = sum |xi|^2 - |sum xi|^2 / n to a float32
      // difference of two nearly equal numbers. The fit is covariant in its
      // origin: the rotation a3 is the same and the displacement about c1 is
      // a = b - a3 J o (J: quarter turn), o = U_o - dt v1.
      //
      // Only points in contact at P^n can be in the friction set, and they are
      // few (the feet), so they are first compacted into an LDS list (slot by
      // slot, in lane order) and the segment's lanes then share the list: one
      // pass of G candidates instead of PPL mostly idle slots.
      int n_cand = 0;
      for (unsigned rest = kap_slots; rest != 0u; rest &= rest - 1u) {
        const int p = __builtin_ctz(rest);
        const bool hit = (kap >> p) & 1u;
        const unsigned long long m = seg_bits<G>(__ballot(hit), seg);
        if (hit) cand[n_cand + __popcll(m & ((1ull << sl) - 1ull))] = sl + p * G;
        n_cand += __popcll(m);
      }
      __builtin_amdgcn_wave_barrier();
      // The trial displacement of the CoG enters the slip as dt v1 itself, not
      // as c1 - c: c1 is rounded to float32 (half an ulp, 1.2e-7 m at |c| ~ 2 m),
      // and a fit that took that rounding for slip would return it as a
      // velocity change of 1.2e-7 m / dt.
      const float dcx = dt * v1[0], dcy = dt * v1[1], dcz = dt * v1[2];
      float mn = 0.f, Sx = 0.f, Sy = 0.f, S2 = 0.f, Dx = 0.f, Dy = 0.f, Cd = 0.f, Wt = 0.f;
      // the six-degree fit's moments, in double (the moments about a set member
      // lose digits to the centroid's removal when the set is wide and its
      // slips large): Sx Sy Sz, Dx Dy Dz, sum s s^T (xx yy zz xy xz yz) and
      // sum s x delta (3)
      double dm[15];
#pragma unroll
      for (int i = 0; i < 15; ++i) dm[i] = 0.0;
      float ox_ = 0.f, oy_ = 0.f, oz_ = 0.f;  // origin of the moments (about c), see above
      bool have_o = false;
      for (int e0 = 0; __any(e0 < n_cand); e0 += G) {
        const int e = e0 + sl;
        bool inS = false;
        float Ux = 0.f, Uy = 0.f, Uz = 0.f, dx = 0.f, dy = 0.f, dz = 0.f, wk = 1.f;
        if (e < n_cand) {
          const int kk = pt_off + cand[e];
          const float4 rho = a.pts[kk];
          const int lk = a.pt_link[kk];
          // r = T rho - g_b at the new joint angles, and its increment this frame
          const float4 t0 = T[lk][0], t1 = T[lk][1], t2 = T[lk][2];
          const float rx = t0.x * rho.x + t0.y * rho.y + t0.z * rho.z + t0.w - gb[0];
          const float ry = t1.x * rho.x + t1.y * rho.y + t1.z * rho.z + t1.w - gb[1];
          const float rz = t2.x * rho.x + t2.y * rho.y + t2.z * rho.z + t2.w - gb[2];
          const float ux = R1[0] * rx + R1[1] * ry + R1[2] * rz;
          const float uy = R1[3] * rx + R1[4] * ry + R1[5] * rz;
          const float uz = R1[6] * rx + R1[7] * ry + R1[8] * rz;
          const float Px = c1[0] + ux, Py = c1[1] + uy, Pz = c1[2] + uz;
          if (hf_at<BIL>(a, Px, Py) - Pz > 0.f) {
            inS = true;
            float drx = 0.f, dry = 0.f, drz = 0.f;
            if (fk_now) {
              const float4 d0 = dT[lk][0], d1 = dT[lk][1], d2 = dT[lk][2];
              drx = d0.x * rho.x + d0.y * rho.y + d0.z * rho.z + d0.w - dgb[0];
              dry = d1.x * rho.x + d1.y * rho.y + d1.z * rho.z + d1.w - dgb[1];
              drz = d2.x * rho.x + d2.y * rho.y + d2.z * rho.z + d2.w - dgb[2];
            }
            const float qx = rx - drx, qy = ry - dry, qz = rz - drz;  // r_old
            Ux = R[0] * qx + R[1] * qy + R[2] * qz;
            Uy = R[3] * qx + R[4] * qy + R[5] * qz;
            Uz = R[6] * qx + R[7] * qy + R[8] * qz;
            dx = (Eb[0] * Ux + Eb[1] * Uy + Eb[2] * Uz) + (R1[0] * drx + R1[1] * dry + R1[2] * drz) +
                 dcx;
            dy = (Eb[3] * Ux + Eb[4] * Uy + Eb[5] * Uz) + (R1[3] * drx + R1[4] * dry + R1[5] * drz) +
                 dcy;
            if constexpr (SIX)
              dz = (Eb[6] * Ux + Eb[7] * Uy + Eb[8] * Uz) +
                   (R1[6] * drx + R1[7] * dry + R1[8] * drz) + dcz;
            if (!SIX && a.fric_w) {  // the six-degree fit is not force-weighted
              // weighted by the force pressing the point at P^n, the normal
              // force of detection recomputed from the point before this
              // frame's joint update (the position P^n = c + U)
              const float dn = hf_at<BIL>(a, c[0] + Ux, c[1] + Uy) - (c[2] + Uz);
              const float vz = v[2] + (w[0] * Uy - w[1] * Ux);
              wk = dn > 0.f ? fmaxf(a.kn * dn * (1.f - a.zeta * vz), 0.f) : 0.f;
            }
          }
        }
        // the origin: U of the segment's first friction-set point
        const unsigned long long m = seg_bits<G>(__ballot(inS), seg);
        const int src = seg * G + (m ? (int)__builtin_ctzll(m) : sl);
        const float bx = __shfl(Ux, src), by = __shfl(Uy, src);
        const float bz = SIX ? __shfl(Uz, src) : 0.f;
        if (!have_o && m != 0ull) {
          ox_ = bx;
          oy_ = by;
          oz_ = bz;
          have_o = true;
        }
        if (inS) {
          const float sx = Ux - ox_, sy = Uy - oy_;
          mn += 1.f;
          Wt += wk;
          Sx += wk * sx;
          Sy += wk * sy;
          S2 += wk * (sx * sx + sy * sy);
          Dx += wk * dx;
          Dy += wk * dy;
          Cd += wk * (sx * dy - sy * dx);
          if constexpr (SIX) {
            const double ex = sx, ey = sy, ez = (double)Uz - (double)oz_;
            const double fx = dx, fy = dy, fz = dz;
            dm[0] += ex;
            dm[1] += ey;
            dm[2] += ez;
            dm[3] += fx;
            dm[4] += fy;
            dm[5] += fz;
            dm[6] += ex * ex;
            dm[7] += ey * ey;
            dm[8] += ez * ez;
            dm[9] += ex * ey;
            dm[10] += ex * ez;
            dm[11] += ey * ez;
            dm[12] += ey * fz - ez * fy;
            dm[13] += ez * fx - ex * fz;
            dm[14] += ex * fy - ey * fx;
          }
        }
      }
      if constexpr (SIX) seg_sum_nd<G>(dm);
      {
        float m7[7] = {mn, Sx, Sy, S2, Dx, Dy, Cd};
        seg_sum_n<G>(m7);
        mn = m7[0]; Sx = m7[1]; Sy = m7[2]; S2 = m7[3]; Dx = m7[4]; Dy = m7[5]; Cd = m7[6];
      }
      const float Wn = a.fric_w ? seg_sum<G>(Wt) : mn;  // total weight (count if unweighted)

      // S6 closed form of eqs. (4)-(6) and S7 static-friction cap. In these
      // moments a3 = [sum xi x delta - (Sx Dy - Sy Dx)/n] / (sum |xi|^2 - |S|^2/n),
      // a = (D + a3 J^T S)/n, the mean slip is D/n. With the force weighting
      // every sum carries the point's weight and n becomes the total weight.
      float a1 = 0.f, a2 = 0.f, a3 = 0.f, lam = 0.f;
      float az = 0.f, th6[3] = {0.f, 0.f, 0.f};  // six-degree fit: a_z and the rotation
      if (mn > 0.f && Wn > 0.f) {
        const float inv_n = rcp(Wn);
        const float D = S2 - (Sx * Sx + Sy * Sy) * inv_n;
        if (mn >= 2.f && D > Wn * a.eps * a.eps) a3 = (Cd - (Sx * Dy - Sy * Dx) * inv_n) * rcp(D);
        a1 = (Dx + Sy * a3) * inv_n + a3 * (oy_ - dcy);
        a2 = (Dy - Sx * a3) * inv_n - a3 * (ox_ - dcx);
        if constexpr (SIX) {
          // The six-degree fit (the refinement closing Sec. III-C, in 3-D), in
          // double: the rotation th = J^-1 b with J = sum (|e|^2 1 - e e^T) the
          // set's spread tensor about its centroid and b = sum e x delta the
          // slips' moment there, when J - t 1 is positive definite (its leading
          // minors, Sylvester) for t = max(n eps^2, 1e-3 tr J): a set thinner
          // than that about some axis (a leg lying on the ground) would have
          // the rotation about it set by the rounding of the slips; else the
          // ground-plane fit (yaw, or none) with the mean vertical slip. The
          // displacement at the predicted CoG: a = D/n - th x (S/n + o - dt v1).
          const double n6 = mn, in6 = 1.0 / n6;
          const double Sx6 = dm[0], Sy6 = dm[1], Sz6 = dm[2];
          const double Dx6 = dm[3], Dy6 = dm[4], Dz6 = dm[5];
          const double Qxx = dm[6] - Sx6 * Sx6 * in6, Qyy = dm[7] - Sy6 * Sy6 * in6;
          const double Qzz = dm[8] - Sz6 * Sz6 * in6, Qxy = dm[9] - Sx6 * Sy6 * in6;
          const double Qxz = dm[10] - Sx6 * Sz6 * in6, Qyz = dm[11] - Sy6 * Sz6 * in6;
          const double J00 = Qyy + Qzz, J11 = Qxx + Qzz, J22 = Qxx + Qyy;
          const double J01 = -Qxy, J02 = -Qxz, J12 = -Qyz;
          const double bx6 = dm[12] - (Sy6 * Dz6 - Sz6 * Dy6) * in6;
          const double by6 = dm[13] - (Sz6 * Dx6 - Sx6 * Dz6) * in6;
          const double bz6 = dm[14] - (Sx6 * Dy6 - Sy6 * Dx6) * in6;
          const double e2 = (double)a.eps * (double)a.eps;
          const double t = fmax(n6 * e2, (double)kSixDofCond * (J00 + J11 + J22));
          const double k00 = J00 - t, k11 = J11 - t, k22 = J22 - t;
          const double m2 = k00 * k11 - J01 * J01;
          const double m3 = k00 * (k11 * k22 - J12 * J12) - J01 * (J01 * k22 - J12 * J02) +
                            J02 * (J01 * J12 - k11 * J02);
          double t0 = 0.0, t1 = 0.0, t2 = 0.0;
          if (mn >= 3.f && k00 > 0.0 && m2 > 0.0 && m3 > 0.0) {
            const double c00 = J11 * J22 - J12 * J12, c11 = J00 * J22 - J02 * J02;
            const double c22 = J00 * J11 - J01 * J01, c01 = J02 * J12 - J01 * J22;
            const double c02 = J01 * J12 - J02 * J11, c12 = J01 * J02 - J00 * J12;
            const double id = 1.0 / (J00 * c00 + J01 * c01 + J02 * c02);
            t0 = (c00 * bx6 + c01 * by6 + c02 * bz6) * id;
            t1 = (c01 * bx6 + c11 * by6 + c12 * bz6) * id;
            t2 = (c02 * bx6 + c12 * by6 + c22 * bz6) * id;
          } else if (mn >= 2.f && J22 > n6 * e2) {
            t2 = bz6 / J22;
          }
          const double gx = Sx6 * in6 + (double)ox_ - (double)dcx;
          const double gy = Sy6 * in6 + (double)oy_ - (double)dcy;
          const double gz = Sz6 * in6 + (double)oz_ - (double)dcz;
          th6[0] = (float)t0;
          th6[1] = (float)t1;
          th6[2] = (float)t2;
          a1 = (float)(Dx6 * in6 - (t1 * gz - t2 * gy));
          a2 = (float)(Dy6 * in6 - (t2 * gx - t0 * gz));
          az = (float)(Dz6 * in6 - (t0 * gy - t1 * gx));
          Dx = (float)Dx6;
          Dy = (float)Dy6;
        }
        const float sbx = Dx * inv_n, sby = Dy * inv_n;
        const float Ff = M * __builtin_amdgcn_sqrtf(sbx * sbx + sby * sby) * (inv_dt * inv_dt);
        lam = (a.mu_inf || Ff <= a.mu * F) ? 1.f : a.mu * F * rcp(Ff);
      }

      // S8 correction and commit
      float c2[3], v2[3], w2[3], Q2[4];
      if constexpr (!SIX) {
        float alpha, sh, ch;
        if (!__any(!(fabsf(a3) < 0.1f))) {
          // |a3| < 0.1: asin from its series to float32 precision (the next term
          // is below 3e-10 relative), and the half-angle rotation |beta| < 0.06
          // from the sine and cosine series
          const float x2 = a3 * a3;
          alpha = a3 * (1.f + x2 * ((1.f / 6.f) + x2 * ((3.f / 40.f) + x2 * (5.f / 112.f))));
          const float be = -0.5f * lam * alpha, b2 = be * be;
          sh = be * (1.f - b2 * (1.f / 6.f) * (1.f - b2 * (1.f / 20.f)));
          ch = 1.f - 0.5f * b2 * (1.f - b2 * (1.f / 12.f) * (1.f - b2 * (1.f / 30.f)));
        } else {
          alpha = asinf(fminf(fmaxf(a3, -1.f), 1.f));
          sin_cos(-0.5f * lam * alpha, &sh, &ch);
        }
        Q2[0] = ch * Q1[0] - sh * Q1[3];
        Q2[1] = ch * Q1[1] - sh * Q1[2];
        Q2[2] = ch * Q1[2] + sh * Q1[1];
        Q2[3] = ch * Q1[3] + sh * Q1[0];
        // c'' = c + (dt v1 - lam a): the small trial step and correction first,
        // one rounding onto the position
        c2[0] = c[0] + (dcx - lam * a1);
        c2[1] = c[1] + (dcy - lam * a2);
        c2[2] = c1[2];
        v2[0] = v1[0] - lam * a1 * inv_dt;
        v2[1] = v1[1] - lam * a2 * inv_dt;
        v2[2] = v1[2];
        w2[0] = w1[0];
        w2[1] = w1[1];
        w2[2] = w1[2] - lam * alpha * inv_dt;
      } else {
        // back by the capped six-degree motion: displacement lam a, rotation
        // by lam asin|th| about th/|th| (|th| is the sine of the angle, as a3
        // of the yaw)
        const float s2 = th6[0] * th6[0] + th6[1] * th6[1] + th6[2] * th6[2];
        const float sn = __builtin_amdgcn_sqrtf(s2);
        const float in = sn > 0.f ? rcp(sn) : 0.f;
        float alpha, sh, ch;
        if (!__any(!(sn < 0.1f))) {
          alpha = sn * (1.f + s2 * ((1.f / 6.f) + s2 * ((3.f / 40.f) + s2 * (5.f / 112.f))));
          const float be = -0.5f * lam * alpha, b2 = be * be;
          sh = be * (1.f - b2 * (1.f / 6.f) * (1.f - b2 * (1.f / 20.f)));
          ch = 1.f - 0.5f * b2 * (1.f - b2 * (1.f / 12.f) * (1.f - b2 * (1.f / 30.f)));
        } else {
          alpha = asinf(fminf(sn, 1.f));
          sin_cos(-0.5f * lam * alpha, &sh, &ch);
        }
        const float nx = th6[0] * in, ny = th6[1] * in, nz = th6[2] * in;
        const float qx = sh * nx, qy = sh * ny, qz = sh * nz;
        Q2[0] = ch * Q1[0] - qx * Q1[1] - qy * Q1[2] - qz * Q1[3];
        Q2[1] = ch * Q1[1] + qx * Q1[0] + qy * Q1[3] - qz * Q1[2];
        Q2[2] = ch * Q1[2] - qx * Q1[3] + qy * Q1[0] + qz * Q1[1];
        Q2[3] = ch * Q1[3] + qx * Q1[2] - qy * Q1[1] + qz * Q1[0];
        c2[0] = c[0] + (dcx - lam * a1);
        c2[1] = c[1] + (dcy - lam * a2);
        c2[2] = c[2] + (dcz - lam * az);
        v2[0] = v1[0] - lam * a1 * inv_dt;
        v2[1] = v1[1] - lam * a2 * inv_dt;
        v2[2] = v1[2] - lam * az * inv_dt;
        const float ra = lam * alpha * inv_dt;
        w2[0] = w1[0] - ra * nx;
        w2[1] = w1[1] - ra * ny;
        w2[2] = w1[2] - ra * nz;
      }

      // S9 telemetry and health
      float R2[9];
      quat_to_mat(Q2[0], Q2[1], Q2[2], Q2[3], R2);
      const float ox = c2[0] - (R2[0] * gb[0] + R2[1] * gb[1] + R2[2] * gb[2]);
      const float oy = c2[1] - (R2[3] * gb[0] + R2[4] * gb[1] + R2[5] * gb[2]);
      const float oz = c2[2] - (R2[6] * gb[0] + R2[7] * gb[1] + R2[8] * gb[2]);
      const float th = oz - hf_at<BIL>(a, ox, oy);
      bool fin = true;
  #pragma unroll
      for (int i = 0; i < 3; ++i) fin = fin && isfinite(c2[i]) && isfinite(v2[i]) && isfinite(w2[i]);
  #pragma unroll
      for (int i = 0; i < 4; ++i) fin = fin && isfinite(Q2[i]);
      const float vv = v2[0] * v2[0] + v2[1] * v2[1] + v2[2] * v2[2];
      const float ww = w2[0] * w2[0] + w2[1] * w2[1] + w2[2] * w2[2];
      const int bad = (fin ? 0 : 1) | ((vv > 2500.f || ww > 250000.f) ? 2 : 0);

      if (active) {
  #pragma unroll
        for (int i = 0; i < 3; ++i) {
          c[i] = c2[i];
          v[i] = v2[i];
          w[i] = w2[i];
        }
  #pragma unroll
        for (int i = 0; i < 4; ++i) Q[i] = Q2[i];
  #pragma unroll
        for (int i = 0; i < 9; ++i) Rq[i] = R2[i];
        tele[0] += (double)th;
        tele[1] += (double)nc;
        tele[2] += (mn > 0.f && Wn > 0.f && lam < 1.f) ? 1.0 : 0.0;
        fl = bad;
        n += 1;
      }
    }
    if (MODE != kStep || s == a.n_steps) break;
    const bool active = valid && fl == 0;
    const float* R = Rq;

    // S1 + S2: detection at P^n and normal forces.
    // Broad phase: a link whose box of points lies wholly above the highest
    // entry of the height map has no point in contact, so its points are not
    // tested (they would add exactly nothing); a point slot no lane of the
    // wave needs is skipped as a whole. The box's lowest world height is its
    // centre's minus sum_j |w_j| e_j, w = the world z row of the link's axes.
    // The verdicts go round the wave as ballots, one bit per link lane.
    unsigned long long tmask[LPL];
#pragma unroll
    for (int l = 0; l < LPL; ++l) {
      const int li = sl + l * G;
      bool tl = false;
      if (lv[l]) {
        const float4 r0 = T[li][0], r1 = T[li][1], r2 = T[li][2];
        const float4 b0 = LK[li].box0, b1 = LK[li].I1_box;
        const float bx[6] = {b0.x, b0.y, b0.z, b0.w, b1.z, b1.w};
        const float y0 = r0.x * bx[0] + r0.y * bx[1] + r0.z * bx[2] + r0.w - gb[0];
        const float y1 = r1.x * bx[0] + r1.y * bx[1] + r1.z * bx[2] + r1.w - gb[1];
        const float y2 = r2.x * bx[0] + r2.y * bx[1] + r2.z * bx[2] + r2.w - gb[2];
        const float zc = c[2] + (R[6] * y0 + R[7] * y1 + R[8] * y2);
        const float wx = R[6] * r0.x + R[7] * r1.x + R[8] * r2.x;
        const float wy = R[6] * r0.y + R[7] * r1.y + R[8] * r2.y;
        const float wz = R[6] * r0.z + R[7] * r1.z + R[8] * r2.z;
        const float ez = fabsf(wx) * bx[3] + fabsf(wy) * bx[4] + fabsf(wz) * bx[5];
        tl = zc - ez <= a.hf_max + 1e-3f;
      }
      tmask[l] = __ballot(tl);
    }
    // the slots past the first NRC that some lane must test (bit p: slot p)
    unsigned act;
    {
      unsigned meet = 0u;
#pragma unroll
      for (int l = 0; l < LPL; ++l) meet |= (unsigned)(hi_half ? tmask[l] >> 32 : tmask[l]) & smask[l];
      const unsigned long long b = __ballot(meet != 0u);
      act = (unsigned)b | (unsigned)(b >> 32);
    }
    // whether link lk of this lane's robot may touch: its lane's bit
    auto touches = [&](int lk) __attribute__((always_inline)) {
      const int l = LPL == 1 ? 0 : lk / G;
      unsigned long long m = tmask[0];
#pragma unroll
      for (int q = 1; q < LPL; ++q) m = l == q ? tmask[q] : m;
      return ((m >> (seg * G + (lk - l * G))) & 1ull) != 0ull;
    };
    kap = 0u;
    kap_slots = 0u;
    F = 0.f;
    tx = 0.f;
    ty = 0.f;
    nc = 0.f;
    // The first NRC slots (the leaf links' points, whose points are in
    // registers) are tested without branches: every lane's point is placed
    // and looked up, and only those of links that may touch count. Their
    // look-ups then travel together instead of one guarded chain per slot.
    {
      float dd[NRC], uxs[NRC], uys[NRC];
      bool need[NRC];
#pragma unroll
      for (int p = 0; p < NRC; ++p) {
        const int lk = (int)((plk[p / 5] >> (6 * (p % 5))) & 63u);
        need[p] = sl + p * G < N && touches(lk);
        const float4 r0 = T[lk][0], r1 = T[lk][1], r2 = T[lk][2];
        const float rx = r0.x * rc[p][0] + r0.y * rc[p][1] + r0.z * rc[p][2] + r0.w - gb[0];
        const float ry = r1.x * rc[p][0] + r1.y * rc[p][1] + r1.z * rc[p][2] + r1.w - gb[1];
        const float rz = r2.x * rc[p][0] + r2.y * rc[p][1] + r2.z * rc[p][2] + r2.w - gb[2];
        const float ux = R[0] * rx + R[1] * ry + R[2] * rz;
        const float uy = R[3] * rx + R[4] * ry + R[5] * rz;
        const float uz = R[6] * rx + R[7] * ry + R[8] * rz;
        const float Px = c[0] + ux, Py = c[1] + uy, Pz = c[2] + uz;
        dd[p] = hf_at<BIL>(a, Px, Py) - Pz;
        uxs[p] = ux;
        uys[p] = uy;
      }
#pragma unroll
      for (int p = 0; p < NRC; ++p) {
        const bool hit = need[p] && dd[p] > 0.f;
        if (hit) {
          kap |= 1u << p;
          const float vz = v[2] + (w[0] * uys[p] - w[1] * uxs[p]);
          const float f = fmaxf(a.kn * dd[p] * (1.f - a.zeta * vz), 0.f);
          F += f;
          tx += uys[p] * f;
          ty -= uxs[p] * f;
          nc += 1.f;
        }
        if (__ballot(hit) != 0ull) kap_slots |= 1u << p;
      }
    }
#pragma unroll
    for (int p = NRC; p < PPL; ++p) {
      if (!((act >> p) & 1u)) continue;
      const int k = sl + p * G;
      const bool ok = k < N;
      const int kk = pt_off + (ok ? k : 0);
      const int lk = (int)((plk[p / 5] >> (6 * (p % 5))) & 63u);
      bool hit = false;
      if (ok && touches(lk)) {
        const float4 rho = a.pts[kk];
        const float4 r0 = T[lk][0], r1 = T[lk][1], r2 = T[lk][2];
        const float rx = r0.x * rho.x + r0.y * rho.y + r0.z * rho.z + r0.w - gb[0];
        const float ry = r1.x * rho.x + r1.y * rho.y + r1.z * rho.z + r1.w - gb[1];
        const float rz = r2.x * rho.x + r2.y * rho.y + r2.z * rho.z + r2.w - gb[2];
        const float ux = R[0] * rx + R[1] * ry + R[2] * rz;
        const float uy = R[3] * rx + R[4] * ry + R[5] * rz;
        const float uz = R[6] * rx + R[7] * ry + R[8] * rz;
        const float Px = c[0] + ux, Py = c[1] + uy, Pz = c[2] + uz;
        const float d = hf_at<BIL>(a, Px, Py) - Pz;
        if (d > 0.f) {
          hit = true;
          kap |= 1u << p;
          const float vz = v[2] + (w[0] * uy - w[1] * ux);
          const float f = fmaxf(a.kn * d * (1.f - a.zeta * vz), 0.f);
          F += f;
          tx += uy * f;
          ty -= ux * f;
          nc += 1.f;
        }
      }
      if (__ballot(hit) != 0ull) kap_slots |= 1u << p;
      group_fence(p);
    }
    {
      float f4[4] = {F, tx, ty, nc};
      seg_sum_n<G>(f4);
      F = f4[0]; tx = f4[1]; ty = f4[2]; nc = f4[3];
    }

    // S3: joint-angle determination every K frames (c, Q, v, w kept)
    const bool upd = (n % a.K) == 0;
    fk_now = __any(upd);
    if (fk_now) {
      const bool take = upd && active;
#pragma unroll
      for (int l = 0; l < LPL; ++l) {
        float qn = command(l);
        // motors' speed: at most rate K dt towards the command per update
        if (a.rate_step > 0.f) qn = fminf(fmaxf(qn, q[l] - a.rate_step), q[l] + a.rate_step);
        dql[l] = take ? qn - q[l] : 0.f;
        qp[l] = take ? q[l] : qp[l];
        q[l] = take ? qn : q[l];
      }
      fk_pending = true;
    }
  }

  if (MODE == kPlace) {
    float R[9];
    quat_to_mat(Q[0], Q[1], Q[2], Q[3], R);
#pragma unroll
    for (int i = 0; i < 3; ++i) c[i] += R[3 * i] * gb[0] + R[3 * i + 1] * gb[1] + R[3 * i + 2] * gb[2];
  }

  if (MODE == kPoints) {
    float R[9];
    quat_to_mat(Q[0], Q[1], Q[2], Q[3], R);
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
      const int k = sl + p * G;
      float r[3];
      if (body_point(k, r) && valid) {
        float* o = a.points_out + ((size_t)inst * a.n_max + a.pt_orig[pt_off + k]) * 3;
        o[0] = c[0] + (R[0] * r[0] + R[1] * r[1] + R[2] * r[2]);
        o[1] = c[1] + (R[3] * r[0] + R[4] * r[1] + R[5] * r[2]);
        o[2] = c[2] + (R[6] * r[0] + R[7] * r[1] + R[8] * r[2]);
      }
    }
  }

  // ---- write back
  if (valid && MODE != kPoints) {
    // The addresses are formed here from fresh copies of the state pointers
    // and the instance index: formed once in the prologue and kept, they
    // would be held (spilled) through the whole launch.
    float* so = a.st;
    int* sp = a.step;
    int* fp = a.flags;
    double* tp = a.tele;
    int iw = inst;
    asm volatile("" : "+s"(so), "+s"(sp), "+s"(fp), "+s"(tp));
    asm volatile("" : "+v"(iw));
    if (sl == 0) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        so[(size_t)i * I + iw] = c[i];
        so[(size_t)(7 + i) * I + iw] = v[i];
        so[(size_t)(10 + i) * I + iw] = w[i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) so[(size_t)(3 + i) * I + iw] = Q[i];
      sp[iw] = n;
      fp[iw] = fl;
#pragma unroll
      for (int i = 0; i < TELE_N; ++i) tp[(size_t)i * I + iw] = tele[i];
    }
#pragma unroll
    for (int l = 0; l < LPL; ++l) {
      const int li = sl + l * G;
      if (lj[l]) {
        so[(size_t)(BODY_ROWS + li - 1) * I + iw] = q[l];
        so[(size_t)(BODY_ROWS + a.j_max + li - 1) * I + iw] = qp[l];
      }
    }
  }
}

// Residency: capping the registers at 256 (two waves per SIMD) for the
// one-link-per-lane shapes of a 64-lane segment with at most 6 points per lane
// and of a 32-lane segment with at most 12 points per lane keeps two waves
// resident to hide gather, LDS and DPP latency; with the body points rebuilt
// from LDS these shapes fit the cap with few or no spills (on 4,096 hexapods
// the 32-lane shape went from 16.6 to 9.1 us per frame with the cap). Larger
// shapes would spill badly under the cap and keep the compiler's choice.
template <int G, int PPL, int LPL>
constexpr int kMinWavesPerEU = ((G == 64 && PPL <= 6) || (G == 32 && PPL <= 12 && LPL == 1)) ? 2 : 1;

template <int G, int PPL, int LPL, int MODE, bool BIL = false, bool SIX = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kMinWavesPerEU<G, PPL, LPL>, 8)))
void step_kernel(const StepArgs a) {
  constexpr int IPW = 64 / G;
  constexpr int LMAX = G * LPL;
  __shared__ LinkT T[IPW][LMAX];
  __shared__ LinkT dT[IPW][LMAX];
  __shared__ int cand[IPW][G * PPL];  // contact points of a frame, compacted
  __shared__ LinkConst LK[IPW][LMAX]; // constants of every link of the robot
  const int lane = threadIdx.x;
  const int seg = lane / G;
  const int sl = lane - seg * G;
  for (int it = 0;; ++it) {
    int tb;
    if (a.queue) {
      int v = 0;
      if (lane == 0) v = atomicAdd(a.queue, 1);
      tb = __builtin_amdgcn_readfirstlane(v);
    } else {
      if (it > 0) break;
      // Workgroups go to the chip's XCDs in turn (workgroup b to XCD b mod 8),
      // and each XCD has its own L2. Block b takes the (b / 8)-th task block of
      // a contiguous share of its XCD, so the robots of one XCD are adjacent
      // in the struct-of-arrays state: a cache line of a state row is read
      // and written by one L2 instead of partly by each of eight. Any grid
      // size maps one-to-one.
      const int nb = (int)gridDim.x, x = (int)(blockIdx.x % kXcds);
      const int q = nb / (int)kXcds, r = nb % (int)kXcds;
      tb = x * q + (x < r ? x : r) + (int)(blockIdx.x / kXcds);
    }
    if (tb >= a.n_blocks) break;
    run_block<G, PPL, LPL, MODE, BIL, SIX>(a, T[seg], dT[seg], cand[seg], LK[seg], tb,
                                      seg, sl);
    __syncthreads();
  }
}

__global__ void zero_kernel(int* p) { *p = 0; }

__global__ void zero_n_kernel(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace

// The built shapes: (G, PPL, LPL).
#define NPX_SHAPES(X)                                                                  \
  X(64, 2, 1) X(64, 4, 1) X(64, 6, 1) X(64, 8, 1) X(64, 10, 1) X(64, 12, 1) X(64, 16, 1) \
  X(32, 4, 1) X(32, 8, 1) X(32, 12, 1) X(32, 12, 2) X(32, 16, 2) X(32, 20, 2)           \
  X(16, 8, 2) X(16, 16, 2) X(16, 24, 2) X(16, 24, 3)

bool pick_shape(int G, int n_max, int l_max, Shape* out) {
  bool found = false;
  Shape best{0, 1 << 30, 1 << 30};
#define NPX_PICK(g, ppl, lpl)                                                          \
  if (g == G && g * ppl >= n_max && g * lpl >= l_max &&                                \
      (ppl < best.PPL || (ppl == best.PPL && lpl < best.LPL))) {                       \
    best = Shape{g, ppl, lpl};                                                         \
    found = true;                                                                      \
  }
  NPX_SHAPES(NPX_PICK)
#undef NPX_PICK
  if (found) *out = best;
  return found;
}

hipError_t launch_step(const StepArgs& a, const Shape& s, int grid, hipStream_t stream) {
#define NPX_LAUNCH(g, ppl, lpl)                                                        \
  if (s.G == g && s.PPL == ppl && s.LPL == lpl) {                                      \
    if (a.place)                                                                       \
      hipLaunchKernelGGL((step_kernel<g, ppl, lpl, kPlace>), dim3(grid), dim3(64), 0,   \
                         stream, a);                                                   \
    else if (a.points_out)                                                             \
      hipLaunchKernelGGL((step_kernel<g, ppl, lpl, kPoints>), dim3(grid), dim3(64), 0,  \
                         stream, a);                                                   \
    else if (a.hf_bilinear && a.fric6)                                                 \
      hipLaunchKernelGGL((step_kernel<g, ppl, lpl, kStep, true, true>), dim3(grid),     \
                         dim3(64), 0, stream, a);                                      \
    else if (a.fric6)                                                                  \
      hipLaunchKernelGGL((step_kernel<g, ppl, lpl, kStep, false, true>), dim3(grid),    \
                         dim3(64), 0, stream, a);                                      \
    else if (a.hf_bilinear)                                                            \
      hipLaunchKernelGGL((step_kernel<g, ppl, lpl, kStep, true>), dim3(grid), dim3(64), 0, \
                         stream, a);                                                   \
    else                                                                               \
      hipLaunchKernelGGL((step_kernel<g, ppl, lpl, kStep>), dim3(grid), dim3(64), 0,    \
                         stream, a);                                                   \
    return hipGetLastError();                                                          \
  }
  NPX_SHAPES(NPX_LAUNCH)
#undef NPX_LAUNCH
  return hipErrorInvalidValue;
}

int resident_blocks_per_cu(const Shape& s) {
  int nb = 0;
#define NPX_OCC(g, ppl, lpl)                                                           \
  if (s.G == g && s.PPL == ppl && s.LPL == lpl)                                        \
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_kernel<g, ppl, lpl, kStep>, 64, 0);
  NPX_SHAPES(NPX_OCC)
#undef NPX_OCC
  return nb;
}

hipError_t launch_zero(int* p, hipStream_t stream) {
  hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(1), 0, stream, p);
  return hipGetLastError();
}

hipError_t launch_zero_n(int* p, int n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_n_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

}  // namespace npx
