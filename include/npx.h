/*
 * npx.h -- C ABI of the MI355X-native batched legged-robot step of NeoPhysIx
 * (Fischer & Ihme, arXiv 2411.05799).
 *
 * A robot is a set of mass points grouped into rigid links joined by hinges
 * (Sec. III-A, IV-A/B). Many robots ("instances") are stepped together on one
 * GPU; each step is the paper's frame: point-cloud collision against a
 * height-map look-up table (Sec. III-A), kinematic joint-angle determination
 * (Sec. III-B), friction estimated by least squares of the contact-point
 * motion (Sec. III-C, eqs. 1-6) capped by the maximum static friction, and
 * integration. The user's move() of Fig. 1 becomes controller data.
 *
 * Conventions for every entry point:
 *  - SI units, z up, right-hand rule for hinge angles, quaternions (w,x,y,z).
 *  - Every call returns npx_status (NPX_OK = 0); on failure npx_last_error()
 *    holds a thread-local message. No exception crosses the ABI.
 *  - Host pointers are only read during the call; the world copies what it
 *    needs. Device pointers (the *_on_device flags) must be HIP device memory
 *    of the world's device and stay valid only for the call.
 *  - Per-instance fields are struct-of-arrays: component-major [comp][I].
 *  - npx_step_n is asynchronous on the given HIP stream; npx_read_state and
 *    npx_write_state first synchronise the stream of the last npx_step_n.
 *    Kernel faults surface as NPX_EHIP at the next synchronising call.
 *  - Numerical blow-ups are not errors: the instance is flagged (field
 *    NPX_F_FLAGS) and frozen, the others continue.
 */
#ifndef NPX_H
#define NPX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NPX_OK = 0,
  NPX_EINVAL = -1,       /* bad argument or inconsistent tables */
  NPX_ENOMEM = -2,       /* device or host allocation failed */
  NPX_EHIP = -3,         /* a HIP runtime call or kernel failed */
  NPX_ESTATE = -4,       /* call not valid in the object's current state */
  NPX_EUNSUPPORTED = -5  /* shape beyond what the kernels are built for */
} npx_status;

#define NPX_MAX_JOINTS 63    /* links per robot <= 64 */
#define NPX_MAX_POINTS 1024  /* mass points per robot */

const char* npx_last_error(void);
int npx_version(void);

/* ---------------------------------------------------------------------- */
/* Morphology tables (the finalised robot of Sec. IV, construction frame) */
/* ---------------------------------------------------------------------- */
/* points  [n_points][4]: x, y, z (construction frame = torso frame at the zero
 *         pose) and mass of each mass point (Sec. III-A).
 * pt_link [n_points]: link that owns the point; link 0 is the torso.
 * parent  [n_links]: parent link, parent[0] = -1, parent[l] < l.
 * joint   [n_links][8]: hinge of link l (createJoint, Sec. IV-B / Appendix):
 *         anchor xyz and axis xyz in the construction frame, then the lower
 *         and upper limit in rad (|limit| >= 1e30 means none). Row 0 unused.
 *         Joint j drives link j+1; J = n_links - 1. */
typedef struct {
  int32_t n_points;
  int32_t n_links;
  const float* points;
  const int32_t* pt_link;
  const int32_t* parent;
  const float* joint;
} npx_morph_tables;

/* ---------------------------------------------------------------------- */
/* Construction API of the paper (Sec. IV, appendix) -> morphology tables  */
/* ---------------------------------------------------------------------- */
/* Host only; nothing touches a device. Body-creating calls return the new
 * body id (>= 0) or a negative npx_status; npx_morph_last_error() explains a
 * failure. Bodies are made of mass points with the body's mass spread evenly
 * (Sec. III-A); each has a reference point (point: its position; box, sphere:
 * centre; cylinder: axis midpoint; ray: start) and an orientation. The morph
 * object owns everything it returns; npx_morph_get_tables views stay valid until
 * npx_morph_free. Calls that change a finalised morph return NPX_ESTATE. */
typedef struct npx_morph npx_morph;
npx_status npx_morph_new(npx_morph** out);
void npx_morph_free(npx_morph* m); /* NULL-safe */
const char* npx_morph_last_error(void);
/* simplifyMode (Sec. IV-C): for cylinders and spheres created afterwards,
 * 0 none, 1 the 8 corners of their bounding box, 2 two points, >= 3 one point. */
npx_status npx_simplify_mode(npx_morph* m, int mode);
int npx_create_point(npx_morph* m, double x, double y, double z, double mass);
/* 8 corner points; w along x, h along z, d along y, centre (x, y, z). */
int npx_create_box(npx_morph* m, double w, double h, double d, double x, double y, double z,
                   double mass);
/* The same box with its two faces normal to z (bottom and top) each carrying a
 * grid_nx x grid_ny lattice of points that spans the face, corners included
 * (2 * grid_nx * grid_ny points, the mass spread equally). Contact is found at
 * mass points only (Sec. III-A), so a box resting on uneven ground with its 8
 * corners alone is held at the corners; the lattice lets the face between them
 * touch. grid 0, 0 is npx_create_box; otherwise both counts must lie in
 * [2, 64] (else NPX_EINVAL). Returns the body id or a negative status. */
int npx_create_box_grid(npx_morph* m, double w, double h, double d, double x, double y, double z,
                        double mass, int grid_nx, int grid_ny);
/* ring_pts points on each end cap ring of radius rr (mode 0). */
int npx_create_cylinder(npx_morph* m, double x1, double y1, double z1, double x2, double y2,
                        double z2, double rr, double mass, int ring_pts);
/* the 12 vertices of a regular icosahedron of radius rr (mode 0). */
int npx_create_sphere(npx_morph* m, double x, double y, double z, double rr, double mass);
/* no mass points; never collides. Glued (npx_connect_bodies) to a body of a
 * link, it becomes that link's range sensor (npx_world_ray_ranges). */
int npx_create_ray(npx_morph* m, double x1, double y1, double z1, double x2, double y2, double z2);
/* connectBodies: glue two bodies into one rigid link. */
npx_status npx_connect_bodies(npx_morph* m, int id1, int id2);
/* createJoint: hinge; anchor and axis in body 1's frame; body 1's link is the
 * parent, body 2's the child. Returns the joint id. */
int npx_create_joint(npx_morph* m, int id1, int id2, double anX, double anY, double anZ,
                     double aX, double aY, double aZ);
/* range of motion of a joint (default unlimited). */
npx_status npx_set_joint_limits(npx_morph* m, int joint, double lo, double hi);
/* moveBody: put the body's reference point at (tx, ty, tz). */
npx_status npx_move_body(npx_morph* m, int id, double tx, double ty, double tz);
/* rotateBody: roll alpha about x, then pitch beta about y, then yaw gamma about
 * z (fixed construction axes, right-hand rule), about the reference point. */
npx_status npx_rotate_body(npx_morph* m, int id, double alpha, double beta, double gamma);
/* getMaxBodyID: the number of body ids handed out. */
int npx_get_max_body_id(const npx_morph* m);
/* finalizeConstruction: links = glued groups, root = the link of body 0, links
 * ordered parents first; fails on a joint inside a link, a link with two
 * parent joints or a body not reachable from the root. */
npx_status npx_finalize_construction(npx_morph* m);
npx_status npx_morph_get_tables(const npx_morph* m, npx_morph_tables* out);
/* The finalised morph's range-sensor rays (Sec. IV, createRay): those glued
 * to a link, in creation order. rays [n][6]: start then end point in the
 * construction frame (the frame of the tables' points, after the bodies'
 * moves and rotations); ray_link [n]: the link each rides on. Views owned by
 * the morph, valid until npx_morph_free; NPX_ESTATE before finalisation. */
npx_status npx_morph_get_rays(const npx_morph* m, int32_t* n_rays, const float** rays,
                              const int32_t** ray_link);
/* index of a joint id in the tables' joint order (the controller's order). */
int npx_morph_joint_index(const npx_morph* m, int joint_id);

/* ---------------------------------------------------------------------- */
/* World: instances, terrain, physical constants                          */
/* ---------------------------------------------------------------------- */
typedef struct {
  double dt;              /* frame length, s (> 0) */
  int32_t joint_interval; /* joints are set every K frames (Sec. III-B), K >= 1 */
  double g[3];            /* gravity */
  double mu;              /* friction coefficient; +inf = pure stick */
  double k_n;             /* normal penalty stiffness per contact point, N/m */
  double zeta;            /* Hunt-Crossley damping, s/m */
  double eps_lsq;         /* rotation is fitted only if the contact spread > eps, m */
  /* height-map look-up table (Sec. III-A): cell (i, j) covers
   * [x0 + i/s, x0 + (i+1)/s) x [y0 + j/s, y0 + (j+1)/s); outside clamps. */
  int32_t hf_nx, hf_ny;
  double hf_s, hf_x0, hf_y0;
  const float* hf_heights; /* host [hf_ny][hf_nx] */
  int64_t n_instances;
  int32_t n_morphs;
  const npx_morph_tables* morphs;  /* host [n_morphs] */
  const int32_t* instance_morph;   /* host [n_instances] */
  const float* init_pose;          /* host [n_instances][7]: torso-origin xyz, quaternion;
                                      the robot starts at rest with q = q_cmd(0) and its
                                      CoG where that pose puts it */
  const float* ctrl;               /* host [n_instances][J_max][3] sinusoid controller
                                      (see npx_set_controller), J_max = max(1, max
                                      n_links - 1); NULL = all zero */
  int32_t friction_weighting;      /* 0: the friction fit of eqs. (4)-(6) as printed;
                                      1: every point's terms weighted by the normal
                                      force pressing it at the frame's start (the
                                      refinement closing Sec. III-C); other values
                                      are rejected */
  int32_t hf_bilinear;             /* 0: the height map as the paper's look-up table;
                                      1: its entries are heights at the cell centres,
                                      read bilinearly between the four around (held
                                      beyond the outer centres); other values are
                                      rejected */
  double max_joint_rate;           /* rad/s a joint may turn (the motors' speed,
                                      Sec. III-B): each joint update moves a joint
                                      from its angle towards its command by at most
                                      max_joint_rate K dt; 0 or +inf: no limit;
                                      negative or NaN: rejected */
  int32_t friction_6dof;           /* 0: the friction fit in the ground plane
                                      (eqs. (4)-(6): displacement and yaw);
                                      1: the fit over the full rigid motion in
                                      3-D (rotations about the other two axes
                                      as well, the refinement closing Sec.
                                      III-C): displacement and rotation vector
                                      of the contact points from P^n to P*, the
                                      ground-plane fit with the mean vertical
                                      slip when the set's spread is too small to
                                      fix a 3-D rotation; the robot is moved
                                      back by the whole fitted motion under the
                                      same static-friction cap; other values,
                                      and 1 together with friction_weighting
                                      (when the force sits on points along one
                                      line, a point of near-zero force would
                                      decide the roll about it), are rejected */
  void* ext_device_buffers[4];     /* optional caller-owned device memory (a torch
                                      tensor's storage, say) that holds the world's
                                      state in place of its own allocation, so the
                                      caller reads it with no copy; a NULL entry is
                                      allocated by the world:
                                      [0] float [13 + 2 J_max][n_instances]: CoG,
                                          quaternion, velocity, angular velocity,
                                          joint angles, joint angles before the last
                                          update (NPX_F_BODY, NPX_F_JOINT,
                                          NPX_F_JOINT_PREV one after the other);
                                      [1] int32 [n_instances] frame counters;
                                      [2] int32 [n_instances] health flags;
                                      [3] double [4][n_instances] telemetry sums.
                                      Each must be device memory of the current
                                      device, 16-byte aligned, inside one
                                      allocation that holds the bytes named (else
                                      NPX_EINVAL). The caller keeps it alive and
                                      unmoved until npx_destroy_world, which does
                                      not free it. npx_create_world writes the
                                      start state into it; after an npx_step_n has
                                      completed on its stream it holds that state. */
} npx_world_desc;

typedef struct npx_world npx_world;

/* Creates a world on the current HIP device; copies every host input. */
npx_status npx_create_world(const npx_world_desc* desc, npx_world** out);

/* NULL-safe. Waits for the world's pending work, then frees it. */
void npx_destroy_world(npx_world* w);

/* Sizes: instances, joint stride J_max (max joints over morphologies) and
 * N_max (max points). Any pointer may be NULL. */
npx_status npx_world_dims(const npx_world* w, int64_t* n_instances, int32_t* j_max,
                          int32_t* n_max);

/* Controller (the user's move() of Fig. 1, as data). Replaces the parameters
 * for the frames that follow; the state is not touched.
 * kind NPX_CTRL_SINUSOID: params [n_instances][J_max][3] = (A, f, phi): joint j
 * is commanded A sin(2 pi f t + phi) rad at t = n dt, clamped to its limits.
 * n_floats must equal n_instances * J_max * 3. */
#define NPX_CTRL_SINUSOID 0
/* kind NPX_CTRL_TARGETS: params [n_instances][J_max] = joint target angles
 * (rad), commanded from the next joint update on, clamped to the limits (held
 * as the sinusoid rows (target, 0, pi/2)). n_floats = n_instances * J_max. */
#define NPX_CTRL_TARGETS 1
npx_status npx_set_controller(npx_world* w, int kind, const float* params, size_t n_floats,
                              int params_on_device);

/* Advances every instance by n frames (n >= 0), asynchronously on hip_stream
 * (a hipStream_t; NULL = default stream). */
npx_status npx_step_n(npx_world* w, int64_t n, void* hip_stream);

/* npx_step_n for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same frames, bit for bit, for the world's launch settings, with no
 * allocation of any kind. Chunks of launch.chunk_steps frames are launched
 * directly (no graph is instantiated); in persistent mode their task-queue
 * counters, one per chunk, are a static device array of NPX_NOALLOC_MAX_CHUNKS
 * ints that every GPU holds until the process ends, cleared by a fill kernel
 * at the start of each call. All calls on one GPU share that array: calls
 * that overlap on one GPU (concurrent streams, threads) race. Returns
 * NPX_EINVAL when n needs more than NPX_NOALLOC_MAX_CHUNKS chunk launches
 * (nothing is launched then), NPX_EHIP on a launch error. */
#define NPX_NOALLOC_MAX_CHUNKS 4096
npx_status npx_step_n_noalloc(npx_world* w, int64_t n, void* hip_stream);

/* State fields, SoA [comp][n_instances]. */
enum {
  NPX_F_COG = 0,        /* float [3][I]  world centre of gravity */
  NPX_F_QUAT = 1,       /* float [4][I]  torso orientation (w,x,y,z) */
  NPX_F_VEL = 2,        /* float [3][I]  CoG velocity */
  NPX_F_OMEGA = 3,      /* float [3][I]  angular velocity, world frame */
  NPX_F_JOINT = 4,      /* float [J_max][I] applied joint angles */
  NPX_F_JOINT_PREV = 5, /* float [J_max][I] joint angles before the last update */
  NPX_F_STEP = 6,       /* int32 [I] frame counter n (t = n dt) */
  NPX_F_FLAGS = 7,      /* int32 [I] health flags, non-zero = frozen */
  NPX_F_TELE = 8,       /* double [4][I] telemetry sums: torso height above the
                           cell under it, contact points, slipping frames, 0 */
  NPX_F_BODY = 9        /* float [13][I] COG, QUAT, VEL, OMEGA in one block */
};
#define NPX_FLAG_NONFINITE 1
#define NPX_FLAG_SPEED 2 /* |v| > 50 m/s or |omega| > 500 rad/s */

/* Copies a field to dst (bytes must equal the field size). Synchronous. */
npx_status npx_read_state(npx_world* w, int field, void* dst, size_t bytes, int dst_on_device);
/* Overwrites a field from src (bytes must equal the field size). Synchronous.
 * Used for checkpoint/resume and to start parity windows from given states. */
npx_status npx_write_state(npx_world* w, int field, const void* src, size_t bytes,
                           int src_on_device);

/* World positions of every mass point at the current state, computed by the
 * step's own transform path: float [n_instances][N_max][3] (rows past an
 * instance's point count are zero). Synchronous. */
npx_status npx_read_points(npx_world* w, float* dst, size_t bytes, int dst_on_device);

/* ---------------------------------------------------------------------- */
/* Range sensors: the rays of the construction API (Sec. IV, createRay)    */
/* ---------------------------------------------------------------------- */
/* Sets the rays of every instance of morphology `morph` (replacing earlier
 * ones). rays: host [n_rays][6], start then end point in that morphology's
 * construction frame (the frame of its table points, as npx_morph_get_rays
 * lists them); ray_link: host [n_rays], the link each rides on, in
 * [0, n_links). 0 <= n_rays <= 64 (0 removes them). A ray may cross at most
 * 65,536 cells of the height map (s sqrt(2) length + 4 <= 65,536), else
 * NPX_EINVAL. Copies the tables; synchronous (waits for the device). */
npx_status npx_world_set_rays(npx_world* w, int32_t morph, int32_t n_rays, const float* rays,
                              const int32_t* ray_link);
/* Range of every ray at the current state, asynchronously on hip_stream:
 * dst device float [n_instances][ld], ld >= the largest ray count of any
 * morphology (and >= 1). A ray rides on its link like a massless point: an
 * end p is at c + R(Q)(T_link p - g_b), the transform of the mass points
 * (Sec. III-A, III-B). dst[i][k] = the distance from ray k's start to the
 * first point of the segment that is at or below the ground, the ground
 * being the step's look-up table (Sec. III-A: the height of the cell a
 * point's floor indices name, clamped to the map); 0 when the start is at or
 * below it; the ray's length when no point is. NaN for a non-finite state.
 * Entries past an instance's own ray count are not written. NPX_EINVAL for a
 * world that reads its map bilinearly or for ld too small. */
npx_status npx_world_ray_ranges(npx_world* w, float* dst, int64_t ld, void* hip_stream);

/* ---------------------------------------------------------------------- */
/* Machine-code controller (Sec. V, the interpreter's command table)       */
/* ---------------------------------------------------------------------- */
/* Foot contact sensors of morphology `morph`: sensor s reads 1 when any mass
 * point of link links[s] is in contact (strictly below the ground, the step's
 * own test), else 0; sensor numbers past n read 0. links: host [n], each in
 * [0, n_links); 0 <= n <= 32. Synchronous. */
npx_status npx_world_set_sensors(npx_world* w, int32_t morph, int32_t n, const int32_t* links);
/* Runs every instance's machine-code program for n_updates joint updates:
 * each update reads the foot sensors at the current state, executes n_instr
 * instructions, writes the joint targets as the controller's commands
 * (A = target, f = 0, phi = pi/2, replacing npx_set_controller's parameters)
 * and advances the world by K frames; asynchronous on hip_stream.
 * programs: device uint8 [n_instances][32]. Byte = 3-bit command, 5-bit
 * argument: 0 move motor (joint) arg left, 1 right (target -/+ motor_step rad,
 * held within the joint's limits; arg >= J does nothing), 2 accumulator =
 * sensor arg, 3 accumulator = arg, 4 jump to address arg if the accumulator is
 * non-zero, 5 accumulator = NOT accumulator, 6 increment, 7 decrement (8 bits,
 * wrapping); the program counter wraps from 31 to 0.
 * vm: device int32 [n_instances][2] (program counter, accumulator), read and
 * written, carried between calls. targets: device float [n_instances][ld],
 * ld >= J_max, read and written. 0 <= n_instr <= 4096; motor_step finite,
 * >= 0. */
npx_status npx_gp_run(npx_world* w, const uint8_t* programs, int32_t* vm, float* targets,
                      int64_t ld_targets, int32_t n_updates, int32_t n_instr, float motor_step,
                      void* hip_stream);

/* ---------------------------------------------------------------------- */
/* Launch shape (chosen by the autotuner or set by hand)                   */
/* ---------------------------------------------------------------------- */
typedef struct {
  int32_t lanes_per_instance; /* 16, 32 or 64 lanes of a wave per robot */
  int32_t persistent;         /* 1: resident grid pulling tasks from a queue */
  int32_t chunk_steps;        /* frames per kernel launch (state stays in registers) */
  int32_t use_graph;          /* 1: replay the launches of a persistent chunk (queue
                                 reset, then the step) from cached hipGraphs; a chunk
                                 of one kernel is always launched directly */
  int32_t waves_per_cu;       /* resident waves per CU in persistent mode */
} npx_launch;

npx_status npx_get_launch(const npx_world* w, npx_launch* out);
/* Rejects shapes the kernels are not built for with NPX_EUNSUPPORTED. */
npx_status npx_set_launch(npx_world* w, const npx_launch* cfg);

/* Times `steps` frames of each candidate launch shape on a scratch copy of the
 * state (the world's state is untouched), applies the fastest and writes it to
 * best; a persistent shape counts as fastest only when it is more than 3%
 * faster than every direct one. times_ms (may be NULL) receives one time per
 * candidate tried, at most max_results; n_tried receives the count. */
npx_status npx_autotune(npx_world* w, int32_t steps, void* hip_stream, npx_launch* best,
                        npx_launch* tried, float* times_ms, int32_t max_results,
                        int32_t* n_tried);

/* Algorithmic FP32 operations of one frame of instance i, counted from the
 * step's formulas (the roofline numerator). */
npx_status npx_flops_per_step(const npx_world* w, int64_t i, double* flops);

/* ==== Learned surrogate: the 10-frame state-delta network ====================
 * The surrogate is a plain multilayer perceptron, n_in -> n_hidden (x
 * n_hidden_layers, SiLU after each) -> n_out, that predicts the change of an
 * instance's state over the next 10 frames from features of its current state,
 * so that controller candidates can be ranked without stepping them; the
 * stepping path above stays the judge of every candidate it ranks highly.  The
 * paper has no learned component: this object serves batched controller search
 * around its simulator.
 *
 * Precision: NPX_SUR_BF16 keeps FP32 master weights and runs every product on
 * BF16 operands with FP32 accumulation; NPX_SUR_FP32 uses FP32 operands
 * throughout (for checking gradients).  Inputs and targets are standardised
 * inside, (x - mean) / std per column with the statistics given to
 * npx_sur_set_norm (identity until then); outputs come back in raw units.
 *
 * Parameters, in the flat order every call uses: for each layer in turn its
 * weights W [out][in] row-major, then its biases b [out].
 *
 * Buffers passed to forward/grad/train_step are device pointers: inputs x
 * [rows][ldx] FP32 (the first n_in columns are read), targets y [rows][ldy]
 * FP32, an optional row index list rows[batch] (int32, NULL = rows 0..batch-1)
 * that gathers the batch, outputs [batch][ldy] FP32.  Calls are asynchronous
 * on `stream` and share the object's work buffers: calls on one object that
 * overlap in time race.  get/set_params and set_norm synchronise the device. */
typedef struct npx_sur npx_sur;

enum { NPX_SUR_BF16 = 0, NPX_SUR_FP32 = 1 };

typedef struct {
  int32_t n_in, n_hidden, n_hidden_layers, n_out;
  int32_t max_batch;   /* largest batch of any call, <= 2^24 */
  int32_t precision;   /* NPX_SUR_BF16 or NPX_SUR_FP32 */
  int32_t training;    /* nonzero: also allocate backward and Adam buffers */
  uint64_t seed;       /* initial weights and biases ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)) */
} npx_sur_desc;

/* NPX_EINVAL for a bad shape (n_hidden_layers 1..7), NPX_ENOMEM when device
 * memory runs out.  The object owns all its device memory. */
npx_status npx_sur_create(const npx_sur_desc* d, npx_sur** out);
void npx_sur_destroy(npx_sur* s);  /* NULL-safe; waits for the device */
npx_status npx_sur_param_count(const npx_sur* s, int64_t* n);
/* n must equal the parameter count; setting resets the Adam moments and step. */
npx_status npx_sur_get_params(npx_sur* s, float* dst, int64_t n, int dst_on_device);
npx_status npx_sur_set_params(npx_sur* s, const float* src, int64_t n, int src_on_device);
/* Host arrays: x_mean, x_std [n_in], y_mean, y_std [n_out].  A standard
 * deviation <= 1e-12 (a constant column) is replaced by 1. */
npx_status npx_sur_set_norm(npx_sur* s, const float* x_mean, const float* x_std,
                            const float* y_mean, const float* y_std);
/* Adam moment decay rates and epsilon (defaults 0.9, 0.999, 1e-8). */
npx_status npx_sur_set_adam(npx_sur* s, double beta1, double beta2, double eps);
/* y[b] = network(x[rows[b]]) in raw units, b < batch <= max_batch.  Each
 * call is deterministic; a BF16 network whose hidden width is a multiple of
 * 128 (up to 384) runs whole 128-row blocks in one kernel and other batches
 * layer by layer, so a row's result can differ in the last bits between
 * batches of the two kinds. */
npx_status npx_sur_forward(npx_sur* s, const float* x, int64_t ldx, const int32_t* rows,
                           int64_t batch, float* y, int64_t ldy, void* stream);
/* Loss = mean over the batch and the n_out columns of the squared error of the
 * standardised prediction against the standardised target; writes it to
 * loss[0] (device, may be NULL) and its gradient with respect to the
 * parameters to grad[param_count] (device, flat order, may be NULL).  Needs
 * `training`; NPX_ESTATE otherwise. */
npx_status npx_sur_grad(npx_sur* s, const float* x, int64_t ldx, const float* y, int64_t ldy,
                        const int32_t* rows, int64_t batch, float* loss, float* grad,
                        void* stream);
/* npx_sur_grad, then one Adam step of size lr on the FP32 master weights. */
npx_status npx_sur_train_step(npx_sur* s, const float* x, int64_t ldx, const float* y,
                              int64_t ldy, const int32_t* rows, int64_t batch, double lr,
                              float* loss, void* stream);
/* Training noise: while set, every npx_sur_grad / npx_sur_train_step call adds
 * noise[b][j] (device, [batch][ldn], raw units) to input column col0 + j of
 * batch row b and subtracts it from target column col0 + j, so that the network
 * learns to return a perturbed state to the recorded next state (the columns
 * must exist in both).  The caller owns the buffer and refills it between
 * calls; noise == NULL switches it off.  Inference never sees it. */
npx_status npx_sur_set_noise(npx_sur* s, const float* noise, int64_t ldn, int32_t col0,
                             int32_t ncols);
/* Column means and population standard deviations (FP64 accumulation) of a
 * device matrix x [rows][ldx], first `cols` columns, into device arrays
 * mean, std [cols].  Synchronises `stream`. */
npx_status npx_sur_norm_stats(const float* x, int64_t ldx, int64_t rows, int32_t cols,
                              float* mean, float* std, void* stream);

/* ---- The simulator side of the surrogate ------------------------------------
 * State row of an instance, width 13 + 2 J (J = the world's joint stride, the
 * largest joint count over its morphologies): c (3, world CoG), Q (4, w x y z),
 * v (3), omega (3), q (J), q_prev (J); joints past an instance's own count are
 * 0.  The heading frame of a state: psi is the heading of the torso x axis on
 * the ground plane; vectors are turned by -psi about z and orientations are
 * left-multiplied by the yaw quaternion of -psi, negated if that leaves w < 0
 * (the sign chosen for the state's own orientation also applies to changes of
 * it).  Network input, width 13 + 12 J + 64:
 *   [0, 13)          0, 0, c_z - h(c_x, c_y), then Q, v, omega in the heading frame
 *   [13, 13 + J)     q;   [13 + J, 13 + 2 J)   (q - q_prev) / dt
 *   [13 + 2 J, 13 + 12 J)   the clamped commanded angles the next 10 frames
 *                    apply, frames n .. n + 9, frame-major
 *   [13 + 12 J, +64) an 8 x 8 patch of the height map at 0.08 m spacing,
 *                    centred on the CoG and turned with the torso heading (the
 *                    torso x axis on the ground plane), each sample minus
 *                    h(c_x, c_y); index 8 a + b, a along the heading, b to its left.
 * Frame n is the frame about to be stepped.  All buffers are device pointers,
 * row-major with the given row stride (in floats); calls are asynchronous on
 * `stream` and are ordered after earlier work on the world only through it. */
npx_status npx_sur_widths(const npx_world* w, int32_t* state_width, int32_t* feature_width);
/* s[i] = state row of instance i. */
npx_status npx_world_rows(npx_world* w, float* s, int64_t lds, void* stream);
/* State of instance i = s[i] (the inverse of npx_world_rows; the frame
 * counters, flags and telemetry are left as they are). */
npx_status npx_world_set_rows(npx_world* w, const float* s, int64_t lds, void* stream);
/* x[i] = network input of instance i, from the state rows s (s != NULL, at
 * frame `frame` >= 0) or from the world's own state and step counters (s ==
 * NULL), with the world's controllers and height map. */
npx_status npx_sur_features(npx_world* w, const float* s, int64_t lds, int64_t frame, float* x,
                            int64_t ldx, void* stream);
/* y[i] = (world state row of i) - s0[i], the body entries turned into the heading
 * frame of s0[i]: the training target after stepping.  y may alias s0. */
npx_status npx_sur_delta(npx_world* w, const float* s0, int64_t lds, float* y, int64_t ldy,
                         void* stream);
/* Rollout update of rows s at frame n: the body rows gain dy turned back from the
 * heading frame of s (Q renormalised),
 * q and q_prev become the clamped commands of frames n + 9 and n + 8 (what the
 * step sets).  Needs joint_interval == 1 (NPX_EUNSUPPORTED otherwise). */
npx_status npx_sur_advance(npx_world* w, float* s, int64_t lds, const float* dy, int64_t lddy,
                           int64_t frame, void* stream);
/* Joint-torque proxy of the controller-search fitness: each point carries its
 * weight m_k g; the points less than 0.002 m above the height map share the
 * robot's weight M |g| as an upward load; the torque of joint j is the moment
 * of the loads on all points distal to it, about its anchor, on its axis.
 * acc[i] (+)= mean over the instance's joints of |tau_j|, from rows s or (s ==
 * NULL) the world's state.  Up to 64 links. */
npx_status npx_sur_torque(npx_world* w, const float* s, int64_t lds, float* acc, int accumulate,
                          void* stream);
/* n_calls surrogate calls from rows s at frame frame0: per call the inputs
 * (written standardised straight into the network's own input rows), the
 * network (into y_work [I][ldy]), the update of s, and (tau_acc != NULL) the
 * torque proxy added to tau_acc[i].  The results equal those of
 * npx_sur_features + npx_sur_forward + npx_sur_advance (+ npx_sur_torque) call
 * by call.  x_work [I][ldx] (ldx >= the feature width) is checked but holds
 * nothing defined afterwards.  The network's widths must match the world's
 * and its max_batch must cover the instances. */
npx_status npx_sur_rollout(npx_sur* net, npx_world* w, float* s, int64_t lds, int64_t frame0,
                           int32_t n_calls, float* x_work, int64_t ldx, float* y_work,
                           int64_t ldy, float* tau_acc, void* stream);

/* The controller search's selection step (Sec. V, the surrogate screen): the
 * fitness of each of n candidates, f_i = (p1_i - p0_i) . h_i - torque_weight *
 * tau_i / n_calls, where p0_i and p1_i are columns 0 and 1 (the CoG's ground
 * position) of row i of s0 and s1 (row stride lds floats, >= 2), h_i the unit
 * start heading (heading [n][2]) and tau_i the torque proxy summed over
 * n_calls calls; f_i = -inf where flags[i] != 0 (flags may be NULL) or f_i is
 * not finite, and -0 counts as +0. fitness [n] receives every f_i; top [n_top]
 * the indices of the n_top largest, best first, equal values by the lower
 * index (n_top = 0: fitness only). All pointers are device memory; the call is
 * asynchronous on `stream` and takes its sort's scratch from the stream-
 * ordered allocator (freed on the stream). Errors: NPX_EINVAL for n < 0,
 * n > 2^31 - 1, n_top outside [0, n], n_calls < 1, lds < 2 or a NULL buffer
 * that is needed; NPX_ENOMEM, NPX_EHIP. */
npx_status npx_sur_screen_select(const float* s0, const float* s1, int64_t lds,
                                 const float* heading, const float* tau, int32_t n_calls,
                                 float torque_weight, const int32_t* flags, int64_t n,
                                 int32_t n_top, float* fitness, int32_t* top, void* stream);

#ifdef __cplusplus
}
#endif
#endif
