/*
 * npx_oracle.h -- FP64 CPU oracle of the NeoPhysIx per-frame step
 * (Fischer & Ihme, "NeoPhysIx: An Ultra Fast 3D Physical Simulator as
 * Development Tool for AI Algorithms", arXiv 2411.05799).
 *
 * TEST INFRASTRUCTURE ONLY. This library is the plain, slow, obviously correct
 * reference that the GPU path is checked against. Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg may load it. It shares no code,
 * header, table or constant with the GPU library; both read the same float32
 * input arrays and nothing else.
 *
 * Every quantity is double precision, round-to-nearest, built without
 * fast-math and with floating-point contraction off.
 *
 * Parity pins: every step part is pinned by a closed form, an invariant, a
 * textbook routine or brute force (see tests/test_oracle_pins.py). The whole
 * step composed over long chaotic horizons has no closed form: beyond those
 * pins its parity is unpinned.
 */
#ifndef NPX_ORACLE_H
#define NPX_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* One robot: mass points in the construction frame and its hinge tree. */
typedef struct {
  int n_points;
  int n_links;
  const float* points;  /* [n_points][4] x, y, z, mass */
  const int* pt_link;   /* [n_points] */
  const int* parent;    /* [n_links], parent[0] = -1, parent[l] < l */
  const float* joint;   /* [n_links][8] anchor xyz, axis xyz, lo, hi */
} orc_morph;

typedef struct {
  double dt;
  int K;          /* joint-update interval (steps) */
  double g[3];
  double mu;      /* friction coefficient, +inf = always stick */
  double k_n;     /* normal stiffness per point */
  double zeta;    /* Hunt-Crossley damping */
  double eps;     /* LSQ spread threshold */
  int weighted;   /* 1: each point's terms in the friction fit weighted by its
                     normal force (Sec. III-C, closing remark) */
  int hf_bilinear; /* 1: the table's entries are heights at cell centres,
                      interpolated bilinearly (0: the paper's look-up table) */
  int hf_nx, hf_ny;
  double hf_s, hf_x0, hf_y0;
  const float* hf; /* [hf_ny][hf_nx] */
  double max_rate; /* > 0: a joint turns at most max_rate rad/s, so one joint
                      update moves it by at most max_rate K dt towards its
                      command (the motors' speed, Sec. III-B); 0 or +inf: no limit */
  int six_dof;     /* 1: the friction fit takes the full rigid motion in 3-D
                      (rotations about the other two axes as well, the
                      refinement closing Sec. III-C; see orc_lsq6_w) and the
                      correction moves the robot back by all of it; not with
                      weighted (the step functions return -1) */
} orc_params;

/* The six-degree fit takes a 3-D rotation only when the smallest eigenvalue
 * of the contact set's spread tensor is at least this fraction of its trace
 * (see orc_lsq6_w). */
#define ORC_SIX_DOF_COND 1e-3

/* Per-instance state vector (double), fixed offsets; q and q_prev follow. */
enum {
  ORC_C = 0,       /* world centre of gravity (3) */
  ORC_Q = 3,       /* torso orientation quaternion w, x, y, z (4) */
  ORC_V = 7,       /* CoG velocity (3) */
  ORC_W = 10,      /* angular velocity, world frame (3) */
  ORC_STEP = 13,   /* step counter n, t = n * dt */
  ORC_FLAGS = 14,  /* health flags; non-zero freezes the instance */
  ORC_TELE = 15,   /* telemetry accumulators (4) */
  ORC_HDR = 19     /* q[J] starts here, then q_prev[J] */
};
#define ORC_STATE_LEN(J) (ORC_HDR + 2 * (J))

/* Per-step diagnostics written by orc_step when diag != NULL. */
enum {
  ORC_D_FN = 0,      /* total normal force F_N */
  ORC_D_TAU = 1,     /* torque about the CoG (3) */
  ORC_D_NC = 4,      /* points in contact at P^n */
  ORC_D_NS = 5,      /* points in the friction set */
  ORC_D_A = 6,       /* a1, a2, a3 (3) */
  ORC_D_LAMBDA = 9,  /* static-friction cap factor */
  ORC_D_FF = 10,     /* friction force estimate */
  ORC_D_A6 = 11,     /* six-degree fit: displacement (3), rotation vector (3) */
  ORC_D_LEN = 17
};

/* Flag bits. */
#define ORC_FLAG_NONFINITE 1
#define ORC_FLAG_SPEED 2

/* A fragile decision of one step: an integer outcome decided by floating point
 * that a change of the inputs far below the parity tolerances could turn the
 * other way. A float32 evaluation of the same step may take it either way, so
 * the parity checks log these and, for a frame that disagrees, re-run the
 * step with one of them taken the other way (a "flip"). */
enum {
  ORC_FR_S1 = 0,       /* stage: detection at P^n (S1, and the S2 force) */
  ORC_FR_S5 = 1,       /* stage: detection at the predicted P* (S5) */
  ORC_FR_FIT = 2,      /* stage: the friction fit and its cap (S6-S7) */
  ORC_FR_S9 = 3        /* stage: the telemetry look-up under the torso origin */
};
enum {
  ORC_FK_EDGE_X = 0,   /* look-up within the margin of a cell edge along x; flip:
                          the cell on the other side of that edge */
  ORC_FK_EDGE_Y = 1,   /* the same along y */
  ORC_FK_CONTACT = 2,  /* |stored height - z| below the margin; flip: the contact
                          test inverted */
  ORC_FK_SPREAD = 3,   /* spread test of the fit within a relative margin of
                          n eps^2; flip: the other branch (rotation fitted or not) */
  ORC_FK_CAP = 4       /* friction estimate within a relative margin of mu F_N;
                          only the slipping-frame counter depends on it (the cap
                          factor is continuous there); flip: the count inverted */
};
typedef struct {
  int stage;      /* ORC_FR_* */
  int point;      /* point index k (-1 for the fit) */
  int kind;       /* ORC_FK_* */
  double dist;    /* distance to the edge or to zero depth (m), or the relative
                     distance to the threshold */
} orc_fragile;

int orc_version(void);

/* Forward kinematics at joint angles q: torso-frame points y [N][3], CoG g_b,
 * inertia about the CoG I_b [3][3] (row-major), total mass. */
void orc_fk(const orc_morph* m, const double* q, double* y, double* g_b, double* I_b,
            double* mass);

/* Height-map look-up: cell indices and the stored height. */
void orc_cell(const orc_params* p, double x, double y, int* i, int* j);
double orc_height(const orc_params* p, double x, double y);

/* Range sensor (a ray of the construction API, Sec. IV, read against the
 * look-up-table ground of Sec. III-A): the distance from A to the first point
 * of the segment A -> B whose height is at or below the stored height of the
 * cell it lies in, or |B - A| when there is none (0 when A is at or below).
 * Nearest-cell ground only (p->hf_bilinear is ignored). */
double orc_ray_range(const orc_params* p, const double A[3], const double B[3]);

/* Friction least squares on n point pairs (ground-plane coordinates):
 * src [n][2] at t, dst [n][2] at t+1. Writes a1, a2, a3. Returns the number of
 * unknowns solved (0 none, 2 translation only, 3 full). */
int orc_lsq(int n, const double* src, const double* dst, double eps, double* a);
/* The same fit with pair i's residuals weighted by wt[i] >= 0 (wt == NULL:
 * all 1). Returns 3 (rotation fitted), 2 (displacement only) or 0 (no pair,
 * or all weights zero: no motion). */
int orc_lsq_w(int n, const double* src, const double* dst, const double* wt, double eps,
              double* a);
/* The six-degree-of-freedom friction fit on n point pairs in 3-D (src [n][3]
 * at t, dst [n][3] at t+1, about the origin of the coordinates), pair i
 * weighted by wt[i] (NULL: 1): a[0..2] the displacement, a[3..5] the
 * rotation vector of the least-squares small rigid motion, when the set's
 * spread tensor about its centroid has its smallest eigenvalue above W eps^2
 * and ORC_SIX_DOF_COND times its trace;
 * else the ground-plane fit of orc_lsq_w on the x, y components (in a[0],
 * a[1], a[5]) with the mean vertical slip in a[2]. Returns 6, 3, 2, 0, or -1
 * when out of memory. */
int orc_lsq6_w(int n, const double* src, const double* dst, const double* wt, double eps,
               double* a);
/* Smallest eigenvalue of a symmetric 3x3 matrix (row-major). */
double orc_sym3_min_eig(const double* A);

/* State from a start pose [7] = torso origin xyz + quaternion, at rest. */
int orc_init_state(const orc_morph* m, const orc_params* p, const float* ctrl,
                   const float* pose, double* state);

/* World positions of all points for a state [N][3]. */
void orc_points(const orc_morph* m, const double* state, double* P);

/* One step n -> n+1. Returns 0, or -1 on invalid input. */
int orc_step(const orc_morph* m, const orc_params* p, const float* ctrl, double* state,
             double* diag);

/* One step that also logs its fragile decisions: every look-up of a point at
 * or below the higher of the two cells' heights (plus margins[0] metres) whose
 * coordinate lies within margins[0] of a cell edge, the telemetry look-up
 * within margins[0] of an edge between cells of different height, every
 * contact test with |depth| < margins[0], the fit's spread test within
 * margins[1] (relative) of its threshold and the static-friction comparison
 * within margins[2] (relative). Up to log_cap entries go to log (n_log gets
 * the count, which may exceed log_cap). flips[0..n_flips) are decisions taken
 * the other way; zero margins and no flips give exactly orc_step. */
int orc_step_ex(const orc_morph* m, const orc_params* p, const float* ctrl, double* state,
                double* diag, const double* margins, orc_fragile* log, int log_cap,
                int* n_log, const orc_fragile* flips, int n_flips);

/* n_steps steps of one instance. */
int orc_run(const orc_morph* m, const orc_params* p, const float* ctrl, double* state,
            long n_steps);

/* n_steps steps of n_inst independent instances on up to n_threads threads
 * (n_threads <= 0: all). Returns the thread count used, or -1 for parameters
 * the step does not take. */
int orc_run_batch(int n_inst, const orc_morph* morphs, const int* inst_morph,
                  const orc_params* p, const float* const* ctrl, double* const* states,
                  long n_steps, int n_threads);

#ifdef __cplusplus
}
#endif
#endif
