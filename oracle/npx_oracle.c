/*
 * npx_oracle.c -- FP64 CPU oracle of the NeoPhysIx per-frame step.
 *
 * TEST INFRASTRUCTURE ONLY (see npx_oracle.h). Plain loops in the order the
 * step is defined; no blocking, fusion or reordering. Where the paper is
 * silent, the reading used is named in the comment of the part it fixes.
 *
 * The step, n -> n+1 at t = n dt, for one robot treated as a single rigid body
 * made of mass points (Sec. III-A, III-B):
 *   S0  controller: commanded joint angles (the user's move() of Fig. 1)
 *   S1  point-cloud collision against the height-map look-up table (Sec. III-A)
 *   S2  normal penalty force per contact point, summed to force and torque
 *       (the paper gives no normal response; reading: Hunt-Crossley penalty)
 *   S3  joint-angle determination: joints are set kinematically, the robot
 *       stays one rigid body and its world CoG is kept (Sec. III-B)
 *   S4  trial integration (semi-implicit Euler) to the predicted points P*
 *   S5  friction set: points in contact at both t and t+1 (Sec. III-C, eq. 3)
 *   S6  least-squares displacement + rotation of the contact points, the
 *       linearised rigid map (eqs. 1-2) solved through the normal equations
 *       (eqs. 4-6), in the ground plane, about the predicted CoG
 *   S7  cap by the maximum static friction mu F_N (Sec. III-C)
 *   S8  move the robot back by the (capped) fitted motion, with the matching
 *       velocity change, and commit
 *   S9  telemetry and health flags (not physics)
 */
#include "npx_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_version(void) { return 1; }

/* ------------------------------------------------------------------------- */
/* small dense linear algebra, row-major 3x3                                  */
/* ------------------------------------------------------------------------- */

static void m3_mul(const double* A, const double* B, double* C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
      C[3 * i + j] = s;
    }
}

static void m3_vec(const double* A, const double* x, double* y) {
  for (int i = 0; i < 3; ++i) y[i] = A[3 * i] * x[0] + A[3 * i + 1] * x[1] + A[3 * i + 2] * x[2];
}

static void m3_transpose(const double* A, double* T) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) T[3 * j + i] = A[3 * i + j];
}

static void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

static double det3(const double* A) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* Gaussian elimination with partial pivoting on a copy of A. Returns 0 when a
 * pivot vanishes. */
static int solve3(const double* A_in, const double* b_in, double* x) {
  double A[9], b[3];
  memcpy(A, A_in, sizeof A);
  memcpy(b, b_in, sizeof b);
  for (int col = 0; col < 3; ++col) {
    int piv = col;
    for (int r = col + 1; r < 3; ++r)
      if (fabs(A[3 * r + col]) > fabs(A[3 * piv + col])) piv = r;
    if (A[3 * piv + col] == 0.0) return 0;
    if (piv != col) {
      for (int k = 0; k < 3; ++k) {
        double t = A[3 * col + k];
        A[3 * col + k] = A[3 * piv + k];
        A[3 * piv + k] = t;
      }
      double t = b[col];
      b[col] = b[piv];
      b[piv] = t;
    }
    for (int r = col + 1; r < 3; ++r) {
      double f = A[3 * r + col] / A[3 * col + col];
      for (int k = col; k < 3; ++k) A[3 * r + k] -= f * A[3 * col + k];
      b[r] -= f * b[col];
    }
  }
  for (int r = 2; r >= 0; --r) {
    double s = b[r];
    for (int k = r + 1; k < 3; ++k) s -= A[3 * r + k] * x[k];
    x[r] = s / A[3 * r + r];
  }
  return 1;
}

/* Gaussian elimination with partial pivoting on an n x n system (n <= 6),
 * on copies. Returns 0 when a pivot vanishes. */
static int solve_n(int n, const double* A_in, const double* b_in, double* x) {
  double A[36], b[6];
  memcpy(A, A_in, sizeof(double) * n * n);
  memcpy(b, b_in, sizeof(double) * n);
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabs(A[n * r + col]) > fabs(A[n * piv + col])) piv = r;
    if (A[n * piv + col] == 0.0) return 0;
    if (piv != col) {
      for (int k = 0; k < n; ++k) {
        double t = A[n * col + k];
        A[n * col + k] = A[n * piv + k];
        A[n * piv + k] = t;
      }
      double t = b[col];
      b[col] = b[piv];
      b[piv] = t;
    }
    for (int r = col + 1; r < n; ++r) {
      double f = A[n * r + col] / A[n * col + col];
      for (int k = col; k < n; ++k) A[n * r + k] -= f * A[n * col + k];
      b[r] -= f * b[col];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double s = b[r];
    for (int k = r + 1; k < n; ++k) s -= A[n * r + k] * x[k];
    x[r] = s / A[n * r + r];
  }
  return 1;
}

/* Smallest eigenvalue of a symmetric 3x3 matrix: the roots of its
 * characteristic cubic in trigonometric form. With q = tr A / 3 and
 * B = (A - q 1) / p, p^2 = |A - q 1|_F^2 / 6, the eigenvalues are
 * q + 2 p cos(phi + 2 pi k / 3), phi = acos(det B / 2) / 3; k = 1 gives the
 * smallest. */
static double sym3_min_eig(const double* A) {
  const double q = (A[0] + A[4] + A[8]) / 3.0;
  const double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
  const double d0 = A[0] - q, d1 = A[4] - q, d2 = A[8] - q;
  const double p2 = d0 * d0 + d1 * d1 + d2 * d2 + 2.0 * off;
  if (!(p2 > 0.0)) return q;
  const double pp = sqrt(p2 / 6.0);
  double B[9];
  for (int i = 0; i < 9; ++i) B[i] = A[i] / pp;
  B[0] -= q / pp; B[4] -= q / pp; B[8] -= q / pp;
  double r = 0.5 * det3(B);
  r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
  const double phi = acos(r) / 3.0;
  return q + 2.0 * pp * cos(phi + 2.0 * acos(-1.0) / 3.0);
}

double orc_sym3_min_eig(const double* A) { return sym3_min_eig(A); }

/* Rotation matrix of a unit quaternion (w, x, y, z). */
static void quat_to_mat(const double* Q, double* R) {
  double w = Q[0], x = Q[1], y = Q[2], z = Q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* Hamilton product a (x) b. */
static void quat_mul(const double* a, const double* b, double* o) {
  double w = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  double x = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
  double y = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
  double z = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
  o[0] = w; o[1] = x; o[2] = y; o[3] = z;
}

static void quat_normalize(double* Q) {
  double n = sqrt(Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2] + Q[3] * Q[3]);
  for (int i = 0; i < 4; ++i) Q[i] /= n;
}

/* Unit quaternion of the rotation vector th (angle |th| about th/|th|). */
static void quat_exp(const double* th, double* o) {
  double a = sqrt(th[0] * th[0] + th[1] * th[1] + th[2] * th[2]);
  if (a < 1e-12) {
    o[0] = 1.0; o[1] = 0.5 * th[0]; o[2] = 0.5 * th[1]; o[3] = 0.5 * th[2];
    return;
  }
  double s = sin(0.5 * a) / a;
  o[0] = cos(0.5 * a); o[1] = s * th[0]; o[2] = s * th[1]; o[3] = s * th[2];
}

/* Rotation by angle th about the unit axis a (Rodrigues' formula). */
static void axis_angle(const double* a, double th, double* R) {
  double c = cos(th), s = sin(th), C = 1.0 - c;
  double x = a[0], y = a[1], z = a[2];
  R[0] = c + x * x * C;     R[1] = x * y * C - z * s; R[2] = x * z * C + y * s;
  R[3] = y * x * C + z * s; R[4] = c + y * y * C;     R[5] = y * z * C - x * s;
  R[6] = z * x * C - y * s; R[7] = z * y * C + x * s; R[8] = c + z * z * C;
}

/* ------------------------------------------------------------------------- */
/* forward kinematics and mass properties (Sec. III-A mass points, III-B)     */
/* ------------------------------------------------------------------------- */

/* Link l moves with its parent and turns by q[l-1] about its hinge, whose
 * anchor and axis are given in the construction frame (createJoint, Sec. IV-B):
 *   T_l(x) = T_parent(Rot(a_l, q)(x - o_l) + o_l),  T_0 = identity.
 * Body points y_k = T_link(k)(rho_k). The CoG and inertia are the plain mass
 * point sums. */
void orc_fk(const orc_morph* m, const double* q, double* y, double* g_b, double* I_b,
            double* mass) {
  int L = m->n_links, N = m->n_points;
  double* R = (double*)malloc(sizeof(double) * 9 * L);
  double* t = (double*)malloc(sizeof(double) * 3 * L);
  for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0) ? 1.0 : 0.0;
  t[0] = t[1] = t[2] = 0.0;
  for (int l = 1; l < L; ++l) {
    const float* jt = m->joint + 8 * l;
    int p = m->parent[l];
    double o[3] = {jt[0], jt[1], jt[2]};
    double a[3] = {jt[3], jt[4], jt[5]};
    double an = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    a[0] /= an; a[1] /= an; a[2] /= an;
    double Rj[9], Ro[3], u[3], w[3];
    axis_angle(a, q[l - 1], Rj);
    m3_mul(R + 9 * p, Rj, R + 9 * l);
    m3_vec(Rj, o, Ro);
    for (int i = 0; i < 3; ++i) u[i] = o[i] - Ro[i];
    m3_vec(R + 9 * p, u, w);
    for (int i = 0; i < 3; ++i) t[3 * l + i] = w[i] + t[3 * p + i];
  }
  double M = 0.0, gs[3] = {0, 0, 0};
  for (int k = 0; k < N; ++k) {
    const float* pt = m->points + 4 * k;
    int l = m->pt_link[k];
    double rho[3] = {pt[0], pt[1], pt[2]}, yk[3];
    m3_vec(R + 9 * l, rho, yk);
    for (int i = 0; i < 3; ++i) {
      y[3 * k + i] = yk[i] + t[3 * l + i];
      gs[i] += (double)pt[3] * y[3 * k + i];
    }
    M += pt[3];
  }
  for (int i = 0; i < 3; ++i) g_b[i] = gs[i] / M;
  for (int i = 0; i < 9; ++i) I_b[i] = 0.0;
  for (int k = 0; k < N; ++k) {
    double mk = m->points[4 * k + 3];
    double r[3] = {y[3 * k] - g_b[0], y[3 * k + 1] - g_b[1], y[3 * k + 2] - g_b[2]};
    double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) I_b[3 * i + j] += mk * ((i == j ? rr : 0.0) - r[i] * r[j]);
  }
  *mass = M;
  free(R);
  free(t);
}

/* ------------------------------------------------------------------------- */
/* height-map look-up (Sec. III-A)                                            */
/* ------------------------------------------------------------------------- */

/* The x-y coordinates are scaled by s and turned into integer indices of a 2-D
 * table. Reading: index = floor(s (x - x0)), clamped onto the table (a NaN
 * coordinate maps to cell 0), evaluated in double like the rest of the
 * oracle. */
static int cell_index(double x, double x0, double s, int n) {
  double u = s * (x - x0);
  if (!(u >= 0.0)) return 0;
  if (u >= (double)(n - 1)) return n - 1;
  return (int)floor(u);
}

/* The interior cell edge nearest to x along one axis (the edges between cells
 * sit at the integers 1..n-1 of u = s (x - x0)): returns the distance to it in
 * metres (+inf when the axis has one cell or x is NaN) and writes the cell on
 * its other side from cell i. */
static double nearest_edge(double x, double x0, double s, int n, int i, int* other) {
  double u = s * (x - x0);
  *other = i;
  if (n < 2 || !(u == u)) return INFINITY;
  double e = floor(u + 0.5);
  if (e < 1.0) e = 1.0;
  if (e > (double)(n - 1)) e = (double)(n - 1);
  *other = (i >= (int)e) ? (int)e - 1 : (int)e;
  return fabs(u - e) / s;
}

void orc_cell(const orc_params* p, double x, double y, int* i, int* j) {
  *i = cell_index(x, p->hf_x0, p->hf_s, p->hf_nx);
  *j = cell_index(y, p->hf_y0, p->hf_s, p->hf_ny);
}

static int cmp_double(const void* a, const void* b) {
  const double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

/* The segment is split at every parameter t where it crosses a grid line
 * x = x0 + k/s or y = y0 + k/s; inside each piece it stays in one cell (the
 * cell of the piece's midpoint), whose ground is flat, and its height is
 * linear in t. The first piece that starts at or below its cell's height, or
 * ends there, holds the first ground point. */
double orc_ray_range(const orc_params* p, const double A[3], const double B[3]) {
  const double d[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
  const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  const double s = p->hf_s;
  const double org[2] = {p->hf_x0, p->hf_y0};
  int cap = 2;
  for (int a = 0; a < 2; ++a) cap += (int)(fabs(d[a]) * s) + 2;
  double* t = (double*)malloc(sizeof(double) * cap);
  int n = 0;
  t[n++] = 0.0;
  t[n++] = 1.0;
  for (int a = 0; a < 2; ++a) {
    if (d[a] == 0.0) continue;
    const double u0 = (A[a] - org[a]) * s, u1 = (B[a] - org[a]) * s;
    const double lo = fmin(u0, u1), hi = fmax(u0, u1);
    for (double k = floor(lo) + 1.0; k < hi; k += 1.0) {
      const double tk = (org[a] + k / s - A[a]) / d[a];
      if (tk > 0.0 && tk < 1.0 && n < cap) t[n++] = tk;
    }
  }
  qsort(t, n, sizeof(double), cmp_double);
  double out = len;
  for (int q = 0; q + 1 < n; ++q) {
    const double ta = t[q], tb = t[q + 1];
    if (!(tb > ta)) continue;
    const double tm = 0.5 * (ta + tb);
    int i, j;
    orc_cell(p, A[0] + tm * d[0], A[1] + tm * d[1], &i, &j);
    const double h = p->hf[(size_t)j * p->hf_nx + i];
    const double za = A[2] + ta * d[2], zb = A[2] + tb * d[2];
    if (za <= h) { out = ta * len; break; }
    if (zb <= h) { out = (h - A[2]) / d[2] * len; break; }
  }
  free(t);
  return out;
}

/* One axis of the bilinear reading: the lower centre index and the fraction
 * towards the next, the coordinate held inside the outer centres. */
static void centre_axis(double x, double x0, double s, int n, int* i0, double* f) {
  double u = (x - x0) * s - 0.5;
  if (!(u > 0.0)) u = 0.0;
  if (u > (double)(n - 1)) u = (double)(n - 1);
  int i = (int)floor(u);
  if (i > n - 2) i = n - 2;
  if (i < 0) i = 0;
  *i0 = i;
  *f = n >= 2 ? u - (double)i : 0.0;
}

double orc_height(const orc_params* p, double x, double y) {
  if (p->hf_bilinear) {
    /* reading of the "smoother ground" option: entry (i, j) is the height at
     * the centre of cell (i, j); bilinear between the four centres around */
    int i0, j0;
    double fu, fw;
    centre_axis(x, p->hf_x0, p->hf_s, p->hf_nx, &i0, &fu);
    centre_axis(y, p->hf_y0, p->hf_s, p->hf_ny, &j0, &fw);
    const int i1 = p->hf_nx >= 2 ? i0 + 1 : i0, j1 = p->hf_ny >= 2 ? j0 + 1 : j0;
    const double h00 = p->hf[(long)j0 * p->hf_nx + i0], h10 = p->hf[(long)j0 * p->hf_nx + i1];
    const double h01 = p->hf[(long)j1 * p->hf_nx + i0], h11 = p->hf[(long)j1 * p->hf_nx + i1];
    return (1.0 - fu) * (1.0 - fw) * h00 + fu * (1.0 - fw) * h10 + (1.0 - fu) * fw * h01 +
           fu * fw * h11;
  }
  int i, j;
  orc_cell(p, x, y, &i, &j);
  return (double)p->hf[(long)j * p->hf_nx + i];
}

/* ------------------------------------------------------------------------- */
/* fragile decisions (for the parity checks; no effect on the step's result    */
/* unless a flip is requested)                                                */
/* ------------------------------------------------------------------------- */

typedef struct {
  double margin_m, margin_spread, margin_cap;
  orc_fragile* log;
  int log_cap, n_log;
  const orc_fragile* flips;
  int n_flips;
} fragile_ctx;

static int is_flipped(const fragile_ctx* fc, int stage, int point, int kind) {
  if (!fc) return 0;
  for (int i = 0; i < fc->n_flips; ++i)
    if (fc->flips[i].stage == stage && fc->flips[i].point == point && fc->flips[i].kind == kind)
      return 1;
  return 0;
}

static void note_fragile(fragile_ctx* fc, int stage, int point, int kind, double dist) {
  if (!fc) return;
  if (fc->n_log < fc->log_cap) {
    orc_fragile* e = fc->log + fc->n_log;
    e->stage = stage;
    e->point = point;
    e->kind = kind;
    e->dist = dist;
  }
  fc->n_log++;
}

/* Depth below the ground (stored height - z) of point k seen at `stage`: the
 * step's own look-up, with the look-ups near a cell edge that could change the
 * point's contact or depth logged (the point is at or below the higher of the
 * two cells) and requested flips applied. */
static double probe_depth(const orc_params* p, fragile_ctx* fc, int stage, int k, double x,
                          double y, double z) {
  if (p->hf_bilinear || !fc) return orc_height(p, x, y) - z;
  int i = cell_index(x, p->hf_x0, p->hf_s, p->hf_nx);
  int j = cell_index(y, p->hf_y0, p->hf_s, p->hf_ny);
  int oi, oj;
  const double ex = nearest_edge(x, p->hf_x0, p->hf_s, p->hf_nx, i, &oi);
  const double ey = nearest_edge(y, p->hf_y0, p->hf_s, p->hf_ny, j, &oj);
  const long nx = p->hf_nx;
  const double h = p->hf[(long)j * nx + i];
  if (ex < fc->margin_m) {
    const double hb = p->hf[(long)j * nx + oi];
    if (hb != h && z < fmax(h, hb) + fc->margin_m) note_fragile(fc, stage, k, ORC_FK_EDGE_X, ex);
  }
  if (ey < fc->margin_m) {
    const double hb = p->hf[(long)oj * nx + i];
    if (hb != h && z < fmax(h, hb) + fc->margin_m) note_fragile(fc, stage, k, ORC_FK_EDGE_Y, ey);
  }
  if (is_flipped(fc, stage, k, ORC_FK_EDGE_X)) i = oi;
  if (is_flipped(fc, stage, k, ORC_FK_EDGE_Y)) j = oj;
  return (double)p->hf[(long)j * nx + i] - z;
}

/* The contact test "strictly below the ground" of point k at `stage`, logged
 * when |depth| is below the margin, inverted when flipped. */
static int probe_contact(fragile_ctx* fc, int stage, int k, double d) {
  int kap = d > 0.0;
  if (fc) {
    if (fabs(d) < fc->margin_m) note_fragile(fc, stage, k, ORC_FK_CONTACT, fabs(d));
    if (is_flipped(fc, stage, k, ORC_FK_CONTACT)) kap = !kap;
  }
  return kap;
}

/* ------------------------------------------------------------------------- */
/* friction least squares (Sec. III-C, eqs. 1-6)                              */
/* ------------------------------------------------------------------------- */

/* Fit dst ~ [[1, -a3], [a3, 1]] src + (a1, a2) over the point pairs (eq. 2) by
 * least squares (eq. 3). Each pair contributes two residual rows whose
 * derivatives in (a1, a2, a3) are (1, 0, -y) and (0, 1, x); summing
 * J^T J a = J^T (dst - src) gives the three linear equations (4)-(6).
 * Reading: with one pair, or pairs with no spread (sum |src - mean|^2 <= n eps^2),
 * the rotation is not determined and only the displacement is fitted. */
int orc_lsq(int n, const double* src, const double* dst, double eps, double* a) {
  return orc_lsq_w(n, src, dst, NULL, eps, a);
}

/* Weighted reading of the closing remark of Sec. III-C: pair i's two
 * residuals enter the sum of squares times its weight w_i, so every sum of
 * eqs. (4)-(6) gains the factor w_i; the spread test and the
 * displacement-only fallback use the weighted spread and the total weight W
 * in place of n. */
static int lsq_core(int n, const double* src, const double* dst, const double* wt, double eps,
                    double* a, fragile_ctx* fc) {
  a[0] = a[1] = a[2] = 0.0;
  if (n <= 0) return 0;
  double A[9] = {0}, b[3] = {0};
  double W = 0, sx = 0, sy = 0, s2 = 0;
  for (int i = 0; i < n; ++i) {
    double wi = wt ? wt[i] : 1.0;
    double x = src[2 * i], y = src[2 * i + 1];
    double dx = dst[2 * i] - x, dy = dst[2 * i + 1] - y;
    double r1[3] = {1.0, 0.0, -y}; /* d/da of the x-residual */
    double r2[3] = {0.0, 1.0, x};  /* d/da of the y-residual */
    for (int u = 0; u < 3; ++u) {
      for (int v = 0; v < 3; ++v) A[3 * u + v] += wi * (r1[u] * r1[v] + r2[u] * r2[v]);
      b[u] += wi * (r1[u] * dx + r2[u] * dy);
    }
    W += wi;
    sx += wi * x; sy += wi * y; s2 += wi * (x * x + y * y);
  }
  if (!(W > 0.0)) return 0;
  double spread = s2 - (sx * sx + sy * sy) / W;
  int full = n >= 2 && spread > W * eps * eps;
  if (fc && n >= 2) {
    /* the spread is a difference of sums of size s2: its rounding scales with s2 */
    const double gap = fabs(spread - W * eps * eps), scale = W * eps * eps + s2;
    if (gap < fc->margin_spread * scale)
      note_fragile(fc, ORC_FR_FIT, -1, ORC_FK_SPREAD, gap / scale);
    if (is_flipped(fc, ORC_FR_FIT, -1, ORC_FK_SPREAD)) full = !full;
  }
  if (full && solve3(A, b, a)) return 3;
  a[0] = b[0] / W;
  a[1] = b[1] / W;
  a[2] = 0.0;
  return 2;
}

int orc_lsq_w(int n, const double* src, const double* dst, const double* wt, double eps,
              double* a) {
  return lsq_core(n, src, dst, wt, eps, a, NULL);
}

/* The six-degree-of-freedom fit (the refinement closing Sec. III-C, rotations
 * about the other two axes as well), in 3-D: the small rigid motion, a
 * displacement a and a rotation vector th about the origin of the
 * coordinates, that best carries the set's points at t (src [n][3]) onto
 * their points at t+1 (dst [n][3]), minimizing
 *   sum_i w_i |dst_i - (src_i + a + th x src_i)|^2
 * (th x src is the first-order term of the rotation, as a3 is of the yaw in
 * eq. 2). The residual of pair i is linear in x = (a, th): its component c
 * has the gradient (e_c, e_0 x src_i . e_c, e_1 x src_i . e_c, e_2 x src_i .
 * e_c), and the fit solves the 6 x 6 normal equations sum_i w_i G_i^T G_i x =
 * sum_i w_i G_i^T (dst_i - src_i). It is solved when the spread tensor of the
 * set about its centroid, S = sum_i w_i (|e_i|^2 1 - e_i e_i^T), e_i = src_i -
 * centroid, has its smallest eigenvalue above both W eps^2 and
 * ORC_SIX_DOF_COND tr S (three or more points, not on one line, and not so
 * close to a line that the rotation about it would be set by slips of
 * 1e-8 m: a bound of 1e3 on the ratio of the largest to the smallest
 * eigenvalue, within a factor of 3); else
 * the ground-plane fit of eqs. (4)-(6) on the x, y components (yaw and
 * horizontal displacement, or displacement only, by its own spread test) with
 * the weighted mean vertical slip as the vertical displacement and no roll or
 * pitch. Writes a[0..2] the displacement and a[3..5] the rotation; returns 6,
 * 3 (yaw only), 2 (displacement only) or 0 (no pair, or all weights zero). */
static int lsq6_core(int n, const double* src, const double* dst, const double* wt, double eps,
                     double* a, double* s2d, double* d2d, fragile_ctx* fc) {
  for (int i = 0; i < 6; ++i) a[i] = 0.0;
  if (n <= 0) return 0;
  double Nm[36] = {0}, rhs[6] = {0}, W = 0.0, cen[3] = {0, 0, 0}, s2 = 0.0;
  for (int i = 0; i < n; ++i) {
    const double wi = wt ? wt[i] : 1.0;
    const double* x = src + 3 * i;
    double d[3];
    for (int c = 0; c < 3; ++c) d[c] = dst[3 * i + c] - x[c];
    double G[3][6];
    for (int c = 0; c < 3; ++c) {
      for (int k = 0; k < 3; ++k) G[c][k] = c == k ? 1.0 : 0.0;
      for (int k = 0; k < 3; ++k) {
        double e[3] = {0, 0, 0}, ex[3];
        e[k] = 1.0;
        cross3(e, x, ex);
        G[c][3 + k] = ex[c];
      }
    }
    for (int u = 0; u < 6; ++u) {
      for (int v = 0; v < 6; ++v)
        for (int c = 0; c < 3; ++c) Nm[6 * u + v] += wi * G[c][u] * G[c][v];
      for (int c = 0; c < 3; ++c) rhs[u] += wi * G[c][u] * d[c];
    }
    W += wi;
    for (int c = 0; c < 3; ++c) cen[c] += wi * x[c];
    s2 += wi * (x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  }
  if (!(W > 0.0)) return 0;
  for (int c = 0; c < 3; ++c) cen[c] /= W;
  double S[9] = {0};
  for (int i = 0; i < n; ++i) {
    const double wi = wt ? wt[i] : 1.0;
    const double e[3] = {src[3 * i] - cen[0], src[3 * i + 1] - cen[1], src[3 * i + 2] - cen[2]};
    const double ee = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) S[3 * r + c] += wi * ((r == c ? ee : 0.0) - e[r] * e[c]);
  }
  const double lmin = sym3_min_eig(S);
  const double thr = fmax(W * eps * eps, ORC_SIX_DOF_COND * (S[0] + S[4] + S[8]));
  int full = n >= 3 && lmin > thr;
  if (fc && n >= 3) {
    const double gap = fabs(lmin - thr), scale = thr + s2;
    if (gap < fc->margin_spread * scale)
      note_fragile(fc, ORC_FR_FIT, -2, ORC_FK_SPREAD, gap / scale);
    if (is_flipped(fc, ORC_FR_FIT, -2, ORC_FK_SPREAD)) full = !full;
  }
  if (full && solve_n(6, Nm, rhs, a)) return 6;
  /* the ground-plane fit, and the mean vertical slip */
  double dz = 0.0;
  for (int i = 0; i < n; ++i) {
    const double wi = wt ? wt[i] : 1.0;
    s2d[2 * i] = src[3 * i];
    s2d[2 * i + 1] = src[3 * i + 1];
    d2d[2 * i] = dst[3 * i];
    d2d[2 * i + 1] = dst[3 * i + 1];
    dz += wi * (dst[3 * i + 2] - src[3 * i + 2]);
  }
  double a3[3];
  int r = lsq_core(n, s2d, d2d, wt, eps, a3, fc);
  for (int i = 0; i < 6; ++i) a[i] = 0.0;
  a[0] = a3[0];
  a[1] = a3[1];
  a[2] = dz / W;
  a[5] = a3[2];
  return r;
}

int orc_lsq6_w(int n, const double* src, const double* dst, const double* wt, double eps,
               double* a) {
  double* s2d = (double*)malloc(sizeof(double) * 2 * (n > 0 ? n : 1));
  double* d2d = (double*)malloc(sizeof(double) * 2 * (n > 0 ? n : 1));
  int r = (s2d && d2d) ? lsq6_core(n, src, dst, wt, eps, a, s2d, d2d, NULL) : -1;
  free(s2d);
  free(d2d);
  return r;
}

/* ------------------------------------------------------------------------- */
/* the step                                                                   */
/* ------------------------------------------------------------------------- */

typedef struct {
  double *y, *r, *P, *Ps, *src, *dst, *src3, *dst3, *f, *wt, *d;
  int* kap;
} work_t;

static int work_alloc(work_t* w, int N) {
  w->y = (double*)malloc(sizeof(double) * 3 * N);
  w->r = (double*)malloc(sizeof(double) * 3 * N);
  w->P = (double*)malloc(sizeof(double) * 3 * N);
  w->Ps = (double*)malloc(sizeof(double) * 3 * N);
  w->src = (double*)malloc(sizeof(double) * 2 * N);
  w->dst = (double*)malloc(sizeof(double) * 2 * N);
  w->src3 = (double*)malloc(sizeof(double) * 3 * N);
  w->dst3 = (double*)malloc(sizeof(double) * 3 * N);
  w->kap = (int*)malloc(sizeof(int) * N);
  w->f = (double*)malloc(sizeof(double) * N);
  w->wt = (double*)malloc(sizeof(double) * N);
  w->d = (double*)malloc(sizeof(double) * N);
  return w->y && w->r && w->P && w->Ps && w->src && w->dst && w->src3 && w->dst3 && w->kap &&
         w->f && w->wt && w->d;
}

static void work_free(work_t* w) {
  free(w->y); free(w->r); free(w->P); free(w->Ps); free(w->src); free(w->dst); free(w->kap);
  free(w->src3); free(w->dst3);
  free(w->f); free(w->wt); free(w->d);
}

/* Step parameters the oracle takes: the six-degree fit is not combined with
 * the force weighting (with the force on points along one line, a point of
 * near-zero force would decide the roll about it). */
static int params_ok(const orc_params* p) {
  return p->K >= 1 && p->dt > 0.0 && !(p->six_dof && p->weighted);
}

static int morph_ok(const orc_morph* m) {
  if (!m || m->n_points <= 0 || m->n_links <= 0) return 0;
  if (m->parent[0] != -1) return 0;
  for (int l = 1; l < m->n_links; ++l)
    if (m->parent[l] < 0 || m->parent[l] >= l) return 0;
  for (int k = 0; k < m->n_points; ++k)
    if (m->pt_link[k] < 0 || m->pt_link[k] >= m->n_links) return 0;
  return 1;
}

/* S0: commanded angle of joint j at time t, clamped to its limits. */
static double command(const orc_morph* m, const float* ctrl, int j, double t) {
  const double two_pi = 6.283185307179586476925286766559;
  double A = ctrl[3 * j], f = ctrl[3 * j + 1], phi = ctrl[3 * j + 2];
  double qh = A * sin(two_pi * f * t + phi);
  double lo = m->joint[8 * (j + 1) + 6], hi = m->joint[8 * (j + 1) + 7];
  if (qh < lo) qh = lo;
  if (qh > hi) qh = hi;
  return qh;
}

/* Principal inertia test shared by the oracle's integrator: an inertia with
 * det <= 1e-9 (trace/3)^3 (a point or a line of points) gets no angular
 * acceleration. */
static int inertia_regular(const double* I) {
  double tr = (I[0] + I[4] + I[8]) / 3.0;
  return tr > 0.0 && det3(I) > 1e-9 * tr * tr * tr;
}

/* Height of the torso origin c - R g_b above the stored ground under it (the
 * look-up logged and flippable like the step's own, stage S9). */
static double torso_height(const orc_params* p, const double* st, const double* g_b,
                           fragile_ctx* fc) {
  double R[9], Rg[3];
  quat_to_mat(st + ORC_Q, R);
  m3_vec(R, g_b, Rg);
  double o[3] = {st[ORC_C] - Rg[0], st[ORC_C + 1] - Rg[1], st[ORC_C + 2] - Rg[2]};
  if (p->hf_bilinear || !fc) return o[2] - orc_height(p, o[0], o[1]);
  int i = cell_index(o[0], p->hf_x0, p->hf_s, p->hf_nx);
  int j = cell_index(o[1], p->hf_y0, p->hf_s, p->hf_ny);
  int oi, oj;
  const double ex = nearest_edge(o[0], p->hf_x0, p->hf_s, p->hf_nx, i, &oi);
  const double ey = nearest_edge(o[1], p->hf_y0, p->hf_s, p->hf_ny, j, &oj);
  const long nx = p->hf_nx;
  const double h = p->hf[(long)j * nx + i];
  if (ex < fc->margin_m && p->hf[(long)j * nx + oi] != h)
    note_fragile(fc, ORC_FR_S9, -1, ORC_FK_EDGE_X, ex);
  if (ey < fc->margin_m && p->hf[(long)oj * nx + i] != h)
    note_fragile(fc, ORC_FR_S9, -1, ORC_FK_EDGE_Y, ey);
  if (is_flipped(fc, ORC_FR_S9, -1, ORC_FK_EDGE_X)) i = oi;
  if (is_flipped(fc, ORC_FR_S9, -1, ORC_FK_EDGE_Y)) j = oj;
  return o[2] - (double)p->hf[(long)j * nx + i];
}

static int step_ws(const orc_morph* m, const orc_params* p, const float* ctrl, double* st,
                   double* diag, work_t* w, fragile_ctx* fc) {
  const int N = m->n_points, J = m->n_links - 1;
  if (st[ORC_FLAGS] != 0.0) return 0; /* frozen instance */
  const long n = (long)st[ORC_STEP];
  const double dt = p->dt, t = (double)n * dt;
  double* q = st + ORC_HDR;
  double* q_prev = q + J;
  double* c = st + ORC_C;
  double* Q = st + ORC_Q;
  double* v = st + ORC_V;
  double* om = st + ORC_W;

  /* body points about the CoG at the current joint angles */
  double g_b[3], I_b[9], M;
  orc_fk(m, q, w->y, g_b, I_b, &M);
  for (int k = 0; k < N; ++k)
    for (int i = 0; i < 3; ++i) w->r[3 * k + i] = w->y[3 * k + i] - g_b[i];

  /* S1: detection at P^n (strictly below the stored height is contact) */
  double R[9];
  quat_to_mat(Q, R);
  int n_contact = 0;
  for (int k = 0; k < N; ++k) {
    double Rr[3];
    m3_vec(R, w->r + 3 * k, Rr);
    for (int i = 0; i < 3; ++i) w->P[3 * k + i] = c[i] + Rr[i];
    w->d[k] = probe_depth(p, fc, ORC_FR_S1, k, w->P[3 * k], w->P[3 * k + 1], w->P[3 * k + 2]);
    w->kap[k] = probe_contact(fc, ORC_FR_S1, k, w->d[k]);
    n_contact += w->kap[k];
  }

  /* S2: per-point normal force along +z, summed to force and torque about c */
  double F = 0.0, tau[3] = {0, 0, 0};
  for (int k = 0; k < N; ++k) {
    w->f[k] = 0.0;
    if (!w->kap[k]) continue;
    double arm[3] = {w->P[3 * k] - c[0], w->P[3 * k + 1] - c[1], w->P[3 * k + 2] - c[2]};
    double wxa[3];
    cross3(om, arm, wxa);
    double uz = v[2] + wxa[2];
    double f = p->k_n * w->d[k] * (1.0 - p->zeta * uz);
    if (f < 0.0) f = 0.0;
    w->f[k] = f;
    double fz[3] = {0.0, 0.0, f}, tk[3];
    cross3(arm, fz, tk);
    F += f;
    for (int i = 0; i < 3; ++i) tau[i] += tk[i];
  }

  /* S3: joint-angle determination every K steps; c, Q, v, omega are kept */
  if (n % p->K == 0) {
    /* reading of the motors' speed (Sec. III-B: joints reach their targets only
     * if the motors are fast enough): with a rate limit, a joint moves from its
     * angle towards the command by at most max_rate K dt per update */
    const int limited = p->max_rate > 0.0 && !isinf(p->max_rate);
    const double dmax = p->max_rate * p->K * p->dt;
    for (int j = 0; j < J; ++j) {
      q_prev[j] = q[j];
      double qn = command(m, ctrl, j, t);
      if (limited) {
        if (qn > q[j] + dmax) qn = q[j] + dmax;
        if (qn < q[j] - dmax) qn = q[j] - dmax;
      }
      q[j] = qn;
    }
    orc_fk(m, q, w->y, g_b, I_b, &M);
    for (int k = 0; k < N; ++k)
      for (int i = 0; i < 3; ++i) w->r[3 * k + i] = w->y[3 * k + i] - g_b[i];
  }

  /* S4: trial integration, semi-implicit Euler */
  double v1[3], om1[3], c1[3], Q1[4];
  for (int i = 0; i < 3; ++i) v1[i] = v[i] + dt * p->g[i];
  v1[2] += dt * F / M;
  {
    double Rt[9], tmp[9], Iw[9], Lw[3], gyro[3], rhs[3], acc[3] = {0, 0, 0};
    m3_transpose(R, Rt);
    m3_mul(R, I_b, tmp);
    m3_mul(tmp, Rt, Iw);
    m3_vec(Iw, om, Lw);
    cross3(om, Lw, gyro);
    for (int i = 0; i < 3; ++i) rhs[i] = tau[i] - gyro[i];
    if (!(inertia_regular(I_b) && solve3(Iw, rhs, acc))) acc[0] = acc[1] = acc[2] = 0.0;
    for (int i = 0; i < 3; ++i) om1[i] = om[i] + dt * acc[i];
  }
  for (int i = 0; i < 3; ++i) c1[i] = c[i] + dt * v1[i];
  {
    double th[3] = {dt * om1[0], dt * om1[1], dt * om1[2]}, dq[4];
    quat_exp(th, dq);
    quat_mul(dq, Q, Q1);
    quat_normalize(Q1);
  }
  double R1[9];
  quat_to_mat(Q1, R1);

  /* S5: predicted points P*, friction set = contact at both P^n and P* */
  int nS = 0;
  for (int k = 0; k < N; ++k) {
    double Rr[3];
    m3_vec(R1, w->r + 3 * k, Rr);
    for (int i = 0; i < 3; ++i) w->Ps[3 * k + i] = c1[i] + Rr[i];
    if (!w->kap[k]) continue; /* only points in contact at P^n can join the set */
    double ds = probe_depth(p, fc, ORC_FR_S5, k, w->Ps[3 * k], w->Ps[3 * k + 1], w->Ps[3 * k + 2]);
    if (probe_contact(fc, ORC_FR_S5, k, ds)) {
      /* ground-plane coordinates about the predicted CoG c1 */
      w->src[2 * nS] = w->P[3 * k] - c1[0];
      w->src[2 * nS + 1] = w->P[3 * k + 1] - c1[1];
      w->dst[2 * nS] = w->Ps[3 * k] - c1[0];
      w->dst[2 * nS + 1] = w->Ps[3 * k + 1] - c1[1];
      for (int i = 0; i < 3; ++i) {  /* the same in 3-D, for the six-degree fit */
        w->src3[3 * nS + i] = w->P[3 * k + i] - c1[i];
        w->dst3[3 * nS + i] = w->Ps[3 * k + i] - c1[i];
      }
      w->wt[nS] = w->f[k];  /* the force pressing the point at P^n */
      ++nS;
    }
  }

  /* S6: least-squares displacement and rotation of the contact points */
  double a[3], a6[6] = {0, 0, 0, 0, 0, 0};
  const double* wt = p->weighted ? w->wt : NULL;
  int fit;
  if (p->six_dof) {
    /* the src/dst arrays serve as the ground-plane fallback's scratch */
    fit = lsq6_core(nS, w->src3, w->dst3, wt, p->eps, a6, w->src, w->dst, fc);
    a[0] = a6[0];
    a[1] = a6[1];
    a[2] = a6[5];
  } else {
    fit = lsq_core(nS, w->src, w->dst, wt, p->eps, a, fc);
  }

  /* S7: cap by the maximum static friction mu F_N (the mean slip is weighted
   * like the fit) */
  double lam = 0.0, Ff = 0.0;
  if (fit > 0) {
    double sbx = 0.0, sby = 0.0, W = 0.0;
    for (int i = 0; i < nS; ++i) {
      double wi = wt ? wt[i] : 1.0;
      sbx += wi * (w->dst3[3 * i] - w->src3[3 * i]);
      sby += wi * (w->dst3[3 * i + 1] - w->src3[3 * i + 1]);
      W += wi;
    }
    sbx /= W;
    sby /= W;
    Ff = M * sqrt(sbx * sbx + sby * sby) / (dt * dt);
    if (isinf(p->mu) || Ff <= p->mu * F) lam = 1.0;
    else lam = p->mu * F / Ff;
  }
  /* the slipping-frame count is the only thing the cap's comparison decides
   * (lambda is continuous across it) */
  int slipping = fit > 0 && lam < 1.0;
  if (fc && fit > 0 && !isinf(p->mu)) {
    const double gap = fabs(Ff - p->mu * F), scale = fmax(Ff, p->mu * F);
    if (scale > 0.0 && gap < fc->margin_cap * scale)
      note_fragile(fc, ORC_FR_FIT, -1, ORC_FK_CAP, gap / scale);
    if (is_flipped(fc, ORC_FR_FIT, -1, ORC_FK_CAP)) slipping = !slipping;
  }

  /* S8: move back by the capped fitted motion (translation, then the rotation
   * about the CoG) and remove the matching velocity */
  if (p->six_dof) {
    /* the rotation vector's length is the sine of the angle (as a3 is of the
     * yaw in eq. 5): angle asin(|th|) about th / |th| */
    const double* th = a6 + 3;
    const double s = sqrt(th[0] * th[0] + th[1] * th[1] + th[2] * th[2]);
    const double ang = asin(s > 1.0 ? 1.0 : s);
    double phi[3] = {0.0, 0.0, 0.0}, back[3], qb[4], Q2[4];
    if (s > 0.0)
      for (int i = 0; i < 3; ++i) phi[i] = ang * th[i] / s;
    for (int i = 0; i < 3; ++i) back[i] = -lam * phi[i];
    quat_exp(back, qb);
    quat_mul(qb, Q1, Q2);
    for (int i = 0; i < 3; ++i) {
      c[i] = c1[i] - lam * a6[i];
      v[i] = v1[i] - lam * a6[i] / dt;
      om[i] = om1[i] - lam * phi[i] / dt;
    }
    for (int i = 0; i < 4; ++i) Q[i] = Q2[i];
  } else {
    double a3 = a[2] < -1.0 ? -1.0 : (a[2] > 1.0 ? 1.0 : a[2]);
    double alpha = asin(a3);
    double Q2[4];
    {
      double half = -0.5 * lam * alpha;
      double qz[4] = {cos(half), 0.0, 0.0, sin(half)};
      quat_mul(qz, Q1, Q2);
    }
    c[0] = c1[0] - lam * a[0];
    c[1] = c1[1] - lam * a[1];
    c[2] = c1[2];
    for (int i = 0; i < 4; ++i) Q[i] = Q2[i];
    v[0] = v1[0] - lam * a[0] / dt;
    v[1] = v1[1] - lam * a[1] / dt;
    v[2] = v1[2];
    om[0] = om1[0];
    om[1] = om1[1];
    om[2] = om1[2] - lam * alpha / dt;
  }

  /* S9: telemetry and health */
  st[ORC_TELE + 0] += torso_height(p, st, g_b, fc);
  st[ORC_TELE + 1] += n_contact;
  st[ORC_TELE + 2] += slipping ? 1.0 : 0.0;
  int bad = 0;
  for (int i = 0; i < 13; ++i)
    if (!isfinite(st[i])) bad |= ORC_FLAG_NONFINITE;
  double vv = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  double ww = sqrt(om[0] * om[0] + om[1] * om[1] + om[2] * om[2]);
  if (vv > 50.0 || ww > 500.0) bad |= ORC_FLAG_SPEED;
  st[ORC_FLAGS] = (double)bad;
  st[ORC_STEP] = (double)(n + 1);

  if (diag) {
    diag[ORC_D_FN] = F;
    for (int i = 0; i < 3; ++i) diag[ORC_D_TAU + i] = tau[i];
    diag[ORC_D_NC] = n_contact;
    diag[ORC_D_NS] = nS;
    for (int i = 0; i < 3; ++i) diag[ORC_D_A + i] = a[i];
    for (int i = 0; i < 6; ++i) diag[ORC_D_A6 + i] = a6[i];
    diag[ORC_D_LAMBDA] = lam;
    diag[ORC_D_FF] = Ff;
  }
  return 0;
}

int orc_init_state(const orc_morph* m, const orc_params* p, const float* ctrl,
                   const float* pose, double* st) {
  (void)p;
  if (!morph_ok(m)) return -1;
  const int J = m->n_links - 1, N = m->n_points;
  memset(st, 0, sizeof(double) * ORC_STATE_LEN(J));
  double* q = st + ORC_HDR;
  for (int j = 0; j < J; ++j) {
    q[j] = command(m, ctrl, j, 0.0);
    q[J + j] = q[j];
  }
  double Q[4] = {pose[3], pose[4], pose[5], pose[6]};
  quat_normalize(Q);
  double* y = (double*)malloc(sizeof(double) * 3 * N);
  double g_b[3], I_b[9], M, R[9], Rg[3];
  orc_fk(m, q, y, g_b, I_b, &M);
  free(y);
  quat_to_mat(Q, R);
  m3_vec(R, g_b, Rg);
  for (int i = 0; i < 3; ++i) st[ORC_C + i] = (double)pose[i] + Rg[i];
  for (int i = 0; i < 4; ++i) st[ORC_Q + i] = Q[i];
  return 0;
}

void orc_points(const orc_morph* m, const double* st, double* P) {
  const int N = m->n_points, J = m->n_links - 1;
  (void)J;
  double* y = (double*)malloc(sizeof(double) * 3 * N);
  double g_b[3], I_b[9], M, R[9];
  orc_fk(m, st + ORC_HDR, y, g_b, I_b, &M);
  quat_to_mat(st + ORC_Q, R);
  for (int k = 0; k < N; ++k) {
    double r[3] = {y[3 * k] - g_b[0], y[3 * k + 1] - g_b[1], y[3 * k + 2] - g_b[2]}, Rr[3];
    m3_vec(R, r, Rr);
    for (int i = 0; i < 3; ++i) P[3 * k + i] = st[ORC_C + i] + Rr[i];
  }
  free(y);
}

int orc_step(const orc_morph* m, const orc_params* p, const float* ctrl, double* st,
             double* diag) {
  if (!morph_ok(m) || !params_ok(p)) return -1;
  work_t w;
  if (!work_alloc(&w, m->n_points)) {
    work_free(&w);
    return -1;
  }
  int rc = step_ws(m, p, ctrl, st, diag, &w, NULL);
  work_free(&w);
  return rc;
}

int orc_step_ex(const orc_morph* m, const orc_params* p, const float* ctrl, double* st,
                double* diag, const double* margins, orc_fragile* log, int log_cap,
                int* n_log, const orc_fragile* flips, int n_flips) {
  if (!morph_ok(m) || !params_ok(p) || log_cap < 0 || n_flips < 0) return -1;
  work_t w;
  if (!work_alloc(&w, m->n_points)) {
    work_free(&w);
    return -1;
  }
  fragile_ctx fc = {margins ? margins[0] : 0.0, margins ? margins[1] : 0.0,
                    margins ? margins[2] : 0.0, log, log ? log_cap : 0, 0,
                    flips, flips ? n_flips : 0};
  int rc = step_ws(m, p, ctrl, st, diag, &w, &fc);
  if (n_log) *n_log = fc.n_log;
  work_free(&w);
  return rc;
}

int orc_run(const orc_morph* m, const orc_params* p, const float* ctrl, double* st,
            long n_steps) {
  if (!morph_ok(m) || !params_ok(p) || n_steps < 0) return -1;
  work_t w;
  if (!work_alloc(&w, m->n_points)) {
    work_free(&w);
    return -1;
  }
  for (long s = 0; s < n_steps; ++s) step_ws(m, p, ctrl, st, NULL, &w, NULL);
  work_free(&w);
  return 0;
}

int orc_run_batch(int n_inst, const orc_morph* morphs, const int* inst_morph,
                  const orc_params* p, const float* const* ctrl, double* const* states,
                  long n_steps, int n_threads) {
  if (!params_ok(p)) return -1;
  int used = 1;
#ifdef _OPENMP
  if (n_threads <= 0) n_threads = omp_get_max_threads();
  used = n_threads;
#pragma omp parallel for schedule(static) num_threads(n_threads)
#endif
  for (int i = 0; i < n_inst; ++i)
    orc_run(&morphs[inst_morph[i]], p, ctrl[i], states[i], n_steps);
  return used;
}
