// The robot construction interface of the paper (Sec. IV and its appendix):
// bodies made of mass points, glued into rigid links, joined by hinges, then
// finalised into the morphology tables that npx_create_world takes. Host code.
//
// Readings where the paper's API text is terse:
//  * every body has a reference point (point: its position; box and sphere:
//    the centre; cylinder: the midpoint of its axis; ray: its start point) and
//    carries its own orientation, changed by rotateBody;
//  * createBox(w, h, d, ...): w along x, h along z, d along y; 8 corner points;
//  * moveBody places the body's reference point at (tx, ty, tz) of the
//    construction frame; rotateBody turns the body about its reference point by
//    roll alpha (x), then pitch beta (y), then yaw gamma (z), each about the
//    fixed construction axes, right-hand rule: R = Rz(gamma) Ry(beta) Rx(alpha);
//  * createJoint(id1, id2, anchor, axis): anchor and axis are given in body
//    1's frame (its reference point and orientation at the time of the call);
//    the link holding body 1 is the parent, the link holding body 2 the child;
//  * simplifyMode applies to cylinders and spheres created afterwards
//    (Sec. IV-C): 1 box (the 8 corners of the bounding box), 2 two points,
//    >= 3 one point at the reference point;
//  * a ray has no mass points and never collides; glued to a body of a link,
//    it is that link's range sensor (its start and end follow the body's
//    moves and rotations); a ray glued to no link is not listed;
//  * the root link is the link holding body 0.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "npx.h"

namespace {

constexpr double kPi = 3.14159265358979323846;
thread_local std::string g_morph_err;

npx_status bad(npx_status s, const char* msg) {
  g_morph_err = msg;
  return s;
}

struct V3 {
  double x, y, z;
};

V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
V3 mul(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
double norm(V3 a) { return std::sqrt(dot(a, a)); }

struct M3 {
  double m[9];
  static M3 eye() { return M3{{1, 0, 0, 0, 1, 0, 0, 0, 1}}; }
  V3 operator*(V3 v) const {
    return {m[0] * v.x + m[1] * v.y + m[2] * v.z, m[3] * v.x + m[4] * v.y + m[5] * v.z,
            m[6] * v.x + m[7] * v.y + m[8] * v.z};
  }
  M3 operator*(const M3& o) const {
    M3 r{};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        r.m[3 * i + j] = m[3 * i] * o.m[j] + m[3 * i + 1] * o.m[3 + j] + m[3 * i + 2] * o.m[6 + j];
    return r;
  }
  M3 transpose() const {
    return M3{{m[0], m[3], m[6], m[1], m[4], m[7], m[2], m[5], m[8]}};
  }
};

M3 rot_x(double a) {
  double c = std::cos(a), s = std::sin(a);
  return M3{{1, 0, 0, 0, c, -s, 0, s, c}};
}
M3 rot_y(double a) {
  double c = std::cos(a), s = std::sin(a);
  return M3{{c, 0, s, 0, 1, 0, -s, 0, c}};
}
M3 rot_z(double a) {
  double c = std::cos(a), s = std::sin(a);
  return M3{{c, -s, 0, s, c, 0, 0, 0, 1}};
}

struct Body {
  V3 ref;                 // reference point (construction frame)
  M3 orient;              // body axes in the construction frame
  std::vector<V3> local;  // points in the body frame
  double mass = 0;
  bool ray = false;
  V3 ray_end;             // a ray's end point in the body frame (its start is ref)
};

struct Joint {
  int body1, body2;
  V3 anchor_local, axis_local;  // in body 1's frame at creation
  V3 anchor, axis;              // construction frame, fixed at creation
  double lo = -1e30, hi = 1e30;
};

}  // namespace

struct npx_morph {
  int simplify = 0;
  bool final = false;
  std::vector<Body> bodies;
  std::vector<int> glue;  // union-find parent over bodies
  std::vector<Joint> joints;
  // finalised tables
  std::vector<float> points, joint_rows;
  std::vector<int32_t> pt_link, parent, joint_of_link, link_of_joint;
  std::vector<float> rays;       // [n][6] start, end (construction frame)
  std::vector<int32_t> ray_link; // [n]
};

namespace {

int find(npx_morph* m, int b) {
  while (m->glue[b] != b) b = m->glue[b] = m->glue[m->glue[b]];
  return b;
}

int add_body(npx_morph* m, Body b) {
  if (m->final) {
    g_morph_err = "construction is finalised";
    return NPX_ESTATE;
  }
  m->bodies.push_back(std::move(b));
  m->glue.push_back((int)m->glue.size());
  return (int)m->bodies.size() - 1;
}

bool valid_body(const npx_morph* m, int id) {
  return m && id >= 0 && id < (int)m->bodies.size();
}

// Two unit vectors perpendicular to d.
void basis(V3 d, V3* e1, V3* e2) {
  V3 h = std::fabs(d.z) < 0.9 ? V3{0, 0, 1} : V3{1, 0, 0};
  *e1 = mul(cross(d, h), 1.0 / norm(cross(d, h)));
  *e2 = cross(d, *e1);
}

}  // namespace

extern "C" {

const char* npx_morph_last_error(void) { return g_morph_err.c_str(); }

npx_status npx_morph_new(npx_morph** out) {
  if (!out) return bad(NPX_EINVAL, "null argument");
  *out = new npx_morph();
  return NPX_OK;
}

void npx_morph_free(npx_morph* m) { delete m; }

npx_status npx_simplify_mode(npx_morph* m, int mode) {
  if (!m || mode < 0) return bad(NPX_EINVAL, "bad simplify mode");
  if (m->final) return bad(NPX_ESTATE, "construction is finalised");
  m->simplify = mode;
  return NPX_OK;
}

int npx_create_point(npx_morph* m, double x, double y, double z, double mass) {
  if (!m || !(mass >= 0)) return bad(NPX_EINVAL, "bad point");
  Body b;
  b.ref = {x, y, z};
  b.orient = M3::eye();
  b.local = {{0, 0, 0}};
  b.mass = mass;
  return add_body(m, b);
}

int npx_create_box(npx_morph* m, double w, double h, double d, double x, double y, double z,
                   double mass) {
  if (!m || !(w >= 0 && h >= 0 && d >= 0 && mass >= 0)) return bad(NPX_EINVAL, "bad box");
  Body b;
  b.ref = {x, y, z};
  b.orient = M3::eye();
  for (int sx = -1; sx <= 1; sx += 2)
    for (int sy = -1; sy <= 1; sy += 2)
      for (int sz = -1; sz <= 1; sz += 2) b.local.push_back({sx * w / 2, sy * d / 2, sz * h / 2});
  b.mass = mass;
  return add_body(m, b);
}

int npx_create_box_grid(npx_morph* m, double w, double h, double d, double x, double y, double z,
                        double mass, int grid_nx, int grid_ny) {
  if (grid_nx == 0 && grid_ny == 0) return npx_create_box(m, w, h, d, x, y, z, mass);
  if (!m || !(w >= 0 && h >= 0 && d >= 0 && mass >= 0) || grid_nx < 2 || grid_ny < 2 ||
      grid_nx > 64 || grid_ny > 64)
    return bad(NPX_EINVAL, "bad box grid (0, 0 or both in [2, 64])");
  Body b;
  b.ref = {x, y, z};
  b.orient = M3::eye();
  for (int sz = -1; sz <= 1; sz += 2)
    for (int j = 0; j < grid_ny; ++j)
      for (int i = 0; i < grid_nx; ++i)
        b.local.push_back({w * ((double)i / (grid_nx - 1) - 0.5),
                           d * ((double)j / (grid_ny - 1) - 0.5), sz * h / 2});
  b.mass = mass;
  return add_body(m, b);
}

int npx_create_cylinder(npx_morph* m, double x1, double y1, double z1, double x2, double y2,
                        double z2, double rr, double mass, int ring_pts) {
  if (!m || !(rr >= 0 && mass >= 0) || ring_pts < 1) return bad(NPX_EINVAL, "bad cylinder");
  V3 p1{x1, y1, z1}, p2{x2, y2, z2};
  V3 axis = sub(p2, p1);
  double len = norm(axis);
  if (!(len > 0)) return bad(NPX_EINVAL, "cylinder of zero length");
  V3 d = mul(axis, 1.0 / len), e1, e2;
  basis(d, &e1, &e2);
  Body b;
  b.ref = mul(add(p1, p2), 0.5);
  // body frame: x = e1, y = e2, z = axis
  b.orient = M3{{e1.x, e2.x, d.x, e1.y, e2.y, d.y, e1.z, e2.z, d.z}};
  const double hl = len / 2;
  if (m->simplify == 0) {
    for (double zc : {-hl, hl})
      for (int k = 0; k < ring_pts; ++k) {
        double a = 2.0 * kPi * k / ring_pts;
        b.local.push_back({rr * std::cos(a), rr * std::sin(a), zc});
      }
  } else if (m->simplify == 1) {
    for (int sx = -1; sx <= 1; sx += 2)
      for (int sy = -1; sy <= 1; sy += 2)
        for (int sz = -1; sz <= 1; sz += 2) b.local.push_back({sx * rr, sy * rr, sz * hl});
  } else if (m->simplify == 2) {
    b.local = {{0, 0, -hl}, {0, 0, hl}};
  } else {
    b.local = {{0, 0, 0}};
  }
  b.mass = mass;
  return add_body(m, b);
}

int npx_create_sphere(npx_morph* m, double x, double y, double z, double rr, double mass) {
  if (!m || !(rr >= 0 && mass >= 0)) return bad(NPX_EINVAL, "bad sphere");
  Body b;
  b.ref = {x, y, z};
  b.orient = M3::eye();
  if (m->simplify == 0) {
    // the 12 vertices of a regular icosahedron on the sphere
    const double t = (1.0 + std::sqrt(5.0)) / 2.0, s = rr / std::sqrt(1.0 + t * t);
    const double v[12][3] = {{-1, t, 0}, {1, t, 0}, {-1, -t, 0}, {1, -t, 0},
                             {0, -1, t}, {0, 1, t}, {0, -1, -t}, {0, 1, -t},
                             {t, 0, -1}, {t, 0, 1}, {-t, 0, -1}, {-t, 0, 1}};
    for (auto& p : v) b.local.push_back({p[0] * s, p[1] * s, p[2] * s});
  } else if (m->simplify == 1) {
    for (int sx = -1; sx <= 1; sx += 2)
      for (int sy = -1; sy <= 1; sy += 2)
        for (int sz = -1; sz <= 1; sz += 2) b.local.push_back({sx * rr, sy * rr, sz * rr});
  } else if (m->simplify == 2) {
    b.local = {{0, 0, -rr}, {0, 0, rr}};
  } else {
    b.local = {{0, 0, 0}};
  }
  b.mass = mass;
  return add_body(m, b);
}

int npx_create_ray(npx_morph* m, double x1, double y1, double z1, double x2, double y2, double z2) {
  if (!m) return bad(NPX_EINVAL, "null morph");
  Body b;
  b.ref = {x1, y1, z1};
  b.orient = M3::eye();
  b.ray = true;
  b.ray_end = {x2 - x1, y2 - y1, z2 - z1};
  return add_body(m, b);
}

npx_status npx_connect_bodies(npx_morph* m, int id1, int id2) {
  if (!valid_body(m, id1) || !valid_body(m, id2)) return bad(NPX_EINVAL, "unknown body id");
  if (m->final) return bad(NPX_ESTATE, "construction is finalised");
  int a = find(m, id1), b = find(m, id2);
  if (a != b) m->glue[std::max(a, b)] = std::min(a, b);
  return NPX_OK;
}

int npx_create_joint(npx_morph* m, int id1, int id2, double anX, double anY, double anZ,
                     double aX, double aY, double aZ) {
  if (!valid_body(m, id1) || !valid_body(m, id2) || id1 == id2)
    return bad(NPX_EINVAL, "unknown or equal body ids");
  if (m->final) return bad(NPX_ESTATE, "construction is finalised");
  V3 ax{aX, aY, aZ};
  if (!(norm(ax) > 0)) return bad(NPX_EINVAL, "joint axis is zero");
  const Body& b1 = m->bodies[id1];
  Joint j;
  j.body1 = id1;
  j.body2 = id2;
  j.anchor_local = {anX, anY, anZ};
  j.axis_local = ax;
  j.anchor = add(b1.ref, b1.orient * j.anchor_local);
  j.axis = b1.orient * mul(ax, 1.0 / norm(ax));
  m->joints.push_back(j);
  return (int)m->joints.size() - 1;
}

npx_status npx_set_joint_limits(npx_morph* m, int joint, double lo, double hi) {
  if (!m || joint < 0 || joint >= (int)m->joints.size() || !(lo <= hi))
    return bad(NPX_EINVAL, "bad joint or limits");
  if (m->final) return bad(NPX_ESTATE, "construction is finalised");
  m->joints[joint].lo = lo;
  m->joints[joint].hi = hi;
  return NPX_OK;
}

npx_status npx_move_body(npx_morph* m, int id, double tx, double ty, double tz) {
  if (!valid_body(m, id)) return bad(NPX_EINVAL, "unknown body id");
  if (m->final) return bad(NPX_ESTATE, "construction is finalised");
  m->bodies[id].ref = {tx, ty, tz};
  return NPX_OK;
}

npx_status npx_rotate_body(npx_morph* m, int id, double alpha, double beta, double gamma) {
  if (!valid_body(m, id)) return bad(NPX_EINVAL, "unknown body id");
  if (m->final) return bad(NPX_ESTATE, "construction is finalised");
  Body& b = m->bodies[id];
  b.orient = rot_z(gamma) * rot_y(beta) * rot_x(alpha) * b.orient;
  return NPX_OK;
}

int npx_get_max_body_id(const npx_morph* m) { return m ? (int)m->bodies.size() : NPX_EINVAL; }

npx_status npx_finalize_construction(npx_morph* m) {
  if (!m) return bad(NPX_EINVAL, "null morph");
  if (m->final) return bad(NPX_ESTATE, "already finalised");
  if (m->bodies.empty()) return bad(NPX_EINVAL, "no bodies");
  const int B = (int)m->bodies.size();
  // links = glued groups of bodies; the root is the group holding body 0
  std::vector<int> group(B), link_of_group(B, -1);
  for (int b = 0; b < B; ++b) group[b] = find(m, b);
  // each joint joins the group of body 1 (parent) to the group of body 2 (child)
  const int NJ = (int)m->joints.size();
  std::vector<int> jparent(NJ), jchild(NJ);
  std::vector<int> parent_joint(B, -1);
  for (int j = 0; j < NJ; ++j) {
    jparent[j] = group[m->joints[j].body1];
    jchild[j] = group[m->joints[j].body2];
    if (jparent[j] == jchild[j]) return bad(NPX_EINVAL, "joint between glued bodies");
    if (parent_joint[jchild[j]] >= 0) return bad(NPX_EINVAL, "a link has two parent joints");
    parent_joint[jchild[j]] = j;
  }
  const int root = group[0];
  if (parent_joint[root] >= 0) return bad(NPX_EINVAL, "the root link has a parent joint");
  // breadth-first from the root, children in joint order: parents precede children
  std::vector<int> order{root};
  link_of_group[root] = 0;
  for (size_t k = 0; k < order.size(); ++k)
    for (int j = 0; j < NJ; ++j)
      if (jparent[j] == order[k]) {
        link_of_group[jchild[j]] = (int)order.size();
        order.push_back(jchild[j]);
      }
  for (int b = 0; b < B; ++b)
    if (link_of_group[group[b]] < 0 && !m->bodies[b].ray)
      return bad(NPX_EINVAL, "a body is not connected to the root by joints");
  const int L = (int)order.size();
  m->parent.assign(L, -1);
  m->joint_of_link.assign(L, -1);
  m->link_of_joint.assign(NJ, -1);
  m->joint_rows.assign(8 * L, 0.f);
  for (int j = 0; j < NJ; ++j) {
    int l = link_of_group[jchild[j]];
    if (l < 0) continue;
    m->parent[l] = link_of_group[jparent[j]];
    m->joint_of_link[l] = j;
    m->link_of_joint[j] = l;
    const Joint& J = m->joints[j];
    float* r = &m->joint_rows[8 * l];
    r[0] = (float)J.anchor.x; r[1] = (float)J.anchor.y; r[2] = (float)J.anchor.z;
    r[3] = (float)J.axis.x; r[4] = (float)J.axis.y; r[5] = (float)J.axis.z;
    r[6] = (float)J.lo; r[7] = (float)J.hi;
  }
  for (int b = 0; b < B; ++b) {
    const Body& bd = m->bodies[b];
    if (bd.ray || bd.local.empty()) continue;
    const double mk = bd.mass / bd.local.size();
    for (const V3& p : bd.local) {
      V3 w = add(bd.ref, bd.orient * p);
      m->points.insert(m->points.end(), {(float)w.x, (float)w.y, (float)w.z, (float)mk});
      m->pt_link.push_back(link_of_group[group[b]]);
    }
  }
  if (m->points.empty()) return bad(NPX_EINVAL, "no mass points");
  m->rays.clear();
  m->ray_link.clear();
  for (int b = 0; b < B; ++b) {
    const Body& bd = m->bodies[b];
    const int l = link_of_group[group[b]];
    if (!bd.ray || l < 0) continue;
    const V3 e = add(bd.ref, bd.orient * bd.ray_end);
    m->rays.insert(m->rays.end(), {(float)bd.ref.x, (float)bd.ref.y, (float)bd.ref.z,
                                   (float)e.x, (float)e.y, (float)e.z});
    m->ray_link.push_back(l);
  }
  m->final = true;
  return NPX_OK;
}

npx_status npx_morph_get_tables(const npx_morph* m, npx_morph_tables* out) {
  if (!m || !out) return bad(NPX_EINVAL, "null argument");
  if (!m->final) return bad(NPX_ESTATE, "construction is not finalised");
  out->n_points = (int32_t)m->pt_link.size();
  out->n_links = (int32_t)m->parent.size();
  out->points = m->points.data();
  out->pt_link = m->pt_link.data();
  out->parent = m->parent.data();
  out->joint = m->joint_rows.data();
  return NPX_OK;
}

npx_status npx_morph_get_rays(const npx_morph* m, int32_t* n_rays, const float** rays,
                              const int32_t** ray_link) {
  if (!m || !n_rays || !rays || !ray_link) return bad(NPX_EINVAL, "null argument");
  if (!m->final) return bad(NPX_ESTATE, "construction is not finalised");
  *n_rays = (int32_t)m->ray_link.size();
  *rays = m->rays.data();
  *ray_link = m->ray_link.data();
  return NPX_OK;
}

int npx_morph_joint_index(const npx_morph* m, int joint_id) {
  if (!m || !m->final || joint_id < 0 || joint_id >= (int)m->link_of_joint.size())
    return bad(NPX_EINVAL, "bad joint id or not finalised");
  int l = m->link_of_joint[joint_id];
  return l < 0 ? NPX_EINVAL : l - 1;
}

}  // extern "C"
