// mesh_dev.hpp -- device geometry of the triangulated body (the deforming bodies of Sec. IV.C):
// crossing of a +x ray with a triangle (inside test by crossing parity), ray-triangle link
// fractions with the barycentric wall velocity, and the velocity of the closest surface point.
// Every predicate and intersection is FP64 with the operations in the order written and no
// contraction, so that masks are reproducible bit for bit.  Candidate triangles come from the
// uniform grid of MeshDev (spacing >= 2): a lattice link spans at most two cells per axis and a
// point within distance h of p lies in the cells around p's cell.
#pragma once

#include "elbm_internal.hpp"

namespace elbm {

__device__ inline double m_edge(const double* a, const double* b, double py, double pz) {
#pragma clang fp contract(off)
  const double l = (b[1] - a[1]) * (pz - a[2]);
  const double r = (b[2] - a[2]) * (py - a[1]);
  return l - r;
}

// half-plane rule: an edge a -> b of a positively oriented projected triangle owns the points on
// it iff dz > 0, or dz = 0 and dy < 0 (each point of a shared edge or vertex is owned once)
__device__ inline bool m_owns(const double* a, const double* b) {
#pragma clang fp contract(off)
  const double dy = b[1] - a[1], dz = b[2] - a[2];
  return dz > 0.0 || (dz == 0.0 && dy < 0.0);
}

// Does the +x ray through (y, z) cross triangle (A, B, C)?  If so, xc = x of the crossing.
__device__ inline bool mesh_crossing(const double* A, const double* B0, const double* C0, double y, double z,
                                     double& xc) {
#pragma clang fp contract(off)
  const double* B = B0;
  const double* C = C0;
  const double area = m_edge(A, B, C[1], C[2]);
  if (area == 0.0) return false;
  if (area < 0.0) {
    B = C0;
    C = B0;
  }
  const double w0 = m_edge(B, C, y, z), w1 = m_edge(C, A, y, z), w2 = m_edge(A, B, y, z);
  if (w0 < 0.0 || (w0 == 0.0 && !m_owns(B, C))) return false;
  if (w1 < 0.0 || (w1 == 0.0 && !m_owns(C, A))) return false;
  if (w2 < 0.0 || (w2 == 0.0 && !m_owns(A, B))) return false;
  double num = w0 * A[0];
  num = num + w1 * B[0];
  num = num + w2 * C[0];
  double den = w0 + w1;
  den = den + w2;
  xc = num / den;
  return true;
}

__device__ inline double m_dot(const double* a, const double* b) {
#pragma clang fp contract(off)
  double s = a[0] * b[0];
  s = s + a[1] * b[1];
  return s + a[2] * b[2];
}
__device__ inline void m_sub(const double* a, const double* b, double* o) {
  o[0] = a[0] - b[0];
  o[1] = a[1] - b[1];
  o[2] = a[2] - b[2];
}
__device__ inline void m_cross(const double* a, const double* b, double* o) {
#pragma clang fp contract(off)
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// Ray o + s d against (A, B, C): o + s d = A + u (B - A) + v (C - A) by scalar triple products.
__device__ inline bool ray_triangle(const double* o, const double* d, const double* A, const double* B,
                                    const double* C, double& s, double& u, double& v) {
#pragma clang fp contract(off)
  double e1[3], e2[3], p[3], tv[3], qv[3];
  m_sub(B, A, e1);
  m_sub(C, A, e2);
  m_cross(d, e2, p);
  const double det = m_dot(e1, p);
  if (det == 0.0) return false;
  const double inv = 1.0 / det;
  m_sub(o, A, tv);
  const double uu = m_dot(tv, p) * inv;
  if (uu < 0.0 || uu > 1.0) return false;
  m_cross(tv, e1, qv);
  const double vv = m_dot(d, qv) * inv;
  if (vv < 0.0 || uu + vv > 1.0) return false;
  s = m_dot(e2, qv) * inv;
  u = uu;
  v = vv;
  return true;
}

// Closest point of (A, B, C) to p: the projection onto the plane when inside (weights from the
// Gram system of the edges), else the closest point of the three edges.  Returns the squared
// distance; w = barycentric weights of the closest point.
__device__ inline double closest_on_triangle(const double* p, const double* A, const double* B, const double* C,
                                             double* w) {
#pragma clang fp contract(off)
  double e1[3], e2[3], ap[3];
  m_sub(B, A, e1);
  m_sub(C, A, e2);
  m_sub(p, A, ap);
  const double d00 = m_dot(e1, e1), d01 = m_dot(e1, e2), d11 = m_dot(e2, e2);
  const double d20 = m_dot(ap, e1), d21 = m_dot(ap, e2);
  const double den = d00 * d11 - d01 * d01;
  if (den > 0.0) {
    const double lb = (d11 * d20 - d01 * d21) / den;
    const double lc = (d00 * d21 - d01 * d20) / den;
    const double la = 1.0 - lb - lc;
    if (la >= 0.0 && lb >= 0.0 && lc >= 0.0) {
      double q[3], r[3];
      for (int a = 0; a < 3; ++a) q[a] = A[a] + lb * e1[a] + lc * e2[a];
      m_sub(p, q, r);
      w[0] = la;
      w[1] = lb;
      w[2] = lc;
      return m_dot(r, r);
    }
  }
  const double* P0[3] = {A, B, C};
  const double* P1[3] = {B, C, A};
  double best = INFINITY;
  for (int e = 0; e < 3; ++e) {
    double d[3], r0[3];
    m_sub(P1[e], P0[e], d);
    m_sub(p, P0[e], r0);
    const double dd = m_dot(d, d);
    double tau = dd > 0.0 ? m_dot(r0, d) / dd : 0.0;
    if (tau < 0.0) tau = 0.0;
    if (tau > 1.0) tau = 1.0;
    double q[3], r[3];
    for (int a = 0; a < 3; ++a) q[a] = P0[e][a] + tau * d[a];
    m_sub(p, q, r);
    const double d2 = m_dot(r, r);
    if (d2 < best) {
      best = d2;
      w[0] = w[1] = w[2] = 0.0;
      w[e] = 1.0 - tau;
      w[e == 2 ? 0 : e + 1] = tau;
    }
  }
  return best;
}

__device__ inline void bary_velocity(const double* V, const int32_t* t3, const double* w, double* out) {
#pragma clang fp contract(off)
  const double* va = V + 3 * t3[0];
  const double* vb = V + 3 * t3[1];
  const double* vc = V + 3 * t3[2];
  for (int a = 0; a < 3; ++a) {
    double s = w[0] * va[a];
    s = s + w[1] * vb[a];
    out[a] = s + w[2] * vc[a];
  }
}

__device__ inline int mesh_cell_index(const MeshDev& m, int cx, int cy, int cz) {
  return (cz * m.dim[1] + cy) * m.dim[0] + cx;
}

// Velocity of the surface point closest to p among the triangles of the cells around p's cell
// (lowest triangle index among equal distances); 0 if there is none.
__device__ inline void mesh_closest_velocity(const MeshDev& m, int lvl, const double* p, double* out) {
  const MeshLevel& L = m.lv[lvl];
  int c0[3];
  for (int a = 0; a < 3; ++a) c0[a] = mesh_cell(m, a, p[a]);
  double best = INFINITY, bw[3] = {1.0, 0.0, 0.0};
  int bk = -1;
  for (int cz = max(c0[2] - 1, 0); cz <= min(c0[2] + 1, m.dim[2] - 1); ++cz)
    for (int cy = max(c0[1] - 1, 0); cy <= min(c0[1] + 1, m.dim[1] - 1); ++cy)
      for (int cx = max(c0[0] - 1, 0); cx <= min(c0[0] + 1, m.dim[0] - 1); ++cx) {
        const int c = mesh_cell_index(m, cx, cy, cz);
        const int e1 = min(L.start[c + 1], m.cap);
        for (int e = L.start[c]; e < e1; ++e) {
          const int k = L.items[e];
          if ((unsigned)k >= (unsigned)m.nt) continue;
          const int32_t* t3 = m.tri + 3 * k;
          double w[3];
          const double d2 = closest_on_triangle(p, L.X + 3 * t3[0], L.X + 3 * t3[1], L.X + 3 * t3[2], w);
          if (d2 < best || (d2 == best && k < bk)) {
            best = d2;
            bk = k;
            bw[0] = w[0];
            bw[1] = w[1];
            bw[2] = w[2];
          }
        }
      }
  if (bk < 0) {
    out[0] = out[1] = out[2] = 0.0;
    return;
  }
  bary_velocity(L.V, m.tri + 3 * bk, bw, out);
}

// The same in the lane-parallel form (one node per group of GROUP lanes, all lanes calling): the
// lanes share out the candidate triangles, then the group takes the minimum of (distance, index),
// which makes the result that of mesh_closest_velocity.
__device__ inline void mesh_closest_velocity_group(const MeshDev& m, int lvl, const double* p, int lane, double* out) {
  const MeshLevel& L = m.lv[lvl];
  int c0[3];
  for (int a = 0; a < 3; ++a) c0[a] = mesh_cell(m, a, p[a]);
  double best = INFINITY, bw[3] = {1.0, 0.0, 0.0};
  int bk = INT32_MAX;
  for (int cz = max(c0[2] - 1, 0); cz <= min(c0[2] + 1, m.dim[2] - 1); ++cz)
    for (int cy = max(c0[1] - 1, 0); cy <= min(c0[1] + 1, m.dim[1] - 1); ++cy)
      for (int cx = max(c0[0] - 1, 0); cx <= min(c0[0] + 1, m.dim[0] - 1); ++cx) {
        const int c = mesh_cell_index(m, cx, cy, cz);
        const int e1 = min(L.start[c + 1], m.cap);
        for (int e = L.start[c] + lane; e < e1; e += GROUP) {
          const int k = L.items[e];
          if ((unsigned)k >= (unsigned)m.nt) continue;
          const int32_t* t3 = m.tri + 3 * k;
          double w[3];
          const double d2 = closest_on_triangle(p, L.X + 3 * t3[0], L.X + 3 * t3[1], L.X + 3 * t3[2], w);
          if (d2 < best || (d2 == best && k < bk)) {
            best = d2;
            bk = k;
            bw[0] = w[0];
            bw[1] = w[1];
            bw[2] = w[2];
          }
        }
      }
  // group minimum of (best, bk), then the weights from the lane that holds it
  double gb = best;
  int gk = bk;
#pragma unroll
  for (int o = GROUP / 2; o > 0; o >>= 1) {
    const double ob = __shfl_xor(gb, o, GROUP);
    const int ok = __shfl_xor(gk, o, GROUP);
    if (ob < gb || (ob == gb && ok < gk)) {
      gb = ob;
      gk = ok;
    }
  }
  if (gk == INT32_MAX) {
    out[0] = out[1] = out[2] = 0.0;
    return;
  }
  const uint64_t own = __ballot(bk == gk && best == gb);
  const int src = __ffsll((unsigned long long)(own >> (threadIdx.x & 32u)) & 0xffffffffull) - 1;
  double w[3];
  for (int a = 0; a < 3; ++a) w[a] = __shfl(bw[a], src, GROUP);
  bary_velocity(L.V, m.tri + 3 * gk, w, out);
}

// Link of fluid node xb in direction i at level t+1: q = the smallest s in (0, 1] where xb - s c_i
// meets a triangle, uw barycentric there; otherwise q = 1/2 and the closest-point velocity of the
// link's midpoint.
__device__ inline void mesh_link(const MeshDev& m, const double* xb, int i, double& q, double* uw) {
#pragma clang fp contract(off)
  const MeshLevel& L = m.lv[1];
  const double d[3] = {-(double)cx(i), -(double)cy(i), -(double)cz(i)};
  int lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    const double e = xb[a] + d[a];
    lo[a] = mesh_cell(m, a, fmin(xb[a], e));
    hi[a] = mesh_cell(m, a, fmax(xb[a], e));
  }
  double best = INFINITY, bu = 0.0, bv = 0.0;
  int bk = -1;
  for (int cz = lo[2]; cz <= hi[2]; ++cz)
    for (int cy = lo[1]; cy <= hi[1]; ++cy)
      for (int cx = lo[0]; cx <= hi[0]; ++cx) {
        const int c = mesh_cell_index(m, cx, cy, cz);
        const int e1 = min(L.start[c + 1], m.cap);
        for (int e = L.start[c]; e < e1; ++e) {
          const int k = L.items[e];
          if ((unsigned)k >= (unsigned)m.nt) continue;
          const int32_t* t3 = m.tri + 3 * k;
          double s, u, v;
          if (!ray_triangle(xb, d, L.X + 3 * t3[0], L.X + 3 * t3[1], L.X + 3 * t3[2], s, u, v)) continue;
          if (!(s > 0.0 && s <= 1.0)) continue;
          if (s < best || (s == best && k < bk)) {
            best = s;
            bk = k;
            bu = u;
            bv = v;
          }
        }
      }
  if (bk >= 0) {
    const double w[3] = {1.0 - bu - bv, bu, bv};
    q = best;
    bary_velocity(L.V, m.tri + 3 * bk, w, uw);
    return;
  }
  const double mid[3] = {xb[0] + 0.5 * d[0], xb[1] + 0.5 * d[1], xb[2] + 0.5 * d[2]};
  q = 0.5;
  mesh_closest_velocity(m, 1, mid, uw);
}

}  // namespace elbm
