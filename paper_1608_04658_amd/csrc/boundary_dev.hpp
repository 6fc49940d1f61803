// boundary_dev.hpp -- device helpers of the wall treatment (Sec. III) shared by the forward
// boundary kernel and its adjoint: node indexing, the previous-step velocity gradient stencil and
// the geometry of a boundary link.
#pragma once

#include "elbm_internal.hpp"

namespace elbm {

struct GeoArgs {
  uint8_t* flags;
  int32_t nx, ny, nz;
  int32_t channel;
  Box box;
};

__device__ __forceinline__ void box_node(const Box& b, long idx, int& x, int& y, int& z) {
  x = b.lo[0] + (int)(idx % b.n[0]);
  y = b.lo[1] + (int)((idx / b.n[0]) % b.n[1]);
  z = b.lo[2] + (int)(idx / ((long)b.n[0] * b.n[1]));
}

__device__ __forceinline__ int first_body(const Bodies& bd, bool at_t1, double x, double y, double z) {
  for (int k = 0; k < bd.nb; ++k)
    if (inside_body(bd.b[k], at_t1 ? bd.b[k].c1 : bd.b[k].c0, x, y, z)) return k;
  return -1;
}

// Periodic index for any offset (stencils reach +-2, lattices may be 1 or 2 nodes thick).
__device__ __forceinline__ int wrap(int v, int n) { return ((v % n) + n) % n; }

struct BArgs {
  const void* A;
  void* B;
  const uint8_t* flags;
  const float* macro;
  const float* F;
  const int32_t* list;
  const uint32_t* dyn_count;
  double* brec;
  int64_t n_static;
  int64_t cap;
  int32_t moving;
  int32_t nx, ny, nz;
  int64_t N;
  int32_t channel;
  int32_t fp64;
  int32_t stream_only;
  float beta, inv_beta, thr;
  double rho0;
  double u_in[3];
};

__device__ __forceinline__ long node_at(const BArgs& a, int x, int y, int z) {
  return ((long)z * a.ny + y) * a.nx + x;
}

// Node x + d, or -1 when it does not exist (outside [0, nx) in channel mode).
__device__ __forceinline__ long neighbour(const BArgs& a, int x, int y, int z, int dx, int dy, int dz) {
  int X = x + dx;
  if (a.channel) {
    if (X < 0 || X >= a.nx) return -1;
  } else {
    X = wrap(X, a.nx);
  }
  return node_at(a, X, wrap(y + dy, a.ny), wrap(z + dz, a.nz));
}

// Velocity gradient by finite differences on U^t (Sec. III), G[3a+b] = d u_a / d x_b.  Per axis:
// central if both neighbours are usable (exist and fluid at t+1), else second-order one-sided
// (forward side first), else first-order one-sided, else 0.
__device__ inline void grad_u(const BArgs& a, int x, int y, int z, long n0, float (&G)[9]) {
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int e0 = b == 0, e1 = b == 1, e2 = b == 2;
    const long p1 = neighbour(a, x, y, z, e0, e1, e2), p2 = neighbour(a, x, y, z, 2 * e0, 2 * e1, 2 * e2);
    const long m1 = neighbour(a, x, y, z, -e0, -e1, -e2), m2 = neighbour(a, x, y, z, -2 * e0, -2 * e1, -2 * e2);
    const bool op1 = p1 >= 0 && !(a.flags[p1] & FL_SOLID), op2 = p2 >= 0 && !(a.flags[p2] & FL_SOLID);
    const bool om1 = m1 >= 0 && !(a.flags[m1] & FL_SOLID), om2 = m2 >= 0 && !(a.flags[m2] & FL_SOLID);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float* U = a.macro + c * a.N;
      float d;
      if (op1 && om1) d = 0.5f * (U[p1] - U[m1]);
      else if (op1 && op2) d = 0.5f * (-3.f * U[n0] + 4.f * U[p1] - U[p2]);
      else if (om1 && om2) d = 0.5f * (3.f * U[n0] - 4.f * U[m1] + U[m2]);
      else if (op1) d = U[p1] - U[n0];
      else if (om1) d = U[n0] - U[m1];
      else d = 0.f;
      G[3 * c + b] = d;
    }
  }
}

// Geometry of boundary link i (i in Dbar) at node (x,y,z): link fraction q, wall velocity u_w and
// owning body (-1 for the inlet wall at x = -1/2).  q is the ray parameter where x - s c_i meets
// the surface (FP64): sphere (|d|^2 - R^2)/(d.c_i + sqrt((d.c_i)^2 - |c_i|^2 (|d|^2 - R^2))),
// plane n.d / n.c_i, d = x - centre(t+1).
__device__ inline void link_geometry(const BArgs& a, const Bodies& bd, int i, int x, int y, int z, double& q, double (&uw)[3],
                              int& kb) {
  int sx = x - cx(i);
  if (a.channel && sx < 0) {
    kb = -1;
    q = ((double)x + 0.5) / (double)cx(i);
    uw[0] = a.u_in[0];
    uw[1] = a.u_in[1];
    uw[2] = a.u_in[2];
    return;
  }
  if (a.channel) sx = sx >= a.nx ? a.nx - 1 : sx;
  else sx = wrap(sx, a.nx);
  const int sy = wrap(y - cy(i), a.ny), sz = wrap(z - cz(i), a.nz);
  kb = first_body(bd, true, sx, sy, sz);
  if (kb < 0) kb = 0;
  const BodyDev& b = bd.b[kb];
  const double v[3] = {(double)cx(i), (double)cy(i), (double)cz(i)};
  const double d[3] = {x - b.c1[0], y - b.c1[1], z - b.c1[2]};
  if (b.kind == ELBM_BODY_SPHERE) {
    const double dv = d[0] * v[0] + d[1] * v[1] + d[2] * v[2];
    const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] - b.r2;
    double disc = dv * dv - vv * dd;
    disc = disc < 0.0 ? 0.0 : disc;
    q = dd / (dv + sqrt(disc));
  } else {
    const double nd = b.n[0] * d[0] + b.n[1] * d[1] + b.n[2] * d[2];
    const double nv = b.n[0] * v[0] + b.n[1] * v[1] + b.n[2] * v[2];
    q = nd / nv;
  }
  const double r[3] = {d[0] - q * v[0], d[1] - q * v[1], d[2] - q * v[2]};  // x_w - centre
  uw[0] = b.U1[0] + (b.omega[1] * r[2] - b.omega[2] * r[1]);
  uw[1] = b.U1[1] + (b.omega[2] * r[0] - b.omega[0] * r[2]);
  uw[2] = b.U1[2] + (b.omega[0] * r[1] - b.omega[1] * r[0]);
}

// Refill of a node uncovered at t+1 (Sec. III): Grad's distribution with the wall velocity of the
// body that held the node at t (taken at t+1), the mean R^t of the neighbours fluid at t and t+1
// (rho0 if none) and the pressure tensor with the finite-difference gradient of U^t.
__device__ inline void refill_pops(const BArgs& a, const Bodies& bd, int x, int y, int z, long n, float (&f)[27],
                                   int& kb, float& ravg, int& m, float (&uw)[3], float (&G)[9]) {
  kb = first_body(bd, false, x, y, z);
  if (kb < 0) kb = 0;
  const BodyDev& b = bd.b[kb];
  const double r[3] = {x - b.c1[0], y - b.c1[1], z - b.c1[2]};
  uw[0] = (float)(b.U1[0] + (b.omega[1] * r[2] - b.omega[2] * r[1]));
  uw[1] = (float)(b.U1[1] + (b.omega[2] * r[0] - b.omega[0] * r[2]));
  uw[2] = (float)(b.U1[2] + (b.omega[0] * r[1] - b.omega[1] * r[0]));
  float rs = 0.f;
  m = 0;
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    if (i == 13) continue;
    const long nn = neighbour(a, x, y, z, cx(i), cy(i), cz(i));
    if (nn < 0 || (a.flags[nn] & (FL_SOLID | FL_SOLID_PREV))) continue;
    rs += a.macro[3 * a.N + nn];
    ++m;
  }
  ravg = m ? rs / (float)m : (float)a.rho0;
  float Pi[6];
  grad_u(a, x, y, z, n, G);
  pressure_tensor(ravg, uw, G, a.beta, Pi);
#pragma unroll
  for (int i = 0; i < 27; ++i) f[i] = grad_pop(i, ravg, uw, Pi);
}

}  // namespace elbm
