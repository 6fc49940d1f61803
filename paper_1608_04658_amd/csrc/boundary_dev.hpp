// boundary_dev.hpp -- device helpers of the wall treatment (Sec. III) shared by the forward
// boundary kernel and its adjoint: node indexing, the previous-step velocity gradient stencil and
// the geometry of a boundary link.
#pragma once

#include "elbm_internal.hpp"
#include "lanes_dev.hpp"
#include "mesh_dev.hpp"

namespace elbm {

struct GeoArgs {
  uint8_t* flags;
  int32_t nx, ny, nz;
  int32_t channel;
  Box box;
};

// Node of linear index idx in a box (x fastest).  A box lies inside the lattice (< 2^31 nodes), so
// 32-bit divisions suffice (a 64-bit one is a long software sequence on the GPU).
__device__ __forceinline__ void box_node(const Box& b, long idx, int& x, int& y, int& z) {
  const uint32_t i = (uint32_t)idx, nx = (uint32_t)b.n[0], ny = (uint32_t)b.n[1];
  const uint32_t q = i / nx;
  x = b.lo[0] + (int)(i - q * nx);
  y = b.lo[1] + (int)(q % ny);
  z = b.lo[2] + (int)(q / ny);
}

// Two disjoint boxes walked by one launch (the body box and the inlet slab): index idx < count of
// the first lies in it, the rest in the second.
__device__ __forceinline__ void box2_node(const Box2& bb, long idx, int& x, int& y, int& z) {
  const long c0 = bb.b[0].count();
  if (idx < c0) box_node(bb.b[0], idx, x, y, z);
  else box_node(bb.b[1], idx - c0, x, y, z);
}

__device__ __forceinline__ int first_body(const Bodies& bd, bool at_t1, double x, double y, double z) {
  for (int k = 0; k < bd.nb; ++k)
    if (inside_body(bd.b[k], at_t1 ? bd.b[k].c1 : bd.b[k].c0, x, y, z)) return k;
  return -1;
}

// Body owning a node known to be solid: the first analytic body containing it, else the
// triangulated body (which comes last in the body array), else body 0.
__device__ __forceinline__ int owner_body(const Bodies& bd, bool at_t1, double x, double y, double z) {
  const int k = first_body(bd, at_t1, x, y, z);
  if (k >= 0) return k;
  return bd.mesh >= 0 ? bd.mesh : 0;
}

// Periodic index for any offset (stencils reach +-2, lattices may be 1 or 2 nodes thick); the
// integer division only where the offset exceeds one period.
__device__ __forceinline__ int wrap(int v, int n) {
  if (v >= 0 && v < n) return v;
  if (v < 0 && v + n >= 0) return v + n;
  if (v >= n && v - n < n) return v - n;
  return ((v % n) + n) % n;
}

struct BArgs {
  const void* A;
  void* B;
  const uint8_t* flags;
  const float* macro;  // U^t, R^t planes
  float* slab_next;    // channel mode: staging of U^{t+1}, R^{t+1} for x < 3 ([4][nz][ny][3])
  const float* F;
  const int32_t* list;
  const uint32_t* dyn_count;
  double* brec;
  uint32_t* fix_list;   // FP64 fix-up queue (wall nodes enter it tagged FIX_PRE)
  uint32_t* fix_count;  // its length for this step
  DevCounters* diag;    // failure flag and gamma range (k_boundary)
  int32_t stats;        // 1: record the gamma range
  int64_t n_static;
  int64_t lo, hi;  // k_boundary: list entries [lo, min(hi, count)) (hi < 0: to the end)
  int64_t cap;
  int32_t moving;
  int32_t nx, ny, nz;
  int64_t N;
  PopLayout lay;  // placement of the populations in A and B
  int32_t channel;
  int32_t fp64;
  int32_t stream_only;
  int32_t stab;  // STAB_* of the context
  float beta, inv_beta, thr;
  double beta64;  // beta in FP64 (the reverse step's arithmetic)
  double rho0;
  double u_in[3];
};

__device__ __forceinline__ long node_at(const BArgs& a, int x, int y, int z) {
  return ((long)z * a.ny + y) * a.nx + x;
}
// Coordinates of node n (n < 2^31: 32-bit divisions).
__device__ __forceinline__ void node_xyz(const BArgs& a, long n, int& x, int& y, int& z) {
  const uint32_t m = (uint32_t)n, nx = (uint32_t)a.nx, ny = (uint32_t)a.ny;
  const uint32_t r = m / nx;
  x = (int)(m - r * nx);
  y = (int)(r % ny);
  z = (int)(r / ny);
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

// Index of the direction (dx, dy, dz).
__host__ __device__ constexpr int dir_index(int dx, int dy, int dz) { return 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1); }

// ---------------------------------------------------------------------------------------------
// Lane-parallel form of the wall kernels (lanes_dev.hpp): one listed node per group of 32 lanes,
// lane i < 27 owns direction i, lanes 27..31 (and lane 13 for a sixth) fetch the nodes two steps
// away along the axes.  Per-direction work runs side by side across the lanes instead of as 27
// unrolled copies in one thread.
__host__ __device__ constexpr int far_lane(int k) { return k < 5 ? 27 + k : 13; }

__device__ __forceinline__ long far_node(const BArgs& a, int x, int y, int z, int k) {
  const int b = k >> 1, s = (k & 1) ? -2 : 2;
  return neighbour(a, x, y, z, b == 0 ? s : 0, b == 1 ? s : 0, b == 2 ? s : 0);
}
// Element of direction i pulled into node (x, y, z): the population at x - c_i (x clamped to the
// lattice in channel mode).
__device__ __forceinline__ int64_t pull_pop(const BArgs& a, int x, int y, int z, int i) {
  int sx = x - cx(i);
  if (a.channel) sx = sx >= a.nx ? a.nx - 1 : (sx < 0 ? 0 : sx);
  else sx = wrap(sx, a.nx);
  return pop_off(a.lay, i, sx, wrap(y - cy(i), a.ny), wrap(z - cz(i), a.nz));
}

// This lane's view of a listed node's neighbourhood; the masks are the same on every lane.
struct LaneNb {
  long n;
  int x, y, z;
  uint32_t fluid;   // bit i: x + c_i exists and is fluid at t+1 (i = 13: the node itself)
  uint32_t fluid0;  // bit i: x + c_i exists and is fluid at t and t+1
  uint32_t dbar;    // bit i: population i is missing (source solid at t+1 or beyond the inlet)
  uint32_t far;     // bit 2b: x + 2 e_b exists and is fluid at t+1; bit 2b+1: x - 2 e_b
  float f, fo;      // pulled deviation of direction lane (0 where missing); own deviation A_lane(x)
  float U[3];       // U^t at x + c_lane where fluid at t+1
  float V[3];       // U^t at the far node of this lane where fluid at t+1
  float R;          // R^t at x + c_lane where fluid at t and t+1
};

// All lanes of the group must call this together (it shuffles and ballots).
template <int S, bool POPS, bool RHO>
__device__ inline void lane_gather(const BArgs& a, const typename Codec<S>::E* A, long n, int lane, LaneNb& h) {
  using C = Codec<S>;
  h.n = n;
  int x, y, z;
  node_xyz(a, n, x, y, z);
  h.x = x;
  h.y = y;
  h.z = z;
  const bool own = lane < 27;
  const int i = own ? lane : 13;
  const long m = neighbour(a, x, y, z, cx(i), cy(i), cz(i));
  const int fk = lane >= 27 ? lane - 27 : (lane == 13 ? 5 : -1);
  const long mf = fk >= 0 ? far_node(a, x, y, z, fk) : -1;
  const uint8_t fl = m >= 0 ? a.flags[m] : FL_SOLID;
  const uint8_t ff = mf >= 0 ? a.flags[mf] : FL_SOLID;
  h.fluid = gballot(own && m >= 0 && !(fl & FL_SOLID));
  h.fluid0 = gballot(own && m >= 0 && !(fl & (FL_SOLID | FL_SOLID_PREV)));
  const uint32_t fb = gballot(fk >= 0 && !(ff & FL_SOLID));
  h.far = ((fb >> 27) & 31u) | (((fb >> 13) & 1u) << 5);
  // source of direction i: the neighbour in direction opp(i), or (0, -cy, -cz) where the outlet
  // clamps x; through the inlet it is missing
  const int sx = x - cx(i);
  const int s = (a.channel && sx >= a.nx) ? dir_index(0, -cy(i), -cz(i)) : opp(i);
  const int fls = __shfl((int)fl, s, GROUP);
  const bool miss = own && ((a.channel && sx < 0) || (fls & FL_SOLID));
  h.dbar = gballot(miss);
  h.f = 0.f;
  h.fo = 0.f;
  if (POPS && own) {
    h.fo = C::load_dev(A + pop_off(a.lay, i, x, y, z));
    if (!miss) h.f = C::load_dev(A + pull_pop(a, x, y, z, i));
  }
  const bool uf = own && ((h.fluid >> i) & 1u);
#pragma unroll
  for (int c = 0; c < 3; ++c) h.U[c] = uf ? a.macro[c * a.N + m] : 0.f;
  const bool vf = fk >= 0 && ((h.far >> fk) & 1u);
#pragma unroll
  for (int c = 0; c < 3; ++c) h.V[c] = vf ? a.macro[c * a.N + mf] : 0.f;
  h.R = (RHO && own && ((h.fluid0 >> i) & 1u)) ? a.macro[3 * a.N + m] : 0.f;
}

// grad_u on the group's gathered stencil (same rule and arithmetic); every lane gets G.
__device__ inline void grad_u_grp(const LaneNb& h, float (&G)[9]) {
  float u0[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) u0[c] = __shfl(h.U[c], 13, GROUP);
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int ip = dir_index(b == 0, b == 1, b == 2), im = dir_index(-(b == 0), -(b == 1), -(b == 2));
    const bool op1 = (h.fluid >> ip) & 1u, om1 = (h.fluid >> im) & 1u;
    const bool op2 = (h.far >> (2 * b)) & 1u, om2 = (h.far >> (2 * b + 1)) & 1u;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float up1 = __shfl(h.U[c], ip, GROUP), um1 = __shfl(h.U[c], im, GROUP);
      const float up2 = __shfl(h.V[c], far_lane(2 * b), GROUP), um2 = __shfl(h.V[c], far_lane(2 * b + 1), GROUP);
      float d;
      if (op1 && om1) d = 0.5f * (up1 - um1);
      else if (op1 && op2) d = 0.5f * (-3.f * u0[c] + 4.f * up1 - up2);
      else if (om1 && om2) d = 0.5f * (3.f * u0[c] - 4.f * um1 + um2);
      else if (op1) d = up1 - u0[c];
      else if (om1) d = u0[c] - um1;
      else d = 0.f;
      G[3 * c + b] = d;
    }
  }
}

// Geometry of boundary link i (i in Dbar) at node (x,y,z): link fraction q, wall velocity u_w and
// owning body (-1 for the inlet wall at x = -1/2).  q is the ray parameter where x - s c_i meets
// the surface (FP64): sphere (|d|^2 - R^2)/(d.c_i + sqrt((d.c_i)^2 - |c_i|^2 (|d|^2 - R^2))),
// plane n.d / n.c_i, d = x - centre(t+1).
// MESH: the body set may hold a triangulated body (a separate instantiation keeps its register
// cost out of the analytic-body kernels).
template <bool MESH>
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
  kb = MESH ? owner_body(bd, true, sx, sy, sz) : max(first_body(bd, true, sx, sy, sz), 0);
  const BodyDev& b = bd.b[kb];
  if (MESH && b.kind == ELBM_BODY_MESH) {
    const double xb[3] = {(double)x, (double)y, (double)z};
    mesh_link(bd.m, xb, i, q, uw);
    return;
  }
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
  double U1[3], W1[3];
  body_U1(bd, kb, U1);
  body_W1(bd, kb, W1);
  uw[0] = U1[0] + (W1[1] * r[2] - W1[2] * r[1]);
  uw[1] = U1[1] + (W1[2] * r[0] - W1[0] * r[2]);
  uw[2] = U1[2] + (W1[0] * r[1] - W1[1] * r[0]);
}

// Reconstruction at a wall node in the lane-parallel form (Sec. III): this lane's link (when its
// population is missing), the group's targets rho_tgt = rho_stat + rho_dyn and u_tgt, the
// finite-difference gradient of U^t, the pressure tensor, and this lane's Grad population.
// All lanes of the group call it together (uniform dmask != 0).
struct WallLane {
  bool mine;     // this lane's population is missing
  double q;      // link fraction (mine)
  double uw[3];  // wall velocity at the link (mine)
  int kb;        // body of the link, -1 for the inlet (mine)
  float fb;      // bounce-back value: deviation of A^t_{opp(lane)}(x)
  float fs;      // Grad population f*_lane (absolute; mine)
  float rt;      // rho_tgt
  float ut[3];   // u_tgt
  float G[9];    // grad U^t
  float Pi[6];   // pressure tensor
  int nD;        // number of missing populations
};

template <bool MESH>
__device__ inline void wall_targets(const BArgs& a, const Bodies& bd, const LaneNb& h, int lane, WallLane& w) {
  const int i = lane < 27 ? lane : 13;
  w.mine = lane < 27 && ((h.dbar >> lane) & 1u);
  w.q = 0.0;
  w.uw[0] = w.uw[1] = w.uw[2] = 0.0;
  w.kb = -1;
  if (w.mine) link_geometry<MESH>(a, bd, i, h.x, h.y, h.z, w.q, w.uw, w.kb);
  w.fb = __shfl(h.fo, opp(i), GROUP);
  float tu[3] = {0.f, 0.f, 0.f}, trs = 0.f, trd = 0.f;
  if (w.mine) {
    const bool fluid = (h.fluid >> lane) & 1u;
    const float qf = (float)w.q, inv = 1.f / (1.f + qf);
#pragma unroll
    for (int c = 0; c < 3; ++c) tu[c] = (qf * (fluid ? h.U[c] : (float)w.uw[c]) + (float)w.uw[c]) * inv;
    trs = w.fb;
    trd = (float)(6.0 * wd(i) * a.rho0 * (cx(i) * w.uw[0] + cy(i) * w.uw[1] + cz(i) * w.uw[2]));
  } else if (lane < 27) {
    trs = h.f;
  }
  const float rstat = gsum(trs), rdyn = gsum(trd);  // rstat: sum of deviations (weights add to 1)
  w.nD = __popc(h.dbar);
  const float invn = 1.f / (float)w.nD;
#pragma unroll
  for (int c = 0; c < 3; ++c) w.ut[c] = gsum(tu[c]) * invn;
  w.rt = 1.f + rstat + rdyn;
  grad_u_grp(h, w.G);
  pressure_tensor(w.rt, w.ut, w.G, a.beta, w.Pi);
  w.fs = w.mine ? grad_pop(i, w.rt, w.ut, w.Pi) : 0.f;
}

}  // namespace elbm
