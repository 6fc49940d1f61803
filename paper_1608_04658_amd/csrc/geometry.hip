// geometry.hip -- moving-wall boundary treatment of the KBC step on gfx950 (Sec. III):
// solid masks, the compacted list of boundary and refill nodes, the previous-step macroscopic
// field, reconstruction of the missing populations with Grad's distribution at target values
// (eqs. grad, pressure, pressure2), refill of uncovered nodes, and the momentum-exchange force
// (Sec. IV.A).
//
// The boundary work touches a few thousand nodes per step.  It runs in its own kernels over a
// compacted node list so that the bulk sweep keeps its register budget and its wavefronts stay
// convergent; the bulk sweep skips every flagged node.  Force sums are deterministic: each list
// entry writes its own FP64 record and a separate kernel reduces the records in list order.
#include <math.h>

#include <algorithm>
#include <stdio.h>

#include "context.hpp"
#include "boundary_dev.hpp"

namespace elbm {

constexpr int BOX_MARGIN = 5;

BArgs boundary_args(elbm_ctx* c, const void* A, void* B);

// ---------------------------------------------------------------------------------------------
// Host kinematics, FP64, in the order written in elbm.h.
void host_kinematics(const elbm_body& b, double t, double c[3], double U[3]) {
#pragma clang fp contract(off)
  double sn = 0.0, cs = 0.0, om = 0.0;
  if (b.period != 0.0) {
    const double ph = ((2.0 * M_PI) * t) / b.period;
    sn = sin(ph);
    cs = cos(ph);
    om = (2.0 * M_PI) / b.period;
  }
  for (int a = 0; a < 3; ++a) {
    c[a] = b.center[a] + (b.amp * sn) * b.dir[a] + b.vel[a] * t;
    U[a] = (b.amp * om * cs) * b.dir[a] + b.vel[a];
  }
}

Bodies make_bodies(const elbm_ctx* c, double t) {
  Bodies bd;
  bd.nb = c->nb;
  bd.mesh = c->mesh_body;
  bd.m = MeshDev{};
  if (c->mesh_body >= 0) {
    // level t in slot mesh_cur; level t+1 in the other slot once elbm_mesh_next supplied it
    const int s0 = c->mesh_cur, s1 = c->mesh_next_set ? c->mesh_cur ^ 1 : c->mesh_cur;
    bd.m = c->mesh_grid;
    bd.m.tri = c->mesh_tri;
    bd.m.nt = c->mesh_nt;
    const int sl[2] = {s0, s1};
    for (int l = 0; l < 2; ++l) {
      bd.m.lv[l].X = c->mesh_X[sl[l]];
      bd.m.lv[l].V = c->mesh_V[sl[l]];
      bd.m.lv[l].start = c->mesh_start[sl[l]];
      bd.m.lv[l].items = c->mesh_items[sl[l]];
    }
  }
  for (int k = 0; k < c->nb; ++k) {
    const elbm_body& b = c->bodies[k];
    BodyDev& d = bd.b[k];
    d.kind = b.kind;
    d.pad = 0;
    if (b.kind == ELBM_BODY_MESH) {
      const int s1 = c->mesh_next_set ? c->mesh_cur ^ 1 : c->mesh_cur;
      for (int a = 0; a < 3; ++a) {
        d.c0[a] = c->mesh_ref[c->mesh_cur][a];
        d.c1[a] = c->mesh_ref[s1][a];
        d.U0[a] = d.U1[a] = 0.0;
        d.n[a] = d.omega[a] = 0.0;
      }
      d.radius = 0.0;
      d.r2 = 0.0;
      continue;
    }
    if (c->freeb[k].on) {
      // explicit Euler of Newton's equations: position and velocity at t (fb.xt, fb.ut, derived
      // by the step loop), position at t+1; the velocity at t+1 is the device integrator's
      const auto& fb = c->freeb[k];
      for (int a = 0; a < 3; ++a) {
        d.c0[a] = fb.xt[a];
        d.U0[a] = fb.ut[a];
        d.c1[a] = fb.xt[a] + fb.ut[a];
        d.U1[a] = 0.0;
      }
    } else {
      host_kinematics(b, t, d.c0, d.U0);
      host_kinematics(b, t + 1.0, d.c1, d.U1);
    }
    d.radius = b.radius;
    d.r2 = b.radius * b.radius;
    for (int a = 0; a < 3; ++a) {
      d.n[a] = b.normal[a];
      // a free body's angular velocity at t (its value at t+1 comes from the device integrator)
      d.omega[a] = c->freeb[k].on ? c->freeb[k].wt[a] : b.omega[a];
    }
  }
  for (int k = c->nb; k < ELBM_MAX_BODIES; ++k) bd.b[k] = BodyDev{};
  bd.U1dev = c->free_U1;
  bd.W1dev = c->free_U1 + 3 * ELBM_MAX_BODIES;
  bd.free_mask = 0;
  for (int k = 0; k < c->nb; ++k)
    if (c->freeb[k].on) bd.free_mask |= 1u << k;
  bd.pad2 = 0;
  return bd;
}

// Axis-aligned box covering every body at t and t+1 plus a margin (the whole axis when the box
// would cross a periodic face, or for planes not normal to an axis).
Box union_box(const elbm_ctx* c, const Bodies& bd) {
  const int dims[3] = {c->p.nx, c->p.ny, c->p.nz};
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  bool full[3] = {false, false, false};
  for (int k = 0; k < bd.nb; ++k) {
    const BodyDev& b = bd.b[k];
    if (b.kind == ELBM_BODY_MESH) {
      for (int a = 0; a < 3; ++a) {
        lo[a] = fmin(lo[a], c->mesh_lo[a] - BOX_MARGIN);
        hi[a] = fmax(hi[a], c->mesh_hi[a] + BOX_MARGIN);
      }
    } else if (b.kind == ELBM_BODY_SPHERE) {
      for (int a = 0; a < 3; ++a) {
        lo[a] = fmin(lo[a], fmin(b.c0[a], b.c1[a]) - b.radius - BOX_MARGIN);
        hi[a] = fmax(hi[a], fmax(b.c0[a], b.c1[a]) + b.radius + BOX_MARGIN);
      }
    } else {
      int axis = -1;
      for (int a = 0; a < 3; ++a)
        if (fabs(b.n[a]) == 1.0) axis = a;
      for (int a = 0; a < 3; ++a) {
        if (a == axis) {
          lo[a] = fmin(lo[a], fmin(b.c0[a], b.c1[a]) - BOX_MARGIN);
          hi[a] = fmax(hi[a], fmax(b.c0[a], b.c1[a]) + BOX_MARGIN);
        } else {
          full[a] = true;
        }
      }
    }
  }
  Box box;
  for (int a = 0; a < 3; ++a) {
    int l = (int)floor(lo[a]), h = (int)ceil(hi[a]);
    const bool periodic = !(a == 0 && c->p.bc_x == ELBM_BC_CHANNEL);
    if (full[a] || bd.nb == 0) {
      l = 0;
      h = dims[a] - 1;
    } else if (l < 0 || h > dims[a] - 1) {
      if (periodic) {
        l = 0;
        h = dims[a] - 1;
      } else {
        l = l < 0 ? 0 : l;
        h = h > dims[a] - 1 ? dims[a] - 1 : h;
      }
    }
    box.lo[a] = l;
    box.n[a] = h - l + 1;
    if (box.n[a] < 1) box.n[a] = 1;
  }
  return box;
}

// The boxes where the wall rules read U^t and R^t: around the bodies and, with slab in channel
// mode, the inlet slab x < 3 (the body box without the slab's columns, so the two are disjoint).
Box2 macro_boxes(const elbm_ctx* c, const Bodies& bd, bool slab) {
  Box2 bb;
  Box sl = full_box(c);
  sl.n[0] = 0;
  if (slab && c->p.bc_x == ELBM_BC_CHANNEL) sl.n[0] = c->p.nx < 3 ? c->p.nx : 3;
  Box ub = full_box(c);
  ub.n[0] = 0;
  if (c->nb > 0) {
    ub = union_box(c, bd);
    const int cut = sl.n[0] - ub.lo[0];  // columns of the body box inside the slab
    if (cut > 0) {
      ub.lo[0] += cut;
      ub.n[0] = ub.n[0] > cut ? ub.n[0] - cut : 0;
    }
  }
  bb.b[0] = ub;
  bb.b[1] = sl;
  return bb;
}

Box full_box(const elbm_ctx* c) {
  Box b;
  b.lo[0] = b.lo[1] = b.lo[2] = 0;
  b.n[0] = c->p.nx;
  b.n[1] = c->p.ny;
  b.n[2] = c->p.nz;
  return b;
}

// Masks at a single time level (set-up): solid at t and "t+1" alike.
__global__ void k_flags_init(GeoArgs g, Bodies bd) {
  const long total = g.box.count();
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    int x, y, z;
    box_node(g.box, idx, x, y, z);
    const long n = ((long)z * g.ny + y) * g.nx + x;
    const bool s = first_body(bd, false, x, y, z) >= 0;
    g.flags[n] = s ? (FL_SOLID | FL_SOLID_PREV) : 0;
  }
}

// Advance masks t -> t+1 inside the box: previous <- current, current <- inside at t+1.
__global__ void k_flags_update(GeoArgs g, Bodies bd) {
  const long total = g.box.count();
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    int x, y, z;
    box_node(g.box, idx, x, y, z);
    const long n = ((long)z * g.ny + y) * g.nx + x;
    const uint8_t old = g.flags[n];
    const bool s1 = first_body(bd, true, x, y, z) >= 0;
    uint8_t nf = old & (uint8_t)~(FL_SOLID | FL_SOLID_PREV);
    if (old & FL_SOLID) nf |= FL_SOLID_PREV;
    if (s1) nf |= FL_SOLID;
    g.flags[n] = nf;
  }
}

// Missing set Dbar is non-empty (a source x - c_i is solid at t+1, or lies through the inlet) or
// the node was solid at t (refill).  The 26 flag loads are independent (no early exit).
__device__ __forceinline__ bool is_boundary(const GeoArgs& g, int x, int y, int z, uint8_t fl) {
  if (fl & FL_SOLID) return false;
  if (fl & FL_SOLID_PREV) return true;
  if (g.channel && x == 0) return true;
  uint8_t acc = 0;
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    if (i == 13) continue;
    int sx = x - cx(i);
    if (g.channel) sx = sx >= g.nx ? g.nx - 1 : sx;
    else sx = sx < 0 ? sx + g.nx : (sx >= g.nx ? sx - g.nx : sx);
    const int ty = y - cy(i), tz = z - cz(i);
    const int sy = ty < 0 ? ty + g.ny : (ty >= g.ny ? ty - g.ny : ty);
    const int sz = tz < 0 ? tz + g.nz : (tz >= g.nz ? tz - g.nz : tz);
    acc |= g.flags[((long)sz * g.ny + sy) * g.nx + sx];
  }
  return (acc & FL_SOLID) != 0;
}

// Ordered compaction of the boundary nodes of a box (deterministic: the box's linear order), in
// three passes: mark + per-block counts, one-block exclusive scan of the counts, emit (two for small
// boxes: k_scan_emit_fused).  Sets
// FL_SPECIAL on listed nodes and clears it on the other box nodes; with skip_inlet the x = 0 face
// keeps its flags and is not listed (it sits in the static part of the list).
constexpr int SCAN_BLOCK = 256;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t& total) {
  return block_scan_inclusive<SCAN_BLOCK / 64>(v, sh, total) - v;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_mark(GeoArgs g, int skip_inlet, uint32_t* block_count) {
  __shared__ uint32_t sh[SCAN_BLOCK / 64];
  const long idx = blockIdx.x * (long)SCAN_BLOCK + threadIdx.x;
  uint32_t isb = 0;
  if (idx < g.box.count()) {
    int x, y, z;
    box_node(g.box, idx, x, y, z);
    const long n = ((long)z * g.ny + y) * g.nx + x;
    if (!(skip_inlet && g.channel && x == 0)) {
      const uint8_t fl = g.flags[n];
      isb = is_boundary(g, x, y, z, fl) ? 1u : 0u;
      const uint8_t nf = isb ? (uint8_t)(fl | FL_SPECIAL) : (uint8_t)(fl & ~FL_SPECIAL);
      if (nf != fl) g.flags[n] = nf;
    }
  }
  uint32_t total;
  block_exclusive_scan(isb, sh, total);
  if (threadIdx.x == 0) block_count[blockIdx.x] = total;
}

// One workgroup: block_offset = exclusive scan of block_count; *count_out = total.
__global__ __launch_bounds__(1024) void k_scan_offsets(const uint32_t* block_count, uint32_t* block_offset, long nblk,
                                                       int64_t base, int64_t cap, uint32_t* count_out,
                                                       uint32_t* overflow) {
  __shared__ uint32_t wsum[16];
  uint32_t running = 0;
  for (long start = 0; start < nblk; start += 1024) {
    const long i = start + threadIdx.x;
    const uint32_t v = i < nblk ? block_count[i] : 0u;
    uint32_t total;
    const uint32_t incl = scan1024_inclusive(v, wsum, total);
    if (i < nblk) block_offset[i] = running + incl - v;
    running += total;
  }
  if (threadIdx.x == 0) {
    *count_out = running;
    if (base + (int64_t)running > cap) atomicOr(overflow, 1u);
  }
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_emit(GeoArgs g, int skip_inlet, const uint32_t* block_offset,
                                                          int32_t* list, int64_t base, int64_t cap) {
  __shared__ uint32_t sh[SCAN_BLOCK / 64];
  const long idx = blockIdx.x * (long)SCAN_BLOCK + threadIdx.x;
  uint32_t isb = 0;
  long n = 0;
  if (idx < g.box.count()) {
    int x, y, z;
    box_node(g.box, idx, x, y, z);
    n = ((long)z * g.ny + y) * g.nx + x;
    isb = (!(skip_inlet && g.channel && x == 0) && (g.flags[n] & FL_SPECIAL)) ? 1u : 0u;
  }
  uint32_t total;
  const uint32_t ex = block_exclusive_scan(isb, sh, total);
  if (isb) {
    const int64_t pos = base + (int64_t)block_offset[blockIdx.x] + ex;
    if (pos < cap) list[pos] = (int32_t)n;
  }
}

// Emit pass for boxes of at most SCAN_FUSED blocks, which saves the one-workgroup pass: each
// workgroup sums the counts of the blocks before it itself (at most SCAN_FUSED / SCAN_BLOCK loads per
// thread), and the last one stores the total and the overflow bit.
constexpr long SCAN_FUSED = 2048;

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_emit_fused(GeoArgs g, int skip_inlet, const uint32_t* block_count,
                                                                int32_t* list, int64_t base, int64_t cap,
                                                                uint32_t* count_out, uint32_t* overflow) {
  __shared__ uint32_t sh[SCAN_BLOCK / 64];
  uint32_t part = 0;
  for (long j = threadIdx.x; j < (long)blockIdx.x; j += SCAN_BLOCK) part += block_count[j];
  uint32_t prefix;
  block_exclusive_scan(part, sh, prefix);  // the workgroup's sum: the counts of all earlier blocks
  const long idx = blockIdx.x * (long)SCAN_BLOCK + threadIdx.x;
  uint32_t isb = 0;
  long n = 0;
  if (idx < g.box.count()) {
    int x, y, z;
    box_node(g.box, idx, x, y, z);
    n = ((long)z * g.ny + y) * g.nx + x;
    isb = (!(skip_inlet && g.channel && x == 0) && (g.flags[n] & FL_SPECIAL)) ? 1u : 0u;
  }
  uint32_t total;
  const uint32_t ex = block_exclusive_scan(isb, sh, total);
  if (isb) {
    const int64_t pos = base + (int64_t)prefix + ex;
    if (pos < cap) list[pos] = (int32_t)n;
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    const uint32_t all = prefix + total;
    *count_out = all;
    if (base + (int64_t)all > cap) atomicOr(overflow, 1u);
  }
}

// Previous-step macroscopic field U^t, R^t on a box: moments of A^t with U = (j - F/2)/rho at
// nodes fluid at t; rigid-body velocity (R = rho0) at nodes solid at t.
template <int S, bool MESH>
__global__ void k_macro(const typename Codec<S>::E* A, PopLayout lay, const uint8_t* flags, float* macro, const float* F,
                        Box2 box, int32_t nx, int32_t ny, int64_t N, double rho0, Bodies bd) {
  using C = Codec<S>;
  const long total = box.count();
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    int x, y, z;
    box2_node(box, idx, x, y, z);
    const long n = ((long)z * ny + y) * nx + x;
    float U[3], R;
    if (flags[n] & FL_SOLID_PREV) {
      const int k = MESH ? owner_body(bd, false, x, y, z) : max(first_body(bd, false, x, y, z), 0);
      const BodyDev& b = bd.b[k];
      if (MESH && b.kind == ELBM_BODY_MESH) {
        // U^t of a node solid at t is read only once the node is fluid at t+1 (finite differences
        // and u_f use nodes fluid at t+1): k_mesh_uncovered writes it at the uncovered nodes
        U[0] = U[1] = U[2] = 0.f;
      } else {
        const double r[3] = {x - b.c0[0], y - b.c0[1], z - b.c0[2]};
        U[0] = (float)(b.U0[0] + (b.omega[1] * r[2] - b.omega[2] * r[1]));
        U[1] = (float)(b.U0[1] + (b.omega[2] * r[0] - b.omega[0] * r[2]));
        U[2] = (float)(b.U0[2] + (b.omega[0] * r[1] - b.omega[1] * r[0]));
      }
      R = (float)rho0;
    } else {
      float dr = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;  // from the stored deviations f - W
#pragma unroll
      for (int i = 0; i < 27; ++i) {
        const float v = C::load_dev(A + pop_off(lay, i, x, y, z));
        dr += v;
        jx += cx(i) * v;
        jy += cy(i) * v;
        jz += cz(i) * v;
      }
      const float rho = 1.f + dr;
      if (F) {
        jx -= 0.5f * F[n];
        jy -= 0.5f * F[N + n];
        jz -= 0.5f * F[2 * N + n];
      }
      U[0] = jx / rho;
      U[1] = jy / rho;
      U[2] = jz / rho;
      R = rho;
    }
    macro[n] = U[0];
    macro[N + n] = U[1];
    macro[2 * N + n] = U[2];
    macro[3 * N + n] = R;
  }
}

// U^t at the nodes the triangulated body uncovers in this step (solid at t, fluid at t+1; all in
// the dynamic list): the velocity of the closest surface point at t, one node per group of lanes.
__global__ __launch_bounds__(64) void k_mesh_uncovered(const BArgs a, const Bodies bd, float* macro) {
  int64_t count = a.n_static + (int64_t)*a.dyn_count;
  if (count > a.cap) count = a.cap;
  const int lane = threadIdx.x & (GROUP - 1), g = threadIdx.x / GROUP;
  for (int64_t k = a.n_static + 2 * (int64_t)blockIdx.x + g; k < count; k += 2 * (int64_t)gridDim.x) {
    const long n = a.list[k];
    const uint8_t fl = a.flags[n];
    if (!(fl & FL_SOLID_PREV) || (fl & FL_SOLID)) continue;  // uniform over the group
    int x, y, z;
    node_xyz(a, n, x, y, z);
    if (owner_body(bd, false, x, y, z) != bd.mesh) continue;
    const double p[3] = {(double)x, (double)y, (double)z};
    double v[3];
    mesh_closest_velocity_group(bd.m, 0, p, lane, v);
    if (lane == 0)
      for (int c = 0; c < 3; ++c) macro[c * a.N + n] = (float)v[c];
  }
}

// ---------------------------------------------------------------------------------------------
// Refill before streaming: the uncovered nodes of the step get their Grad populations written into
// the current buffer A^t, where their neighbours (and the node itself) pull them.  One node per
// group of 32 lanes; only the dynamic (body) part of the list can hold uncovered nodes.
template <int S, bool MESH>
__global__ __launch_bounds__(64) void k_refill(const BArgs a, const Bodies bd, void* Aw) {
  using C = Codec<S>;
  using E = typename C::E;
  E* __restrict__ A = (E*)Aw;
  int64_t count = a.n_static + (a.moving ? (int64_t)*a.dyn_count : 0);
  if (count > a.cap) count = a.cap;
  const int lane = threadIdx.x & (GROUP - 1), g = threadIdx.x / GROUP;
  for (int64_t k = a.n_static + 2 * (int64_t)blockIdx.x + g; k < count; k += 2 * (int64_t)gridDim.x) {
    const long n = a.list[k];
    if (!(a.flags[n] & FL_SOLID_PREV)) continue;  // uniform over the group
    LaneNb h;
    lane_gather<S, false, true>(a, A, n, lane, h);
    const int kb = MESH ? owner_body(bd, false, h.x, h.y, h.z) : max(first_body(bd, false, h.x, h.y, h.z), 0);
    const BodyDev& b = bd.b[kb];
    float uw[3];
    if (MESH && b.kind == ELBM_BODY_MESH) {
      // the body's velocity at the node: that of the closest surface point at t+1 (candidate
      // triangles shared out over the group's lanes)
      const double p[3] = {(double)h.x, (double)h.y, (double)h.z};
      double v[3];
      mesh_closest_velocity_group(bd.m, 1, p, lane, v);
      for (int a = 0; a < 3; ++a) uw[a] = (float)v[a];
    } else {
      const double r[3] = {h.x - b.c1[0], h.y - b.c1[1], h.z - b.c1[2]};
      double U1[3], W1[3];
      body_U1(bd, kb, U1);
      body_W1(bd, kb, W1);
      uw[0] = (float)(U1[0] + (W1[1] * r[2] - W1[2] * r[1]));
      uw[1] = (float)(U1[1] + (W1[2] * r[0] - W1[0] * r[2]));
      uw[2] = (float)(U1[2] + (W1[0] * r[1] - W1[1] * r[0]));
    }
    const uint32_t nbm = h.fluid0 & ~(1u << 13);
    const float rs = gsum(lane != 13 ? h.R : 0.f);
    const int m = __popc(nbm);
    const float ravg = m ? rs / (float)m : (float)a.rho0;
    float G[9], Pi[6];
    grad_u_grp(h, G);
    pressure_tensor(ravg, uw, G, a.beta, Pi);
    if (lane < 27) C::store(A + pop_off(a.lay, lane, h.x, h.y, h.z), grad_pop(lane, ravg, uw, Pi), wf(lane));
  }
}

// Wall nodes (Sec. III): Grad reconstruction of the missing populations, the momentum exchange of
// each link (Sec. IV.A), then the KBC collision of the node.  One node per group of 32 lanes, one
// direction per lane, sums over directions as butterfly reductions.
template <int S, bool FORCE, int STAB, bool MESH>
__global__ __launch_bounds__(64) void k_boundary(const BArgs a, const Bodies bd) {
  using C = Codec<S>;
  using E = typename C::E;
  const E* __restrict__ A = (const E*)a.A;
  E* __restrict__ B = (E*)a.B;
  __shared__ float sh[2][GROUP];
  int64_t count = a.n_static + (a.moving ? (int64_t)*a.dyn_count : 0);
  if (count > a.cap) count = a.cap;
  if (a.hi >= 0 && count > a.hi) count = a.hi;
  const int nb = bd.nb;
  const int lane = threadIdx.x & (GROUP - 1), g = threadIdx.x / GROUP;
  const int i = lane < 27 ? lane : 13;
  for (int64_t base = a.lo + 2 * (int64_t)blockIdx.x; base < count; base += 2 * (int64_t)gridDim.x) {
    // the loop is uniform over the block (barriers below); a group past the end repeats the
    // block's first node and stores nothing
    const int64_t k = base + g;
    const bool active = k < count;
    const long n = a.list[active ? k : base];
    LaneNb h;
    lane_gather<S, true, false>(a, A, n, lane, h);
    double* rec = a.brec + k * nb * 6;
    // f holds deviations from the weights throughout, so that pulled populations pass through
    // unchanged in every storage form
    float fi = h.f;
    const uint32_t dmask = h.dbar;
    if (dmask) {  // missing populations at a wall (Sec. III); uniform over the group
      WallLane w;
      wall_targets<MESH>(a, bd, h, lane, w);
      double dF[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      if (w.mine) {
        fi = w.fs - wf(i);
        if (w.kb >= 0) {
          // Galilean-invariant momentum exchange of the link
          const double fbd = wd(opp(i)) + (double)w.fb;
          const double c[3] = {(double)cx(i), (double)cy(i), (double)cz(i)};
#pragma unroll
          for (int e = 0; e < 3; ++e) dF[e] = fbd * (-c[e] - w.uw[e]) - (double)w.fs * (c[e] - w.uw[e]);
          const BodyDev& b = bd.b[w.kb];
          const double r[3] = {h.x - w.q * c[0] - b.c1[0], h.y - w.q * c[1] - b.c1[1], h.z - w.q * c[2] - b.c1[2]};
          dF[3] = r[1] * dF[2] - r[2] * dF[1];
          dF[4] = r[2] * dF[0] - r[0] * dF[2];
          dF[5] = r[0] * dF[1] - r[1] * dF[0];
        }
      }
      if (gballot(w.mine && w.kb >= 0)) {  // uniform over the group; inlet-only nodes skip the sums
        for (int bb = 0; bb < nb; ++bb) {
#pragma unroll
          for (int e = 0; e < 6; ++e) {
            const double v = gsum(w.kb == bb ? dF[e] : 0.0);
            if (active && lane == e) rec[bb * 6 + e] = v;
          }
        }
      } else if (active) {
        for (int jj = lane; jj < nb * 6; jj += GROUP) rec[jj] = 0.0;
      }
    } else if (active) {
      for (int j = lane; j < nb * 6; j += GROUP) rec[j] = 0.0;
    }
    if (a.stream_only) {
      if (active && lane < 27) C::store_dev(B + pop_off(a.lay, lane, h.x, h.y, h.z), fi);
      continue;
    }
    float Fx = 0.f, Fy = 0.f, Fz = 0.f;
    if (FORCE) {
      Fx = a.F[n];
      Fy = a.F[a.N + n];
      Fz = a.F[2 * a.N + n];
    }
    KbcOut<float> r;
    const float fpost = kbc_collide_lanes<float, FORCE, STAB>(lane, fi, a.beta, a.inv_beta, Fx, Fy, Fz, r);
    // <dh|dh> at the FP32 noise floor (equal on all lanes of the group): store the pre-collision
    // deviations and queue the node for the FP64 collision of k_fixup
    const bool fp64 = a.fp64 && needs_fp64(r, a.thr);
    if (active && lane == 0) {
      // failure detection and the gamma range (r is equal on all lanes of the group)
      if (!r.dom) atomicOr(&a.diag->nonfinite, 2u);
      if (a.stats) {
        atomicMin(&a.diag->gamma_lo, f32_key(r.gamma));
        atomicMax(&a.diag->gamma_hi, f32_key(r.gamma));
      }
    }
    if (active && lane < 27) C::store_dev(B + pop_off(a.lay, lane, h.x, h.y, h.z), fp64 ? fi : fpost);
    if (fp64 && active && lane == 0) a.fix_list[atomicAdd(a.fix_count, 1u)] = (uint32_t)n | FIX_PRE;
    // inlet slab: U, R of the new state, summed in direction order on the group's first lane
    sh[g][lane] = fpost;
    __syncthreads();
    if (lane == 0 && active && !fp64 && a.slab_next && h.x < 3) {
      float f[27];
#pragma unroll
      for (int q = 0; q < 27; ++q) f[q] = sh[g][q];
      macro_from_post<S, FORCE>(f, Fx, Fy, Fz, a.slab_next, (size_t)3 * a.ny * a.nz, slab_index(h.x, h.y, h.z, a.ny));
    }
    __syncthreads();
  }
}

// Deterministic per-body force sum in two levels: FORCE_PARTS workgroups each own a fixed
// contiguous range of list entries and reduce every (body, component) in a fixed order; one
// workgroup then adds the partial sums in order.
constexpr int FORCE_PARTS = 64;
__global__ __launch_bounds__(256) void k_force_partial(const double* brec, const uint32_t* dyn_count, int64_t n_static,
                                                       int64_t cap, int32_t moving, int32_t nb, double* partial) {
  __shared__ double sh[256];
  int64_t count = n_static + (moving ? (int64_t)*dyn_count : 0);
  if (count > cap) count = cap;
  const int64_t chunk = (count + FORCE_PARTS - 1) / FORCE_PARTS;
  const int64_t k0 = blockIdx.x * chunk, k1 = k0 + chunk < count ? k0 + chunk : count;
  for (int comp = 0; comp < nb * 6; ++comp) {
    double s = 0.0;
    for (int64_t k = k0 + threadIdx.x; k < k1; k += 256) s += brec[k * nb * 6 + comp];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (threadIdx.x < (unsigned)off) sh[threadIdx.x] += sh[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x * ELBM_MAX_BODIES * 6 + comp] = sh[0];
    __syncthreads();
  }
}

__global__ void k_force_final(const double* partial, int32_t nb, double* out) {
  const int comp = threadIdx.x;
  if (comp >= nb * 6) return;
  double s = 0.0;
  for (int p = 0; p < FORCE_PARTS; ++p) s += partial[p * ELBM_MAX_BODIES * 6 + comp];
  out[comp] = s;
}

// ---------------------------------------------------------------------------------------------
// Free bodies on the device (Sec. IV.A, explicit Euler with unit time step):
//   x(t+1) = x(t) + u(t),  u(t+1) = u(t) + F(t)/m + (1 - 1/density_ratio) g,
// F(t) the momentum-exchange force of the step that produced t.  The sums are written in the
// order of the host's derivation, so both sides agree bit for bit.
struct FreeParams {
  double m[ELBM_MAX_BODIES];
  double I[ELBM_MAX_BODIES];     // moment of inertia; 0 for a body that does not rotate freely
  double ab[ELBM_MAX_BODIES][3];
  FreeState s[ELBM_MAX_BODIES];  // k_free_write: the state to store
  uint32_t mask;
};

__device__ inline double euler_u(double u, double F, double m, double ab) {
#pragma clang fp contract(off)
  return u + F / m + ab;
}

__device__ inline double euler_w(double w, double M, double I) {
#pragma clang fp contract(off)
  return I > 0.0 ? w + M / I : w;
}

// State of one level from the host, and the velocities at the next level (U1 [MAX_BODIES][3]
// translational, then [MAX_BODIES][3] angular).
__global__ void k_free_write(FreeParams p, FreeState* slot, double* U1) {
  const int k = threadIdx.x;
  if (k >= ELBM_MAX_BODIES || !((p.mask >> k) & 1u)) return;
  slot[k] = p.s[k];
  for (int a = 0; a < 3; ++a) {
    U1[3 * k + a] = euler_u(p.s[k].u[a], p.s[k].F[a], p.m[k], p.ab[k][a]);
    U1[3 * ELBM_MAX_BODIES + 3 * k + a] = euler_w(p.s[k].w[a], p.s[k].M[a], p.I[k]);
  }
}

// After the step t -> t+1: the state of level t+1 from that of level t and the step's force (in
// the ring), and the velocity at t+2 for the next step.
__global__ void k_free_commit(FreeParams p, const FreeState* prev, FreeState* next, const double* force, double* U1) {
#pragma clang fp contract(off)
  const int k = threadIdx.x;
  if (k >= ELBM_MAX_BODIES || !((p.mask >> k) & 1u)) return;
  FreeState s;
  for (int a = 0; a < 3; ++a) {
    s.x[a] = prev[k].x[a] + prev[k].u[a];
    s.u[a] = euler_u(prev[k].u[a], prev[k].F[a], p.m[k], p.ab[k][a]);
    s.F[a] = force[6 * k + a];
    s.w[a] = euler_w(prev[k].w[a], prev[k].M[a], p.I[k]);
    s.M[a] = force[6 * k + 3 + a];
  }
  next[k] = s;
  for (int a = 0; a < 3; ++a) {
    U1[3 * k + a] = euler_u(s.u[a], s.F[a], p.m[k], p.ab[k][a]);
    U1[3 * ELBM_MAX_BODIES + 3 * k + a] = euler_w(s.w[a], s.M[a], p.I[k]);
  }
}

static FreeParams free_params(const elbm_ctx* c) {
  FreeParams p{};
  for (int k = 0; k < c->nb; ++k) {
    if (!c->freeb[k].on) continue;
    p.mask |= 1u << k;
    p.m[k] = c->freeb[k].m;
    p.I[k] = c->freeb[k].I;
    for (int a = 0; a < 3; ++a) {
      p.ab[k][a] = c->freeb[k].ab[a];
      p.s[k].x[a] = c->freeb[k].x[a];
      p.s[k].u[a] = c->freeb[k].u[a];
      p.s[k].F[a] = c->freeb[k].F[a];
      p.s[k].w[a] = c->freeb[k].w[a];
      p.s[k].M[a] = c->freeb[k].M[a];
    }
  }
  return p;
}

// The host copy (level free_lv) to the device ring, and the velocity at the next level.
hipError_t free_init(elbm_ctx* c) {
  if (!c->n_free) return hipSuccess;
  const FreeParams p = free_params(c);
  FreeState* slot = c->free_hist + (size_t)(c->free_lv % FREE_HIST) * ELBM_MAX_BODIES;
  hipLaunchKernelGGL(k_free_write, dim3(1), dim3(64), 0, c->stream, p, slot, c->free_U1);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(c->free_ev[c->free_lv % FREE_HIST], c->stream);
  return e;
}

// Integrate after the step c->t -> c->t + 1 (its force reduced into the ring).
hipError_t free_commit(elbm_ctx* c) {
  if (!c->n_free) return hipSuccess;
  const FreeParams p = free_params(c);
  const FreeState* prev = c->free_hist + (size_t)(c->t % FREE_HIST) * ELBM_MAX_BODIES;
  FreeState* next = c->free_hist + (size_t)((c->t + 1) % FREE_HIST) * ELBM_MAX_BODIES;
  const double* force = c->ring + (size_t)((c->t + 1) % c->p.force_ring) * ELBM_MAX_BODIES * 6;
  hipLaunchKernelGGL(k_free_commit, dim3(1), dim3(64), 0, c->stream, p, prev, next, force, c->free_U1);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(c->free_ev[(c->t + 1) % FREE_HIST], c->stream);
  return e;
}

// ---------------------------------------------------------------------------------------------
dim3 grid_for(long n) {
  long b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

static GeoArgs geo_args(elbm_ctx* c, const Box& box) {
  GeoArgs g;
  g.flags = c->flags;
  g.nx = c->p.nx;
  g.ny = c->p.ny;
  g.nz = c->p.nz;
  g.channel = c->p.bc_x == ELBM_BC_CHANNEL;
  g.box = box;
  return g;
}

template <int S>
static void macro_launch(elbm_ctx* c, const void* A, const Box2& box, const Bodies& bd) {
  if (bd.mesh >= 0)
    hipLaunchKernelGGL((k_macro<S, true>), grid_for(box.count()), dim3(256), 0, c->stream,
                       (const typename Codec<S>::E*)A, c->lay, (const uint8_t*)c->flags, c->macro, c->bodyforce, box, c->p.nx,
                       c->p.ny, (int64_t)c->N, c->p.rho0, bd);
  else
    hipLaunchKernelGGL((k_macro<S, false>), grid_for(box.count()), dim3(256), 0, c->stream,
                       (const typename Codec<S>::E*)A, c->lay, (const uint8_t*)c->flags, c->macro, c->bodyforce, box, c->p.nx,
                       c->p.ny, (int64_t)c->N, c->p.rho0, bd);
}

static void macro_box(elbm_ctx* c, const void* A, const Box2& box, const Bodies& bd) {
  switch (c->p.storage) {
    case ELBM_STORAGE_F32: macro_launch<ELBM_STORAGE_F32>(c, A, box, bd); break;
    case ELBM_STORAGE_F16: macro_launch<ELBM_STORAGE_F16>(c, A, box, bd); break;
    default: macro_launch<ELBM_STORAGE_BF16>(c, A, box, bd);
  }
}

// The inlet slab's U, R from the staging written by the previous step's producers.
__global__ void k_slab_copy(const float* slab, float* macro, int32_t nx, int32_t ny, int32_t nz, int64_t N) {
  const long per = 3L * ny * nz;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < 4 * per; k += (long)gridDim.x * blockDim.x) {
    const int c = (int)(k / per);
    const long r = k % per;
    const int x = (int)(r % 3), y = (int)((r / 3) % ny), z = (int)(r / (3L * ny));
    if (x < nx) macro[c * N + ((long)z * ny + y) * nx + x] = slab[k];
  }
}

// U^t, R^t of the populations A around the bodies and, with slab, on the inlet slab.
hipError_t macro_fields(elbm_ctx* c, const void* A, const Bodies& bd, bool slab) {
  const Box2 bb = macro_boxes(c, bd, slab);
  if (bb.count() > 0) macro_box(c, A, bb, bd);
  return hipGetLastError();
}

// Ordered compaction of the boundary nodes of box into list[base ...]; count to cnt->dyn_count.
static hipError_t scan_box(elbm_ctx* c, const Box& box, int64_t base, int skip_inlet) {
  const long nblk = (box.count() + SCAN_BLOCK - 1) / SCAN_BLOCK;
  if (nblk > c->scan_blocks) return hipErrorInvalidValue;
  uint32_t* counts = c->scan_tmp;
  uint32_t* offsets = c->scan_tmp + c->scan_blocks;
  const GeoArgs g = geo_args(c, box);
  hipLaunchKernelGGL(k_scan_mark, dim3((unsigned)nblk), dim3(SCAN_BLOCK), 0, c->stream, g, skip_inlet, counts);
  if (nblk >= 1 && nblk <= SCAN_FUSED) {
    hipLaunchKernelGGL(k_scan_emit_fused, dim3((unsigned)nblk), dim3(SCAN_BLOCK), 0, c->stream, g, skip_inlet,
                       (const uint32_t*)counts, c->blist, base, c->blist_cap, &c->cnt->dyn_count, &c->cnt->overflow);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(1024), 0, c->stream, (const uint32_t*)counts, offsets, nblk, base,
                     c->blist_cap, &c->cnt->dyn_count, &c->cnt->overflow);
  hipLaunchKernelGGL(k_scan_emit, dim3((unsigned)nblk), dim3(SCAN_BLOCK), 0, c->stream, g, skip_inlet,
                     (const uint32_t*)offsets, c->blist, base, c->blist_cap);
  return hipGetLastError();
}

// Set-up at the current time level: masks everywhere, then the static part of the boundary list
// (all boundary nodes for fixed geometry; only the inlet face when bodies move).
hipError_t geometry_init(elbm_ctx* c) {
  c->slab_valid = false;  // the populations were set from outside
  const Bodies bd = make_bodies(c, (double)c->t);
  const Box fb = full_box(c);
  GeoArgs g = geo_args(c, fb);
  hipLaunchKernelGGL(k_flags_init, grid_for(fb.count()), dim3(256), 0, c->stream, g, bd);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (c->mesh_body >= 0) {
    e = mesh_mask(c, bd, 0, FL_SOLID | FL_SOLID_PREV);
    if (e != hipSuccess) return e;
  }
  Box sb = fb;
  const bool channel = c->p.bc_x == ELBM_BC_CHANNEL;
  if (c->moving) {
    if (channel) {
      sb.n[0] = 1;  // inlet face only
    } else {
      c->n_static = 0;
      return hipSuccess;
    }
  } else if (c->nb == 0 && !channel) {
    c->n_static = 0;
    return hipSuccess;
  }
  e = scan_box(c, sb, 0, 0);
  if (e != hipSuccess) return e;
  uint32_t n = 0;
  e = hipMemcpyAsync(&n, &c->cnt->dyn_count, sizeof n, hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return e;
  c->n_static = (int64_t)n;
  return hipSuccess;
}

// Per step, before the sweep: masks at t+1 and the dynamic list (moving bodies), then U^t, R^t
// around the bodies and on the inlet slab.
hipError_t geometry_pre_step(elbm_ctx* c, const Bodies& bd) {
  const bool channel = c->p.bc_x == ELBM_BC_CHANNEL;
  if (c->nb == 0 && !channel) return hipSuccess;
  Box ub = union_box(c, bd);
  if (c->moving) {
    GeoArgs g = geo_args(c, ub);
    hipLaunchKernelGGL(k_flags_update, grid_for(ub.count()), dim3(256), 0, c->stream, g, bd);
    if (c->mesh_body >= 0) {
      const hipError_t em = mesh_mask(c, bd, 1, FL_SOLID);
      if (em != hipSuccess) return em;
    }
    const hipError_t e = scan_box(c, ub, c->n_static, 1);
    if (e != hipSuccess) return e;
  }
  // the inlet slab of the current state was staged by the step that produced it, unless the state
  // was set from outside since then
  if (c->slab_valid) {
    hipLaunchKernelGGL(k_slab_copy, grid_for(4L * 3 * c->p.ny * c->p.nz), dim3(256), 0, c->stream, c->slab_next,
                       c->macro, c->p.nx, c->p.ny, c->p.nz, (int64_t)c->N);
  }
  hipError_t e = macro_fields(c, c->pop[c->cur], bd, !c->slab_valid);
  if (e != hipSuccess || bd.mesh < 0) return e;
  const BArgs a = boundary_args(c, c->pop[c->cur], nullptr);
  const dim3 g((unsigned)std::min<int64_t>(std::max<int64_t>((a.cap - a.n_static + 1) / 2, 1), 4096)), b(64);
  hipLaunchKernelGGL(k_mesh_uncovered, g, b, 0, c->stream, a, bd, c->macro);
  return hipGetLastError();
}

// Masks of both time levels of the step t -> t+1 recomputed from the kinematics alone (so that a
// reverse sweep can visit the steps in any order), the inlet face marked, then the dynamic list.
__global__ void k_flags_two(GeoArgs g, Bodies bd) {
  const long total = g.box.count();
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    int x, y, z;
    box_node(g.box, idx, x, y, z);
    const long n = ((long)z * g.ny + y) * g.nx + x;
    const bool s1 = first_body(bd, true, x, y, z) >= 0;
    const bool s0 = first_body(bd, false, x, y, z) >= 0;
    uint8_t f = (s1 ? FL_SOLID : 0) | (s0 ? FL_SOLID_PREV : 0);
    if (g.channel && x == 0 && !s1) f |= FL_SPECIAL;
    g.flags[n] = f;
  }
}

hipError_t geometry_for_step(elbm_ctx* c, const Bodies& bd) {
  if (!c->moving) return hipSuccess;  // fixed geometry: masks and list from the set-up hold
  const Box fb = full_box(c);
  hipLaunchKernelGGL(k_flags_two, grid_for(fb.count()), dim3(256), 0, c->stream, geo_args(c, fb), bd);
  return scan_box(c, union_box(c, bd), c->n_static, 1);
}

template <int S, int STAB>
static void boundary_launch_st(elbm_ctx* c, const BArgs& a, const Bodies& bd) {
  // two list entries per 64-lane workgroup
  const dim3 g((unsigned)std::min<int64_t>(std::max<int64_t>((a.cap + 1) / 2, 1), 16384)), b(64);
  if (bd.mesh < 0) {
    if (c->bodyforce) hipLaunchKernelGGL((k_boundary<S, true, STAB, false>), g, b, 0, c->stream, a, bd);
    else hipLaunchKernelGGL((k_boundary<S, false, STAB, false>), g, b, 0, c->stream, a, bd);
    return;
  }
  // with a triangulated body: the static entries (the inlet face; no body is that close to it) in
  // the plain instantiation, the dynamic ones in the one that carries the mesh geometry
  BArgs as = a, ad = a;
  as.hi = a.n_static;
  ad.lo = a.n_static;
  const dim3 gs((unsigned)std::min<int64_t>(std::max<int64_t>((a.n_static + 1) / 2, 1), 16384));
  const dim3 gd((unsigned)std::min<int64_t>(std::max<int64_t>((a.cap - a.n_static + 1) / 2, 1), 16384));
  if (a.n_static > 0) {
    if (c->bodyforce) hipLaunchKernelGGL((k_boundary<S, true, STAB, false>), gs, b, 0, c->stream, as, bd);
    else hipLaunchKernelGGL((k_boundary<S, false, STAB, false>), gs, b, 0, c->stream, as, bd);
  }
  if (c->bodyforce) hipLaunchKernelGGL((k_boundary<S, true, STAB, true>), gd, b, 0, c->stream, ad, bd);
  else hipLaunchKernelGGL((k_boundary<S, false, STAB, true>), gd, b, 0, c->stream, ad, bd);
}

template <int S>
static void boundary_launch(elbm_ctx* c, const BArgs& a, const Bodies& bd) {
  switch (c->stab) {
    case STAB_EXACT: boundary_launch_st<S, STAB_EXACT>(c, a, bd); break;
    case STAB_LBGK: boundary_launch_st<S, STAB_LBGK>(c, a, bd); break;
    case STAB_KBC | STAB_CENTRAL: boundary_launch_st<S, STAB_KBC | STAB_CENTRAL>(c, a, bd); break;
    default: boundary_launch_st<S, STAB_KBC>(c, a, bd);
  }
}

BArgs boundary_args(elbm_ctx* c, const void* A, void* B) {
  const bool channel = c->p.bc_x == ELBM_BC_CHANNEL;
  BArgs a;
  a.A = A;
  a.B = B;
  a.flags = c->flags;
  a.macro = c->macro;
  a.F = c->bodyforce;
  a.list = c->blist;
  a.dyn_count = &c->cnt->dyn_count;
  a.brec = c->brec;
  a.fix_list = (uint32_t*)c->fix_list;
  a.fix_count = &c->cnt->fix_count[c->fix_par];
  a.diag = c->cnt;
  a.stats = c->gamma_stats ? 1 : 0;
  a.slab_next = (channel && !(c->p.flags & ELBM_FLAG_STREAM_ONLY)) ? c->slab_next : nullptr;
  a.n_static = c->n_static;
  a.lo = 0;
  a.hi = -1;
  a.cap = c->blist_cap;
  a.moving = c->moving ? 1 : 0;
  a.nx = c->p.nx;
  a.ny = c->p.ny;
  a.nz = c->p.nz;
  a.N = c->N;
  a.lay = c->lay;
  a.channel = channel ? 1 : 0;
  a.fp64 = !(c->p.flags & ELBM_FLAG_NO_FP64);
  a.stream_only = (c->p.flags & ELBM_FLAG_STREAM_ONLY) != 0;
  a.stab = c->stab;
  a.beta = (float)c->beta;
  a.inv_beta = (float)(1.0 / c->beta);
  a.beta64 = c->beta;
  a.thr = (float)c->fp64_thr;
  a.rho0 = c->p.rho0;
  for (int e = 0; e < 3; ++e) a.u_in[e] = c->p.u_inlet[e];
  return a;
}

hipError_t launch_refill(elbm_ctx* c, const Bodies& bd, void* A) {
  if (!c->moving) return hipSuccess;  // fixed bodies uncover nothing
  const BArgs a = boundary_args(c, A, nullptr);
  const int64_t dyn = a.cap - a.n_static;
  const dim3 g((unsigned)std::min<int64_t>(std::max<int64_t>((dyn + 1) / 2, 1), 4096)), b(64);
  const bool mesh = bd.mesh >= 0;
  switch (c->p.storage) {
    case ELBM_STORAGE_F32:
      if (mesh) hipLaunchKernelGGL((k_refill<ELBM_STORAGE_F32, true>), g, b, 0, c->stream, a, bd, A);
      else hipLaunchKernelGGL((k_refill<ELBM_STORAGE_F32, false>), g, b, 0, c->stream, a, bd, A);
      break;
    case ELBM_STORAGE_F16:
      if (mesh) hipLaunchKernelGGL((k_refill<ELBM_STORAGE_F16, true>), g, b, 0, c->stream, a, bd, A);
      else hipLaunchKernelGGL((k_refill<ELBM_STORAGE_F16, false>), g, b, 0, c->stream, a, bd, A);
      break;
    default:
      if (mesh) hipLaunchKernelGGL((k_refill<ELBM_STORAGE_BF16, true>), g, b, 0, c->stream, a, bd, A);
      else hipLaunchKernelGGL((k_refill<ELBM_STORAGE_BF16, false>), g, b, 0, c->stream, a, bd, A);
  }
  return hipGetLastError();
}

hipError_t launch_boundary(elbm_ctx* c, const Bodies& bd) {
  const bool channel = c->p.bc_x == ELBM_BC_CHANNEL;
  if (c->nb == 0 && !channel) return hipSuccess;
  const BArgs a = boundary_args(c, c->pop[c->cur], c->pop[c->cur ^ 1]);
  switch (c->p.storage) {
    case ELBM_STORAGE_F32: boundary_launch<ELBM_STORAGE_F32>(c, a, bd); break;
    case ELBM_STORAGE_F16: boundary_launch<ELBM_STORAGE_F16>(c, a, bd); break;
    default: boundary_launch<ELBM_STORAGE_BF16>(c, a, bd);
  }
  return hipGetLastError();
}

hipError_t launch_force_reduce(elbm_ctx* c) {
  if (c->nb == 0) return hipSuccess;
  const int slot = (int)((c->t + 1) % c->p.force_ring);
  double* out = c->ring + (size_t)slot * ELBM_MAX_BODIES * 6;
  hipLaunchKernelGGL(k_force_partial, dim3(FORCE_PARTS), dim3(256), 0, c->stream, (const double*)c->brec,
                     (const uint32_t*)&c->cnt->dyn_count, c->n_static, c->blist_cap, (int32_t)(c->moving ? 1 : 0),
                     (int32_t)c->nb, c->force_partial);
  hipLaunchKernelGGL(k_force_final, dim3(1), dim3(64), 0, c->stream, (const double*)c->force_partial, (int32_t)c->nb,
                     out);
  return hipGetLastError();
}

}  // namespace elbm
