// adjoint.hip -- hand-written reverse mode of one step of the forward path (an addition of this
// library, not part of the paper): given dL/dA^{t+1} it produces dL/dA^t and accumulates dL/dF for
// the body-force field and dL/d(amp) for each body's oscillation amplitude.  The forward step it
// differentiates is exactly the one of sweep.hip and geometry.hip: pull streaming, the KBC
// collision of Sec. II (stabiliser included), the moving-wall Grad reconstruction and the
// momentum-exchange force of Sec. III / IV.A.  The solid masks are piecewise constant in the
// parameters, so their derivative is zero (the topology of each step is that of the forward run).
//
// Data flow of a reverse step (all on the context's stream):
//   k_adj_bulk      per fluid node: collision VJP, then the transpose of the pull -- every
//                   (source, direction) entry of dL/dA^t is written exactly once by the node that
//                   pulled it, so the scatter needs no atomics;  solid nodes write zeros; in channel
//                   mode the face nodes also zero the entries no node pulls (the wall adjoint then
//                   adds the inlet bounce-back terms).
//   k_adj_boundary  per boundary/refill node: the adjoint of the reconstruction (Grad populations,
//                   targets, finite-difference gradient, force term of the loss); contributions to
//                   U^t and R^t of other nodes go to FP64 accumulators.
//   k_adj_outlet    channel mode: the outlet copy, added after the wall adjoint.
//   k_adj_refill    the completed dL/dA^t of refilled nodes sent through Grad's distribution.
//   k_adj_macro     the accumulated dL/dU^t, dL/dR^t turned into dL/dA^t (nodes fluid at t) or
//                   into dL/d(amp) (nodes solid at t, whose U^t is the rigid-body velocity).
//
// Every collision VJP runs in FP64 on the exactly widened stored deviations (f = W + d): the
// derivative of the stabiliser carries 1/<dh|dh>, so an FP32 evaluation loses the digits of dh
// that decide it at weakly disturbed nodes (an FP32 VJP missed a smooth body-force gradient by
// 7.5e-4 on a small channel; FP64 by 6e-7).  Adjoint fields stay FP32 in memory.
#include <algorithm>

#include "context.hpp"
#include "boundary_dev.hpp"

namespace elbm {

// FP64 reciprocal from the hardware estimate and two Newton steps (within an ulp of 1/x; the
// IEEE division sequence costs twice the instructions).
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

// One velocity component's equilibrium factors phi(c, u) = w(c) (2 - s) X^c (c = -1, 0, 1; the rule
// of axis_phi, s = sqrt(1 + 3u^2), X = (2u + s)/(1 - u)), their reciprocals and their log-derivatives
// d ln phi(c, u) / du = d0 + c dX with d0 = -3u / (s (2 - s)) and dX = (2 + 3u/s)/(2u + s) + 1/(1 - u).
// Since s^2 - 4u^2 = 1 - u^2, phi(+1) phi(-1) = ((2 - s)/6)^2 and phi(0) = (2/3)(2 - s): the three
// reciprocals follow from 1/(2 - s); 1 + u and 1 - u share one reciprocal, s and 2u + s another
// (three in all, with the square root).
__device__ __forceinline__ void axis_phi_dln(double u, double (&ph)[3], double (&D)[3], double (&iph)[3]) {
  const double s = sqrt_(3.0 * u * u + 1.0);
  const double g = 2.0 - s, w = 2.0 * u + s;
  const double ig = rcp64(g), rpm = rcp64((1.0 + u) * (1.0 - u)), rsw = rcp64(s * w);
  const double ip = (1.0 - u) * rpm, im = (1.0 + u) * rpm, is = w * rsw, iw = s * rsw;
  ph[0] = g * ((s - 2.0 * u) * ip) * (1.0 / 6.0);
  ph[1] = g * (2.0 / 3.0);
  ph[2] = g * (w * im) * (1.0 / 6.0);
  const double q = 36.0 * ig * ig;
  iph[0] = ph[2] * q;
  iph[1] = 1.5 * ig;
  iph[2] = ph[0] * q;
  const double d0 = -3.0 * u * is * ig;
  const double dX = (2.0 + 3.0 * u * is) * iw + im;
  D[0] = d0 - dX;
  D[1] = d0;
  D[2] = d0 + dX;
}
__device__ __forceinline__ void axis_phi_dln(double u, double (&ph)[3], double (&D)[3]) {
  double iph[3];
  axis_phi_dln(u, ph, D, iph);
}

template <typename T> struct VjpOut {
  T b;
  T rho;
};

// Vector-Jacobian product of kbc_collide: g = (d f'/d f)^T gp and gF = (d f'/d F)^T gp.
// The equilibrium and its reciprocal come from per-axis factors (feq_i = rho phi_x phi_y phi_z),
// so no division runs per direction; the equilibrium's cotangent is folded into the four sums it
// feeds (d/drho and d/du of feq) as soon as each term is known, so no per-direction array besides
// gp, the deviations and g stays live.
template <typename T, bool FORCE>
__device__ inline VjpOut<T> kbc_vjp(const T (&f)[27], const T (&gp)[27], const T beta, const T Fx, const T Fy,
                                    const T Fz, T (&g)[27], T (&gF)[3], bool lbgk = false) {
  T rho = T(0), jx = T(0), jy = T(0), jz = T(0);
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    rho += f[i];
    jx += T(cx(i)) * f[i];
    jy += T(cy(i)) * f[i];
    jz += T(cz(i)) * f[i];
  }
  const T irho = rcp64(rho);
  const T ux = jx * irho, uy = jy * irho, uz = jz * irho;
  T px[3], py[3], pz[3], ipz[3], pxy[9], ipxy[9], Dx[3], Dy[3], Dz[3];
  {
    T ipx[3], ipy[3];
    axis_phi_dln(ux, px, Dx, ipx);
    axis_phi_dln(uy, py, Dy, ipy);
    axis_phi_dln(uz, pz, Dz, ipz);
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        pxy[3 * l + k] = rho * px[k] * py[l];
        ipxy[3 * l + k] = irho * ipx[k] * ipy[l];
      }
  }
  auto FE = [&](int i) -> T { return pxy[3 * (cy(i) + 1) + cx(i) + 1] * pz[cz(i) + 1]; };
  auto IFE = [&](int i) -> T { return ipxy[3 * (cy(i) + 1) + cx(i) + 1] * ipz[cz(i) + 1]; };
  T dh[27];
  T M200 = 0, M020 = 0, M002 = 0, M110 = 0, M101 = 0, M011 = 0;
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const T d = f[i] - FE(i);
    dh[i] = d;
    M200 += T(cx(i) * cx(i)) * d;
    M020 += T(cy(i) * cy(i)) * d;
    M002 += T(cz(i) * cz(i)) * d;
    M110 += T(cx(i) * cy(i)) * d;
    M101 += T(cx(i) * cz(i)) * d;
    M011 += T(cy(i) * cz(i)) * d;
  }
  const T tr3 = (M200 + M020 + M002) * T(1.0 / 3.0);
  const T sfx = T(0.5) * (M200 - tr3), sfy = T(0.5) * (M020 - tr3), sfz = T(0.5) * (M002 - tr3);
  const T sxy = T(0.25) * M110, sxz = T(0.25) * M101, syz = T(0.25) * M011;
  auto DS = [&](int i) -> T {
    if (nnz(i) == 1) return cx(i) ? sfx : (cy(i) ? sfy : sfz);
    if (nnz(i) == 2) {
      if (cz(i) == 0) return T(cx(i) * cy(i)) * sxy;
      if (cy(i) == 0) return T(cx(i) * cz(i)) * sxz;
      return T(cy(i) * cz(i)) * syz;
    }
    return T(0);
  };
  T a = T(0), b = T(0), g_gam = T(0);
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    dh[i] -= DS(i);
    const T th = dh[i] * IFE(i);
    b += th * dh[i];
    a += th * DS(i);
    g_gam += gp[i] * dh[i];
  }
  const bool guard = lbgk || !(b > T(1e-30));  // gamma fixed at 2: no derivative through it
  const T ib = rcp64(beta);
  const T inv_b = guard ? T(0) : rcp64(b);
  const T gam = guard ? T(2) : ib - (T(2) - ib) * a * inv_b;
  // reverse
  g_gam *= -beta;
  const T g_a = -(T(2) - ib) * inv_b * g_gam;
  const T g_b = (T(2) - ib) * a * inv_b * inv_b * g_gam;
  // S0, Sx, Sy, Sz: sums of (dL/dfeq_i) feq_i times 1 and d ln feq_i / du
  T S0 = T(0), Sx = T(0), Sy = T(0), Sz = T(0);
  T gDx = 0, gDy = 0, gDz = 0, gPxy = 0, gPxz = 0, gPyz = 0;
  const T bg = beta * gam;
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const T ds = DS(i), h = dh[i], ife = IFE(i);
    const T g_dh = -bg * gp[i] + (g_a * ds + T(2) * g_b * h) * ife;
    const T g_ds = -T(2) * beta * gp[i] + g_a * h * ife - g_dh;
    const T ge = -(g_a * ds + g_b * h) * h * ife - g_dh * FE(i);
    S0 += ge;
    Sx += ge * Dx[cx(i) + 1];
    Sy += ge * Dy[cy(i) + 1];
    Sz += ge * Dz[cz(i) + 1];
    g[i] = gp[i] + g_dh;
    if (nnz(i) == 1) {
      if (cx(i)) gDx += T(0.5) * g_ds;
      else if (cy(i)) gDy += T(0.5) * g_ds;
      else gDz += T(0.5) * g_ds;
    } else if (nnz(i) == 2) {
      if (cz(i) == 0) gPxy += T(0.25) * T(cx(i) * cy(i)) * g_ds;
      else if (cy(i) == 0) gPxz += T(0.25) * T(cx(i) * cz(i)) * g_ds;
      else gPyz += T(0.25) * T(cy(i) * cz(i)) * g_ds;
    }
  }
  const T gm = (gDx + gDy + gDz) * T(1.0 / 3.0);
  const T gM200 = gDx - gm, gM020 = gDy - gm, gM002 = gDz - gm;
  T g_rho = T(0), gux = T(0), guy = T(0), guz = T(0);
  gF[0] = gF[1] = gF[2] = T(0);
  T qx[3], qy[3], qz[3], D1x[3], D1y[3], D1z[3], u1x = T(0), u1y = T(0), u1z = T(0);
  T gr1 = T(0), g1x = T(0), g1y = T(0), g1z = T(0);
  if (FORCE) {
    // f' += feq(rho, u + F/rho) - feq(rho, u)
    u1x = ux + Fx * irho;
    u1y = uy + Fy * irho;
    u1z = uz + Fz * irho;
    axis_phi_dln(u1x, qx, D1x);
    axis_phi_dln(u1y, qy, D1y);
    axis_phi_dln(u1z, qz, D1z);
  }
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const T e = gM200 * T(cx(i) * cx(i)) + gM020 * T(cy(i) * cy(i)) + gM002 * T(cz(i) * cz(i)) +
                gPxy * T(cx(i) * cy(i)) + gPxz * T(cx(i) * cz(i)) + gPyz * T(cy(i) * cz(i));
    g[i] += e;
    T ge = -e;
    if (FORCE) {
      const T g1 = gp[i] * rho * qx[cx(i) + 1] * qy[cy(i) + 1] * qz[cz(i) + 1];
      gr1 += g1;
      g1x += g1 * D1x[cx(i) + 1];
      g1y += g1 * D1y[cy(i) + 1];
      g1z += g1 * D1z[cz(i) + 1];
      ge -= gp[i];
    }
    ge *= FE(i);
    S0 += ge;
    Sx += ge * Dx[cx(i) + 1];
    Sy += ge * Dy[cy(i) + 1];
    Sz += ge * Dz[cz(i) + 1];
  }
  if (FORCE) {
    g_rho += gr1 * irho - (g1x * Fx + g1y * Fy + g1z * Fz) * irho * irho;
    gux += g1x;
    guy += g1y;
    guz += g1z;
    gF[0] = g1x * irho;
    gF[1] = g1y * irho;
    gF[2] = g1z * irho;
  }
  g_rho += S0 * irho;
  gux += Sx;
  guy += Sy;
  guz += Sz;
  const T gjx = gux * irho, gjy = guy * irho, gjz = guz * irho;
  g_rho -= (gux * ux + guy * uy + guz * uz) * irho;
#pragma unroll
  for (int i = 0; i < 27; ++i) g[i] += g_rho + T(cx(i)) * gjx + T(cy(i)) * gjy + T(cz(i)) * gjz;
  return VjpOut<T>{b, rho};
}

struct AdjArgs {
  const float* lam_in;
  float* lam_out;
  float* side;
  float* gF;
  double* gUR;
  const double* m64;  // U^t, R^t in FP64 (4 N) around the bodies and on the inlet slab
  double* r64;        // FP64 refill populations of the uncovered nodes, [list slot][27]
  int32_t* slot;      // list slot of each uncovered node
};

struct AdjBodyArgs {
  double dc1[ELBM_MAX_BODIES][3];  // d c(t+1) / d amp
  double dU1[ELBM_MAX_BODIES][3];  // d U(t+1) / d amp
  double dU0[ELBM_MAX_BODIES][3];  // d U(t) / d amp
  double w[ELBM_MAX_BODIES][3];    // dL / dF_body(t+1)
  double* gamp;                    // [MAX_BODIES] accumulators
  int32_t loss;
  int32_t pad;
};

// Transpose of the pull: entry (x - c_i, i) of dL/dA^t receives v.  Channel mode: nothing for a
// source through the inlet; the outlet copy goes to the side buffer, keyed by the destination.
__device__ inline void adj_push(const BArgs& a, const AdjArgs& j, int i, int x, int y, int z, float v) {
  int sx = x - cx(i);
  if (a.channel) {
    if (sx < 0) return;
    if (sx >= a.nx) {
      j.side[(size_t)(i / 3) * a.ny * a.nz + (size_t)z * a.ny + y] = v;
      return;
    }
  } else {
    sx = wrap(sx, a.nx);
  }
  j.lam_out[(size_t)i * a.N + node_at(a, sx, wrap(y - cy(i), a.ny), wrap(z - cz(i), a.nz))] = v;
}

__device__ inline long pull_source(const BArgs& a, int i, int x, int y, int z) {
  int sx = x - cx(i);
  if (a.channel) sx = sx >= a.nx ? a.nx - 1 : (sx < 0 ? 0 : sx);
  else sx = wrap(sx, a.nx);
  return node_at(a, sx, wrap(y - cy(i), a.ny), wrap(z - cz(i), a.nz));
}

// Pull sources of a node, computed once, split for the addressing as in the bulk sweep: per source
// plane z - cz its element offset in the population layout and its first node (uniform over a
// workgroup: z is the grid's z), per source row y - cy its in-plane offsets, and the 3 source x
// (clamped to the outlet in channel mode; periodic in y and z).  Loads and stores go through buffer
// resources on the uniform bases with 32-bit in-plane byte offsets (the plane-size limit of the
// context and fewer than 2^30 nodes for the adjoint keep them below 2^32).  The transpose of the pull
// writes to the same entries, except beyond the inlet (nothing) and beyond the outlet (the side
// buffer).
struct PullIdx {
  int64_t zb[3];   // zb[cz+1]: element offset of source plane z - cz (population layout)
  uint32_t zn[3];  // zn[cz+1]: node index of the first node of source plane z - cz
  uint32_t yo[3];  // yo[cy+1]: element offset of source row y - cy inside its plane
  uint32_t yn[3];  // yn[cy+1]: node offset of source row y - cy inside its plane
  uint32_t xs[3];  // xs[cx+1]: source x
  bool in_lo;      // channel: x - 1 < 0 (cx = +1 comes through the inlet)
  bool out_hi;     // channel: x + 1 >= nx (cx = -1 comes from beyond the outlet, copied)
};

__device__ inline void pull_idx(const BArgs& a, int x, int y, int z, PullIdx& P) {
  const int xm = x + 1, xp = x - 1;
  if (a.channel) {
    P.xs[0] = xm < a.nx ? xm : a.nx - 1;
    P.xs[2] = xp >= 0 ? xp : 0;
  } else {
    P.xs[0] = xm == a.nx ? 0 : xm;
    P.xs[2] = xp < 0 ? a.nx - 1 : xp;
  }
  P.xs[1] = x;
  P.in_lo = a.channel && xp < 0;
  P.out_hi = a.channel && xm >= a.nx;
  const int ys[3] = {y + 1 == a.ny ? 0 : y + 1, y, y == 0 ? a.ny - 1 : y - 1};
  const int zs[3] = {z + 1 == a.nz ? 0 : z + 1, z, z == 0 ? a.nz - 1 : z - 1};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    P.zb[k] = (int64_t)zs[k] * a.ny * a.lay.rs;
    P.zn[k] = (uint32_t)zs[k] * (uint32_t)a.ny * (uint32_t)a.nx;
    P.yo[k] = (uint32_t)ys[k] * (uint32_t)a.lay.rs;
    P.yn[k] = (uint32_t)ys[k] * (uint32_t)a.nx;
  }
}

// Node pulled into direction i.
__device__ __forceinline__ uint32_t pull_src_idx(const BArgs& a, const PullIdx& P, int i) {
  return P.zn[cz(i) + 1] + P.yn[cy(i) + 1] + P.xs[cx(i) + 1];
}

// Deviation of population i of the node pulled into direction i, in A^t.
template <int S>
__device__ __forceinline__ float pull_load(const BArgs& a, const PullIdx& P, int i) {
  using E = typename Codec<S>::E;
  const E* base = (const E*)a.A + (P.zb[cz(i) + 1] + (int64_t)i * a.lay.si);
  const uint32_t off = (P.yo[cy(i) + 1] + P.xs[cx(i) + 1]) * (uint32_t)sizeof(E);
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, BUF_ALL, BUF_WORD3);
  if constexpr (sizeof(E) == 4) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  } else {
    const E e = __builtin_bit_cast(E, __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0));
    return Codec<S>::load_dev(&e);
  }
}

// Entry n of direction i of an adjoint field ([27][N] FP32), through a buffer resource on the
// direction's base.
__device__ __forceinline__ float dir_load(const float* f, const BArgs& a, int i, uint32_t n) {
  const __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc((void*)(f + (int64_t)i * a.N), (short)0, BUF_ALL, BUF_WORD3);
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, n * 4u, 0, 0));
}
__device__ __forceinline__ void dir_store(float* f, const BArgs& a, int i, uint32_t n, float v) {
  const __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc((void*)(f + (int64_t)i * a.N), (short)0, BUF_ALL, BUF_WORD3);
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, n * 4u, 0, 0);
}

// Transpose of the pull for direction i of node (y, z): entry (x - c_i, i) of dL/dA^t receives v.
__device__ __forceinline__ void push_idx(const BArgs& a, const AdjArgs& j, const PullIdx& P, int i, int y, int z,
                                         float v) {
  if (cx(i) == 1 && P.in_lo) return;
  if (cx(i) == -1 && P.out_hi) {
    j.side[(size_t)(i / 3) * a.ny * a.nz + (size_t)z * a.ny + y] = v;
    return;
  }
  dir_store(j.lam_out, a, i, pull_src_idx(a, P, i), v);
}

template <int S, bool FLAGS, bool FORCE>
__global__ __launch_bounds__(256) void k_adj_bulk(const BArgs a, const AdjArgs j) {
  using C = Codec<S>;
  using E = typename C::E;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= a.nx || y >= a.ny) return;
  const long n = node_at(a, x, y, z);
  if (FLAGS && a.channel && (x == 0 || x == a.nx - 1)) {
    // channel faces: the entries no node pulls (x = 0 moving in -x, x = nx-1 moving in +x) start at
    // zero; the wall kernel, launched next, adds the inlet's bounce-back terms to those at x = 0
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      if (x == 0) j.lam_out[(3 * k) * a.N + n] = 0.f;
      if (x == a.nx - 1) j.lam_out[(3 * k + 2) * a.N + n] = 0.f;
    }
  }
  const uint8_t fl = FLAGS ? a.flags[n] : (uint8_t)0;
  if (fl & FL_SPECIAL) return;
  PullIdx P;
  pull_idx(a, x, y, z, P);
  if (fl & FL_SOLID) {
    // a source fluid at t+1 is a wall node whose missing population this one is: the wall kernel
    // writes the entry (the bounce-back term), so it is left alone here
#pragma unroll
    for (int i = 0; i < 27; ++i) {
      const bool beyond = (cx(i) == 1 && P.in_lo) || (cx(i) == -1 && P.out_hi);
      if (beyond || (a.flags[pull_src_idx(a, P, i)] & FL_SOLID)) push_idx(a, j, P, i, y, z, 0.f);
    }
    return;
  }
  double f[27], gp[27], g[27], gF[3];
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    f[i] = (double)pull_load<S>(a, P, i) + wd(i);  // exact widening
    gp[i] = (double)dir_load(j.lam_in, a, i, (uint32_t)n);
  }
  if (FLAGS && (fl & FL_NEAR_REFILL)) {
    // a source uncovered in this step: its refill value unrounded (the stored one is rounded)
    for (int i = 0; i < 27; ++i) {
      const uint32_t s = pull_src_idx(a, P, i);
      if ((a.flags[s] & (FL_SOLID_PREV | FL_SOLID)) == FL_SOLID_PREV) {
        const uint32_t sl = (uint32_t)j.slot[s];
        if (sl < (uint32_t)a.cap) f[i] = j.r64[(size_t)sl * 27 + i];
      }
    }
  }
  double Fx = 0.0, Fy = 0.0, Fz = 0.0;
  if (FORCE) {
    Fx = a.F[n];
    Fy = a.F[a.N + n];
    Fz = a.F[2 * a.N + n];
  }
  kbc_vjp<double, FORCE>(f, gp, a.beta64, Fx, Fy, Fz, g, gF, a.stab == STAB_LBGK);
#pragma unroll
  for (int i = 0; i < 27; ++i) push_idx(a, j, P, i, y, z, (float)g[i]);
  if (FORCE && j.gF) {
    j.gF[n] += (float)gF[0];
    j.gF[a.N + n] += (float)gF[1];
    j.gF[2 * a.N + n] += (float)gF[2];
  }
}

// Adjoint of Grad's distribution f*_i(rho, u, Pi) (eq. grad), accumulated over directions.
template <typename T>
__device__ inline void grad_pop_vjp(int i, T gfs, T rho, const T (&u)[3], T& gr, T (&gu)[3], T (&gP)[6]) {
  const T W = T(wd(i));
  const T c[3] = {T(cx(i)), T(cy(i)), T(cz(i))};
  const T cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
  const T c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
  gr += gfs * W * (T(1) + T(3) * cu - T(1.5) * (c2 - T(1)));
  gu[0] += gfs * T(3) * rho * W * c[0];
  gu[1] += gfs * T(3) * rho * W * c[1];
  gu[2] += gfs * T(3) * rho * W * c[2];
  const T t = T(1.0 / 3.0);
  gP[0] += gfs * T(4.5) * W * (c[0] * c[0] - t);
  gP[1] += gfs * T(4.5) * W * (c[1] * c[1] - t);
  gP[2] += gfs * T(4.5) * W * (c[2] * c[2] - t);
  gP[3] += gfs * T(9) * W * c[0] * c[1];
  gP[4] += gfs * T(9) * W * c[0] * c[2];
  gP[5] += gfs * T(9) * W * c[1] * c[2];
}

// Adjoint of the pressure tensor (eqs. pressure, pressure2) in the packed order xx,yy,zz,xy,xz,yz.
template <typename T>
__device__ inline void pressure_vjp(T rho, const T (&u)[3], const T (&G)[9], T beta, const T (&gP)[6], T& gr,
                                    T (&gu)[3], T (&gG)[9]) {
  const T k = rho / (T(6) * beta), kr = T(1) / (T(6) * beta);
  const T t = T(1.0 / 3.0);
  gr += gP[0] * (t + u[0] * u[0] - T(2) * kr * G[0]) + gP[1] * (t + u[1] * u[1] - T(2) * kr * G[4]) +
        gP[2] * (t + u[2] * u[2] - T(2) * kr * G[8]) + gP[3] * (u[0] * u[1] - kr * (G[1] + G[3])) +
        gP[4] * (u[0] * u[2] - kr * (G[2] + G[6])) + gP[5] * (u[1] * u[2] - kr * (G[5] + G[7]));
  gu[0] += T(2) * rho * u[0] * gP[0] + rho * u[1] * gP[3] + rho * u[2] * gP[4];
  gu[1] += T(2) * rho * u[1] * gP[1] + rho * u[0] * gP[3] + rho * u[2] * gP[5];
  gu[2] += T(2) * rho * u[2] * gP[2] + rho * u[0] * gP[4] + rho * u[1] * gP[5];
  gG[0] = -T(2) * k * gP[0];
  gG[4] = -T(2) * k * gP[1];
  gG[8] = -T(2) * k * gP[2];
  gG[1] = gG[3] = -k * gP[3];
  gG[2] = gG[6] = -k * gP[4];
  gG[5] = gG[7] = -k * gP[5];
}

__device__ inline void addU(const BArgs& a, const AdjArgs& j, int comp, long node, double v) {
  if (v != 0.0) atomicAdd(&j.gUR[comp * a.N + node], v);
}

// Transpose of the finite-difference stencil of grad_u for one (axis b, component c) pair:
// g = dL/dG[3c+b] -> dL/dU^t at the stencil nodes (FP64 accumulators).
__device__ inline void grad_u_vjp_one(const BArgs& a, const AdjArgs& j, const LaneNb& h, int b, int c, double g) {
  if (g == 0.0) return;
  const int ip = dir_index(b == 0, b == 1, b == 2), im = dir_index(-(b == 0), -(b == 1), -(b == 2));
  const bool op1 = (h.fluid >> ip) & 1u, om1 = (h.fluid >> im) & 1u;
  const bool op2 = (h.far >> (2 * b)) & 1u, om2 = (h.far >> (2 * b + 1)) & 1u;
  const long n0 = h.n;
  const long p1 = neighbour(a, h.x, h.y, h.z, cx(ip), cy(ip), cz(ip));
  const long m1 = neighbour(a, h.x, h.y, h.z, cx(im), cy(im), cz(im));
  const long p2 = far_node(a, h.x, h.y, h.z, 2 * b), m2 = far_node(a, h.x, h.y, h.z, 2 * b + 1);
  if (op1 && om1) {
    addU(a, j, c, p1, 0.5 * g);
    addU(a, j, c, m1, -0.5 * g);
  } else if (op1 && op2) {
    addU(a, j, c, n0, -1.5 * g);
    addU(a, j, c, p1, 2.0 * g);
    addU(a, j, c, p2, -0.5 * g);
  } else if (om1 && om2) {
    addU(a, j, c, n0, 1.5 * g);
    addU(a, j, c, m1, -2.0 * g);
    addU(a, j, c, m2, 0.5 * g);
  } else if (op1) {
    addU(a, j, c, p1, g);
    addU(a, j, c, n0, -g);
  } else if (om1) {
    addU(a, j, c, n0, g);
    addU(a, j, c, m1, -g);
  }
}

// The collision VJP in the lane-parallel form of the wall kernels (FP64): lane i < 27 holds f_i
// (absolute) and gp_i = dL/df'_i and receives g_i = dL/df_i; lanes >= 27 pass zeros.  Same
// arithmetic as kbc_vjp, with every sum over directions a butterfly reduction inside the group.
template <bool FORCE>
__device__ inline double kbc_vjp_lanes(int lane, double f, double gp, double beta, double Fx, double Fy, double Fz,
                                       double (&gF)[3], bool lbgk = false) {
  const bool own = lane < 27;
  const int i = own ? lane : 13;
  const double ci[3] = {(double)cx(i), (double)cy(i), (double)cz(i)};
  if (!own) {
    f = 0.0;
    gp = 0.0;
  }
  const double rho = gsum(f), jx = gsum(ci[0] * f), jy = gsum(ci[1] * f), jz = gsum(ci[2] * f);
  const double irho = rcp64(rho);
  const double ux = jx * irho, uy = jy * irho, uz = jz * irho;
  double px[3], py[3], pz[3], Dx[3], Dy[3], Dz[3], ipx[3], ipy[3], ipz[3];
  axis_phi_dln(ux, px, Dx, ipx);
  axis_phi_dln(uy, py, Dy, ipy);
  axis_phi_dln(uz, pz, Dz, ipz);
  const double fe = rho * px[cx(i) + 1] * py[cy(i) + 1] * pz[cz(i) + 1];
  const double d = own ? f - fe : 0.0;
  const double M200 = gsum(ci[0] * ci[0] * d), M020 = gsum(ci[1] * ci[1] * d), M002 = gsum(ci[2] * ci[2] * d);
  const double M110 = gsum(ci[0] * ci[1] * d), M101 = gsum(ci[0] * ci[2] * d), M011 = gsum(ci[1] * ci[2] * d);
  const double tr3 = (M200 + M020 + M002) * (1.0 / 3.0);
  const double sfx = 0.5 * (M200 - tr3), sfy = 0.5 * (M020 - tr3), sfz = 0.5 * (M002 - tr3);
  const double sxy = 0.25 * M110, sxz = 0.25 * M101, syz = 0.25 * M011;
  double ds = 0.0;
  if (nnz(i) == 1) ds = cx(i) ? sfx : (cy(i) ? sfy : sfz);
  else if (nnz(i) == 2) ds = cz(i) == 0 ? ci[0] * ci[1] * sxy : (cy(i) == 0 ? ci[0] * ci[2] * sxz : ci[1] * ci[2] * syz);
  if (!own) ds = 0.0;
  const double ife = own ? irho * ipx[cx(i) + 1] * ipy[cy(i) + 1] * ipz[cz(i) + 1] : 0.0;
  const double h = d - ds, th = h * ife;
  const double b = gsum(th * h), a = gsum(th * ds), ggh = gsum(gp * h);
  const bool guard = lbgk || !(b > 1e-30);  // gamma fixed at 2: no derivative through it
  const double ib = rcp64(beta);
  const double inv_b = guard ? 0.0 : rcp64(b);
  const double gam = guard ? 2.0 : ib - (2.0 - ib) * a * inv_b;
  // reverse
  const double g_gam = -beta * ggh;
  const double g_a = guard ? 0.0 : -(2.0 - ib) * inv_b * g_gam;
  const double g_b = guard ? 0.0 : (2.0 - ib) * a * inv_b * inv_b * g_gam;
  const double g_dh = own ? -beta * gam * gp + (g_a * ds + 2.0 * g_b * h) * ife : 0.0;
  const double g_ds = own ? -2.0 * beta * gp + g_a * h * ife - g_dh : 0.0;
  double gfe = own ? -(g_a * ds * h + g_b * h * h) * ife * ife - g_dh : 0.0;
  // g_ds onto the deviatoric moments
  const bool face = nnz(i) == 1, edge = nnz(i) == 2;
  const double gDx = gsum(face && cx(i) ? 0.5 * g_ds : 0.0), gDy = gsum(face && cy(i) ? 0.5 * g_ds : 0.0);
  const double gDz = gsum(face && cz(i) ? 0.5 * g_ds : 0.0);
  const double gPxy = gsum(edge && cz(i) == 0 ? 0.25 * ci[0] * ci[1] * g_ds : 0.0);
  const double gPxz = gsum(edge && cy(i) == 0 ? 0.25 * ci[0] * ci[2] * g_ds : 0.0);
  const double gPyz = gsum(edge && cx(i) == 0 ? 0.25 * ci[1] * ci[2] * g_ds : 0.0);
  const double gm = (gDx + gDy + gDz) * (1.0 / 3.0);
  const double e = (gDx - gm) * ci[0] * ci[0] + (gDy - gm) * ci[1] * ci[1] + (gDz - gm) * ci[2] * ci[2] +
                   gPxy * ci[0] * ci[1] + gPxz * ci[0] * ci[2] + gPyz * ci[1] * ci[2];
  gfe -= own ? e : 0.0;
  double g_rho = 0.0, gux = 0.0, guy = 0.0, guz = 0.0;
  gF[0] = gF[1] = gF[2] = 0.0;
  if (FORCE) {
    // f' += feq(rho, u + F/rho) - feq(rho, u)
    const double u1x = ux + Fx * irho, u1y = uy + Fy * irho, u1z = uz + Fz * irho;
    double qx[3], qy[3], qz[3], D1x[3], D1y[3], D1z[3];
    axis_phi_dln(u1x, qx, D1x);
    axis_phi_dln(u1y, qy, D1y);
    axis_phi_dln(u1z, qz, D1z);
    const double ge1 = own ? gp * rho * qx[cx(i) + 1] * qy[cy(i) + 1] * qz[cz(i) + 1] : 0.0;
    const double gr1 = gsum(ge1);
    const double g1x = gsum(ge1 * D1x[cx(i) + 1]), g1y = gsum(ge1 * D1y[cy(i) + 1]);
    const double g1z = gsum(ge1 * D1z[cz(i) + 1]);
    gfe -= gp;
    g_rho += gr1 * irho - (g1x * Fx + g1y * Fy + g1z * Fz) * irho * irho;
    gux += g1x;
    guy += g1y;
    guz += g1z;
    gF[0] = g1x * irho;
    gF[1] = g1y * irho;
    gF[2] = g1z * irho;
  }
  const double ge = own ? gfe * fe : 0.0;
  g_rho += gsum(ge) * irho;
  gux += gsum(ge * Dx[cx(i) + 1]);
  guy += gsum(ge * Dy[cy(i) + 1]);
  guz += gsum(ge * Dz[cz(i) + 1]);
  const double gjx = gux * irho, gjy = guy * irho, gjz = guz * irho;
  g_rho -= (gux * ux + guy * uy + guz * uz) * irho;
  return gp + g_dh + e + g_rho + ci[0] * gjx + ci[1] * gjy + ci[2] * gjz;
}

// ---------------------------------------------------------------------------------------------
// The point of linearisation.  The stabiliser's derivative changes fast with the state (its
// curvature goes with 1/<dh|dh>), so a reverse step evaluated at populations rounded to FP32
// differs from the derivative at the exact state by far more than FP32 rounding: at inlet nodes
// of a state with relative noise 1e-3, FP32 Grad populations moved dL/dA^t by up to 1e-4 of its
// size.  The reverse step therefore rebuilds its forward quantities in FP64 from the stored state:
// U^t and R^t (k_macro64), the wall targets and Grad populations (wall_targets64), the refill
// values (k_adj_refill); only the adjoint fields themselves are stored in FP32.

// U^t, R^t in FP64 on a box: the rule of k_macro (moments of A^t with U = (j - F/2)/rho at nodes
// fluid at t, the rigid-body velocity and rho0 at nodes solid at t) from the exactly widened
// stored deviations.
template <int S>
__global__ void k_macro64(const typename Codec<S>::E* A, PopLayout lay, const uint8_t* flags, double* m64,
                          const float* F, Box2 box, int32_t nx, int32_t ny, int64_t N, double rho0, Bodies bd) {
  using C = Codec<S>;
  const long total = box.count();
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    int x, y, z;
    box2_node(box, idx, x, y, z);
    const long n = ((long)z * ny + y) * nx + x;
    double U[3], R;
    if (flags[n] & FL_SOLID_PREV) {
      const BodyDev& b = bd.b[max(first_body(bd, false, x, y, z), 0)];
      const double r[3] = {x - b.c0[0], y - b.c0[1], z - b.c0[2]};
      U[0] = b.U0[0] + (b.omega[1] * r[2] - b.omega[2] * r[1]);
      U[1] = b.U0[1] + (b.omega[2] * r[0] - b.omega[0] * r[2]);
      U[2] = b.U0[2] + (b.omega[0] * r[1] - b.omega[1] * r[0]);
      R = rho0;
    } else {
      double dr = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
      for (int i = 0; i < 27; ++i) {
        const double v = (double)C::load_dev(A + pop_off(lay, i, x, y, z));
        dr += v;
        jx += cx(i) * v;
        jy += cy(i) * v;
        jz += cz(i) * v;
      }
      const double rho = 1.0 + dr;
      if (F) {
        jx -= 0.5 * (double)F[n];
        jy -= 0.5 * (double)F[N + n];
        jz -= 0.5 * (double)F[2 * N + n];
      }
      const double irho = 1.0 / rho;
      U[0] = jx * irho;
      U[1] = jy * irho;
      U[2] = jz * irho;
      R = rho;
    }
    m64[n] = U[0];
    m64[N + n] = U[1];
    m64[2 * N + n] = U[2];
    m64[3 * N + n] = R;
  }
}

// This lane's FP64 U^t, R^t of the stencil gathered by lane_gather (same masks).
struct LaneU64 {
  double U[3];  // U^t at x + c_lane where fluid at t+1
  double V[3];  // U^t at the far node of this lane where fluid at t+1
  double R;     // R^t at x + c_lane where fluid at t and t+1
};

__device__ inline void lane_u64(const BArgs& a, const double* m64, const LaneNb& h, int lane, LaneU64& u) {
  const bool own = lane < 27;
  const int i = own ? lane : 13;
  const long m = neighbour(a, h.x, h.y, h.z, cx(i), cy(i), cz(i));
  const int fk = lane >= 27 ? lane - 27 : (lane == 13 ? 5 : -1);
  const bool uf = own && ((h.fluid >> i) & 1u);
  const bool vf = fk >= 0 && ((h.far >> fk) & 1u);
  const long mf = vf ? far_node(a, h.x, h.y, h.z, fk) : -1;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    u.U[c] = uf ? m64[c * a.N + m] : 0.0;
    u.V[c] = vf ? m64[c * a.N + mf] : 0.0;
  }
  u.R = (own && ((h.fluid0 >> i) & 1u)) ? m64[3 * a.N + m] : 0.0;
}

// grad_u_grp on the FP64 stencil.
__device__ inline void grad_u_grp64(const LaneNb& h, const LaneU64& u, double (&G)[9]) {
  double u0[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) u0[c] = __shfl(u.U[c], 13, GROUP);
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int ip = dir_index(b == 0, b == 1, b == 2), im = dir_index(-(b == 0), -(b == 1), -(b == 2));
    const bool op1 = (h.fluid >> ip) & 1u, om1 = (h.fluid >> im) & 1u;
    const bool op2 = (h.far >> (2 * b)) & 1u, om2 = (h.far >> (2 * b + 1)) & 1u;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double up1 = __shfl(u.U[c], ip, GROUP), um1 = __shfl(u.U[c], im, GROUP);
      const double up2 = __shfl(u.V[c], far_lane(2 * b), GROUP), um2 = __shfl(u.V[c], far_lane(2 * b + 1), GROUP);
      double d;
      if (op1 && om1) d = 0.5 * (up1 - um1);
      else if (op1 && op2) d = 0.5 * (-3.0 * u0[c] + 4.0 * up1 - up2);
      else if (om1 && om2) d = 0.5 * (3.0 * u0[c] - 4.0 * um1 + um2);
      else if (op1) d = up1 - u0[c];
      else if (om1) d = u0[c] - um1;
      else d = 0.0;
      G[3 * c + b] = d;
    }
  }
}

// wall_targets in FP64: this lane's link, the group's targets, the gradient of U^t, the pressure
// tensor and this lane's Grad population (absolute), from the FP64 U^t and the exactly widened
// stored deviations.
struct WallLane64 {
  bool mine;
  double q, uw[3];
  int kb;
  double fb;  // bounce-back value: deviation of A^t_{opp(lane)}(x)
  double fs;  // f*_lane (absolute; mine)
  double rt, ut[3], G[9], Pi[6];
  int nD;
};

// fdev: this lane's pulled deviation (0 where missing), fodev: the node's own deviation of this
// lane's direction, both in FP64.
__device__ inline void wall_targets64(const BArgs& a, const Bodies& bd, const LaneNb& h, const LaneU64& u, int lane,
                                      double fdev, double fodev, WallLane64& w) {
  const int i = lane < 27 ? lane : 13;
  w.mine = lane < 27 && ((h.dbar >> lane) & 1u);
  w.q = 0.0;
  w.uw[0] = w.uw[1] = w.uw[2] = 0.0;
  w.kb = -1;
  if (w.mine) link_geometry<false>(a, bd, i, h.x, h.y, h.z, w.q, w.uw, w.kb);
  w.fb = __shfl(fodev, opp(i), GROUP);
  double tu[3] = {0.0, 0.0, 0.0}, trs = 0.0, trd = 0.0;
  if (w.mine) {
    const bool fluid = (h.fluid >> lane) & 1u;
    const double inv = 1.0 / (1.0 + w.q);
#pragma unroll
    for (int c = 0; c < 3; ++c) tu[c] = (w.q * (fluid ? u.U[c] : w.uw[c]) + w.uw[c]) * inv;
    trs = w.fb;
    trd = 6.0 * wd(i) * a.rho0 * (cx(i) * w.uw[0] + cy(i) * w.uw[1] + cz(i) * w.uw[2]);
  } else if (lane < 27) {
    trs = fdev;
  }
  const double rstat = gsum(trs), rdyn = gsum(trd);  // rstat: sum of deviations (weights add to 1)
  w.nD = __popc(h.dbar);
  const double invn = 1.0 / (double)w.nD;
#pragma unroll
  for (int c = 0; c < 3; ++c) w.ut[c] = gsum(tu[c]) * invn;
  w.rt = 1.0 + rstat + rdyn;
  grad_u_grp64(h, u, w.G);
  pressure_tensor(w.rt, w.ut, w.G, a.beta64, w.Pi);
  w.fs = w.mine ? grad_pop(i, w.rt, w.ut, w.Pi) : 0.0;
}

// Adjoint of the boundary rules of Secs. III / IV.A at the listed nodes, in the lane-parallel
// form of the forward wall kernel: one node per group of 32 lanes, lane i < 27 owning direction
// i.  The reconstruction is rebuilt in FP64 (wall_targets64); the FP64 collision VJP and the
// reverse of the reconstruction run per lane with butterfly sums.  Listed nodes without missing
// populations (inlet and outlet rows, refill nodes) take the plain collision VJP here: their
// forward values are the wall kernel's, and the adjoint bulk kernel skips FL_SPECIAL nodes.
template <int S, bool FORCE>
__global__ __launch_bounds__(64) void k_adj_boundary(const BArgs a, const Bodies bd, const AdjArgs j,
                                                     const AdjBodyArgs p) {
  using C = Codec<S>;
  using E = typename C::E;
  const E* __restrict__ A = (const E*)a.A;
  int64_t count = a.n_static + (a.moving ? (int64_t)*a.dyn_count : 0);
  if (count > a.cap) count = a.cap;
  const int lane = threadIdx.x & (GROUP - 1), g = threadIdx.x / GROUP;
  const int i = lane < 27 ? lane : 13;
  for (int64_t base = 2 * (int64_t)blockIdx.x; base < count; base += 2 * (int64_t)gridDim.x) {
    // a group past the end repeats the block's first node and writes nothing
    const int64_t k = base + g;
    const long n = a.list[k < count ? k : base];
    LaneNb h;
    lane_gather<S, true, false>(a, A, n, lane, h);
    const bool active = k < count;
    const double gpi = lane < 27 ? (double)j.lam_in[(long)i * a.N + n] : 0.0;
    const uint32_t dmask = h.dbar;
    // FP64 deviations: the stored ones widened exactly, except at nodes uncovered in this step,
    // whose refill values are taken unrounded -- the node's own (a refill node) and pulled ones
    double fdev = (double)h.f, fodev = (double)h.fo;
    if (lane < 27) {
      if ((a.flags[n] & (FL_SOLID_PREV | FL_SOLID)) == FL_SOLID_PREV) {
        const uint32_t sl = (uint32_t)j.slot[n];
        if (sl < (uint32_t)a.cap) fodev = j.r64[(size_t)sl * 27 + i] - wd(i);
      }
      if (!((dmask >> lane) & 1u)) {
        int sx = h.x - cx(i);
        if (a.channel) sx = sx >= a.nx ? a.nx - 1 : sx;
        else sx = wrap(sx, a.nx);
        const long s = node_at(a, sx, wrap(h.y - cy(i), a.ny), wrap(h.z - cz(i), a.nz));
        if ((a.flags[s] & (FL_SOLID_PREV | FL_SOLID)) == FL_SOLID_PREV) {
          const uint32_t sl = (uint32_t)j.slot[s];
          if (sl < (uint32_t)a.cap) fdev = j.r64[(size_t)sl * 27 + i] - wd(i);
        }
      }
    }
    WallLane64 w;
    w.mine = false;
    if (dmask) {
      LaneU64 u;
      lane_u64(a, j.m64, h, lane, u);
      wall_targets64(a, bd, h, u, lane, fdev, fodev, w);
    }
    // collision input: f*_i (absolute) where missing, else the pulled value in FP64
    const double fdi = lane < 27 ? (((dmask >> lane) & 1u) ? w.fs : wd(i) + fdev) : 0.0;
    double Fx = 0.0, Fy = 0.0, Fz = 0.0;
    if (FORCE) {
      Fx = a.F[n];
      Fy = a.F[a.N + n];
      Fz = a.F[2 * a.N + n];
    }
    double gFn[3];
    const double gi = kbc_vjp_lanes<FORCE>(lane, fdi, gpi, a.beta64, Fx, Fy, Fz, gFn, a.stab == STAB_LBGK);
    if (FORCE && j.gF && active && lane == 0) {
      j.gF[n] += (float)gFn[0];
      j.gF[a.N + n] += (float)gFn[1];
      j.gF[2 * a.N + n] += (float)gFn[2];
    }
    if (!dmask) {
      if (active && lane < 27) adj_push(a, j, i, h.x, h.y, h.z, (float)gi);
    } else {
      double grl = 0.0, gul[3] = {0.0, 0.0, 0.0}, gPl[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, ga = 0.0;
      if (w.mine) {
        double gfs = gi;
        if (p.loss && w.kb >= 0)
          gfs -= p.w[w.kb][0] * (cx(i) - w.uw[0]) + p.w[w.kb][1] * (cy(i) - w.uw[1]) + p.w[w.kb][2] * (cz(i) - w.uw[2]);
        grad_pop_vjp(i, gfs, w.rt, w.ut, grl, gul, gPl);
      }
      double gr = gsum(grl), gu[3], gP[6], gG[9];
#pragma unroll
      for (int c = 0; c < 3; ++c) gu[c] = gsum(gul[c]);
#pragma unroll
      for (int c = 0; c < 6; ++c) gP[c] = gsum(gPl[c]);
      pressure_vjp(w.rt, w.ut, w.G, a.beta64, gP, gr, gu, gG);
      if (active && lane < 27) {
        if (!w.mine) {
          adj_push(a, j, i, h.x, h.y, h.z, (float)(gi + gr));
        } else {
          double vbb = gr;
          double guw[3];
          const double qd = w.q, inv = 1.0 / (w.nD * (1.0 + qd));
          const double cv[3] = {(double)cx(i), (double)cy(i), (double)cz(i)};
#pragma unroll
          for (int c = 0; c < 3; ++c) guw[c] = gr * 6.0 * wd(i) * a.rho0 * cv[c] + gu[c] * inv;
          if (p.loss && w.kb >= 0) {
            const double fbd = wd(opp(i)) + w.fb;
            vbb += p.w[w.kb][0] * (-cv[0] - w.uw[0]) + p.w[w.kb][1] * (-cv[1] - w.uw[1]) +
                   p.w[w.kb][2] * (-cv[2] - w.uw[2]);
#pragma unroll
            for (int c = 0; c < 3; ++c) guw[c] += p.w[w.kb][c] * (w.fs - fbd);
          }
          // the only writer of this entry: its puller, the solid node, leaves it to this kernel
          j.lam_out[(long)opp(i) * a.N + n] = (float)vbb;
          if (!(a.channel && h.x - cx(i) < 0)) adj_push(a, j, i, h.x, h.y, h.z, 0.f);
          // u_f and q
          double uf[3];
          if ((h.fluid >> lane) & 1u) {
            const long nf = neighbour(a, h.x, h.y, h.z, cx(i), cy(i), cz(i));
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              uf[c] = j.m64[c * a.N + nf];
              addU(a, j, c, nf, gu[c] * qd * inv);
            }
          } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              uf[c] = w.uw[c];
              guw[c] += gu[c] * qd * inv;
            }
          }
          if (w.kb >= 0) {
            const double gq =
                (gu[0] * (uf[0] - w.uw[0]) + gu[1] * (uf[1] - w.uw[1]) + gu[2] * (uf[2] - w.uw[2])) * inv / (1.0 + qd);
            const BodyDev& b = bd.b[w.kb];
            double dqdc[3];
            if (b.kind == ELBM_BODY_SPHERE) {
              const double r[3] = {h.x - b.c1[0] - qd * cv[0], h.y - b.c1[1] - qd * cv[1], h.z - b.c1[2] - qd * cv[2]};
              const double rv = r[0] * cv[0] + r[1] * cv[1] + r[2] * cv[2];
#pragma unroll
              for (int c = 0; c < 3; ++c) dqdc[c] = -r[c] / rv;
            } else {
              const double nv = b.n[0] * cv[0] + b.n[1] * cv[1] + b.n[2] * cv[2];
#pragma unroll
              for (int c = 0; c < 3; ++c) dqdc[c] = -b.n[c] / nv;
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) ga += guw[c] * p.dU1[w.kb][c] + gq * dqdc[c] * p.dc1[w.kb][c];
          }
        }
      }
      // dL/d(amp) of the group's links, summed over the group first: one atomic per node and body
      // (per-link atomics on the one address serialise)
      for (int kb = 0; kb < bd.nb; ++kb) {
        const double sg = gsum(w.mine && w.kb == kb ? ga : 0.0);
        if (active && lane == 0 && sg != 0.0) atomicAdd(&p.gamp[kb], sg);
      }
      // transpose of the gradient stencil: lanes 0..8 take one (axis, component) pair each
      if (active && lane < 9) grad_u_vjp_one(a, j, h, lane / 3, lane % 3, gG[3 * (lane % 3) + lane / 3]);
    }
  }
}

// Flag bit FL_NEAR_REFILL of the nodes next to an uncovered node (set = true, or cleared); 32-bit
// atomics on the word holding the flag byte (the flag array is padded to 256 bytes).
__device__ inline void mark_near(uint8_t* flags, long m, bool set) {
  uint32_t* word = (uint32_t*)(flags + (m & ~3L));
  const uint32_t bit = (uint32_t)FL_NEAR_REFILL << (8 * (m & 3));
  if (set) atomicOr(word, bit);
  else atomicAnd(word, ~bit);
}

// The refill of the step in FP64 (k_refill's rule, from the FP64 U^t and R^t): the populations of
// each uncovered node go to its list slot of the table r64, the slot to the node's entry of slot[],
// and the node's neighbours that are fluid at t+1 get FL_NEAR_REFILL, so that the reverse kernels
// read the unrounded values where they pull from it.
__global__ __launch_bounds__(64) void k_adj_refill64(const BArgs a, const Bodies bd, const AdjArgs j) {
  int64_t count = a.n_static + (a.moving ? (int64_t)*a.dyn_count : 0);
  if (count > a.cap) count = a.cap;
  const int lane = threadIdx.x & (GROUP - 1), g = threadIdx.x / GROUP;
  for (int64_t k = a.n_static + 2 * (int64_t)blockIdx.x + g; k < count; k += 2 * (int64_t)gridDim.x) {
    const long n = a.list[k];
    if (!(a.flags[n] & FL_SOLID_PREV)) continue;  // uniform over the group
    LaneNb h;
    lane_gather<ELBM_STORAGE_F32, false, false>(a, nullptr, n, lane, h);
    LaneU64 u;
    lane_u64(a, j.m64, h, lane, u);
    int kb = first_body(bd, false, h.x, h.y, h.z);
    if (kb < 0) kb = 0;
    const BodyDev& b = bd.b[kb];
    const double r[3] = {h.x - b.c1[0], h.y - b.c1[1], h.z - b.c1[2]};
    double uw[3];
    uw[0] = b.U1[0] + (b.omega[1] * r[2] - b.omega[2] * r[1]);
    uw[1] = b.U1[1] + (b.omega[2] * r[0] - b.omega[0] * r[2]);
    uw[2] = b.U1[2] + (b.omega[0] * r[1] - b.omega[1] * r[0]);
    const uint32_t nbm = h.fluid0 & ~(1u << 13);
    const double rs = gsum(lane != 13 ? u.R : 0.0);
    const int m = __popc(nbm);
    const double ravg = m ? rs / (double)m : a.rho0;
    double G[9], Pi[6];
    grad_u_grp64(h, u, G);
    pressure_tensor(ravg, uw, G, a.beta64, Pi);
    if (lane < 27) j.r64[(size_t)k * 27 + lane] = grad_pop(lane, ravg, uw, Pi);
    if (lane == 0) j.slot[n] = (int32_t)k;
    if (lane < 27 && lane != 13 && ((h.fluid >> lane) & 1u))
      mark_near(const_cast<uint8_t*>(a.flags), neighbour(a, h.x, h.y, h.z, cx(lane), cy(lane), cz(lane)), true);
  }
}

// Adjoint of the refill (which writes Grad's distribution into A^t at the nodes uncovered by the
// step): the completed dL/dA^t of a refill node goes through Grad's distribution to R^t of its
// neighbours, U^t of its stencil and the body's amplitude; the node's own entries are then zero
// (its stored A^t is overwritten and influences nothing).  FP64, from the FP64 U^t and R^t.
__global__ __launch_bounds__(64) void k_adj_refill(const BArgs a, const Bodies bd, const AdjArgs j,
                                                   const AdjBodyArgs p) {
  int64_t count = a.n_static + (a.moving ? (int64_t)*a.dyn_count : 0);
  if (count > a.cap) count = a.cap;
  const int lane = threadIdx.x & (GROUP - 1), g = threadIdx.x / GROUP;
  for (int64_t k = a.n_static + 2 * (int64_t)blockIdx.x + g; k < count; k += 2 * (int64_t)gridDim.x) {
    const long n = a.list[k];
    if (!(a.flags[n] & FL_SOLID_PREV)) continue;  // uniform over the group
    LaneNb h;
    lane_gather<ELBM_STORAGE_F32, false, false>(a, nullptr, n, lane, h);
    LaneU64 u;
    lane_u64(a, j.m64, h, lane, u);
    // forward recomputation, as k_refill
    int kb = first_body(bd, false, h.x, h.y, h.z);
    if (kb < 0) kb = 0;
    const BodyDev& b = bd.b[kb];
    const double r[3] = {h.x - b.c1[0], h.y - b.c1[1], h.z - b.c1[2]};
    double uw[3];
    uw[0] = b.U1[0] + (b.omega[1] * r[2] - b.omega[2] * r[1]);
    uw[1] = b.U1[1] + (b.omega[2] * r[0] - b.omega[0] * r[2]);
    uw[2] = b.U1[2] + (b.omega[0] * r[1] - b.omega[1] * r[0]);
    const uint32_t nbm = h.fluid0 & ~(1u << 13);
    const double rs = gsum(lane != 13 ? u.R : 0.0);
    const int m = __popc(nbm);
    const double ravg = m ? rs / (double)m : a.rho0;
    double G[9], Pi[6];
    grad_u_grp64(h, u, G);
    pressure_tensor(ravg, uw, G, a.beta64, Pi);
    // reverse: the completed dL/dA^t of the refilled entries goes through Grad's distribution;
    // the entries themselves were overwritten, so their adjoint restarts at zero
    double grl = 0.0, gul[3] = {0.0, 0.0, 0.0}, gPl[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (lane < 27) {
      const double gi = (double)j.lam_out[(long)lane * a.N + n];
      j.lam_out[(long)lane * a.N + n] = 0.f;
      grad_pop_vjp(lane, gi, ravg, uw, grl, gul, gPl);
    }
    double gr = gsum(grl), gu[3], gP[6], gG[9];
#pragma unroll
    for (int c = 0; c < 3; ++c) gu[c] = gsum(gul[c]);
#pragma unroll
    for (int c = 0; c < 6; ++c) gP[c] = gsum(gPl[c]);
    pressure_vjp(ravg, uw, G, a.beta64, gP, gr, gu, gG);
    if (m && lane < 27 && ((nbm >> lane) & 1u))
      atomicAdd(&j.gUR[3 * a.N + neighbour(a, h.x, h.y, h.z, cx(lane), cy(lane), cz(lane))], gr / (double)m);
    if (lane == 0) atomicAdd(&p.gamp[kb], gu[0] * p.dU1[kb][0] + gu[1] * p.dU1[kb][1] + gu[2] * p.dU1[kb][2]);
    if (lane < 9) grad_u_vjp_one(a, j, h, lane / 3, lane % 3, gG[3 * (lane % 3) + lane / 3]);
    // every reader of the marks (bulk and wall kernels) has run: clear them
    if (lane < 27 && lane != 13 && ((h.fluid >> lane) & 1u))
      mark_near(const_cast<uint8_t*>(a.flags), neighbour(a, h.x, h.y, h.z, cx(lane), cy(lane), cz(lane)), false);
  }
}

// Channel faces, after the boundary adjoint: add the outlet-copy contributions of the side buffer.
// One thread per (direction k with c_x = -1, y, z); for each k the targets are distinct.
__global__ __launch_bounds__(256) void k_adj_outlet(const BArgs a, const AdjArgs j) {
  const long face = (long)a.ny * a.nz, total = 9 * face;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const int k = (int)(idx / face);
    const long r = idx - k * face;
    const int y = (int)(r % a.ny), z = (int)(r / a.ny);
    const int i = 3 * k;
    const long tgt = node_at(a, a.nx - 1, wrap(y - cy(i), a.ny), wrap(z - cz(i), a.nz));
    j.lam_out[i * a.N + tgt] += j.side[(size_t)k * face + (size_t)z * a.ny + y];
  }
}

// dL/dU^t, dL/dR^t -> dL/dA^t at nodes fluid at t (U = (j - F/2)/rho, R = rho), or dL/d(amp) at
// nodes solid at t (U = rigid-body velocity at t).  Clears the accumulators it consumes.
// Launched on the boxes where the wall rules read U^t and R^t (around the bodies, the inlet slab),
// which hold every accumulated entry.
__global__ __launch_bounds__(256) void k_adj_macro(const BArgs a, const Bodies bd, const AdjArgs j, const AdjBodyArgs p,
                                                   const Box2 box) {
  const long total = box.count();
  double acc[ELBM_MAX_BODIES];  // this thread's dL/d(amp) per body, summed over the wave at the end
#pragma unroll
  for (int q = 0; q < ELBM_MAX_BODIES; ++q) acc[q] = 0.0;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    int bx, by, bz;
    box2_node(box, idx, bx, by, bz);
    const long n = node_at(a, bx, by, bz);
    // every operand is loaded up front, independent of the others (one memory round trip): the
    // accumulators, the FP64 U^t and R^t of k_macro64 (the same rule: U = (j - F/2)/rho from the
    // exactly widened stored deviations), the node's 27 entries of dL/dA^t and its flags
    const double gU0 = j.gUR[n], gU1 = j.gUR[a.N + n], gU2 = j.gUR[2 * a.N + n], gR = j.gUR[3 * a.N + n];
    const double U0 = j.m64[n], U1 = j.m64[a.N + n], U2 = j.m64[2 * a.N + n], rho = j.m64[3 * a.N + n];
    const uint8_t fl = a.flags[n];
    float lam[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) lam[i] = j.lam_out[i * a.N + n];
    if (gU0 == 0.0 && gU1 == 0.0 && gU2 == 0.0 && gR == 0.0) continue;
    j.gUR[n] = 0.0;
    j.gUR[a.N + n] = 0.0;
    j.gUR[2 * a.N + n] = 0.0;
    j.gUR[3 * a.N + n] = 0.0;
    if (fl & FL_SOLID_PREV) {
      int x, y, z;
      node_xyz(a, n, x, y, z);
      int kb = first_body(bd, false, x, y, z);
      if (kb < 0) kb = 0;
      const double v = gU0 * p.dU0[kb][0] + gU1 * p.dU0[kb][1] + gU2 * p.dU0[kb][2];
#pragma unroll
      for (int q = 0; q < ELBM_MAX_BODIES; ++q) acc[q] += q == kb ? v : 0.0;
      continue;
    }
    const double irho = 1.0 / rho;
    const double h0 = gU0 * irho, h1 = gU1 * irho, h2 = gU2 * irho;
    const double base = gR - (h0 * U0 + h1 * U1 + h2 * U2);
#pragma unroll
    for (int i = 0; i < 27; ++i) j.lam_out[i * a.N + n] = lam[i] + (float)(base + h0 * cx(i) + h1 * cy(i) + h2 * cz(i));
    if (a.F && j.gF) {
      j.gF[n] -= (float)(0.5 * h0);
      j.gF[a.N + n] -= (float)(0.5 * h1);
      j.gF[2 * a.N + n] -= (float)(0.5 * h2);
    }
  }
  // one atomic per wave and body (every lane of the launch reaches this point)
  for (int q = 0; q < bd.nb; ++q) {
    double v = acc[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0 && v != 0.0) atomicAdd(&p.gamp[q], v);
  }
}

// ---------------------------------------------------------------------------------------------
static BArgs bargs(elbm_ctx* c, const void* A) {
  BArgs a;
  a.A = A;
  a.B = nullptr;
  a.flags = c->flags;
  a.macro = c->macro;
  a.F = c->bodyforce;
  a.list = c->blist;
  a.dyn_count = &c->cnt->dyn_count;
  a.brec = c->brec;
  a.fix_list = nullptr;  // the adjoint kernels queue nothing
  a.fix_count = nullptr;
  a.diag = c->cnt;
  a.stats = 0;
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
  a.channel = c->p.bc_x == ELBM_BC_CHANNEL;
  a.fp64 = !(c->p.flags & ELBM_FLAG_NO_FP64);
  a.stream_only = 0;
  a.stab = c->stab;
  a.beta = (float)c->beta;
  a.inv_beta = (float)(1.0 / c->beta);
  a.beta64 = c->beta;
  a.thr = (float)c->fp64_thr;
  a.rho0 = c->p.rho0;
  for (int e = 0; e < 3; ++e) a.u_in[e] = c->p.u_inlet[e];
  return a;
}

static void amp_derivatives(const elbm_body& b, double t, double dc[3], double dU[3]) {
  double sn = 0.0, cs = 0.0, om = 0.0;
  if (b.period != 0.0) {
    const double ph = ((2.0 * M_PI) * t) / b.period;
    sn = sin(ph);
    cs = cos(ph);
    om = (2.0 * M_PI) / b.period;
  }
  for (int a = 0; a < 3; ++a) {
    dc[a] = sn * b.dir[a];
    dU[a] = (om * cs) * b.dir[a];
  }
}

// FP64 U^t, R^t on the boxes where the wall rules read them.
template <int S>
static void macro64_fields(elbm_ctx* c, const void* A, const Bodies& bd) {
  const Box2 bb = macro_boxes(c, bd, true);
  if (bb.count() == 0) return;
  hipLaunchKernelGGL((k_macro64<S>), grid_for(bb.count()), dim3(256), 0, c->stream, (const typename Codec<S>::E*)A,
                     c->lay, (const uint8_t*)c->flags, c->adj_macro64, c->bodyforce, bb, c->p.nx, c->p.ny,
                     (int64_t)c->N, c->p.rho0, bd);
}

template <int S>
static hipError_t adj_launch(elbm_ctx* c, const BArgs& a, const Bodies& bd, const AdjArgs& j, const AdjBodyArgs& p) {
  int bx = 256;
  while (bx > 32 && (c->p.nx % bx) != 0) bx >>= 1;
  if (c->p.nx < bx) bx = 32;
  const dim3 blk(bx, 256 / bx, 1);
  const dim3 grd((c->p.nx + bx - 1) / bx, (c->p.ny + blk.y - 1) / blk.y, c->p.nz);
  const bool geo = c->flags != nullptr, force = c->bodyforce != nullptr;
  if (geo) macro64_fields<S>(c, a.A, bd);
  if (geo && c->moving) {
    const dim3 gr((unsigned)std::min<int64_t>(std::max<int64_t>((a.cap - a.n_static + 1) / 2, 1), 1024));
    hipLaunchKernelGGL(k_adj_refill64, gr, dim3(64), 0, c->stream, a, bd, j);
  }
  const dim3 gf = grid_for(9L * c->p.ny * c->p.nz);
  if (geo && force) hipLaunchKernelGGL((k_adj_bulk<S, true, true>), grd, blk, 0, c->stream, a, j);
  else if (geo) hipLaunchKernelGGL((k_adj_bulk<S, true, false>), grd, blk, 0, c->stream, a, j);
  else if (force) hipLaunchKernelGGL((k_adj_bulk<S, false, true>), grd, blk, 0, c->stream, a, j);
  else hipLaunchKernelGGL((k_adj_bulk<S, false, false>), grd, blk, 0, c->stream, a, j);
  if (geo) {
    // a grid-stride loop over the list: about two groups per SIMD (the list length is on the device)
    const dim3 gb((unsigned)std::min<int64_t>(std::max<int64_t>((a.cap + 1) / 2, 1), 2048));
    if (force) hipLaunchKernelGGL((k_adj_boundary<S, true>), gb, dim3(64), 0, c->stream, a, bd, j, p);
    else hipLaunchKernelGGL((k_adj_boundary<S, false>), gb, dim3(64), 0, c->stream, a, bd, j, p);
    if (a.channel) hipLaunchKernelGGL(k_adj_outlet, gf, dim3(256), 0, c->stream, a, j);
    if (c->moving) {
      const dim3 gr((unsigned)std::min<int64_t>(std::max<int64_t>((a.cap - a.n_static + 1) / 2, 1), 1024));
      hipLaunchKernelGGL(k_adj_refill, gr, dim3(64), 0, c->stream, a, bd, j, p);
    }
    const Box2 bb = macro_boxes(c, bd, true);
    if (bb.count() > 0)
      hipLaunchKernelGGL(k_adj_macro, grid_for(bb.count()), dim3(256), 0, c->stream, a, bd, j, p, bb);
  }
  return hipGetLastError();
}

hipError_t launch_adjoint(elbm_ctx* c, int64_t t, const void* A, const float* lam_in, float* lam_out,
                          const double* w_force, float* gF) {
  const Bodies bd = make_bodies(c, (double)t);
  if (c->flags) {
    hipError_t e = geometry_for_step(c, bd);
    if (e != hipSuccess) return e;
    e = macro_fields(c, A, bd, true);
    if (e != hipSuccess) return e;
    // the forward step refills uncovered nodes into A^t before streaming; do the same here
    e = launch_refill(c, bd, const_cast<void*>(A));
    if (e != hipSuccess) return e;
  }
  const BArgs a = bargs(c, A);
  AdjArgs j;
  j.lam_in = lam_in;
  j.lam_out = lam_out;
  j.side = c->adj_side;
  j.gF = gF;
  j.gUR = c->adj_gUR;
  j.m64 = c->adj_macro64;
  j.r64 = c->adj_refill64;
  j.slot = c->adj_slot;
  AdjBodyArgs p{};
  p.gamp = c->adj_gamp;
  p.loss = w_force != nullptr;
  for (int k = 0; k < c->nb; ++k) {
    amp_derivatives(c->bodies[k], (double)t + 1.0, p.dc1[k], p.dU1[k]);
    double dc0[3];
    amp_derivatives(c->bodies[k], (double)t, dc0, p.dU0[k]);
    for (int e = 0; e < 3; ++e) p.w[k][e] = w_force ? w_force[3 * k + e] : 0.0;
  }
  switch (c->p.storage) {
    case ELBM_STORAGE_F32: return adj_launch<ELBM_STORAGE_F32>(c, a, bd, j, p);
    case ELBM_STORAGE_F16: return adj_launch<ELBM_STORAGE_F16>(c, a, bd, j, p);
    default: return adj_launch<ELBM_STORAGE_BF16>(c, a, bd, j, p);
  }
}

}  // namespace elbm
