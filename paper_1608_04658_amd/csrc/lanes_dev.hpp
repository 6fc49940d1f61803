// lanes_dev.hpp -- the lane-parallel form of the per-node work: one node per group of GROUP = 32
// lanes (two per wavefront), lane i < 27 owning direction i.  Sums and extrema over the directions
// are butterfly reductions inside the group (fixed order, deterministic); the KBC collision of
// Sec. II in this form serves the wall kernel (FP32) and the FP64 fix-up kernel.
#pragma once

#include "elbm_internal.hpp"

namespace elbm {

// Reductions over the lanes of the calling group (GROUP = 32 is defined with the shared
// declarations); every lane receives the result, bit-identical on all lanes.  Four steps inside each
// 16-lane row through DPP operand modifiers (lane pairs 1, 2 apart, then the mirror images in each
// 8-lane half and in the row), which the compiler folds into the arithmetic instruction, and one
// exchange of the two rows of the group through ds_swizzle (lane l and l ^ 16): one LDS-pipe step
// where a shuffle butterfly takes five.  The pairs of every step hold identical partial results,
// so each lane adds the same two values.
template <int CTRL>
__device__ __forceinline__ float dpp32(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp64(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ float row_swap(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, v), 0x401F));
}
__device__ __forceinline__ double row_swap(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)(uint32_t)b, 0x401F);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(uint32_t)(b >> 32), 0x401F);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
static_assert(GROUP == 32, "the group reductions cover two 16-lane rows");
constexpr int DPP_XOR1 = 0xB1;      // quad_perm [1, 0, 3, 2]
constexpr int DPP_XOR2 = 0x4E;      // quad_perm [2, 3, 0, 1]
constexpr int DPP_HMIRROR = 0x141;  // row_half_mirror: lane 7 - l in each 8-lane half
constexpr int DPP_MIRROR = 0x140;   // row_mirror: lane 15 - l in each row
template <typename T, typename Op>
__device__ __forceinline__ T greduce(T v, Op op) {
  if constexpr (sizeof(T) == 4) {
    v = op(v, dpp32<DPP_XOR1>(v));
    v = op(v, dpp32<DPP_XOR2>(v));
    v = op(v, dpp32<DPP_HMIRROR>(v));
    v = op(v, dpp32<DPP_MIRROR>(v));
  } else {
    v = op(v, dpp64<DPP_XOR1>(v));
    v = op(v, dpp64<DPP_XOR2>(v));
    v = op(v, dpp64<DPP_HMIRROR>(v));
    v = op(v, dpp64<DPP_MIRROR>(v));
  }
  return op(v, row_swap(v));
}
__device__ __forceinline__ float gsum(float v) {
  return greduce(v, [](float x, float y) { return x + y; });
}
__device__ __forceinline__ double gsum(double v) {
  return greduce(v, [](double x, double y) { return x + y; });
}
__device__ __forceinline__ float gmax(float v) {
  return greduce(v, [](float x, float y) { return fmaxf(x, y); });
}
__device__ __forceinline__ float gmin(float v) {
  return greduce(v, [](float x, float y) { return fminf(x, y); });
}
__device__ __forceinline__ double gmax(double v) {
  return greduce(v, [](double x, double y) { return fmax(x, y); });
}
__device__ __forceinline__ double gmin(double v) {
  return greduce(v, [](double x, double y) { return fmin(x, y); });
}
// Bit l = predicate of lane l of the calling group.
__device__ __forceinline__ uint32_t gballot(bool p) {
  const unsigned long long b = __ballot(p);
  return (uint32_t)(b >> (threadIdx.x & 32u));
}

// The KBC collision (Sec. II) in the lane-parallel form of the wall and FP64 fix-up kernels: lane
// i < 27 holds d_i = f_i - W_i and receives the post-collision deviation; lanes >= 27 pass zeros.
// Same formulas as kbc_collide<T>, with every sum over directions a butterfly reduction inside the
// group.  r receives gamma, <dh|dh>, rho and the shear estimate for the FP64 rule (equal on all
// lanes of the group).
template <typename T, bool FORCE, int STAB = STAB_KBC>
__device__ inline T kbc_collide_lanes(int lane, T d, T beta, T inv_beta, T Fx, T Fy, T Fz, KbcOut<T>& r) {
  const bool own = lane < 27;
  const int i = own ? lane : 13;
  if (!own) d = T(0);
  const T c0 = (T)cx(i), c1 = (T)cy(i), c2 = (T)cz(i);
  const T dr = gsum(d), jx = gsum(c0 * d), jy = gsum(c1 * d), jz = gsum(c2 * d);
  const T Q200 = gsum(c0 * c0 * d), Q020 = gsum(c1 * c1 * d), Q002 = gsum(c2 * c2 * d);
  const T Q110 = gsum(c0 * c1 * d), Q101 = gsum(c0 * c2 * d), Q011 = gsum(c1 * c2 * d);
  const T rho = T(1) + dr;
  const T rinv = rcp_(rho);
  const T ux = jx * rinv, uy = jy * rinv, uz = jz * rinv;
  T ex[3], ey[3], ez[3], psx[3], psy[3], psz[3], sx, sy, sz;
  axis_dev(ux, ex, psx, sx);
  axis_dev(uy, ey, psy, sy);
  axis_dev(uz, ez, psz, sz);
  const T third = T(1.0 / 3.0);
  const T dM200 = Q200 - (dr * (T(1) + T(2) * sx) + T(2) * sx) * third;
  const T dM020 = Q020 - (dr * (T(1) + T(2) * sy) + T(2) * sy) * third;
  const T dM002 = Q002 - (dr * (T(1) + T(2) * sz) + T(2) * sz) * third;
  const T tr3 = (dM200 + dM020 + dM002) * third;
  const T sfx = T(0.5) * (dM200 - tr3), sfy = T(0.5) * (dM020 - tr3), sfz = T(0.5) * (dM002 - tr3);
  const T sxy = T(0.25) * (Q110 - jx * uy), sxz = T(0.25) * (Q101 - jx * uz), syz = T(0.25) * (Q011 - jy * uz);
  // feq_i - W_i = W_i (dr + rho P_i)
  const T a_ = ey[cy(i) + 1], b_ = ez[cz(i) + 1];
  const T pyz = a_ + b_ + a_ * b_;
  const T e_ = ex[cx(i) + 1];
  const T P = e_ + pyz + e_ * pyz;
  const T fdev = T(wd(i)) * (dr + rho * P);
  constexpr bool CENTRAL = (STAB & STAB_CENTRAL) != 0;
  T ds = T(0);
  if (CENTRAL) {
    // shear part through the dual basis of the shifted velocities, as in kbc_collide
    T cbx[3][3], cby[3][3], cbz[3][3];
    central_basis(ux, cbx);
    central_basis(uy, cby);
    central_basis(uz, cbz);
    const int x = cx(i) + 1, y = cy(i) + 1, z = cz(i) + 1;
    ds = (T(2) * sfx) * cbx[2][x] * cby[0][y] * cbz[0][z] + (T(2) * sfy) * cbx[0][x] * cby[2][y] * cbz[0][z] +
         (T(2) * sfz) * cbx[0][x] * cby[0][y] * cbz[2][z] + (T(4) * sxy) * cbx[1][x] * cby[1][y] * cbz[0][z] +
         (T(4) * sxz) * cbx[1][x] * cby[0][y] * cbz[1][z] + (T(4) * syz) * cbx[0][x] * cby[1][y] * cbz[1][z];
  } else if (nnz(i) == 1) {
    ds = cx(i) ? sfx : (cy(i) ? sfy : sfz);
  } else if (nnz(i) == 2) {
    ds = cz(i) == 0 ? c0 * c1 * sxy : (cy(i) == 0 ? c0 * c2 * sxz : c1 * c2 * syz);
  }
  if (!own) ds = T(0);
  T h = own ? (d - fdev) - ds : T(0);
  // remove the rounding residue of the mass and momentum of dh (rest and face populations)
  const T hm = gsum(h), hx = gsum(c0 * h), hy = gsum(c1 * h), hz = gsum(c2 * h);
  if (own) {
    if (i == 13) h -= hm;
    else if (i == 14) h -= T(0.5) * hx;
    else if (i == 12) h += T(0.5) * hx;
    else if (i == 16) h -= T(0.5) * hy;
    else if (i == 10) h += T(0.5) * hy;
    else if (i == 22) h -= T(0.5) * hz;
    else if (i == 4) h += T(0.5) * hz;
  }
  const T ife = (rinv * (psy[cy(i) + 1] * psz[cz(i) + 1])) * psx[cx(i) + 1];
  const T th = h * ife;
  const T b = gsum(th * h), a = gsum(th * ds);
  T gamma = (b > T(1e-30)) ? inv_beta - (T(2) - inv_beta) * ratio_(a, b) : T(2);
  if ((STAB & 3) == STAB_LBGK) gamma = T(2);
  if ((STAB & 3) == STAB_EXACT && b > T(1e-30)) {
    // bracketed Newton on eq. gamma_min, as in kbc_collide (sums and extrema over the group)
    T clo = T(-1e6), chi = T(1e6);
    if (own) {
      // argument of the logarithm = p0 + p1 g
      const T p0 = T(1) + (h - (T(2) * beta - T(1)) * ds) * ife, p1 = -beta * h * ife;
      if (p1 > T(0)) clo = -p0 / p1;
      else if (p1 < T(0)) chi = -p0 / p1;
    }
    T lo = fmax(gmax(clo), T(-1e6)), hi = fmin(gmin(chi), T(1e6));
    if (lo < hi) {
      const T tol = sizeof(T) == 4 ? T(1e-6) : T(1e-13);
      T g = (gamma > lo && gamma < hi) ? gamma : T(0.5) * (lo + hi);
      for (int it = 0; it < 64; ++it) {
        T Gl = T(0), dGl = T(0), Gal = T(0);
        const bool okl = own ? gamma_term(g, beta, h, ds, ife, Gl, dGl, Gal) : true;
        const T G = gsum(Gl), dG = gsum(dGl), Ga = gsum(Gal);
        const bool bad = gballot(!okl) != 0u;
        if (!bad && fabs(G) <= T(64) * eps_of<T>() * Ga) break;
        T gn;
        if (bad || !(dG < T(0))) {
          if (g < T(0.5) * (lo + hi)) lo = g;
          else hi = g;
          gn = T(0.5) * (lo + hi);
        } else {
          if (G > T(0)) lo = g;
          else hi = g;
          gn = g - G / dG;
          if (!(gn > lo && gn < hi)) gn = T(0.5) * (lo + hi);
        }
        const bool done = !(fabs(gn - g) > tol * fabs(gn));
        g = gn;
        if (done) break;
      }
      if (g > T(0)) gamma = g;
    }
  }
  const T s2 = CENTRAL ? gsum(ds * ds * ife)
                       : (T(27) * (sfx * sfx + sfy * sfy + sfz * sfz) + T(216) * (sxy * sxy + sxz * sxz + syz * syz)) * rinv;
  T out = d - (T(2) * beta) * ds - (beta * gamma) * h;
  if (FORCE) {
    const double rr = (double)rho;
    double p0[3], q0[3], w0[3], p1[3], q1[3], w1[3];
    axis_phi((double)ux, p0);
    axis_phi((double)uy, q0);
    axis_phi((double)uz, w0);
    axis_phi((double)ux + (double)Fx / rr, p1);
    axis_phi((double)uy + (double)Fy / rr, q1);
    axis_phi((double)uz + (double)Fz / rr, w1);
    const double e0 = rr * p0[cx(i) + 1] * q0[cy(i) + 1] * w0[cz(i) + 1];
    const double e1 = rr * p1[cx(i) + 1] * q1[cy(i) + 1] * w1[cz(i) + 1];
    out = (T)((double)out + (e1 - e0));
  }
  const bool dom = rho > T(0) && rho < T(FLT_BIG) && fabs(ux) < T(1) && fabs(uy) < T(1) && fabs(uz) < T(1);
  r = KbcOut<T>{gamma, b, rho, s2, dom};
  return own ? out : T(0);
}

}  // namespace elbm
