// elbm_internal.hpp -- shared declarations of the gfx950 entropic lattice Boltzmann library.
//
// Device helpers for the D3Q27 KBC step (Dorschner, Chikatamarla, Karlin, arXiv:1608.04658):
// lattice tables, the KBC collision (Sec. II), Grad's distribution and pressure tensor
// (Sec. III, eqs. grad, pressure, pressure2), population storage codecs, the structures the
// kernels receive (bodies, the triangulated surface, counters) and block-level scans.  The
// host-side context is in context.hpp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "elbm.h"

namespace elbm {

// ---------------------------------------------------------------------------------------------
// D3Q27 lattice.  i = 9 (cz+1) + 3 (cy+1) + (cx+1); opposite direction 26 - i; rest i = 13.
// Weights are the tensor products of w(0) = 2/3, w(+-1) = 1/6 (c_s^2 = 1/3).
__host__ __device__ constexpr int cx(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int cy(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int cz(int i) { return i / 9 - 1; }
__host__ __device__ constexpr int opp(int i) { return 26 - i; }
__host__ __device__ constexpr double w1d(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
__host__ __device__ constexpr double wd(int i) { return w1d(cx(i)) * w1d(cy(i)) * w1d(cz(i)); }
__host__ __device__ constexpr float wf(int i) { return (float)wd(i); }
__host__ __device__ constexpr int nnz(int i) { return (cx(i) != 0) + (cy(i) != 0) + (cz(i) != 0); }

// node flag bits
constexpr uint8_t FL_SOLID = 1;       // solid at the time level being produced (t+1)
constexpr uint8_t FL_SOLID_PREV = 2;  // solid at the previous time level (t)
constexpr uint8_t FL_SPECIAL = 4;     // handled by the boundary kernel (missing populations or refill)
constexpr uint8_t FL_NEAR_REFILL = 8; // reverse step only: pulls from a node uncovered in the step

// FP64 fix-up queue entries: node index, with this bit set when the node's pre-collision
// deviations already sit in the output buffer (wall nodes) instead of being pulled from A^t.
constexpr uint32_t FIX_PRE = 0x80000000u;

// ---------------------------------------------------------------------------------------------
// Placement of the populations in a population array.  Direction i of the node in column x of
// lattice row r = z ny + y sits at element r rs + i si + x:
//   structure of arrays [27][nz][ny][nx]:  rs = nx,     si = N;
//   rows interleaved    [nz][ny][27][nx]:  rs = 27 nx,  si = nx.
// Both keep x fastest, so a wavefront's access to one direction is one contiguous run either way.
// The interleaved form puts the 27 streams of a row next to each other: the 27 x 9 rows a workgroup
// gathers lie in 9 runs of 27 nx elements instead of 243 places up to 27 N apart.
struct PopLayout {
  int64_t si;  // stride between directions
  int64_t rs;  // stride between lattice rows
  int32_t nx, ny;
  int32_t interleaved;
  int32_t pad;
};
__host__ __device__ __forceinline__ int64_t pop_off(const PopLayout& L, int i, int x, int y, int z) {
  return ((int64_t)z * L.ny + y) * L.rs + (int64_t)i * L.si + x;
}
// Offset of direction 0 of node n = (z ny + y) nx + x (n < 2^31); direction i adds i si.
__device__ __forceinline__ int64_t pop_base_n(const PopLayout& L, int64_t n) {
  const uint32_t r = (uint32_t)n / (uint32_t)L.nx;
  const int x = (int)((uint32_t)n - r * (uint32_t)L.nx);
  return (int64_t)r * L.rs + x;
}

// ---------------------------------------------------------------------------------------------
// Population storage: every format stores the deviation d = f - W_i from the lattice weight (FP32,
// or FP16 / BF16 rounded to nearest even); arithmetic is FP32 (FP64 on the recomputation path).
// load/store take absolute populations, load_dev/store_dev deviations.
// Raw buffer resources on gfx950 (CDNA): fourth descriptor word of an untyped 32-bit buffer, and the
// cache-policy operand of a non-temporal access.
constexpr int BUF_WORD3 = 0x00020000;
constexpr int BUF_NT = 2;
constexpr int BUF_ALL = (int)0xFFFFFFFFu;  // record count: no range check on the 32-bit offsets

template <int S> struct Codec;
template <> struct Codec<ELBM_STORAGE_F32> {
  using E = float;
  static __device__ __forceinline__ float load(const E* p, float w) { return *p + w; }
  static __device__ __forceinline__ void store(E* p, float v, float w) { *p = v - w; }
  static __device__ __forceinline__ float load_dev(const E* p) { return *p; }
  static __device__ __forceinline__ void store_dev(E* p, float d) { *p = d; }
};
template <> struct Codec<ELBM_STORAGE_F16> {
  using E = _Float16;
  static __device__ __forceinline__ float load(const E* p, float w) { return (float)(*p) + w; }
  static __device__ __forceinline__ void store(E* p, float v, float w) { *p = (_Float16)(v - w); }
  static __device__ __forceinline__ float load_dev(const E* p) { return (float)(*p); }
  static __device__ __forceinline__ void store_dev(E* p, float d) { *p = (_Float16)d; }
};
// binary32 -> bfloat16, round to nearest even: gfx950's conversion instruction (v_cvt_pk_bf16_f32,
// one VALU operation where the integer form takes five per value; NaN stays a quiet NaN).  The empty
// asm statement (no instruction) makes v an opaque binary32 value: without it the compiler fuses a
// preceding (float) of a double into one double -> bfloat16 rounding, which differs from rounding
// the binary32 value at ties, and the stored populations would no longer be the rounding of the
// binary32 deviations that the inlet-slab staging and the tests assume.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float v) {
  __asm__("" : "+v"(v));
  return __builtin_bit_cast(uint16_t, (__bf16)v);
}
template <> struct Codec<ELBM_STORAGE_BF16> {
  using E = uint16_t;
  static __device__ __forceinline__ float load(const E* p, float w) { return __uint_as_float(((uint32_t)*p) << 16) + w; }
  static __device__ __forceinline__ void store(E* p, float v, float w) { *p = f32_to_bf16_rne(v - w); }
  static __device__ __forceinline__ float load_dev(const E* p) { return __uint_as_float(((uint32_t)*p) << 16); }
  static __device__ __forceinline__ void store_dev(E* p, float d) { *p = f32_to_bf16_rne(d); }
};

// U, R of a node's post-collision state as stored (the deviations rounded to the storage format,
// summed in direction order exactly as the previous-step field kernel sums them), written to 4
// planes (U_x, U_y, U_z, R) of dst with the given plane stride.  U = (j - F/2) / rho.
template <int S, bool FORCE>
__device__ inline void macro_from_post(const float (&d)[27], float Fx, float Fy, float Fz, float* dst, size_t stride,
                                       size_t idx) {
  using C = Codec<S>;
  float dr = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    typename C::E e;
    C::store_dev(&e, d[i]);
    const float v = C::load_dev(&e);
    dr += v;
    jx += cx(i) * v;
    jy += cy(i) * v;
    jz += cz(i) * v;
  }
  const float rho = 1.f + dr;
  if (FORCE) {
    jx -= 0.5f * Fx;
    jy -= 0.5f * Fy;
    jz -= 0.5f * Fz;
  }
  dst[idx] = jx / rho;
  dst[stride + idx] = jy / rho;
  dst[2 * stride + idx] = jz / rho;
  dst[3 * stride + idx] = rho;
}

// Inlet slab staging: U, R of the nodes x < 3 as [4][nz][ny][3]; index of node (x, y, z).
__host__ __device__ inline size_t slab_index(int x, int y, int z, int ny) { return ((size_t)z * ny + y) * 3 + x; }

inline size_t storage_bytes(int s) { return s == ELBM_STORAGE_F32 ? 4 : 2; }

// ---------------------------------------------------------------------------------------------
// Arithmetic helpers (FP32: hardware reciprocal and square root; FP64: IEEE division).
__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_(double x) { return 1.0 / x; }
__device__ __forceinline__ float log1p_(float x) { return log1pf(x); }
__device__ __forceinline__ double log1p_(double x) { return log1p(x); }

// Stabiliser of the collision: the paper's analytic approximation (default), the exact root of
// eq. gamma_min, or gamma = 2 (LBGK, for comparisons).
constexpr int STAB_KBC = 0, STAB_EXACT = 1, STAB_LBGK = 2;
// bit added to the stabiliser code: the shear part from central moments (with STAB_KBC only)
constexpr int STAB_CENTRAL = 4;

// Dual basis of the shifted velocities c - u, c in {-1, 0, 1}, for moments taken in the frame
// moving with u: cb[p][c + 1] = coefficient of xi^p in the Lagrange polynomial of the points
// {-1 - u, -u, 1 - u} that is 1 at c - u (at u = 0: 1 - c^2, c/2, 3c^2/2 - 1).
template <typename T>
__device__ __forceinline__ void central_basis(T u, T (&cb)[3][3]) {
  cb[0][0] = T(0.5) * u * (u - T(1));
  cb[1][0] = u - T(0.5);
  cb[2][0] = T(0.5);
  cb[0][1] = T(1) - u * u;
  cb[1][1] = T(-2) * u;
  cb[2][1] = T(-1);
  cb[0][2] = T(0.5) * u * (u + T(1));
  cb[1][2] = u + T(0.5);
  cb[2][2] = T(0.5);
}

// Term of direction i in the root condition of eq. gamma_min,
//   G(g) = sum_i dh_i ln(1 + ((1 - beta g) dh_i - (2 beta - 1) ds_i) / feq_i) = 0,
// which makes H(f') stationary along the stabiliser, and in G' = -beta sum dh_i^2 / (feq_i + ...) < 0;
// false where the argument of the logarithm is not positive (outside the admissible interval).
// Gabs accumulates |term|, the scale of the rounding error of G.
template <typename T>
__device__ __forceinline__ bool gamma_term(T g, T beta, T dh, T ds, T ife, T& G, T& dG, T& Gabs) {
  const T x = ((T(1) - beta * g) * dh - (T(2) * beta - T(1)) * ds) * ife;
  const T t = dh * log1p_(x);
  G += t;
  Gabs += fabs(t);
  dG -= beta * dh * dh * ife / (T(1) + x);
  return x > T(-1);
}
template <typename T>
__host__ __device__ constexpr T eps_of() { return sizeof(T) == 4 ? T(1.1920928955078125e-7) : T(2.220446049250313e-16); }
__device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_(double x) { return __builtin_sqrt(x); }

// Factorised entropic equilibrium (eq. feq_min) per axis, relative to the weights:
//   feq_i = rho W_i prod_a g_a(c_ia),  g(c) = (2 - s) X^c / 1,  X = (2u + s)/(1 - u),  s = sqrt(1 + 3u^2),
// written as g(c) = 1 + e(c) with the small parts evaluated without cancellation:
//   e(0)  = -(s - 1),                          s - 1 = 3u^2 / (1 + s)
//   e(+1) = (u (5 - 2s - 3u) + 2 (s - 1)) / (1 - u)
//   e(-1) = (u (s - 4) - 2 (s - 1)) / (2u + s)
// and the reciprocals 1/(w(c) g(c)) for the entropic scalar product.  Since s^2 = 1 + 3u^2, the two
// moving factors multiply to g(+1) g(-1) = (2 - s)^2, so all three reciprocals follow from 1/(2 - s):
// 1/(w g(-1)) = 6 g(+1)/(2 - s)^2, 1/(w g(+1)) = 6 g(-1)/(2 - s)^2, 1/(w g(0)) = (3/2)/(2 - s); the
// two denominators of e(+-1) share one reciprocal as well (four reciprocals per axis instead of seven).
template <typename T>
__device__ __forceinline__ void axis_dev(T u, T (&e)[3], T (&ps)[3], T& sm1) {
  const T s = sqrt_(T(3) * u * u + T(1));
  sm1 = T(3) * u * u * rcp_(T(1) + s);
  e[1] = -sm1;
  const T dp = T(1) - u, dm = T(2) * u + s;
  const T rpm = rcp_(dp * dm);
  e[2] = (u * (T(5) - T(2) * s - T(3) * u) + T(2) * sm1) * (dm * rpm);
  e[0] = (u * (s - T(4)) - T(2) * sm1) * (dp * rpm);
  const T r = rcp_(T(1) - sm1);  // 1/(2 - s)
  const T q = T(6) * r * r;
  ps[0] = q * (T(1) + e[2]);
  ps[1] = T(1.5) * r;
  ps[2] = q * (T(1) + e[0]);
}

// a/b for the stabiliser: FP32 through the hardware reciprocal (the ratio needs no correctly rounded
// quotient), FP64 as an IEEE division.
__device__ __forceinline__ float ratio_(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double ratio_(double a, double b) { return a / b; }

template <typename T>
__device__ __forceinline__ void axis_phi(T u, T (&ph)[3]) {
  const T s = sqrt_(T(3) * u * u + T(1));
  const T g = T(2) - s;
  ph[0] = g * ((s - T(2) * u) / (T(1) + u)) * T(1.0 / 6.0);
  ph[1] = g * T(2.0 / 3.0);
  ph[2] = g * ((T(2) * u + s) / (T(1) - u)) * T(1.0 / 6.0);
}

// Entropic equilibrium of all 27 directions (double precision, used for initial states and the
// body-force increment).
__device__ __forceinline__ void feq_all(double rho, double ux, double uy, double uz, double (&fe)[27]) {
  double px[3], py[3], pz[3];
  axis_phi(ux, px);
  axis_phi(uy, py);
  axis_phi(uz, pz);
#pragma unroll
  for (int i = 0; i < 27; ++i) fe[i] = rho * px[cx(i) + 1] * py[cy(i) + 1] * pz[cz(i) + 1];
}

template <typename T> struct KbcOut {
  T gamma;
  T b;    // <dh|dh>
  T rho;
  T s2;   // <ds|ds> estimated with feq ~ rho W (used only to decide on the FP64 path)
  bool dom;  // 0 < rho < inf and every |u_a| < 1: the entropic equilibrium is positive (a NaN or an
             // infinite population fails this test through rho or u)
};

// Largest finite binary32 value (the upper end of the density test).
constexpr float FLT_BIG = 3.4028234663852886e38f;

// Order-preserving map of binary32 values to uint32 (for atomic min/max of gamma).
__device__ __forceinline__ uint32_t f32_key(float v) {
  const uint32_t b = __float_as_uint(v);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__host__ __device__ inline float f32_unkey(uint32_t k) {
  const uint32_t b = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  float v;
  __builtin_memcpy(&v, &b, 4);
  return v;
}

// FP64 recomputation rule: <dh|dh> is at the FP32 noise floor (the ratio <ds|dh>/<dh|dh> is then
// ill-conditioned) while the shear part is not (otherwise gamma dh, bounded by the shear part, is
// itself at the noise floor and the FP32 result is as good as an FP64 one).
template <typename T>
__device__ __forceinline__ bool needs_fp64(const KbcOut<T>& r, T thr) {
  return !(r.b >= thr * r.rho) && !(r.s2 < thr * r.rho);
}

// KBC collision of one node, in place on the deviations d_i = f_i - W_i (Sec. II, eqs. kineticEq
// and kbc_relax).  The mirror-state update is applied in its equivalent increment form
//   f' = f - beta (2 ds + gamma dh),
// with ds, dh the deviations of the shear part s and the higher-order part h from equilibrium:
//   - raw moments of d by a separable 1-D transform along x, y, z (rho - 1, j, second moments);
//   - feq - W from the factorised closed form relative to the weights, 1/feq from reciprocal
//     factors;
//   - ds from the deviatoric second moments of df = f - feq through the dual basis
//     phi_0 = 1 - c^2, phi_1 = c/2, phi_2 = 3c^2/2 - 1 (faces: D_aa/2, edges: c_a c_b P_ab/4,
//     rest and corners: 0); the equilibrium second moments are rho (2 s_a - 1)/3 and rho u_a u_b;
//   - dh = df - ds, with the rounding residue of its mass and momentum removed;
//   - gamma = 1/beta - (2 - 1/beta) <ds|dh>/<dh|dh>, <X|Y> = sum X Y / feq; gamma = 2 when
//     <dh|dh> <= 1e-30 (then dh is zero to round-off and f' does not depend on it).  STAB selects
//     this analytic stabiliser (the paper's choice), the exact root of eq. gamma_min (Newton from
//     the analytic value), or gamma = 2 (LBGK); with the STAB_CENTRAL bit, ds is rebuilt from the
//     same deviatoric moments (central ones equal the raw ones for df, which carries no mass or
//     momentum) through the dual basis of the shifted velocities c - u (central_basis).
// Working in deviations keeps every difference between O(1) numbers out of the FP32 arithmetic.
// FORCE adds the exact-difference body-force increment feq(rho, u + F/rho) - feq(rho, u),
// evaluated in FP64 to avoid cancellation.
template <typename T, bool FORCE, int STAB = STAB_KBC>
__device__ __forceinline__ KbcOut<T> kbc_collide(T (&d)[27], const T beta, const T inv_beta, const T Fx, const T Fy,
                                                 const T Fz) {
  // separable raw-moment transform: (a, b, c) at c = -1, 0, +1  ->  (a+b+c, c-a, a+c)
  T m0[9], m1[9], m2[9];
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    const T a = d[3 * r], b = d[3 * r + 1], c = d[3 * r + 2];
    const T ac = a + c;
    m0[r] = ac + b;
    m1[r] = c - a;
    m2[r] = ac;
  }
  T m00[3], m01[3], m02[3], m10[3], m11[3], m20[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    {
      const T a = m0[3 * k], b = m0[3 * k + 1], c = m0[3 * k + 2];
      const T ac = a + c;
      m00[k] = ac + b;
      m01[k] = c - a;
      m02[k] = ac;
    }
    {
      const T a = m1[3 * k], b = m1[3 * k + 1], c = m1[3 * k + 2];
      m10[k] = (a + c) + b;
      m11[k] = c - a;
    }
    m20[k] = (m2[3 * k] + m2[3 * k + 2]) + m2[3 * k + 1];
  }
  const T dr = (m00[0] + m00[2]) + m00[1];  // rho - 1
  const T jz = m00[2] - m00[0];
  const T Q002 = m00[0] + m00[2];           // second moments of d (those of W are 1/3 and 0)
  const T jy = (m01[0] + m01[2]) + m01[1];
  const T Q011 = m01[2] - m01[0];
  const T Q020 = (m02[0] + m02[2]) + m02[1];
  const T jx = (m10[0] + m10[2]) + m10[1];
  const T Q101 = m10[2] - m10[0];
  const T Q110 = (m11[0] + m11[2]) + m11[1];
  const T Q200 = (m20[0] + m20[2]) + m20[1];

  const T rho = T(1) + dr;
  const T rinv = rcp_(rho);
  const T ux = jx * rinv, uy = jy * rinv, uz = jz * rinv;
  T ex[3], ey[3], ez[3], psx[3], psy[3], psz[3], sx, sy, sz;
  axis_dev(ux, ex, psx, sx);
  axis_dev(uy, ey, psy, sy);
  axis_dev(uz, ez, psz, sz);

  // deviatoric moments of df: M200 - rho (2 s - 1)/3 = Q200 - (dr (1 + 2 (s-1)) + 2 (s-1))/3
  const T third = T(1.0 / 3.0);
  const T dM200 = Q200 - (dr * (T(1) + T(2) * sx) + T(2) * sx) * third;
  const T dM020 = Q020 - (dr * (T(1) + T(2) * sy) + T(2) * sy) * third;
  const T dM002 = Q002 - (dr * (T(1) + T(2) * sz) + T(2) * sz) * third;
  const T tr3 = (dM200 + dM020 + dM002) * third;
  const T sfx = T(0.5) * (dM200 - tr3), sfy = T(0.5) * (dM020 - tr3), sfz = T(0.5) * (dM002 - tr3);
  const T sxy = T(0.25) * (Q110 - jx * uy), sxz = T(0.25) * (Q101 - jx * uz), syz = T(0.25) * (Q011 - jy * uz);
  constexpr bool CENTRAL = (STAB & STAB_CENTRAL) != 0;
  T cbx[3][3], cby[3][3], cbz[3][3];
  if (CENTRAL) {
    central_basis(ux, cbx);
    central_basis(uy, cby);
    central_basis(uz, cbz);
  }
  // shear part of direction i: raw basis (faces D_aa/2, edges c_a c_b P_ab/4), or central
  auto ds_of = [&](int i) -> T {
    if (CENTRAL) {
      const int x = cx(i) + 1, y = cy(i) + 1, z = cz(i) + 1;
      const T dx = T(2) * sfx, dy = T(2) * sfy, dz = T(2) * sfz;
      const T pxy = T(4) * sxy, pxz = T(4) * sxz, pyz = T(4) * syz;
      return dx * cbx[2][x] * cby[0][y] * cbz[0][z] + dy * cbx[0][x] * cby[2][y] * cbz[0][z] +
             dz * cbx[0][x] * cby[0][y] * cbz[2][z] + pxy * cbx[1][x] * cby[1][y] * cbz[0][z] +
             pxz * cbx[1][x] * cby[0][y] * cbz[1][z] + pyz * cbx[0][x] * cby[1][y] * cbz[1][z];
    }
    T ds = T(0);
    if (nnz(i) == 1) ds = cx(i) ? sfx : (cy(i) ? sfy : sfz);
    if (nnz(i) == 2) {
      if (cz(i) == 0) ds = T(cx(i) * cy(i)) * sxy;
      else if (cy(i) == 0) ds = T(cx(i) * cz(i)) * sxz;
      else ds = T(cy(i) * cz(i)) * syz;
    }
    return ds;
  };

  // feq_i - W_i = W_i (dr + rho P_i),  P_i = prod (1 + e) - 1 expanded without cancellation; with
  // the y and z factors of a row of three directions (c_y, c_z fixed) in p_yz = (1 + e_y)(1 + e_z) - 1:
  // dr + rho P_i = (dr + rho p_yz) + e_x rho (1 + p_yz)
  T dh[27];
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    const T a_ = ey[cy(3 * r) + 1], b_ = ez[cz(3 * r) + 1];
    const T pyz = a_ + b_ + a_ * b_;
    const T Y = rho * pyz + rho, Z = rho * pyz + dr;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int i = 3 * r + k;
      const T fdev = T(wd(i)) * (ex[k] * Y + Z);
      dh[i] = (d[i] - fdev) - ds_of(i);
    }
  }
  // mass and momentum of dh by the separable transform used for the moments of d
  T hm, hx, hy, hz;
  {
    T r0[9], r1[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      const T a = dh[3 * r], b = dh[3 * r + 1], c = dh[3 * r + 2];
      r0[r] = (a + c) + b;
      r1[r] = c - a;
    }
    T q00[3], q01[3], q10[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      q00[k] = (r0[3 * k] + r0[3 * k + 2]) + r0[3 * k + 1];
      q01[k] = r0[3 * k + 2] - r0[3 * k];
      q10[k] = (r1[3 * k] + r1[3 * k + 2]) + r1[3 * k + 1];
    }
    hm = (q00[0] + q00[2]) + q00[1];
    hz = q00[2] - q00[0];
    hy = (q01[0] + q01[2]) + q01[1];
    hx = (q10[0] + q10[2]) + q10[1];
  }
  // dh has zero mass and momentum in exact arithmetic; remove the rounding residue (its kinematic
  // part in the dual basis: mass on the rest population, momentum on the face pairs) so that the
  // update conserves rho and j to the rounding of the store alone.
  dh[13] -= hm;
  dh[14] -= T(0.5) * hx;
  dh[12] += T(0.5) * hx;
  dh[16] -= T(0.5) * hy;
  dh[10] += T(0.5) * hy;
  dh[22] -= T(0.5) * hz;
  dh[4] += T(0.5) * hz;
  // <ds|dh> and <dh|dh>: 1/feq_i = (1/rho) psx psy psz, summed along x inside each row first
  T a = T(0), b = T(0), s2c = T(0);
  if (CENTRAL) {
#pragma unroll
    for (int i = 0; i < 27; ++i) {
      const T ife = (rinv * (psy[cy(i) + 1] * psz[cz(i) + 1])) * psx[cx(i) + 1];
      const T ds = ds_of(i);
      const T th = dh[i] * ife;
      b += th * dh[i];
      a += th * ds;
      s2c += ds * ds * ife;
    }
  } else {
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      T br = T(0), ar = T(0);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int i = 3 * r + k;
        const T th = dh[i] * psx[k];
        br += th * dh[i];
        if (nnz(i) == 1 || nnz(i) == 2) ar += th * ds_of(i);
      }
      const T w = psy[cy(3 * r) + 1] * psz[cz(3 * r) + 1];
      b += w * br;
      a += w * ar;
    }
    b *= rinv;
    a *= rinv;
  }
  T gamma = (b > T(1e-30)) ? inv_beta - (T(2) - inv_beta) * ratio_(a, b) : T(2);
  if ((STAB & 3) == STAB_LBGK) gamma = T(2);
  if ((STAB & 3) == STAB_EXACT && b > T(1e-30)) {
    // Root of eq. gamma_min inside the admissible interval (lo, hi), where every argument of the
    // logarithm, p0_i + p1_i g, is positive. G falls from +inf at lo to -inf at hi, so the root is
    // unique. Newton from the analytic value (its first-order approximation) inside a bracket that
    // shrinks with the sign of G; a step that leaves the bracket is replaced by bisection. Stops
    // at a relative step below tol or where |G| is at the rounding level of its sum.
    T lo = T(-1e6), hi = T(1e6);
#pragma unroll
    for (int i = 0; i < 27; ++i) {
      const T ife = (rinv * (psy[cy(i) + 1] * psz[cz(i) + 1])) * psx[cx(i) + 1];
      const T ds = ds_of(i);
      const T p0 = T(1) + (dh[i] - (T(2) * beta - T(1)) * ds) * ife, p1 = -beta * dh[i] * ife;
      if (p1 > T(0)) lo = fmax(lo, -p0 / p1);
      else if (p1 < T(0)) hi = fmin(hi, -p0 / p1);
    }
    if (lo < hi) {
      const T tol = sizeof(T) == 4 ? T(1e-6) : T(1e-13);
      T g = (gamma > lo && gamma < hi) ? gamma : T(0.5) * (lo + hi);
      for (int it = 0; it < 64; ++it) {
        T G = T(0), dG = T(0), Ga = T(0);
        bool ok = true;
#pragma unroll
        for (int i = 0; i < 27; ++i) {
          const T ife = (rinv * (psy[cy(i) + 1] * psz[cz(i) + 1])) * psx[cx(i) + 1];
          const T ds = ds_of(i);
          ok = gamma_term(g, beta, dh[i], ds, ife, G, dG, Ga) && ok;
        }
        // G at its rounding level: g is the root as far as the arithmetic can tell
        if (ok && fabs(G) <= T(64) * eps_of<T>() * Ga) break;
        T gn;
        if (!ok || !(dG < T(0))) {
          // rounding put an argument at or below zero: g sits at an end of the interval
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
  // faces: W = 2/27 (2 per axis), edges: W = 1/54 (4 per plane)
  const T s2 = CENTRAL ? s2c
                       : (T(27) * (sfx * sfx + sfy * sfy + sfz * sfz) + T(216) * (sxy * sxy + sxz * sxz + syz * syz)) * rinv;
  const T bg = beta * gamma, b2 = T(2) * beta;
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const T ds = ds_of(i);
    d[i] = d[i] - b2 * ds - bg * dh[i];
  }
  if (FORCE) {
    const double r = (double)rho;
    double e0[27], e1[27];
    feq_all(r, (double)ux, (double)uy, (double)uz, e0);
    feq_all(r, (double)ux + (double)Fx / r, (double)uy + (double)Fy / r, (double)uz + (double)Fz / r, e1);
#pragma unroll
    for (int i = 0; i < 27; ++i) d[i] = (T)((double)d[i] + (e1[i] - e0[i]));
  }
  const bool dom = rho > T(0) && rho < T(FLT_BIG) && fabs(ux) < T(1) && fabs(uy) < T(1) && fabs(uz) < T(1);
  return KbcOut<T>{gamma, b, rho, s2, dom};
}

// Grad's distribution (eq. grad) with c_s^2 = 1/3:
//   f*_i = W_i [rho + 3 rho c.u + (9/2) (Pi - rho/3 I) : (c c - I/3)].
template <typename T>
__device__ __forceinline__ T grad_pop(int i, T rho, const T (&u)[3], const T (&Pi)[6]) {
  // Pi packed as xx, yy, zz, xy, xz, yz
  const T c[3] = {T(cx(i)), T(cy(i)), T(cz(i))};
  const T cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
  const T r3 = rho * T(1.0 / 3.0);
  const T Axx = Pi[0] - r3, Ayy = Pi[1] - r3, Azz = Pi[2] - r3;
  const T t = T(1.0 / 3.0);
  const T PQ = Axx * (c[0] * c[0] - t) + Ayy * (c[1] * c[1] - t) + Azz * (c[2] * c[2] - t) +
               T(2) * (Pi[3] * c[0] * c[1] + Pi[4] * c[0] * c[2] + Pi[5] * c[1] * c[2]);
  return T(wd(i)) * (rho + T(3) * rho * cu + T(4.5) * PQ);
}

// Pressure tensor (eqs. pressure, pressure2): Pi = rho/3 I + rho u u - (rho/3)/(2 beta) (G + G^T),
// G[a][b] = d u_a / d x_b.
template <typename T>
__device__ __forceinline__ void pressure_tensor(T rho, const T (&u)[3], const T (&G)[9], T beta, T (&Pi)[6]) {
  const T k = rho * T(1.0 / 3.0) / (T(2) * beta);
  const T r3 = rho * T(1.0 / 3.0);
  Pi[0] = r3 + rho * u[0] * u[0] - k * T(2) * G[0];
  Pi[1] = r3 + rho * u[1] * u[1] - k * T(2) * G[4];
  Pi[2] = r3 + rho * u[2] * u[2] - k * T(2) * G[8];
  Pi[3] = rho * u[0] * u[1] - k * (G[1] + G[3]);
  Pi[4] = rho * u[0] * u[2] - k * (G[2] + G[6]);
  Pi[5] = rho * u[1] * u[2] - k * (G[5] + G[7]);
}

// ---------------------------------------------------------------------------------------------
// Bodies as seen by kernels: kinematics evaluated on the host (FP64) at t and t+1.
struct BodyDev {
  int32_t kind;
  int32_t pad;
  double c0[3];      // centre at t
  double c1[3];      // centre at t+1
  double U0[3];      // velocity at t
  double U1[3];      // velocity at t+1
  double r2;         // radius^2
  double radius;
  double n[3];       // plane normal
  double omega[3];
};

// Triangulated body: vertex data of one time level, binned into a uniform grid of cells (spacing
// h >= 2) by triangle bounding box; cell c lists items[start[c] .. start[c+1]).
struct MeshLevel {
  const double* X;       // [nv][3] positions
  const double* V;       // [nv][3] velocities
  const int32_t* start;  // [ncell + 1]
  const int32_t* items;  // triangle indices
};

struct MeshDev {
  const int32_t* tri;  // [nt][3]
  int32_t nt;
  int32_t ncell;
  double org[3];       // corner of cell (0, 0, 0)
  double inv_h;
  int32_t dim[3];
  int32_t cap;         // capacity of items (entries past it, after an overflow, are not read)
  MeshLevel lv[2];     // time levels t and t+1
};

// Grid cell of coordinate v along axis a (clamped to the grid): monotone in v, so a triangle's
// bounding box covers the cell of every point of the triangle.
__host__ __device__ inline int mesh_cell(const MeshDev& m, int a, double v) {
  int c = (int)floor((v - m.org[a]) * m.inv_h);
  c = c < 0 ? 0 : c;
  return c > m.dim[a] - 1 ? m.dim[a] - 1 : c;
}

struct Bodies {
  int32_t nb;
  int32_t mesh;  // index of the triangulated body, -1 if none
  BodyDev b[ELBM_MAX_BODIES];
  MeshDev m;
  // free bodies: their velocity at t+1 depends on the force of the step that produced t, which the
  // device-side integrator holds; U1dev [MAX_BODIES][3] replaces b[k].U1 where bit k of free_mask is set
  const double* U1dev;
  const double* W1dev;  // [MAX_BODIES][3] angular velocity at t+1 of the free bodies
  uint32_t free_mask;
  int32_t pad2;
};

// Translational velocity of body k at t+1.
__device__ inline void body_U1(const Bodies& bd, int k, double* u) {
  if ((bd.free_mask >> k) & 1u) {
    u[0] = bd.U1dev[3 * k];
    u[1] = bd.U1dev[3 * k + 1];
    u[2] = bd.U1dev[3 * k + 2];
  } else {
    u[0] = bd.b[k].U1[0];
    u[1] = bd.b[k].U1[1];
    u[2] = bd.b[k].U1[2];
  }
}

// Angular velocity of body k at t+1 (b[k].omega holds the one at t).
__device__ inline void body_W1(const Bodies& bd, int k, double* w) {
  if ((bd.free_mask >> k) & 1u) {
    w[0] = bd.W1dev[3 * k];
    w[1] = bd.W1dev[3 * k + 1];
    w[2] = bd.W1dev[3 * k + 2];
  } else {
    w[0] = bd.b[k].omega[0];
    w[1] = bd.b[k].omega[1];
    w[2] = bd.b[k].omega[2];
  }
}

// State of a free body at one time level: position, velocity, and the force of the step that
// produced the level (explicit Euler of Newton's equations, Sec. IV.A).
struct FreeState {
  double x[3], u[3], F[3];
  double w[3], M[3];  // angular velocity and the torque of the step that produced the level
};

// Strictly-inside test (FP64, operations in the written order, no contraction).
// (A triangulated body is never inside here: its mask comes from the crossing count.)
__host__ __device__ inline bool inside_body(const BodyDev& b, const double* c, double x, double y, double z) {
#pragma clang fp contract(off)
  if (b.kind == ELBM_BODY_MESH) return false;
  if (b.kind == ELBM_BODY_SPHERE) {
    const double dx = x - c[0], dy = y - c[1], dz = z - c[2];
    double d2 = dx * dx;
    d2 = d2 + dy * dy;
    d2 = d2 + dz * dz;
    return d2 < b.r2;
  }
  double s = b.n[0] * (x - c[0]);
  s = s + b.n[1] * (y - c[1]);
  s = s + b.n[2] * (z - c[2]);
  return s < 0.0;
}

// ---------------------------------------------------------------------------------------------
// Device-resident counters.
struct DevCounters {
  // FP64 fix-up queue lengths of the steps of even and odd parity: a step appends to its own and
  // its fix-up kernel clears the other one, which the next step then uses (no host round trip,
  // no grid-wide ticket); the last step's length stays readable until the next fix-up
  uint32_t fix_count[2];
  uint32_t dyn_count;     // dynamic boundary nodes this step
  uint32_t overflow;      // sticky: 1 boundary list, 2 mesh vertex outside its box or grid full,
                          // 4 more crossings on a lattice row than the mask kernel holds,
                          // 8 mesh vertex index out of range
  uint32_t nonfinite;     // sticky: a collided node had a non-finite state or one outside the
                          // domain of the entropic equilibrium (1 bulk sweep, 2 wall kernel)
  uint32_t gamma_lo, gamma_hi;  // f32_key of the smallest and largest gamma since the last read
  uint32_t pad;
};

// Lanes per node in the lane-parallel boundary kernels (two nodes per wavefront of 64).
constexpr int GROUP = 32;

// Inclusive prefix sum over a workgroup of NW wavefronts of 64: shuffles within each wavefront,
// one shared array wsum[NW] of the wavefront totals; total = the workgroup's sum.  Every thread of
// the workgroup must call it.
template <int NW, typename T>
__device__ inline T block_scan_inclusive(T v, T* wsum, T& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  if (lane == 63) wsum[wave] = v;
  __syncthreads();
  if (wave == 0) {
    T s = lane < NW ? wsum[lane] : T(0);
#pragma unroll
    for (int off = 1; off < NW; off <<= 1) {
      const T u = __shfl_up(s, off, 64);
      if (lane >= off) s += u;
    }
    if (lane < NW) wsum[lane] = s;
  }
  __syncthreads();
  if (wave > 0) v += wsum[wave - 1];
  total = wsum[NW - 1];
  __syncthreads();
  return v;
}

template <typename T>
__device__ inline T scan1024_inclusive(T v, T* wsum, T& total) {
  return block_scan_inclusive<16>(v, wsum, total);
}

struct Box {
  int lo[3];
  int n[3];
  __host__ __device__ long count() const { return (long)n[0] * n[1] * n[2]; }
};
struct Box2 {
  Box b[2];
  __host__ __device__ long count() const { return b[0].count() + b[1].count(); }
};

}  // namespace elbm
