/*
 * elbm_oracle_adjoint.cpp -- FP64 CPU adjoint of one time step of the oracle (the step of
 * elbm_oracle.c: pull streaming, moving-wall Grad reconstruction and refill of Sec. III,
 * momentum-exchange force of Sec. IV.A, KBC collision of Sec. II, eqs. kineticEq, kbc_relax,
 * feq_min, grad, pressure, pressure2).
 *
 * TEST INFRASTRUCTURE ONLY.  The product library never links, loads or calls this file; only the
 * test suite uses it.  It shares no code, header or table with the GPU implementation, and it does
 * not call the forward oracle either: the step is restated below, so that the tests can check the
 * two restatements against each other (values to rounding, derivatives against finite differences
 * of the forward oracle).
 *
 * What it computes.  With the solid masks of t and t+1 held fixed (a mask is piecewise constant in
 * every parameter, so its derivative is zero), one step maps the post-collision populations A^t,
 * the body-force field F and each body's oscillation amplitude amp_k to A^{t+1} and to the
 * momentum-exchange force F_k(t+1) on each body.  For the scalar
 *     L = <lam, A^{t+1}> + sum_k w_k . F_k(t+1)
 * it returns dL/dA^t (27 N values) and adds dL/dF (3 N) and dL/d(amp_k).
 *
 * How.  Every node-local map of the step -- the collision at a node, the reconstruction of the
 * missing populations at a boundary node together with its link forces, the refill of an uncovered
 * node, the moments behind the previous-step fields U^t, R^t -- is written once on a generic
 * scalar type.  On doubles it is the forward step; on forward-mode dual numbers (a value and 32
 * tangent components, each operation applying its derivative rule) it gives exact derivatives.
 * Seeding the tangents with unit vectors of a map's inputs yields its full Jacobian J, and the
 * adjoint applies J^T to the adjoint of the map's outputs.  The linear structure between the
 * maps -- the pull, the outlet copy, the finite-difference stencil, the neighbour average of the
 * refill density -- is transposed by adding each input's adjoint to the entry it was read from.
 * No finite differences, no approximation: FP64 rounding only.
 *
 * Readings are those of the forward oracle (same definitions of the missing set, link fraction,
 * wall velocity, targets, stencil, refill, force, time levels).  Supported: analytic stabiliser and
 * gamma = 2, raw moment basis, spheres and planes with prescribed motion (rotation included).  Not
 * supported (returns an error): the exact stabiliser, the central-moment variant, freely moving
 * and triangulated bodies.
 *
 * Population layout: f[i * N + n], node n = (z * ny + y) * nx + x; vector fields [3][N].
 */
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

constexpr int NQ = 27;
constexpr int MAXB = 8;
constexpr int ND = 32;  // tangent components carried by one dual number

// D3Q27: i = 9 (cz+1) + 3 (cy+1) + (cx+1); opposite 26 - i; rest 13.
int cxi(int i) { return i % 3 - 1; }
int cyi(int i) { return (i / 3) % 3 - 1; }
int czi(int i) { return i / 9 - 1; }
int cc(int i, int a) { return a == 0 ? cxi(i) : (a == 1 ? cyi(i) : czi(i)); }
int dir_of(int x, int y, int z) { return 9 * (z + 1) + 3 * (y + 1) + (x + 1); }
double w1(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
double wgt(int i) { return w1(cxi(i)) * w1(cyi(i)) * w1(czi(i)); }
const double CS2 = 1.0 / 3.0;

// ------------------------------------------------------------------------------------------------
// Forward-mode dual numbers: value v and tangent d (the derivative along ND seeded directions).
struct Uninit {};
struct D {
  double v;
  double d[ND];
  D() : v(0.0) { std::memset(d, 0, sizeof d); }
  D(double x) : v(x) { std::memset(d, 0, sizeof d); }  // a constant
  explicit D(Uninit) {}                                 // every field written by the caller
};
inline D operator+(const D& a, const D& b) { D r{Uninit{}}; r.v = a.v + b.v; for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
inline D operator-(const D& a, const D& b) { D r{Uninit{}}; r.v = a.v - b.v; for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
inline D operator-(const D& a) { D r{Uninit{}}; r.v = -a.v; for (int k = 0; k < ND; ++k) r.d[k] = -a.d[k]; return r; }
inline D operator*(const D& a, const D& b) {
  D r{Uninit{}};
  r.v = a.v * b.v;
  for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
inline D operator/(const D& a, const D& b) {
  D r{Uninit{}};
  r.v = a.v / b.v;
  const double ib = 1.0 / b.v;
  for (int k = 0; k < ND; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
  return r;
}
inline D operator+(const D& a, double b) { D r = a; r.v += b; return r; }
inline D operator+(double a, const D& b) { return b + a; }
inline D operator-(const D& a, double b) { D r = a; r.v -= b; return r; }
inline D operator-(double a, const D& b) { D r = -b; r.v += a; return r; }
inline D operator*(const D& a, double b) { D r{Uninit{}}; r.v = a.v * b; for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * b; return r; }
inline D operator*(double a, const D& b) { return b * a; }
inline D operator/(const D& a, double b) { D r{Uninit{}}; r.v = a.v / b; for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] / b; return r; }
inline D operator/(double a, const D& b) { return D(a) / b; }
inline D& operator+=(D& a, const D& b) { a = a + b; return a; }
inline D& operator-=(D& a, const D& b) { a = a - b; return a; }
inline D& operator/=(D& a, double b) { a = a / b; return a; }
inline D sqrt_(const D& a) {
  D r{Uninit{}};
  r.v = std::sqrt(a.v);
  const double s = r.v > 0.0 ? 0.5 / r.v : 0.0;  // the root of 0 (a tangent ray) has no derivative
  for (int k = 0; k < ND; ++k) r.d[k] = s * a.d[k];
  return r;
}
inline double sqrt_(double a) { return std::sqrt(a); }
inline double val(double a) { return a; }
inline double val(const D& a) { return a.v; }

// ------------------------------------------------------------------------------------------------
// Node-local maps, generic in the scalar S (double or D).

// Entropic equilibrium, product form (eq. feq_min):
//   feq_i = rho prod_a w(c_ia) (2 - s_a) [(2 u_a + s_a)/(1 - u_a)]^{c_ia},  s_a = sqrt(1 + 3 u_a^2).
template <class S>
void feq(const S& rho, const S u[3], S out[NQ]) {
  S phi[3][3];
  for (int a = 0; a < 3; ++a) {
    const S s = sqrt_(1.0 + 3.0 * u[a] * u[a]);
    const S X = (2.0 * u[a] + s) / (1.0 - u[a]);
    phi[a][0] = w1(-1) * (2.0 - s) / X;
    phi[a][1] = w1(0) * (2.0 - s);
    phi[a][2] = w1(1) * (2.0 - s) * X;
  }
  for (int i = 0; i < NQ; ++i) out[i] = rho * phi[0][cxi(i) + 1] * phi[1][cyi(i) + 1] * phi[2][czi(i) + 1];
}

int ipow(int c, int p) { int r = 1; for (int k = 0; k < p; ++k) r *= c; return r; }

template <class S>
S raw_moment(const S f[NQ], int p, int q, int r) {
  S m(0.0);
  for (int i = 0; i < NQ; ++i) {
    const int w = ipow(cxi(i), p) * ipow(cyi(i), q) * ipow(czi(i), r);
    if (w) m += f[i] * (double)w;
  }
  return m;
}

// 1-D dual basis of the raw moments: phi_0 = 1 - c^2, phi_1 = c/2, phi_2 = 3 c^2/2 - 1.
double phib(int p, int c) { return p == 0 ? 1.0 - c * c : (p == 1 ? 0.5 * c : 1.5 * c * c - 1.0); }
double basis(int p, int q, int r, int i) { return phib(p, cxi(i)) * phib(q, cyi(i)) * phib(r, czi(i)); }

// KBC parts (Sec. II): k from the conserved moments, s from the deviatoric stress.
template <class S>
void kinematic_part(const S f[NQ], S k[NQ]) {
  const S M000 = raw_moment(f, 0, 0, 0), M100 = raw_moment(f, 1, 0, 0), M010 = raw_moment(f, 0, 1, 0),
          M001 = raw_moment(f, 0, 0, 1);
  for (int i = 0; i < NQ; ++i)
    k[i] = M000 * basis(0, 0, 0, i) + M100 * basis(1, 0, 0, i) + M010 * basis(0, 1, 0, i) + M001 * basis(0, 0, 1, i);
}

template <class S>
void shear_part(const S f[NQ], S s[NQ]) {
  const S M200 = raw_moment(f, 2, 0, 0), M020 = raw_moment(f, 0, 2, 0), M002 = raw_moment(f, 0, 0, 2);
  const S M110 = raw_moment(f, 1, 1, 0), M101 = raw_moment(f, 1, 0, 1), M011 = raw_moment(f, 0, 1, 1);
  const S T = M200 + M020 + M002;
  const S D200 = M200 - T / 3.0, D020 = M020 - T / 3.0, D002 = M002 - T / 3.0;
  for (int i = 0; i < NQ; ++i)
    s[i] = D200 * basis(2, 0, 0, i) + D020 * basis(0, 2, 0, i) + D002 * basis(0, 0, 2, i) + M110 * basis(1, 1, 0, i) +
           M101 * basis(1, 0, 1, i) + M011 * basis(0, 1, 1, i);
}

// KBC collision (eqs. kineticEq, kbc_relax): f' = (1 - beta) f + beta [k + (2 s_eq - s) + (1 - gamma) h
// + gamma h_eq], with gamma = 1/beta - (2 - 1/beta) <ds|dh>/<dh|dh> (entropic scalar product with
// weights 1/feq), gamma = 2 where <dh|dh> <= 1e-30 (the value decides; gamma is then constant) or
// when lbgk is set.  Body force: f' += feq(rho, u + F/rho) - feq(rho, u).
template <class S>
void collide(S f[NQ], double beta, const S* F, bool lbgk) {
  const S rho = raw_moment(f, 0, 0, 0);
  const S u[3] = {raw_moment(f, 1, 0, 0) / rho, raw_moment(f, 0, 1, 0) / rho, raw_moment(f, 0, 0, 1) / rho};
  S fe[NQ], k[NQ], s[NQ], h[NQ], seq[NQ], heq[NQ], keq[NQ], ds[NQ], dh[NQ];
  feq(rho, u, fe);
  kinematic_part(f, k);
  kinematic_part(fe, keq);
  shear_part(f, s);
  shear_part(fe, seq);
  for (int i = 0; i < NQ; ++i) {
    h[i] = f[i] - k[i] - s[i];
    heq[i] = fe[i] - keq[i] - seq[i];
    ds[i] = s[i] - seq[i];
    dh[i] = h[i] - heq[i];
  }
  S a(0.0), b(0.0);
  for (int i = 0; i < NQ; ++i) {
    a += ds[i] * dh[i] / fe[i];
    b += dh[i] * dh[i] / fe[i];
  }
  S gamma(2.0);
  if (!lbgk && val(b) > 1e-30) gamma = 1.0 / beta - (2.0 - 1.0 / beta) * a / b;
  for (int i = 0; i < NQ; ++i) {
    const S fmirr = k[i] + (2.0 * seq[i] - s[i]) + ((1.0 - gamma) * h[i] + gamma * heq[i]);
    f[i] = (1.0 - beta) * f[i] + beta * fmirr;
  }
  if (F) {
    const S u2[3] = {u[0] + F[0] / rho, u[1] + F[1] / rho, u[2] + F[2] / rho};
    S fe2[NQ];
    feq(rho, u2, fe2);
    for (int i = 0; i < NQ; ++i) f[i] += fe2[i] - fe[i];
  }
}

// Grad's distribution (eq. grad) with the pressure tensor of eqs. pressure, pressure2:
//   Pi = rho c_s^2 I + rho u u - (rho c_s^2/(2 beta)) (G + G^T),  G[3a+b] = d u_a/d x_b,
//   f*_i = W_i [rho + (rho/c_s^2) c_i.u + (1/(2 c_s^4)) (Pi - rho c_s^2 I):(c_i c_i - c_s^2 I)].
template <class S>
void pressure(const S& rho, const S u[3], const S G[9], double beta, S Pi[9]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      Pi[3 * a + b] = rho * CS2 * (a == b ? 1.0 : 0.0) + rho * u[a] * u[b] -
                      rho * CS2 / (2.0 * beta) * (G[3 * a + b] + G[3 * b + a]);
}

template <class S>
void grad_dist(const S& rho, const S u[3], const S Pi[9], S out[NQ]) {
  for (int i = 0; i < NQ; ++i) {
    S cu(0.0), PQ(0.0);
    for (int a = 0; a < 3; ++a) cu += u[a] * (double)cc(i, a);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        const double d = a == b ? 1.0 : 0.0;
        PQ += (Pi[3 * a + b] - rho * CS2 * d) * ((double)(cc(i, a) * cc(i, b)) - CS2 * d);
      }
    out[i] = wgt(i) * (rho + rho / CS2 * cu + PQ / (2.0 * CS2 * CS2));
  }
}

// ------------------------------------------------------------------------------------------------
// Grid and bodies: the same records as the forward oracle passes (layout of its or_grid/or_body).
struct Grid {
  int32_t nx, ny, nz;
  int32_t channel;
  double beta;
  double rho0;
  double u_in[3];
  int32_t stream_only;
  int32_t stabiliser;  // 0 analytic, 1 exact (not supported here), 2 gamma = 2
  int32_t central;     // not supported here
};

struct Body {
  int32_t kind;        // 0 sphere, 1 plane (2, triangulated: not supported here)
  int32_t tracked;     // freely moving: not supported here
  double p0[3];
  double radius;
  double normal[3];
  double amp, period;
  double dir[3];
  double vel[3];
  double omega[3];
  double track_t;
  double track_c[2][3];
  double track_U[2][3];
  const double* mesh_X[2];
  const double* mesh_V[2];
  const int32_t* mesh_tri;
  int32_t mesh_nv, mesh_nt;
  double mesh_t;
  double track_W[2][3];
};

// Prescribed motion (the forward oracle's parametrisation, FP64, same operation order):
//   c(t) = p0 + (amp sin(2 pi t/T)) dir + vel t,   U(t) = (amp (2 pi/T) cos(2 pi t/T)) dir + vel.
template <class S>
void kinematics(const Body& b, double t, const S& amp, S c[3], S U[3]) {
  double sn = 0.0, cs = 0.0, om = 0.0;
  if (b.period != 0.0) {
    const double ph = ((2.0 * M_PI) * t) / b.period;
    sn = std::sin(ph);
    cs = std::cos(ph);
    om = (2.0 * M_PI) / b.period;
  }
  for (int a = 0; a < 3; ++a) {
    c[a] = b.p0[a] + (amp * sn) * b.dir[a] + b.vel[a] * t;
    U[a] = (amp * om * cs) * b.dir[a] + b.vel[a];
  }
}

// Rigid-body velocity at x: U + omega x (x - c).
template <class S>
void rigid_velocity(const Body& b, const S c[3], const S U[3], const S x[3], S out[3]) {
  const S r[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
  const double* w = b.omega;
  out[0] = U[0] + (w[1] * r[2] - w[2] * r[1]);
  out[1] = U[1] + (w[2] * r[0] - w[0] * r[2]);
  out[2] = U[2] + (w[0] * r[1] - w[1] * r[0]);
}

// Link fraction q_i (Sec. III): x_w = x_b - q c_i on the surface.  Sphere: smallest root of
// |x_b - s c_i - c|^2 = R^2 written as (|d|^2 - R^2)/(d.c_i + sqrt(disc)), a negative disc taken
// as 0; plane: n.(x_b - c)/n.c_i.
template <class S>
S link_fraction(const Body& b, const S c[3], const double xb[3], int i) {
  const double v[3] = {(double)cxi(i), (double)cyi(i), (double)czi(i)};
  const S d[3] = {xb[0] - c[0], xb[1] - c[1], xb[2] - c[2]};
  if (b.kind == 0) {
    const S dv = d[0] * v[0] + d[1] * v[1] + d[2] * v[2];
    const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const S dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] - b.radius * b.radius;
    S disc = dv * dv - vv * dd;
    if (val(disc) < 0.0) disc = S(0.0);
    return dd / (dv + sqrt_(disc));
  }
  const S nd = b.normal[0] * d[0] + b.normal[1] * d[1] + b.normal[2] * d[2];
  const double nv = b.normal[0] * v[0] + b.normal[1] * v[1] + b.normal[2] * v[2];
  return nd / nv;
}

// Finite-difference velocity gradient on U^t (Sec. III; the oracle's stencil reading): per axis b,
// central if the nodes at +-1 are usable; else second-order one-sided over +1, +2 (forward first)
// or -1, -2; else first-order one-sided; else 0.  Un[j]: U at x + c_j (Un[13] = U(x)); Ufar[2b],
// Ufar[2b+1]: U at x + 2 e_b, x - 2 e_b; ok1[j], okfar[.]: usable (exists, fluid at t+1).
template <class S>
void grad_u(const S Un[NQ][3], const S Ufar[6][3], const bool ok1[NQ], const bool okfar[6], S G[9]) {
  for (int b = 0; b < 3; ++b) {
    const int ip = dir_of(b == 0, b == 1, b == 2), im = dir_of(-(b == 0), -(b == 1), -(b == 2));
    const bool p1 = ok1[ip], m1 = ok1[im], p2 = okfar[2 * b], m2 = okfar[2 * b + 1];
    for (int a = 0; a < 3; ++a) {
      S d(0.0);
      if (p1 && m1) d = 0.5 * (Un[ip][a] - Un[im][a]);
      else if (p1 && p2) d = 0.5 * (-3.0 * Un[13][a] + 4.0 * Un[ip][a] - Ufar[2 * b][a]);
      else if (m1 && m2) d = 0.5 * (3.0 * Un[13][a] - 4.0 * Un[im][a] + Ufar[2 * b + 1][a]);
      else if (p1) d = Un[ip][a] - Un[13][a];
      else if (m1) d = Un[13][a] - Un[im][a];
      G[3 * a + b] = d;
    }
  }
}

// ------------------------------------------------------------------------------------------------
// Lattice helpers.
struct Lat {
  const Grid* g;
  long N;
  long node(int x, int y, int z) const { return ((long)z * g->ny + y) * g->nx + x; }
  void xyz(long n, int& x, int& y, int& z) const {
    x = (int)(n % g->nx);
    y = (int)((n / g->nx) % g->ny);
    z = (int)(n / ((long)g->nx * g->ny));
  }
  // neighbour x + (dx, dy, dz): periodic in y, z and (periodic mode) x; -1 outside a channel
  long nbr(int x, int y, int z, int dx, int dy, int dz) const {
    int X = x + dx, Y = y + dy, Z = z + dz;
    if (g->channel) {
      if (X < 0 || X >= g->nx) return -1;
    } else {
      X = ((X % g->nx) + g->nx) % g->nx;
    }
    Y = ((Y % g->ny) + g->ny) % g->ny;
    Z = ((Z % g->nz) + g->nz) % g->nz;
    return node(X, Y, Z);
  }
};

// Node-local neighbourhood of the stencil maps: nodes x + c_j (27, j = 13 the node) and x +- 2 e_b.
struct Hood {
  long n1[NQ];   // -1 where it does not exist
  long nfar[6];
};

Hood hood(const Lat& L, int x, int y, int z) {
  Hood h;
  for (int j = 0; j < NQ; ++j) h.n1[j] = L.nbr(x, y, z, cxi(j), cyi(j), czi(j));
  for (int b = 0; b < 3; ++b) {
    h.nfar[2 * b] = L.nbr(x, y, z, 2 * (b == 0), 2 * (b == 1), 2 * (b == 2));
    h.nfar[2 * b + 1] = L.nbr(x, y, z, -2 * (b == 0), -2 * (b == 1), -2 * (b == 2));
  }
  return h;
}

// J^T gout of a node-local map fn(x[nin]) -> out[nout], evaluated on dual numbers with the inputs'
// unit tangents seeded ND at a time.  out0 (optional) receives the map's values.
template <class Fn>
void local_vjp(int nin, const double* x, int nout, const double* gout, double* gin, Fn fn, double* out0 = nullptr) {
  std::vector<D> xin(nin), out(nout);
  for (int k0 = 0; k0 < nin; k0 += ND) {
    for (int k = 0; k < nin; ++k) {
      xin[k] = D(x[k]);
      if (k >= k0 && k < k0 + ND) xin[k].d[k - k0] = 1.0;
    }
    fn(xin.data(), out.data());
    for (int k = k0; k < std::min(nin, k0 + ND); ++k) {
      double s = 0.0;
      for (int o = 0; o < nout; ++o) s += gout[o] * out[o].d[k - k0];
      gin[k] = s;
    }
    if (out0 && k0 == 0)
      for (int o = 0; o < nout; ++o) out0[o] = out[o].v;
  }
}

// The frozen, non-differentiable data of a fluid node's step at t+1 (masks only).
struct Links {
  bool inD[NQ];      // population i is missing (source solid at t+1, or through the inlet)
  int body[NQ];      // body hit by a missing link (-1: the inlet)
  long src[NQ];      // pull source of a present population
  int nD;
};

Links links_of(const Lat& L, const uint8_t* solid_t1, int x, int y, int z) {
  const Grid* g = L.g;
  Links k;
  k.nD = 0;
  for (int i = 0; i < NQ; ++i) {
    k.inD[i] = false;
    k.body[i] = -1;
    k.src[i] = -1;
    int sx = x - cxi(i);
    if (g->channel && sx < 0) {  // through the inlet face
      k.inD[i] = true;
      ++k.nD;
      continue;
    }
    long src;
    if (g->channel) {
      if (sx >= g->nx) sx = g->nx - 1;  // the outlet copy
      src = L.nbr(sx, y, z, 0, -cyi(i), -czi(i));
    } else {
      src = L.nbr(x, y, z, -cxi(i), -cyi(i), -czi(i));
    }
    if (solid_t1[src]) {
      k.inD[i] = true;
      k.body[i] = solid_t1[src] - 1;
      ++k.nD;
      continue;
    }
    k.src[i] = src;
  }
  return k;
}

// Inputs of the reconstruction map at a boundary node, in this order:
//   [0, 27)    f_i pulled (present populations; the others unused)
//   [27, 54)   A_w at the node itself in direction opp(i), for missing i (bounce-back value)
//   [54, 135)  U^t at x + c_j, j = 0..26, 3 components each
//   [135, 153) U^t at x +- 2 e_b
//   [153, 153 + nb)  amplitude of each body
// Outputs: [0, 27) the population entering the collision (pulled or reconstructed), then 3 per
// body: the momentum-exchange force of the node's links.
constexpr int RI_FIN = 0, RI_FO = 27, RI_UN = 54, RI_UF = 135, RI_AMP = 153;

template <class S>
void reconstruct(const Grid& g, const Body* bodies, int nb, double t1, const Links& lk, const bool ok1[NQ],
                 const bool okfar[6], const double xb[3], const S* in, S* out) {
  S c1[MAXB][3], U1[MAXB][3];
  for (int k = 0; k < nb; ++k) kinematics(bodies[k], t1, in[RI_AMP + k], c1[k], U1[k]);
  S Un[NQ][3], Ufar[6][3];
  for (int j = 0; j < NQ; ++j)
    for (int a = 0; a < 3; ++a) Un[j][a] = in[RI_UN + 3 * j + a];
  for (int j = 0; j < 6; ++j)
    for (int a = 0; a < 3; ++a) Ufar[j][a] = in[RI_UF + 3 * j + a];
  S f[NQ];
  for (int i = 0; i < NQ; ++i) f[i] = lk.inD[i] ? S(0.0) : in[RI_FIN + i];
  for (int k = 0; k < nb; ++k)
    for (int a = 0; a < 3; ++a) out[NQ + 3 * k + a] = S(0.0);
  if (lk.nD) {
    S q[NQ], uw[NQ][3], ut[3] = {S(0.0), S(0.0), S(0.0)}, rstat(0.0), rdyn(0.0);
    for (int i = 0; i < NQ; ++i) {
      if (!lk.inD[i]) {
        rstat += f[i];
        continue;
      }
      rstat += in[RI_FO + i];
      const int k = lk.body[i];
      if (k < 0) {
        q[i] = S((xb[0] + 0.5) / cxi(i));
        for (int a = 0; a < 3; ++a) uw[i][a] = S(g.u_in[a]);
      } else {
        q[i] = link_fraction(bodies[k], c1[k], xb, i);
        const S xw[3] = {xb[0] - q[i] * (double)cxi(i), xb[1] - q[i] * (double)cyi(i), xb[2] - q[i] * (double)czi(i)};
        rigid_velocity(bodies[k], c1[k], U1[k], xw, uw[i]);
      }
      S uf[3];
      for (int a = 0; a < 3; ++a) uf[a] = ok1[i] ? Un[i][a] : uw[i][a];
      for (int a = 0; a < 3; ++a) ut[a] += (q[i] * uf[a] + uw[i][a]) / (1.0 + q[i]);
      rdyn += 6.0 * wgt(i) * g.rho0 *
              ((double)cxi(i) * uw[i][0] + (double)cyi(i) * uw[i][1] + (double)czi(i) * uw[i][2]);
    }
    for (int a = 0; a < 3; ++a) ut[a] /= (double)lk.nD;
    const S rtgt = rstat + rdyn;
    S G[9], Pi[9], fs[NQ];
    grad_u(Un, Ufar, ok1, okfar, G);
    pressure(rtgt, ut, G, g.beta, Pi);
    grad_dist(rtgt, ut, Pi, fs);
    for (int i = 0; i < NQ; ++i) {
      if (!lk.inD[i]) continue;
      f[i] = fs[i];
      const int k = lk.body[i];
      if (k < 0) continue;
      const S fo = in[RI_FO + i];
      for (int a = 0; a < 3; ++a)
        out[NQ + 3 * k + a] += fo * (-(double)cc(i, a) - uw[i][a]) - fs[i] * ((double)cc(i, a) - uw[i][a]);
    }
  }
  for (int i = 0; i < NQ; ++i) out[i] = f[i];
}

// Refill of a node uncovered at t+1 (Sec. III): Grad's distribution at the wall velocity of the
// node (the body that held it at t, velocity at t+1), the mean R^t of the neighbours fluid at t
// and t+1 (rho0 if none), and the pressure tensor of the stencil gradient.  Inputs:
//   [0, 27) R^t at x + c_j;  [27, 108) U^t at x + c_j;  [108, 126) U^t at x +- 2 e_b;  then amp.
constexpr int FI_R = 0, FI_UN = 27, FI_UF = 108, FI_AMP = 126;

template <class S>
void refill(const Grid& g, const Body& b, double t1, const bool cnt[NQ], const bool ok1[NQ], const bool okfar[6],
            const double xb[3], const S* in, S* out) {
  S c1[3], U1[3];
  kinematics(b, t1, in[FI_AMP], c1, U1);
  const S xs[3] = {S(xb[0]), S(xb[1]), S(xb[2])};
  S uw[3];
  rigid_velocity(b, c1, U1, xs, uw);
  S rs(0.0);
  int m = 0;
  for (int j = 0; j < NQ; ++j) {
    if (!cnt[j]) continue;
    rs += in[FI_R + j];
    ++m;
  }
  const S ravg = m ? rs / (double)m : S(g.rho0);
  S Un[NQ][3], Ufar[6][3];
  for (int j = 0; j < NQ; ++j)
    for (int a = 0; a < 3; ++a) Un[j][a] = in[FI_UN + 3 * j + a];
  for (int j = 0; j < 6; ++j)
    for (int a = 0; a < 3; ++a) Ufar[j][a] = in[FI_UF + 3 * j + a];
  S G[9], Pi[9];
  grad_u(Un, Ufar, ok1, okfar, G);
  pressure(ravg, uw, G, g.beta, Pi);
  grad_dist(ravg, uw, Pi, out);
}

// U^t, R^t of a node fluid at t (the forward oracle's reading): U = (j - F/2)/rho, R = rho.
// Inputs: A^t (27), F (3).  Outputs: U (3), R.
template <class S>
void macro_fluid(const S* in, S* out) {
  const S* f = in;
  const S rho = raw_moment(f, 0, 0, 0);
  const S j[3] = {raw_moment(f, 1, 0, 0), raw_moment(f, 0, 1, 0), raw_moment(f, 0, 0, 1)};
  for (int a = 0; a < 3; ++a) out[a] = (j[a] - 0.5 * in[NQ + a]) / rho;
  out[3] = rho;
}

int check(const Grid* g, const Body* bodies, int nb) {
  if (nb < 0 || nb > MAXB) return -1;
  if (g->stabiliser == 1 || g->central) return -4;
  for (int k = 0; k < nb; ++k)
    if (bodies[k].tracked || (bodies[k].kind != 0 && bodies[k].kind != 1)) return -3;
  return 0;
}

}  // namespace

// ==================================================================================================
extern "C" {

/* Single-node maps, for the tests of each piece against finite differences of the forward oracle. */

// KBC collision of one node (value): f in place; F may be NULL; lbgk = 1 for gamma = 2.
void oa_collide(double f[NQ], double beta, const double* F, int lbgk) { collide<double>(f, beta, F, lbgk != 0); }

// (d f'/d f)^T gout and (d f'/d F)^T gout of the collision at f (F may be NULL, then gF is untouched).
void oa_collide_vjp(const double f[NQ], double beta, const double* F, int lbgk, const double gout[NQ],
                    double gf[NQ], double gF[3]) {
  double x[NQ + 3], gin[NQ + 3];
  for (int i = 0; i < NQ; ++i) x[i] = f[i];
  for (int a = 0; a < 3; ++a) x[NQ + a] = F ? F[a] : 0.0;
  const bool force = F != nullptr;
  local_vjp(NQ + 3, x, NQ, gout, gin, [&](const D* in, D* out) {
    for (int i = 0; i < NQ; ++i) out[i] = in[i];
    collide<D>(out, beta, force ? in + NQ : nullptr, lbgk != 0);
  });
  for (int i = 0; i < NQ; ++i) gf[i] = gin[i];
  if (F)
    for (int a = 0; a < 3; ++a) gF[a] = gin[NQ + a];
}

// Grad's distribution at (rho, u, Pi(rho, u, G)) and its transposed derivative: g_rho, g_u[3], g_G[9].
void oa_grad_pressure_vjp(double rho, const double u[3], const double G[9], double beta, const double gout[NQ],
                          double out[NQ], double* g_rho, double g_u[3], double g_G[9]) {
  double x[13], gin[13];
  x[0] = rho;
  for (int a = 0; a < 3; ++a) x[1 + a] = u[a];
  for (int k = 0; k < 9; ++k) x[4 + k] = G[k];
  local_vjp(13, x, NQ, gout, gin, [&](const D* in, D* o) {
    D Pi[9];
    pressure(in[0], in + 1, in + 4, beta, Pi);
    grad_dist(in[0], in + 1, Pi, o);
  }, out);
  *g_rho = gin[0];
  for (int a = 0; a < 3; ++a) g_u[a] = gin[1 + a];
  for (int k = 0; k < 9; ++k) g_G[k] = gin[4 + k];
}

// Link fraction of body b (centre c) along direction i from xb, and dq/dc.
double oa_link_fraction(const Body* b, const double c[3], const double xb[3], int i, double dq_dc[3]) {
  double gin[3], q = 0.0;
  const double one = 1.0;
  local_vjp(3, c, 1, &one, gin, [&](const D* in, D* o) { o[0] = link_fraction(*b, in, xb, i); }, &q);
  for (int a = 0; a < 3; ++a) dq_dc[a] = gin[a];
  return q;
}

/* One adjoint step (see the file header).  A_t, lam: [27][N]; solid_t, solid_t1: [N], 0 = fluid,
 * 1 + k = inside body k; F: [3][N] or NULL; w_force: [nb][3] or NULL.  Outputs: lam_out [27][N]
 * (overwritten); gF [3][N] (added to, may be NULL when F is NULL); gamp [nb] (added to).  A_t1
 * [27][N] and forces [nb][3] (optional, NULL to skip) receive the forward step's values, for the
 * check against the forward oracle.  Returns 0, or -1 bad arguments, -2 out of memory,
 * -3 unsupported body, -4 unsupported collision variant. */
int oa_adjoint_step(const Grid* g, const Body* bodies, int nb, double t, const double* A_t, const uint8_t* solid_t,
                    const uint8_t* solid_t1, const double* F, const double* lam, const double* w_force,
                    double* lam_out, double* gF, double* gamp, double* A_t1, double* forces) {
  const int rc = check(g, bodies, nb);
  if (rc) return rc;
  if (!A_t || !solid_t || !solid_t1 || !lam || !lam_out || (nb > 0 && !gamp)) return -1;
  Lat L{g, (long)g->nx * g->ny * g->nz};
  const long N = L.N;
  const double t1 = t + 1.0;
  const bool lbgk = g->stabiliser == 2;
  double amp[MAXB];
  for (int k = 0; k < nb; ++k) amp[k] = bodies[k].amp;
  double c0[MAXB][3], U0[MAXB][3];
  for (int k = 0; k < nb; ++k) kinematics<double>(bodies[k], t, amp[k], c0[k], U0[k]);

  std::vector<double> U(3 * N), R(N), Aw(A_t, A_t + NQ * N);
  // ---- forward: U^t, R^t (fluid at t: moments; solid at t: rigid-body velocity, rho0)
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; ++n) {
    double o[4];
    if (solid_t[n]) {
      const int k = solid_t[n] - 1;
      int x, y, z;
      L.xyz(n, x, y, z);
      const double xp[3] = {(double)x, (double)y, (double)z};
      rigid_velocity<double>(bodies[k], c0[k], U0[k], xp, o);
      o[3] = g->rho0;
    } else {
      double in[NQ + 3];
      for (int i = 0; i < NQ; ++i) in[i] = A_t[i * N + n];
      for (int a = 0; a < 3; ++a) in[NQ + a] = F ? F[a * N + n] : 0.0;
      macro_fluid<double>(in, o);
    }
    for (int a = 0; a < 3; ++a) U[a * N + n] = o[a];
    R[n] = o[3];
  }
  // local stencil data: usable = exists and fluid at t+1
  auto usable = [&](long m) { return m >= 0 && !solid_t1[m]; };
  auto gather_U = [&](const Hood& h, double* dst) {  // 27 x 3 then 6 x 3
    for (int j = 0; j < NQ; ++j)
      for (int a = 0; a < 3; ++a) dst[3 * j + a] = h.n1[j] >= 0 ? U[a * N + h.n1[j]] : 0.0;
    for (int j = 0; j < 6; ++j)
      for (int a = 0; a < 3; ++a) dst[3 * NQ + 3 * j + a] = h.nfar[j] >= 0 ? U[a * N + h.nfar[j]] : 0.0;
  };
  // ---- forward: refill of the nodes uncovered at t+1 (written into A_w before streaming)
  std::vector<long> refills;
  for (long n = 0; n < N; ++n)
    if (solid_t[n] && !solid_t1[n]) refills.push_back(n);
  const long nref = (long)refills.size();
  constexpr int NFI = FI_AMP + 1;
  std::vector<double> fin_refill((size_t)nref * NFI);
#pragma omp parallel for schedule(dynamic, 4)
  for (long r = 0; r < nref; ++r) {
    const long n = refills[r];
    int x, y, z;
    L.xyz(n, x, y, z);
    const Hood h = hood(L, x, y, z);
    const int k = solid_t[n] - 1;
    bool cnt[NQ], ok1[NQ], okfar[6];
    for (int j = 0; j < NQ; ++j) {
      cnt[j] = j != 13 && h.n1[j] >= 0 && !solid_t[h.n1[j]] && !solid_t1[h.n1[j]];
      ok1[j] = usable(h.n1[j]);
    }
    for (int j = 0; j < 6; ++j) okfar[j] = usable(h.nfar[j]);
    double* in = &fin_refill[(size_t)r * NFI];
    for (int j = 0; j < NQ; ++j) in[FI_R + j] = h.n1[j] >= 0 ? R[h.n1[j]] : 0.0;
    gather_U(h, in + FI_UN);
    in[FI_AMP] = amp[k];
    const double xb[3] = {(double)x, (double)y, (double)z};
    double out[NQ];
    refill<double>(*g, bodies[k], t1, cnt, ok1, okfar, xb, in, out);
    for (int i = 0; i < NQ; ++i) Aw[i * N + n] = out[i];
  }

  // ---- per fluid node at t+1: the population entering the collision, the collision, and the
  // adjoint of the collision (G_f = (d f'/d f)^T lam, dL/dF of the node)
  constexpr int NRI = RI_AMP + MAXB;
  std::vector<double> Gf((size_t)NQ * N, 0.0);
  std::vector<double> fz((size_t)g->nz * MAXB * 3, 0.0);  // forces per z plane (fixed order)
  std::vector<char> isbnd(N, 0);
  std::vector<double> gFl(F ? 3 * N : 0, 0.0);
#pragma omp parallel for schedule(dynamic, 1)
  for (int z = 0; z < g->nz; ++z)
    for (int y = 0; y < g->ny; ++y)
      for (int x = 0; x < g->nx; ++x) {
        const long n = L.node(x, y, z);
        if (solid_t1[n]) {
          if (A_t1)
            for (int i = 0; i < NQ; ++i) A_t1[i * N + n] = A_t[i * N + n];
          continue;
        }
        const Links lk = links_of(L, solid_t1, x, y, z);
        double f[NQ];
        if (lk.nD) {
          isbnd[n] = 1;
          const Hood h = hood(L, x, y, z);
          bool ok1[NQ], okfar[6];
          for (int j = 0; j < NQ; ++j) ok1[j] = usable(h.n1[j]);
          for (int j = 0; j < 6; ++j) okfar[j] = usable(h.nfar[j]);
          double in[NRI] = {0.0}, out[NQ + 3 * MAXB];
          for (int i = 0; i < NQ; ++i) {
            if (!lk.inD[i]) in[RI_FIN + i] = Aw[i * N + lk.src[i]];
            else in[RI_FO + i] = Aw[(26 - i) * N + n];
          }
          gather_U(h, in + RI_UN);
          for (int k = 0; k < nb; ++k) in[RI_AMP + k] = amp[k];
          const double xb[3] = {(double)x, (double)y, (double)z};
          reconstruct<double>(*g, bodies, nb, t1, lk, ok1, okfar, xb, in, out);
          for (int i = 0; i < NQ; ++i) f[i] = out[i];
          for (int k = 0; k < nb; ++k)
            for (int a = 0; a < 3; ++a) fz[((size_t)z * MAXB + k) * 3 + a] += out[NQ + 3 * k + a];
        } else {
          for (int i = 0; i < NQ; ++i) f[i] = Aw[i * N + lk.src[i]];
        }
        double Fn[3] = {0.0, 0.0, 0.0};
        if (F)
          for (int a = 0; a < 3; ++a) Fn[a] = F[a * N + n];
        if (A_t1) {
          double fp[NQ];
          std::memcpy(fp, f, sizeof fp);
          if (!g->stream_only) collide<double>(fp, g->beta, F ? Fn : nullptr, lbgk);
          for (int i = 0; i < NQ; ++i) A_t1[i * N + n] = fp[i];
        }
        double gl[NQ];
        for (int i = 0; i < NQ; ++i) gl[i] = lam[i * N + n];
        if (g->stream_only) {
          for (int i = 0; i < NQ; ++i) Gf[i * N + n] = gl[i];
          continue;
        }
        double gf[NQ], gFn[3] = {0.0, 0.0, 0.0};
        oa_collide_vjp(f, g->beta, F ? Fn : nullptr, lbgk ? 1 : 0, gl, gf, gFn);
        for (int i = 0; i < NQ; ++i) Gf[i * N + n] = gf[i];
        if (F)
          for (int a = 0; a < 3; ++a) gFl[a * N + n] += gFn[a];
      }
  if (forces) {
    for (int k = 0; k < nb; ++k)
      for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int z = 0; z < g->nz; ++z) s += fz[((size_t)z * MAXB + k) * 3 + a];
        forces[3 * k + a] = s;
      }
  }

  // ---- reverse
  std::vector<double> gA((size_t)NQ * N, 0.0), gAw((size_t)NQ * N, 0.0), gU(3 * N, 0.0), gR(N, 0.0);
  double gampl[MAXB] = {0.0};
  // nodes solid at t+1 keep their populations: A^{t+1} = A^t there
  for (long n = 0; n < N; ++n)
    if (solid_t1[n])
      for (int i = 0; i < NQ; ++i) gA[i * N + n] += lam[i * N + n];
  // boundary nodes: the reconstruction map's input adjoints (computed in parallel, added in order)
  std::vector<long> bnodes;
  for (long n = 0; n < N; ++n)
    if (isbnd[n]) bnodes.push_back(n);
  const long nbn = (long)bnodes.size();
  std::vector<double> gin_b((size_t)nbn * NRI, 0.0);
#pragma omp parallel for schedule(dynamic, 4)
  for (long r = 0; r < nbn; ++r) {
    const long n = bnodes[r];
    int x, y, z;
    L.xyz(n, x, y, z);
    const Links lk = links_of(L, solid_t1, x, y, z);
    const Hood h = hood(L, x, y, z);
    bool ok1[NQ], okfar[6];
    for (int j = 0; j < NQ; ++j) ok1[j] = usable(h.n1[j]);
    for (int j = 0; j < 6; ++j) okfar[j] = usable(h.nfar[j]);
    const int nin = RI_AMP + nb;
    double in[NRI] = {0.0}, gout[NQ + 3 * MAXB];
    for (int i = 0; i < NQ; ++i) {
      if (!lk.inD[i]) in[RI_FIN + i] = Aw[i * N + lk.src[i]];
      else in[RI_FO + i] = Aw[(26 - i) * N + n];
    }
    gather_U(h, in + RI_UN);
    for (int k = 0; k < nb; ++k) in[RI_AMP + k] = amp[k];
    for (int i = 0; i < NQ; ++i) gout[i] = Gf[i * N + n];
    for (int k = 0; k < nb; ++k)
      for (int a = 0; a < 3; ++a) gout[NQ + 3 * k + a] = w_force ? w_force[3 * k + a] : 0.0;
    const double xb[3] = {(double)x, (double)y, (double)z};
    local_vjp(nin, in, NQ + 3 * nb, gout, &gin_b[(size_t)r * NRI], [&](const D* xin, D* o) {
      reconstruct<D>(*g, bodies, nb, t1, lk, ok1, okfar, xb, xin, o);
    });
  }
  // transpose of the pull (interior nodes: G_f goes to the pulled entry) and of the reconstruction
  long bi = 0;
  for (int z = 0; z < g->nz; ++z)
    for (int y = 0; y < g->ny; ++y)
      for (int x = 0; x < g->nx; ++x) {
        const long n = L.node(x, y, z);
        if (solid_t1[n]) continue;
        if (!isbnd[n]) {
          const Links lk = links_of(L, solid_t1, x, y, z);
          for (int i = 0; i < NQ; ++i) gAw[i * N + lk.src[i]] += Gf[i * N + n];
          continue;
        }
        const double* gi = &gin_b[(size_t)bi++ * NRI];
        const Links lk = links_of(L, solid_t1, x, y, z);
        const Hood h = hood(L, x, y, z);
        for (int i = 0; i < NQ; ++i) {
          if (!lk.inD[i]) gAw[i * N + lk.src[i]] += gi[RI_FIN + i];
          else gAw[(26 - i) * N + n] += gi[RI_FO + i];
        }
        for (int j = 0; j < NQ; ++j)
          if (h.n1[j] >= 0)
            for (int a = 0; a < 3; ++a) gU[a * N + h.n1[j]] += gi[RI_UN + 3 * j + a];
        for (int j = 0; j < 6; ++j)
          if (h.nfar[j] >= 0)
            for (int a = 0; a < 3; ++a) gU[a * N + h.nfar[j]] += gi[RI_UF + 3 * j + a];
        for (int k = 0; k < nb; ++k) gampl[k] += gi[RI_AMP + k];
      }
  // refill nodes: their A_w entries came from the refill map, not from A^t
  std::vector<double> gin_r((size_t)nref * NFI, 0.0);
#pragma omp parallel for schedule(dynamic, 4)
  for (long r = 0; r < nref; ++r) {
    const long n = refills[r];
    int x, y, z;
    L.xyz(n, x, y, z);
    const Hood h = hood(L, x, y, z);
    const int k = solid_t[n] - 1;
    bool cnt[NQ], ok1[NQ], okfar[6];
    for (int j = 0; j < NQ; ++j) {
      cnt[j] = j != 13 && h.n1[j] >= 0 && !solid_t[h.n1[j]] && !solid_t1[h.n1[j]];
      ok1[j] = usable(h.n1[j]);
    }
    for (int j = 0; j < 6; ++j) okfar[j] = usable(h.nfar[j]);
    double gout[NQ];
    for (int i = 0; i < NQ; ++i) gout[i] = gAw[i * N + n];
    const double xb[3] = {(double)x, (double)y, (double)z};
    local_vjp(NFI, &fin_refill[(size_t)r * NFI], NQ, gout, &gin_r[(size_t)r * NFI], [&](const D* xin, D* o) {
      refill<D>(*g, bodies[k], t1, cnt, ok1, okfar, xb, xin, o);
    });
  }
  std::vector<char> isref(N, 0);
  for (long r = 0; r < nref; ++r) {
    const long n = refills[r];
    isref[n] = 1;
    int x, y, z;
    L.xyz(n, x, y, z);
    const Hood h = hood(L, x, y, z);
    const double* gi = &gin_r[(size_t)r * NFI];
    for (int j = 0; j < NQ; ++j)
      if (h.n1[j] >= 0) {
        gR[h.n1[j]] += gi[FI_R + j];
        for (int a = 0; a < 3; ++a) gU[a * N + h.n1[j]] += gi[FI_UN + 3 * j + a];
      }
    for (int j = 0; j < 6; ++j)
      if (h.nfar[j] >= 0)
        for (int a = 0; a < 3; ++a) gU[a * N + h.nfar[j]] += gi[FI_UF + 3 * j + a];
    gampl[solid_t[n] - 1] += gi[FI_AMP];
  }
  for (long n = 0; n < N; ++n)
    if (!isref[n])
      for (int i = 0; i < NQ; ++i) gA[i * N + n] += gAw[i * N + n];
  // U^t, R^t: moments of A^t at nodes fluid at t, the rigid-body velocity at nodes solid at t
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; ++n) {
    const double go[4] = {gU[n], gU[N + n], gU[2 * N + n], gR[n]};
    if (go[0] == 0.0 && go[1] == 0.0 && go[2] == 0.0 && go[3] == 0.0) continue;
    if (solid_t[n]) continue;  // handled below (amplitude, serial)
    double in[NQ + 3], gi[NQ + 3];
    for (int i = 0; i < NQ; ++i) in[i] = A_t[i * N + n];
    for (int a = 0; a < 3; ++a) in[NQ + a] = F ? F[a * N + n] : 0.0;
    local_vjp(NQ + 3, in, 4, go, gi, [&](const D* xin, D* o) { macro_fluid<D>(xin, o); });
    for (int i = 0; i < NQ; ++i) gA[i * N + n] += gi[i];
    if (F)
      for (int a = 0; a < 3; ++a) gFl[a * N + n] += gi[NQ + a];
  }
  for (long n = 0; n < N; ++n) {
    if (!solid_t[n]) continue;
    const double go[3] = {gU[n], gU[N + n], gU[2 * N + n]};
    if (go[0] == 0.0 && go[1] == 0.0 && go[2] == 0.0) continue;
    const int k = solid_t[n] - 1;
    int x, y, z;
    L.xyz(n, x, y, z);
    double gi = 0.0;
    const double a0 = amp[k];
    local_vjp(1, &a0, 3, go, &gi, [&](const D* xin, D* o) {
      D c[3], Ub[3];
      kinematics(bodies[k], t, xin[0], c, Ub);
      const D xp[3] = {D((double)x), D((double)y), D((double)z)};
      rigid_velocity(bodies[k], c, Ub, xp, o);
    });
    gampl[k] += gi;
  }
  std::memcpy(lam_out, gA.data(), sizeof(double) * NQ * N);
  if (gF && F)
    for (long m = 0; m < 3 * N; ++m) gF[m] += gFl[m];
  for (int k = 0; k < nb; ++k) gamp[k] += gampl[k];
  return 0;
}

}  // extern "C"
