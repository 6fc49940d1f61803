/*
 * elbm_oracle.c -- plain, slow FP64 CPU reference ("oracle") for one time step
 * of the entropic multi-relaxation-time (KBC) lattice Boltzmann method with
 * moving-wall Grad boundary conditions, after Dorschner, Chikatamarla and
 * Karlin, "Entropic lattice Boltzmann method for moving and deforming
 * geometries in three dimensions" (arXiv:1608.04658).
 *
 * TEST INFRASTRUCTURE ONLY.  The product library never links, loads or calls
 * this file.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or constant with the
 * GPU implementation; its lattice tables are its own.
 *
 * Every routine restates a passage of the paper and names it (section and
 * equation label).  Where the paper is silent the code says "reading:" and
 * states the choice made.  No blocking, fusion or reordering is done beyond
 * what the equations state: one scalar loop per node, FP64 throughout.
 *
 * Population layout used by every array here: f[i * N + n], with the node
 * index n = (z * ny + y) * nx + x and N = nx * ny * nz.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NQ 27
#define MAXB 8

/* ------------------------------------------------------------------------ */
/* Lattice (Sec. II): the standard D3Q27 velocity set c_i in {-1,0,1}^3 with
 * sound speed c_s^2 = 1/3.  Enumeration: i = 9 (cz+1) + 3 (cy+1) + (cx+1),
 * so the opposite direction of i is 26 - i and the rest velocity is i = 13.
 * Reading: the paper names the lattice but does not print its weights; they
 * are the tensor-product weights W_i = w(cx) w(cy) w(cz) with w(0) = 2/3 and
 * w(+-1) = 1/6. */
static int cxi(int i) { return i % 3 - 1; }
static int cyi(int i) { return (i / 3) % 3 - 1; }
static int czi(int i) { return i / 9 - 1; }
static int ci(int i, int a) { return a == 0 ? cxi(i) : (a == 1 ? cyi(i) : czi(i)); }
static int opp(int i) { return 26 - i; }
static double w1(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
static double wgt(int i) { return w1(cxi(i)) * w1(cyi(i)) * w1(czi(i)); }
static const double CS2 = 1.0 / 3.0;

void or_lattice(int32_t c[NQ * 3], double w[NQ]) {
  for (int i = 0; i < NQ; ++i) {
    c[3 * i] = cxi(i); c[3 * i + 1] = cyi(i); c[3 * i + 2] = czi(i);
    w[i] = wgt(i);
  }
}

/* Raw moment M_pqr = sum_i f_i cx^p cy^q cz^r. */
static double ipow(int c, int p) { double r = 1.0; for (int k = 0; k < p; ++k) r *= c; return r; }
static double moment(const double f[NQ], int p, int q, int r) {
  double m = 0.0;
  for (int i = 0; i < NQ; ++i) m += f[i] * ipow(cxi(i), p) * ipow(cyi(i), q) * ipow(czi(i), r);
  return m;
}

/* Chapman-Enskog relation of Sec. II, nu = c_s^2 (1/(2 beta) - 1/2), solved for beta. */
double or_beta_from_nu(double nu) { return 1.0 / (2.0 * nu / CS2 + 1.0); }

/* ------------------------------------------------------------------------ */
/* Entropic equilibrium (eq. feq_min): the minimiser of H(f) = sum f ln(f/W)
 * at fixed rho and j.  Reading: the "exact solution" the paper cites is the
 * closed form that factorises over the three Cartesian axes,
 *   feq_i = rho prod_a w(c_ia) (2 - s_a) [(2 u_a + s_a) / (1 - u_a)]^{c_ia},
 *   s_a = sqrt(1 + 3 u_a^2).
 * Tests check it against the definition: the constraints and the stationarity
 * (KKT) condition of the minimisation, and a numerical minimiser. */
void or_feq(double rho, const double u[3], double feq[NQ]) {
  double phi[3][3];
  for (int a = 0; a < 3; ++a) {
    double s = sqrt(1.0 + 3.0 * u[a] * u[a]);
    double X = (2.0 * u[a] + s) / (1.0 - u[a]);
    phi[a][0] = w1(-1) * (2.0 - s) / X;
    phi[a][1] = w1(0) * (2.0 - s);
    phi[a][2] = w1(1) * (2.0 - s) * X;
  }
  for (int i = 0; i < NQ; ++i)
    feq[i] = rho * phi[0][cxi(i) + 1] * phi[1][cyi(i) + 1] * phi[2][czi(i) + 1];
}

/* ------------------------------------------------------------------------ */
/* KBC decomposition f = k + s + h (Sec. II).
 * Reading: the "natural moment basis" is the raw moments M_pqr, p,q,r in {0,1,2};
 * a population set is rebuilt from them with the 1-D dual basis
 *   phi_0(c) = 1 - c^2,  phi_1(c) = c/2,  phi_2(c) = 3 c^2 / 2 - 1,
 * i.e. f_i = sum_pqr M_pqr phi_p(cx) phi_q(cy) phi_r(cz).
 *   k: the locally conserved moments rho = M000, j = (M100, M010, M001).
 *   s: the deviatoric stress -- the traceless part of the diagonal second
 *      moments and the three off-diagonal ones.
 *   h: everything else, including the trace of the stress, whose relaxation
 *      with gamma*beta is what the bulk-viscosity relation of Sec. II states. */
static double phib(int p, int c) {
  if (p == 0) return 1.0 - c * c;
  if (p == 1) return 0.5 * c;
  return 1.5 * c * c - 1.0;
}
static double basis(int p, int q, int r, int i) { return phib(p, cxi(i)) * phib(q, cyi(i)) * phib(r, czi(i)); }

/* Central-moment member of the KBC family (an addition; the paper uses the raw basis): moments in
 * the frame moving with the node's velocity u,
 *   M^c_pqr = sum_i f_i (cx - ux)^p (cy - uy)^q (cz - uz)^r,
 * and populations rebuilt from them with the 1-D dual basis of the shifted velocities
 * c - u in {-1 - u, -u, 1 - u}: psi_p(c; u) is the coefficient of xi^p in the Lagrange
 * polynomial of the three points that is 1 at c - u and 0 at the other two.  s is again the
 * deviatoric part of the second moments, now central.  At u = 0 the basis is the raw one. */
static void psi_central(double u, double psi[3][3]) { /* psi[p][c + 1] */
  for (int c = -1; c <= 1; ++c) {
    double a = 0.0, b = 0.0, den = 1.0;
    int n = 0;
    for (int k = -1; k <= 1; ++k) {
      if (k == c) continue;
      const double node = (double)k - u;
      if (n == 0) a = node; else b = node;
      den *= (double)(c - k);
      ++n;
    }
    psi[0][c + 1] = a * b / den;   /* (xi - a)(xi - b) = xi^2 - (a + b) xi + a b */
    psi[1][c + 1] = -(a + b) / den;
    psi[2][c + 1] = 1.0 / den;
  }
}

static double central_moment(const double f[NQ], const double u[3], int p, int q, int r) {
  double m = 0.0;
  for (int i = 0; i < NQ; ++i)
    m += f[i] * pow(cxi(i) - u[0], p) * pow(cyi(i) - u[1], q) * pow(czi(i) - u[2], r);
  return m;
}

void or_shear_part_central(const double f[NQ], const double u[3], double s[NQ]) {
  double px[3][3], py[3][3], pz[3][3];
  psi_central(u[0], px);
  psi_central(u[1], py);
  psi_central(u[2], pz);
  double M200 = central_moment(f, u, 2, 0, 0), M020 = central_moment(f, u, 0, 2, 0), M002 = central_moment(f, u, 0, 0, 2);
  double M110 = central_moment(f, u, 1, 1, 0), M101 = central_moment(f, u, 1, 0, 1), M011 = central_moment(f, u, 0, 1, 1);
  double T = M200 + M020 + M002;
  double D200 = M200 - T / 3.0, D020 = M020 - T / 3.0, D002 = M002 - T / 3.0;
  for (int i = 0; i < NQ; ++i) {
    const int x = cxi(i) + 1, y = cyi(i) + 1, z = czi(i) + 1;
    s[i] = D200 * px[2][x] * py[0][y] * pz[0][z] + D020 * px[0][x] * py[2][y] * pz[0][z] +
           D002 * px[0][x] * py[0][y] * pz[2][z] + M110 * px[1][x] * py[1][y] * pz[0][z] +
           M101 * px[1][x] * py[0][y] * pz[1][z] + M011 * px[0][x] * py[1][y] * pz[1][z];
  }
}

static void kinematic_part(const double f[NQ], double k[NQ]) {
  double M000 = moment(f, 0, 0, 0), M100 = moment(f, 1, 0, 0), M010 = moment(f, 0, 1, 0),
         M001 = moment(f, 0, 0, 1);
  for (int i = 0; i < NQ; ++i)
    k[i] = M000 * basis(0, 0, 0, i) + M100 * basis(1, 0, 0, i) + M010 * basis(0, 1, 0, i) +
           M001 * basis(0, 0, 1, i);
}

void or_shear_part(const double f[NQ], double s[NQ]) {
  double M200 = moment(f, 2, 0, 0), M020 = moment(f, 0, 2, 0), M002 = moment(f, 0, 0, 2);
  double M110 = moment(f, 1, 1, 0), M101 = moment(f, 1, 0, 1), M011 = moment(f, 0, 1, 1);
  double T = M200 + M020 + M002;
  double D200 = M200 - T / 3.0, D020 = M020 - T / 3.0, D002 = M002 - T / 3.0;
  for (int i = 0; i < NQ; ++i)
    s[i] = D200 * basis(2, 0, 0, i) + D020 * basis(0, 2, 0, i) + D002 * basis(0, 0, 2, i) +
           M110 * basis(1, 1, 0, i) + M101 * basis(1, 0, 1, i) + M011 * basis(0, 1, 1, i);
}

/* Entropic scalar product <X|Y> = sum_i X_i Y_i / feq_i (Sec. II). */
static double esp(const double X[NQ], const double Y[NQ], const double feq[NQ]) {
  double r = 0.0;
  for (int i = 0; i < NQ; ++i) r += X[i] * Y[i] / feq[i];
  return r;
}

/* One KBC collision at one node (eqs. kineticEq, kbc_relax):
 *   f' = (1 - beta) f + beta f_mirr,
 *   f_mirr = k + (2 s_eq - s) + ((1 - gamma) h + gamma h_eq),
 * with the analytic stabiliser of Sec. II
 *   gamma = 1/beta - (2 - 1/beta) <ds|dh> / <dh|dh>.
 * Reading (the paper is silent on <dh|dh> = 0): if <dh|dh> <= 1e-30 then
 * gamma = 2, the LBGK value; dh is then zero to round-off and f' does not
 * depend on gamma.
 * Body force F (not part of the paper; an addition of this library): exact-
 * difference shift f' += feq(rho, u + F/rho) - feq(rho, u).  Pass F = NULL for
 * none.  gamma_fixed > 0 replaces the stabiliser by that constant (tests).
 * Returns gamma; *guard is set to 1 when the <dh|dh> rule was used. */
static double collide_basis(double f[NQ], double beta, const double *F, double gamma_fixed, int *guard, int central);
double or_collide_ex(double f[NQ], double beta, const double *F, double gamma_fixed, int *guard) {
  return collide_basis(f, beta, F, gamma_fixed, guard, 0);
}

/* The same collision with the central-moment s of or_shear_part_central (central = 1). */
double or_collide_central(double f[NQ], double beta, const double *F, double gamma_fixed, int *guard) {
  return collide_basis(f, beta, F, gamma_fixed, guard, 1);
}

static double collide_basis(double f[NQ], double beta, const double *F, double gamma_fixed, int *guard, int central) {
  double rho = moment(f, 0, 0, 0);
  double u[3] = {moment(f, 1, 0, 0) / rho, moment(f, 0, 1, 0) / rho, moment(f, 0, 0, 1) / rho};
  double feq[NQ], k[NQ], s[NQ], h[NQ], seq[NQ], heq[NQ], keq[NQ], ds[NQ], dh[NQ];
  or_feq(rho, u, feq);
  kinematic_part(f, k);
  kinematic_part(feq, keq);
  if (central) {
    or_shear_part_central(f, u, s);
    or_shear_part_central(feq, u, seq);
  } else {
    or_shear_part(f, s);
    or_shear_part(feq, seq);
  }
  for (int i = 0; i < NQ; ++i) {
    h[i] = f[i] - k[i] - s[i];
    heq[i] = feq[i] - keq[i] - seq[i];
    ds[i] = s[i] - seq[i];
    dh[i] = h[i] - heq[i];
  }
  double a = esp(ds, dh, feq), b = esp(dh, dh, feq);
  double gamma;
  int g = 0;
  if (gamma_fixed > 0.0) {
    gamma = gamma_fixed;
  } else if (b > 1e-30) {
    gamma = 1.0 / beta - (2.0 - 1.0 / beta) * a / b;
  } else {
    gamma = 2.0;
    g = 1;
  }
  if (guard) *guard = g;
  for (int i = 0; i < NQ; ++i) {
    double fmirr = k[i] + (2.0 * seq[i] - s[i]) + ((1.0 - gamma) * h[i] + gamma * heq[i]);
    f[i] = (1.0 - beta) * f[i] + beta * fmirr;
  }
  if (F) {
    double u2[3] = {u[0] + F[0] / rho, u[1] + F[1] / rho, u[2] + F[2] / rho};
    double feq2[NQ];
    or_feq(rho, u2, feq2);
    for (int i = 0; i < NQ; ++i) f[i] += feq2[i] - feq[i];
  }
  return gamma;
}

double or_collide(double f[NQ], double beta, const double *F) { return or_collide_ex(f, beta, F, 0.0, 0); }

/* Exact stabiliser (eq. gamma_min): the root in gamma of
 *   G(gamma) = sum_i dh_i ln[1 + ((1 - beta gamma) dh_i - (2 beta - 1) ds_i) / feq_i] = 0,
 * i.e. the gamma that minimises H(f') along the one-parameter family of
 * post-collision states.  G decreases in gamma wherever every argument of the
 * logarithm is positive; the root is bracketed inside that interval and found
 * by bisection.  Used by tests only (the paper uses the analytic
 * approximation).  Returns NAN if no root is bracketed. */
double or_gamma_exact(const double f_in[NQ], double beta) {
  double f[NQ];
  memcpy(f, f_in, sizeof f);
  double rho = moment(f, 0, 0, 0);
  double u[3] = {moment(f, 1, 0, 0) / rho, moment(f, 0, 1, 0) / rho, moment(f, 0, 0, 1) / rho};
  double feq[NQ], s[NQ], seq[NQ], df[NQ], ds[NQ], dh[NQ];
  or_feq(rho, u, feq);
  for (int i = 0; i < NQ; ++i) df[i] = f[i] - feq[i];
  or_shear_part(f, s);
  or_shear_part(feq, seq);
  for (int i = 0; i < NQ; ++i) { ds[i] = s[i] - seq[i]; dh[i] = df[i] - ds[i]; }
  /* admissible interval: 1 + ((1 - beta g) dh - (2 beta - 1) ds)/feq > 0 for all i */
  double lo = -1e300, hi = 1e300;
  for (int i = 0; i < NQ; ++i) {
    double c0 = 1.0 + (dh[i] - (2.0 * beta - 1.0) * ds[i]) / feq[i];
    double c1 = -beta * dh[i] / feq[i];  /* argument = c0 + c1 * g */
    if (c1 > 0) { double g0 = -c0 / c1; if (g0 > lo) lo = g0; }
    else if (c1 < 0) { double g0 = -c0 / c1; if (g0 < hi) hi = g0; }
  }
  if (!(lo < hi)) return NAN;
  double a = lo, b = hi;
  if (a < -1e6) a = -1e6;
  if (b > 1e6) b = 1e6;
  /* shrink to the open interval */
  double span = b - a;
  a += 1e-12 * span; b -= 1e-12 * span;
  double Ga = 0, Gb = 0;
  for (int i = 0; i < NQ; ++i) {
    Ga += dh[i] * log(1.0 + ((1.0 - beta * a) * dh[i] - (2.0 * beta - 1.0) * ds[i]) / feq[i]);
    Gb += dh[i] * log(1.0 + ((1.0 - beta * b) * dh[i] - (2.0 * beta - 1.0) * ds[i]) / feq[i]);
  }
  if (!(Ga >= 0 && Gb <= 0)) return NAN;
  for (int it = 0; it < 400; ++it) {
    double m = 0.5 * (a + b);
    if (m == a || m == b) break;
    double G = 0;
    for (int i = 0; i < NQ; ++i)
      G += dh[i] * log(1.0 + ((1.0 - beta * m) * dh[i] - (2.0 * beta - 1.0) * ds[i]) / feq[i]);
    if (G > 0) a = m; else b = m;
  }
  return 0.5 * (a + b);
}

/* Discrete H-function H(f) = sum_i f_i ln(f_i / W_i) (eq. feq_min). */
double or_H(const double f[NQ]) {
  double H = 0;
  for (int i = 0; i < NQ; ++i) H += f[i] * log(f[i] / wgt(i));
  return H;
}

/* ------------------------------------------------------------------------ */
/* Grad's distribution (eq. grad):
 *   f*_i = W_i [rho + (rho/c_s^2) c_i.u + (1/(2 c_s^4)) (Pi - rho c_s^2 I):(c_i c_i - c_s^2 I)]. */
void or_grad_dist(double rho, const double u[3], const double Pi[9], double out[NQ]) {
  for (int i = 0; i < NQ; ++i) {
    double cu = 0, PQ = 0;
    for (int a = 0; a < 3; ++a) cu += ci(i, a) * u[a];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double d = (a == b) ? 1.0 : 0.0;
        PQ += (Pi[3 * a + b] - rho * CS2 * d) * (ci(i, a) * ci(i, b) - CS2 * d);
      }
    out[i] = wgt(i) * (rho + rho / CS2 * cu + PQ / (2.0 * CS2 * CS2));
  }
}

/* Pressure tensor (eqs. pressure, pressure2):
 *   Pi = rho c_s^2 I + rho u u - (rho c_s^2 / (2 beta)) (grad u + grad u^T),
 * with G[a][b] = d u_a / d x_b. */
void or_pressure(double rho, const double u[3], const double G[9], double beta, double Pi[9]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      Pi[3 * a + b] = rho * CS2 * (a == b ? 1.0 : 0.0) + rho * u[a] * u[b] -
                      rho * CS2 / (2.0 * beta) * (G[3 * a + b] + G[3 * b + a]);
}

/* ------------------------------------------------------------------------ */
/* Grid, bodies and kinematics.  Bodies and their prescribed motion are the
 * paper's "objects" (Sec. III); the kinematic law below is this library's
 * parametrisation of them:
 *   centre c(t)   = p0 + (amp sin(((2 pi) t) / period)) dir + vel t
 *   velocity U(t) = (amp ((2 pi) / period) cos(((2 pi) t) / period)) dir + vel
 *   wall velocity u_w(x) = U(t) + omega x (x - c(t)).
 * Every product and sum is evaluated in the order written, in FP64, so that a
 * second implementation following the same formula gets the same bits. */
typedef struct {
  int32_t nx, ny, nz;
  int32_t channel;   /* 0: periodic in x;  1: inlet at x = 0, outlet at x = nx-1 */
  double beta;
  double rho0;
  double u_in[3];
  int32_t stream_only; /* 1: skip the collision (streaming-permutation tests) */
  int32_t stabiliser;  /* 0: the analytic gamma of Sec. II; 1: the exact root of eq. gamma_min
                          (or_gamma_exact; the analytic one where no root is bracketed);
                          2: gamma = 2 (LBGK) */
  int32_t central;     /* 1: central-moment s (or_shear_part_central), with stabiliser 0 */
} or_grid;

typedef struct {
  int32_t kind;      /* 0: sphere, 1: half-space bounded by a plane, 2: closed triangulated
                        surface (the deforming bodies of Sec. IV.C) */
  int32_t tracked;   /* 1: centre and velocity come from the track below (a freely moving body
                        whose motion the caller integrates), not from the prescribed motion */
  double p0[3];      /* sphere centre, or a point of the plane, at t = 0 */
  double radius;
  double normal[3];  /* plane: unit normal pointing into the fluid */
  double amp, period;
  double dir[3];
  double vel[3];
  double omega[3];
  double track_t;         /* tracked: the time level t of track_c[0], track_U[0] */
  double track_c[2][3];   /* tracked: centre at t and t + 1 */
  double track_U[2][3];   /* tracked: translational velocity at t and t + 1 */
  /* kind 2: vertex positions and velocities [nv][3] at the time levels mesh_t (index 0) and
     mesh_t + 1 (index 1), triangles [nt][3] (vertex indices).  The centre used for the torque is
     the track (tracked = 1). */
  const double *mesh_X[2];
  const double *mesh_V[2];
  const int32_t *mesh_tri;
  int32_t mesh_nv, mesh_nt;
  double mesh_t;
  double track_W[2][3];   /* tracked: angular velocity at t and t + 1 (a freely rotating sphere) */
} or_body;

typedef struct {
  int64_t boundary_nodes, links, refill_nodes, gamma_guard;
  double gamma_min, gamma_max;
  int64_t exact_fallback;  /* stabiliser 1: nodes where no positive root was bracketed */
} or_stats;

void or_kinematics(const or_body *b, double t, double c[3], double U[3]) {
  if (b->tracked) {
    const int k = (t == b->track_t) ? 0 : ((t == b->track_t + 1.0) ? 1 : -1);
    for (int a = 0; a < 3; ++a) {
      c[a] = k >= 0 ? b->track_c[k][a] : NAN;
      U[a] = k >= 0 ? b->track_U[k][a] : NAN;
    }
    return;
  }
  double ph = 0.0, sn = 0.0, cs = 0.0, om = 0.0;
  if (b->period != 0.0) {
    ph = ((2.0 * M_PI) * t) / b->period;
    sn = sin(ph);
    cs = cos(ph);
    om = (2.0 * M_PI) / b->period;
  }
  for (int a = 0; a < 3; ++a) {
    c[a] = b->p0[a] + (b->amp * sn) * b->dir[a] + b->vel[a] * t;
    U[a] = (b->amp * om * cs) * b->dir[a] + b->vel[a];
  }
}

/* Angular velocity of body b at time t: the prescribed omega, or the track of a tracked body. */
static void body_omega(const or_body *b, double t, double W[3]) {
  if (b->tracked) {
    const int k = (t == b->track_t) ? 0 : ((t == b->track_t + 1.0) ? 1 : -1);
    for (int a = 0; a < 3; ++a) W[a] = k >= 0 ? b->track_W[k][a] : NAN;
    return;
  }
  for (int a = 0; a < 3; ++a) W[a] = b->omega[a];
}

/* Rigid-body velocity U + W x (x - c) at time t. */
static void rigid_velocity(const or_body *b, const double c[3], const double U[3], double t, const double x[3],
                           double out[3]) {
  double r[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
  double w[3];
  body_omega(b, t, w);
  out[0] = U[0] + (w[1] * r[2] - w[2] * r[1]);
  out[1] = U[1] + (w[2] * r[0] - w[0] * r[2]);
  out[2] = U[2] + (w[0] * r[1] - w[1] * r[0]);
}

/* Velocity of body b at the point x at time level t: rigid motion, or for a triangulated body the
 * velocity of the closest surface point. */
static int mesh_level(const or_body *b, double t);
void or_mesh_closest_velocity(const double *X, const double *V, const int32_t *tri, int nt, const double p[3],
                              double out[3], double *dist2);
static void body_velocity(const or_body *b, const double c[3], const double U[3], double t, const double x[3],
                          double out[3]) {
  if (b->kind == 2) {
    const int lv = mesh_level(b, t);
    out[0] = out[1] = out[2] = 0.0;
    if (lv >= 0) or_mesh_closest_velocity(b->mesh_X[lv], b->mesh_V[lv], b->mesh_tri, b->mesh_nt, x, out, 0);
    return;
  }
  rigid_velocity(b, c, U, t, x, out);
}


/* ------------------------------------------------------------------------ */
/* Triangulated bodies (Sec. IV.C: the swimmer is a triangulated surface; the wall velocity at
 * the link intersections is the barycentric interpolation of the vertex velocities).
 * Readings (the paper gives no algorithm for these):
 *  - inside: a node is solid iff a ray from it along +x crosses the surface an odd number of
 *    times.  A triangle is crossed iff the node's (y, z) lies in its projection onto the y-z
 *    plane; points on a projected edge or vertex belong to exactly one of the triangles sharing
 *    it (half-plane rule on the edge direction), so rays through edges and vertices count each
 *    surface crossing once; triangles with zero projected area are not crossed.  The crossing
 *    is at x_c = (w0 x_A + w1 x_B + w2 x_C) / (w0 + w1 + w2) with the projected edge functions
 *    w, and counts iff x_c > x.  FP64, operations in the written order, no fused multiply-add.
 *  - link fraction: q_i = the smallest s in (0, 1] at which the segment x_b - s c_i meets a
 *    triangle (ray-triangle intersection with barycentric coordinates u, v of the hit), the
 *    wall velocity (1 - u - v) V_A + u V_B + v V_C; where rounding lets the segment slip between
 *    triangles, q = 1/2 and the velocity of the surface point closest to x_b - c_i / 2.
 *  - velocity of the body at a node (solid nodes of U^t, refill): that of the closest surface
 *    point, barycentric in its triangle; ties go to the lowest triangle index. */
static double edge_fn(const double *a, const double *b, double py, double pz) {
  double l = (b[1] - a[1]) * (pz - a[2]);
  double r = (b[2] - a[2]) * (py - a[1]);
  return l - r;
}

/* half-plane rule: an edge a -> b of a positively oriented projected triangle owns the points on
 * it iff its direction has dz > 0, or dz = 0 and dy < 0 */
static int edge_owns(const double *a, const double *b) {
  double dy = b[1] - a[1], dz = b[2] - a[2];
  return dz > 0.0 || (dz == 0.0 && dy < 0.0);
}

int or_mesh_crossing(const double A[3], const double B0[3], const double C0[3], double y, double z, double *xc) {
  const double *B = B0, *C = C0;
  double area = edge_fn(A, B, C[1], C[2]);
  if (area == 0.0) return 0;
  if (area < 0.0) { B = C0; C = B0; }
  double w0 = edge_fn(B, C, y, z), w1 = edge_fn(C, A, y, z), w2 = edge_fn(A, B, y, z);
  if (w0 < 0.0 || (w0 == 0.0 && !edge_owns(B, C))) return 0;
  if (w1 < 0.0 || (w1 == 0.0 && !edge_owns(C, A))) return 0;
  if (w2 < 0.0 || (w2 == 0.0 && !edge_owns(A, B))) return 0;
  double num = w0 * A[0];
  num = num + w1 * B[0];
  num = num + w2 * C[0];
  double den = w0 + w1;
  den = den + w2;
  *xc = num / den;
  return 1;
}

int or_mesh_inside(const double *X, const int32_t *tri, int nt, double x, double y, double z) {
  int odd = 0;
  for (int k = 0; k < nt; ++k) {
    double xc;
    if (or_mesh_crossing(X + 3 * tri[3 * k], X + 3 * tri[3 * k + 1], X + 3 * tri[3 * k + 2], y, z, &xc) && xc > x)
      odd ^= 1;
  }
  return odd;
}

static void sub3(const double *a, const double *b, double *o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static double dot3(const double *a, const double *b) { double s = a[0] * b[0]; s = s + a[1] * b[1]; return s + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

/* Ray o + s d against triangle (A, B, C): returns 1 with s and the barycentric weights (u, v)
 * of B and C when the ray meets the triangle (u, v >= 0, u + v <= 1), via the solution of
 * o + s d = A + u (B - A) + v (C - A) by Cramer's rule with scalar triple products. */
int or_ray_triangle(const double o[3], const double d[3], const double *A, const double *B, const double *C,
                    double *s, double *u, double *v) {
  double e1[3], e2[3], p[3], tv[3], qv[3];
  sub3(B, A, e1);
  sub3(C, A, e2);
  cross3(d, e2, p);
  double det = dot3(e1, p);
  if (det == 0.0) return 0;
  double inv = 1.0 / det;
  sub3(o, A, tv);
  double uu = dot3(tv, p) * inv;
  if (uu < 0.0 || uu > 1.0) return 0;
  cross3(tv, e1, qv);
  double vv = dot3(d, qv) * inv;
  if (vv < 0.0 || uu + vv > 1.0) return 0;
  *s = dot3(e2, qv) * inv;
  *u = uu;
  *v = vv;
  return 1;
}

/* Closest point of triangle (A, B, C) to p: the orthogonal projection onto its plane when that
 * lies inside (barycentric weights from the 2x2 Gram system of the edges), else the closest point
 * on its three edges.  Returns the squared distance and the weights (wa, wb, wc). */
double or_closest_on_triangle(const double p[3], const double *A, const double *B, const double *C, double w[3]) {
  double e1[3], e2[3], ap[3];
  sub3(B, A, e1);
  sub3(C, A, e2);
  sub3(p, A, ap);
  double d00 = dot3(e1, e1), d01 = dot3(e1, e2), d11 = dot3(e2, e2);
  double d20 = dot3(ap, e1), d21 = dot3(ap, e2);
  double den = d00 * d11 - d01 * d01;
  if (den > 0.0) {
    double lb = (d11 * d20 - d01 * d21) / den;
    double lc = (d00 * d21 - d01 * d20) / den;
    double la = 1.0 - lb - lc;
    if (la >= 0.0 && lb >= 0.0 && lc >= 0.0) {
      double q[3], r[3];
      for (int a = 0; a < 3; ++a) q[a] = A[a] + lb * e1[a] + lc * e2[a];
      sub3(p, q, r);
      w[0] = la; w[1] = lb; w[2] = lc;
      return dot3(r, r);
    }
  }
  /* edges P0 -> P1 with the weight indices of their end points */
  const double *P[3][2] = {{A, B}, {B, C}, {C, A}};
  const int idx[3][2] = {{0, 1}, {1, 2}, {2, 0}};
  double best = INFINITY;
  for (int e = 0; e < 3; ++e) {
    double d[3], r0[3];
    sub3(P[e][1], P[e][0], d);
    sub3(p, P[e][0], r0);
    double dd = dot3(d, d);
    double tau = dd > 0.0 ? dot3(r0, d) / dd : 0.0;
    if (tau < 0.0) tau = 0.0;
    if (tau > 1.0) tau = 1.0;
    double q[3], r[3];
    for (int a = 0; a < 3; ++a) q[a] = P[e][0][a] + tau * d[a];
    sub3(p, q, r);
    double d2 = dot3(r, r);
    if (d2 < best) {
      best = d2;
      w[0] = w[1] = w[2] = 0.0;
      w[idx[e][0]] = 1.0 - tau;
      w[idx[e][1]] = tau;
    }
  }
  return best;
}

static void bary_velocity(const double *V, const int32_t *t3, const double w[3], double out[3]) {
  const double *va = V + 3 * t3[0], *vb = V + 3 * t3[1], *vc = V + 3 * t3[2];
  for (int a = 0; a < 3; ++a) {
    double s = w[0] * va[a];
    s = s + w[1] * vb[a];
    out[a] = s + w[2] * vc[a];
  }
}

/* Velocity of the surface point closest to p (lowest triangle index among equals). */
void or_mesh_closest_velocity(const double *X, const double *V, const int32_t *tri, int nt, const double p[3],
                              double out[3], double *dist2) {
  double best = INFINITY, bw[3] = {1.0, 0.0, 0.0};
  int bk = 0;
  for (int k = 0; k < nt; ++k) {
    double w[3];
    const int32_t *t3 = tri + 3 * k;
    double d2 = or_closest_on_triangle(p, X + 3 * t3[0], X + 3 * t3[1], X + 3 * t3[2], w);
    if (d2 < best) { best = d2; bk = k; bw[0] = w[0]; bw[1] = w[1]; bw[2] = w[2]; }
  }
  if (nt > 0) bary_velocity(V, tri + 3 * bk, bw, out);
  else out[0] = out[1] = out[2] = 0.0;
  if (dist2) *dist2 = best;
}

/* Link of the fluid node xb in direction i against the surface: returns 1 with q and the wall
 * velocity for a hit in (0, 1], else 0 with the fallback values. */
int or_mesh_link(const double *X, const double *V, const int32_t *tri, int nt, const double xb[3], int i, double *q,
                 double uw[3]) {
  double d[3] = {-(double)cxi(i), -(double)cyi(i), -(double)czi(i)};
  double best = INFINITY, bu = 0.0, bv = 0.0;
  int bk = -1;
  for (int k = 0; k < nt; ++k) {
    const int32_t *t3 = tri + 3 * k;
    double s, u, v;
    if (!or_ray_triangle(xb, d, X + 3 * t3[0], X + 3 * t3[1], X + 3 * t3[2], &s, &u, &v)) continue;
    if (!(s > 0.0 && s <= 1.0)) continue;
    if (s < best) { best = s; bk = k; bu = u; bv = v; }
  }
  if (bk >= 0) {
    double w[3] = {1.0 - bu - bv, bu, bv};
    *q = best;
    bary_velocity(V, tri + 3 * bk, w, uw);
    return 1;
  }
  double mid[3] = {xb[0] + 0.5 * d[0], xb[1] + 0.5 * d[1], xb[2] + 0.5 * d[2]};
  *q = 0.5;
  or_mesh_closest_velocity(X, V, tri, nt, mid, uw, 0);
  return 0;
}

static int mesh_level(const or_body *b, double t) {
  return t == b->mesh_t ? 0 : (t == b->mesh_t + 1.0 ? 1 : -1);
}

/* Inside test.  Reading: a node is solid iff it lies strictly inside the body:
 * |x - c|^2 < R^2 for a sphere, n.(x - c) < 0 for a plane, both evaluated in
 * FP64 with the operations in the order written and no fused multiply-add. */
static int inside(const or_body *b, const double c[3], double t, double x, double y, double z) {
  if (b->kind == 2) {
    const int lv = mesh_level(b, t);
    return lv >= 0 && or_mesh_inside(b->mesh_X[lv], b->mesh_tri, b->mesh_nt, x, y, z);
  }
  if (b->kind == 0) {
    double dx = x - c[0], dy = y - c[1], dz = z - c[2];
    double d2 = dx * dx;
    d2 = d2 + dy * dy;
    d2 = d2 + dz * dz;
    double r2 = b->radius * b->radius;
    return d2 < r2;
  }
  double s = b->normal[0] * (x - c[0]);
  s = s + b->normal[1] * (y - c[1]);
  s = s + b->normal[2] * (z - c[2]);
  return s < 0.0;
}

/* Solid mask at time t: out[n] = 0 for fluid, else 1 + index of the first body
 * (in the given order) containing node n. */
void or_solid_mask(const or_grid *g, const or_body *bodies, int nb, double t, uint8_t *out) {
  double c[MAXB][3], U[3];
  for (int k = 0; k < nb; ++k) or_kinematics(&bodies[k], t, c[k], U);
  long N = (long)g->nx * g->ny * g->nz;
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; ++n) {
    int x = (int)(n % g->nx), y = (int)((n / g->nx) % g->ny), z = (int)(n / ((long)g->nx * g->ny));
    uint8_t v = 0;
    for (int k = 0; k < nb && !v; ++k)
      if (inside(&bodies[k], c[k], t, x, y, z)) v = (uint8_t)(k + 1);
    out[n] = v;
  }
}

/* Wall distance fraction along a boundary link (Sec. III):
 * q_i = |x_b - x_w,i| / |c_i|, where x_w,i is where the segment from the fluid
 * node x_b towards x_b - c_i first meets the body surface.  With s the ray
 * parameter (x_w = x_b - s c_i), q_i = s.  Sphere: smallest root of
 * |x_b - s c_i - c|^2 = R^2, written as (|d|^2 - R^2) / (d.c_i + sqrt(disc)),
 * d = x_b - c, disc = (d.c_i)^2 - |c_i|^2 (|d|^2 - R^2).  Plane: s =
 * n.(x_b - c) / n.c_i.  No clamping (a frozen-topology run may move the
 * surface slightly past the node; a negative discriminant is taken as 0). */
double or_q(const or_body *b, const double c[3], const double xb[3], int i) {
  if (b->kind == 2) {  /* the later of the two time levels, as the step uses it */
    double q = 0.5, uw[3];
    or_mesh_link(b->mesh_X[1], b->mesh_V[1], b->mesh_tri, b->mesh_nt, xb, i, &q, uw);
    return q;
  }
  double v[3] = {cxi(i), cyi(i), czi(i)};
  double d[3] = {xb[0] - c[0], xb[1] - c[1], xb[2] - c[2]};
  if (b->kind == 0) {
    double dv = d[0] * v[0] + d[1] * v[1] + d[2] * v[2];
    double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] - b->radius * b->radius;
    double disc = dv * dv - vv * dd;
    if (disc < 0) disc = 0;
    return dd / (dv + sqrt(disc));
  }
  double nd = b->normal[0] * d[0] + b->normal[1] * d[1] + b->normal[2] * d[2];
  double nv = b->normal[0] * v[0] + b->normal[1] * v[1] + b->normal[2] * v[2];
  return nd / nv;
}

/* ------------------------------------------------------------------------ */
/* Neighbour lookup: periodic wrap on periodic axes; in channel mode x is not
 * periodic and a neighbour outside [0, nx) does not exist (returns -1). */
static long nbr(const or_grid *g, int x, int y, int z, int dx, int dy, int dz) {
  int X = x + dx, Y = y + dy, Z = z + dz;
  if (g->channel) {
    if (X < 0 || X >= g->nx) return -1;
  } else {
    X = ((X % g->nx) + g->nx) % g->nx;
  }
  Y = ((Y % g->ny) + g->ny) % g->ny;
  Z = ((Z % g->nz) + g->nz) % g->nz;
  return ((long)Z * g->ny + Y) * g->nx + X;
}

/* Velocity gradient by finite differences on the previous-step velocity field
 * U^t (Sec. III).  Reading (the paper names no stencil): per axis, using only
 * stencil nodes that exist and are fluid at t+1 ("usable"):
 *   both neighbours usable           -> central      (u+1 - u-1) / 2
 *   two nodes usable on one side     -> one-sided    (-3 u0 + 4 u1 - u2) / 2 (sign by side)
 *   one node usable on one side      -> one-sided    u1 - u0  (sign by side)
 *   none                             -> 0.
 * The forward side is tried before the backward side.  G[3a+b] = d u_a / d x_b. */
void or_grad_u(const or_grid *g, const double *U, const uint8_t *solid_t1, int x, int y, int z, double G[9]) {
  long N = (long)g->nx * g->ny * g->nz;
  long n0 = ((long)z * g->ny + y) * g->nx + x;
  for (int b = 0; b < 3; ++b) {
    int e[3] = {0, 0, 0};
    long p[3], m[3];  /* p[k]: node at +k (k = 1, 2), m[k]: node at -k */
    int okp[3], okm[3];
    for (int k = 1; k <= 2; ++k) {
      e[b] = k;
      p[k] = nbr(g, x, y, z, e[0], e[1], e[2]);
      e[b] = -k;
      m[k] = nbr(g, x, y, z, e[0], e[1], e[2]);
      e[b] = 0;
      okp[k] = p[k] >= 0 && !solid_t1[p[k]];
      okm[k] = m[k] >= 0 && !solid_t1[m[k]];
    }
    for (int a = 0; a < 3; ++a) {
      const double *Ua = U + a * N;
      double d;
      if (okp[1] && okm[1]) d = 0.5 * (Ua[p[1]] - Ua[m[1]]);
      else if (okp[1] && okp[2]) d = 0.5 * (-3.0 * Ua[n0] + 4.0 * Ua[p[1]] - Ua[p[2]]);
      else if (okm[1] && okm[2]) d = 0.5 * (3.0 * Ua[n0] - 4.0 * Ua[m[1]] + Ua[m[2]]);
      else if (okp[1]) d = Ua[p[1]] - Ua[n0];
      else if (okm[1]) d = Ua[n0] - Ua[m[1]];
      else d = 0.0;
      G[3 * a + b] = d;
    }
  }
}

/* Macroscopic fields of the previous step, U^t and R^t (Sec. III: "the velocity
 * values from the previous time step").  Reading: for a node fluid at t they
 * are the moments of its stored post-collision populations A^t, with the
 * velocity shifted back by half the body force, U = (j - F/2)/rho; for a node
 * solid at t, U^t is the rigid-body velocity there and R^t = rho0. */
void or_macro(const or_grid *g, const or_body *bodies, int nb, double t, const double *A, const uint8_t *solid_t,
              const double *F, double *U, double *R) {
  long N = (long)g->nx * g->ny * g->nz;
  double c[MAXB][3], Ub[MAXB][3];
  for (int k = 0; k < nb; ++k) or_kinematics(&bodies[k], t, c[k], Ub[k]);
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; ++n) {
    if (solid_t[n]) {
      int k = solid_t[n] - 1;
      double xp[3] = {(double)(n % g->nx), (double)((n / g->nx) % g->ny), (double)(n / ((long)g->nx * g->ny))};
      double v[3];
      body_velocity(&bodies[k], c[k], Ub[k], t, xp, v);
      for (int a = 0; a < 3; ++a) U[a * N + n] = v[a];
      R[n] = g->rho0;
      continue;
    }
    double f[NQ];
    for (int i = 0; i < NQ; ++i) f[i] = A[i * N + n];
    double rho = moment(f, 0, 0, 0);
    double j[3] = {moment(f, 1, 0, 0), moment(f, 0, 1, 0), moment(f, 0, 0, 1)};
    for (int a = 0; a < 3; ++a) {
      double Fa = F ? F[a * N + n] : 0.0;
      U[a * N + n] = (j[a] - 0.5 * Fa) / rho;
    }
    R[n] = rho;
  }
}

/* ------------------------------------------------------------------------ */
/* Refill of uncovered nodes (Sec. III): a node solid at t and fluid at t+1 has no
 * populations of its own.  It receives Grad's distribution with the wall velocity at the node, a
 * local density average and the pressure tensor of eqs. pressure/pressure2.
 * Readings: the refill takes place before streaming, so the refilled populations are the node's
 * state at t -- its neighbours pull them and the node itself then streams, meets the wall and
 * collides like any other fluid node; the density average is over the 26 neighbours fluid at both
 * t and t+1 (rho0 if none); the body is the one that held the node at t, its velocity taken at t+1;
 * the gradient is the finite difference of U^t at the node.
 * Writes A_w = A_t with the refill nodes replaced; U, R are U^t, R^t of or_macro. */
void or_refill_state(const or_grid *g, const or_body *bodies, int nb, double t, const double *A_t,
                     const uint8_t *solid_t, const uint8_t *solid_t1, const double *U, const double *R,
                     double *A_w, int64_t *count) {
  const long N = (long)g->nx * g->ny * g->nz;
  double c1[MAXB][3], U1[MAXB][3];
  for (int k = 0; k < nb; ++k) or_kinematics(&bodies[k], t + 1.0, c1[k], U1[k]);
  memcpy(A_w, A_t, sizeof(double) * NQ * N);
  int64_t cnt = 0;
#pragma omp parallel for schedule(static) reduction(+ : cnt)
  for (long n = 0; n < N; ++n) {
    if (!(solid_t[n] && !solid_t1[n])) continue;
    const int x = (int)(n % g->nx), y = (int)((n / g->nx) % g->ny), z = (int)(n / ((long)g->nx * g->ny));
    const double xb[3] = {x, y, z};
    const int k = solid_t[n] - 1;
    double uw[3];
    body_velocity(&bodies[k], c1[k], U1[k], t + 1.0, xb, uw);
    double rs = 0.0;
    int m = 0;
    for (int i = 0; i < NQ; ++i) {
      if (i == 13) continue;
      long nn = nbr(g, x, y, z, cxi(i), cyi(i), czi(i));
      if (nn < 0 || solid_t[nn] || solid_t1[nn]) continue;
      rs += R[nn];
      ++m;
    }
    double rho_avg = m ? rs / m : g->rho0;
    double G[9], Pi[9], f[NQ];
    or_grad_u(g, U, solid_t1, x, y, z, G);
    or_pressure(rho_avg, uw, G, g->beta, Pi);
    or_grad_dist(rho_avg, uw, Pi, f);
    for (int i = 0; i < NQ; ++i) A_w[i * N + n] = f[i];
    ++cnt;
  }
  if (count) *count = cnt;
}

/* ------------------------------------------------------------------------ */
/* One time step t -> t+1 (Secs. II and III).
 *   A_t     : post-collision populations at t (27 N)
 *   solid_t : solid mask at t, solid_t1 : solid mask at t+1 (or_solid_mask)
 *   F       : body-force field (3 N, component-major) or NULL
 *   A_t1    : output populations at t+1 (27 N).  Solid nodes keep A_t.
 *   forces  : output, per body 6 doubles (force[3], torque[3]) of the links
 *             used while producing A_t1
 * First the nodes uncovered by the bodies are refilled (or_refill_state), then for
 * each node fluid at t+1:
 *  - pull streaming f_i = A_t,i(x - c_i) for the populations whose
 *    source exists and is fluid at t+1.  The others form the missing set Dbar
 *    (reading: streamed from a node solid at t+1, or through the inlet face)
 *    and are rebuilt with Grad's distribution at target values (Sec. III):
 *      u_tgt = (1/n) sum_Dbar (q_i u_f,i + u_w,i) / (1 + q_i)
 *      rho_tgt = sum_Dbar f_i^bb + sum_notDbar f_i + sum_Dbar 6 W_i rho0 c_i.u_w,i
 *    with f_i^bb = A_t at x in the opposite direction, u_f,i = U^t(x + c_i)
 *    (reading: u_w,i if that node is not fluid at t+1), Pi from eqs.
 *    pressure/pressure2 at (rho_tgt, u_tgt) with the finite-difference
 *    gradient above.  Only the Dbar populations are replaced.
 *    Momentum exchange (Sec. IV.A, Galilean-invariant form; reading of the
 *    cited formula): per link dF = A_t,ibar(x) (c_ibar - u_w) - f*_i (c_i - u_w),
 *    torque (x_w - c) x dF, summed per body.
 *  - then the KBC collision (with the body force if F != NULL).
 * Channel mode (an addition of this library, not from the paper): the inlet
 * face x = 0 is a moving wall at x = -1/2 (q = 1/2) with velocity u_in, not
 * counted in any body force; the outlet x = nx-1 takes its missing
 * populations (c_x = -1) from its own column, i.e. the value streamed into
 * the upstream neighbour (zero-gradient copy). */
int or_step(const or_grid *g, const or_body *bodies, int nb, double t, const double *A_t,
            const uint8_t *solid_t, const uint8_t *solid_t1, const double *F, double *A_t1,
            double *forces, or_stats *st) {
  if (nb > MAXB) return -1;
  const long N = (long)g->nx * g->ny * g->nz;
  const double beta = g->beta;
  double *U = (double *)malloc(sizeof(double) * 3 * N);
  double *R = (double *)malloc(sizeof(double) * N);
  double *fz = (double *)calloc((size_t)g->nz * MAXB * 6, sizeof(double));
  int64_t *cnt = (int64_t *)calloc((size_t)g->nz * 4, sizeof(int64_t));
  double *gmin = (double *)malloc(sizeof(double) * g->nz), *gmax = (double *)malloc(sizeof(double) * g->nz);
  if (!U || !R || !fz || !cnt || !gmin || !gmax) return -2;
  or_macro(g, bodies, nb, t, A_t, solid_t, F, U, R);
  double *Aw = (double *)malloc(sizeof(double) * NQ * N);
  if (!Aw) return -2;
  int64_t nrefill = 0;
  or_refill_state(g, bodies, nb, t, A_t, solid_t, solid_t1, U, R, Aw, &nrefill);
  double c1[MAXB][3], U1[MAXB][3];
  for (int k = 0; k < nb; ++k) or_kinematics(&bodies[k], t + 1.0, c1[k], U1[k]);

#pragma omp parallel for schedule(static)
  for (int z = 0; z < g->nz; ++z) {
    gmin[z] = 1e300; gmax[z] = -1e300;
    for (int y = 0; y < g->ny; ++y)
      for (int x = 0; x < g->nx; ++x) {
        long n = ((long)z * g->ny + y) * g->nx + x;
        if (solid_t1[n]) {
          for (int i = 0; i < NQ; ++i) A_t1[i * N + n] = A_t[i * N + n];
          continue;
        }
        double xb[3] = {x, y, z};
        double f[NQ];
        {
          int inD[NQ], bodyof[NQ];
          double q[NQ], uwm[NQ][3];  /* uwm: wall velocity of links into a triangulated body */
          int nD = 0;
          for (int i = 0; i < NQ; ++i) {
            inD[i] = 0; bodyof[i] = -1; q[i] = 0;
            int sx = x - cxi(i);
            if (g->channel && sx < 0) {            /* through the inlet face */
              inD[i] = 1; bodyof[i] = -1; q[i] = (xb[0] + 0.5) / cxi(i);
              ++nD;
              continue;
            }
            long src;
            if (g->channel) {
              if (sx >= g->nx) sx = g->nx - 1;               /* outlet copy */
              src = nbr(g, sx, y, z, 0, -cyi(i), -czi(i));
            } else {
              src = nbr(g, x, y, z, -cxi(i), -cyi(i), -czi(i));
            }
            if (solid_t1[src]) {
              inD[i] = 1; bodyof[i] = solid_t1[src] - 1;
              const or_body *bb = &bodies[bodyof[i]];
              if (bb->kind == 2) {
                const int lv = mesh_level(bb, t + 1.0);
                q[i] = 0.5;
                uwm[i][0] = uwm[i][1] = uwm[i][2] = 0.0;
                if (lv >= 0) or_mesh_link(bb->mesh_X[lv], bb->mesh_V[lv], bb->mesh_tri, bb->mesh_nt, xb, i, &q[i], uwm[i]);
              } else {
                q[i] = or_q(bb, c1[bodyof[i]], xb, i);
              }
              ++nD;
              continue;
            }
            f[i] = Aw[i * N + src];
          }
          if (nD) {
            double uw[NQ][3], ut[3] = {0, 0, 0}, rstat = 0, rdyn = 0;
            for (int i = 0; i < NQ; ++i) {
              if (!inD[i]) { rstat += f[i]; continue; }
              rstat += Aw[opp(i) * N + n];
              if (bodyof[i] < 0) {
                for (int a = 0; a < 3; ++a) uw[i][a] = g->u_in[a];
              } else if (bodies[bodyof[i]].kind == 2) {
                for (int a = 0; a < 3; ++a) uw[i][a] = uwm[i][a];
              } else {
                double xw[3] = {xb[0] - q[i] * cxi(i), xb[1] - q[i] * cyi(i), xb[2] - q[i] * czi(i)};
                rigid_velocity(&bodies[bodyof[i]], c1[bodyof[i]], U1[bodyof[i]], t + 1.0, xw, uw[i]);
              }
              double uf[3];
              long nf = nbr(g, x, y, z, cxi(i), cyi(i), czi(i));
              if (nf >= 0 && !solid_t1[nf]) {
                for (int a = 0; a < 3; ++a) uf[a] = U[a * N + nf];
              } else {
                for (int a = 0; a < 3; ++a) uf[a] = uw[i][a];
              }
              for (int a = 0; a < 3; ++a) ut[a] += (q[i] * uf[a] + uw[i][a]) / (1.0 + q[i]);
              rdyn += 6.0 * wgt(i) * g->rho0 * (cxi(i) * uw[i][0] + cyi(i) * uw[i][1] + czi(i) * uw[i][2]);
            }
            for (int a = 0; a < 3; ++a) ut[a] /= nD;
            double rtgt = rstat + rdyn;
            double G[9], Pi[9], fs[NQ];
            or_grad_u(g, U, solid_t1, x, y, z, G);
            or_pressure(rtgt, ut, G, beta, Pi);
            or_grad_dist(rtgt, ut, Pi, fs);
            for (int i = 0; i < NQ; ++i) {
              if (!inD[i]) continue;
              f[i] = fs[i];
              int k = bodyof[i];
              cnt[4 * z + 1]++;
              if (k < 0) continue;
              double fo = Aw[opp(i) * N + n];
              double dF[3], xw[3];
              for (int a = 0; a < 3; ++a) {
                dF[a] = fo * (-ci(i, a) - uw[i][a]) - fs[i] * (ci(i, a) - uw[i][a]);
                xw[a] = xb[a] - q[i] * ci(i, a) - c1[k][a];
              }
              double *acc = fz + ((size_t)z * MAXB + k) * 6;
              for (int a = 0; a < 3; ++a) acc[a] += dF[a];
              acc[3] += xw[1] * dF[2] - xw[2] * dF[1];
              acc[4] += xw[2] * dF[0] - xw[0] * dF[2];
              acc[5] += xw[0] * dF[1] - xw[1] * dF[0];
            }
            cnt[4 * z + 0]++;
          }
        }
        double Fn[3];
        if (F) for (int a = 0; a < 3; ++a) Fn[a] = F[a * N + n];
        int guard = 0;
        double gam = 2.0;
        if (!g->stream_only) {
          double gfix = 0.0;
          if (g->stabiliser == 2) gfix = 2.0;
          if (g->stabiliser == 1) {
            const double ge = or_gamma_exact(f, beta);
            if (isfinite(ge) && ge > 0.0) gfix = ge;
            else cnt[4 * z + 2]++;
          }
          gam = g->central ? or_collide_central(f, beta, F ? Fn : 0, gfix, &guard)
                           : or_collide_ex(f, beta, F ? Fn : 0, gfix, &guard);
        }
        cnt[4 * z + 3] += guard;
        if (gam < gmin[z]) gmin[z] = gam;
        if (gam > gmax[z]) gmax[z] = gam;
        for (int i = 0; i < NQ; ++i) A_t1[i * N + n] = f[i];
      }
  }
  for (int k = 0; k < nb; ++k)
    for (int c = 0; c < 6; ++c) {
      double s = 0;
      for (int z = 0; z < g->nz; ++z) s += fz[((size_t)z * MAXB + k) * 6 + c];
      forces[6 * k + c] = s;
    }
  if (st) {
    memset(st, 0, sizeof *st);
    st->gamma_min = 1e300; st->gamma_max = -1e300;
    for (int z = 0; z < g->nz; ++z) {
      st->boundary_nodes += cnt[4 * z]; st->links += cnt[4 * z + 1];
      st->gamma_guard += cnt[4 * z + 3];
      st->exact_fallback += cnt[4 * z + 2];
      if (gmin[z] < st->gamma_min) st->gamma_min = gmin[z];
      if (gmax[z] > st->gamma_max) st->gamma_max = gmax[z];
    }
    st->refill_nodes = nrefill;
  }
  free(Aw); free(U); free(R); free(fz); free(cnt); free(gmin); free(gmax);
  return 0;
}

/* Initial state A^0 = feq(rho, u) at every node (an equilibrium state is left
 * unchanged by the collision, so it is a valid post-collision state).
 * rho may be NULL (rho = 1 everywhere); u is 3 N, component-major. */
void or_init_equilibrium(long N, const double *rho, const double *u, double *A) {
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; ++n) {
    double uu[3] = {u[n], u[N + n], u[2 * N + n]}, feq[NQ];
    or_feq(rho ? rho[n] : 1.0, uu, feq);
    for (int i = 0; i < NQ; ++i) A[i * N + n] = feq[i];
  }
}

/* Moments of every node of a population field: rho (N) and j (3 N). */
void or_moments(long N, const double *A, double *rho, double *j) {
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; ++n) {
    double f[NQ];
    for (int i = 0; i < NQ; ++i) f[i] = A[i * N + n];
    rho[n] = moment(f, 0, 0, 0);
    j[n] = moment(f, 1, 0, 0);
    j[N + n] = moment(f, 0, 1, 0);
    j[2 * N + n] = moment(f, 0, 0, 1);
  }
}

int or_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
