/*
 * elbm.h -- C ABI of the MI355X (gfx950) entropic lattice Boltzmann library.
 *
 * The library advances the D3Q27 entropic multi-relaxation-time (KBC) lattice
 * Boltzmann method with moving-wall Grad boundary conditions of Dorschner,
 * Chikatamarla and Karlin (arXiv:1608.04658): pull streaming, moments,
 * entropic equilibrium, KBC collision with a per-node stabiliser gamma (Sec. II,
 * eqs. kineticEq, kbc_relax, feq_min), reconstruction of the missing populations
 * at moving walls with Grad's distribution and refill of uncovered nodes
 * (Sec. III, eqs. grad, pressure, pressure2), and the momentum-exchange force on
 * each body (Sec. IV.A).
 *
 * Conventions shared by every entry point
 *  - Return value: ELBM_OK (0) or a negative ELBM_E* code.  No exception crosses
 *    the ABI.  elbm_last_error() describes the last failure of a context.
 *  - Memory: the caller owns all device memory.  elbm_workspace_bytes() sizes
 *    one device buffer that the caller allocates (256-byte aligned) and hands
 *    to elbm_create(); the library carves its fields out of it and never calls
 *    hipMalloc or hipFree.  Host memory passed in is only read or written during
 *    the call.  "dev" pointers are device pointers, "host" pointers host ones.
 *  - Streams: every kernel is enqueued on the stream given to elbm_create()
 *    (or elbm_set_stream()).  Calls return without waiting for the GPU unless
 *    stated ("synchronises").
 *  - Layout: N = nx*ny*nz nodes, node n = (z*ny + y)*nx + x (x fastest).
 *    Population arrays exchanged through the ABI (FP64 reads and writes,
 *    adjoint fields) are structure-of-arrays [27][N]; the storage arrays
 *    inside the workspace follow elbm_info.layout.  Velocity i has
 *    c_i = (i%3 - 1, (i/3)%3 - 1, i/9 - 1), so the opposite of i is 26 - i.
 *    Vector fields are [3][N].
 *  - One context per host thread at a time; contexts are independent.
 */
#ifndef ELBM_H
#define ELBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ELBM_OK 0
#define ELBM_EINVAL (-1)     /* bad argument */
#define ELBM_ENOSPACE (-2)   /* workspace too small, or a device list overflowed */
#define ELBM_EDEVICE (-3)    /* a HIP call failed */
#define ELBM_ESTATE (-4)     /* call not valid in the context's current state */
#define ELBM_ENONFINITE (-5) /* a collided node had a non-finite state, or one where the entropic
                                equilibrium is not positive (rho <= 0 or some |u_a| >= 1, where an
                                feq_i <= 0 and the entropic scalar product is undefined) */

/* storage of the populations in HBM */
#define ELBM_STORAGE_F32 0   /* d_i = f_i - W_i as binary32 */
#define ELBM_STORAGE_F16 1   /* d_i = f_i - W_i as binary16 (round to nearest even) */
#define ELBM_STORAGE_BF16 2  /* d_i = f_i - W_i as bfloat16 (round to nearest even) */

/* placement of the 27 N elements of a population array in the workspace (elbm_info.layout; the
 * same for both time levels and for elbm_save_state).  This version stores every format as
 * ELBM_LAYOUT_ROWS; ELBM_LAYOUT_SOA names the plain form for readers of raw checkpoints. */
#define ELBM_LAYOUT_SOA 0    /* [27][nz][ny][nx] */
#define ELBM_LAYOUT_ROWS 1   /* [nz][ny][27][nx]: the 27 directions of each lattice row together */

/* x-direction boundary (y and z are always periodic) */
#define ELBM_BC_PERIODIC 0
#define ELBM_BC_CHANNEL 1    /* inlet at x = 0 (moving wall at x = -1/2 with velocity u_inlet,
                                link fraction 1/2, not counted as a body); outlet at x = nx-1
                                (a population entering from x = nx takes the value streamed into
                                x = nx-2 in the same direction) */

#define ELBM_BODY_SPHERE 0
#define ELBM_BODY_PLANE 1    /* solid half-space n.(x - c) < 0, normal pointing into the fluid */
#define ELBM_BODY_MESH 2     /* closed triangulated surface set by elbm_set_mesh (at most one per
                                context, last in the body array; see elbm_set_mesh) */

#define ELBM_MAX_BODIES 8

/* elbm_params.flags */
#define ELBM_FLAG_BODY_FORCE 1u   /* a per-node body-force field will be bound */
#define ELBM_FLAG_STREAM_ONLY 2u  /* no collision: the step is the streaming permutation alone */
#define ELBM_FLAG_NO_FP64 4u      /* disable the FP64 recomputation of near-equilibrium nodes */
#define ELBM_FLAG_ADJOINT 8u      /* reserve workspace for elbm_adjoint_step */
#define ELBM_FLAG_EXACT_GAMMA 16u /* stabiliser = the exact root of eq. gamma_min (Newton from the
                                     analytic value) instead of the paper's analytic approximation;
                                     not with ELBM_FLAG_ADJOINT */
#define ELBM_FLAG_LBGK 32u        /* stabiliser gamma = 2 (plain LBGK), for comparisons */
#define ELBM_FLAG_CENTRAL 64u     /* central-moment member of the KBC family: the shear part s is
                                     rebuilt from the deviatoric second moments through the dual
                                     basis of the velocities c - u shifted by the node's velocity
                                     (at u = 0 the raw basis of the paper); with the analytic
                                     stabiliser only, not with ELBM_FLAG_ADJOINT */

typedef struct elbm_params {
  int32_t nx, ny, nz;   /* lattice size, each >= 1 (channel mode: nx >= 4), N < 2^31 */
  int32_t storage;      /* ELBM_STORAGE_* */
  int32_t bc_x;         /* ELBM_BC_* */
  int32_t max_bodies;   /* 0 .. ELBM_MAX_BODIES; 0 = no geometry at all */
  uint32_t flags;       /* ELBM_FLAG_* */
  int32_t force_ring;   /* per-step force records kept on the device (>= 1 if max_bodies > 0) */
  int64_t max_boundary; /* capacity of the boundary-node list; 0 = library default */
  double nu;            /* kinematic viscosity; beta = 1/(6 nu + 1) (Sec. II, Chapman-Enskog) */
  double rho0;          /* reference density of the displacement term of Sec. III (1.0) */
  double u_inlet[3];    /* ELBM_BC_CHANNEL inlet velocity */
  double fp64_threshold;/* nodes with <dh|dh> < thr*rho and <ds|ds> >= thr*rho get the
                           collision recomputed in FP64; 0 = 1e-12 */
  int32_t max_mesh_vertices;  /* capacity for one triangulated body (0 = none) */
  int32_t max_mesh_triangles;
} elbm_params;

/* A rigid body with prescribed motion (Sec. III).  Every quantity is evaluated
 * in FP64 in the order written:
 *   centre   c(t) = center + (amp * sin(((2*pi)*t)/period)) * dir + vel * t
 *   velocity U(t) = (amp * ((2*pi)/period) * cos(((2*pi)*t)/period)) * dir + vel
 *   wall velocity at a point x: U(t) + omega x (x - c(t))
 * (period = 0 means no oscillation).  A node x is solid at t iff it lies strictly
 * inside: |x - c|^2 < radius^2 (sphere, squares and sums left to right, no fused
 * multiply-add) or n.(x - c) < 0 (plane).  The first body in the array that
 * contains a node owns it. */
/* Free motion (two-way coupling; Newton's equations of the settling-sphere case of Sec. IV.A):
 * a sphere with motion = ELBM_MOTION_FREE is moved by the momentum-exchange force F, gravity
 * and buoyancy, integrated with explicit Euler and unit time step,
 *   x(t+1) = x(t) + u(t),   u(t+1) = u(t) + F(t)/m + (1 - 1/density_ratio) g,
 *   m = density_ratio * rho0 * (4/3) pi radius^3,
 * where F(t) is the force of the step that produced time level t (zero at the time level at
 * which the geometry is set).  center and vel are the position and velocity at the current
 * time level; amp and period must be 0, and omega too unless the sphere rotates freely.
 * With motion = ELBM_MOTION_FREE_ROTATING the torque M about the centre (of the same step) also
 * turns the sphere:  w(t+1) = w(t) + M(t)/I,  I = (2/5) m radius^2 (solid sphere), omega being
 * w at the current time level; the wall velocity is u + w x (x - c).  The integration runs on the
 * device after each step; the host reads the state one step behind (no step waits for the
 * previous one to end).  A free sphere must stay at least 3 nodes inside every face (6 from the
 * inlet and outlet in channel mode); a step that would take it closer fails with ELBM_ESTATE.
 * Not available with ELBM_FLAG_ADJOINT. */
#define ELBM_MOTION_PRESCRIBED 0
#define ELBM_MOTION_FREE 1
#define ELBM_MOTION_FREE_ROTATING 2

typedef struct elbm_body {
  int32_t kind;         /* ELBM_BODY_* */
  int32_t motion;       /* ELBM_MOTION_PRESCRIBED or ELBM_MOTION_FREE */
  double center[3];
  double radius;
  double normal[3];     /* plane only: unit normal into the fluid */
  double amp;
  double period;
  double dir[3];
  double vel[3];
  double omega[3];
  double density_ratio; /* free motion: rho_s / rho_f (> 0) */
  double gravity[3];    /* free motion: gravitational acceleration (lattice units) */
} elbm_body;

typedef struct elbm_info {
  int64_t t;              /* time level of the current populations */
  int64_t nodes;          /* N */
  double beta;
  size_t pop_bytes;       /* bytes of one population array */
  size_t pop_offset;      /* byte offset of the current populations A^t in the workspace; SIZE_MAX
                             while they are in a caller's buffer (elbm_step_into) */
  size_t flags_offset;    /* byte offset of the uint8 node flags (0 if no geometry) */
  int32_t storage;
  int32_t nbodies;
  int64_t boundary_nodes; /* boundary + refill nodes of the last step (synchronises) */
  int64_t fp64_nodes;     /* nodes recomputed in FP64 during the last step (synchronises) */
  int32_t layout;         /* ELBM_LAYOUT_* of the population arrays */
  int32_t pad;
  double gamma_min;       /* with elbm_set_diagnostics(ctx, 1): smallest and largest stabiliser gamma */
  double gamma_max;       /* of the nodes collided since the last elbm_get_info (0 if none) */
  int32_t nonfinite;      /* nonzero once a step met a state that ELBM_ENONFINITE describes (bit 0 in
                             the bulk sweep, bit 1 at a wall node); cleared when populations are set */
  int32_t gamma_stats;    /* 1 while the gamma range is recorded */
} elbm_info;

/* Bytes of device workspace a context with these parameters needs. */
int elbm_workspace_bytes(const elbm_params* p, size_t* bytes);

/* Create a context.  stream: a hipStream_t (NULL = default stream).  workspace:
 * dev, >= elbm_workspace_bytes(p), 256-byte aligned, owned by the caller and
 * kept alive until elbm_destroy().  The populations are undefined until
 * elbm_init_equilibrium() or elbm_write_populations(). */
int elbm_create(const elbm_params* p, void* stream, void* workspace, size_t ws_bytes, struct elbm_ctx** out);

/* Free the context's host-side state (the workspace stays the caller's). */
int elbm_destroy(struct elbm_ctx* ctx);

int elbm_set_stream(struct elbm_ctx* ctx, void* stream);

/* A^0 = feq(rho, u) at every node (the entropic equilibrium of eq. feq_min),
 * computed in FP64 and rounded to the storage format; sets t = 0.
 * rho_dev: dev [N] FP64, or NULL for rho = 1; u_dev: dev [3][N] FP64. */
int elbm_init_equilibrium(struct elbm_ctx* ctx, const double* rho_dev, const double* u_dev);

/* Replace the populations with pop_dev (dev [27][N] FP64, rounded to the storage
 * format) and set the time level to t. */
int elbm_write_populations(struct elbm_ctx* ctx, const double* pop_dev, int64_t t);

/* Copy the current populations to pop_dev (dev [27][N] FP64, widened exactly). */
int elbm_read_populations(struct elbm_ctx* ctx, double* pop_dev);

/* Set the bodies (host array of nb <= max_bodies records; nb = 0 removes them)
 * and compute the solid mask at the current time level.  In channel mode a body
 * must stay at least 6 nodes away from the inlet and outlet faces. */
int elbm_set_geometry(struct elbm_ctx* ctx, const elbm_body* bodies, int32_t nb);

/* Triangulated body (the deforming geometries of Sec. IV.C: a closed triangulated surface whose
 * wall velocity at each link intersection is the barycentric interpolation of its vertex
 * velocities).  Sets the surface at the current time level: tris_dev dev [nt][3] int32 vertex
 * indices; verts_dev, vels_dev dev [nv][3] FP64 positions and velocities (vels_dev NULL = at rest);
 * box_lo, box_hi host double[3]: a box the surface stays inside for the whole run (it bounds the
 * per-step mask and list work; a vertex outside it makes the next elbm_force/elbm_force_history
 * fail with ELBM_ENOSPACE); center: host double[3], the point torques are taken about (NULL = the
 * box centre).  The arrays are copied on the context's stream.  Call before elbm_set_geometry
 * with a body of kind ELBM_BODY_MESH (its other fields are ignored), which must be the last body.
 * Definitions (FP64, operations in the written order, no fused multiply-add):
 *  - a node is solid iff the ray from it along +x crosses the surface an odd number of times; a
 *    triangle is crossed iff the node's (y, z) lies in its projection onto the y-z plane, points on
 *    a projected edge belonging to that edge's triangle iff the edge direction of the positively
 *    oriented projection has dz > 0, or dz = 0 and dy < 0; triangles of zero projected area are
 *    never crossed; the crossing is at x_c = (w0 x_A + w1 x_B + w2 x_C)/(w0 + w1 + w2) (projected
 *    edge functions w) and counts iff x_c > x;
 *  - link fraction q_i: the smallest s in (0, 1] where x - s c_i meets a triangle (ray-triangle
 *    intersection solved by scalar triple products), the wall velocity barycentric there; if
 *    rounding lets the segment pass between triangles, q = 1/2 and the velocity of the surface
 *    point closest to x - c_i/2;
 *  - velocity of the body at a node (refill, solid nodes' U^t): that of the closest surface point
 *    within the neighbouring cells of a grid of spacing >= 2 (0 if none; nodes where it is used lie
 *    within one lattice spacing of the surface).
 * The surface must stay at least 3 nodes inside every face.  Not with ELBM_FLAG_ADJOINT. */
int elbm_set_mesh(struct elbm_ctx* ctx, const int32_t* tris_dev, int32_t nt, const double* verts_dev,
                  const double* vels_dev, int32_t nv, const double box_lo[3], const double box_hi[3],
                  const double center[3]);

/* The triangulated body's vertex positions and velocities (same layout, the nv vertices of
 * elbm_set_mesh, same triangles) at the next time level, t+1, for the next step.  Without a call before a step the surface keeps its current
 * level (positions and velocities).  center: host double[3] or NULL (keep). */
int elbm_mesh_next(struct elbm_ctx* ctx, const double* verts_dev, const double* vels_dev, const double center[3]);

/* Position and velocity of body `body` at the current time level (host arrays of 3):
 * the prescribed motion evaluated at t, or the integrated state of a free body (synchronises). */
int elbm_body_state(struct elbm_ctx* ctx, int32_t body, double pos[3], double vel[3]);

/* Angular velocity of body `body` at the current time level (host array of 3): the prescribed
 * omega, or the integrated one of a freely rotating sphere (synchronises). */
int elbm_body_spin(struct elbm_ctx* ctx, int32_t body, double omega[3]);

/* Bind a body-force field F_dev (dev [3][N] FP32, borrowed until replaced) or
 * NULL for none.  Needs ELBM_FLAG_BODY_FORCE.  The collision adds
 * feq(rho, u + F/rho) - feq(rho, u); the reported velocity is (j + F/2)/rho. */
int elbm_set_body_force(struct elbm_ctx* ctx, const float* F_dev);

/* Advance nsteps >= 0 time steps (Secs. II-III): per step the geometry at t+1,
 * pull streaming, reconstruction of missing populations at walls, refill of
 * uncovered nodes, KBC collision, store, and the force on each body. */
int elbm_step(struct elbm_ctx* ctx, int32_t nsteps);

/* Flags of elbm_step_into. */
#define ELBM_STEP_SKIP_FORCE 1u /* the force of the step is not summed: its slot of the force ring keeps
                                   what it held (a recompute of levels whose forces an earlier pass
                                   recorded); not with free bodies, whose motion needs it */

/* One step of elbm_step that stores A^{t+1} in the caller's device buffer pop_next_dev
 * (27 N elements in the storage format and layout of elbm_save_state, 16-byte aligned, disjoint
 * from the current populations) instead of the workspace, and makes that buffer the current
 * population: the next step reads it and the refill of that step writes the uncovered nodes of
 * it in place.  The buffer is borrowed until the next elbm_step writes the workspace again or
 * elbm_write_populations / elbm_init_equilibrium / elbm_load_state replaces the populations;
 * elbm_get_info reports pop_offset = SIZE_MAX meanwhile.  step_flags: 0 or ELBM_STEP_SKIP_FORCE.
 * Lets a checkpointed reverse sweep keep every recomputed level without a copy.  ELBM_EINVAL for
 * NULL, misaligned or overlapping buffers, for unknown flags and for ELBM_STEP_SKIP_FORCE on a
 * context with free bodies. */
int elbm_step_into(struct elbm_ctx* ctx, void* pop_next_dev, uint32_t step_flags);

/* Force and torque on body `body` from the step that produced time level
 * `step` (1 <= step <= t, within the last force_ring steps): momentum exchange
 * of Sec. IV.A, torque about the body centre.  F, M: host double[3].
 * Synchronises.  Returns ELBM_ENOSPACE after a list overflow and ELBM_ENONFINITE once a step met
 * a failed state (see elbm_set_diagnostics). */
int elbm_force(struct elbm_ctx* ctx, int32_t body, int64_t step, double F[3], double M[3]);

/* Forces of `count` consecutive steps starting at time level `first`:
 * out_host [count][6] = (Fx, Fy, Fz, Mx, My, Mz).  Synchronises. */
int elbm_force_history(struct elbm_ctx* ctx, int32_t body, int64_t first, int32_t count, double* out_host);

/* Node flags at the current time level: out_dev (dev [N] uint8), bit 0 = solid. */
int elbm_read_flags(struct elbm_ctx* ctx, uint8_t* out_dev);

/* Context information (synchronises for the per-step counters).  Fills *out, then returns
 * ELBM_ENOSPACE if the boundary list has overflowed its capacity (the steps since are wrong at the
 * nodes that did not fit), else ELBM_OK.  A failed state is reported in out->nonfinite (and by
 * elbm_force, which returns ELBM_ENONFINITE); the gamma range restarts after each call. */
int elbm_get_info(struct elbm_ctx* ctx, elbm_info* out);

/* Failure detection is always on: every collided node tests that its state is finite and inside the
 * domain of the entropic equilibrium (Sec. II, eq. feq_min: rho > 0 and |u_a| < 1 for all a, so
 * that every feq_i > 0 and the entropic scalar product is defined), one vote per wavefront.
 * gamma_stats = 1 also records the range of the stabiliser gamma of the collided nodes (a
 * wavefront-wide min/max and one pair of atomics per wavefront in the bulk sweep; FP32 gamma for
 * nodes recomputed in FP64), reported and restarted by elbm_get_info; 0 stops it. */
int elbm_set_diagnostics(struct elbm_ctx* ctx, int32_t gamma_stats);

/* Copy the current populations, in the context's storage format and layout (27 N elements of 4
 * or 2 bytes, placed as elbm_info.layout says), to pop_dev (dev).  Used for checkpoints. */
int elbm_save_state(struct elbm_ctx* ctx, void* pop_dev);

/* Replace the current populations by pop_dev (dev, storage format, as written by
 * elbm_save_state) and set the time level to t; the geometry is recomputed for t. */
int elbm_load_state(struct elbm_ctx* ctx, const void* pop_dev, int64_t t);

/* One reverse step of the adjoint of elbm_step for the step t -> t+1 (an addition of this
 * library; the forward step it differentiates is the one of Secs. II-III and IV.A):
 *   lam_out = (dA^{t+1}/dA^t)^T lam_in + dL_t/dA^t,
 * where L_t = sum_b w_force[3b..3b+2] . F_b(t+1) is the loss term on the momentum-exchange force
 * of that step (w_force: host double[nbodies][3], NULL for none).  Also accumulates
 *   gF_dev += dL/dF (dev [3][N] FP32, body-force field; NULL to skip)
 * and, inside the context, dL/d(amp) of every body (elbm_adjoint_param_grad).
 * pop_t_dev: dev, the populations A^t in the storage format and layout (as elbm_save_state writes
 * them, e.g. recomputed from a checkpoint); the
 * entries of nodes uncovered by the step are overwritten with their refill values, as the forward
 * step does with its own buffer;
 * lam_in_dev, lam_out_dev: dev [27][N] FP32, distinct.  The solid masks of the step are those of
 * the forward run (their derivative is zero).  Needs ELBM_FLAG_ADJOINT and bodies without
 * rotation.  Overwrites the context's geometry state: call elbm_load_state before stepping on. */
int elbm_adjoint_step(struct elbm_ctx* ctx, int64_t t, void* pop_t_dev, const float* lam_in_dev,
                      float* lam_out_dev, const double* w_force, float* gF_dev);

/* dL/d(amp) of each body accumulated by elbm_adjoint_step (g_amp: host double[nbodies]);
 * reset = 1 clears the accumulators afterwards.  Synchronises. */
int elbm_adjoint_param_grad(struct elbm_ctx* ctx, double* g_amp, int32_t reset);

/* Per-step timing of the bulk sweep kernel with HIP events recorded on the context's stream
 * around each launch.  enable = 1 starts (and clears) the record, 0 stops it. */
int elbm_set_timing(struct elbm_ctx* ctx, int32_t enable);

/* Sum of the recorded sweep-kernel durations in ms and the number of launches (synchronises). */
int elbm_get_timing(struct elbm_ctx* ctx, double* sweep_ms, int64_t* launches);

/* Text of the last error of ctx (or of the last failed elbm_create if ctx is NULL). */
const char* elbm_last_error(const struct elbm_ctx* ctx);

/* Context-free KBC collision of n independent nodes (Sec. II): f_in_dev, f_out_dev
 * dev [27][n] FP32, gamma_dev dev [n] FP32 (or NULL), F_dev dev [3][n] FP32 or
 * NULL.  Uses the same device code as elbm_step, FP64 recomputation included
 * unless fp64_threshold < 0.  flags: 0, ELBM_FLAG_EXACT_GAMMA, ELBM_FLAG_LBGK or
 * ELBM_FLAG_CENTRAL (the variant).  stream: hipStream_t. */
int elbm_collide_nodes(const float* f_in_dev, float* f_out_dev, float* gamma_dev, const float* F_dev,
                       int64_t n, double nu, double fp64_threshold, uint32_t flags, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): one time step of a periodic box without bodies, the
 * work of elbm_step on such a context (pull streaming, KBC collision, FP64 recomputation of the
 * nodes the threshold selects), with no context and no workspace.  p: the parameters of such a
 * context (bc_x = ELBM_BC_PERIODIC, max_bodies = 0; flags only ELBM_FLAG_NO_FP64,
 * ELBM_FLAG_EXACT_GAMMA, ELBM_FLAG_LBGK, ELBM_FLAG_CENTRAL, ELBM_FLAG_STREAM_ONLY; the other
 * fields as elbm_create reads them).  pop_in_dev: dev, A^t, 27 N elements in the storage format
 * and layout that elbm_save_state writes (ELBM_LAYOUT_ROWS); pop_out_dev: dev, receives A^{t+1} in
 * the same form; the two must not overlap; both stay the caller's.  stream: a hipStream_t of the
 * current device.  Returns ELBM_EINVAL (elbm_last_error(NULL) says why) for other parameters, for
 * N > 8 388 608 nodes, or for overlapping arrays; ELBM_EDEVICE if a HIP call fails.
 * The library allocates nothing here: the FP64 queue and its counters live in a static device array
 * of 32 MiB + 256 bytes that each GPU the library runs on holds until the process ends.  Every call
 * on one GPU shares that array: calls that overlap in time on one GPU (several streams or host
 * threads) race and must be ordered by the caller. */
int elbm_step_periodic_noalloc(const elbm_params* p, const void* pop_in_dev, void* pop_out_dev, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ELBM_H */
