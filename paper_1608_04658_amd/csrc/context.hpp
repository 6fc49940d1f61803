// context.hpp -- host side of the library: the context behind the C ABI (device buffers carved out
// of the caller's workspace, geometry and time-level state) and the kernel launchers of the
// source files.  Device code lives in elbm_internal.hpp and the *_dev.hpp headers.
#pragma once

#include "elbm_internal.hpp"

// ---------------------------------------------------------------------------------------------
// The context behind the C ABI.
struct elbm_ctx {
  elbm_params p;
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  int64_t N;
  double beta;
  double fp64_thr;
  // carved fields (device)
  void* pop[2];
  int cur;                 // pop[cur] holds A^t
  void* own[2];            // the workspace's two population buffers (pop[] may point to a caller's
                           // buffer after elbm_step_into; a step always writes into own[] otherwise)
  elbm::PopLayout lay;     // placement of the populations in pop[0], pop[1] (pop_layout)
  uint8_t* flags;          // N (geometry only)
  float* macro;            // 4 N: U (3 N) then R (N) (geometry only)
  int32_t* blist;          // boundary list (geometry only)
  int64_t blist_cap;
  int64_t n_static;        // static part (channel inlet face, or all entries for static geometry)
  double* brec;            // per-list-entry force records [cap][nb][6]
  uint32_t* scan_tmp;      // 2 x scan_blocks: per-block counts and offsets of the list compaction
  int64_t scan_blocks;
  double* ring;            // [force_ring][MAX_BODIES][6]
  double* force_partial;   // [64][MAX_BODIES][6] partial sums of the force reduction
  int32_t* fix_list;       // N
  elbm::DevCounters* cnt;
  int fix_par;             // parity of the FP64 queue counter of the next step (DevCounters::fix_count)
  double* scratch64;       // small FP64 scratch (force sums)
  bool gamma_stats;        // record the range of gamma (elbm_set_diagnostics)
  const float* bodyforce;
  // geometry state
  int32_t nb;
  elbm_body bodies[ELBM_MAX_BODIES];
  bool moving;
  // free bodies (two-way coupling), integrated on the device: after each step a one-workgroup
  // kernel advances the state (elbm::FreeState, a ring over time levels) with the step's force and
  // writes the velocity at t+1 for the next step.  The host keeps a copy of the state at one time
  // level (free_lv), read one step behind the device, from which it derives the positions it
  // needs to place the geometry work (exact, the same FP64 operations as the device).
  struct FreeBody {
    bool on;
    double x[3], u[3], F[3];  // state at level free_lv
    double w[3], M[3];        // angular velocity and torque at level free_lv (rotating spheres)
    double m, ab[3];          // mass, (1 - 1/density_ratio) g
    double I;                 // (2/5) m R^2 for a freely rotating sphere, else 0
    double xt[3], ut[3], wt[3];  // position and velocities at the level of the step being launched
  } freeb[ELBM_MAX_BODIES];
  int n_free;
  int64_t free_lv;
  elbm::FreeState* free_hist;  // device [FREE_HIST][MAX_BODIES]
  double* free_U1;             // device [2][MAX_BODIES][3]: velocity, then angular velocity, at t+1
  hipStream_t aux;             // reads of the state, behind an event of the main stream
  hipEvent_t free_ev[4];       // recorded after the state of level t is written (slot t % FREE_HIST)
  int stab;         // STAB_KBC, STAB_EXACT or STAB_LBGK (from the context flags)
  // triangulated body (elbm_set_mesh): slot mesh_cur holds time level t; slot mesh_cur ^ 1 level
  // t+1 when mesh_next_set (else level t+1 = level t)
  int mesh_body;           // body index, -1 if none
  bool mesh_set;
  int32_t mesh_nv, mesh_nt;
  int mesh_cur;
  bool mesh_next_set;
  double mesh_ref[2][3];   // torque centre per slot
  double mesh_lo[3], mesh_hi[3];
  elbm::MeshDev mesh_grid; // grid geometry (pointers of slot 0/1 filled per use)
  int32_t* mesh_tri;
  double* mesh_X[2];
  double* mesh_V[2];
  int32_t* mesh_start[2];
  int32_t* mesh_items[2];
  int32_t* mesh_cursor;    // [MESH_CELLS] binning counters
  int64_t mesh_cap;        // items per slot
  bool slab_valid;  // slab_next holds U, R of the inlet slab of the current state (written by the
                    // kernels that produced it)
  float* slab_next; // channel mode: [4][nz][ny][3] staging of U, R for x < 3
  int64_t t;
  char err[256];
  // adjoint (ELBM_FLAG_ADJOINT)
  double* adj_gUR;         // 4 N: dL/dU^t (3 N) and dL/dR^t (N), FP64 scatter targets
  float* adj_side;         // 9 ny nz: outlet-copy adjoint contributions
  double* adj_gamp;        // [MAX_BODIES] dL/d(amplitude)
  double* adj_macro64;     // 4 N: U^t (3 N), R^t (N) in FP64 around the bodies and on the inlet slab,
                           // the point at which the reverse step linearises the wall rules
  double* adj_refill64;    // [blist_cap][27]: FP64 refill populations of the uncovered nodes, by list slot
  int32_t* adj_slot;       // N: list slot of an uncovered node (read only where the flags say refill)
  // sweep timing (HIP events around each bulk-sweep launch)
  bool timing;
  hipEvent_t* ev;
  int64_t ev_cap, ev_used;
};

namespace elbm {
// kernel launchers (defined in sweep.hip / geometry.hip)
PopLayout pop_layout(const elbm_params& p);
hipError_t launch_sweep(elbm_ctx* c);
hipError_t launch_fixup(elbm_ctx* c);
hipError_t launch_init_eq(elbm_ctx* c, const double* rho, const double* u);
hipError_t launch_write_pop(elbm_ctx* c, const double* src);
hipError_t launch_read_pop(elbm_ctx* c, double* dst);
hipError_t launch_collide_nodes(const float* fin, float* fout, float* gam, const float* F, int64_t n, double beta,
                                double thr, int stab, hipStream_t s);
hipError_t geometry_init(elbm_ctx* c);
hipError_t geometry_pre_step(elbm_ctx* c, const Bodies& bd);
hipError_t launch_boundary(elbm_ctx* c, const Bodies& bd);
hipError_t launch_refill(elbm_ctx* c, const Bodies& bd, void* A);
hipError_t launch_force_reduce(elbm_ctx* c);
hipError_t launch_adjoint(elbm_ctx* c, int64_t t, const void* A, const float* lam_in, float* lam_out,
                          const double* w_force, float* gF);
void host_kinematics(const elbm_body& b, double t, double c[3], double U[3]);
hipError_t macro_fields(elbm_ctx* c, const void* A, const Bodies& bd, bool slab);
hipError_t geometry_for_step(elbm_ctx* c, const Bodies& bd);
Box union_box(const elbm_ctx* c, const Bodies& bd);
Box full_box(const elbm_ctx* c);
Box2 macro_boxes(const elbm_ctx* c, const Bodies& bd, bool slab);
dim3 grid_for(long n);
Bodies make_bodies(const elbm_ctx* c, double t);
constexpr int MESH_CELLS = 1 << 16;
constexpr int FREE_HIST = 4;
hipError_t free_init(elbm_ctx* c);
hipError_t free_commit(elbm_ctx* c);
hipError_t mesh_upload(elbm_ctx* c, int slot, const double* X, const double* V);
hipError_t mesh_copy_tris(elbm_ctx* c, const int32_t* tris, int32_t nt);
hipError_t mesh_mask(elbm_ctx* c, const Bodies& bd, int level, uint8_t bits);
}  // namespace elbm
