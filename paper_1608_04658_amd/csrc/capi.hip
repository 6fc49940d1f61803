// capi.hip -- the C ABI of include/elbm.h: context set-up over a caller-owned device workspace,
// the per-step launch sequence, and force/state readback.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>

#include "context.hpp"

using namespace elbm;

static char g_create_err[256] = "";

static int fail(elbm_ctx* c, int code, const char* fmt, ...) {
  char* buf = c ? c->err : g_create_err;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, 256, fmt, ap);
  va_end(ap);
  return code;
}

#define HIP_OK(c, expr)                                                                    \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail((c), ELBM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

namespace {

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
  size_t pop[2], cnt, fix_list, flags, macro, slab, blist, brec, ring, force_partial, scratch, scan_tmp, adj_gUR, adj_side,
      adj_gamp, adj_macro64, adj_refill64, adj_slot, mesh_tri, mesh_X[2], mesh_V[2], mesh_start[2], mesh_items[2], mesh_cursor, free_hist, free_U1, total;
  int64_t mesh_cap;
  int64_t scan_blocks;
  int64_t cap;
  bool geometry;
};

bool has_geometry(const elbm_params* p) { return p->max_bodies > 0 || p->bc_x == ELBM_BC_CHANNEL; }

int64_t default_cap(const elbm_params* p) {
  const int64_t N = (int64_t)p->nx * p->ny * p->nz;
  const int64_t surf = 2 * ((int64_t)p->nx * p->ny + (int64_t)p->ny * p->nz + (int64_t)p->nx * p->nz) + 65536;
  return surf < N ? surf : N;
}

int validate(const elbm_params* p, char* err) {
  if (!p) return snprintf(err, 256, "params is NULL"), ELBM_EINVAL;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return snprintf(err, 256, "lattice size must be >= 1"), ELBM_EINVAL;
  const double N = (double)p->nx * p->ny * p->nz;
  if (N >= 2147483648.0) return snprintf(err, 256, "more than 2^31-1 nodes"), ELBM_EINVAL;
  if (27.0 * 4.0 * p->nx * p->ny >= 4294967296.0)
    return snprintf(err, 256, "a z plane of the populations exceeds 4 GiB (nx ny too large)"), ELBM_EINVAL;
  if (p->storage < 0 || p->storage > 2) return snprintf(err, 256, "bad storage %d", p->storage), ELBM_EINVAL;
  if (p->bc_x != ELBM_BC_PERIODIC && p->bc_x != ELBM_BC_CHANNEL) return snprintf(err, 256, "bad bc_x"), ELBM_EINVAL;
  if (p->bc_x == ELBM_BC_CHANNEL && p->nx < 4) return snprintf(err, 256, "channel needs nx >= 4"), ELBM_EINVAL;
  if (p->max_bodies < 0 || p->max_bodies > ELBM_MAX_BODIES) return snprintf(err, 256, "bad max_bodies"), ELBM_EINVAL;
  if (p->force_ring < 0 || (p->max_bodies > 0 && p->force_ring < 1))
    return snprintf(err, 256, "force_ring must be >= 1 (>= 0 without bodies)"), ELBM_EINVAL;
  if (!(p->nu > 0.0) || !isfinite(p->nu)) return snprintf(err, 256, "nu must be positive"), ELBM_EINVAL;
  if (p->max_boundary < 0) return snprintf(err, 256, "bad max_boundary"), ELBM_EINVAL;
  if ((p->flags & ELBM_FLAG_EXACT_GAMMA) && (p->flags & ELBM_FLAG_LBGK))
    return snprintf(err, 256, "ELBM_FLAG_EXACT_GAMMA and ELBM_FLAG_LBGK exclude each other"), ELBM_EINVAL;
  if ((p->flags & ELBM_FLAG_ADJOINT) && N >= 1073741824.0)  // 32-bit byte offsets into each adjoint direction
    return snprintf(err, 256, "the adjoint needs fewer than 2^30 nodes"), ELBM_EINVAL;
  if ((p->flags & ELBM_FLAG_EXACT_GAMMA) && (p->flags & ELBM_FLAG_ADJOINT))
    return snprintf(err, 256, "the adjoint differentiates the analytic stabiliser only"), ELBM_EINVAL;
  if ((p->flags & ELBM_FLAG_CENTRAL) && (p->flags & (ELBM_FLAG_EXACT_GAMMA | ELBM_FLAG_LBGK | ELBM_FLAG_ADJOINT)))
    return snprintf(err, 256, "ELBM_FLAG_CENTRAL goes with the analytic stabiliser and without the adjoint"),
           ELBM_EINVAL;
  if (p->max_mesh_vertices < 0 || p->max_mesh_triangles < 0 || p->max_mesh_triangles > (1 << 24) ||
      p->max_mesh_vertices > (1 << 24))
    return snprintf(err, 256, "bad mesh capacity"), ELBM_EINVAL;
  if ((p->max_mesh_triangles > 0) != (p->max_mesh_vertices > 0))
    return snprintf(err, 256, "mesh capacity needs both vertices and triangles"), ELBM_EINVAL;
  if (p->max_mesh_triangles > 0 && p->max_bodies < 1)
    return snprintf(err, 256, "a triangulated body needs max_bodies >= 1"), ELBM_EINVAL;
  if (p->max_mesh_triangles > 0 && (p->flags & ELBM_FLAG_ADJOINT))
    return snprintf(err, 256, "no triangulated bodies with the adjoint"), ELBM_EINVAL;
  return ELBM_OK;
}

Layout layout(const elbm_params* p) {
  Layout L{};
  const size_t N = (size_t)p->nx * p->ny * p->nz;
  const size_t es = storage_bytes(p->storage);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  L.pop[0] = take(27 * N * es);
  L.pop[1] = take(27 * N * es);
  L.cnt = take(sizeof(DevCounters));
  L.scratch = take(64 * sizeof(double));
  L.fix_list = take(4 * N);
  L.geometry = has_geometry(p);
  L.cap = 0;
  if (L.geometry) {
    L.cap = p->max_boundary > 0 ? p->max_boundary : default_cap(p);
    const int nbm = p->max_bodies > 0 ? p->max_bodies : 1;
    const int ring = p->force_ring > 0 ? p->force_ring : 1;
    L.flags = take(N);
    L.macro = take(16 * N);
    if (p->bc_x == ELBM_BC_CHANNEL) L.slab = take(sizeof(float) * 4 * 3 * (size_t)p->ny * p->nz);
    L.blist = take(4 * (size_t)L.cap);
    L.brec = take(sizeof(double) * 6 * nbm * (size_t)L.cap);
    L.ring = take(sizeof(double) * 6 * ELBM_MAX_BODIES * ring);
    L.force_partial = take(sizeof(double) * 64 * 6 * ELBM_MAX_BODIES);
    L.free_hist = take(sizeof(FreeState) * FREE_HIST * ELBM_MAX_BODIES);
    L.free_U1 = take(sizeof(double) * 6 * ELBM_MAX_BODIES);
    L.scan_blocks = (int64_t)((N + 255) / 256);
    L.scan_tmp = take(sizeof(uint32_t) * 2 * (size_t)L.scan_blocks);
  }
  if (p->flags & ELBM_FLAG_ADJOINT) {
    L.adj_gUR = take(sizeof(double) * 4 * N);
    L.adj_side = take(sizeof(float) * 9 * (size_t)p->ny * p->nz);
    L.adj_gamp = take(sizeof(double) * ELBM_MAX_BODIES);
    L.adj_macro64 = take(sizeof(double) * 4 * N);
    L.adj_refill64 = take(sizeof(double) * 27 * (size_t)(L.cap > 0 ? L.cap : 1));
    L.adj_slot = take(sizeof(int32_t) * N);
  }
  if (p->max_mesh_triangles > 0) {
    const size_t nv = (size_t)p->max_mesh_vertices, nt = (size_t)p->max_mesh_triangles;
    L.mesh_cap = 16 * (int64_t)nt + 4096;  // triangle-in-cell entries per time level
    L.mesh_tri = take(sizeof(int32_t) * 3 * nt);
    for (int s = 0; s < 2; ++s) {
      L.mesh_X[s] = take(sizeof(double) * 3 * nv);
      L.mesh_V[s] = take(sizeof(double) * 3 * nv);
      L.mesh_start[s] = take(sizeof(int32_t) * (MESH_CELLS + 1));
      L.mesh_items[s] = take(sizeof(int32_t) * (size_t)L.mesh_cap);
    }
    L.mesh_cursor = take(sizeof(int32_t) * MESH_CELLS);
  }
  L.total = off;
  return L;
}

bool body_moves(const elbm_body& b) {
  if (b.kind == ELBM_BODY_SPHERE)
    return (b.amp != 0.0 && b.period != 0.0) || b.vel[0] != 0.0 || b.vel[1] != 0.0 || b.vel[2] != 0.0;
  const double dn = b.dir[0] * b.normal[0] + b.dir[1] * b.normal[1] + b.dir[2] * b.normal[2];
  const double vn = b.vel[0] * b.normal[0] + b.vel[1] * b.normal[1] + b.vel[2] * b.normal[2];
  return (b.amp != 0.0 && b.period != 0.0 && dn != 0.0) || vn != 0.0;
}

// A free sphere centred at x: at least 3 nodes inside every face, 6 from the inlet and outlet.
bool free_inside(const elbm_ctx* c, const double x[3], double r) {
  const int n[3] = {c->p.nx, c->p.ny, c->p.nz};
  for (int a = 0; a < 3; ++a) {
    const double m = (a == 0 && c->p.bc_x == ELBM_BC_CHANNEL) ? 6.0 : 3.0;
    if (!(x[a] - r >= m) || !(x[a] + r <= n[a] - 1.0 - m)) return false;
  }
  return true;
}

// The device's free-body state of level lv into the host copy (waits for that level only).
hipError_t free_read_level(elbm_ctx* c, int64_t lv) {
  FreeState st[ELBM_MAX_BODIES];
  hipError_t e = hipStreamWaitEvent(c->aux, c->free_ev[lv % FREE_HIST], 0);
  if (e == hipSuccess)
    e = hipMemcpyAsync(st, c->free_hist + (size_t)(lv % FREE_HIST) * ELBM_MAX_BODIES, sizeof st,
                       hipMemcpyDeviceToHost, c->aux);
  if (e == hipSuccess) e = hipStreamSynchronize(c->aux);
  if (e != hipSuccess) return e;
  for (int k = 0; k < c->nb; ++k) {
    if (!c->freeb[k].on) continue;
    for (int a = 0; a < 3; ++a) {
      c->freeb[k].x[a] = st[k].x[a];
      c->freeb[k].u[a] = st[k].u[a];
      c->freeb[k].F[a] = st[k].F[a];
      c->freeb[k].w[a] = st[k].w[a];
      c->freeb[k].M[a] = st[k].M[a];
    }
  }
  c->free_lv = lv;
  return hipSuccess;
}

// Position and velocity at level c->t from the host copy at level c->t or c->t - 1 (explicit Euler
// in the operation order of the device integrator).
void free_derive(elbm_ctx* c) {
#pragma clang fp contract(off)
  for (int k = 0; k < c->nb; ++k) {
    auto& fb = c->freeb[k];
    if (!fb.on) continue;
    for (int a = 0; a < 3; ++a) {
      if (c->free_lv == c->t) {
        fb.xt[a] = fb.x[a];
        fb.ut[a] = fb.u[a];
        fb.wt[a] = fb.w[a];
      } else {
        fb.xt[a] = fb.x[a] + fb.u[a];
        fb.ut[a] = fb.u[a] + fb.F[a] / fb.m + fb.ab[a];
        fb.wt[a] = fb.I > 0.0 ? fb.w[a] + fb.M[a] / fb.I : fb.w[a];
      }
    }
  }
}

// The free bodies keep their state when the populations are replaced at level t: it is read back
// (synchronises) and stored again as the state of level t.
hipError_t free_reanchor(elbm_ctx* c, int64_t t) {
  if (!c->n_free) return hipSuccess;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess && c->free_lv != c->t) e = free_read_level(c, c->t);
  if (e != hipSuccess) return e;
  c->free_lv = t;
  const int64_t t_old = c->t;
  c->t = t;
  free_derive(c);
  c->t = t_old;
  return free_init(c);
}

// Failure flag cleared (with_flag) and the gamma range emptied (lo = all ones, hi = 0).
hipError_t diag_reset(elbm_ctx* c, bool with_flag) {
  hipError_t e = hipSuccess;
  if (with_flag) e = hipMemsetAsync(&c->cnt->nonfinite, 0, sizeof(uint32_t), c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(&c->cnt->gamma_lo, 0xFF, sizeof(uint32_t), c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(&c->cnt->gamma_hi, 0, sizeof(uint32_t), c->stream);
  return e;
}

}  // namespace

// geometry_init, and the static part of the boundary list checked against its capacity.
static int geo_init(elbm_ctx* c) {
  HIP_OK(c, geometry_init(c));
  if (c->n_static > c->blist_cap)
    return fail(c, ELBM_ENOSPACE, "the static boundary list needs %lld entries, max_boundary allows %lld",
                (long long)c->n_static, (long long)c->blist_cap);
  return ELBM_OK;
}

extern "C" {

int elbm_workspace_bytes(const elbm_params* p, size_t* bytes) {
  const int rc = validate(p, g_create_err);
  if (rc) return rc;
  if (!bytes) return fail(nullptr, ELBM_EINVAL, "bytes is NULL");
  *bytes = layout(p).total;
  return ELBM_OK;
}

// The context's own streams and events (those that exist).
static void release_streams(elbm_ctx* c) {
  for (int k = 0; k < FREE_HIST; ++k)
    if (c->free_ev[k]) (void)hipEventDestroy(c->free_ev[k]);
  if (c->aux) (void)hipStreamDestroy(c->aux);
}

int elbm_create(const elbm_params* p, void* stream, void* workspace, size_t ws_bytes, elbm_ctx** out) {
  const int rc = validate(p, g_create_err);
  if (rc) return rc;
  if (!out) return fail(nullptr, ELBM_EINVAL, "out is NULL");
  *out = nullptr;
  const Layout L = layout(p);
  if (!workspace) return fail(nullptr, ELBM_EINVAL, "workspace is NULL");
  if (((uintptr_t)workspace) % ALIGN) return fail(nullptr, ELBM_EINVAL, "workspace not 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(nullptr, ELBM_ENOSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
  elbm_ctx* c = new (std::nothrow) elbm_ctx();
  if (!c) return fail(nullptr, ELBM_EINVAL, "out of host memory");
  c->p = *p;
  if (c->p.rho0 == 0.0) c->p.rho0 = 1.0;
  c->stream = (hipStream_t)stream;
  c->ws = (char*)workspace;
  c->ws_bytes = ws_bytes;
  c->N = (int64_t)p->nx * p->ny * p->nz;
  c->beta = 1.0 / (6.0 * p->nu + 1.0);
  c->fp64_thr = p->fp64_threshold > 0.0 ? p->fp64_threshold : 1e-12;
  c->stab = (p->flags & ELBM_FLAG_EXACT_GAMMA) ? STAB_EXACT : ((p->flags & ELBM_FLAG_LBGK) ? STAB_LBGK : STAB_KBC);
  if (p->flags & ELBM_FLAG_CENTRAL) c->stab |= STAB_CENTRAL;
  c->pop[0] = c->ws + L.pop[0];
  c->pop[1] = c->ws + L.pop[1];
  c->own[0] = c->pop[0];
  c->own[1] = c->pop[1];
  c->cur = 0;
  c->lay = pop_layout(c->p);
  c->cnt = (DevCounters*)(c->ws + L.cnt);
  c->scratch64 = (double*)(c->ws + L.scratch);
  c->fix_list = (int32_t*)(c->ws + L.fix_list);
  c->flags = L.geometry ? (uint8_t*)(c->ws + L.flags) : nullptr;
  c->macro = L.geometry ? (float*)(c->ws + L.macro) : nullptr;
  c->slab_next = (L.geometry && p->bc_x == ELBM_BC_CHANNEL) ? (float*)(c->ws + L.slab) : nullptr;
  c->slab_valid = false;
  c->blist = L.geometry ? (int32_t*)(c->ws + L.blist) : nullptr;
  c->brec = L.geometry ? (double*)(c->ws + L.brec) : nullptr;
  c->ring = L.geometry ? (double*)(c->ws + L.ring) : nullptr;
  c->force_partial = L.geometry ? (double*)(c->ws + L.force_partial) : nullptr;
  const bool adj = (p->flags & ELBM_FLAG_ADJOINT) != 0;
  c->adj_gUR = adj ? (double*)(c->ws + L.adj_gUR) : nullptr;
  c->adj_side = adj ? (float*)(c->ws + L.adj_side) : nullptr;
  c->adj_gamp = adj ? (double*)(c->ws + L.adj_gamp) : nullptr;
  c->adj_macro64 = adj ? (double*)(c->ws + L.adj_macro64) : nullptr;
  c->adj_refill64 = adj ? (double*)(c->ws + L.adj_refill64) : nullptr;
  c->adj_slot = adj ? (int32_t*)(c->ws + L.adj_slot) : nullptr;
  const bool mesh = p->max_mesh_triangles > 0;
  c->mesh_body = -1;
  c->mesh_set = false;
  c->mesh_nv = c->mesh_nt = 0;
  c->mesh_cur = 0;
  c->mesh_next_set = false;
  c->mesh_grid = MeshDev{};
  c->mesh_cap = mesh ? L.mesh_cap : 0;
  c->mesh_tri = mesh ? (int32_t*)(c->ws + L.mesh_tri) : nullptr;
  c->mesh_cursor = mesh ? (int32_t*)(c->ws + L.mesh_cursor) : nullptr;
  for (int s = 0; s < 2; ++s) {
    c->mesh_X[s] = mesh ? (double*)(c->ws + L.mesh_X[s]) : nullptr;
    c->mesh_V[s] = mesh ? (double*)(c->ws + L.mesh_V[s]) : nullptr;
    c->mesh_start[s] = mesh ? (int32_t*)(c->ws + L.mesh_start[s]) : nullptr;
    c->mesh_items[s] = mesh ? (int32_t*)(c->ws + L.mesh_items[s]) : nullptr;
  }
  c->blist_cap = L.cap;
  c->scan_tmp = L.geometry ? (uint32_t*)(c->ws + L.scan_tmp) : nullptr;
  c->scan_blocks = L.geometry ? L.scan_blocks : 0;
  c->n_static = 0;
  c->bodyforce = nullptr;
  c->nb = 0;
  c->moving = false;
  c->n_free = 0;
  c->free_lv = 0;
  c->free_hist = L.geometry ? (FreeState*)(c->ws + L.free_hist) : nullptr;
  c->free_U1 = L.geometry ? (double*)(c->ws + L.free_U1) : nullptr;
  c->aux = nullptr;
  for (int k = 0; k < FREE_HIST; ++k) c->free_ev[k] = nullptr;
  for (int k = 0; k < ELBM_MAX_BODIES; ++k) c->freeb[k].on = false;
  c->t = 0;
  c->err[0] = 0;
  c->timing = false;
  c->ev = nullptr;
  c->ev_cap = c->ev_used = 0;
  hipError_t e = hipMemsetAsync(c->cnt, 0, sizeof(DevCounters), c->stream);
  if (e == hipSuccess && L.geometry) e = hipMemsetAsync(c->flags, 0, (size_t)c->N, c->stream);
  if (e == hipSuccess && L.geometry)  // the ring as layout() sized it
    e = hipMemsetAsync(c->ring, 0, sizeof(double) * 6 * ELBM_MAX_BODIES * (size_t)(p->force_ring > 0 ? p->force_ring : 1),
                       c->stream);
  if (e == hipSuccess) e = diag_reset(c, true);
  if (e == hipSuccess && L.geometry) e = hipMemsetAsync(c->macro, 0, 16 * (size_t)c->N, c->stream);
  if (e == hipSuccess && adj) e = hipMemsetAsync(c->adj_gUR, 0, sizeof(double) * 4 * (size_t)c->N, c->stream);
  if (e == hipSuccess && adj) e = hipMemsetAsync(c->adj_side, 0, sizeof(float) * 9 * (size_t)p->ny * p->nz, c->stream);
  if (e == hipSuccess && adj) e = hipMemsetAsync(c->adj_gamp, 0, sizeof(double) * ELBM_MAX_BODIES, c->stream);
  if (e == hipSuccess && adj) e = hipMemsetAsync(c->adj_macro64, 0, sizeof(double) * 4 * (size_t)c->N, c->stream);
  if (e == hipSuccess && adj) e = hipMemsetAsync(c->adj_slot, 0xFF, sizeof(int32_t) * (size_t)c->N, c->stream);
  if (e == hipSuccess && L.geometry) e = hipMemsetAsync(c->free_U1, 0, sizeof(double) * 6 * ELBM_MAX_BODIES, c->stream);
  if (e == hipSuccess && L.geometry) e = hipStreamCreate(&c->aux);  // default priority
  for (int k = 0; k < FREE_HIST && e == hipSuccess && L.geometry; ++k)
    e = hipEventCreateWithFlags(&c->free_ev[k], hipEventDisableTiming);
  if (e != hipSuccess) {
    release_streams(c);
    delete c;
    return fail(nullptr, ELBM_EDEVICE, "context set-up: %s", hipGetErrorString(e));
  }
  if (L.geometry) {
    // channel without bodies: the inlet face is the static boundary list
    const int g = geometry_init(c);
    const bool over = g == hipSuccess && c->n_static > c->blist_cap;
    if (g != hipSuccess || over) {
      release_streams(c);
      const long long ns = (long long)c->n_static, cap = (long long)c->blist_cap;
      delete c;
      if (over)
        return fail(nullptr, ELBM_ENOSPACE, "the static boundary list needs %lld entries, max_boundary allows %lld", ns, cap);
      return fail(nullptr, ELBM_EDEVICE, "geometry set-up failed");
    }
  }
  *out = c;
  return ELBM_OK;
}

static void free_events(elbm_ctx* c) {
  if (c->ev) {
    for (int64_t k = 0; k < 2 * c->ev_cap; ++k)
      if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
    free(c->ev);
  }
  c->ev = nullptr;
  c->ev_cap = c->ev_used = 0;
}

int elbm_destroy(elbm_ctx* c) {
  if (!c) return ELBM_EINVAL;
  free_events(c);
  release_streams(c);
  delete c;
  return ELBM_OK;
}

int elbm_set_stream(elbm_ctx* c, void* stream) {
  if (!c) return ELBM_EINVAL;
  c->stream = (hipStream_t)stream;
  return ELBM_OK;
}

int elbm_init_equilibrium(elbm_ctx* c, const double* rho_dev, const double* u_dev) {
  if (!c) return ELBM_EINVAL;
  if (!u_dev) return fail(c, ELBM_EINVAL, "u_dev is NULL");
  // both buffers: nodes that stay solid are never written by a step
  HIP_OK(c, free_reanchor(c, 0));
  c->pop[0] = c->own[0];
  c->pop[1] = c->own[1];
  c->cur = 1;
  HIP_OK(c, launch_init_eq(c, rho_dev, u_dev));
  c->cur = 0;
  c->t = 0;
  HIP_OK(c, launch_init_eq(c, rho_dev, u_dev));
  HIP_OK(c, diag_reset(c, true));
  if (c->flags) return geo_init(c);
  return ELBM_OK;
}

int elbm_write_populations(elbm_ctx* c, const double* pop_dev, int64_t t) {
  if (!c) return ELBM_EINVAL;
  if (!pop_dev || t < 0) return fail(c, ELBM_EINVAL, "bad arguments");
  HIP_OK(c, free_reanchor(c, t));
  c->t = t;
  c->pop[0] = c->own[0];
  c->pop[1] = c->own[1];
  HIP_OK(c, launch_write_pop(c, pop_dev));
  HIP_OK(c, diag_reset(c, true));
  if (c->flags) return geo_init(c);
  return ELBM_OK;
}

int elbm_read_populations(elbm_ctx* c, double* pop_dev) {
  if (!c) return ELBM_EINVAL;
  if (!pop_dev) return fail(c, ELBM_EINVAL, "pop_dev is NULL");
  HIP_OK(c, launch_read_pop(c, pop_dev));
  return ELBM_OK;
}

int elbm_set_geometry(elbm_ctx* c, const elbm_body* bodies, int32_t nb) {
  if (!c) return ELBM_EINVAL;
  if (nb < 0 || nb > c->p.max_bodies) return fail(c, ELBM_EINVAL, "nb = %d exceeds max_bodies = %d", nb, c->p.max_bodies);
  if (nb > 0 && !bodies) return fail(c, ELBM_EINVAL, "bodies is NULL");
  bool moving = false;
  for (int k = 0; k < nb; ++k) {
    const elbm_body& b = bodies[k];
    if (b.kind == ELBM_BODY_MESH) {
      if (!c->mesh_set) return fail(c, ELBM_ESTATE, "body %d: no triangulated surface set (elbm_set_mesh)", k);
      if (k != nb - 1) return fail(c, ELBM_EINVAL, "body %d: the triangulated body must be the last body", k);
      if (b.motion != ELBM_MOTION_PRESCRIBED) return fail(c, ELBM_EINVAL, "body %d: a triangulated body moves as given", k);
      moving = true;
      continue;
    }
    if (b.kind != ELBM_BODY_SPHERE && b.kind != ELBM_BODY_PLANE) return fail(c, ELBM_EINVAL, "body %d: bad kind", k);
    if (b.motion != ELBM_MOTION_PRESCRIBED && b.motion != ELBM_MOTION_FREE && b.motion != ELBM_MOTION_FREE_ROTATING)
      return fail(c, ELBM_EINVAL, "body %d: bad motion", k);
    if (b.motion != ELBM_MOTION_PRESCRIBED) {
      if (b.kind != ELBM_BODY_SPHERE || !(b.radius > 0.0)) return fail(c, ELBM_EINVAL, "body %d: free motion needs a sphere", k);
      if (!(b.density_ratio > 0.0) || !isfinite(b.density_ratio))
        return fail(c, ELBM_EINVAL, "body %d: density_ratio must be positive", k);
      if (b.amp != 0.0 || b.period != 0.0)
        return fail(c, ELBM_EINVAL, "body %d: a free body has no prescribed oscillation", k);
      if (b.motion == ELBM_MOTION_FREE && (b.omega[0] != 0.0 || b.omega[1] != 0.0 || b.omega[2] != 0.0))
        return fail(c, ELBM_EINVAL, "body %d: omega needs ELBM_MOTION_FREE_ROTATING", k);
      if (c->p.flags & ELBM_FLAG_ADJOINT) return fail(c, ELBM_EINVAL, "body %d: no free bodies with the adjoint", k);
      if (!free_inside(c, b.center, b.radius))
        return fail(c, ELBM_EINVAL, "body %d: free sphere too close to a face", k);
      moving = true;
      continue;
    }
    if (b.kind == ELBM_BODY_SPHERE && !(b.radius > 0.0)) return fail(c, ELBM_EINVAL, "body %d: radius <= 0", k);
    if (b.kind == ELBM_BODY_PLANE) {
      const double nn = b.normal[0] * b.normal[0] + b.normal[1] * b.normal[1] + b.normal[2] * b.normal[2];
      if (fabs(nn - 1.0) > 1e-12) return fail(c, ELBM_EINVAL, "body %d: plane normal not unit", k);
    }
    if (b.kind == ELBM_BODY_SPHERE && c->p.bc_x == ELBM_BC_CHANNEL) {
      const double ex = b.radius + fabs(b.amp * b.dir[0]);
      if (b.vel[0] != 0.0 || b.center[0] - ex < 6.0 || b.center[0] + ex > c->p.nx - 7.0)
        return fail(c, ELBM_EINVAL, "body %d: sphere must stay 6 nodes from inlet and outlet", k);
    }
    if ((c->p.flags & ELBM_FLAG_ADJOINT) && (b.omega[0] != 0.0 || b.omega[1] != 0.0 || b.omega[2] != 0.0))
      return fail(c, ELBM_EINVAL, "body %d: the adjoint supports bodies without rotation", k);
    moving = moving || body_moves(b);
  }
  c->nb = nb;
  c->mesh_body = (nb > 0 && bodies[nb - 1].kind == ELBM_BODY_MESH) ? nb - 1 : -1;
  c->n_free = 0;
  c->free_lv = c->t;
  for (int k = 0; k < ELBM_MAX_BODIES; ++k) c->freeb[k].on = false;
  for (int k = 0; k < nb; ++k) {
    c->bodies[k] = bodies[k];
    const elbm_body& b = bodies[k];
    if (b.motion == ELBM_MOTION_PRESCRIBED) continue;
    auto& fb = c->freeb[k];
    fb.on = true;
    fb.m = b.density_ratio * c->p.rho0 * (4.0 / 3.0) * M_PI * b.radius * b.radius * b.radius;
    const bool rot = b.motion == ELBM_MOTION_FREE_ROTATING;
    fb.I = rot ? 0.4 * fb.m * b.radius * b.radius : 0.0;
    for (int a = 0; a < 3; ++a) {
      fb.x[a] = b.center[a];
      fb.u[a] = b.vel[a];
      fb.F[a] = 0.0;
      fb.w[a] = rot ? b.omega[a] : 0.0;
      fb.M[a] = 0.0;
      fb.ab[a] = (1.0 - 1.0 / b.density_ratio) * b.gravity[a];
      fb.xt[a] = b.center[a];
      fb.ut[a] = b.vel[a];
      fb.wt[a] = fb.w[a];
    }
    c->n_free += 1;
  }
  if (c->n_free) HIP_OK(c, free_init(c));
  c->moving = moving;
  if (!c->flags) {
    if (nb > 0) return fail(c, ELBM_ESTATE, "context created with max_bodies = 0");
    return ELBM_OK;
  }
  return geo_init(c);
}

int elbm_set_mesh(elbm_ctx* c, const int32_t* tris_dev, int32_t nt, const double* verts_dev, const double* vels_dev,
                  int32_t nv, const double box_lo[3], const double box_hi[3], const double center[3]) {
  if (!c) return ELBM_EINVAL;
  if (!c->mesh_tri) return fail(c, ELBM_ESTATE, "context created without mesh capacity");
  if (!tris_dev || !verts_dev || !box_lo || !box_hi) return fail(c, ELBM_EINVAL, "NULL argument");
  if (nt < 1 || nt > c->p.max_mesh_triangles || nv < 3 || nv > c->p.max_mesh_vertices)
    return fail(c, ELBM_EINVAL, "nt = %d, nv = %d outside the capacity (%d, %d)", nt, nv, c->p.max_mesh_triangles,
                c->p.max_mesh_vertices);
  const int dims[3] = {c->p.nx, c->p.ny, c->p.nz};
  double ext[3];
  for (int a = 0; a < 3; ++a) {
    const double m = (a == 0 && c->p.bc_x == ELBM_BC_CHANNEL) ? 6.0 : 3.0;
    if (!(box_lo[a] < box_hi[a]) || !(box_lo[a] >= m) || !(box_hi[a] <= dims[a] - 1.0 - m))
      return fail(c, ELBM_EINVAL, "mesh box must lie %s nodes inside the faces", c->p.bc_x == ELBM_BC_CHANNEL ? "3 (6 in x)" : "3");
    ext[a] = box_hi[a] - box_lo[a];
  }
  // cells of spacing h >= 2 with one cell of margin on every side, at most MESH_CELLS of them
  double h = 2.0;
  int dim[3];
  for (int it = 0; it < 64; ++it) {
    long n = 1;
    for (int a = 0; a < 3; ++a) {
      dim[a] = (int)floor(ext[a] / h) + 3;
      n *= dim[a];
    }
    if (n <= MESH_CELLS) break;
    h *= 1.25;
  }
  if ((long)dim[0] * dim[1] * dim[2] > MESH_CELLS) return fail(c, ELBM_EINVAL, "mesh box too large for the cell grid");
  MeshDev& g = c->mesh_grid;
  g = MeshDev{};
  g.inv_h = 1.0 / h;
  g.ncell = dim[0] * dim[1] * dim[2];
  for (int a = 0; a < 3; ++a) {
    g.dim[a] = dim[a];
    g.org[a] = box_lo[a] - h;
    // the node region of the mask and the list: the whole grid
    c->mesh_lo[a] = g.org[a];
    c->mesh_hi[a] = g.org[a] + dim[a] * h;
  }
  c->mesh_nt = nt;
  c->mesh_nv = nv;
  c->mesh_cur = 0;
  c->mesh_next_set = false;
  for (int a = 0; a < 3; ++a) {
    const double r = center ? center[a] : 0.5 * (box_lo[a] + box_hi[a]);
    c->mesh_ref[0][a] = c->mesh_ref[1][a] = r;
  }
  g.cap = (int32_t)std::min<int64_t>(c->mesh_cap, INT32_MAX);
  HIP_OK(c, mesh_copy_tris(c, tris_dev, nt));
  HIP_OK(c, mesh_upload(c, 0, verts_dev, vels_dev));
  c->mesh_set = true;
  return ELBM_OK;
}

// verts_dev / vels_dev hold the nv vertices of elbm_set_mesh (their size cannot be checked here).
int elbm_mesh_next(elbm_ctx* c, const double* verts_dev, const double* vels_dev, const double center[3]) {
  if (!c) return ELBM_EINVAL;
  if (!c->mesh_set) return fail(c, ELBM_ESTATE, "no triangulated surface set");
  if (!verts_dev) return fail(c, ELBM_EINVAL, "verts_dev is NULL");
  const int s1 = c->mesh_cur ^ 1;
  HIP_OK(c, mesh_upload(c, s1, verts_dev, vels_dev));
  for (int a = 0; a < 3; ++a) c->mesh_ref[s1][a] = center ? center[a] : c->mesh_ref[c->mesh_cur][a];
  c->mesh_next_set = true;
  return ELBM_OK;
}

int elbm_body_state(elbm_ctx* c, int32_t body, double pos[3], double vel[3]) {
  if (!c) return ELBM_EINVAL;
  if (body < 0 || body >= c->nb || !pos || !vel) return fail(c, ELBM_EINVAL, "bad arguments");
  if (c->freeb[body].on) {
    HIP_OK(c, hipStreamSynchronize(c->stream));
    if (c->free_lv != c->t) HIP_OK(c, free_read_level(c, c->t));
    for (int a = 0; a < 3; ++a) {
      pos[a] = c->freeb[body].x[a];
      vel[a] = c->freeb[body].u[a];
    }
  } else if (body == c->mesh_body) {
    for (int a = 0; a < 3; ++a) {
      pos[a] = c->mesh_ref[c->mesh_cur][a];
      vel[a] = 0.0;
    }
  } else {
    host_kinematics(c->bodies[body], (double)c->t, pos, vel);
  }
  return ELBM_OK;
}

int elbm_body_spin(elbm_ctx* c, int32_t body, double omega[3]) {
  if (!c) return ELBM_EINVAL;
  if (body < 0 || body >= c->nb || !omega) return fail(c, ELBM_EINVAL, "bad arguments");
  if (c->freeb[body].on) {
    HIP_OK(c, hipStreamSynchronize(c->stream));
    if (c->free_lv != c->t) HIP_OK(c, free_read_level(c, c->t));
    for (int a = 0; a < 3; ++a) omega[a] = c->freeb[body].w[a];
  } else {
    for (int a = 0; a < 3; ++a) omega[a] = c->bodies[body].omega[a];
  }
  return ELBM_OK;
}

int elbm_set_body_force(elbm_ctx* c, const float* F_dev) {
  if (!c) return ELBM_EINVAL;
  if (F_dev && !(c->p.flags & ELBM_FLAG_BODY_FORCE)) return fail(c, ELBM_ESTATE, "ELBM_FLAG_BODY_FORCE not set");
  c->bodyforce = F_dev;
  c->slab_valid = false;  // U = (j - F/2) / rho depends on the field
  return ELBM_OK;
}

// One step t -> t+1 writing A^{t+1} into dst (NULL: the workspace buffer of the other slot);
// force = false leaves the force of the step unsummed (its ring slot keeps what it held).
static int one_step(elbm_ctx* c, void* dst, bool force = true) {
  const bool geo = c->flags != nullptr;
  c->pop[c->cur ^ 1] = dst ? dst : c->own[c->cur ^ 1];
  {
    if (c->n_free) {
      // positions at t and t+1 from the state of level t or t-1 (the latter read one step behind
      // the device: the step before is still running meanwhile)
      if (c->free_lv < c->t - 1) HIP_OK(c, free_read_level(c, c->t - 1));
      free_derive(c);
      for (int k = 0; k < c->nb; ++k) {
        if (!c->freeb[k].on) continue;
        double x1[3];
        for (int a = 0; a < 3; ++a) x1[a] = c->freeb[k].xt[a] + c->freeb[k].ut[a];
        if (!free_inside(c, x1, c->bodies[k].radius))
          return fail(c, ELBM_ESTATE, "free body %d would come closer than allowed to a face at t = %lld", k,
                      (long long)(c->t + 1));
      }
    }
    Bodies bd;
    if (geo) {
      bd = make_bodies(c, (double)c->t);
      HIP_OK(c, geometry_pre_step(c, bd));
      HIP_OK(c, launch_refill(c, bd, c->pop[c->cur]));
    }
    const bool rec = c->timing && c->ev_used < c->ev_cap;
    if (rec) HIP_OK(c, hipEventRecord(c->ev[2 * c->ev_used], c->stream));
    HIP_OK(c, launch_sweep(c));
    if (rec) {
      HIP_OK(c, hipEventRecord(c->ev[2 * c->ev_used + 1], c->stream));
      c->ev_used += 1;
    }
    if (geo) HIP_OK(c, launch_boundary(c, bd));
    HIP_OK(c, launch_fixup(c));  // bulk and wall nodes queued for the FP64 collision
    c->fix_par ^= 1;
    if (geo && force) HIP_OK(c, launch_force_reduce(c));
    if (c->n_free) HIP_OK(c, free_commit(c));  // the free bodies' state of level t+1 on the device
    if (c->mesh_next_set) {
      c->mesh_cur ^= 1;
      c->mesh_next_set = false;
    }
    c->cur ^= 1;
    c->t += 1;
    // the sweep, the wall kernel and the fix-up staged U, R of the new state's inlet slab
    c->slab_valid = c->slab_next != nullptr && !(c->p.flags & ELBM_FLAG_STREAM_ONLY);
  }
  return ELBM_OK;
}

int elbm_step(elbm_ctx* c, int32_t nsteps) {
  if (!c) return ELBM_EINVAL;
  if (nsteps < 0) return fail(c, ELBM_EINVAL, "nsteps < 0");
  for (int32_t s = 0; s < nsteps; ++s) {
    const int rc = one_step(c, nullptr);
    if (rc) return rc;
  }
  return ELBM_OK;
}

int elbm_step_into(elbm_ctx* c, void* pop_next_dev, uint32_t step_flags) {
  if (!c) return ELBM_EINVAL;
  if (!pop_next_dev) return fail(c, ELBM_EINVAL, "pop_next_dev is NULL");
  if (step_flags & ~(uint32_t)ELBM_STEP_SKIP_FORCE) return fail(c, ELBM_EINVAL, "unknown step flags 0x%x", step_flags);
  const bool skip_force = (step_flags & ELBM_STEP_SKIP_FORCE) != 0;
  if (skip_force && c->n_free) return fail(c, ELBM_EINVAL, "free bodies need the force of every step");
  const size_t bytes = 27 * (size_t)c->N * storage_bytes(c->p.storage);
  const char* a0 = (const char*)c->pop[c->cur];
  const char* b0 = (const char*)pop_next_dev;
  if (a0 < b0 + bytes && b0 < a0 + bytes) return fail(c, ELBM_EINVAL, "pop_next_dev overlaps the current populations");
  if (((uintptr_t)pop_next_dev) % 16) return fail(c, ELBM_EINVAL, "pop_next_dev must be 16-byte aligned");
  return one_step(c, pop_next_dev, !skip_force);
}

int elbm_force_history(elbm_ctx* c, int32_t body, int64_t first, int32_t count, double* out_host) {
  if (!c) return ELBM_EINVAL;
  if (body < 0 || body >= c->nb) return fail(c, ELBM_EINVAL, "no body %d", body);
  if (count < 0 || !out_host) return fail(c, ELBM_EINVAL, "bad arguments");
  const int64_t ring = c->p.force_ring;
  if (first < 1 || first + count - 1 > c->t || first <= c->t - ring)
    return fail(c, ELBM_EINVAL, "steps %lld..%lld not in the force ring (t = %lld, ring = %lld)", (long long)first,
                (long long)(first + count - 1), (long long)c->t, (long long)ring);
  HIP_OK(c, hipStreamSynchronize(c->stream));
  uint32_t ov = 0;
  HIP_OK(c, hipMemcpy(&ov, &c->cnt->overflow, sizeof ov, hipMemcpyDeviceToHost));
  if (ov & 1u) return fail(c, ELBM_ENOSPACE, "boundary list overflowed its capacity (%lld)", (long long)c->blist_cap);
  if (ov & 2u) return fail(c, ELBM_ENOSPACE, "a mesh vertex left the declared box, or the mesh grid is full");
  if (ov & 4u) return fail(c, ELBM_ENOSPACE, "a lattice row crosses the mesh more than 32 times");
  if (ov & 8u) return fail(c, ELBM_EINVAL, "a mesh triangle has a vertex index outside [0, nv)");
  uint32_t nf = 0;
  HIP_OK(c, hipMemcpy(&nf, &c->cnt->nonfinite, sizeof nf, hipMemcpyDeviceToHost));
  if (nf)
    return fail(c, ELBM_ENONFINITE, "a node had a non-finite state or one where the entropic equilibrium is not "
                "positive (rho <= 0 or |u_a| >= 1) in the %s", (nf & 1u) ? "bulk sweep" : "wall kernel");
  for (int32_t k = 0; k < count; ++k) {
    const int64_t step = first + k;
    const int slot = (int)(step % ring);
    HIP_OK(c, hipMemcpy(out_host + 6 * k, c->ring + ((size_t)slot * ELBM_MAX_BODIES + body) * 6, 6 * sizeof(double),
                        hipMemcpyDeviceToHost));
  }
  return ELBM_OK;
}

int elbm_force(elbm_ctx* c, int32_t body, int64_t step, double F[3], double M[3]) {
  double rec[6];
  const int rc = elbm_force_history(c, body, step, 1, rec);
  if (rc) return rc;
  for (int a = 0; a < 3; ++a) {
    if (F) F[a] = rec[a];
    if (M) M[a] = rec[3 + a];
  }
  return ELBM_OK;
}

int elbm_read_flags(elbm_ctx* c, uint8_t* out_dev) {
  if (!c) return ELBM_EINVAL;
  if (!out_dev) return fail(c, ELBM_EINVAL, "out_dev is NULL");
  if (!c->flags) {
    HIP_OK(c, hipMemsetAsync(out_dev, 0, (size_t)c->N, c->stream));
    return ELBM_OK;
  }
  HIP_OK(c, hipMemcpyAsync(out_dev, c->flags, (size_t)c->N, hipMemcpyDeviceToDevice, c->stream));
  return ELBM_OK;
}

int elbm_get_info(elbm_ctx* c, elbm_info* out) {
  if (!c || !out) return ELBM_EINVAL;
  memset(out, 0, sizeof *out);
  out->t = c->t;
  out->nodes = c->N;
  out->beta = c->beta;
  out->pop_bytes = 27 * (size_t)c->N * storage_bytes(c->p.storage);
  out->pop_offset = c->pop[c->cur] == c->own[c->cur] ? (size_t)((char*)c->pop[c->cur] - c->ws) : (size_t)-1;
  out->flags_offset = c->flags ? (size_t)((char*)c->flags - c->ws) : 0;
  out->storage = c->p.storage;
  out->layout = c->lay.interleaved ? ELBM_LAYOUT_ROWS : ELBM_LAYOUT_SOA;
  out->nbodies = c->nb;
  HIP_OK(c, hipStreamSynchronize(c->stream));
  DevCounters h;
  HIP_OK(c, hipMemcpy(&h, c->cnt, sizeof h, hipMemcpyDeviceToHost));
  out->boundary_nodes = c->flags ? c->n_static + (c->moving ? (int64_t)h.dyn_count : 0) : 0;
  out->fp64_nodes = h.fix_count[c->fix_par ^ 1];
  out->nonfinite = (int32_t)h.nonfinite;
  out->gamma_stats = c->gamma_stats ? 1 : 0;
  const bool seen = c->gamma_stats && h.gamma_lo != 0xFFFFFFFFu;
  out->gamma_min = seen ? (double)f32_unkey(h.gamma_lo) : 0.0;
  out->gamma_max = seen ? (double)f32_unkey(h.gamma_hi) : 0.0;
  if (c->gamma_stats) HIP_OK(c, diag_reset(c, false));  // the range restarts with the next step
  if (h.overflow & 1u)
    return fail(c, ELBM_ENOSPACE, "boundary list overflowed its capacity (%lld)", (long long)c->blist_cap);
  return ELBM_OK;
}

int elbm_set_diagnostics(elbm_ctx* c, int32_t gamma_stats) {
  if (!c) return ELBM_EINVAL;
  c->gamma_stats = gamma_stats != 0;
  HIP_OK(c, diag_reset(c, false));
  return ELBM_OK;
}

int elbm_save_state(elbm_ctx* c, void* pop_dev) {
  if (!c) return ELBM_EINVAL;
  if (!pop_dev) return fail(c, ELBM_EINVAL, "pop_dev is NULL");
  const size_t bytes = 27 * (size_t)c->N * storage_bytes(c->p.storage);
  HIP_OK(c, hipMemcpyAsync(pop_dev, c->pop[c->cur], bytes, hipMemcpyDeviceToDevice, c->stream));
  return ELBM_OK;
}

int elbm_load_state(elbm_ctx* c, const void* pop_dev, int64_t t) {
  if (!c) return ELBM_EINVAL;
  if (!pop_dev || t < 0) return fail(c, ELBM_EINVAL, "bad arguments");
  const size_t bytes = 27 * (size_t)c->N * storage_bytes(c->p.storage);
  c->pop[0] = c->own[0];
  c->pop[1] = c->own[1];
  HIP_OK(c, hipMemcpyAsync(c->pop[c->cur], pop_dev, bytes, hipMemcpyDeviceToDevice, c->stream));
  HIP_OK(c, free_reanchor(c, t));
  c->t = t;
  HIP_OK(c, diag_reset(c, true));
  if (c->flags) return geo_init(c);
  return ELBM_OK;
}

int elbm_adjoint_step(elbm_ctx* c, int64_t t, void* pop_t_dev, const float* lam_in_dev, float* lam_out_dev,
                      const double* w_force, float* gF_dev) {
  if (!c) return ELBM_EINVAL;
  if (!c->adj_gUR) return fail(c, ELBM_ESTATE, "context created without ELBM_FLAG_ADJOINT");
  if (!pop_t_dev || !lam_in_dev || !lam_out_dev || t < 0) return fail(c, ELBM_EINVAL, "bad arguments");
  if (lam_in_dev == lam_out_dev) return fail(c, ELBM_EINVAL, "lam_in and lam_out must not alias");
  if (gF_dev && !c->bodyforce) return fail(c, ELBM_ESTATE, "gF requested but no body-force field is bound");
  if (c->p.flags & ELBM_FLAG_STREAM_ONLY) return fail(c, ELBM_ESTATE, "no adjoint in stream-only mode");
  c->slab_valid = false;  // the reverse step recomputes U^t, R^t of its own state
  HIP_OK(c, launch_adjoint(c, t, pop_t_dev, lam_in_dev, lam_out_dev, w_force, gF_dev));
  return ELBM_OK;
}

int elbm_adjoint_param_grad(elbm_ctx* c, double* g_amp, int32_t reset) {
  if (!c) return ELBM_EINVAL;
  if (!c->adj_gamp) return fail(c, ELBM_ESTATE, "context created without ELBM_FLAG_ADJOINT");
  if (!g_amp) return fail(c, ELBM_EINVAL, "g_amp is NULL");
  HIP_OK(c, hipStreamSynchronize(c->stream));
  double h[ELBM_MAX_BODIES];
  HIP_OK(c, hipMemcpy(h, c->adj_gamp, sizeof h, hipMemcpyDeviceToHost));
  for (int k = 0; k < c->nb; ++k) g_amp[k] = h[k];
  if (reset) HIP_OK(c, hipMemsetAsync(c->adj_gamp, 0, sizeof(double) * ELBM_MAX_BODIES, c->stream));
  return ELBM_OK;
}

int elbm_set_timing(elbm_ctx* c, int32_t enable) {
  if (!c) return ELBM_EINVAL;
  c->ev_used = 0;
  c->timing = enable != 0;
  if (c->timing && !c->ev) {
    const int64_t cap = 8192;
    c->ev = (hipEvent_t*)calloc(2 * cap, sizeof(hipEvent_t));
    if (!c->ev) return fail(c, ELBM_EINVAL, "out of host memory");
    c->ev_cap = cap;
    for (int64_t k = 0; k < 2 * cap; ++k) HIP_OK(c, hipEventCreate(&c->ev[k]));
  }
  return ELBM_OK;
}

int elbm_get_timing(elbm_ctx* c, double* sweep_ms, int64_t* launches) {
  if (!c || !sweep_ms || !launches) return ELBM_EINVAL;
  double total = 0.0;
  if (c->ev_used) HIP_OK(c, hipEventSynchronize(c->ev[2 * c->ev_used - 1]));
  for (int64_t k = 0; k < c->ev_used; ++k) {
    float ms = 0.f;
    HIP_OK(c, hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]));
    total += ms;
  }
  *sweep_ms = total;
  *launches = c->ev_used;
  return ELBM_OK;
}

const char* elbm_last_error(const elbm_ctx* c) { return c ? c->err : g_create_err; }

int elbm_collide_nodes(const float* f_in_dev, float* f_out_dev, float* gamma_dev, const float* F_dev, int64_t n,
                       double nu, double fp64_threshold, uint32_t flags, void* stream) {
  if (!f_in_dev || !f_out_dev || n < 0 || !(nu > 0.0)) return fail(nullptr, ELBM_EINVAL, "bad arguments");
  if ((flags & ELBM_FLAG_EXACT_GAMMA) && (flags & ELBM_FLAG_LBGK)) return fail(nullptr, ELBM_EINVAL, "bad flags");
  if ((flags & ELBM_FLAG_CENTRAL) && (flags & (ELBM_FLAG_EXACT_GAMMA | ELBM_FLAG_LBGK)))
    return fail(nullptr, ELBM_EINVAL, "ELBM_FLAG_CENTRAL goes with the analytic stabiliser");
  if (n == 0) return ELBM_OK;
  const double beta = 1.0 / (6.0 * nu + 1.0);
  const double thr = fp64_threshold < 0.0 ? -1.0 : (fp64_threshold == 0.0 ? 1e-12 : fp64_threshold);
  int stab = (flags & ELBM_FLAG_EXACT_GAMMA) ? STAB_EXACT : ((flags & ELBM_FLAG_LBGK) ? STAB_LBGK : STAB_KBC);
  if (flags & ELBM_FLAG_CENTRAL) stab |= STAB_CENTRAL;
  hipError_t e = launch_collide_nodes(f_in_dev, f_out_dev, gamma_dev, F_dev, n, beta, thr, stab, (hipStream_t)stream);
  if (e != hipSuccess) return fail(nullptr, ELBM_EDEVICE, "collide: %s", hipGetErrorString(e));
  return ELBM_OK;
}


}  // extern "C"

// ---------------------------------------------------------------------------------------------
// elbm_step_periodic_noalloc: one step of a periodic box without bodies for callers that cannot
// allocate device memory.  elbm_step keeps the FP64 recomputation queue (one entry per node) and
// its counters in the caller's workspace; here they live in the file-scope device array below,
// one copy per GPU, held from the library's first load on that GPU until the process ends.  Its
// device address is taken once per device with hipGetSymbolAddress; host code passes only that
// address to kernels (the array's own name is a host-side stand-in, not a device address).
namespace {
constexpr size_t NOALLOC_COUNTER_BYTES = 256;
constexpr int64_t NOALLOC_MAX_NODES = (int64_t)1 << 23;  // 8 388 608 nodes, e.g. 256 x 256 x 128
constexpr size_t NOALLOC_BYTES = NOALLOC_COUNTER_BYTES + sizeof(uint32_t) * (size_t)NOALLOC_MAX_NODES;
constexpr int NOALLOC_MAX_DEVICES = 64;
static_assert(sizeof(DevCounters) <= NOALLOC_COUNTER_BYTES, "counters must fit their slot");
}  // namespace

// [counters: NOALLOC_COUNTER_BYTES][FP64 queue: one uint32 per node, NOALLOC_MAX_NODES entries]
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
std::mutex g_noalloc_mu;
char* g_noalloc_ptr[NOALLOC_MAX_DEVICES];  // device address of `scratch` on each device, or null

// The per-call counters must start at zero: a kernel clears them (no memset node, so the call
// can be captured into a graph).
__global__ void k_noalloc_clear(uint32_t* counters, int n) {
  for (int k = threadIdx.x; k < n; k += blockDim.x) counters[k] = 0u;
}

// Address of the scratch array on the current device (taken on the first call there).
hipError_t noalloc_scratch(char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_noalloc_ptr[dev] = (char*)p;
  }
  *out = g_noalloc_ptr[dev];
  return hipSuccess;
}
}  // namespace

extern "C" int elbm_step_periodic_noalloc(const elbm_params* p, const void* pop_in_dev, void* pop_out_dev,
                                          void* stream) {
  const int rc = validate(p, g_create_err);
  if (rc) return rc;
  if (!pop_in_dev || !pop_out_dev) return fail(nullptr, ELBM_EINVAL, "pop_in_dev and pop_out_dev must be set");
  if (p->bc_x != ELBM_BC_PERIODIC || p->max_bodies != 0)
    return fail(nullptr, ELBM_EINVAL, "the allocation-free step serves a periodic box without bodies");
  const uint32_t allowed = ELBM_FLAG_NO_FP64 | ELBM_FLAG_EXACT_GAMMA | ELBM_FLAG_LBGK | ELBM_FLAG_CENTRAL |
                           ELBM_FLAG_STREAM_ONLY;
  if (p->flags & ~allowed)
    return fail(nullptr, ELBM_EINVAL, "flags 0x%x: no body force or adjoint in the allocation-free step",
                p->flags & ~allowed);
  const int64_t N = (int64_t)p->nx * p->ny * p->nz;
  if (N > NOALLOC_MAX_NODES)
    return fail(nullptr, ELBM_EINVAL, "%lld nodes exceed the %lld of the allocation-free step's scratch",
                (long long)N, (long long)NOALLOC_MAX_NODES);
  const size_t bytes = 27 * (size_t)N * storage_bytes(p->storage);
  const char* a0 = (const char*)pop_in_dev;
  const char* b0 = (const char*)pop_out_dev;
  if (a0 < b0 + bytes && b0 < a0 + bytes) return fail(nullptr, ELBM_EINVAL, "pop_in_dev and pop_out_dev overlap");
  char* scr = nullptr;
  hipError_t e = noalloc_scratch(&scr);
  if (e != hipSuccess) return fail(nullptr, ELBM_EDEVICE, "scratch address: %s", hipGetErrorString(e));
  // a context on the host stack: the same sweep and FP64 kernels as elbm_step, their queue and
  // counters in the scratch array, the populations the caller's
  elbm_ctx c{};
  c.p = *p;
  c.stream = (hipStream_t)stream;
  c.N = N;
  c.beta = 1.0 / (6.0 * p->nu + 1.0);
  c.fp64_thr = p->fp64_threshold > 0.0 ? p->fp64_threshold : 1e-12;
  c.stab = (p->flags & ELBM_FLAG_EXACT_GAMMA) ? STAB_EXACT : ((p->flags & ELBM_FLAG_LBGK) ? STAB_LBGK : STAB_KBC);
  if (p->flags & ELBM_FLAG_CENTRAL) c.stab |= STAB_CENTRAL;
  c.pop[0] = const_cast<void*>(pop_in_dev);
  c.pop[1] = pop_out_dev;
  c.cur = 0;
  c.lay = pop_layout(c.p);
  c.cnt = (DevCounters*)scr;
  c.fix_list = (int32_t*)(scr + NOALLOC_COUNTER_BYTES);
  c.fix_par = 0;
  hipLaunchKernelGGL(k_noalloc_clear, dim3(1), dim3(64), 0, c.stream, (uint32_t*)scr,
                     (int)(NOALLOC_COUNTER_BYTES / sizeof(uint32_t)));
  e = hipGetLastError();
  if (e == hipSuccess) e = launch_sweep(&c);
  if (e == hipSuccess) e = launch_fixup(&c);
  if (e != hipSuccess) return fail(nullptr, ELBM_EDEVICE, "allocation-free step: %s", hipGetErrorString(e));
  return ELBM_OK;
}
