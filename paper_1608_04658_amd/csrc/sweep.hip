// sweep.hip -- the fused bulk sweep of the D3Q27 KBC step on gfx950: pull streaming, moments,
// entropic equilibrium, KBC collision with the per-node stabiliser, store (Sec. II,
// eqs. kineticEq, kbc_relax, feq_min), plus the FP64 recomputation of near-equilibrium nodes.
//
// One thread per node, x fastest inside a wavefront: every load and store of a population
// array is a contiguous 64-lane access (the +-x shifted loads straddle one extra cache line,
// which the neighbouring lanes of the same workgroup bring into L2).  Each direction of each
// lattice row is one contiguous run in either population layout (PopLayout), so every population
// streams through HBM exactly once per step.
#include "context.hpp"
#include "lanes_dev.hpp"

namespace elbm {

struct SweepArgs {
  const void* A;
  void* B;
  const uint8_t* flags;
  const float* F;
  uint32_t* fix_list;
  uint32_t* fix_count;  // this step's FP64 queue length
  uint32_t* fix_clear;  // the other parity's, cleared by the fix-up kernel for the next step
  DevCounters* diag;    // failure flag and gamma range
  int32_t stats;        // 1: record the gamma range (listed nodes excluded: the wall kernel's)
  float* slab_next;  // [4][nz][ny][3] staging of U, R for x < 3 (written when slab is set)
  PopLayout lay;
  int32_t nx, ny, nz;
  uint32_t N;
  float beta, inv_beta, thr;
  int32_t channel;
  int32_t fp64;
  int32_t stream_only;
  int32_t slab;    // channel mode: the producers of A^{t+1} write U, R of the inlet slab x < 3
  int32_t remap;   // 1-D grid of tiles, each XCD taking a contiguous chunk (see sweep_shape)
  int32_t gx, gy;  // tiles along x and y
  int32_t tiles;   // gx * gy * nz
};

// Source coordinates of the pull for each velocity component, split for the addressing: the
// element offset zb[cz+1] of the first row of source plane z - cz (uniform over a workgroup of the
// bulk sweep, so the per-direction bases stay scalar) and the in-plane offsets
// lo[3 (cy+1) + (cx+1)] = (y - cy) rs + (x - cx) (elements, < 2^32 / 4 by the plane-size limit of
// the context); periodic in y and z; periodic in x or, in channel mode, clamped (the outlet copy;
// x = 0 is never gathered by the bulk path).
__device__ __forceinline__ void gather_offsets(int x, int y, int z, const SweepArgs& a, int64_t (&zb)[3],
                                               uint32_t (&lo)[9]) {
  int xs[3];
  if (a.channel) {
    xs[0] = min(x + 1, a.nx - 1);
    xs[2] = max(x - 1, 0);
  } else {
    xs[0] = x + 1 == a.nx ? 0 : x + 1;
    xs[2] = x == 0 ? a.nx - 1 : x - 1;
  }
  xs[1] = x;
  const int ym = (y + 1 == a.ny) ? 0 : y + 1, yp = (y == 0) ? a.ny - 1 : y - 1;
  const int zm = (z + 1 == a.nz) ? 0 : z + 1, zp = (z == 0) ? a.nz - 1 : z - 1;
  const int ys[3] = {ym, y, yp};  // source y for cy = -1, 0, +1
  const int zs[3] = {zm, z, zp};
  const uint32_t rs = (uint32_t)a.lay.rs;
#pragma unroll
  for (int k = 0; k < 3; ++k) zb[k] = (int64_t)zs[k] * a.ny * a.lay.rs;
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int k = 0; k < 3; ++k) lo[3 * j + k] = (uint32_t)ys[j] * rs + (uint32_t)xs[k];
}

// Element i of the pull: base of direction i in source plane z - cz_i, plus the in-plane byte
// offset in 32 bits.
template <typename E>
__device__ __forceinline__ const E* pull_ptr(const E* A, const SweepArgs& a, const int64_t (&zb)[3],
                                             const uint32_t (&lo)[9], int i) {
  const E* base = A + (zb[cz(i) + 1] + (int64_t)i * a.lay.si);
  return (const E*)((const char*)base + lo[3 * (cy(i) + 1) + cx(i) + 1] * (uint32_t)sizeof(E));
}

// The plain collision (no body force; the analytic stabiliser or LBGK) runs at five waves per SIMD
// (at most 102 VGPRs): the compiler's own choice is 111 VGPRs, four waves, which measured about 0.5 %
// slower for the 2-byte sweeps.  The other forms need more registers and keep the compiler's choice
// (bounding them spills to scratch).
template <bool FORCE, int STAB>
constexpr int sweep_min_waves() { return (FORCE || (STAB & 3) == STAB_EXACT || (STAB & STAB_CENTRAL)) ? 1 : 5; }

template <int S, bool FLAGS, bool FORCE, int STAB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sweep_min_waves<FORCE, STAB>())))
void k_sweep(const SweepArgs a) {
  using C = Codec<S>;
  using E = typename C::E;
  int tx = blockIdx.x, ty = blockIdx.y, z = blockIdx.z;
  if (a.remap) {
    // workgroups are dispatched round-robin over the 8 XCDs; give each XCD a contiguous range of
    // tiles, so that the x-neighbouring tiles of a row, which share the cache lines at their
    // edges, run on the same XCD (same L2) at about the same time
    const int b = blockIdx.x, xcd = b & 7, j = b >> 3, q = a.tiles >> 3, r = a.tiles & 7;
    const int t = (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + j;
    tx = t % a.gx;
    ty = (t / a.gx) % a.gy;
    z = t / (a.gx * a.gy);
  }
  const int x = tx * blockDim.x + threadIdx.x;
  const int y = ty * blockDim.y + threadIdx.y;
  if (x >= a.nx || y >= a.ny) return;
  const uint32_t n = (uint32_t)((z * a.ny + y) * a.nx + x);
  // the flag byte is loaded together with the 27 gathers (all sources are in range for every
  // node), so that waiting for it does not delay them; solid nodes then leave.  Listed nodes
  // (FL_SPECIAL) run through and store like the others: the wall kernel, launched after the sweep
  // on the same stream, overwrites all 27 of their populations, and storing them here keeps every
  // written cache line whole (a masked lane per row, as at the inlet face, turns each of the row's
  // line writes into a partial one: 600 against 543 us on a 384x192x192 channel).  They enter
  // neither the FP64 queue nor the inlet-slab staging, which the wall kernel owns for them.
  const uint8_t fl = FLAGS ? a.flags[n] : (uint8_t)0;
  const bool skip = FLAGS && (fl & FL_SOLID);
  const bool listed = FLAGS && (fl & FL_SPECIAL);
  int64_t zb[3];
  uint32_t lo[9];
  gather_offsets(x, y, z, a, zb, lo);
  const E* __restrict__ A = (const E*)a.A;
  float f[27];  // deviations f - W
#pragma unroll
  for (int i = 0; i < 27; ++i) f[i] = C::load_dev(pull_ptr(A, a, zb, lo, i));
  if (FLAGS) {
    // compiler-only barrier: keeps the gathers issued above the branch (no machine instruction)
    __asm__ volatile("" ::: "memory");
    if (skip) return;
  }
  if (!a.stream_only) {
    float Fx = 0.f, Fy = 0.f, Fz = 0.f;
    if (FORCE) {
      Fx = a.F[n];
      Fy = a.F[a.N + n];
      Fz = a.F[2 * (size_t)a.N + n];
    }
    const KbcOut<float> r = kbc_collide<float, FORCE, STAB>(f, a.beta, a.inv_beta, Fx, Fy, Fz);
    // failure detection: a non-finite state, or one where the entropic equilibrium is not positive
    // (the tests of r.dom); one ballot per wavefront, an atomic only where a node fails.  Listed
    // nodes pulled from solid nodes here and are checked by the wall kernel.
    const uint64_t bad = __ballot(!r.dom && !listed);
    if (bad && __lane_id() == (uint32_t)(__ffsll((unsigned long long)bad) - 1)) atomicOr(&a.diag->nonfinite, 1u);
    if (a.stats) {
      // gamma range over the wavefront's active lanes (exec-aware reduction), one atomic pair
      const unsigned long long act = __ballot(1);
      const uint32_t lo = __reduce_min_sync(act, listed ? 0xFFFFFFFFu : f32_key(r.gamma));
      const uint32_t hi = __reduce_max_sync(act, listed ? 0u : f32_key(r.gamma));
      if (__lane_id() == (uint32_t)(__ffsll(act) - 1)) {
        atomicMin(&a.diag->gamma_lo, lo);
        atomicMax(&a.diag->gamma_hi, hi);
      }
    }
    if (a.fp64) {
      // one queue reservation per wavefront for all of its nodes that need the FP64 collision
      const bool q = needs_fp64(r, a.thr) && !listed;
      const uint64_t m = __ballot(q);
      if (m) {
        const int lane = (int)__lane_id();
        const int leader = __ffsll((unsigned long long)m) - 1;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(a.fix_count, (uint32_t)__popcll(m));
        base = __shfl(base, leader);
        if (q) a.fix_list[base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = n;
      }
    }
    if (FLAGS && a.slab && x < 3 && !listed)
      macro_from_post<S, FORCE>(f, Fx, Fy, Fz, a.slab_next, (size_t)3 * a.ny * a.nz, slab_index(x, y, z, a.ny));
  }
  // Non-temporal stores (the next step reads this buffer only after the whole sweep, so keeping the
  // write stream out of the caches wins; measured for FP32 and for 2-byte storage alike), each
  // through a buffer resource on its direction's base in this plane (scalar registers) with the
  // lane's 32-bit in-plane byte offset: no per-store 64-bit address arithmetic on the vector ALU,
  // which the ALU-bound 2-byte sweeps feel.
  E* __restrict__ B = (E*)a.B;
  const uint32_t off = ((uint32_t)y * (uint32_t)a.lay.rs + (uint32_t)x) * (uint32_t)sizeof(E);
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    E v;
    C::store_dev(&v, f[i]);
    const __amdgpu_buffer_rsrc_t dst =
        __builtin_amdgcn_make_buffer_rsrc((void*)(B + (zb[1] + (int64_t)i * a.lay.si)), (short)0, BUF_ALL, BUF_WORD3);
    if constexpr (sizeof(E) == 4) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), dst, off, 0, BUF_NT);
    else __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), dst, off, 0, BUF_NT);
  }
}

// FP64 recomputation of the nodes whose <dh|dh> fell below the FP32 threshold: the same gather
// and the same collision in double precision, rounded once on store.  Two forms, chosen on the
// device from the queue length (uniform over the grid):
//  - a short queue (a few thousand nodes, as around a moving body in a stream) is bound by the
//    chain of dependent FP64 operations of one node: one node per group of 32 lanes, lane i < 27
//    owning direction i (kbc_collide_lanes, sums as butterfly reductions in the group); sphere384,
//    ~2.7 k nodes: 8.6 us against 17.4 us with one thread per node;
//  - a long queue (a fluid largely at rest, ~10^5 nodes) is bound by FP64 throughput, where the
//    shuffles of the lane form cost more than they save: one node per thread (the settling sphere:
//    30 us against 191 us in the lane form).
// The queue length of the other parity is cleared here for the next step, so the kernel is
// launched every step without a host round trip.
constexpr uint32_t FIX_LANES_MAX = 8192;  // queue lengths served by the lane form

template <int S, bool FORCE, int STAB>
__global__ __launch_bounds__(256) void k_fixup(const SweepArgs a) {
  using C = Codec<S>;
  using E = typename C::E;
  const uint32_t count = __atomic_load_n(a.fix_count, __ATOMIC_RELAXED);
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.fix_clear = 0u;
  const E* __restrict__ A = (const E*)a.A;
  E* __restrict__ B = (E*)a.B;
  const double beta = (double)a.beta;
  if (count <= FIX_LANES_MAX) {
    const int lane = threadIdx.x & (GROUP - 1);
    const bool own = lane < 27;
    const int i = own ? lane : 13;
    const uint32_t per_block = blockDim.x / GROUP;
    for (uint32_t k = blockIdx.x * per_block + threadIdx.x / GROUP; k < count; k += gridDim.x * per_block) {
      const uint32_t e = a.fix_list[k];
      const uint32_t n = e & ~FIX_PRE;
      if (n >= a.N) continue;  // never written so; guards the accesses below (uniform over the group)
      const int x = (int)(n % (uint32_t)a.nx);
      const int y = (int)((n / (uint32_t)a.nx) % (uint32_t)a.ny);
      const int z = (int)(n / ((uint32_t)a.nx * (uint32_t)a.ny));
      double d = 0.0;  // deviation f_i - W_i of this lane's direction
      if (own) {
        if (e & FIX_PRE) {
          // wall node: its reconstructed pre-collision deviations were left in B
          d = (double)C::load_dev(B + pop_off(a.lay, i, x, y, z));
        } else {
          // the pull of the bulk sweep: x - c_i, periodic in y and z, in x periodic or clamped
          int sx = x - cx(i), sy = y - cy(i), sz = z - cz(i);
          if (a.channel) sx = min(max(sx, 0), a.nx - 1);
          else sx = sx < 0 ? sx + a.nx : (sx >= a.nx ? sx - a.nx : sx);
          sy = sy < 0 ? sy + a.ny : (sy >= a.ny ? sy - a.ny : sy);
          sz = sz < 0 ? sz + a.nz : (sz >= a.nz ? sz - a.nz : sz);
          d = (double)C::load_dev(A + pop_off(a.lay, i, sx, sy, sz));
        }
      }
      double Fx = 0, Fy = 0, Fz = 0;
      if (FORCE) {
        Fx = a.F[n];
        Fy = a.F[a.N + n];
        Fz = a.F[2 * (size_t)a.N + n];
      }
      KbcOut<double> r;
      const double post = kbc_collide_lanes<double, FORCE, STAB>(lane, d, beta, 1.0 / beta, Fx, Fy, Fz, r);
      const float out = (float)post;
      if (own) C::store_dev(B + pop_off(a.lay, i, x, y, z), out);
      if (a.slab && x < 3) {
        // U, R of the stored state for the inlet slab, summed in direction order on the first lane
        float o[27];
#pragma unroll
        for (int j = 0; j < 27; ++j) o[j] = __shfl(out, j, GROUP);
        if (lane == 0)
          macro_from_post<S, FORCE>(o, (float)Fx, (float)Fy, (float)Fz, a.slab_next, (size_t)3 * a.ny * a.nz,
                                    slab_index(x, y, z, a.ny));
      }
    }
    return;
  }
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < count; k += gridDim.x * blockDim.x) {
    const uint32_t e = a.fix_list[k];
    const uint32_t n = e & ~FIX_PRE;
    if (n >= a.N) continue;  // never written so; guards the accesses below
    const int x = (int)(n % (uint32_t)a.nx);
    const int y = (int)((n / (uint32_t)a.nx) % (uint32_t)a.ny);
    const int z = (int)(n / ((uint32_t)a.nx * (uint32_t)a.ny));
    double f[27];  // deviations f - W
    if (e & FIX_PRE) {
#pragma unroll
      for (int i = 0; i < 27; ++i) f[i] = (double)C::load_dev(B + pop_off(a.lay, i, x, y, z));
    } else {
      int64_t zb[3];
      uint32_t lo[9];
      gather_offsets(x, y, z, a, zb, lo);
#pragma unroll
      for (int i = 0; i < 27; ++i) f[i] = (double)C::load_dev(pull_ptr(A, a, zb, lo, i));
    }
    double Fx = 0, Fy = 0, Fz = 0;
    if (FORCE) {
      Fx = a.F[n];
      Fy = a.F[a.N + n];
      Fz = a.F[2 * (size_t)a.N + n];
    }
    kbc_collide<double, FORCE, STAB>(f, beta, 1.0 / beta, Fx, Fy, Fz);
    float out[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) {
      out[i] = (float)f[i];
      C::store_dev(B + pop_off(a.lay, i, x, y, z), out[i]);
    }
    if (a.slab && x < 3)
      macro_from_post<S, FORCE>(out, (float)Fx, (float)Fy, (float)Fz, a.slab_next, (size_t)3 * a.ny * a.nz,
                                slab_index(x, y, z, a.ny));
  }
}

// Population layout: rows interleaved for every storage format.  Measured on the bulk sweep against
// structure of arrays (same kernel, only the strides differ): 512^3 FP32 6.04-6.07 TB/s against
// 5.36-5.53, FP16 5.05-5.07 against 4.79-4.81 (with the tile shapes below), BF16 4.87-4.91 against
// 4.74-4.76; 384-wide channels +3-5 %; 256^3 equal within noise.
PopLayout pop_layout(const elbm_params& p) {
  PopLayout L;
  L.nx = p.nx;
  L.ny = p.ny;
  L.pad = 0;
  L.interleaved = 1;
  L.rs = 27 * (int64_t)p.nx;
  L.si = p.nx;
  return L;
}

static SweepArgs sweep_args(elbm_ctx* c) {
  SweepArgs a;
  a.A = c->pop[c->cur];
  a.B = c->pop[c->cur ^ 1];
  a.flags = c->flags;
  a.F = c->bodyforce;
  a.fix_list = (uint32_t*)c->fix_list;
  a.fix_count = &c->cnt->fix_count[c->fix_par];
  a.fix_clear = &c->cnt->fix_count[c->fix_par ^ 1];
  a.diag = c->cnt;
  a.stats = c->gamma_stats ? 1 : 0;
  a.nx = c->p.nx;
  a.ny = c->p.ny;
  a.nz = c->p.nz;
  a.N = (uint32_t)c->N;
  a.beta = (float)c->beta;
  a.inv_beta = (float)(1.0 / c->beta);
  a.thr = (float)c->fp64_thr;
  a.channel = c->p.bc_x == ELBM_BC_CHANNEL;
  a.fp64 = !(c->p.flags & ELBM_FLAG_NO_FP64) && !(c->p.flags & ELBM_FLAG_STREAM_ONLY);
  a.stream_only = (c->p.flags & ELBM_FLAG_STREAM_ONLY) != 0;
  a.slab_next = c->slab_next;
  a.lay = c->lay;
  a.slab = (c->flags != nullptr && a.channel && !a.stream_only && c->slab_next) ? 1 : 0;
  a.remap = 0;
  a.gx = a.gy = a.tiles = 0;
  return a;
}

// Launch shape: 256-thread workgroups, x-extent bx, the rest along y.  Rows up to 256 wide: the
// widest power of two <= 256 dividing nx (at least 32).  Longer rows, measured with the interleaved
// layout: bx = 128 where it divides nx and 256 does not (384: 6.03-6.06 TB/s against 4.74-4.79 with
// a ragged 256-wide tile), bx = 256 where it divides nx (512^3 FP16 5.05-5.07 against 4.86-4.98 with
// 128), except 512-wide FP32 rows, which keep 128 (256-wide tiles 5.68-6.05 TB/s, not distinguishable
// in the noise); bx = 256 with a ragged last tile otherwise (1600-wide channel: 5.42-5.50 TB/s against
// 4.86-4.95 with 128 and 4.90-4.95 with 64).
// Tile order: FP32 rows of four or more tiles run in an XCD-contiguous order, so that the tiles of a
// row, which share the cache lines at their edges, sit on one XCD's L2 (512^3: 5.72-5.73 TB/s
// against 5.27-5.28 in dispatch order, reads 1.0003x the algorithmic bytes; 1600-wide channel:
// 9.66-9.67 ms against 9.83-10.18); fewer tiles per row (384: 533-539 us against 558 us remapped)
// and the 2-byte forms (4.67 against 5.20 TB/s) keep the dispatch order.  Workgroups are dispatched
// round-robin over the 8 XCDs; k_sweep remaps the 1-D grid so that each XCD takes a contiguous range
// of tiles.  The 1-D tile grid also serves shapes beyond the 65535 limit of the y and z grid extents.
static void sweep_shape(SweepArgs& a, int storage, dim3& grid, dim3& block) {
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  int bx;
  if (nx <= 256) {
    bx = 256;
    while (bx > 32 && (nx % bx) != 0) bx >>= 1;
    if (nx < bx) bx = 32;
  } else if (nx % 256 == 0) {
    bx = (storage == ELBM_STORAGE_F32 && nx == 512) ? 128 : 256;
  } else if (nx % 128 == 0 && nx <= 512) {
    bx = 128;
  } else {
    bx = 256;
  }
  const int by = 256 / bx;
  block = dim3(bx, by, 1);
  a.gx = (nx + bx - 1) / bx;
  a.gy = (ny + by - 1) / by;
  a.tiles = a.gx * a.gy * nz;
  const bool remap = (storage == ELBM_STORAGE_F32 && a.gx >= 4) || a.gy > 65535 || nz > 65535;
  a.remap = remap ? 1 : 0;
  grid = remap ? dim3(a.tiles, 1, 1) : dim3(a.gx, a.gy, nz);
}

template <int S, int STAB>
static hipError_t sweep_st(elbm_ctx* c, const SweepArgs& a, dim3 g, dim3 b) {
  const bool flags = c->flags != nullptr;
  const bool force = c->bodyforce != nullptr;
  if (flags && force) hipLaunchKernelGGL((k_sweep<S, true, true, STAB>), g, b, 0, c->stream, a);
  else if (flags) hipLaunchKernelGGL((k_sweep<S, true, false, STAB>), g, b, 0, c->stream, a);
  else if (force) hipLaunchKernelGGL((k_sweep<S, false, true, STAB>), g, b, 0, c->stream, a);
  else hipLaunchKernelGGL((k_sweep<S, false, false, STAB>), g, b, 0, c->stream, a);
  return hipGetLastError();
}

template <int S>
static hipError_t sweep_s(elbm_ctx* c, const SweepArgs& a, dim3 g, dim3 b) {
  switch (c->stab) {
    case STAB_EXACT: return sweep_st<S, STAB_EXACT>(c, a, g, b);
    case STAB_LBGK: return sweep_st<S, STAB_LBGK>(c, a, g, b);
    case STAB_KBC | STAB_CENTRAL: return sweep_st<S, STAB_KBC | STAB_CENTRAL>(c, a, g, b);
    default: return sweep_st<S, STAB_KBC>(c, a, g, b);
  }
}

hipError_t launch_sweep(elbm_ctx* c) {
  SweepArgs a = sweep_args(c);
  dim3 g, b;
  sweep_shape(a, c->p.storage, g, b);
  switch (c->p.storage) {
    case ELBM_STORAGE_F32: return sweep_s<ELBM_STORAGE_F32>(c, a, g, b);
    case ELBM_STORAGE_F16: return sweep_s<ELBM_STORAGE_F16>(c, a, g, b);
    default: return sweep_s<ELBM_STORAGE_BF16>(c, a, g, b);
  }
}

template <int S, int STAB>
static hipError_t fixup_st(elbm_ctx* c, const SweepArgs& a) {
  // the queue length is known only on the device: enough workgroups for two waves per SIMD
  const dim3 g(512), b(256);
  if (c->bodyforce) hipLaunchKernelGGL((k_fixup<S, true, STAB>), g, b, 0, c->stream, a);
  else hipLaunchKernelGGL((k_fixup<S, false, STAB>), g, b, 0, c->stream, a);
  return hipGetLastError();
}

template <int S>
static hipError_t fixup_s(elbm_ctx* c, const SweepArgs& a) {
  switch (c->stab) {
    case STAB_EXACT: return fixup_st<S, STAB_EXACT>(c, a);
    case STAB_LBGK: return fixup_st<S, STAB_LBGK>(c, a);
    case STAB_KBC | STAB_CENTRAL: return fixup_st<S, STAB_KBC | STAB_CENTRAL>(c, a);
    default: return fixup_st<S, STAB_KBC>(c, a);
  }
}

hipError_t launch_fixup(elbm_ctx* c) {
  const SweepArgs a = sweep_args(c);
  if (!a.fp64) return hipSuccess;
  switch (c->p.storage) {
    case ELBM_STORAGE_F32: return fixup_s<ELBM_STORAGE_F32>(c, a);
    case ELBM_STORAGE_F16: return fixup_s<ELBM_STORAGE_F16>(c, a);
    default: return fixup_s<ELBM_STORAGE_BF16>(c, a);
  }
}

// ---------------------------------------------------------------------------------------------
// Conversions between FP64 population arrays and the storage format.
template <int S> __device__ __forceinline__ void store_d(typename Codec<S>::E* p, double v, int i);
template <> __device__ __forceinline__ void store_d<ELBM_STORAGE_F32>(float* p, double v, int i) {
  *p = (float)(v - wd(i));
}
template <> __device__ __forceinline__ void store_d<ELBM_STORAGE_F16>(_Float16* p, double v, int i) {
  float d = (float)(v - wd(i));
  __asm__("" : "+v"(d));  // round the binary32 deviation, as every other store does (see f32_to_bf16_rne)
  *p = (_Float16)d;
}
template <> __device__ __forceinline__ void store_d<ELBM_STORAGE_BF16>(uint16_t* p, double v, int i) {
  *p = f32_to_bf16_rne((float)(v - wd(i)));
}
template <int S> __device__ __forceinline__ double load_d(const typename Codec<S>::E* p, int i);
template <> __device__ __forceinline__ double load_d<ELBM_STORAGE_F32>(const float* p, int i) {
  return (double)*p + wd(i);
}
template <> __device__ __forceinline__ double load_d<ELBM_STORAGE_F16>(const _Float16* p, int i) {
  return (double)(float)*p + wd(i);
}
template <> __device__ __forceinline__ double load_d<ELBM_STORAGE_BF16>(const uint16_t* p, int i) {
  return (double)__uint_as_float(((uint32_t)*p) << 16) + wd(i);
}

template <int S>
__global__ __launch_bounds__(256) void k_init_eq(typename Codec<S>::E* A, PopLayout L, const double* rho,
                                                 const double* u, int64_t N) {
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
    double fe[27];
    feq_all(rho ? rho[n] : 1.0, u[n], u[N + n], u[2 * N + n], fe);
    const int64_t b = pop_base_n(L, n);
#pragma unroll
    for (int i = 0; i < 27; ++i) store_d<S>(A + b + i * L.si, fe[i], i);
  }
}

template <int S>
__global__ __launch_bounds__(256) void k_write_pop(typename Codec<S>::E* A, PopLayout L, const double* src, int64_t N) {
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = pop_base_n(L, n);
#pragma unroll
    for (int i = 0; i < 27; ++i) store_d<S>(A + b + i * L.si, src[i * N + n], i);
  }
}

template <int S>
__global__ __launch_bounds__(256) void k_read_pop(const typename Codec<S>::E* A, PopLayout L, double* dst, int64_t N) {
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = pop_base_n(L, n);
#pragma unroll
    for (int i = 0; i < 27; ++i) dst[i * N + n] = load_d<S>(A + b + i * L.si, i);
  }
}

static dim3 grid_1d(int64_t N) {
  int64_t b = (N + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

hipError_t launch_init_eq(elbm_ctx* c, const double* rho, const double* u) {
  void* A = c->pop[c->cur];
  switch (c->p.storage) {
    case ELBM_STORAGE_F32:
      hipLaunchKernelGGL(k_init_eq<ELBM_STORAGE_F32>, grid_1d(c->N), dim3(256), 0, c->stream, (float*)A, c->lay, rho, u, c->N);
      break;
    case ELBM_STORAGE_F16:
      hipLaunchKernelGGL(k_init_eq<ELBM_STORAGE_F16>, grid_1d(c->N), dim3(256), 0, c->stream, (_Float16*)A, c->lay, rho, u, c->N);
      break;
    default:
      hipLaunchKernelGGL(k_init_eq<ELBM_STORAGE_BF16>, grid_1d(c->N), dim3(256), 0, c->stream, (uint16_t*)A, c->lay, rho, u, c->N);
  }
  return hipGetLastError();
}

hipError_t launch_write_pop(elbm_ctx* c, const double* src) {
  void* A = c->pop[c->cur];
  switch (c->p.storage) {
    case ELBM_STORAGE_F32:
      hipLaunchKernelGGL(k_write_pop<ELBM_STORAGE_F32>, grid_1d(c->N), dim3(256), 0, c->stream, (float*)A, c->lay, src, c->N);
      break;
    case ELBM_STORAGE_F16:
      hipLaunchKernelGGL(k_write_pop<ELBM_STORAGE_F16>, grid_1d(c->N), dim3(256), 0, c->stream, (_Float16*)A, c->lay, src, c->N);
      break;
    default:
      hipLaunchKernelGGL(k_write_pop<ELBM_STORAGE_BF16>, grid_1d(c->N), dim3(256), 0, c->stream, (uint16_t*)A, c->lay, src, c->N);
  }
  return hipGetLastError();
}

hipError_t launch_read_pop(elbm_ctx* c, double* dst) {
  const void* A = c->pop[c->cur];
  switch (c->p.storage) {
    case ELBM_STORAGE_F32:
      hipLaunchKernelGGL(k_read_pop<ELBM_STORAGE_F32>, grid_1d(c->N), dim3(256), 0, c->stream, (const float*)A, c->lay, dst, c->N);
      break;
    case ELBM_STORAGE_F16:
      hipLaunchKernelGGL(k_read_pop<ELBM_STORAGE_F16>, grid_1d(c->N), dim3(256), 0, c->stream, (const _Float16*)A, c->lay,
                         dst, c->N);
      break;
    default:
      hipLaunchKernelGGL(k_read_pop<ELBM_STORAGE_BF16>, grid_1d(c->N), dim3(256), 0, c->stream, (const uint16_t*)A, c->lay,
                         dst, c->N);
  }
  return hipGetLastError();
}

// Context-free collision of independent nodes (unit tests of the collision alone).
template <int STAB>
__global__ __launch_bounds__(256) void k_collide_nodes(const float* fin, float* fout, float* gam, const float* F,
                                                       int64_t n, float beta, float inv_beta, float thr) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    float f[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) f[i] = fin[i * n + k] - wf(i);
    const float Fx = F ? F[k] : 0.f, Fy = F ? F[n + k] : 0.f, Fz = F ? F[2 * n + k] : 0.f;
    KbcOut<float> r;
    if (F) r = kbc_collide<float, true, STAB>(f, beta, inv_beta, Fx, Fy, Fz);
    else r = kbc_collide<float, false, STAB>(f, beta, inv_beta, Fx, Fy, Fz);
    float g = r.gamma;
    if (thr >= 0.f && needs_fp64(r, thr)) {
      double d[27];
#pragma unroll
      for (int i = 0; i < 27; ++i) d[i] = (double)fin[i * n + k] - wd(i);
      KbcOut<double> r2;
      if (F) r2 = kbc_collide<double, true, STAB>(d, (double)beta, 1.0 / (double)beta, Fx, Fy, Fz);
      else r2 = kbc_collide<double, false, STAB>(d, (double)beta, 1.0 / (double)beta, 0.0, 0.0, 0.0);
#pragma unroll
      for (int i = 0; i < 27; ++i) f[i] = (float)(d[i] + wd(i));
      g = (float)r2.gamma;
    } else {
#pragma unroll
      for (int i = 0; i < 27; ++i) f[i] += wf(i);
    }
#pragma unroll
    for (int i = 0; i < 27; ++i) fout[i * n + k] = f[i];
    if (gam) gam[k] = g;
  }
}

hipError_t launch_collide_nodes(const float* fin, float* fout, float* gam, const float* F, int64_t n, double beta,
                                double thr, int stab, hipStream_t s) {
  const float b = (float)beta, ib = (float)(1.0 / beta), th = (float)thr;
  if (stab == STAB_EXACT)
    hipLaunchKernelGGL(k_collide_nodes<STAB_EXACT>, grid_1d(n), dim3(256), 0, s, fin, fout, gam, F, n, b, ib, th);
  else if (stab == STAB_LBGK)
    hipLaunchKernelGGL(k_collide_nodes<STAB_LBGK>, grid_1d(n), dim3(256), 0, s, fin, fout, gam, F, n, b, ib, th);
  else if (stab == (STAB_KBC | STAB_CENTRAL))
    hipLaunchKernelGGL(k_collide_nodes<STAB_KBC | STAB_CENTRAL>, grid_1d(n), dim3(256), 0, s, fin, fout, gam, F, n, b,
                       ib, th);
  else
    hipLaunchKernelGGL(k_collide_nodes<STAB_KBC>, grid_1d(n), dim3(256), 0, s, fin, fout, gam, F, n, b, ib, th);
  return hipGetLastError();
}

}  // namespace elbm
