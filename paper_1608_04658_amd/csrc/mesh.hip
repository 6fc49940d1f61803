// mesh.hip -- the triangulated body (the deforming geometries of Sec. IV.C): upload of a time
// level of vertex positions and velocities, binning of the triangles into a uniform grid on the
// device (count, scan, fill; no host round trip), and the solid mask by crossing parity, one
// lattice row per thread.
#include <math.h>

#include <algorithm>

#include "context.hpp"
#include "mesh_dev.hpp"

namespace elbm {

constexpr int ROW_CROSSINGS = 32;  // crossings held per lattice row (a closed surface: a few)

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    p[k] = v;
}

// Triangles with every vertex index checked: an index outside [0, nv) becomes 0 and is flagged.
__global__ void k_copy_tris(int32_t* dst, const int32_t* src, int64_t n, int32_t nv, uint32_t* overflow) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = src[k];
    const bool ok = v >= 0 && v < nv;
    if (!ok) atomicOr(overflow, 8u);
    dst[k] = ok ? v : 0;
  }
}

__global__ void k_copy_or_zero(double* dst, const double* src, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    dst[k] = src ? src[k] : 0.0;
}

// Cell range of triangle k's bounding box; flags a vertex outside the declared box.
__device__ inline void tri_cells(const MeshDev& m, const double* X, int k, int* lo, int* hi, uint32_t* overflow) {
  const int32_t* t3 = m.tri + 3 * k;
  for (int a = 0; a < 3; ++a) {
    const double v0 = X[3 * t3[0] + a], v1 = X[3 * t3[1] + a], v2 = X[3 * t3[2] + a];
    const double mn = fmin(v0, fmin(v1, v2)), mx = fmax(v0, fmax(v1, v2));
    const double lim = m.org[a] + (double)m.dim[a] / m.inv_h;
    if (!(mn >= m.org[a]) || !(mx < lim)) atomicOr(overflow, 2u);
    lo[a] = mesh_cell(m, a, mn);
    hi[a] = mesh_cell(m, a, mx);
  }
}

__global__ void k_mesh_count(MeshDev m, const double* X, int32_t* cnt, uint32_t* overflow) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < m.nt; k += gridDim.x * blockDim.x) {
    int lo[3], hi[3];
    tri_cells(m, X, k, lo, hi, overflow);
    for (int cz = lo[2]; cz <= hi[2]; ++cz)
      for (int cy = lo[1]; cy <= hi[1]; ++cy)
        for (int cx = lo[0]; cx <= hi[0]; ++cx) atomicAdd(&cnt[mesh_cell_index(m, cx, cy, cz)], 1);
  }
}

// One workgroup: start = exclusive scan of cnt (start[ncell] = total); cnt is cleared for the fill.
__global__ __launch_bounds__(1024) void k_mesh_scan(int32_t* cnt, int32_t* start, int32_t ncell, int64_t cap,
                                                    uint32_t* overflow) {
  __shared__ int32_t wsum[16];
  // The loads of eight consecutive 1024-cell chunks are issued together, so the chunk scans wait
  // for memory once per 8192 cells.
  constexpr int CHUNKS = 8;
  int32_t running = 0;
  for (int64_t base = 0; base < ncell; base += 1024 * CHUNKS) {
    int32_t v[CHUNKS];
#pragma unroll
    for (int k = 0; k < CHUNKS; ++k) {
      const int64_t i = base + k * 1024 + threadIdx.x;
      v[k] = i < ncell ? cnt[i] : 0;
    }
#pragma unroll
    for (int k = 0; k < CHUNKS; ++k) {
      const int64_t i = base + k * 1024 + threadIdx.x;
      int32_t total;
      const int32_t incl = scan1024_inclusive(v[k], wsum, total);
      if (i < ncell) {
        start[i] = running + incl - v[k];
        cnt[i] = 0;
      }
      running += total;
    }
  }
  if (threadIdx.x == 0) {
    start[ncell] = running;
    if ((int64_t)running > cap) atomicOr(overflow, 2u);
  }
}

__global__ void k_mesh_fill(MeshDev m, const double* X, const int32_t* start, int32_t* cursor, int32_t* items,
                            int64_t cap, uint32_t* overflow) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < m.nt; k += gridDim.x * blockDim.x) {
    int lo[3], hi[3];
    tri_cells(m, X, k, lo, hi, overflow);
    for (int cz = lo[2]; cz <= hi[2]; ++cz)
      for (int cy = lo[1]; cy <= hi[1]; ++cy)
        for (int cx = lo[0]; cx <= hi[0]; ++cx) {
          const int c = mesh_cell_index(m, cx, cy, cz);
          const int64_t pos = (int64_t)start[c] + atomicAdd(&cursor[c], 1);
          if (pos < cap) items[pos] = k;
        }
  }
}

// Solid mask of the triangulated body on a box, one wavefront per (y, z) row: the lanes share out
// the cells along x and collect the x of every crossing of the +x ray through (y, z) (each
// triangle once: in the cell of its bounding box's lowest x), then share out the nodes of the row
// and mark those with an odd number of crossings beyond them (the order of the list is immaterial).
constexpr int MASK_ROWS = 4;  // wavefronts (rows) per workgroup
__global__ __launch_bounds__(64 * MASK_ROWS) void k_mesh_mask(MeshDev m, int lvl, uint8_t* flags, int32_t nx,
                                                              int32_t ny, Box box, uint8_t bits, uint32_t* overflow) {
  __shared__ double xs[MASK_ROWS][ROW_CROSSINGS];
  __shared__ int cnt[MASK_ROWS];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const MeshLevel& L = m.lv[lvl];
  const long rows = (long)box.n[1] * box.n[2];
  const long r = blockIdx.x * (long)MASK_ROWS + w;
  const bool active = r < rows;  // uniform over the wavefront
  const int y = active ? box.lo[1] + (int)(r % box.n[1]) : 0, z = active ? box.lo[2] + (int)(r / box.n[1]) : 0;
  if (lane == 0) cnt[w] = 0;
  __syncthreads();
  if (active) {
    const double yd = (double)y, zd = (double)z;
    const int cy = mesh_cell(m, 1, yd), cz = mesh_cell(m, 2, zd);
    for (int cx = lane; cx < m.dim[0]; cx += 64) {
      const int c = mesh_cell_index(m, cx, cy, cz);
      const int e1 = min(L.start[c + 1], m.cap);
      for (int e = L.start[c]; e < e1; ++e) {
        const int k = L.items[e];
        if ((unsigned)k >= (unsigned)m.nt) continue;
        const int32_t* t3 = m.tri + 3 * k;
        const double* A = L.X + 3 * t3[0];
        const double* B = L.X + 3 * t3[1];
        const double* C = L.X + 3 * t3[2];
        if (mesh_cell(m, 0, fmin(A[0], fmin(B[0], C[0]))) != cx) continue;
        double xc;
        if (!mesh_crossing(A, B, C, yd, zd, xc)) continue;
        const int j = atomicAdd(&cnt[w], 1);
        if (j < ROW_CROSSINGS) xs[w][j] = xc;
        else atomicOr(overflow, 4u);
      }
    }
  }
  __syncthreads();
  if (!active) return;
  const int nc = min(cnt[w], ROW_CROSSINGS);
  if (nc == 0) return;
  for (int x = box.lo[0] + lane; x < box.lo[0] + box.n[0]; x += 64) {
    const double xd = (double)x;
    int odd = 0;
    for (int j = 0; j < nc; ++j) odd ^= (xs[w][j] > xd) ? 1 : 0;
    if (odd) {
      const long n = ((long)z * ny + y) * nx + x;
      flags[n] |= bits;
    }
  }
}

hipError_t mesh_copy_tris(elbm_ctx* c, const int32_t* tris, int32_t nt) {
  const int64_t n = 3 * (int64_t)nt;
  hipLaunchKernelGGL(k_copy_tris, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096))),
                     dim3(256), 0, c->stream, c->mesh_tri, tris, n, c->mesh_nv, &c->cnt->overflow);
  return hipGetLastError();
}

static MeshDev mesh_dev_for_slot(const elbm_ctx* c, int slot) {
  MeshDev m = c->mesh_grid;
  m.tri = c->mesh_tri;
  m.nt = c->mesh_nt;
  for (int l = 0; l < 2; ++l) {
    m.lv[l].X = c->mesh_X[slot];
    m.lv[l].V = c->mesh_V[slot];
    m.lv[l].start = c->mesh_start[slot];
    m.lv[l].items = c->mesh_items[slot];
  }
  return m;
}

// Copy a time level into slot (V NULL = at rest) and bin its triangles.
hipError_t mesh_upload(elbm_ctx* c, int slot, const double* X, const double* V) {
  const int64_t n3 = 3 * (int64_t)c->mesh_nv;
  const dim3 b(256);
  const dim3 gv((unsigned)std::max<int64_t>(1, std::min<int64_t>((n3 + 255) / 256, 4096)));
  hipLaunchKernelGGL(k_copy_or_zero, gv, b, 0, c->stream, c->mesh_X[slot], X, n3);
  hipLaunchKernelGGL(k_copy_or_zero, gv, b, 0, c->stream, c->mesh_V[slot], V, n3);
  const MeshDev m = mesh_dev_for_slot(c, slot);
  const dim3 gt((unsigned)std::max(1, std::min((c->mesh_nt + 255) / 256, 4096)));
  hipLaunchKernelGGL(k_fill_i32, dim3((m.ncell + 255) / 256), b, 0, c->stream, c->mesh_cursor, (int64_t)m.ncell, 0);
  hipLaunchKernelGGL(k_mesh_count, gt, b, 0, c->stream, m, (const double*)c->mesh_X[slot], c->mesh_cursor,
                     &c->cnt->overflow);
  hipLaunchKernelGGL(k_mesh_scan, dim3(1), dim3(1024), 0, c->stream, c->mesh_cursor, c->mesh_start[slot], m.ncell,
                     c->mesh_cap, &c->cnt->overflow);
  hipLaunchKernelGGL(k_mesh_fill, gt, b, 0, c->stream, m, (const double*)c->mesh_X[slot],
                     (const int32_t*)c->mesh_start[slot], c->mesh_cursor, c->mesh_items[slot], c->mesh_cap,
                     &c->cnt->overflow);
  return hipGetLastError();
}

// OR `bits` into the flags of the nodes inside the triangulated body at level lvl of bd.m.
hipError_t mesh_mask(elbm_ctx* c, const Bodies& bd, int lvl, uint8_t bits) {
  Box box;
  const int dims[3] = {c->p.nx, c->p.ny, c->p.nz};
  for (int a = 0; a < 3; ++a) {
    int l = (int)ceil(c->mesh_lo[a]), h = (int)floor(c->mesh_hi[a]);
    l = l < 0 ? 0 : l;
    h = h > dims[a] - 1 ? dims[a] - 1 : h;
    box.lo[a] = l;
    box.n[a] = h >= l ? h - l + 1 : 0;
  }
  const long rows = (long)box.n[1] * box.n[2];
  if (rows == 0 || box.n[0] == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mesh_mask, dim3((unsigned)((rows + MASK_ROWS - 1) / MASK_ROWS)), dim3(64 * MASK_ROWS), 0,
                     c->stream, bd.m, lvl, c->flags, c->p.nx, c->p.ny, box, bits, &c->cnt->overflow);
  return hipGetLastError();
}

}  // namespace elbm
