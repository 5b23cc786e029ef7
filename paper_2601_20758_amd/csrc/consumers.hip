// Consumers of a density grid on the device, so a grid never has to cross
// PCIe for them: the density at arbitrary positions (trilinear interpolation
// of the surrounding grid nodes, Section 3.1 after Eq. 8), the selection of
// the points whose density reaches a threshold (the region a Marching Cubes
// iso-surface of the grid bounds, Section 4.1), the Marching Cubes
// classification of the grid's cells against that threshold, the per-brick
// value range that drives adaptive refinement, and the copy of a view's
// lattice nodes out of cached blocks.
//
// Arithmetic: double, every operation rounded, no contraction (the library
// is built with -ffp-contract=off), in this fixed order per axis
//   f = ((p - lo) * (res - 1)) / (hi - lo), cell c = floor(f) clamped to
//   [0, res - 2], t = f - c clamped to [0, 1],
// and the eight corner terms ((wx * wy) * wz) * value accumulated z-major,
// then y, then x, so a threshold decision is the same as the definition's.
#include <algorithm>

#include "sfk_device.h"

namespace sfk {

struct GridGeom {
  double lo[3], hi[3];
  int32_t res[3];
  int32_t pad_;
};

__device__ __forceinline__ bool in_closed_box(const GridGeom& g, float x, float y, float z) {
  const double p[3] = {(double)x, (double)y, (double)z};
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (!(p[k] >= g.lo[k] && p[k] <= g.hi[k])) return false;
  return true;
}

__device__ __forceinline__ double trilinear_at(const float* __restrict__ grid, const GridGeom& g,
                                               float x, float y, float z) {
  const double p[3] = {(double)x, (double)y, (double)z};
  int c[3];
  double t[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double f = ((p[k] - g.lo[k]) * (double)(g.res[k] - 1)) / (g.hi[k] - g.lo[k]);
    int ci = (int)floor(f);
    ci = max(0, min(ci, g.res[k] - 2));
    double tt = f - (double)ci;
    tt = fmin(fmax(tt, 0.0), 1.0);
    c[k] = ci;
    t[k] = tt;
  }
  double acc = 0.0;
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        const double w = ((dx ? t[0] : 1.0 - t[0]) * (dy ? t[1] : 1.0 - t[1])) *
                         (dz ? t[2] : 1.0 - t[2]);
        const int64_t idx =
            (int64_t)(c[0] + dx) +
            (int64_t)g.res[0] * ((int64_t)(c[1] + dy) + (int64_t)g.res[1] * (int64_t)(c[2] + dz));
        acc += w * (double)grid[idx];
      }
  return acc;
}

// density at each point (0 outside the closed box), rounded once to float
__global__ __launch_bounds__(256) void k_sample(const float* __restrict__ grid, GridGeom g,
                                                const float* __restrict__ xyz, int64_t n,
                                                float* __restrict__ out) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    const float x = xyz[3 * j], y = xyz[3 * j + 1], z = xyz[3 * j + 2];
    out[j] = in_closed_box(g, x, y, z) ? (float)trilinear_at(grid, g, x, y, z) : 0.0f;
  }
}

// 1 where the point lies in the closed box and its density is >= iso
__global__ __launch_bounds__(256) void k_select_flags(const float* __restrict__ grid, GridGeom g,
                                                      double iso, const float* __restrict__ xyz,
                                                      int64_t n, int32_t* __restrict__ flags) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    const float x = xyz[3 * j], y = xyz[3 * j + 1], z = xyz[3 * j + 2];
    flags[j] = (in_closed_box(g, x, y, z) && trilinear_at(grid, g, x, y, z) >= iso) ? 1 : 0;
  }
}

// ascending indices of the flagged entries (the first `cap` of them)
__global__ __launch_bounds__(256) void k_compact_index(const int32_t* __restrict__ flags,
                                                       const int64_t* __restrict__ pos, int64_t n,
                                                       int64_t* __restrict__ idx, int64_t cap) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x)
    if (flags[j] && pos[j] < cap) idx[pos[j]] = j;
}

// Marching Cubes case of every cell (bit dx + 2 dy + 4 dz set when that
// corner's value is >= iso); flag = case not in {0, 255}
__global__ __launch_bounds__(256) void k_iso_flags(const float* __restrict__ grid, GridGeom g,
                                                   double iso, int64_t n_cells,
                                                   int32_t* __restrict__ flags,
                                                   uint8_t* __restrict__ case_all) {
  const int64_t cx = g.res[0] - 1, cy = g.res[1] - 1;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n_cells;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = q % cx, j = (q / cx) % cy, k = q / (cx * cy);
    int cs = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int dx = b & 1, dy = (b >> 1) & 1, dz = (b >> 2) & 1;
      const double v = (double)grid[(i + dx) + (int64_t)g.res[0] * ((j + dy) + (int64_t)g.res[1] * (k + dz))];
      if (v >= iso) cs |= 1 << b;
    }
    case_all[q] = (uint8_t)cs;
    flags[q] = (cs != 0 && cs != 255) ? 1 : 0;
  }
}

__global__ __launch_bounds__(256) void k_compact_cells(const int32_t* __restrict__ flags,
                                                       const int64_t* __restrict__ pos,
                                                       const uint8_t* __restrict__ case_all,
                                                       int64_t n, int64_t* __restrict__ cells,
                                                       uint8_t* __restrict__ cases, int64_t cap) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x)
    if (flags[q] && pos[q] < cap) {
      cells[pos[q]] = q;
      cases[pos[q]] = case_all[q];
    }
}

// ---------------------------------------------------------------------------
// Marching Cubes triangles (Section 4.1; Lorensen and Cline 1987). The case
// table is computed at compile time from the cube's faces:
//   corner c = dx + 2 dy + 4 dz, inside when its value is >= iso;
//   edge ids: along x dy + 2 dz, along y 4 + dx + 2 dz, along z 8 + dx + 2 dy;
//   each face walked counterclockwise as seen from outside the cube
//   (face normal k, side v, a = k+1, b = k+2 mod 3: (a, b) corners
//   00, 10, 11, 01 for v = 1, 00, 01, 11, 10 for v = 0);
//   an edge crossed inside -> outside in that walk is joined to the nearest
//   crossed edge before it in the walk (faces with four crossings cut off
//   their inside corners: the rule sees only the face, so both cells of a
//   face agree and the surface is closed);
//   the joins form loops, started at their smallest edge, in ascending
//   order; a loop w0 .. w(L-1) is fanned from the first apex a whose
//   diagonals never join two edges of one face, as the triangles
//   (w(a), w(a+i+1), w(a+i)), i = 1 .. L-2: normals point outward (from
//   values >= iso to values below).
// Vertex on an edge from its lower corner p to q: t = (iso - f_p) /
// (f_q - f_p), coordinate x_p + t (x_q - x_p) on the edge's axis, node
// coordinates on the others, in double, rounded once to float.
// ---------------------------------------------------------------------------

struct McCases {
  int8_t ntri[256];
  int8_t edge[256][15];
};

// edge between corners c and c ^ (1 << axis)
constexpr int mc_edge(int c, int axis) {
  const int x = c & 1, y = (c >> 1) & 1, z = (c >> 2) & 1;
  return axis == 0 ? y + 2 * z : axis == 1 ? 4 + x + 2 * z : 8 + x + 2 * y;
}

// the two faces (normal axis, side) an edge lies on, as axis * 2 + side
constexpr bool mc_common_face(int e, int f) {
  int fe[2] = {0, 0}, ff[2] = {0, 0};
  const int es[2] = {e, f};
  for (int w = 0; w < 2; ++w) {
    const int axis = es[w] >> 2, bits = es[w] & 3;
    const int n0 = axis == 0 ? 1 : 0;  // the lower of the two other axes
    const int n1 = axis == 2 ? 1 : 2;  // the upper one
    int* out = w == 0 ? fe : ff;
    out[0] = n0 * 2 + (bits & 1);
    out[1] = n1 * 2 + (bits >> 1);
  }
  return fe[0] == ff[0] || fe[0] == ff[1] || fe[1] == ff[0] || fe[1] == ff[1];
}

constexpr McCases mc_cases() {
  McCases t{};
  for (int cs = 0; cs < 256; ++cs) {
    int next[12] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};
    bool cut[12] = {};
    for (int k = 0; k < 3; ++k)
      for (int v = 0; v < 2; ++v) {
        const int a = (k + 1) % 3, b = (k + 2) % 3;
        int corner[4] = {0, 0, 0, 0};
        for (int i = 0; i < 4; ++i) {
          // counterclockwise from outside: (0,0),(1,0),(1,1),(0,1) on the
          // upper face, reversed (0,0),(0,1),(1,1),(1,0) on the lower one
          const int ua = (i == 1 || i == 2) ? 1 : 0, ub = (i >= 2) ? 1 : 0;
          const int ca = v ? ua : ub, cb = v ? ub : ua;
          corner[i] = (v << k) | (ca << a) | (cb << b);
        }
        bool in[4] = {}, crossed[4] = {};
        int edge[4] = {0, 0, 0, 0};
        for (int i = 0; i < 4; ++i) in[i] = ((cs >> corner[i]) & 1) != 0;
        for (int i = 0; i < 4; ++i) {
          const int c0 = corner[i], c1 = corner[(i + 1) & 3];
          const int d = c0 ^ c1;
          const int axis = d == 1 ? 0 : d == 2 ? 1 : 2;
          edge[i] = mc_edge(c0 & ~d, axis);
          crossed[i] = in[i] != in[(i + 1) & 3];
          if (crossed[i]) cut[edge[i]] = true;
        }
        for (int i = 0; i < 4; ++i) {
          if (!(in[i] && !in[(i + 1) & 3])) continue;
          for (int back = 1; back < 4; ++back) {
            const int j = (i + 4 - back) & 3;
            if (crossed[j]) {
              next[edge[i]] = edge[j];
              break;
            }
          }
        }
      }
    bool used[12] = {};
    int n = 0;
    for (int e0 = 0; e0 < 12; ++e0) {
      if (!cut[e0] || used[e0]) continue;
      int w[12] = {}, len = 0;
      for (int x = e0; len < 12;) {
        used[x] = true;
        w[len++] = x;
        x = next[x];
        if (x == e0 || x < 0) break;
      }
      int apex = 0;
      for (int a = 0; a < len; ++a) {
        bool clean = true;
        for (int i = 2; i + 1 < len; ++i)
          if (mc_common_face(w[a], w[(a + i) % len])) clean = false;
        if (clean) {
          apex = a;
          break;
        }
      }
      for (int i = 1; i + 1 < len; ++i) {
        t.edge[cs][3 * n] = (int8_t)w[apex];
        t.edge[cs][3 * n + 1] = (int8_t)w[(apex + i + 1) % len];
        t.edge[cs][3 * n + 2] = (int8_t)w[(apex + i) % len];
        ++n;
      }
    }
    t.ntri[cs] = (int8_t)n;
  }
  return t;
}

__constant__ McCases kMcCases = mc_cases();

// the same table on the host (test export)
int mc_case_host(int cs, int8_t* edges) {
  static constexpr McCases t = mc_cases();
  for (int i = 0; i < 3 * t.ntri[cs]; ++i) edges[i] = t.edge[cs][i];
  return t.ntri[cs];
}

// triangles of each cell (from the cell's case)
__global__ __launch_bounds__(256) void k_iso_tri_count(const uint8_t* __restrict__ case_all,
                                                       int64_t n_cells,
                                                       int32_t* __restrict__ cnt) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n_cells;
       q += (int64_t)gridDim.x * blockDim.x)
    cnt[q] = kMcCases.ntri[case_all[q]];
}

__device__ __forceinline__ double node_x(const GridGeom& g, int k, int64_t i) {
  return g.lo[k] + ((double)i * (g.hi[k] - g.lo[k])) / (double)(g.res[k] - 1);
}

// the triangles of every cell at their offsets (the first `cap` of them):
// 9 floats each, three vertices (x, y, z)
__global__ __launch_bounds__(256) void k_iso_emit(const float* __restrict__ grid, GridGeom g,
                                                  double iso, const uint8_t* __restrict__ case_all,
                                                  const int64_t* __restrict__ pos,
                                                  int64_t n_cells, float* __restrict__ tris,
                                                  int64_t cap) {
  const int64_t cx = g.res[0] - 1, cy = g.res[1] - 1;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n_cells;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int cs = case_all[q];
    const int nt = kMcCases.ntri[cs];
    if (nt == 0) continue;
    const int64_t base = pos[q];
    if (base >= cap) continue;
    const int64_t ci[3] = {q % cx, (q / cx) % cy, q / (cx * cy)};
    double f[8];
#pragma unroll
    for (int c = 0; c < 8; ++c)
      f[c] = (double)grid[(ci[0] + (c & 1)) +
                          (int64_t)g.res[0] * ((ci[1] + ((c >> 1) & 1)) +
                                               (int64_t)g.res[1] * (ci[2] + ((c >> 2) & 1)))];
    for (int tr = 0; tr < nt && base + tr < cap; ++tr) {
      float* out = tris + 9 * (base + tr);
      for (int vtx = 0; vtx < 3; ++vtx) {
        const int e = kMcCases.edge[cs][3 * tr + vtx];
        const int axis = e >> 2, bits = e & 3;
        // lower corner of the edge: its two other coordinates from the id
        const int o0 = axis == 0 ? 1 : 0, o1 = axis == 2 ? 1 : 2;
        const int p = ((bits & 1) << o0) | ((bits >> 1) << o1);
        const int qc = p | (1 << axis);
        const double t = (iso - f[p]) / (f[qc] - f[p]);
        for (int d = 0; d < 3; ++d) {
          const int64_t idx = ci[d] + ((p >> d) & 1);
          double x = node_x(g, d, idx);
          if (d == axis) x = x + t * (node_x(g, d, idx + 1) - x);
          out[3 * vtx + d] = (float)x;
        }
      }
    }
  }
}

// Lattice nodes g0 + (i, j, k) of a view, copied out of cached blocks of B^3
// nodes (x fastest inside a block). table[] holds the cache slot of each
// block of the range b0 .. b0 + nb - 1 (x fastest); every node of the grid
// falls in that range by construction, and a node that did not would be
// written as 0 rather than read out of bounds.
struct GatherGeom {
  int64_t g0[3], b0[3];
  int32_t res[3], nb[3];
  int32_t B;
  int32_t pad_;
  int64_t n_slots;
};

__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b) {
  return a >= 0 ? a / b : -((-a + b - 1) / b);
}

__global__ __launch_bounds__(256) void k_view_gather(const float* __restrict__ cache,
                                                     const int32_t* __restrict__ table,
                                                     GatherGeom G, float* __restrict__ out) {
  const int64_t n = (int64_t)G.res[0] * G.res[1] * G.res[2];
  const int64_t B = G.B;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = q % G.res[0], j = (q / G.res[0]) % G.res[1], k = q / ((int64_t)G.res[0] * G.res[1]);
    const int64_t g[3] = {G.g0[0] + i, G.g0[1] + j, G.g0[2] + k};
    int64_t b[3], l[3];
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int64_t bb = floor_div(g[a], B);
      l[a] = g[a] - bb * B;
      b[a] = bb - G.b0[a];
      ok = ok && b[a] >= 0 && b[a] < G.nb[a];
    }
    float v = 0.0f;
    if (ok) {
      const int32_t slot = table[b[0] + (int64_t)G.nb[0] * (b[1] + (int64_t)G.nb[1] * b[2])];
      if (slot >= 0 && slot < G.n_slots) v = cache[(int64_t)slot * B * B * B + l[0] + B * (l[1] + B * l[2])];
    }
    out[q] = v;
  }
}

// Smallest and largest node value of each brick (one workgroup per brick).
__global__ __launch_bounds__(256) void k_brick_minmax(const BrickDesc* __restrict__ d, int32_t n,
                                                      float* __restrict__ mn,
                                                      float* __restrict__ mx) {
  __shared__ float s_lo[256], s_hi[256];
  for (int32_t b = blockIdx.x; b < n; b += gridDim.x) {
    const BrickDesc D = d[b];
    const int64_t nx = D.cells[0] + 1, ny = D.cells[1] + 1, nz = D.cells[2] + 1;
    float lo = __builtin_huge_valf(), hi = -__builtin_huge_valf();
    for (int64_t q = threadIdx.x; q < nx * ny * nz; q += blockDim.x) {
      const int64_t i = q % nx, j = (q / nx) % ny, k = q / (nx * ny);
      const float v = D.grid[(D.n0[0] + i) +
                             (int64_t)D.res[0] * ((D.n0[1] + j) + (int64_t)D.res[1] * (D.n0[2] + k))];
      lo = fminf(lo, v);
      hi = fmaxf(hi, v);
    }
    s_lo[threadIdx.x] = lo;
    s_hi[threadIdx.x] = hi;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) {
        s_lo[threadIdx.x] = fminf(s_lo[threadIdx.x], s_lo[threadIdx.x + off]);
        s_hi[threadIdx.x] = fmaxf(s_hi[threadIdx.x], s_hi[threadIdx.x + off]);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      mn[b] = s_lo[0];
      mx[b] = s_hi[0];
    }
    __syncthreads();
  }
}

static GridGeom geom_of(const double lo[3], const double hi[3], const int32_t res[3]) {
  GridGeom g{};
  for (int k = 0; k < 3; ++k) {
    g.lo[k] = lo[k];
    g.hi[k] = hi[k];
    g.res[k] = res[k];
  }
  return g;
}

static unsigned grid_of(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536));
}

hipError_t launch_sample(const float* grid, const double lo[3], const double hi[3],
                         const int32_t res[3], const float* xyz, int64_t n, float* out,
                         hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sample, dim3(grid_of(n)), dim3(256), 0, s, grid, geom_of(lo, hi, res), xyz,
                     n, out);
  return hipGetLastError();
}

hipError_t launch_select_flags(const float* grid, const double lo[3], const double hi[3],
                               const int32_t res[3], double iso, const float* xyz, int64_t n,
                               int32_t* flags, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_select_flags, dim3(grid_of(n)), dim3(256), 0, s, grid,
                     geom_of(lo, hi, res), iso, xyz, n, flags);
  return hipGetLastError();
}

hipError_t launch_compact_index(const int32_t* flags, const int64_t* pos, int64_t n, int64_t* idx,
                                int64_t cap, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_compact_index, dim3(grid_of(n)), dim3(256), 0, s, flags, pos, n, idx, cap);
  return hipGetLastError();
}

hipError_t launch_iso_flags(const float* grid, const int32_t res[3], double iso, int64_t n_cells,
                            int32_t* flags, uint8_t* case_all, hipStream_t s) {
  if (n_cells <= 0) return hipSuccess;
  const double z[3] = {0.0, 0.0, 0.0};
  hipLaunchKernelGGL(k_iso_flags, dim3(grid_of(n_cells)), dim3(256), 0, s, grid,
                     geom_of(z, z, res), iso, n_cells, flags, case_all);
  return hipGetLastError();
}

hipError_t launch_compact_cells(const int32_t* flags, const int64_t* pos, const uint8_t* case_all,
                                int64_t n, int64_t* cells, uint8_t* cases, int64_t cap,
                                hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_compact_cells, dim3(grid_of(n)), dim3(256), 0, s, flags, pos, case_all, n,
                     cells, cases, cap);
  return hipGetLastError();
}

hipError_t launch_iso_tri_count(const uint8_t* case_all, int64_t n_cells, int32_t* cnt,
                                hipStream_t s) {
  if (n_cells <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_iso_tri_count, dim3(grid_of(n_cells)), dim3(256), 0, s, case_all, n_cells,
                     cnt);
  return hipGetLastError();
}

hipError_t launch_iso_emit(const float* grid, const double lo[3], const double hi[3],
                           const int32_t res[3], double iso, const uint8_t* case_all,
                           const int64_t* pos, int64_t n_cells, float* tris, int64_t cap,
                           hipStream_t s) {
  if (n_cells <= 0 || cap <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_iso_emit, dim3(grid_of(n_cells)), dim3(256), 0, s, grid,
                     geom_of(lo, hi, res), iso, case_all, pos, n_cells, tris, cap);
  return hipGetLastError();
}

hipError_t launch_brick_minmax(const BrickDesc* d_descs, int32_t n, float* d_min, float* d_max,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_brick_minmax, dim3((unsigned)std::min<int32_t>(n, 65536)), dim3(256), 0, s,
                     d_descs, n, d_min, d_max);
  return hipGetLastError();
}

hipError_t launch_view_gather(const float* cache, int64_t n_slots, int block, const int32_t* table,
                              const int64_t b0[3], const int32_t nb[3], const int64_t g0[3],
                              const int32_t res[3], float* out, hipStream_t s) {
  GatherGeom G{};
  for (int k = 0; k < 3; ++k) {
    G.g0[k] = g0[k];
    G.b0[k] = b0[k];
    G.res[k] = res[k];
    G.nb[k] = nb[k];
  }
  G.B = block;
  G.n_slots = n_slots;
  const int64_t n = (int64_t)res[0] * res[1] * res[2];
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_view_gather, dim3(grid_of(n)), dim3(256), 0, s, cache, table, G, out);
  return hipGetLastError();
}

}  // namespace sfk
