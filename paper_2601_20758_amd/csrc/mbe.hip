// Kernels of the in-box particle set and of the MBE stages (Section 3.1):
// the particles inside a ROI's closed box B are compacted (keeping curve
// order) into a sub-cloud with its own leaves; Eq. 1 takes exact order
// statistics from a radix sort of each axis; the adaptive smoothing length
// (Eqs. 5-6) interpolates the pilot grid at every particle, averages with a
// fixed-order two-level reduction (the paper's shared-memory group
// reduction followed by a mean of the group results, Alg. 3) and writes
// per-particle inverse lengths and weights for the final pass (Eq. 7).
#include "sfk_device.h"

namespace sfk {

// Leaves whose box meets the closed box B (a particle in B lies in its
// leaf's box, so no other leaf holds one); empty leaves never meet it.
__global__ __launch_bounds__(256) void k_leaf_overlap(const NodeBox* __restrict__ leaf_box,
                                                      int32_t n_leaves, double lx, double ly,
                                                      double lz, double hx, double hy, double hz,
                                                      int32_t* __restrict__ flags) {
  for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n_leaves;
       l += (int64_t)gridDim.x * blockDim.x) {
    const NodeBox b = leaf_box[l];
    const bool meet = (double)b.lo[0] <= hx && (double)b.hi[0] >= lx && (double)b.lo[1] <= hy &&
                      (double)b.hi[1] >= ly && (double)b.lo[2] <= hz && (double)b.hi[2] >= lz;
    flags[l] = meet ? 1 : 0;
  }
}

hipError_t launch_leaf_overlap(const NodeBox* leaf_box, int32_t n_leaves, const double* lo,
                               const double* hi, int32_t* flags, hipStream_t s) {
  if (n_leaves <= 0) return hipSuccess;
  const int64_t nb = std::min<int64_t>((n_leaves + 255) / 256, 65536);
  hipLaunchKernelGGL(k_leaf_overlap, dim3((unsigned)nb), dim3(256), 0, s, leaf_box, n_leaves,
                     lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], flags);
  return hipGetLastError();
}

// Indices of the flagged leaves, ascending (pos: exclusive scan of flags).
__global__ __launch_bounds__(256) void k_compact_leaves(const int32_t* __restrict__ flags,
                                                        const int64_t* __restrict__ pos,
                                                        int32_t n_leaves,
                                                        int32_t* __restrict__ cand) {
  for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n_leaves;
       l += (int64_t)gridDim.x * blockDim.x)
    if (flags[l]) cand[pos[l]] = (int32_t)l;
}

hipError_t launch_compact_leaves(const int32_t* flags, const int64_t* pos, int32_t n_leaves,
                                 int32_t* cand, hipStream_t s) {
  if (n_leaves <= 0) return hipSuccess;
  const int64_t nb = std::min<int64_t>((n_leaves + 255) / 256, 65536);
  hipLaunchKernelGGL(k_compact_leaves, dim3((unsigned)nb), dim3(256), 0, s, flags, pos, n_leaves,
                     cand);
  return hipGetLastError();
}

// Slot of the i-th particle examined: all slots in order, or the slots of
// the candidate leaves in order (cand != nullptr).
__device__ __forceinline__ int64_t examined_slot(const int32_t* __restrict__ cand, int64_t i) {
  return cand ? (int64_t)cand[i >> 6] * SFK_LEAF + (i & (SFK_LEAF - 1)) : i;
}

__global__ __launch_bounds__(256) void k_inbox_flags(const float4* __restrict__ pts,
                                                     const int32_t* __restrict__ cand, int64_t n,
                                                     double lx, double ly, double lz, double hx,
                                                     double hy, double hz,
                                                     int32_t* __restrict__ flags) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float4 p = pts[examined_slot(cand, i)];
    const double x = p.x, y = p.y, z = p.z;
    const bool in = p.x < 1.0e29f && x >= lx && x <= hx && y >= ly && y <= hy && z >= lz &&
                    z <= hz;
    flags[i] = in ? 1 : 0;
  }
}

hipError_t launch_inbox_flags(const float4* pts, const int32_t* cand, int64_t n, const double* lo,
                              const double* hi, int32_t* flags, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_inbox_flags, dim3((unsigned)nb), dim3(256), 0, s, pts, cand, n, lo[0],
                     lo[1], lo[2], hi[0], hi[1], hi[2], flags);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_compact(const float4* __restrict__ pts,
                                                 const int32_t* __restrict__ perm,
                                                 const int32_t* __restrict__ cand,
                                                 const int32_t* __restrict__ flags,
                                                 const int64_t* __restrict__ pos, int64_t n,
                                                 int64_t n_slots_out, float4* __restrict__ out_pts,
                                                 int32_t* __restrict__ out_perm,
                                                 float* __restrict__ out_axes, int64_t n_b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (flags[i]) {
      const int64_t j = pos[i];
      const int64_t src = examined_slot(cand, i);
      const float4 p = pts[src];
      out_pts[j] = p;
      out_perm[j] = perm[src];
      if (out_axes) {
        out_axes[j] = p.x;
        out_axes[n_b + j] = p.y;
        out_axes[2 * n_b + j] = p.z;
      }
    }
  }
  for (int64_t j = n_b + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n_slots_out;
       j += (int64_t)gridDim.x * blockDim.x)
    out_pts[j] = make_float4(SFK_SENTINEL, SFK_SENTINEL, SFK_SENTINEL, 0.0f);
}

hipError_t launch_compact(const float4* pts, const int32_t* perm, const int32_t* cand,
                          const int32_t* flags, const int64_t* pos, int64_t n,
                          int64_t n_slots_out, float4* out_pts, int32_t* out_perm,
                          float* out_axes, int64_t n_b, hipStream_t s) {
  const int64_t m = std::max<int64_t>(n, n_slots_out);
  if (m <= 0) return hipSuccess;
  const int64_t nb = std::min<int64_t>((m + 255) / 256, 65536);
  hipLaunchKernelGGL(k_compact, dim3((unsigned)nb), dim3(256), 0, s, pts, perm, cand, flags, pos,
                     n, n_slots_out, out_pts, out_perm, out_axes, n_b);
  return hipGetLastError();
}

// float -> unsigned key with the same order (negative values flipped)
__device__ __forceinline__ uint32_t f2ord(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t u) {
  const uint32_t b = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
  return __uint_as_float(b);
}

// Key = axis index in bits 32-33 above the order bits, so one sort of the
// three axis arrays leaves each axis sorted in its own segment.
__global__ __launch_bounds__(256) void k_axis_keys(const float* __restrict__ axes, int64_t n_b,
                                                   uint64_t* __restrict__ keys,
                                                   uint32_t* __restrict__ vals) {
  const int64_t m = 3 * n_b;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    keys[i] = ((uint64_t)(i / n_b) << 32) | (uint64_t)f2ord(axes[i]);
    vals[i] = (uint32_t)i;
  }
}

hipError_t launch_axis_keys(const float* axes, int64_t n_b, uint64_t* keys, uint32_t* vals,
                            hipStream_t s) {
  if (n_b <= 0) return hipSuccess;
  const int64_t nb = std::min<int64_t>((3 * n_b + 255) / 256, 65536);
  hipLaunchKernelGGL(k_axis_keys, dim3((unsigned)nb), dim3(256), 0, s, axes, n_b, keys, vals);
  return hipGetLastError();
}

// Type-7 percentile of an ascending array held as order keys.
__device__ double pct_type7(const uint64_t* __restrict__ v, int64_t n, double q) {
  const double pos = (double)(n - 1) * q;
  const int64_t i = (int64_t)floor(pos);
  const double f = pos - (double)i;
  const double vi = (double)ord2f((uint32_t)v[i]);
  if (i + 1 >= n) return (double)ord2f((uint32_t)v[n - 1]);
  const double vj = (double)ord2f((uint32_t)v[i + 1]);
  return vi + f * (vj - vi);
}

// Eq. 1: l_k = 2 (P80 - P20) / ln(N_B); a non-positive or non-finite
// result (N_B < 2, or P80 == P20) takes the cap 5 s_k of Eq. 6.
__global__ void k_mbe_ell(const uint64_t* __restrict__ sorted_x, const uint64_t* __restrict__ sorted_y,
                          const uint64_t* __restrict__ sorted_z, int64_t n_b, double lx, double ly,
                          double lz, double hx, double hy, double hz, int rx, int ry, int rz,
                          float* __restrict__ ell_out, int32_t* __restrict__ flags_out) {
  if (threadIdx.x != 0) return;
  int flags = 0;
  for (int k = 0; k < 3; ++k) {
    const uint64_t* v = k == 0 ? sorted_x : (k == 1 ? sorted_y : sorted_z);
    const double lo = k == 0 ? lx : (k == 1 ? ly : lz);
    const double hi = k == 0 ? hx : (k == 1 ? hy : hz);
    const int res = k == 0 ? rx : (k == 1 ? ry : rz);
    const double cap = 5.0 * ((hi - lo) / (double)(res - 1));
    double l = __builtin_nan("");
    if (n_b >= 2) {
      const double p20 = pct_type7(v, n_b, 0.20);
      const double p80 = pct_type7(v, n_b, 0.80);
      l = 2.0 * (p80 - p20) / log((double)n_b);
    }
    if (!(l > 0.0) || !isfinite(l)) {
      l = cap;
      flags |= 1 << k;
    }
    ell_out[k] = (float)l;
  }
  *flags_out = flags;
}

hipError_t launch_mbe_ell(const uint64_t* sorted_keys_xyz, int64_t n_b, const double* lo,
                          const double* hi, const int32_t* res, float* ell_out,
                          int32_t* flags_out, hipStream_t s) {
  hipLaunchKernelGGL(k_mbe_ell, dim3(1), dim3(64), 0, s, sorted_keys_xyz, sorted_keys_xyz + n_b,
                     sorted_keys_xyz + 2 * n_b, n_b, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2],
                     res[0], res[1], res[2], ell_out, flags_out);
  return hipGetLastError();
}

// Trilinear interpolation of the pilot grid at each particle of B
// (f = (p - lo)(res - 1)/(hi - lo), cell clamped to [0, res - 2], t clamped
// to [0, 1]), in double; per-block sums for the mean (fixed order).
struct GridGeo {
  double lo[3], hi[3];
  int res[3];
};

__global__ __launch_bounds__(256) void k_trilinear(const float4* __restrict__ pts, int64_t n_b,
                                                   const float* __restrict__ grid, GridGeo gg,
                                                   double* __restrict__ pden,
                                                   double* __restrict__ block_sums) {
  __shared__ double lds[4];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double val = 0.0;
  if (j < n_b) {
    const float4 p = pts[j];
    const float pc[3] = {p.x, p.y, p.z};
    int ci[3];
    double tt[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double f = ((double)pc[k] - gg.lo[k]) * (double)(gg.res[k] - 1) / (gg.hi[k] - gg.lo[k]);
      int c = (int)floor(f);
      if (c < 0) c = 0;
      if (c > gg.res[k] - 2) c = gg.res[k] - 2;
      double t = f - (double)c;
      if (t < 0.0) t = 0.0;
      if (t > 1.0) t = 1.0;
      ci[k] = c;
      tt[k] = t;
    }
    double a = 0.0;
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          const double wgt = (dx ? tt[0] : 1.0 - tt[0]) * (dy ? tt[1] : 1.0 - tt[1]) *
                             (dz ? tt[2] : 1.0 - tt[2]);
          const int64_t idx = (int64_t)(ci[0] + dx) +
                              (int64_t)gg.res[0] * ((int64_t)(ci[1] + dy) +
                                                    (int64_t)gg.res[1] * (ci[2] + dz));
          a += wgt * (double)grid[idx];
        }
    pden[j] = a;
    val = a;
  }
  val = wave_sum(val);
  if (lane_id() == 0) lds[threadIdx.x >> 6] = val;
  __syncthreads();
  if (threadIdx.x == 0) block_sums[blockIdx.x] = ((lds[0] + lds[1]) + lds[2]) + lds[3];
}

// aveDen = (sum of block sums) / N_B, one block, fixed order.
__global__ __launch_bounds__(256) void k_mean(const double* __restrict__ block_sums, int nblk,
                                              int64_t n_b, double* __restrict__ ave) {
  __shared__ double lds[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) s += block_sums[i];
  s = wave_sum(s);
  if (lane_id() == 0) lds[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *ave = n_b > 0 ? (((lds[0] + lds[1]) + lds[2]) + lds[3]) / (double)n_b : 0.0;
}

// Eq. 6 per particle; pden <= 0 takes the cap.
__global__ __launch_bounds__(256) void k_asl(const double* __restrict__ pden, int64_t n_b,
                                             const double* __restrict__ ave_p, float e0, float e1,
                                             float e2, GridGeo gg, float4* __restrict__ pparam,
                                             float* __restrict__ ell_out) {
  const double ave = *ave_p;
  const float e[3] = {e0, e1, e2};
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n_b;
       j += (int64_t)gridDim.x * blockDim.x) {
    const double pd = pden[j];
    float l[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double cap = 5.0 * ((gg.hi[k] - gg.lo[k]) / (double)(gg.res[k] - 1));
      double v;
      if (pd > 0.0) {
        v = (double)e[k] * cbrt(ave / pd);
        if (v > cap) v = cap;
      } else {
        v = cap;
      }
      l[k] = (float)v;
    }
    const double lx = l[0], ly = l[1], lz = l[2];
    pparam[j] = make_float4((float)(1.0 / lx), (float)(1.0 / ly), (float)(1.0 / lz),
                            (float)(1.0 / (lx * ly * lz)));
    if (ell_out) {
      ell_out[3 * j] = l[0];
      ell_out[3 * j + 1] = l[1];
      ell_out[3 * j + 2] = l[2];
    }
  }
}

hipError_t launch_trilinear_mean(const float4* pts, int64_t n_b, const float* grid,
                                 const double* lo, const double* hi, const int32_t* res,
                                 double* pden, double* block_sums, double* ave, hipStream_t s) {
  if (n_b <= 0) return hipSuccess;
  GridGeo gg;
  for (int k = 0; k < 3; ++k) {
    gg.lo[k] = lo[k];
    gg.hi[k] = hi[k];
    gg.res[k] = res[k];
  }
  const int nblk = (int)((n_b + 255) / 256);
  hipLaunchKernelGGL(k_trilinear, dim3(nblk), dim3(256), 0, s, pts, n_b, grid, gg, pden,
                     block_sums);
  hipLaunchKernelGGL(k_mean, dim3(1), dim3(256), 0, s, block_sums, nblk, n_b, ave);
  return hipGetLastError();
}

hipError_t launch_asl2(const double* pden, int64_t n_b, const double* ave, const float* ell0,
                       const double* lo, const double* hi, const int32_t* res, float4* pparam,
                       float* ell_out, hipStream_t s) {
  if (n_b <= 0) return hipSuccess;
  GridGeo gg;
  for (int k = 0; k < 3; ++k) {
    gg.lo[k] = lo[k];
    gg.hi[k] = hi[k];
    gg.res[k] = res[k];
  }
  const int64_t nb = std::min<int64_t>((n_b + 255) / 256, 65536);
  hipLaunchKernelGGL(k_asl, dim3((unsigned)nb), dim3(256), 0, s, pden, n_b, ave, ell0[0], ell0[1],
                     ell0[2], gg, pparam, ell_out);
  return hipGetLastError();
}

}  // namespace sfk
