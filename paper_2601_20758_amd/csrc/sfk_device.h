// Device helpers shared by the libsfkde kernels (wavefront = 64 lanes).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sfk_internal.h"

namespace sfk {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  return (1ull << lane_id()) - 1ull;
}

__device__ __forceinline__ int popc64(uint64_t m) { return __popcll(m); }

// Make LDS writes of this wavefront visible to its other lanes.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T wave_bcast(T v, int src) { return __shfl(v, src, 64); }

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Lane l's value of a float (l uniform), bit for bit.
__device__ __forceinline__ float readlane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fminf(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    T t = __shfl_up(v, off, 64);
    if (lane >= off) v += t;
  }
  return v;
}

// Exclusive scan over a block of NT threads (NT multiple of 64); returns the
// exclusive prefix and writes the block total to *total.
template <int NT, typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* total, T* lds /* NT/64 */) {
  const int lane = lane_id(), w = threadIdx.x >> 6;
  T inc = wave_incl_scan(v);
  if (lane == 63) lds[w] = inc;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    T s = lds[i];
    if (i < w) off += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return inc - v + off;
}

// Canonical float32 squared distance between two points (no contraction):
// d = a - b per axis, s = (dx*dx + dy*dy) + dz*dz.
__device__ __forceinline__ float canon_d2(float ax, float ay, float az, float bx, float by,
                                          float bz) {
  float dx = __fsub_rn(ax, bx), dy = __fsub_rn(ay, by), dz = __fsub_rn(az, bz);
  return __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
}

// Canonical squared scaled distance of a node to a particle: double
// operations on the float32 particle and inverse-bandwidth values, every
// operation rounded, no contraction (the library is built with
// -ffp-contract=off): u_k = (x_nk - p_k) * ih_k, u2 = (ux^2 + uy^2) + uz^2.
__device__ __forceinline__ double canon_u2(double nx, double ny, double nz, float px, float py,
                                           float pz, float ihx, float ihy, float ihz) {
  const double ux = (nx - (double)px) * (double)ihx;
  const double uy = (ny - (double)py) * (double)ihy;
  const double uz = (nz - (double)pz) * (double)ihz;
  return (ux * ux + uy * uy) + uz * uz;
}

// Lower bound of the canonical scaled distance between any node of box
// [tlo, thi] and any particle of box b with inverse bandwidths >= ih: the
// per-axis gap, rounded the same way as the per-pair arithmetic, so by
// monotonicity of rounding no member can lie in a box that fails this test.
__device__ __forceinline__ double box_gap_u2(const NodeBox& b, double tlx, double tly,
                                             double tlz, double thx, double thy, double thz,
                                             float ihx, float ihy, float ihz) {
  const double gx = fmax(fmax((double)b.lo[0] - thx, tlx - (double)b.hi[0]), 0.0);
  const double gy = fmax(fmax((double)b.lo[1] - thy, tly - (double)b.hi[1]), 0.0);
  const double gz = fmax(fmax((double)b.lo[2] - thz, tlz - (double)b.hi[2]), 0.0);
  const double ux = gx * (double)ihx, uy = gy * (double)ihy, uz = gz * (double)ihz;
  return (ux * ux + uy * uy) + uz * uz;
}

// float32 canonical squared distance lower bound (k-NN selection).
__device__ __forceinline__ float box_gap_d2(const NodeBox& b, float tlx, float tly, float tlz,
                                            float thx, float thy, float thz) {
  float gx = fmaxf(fmaxf(__fsub_rn(b.lo[0], thx), __fsub_rn(tlx, b.hi[0])), 0.0f);
  float gy = fmaxf(fmaxf(__fsub_rn(b.lo[1], thy), __fsub_rn(tly, b.hi[1])), 0.0f);
  float gz = fmaxf(fmaxf(__fsub_rn(b.lo[2], thz), __fsub_rn(tlz, b.hi[2])), 0.0f);
  return __fadd_rn(__fadd_rn(__fmul_rn(gx, gx), __fmul_rn(gy, gy)), __fmul_rn(gz, gz));
}

// Depth-first traversal of the 64-ary box hierarchy by one wavefront.
// test(box, node_global_index) -> bool per lane (lane = one child);
// leaves(child_leaf_index, pass, mask) is called for each group of up to 64
// sibling leaves, in increasing leaf order. Children are pushed in reverse
// so the walk emits leaves in ascending (curve) order.
#define SFK_STACK 384
template <class TestF, class LeafF>
__device__ __forceinline__ void traverse(const TreeView& tv, int32_t* stack, TestF test,
                                         LeafF leaves) {
  if (tv.n_levels <= 0) return;
  const int lane = lane_id();
  int sp = 0;
  int level = tv.n_levels - 1;
  int first = 0;
  int cnt = tv.level_cnt[level];
  while (true) {
    const int child = first + lane;
    const bool valid = lane < cnt;
    bool pass = false;
    if (valid) {
      const int g = tv.level_off[level] + child;
      pass = test(tv.nodes[g], g);
    }
    const uint64_t mask = ballot(pass);
    if (level == 0) {
      leaves(child, pass, mask);
    } else if (mask) {
      const int np = popc64(mask);
      if (pass) {
        const int r = popc64(mask & lanemask_lt());
        stack[sp + np - 1 - r] = ((level - 1) << 27) | child;
      }
      sp += np;
      wave_sync();
    }
    if (sp == 0) break;
    --sp;
    const int e = stack[sp];
    const int pl = e >> 27;        // level of the popped node's children
    const int pn = e & ((1 << 27) - 1);
    level = pl;
    first = pn * SFK_FANOUT;
    cnt = min(SFK_FANOUT, tv.level_cnt[pl] - first);
    wave_sync();
  }
}

// traverse() whose leaf callback returns false to end the walk early.
template <class TestF, class LeafF>
__device__ __forceinline__ void traverse_until(const TreeView& tv, int32_t* stack, TestF test,
                                               LeafF leaves) {
  if (tv.n_levels <= 0) return;
  const int lane = lane_id();
  int sp = 0;
  int level = tv.n_levels - 1;
  int first = 0;
  int cnt = tv.level_cnt[level];
  while (true) {
    const int child = first + lane;
    const bool valid = lane < cnt;
    bool pass = false;
    if (valid) {
      const int g = tv.level_off[level] + child;
      pass = test(tv.nodes[g], g);
    }
    const uint64_t mask = ballot(pass);
    if (level == 0) {
      if (!leaves(child, pass, mask)) return;
    } else if (mask) {
      const int np = popc64(mask);
      if (pass) {
        const int r = popc64(mask & lanemask_lt());
        stack[sp + np - 1 - r] = ((level - 1) << 27) | child;
      }
      sp += np;
      wave_sync();
    }
    if (sp == 0) break;
    --sp;
    const int e = stack[sp];
    const int pl = e >> 27;
    const int pn = e & ((1 << 27) - 1);
    level = pl;
    first = pn * SFK_FANOUT;
    cnt = min(SFK_FANOUT, tv.level_cnt[pl] - first);
    wave_sync();
  }
}

}  // namespace sfk
