// Tree build on the device: bounding box, space-filling curve keys
// (Hilbert or Morton), stable LSD radix sort, leaf buckets of 64 particles
// (float4, curve order), a 64-ary box hierarchy, and the per-particle k-th
// nearest neighbour bandwidth.
//
// The paper builds a k-d tree on the CPU and uploads it (Section 3.2);
// here the index is built where the particles live so only ROI descriptors
// ever cross PCIe.
#include "sfk_device.h"

namespace sfk {

// ---------------------------------------------------------------------------
// bounding box + finiteness check
// ---------------------------------------------------------------------------

__device__ __forceinline__ void bbox_take(float v, int axis, float (&mn)[3], float (&mx)[3],
                                          float& bad) {
  if (!isfinite(v)) {
    bad += 1.0f;
    return;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (axis == k) {
      mn[k] = fminf(mn[k], v);
      mx[k] = fmaxf(mx[k], v);
    }
}

// Per block: min and max per axis and the count of non-finite values. With
// a 16-byte aligned array the 3n floats are read as float4 chunks (chunk j
// starts on axis j mod 3) and the last 3n mod 4 floats one by one.
__global__ __launch_bounds__(256) void k_bbox_partial(const float* __restrict__ xyz, int64_t n,
                                                      int vec, float* __restrict__ partial,
                                                      int nblk) {
  __shared__ float lds[7][4];
  float mn[3] = {3.0e38f, 3.0e38f, 3.0e38f}, mx[3] = {-3.0e38f, -3.0e38f, -3.0e38f};
  float bad = 0.0f;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (vec) {
    const int64_t n4 = (3 * n) / 4;
    const float4* x4 = reinterpret_cast<const float4*>(xyz);
    int r = (int)(tid % 3);
    const int dr = (int)(stride % 3);
    for (int64_t j = tid; j < n4; j += stride) {
      const float4 c = x4[j];
      bbox_take(c.x, r, mn, mx, bad);
      bbox_take(c.y, r + 1 == 3 ? 0 : r + 1, mn, mx, bad);
      bbox_take(c.z, r == 0 ? 2 : r - 1, mn, mx, bad);
      bbox_take(c.w, r, mn, mx, bad);
      r += dr;
      if (r >= 3) r -= 3;
    }
    for (int64_t e = 4 * n4 + tid; e < 3 * n; e += stride) bbox_take(xyz[e], (int)(e % 3), mn, mx, bad);
  } else {
    for (int64_t i = tid; i < n; i += stride) {
#pragma unroll
      for (int k = 0; k < 3; ++k) bbox_take(xyz[3 * i + k], k, mn, mx, bad);
    }
  }
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    mn[k] = wave_min(mn[k]);
    mx[k] = wave_max(mx[k]);
  }
  bad = wave_sum(bad);
  if (lane_id() == 0) {
    for (int k = 0; k < 3; ++k) {
      lds[k][w] = mn[k];
      lds[3 + k][w] = mx[k];
    }
    lds[6][w] = bad;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    const int k = threadIdx.x;
    float v = lds[k][0];
    for (int j = 1; j < 4; ++j) {
      const float u = lds[k][j];
      v = k < 3 ? fminf(v, u) : (k < 6 ? fmaxf(v, u) : v + u);
    }
    partial[k * nblk + blockIdx.x] = v;
  }
}

// One block of 1024 threads combines the partials, all 7 components at once.
__global__ __launch_bounds__(1024) void k_bbox_final(const float* __restrict__ partial, int nblk,
                                                     float* __restrict__ result) {
  __shared__ float lds[7][16];
  float v[7] = {3.0e38f, 3.0e38f, 3.0e38f, -3.0e38f, -3.0e38f, -3.0e38f, 0.0f};
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      const float u = partial[k * nblk + i];
      v[k] = k < 3 ? fminf(v[k], u) : (k < 6 ? fmaxf(v[k], u) : v[k] + u);
    }
  }
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    v[k] = k < 3 ? wave_min(v[k]) : (k < 6 ? wave_max(v[k]) : wave_sum(v[k]));
    if (lane_id() == 0) lds[k][w] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    const int k = threadIdx.x;
    float r = lds[k][0];
    for (int j = 1; j < (int)(blockDim.x >> 6); ++j) {
      const float u = lds[k][j];
      r = k < 3 ? fminf(r, u) : (k < 6 ? fmaxf(r, u) : r + u);
    }
    result[k] = r;
  }
}

hipError_t launch_bbox(const float* xyz, int64_t n, float* partial, int nblk, float* result,
                       hipStream_t s) {
  const int vec = ((uintptr_t)xyz & 15) == 0 ? 1 : 0;
  hipLaunchKernelGGL(k_bbox_partial, dim3(nblk), dim3(256), 0, s, xyz, n, vec, partial, nblk);
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(1024), 0, s, partial, nblk, result);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// space-filling curve keys
// ---------------------------------------------------------------------------

__host__ __device__ __forceinline__ uint64_t spread3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

// Key of the cell (x, y, z) of a 2^bits-per-axis lattice, 3*bits bits.
// Morton: the coordinate bits interleaved, x the most significant of each
// triple. Hilbert: J. Skilling's transpose method (Programming the Hilbert
// curve, AIP Conf. Proc. 707, 2004): from the top bit down, each lower bit
// field is inverted or exchanged with x's according to the current bit, a
// Gray-code step then makes the three words the transposed index, whose
// bits are interleaved like Morton's. Consecutive Hilbert keys are
// face-adjacent cells, so 64 consecutive particles span a more compact box
// than under Morton's jumps.
__host__ __device__ __forceinline__ uint64_t curve_key(uint32_t x, uint32_t y, uint32_t z,
                                                       int bits, int hilbert) {
  if (hilbert) {
    for (uint32_t q = 1u << (bits - 1); q > 1u; q >>= 1) {
      const uint32_t p = q - 1u;
      if (x & q) x ^= p;
      uint32_t t = (x ^ y) & p;
      if (y & q) { x ^= p; t = 0u; }
      x ^= t;
      y ^= t;
      t = (x ^ z) & p;
      if (z & q) { x ^= p; t = 0u; }
      x ^= t;
      z ^= t;
    }
    y ^= x;
    z ^= y;
    uint32_t t = 0u;
    for (uint32_t q = 1u << (bits - 1); q > 1u; q >>= 1)
      if (z & q) t ^= q - 1u;
    x ^= t;
    y ^= t;
    z ^= t;
  }
  return (spread3(x) << 2) | (spread3(y) << 1) | spread3(z);
}

template <typename K>
__global__ __launch_bounds__(256) void k_curve_keys(const float* __restrict__ xyz, int64_t n,
                                                    const float* __restrict__ bbox, int bits,
                                                    int hilbert, K* __restrict__ keys,
                                                    uint32_t* __restrict__ vals) {
  const float cells = (float)(1u << bits);
  float lo[3], sc[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lo[k] = bbox[k];
    const float ext = bbox[3 + k] - bbox[k];
    sc[k] = ext > 0.0f ? cells / ext : 0.0f;
  }
  const uint32_t qmax = (1u << bits) - 1u;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t q[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float f = (xyz[3 * i + k] - lo[k]) * sc[k];
      q[k] = f <= 0.0f ? 0u : (f >= (float)qmax ? qmax : (uint32_t)f);
    }
    keys[i] = (K)curve_key(q[0], q[1], q[2], bits, hilbert);
    vals[i] = (uint32_t)i;
  }
}

hipError_t launch_curve_keys(const float* xyz, int64_t n, const float* bbox, int bits,
                             int hilbert, void* keys, uint32_t* vals, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = std::min<int64_t>((n + 255) / 256, 65536);
  if (3 * bits <= 32)
    hipLaunchKernelGGL(k_curve_keys<uint32_t>, dim3((unsigned)nb), dim3(256), 0, s, xyz, n, bbox,
                       bits, hilbert, (uint32_t*)keys, vals);
  else
    hipLaunchKernelGGL(k_curve_keys<uint64_t>, dim3((unsigned)nb), dim3(256), 0, s, xyz, n, bbox,
                       bits, hilbert, (uint64_t*)keys, vals);
  return hipGetLastError();
}

void curve_keys_host(const uint32_t* cells, int64_t n, int bits, int hilbert, uint64_t* keys) {
  for (int64_t i = 0; i < n; ++i)
    keys[i] = curve_key(cells[3 * i], cells[3 * i + 1], cells[3 * i + 2], bits, hilbert);
}

// ---------------------------------------------------------------------------
// stable LSD radix sort of (u32 or u64 key, u32 value) pairs, 8-bit digits.
// Per pass: block digit histograms (digit-major) -> exclusive scan ->
// scatter. The scatter ranks equal digits inside a wavefront with eight
// ballots (one per digit bit); each wavefront owns a contiguous quarter of
// the block's tile and starts each digit after the earlier wavefronts'
// elements of that digit, so the order of equal keys is preserved; the
// ranked tile is staged in LDS and written out in digit order.
// ---------------------------------------------------------------------------

static constexpr int kRsNT = 256;
static constexpr int kRsItems = 16;
static constexpr int kRsTile = kRsNT * kRsItems;

template <typename K>
__global__ __launch_bounds__(kRsNT) void k_rs_hist(const K* __restrict__ keys, int64_t n,
                                                   int shift, uint32_t* __restrict__ hist,
                                                   int nblk) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll 4
  for (int r = 0; r < kRsItems; ++r) {
    const int64_t g = base + (int64_t)r * kRsNT + threadIdx.x;
    if (g < n) atomicAdd(&h[(uint32_t)(keys[g] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

template <typename K>
__global__ __launch_bounds__(kRsNT) void k_rs_scatter(const K* __restrict__ kin,
                                                      const uint32_t* __restrict__ vin,
                                                      K* __restrict__ kout,
                                                      uint32_t* __restrict__ vout, int64_t n,
                                                      int shift,
                                                      const uint32_t* __restrict__ hist,
                                                      const uint32_t* __restrict__ offs,
                                                      int nblk) {
  // Each wavefront owns a contiguous quarter of the block's tile. Its digit
  // counts give every (wavefront, digit) a first local slot (digits in
  // order, wavefronts in order within a digit); each wavefront then ranks its
  // elements in index order into an LDS copy of the tile (stable), and the
  // tile is written out in that order, so the elements of one digit go to
  // consecutive global positions.
  constexpr int kPerWave = kRsTile / 4;
  __shared__ K stage_k[kRsTile];
  __shared__ uint32_t stage_v[kRsTile];
  __shared__ uint32_t wslot[4][256];  // counts, then next local slot per (wavefront, digit)
  __shared__ uint32_t lstart[256];    // first local slot of each digit
  __shared__ uint32_t gbase[256];     // global position of the digit's first element
  const int tid = threadIdx.x, wave = tid >> 6, lane = lane_id();
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  const int tile_n = (int)min((int64_t)kRsTile, n - base);
  const int w0 = wave * kPerWave;
  for (int d = lane; d < 256; d += 64) wslot[wave][d] = 0;
  wave_sync();
  for (int r = 0; r < kPerWave / 64; ++r) {
    const int li = w0 + r * 64 + lane;
    if (li < tile_n) atomicAdd(&wslot[wave][(uint32_t)(kin[base + li] >> shift) & 255u], 1u);
  }
  // local digit starts: exclusive scan of this block's histogram
  const uint32_t hc = hist[(int64_t)tid * nblk + blockIdx.x];
  uint32_t inc = hc;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(inc, off, 64);
    if (lane >= off) inc += t;
  }
  __shared__ uint32_t wsum[4];
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint32_t start = inc - hc;
  for (int w = 0; w < wave; ++w) start += wsum[w];
  lstart[tid] = start;
  gbase[tid] = offs[(int64_t)tid * nblk + blockIdx.x];
  {
    const uint32_t c0 = wslot[0][tid], c1 = wslot[1][tid], c2 = wslot[2][tid];
    wslot[0][tid] = start;
    wslot[1][tid] = start + c0;
    wslot[2][tid] = start + c0 + c1;
    wslot[3][tid] = start + c0 + c1 + c2;
  }
  __syncthreads();
  const uint64_t lt = lanemask_lt();
  for (int r = 0; r < kPerWave / 64; ++r) {
    const int li = w0 + r * 64 + lane;
    const bool valid = li < tile_n;
    const K key = valid ? kin[base + li] : (K)0;
    const uint32_t val = valid ? vin[base + li] : 0u;
    const uint32_t dig = (uint32_t)(key >> shift) & 255u;
    uint64_t mask = ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dig >> b) & 1u;
      const uint64_t bb = ballot(bit);
      mask &= bit ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)popc64(mask & lt);
    uint32_t slot = 0;
    if (valid) slot = wslot[wave][dig];
    wave_sync();  // every lane has read its digit's slot before the leaders advance it
    if (valid) {
      stage_k[slot + rank] = key;
      stage_v[slot + rank] = val;
      if (rank == 0) wslot[wave][dig] = slot + (uint32_t)popc64(mask);
    }
    wave_sync();
  }
  __syncthreads();
  for (int i = tid; i < tile_n; i += kRsNT) {
    const K key = stage_k[i];
    const uint32_t dig = (uint32_t)(key >> shift) & 255u;
    kout[gbase[dig] + ((uint32_t)i - lstart[dig])] = key;
    vout[gbase[dig] + ((uint32_t)i - lstart[dig])] = stage_v[i];
  }
}

size_t radix_sort_tmp_bytes(int64_t n) {
  const int64_t nblk = (n + kRsTile - 1) / kRsTile;
  const int64_t nh = 256 * nblk;
  return (size_t)nh * 2 * sizeof(uint32_t) + scan_tmp_bytes(nh) + 1024;
}

template <typename K>
static hipError_t radix_sort_impl(K* keys, uint32_t* vals, K* keys_alt, uint32_t* vals_alt,
                                  int64_t n, int key_bits, void* tmp, size_t tmp_bytes,
                                  hipStream_t s, int* result_in_alt) {
  *result_in_alt = 0;
  if (n <= 1) return hipSuccess;
  const int64_t nblk = (n + kRsTile - 1) / kRsTile;
  const int64_t nh = 256 * nblk;
  if (radix_sort_tmp_bytes(n) > tmp_bytes) return hipErrorInvalidValue;
  uint32_t* hist = (uint32_t*)tmp;
  uint32_t* offs = hist + nh;
  void* stmp = (void*)(offs + nh);
  const size_t stmp_bytes = tmp_bytes - (size_t)nh * 2 * sizeof(uint32_t);
  K *ka = keys, *kb = keys_alt;
  uint32_t *va = vals, *vb = vals_alt;
  const int passes = (key_bits + 7) / 8;
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    hipLaunchKernelGGL(k_rs_hist<K>, dim3((unsigned)nblk), dim3(kRsNT), 0, s, ka, n, shift, hist,
                       (int)nblk);
    hipError_t e = scan_exclusive_u32(hist, offs, nh, stmp, stmp_bytes, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rs_scatter<K>, dim3((unsigned)nblk), dim3(kRsNT), 0, s, ka, va, kb, vb,
                       n, shift, hist, offs, (int)nblk);
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  *result_in_alt = (passes & 1) ? 1 : 0;
  return hipGetLastError();
}

hipError_t radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt,
                            uint32_t* vals_alt, int64_t n, int key_bits, void* tmp,
                            size_t tmp_bytes, hipStream_t s, int* result_in_alt) {
  return radix_sort_impl(keys, vals, keys_alt, vals_alt, n, key_bits, tmp, tmp_bytes, s,
                         result_in_alt);
}

hipError_t radix_sort_pairs_u32(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                                uint32_t* vals_alt, int64_t n, int key_bits, void* tmp,
                                size_t tmp_bytes, hipStream_t s, int* result_in_alt) {
  if (key_bits > 32) return hipErrorInvalidValue;
  return radix_sort_impl(keys, vals, keys_alt, vals_alt, n, key_bits, tmp, tmp_bytes, s,
                         result_in_alt);
}

// ---------------------------------------------------------------------------
// leaf layout
// ---------------------------------------------------------------------------

// Sub-blocks of 8 consecutive particles inside a leaf: the k-NN search
// bounds a query's distance to each by the sub-block's box.
constexpr int kKnnSub = 8;                          // particles per sub-block
constexpr int kKnnSubPerLeaf = SFK_LEAF / kKnnSub;  // sub-blocks per leaf
constexpr int kKnnBoxFloats = 8 * kKnnSubPerLeaf;   // a leaf's sub-block boxes, <= 64
static_assert(kKnnBoxFloats <= 64, "a leaf's sub-block boxes are loaded one float per lane");

// One wavefront per leaf. Particle perm[i] of the input goes to slot i as
// (x, y, z, 0), slots from n on get the sentinel, and from the same registers
// the kernel writes the leaf's box (the leaf level of the hierarchy, as
// k_leaf_boxes computes it) and, with sub_box set, the boxes of the leaf's
// sub-blocks: 8 floats per box (lo.xyz, 0, hi.xyz, 0), so one 256-byte line
// holds a leaf's eight. A box without real particles is empty (lo > hi), and
// its distance to any point is infinite.
__global__ __launch_bounds__(256) void k_gather(const float* __restrict__ xyz,
                                                const uint32_t* __restrict__ perm, int64_t n,
                                                int32_t n_leaves, float4* __restrict__ pts,
                                                int32_t* __restrict__ perm_out,
                                                NodeBox* __restrict__ leaf_box,
                                                float4* __restrict__ sub_box) {
  const int lane = lane_id();
  for (int leaf = blockIdx.x * 4 + (threadIdx.x >> 6); leaf < n_leaves; leaf += gridDim.x * 4) {
    const int64_t slot = (int64_t)leaf * SFK_LEAF + lane;
    float4 p = make_float4(SFK_SENTINEL, SFK_SENTINEL, SFK_SENTINEL, 0.0f);
    if (slot < n) {
      const uint32_t j = perm[slot];
      p = make_float4(xyz[3 * (int64_t)j], xyz[3 * (int64_t)j + 1], xyz[3 * (int64_t)j + 2],
                      0.0f);
      perm_out[slot] = (int32_t)j;
    }
    pts[slot] = p;
    const bool real = slot < n && p.x < 1.0e29f;
    const float lo[3] = {real ? p.x : 3.0e38f, real ? p.y : 3.0e38f, real ? p.z : 3.0e38f};
    const float hi[3] = {real ? p.x : -3.0e38f, real ? p.y : -3.0e38f, real ? p.z : -3.0e38f};
    if (sub_box) {  // uniform: every lane of the wave takes part in the shuffles
      float v[6] = {lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]};
#pragma unroll
      for (int off = 1; off < kKnnSub; off <<= 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          v[c] = fminf(v[c], __shfl_xor(v[c], off, 64));
          v[c + 3] = fmaxf(v[c + 3], __shfl_xor(v[c + 3], off, 64));
        }
      }
      if ((lane & (kKnnSub - 1)) == 0) {
        float4* o = sub_box + (slot / kKnnSub) * 2;
        o[0] = make_float4(v[0], v[1], v[2], 0.0f);
        o[1] = make_float4(v[3], v[4], v[5], 0.0f);
      }
    }
    NodeBox b;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      b.lo[k] = wave_min(lo[k]);
      b.hi[k] = wave_max(hi[k]);
    }
    b.count = popc64(ballot(real));
    b.first = leaf * SFK_LEAF;
    if (lane == 0) leaf_box[leaf] = b;
  }
}

hipError_t launch_gather(const float* xyz, const uint32_t* perm, int64_t n, int32_t n_leaves,
                         float4* pts, int32_t* perm_out, NodeBox* leaf_box, float* sub_box,
                         hipStream_t s) {
  if (n_leaves <= 0) return hipSuccess;
  if (n > (int64_t)n_leaves * SFK_LEAF) return hipErrorInvalidValue;
  const int nb = std::min<int>((n_leaves + 3) / 4, 65536);
  hipLaunchKernelGGL(k_gather, dim3(nb), dim3(256), 0, s, xyz, perm, n, n_leaves, pts, perm_out,
                     leaf_box, reinterpret_cast<float4*>(sub_box));
  return hipGetLastError();
}

// One wavefront per leaf: box of the real (non-sentinel) particles. With
// only_if set, the launch does nothing unless *only_if is non-zero (a
// refresh that only particles moved to the sentinel would make necessary).
__global__ __launch_bounds__(256) void k_leaf_boxes(const float4* __restrict__ pts, int64_t n,
                                                    int32_t n_leaves, NodeBox* __restrict__ out,
                                                    const int32_t* __restrict__ only_if) {
  if (only_if && *only_if == 0) return;
  const int lane = lane_id();
  for (int leaf = blockIdx.x * 4 + (threadIdx.x >> 6); leaf < n_leaves; leaf += gridDim.x * 4) {
    const int64_t slot = (int64_t)leaf * SFK_LEAF + lane;
    const float4 p = pts[slot];
    const bool real = slot < n && p.x < 1.0e29f;
    float lo[3] = {real ? p.x : 3.0e38f, real ? p.y : 3.0e38f, real ? p.z : 3.0e38f};
    float hi[3] = {real ? p.x : -3.0e38f, real ? p.y : -3.0e38f, real ? p.z : -3.0e38f};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      lo[k] = wave_min(lo[k]);
      hi[k] = wave_max(hi[k]);
    }
    const int cnt = popc64(ballot(real));
    if (lane == 0) {
      NodeBox b;
      for (int k = 0; k < 3; ++k) {
        b.lo[k] = lo[k];
        b.hi[k] = hi[k];
      }
      b.first = leaf * SFK_LEAF;
      b.count = cnt;
      out[leaf] = b;
    }
  }
}

hipError_t launch_leaf_boxes(const float4* pts, int64_t n, int32_t n_leaves, NodeBox* out,
                             const int32_t* only_if, hipStream_t s) {
  if (n_leaves <= 0) return hipSuccess;
  // grid-stride: a launch that finds only_if clear ends after few blocks
  const int nb = std::min<int>((n_leaves + 3) / 4, 4096);
  hipLaunchKernelGGL(k_leaf_boxes, dim3(nb), dim3(256), 0, s, pts, n, n_leaves, out, only_if);
  return hipGetLastError();
}

// One wavefront per parent: union of up to 64 child boxes (only_if as
// for the leaves).
__global__ __launch_bounds__(256) void k_level_boxes(const NodeBox* __restrict__ child,
                                                     int32_t n_child,
                                                     NodeBox* __restrict__ parent,
                                                     int32_t n_parent,
                                                     const int32_t* __restrict__ only_if) {
  if (only_if && *only_if == 0) return;
  const int lane = lane_id();
  for (int p = blockIdx.x * 4 + (threadIdx.x >> 6); p < n_parent; p += gridDim.x * 4) {
    const int c = p * SFK_FANOUT + lane;
    float lo[3] = {3.0e38f, 3.0e38f, 3.0e38f}, hi[3] = {-3.0e38f, -3.0e38f, -3.0e38f};
    int cnt = 0;
    if (c < n_child) {
      const NodeBox b = child[c];
      if (b.count > 0) {
        for (int k = 0; k < 3; ++k) {
          lo[k] = b.lo[k];
          hi[k] = b.hi[k];
        }
        cnt = b.count;
      }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      lo[k] = wave_min(lo[k]);
      hi[k] = wave_max(hi[k]);
    }
    cnt = wave_sum(cnt);
    if (lane == 0) {
      NodeBox b;
      for (int k = 0; k < 3; ++k) {
        b.lo[k] = lo[k];
        b.hi[k] = hi[k];
      }
      b.first = p * SFK_FANOUT;
      b.count = cnt;
      parent[p] = b;
    }
  }
}

hipError_t launch_level_boxes(const NodeBox* child, int32_t n_child, NodeBox* parent,
                              int32_t n_parent, const int32_t* only_if, hipStream_t s) {
  if (n_parent <= 0) return hipSuccess;
  const int nb = std::min<int>((n_parent + 3) / 4, 4096);
  hipLaunchKernelGGL(k_level_boxes, dim3(nb), dim3(256), 0, s, child, n_child, parent, n_parent,
                     only_if);
  return hipGetLastError();
}

// Per-node minimum inverse bandwidth per axis (largest support) for pruning
// with per-particle bandwidths.
__global__ __launch_bounds__(256) void k_leaf_ih(const float4* __restrict__ pts,
                                                 const float4* __restrict__ pparam,
                                                 int32_t pp_mode, int64_t n, int32_t n_leaves,
                                                 float4* __restrict__ out) {
  const int lane = lane_id();
  for (int leaf = blockIdx.x * 4 + (threadIdx.x >> 6); leaf < n_leaves; leaf += gridDim.x * 4) {
    const int64_t slot = (int64_t)leaf * SFK_LEAF + lane;
    const float4 p = pts[slot];
    const bool real = slot < n && p.x < 1.0e29f;
    float m[3] = {3.0e38f, 3.0e38f, 3.0e38f};
    if (real) {
      if (pp_mode == PP_ANISO) {
        const float4 q = pparam[slot];
        m[0] = q.x;
        m[1] = q.y;
        m[2] = q.z;
      } else {
        m[0] = m[1] = m[2] = p.w;
      }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) m[k] = wave_min(m[k]);
    if (lane == 0) out[leaf] = make_float4(m[0], m[1], m[2], 0.0f);
  }
}

__global__ __launch_bounds__(256) void k_level_ih(const float4* __restrict__ child, int32_t n_child,
                                                  float4* __restrict__ parent, int32_t n_parent) {
  const int lane = lane_id();
  for (int p = blockIdx.x * 4 + (threadIdx.x >> 6); p < n_parent; p += gridDim.x * 4) {
    const int c = p * SFK_FANOUT + lane;
    float m[3] = {3.0e38f, 3.0e38f, 3.0e38f};
    if (c < n_child) {
      const float4 q = child[c];
      m[0] = q.x;
      m[1] = q.y;
      m[2] = q.z;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) m[k] = wave_min(m[k]);
    if (lane == 0) parent[p] = make_float4(m[0], m[1], m[2], 0.0f);
  }
}

hipError_t launch_node_ih(const float4* pts, const float4* pparam, int32_t pp_mode, int64_t n,
                          const NodeBox* nodes, const int32_t* level_off,
                          const int32_t* level_cnt, int n_levels, float4* node_ih,
                          int leaf_done, hipStream_t s) {
  (void)nodes;
  if (n_levels <= 0) return hipSuccess;
  int nb = std::min<int>((level_cnt[0] + 3) / 4, 65536);
  if (!leaf_done)
    hipLaunchKernelGGL(k_leaf_ih, dim3(nb), dim3(256), 0, s, pts, pparam, pp_mode, n,
                       level_cnt[0], node_ih + level_off[0]);
  for (int l = 1; l < n_levels; ++l) {
    nb = std::min<int>((level_cnt[l] + 3) / 4, 65536);
    hipLaunchKernelGGL(k_level_ih, dim3(nb), dim3(256), 0, s, node_ih + level_off[l - 1],
                       level_cnt[l - 1], node_ih + level_off[l], level_cnt[l]);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k-th nearest neighbour squared distance (per-point bandwidth).
// One wavefront per leaf, one query particle per lane; each lane keeps its
// KM smallest squared distances in a sorted register array whose last slot
// is its current k-th smallest (the threshold). The lane's own leaf and its
// nearest neighbours along the curve come first and bound every answer from above by
// real distances. The box hierarchy is then walked with the wavefront's
// largest threshold (a box farther than that cannot hold a closer
// particle); the leaves it yields are kept in a per-wave list and visited
// nearest-first in five distance bands, so thresholds shrink early. Per
// visited leaf a lane takes part only if its own threshold exceeds its
// distance to the leaf box, and per group of 8 particles only if it exceeds
// its distance to that group's box. Exact: the canonical float32 distances
// of the definition, selected without approximation; every pruning bound
// uses the same rounded operations, so by monotonicity of rounding it never
// exceeds a distance it stands for.
// ---------------------------------------------------------------------------

constexpr int kKnnList = 256;                       // leaves held for ordering
constexpr int kKnnBands = 5;                        // distance bands of the visiting order
// Curve neighbours of the query leaf visited first, on each side: more
// seed candidates bound the answers of the leaf's edge lanes more tightly
// before the walk (10M points, k = 32, Morton order: 1 -> 4 per side cut the
// kernel by 5%)
template <int KM>
constexpr int knn_near() {
  return KM >= 32 ? 4 : KM >= 16 ? 2 : 1;
}

// Insert x into the ascending array a, dropping the largest entry. Each new
// entry is the median of (old left neighbour, x, old entry), so the updates
// are independent of each other.
template <int KM>
__device__ __forceinline__ void knn_insert(float (&a)[KM], float x) {
#pragma unroll
  for (int i = KM - 1; i >= 1; --i) a[i] = __builtin_amdgcn_fmed3f(a[i - 1], x, a[i]);
  // min(a[0], x) as one operation: the bound -FLT_MAX lies below every
  // distance, and a -inf entry (only ever read as a left neighbour of
  // another -inf entry or of this one) may become -FLT_MAX harmlessly
  a[0] = __builtin_amdgcn_fmed3f(a[0], x, -3.402823466e38f);
}

// Largest unsigned value over the wavefront (uniform result): DPP row
// shifts and row broadcasts, with 0 (the identity of max) for lanes without
// a source, leave the total in lane 63.
__device__ __forceinline__ unsigned wave_max_u32(unsigned b) {
#define SFK_DPP_MAX(CTRL, ROWS) \
  b = max(b, (unsigned)__builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xf, false))
  SFK_DPP_MAX(0x111, 0xf);  // row_shr:1
  SFK_DPP_MAX(0x112, 0xf);  // row_shr:2
  SFK_DPP_MAX(0x114, 0xf);  // row_shr:4
  SFK_DPP_MAX(0x118, 0xf);  // row_shr:8: lane 15 of each row holds the row's max
  SFK_DPP_MAX(0x142, 0xa);  // row_bcast:15
  SFK_DPP_MAX(0x143, 0xc);  // row_bcast:31: lane 63 holds the total
#undef SFK_DPP_MAX
  return (unsigned)__builtin_amdgcn_readlane((int)b, 63);
}

// Largest of the non-negative floats v (+inf allowed) over the wavefront: on
// such values the order of the bit patterns as unsigned integers is the
// order of the floats.
__device__ __forceinline__ float wave_max_nonneg(float v) {
  return __uint_as_float(wave_max_u32(__float_as_uint(v)));
}

// Ascending bitonic sorting network on a register array (N a power of two;
// every index is a compile-time constant, so each compare-exchange is one
// min and one max).
template <int N>
__device__ __forceinline__ void sort_net(float (&v)[N]) {
#pragma unroll
  for (int size = 2; size <= N; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int j = i ^ stride;
        if (j > i) {
          const float lo = fminf(v[i], v[j]), hi = fmaxf(v[i], v[j]);
          const bool up = (i & size) == 0 || size == N;
          v[i] = up ? lo : hi;
          v[j] = up ? hi : lo;
        }
      }
    }
  }
}

// a (N) and b (M <= N) ascending: a becomes the N smallest of both,
// ascending. With b padded by +inf to N values, the elementwise minimum of a
// and reversed b holds exactly those N values as a bitonic sequence, which
// one half-cleaner cascade sorts; the padding leaves a's first N - M alone.
template <int N, int M>
__device__ __forceinline__ void merge_low(float (&a)[N], const float (&b)[M]) {
  static_assert(M <= N, "merge a shorter run into a longer one");
#pragma unroll
  for (int i = 0; i < M; ++i) a[N - M + i] = fminf(a[N - M + i], b[M - 1 - i]);
#pragma unroll
  for (int stride = N >> 1; stride > 0; stride >>= 1) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int j = i ^ stride;
      if (j > i) {
        const float lo = fminf(a[i], a[j]), hi = fmaxf(a[i], a[j]);
        a[i] = lo;
        a[j] = hi;
      }
    }
  }
}

// float32 squared distance from a point to a box, rounded like canon_d2
__device__ __forceinline__ float pt_box_d2(const float* b, float x, float y, float z) {
  const float gx = fmaxf(fmaxf(__fsub_rn(b[0], x), __fsub_rn(x, b[3])), 0.0f);
  const float gy = fmaxf(fmaxf(__fsub_rn(b[1], y), __fsub_rn(y, b[4])), 0.0f);
  const float gz = fmaxf(fmaxf(__fsub_rn(b[2], z), __fsub_rn(z, b[5])), 0.0f);
  return __fadd_rn(__fadd_rn(__fmul_rn(gx, gx), __fmul_rn(gy, gy)), __fmul_rn(gz, gz));
}

#ifndef SFK_KNN_WAVES
#define SFK_KNN_WAVES 4
#endif
#ifndef SFK_KNN_RUN
#define SFK_KNN_RUN 16
#endif

template <int KM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KM <= 32 ? SFK_KNN_WAVES : 2))) void k_knn(TreeView tv, const float* __restrict__ sub_box, int k,
                                             float* __restrict__ h2_sorted,
                                             const float* __restrict__ skip_if) {
  if (skip_if && *skip_if > 0.0f) return;  // the build fails: non-finite coordinates
  __shared__ float4 lds_pts[4][SFK_LEAF];
  __shared__ int32_t lds_stack[4][SFK_STACK];
  __shared__ float lds_d2[4][kKnnSub * 64];
  __shared__ int32_t lds_lid[4][kKnnList];
  __shared__ float lds_lkey[4][kKnnList];
  __shared__ int32_t lds_ord[4][kKnnList];
  __shared__ float4 lds_sb[4][2 * kKnnSubPerLeaf];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  float4* lp = lds_pts[wave];
  float4* lsb = lds_sb[wave];
  float* ld2 = lds_d2[wave];
  int32_t* stack = lds_stack[wave];
  int32_t* lid = lds_lid[wave];
  float* lkey = lds_lkey[wave];
  int32_t* ord = lds_ord[wave];
  const int nl = tv.n_leaves;
  const NodeBox* leaf_box = tv.nodes + tv.level_off[0];
  for (int leaf = blockIdx.x * 4 + wave; leaf < nl; leaf += gridDim.x * 4) {
    const int64_t my = (int64_t)leaf * SFK_LEAF + lane;
    const float4 q = tv.pts[my];
    const bool real = my < tv.n;
    // The first KM - k slots hold -inf and never move, so the last slot is
    // always the k-th smallest distance seen (no runtime index into a).
    float a[KM];
#pragma unroll
    for (int i = 0; i < KM; ++i) a[i] = i < KM - k ? -__builtin_huge_valf() : __builtin_huge_valf();
    float thr = __builtin_huge_valf();
    const NodeBox qb = leaf_box[leaf];

    // One candidate leaf, its particle for this lane in pc and its eight
    // sub-block boxes over the lanes of sbv (8 floats per box). Lanes 0..7
    // first test one box each against the query leaf's box and the
    // wavefront's largest threshold (a box that fails cannot hold a particle
    // closer to any lane than its threshold); the boxes that pass are tested
    // per lane. Per needed sub-block each lane marks the particles below its
    // threshold; the insertion then runs in rounds, a round inserting every
    // lane's next marked particle, until no lane has one left.
    auto process = [&](int cl, const float4 pc, const float sbv) {
      lp[lane] = pc;
      if (lane < kKnnBoxFloats) reinterpret_cast<float*>(lsb)[lane] = sbv;
      wave_sync();
      const float tnow = wave_max_nonneg(real ? thr : 0.0f);
      bool cpass = false;
      if (lane < kKnnSubPerLeaf) {
        const float4 blo = lsb[2 * lane], bhi = lsb[2 * lane + 1];
        const NodeBox b = {{blo.x, blo.y, blo.z}, 0, {bhi.x, bhi.y, bhi.z}, 0};
        cpass = box_gap_d2(b, qb.lo[0], qb.lo[1], qb.lo[2], qb.hi[0], qb.hi[1], qb.hi[2]) < tnow;
      }
      const uint32_t cand = (uint32_t)ballot(cpass);
      uint32_t need = 0;
#pragma unroll
      for (int j = 0; j < kKnnSubPerLeaf; ++j) {
        if (cand & (1u << j)) {
          const float4 blo = lsb[2 * j], bhi = lsb[2 * j + 1];
          const float bx[6] = {blo.x, blo.y, blo.z, bhi.x, bhi.y, bhi.z};
          if (ballot(real && pt_box_d2(bx, q.x, q.y, q.z) < thr)) need |= 1u << j;
        }
      }
      const int self = cl == leaf ? lane : -1;
      while (need) {
        const int j = __ffs(need) - 1;
        need &= need - 1;
        uint32_t mark = 0;
#pragma unroll
        for (int u = 0; u < kKnnSub; ++u) {
          const float4 p = lp[j * kKnnSub + u];
          const float x = canon_d2(q.x, q.y, q.z, p.x, p.y, p.z);
          ld2[u * 64 + lane] = x;  // own column: no other lane reads it
          if (x < thr) mark |= 1u << u;
        }
        // the query itself and padding lanes never insert
        const int rel = self - j * kKnnSub;
        if ((unsigned)rel < (unsigned)kKnnSub) mark &= ~(1u << rel);
        if (!real) mark = 0;
        const int rounds = (int)wave_max_u32((unsigned)__popc(mark));
        for (int r = 0; r < rounds; ++r) {
          // a lane without a mark reads any slot of its column and inserts +inf
          const int u = (__ffs(mark) - 1) & (kKnnSub - 1);
          const float x = mark ? ld2[u * 64 + lane] : __builtin_huge_valf();
          mark &= mark - 1;
          // lanes with x >= thr only touch entries past the k-th: harmless
          knn_insert<KM>(a, x);
          thr = a[KM - 1];
        }
      }
      wave_sync();
    };
    // process() over the leaves ord[0..count), with the next leaf's
    // particles and sub-block boxes in flight
    auto run = [&](int count) {
      if (count <= 0) return;
      int cl = __builtin_amdgcn_readfirstlane(ord[0]);
      float4 pn = tv.pts[(int64_t)cl * SFK_LEAF + lane];
      float sn = lane < kKnnBoxFloats ? sub_box[(int64_t)cl * kKnnBoxFloats + lane] : 0.0f;
      for (int i = 0; i < count; ++i) {
        const int cur = cl;
        const float4 pc = pn;
        const float sc = sn;
        if (i + 1 < count) {
          cl = __builtin_amdgcn_readfirstlane(ord[i + 1]);
          pn = tv.pts[(int64_t)cl * SFK_LEAF + lane];
          sn = lane < kKnnBoxFloats ? sub_box[(int64_t)cl * kKnnBoxFloats + lane] : 0.0f;
        }
        process(cur, pc, sc);
      }
    };

    // Depth-first walk of the box hierarchy that stops whenever the held
    // list may not take another group of 64 leaves and resumes where it
    // stopped (its stack stays in LDS). It keeps the leaves, other than the
    // first pass's, whose box is within tau of this leaf's box.
    float tau = 0.0f;
    int ln = 0, sp = 0, level = 0, first = 0, cnt = 0;
    bool walk_done = false;
    auto collect = [&]() {
      while (!walk_done && ln <= kKnnList - SFK_FANOUT) {
        const int child = first + lane;
        bool pass = false;
        float key = 0.0f;
        if (lane < cnt) {
          key = box_gap_d2(tv.nodes[tv.level_off[level] + child], qb.lo[0], qb.lo[1], qb.lo[2],
                           qb.hi[0], qb.hi[1], qb.hi[2]);
          pass = key <= tau;
        }
        if (level == 0) {
          const bool take = pass && (child < leaf - knn_near<KM>() || child > leaf + knn_near<KM>());
          const uint64_t tm = ballot(take);
          if (take) {
            const int pos = ln + popc64(tm & lanemask_lt());
            lid[pos] = child;
            lkey[pos] = key;
          }
          ln += popc64(tm);
        } else {
          const uint64_t mask = ballot(pass);
          const int np = popc64(mask);
          if (pass) stack[sp + np - 1 - popc64(mask & lanemask_lt())] = ((level - 1) << 27) | child;
          sp += np;
        }
        wave_sync();
        if (sp == 0) {
          walk_done = true;
          break;
        }
        --sp;
        const int e = stack[sp];
        level = e >> 27;
        first = (e & ((1 << 27) - 1)) * SFK_FANOUT;
        cnt = min(SFK_FANOUT, tv.level_cnt[level] - first);
        wave_sync();
      }
    };
    // Order the held leaves by distance band (limits tau/256, tau/64, tau/16,
    // tau/4, open) into ord[], dropping those no
    // lane needs (thresholds only shrink, so a leaf no lane needs now is
    // never needed); leaf boxes come in 64 at a time, one per lane.
    auto order = [&]() {
      int no = 0;
      float lo_lim = -1.0f;
#pragma unroll 1
      for (int band = 0; band < kKnnBands; ++band) {
        // band limits tau / 4^(kKnnBands - 1 - band); the last one is open
        const float hi_lim = band == kKnnBands - 1
                                 ? __builtin_huge_valf()
                                 : tau * __builtin_ldexpf(1.0f, -2 * (kKnnBands - 1 - band));
        for (int i0 = 0; i0 < ln; i0 += 64) {
          const int i = i0 + lane;
          const float key = i < ln ? lkey[i] : -2.0f;
          const bool inb = key > lo_lim && key <= hi_lim;
          uint64_t m = ballot(inb);
          if (!m) continue;
          const int id = i < ln ? lid[i] : 0;
          NodeBox bb = {};
          if (inb) bb = leaf_box[id];
          while (m) {
            const int b = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            const float bx[6] = {readlane_f(bb.lo[0], b), readlane_f(bb.lo[1], b),
                                 readlane_f(bb.lo[2], b), readlane_f(bb.hi[0], b),
                                 readlane_f(bb.hi[1], b), readlane_f(bb.hi[2], b)};
            if (ballot(real && pt_box_d2(bx, q.x, q.y, q.z) < thr)) {
              if (lane == 0) ord[no] = __builtin_amdgcn_readlane(id, b);
              ++no;
            }
          }
        }
        lo_lim = hi_lim;
      }
      ln = 0;
      wave_sync();
      return no;
    };

    // Phase 0 visits the leaf itself and its curve neighbours, which bound
    // every lane's answer from above; tau is then the wavefront's largest
    // bound. Each later phase visits one collected chunk of the walk. One
    // visiting site keeps a single copy of the insertion code.
    for (int phase = 0;; ++phase) {
      int no;
      if (phase == 0) {
        // the leaf, then its curve neighbours at distance 1, 2, ... knn_near
        no = 0;
        if (k == KM) {
          // The leaf's particles are the lanes' own queries. With no -inf
          // slots, a lane's KM smallest distances to them come from sorting
          // networks over KM of them at a time (the query itself and padding
          // at +inf), merged keeping the lower half: the same values the
          // insertion would keep, without its 64 rounds.
          lp[lane] = q;
          wave_sync();
          auto own = [&](int u) {
            const float4 p = lp[u];
            return u == lane ? __builtin_huge_valf() : canon_d2(q.x, q.y, q.z, p.x, p.y, p.z);
          };
#pragma unroll
          for (int i = 0; i < KM; ++i) a[i] = own(i);
          sort_net<KM>(a);
          // the rest in sorted runs of at most 16, so both arrays stay in
          // registers (10M points, k = 32: k-NN 9.09 -> 8.75 ms against the
          // insertion; whole runs of 32: 8.79 ms; the first 32 sorted and the
          // rest inserted: 8.90 ms)
          constexpr int R = KM > SFK_KNN_RUN ? SFK_KNN_RUN : KM;
#pragma unroll
          for (int c0 = KM; c0 < SFK_LEAF; c0 += R) {
            float b[R];
#pragma unroll
            for (int i = 0; i < R; ++i) b[i] = own(c0 + i);
            sort_net<R>(b);
            merge_low<KM, R>(a, b);
          }
          thr = a[KM - 1];
          wave_sync();
        } else {
          if (lane == 0) ord[0] = leaf;
          ++no;
        }
        for (int d = 1; d <= knn_near<KM>(); ++d) {
          if (leaf - d >= 0) {
            if (lane == 0) ord[no] = leaf - d;
            ++no;
          }
          if (leaf + d < nl) {
            if (lane == 0) ord[no] = leaf + d;
            ++no;
          }
        }
        wave_sync();
      } else {
        collect();
        no = order();
      }
      run(no);
      wave_sync();
      if (phase == 0) {
        tau = wave_max(real ? thr : 0.0f);
        level = tv.n_levels - 1;
        first = 0;
        cnt = tv.level_cnt[level];
        walk_done = tv.n_levels <= 0;
      } else if (walk_done) {
        break;
      }
    }
    if (real) h2_sorted[my] = thr;
  }
}

hipError_t launch_knn(TreeView tv, float* sub_box, int k, float* h2_sorted,
                      const float* skip_if, hipStream_t s) {
  if (tv.n_leaves <= 0) return hipSuccess;
  const int nb = std::min<int>((tv.n_leaves + 3) / 4, 65536);
  if (k <= 8)
    hipLaunchKernelGGL(k_knn<8>, dim3(nb), dim3(256), 0, s, tv, sub_box, k, h2_sorted,
                       skip_if);
  else if (k <= 16)
    hipLaunchKernelGGL(k_knn<16>, dim3(nb), dim3(256), 0, s, tv, sub_box, k, h2_sorted,
                       skip_if);
  else if (k <= 32)
    hipLaunchKernelGGL(k_knn<32>, dim3(nb), dim3(256), 0, s, tv, sub_box, k, h2_sorted,
                       skip_if);
  else
    hipLaunchKernelGGL(k_knn<64>, dim3(nb), dim3(256), 0, s, tv, sub_box, k, h2_sorted,
                       skip_if);
  return hipGetLastError();
}

size_t knn_sub_box_bytes(int32_t n_leaves) {
  return sizeof(float) * 8 * (size_t)n_leaves * kKnnSubPerLeaf;
}

// Per-particle isotropic inverse bandwidth into pts[].w:
// ih = (float)(1 / sqrt((double)h2)) from the k-NN result, or
// ih = (float)(1 / (double)h) from a caller-given bandwidth (original order).
// A zero bandwidth has an empty support: the particle is moved to the
// sentinel position so it is never a member.
// One wavefront per leaf: each particle's inverse bandwidth, and the leaf's
// minimum inverse bandwidth (the leaf level of the node bandwidths, as
// k_leaf_ih computes it from the updated particles).
__global__ __launch_bounds__(256) void k_iso_params(float4* __restrict__ pts,
                                                    const float* __restrict__ h2_sorted,
                                                    const float* __restrict__ h_user,
                                                    const int32_t* __restrict__ perm, int64_t n,
                                                    int32_t n_leaves, float4* __restrict__ leaf_ih,
                                                    int32_t* __restrict__ moved) {
  const int lane = lane_id();
  for (int leaf = blockIdx.x * 4 + (threadIdx.x >> 6); leaf < n_leaves; leaf += gridDim.x * 4) {
    const int64_t i = (int64_t)leaf * SFK_LEAF + lane;
    float m = 3.0e38f;
    if (i < n) {
      float4 p = pts[i];
      double h;
      if (h_user)
        h = (double)h_user[perm[i]];
      else
        h = sqrt((double)h2_sorted[i]);
      if (h > 0.0) {
        p.w = (float)(1.0 / h);
      } else {
        p = make_float4(SFK_SENTINEL, SFK_SENTINEL, SFK_SENTINEL, 1.0f);
        *moved = 1;  // the same value from every such lane
      }
      pts[i] = p;
      if (p.x < 1.0e29f) m = p.w;
    }
    m = wave_min(m);
    if (lane == 0) leaf_ih[leaf] = make_float4(m, m, m, 0.0f);
  }
}

__global__ void k_zero_i32(int32_t* p);

hipError_t launch_iso_params(float4* pts, const float* h2_sorted, const float* h_user_orig,
                             const int32_t* perm, int64_t n, int32_t n_leaves, float4* leaf_ih,
                             int32_t* moved, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, s, moved);
  if (n_leaves <= 0) return hipGetLastError();
  const int nb = std::min<int>((n_leaves + 3) / 4, 65536);
  hipLaunchKernelGGL(k_iso_params, dim3(nb), dim3(256), 0, s, pts, h2_sorted, h_user_orig, perm,
                     n, n_leaves, leaf_ih, moved);
  return hipGetLastError();
}

}  // namespace sfk

namespace sfk {

// Count of values that are not finite and > 0 (per-particle bandwidth check).
__global__ __launch_bounds__(256) void k_count_nonpositive(const float* __restrict__ h, int64_t n,
                                                           int32_t* __restrict__ bad) {
  int c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float v = h[i];
    if (!(v > 0.0f) || !isfinite(v)) ++c;
  }
  c = wave_sum(c);
  if (lane_id() == 0 && c) atomicAdd(bad, c);
}

__global__ void k_zero_i32(int32_t* p) { *p = 0; }

hipError_t launch_count_nonpositive(const float* h, int64_t n, int32_t* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, s, bad);
  if (n > 0) {
    const int64_t nb = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_count_nonpositive, dim3((unsigned)nb), dim3(256), 0, s, h, n, bad);
  }
  return hipGetLastError();
}

// Fill a float buffer with zeros (used instead of memset so the launch can
// live inside a captured graph).
__global__ __launch_bounds__(256) void k_fill_f32(float* __restrict__ p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)nb), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace sfk
