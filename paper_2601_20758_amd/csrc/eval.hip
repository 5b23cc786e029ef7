// ROI evaluation: tile-granular range query over the box hierarchy, a
// device-side work plan (prefix sums, heavy tiles split into chunks of
// leaves), and the persistent work-stealing evaluation kernel.
//
// Paper mapping (Section 3.2): Algorithms 2 and 4 give one thread per grid
// node, a range query of radius max(l) per node (Alg. 2) or a loop over all
// particles (Alg. 4), and a kernel sum per node, gathered (no atomics). Here
// one wavefront owns a tile of tx*ty*tz neighbouring nodes; the tile's
// candidate leaves come from one range query per tile; each lane takes one
// particle of a 64-particle leaf and evaluates it against every node of the
// tile, exploiting the grid's separability (the per-axis squared scaled
// distances are computed once per particle and node row); the per-node sums
// are combined across lanes with a transposing butterfly of wavefront
// shuffles. Heavy tiles are split into chunks of leaves whose partial sums
// are combined in a fixed order, so every grid is bitwise reproducible
// whatever batch it runs in.
#include <type_traits>

#include "sfk_device.h"

namespace sfk {

__device__ __forceinline__ int find_roi(const RoiDev* __restrict__ rois, int n_rois, int64_t t) {
  int lo = 0, hi = n_rois - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (rois[mid].tile_base <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

struct TileGeo {
  int r;
  int i0, j0, k0;
  double lo[3], hi[3];
};

template <int TX, int TY, int TZ>
__device__ __forceinline__ TileGeo tile_geo(const RoiDev* __restrict__ rois, int n_rois,
                                            const double* __restrict__ coords, int64_t t) {
  TileGeo g;
  g.r = find_roi(rois, n_rois, t);
  const RoiDev& R = rois[g.r];
  const int64_t lt = t - R.tile_base;
  const int ti = (int)(lt % R.ntile[0]);
  const int tj = (int)((lt / R.ntile[0]) % R.ntile[1]);
  const int tk = (int)(lt / ((int64_t)R.ntile[0] * R.ntile[1]));
  g.i0 = ti * TX;
  g.j0 = tj * TY;
  g.k0 = tk * TZ;
  const int i1 = min(g.i0 + TX, R.res[0]) - 1;
  const int j1 = min(g.j0 + TY, R.res[1]) - 1;
  const int k1 = min(g.k0 + TZ, R.res[2]) - 1;
  const double* cx = coords + R.coord_off;
  const double* cy = cx + R.res[0];
  const double* cz = cy + R.res[1];
  g.lo[0] = cx[g.i0];
  g.hi[0] = cx[i1];
  g.lo[1] = cy[g.j0];
  g.hi[1] = cy[j1];
  g.lo[2] = cz[g.k0];
  g.hi[2] = cz[k1];
  return g;
}

// Box test shared by the count, fill, evaluation and debug walks.
__device__ __forceinline__ bool tile_box_test(const TreeView& tv, const RoiDev& R,
                                              const TileGeo& g, const NodeBox& b, int gidx) {
  float ihx = R.ih[0], ihy = R.ih[1], ihz = R.ih[2];
  if (R.pp_mode != PP_UNIFORM) {
    const float4 m = tv.node_ih[gidx];
    ihx = m.x;
    ihy = m.y;
    ihz = m.z;
  }
  return box_gap_u2(b, g.lo[0], g.lo[1], g.lo[2], g.hi[0], g.hi[1], g.hi[2], ihx, ihy, ihz) <
         (double)R.c2;
}

// ---------------------------------------------------------------------------
// ROI coordinate tables: x_i = lo + (i*(hi-lo))/(res-1) in double.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double node_coord(const RoiDev& R, int k, int i) {
  const double lo = R.lo[k], hi = R.hi[k];
  const double num = __dmul_rn((double)i, __dsub_rn(hi, lo));
  return __dadd_rn(lo, __ddiv_rn(num, (double)(R.res[k] - 1)));
}

__device__ void roi_list_walk(const TreeView& tv, int r, const RoiDev& R, int32_t* stack,
                              int32_t* __restrict__ roi_leaves, int32_t* __restrict__ roi_nl);

// One block per ROI: the coordinate table, then (first wavefront) the ROI's
// leaf list, described below.
__global__ __launch_bounds__(256) void k_roi_coords(TreeView tv, const BatchHdr* __restrict__ hdr,
                                                    const RoiDev* __restrict__ rois,
                                                    double* __restrict__ coords,
                                                    int32_t* __restrict__ roi_leaves,
                                                    int32_t* __restrict__ roi_nl) {
  __shared__ int32_t lds_stack[SFK_STACK];
  if ((int)blockIdx.x >= hdr->n_rois) return;
  const RoiDev& R = rois[blockIdx.x];
  const int tot = R.res[0] + R.res[1] + R.res[2];
  for (int q = threadIdx.x; q < tot; q += blockDim.x) {
    int k = 0, i = q;
    if (i >= R.res[0]) {
      i -= R.res[0];
      k = 1;
      if (i >= R.res[1]) {
        i -= R.res[1];
        k = 2;
      }
    }
    coords[R.coord_off + q] = node_coord(R, k, i);
  }
  if (threadIdx.x < 64) roi_list_walk(tv, (int)blockIdx.x, R, lds_stack, roi_leaves, roi_nl);
}

hipError_t launch_roi_coords(TreeView tv, const BatchHdr* hdr, const RoiDev* rois, int grid_rois,
                             double* coords, int32_t* roi_leaves, int32_t* roi_nl,
                             hipStream_t s) {
  if (grid_rois <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_roi_coords, dim3(grid_rois), dim3(256), 0, s, tv, hdr, rois, coords,
                     roi_leaves, roi_nl);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// ROI leaf lists: one wavefront per ROI walks the hierarchy once with the
// box of all the ROI's nodes and keeps the passing leaves, ascending, when
// there are at most kRoiListCap of them (else the count is -1 and every tile
// walks). A tile's box lies inside the ROI's and the test is monotone in the
// box (rounded subtractions, products with non-negative inverse bandwidths
// and sums are monotone), so every leaf a tile's walk yields is in the list;
// a tile then tests the list's leaves directly and yields the same leaves in
// the same order, without descending from the root.
// ---------------------------------------------------------------------------

// The box of the first and last nodes, computed as the coordinate table
// computes them.
__device__ void roi_list_walk(const TreeView& tv, int r, const RoiDev& R, int32_t* stack,
                              int32_t* __restrict__ roi_leaves, int32_t* __restrict__ roi_nl) {
  const int lane = lane_id();
  TileGeo g;
  g.r = r;
  g.i0 = g.j0 = g.k0 = 0;
  for (int k = 0; k < 3; ++k) {
    g.lo[k] = node_coord(R, k, 0);
    g.hi[k] = node_coord(R, k, R.res[k] - 1);
  }
  int32_t* out = roi_leaves + (int64_t)r * kRoiListCap;
  int cnt = 0;
  traverse_until(
      tv, stack,
      [&](const NodeBox& b, int gidx) { return tile_box_test(tv, R, g, b, gidx); },
      [&](int child, bool pass, uint64_t mask) {
        const int pos = cnt + popc64(mask & lanemask_lt());
        if (pass && pos < kRoiListCap) out[pos] = child;
        cnt += popc64(mask);
        return cnt <= kRoiListCap;
      });
  if (lane == 0) roi_nl[r] = cnt <= kRoiListCap ? cnt : -1;
}

// A tile's candidate leaves: from its ROI's list when there is one, else by
// a walk from the root. leaves(child, pass, mask) per group of up to 64, in
// ascending leaf order either way.
template <class LeafF>
__device__ __forceinline__ void tile_leaves(const TreeView& tv, int32_t* stack, const RoiDev& R,
                                            const TileGeo& g,
                                            const int32_t* __restrict__ roi_leaves,
                                            const int32_t* __restrict__ roi_nl, LeafF leaves) {
  const int nl = roi_nl[g.r];
  if (nl >= 0) {
    const int32_t* list = roi_leaves + (int64_t)g.r * kRoiListCap;
    for (int i0 = 0; i0 < nl; i0 += 64) {
      const int i = i0 + lane_id();
      int child = 0;
      bool pass = false;
      if (i < nl) {
        child = list[i];
        const int gi = tv.level_off[0] + child;
        pass = tile_box_test(tv, R, g, tv.nodes[gi], gi);
      }
      leaves(child, pass, ballot(pass));
    }
    return;
  }
  traverse(
      tv, stack, [&](const NodeBox& b, int gidx) { return tile_box_test(tv, R, g, b, gidx); },
      leaves);
}

// ---------------------------------------------------------------------------
// tile range query: count pass and fill pass (one wavefront per tile)
// ---------------------------------------------------------------------------

template <int TX, int TY, int TZ>
__global__ __launch_bounds__(256) void k_tile_count(TreeView tv, const BatchHdr* __restrict__ hdr,
                                                    const RoiDev* __restrict__ rois,
                                                    const double* __restrict__ coords,
                                                    const int32_t* __restrict__ roi_leaves,
                                                    const int32_t* __restrict__ roi_nl,
                                                    int32_t* __restrict__ tile_cnt,
                                                    int32_t* __restrict__ tile_done,
                                                    int32_t* __restrict__ tile_slots) {
  __shared__ int32_t lds_stack[4][SFK_STACK];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int64_t n_tiles = hdr->n_tiles;
  const int n_rois = hdr->n_rois;
  const int slot_cap = hdr->slot_cap;
  const int poison = hdr->debug_poison;
  for (int64_t t = (int64_t)blockIdx.x * 4 + wave; t < n_tiles; t += (int64_t)gridDim.x * 4) {
    const TileGeo g = tile_geo<TX, TY, TZ>(rois, n_rois, coords, t);
    const RoiDev& R = rois[g.r];
    int cnt = 0;
    int32_t* slot = tile_slots + t * slot_cap;
    tile_leaves(tv, lds_stack[wave], R, g, roi_leaves, roi_nl,
                [&](int child, bool pass, uint64_t mask) {
                  const int pos = cnt + popc64(mask & lanemask_lt());
                  if (pass && pos < slot_cap)
                    slot[pos] = (poison & 1) && pos >= 64 ? tv.n_leaves + child : child;
                  cnt += popc64(mask);
                });
    if (lane == 0) {
      tile_cnt[t] = cnt;
      tile_done[t] = 0;
    }
  }
}

// How a tile is evaluated. Lists: its leaf list and partial slots fit the
// buffers, one work item per chunk of its list. Walk per chunk: only the
// partial slots fit; one work item per chunk, each walking the hierarchy and
// evaluating the leaves of its chunk. Walk whole tile: one work item walks
// and evaluates every chunk in order. All three visit the same leaves in the
// same order with the same chunk boundaries, so the sums are bitwise equal.
static constexpr int kModeWalkTile = 0;
static constexpr int kModeLists = 1;
static constexpr int kModeWalkChunk = 2;

template <int TX, int TY, int TZ>
__global__ __launch_bounds__(256) void k_tile_fill(
    TreeView tv, const BatchHdr* __restrict__ hdr, const RoiDev* __restrict__ rois,
    const double* __restrict__ coords, const int32_t* __restrict__ roi_leaves,
    const int32_t* __restrict__ roi_nl, const int32_t* __restrict__ tile_slots,
    const int32_t* __restrict__ tile_cnt, const int32_t* __restrict__ tile_fit,
    const int64_t* __restrict__ leaf_off,
    const int64_t* __restrict__ chunk_off, int32_t* __restrict__ leaves,
    int32_t* __restrict__ item_tile, int32_t* __restrict__ claims, double* __restrict__ partials,
    const int64_t* __restrict__ partial_off) {
  __shared__ int32_t lds_stack[4][SFK_STACK];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int64_t n_tiles = hdr->n_tiles;
  const int n_rois = hdr->n_rois;
  const int slot_cap = hdr->slot_cap;
  const int poison = hdr->debug_poison;
  for (int64_t t = (int64_t)blockIdx.x * 4 + wave; t < n_tiles; t += (int64_t)gridDim.x * 4) {
    const int64_t c0 = chunk_off[t], c1 = min(chunk_off[t + 1], hdr->item_cap);
    for (int64_t c = c0 + lane; c < c1; c += 64) item_tile[c] = (int32_t)t;
    const int tc = tile_cnt[t];
    if (tc == 0) {
      // no candidate leaf, hence no work item: the tile's nodes are zero
      constexpr int T = TX * TY * TZ;
      const int r = find_roi(rois, n_rois, t);
      const RoiDev& R = rois[r];
      const int64_t lt = t - R.tile_base;
      const int ti = (int)(lt % R.ntile[0]) * TX, tj = (int)((lt / R.ntile[0]) % R.ntile[1]) * TY;
      const int tk = (int)(lt / ((int64_t)R.ntile[0] * R.ntile[1])) * TZ;
      for (int q = lane; q < T; q += 64) {
        const int gi = ti + q % TX, gj = tj + (q / TX) % TY, gk = tk + q / (TX * TY);
        if (gi < R.res[0] && gj < R.res[1] && gk < R.res[2])
          R.out[(int64_t)gi + (int64_t)R.res[0] * ((int64_t)gj + (int64_t)R.res[1] * gk)] = 0.0f;
      }
      continue;
    }
    if (hdr->splat && tile_fit[t] != kModeWalkTile && chunk_off[t + 1] - c0 > 1) {
      // a brick split over several work items: its integer node sums start at 0
      constexpr int64_t T = (int64_t)TX * TY * TZ;
      unsigned long long* sums = (unsigned long long*)(partials) + partial_off[t] * T;
      for (int64_t i = lane; i < T; i += 64) sums[i] = 0ull;
    }
    if (tile_fit[t] != kModeLists) continue;
    int32_t* out = leaves + leaf_off[t];
    if (tc <= slot_cap) {
      // the count pass kept the whole list, in walk order; an entry that is
      // not a leaf of the tree is an internal error: flag it, copy leaf 0
      bool bad = false;
      for (int i = lane; i < tc; i += 64) {
        int v = tile_slots[t * slot_cap + i];
        if ((unsigned)v >= (unsigned)tv.n_leaves) {
          bad = true;
          v = 0;
        }
        out[i] = (poison & 2) && i >= 64 ? tv.n_leaves + v : v;
      }
      if (bad) claims[kErrWord] = 1;
      continue;
    }
    const TileGeo g = tile_geo<TX, TY, TZ>(rois, n_rois, coords, t);
    const RoiDev& R = rois[g.r];
    int cnt = 0;
    tile_leaves(tv, lds_stack[wave], R, g, roi_leaves, roi_nl,
                [&](int child, bool pass, uint64_t mask) {
                  if (pass) out[cnt + popc64(mask & lanemask_lt())] = child;
                  cnt += popc64(mask);
                });
  }
}

// ---------------------------------------------------------------------------
// work plan: per tile, leaf_off (prefix of candidate leaves), partial_off
// (prefix of partial-sum slots of split tiles), tile_fit (how the tile is
// evaluated, below) and chunk_off (prefix of work items). Three launches over
// blocks of kPlanNT consecutive tiles (coalesced; no block waits for
// another): per-block sums of leaves and partial slots; then each block adds
// the sums of the blocks before it, scans its tiles, decides each tile's mode
// from the prefixes and sums its work items; then the same for the items.
// Block 0 of the last launch writes the totals. A batch of at most kPlanNT
// tiles takes one launch of one block instead.
// ---------------------------------------------------------------------------

static constexpr int kPlanNT = 1024;

// Work items of a tile: one per chunk of its leaves. A tile with no
// candidate leaf has none: the fill pass writes its (zero) nodes.
__device__ __forceinline__ int64_t plan_chunks(int64_t cnt, int chunk_leaves) {
  return cnt > 0 ? (cnt + chunk_leaves - 1) / chunk_leaves : 0;
}

// Partial slots a tile needs: one per chunk when it is split (its chunks'
// sums are combined in chunk order), or one for a split brick (its chunks
// add integer node sums into that one slot).
__device__ __forceinline__ int64_t plan_partials(int64_t nch, int splat) {
  return nch > 1 ? (splat ? 1 : nch) : 0;
}

// sum of v over the block (every thread gets it)
__device__ __forceinline__ int64_t block_sum(int64_t v, int64_t* lds) {
  int64_t tot;
  (void)block_excl_scan<kPlanNT>(v, &tot, lds);
  return tot;
}

// sum of bs[stride * i + k] over the blocks i < nb
__device__ __forceinline__ int64_t sum_before(const int64_t* __restrict__ bs, int stride, int k,
                                              int64_t nb, int64_t* lds) {
  int64_t v = 0;
  for (int64_t i = threadIdx.x; i < nb; i += kPlanNT) v += bs[stride * i + k];
  return block_sum(v, lds);
}

__global__ __launch_bounds__(kPlanNT) void k_plan_sums(const int32_t* __restrict__ tile_cnt,
                                                       const BatchHdr* __restrict__ hdr,
                                                       int chunk_leaves,
                                                       int64_t* __restrict__ bs) {
  __shared__ int64_t lds[kPlanNT / 64];
  const int64_t n_tiles = hdr->n_tiles;
  const int64_t t = (int64_t)blockIdx.x * kPlanNT + threadIdx.x;
  if ((int64_t)blockIdx.x * kPlanNT >= n_tiles) return;  // whole block past the end
  const int64_t cnt = t < n_tiles ? tile_cnt[t] : 0;
  const int64_t nch = plan_chunks(cnt, chunk_leaves);
  const int64_t sl = block_sum(cnt, lds);
  const int64_t sp = block_sum(t < n_tiles ? plan_partials(nch, hdr->splat) : 0, lds);
  if (threadIdx.x == 0) {
    bs[3 * blockIdx.x] = sl;
    bs[3 * blockIdx.x + 1] = sp;
  }
}

__global__ __launch_bounds__(kPlanNT) void k_plan_modes(const int32_t* __restrict__ tile_cnt,
                                                        const BatchHdr* __restrict__ hdr,
                                                        int chunk_leaves, int64_t* __restrict__ bs,
                                                        int64_t* __restrict__ leaf_off,
                                                        int64_t* __restrict__ partial_off,
                                                        int32_t* __restrict__ tile_fit) {
  __shared__ int64_t lds[kPlanNT / 64];
  const int64_t n_tiles = hdr->n_tiles;
  const int64_t leaf_cap = hdr->leaf_cap;
  const int64_t partial_cap = hdr->partial_cap;
  if ((int64_t)blockIdx.x * kPlanNT >= n_tiles) return;
  const int64_t base_l = sum_before(bs, 3, 0, blockIdx.x, lds);
  const int64_t base_p = sum_before(bs, 3, 1, blockIdx.x, lds);
  const int64_t t = (int64_t)blockIdx.x * kPlanNT + threadIdx.x;
  const bool v = t < n_tiles;
  const int64_t cnt = v ? tile_cnt[t] : 0;
  const int64_t nch = plan_chunks(cnt, chunk_leaves);
  const int64_t pneed = v ? plan_partials(nch, hdr->splat) : 0;
  int64_t tot;
  const int64_t lo = base_l + block_excl_scan<kPlanNT>(cnt, &tot, lds);
  const int64_t po = base_p + block_excl_scan<kPlanNT>(pneed, &tot, lds);
  const bool fit_p = pneed == 0 || po + pneed <= partial_cap;
  // bricks never walk per chunk: their items stay within the list capacity
  const int mode = (lo + cnt <= leaf_cap && fit_p)    ? kModeLists
                   : (fit_p && nch > 1 && !hdr->splat) ? kModeWalkChunk
                                                       : kModeWalkTile;
  const int64_t nit = v && cnt > 0 ? (mode == kModeWalkTile ? 1 : nch) : 0;
  if (v) {
    leaf_off[t] = lo;
    partial_off[t] = po;
    tile_fit[t] = mode;
  }
  const int64_t si = block_sum(nit, lds);
  if (threadIdx.x == 0) bs[3 * blockIdx.x + 2] = si;
}

__global__ __launch_bounds__(kPlanNT) void k_plan_items(const int32_t* __restrict__ tile_cnt,
                                                        BatchHdr* __restrict__ hdr,
                                                        int32_t* __restrict__ claims,
                                                        int chunk_leaves,
                                                        const int64_t* __restrict__ bs,
                                                        int64_t* __restrict__ leaf_off,
                                                        int64_t* __restrict__ partial_off,
                                                        int64_t* __restrict__ chunk_off,
                                                        const int32_t* __restrict__ tile_fit) {
  __shared__ int64_t lds[kPlanNT / 64];
  const int64_t n_tiles = hdr->n_tiles;
  const int64_t nb = (n_tiles + kPlanNT - 1) / kPlanNT;
  if (blockIdx.x == 0) {
    // totals (block 0 runs even for an empty batch)
    const int64_t tl = sum_before(bs, 3, 0, nb, lds);
    const int64_t tp = sum_before(bs, 3, 1, nb, lds);
    const int64_t tc = sum_before(bs, 3, 2, nb, lds);
    const int64_t leaf_cap = hdr->leaf_cap, partial_cap = hdr->partial_cap;
    // every thread of this block has read the header before thread 0 writes it
    __syncthreads();
    if (threadIdx.x < kClaimSlices) claims[threadIdx.x * kClaimStride] = 0;
    if (threadIdx.x == 0) {
      leaf_off[n_tiles] = tl;
      partial_off[n_tiles] = tp;
      chunk_off[n_tiles] = tc;
      hdr->total_leaves = tl;
      hdr->n_items = tc;
      hdr->total_partials = tp;
      hdr->overflow = (tl > leaf_cap || tp > partial_cap) ? 1 : 0;
    }
  }
  if ((int64_t)blockIdx.x >= nb) return;
  const int64_t base_c = sum_before(bs, 3, 2, blockIdx.x, lds);
  const int64_t t = (int64_t)blockIdx.x * kPlanNT + threadIdx.x;
  const bool v = t < n_tiles;
  int64_t nit = 0;
  if (v && tile_cnt[t] > 0)
    nit = tile_fit[t] == kModeWalkTile ? 1 : plan_chunks(tile_cnt[t], chunk_leaves);
  int64_t tot;
  const int64_t co = base_c + block_excl_scan<kPlanNT>(nit, &tot, lds);
  if (v) chunk_off[t] = co;
}

// ---------------------------------------------------------------------------
// evaluation
// ---------------------------------------------------------------------------

// One split stage of the transposing reduction: lanes with bit OFF keep the
// upper half of the live accumulators, the others the lower half; each adds
// its partner's copy of the half it keeps.
template <int N, int OFF, typename A, int T>
__device__ __forceinline__ void xsplit(A (&acc)[T]) {
  const bool up = (lane_id() & OFF) != 0;
#pragma unroll
  for (int i = 0; i < N / 2; ++i) {
    const A lo = acc[i], hi = acc[i + N / 2];
    const A send = up ? lo : hi;
    const A keep = up ? hi : lo;
    acc[i] = keep + __shfl_xor(send, OFF, 64);
  }
}

template <int OFF, typename A, int T>
__device__ __forceinline__ void xfold(A (&acc)[T]) {
#pragma unroll
  for (int i = 0; i < T; ++i) acc[i] = acc[i] + __shfl_xor(acc[i], OFF, 64);
}

template <int OFF, typename A, int T>
__device__ __forceinline__ void fold_down(A (&acc)[T]) {
  if constexpr (OFF >= T && OFF >= 1) {
    xfold<OFF>(acc);
    fold_down<OFF / 2>(acc);
  }
}

template <int N, typename A, int T>
__device__ __forceinline__ void split_down(A (&acc)[T]) {
  if constexpr (N >= 2) {
    xsplit<N, N / 2>(acc);
    split_down<N / 2>(acc);
  }
}

// Reduce T per-lane accumulators over the 64 lanes. Afterwards lane l holds
// node (l * NPL + m) in acc[m] for m < NPL = max(1, T/64); for T < 64 the
// lanes first fold in halves down to T lanes' worth, so lane l holds node
// l mod T. Fixed order: deterministic.
template <typename A, int T>
__device__ __forceinline__ void reduce_nodes(A (&acc)[T]) {
  if constexpr (T >= 64) {
    xsplit<T, 32>(acc);
    xsplit<T / 2, 16>(acc);
    xsplit<T / 4, 8>(acc);
    xsplit<T / 8, 4>(acc);
    xsplit<T / 16, 2>(acc);
    xsplit<T / 32, 1>(acc);
  } else {
    fold_down<32>(acc);
    split_down<T>(acc);
  }
}

// leaf ids of a work item staged in LDS at a time
constexpr int kIdBlock = 256;

// -log2(e)/2 in double: exp(-u2/2) = exp2(KG * u2)
#define SFK_KG64 (-0.72134752044448170368)

// The evaluation kernel. Template parameters: tile shape (TX, TY, TZ), kernel
// (Epanechnikov / truncated Gaussian), bandwidth source (uniform, per-particle
// isotropic, per-particle anisotropic) and counting mode. Membership and the
// Epanechnikov value 1 - u2 are double (same rate as unpacked float32 on
// gfx950), each term then rounded once to float32; the Gaussian factors are
// float32 exp2 of the double exponents.
template <int TX, int TY, int TZ, int KK, int PP, bool CNT>
__global__ __launch_bounds__(256) void k_eval(
    TreeView tv, const RoiDev* __restrict__ rois, const double* __restrict__ coords,
    int chunk_leaves, const int64_t* __restrict__ leaf_off, const int64_t* __restrict__ chunk_off,
    const int64_t* __restrict__ partial_off, const int32_t* __restrict__ tile_cnt,
    const int32_t* __restrict__ tile_fit, const int32_t* __restrict__ leaves,
    const int32_t* __restrict__ item_tile, double* __restrict__ partials,
    int32_t* __restrict__ tile_done, BatchHdr* __restrict__ hdr, int32_t* __restrict__ claims) {
  constexpr int T = TX * TY * TZ;
  constexpr int NPL = T >= 64 ? T / 64 : 1;
  // Per-lane node accumulators are float32: a lane adds one term per drained
  // batch of 64 particles (at most chunk_leaves terms per work item), the 64
  // lanes are combined by a 6-level tree and the chunks of a tile in double.
  // Uniform-bandwidth Epanechnikov tiles of at most 16 nodes accumulate in
  // double (registers allow it), which also saves the per-pair conversion.
  constexpr bool kDoubleAcc = T <= 16 && KK == KK_EPAN && PP == PP_UNIFORM && !CNT;
  using Acc = std::conditional_t<kDoubleAcc, double, float>;
  // particle buffers of the leaf pipeline; each pipeline round appends up to
  // NB leaves to the queue before draining it, hence its capacity
  constexpr int NB = 3;
  constexpr int QCAP = 64 * (NB + 1);
  __shared__ int32_t lds_stack[4][SFK_STACK];
  __shared__ float4 lds_qpts[4][QCAP];
  __shared__ float4 lds_qprm[4][PP == PP_ANISO ? QCAP : 1];
  __shared__ int32_t lds_ids[4][kIdBlock];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int64_t n_items = min(hdr->n_items, hdr->item_cap);  // equal by construction
  const int n_rois = hdr->n_rois;
  // XCD-aware work stealing. Workgroups are dispatched round-robin over the
  // 8 XCDs, each with its own L2. The item list is cut into kClaimSlices
  // contiguous (hence spatially coherent) slices, 8 per XCD, each with its own
  // counter on its own cache line: device-scope atomics serialize per line,
  // so spreading them is what lets many light items be claimed quickly. A
  // wave claims single items from its home slice (one of its XCD's eight);
  // when that slice is exhausted, the 64 lanes read all 64 counters at once
  // (plain loads) and the wave moves to the first slice with items left in
  // its order: its XCD's other slices, then the other XCDs'. Which wave takes
  // an item never changes what the item computes.
  const int xcd = blockIdx.x & 7;
  const int sub = (int)(((blockIdx.x >> 3) * 4 + wave) & 7);
  auto slice_at = [&](int pos) { return ((xcd + (pos >> 3)) & 7) * 8 + ((sub + pos) & 7); };
  auto slice_begin = [&](int sl) { return n_items * sl / kClaimSlices; };
  int cur = slice_at(0);
  while (true) {
    int64_t item = -1;
    while (true) {
      const int64_t b = slice_begin(cur), e = slice_begin(cur + 1);
      int idx = 0;
      if (b < e && lane == 0) idx = atomicAdd(&claims[cur * kClaimStride], 1);
      idx = __shfl(idx, 0, 64);
      if (b + idx < e) {
        item = b + idx;
        break;
      }
      const int my = slice_at(lane);
      const int64_t mb = slice_begin(my), me = slice_begin(my + 1);
      const int seen =
          __hip_atomic_load(&claims[my * kClaimStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint64_t open = __ballot(mb + seen < me);
      if (open == 0) break;
      cur = slice_at(__ffsll((unsigned long long)open) - 1);
    }
    if (item < 0) break;
    const int t = item_tile[item];
    const TileGeo g = tile_geo<TX, TY, TZ>(rois, n_rois, coords, t);
    const RoiDev& R = rois[g.r];
    const double* cx = coords + R.coord_off;
    const double* cy = cx + R.res[0];
    const double* cz = cy + R.res[1];
    double nx[TX], ny[TY], nz[TZ];
#pragma unroll
    for (int i = 0; i < TX; ++i) nx[i] = cx[min(g.i0 + i, R.res[0] - 1)];
#pragma unroll
    for (int j = 0; j < TY; ++j) ny[j] = cy[min(g.j0 + j, R.res[1] - 1)];
#pragma unroll
    for (int k = 0; k < TZ; ++k) nz[k] = cz[min(g.k0 + k, R.res[2] - 1)];
    const float uih0 = R.ih[0], uih1 = R.ih[1], uih2 = R.ih[2];
    const double c2 = R.c2;
    const int cnt = tile_cnt[t];  // > 0: tiles with no candidate leaf have no work item
    const int nch = (cnt + chunk_leaves - 1) / chunk_leaves;

    Acc acc[T];
#pragma unroll
    for (int q = 0; q < T; ++q) acc[q] = (Acc)0;

    // Per-wave queue of particles whose support reaches the tile box. Each
    // leaf is loaded one particle per lane and culled against the tile with
    // the same monotone-rounding bound as the tree walk (a culled particle
    // would only add exact zeros); survivors are appended in leaf-then-lane
    // order and evaluated 64 at a time, so lanes stay busy with particles
    // that can matter. The order is fixed, hence so are the sums.
    float4* qp = lds_qpts[wave];
    float4* qa = lds_qprm[wave];
    int32_t* ids = lds_ids[wave];
    int qn = 0;

    auto eval_point = [&](const float4 p, const float4 prm) {
      float ihx, ihy, ihz;
      double w = 1.0;
      if constexpr (PP == PP_UNIFORM) {
        ihx = uih0;
        ihy = uih1;
        ihz = uih2;
      } else if constexpr (PP == PP_ISO) {
        ihx = ihy = ihz = p.w;
        const double ih = (double)p.w;
        w = (ih * ih) * ih;
      } else {
        ihx = prm.x;
        ihy = prm.y;
        ihz = prm.z;
        w = (double)prm.w;
      }
      const double px = p.x, py = p.y, pz = p.z;
      double sx[TX], sy[TY], sz[TZ];
#pragma unroll
      for (int i = 0; i < TX; ++i) {
        const double u = (nx[i] - px) * (double)ihx;
        sx[i] = u * u;
      }
#pragma unroll
      for (int j = 0; j < TY; ++j) {
        const double u = (ny[j] - py) * (double)ihy;
        sy[j] = u * u;
      }
#pragma unroll
      for (int k = 0; k < TZ; ++k) {
        const double u = (nz[k] - pz) * (double)ihz;
        sz[k] = u * u;
      }
      // A row (i, j) of nodes where no lane's particle reaches (sx + sy >= c2
      // for all 64; u2 only grows with sz) adds exact zeros: skipped.
      if constexpr (CNT) {
#pragma unroll
        for (int j = 0; j < TY; ++j)
#pragma unroll
          for (int i = 0; i < TX; ++i) {
            const double tt = sx[i] + sy[j];
            if (!ballot(tt < c2)) continue;
#pragma unroll
            for (int k = 0; k < TZ; ++k) {
              const double u2 = tt + sz[k];
              acc[i + TX * (j + TY * k)] += (u2 < c2) ? 1.0f : 0.0f;
            }
          }
      } else if constexpr (KK == KK_EPAN && PP == PP_UNIFORM) {
        // 1 - u2 = (1 - (sx + sy)) - sz: one subtraction per node (the
        // rounding differs from 1 - ((sx + sy) + sz) by at most an ulp of
        // double; a term at the support's edge is then +-1e-16, not 0)
#pragma unroll
        for (int j = 0; j < TY; ++j)
#pragma unroll
          for (int i = 0; i < TX; ++i) {
            const double om = 1.0 - (sx[i] + sy[j]);
            if (!ballot(om > 0.0)) continue;
#pragma unroll
            for (int k = 0; k < TZ; ++k) {
              Acc& a = acc[i + TX * (j + TY * k)];
              if constexpr (kDoubleAcc)
                a = a + fmax(om - sz[k], 0.0);
              else
                a = a + (float)fmax(om - sz[k], 0.0);
            }
          }
      } else if constexpr (KK == KK_EPAN) {
        const float wf = (float)w;
#pragma unroll
        for (int j = 0; j < TY; ++j)
#pragma unroll
          for (int i = 0; i < TX; ++i) {
            const double tt = sx[i] + sy[j];
            if (!ballot(tt < c2)) continue;
#pragma unroll
            for (int k = 0; k < TZ; ++k) {
              const double u2 = tt + sz[k];
              const float v = (float)fmax(1.0 - u2, 0.0);
              Acc& a = acc[i + TX * (j + TY * k)];
              a = fmaf(wf, v, a);
            }
          }
      } else {
        float ex[TX], ey[TY], ez[TZ];
        const float wf = (float)w;
#pragma unroll
        for (int i = 0; i < TX; ++i) {
          ex[i] = __builtin_amdgcn_exp2f((float)(SFK_KG64 * sx[i]));
          if constexpr (PP != PP_UNIFORM) ex[i] = ex[i] * wf;
        }
#pragma unroll
        for (int j = 0; j < TY; ++j) ey[j] = __builtin_amdgcn_exp2f((float)(SFK_KG64 * sy[j]));
#pragma unroll
        for (int k = 0; k < TZ; ++k) ez[k] = __builtin_amdgcn_exp2f((float)(SFK_KG64 * sz[k]));
#pragma unroll
        for (int j = 0; j < TY; ++j)
#pragma unroll
          for (int i = 0; i < TX; ++i) {
            const double tt = sx[i] + sy[j];
            if (!ballot(tt < c2)) continue;
            const float exy = ex[i] * ey[j];
#pragma unroll
            for (int k = 0; k < TZ; ++k) {
              const double u2 = tt + sz[k];
              const float e = exy * ez[k];
              Acc& a = acc[i + TX * (j + TY * k)];
              a = a + ((u2 < c2) ? e : 0.0f);
            }
          }
      }
    };

    // evaluate queue entries [0, 64) and move the rest to the front
    auto drain64 = [&]() {
      const float4 p = qp[lane];
      float4 prm = make_float4(0.f, 0.f, 0.f, 0.f);
      if constexpr (PP == PP_ANISO) prm = qa[lane];
      // move entries [64, qn) to the front, 64 at a time in ascending order
      for (int e = lane; e + 64 < qn; e += 64) {
        qp[e] = qp[e + 64];
        if constexpr (PP == PP_ANISO) qa[e] = qa[e + 64];
      }
      qn -= 64;
      wave_sync();
      eval_point(p, prm);
    };
    // evaluate what is left (lanes past the end take a far dummy particle)
    auto drain_rest = [&]() {
      if (qn == 0) return;
      float4 p = make_float4(SFK_SENTINEL, SFK_SENTINEL, SFK_SENTINEL, 1.0f);
      float4 prm = make_float4(1.f, 1.f, 1.f, 0.f);
      if (lane < qn) {
        p = qp[lane];
        if constexpr (PP == PP_ANISO) prm = qa[lane];
      }
      qn = 0;
      wave_sync();
      eval_point(p, prm);
    };

    // particle (and, anisotropic, its parameters) of lane `lane` of leaf lid
    auto fetch = [&](int lid, float4& p, float4& prm) {
      const int64_t slot = (int64_t)lid * SFK_LEAF + lane;
      p = tv.pts[slot];
      if constexpr (PP == PP_ANISO) prm = tv.pparam[slot];
    };
    // does the particle's support reach the tile box? (same monotone bound
    // as the tree walk)
    auto keep_of = [&](const float4 p, const float4 prm) {
      float ihx = uih0, ihy = uih1, ihz = uih2;
      if constexpr (PP == PP_ISO) {
        ihx = ihy = ihz = p.w;
      } else if constexpr (PP == PP_ANISO) {
        ihx = prm.x;
        ihy = prm.y;
        ihz = prm.z;
      }
      const double px = p.x, py = p.y, pz = p.z;
      const double gx = fmax(fmax(g.lo[0] - px, px - g.hi[0]), 0.0);
      const double gy = fmax(fmax(g.lo[1] - py, py - g.hi[1]), 0.0);
      const double gz = fmax(fmax(g.lo[2] - pz, pz - g.hi[2]), 0.0);
      const double ux = gx * (double)ihx, uy = gy * (double)ihy, uz = gz * (double)ihz;
      return ((ux * ux + uy * uy) + uz * uz) < c2;
    };
    // append the kept particles of one leaf (lane order) to the queue; the
    // caller makes the writes visible (wave_sync) before the queue is read
    auto push = [&](const float4 p, const float4 prm, bool keep) {
      const uint64_t m = ballot(keep);
      if (keep) {
        const int pos = qn + popc64(m & lanemask_lt());
        qp[pos] = p;
        if constexpr (PP == PP_ANISO) qa[pos] = prm;
      }
      qn += popc64(m);
    };
    auto cull = [&](const float4 p, const float4 prm, bool live) {
      push(p, prm, live && keep_of(p, prm));
      wave_sync();
    };
    auto cull_push = [&](const float4 p, const float4 prm) {
      cull(p, prm, true);
      if (qn >= 64) drain64();
    };
    auto eval_leaf = [&](int lid) {
      float4 p, prm = make_float4(0.f, 0.f, 0.f, 0.f);
      fetch(lid, p, prm);
      cull_push(p, prm);
    };
    auto end_chunk = [&]() {
      drain_rest();
      reduce_nodes(acc);
    };

    auto node_out = [&](int node, double v) {
      const int i = node % TX, j = (node / TX) % TY, k = node / (TX * TY);
      const int gi = g.i0 + i, gj = g.j0 + j, gk = g.k0 + k;
      if (gi < R.res[0] && gj < R.res[1] && gk < R.res[2])
        R.out[(int64_t)gi + (int64_t)R.res[0] * ((int64_t)gj + (int64_t)R.res[1] * gk)] = (float)v;
    };
    auto lane_node = [&](int m) { return T >= 64 ? lane * NPL + m : (lane & (T - 1)); };
    const bool lane_writes = T >= 64 || lane < T;

    const int mode = tile_fit[t];
    const int c = (int)(item - chunk_off[t]);
    // the chunk's per-node sums: the grid values when the tile has one
    // chunk, else a partial slot, the last chunk to finish combining all
    // of them in chunk order (in double)
    auto finish_chunk = [&]() {
      if (nch == 1) {
        if (lane_writes) {
#pragma unroll
          for (int m = 0; m < NPL; ++m) node_out(lane_node(m), (double)acc[m] * R.scale);
        }
      } else {
        const int64_t pbase = (partial_off[t] + c) * T;
        if (lane_writes) {
#pragma unroll
          for (int m = 0; m < NPL; ++m) partials[pbase + lane_node(m)] = (double)acc[m];
        }
        __threadfence();
        int prev = 0;
        if (lane == 0) prev = atomicAdd(&tile_done[t], 1);
        prev = __shfl(prev, 0, 64);
        if (prev == nch - 1) {
          __threadfence();
          if (lane_writes) {
            const int64_t p0 = partial_off[t] * T;
#pragma unroll
            for (int m = 0; m < NPL; ++m) {
              const int node = lane_node(m);
              double s = 0.0;
              for (int cc = 0; cc < nch; ++cc)
                s += __hip_atomic_load(&partials[p0 + (int64_t)cc * T + node], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
              node_out(node, s * R.scale);
            }
          }
        }
      }
    };
    if (mode == kModeLists) {
      const int64_t lb = leaf_off[t] + (int64_t)c * chunk_leaves;
      const int64_t le = min(lb + chunk_leaves, leaf_off[t] + cnt);
      // Software pipeline over NB particle buffers: a buffer is refilled
      // with the leaf NB places ahead as soon as it has been culled, so
      // NB - 1 leaves are in flight during each cull; the loop is unrolled
      // over the buffers so that no register is copied while its load is
      // pending. The leaf ids of a block of the chunk are staged in LDS
      // first, so reading them never waits on the particle loads.
      for (int64_t b0 = lb; b0 < le; b0 += kIdBlock) {
        const int n = (int)min((int64_t)kIdBlock, le - b0);
        // a list entry that is not a leaf of the tree is an internal error:
        // flag it and read leaf 0 instead (never out of bounds)
        bool bad = false;
        for (int i = lane; i < n; i += 64) {
          int v = leaves[b0 + i];
          if ((unsigned)v >= (unsigned)tv.n_leaves) {
            bad = true;
            v = 0;
          }
          ids[i] = v;
        }
        if (bad) claims[kErrWord] = 1;
        wave_sync();
        // Every buffer is refilled unconditionally (past the end with the
        // block's last leaf, culled as empty), which keeps the count of
        // loads in flight the same on every path through the loop.
        float4 pb[NB], ab[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
          pb[u] = ab[u] = make_float4(0.f, 0.f, 0.f, 0.f);
          fetch(__builtin_amdgcn_readfirstlane(ids[min(u, n - 1)]), pb[u], ab[u]);
          // keep buffer order = issue order (the oldest load is consumed first)
          __builtin_amdgcn_sched_barrier(0);
        }
        for (int i = 0; i < n; i += NB) {
          // appends only need to be visible to the drain: one visibility
          // point per round lets the compiler overlap consecutive culls
#pragma unroll
          for (int u = 0; u < NB; ++u) {
            push(pb[u], ab[u], i + u < n && keep_of(pb[u], ab[u]));
            fetch(__builtin_amdgcn_readfirstlane(ids[min(i + u + NB, n - 1)]), pb[u], ab[u]);
          }
          wave_sync();
          while (qn >= 64) drain64();
        }
        wave_sync();
      }
      end_chunk();
      finish_chunk();
    } else if (mode == kModeWalkChunk) {
      // the list did not fit: walk the hierarchy and evaluate the leaves of
      // this chunk (walk order = list order), stopping after its last one
      const int start = c * chunk_leaves, stop = min(start + chunk_leaves, cnt);
      int done = 0;
      traverse_until(
          tv, lds_stack[wave],
          [&](const NodeBox& b, int gidx) { return tile_box_test(tv, R, g, b, gidx); },
          [&](int child, bool pass, uint64_t mask) {
            (void)pass;
            const int np = popc64(mask);
            if (done + np <= start) {
              done += np;
              return true;
            }
            uint64_t mm = mask;
            while (mm && done < stop) {
              const int b = __ffsll((unsigned long long)mm) - 1;
              mm &= mm - 1;
              if (done >= start) eval_leaf(__shfl(child, b, 64));
              ++done;
            }
            return done < stop;
          });
      end_chunk();
      finish_chunk();
    } else {
      // neither list nor partial slots fit: one work item walks the
      // hierarchy with the same leaf order and the same chunk boundaries
      double dacc[NPL];
#pragma unroll
      for (int m = 0; m < NPL; ++m) dacc[m] = 0.0;
      int done = 0;
      traverse(
          tv, lds_stack[wave],
          [&](const NodeBox& b, int gidx) { return tile_box_test(tv, R, g, b, gidx); },
          [&](int child, bool pass, uint64_t mask) {
            (void)pass;
            uint64_t mm = mask;
            while (mm) {
              const int b = __ffsll((unsigned long long)mm) - 1;
              mm &= mm - 1;
              eval_leaf(__shfl(child, b, 64));
              ++done;
              if (nch > 1 && done % chunk_leaves == 0) {
                end_chunk();
#pragma unroll
                for (int m = 0; m < NPL; ++m) dacc[m] += (double)acc[m];
#pragma unroll
                for (int q = 0; q < T; ++q) acc[q] = (Acc)0;
              }
            }
          });
      if (nch == 1) {
        end_chunk();
        if (lane_writes) {
#pragma unroll
          for (int m = 0; m < NPL; ++m) node_out(lane_node(m), (double)acc[m] * R.scale);
        }
      } else {
        if (done % chunk_leaves != 0) {
          end_chunk();
#pragma unroll
          for (int m = 0; m < NPL; ++m) dacc[m] += (double)acc[m];
        }
        if (lane_writes) {
#pragma unroll
          for (int m = 0; m < NPL; ++m) node_out(lane_node(m), dacc[m] * R.scale);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Brick evaluation by scattering (uniform bandwidths). A workgroup owns a
// brick of kBrick^3 nodes and keeps one 64-bit integer sum per node in LDS.
// Each lane takes one particle of a candidate leaf, computes on each axis the
// range of brick nodes whose distance can be inside the support (rounded
// outwards by a relative 1e-9, so the range never misses a member), and
// visits those nodes only. An Epanechnikov term is (1 - (ux^2 + uy^2)) - uz^2
// in double, counted as floor(v * 2^31 + 1/2) units (0 when v <= 0) with
// an LDS atomic; the support counts and the truncated Gaussian decide
// membership by the canonical u2 = (ux^2 + uy^2) + uz^2 < c2 as the
// definition does (the Gaussian's term is exp(-u2/2) in float). The
// per-particle cost follows the support (about (2h/s)^3 nodes, twice the
// members) instead of a whole tile, and integer sums are exact, so the grid
// is the same whatever the order of particles, chunks or workgroups (alone,
// in any batch, in any evaluation mode). The brick's chunks add their sums
// into one 64-bit slot per node with global atomics; the last chunk to
// finish writes the nodes: sum * 2^-31 * scale, rounded once to float.
// Per term the fixed point adds about 2^-32 at most (in units of the
// kernel's peak) to a node sum.
// ---------------------------------------------------------------------------

// Fixed-point units of a scattered term v in [0, 1]: floor(v * 2^31 + 1/2)
// with one rounding (a fused multiply-add), 0 for v <= 0.
__device__ __forceinline__ unsigned int splat_units(double v) {
  return (unsigned int)fma(fmax(v, 0.0), kSplatUnit, 0.5);
}

// The Epanechnikov term (1 - (ux^2 + uy^2)) - uz^2 in fixed point, from the
// units of its two parts: the row part a = 1 - (ux^2 + uy^2) counts
// splat_units(a) (at most 2^31), uz^2 counts floor(uz^2 2^31 + 1/2) saturated
// at 2^32 - 1, and the term is their difference, 0 when it is not positive
// (one saturating subtraction per node; a pair outside the support counts 0
// up to one unit at its edge).
__device__ __forceinline__ unsigned int epan_z_units(double sz) {
  return (unsigned int)fmin(fma(sz, kSplatUnit, 0.5), 4294967295.0);
}
__device__ __forceinline__ unsigned int epan_units(unsigned int row, unsigned int z) {
  return row > z ? row - z : 0u;
}

// One wave claims the next work item (XCD-aware slices as in k_eval); -1
// when every slice is exhausted. `cur` carries the wave's current slice.
__device__ __forceinline__ int64_t claim_item(int32_t* __restrict__ claims, int64_t n_items,
                                              int xcd, int sub, int& cur) {
  const int lane = lane_id();
  auto slice_at = [&](int pos) { return ((xcd + (pos >> 3)) & 7) * 8 + ((sub + pos) & 7); };
  auto slice_begin = [&](int sl) { return n_items * sl / kClaimSlices; };
  while (true) {
    const int64_t b = slice_begin(cur), e = slice_begin(cur + 1);
    int idx = 0;
    if (b < e && lane == 0) idx = atomicAdd(&claims[cur * kClaimStride], 1);
    idx = __shfl(idx, 0, 64);
    if (b + idx < e) return b + idx;
    const int my = slice_at(lane);
    const int64_t mb = slice_begin(my), me = slice_begin(my + 1);
    const int seen =
        __hip_atomic_load(&claims[my * kClaimStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t open = __ballot(mb + seen < me);
    if (open == 0) return -1;
    cur = slice_at(__ffsll((unsigned long long)open) - 1);
  }
}

// -log2(e)/2 (exp(-u2/2) = exp2(KG * u2)), as in k_eval
#define SFK_KG64S (-0.72134752044448170368)

template <int KK, bool CNT>
__global__ __launch_bounds__(256) void k_splat(
    TreeView tv, const RoiDev* __restrict__ rois, const double* __restrict__ coords,
    int chunk_leaves, const int64_t* __restrict__ leaf_off, const int64_t* __restrict__ chunk_off,
    const int64_t* __restrict__ partial_off, const int32_t* __restrict__ tile_cnt,
    const int32_t* __restrict__ tile_fit, const int32_t* __restrict__ leaves,
    const int32_t* __restrict__ item_tile, double* __restrict__ partials,
    int32_t* __restrict__ tile_done, BatchHdr* __restrict__ hdr, int32_t* __restrict__ claims) {
  constexpr int B = kBrick;
  constexpr int T = B * B * B;
  __shared__ unsigned long long sums[T];
  __shared__ double lds_c[3][B];
  __shared__ int32_t lds_stack[4][SFK_STACK];
  __shared__ int64_t lds_item;
  __shared__ int32_t lds_last;
  unsigned long long* gsum = (unsigned long long*)partials;
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int64_t n_items = min(hdr->n_items, hdr->item_cap);
  const int n_rois = hdr->n_rois;
  const int xcd = blockIdx.x & 7;
  const int sub = (int)((blockIdx.x >> 3) & 7);
  int cur = ((xcd + 0) & 7) * 8 + (sub & 7);
  while (true) {
    if (wave == 0) {
      const int64_t it = claim_item(claims, n_items, xcd, sub, cur);
      if (lane == 0) lds_item = it;
    }
    __syncthreads();
    const int64_t item = lds_item;
    if (item < 0) break;
    const int t = item_tile[item];
    const TileGeo g = tile_geo<B, B, B>(rois, n_rois, coords, t);
    const RoiDev& R = rois[g.r];
    const int n_here[3] = {min(B, R.res[0] - g.i0), min(B, R.res[1] - g.j0),
                           min(B, R.res[2] - g.k0)};
    if (threadIdx.x < 3 * B) {
      const int k = threadIdx.x / B, i = threadIdx.x % B;
      const int o = k == 0 ? g.i0 : k == 1 ? g.j0 : g.k0;
      const int off = R.coord_off + (k > 0 ? R.res[0] : 0) + (k > 1 ? R.res[1] : 0);
      lds_c[k][i] = coords[off + min(o + i, R.res[k] - 1)];
    }
    for (int i = threadIdx.x; i < T; i += 256) sums[i] = 0ull;
    __syncthreads();
    const double c2 = R.c2;
    const double lo[3] = {R.lo[0], R.lo[1], R.lo[2]};
    double inv_s[3], half[3];
    const int org[3] = {g.i0, g.j0, g.k0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      inv_s[k] = (double)(R.res[k] - 1) / (R.hi[k] - R.lo[k]);
      // support half-width in node steps, rounded outwards
      half[k] = sqrt(c2) * inv_s[k] / (double)R.ih[k];
      half[k] = half[k] * (1.0 + 1e-9) + 1e-9;
    }
    const double ih[3] = {(double)R.ih[0], (double)R.ih[1], (double)R.ih[2]};

    // scatter one particle (lane's own) into the brick's node sums
    auto splat = [&](const float4 p) {
      const double pp[3] = {(double)p.x, (double)p.y, (double)p.z};
      int a[3], b[3];
      bool empty = false;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double ic = (pp[k] - lo[k]) * inv_s[k] - (double)org[k];
        const double fa = fmax(ceil(ic - half[k]), 0.0);
        const double fb = fmin(floor(ic + half[k]), (double)(n_here[k] - 1));
        empty |= !(fa <= fb);
        a[k] = empty ? 0 : (int)fa;
        b[k] = empty ? -1 : (int)fb;
      }
      if (empty) return;
      // Lanes of a leaf often share their range: each lane starts its walk
      // over the range at its own rotation (lane mod the range size per
      // axis), so the atomics of one instruction spread over the range's
      // nodes instead of queueing on one.
      const int nx = b[0] - a[0] + 1, ny = b[1] - a[1] + 1, nz = b[2] - a[2] + 1;
      const int rx = lane % nx, ry = (lane >> 2) % ny, rz = (lane >> 4) % nz;
      for (int dz = 0; dz < nz; ++dz) {
        int kz = a[2] + dz + rz;
        kz = kz > b[2] ? kz - nz : kz;
        const double uz = (lds_c[2][kz] - pp[2]) * ih[2];
        const double sz = uz * uz;
        const unsigned int zq = epan_z_units(sz);
        for (int dy = 0; dy < ny; ++dy) {
          int jy = a[1] + dy + ry;
          jy = jy > b[1] ? jy - ny : jy;
          const double uy = (lds_c[1][jy] - pp[1]) * ih[1];
          const double sy = uy * uy;
          const int row = B * (jy + B * kz);
          const int sw = (3 * jy + 5 * kz) & (B - 1);  // bank swizzle of the row
          for (int dx = 0; dx < nx; ++dx) {
            int ix = a[0] + dx + rx;
            ix = ix > b[0] ? ix - nx : ix;
            const double ux = (lds_c[0][ix] - pp[0]) * ih[0];
            if constexpr (KK == KK_EPAN && !CNT) {
              // the Epanechnikov term (1 - (ux^2 + uy^2)) - uz^2, quantised
              const unsigned int q = epan_units(splat_units(1.0 - (ux * ux + sy)), zq);
              if (q != 0u) atomicAdd(&sums[row + ((ix + sw) & (B - 1))], (unsigned long long)q);
            } else {
              const double u2 = (ux * ux + sy) + sz;
              if (u2 < c2) {
                unsigned int q;
                if constexpr (CNT) {
                  q = 1u;
                } else {
                  const float e = __builtin_amdgcn_exp2f((float)(SFK_KG64S * u2));
                  q = splat_units((double)e);
                }
                atomicAdd(&sums[row + ((ix + sw) & (B - 1))], (unsigned long long)q);
              }
            }
          }
        }
      }
    };
    // Listed leaves: a leaf's particles that reach the brick (the same
    // outward-rounded ranges as splat) are queued and scattered 64 at a time,
    // so every lane has a particle. In the leaves of sparse and deep ROIs
    // most particles reach no node of the brick, and a lane per leaf
    // particle left most lanes idle. The order of the integer adds does not
    // change the sums. The queue (particle indices, at most 127) lives in the
    // wave's traversal stack, which listed leaves do not use.
    uint32_t* qi = reinterpret_cast<uint32_t*>(lds_stack[wave]);
    static_assert(SFK_STACK >= 2 * SFK_LEAF, "the queue shares the traversal stack");
    int qn = 0;
    auto reaches = [&](const float4 p) {
      const double pp[3] = {(double)p.x, (double)p.y, (double)p.z};
      bool ok = true;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double ic = (pp[k] - lo[k]) * inv_s[k] - (double)org[k];
        ok &= fmax(ceil(ic - half[k]), 0.0) <= fmin(floor(ic + half[k]), (double)(n_here[k] - 1));
      }
      return ok;
    };
    auto offer = [&](const float4 p, int64_t idx) {
      const bool ok = reaches(p);
      const uint64_t m = ballot(ok);
      if (ok) qi[qn + popc64(m & lanemask_lt())] = (uint32_t)idx;
      qn += popc64(m);
      wave_sync();
      if (qn >= 64) {
        const uint32_t mine = qi[lane];
        for (int e = lane; e + 64 < qn; e += 64) qi[e] = qi[e + 64];
        qn -= 64;
        wave_sync();
        splat(tv.pts[mine]);
      }
    };
    auto drain_rest = [&]() {
      if (qn == 0) return;
      const bool have = lane < qn;
      const uint32_t mine = have ? qi[lane] : 0u;
      qn = 0;
      wave_sync();
      if (have) splat(tv.pts[mine]);
    };
    auto do_leaf = [&](int lid) {
      const float4 p = tv.pts[(int64_t)lid * SFK_LEAF + lane];
      splat(p);
    };

    const int cnt = tile_cnt[t];
    const int nch = (cnt + chunk_leaves - 1) / chunk_leaves;
    const int mode = tile_fit[t];
    const int c = (int)(item - chunk_off[t]);
    if (mode == kModeLists) {
      // the chunk's leaves, every fourth to each wave; ids outside the tree
      // are an internal error (flagged, leaf 0 read instead)
      const int64_t lb = leaf_off[t] + (int64_t)c * chunk_leaves;
      const int64_t le = min(lb + chunk_leaves, leaf_off[t] + cnt);
      auto leaf_at = [&](int64_t q) {
        int lid = leaves[q];
        if ((unsigned)lid >= (unsigned)tv.n_leaves) {
          if (lane == 0) claims[kErrWord] = 1;
          lid = 0;
        }
        return __builtin_amdgcn_readfirstlane(lid);
      };
      // the next leaf's particle is in flight while this one is offered
      if (lb + wave < le) {
        int64_t idx = (int64_t)leaf_at(lb + wave) * SFK_LEAF + lane;
        float4 p = tv.pts[idx];
        for (int64_t q = lb + wave; q < le; q += 4) {
          float4 pn = p;
          int64_t nidx = idx;
          if (q + 4 < le) {
            nidx = (int64_t)leaf_at(q + 4) * SFK_LEAF + lane;
            pn = tv.pts[nidx];
          }
          offer(p, idx);
          p = pn;
          idx = nidx;
        }
      }
      drain_rest();
    } else {
      // walking modes: every wave walks the hierarchy (same order) and takes
      // every fourth leaf of the item's range
      const int start = mode == kModeWalkChunk ? c * chunk_leaves : 0;
      const int stop = mode == kModeWalkChunk ? min(start + chunk_leaves, cnt) : cnt;
      int done = 0;
      traverse_until(
          tv, lds_stack[wave],
          [&](const NodeBox& b, int gidx) { return tile_box_test(tv, R, g, b, gidx); },
          [&](int child, bool pass, uint64_t mask) {
            (void)pass;
            uint64_t mm = mask;
            while (mm && done < stop) {
              const int bl = __ffsll((unsigned long long)mm) - 1;
              mm &= mm - 1;
              if (done >= start && ((done - start) & 3) == wave) do_leaf(__shfl(child, bl, 64));
              ++done;
            }
            return done < stop;
          });
    }
    __syncthreads();
    const double unit = CNT ? 1.0 : 1.0 / kSplatUnit;
    // LDS slot n holds node (ix, jy, kz) with n = B (jy + B kz) + ((ix + sw) mod B)
    auto write_node = [&](int n, unsigned long long v) {
      const int jy = (n / B) % B, kz = n / (B * B);
      const int ix = ((n % B) - ((3 * jy + 5 * kz) & (B - 1))) & (B - 1);
      if (ix < n_here[0] && jy < n_here[1] && kz < n_here[2]) {
        const int64_t gi = g.i0 + ix, gj = g.j0 + jy, gk = g.k0 + kz;
        R.out[gi + (int64_t)R.res[0] * (gj + (int64_t)R.res[1] * gk)] =
            (float)(((double)v * unit) * R.scale);
      }
    };
    if (mode == kModeWalkTile || nch == 1) {
      for (int n = threadIdx.x; n < T; n += 256) write_node(n, sums[n]);
    } else {
      unsigned long long* slot = gsum + partial_off[t] * (int64_t)T;
      for (int n = threadIdx.x; n < T; n += 256)
        if (sums[n]) atomicAdd(&slot[n], sums[n]);
      __threadfence();
      __syncthreads();
      if (threadIdx.x == 0) lds_last = atomicAdd(&tile_done[t], 1) == nch - 1 ? 1 : 0;
      __syncthreads();
      if (lds_last) {
        __threadfence();
        for (int n = threadIdx.x; n < T; n += 256)
          write_node(n, __hip_atomic_load(&slot[n], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Particle sweep (uniform bandwidths, dense ROIs). Where a ROI holds many
// particles per node, a tile re-reads each particle in every tile whose
// support-widened box holds it (about (t + 2h/s)^3 / t^3 tiles for a tile
// of t^3 nodes) and tests it against all the tile's nodes, and each tile
// pays a range query. The sweep reads every particle of the ROI's support
// once. A work item is a (ROI, box) pair, the box taken from the
// hierarchy's first interior level (64 leaves, 4096 particles, compact in
// curve order); the workgroup scatters the box's particles into an LDS
// window of the ROI's nodes that the box's support can reach, with the
// brick's terms and fixed point (the same operations in the same order)
// and LDS atomics into private copies of the window (lane l adds to copy
// l mod ncp), then adds the window's nonzero sums into the batch's 64-bit
// node sums with global atomics. Per node the Epanechnikov term is one
// saturating subtraction of fixed-point units (those of 1 - (ux^2 + uy^2),
// taken once per node row, minus those of uz^2), with no membership branch.
// Integer sums make the grid independent of the order of items, particles
// and workgroups, and equal to the brick's grid bit for bit. For spans of 3
// nodes or more the lanes of a wavefront take particles of different leaves
// of the box, so one instruction's atomics spread over the window instead
// of queueing on the few nodes one leaf reaches; spans of 1 and 2 nodes add
// few terms and take one leaf per wavefront, for coalesced loads. Windows
// wider than W nodes on some axis (W = kSweepWin, half that for 1-node
// spans) are swept in blocks of W^3 nodes, each reading the box again.
// ---------------------------------------------------------------------------

// A squared offset past any support (c^2 <= 9): the sweep gives the nodes
// past a particle's z range this value, so their terms are 0.
constexpr double kSweepFar = 1e300;

// Level of the hierarchy whose boxes are the sweep's work items: the first
// interior level (64 leaves a box) when the tree has one, else the leaves.
__device__ __forceinline__ int sweep_level(const TreeView& tv) { return tv.n_levels >= 2 ? 1 : 0; }

// Support half-width of a ROI in node steps on axis k, rounded outwards so
// that a particle's node range never misses a member (as the brick's).
__device__ __forceinline__ double sweep_half(const RoiDev& R, int k, double* inv_s) {
  *inv_s = (double)(R.res[k] - 1) / (R.hi[k] - R.lo[k]);
  const double h = sqrt((double)R.c2) * *inv_s / (double)R.ih[k];
  return h * (1.0 + 1e-9) + 1e-9;
}

// Block 0 zeroes the claim counters (never the error word), every block a
// stride of the node sums of the header's tiles.
__global__ __launch_bounds__(256) void k_sweep_zero(const BatchHdr* __restrict__ hdr,
                                                    unsigned long long* __restrict__ acc,
                                                    int32_t* __restrict__ claims) {
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < kClaimSlices * kClaimStride; i += blockDim.x) claims[i] = 0;
  constexpr int T = kSweep * kSweep * kSweep;
  const int64_t n = hdr->n_tiles * T;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc[i] = 0ull;
}

// One wavefront per (ROI, group of 64 item boxes): the group's parent box
// first (when the level above exists), then one box per lane, with the
// tiles' box test against the box of all the ROI's nodes; passing boxes are
// appended as (ROI << 32 | box).
__global__ __launch_bounds__(256) void k_sweep_list(TreeView tv, BatchHdr* __restrict__ hdr,
                                                    const RoiDev* __restrict__ rois,
                                                    const double* __restrict__ coords,
                                                    int64_t* __restrict__ items,
                                                    int32_t* __restrict__ claims) {
  const int lane = lane_id();
  const int L = sweep_level(tv);
  const int nb = tv.level_cnt[L];
  const int ng = (nb + 63) >> 6;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (ng == 0 || w >= (int64_t)hdr->n_rois * ng) return;
  const int r = (int)(w / ng), grp = (int)(w % ng);
  const RoiDev& R = rois[r];
  TileGeo g;
  g.r = r;
  g.i0 = g.j0 = g.k0 = 0;
  {
    const double* cx = coords + R.coord_off;
    const double* cy = cx + R.res[0];
    const double* cz = cy + R.res[1];
    g.lo[0] = cx[0];
    g.hi[0] = cx[R.res[0] - 1];
    g.lo[1] = cy[0];
    g.hi[1] = cy[R.res[1] - 1];
    g.lo[2] = cz[0];
    g.hi[2] = cz[R.res[2] - 1];
  }
  if (L + 1 < tv.n_levels) {
    const int gp = tv.level_off[L + 1] + grp;
    if (!tile_box_test(tv, R, g, tv.nodes[gp], gp)) return;
  }
  const int b = grp * 64 + lane;
  bool pass = false;
  if (b < nb) {
    const int gi = tv.level_off[L] + b;
    pass = tv.nodes[gi].count > 0 && tile_box_test(tv, R, g, tv.nodes[gi], gi);
  }
  const uint64_t m = ballot(pass);
  if (m == 0) return;
  unsigned long long base = 0;
  if (lane == 0) base = atomicAdd((unsigned long long*)&hdr->n_items, (unsigned long long)popc64(m));
  base = __shfl(base, 0, 64);
  const int64_t pos = (int64_t)base + popc64(m & lanemask_lt());
  if (pass) {
    if (pos < hdr->item_cap)
      items[pos] = ((int64_t)r << 32) | (int64_t)(uint32_t)b;
    else
      claims[kErrWord] = 1;
  }
}

// (1-node spans ask for 6 waves per SIMD, their register bound without
// spills; more waves spilled and were slower)
template <int KK, bool CNT, int NM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NM == 1 ? 6 : 1)))
void k_sweep(TreeView tv, const BatchHdr* __restrict__ hdr, const RoiDev* __restrict__ rois,
             const int64_t* __restrict__ items, unsigned long long* __restrict__ acc,
             int32_t* __restrict__ claims) {
  // Windows of 1-node spans are blocked at 8^3 nodes: their boxes' windows
  // seldom exceed that, and the smaller LDS array lets 6 blocks share a CU
  // (the register bound) to hide more of the memory latency these light
  // particles wait on (2-node spans lost more to re-read blocks than they
  // gained).
  constexpr int W = NM == 1 ? kSweepWin / 2 : kSweepWin;
  constexpr int S = kSweep;
  // the window's node sums, z fastest, with an odd x stride (W^2 + 1 at
  // most) so that threads reading consecutive x fall in different banks
  constexpr int WN = W * (W * W + 1);
  // (the Epanechnikov adds of spans up to 3 nodes are unmasked: a
  // particle's nodes past its z range add 0 up to kSweepMaxNM - 1 words past
  // a copy, hence the padding, which is never read)
  __shared__ unsigned long long sums[WN + kSweepMaxNM];
  // node coordinates of a block, with kSweepMaxNM more past its end so the
  // unrolled per-particle loops read them without clamping
  constexpr int WC = W + kSweepMaxNM;
  __shared__ double lds_c[3][WC];
  __shared__ int64_t lds_item;
  __shared__ int32_t lds_surv[SFK_FANOUT];
  __shared__ int32_t lds_nsurv;
  const int lane = lane_id();
  const int tid = threadIdx.x;
  const int64_t n_items = min((int64_t)hdr->n_items, hdr->item_cap);
  const int L = sweep_level(tv);
  const int xcd = blockIdx.x & 7;
  const int sub = (int)((blockIdx.x >> 3) & 7);
  int cur = ((xcd + 0) & 7) * 8 + (sub & 7);
  bool bad = false;
  while (true) {
    if (tid < 64) {
      const int64_t it = claim_item(claims, n_items, xcd, sub, cur);
      if (lane == 0) lds_item = it;
    }
    __syncthreads();
    const int64_t pos = lds_item;
    __syncthreads();  // lds_item is rewritten by the next claim
    if (pos < 0) break;
    const int64_t item = items[pos];
    const int r = (int)(item >> 32);
    const int b = (int)(item & 0xffffffff);
    // an item outside the batch or the tree is an internal error (flagged,
    // skipped: nothing is read out of bounds)
    if ((unsigned)r >= (unsigned)hdr->n_rois || (unsigned)b >= (unsigned)tv.level_cnt[L]) {
      bad = true;
      continue;
    }
    const RoiDev& R = rois[r];
    const NodeBox box = tv.nodes[tv.level_off[L] + b];
    const int l0 = L == 1 ? b * SFK_FANOUT : b;
    const int nl = L == 1 ? min(SFK_FANOUT, tv.n_leaves - l0) : 1;
    double inv_s[3], half[3], lo[3], ih[3];
    int w0[3], w1[3];
    bool empty = false;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      half[k] = sweep_half(R, k, &inv_s[k]);
      lo[k] = R.lo[k];
      ih[k] = (double)R.ih[k];
      const double fa = fmax(ceil(((double)box.lo[k] - lo[k]) * inv_s[k] - half[k]), 0.0);
      const double fb =
          fmin(floor(((double)box.hi[k] - lo[k]) * inv_s[k] + half[k]), (double)(R.res[k] - 1));
      empty |= !(fa <= fb);
      w0[k] = empty ? 0 : (int)fa;
      w1[k] = empty ? -1 : (int)fb;
    }
    if (empty) continue;
    const double c2 = (double)R.c2;
    const float4* pts = tv.pts + (int64_t)l0 * SFK_LEAF;
    for (int bz = w0[2]; bz <= w1[2]; bz += W)
      for (int by = w0[1]; by <= w1[1]; by += W)
        for (int bx = w0[0]; bx <= w1[0]; bx += W) {
          const int blk0[3] = {bx, by, bz};
          const int nbk[3] = {min(W, w1[0] - bx + 1), min(W, w1[1] - by + 1),
                              min(W, w1[2] - bz + 1)};
          const int nyz = (nbk[1] * nbk[2]) | 1, nw = nbk[0] * nyz;
          // ncp private copies of the window's sums (odd stride, so the
          // copies of one node fall in different banks): lane l adds to copy
          // l mod ncp, so lanes whose particles reach the same node seldom
          // add to the same word
          int ncp = 16;
          while (ncp > 1 && ncp * (nw | 1) > WN) ncp >>= 1;
          const int cs = ncp > 1 ? (nw | 1) : nw;
          const int my_copy = (lane % ncp) * cs;
          if (tid < 3 * WC) {
            const int k = tid / WC, i = tid % WC;
            lds_c[k][i] = node_coord(R, k, blk0[k] + i);
          }
          for (int i = tid; i < ncp * cs; i += 256) sums[i] = 0ull;
          // the box's leaves whose box can reach the block (a particle's node
          // range lies inside its leaf's, so the others add nothing here)
          if (tid < 64) {
            bool reach = false;
            if (lane < nl) {
              const NodeBox lb = tv.nodes[tv.level_off[0] + l0 + lane];
              reach = lb.count > 0;
#pragma unroll
              for (int k = 0; k < 3; ++k) {
                const double fa = fmax(ceil(((double)lb.lo[k] - lo[k]) * inv_s[k] - half[k]),
                                       (double)blk0[k]);
                const double fb = fmin(floor(((double)lb.hi[k] - lo[k]) * inv_s[k] + half[k]),
                                       (double)(blk0[k] + nbk[k] - 1));
                reach &= fa <= fb;
              }
            }
            const uint64_t m = ballot(reach);
            if (reach) lds_surv[popc64(m & lanemask_lt())] = lane;
            if (lane == 0) lds_nsurv = popc64(m);
          }
          __syncthreads();
          const int ns = lds_nsurv;
          auto splat = [&](const float4 p) {
            const double pp[3] = {(double)p.x, (double)p.y, (double)p.z};
            int a[3], n[3];
            bool ok = true;
            if constexpr (NM == 1) {
              // a support under half a spacing reaches at most the nearest
              // node: per axis the node rint(ic), if within the half-width
#pragma unroll
              for (int k = 0; k < 3; ++k) {
                const double ic = (pp[k] - lo[k]) * inv_s[k];
                const double r = rint(ic);
                ok &= fabs(ic - r) <= half[k] && r >= (double)blk0[k] &&
                      r <= (double)(blk0[k] + nbk[k] - 1);
                a[k] = ok ? (int)r - blk0[k] : 0;
                n[k] = 1;
              }
              if (!ok) return;
            } else {
              // the ranges of all three axes first, one exit, then the
              // conversions (no lane mask per axis)
              double fa[3], fb[3];
#pragma unroll
              for (int k = 0; k < 3; ++k) {
                const double ic = (pp[k] - lo[k]) * inv_s[k];
                fa[k] = fmax(ceil(ic - half[k]), (double)blk0[k]);
                fb[k] = fmin(floor(ic + half[k]), (double)(blk0[k] + nbk[k] - 1));
                ok &= fa[k] <= fb[k];
              }
              if (!ok) return;
#pragma unroll
              for (int k = 0; k < 3; ++k) {
                a[k] = (int)fa[k] - blk0[k];
                n[k] = (int)(fb[k] - fa[k]) + 1;
              }
              if (n[0] > NM || n[1] > NM || n[2] > NM) {
                bad = true;
                return;
              }
            }
            // the particle's first node in this lane's copy of the window
            // (stored z fastest, x stride nyz); a node (mx, my, mz) past it
            // is base + mz + nbk2 my + nyz mx, so a row's adds differ only
            // in the immediate offset
            const int base = my_copy + a[2] + nbk[2] * a[1] + nyz * a[0];
            double sx[NM], sy[NM], sz[NM];
#pragma unroll
            for (int m = 0; m < NM; ++m) {
              const double ux = (lds_c[0][a[0] + m] - pp[0]) * ih[0];
              const double uy = (lds_c[1][a[1] + m] - pp[1]) * ih[1];
              const double uz = (lds_c[2][a[2] + m] - pp[2]) * ih[2];
              sx[m] = ux * ux;
              sy[m] = uy * uy;
              // past the particle's z range a huge square makes every term
              // 0 (no add), so the inner loop needs no range test
              sz[m] = m < n[2] ? uz * uz : kSweepFar;
            }
            unsigned int zq[NM];
#pragma unroll
            for (int m = 0; m < NM; ++m) zq[m] = epan_z_units(sz[m]);
#pragma unroll
            for (int my = 0; my < NM; ++my) {
#pragma unroll
              for (int mx = 0; mx < NM; ++mx) {
                if (mx < n[0] && my < n[1]) {
                  const double sxy = sx[mx] + sy[my];
                  const int row = base + nbk[2] * my + nyz * mx;
                  if constexpr (KK == KK_EPAN && !CNT) {
                    // the Epanechnikov term (1 - (ux^2 + uy^2)) - uz^2,
                    // quantised: no membership test (a non-member's term
                    // counts 0); one saturating subtraction per node
                    // Up to 3 nodes per axis every lane adds, a zero where
                    // its term is 0 (no lane mask per node; the LDS has room
                    // for the extra adds). Wider spans add only nonzero
                    // terms: with 216 or more pairs per particle the unmasked
                    // adds made the LDS the bound (6 nodes: 5.9 -> 10 ms on
                    // a full 100M-point box at 256^3).
                    const unsigned int aq = splat_units(1.0 - sxy);
#pragma unroll
                    for (int mz = 0; mz < NM; ++mz) {
                      const unsigned int q = epan_units(aq, zq[mz]);
                      if (NM <= 3 || q != 0u) atomicAdd(&sums[row + mz], (unsigned long long)q);
                    }
                  } else {
#pragma unroll
                    for (int mz = 0; mz < NM; ++mz) {
                      const double u2 = sxy + sz[mz];
                      if (u2 < c2) {
                        unsigned int q;
                        if constexpr (CNT) {
                          q = 1u;
                        } else {
                          const float e = __builtin_amdgcn_exp2f((float)(SFK_KG64S * u2));
                          q = splat_units((double)e);
                        }
                        atomicAdd(&sums[row + mz], (unsigned long long)q);
                      }
                    }
                  }
                }
              }
            }
          };
          // thread tid takes particles q = tid + 256 i of the surviving
          // leaves, in one of two orders
          if (ns > 0 && NM <= 2) {
            // Spans of 1 and 2 nodes add few terms per particle, so the LDS
            // atomics of one leaf's particles seldom meet (16 private copies
            // for their small windows): consecutive lanes take consecutive
            // particles of one leaf, and a wavefront's load is one 1 KB run
            // instead of 64 cache lines (3-node spans lost more to meeting
            // atomics than they gained)
            const bool all = ns == nl;
            const int total = ns * SFK_LEAF;
            int q = tid;
            if (q < total) {
              float4 p = pts[(int64_t)(all ? q >> 6 : lds_surv[q >> 6]) * SFK_LEAF + (q & 63)];
              while (true) {
                const int qn = q + 256;
                const bool more = qn < total;
                float4 pn = p;
                if (more) pn = pts[(int64_t)(all ? qn >> 6 : lds_surv[qn >> 6]) * SFK_LEAF + (qn & 63)];
                splat(p);
                if (!more) break;
                p = pn;
                q = qn;
              }
            }
          } else if (ns > 0) {
            // wider spans: "leaf q mod ns, slot q / ns", so the lanes of a
            // wavefront take particles of different leaves and one
            // instruction's atomics spread over the window
            const int step_slot = 256 / ns, step_leaf = 256 % ns;
            const bool all = ns == nl;  // every leaf reaches: no indirection
            auto leaf_id = [&](int q) { return all ? q : lds_surv[q]; };
            int leaf = tid % ns, slot = tid / ns;
            if (slot < SFK_LEAF) {
              float4 p = pts[(int64_t)leaf_id(leaf) * SFK_LEAF + slot];
              while (true) {
                int nleaf = leaf + step_leaf, nslot = slot + step_slot;
                if (nleaf >= ns) {
                  nleaf -= ns;
                  ++nslot;
                }
                const bool more = nslot < SFK_LEAF;
                float4 pn = p;
                if (more) pn = pts[(int64_t)leaf_id(nleaf) * SFK_LEAF + nslot];
                splat(p);
                if (!more) break;
                p = pn;
                leaf = nleaf;
                slot = nslot;
              }
            }
          }
          __syncthreads();
          // the window's nonzero sums into the batch's node sums: thread t
          // takes x = t mod W of the x rows t / W, t / W + 256 / W, ...
          // (consecutive threads add to consecutive nodes; the row's (y, z)
          // advances without divisions)
          if ((tid & (W - 1)) < nbk[0]) {
            constexpr int RS = 256 / W;
            const int li = tid & (W - 1);
            int lj = tid / W, lk = 0;
            while (lj >= nbk[1]) {
              lj -= nbk[1];
              ++lk;
            }
            while (lk < nbk[2]) {
              const int w = lk + nbk[2] * lj + nyz * li;
              unsigned long long v = 0ull;
              for (int c = 0; c < ncp; ++c) v += sums[c * cs + w];
              if (v != 0ull) {
                const int gi = blk0[0] + li, gj = blk0[1] + lj, gk = blk0[2] + lk;
                const int64_t t = R.tile_base + (gi / S) +
                                  (int64_t)R.ntile[0] * ((gj / S) + (int64_t)R.ntile[1] * (gk / S));
                atomicAdd(&acc[t * (S * S * S) + (gi % S) + S * ((gj % S) + S * (gk % S))], v);
              }
              lj += RS;
              while (lj >= nbk[1]) {
                lj -= nbk[1];
                ++lk;
              }
            }
          }
          __syncthreads();
        }
  }
  if (bad) claims[kErrWord] = 1;
}

// One block per tile of kSweep^3 nodes: sum * 2^-31 * scale, rounded once to
// float (the brick's conversion).
template <bool CNT>
__global__ __launch_bounds__(256) void k_sweep_write(const BatchHdr* __restrict__ hdr,
                                                     const RoiDev* __restrict__ rois,
                                                     const unsigned long long* __restrict__ acc) {
  constexpr int S = kSweep;
  const int64_t n_tiles = hdr->n_tiles;
  const int n_rois = hdr->n_rois;
  const double unit = CNT ? 1.0 : 1.0 / kSplatUnit;
  for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const int r = find_roi(rois, n_rois, t);
    const RoiDev& R = rois[r];
    const int64_t lt = t - R.tile_base;
    const int i0 = (int)(lt % R.ntile[0]) * S;
    const int j0 = (int)((lt / R.ntile[0]) % R.ntile[1]) * S;
    const int k0 = (int)(lt / ((int64_t)R.ntile[0] * R.ntile[1])) * S;
    for (int n = threadIdx.x; n < S * S * S; n += 256) {
      const int gi = i0 + n % S, gj = j0 + (n / S) % S, gk = k0 + n / (S * S);
      if (gi < R.res[0] && gj < R.res[1] && gk < R.res[2])
        R.out[gi + (int64_t)R.res[0] * (gj + (int64_t)R.res[1] * gk)] =
            (float)(((double)acc[t * (S * S * S) + n] * unit) * R.scale);
    }
  }
}

// ---------------------------------------------------------------------------
// debug: support sets of single nodes (one wavefront per node)
// ---------------------------------------------------------------------------

template <int TX, int TY, int TZ>
__global__ __launch_bounds__(256) void k_debug_candidates(TreeView tv, const int32_t* __restrict__ perm,
                                                          const RoiDev* __restrict__ rois,
                                                          const double* __restrict__ coords,
                                                          int64_t node_begin, int64_t node_end,
                                                          int64_t* __restrict__ cnt_out,
                                                          const int64_t* __restrict__ off,
                                                          int32_t* __restrict__ idx_out) {
  __shared__ int32_t lds_stack[4][SFK_STACK];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const RoiDev& R = rois[0];
  const double* cx = coords + R.coord_off;
  const double* cy = cx + R.res[0];
  const double* cz = cy + R.res[1];
  for (int64_t nd = node_begin + (int64_t)blockIdx.x * 4 + wave; nd < node_end;
       nd += (int64_t)gridDim.x * 4) {
    const int ix = (int)(nd % R.res[0]);
    const int iy = (int)((nd / R.res[0]) % R.res[1]);
    const int iz = (int)(nd / ((int64_t)R.res[0] * R.res[1]));
    const int64_t t = (int64_t)(ix / TX) +
                      (int64_t)R.ntile[0] * ((int64_t)(iy / TY) + (int64_t)R.ntile[1] * (iz / TZ));
    const TileGeo g = tile_geo<TX, TY, TZ>(rois, 1, coords, t);
    const double xn = cx[ix], yn = cy[iy], zn = cz[iz];
    int64_t c = 0;
    int32_t* out = off ? idx_out + off[nd - node_begin] : nullptr;
    traverse(
        tv, lds_stack[wave],
        [&](const NodeBox& b, int gidx) { return tile_box_test(tv, R, g, b, gidx); },
        [&](int child, bool pass, uint64_t mask) {
          (void)pass;
          uint64_t mm = mask;
          while (mm) {
            const int b = __ffsll((unsigned long long)mm) - 1;
            mm &= mm - 1;
            const int lid = __shfl(child, b, 64);
            const int64_t slot = (int64_t)lid * SFK_LEAF + lane;
            const float4 p = tv.pts[slot];
            float ihx = R.ih[0], ihy = R.ih[1], ihz = R.ih[2];
            if (R.pp_mode == PP_ISO) {
              ihx = ihy = ihz = p.w;
            } else if (R.pp_mode == PP_ANISO) {
              const float4 q = tv.pparam[slot];
              ihx = q.x;
              ihy = q.y;
              ihz = q.z;
            }
            const bool mem =
                slot < tv.n && canon_u2(xn, yn, zn, p.x, p.y, p.z, ihx, ihy, ihz) < (double)R.c2;
            const uint64_t mb = ballot(mem);
            if (out && mem) out[c + popc64(mb & lanemask_lt())] = perm[slot];
            c += popc64(mb);
          }
        });
    if (!off && lane == 0) cnt_out[nd - node_begin] = c;
  }
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------

bool tile_shape_supported(TileShape ts) {
  return (ts.tx == 4 && ts.ty == 4 && (ts.tz == 4 || ts.tz == 2)) ||
         (ts.tx == 4 && ts.ty == 2 && ts.tz == 2) || (ts.tx == 2 && ts.ty == 2 && ts.tz == 2) ||
         (ts.tx == 1 && ts.ty == 1 && ts.tz == 1) || is_brick(ts) || is_sweep(ts);
}

bool is_brick(TileShape ts) { return ts.tx == kBrick && ts.ty == kBrick && ts.tz == kBrick; }
bool is_sweep(TileShape ts) { return ts.tx == kSweep && ts.ty == kSweep && ts.tz == kSweep; }

hipError_t launch_sweep_list(TreeView tv, BatchHdr* hdr, const RoiDev* rois,
                             const double* coords, int64_t* items, unsigned long long* acc,
                             int32_t* claims, int max_rois, int64_t max_tiles, hipStream_t s) {
  constexpr int64_t T = kSweep * kSweep * kSweep;
  const int zb = (int)std::max<int64_t>(1, std::min<int64_t>((max_tiles * T + 255) / 256, 8192));
  hipLaunchKernelGGL(k_sweep_zero, dim3(zb), dim3(256), 0, s, hdr, acc, claims);
  const int L = tv.n_levels >= 2 ? 1 : 0;
  const int64_t ng = ((int64_t)tv.level_cnt[L] + 63) / 64;
  const int64_t waves = ng * std::max(1, max_rois);
  if (waves > 0)
    hipLaunchKernelGGL(k_sweep_list, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, tv, hdr,
                       rois, coords, items, claims);
  return hipGetLastError();
}

hipError_t launch_sweep_eval(TreeView tv, const BatchHdr* hdr, const RoiDev* rois,
                             const double* coords, int kk, bool cnt, int nm,
                             const int64_t* items, unsigned long long* acc, int32_t* claims,
                             int grid_blocks, int n_cu, int64_t max_tiles, hipStream_t s) {
  (void)coords;
  if (nm < 1 || nm > kSweepMaxNM) return hipErrorInvalidValue;
#define SFK_W(KK, C, NM)                                                                      \
  do {                                                                                        \
    static int occ_ = 0;                                                                      \
    if (occ_ == 0) {                                                                          \
      int b_ = 0;                                                                             \
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b_, k_sweep<KK, C, NM>, 256, 0) !=    \
              hipSuccess ||                                                                   \
          b_ < 1)                                                                             \
        b_ = 1;                                                                               \
      occ_ = b_;                                                                              \
    }                                                                                         \
    const int g_ = grid_blocks > 0 ? grid_blocks : n_cu * occ_;                               \
    hipLaunchKernelGGL((k_sweep<KK, C, NM>), dim3(g_), dim3(256), 0, s, tv, hdr, rois, items, \
                       acc, claims);                                                          \
  } while (0)
#define SFK_W_NM(KK, C)        \
  switch (nm) {                \
    case 1: SFK_W(KK, C, 1); break; \
    case 2: SFK_W(KK, C, 2); break; \
    case 3: SFK_W(KK, C, 3); break; \
    case 4: SFK_W(KK, C, 4); break; \
    case 5: SFK_W(KK, C, 5); break; \
    case 6: SFK_W(KK, C, 6); break; \
    case 7: SFK_W(KK, C, 7); break; \
    default: SFK_W(KK, C, 8); break; \
  }
  if (cnt) {
    SFK_W_NM(KK_EPAN, true);
  } else if (kk == KK_EPAN) {
    SFK_W_NM(KK_EPAN, false);
  } else {
    SFK_W_NM(KK_GAUSS, false);
  }
#undef SFK_W_NM
#undef SFK_W
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int wb = (int)std::max<int64_t>(1, std::min<int64_t>(max_tiles, 16384));
  if (cnt)
    hipLaunchKernelGGL(k_sweep_write<true>, dim3(wb), dim3(256), 0, s, hdr, rois, acc);
  else
    hipLaunchKernelGGL(k_sweep_write<false>, dim3(wb), dim3(256), 0, s, hdr, rois, acc);
  return hipGetLastError();
}

// every shape of the range query (wavefront tiles and bricks)
#define SFK_SHAPE_SWITCH(ts, MACRO)                                  \
  do {                                                               \
    if ((ts).tx == kBrick && (ts).ty == kBrick && (ts).tz == kBrick) { \
      MACRO(kBrick, kBrick, kBrick);                                 \
    } else if ((ts).tx == 4 && (ts).ty == 4 && (ts).tz == 4) {       \
      MACRO(4, 4, 4);                                                \
    } else if ((ts).tx == 4 && (ts).ty == 4 && (ts).tz == 2) {       \
      MACRO(4, 4, 2);                                                \
    } else if ((ts).tx == 4 && (ts).ty == 2 && (ts).tz == 2) {       \
      MACRO(4, 2, 2);                                                \
    } else if ((ts).tx == 2 && (ts).ty == 2 && (ts).tz == 2) {       \
      MACRO(2, 2, 2);                                                \
    } else if ((ts).tx == 1 && (ts).ty == 1 && (ts).tz == 1) {       \
      MACRO(1, 1, 1);                                                \
    } else {                                                         \
      return hipErrorInvalidValue;                                   \
    }                                                                \
  } while (0)

static int grid_for(int64_t waves) {
  const int64_t b = (waves + 3) / 4;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 65536));
}

int tile_grid_blocks(int64_t n_tiles) { return grid_for(n_tiles); }

hipError_t launch_tile_count(TreeView tv, const BatchHdr* hdr, const RoiDev* rois,
                             const double* coords, const int32_t* roi_leaves,
                             const int32_t* roi_nl, TileShape ts, int grid_blocks,
                             int32_t* tile_cnt, int32_t* tile_done, int32_t* tile_slots,
                             hipStream_t s) {
  const int nb = std::max(1, grid_blocks);
#define SFK_L(X, Y, Z)                                                                      \
  hipLaunchKernelGGL((k_tile_count<X, Y, Z>), dim3(nb), dim3(256), 0, s, tv, hdr, rois,  \
                     coords, roi_leaves, roi_nl, tile_cnt, tile_done, tile_slots)
  SFK_SHAPE_SWITCH(ts, SFK_L);
#undef SFK_L
  return hipGetLastError();
}

// The whole plan in one block, for batches of at most kPlanNT tiles.
__global__ __launch_bounds__(kPlanNT) void k_plan_one(const int32_t* __restrict__ tile_cnt,
                                                      BatchHdr* __restrict__ hdr,
                                                      int32_t* __restrict__ claims,
                                                      int chunk_leaves,
                                                      int64_t* __restrict__ leaf_off,
                                                      int64_t* __restrict__ partial_off,
                                                      int64_t* __restrict__ chunk_off,
                                                      int32_t* __restrict__ tile_fit) {
  __shared__ int64_t lds[kPlanNT / 64];
  const int64_t n_tiles = hdr->n_tiles;
  const int64_t leaf_cap = hdr->leaf_cap, partial_cap = hdr->partial_cap;
  const int64_t t = threadIdx.x;
  const bool v = t < n_tiles;
  const int64_t cnt = v ? tile_cnt[t] : 0;
  const int64_t nch = plan_chunks(cnt, chunk_leaves);
  const int64_t pneed = v ? plan_partials(nch, hdr->splat) : 0;
  int64_t tl, tp, tc;
  const int64_t lo = block_excl_scan<kPlanNT>(cnt, &tl, lds);
  const int64_t po = block_excl_scan<kPlanNT>(pneed, &tp, lds);
  const bool fit_p = pneed == 0 || po + pneed <= partial_cap;
  // bricks never walk per chunk: their items stay within the list capacity
  const int mode = (lo + cnt <= leaf_cap && fit_p)    ? kModeLists
                   : (fit_p && nch > 1 && !hdr->splat) ? kModeWalkChunk
                                                       : kModeWalkTile;
  const int64_t nit = v && cnt > 0 ? (mode == kModeWalkTile ? 1 : nch) : 0;
  const int64_t co = block_excl_scan<kPlanNT>(nit, &tc, lds);
  if (v) {
    leaf_off[t] = lo;
    partial_off[t] = po;
    chunk_off[t] = co;
    tile_fit[t] = mode;
  }
  // every thread has read the header above before thread 0 writes it
  __syncthreads();
  if (threadIdx.x < kClaimSlices) claims[threadIdx.x * kClaimStride] = 0;
  if (threadIdx.x == 0) {
    leaf_off[n_tiles] = tl;
    partial_off[n_tiles] = tp;
    chunk_off[n_tiles] = tc;
    hdr->total_leaves = tl;
    hdr->n_items = tc;
    hdr->total_partials = tp;
    hdr->overflow = (tl > leaf_cap || tp > partial_cap) ? 1 : 0;
  }
}

int plan_blocks(int64_t max_tiles) {
  return (int)std::max<int64_t>(1, (max_tiles + kPlanNT - 1) / kPlanNT);
}

hipError_t launch_plan(const int32_t* tile_cnt, BatchHdr* hdr, int32_t* claims, int chunk_leaves,
                       int64_t* leaf_off, int64_t* partial_off, int64_t* chunk_off,
                       int32_t* tile_fit, int64_t* plan_tmp, int64_t max_tiles, hipStream_t s) {
  const int nb = plan_blocks(max_tiles);
  if (nb == 1) {
    hipLaunchKernelGGL(k_plan_one, dim3(1), dim3(kPlanNT), 0, s, tile_cnt, hdr, claims,
                       chunk_leaves, leaf_off, partial_off, chunk_off, tile_fit);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_plan_sums, dim3(nb), dim3(kPlanNT), 0, s, tile_cnt, hdr, chunk_leaves,
                     plan_tmp);
  hipLaunchKernelGGL(k_plan_modes, dim3(nb), dim3(kPlanNT), 0, s, tile_cnt, hdr, chunk_leaves,
                     plan_tmp, leaf_off, partial_off, tile_fit);
  hipLaunchKernelGGL(k_plan_items, dim3(nb), dim3(kPlanNT), 0, s, tile_cnt, hdr, claims,
                     chunk_leaves, plan_tmp, leaf_off, partial_off, chunk_off, tile_fit);
  return hipGetLastError();
}

hipError_t launch_tile_fill(TreeView tv, const BatchHdr* hdr, const RoiDev* rois,
                            const double* coords, const int32_t* roi_leaves,
                            const int32_t* roi_nl, const int32_t* tile_slots, TileShape ts,
                            int grid_blocks, const int32_t* tile_cnt, const int32_t* tile_fit,
                            const int64_t* leaf_off, const int64_t* chunk_off, int32_t* leaves,
                            int32_t* item_tile, int32_t* claims, double* partials,
                            const int64_t* partial_off, hipStream_t s) {
  const int nb = std::max(1, grid_blocks);
#define SFK_L(X, Y, Z)                                                                     \
  hipLaunchKernelGGL((k_tile_fill<X, Y, Z>), dim3(nb), dim3(256), 0, s, tv, hdr, rois,  \
                     coords, roi_leaves, roi_nl, tile_slots, tile_cnt, tile_fit, leaf_off,  \
                     chunk_off, leaves, item_tile, claims, partials, partial_off)
  SFK_SHAPE_SWITCH(ts, SFK_L);
#undef SFK_L
  return hipGetLastError();
}

template <int X, int Y, int Z>
static hipError_t launch_eval_shape(int kk, int pp, bool cnt, int grid, int n_cu, int max_blocks,
                                    hipStream_t s,
                                    TreeView tv, const RoiDev* rois, const double* coords,
                                    int chunk_leaves, const int64_t* leaf_off,
                                    const int64_t* chunk_off, const int64_t* partial_off,
                                    const int32_t* tile_cnt, const int32_t* tile_fit,
                                    const int32_t* leaves, const int32_t* item_tile,
                                    double* partials, int32_t* tile_done, BatchHdr* hdr,
                                    int32_t* claims) {
#define SFK_E(KK, PP, C)                                                                       \
  do {                                                                                         \
    static int occ_ = 0;                                                                       \
    if (occ_ == 0) {                                                                           \
      int b_ = 0;                                                                              \
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b_, k_eval<X, Y, Z, KK, PP, C>, 256,   \
                                                       0) != hipSuccess || b_ < 1)             \
        b_ = 1;                                                                                \
      occ_ = b_;                                                                               \
    }                                                                                          \
    const int g_ = grid > 0 ? grid : std::max(1, std::min(n_cu * occ_, max_blocks));          \
    hipLaunchKernelGGL((k_eval<X, Y, Z, KK, PP, C>), dim3(g_), dim3(256), 0, s, tv, rois,      \
                       coords, chunk_leaves, leaf_off, chunk_off, partial_off, tile_cnt,       \
                       tile_fit, leaves, item_tile, partials, tile_done, hdr, claims);         \
  } while (0)
  if (cnt) {
    if (pp == PP_UNIFORM) SFK_E(KK_EPAN, PP_UNIFORM, true);
    else if (pp == PP_ISO) SFK_E(KK_EPAN, PP_ISO, true);
    else SFK_E(KK_EPAN, PP_ANISO, true);
  } else if (kk == KK_EPAN) {
    if (pp == PP_UNIFORM) SFK_E(KK_EPAN, PP_UNIFORM, false);
    else if (pp == PP_ISO) SFK_E(KK_EPAN, PP_ISO, false);
    else SFK_E(KK_EPAN, PP_ANISO, false);
  } else {
    if (pp == PP_UNIFORM) SFK_E(KK_GAUSS, PP_UNIFORM, false);
    else if (pp == PP_ISO) SFK_E(KK_GAUSS, PP_ISO, false);
    else SFK_E(KK_GAUSS, PP_ANISO, false);
  }
#undef SFK_E
  return hipGetLastError();
}

hipError_t launch_eval(TreeView tv, const BatchHdr* hdr_c, const RoiDev* rois,
                       const double* coords, TileShape ts, int kk, int pp, bool cnt,
                       int chunk_leaves, const int64_t* leaf_off, const int64_t* chunk_off,
                       const int64_t* partial_off, const int32_t* tile_cnt,
                       const int32_t* tile_fit, const int32_t* leaves, const int32_t* item_tile,
                       double* partials, int32_t* tile_done, BatchHdr* hdr, int32_t* claims,
                       int grid_blocks, int n_cu, int max_blocks, hipStream_t s) {
  (void)hdr_c;
  if (is_brick(ts)) {
    if (pp != PP_UNIFORM) return hipErrorInvalidValue;
#define SFK_S(KK, C)                                                                          \
  do {                                                                                        \
    static int occ_ = 0;                                                                      \
    if (occ_ == 0) {                                                                          \
      int b_ = 0;                                                                             \
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b_, k_splat<KK, C>, 256, 0) !=        \
              hipSuccess ||                                                                   \
          b_ < 1)                                                                             \
        b_ = 1;                                                                               \
      occ_ = b_;                                                                              \
    }                                                                                         \
    const int g_ = grid_blocks > 0 ? grid_blocks : std::max(1, std::min(n_cu * occ_, max_blocks)); \
    hipLaunchKernelGGL((k_splat<KK, C>), dim3(g_), dim3(256), 0, s, tv, rois, coords,         \
                       chunk_leaves, leaf_off, chunk_off, partial_off, tile_cnt, tile_fit,    \
                       leaves, item_tile, partials, tile_done, hdr, claims);                  \
  } while (0)
    if (cnt)
      SFK_S(KK_EPAN, true);
    else if (kk == KK_EPAN)
      SFK_S(KK_EPAN, false);
    else
      SFK_S(KK_GAUSS, false);
#undef SFK_S
    return hipGetLastError();
  }
#define SFK_L(X, Y, Z)                                                                        \
  return launch_eval_shape<X, Y, Z>(kk, pp, cnt, grid_blocks, n_cu, max_blocks, s, tv, rois, \
                                    coords,                                                   \
                                    chunk_leaves, leaf_off, chunk_off, partial_off, tile_cnt, \
                                    tile_fit, leaves, item_tile, partials, tile_done, hdr,    \
                                    claims)
  if ((ts).tx == 4 && (ts).ty == 4 && (ts).tz == 4) {
    SFK_L(4, 4, 4);
  } else if ((ts).tx == 4 && (ts).ty == 4 && (ts).tz == 2) {
    SFK_L(4, 4, 2);
  } else if ((ts).tx == 4 && (ts).ty == 2 && (ts).tz == 2) {
    SFK_L(4, 2, 2);
  } else if ((ts).tx == 2 && (ts).ty == 2 && (ts).tz == 2) {
    SFK_L(2, 2, 2);
  } else if ((ts).tx == 1 && (ts).ty == 1 && (ts).tz == 1) {
    SFK_L(1, 1, 1);
  }
#undef SFK_L
  return hipErrorInvalidValue;
}

hipError_t launch_debug_candidates2(TreeView tv, const int32_t* perm, const RoiDev* roi,
                                    const double* coords, TileShape ts, int64_t node_begin,
                                    int64_t node_end, int64_t* cnt, const int64_t* off,
                                    int32_t* idx_out, hipStream_t s) {
  const int64_t nn = node_end - node_begin;
  if (nn <= 0) return hipSuccess;
  const int nb = grid_for(nn);
#define SFK_L(X, Y, Z)                                                                     \
  hipLaunchKernelGGL((k_debug_candidates<X, Y, Z>), dim3(nb), dim3(256), 0, s, tv, perm, \
                     roi, coords, node_begin, node_end, cnt, off, idx_out)
  SFK_SHAPE_SWITCH(ts, SFK_L);
#undef SFK_L
  return hipGetLastError();
}

}  // namespace sfk
