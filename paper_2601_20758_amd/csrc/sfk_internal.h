// Internal device/host structures of libsfkde (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SFK_LEAF 64            // particles per leaf bucket = wavefront width
#define SFK_WAVE 64
#define SFK_FANOUT 64          // children per interior node of the box hierarchy
#define SFK_MAX_LEVELS 8       // 64^7 leaves is far beyond 2^31 particles
#define SFK_SENTINEL 1.0e30f   // coordinate of padding / zero-support particles

// Bounding box of a subtree (32 bytes). For a leaf, first = first particle
// slot; for an interior node, first = first child index on the level below.
struct alignas(16) NodeBox {
  float lo[3];
  int32_t first;
  float hi[3];
  int32_t count;  // real particles in the subtree
};

enum PPMode : int32_t {
  PP_UNIFORM = 0,  // bandwidth from the ROI
  PP_ISO = 1,      // per-particle isotropic inverse bandwidth in pts[].w
  PP_ANISO = 2     // per-particle (ih_x, ih_y, ih_z, w) in pparam[]
};

// Read-only view of a tree passed to kernels by value.
struct TreeView {
  const float4* pts;     // n_leaves*64 slots, curve order, padded with sentinels
  const float4* pparam;  // PP_ANISO only
  const NodeBox* nodes;  // all levels, level 0 = leaves
  const float4* node_ih; // per node: per-axis minimum inverse bandwidth (per-point modes)
  int32_t level_off[SFK_MAX_LEVELS];
  int32_t level_cnt[SFK_MAX_LEVELS];
  int32_t n_levels;      // levels including the leaf level (0 if empty)
  int32_t n_leaves;
  int64_t n;
  int32_t pp_mode;
  int32_t pad_;
};

enum KernelKind : int32_t { KK_EPAN = 0, KK_GAUSS = 1 };

// One ROI of a batch, as the evaluation kernels see it (device copy).
struct alignas(16) RoiDev {
  double lo[3], hi[3];
  int32_t res[3];
  int32_t ntile[3];      // tiles per axis
  int64_t tile_base;     // global index of the ROI's first tile
  float ih[3];           // uniform inverse bandwidth (PP_UNIFORM)
  float c2;              // support threshold on u2 (1 or 9)
  double scale;          // final multiplier C_K * nu (* w for a uniform bandwidth)
  int32_t kernel;        // KernelKind
  int32_t count_mode;    // 1: accumulate support counts instead of density
  int32_t coord_off;     // into the batch coordinate table: x, then y, then z
  float* out;
  int32_t pp_mode;       // PPMode of this evaluation
  int32_t pad_[3];
};

// Device-side header of one batch, staged by the host together with the ROI
// descriptors (so a captured graph can be replayed for any batch that fits
// its buffers); the plan kernel fills in the totals. No host sync.
struct alignas(16) BatchHdr {
  int64_t n_tiles;       // host: tiles of the batch
  int64_t leaf_cap;      // host: capacity of the leaf-list buffer
  int64_t partial_cap;   // host: capacity of the split-tile partial slots
  int64_t item_cap;      // host: capacity of the item buffers
  int32_t n_rois;        // host: descriptors that follow the header
  int32_t slot_cap;      // host: leaves the count pass keeps per tile (<= kTileSlotCap)
  int64_t total_leaves;  // plan: candidate leaves over all tiles
  int64_t n_items;       // plan: work items (tile chunks)
  int64_t total_partials;  // plan: partial-sum slots the split tiles need
  int32_t overflow;      // plan: 1 if some tile's lists did not fit (it walks the tree)
  int32_t debug_poison;  // host, tests only: bit 0 = the count pass stores out-of-range
                         // ids in the slots past the 64th of a tile, bit 1 = the fill
                         // pass stores them in the lists past the 64th entry
  int32_t splat;         // host: 1 = the tiles are bricks evaluated by scattering into
                         // integer node sums; a split brick then needs one partial
                         // slot (its node sums), not one per chunk
  int32_t pad_;
};

// Work-claim counters of the evaluation: kClaimSlices counters, one per
// 128-byte line (kClaimStride int32 apart) so claims on different slices do
// not contend; zeroed by the plan kernel of each batch.
constexpr int kClaimSlices = 64;
constexpr int kClaimStride = 32;
// After the counters, on a line of its own: the sticky error word of the
// workspace. A kernel that reads a leaf id outside the tree from a slot or a
// list sets it (and uses leaf 0 instead, so nothing is read out of bounds);
// the host reads it back after each batch, reports SFK_E_INTERNAL and clears
// it. No kernel clears it.
constexpr int kErrWord = kClaimSlices * kClaimStride;
constexpr size_t kClaimBytes = sizeof(int32_t) * (kClaimSlices + 1) * kClaimStride;
// Leaves held per ROI list (the leaves that can reach any of the ROI's
// nodes); a ROI with more walks the hierarchy per tile instead.
constexpr int kRoiListCap = 256;
// Largest number of leaves the count pass keeps per tile (in walk order);
// the fill pass copies them for tiles with at most that many instead of
// walking again. The capacity of a batch (BatchHdr::slot_cap) follows its
// tile shape: tiles of fewer nodes meet fewer leaves.
constexpr int kTileSlotCap = 256;

// Tile shapes (wavefront = tx*ty*tz nodes, powers of two). The brick shape
// kBrick^3 is not a wavefront's tile: a workgroup scatters particles into
// the brick's node sums (uniform bandwidths only).
struct TileShape { int tx, ty, tz; };
constexpr int kBrick = 16;
// Fixed point of the brick's integer node sums: a term v in [0, 1] counts
// floor(v * 2^31 + 1/2) units (so a sum of up to 2^32 terms fits in 64 bits).
constexpr double kSplatUnit = 2147483648.0;
// Particle sweep (dense uniform-bandwidth ROIs): work items are boxes of the
// hierarchy's first interior level (64 leaves), each scattered once into
// an LDS window of at most kSweepWin^3 nodes and flushed into 64-bit integer
// node sums kept per tile of kSweep^3 nodes (the shape's "tiles": they only
// lay out the sums and the final conversion). A particle's support spans at
// most kSweepMaxNM nodes per axis.
constexpr int kSweep = 8;
constexpr int kSweepWin = 16;
constexpr int kSweepMaxNM = 8;

// ---- host-side launch wrappers (defined in the .hip files) ----
namespace sfk {

// A brick of a node grid for the refinement test: nodes n0 .. n0 + cells of
// `grid` (res nodes per axis, x fastest).
struct BrickDesc {
  const float* grid;
  int32_t res[3];
  int32_t n0[3];
  int32_t cells[3];
  int32_t pad_;
};

// consumers.hip
hipError_t launch_brick_minmax(const BrickDesc* d_descs, int32_t n, float* d_min, float* d_max,
                               hipStream_t s);
hipError_t launch_view_gather(const float* cache, int64_t n_slots, int block, const int32_t* table,
                              const int64_t b0[3], const int32_t nb[3], const int64_t g0[3],
                              const int32_t res[3], float* out, hipStream_t s);
hipError_t launch_sample(const float* grid, const double lo[3], const double hi[3],
                         const int32_t res[3], const float* xyz, int64_t n, float* out,
                         hipStream_t s);
hipError_t launch_select_flags(const float* grid, const double lo[3], const double hi[3],
                               const int32_t res[3], double iso, const float* xyz, int64_t n,
                               int32_t* flags, hipStream_t s);
hipError_t launch_compact_index(const int32_t* flags, const int64_t* pos, int64_t n, int64_t* idx,
                                int64_t cap, hipStream_t s);
hipError_t launch_iso_flags(const float* grid, const int32_t res[3], double iso, int64_t n_cells,
                            int32_t* flags, uint8_t* case_all, hipStream_t s);
hipError_t launch_compact_cells(const int32_t* flags, const int64_t* pos, const uint8_t* case_all,
                                int64_t n, int64_t* cells, uint8_t* cases, int64_t cap,
                                hipStream_t s);
// Marching Cubes triangles: per-cell counts from the cases, then 9 floats per
// triangle at the cells' exclusive-scan offsets (the first `cap` triangles)
// the Marching Cubes case table the kernels use, read on the host:
// 3 * n edge ids of case cs, returns n
int mc_case_host(int cs, int8_t* edges);
hipError_t launch_iso_tri_count(const uint8_t* case_all, int64_t n_cells, int32_t* cnt,
                                hipStream_t s);
hipError_t launch_iso_emit(const float* grid, const double lo[3], const double hi[3],
                           const int32_t res[3], double iso, const uint8_t* case_all,
                           const int64_t* pos, int64_t n_cells, float* tris, int64_t cap,
                           hipStream_t s);

// scan.hip
hipError_t scan_exclusive_i32_i64(const int32_t* in, int64_t* out, int64_t n,
                                  int64_t* total, void* tmp, size_t tmp_bytes, hipStream_t s);
size_t scan_tmp_bytes(int64_t n);
hipError_t scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, void* tmp,
                              size_t tmp_bytes, hipStream_t s);

// build.hip
hipError_t launch_bbox(const float* xyz, int64_t n, float* partial, int nblk, float* result,
                       hipStream_t s);
// keys: uint32_t[n] when 3*bits <= 32, else uint64_t[n]
hipError_t launch_curve_keys(const float* xyz, int64_t n, const float* bbox, int bits,
                             int hilbert, void* keys, uint32_t* vals, hipStream_t s);
// the same key function on the host: cells = n (x, y, z) triples < 2^bits
void curve_keys_host(const uint32_t* cells, int64_t n, int bits, int hilbert, uint64_t* keys);
size_t radix_sort_tmp_bytes(int64_t n);
hipError_t radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt,
                            uint32_t* vals_alt, int64_t n, int key_bits, void* tmp,
                            size_t tmp_bytes, hipStream_t s, int* result_in_alt);
// the same with 32-bit keys (key_bits <= 32)
hipError_t radix_sort_pairs_u32(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                                uint32_t* vals_alt, int64_t n, int key_bits, void* tmp,
                                size_t tmp_bytes, hipStream_t s, int* result_in_alt);
// Sorted particles into n_leaves * SFK_LEAF slots (n <= that), the leaf
// boxes into leaf_box[0, n_leaves), and with sub_box non-null the k-NN
// sub-block boxes (knn_sub_box_bytes(n_leaves))
hipError_t launch_gather(const float* xyz, const uint32_t* perm, int64_t n, int32_t n_leaves,
                         float4* pts, int32_t* perm_out, NodeBox* leaf_box, float* sub_box,
                         hipStream_t s);
// only_if: nullptr, or a device flag; the launch does nothing while it is 0
hipError_t launch_leaf_boxes(const float4* pts, int64_t n, int32_t n_leaves, NodeBox* out,
                             const int32_t* only_if, hipStream_t s);
hipError_t launch_level_boxes(const NodeBox* child, int32_t n_child, NodeBox* parent,
                              int32_t n_parent, const int32_t* only_if, hipStream_t s);
// leaf_done: the leaf level is already written (launch_iso_params)
hipError_t launch_node_ih(const float4* pts, const float4* pparam, int32_t pp_mode,
                          int64_t n, const NodeBox* nodes, const int32_t* level_off,
                          const int32_t* level_cnt, int n_levels, float4* node_ih,
                          int leaf_done, hipStream_t s);
// sub_box: the sub-block boxes launch_gather wrote for this leaf layout;
// skip_if: nullptr, or a device float; while it is > 0 the kernel returns at
// once and h2_sorted is left as it was
hipError_t launch_knn(TreeView tv, float* sub_box, int k, float* h2_sorted,
                      const float* skip_if, hipStream_t s);
size_t knn_sub_box_bytes(int32_t n_leaves);
// moved (device int32): set to 1 when a zero bandwidth moved a particle to
// the sentinel position, else 0; leaf_ih: the leaf level of the node
// bandwidths (n_leaves float4), written from the updated particles
hipError_t launch_iso_params(float4* pts, const float* h2_sorted, const float* h_user_orig,
                             const int32_t* perm, int64_t n, int32_t n_leaves, float4* leaf_ih,
                             int32_t* moved, hipStream_t s);

hipError_t launch_count_nonpositive(const float* h, int64_t n, int32_t* bad, hipStream_t s);
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s);

// eval.hip (every kernel reads the batch sizes from the device header)
// the coordinate tables and the ROI leaf lists (one block per ROI);
// roi_leaves: kRoiListCap int32 per ROI; roi_nl: one int32 per ROI (list
// length, or -1 when the ROI reaches more leaves than a list holds)
hipError_t launch_roi_coords(TreeView tv, const BatchHdr* hdr, const RoiDev* rois, int grid_rois,
                             double* coords, int32_t* roi_leaves, int32_t* roi_nl,
                             hipStream_t s);
// tile_slots: hdr->slot_cap int32 per tile
hipError_t launch_tile_count(TreeView tv, const BatchHdr* hdr, const RoiDev* rois,
                             const double* coords, const int32_t* roi_leaves,
                             const int32_t* roi_nl, TileShape ts, int grid_blocks,
                             int32_t* tile_cnt, int32_t* tile_done, int32_t* tile_slots,
                             hipStream_t s);
// plan_tmp: 3 int64 per block of plan_blocks(max_tiles); max_tiles bounds
// the header's tile count (the grid of a captured graph uses the capacity)
int plan_blocks(int64_t max_tiles);
hipError_t launch_plan(const int32_t* tile_cnt, BatchHdr* hdr, int32_t* claims, int chunk_leaves,
                       int64_t* leaf_off, int64_t* partial_off, int64_t* chunk_off,
                       int32_t* tile_fit, int64_t* plan_tmp, int64_t max_tiles, hipStream_t s);
// claims: the work-claim counters, whose error word the slot copy may set
// partials/partial_off: bricks (hdr->splat) zero the node sums of their
// partial slot here when they are split into several work items
hipError_t launch_tile_fill(TreeView tv, const BatchHdr* hdr, const RoiDev* rois,
                            const double* coords, const int32_t* roi_leaves,
                            const int32_t* roi_nl, const int32_t* tile_slots, TileShape ts,
                            int grid_blocks, const int32_t* tile_cnt, const int32_t* tile_fit,
                            const int64_t* leaf_off, const int64_t* chunk_off, int32_t* leaves,
                            int32_t* item_tile, int32_t* claims, double* partials,
                            const int64_t* partial_off, hipStream_t s);
hipError_t launch_eval(TreeView tv, const BatchHdr* hdr_c, const RoiDev* rois,
                       const double* coords, TileShape ts, int kk, int pp, bool cnt,
                       int chunk_leaves, const int64_t* leaf_off, const int64_t* chunk_off,
                       const int64_t* partial_off, const int32_t* tile_cnt,
                       const int32_t* tile_fit, const int32_t* leaves, const int32_t* item_tile,
                       double* partials, int32_t* tile_done, BatchHdr* hdr, int32_t* claims,
                       int grid_blocks, int n_cu, int max_blocks, hipStream_t s);
hipError_t launch_debug_candidates2(TreeView tv, const int32_t* perm, const RoiDev* roi,
                                    const double* coords, TileShape ts, int64_t node_begin,
                                    int64_t node_end, int64_t* cnt, const int64_t* off,
                                    int32_t* idx_out, hipStream_t s);
bool tile_shape_supported(TileShape ts);
bool is_brick(TileShape ts);
bool is_sweep(TileShape ts);
int tile_grid_blocks(int64_t n_tiles);
// Particle sweep of a batch (uniform bandwidths), in two launches.
// launch_sweep_list: zero the integer node sums of hdr->n_tiles tiles (acc,
// kSweep^3 64-bit sums per tile) and the claim counters, and list the
// (ROI, box) work items into items[0, hdr->item_cap) (count in
// hdr->n_items); max_rois / max_tiles bound the header's counts (the grids
// of a captured graph use the capacities).
// launch_sweep_eval: scatter the items and write every node of every ROI.
// nm: nodes per axis a support can span (1..kSweepMaxNM). A listing past
// the capacity or a support wider than nm sets the error word.
hipError_t launch_sweep_list(TreeView tv, BatchHdr* hdr, const RoiDev* rois,
                             const double* coords, int64_t* items, unsigned long long* acc,
                             int32_t* claims, int max_rois, int64_t max_tiles, hipStream_t s);
hipError_t launch_sweep_eval(TreeView tv, const BatchHdr* hdr, const RoiDev* rois,
                             const double* coords, int kk, bool cnt, int nm,
                             const int64_t* items, unsigned long long* acc, int32_t* claims,
                             int grid_blocks, int n_cu, int64_t max_tiles, hipStream_t s);

// mbe.hip
// leaves whose box meets the closed box [lo, hi]: flags[n_leaves]; their
// indices, ascending, from the flags' exclusive scan
hipError_t launch_leaf_overlap(const NodeBox* leaf_box, int32_t n_leaves, const double* lo,
                               const double* hi, int32_t* flags, hipStream_t s);
hipError_t launch_compact_leaves(const int32_t* flags, const int64_t* pos, int32_t n_leaves,
                                 int32_t* cand, hipStream_t s);
// particles in the closed box among n examined slots: every slot in order
// (cand == nullptr, n = slots) or the 64 slots of each candidate leaf in
// order (n = 64 * candidates); flags and positions index examined slots
hipError_t launch_inbox_flags(const float4* pts, const int32_t* cand, int64_t n, const double* lo,
                              const double* hi, int32_t* flags, hipStream_t s);
hipError_t launch_compact(const float4* pts, const int32_t* perm, const int32_t* cand,
                          const int32_t* flags, const int64_t* pos, int64_t n,
                          int64_t n_slots_out, float4* out_pts, int32_t* out_perm,
                          float* out_axes, int64_t n_b, hipStream_t s);
hipError_t launch_axis_keys(const float* axes, int64_t n_b, uint64_t* keys, uint32_t* vals,
                            hipStream_t s);
hipError_t launch_mbe_ell(const uint64_t* sorted_keys_xyz, int64_t n_b, const double* lo,
                          const double* hi, const int32_t* res, float* ell_out,
                          int32_t* flags_out, hipStream_t s);
hipError_t launch_trilinear_mean(const float4* pts, int64_t n_b, const float* grid,
                                 const double* lo, const double* hi, const int32_t* res,
                                 double* pden, double* block_sums, double* ave, hipStream_t s);
hipError_t launch_asl2(const double* pden, int64_t n_b, const double* ave, const float* ell0,
                       const double* lo, const double* hi, const int32_t* res, float4* pparam,
                       float* ell_out, hipStream_t s);

}  // namespace sfk
