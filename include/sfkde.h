/*
 * sfkde.h -- C ABI of the MI355X (gfx950) ROI kernel density estimation
 * library: on-the-fly density grids over regions of interest of a large
 * particle cloud, after ScaleFree (arXiv 2601.20758).
 *
 * Method references (paper sections, equations, algorithms):
 *   Section 3.1, Eqs. 1-8   the estimator: a uniform node grid over a box B,
 *                           the Epanechnikov kernel (Eq. 4), the pilot
 *                           density (Eqs. 2-3), the initial smoothing length
 *                           (Eq. 1), the mean pilot density (Eq. 5), the
 *                           adaptive smoothing length (Eq. 6) and the final
 *                           density (Eqs. 7-8).
 *   Section 3.2, Alg. 1-4   the GPU pipeline the paper dispatches (pilot,
 *                           adaptive length, final) and its inputs: a spatial
 *                           index over the particles, the positions, the
 *                           grid, the smoothing lengths and the node spacing.
 *
 * Conventions
 *   - Every pointer named d_* is device memory on the context's device; h_*
 *     is host memory. The caller owns both; the library never frees them.
 *   - Positions are float32 AoS, n x 3 (x, y, z).
 *   - A grid has res[0]*res[1]*res[2] float32 values, x fastest:
 *     idx = x + y*res[0] + z*res[0]*res[1] (Algorithms 2 and 4 index the
 *     density buffer this way).
 *   - Grid node i on axis k sits at lo + (i*(hi-lo))/(res-1), evaluated in
 *     double (vertex-centred nodes on the closed box; node spacing
 *     s_k = (hi_k - lo_k)/(res_k - 1)).
 *   - A particle j is in the support of node n when, in double on the
 *     float32 particle and inverse-bandwidth values, u2 < c2 with
 *     u_k = (x_nk - p_jk) * ih_k, u2 = (u_x*u_x + u_y*u_y) + u_z*u_z, every
 *     operation rounded (no fused multiply-add), ih_k the float32 inverse
 *     bandwidth, c2 = 1 (Epanechnikov, Eq. 4 is zero at |x| >= 1) or 9
 *     (Gaussian truncated at 3 sigma).
 *   - Functions return sfk_status and never throw or abort. Arguments are
 *     validated before any device work; on failure nothing is launched and
 *     sfk_last_error() describes the cause.
 *   - One host thread per context. Trees are immutable after build and may
 *     be evaluated by several ROIs at once.
 */
#ifndef SFKDE_H
#define SFKDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SFK_OK = 0,
  SFK_E_INVAL = 1,        /* invalid argument (checked before any launch) */
  SFK_E_NOMEM = 2,        /* allocator returned NULL; the context stays usable */
  SFK_E_BUDGET = 3,       /* request exceeds the context's device-memory budget */
  SFK_E_DEVICE = 4,       /* a HIP runtime call failed */
  SFK_E_NOT_READY = 5,    /* ticket still running (sfk_poll / sfk_wait timeout) */
  SFK_E_CANCELLED = 6,    /* ticket was cancelled before it ran */
  SFK_E_UNSUPPORTED = 7,  /* valid but not supported combination */
  SFK_E_INTERNAL = 8
} sfk_status;

typedef enum {
  SFK_KERNEL_EPANECHNIKOV = 0, /* Eq. 4, C = 15/(8 pi) (Eq. 2, Eq. 7) */
  SFK_KERNEL_GAUSS_TRUNC3 = 1  /* exp(-u2/2) on u2 < 9, renormalised to unit mass */
} sfk_kernel;

typedef enum {
  SFK_BW_FIXED = 0,      /* h per axis as given */
  SFK_BW_ROI_SCALED = 1, /* h_k = h0 * (hi_k - lo_k), h0 = h[0] */
  SFK_BW_PER_POINT = 2,  /* per-particle isotropic h from the tree (k-NN or given) */
  SFK_BW_MBE = 3         /* Section 3.1: Eq. 1 -> pilot -> Eq. 6 -> final (Epanechnikov) */
} sfk_bw;

typedef enum {
  SFK_NORM_PAPER = 0, /* times 1/N: the grid integrates to 1 (Eqs. 2 and 7) */
  SFK_NORM_COUNT = 1  /* no 1/N: the grid integrates to N */
} sfk_norm;

typedef enum {
  SFK_SET_CLOUD = 0,  /* every particle of the tree contributes; N = tree size */
  SFK_SET_IN_ROI = 1  /* only particles in the closed box B; N = N_B (Eq. 1) */
} sfk_set;

typedef enum {
  SFK_CURVE_HILBERT = 0, /* Hilbert order (default): consecutive cells are face
                            neighbours, so leaf and group boxes are compact */
  SFK_CURVE_MORTON = 1   /* Morton (Z) order: the coordinate bits interleaved */
} sfk_curve;

typedef struct sfk_ctx_s* sfk_ctx;
typedef struct sfk_tree_s* sfk_tree;
typedef int64_t sfk_ticket;

/* Device-memory allocator. alloc returns device memory of at least `bytes`
 * (256-byte aligned) or NULL; free releases it. With a NULL allocator the
 * library uses hipMalloc / hipFree. */
typedef struct {
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, size_t bytes, void* user);
  void* user;
} sfk_allocator;

typedef struct {
  int32_t leaf_size;   /* particles per leaf bucket; 0 or 64 (the wavefront width) */
  int32_t knn_k;       /* 0: no per-point bandwidth; 1..64: h_j^2 = k-th smallest
                          squared distance to another particle (self excluded) */
  int32_t key_bits;    /* bits per axis of the sort key, 1..21, 0 = automatic
                          (10..21, about 4 cells per axis per n^(1/3)) */
  int32_t curve;       /* sfk_curve: the order of particles in the leaves */
} sfk_tree_opts;

/* One region-of-interest request (Section 3.1: a box B and its node grid). */
typedef struct {
  double lo[3], hi[3]; /* closed box B, hi > lo */
  int32_t res[3];      /* nodes per axis, each >= 2 */
  int32_t kernel;      /* sfk_kernel */
  int32_t bw;          /* sfk_bw */
  int32_t norm;        /* sfk_norm */
  int32_t set;         /* sfk_set (SFK_BW_MBE requires SFK_SET_IN_ROI) */
  float h[3];          /* FIXED: h per axis; ROI_SCALED: h0 in h[0]; else unused */
  float* d_out;        /* device, res[0]*res[1]*res[2] floats, written in full */
  uint64_t tag;        /* caller's label, unused by the library */
} sfk_roi;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`. hbm_budget_bytes bounds the
 * workspace the context may hold for in-flight batches (0 = no bound).
 * alloc may be NULL. */
sfk_status sfk_ctx_create(int device, const sfk_allocator* alloc,
                          size_t hbm_budget_bytes, sfk_ctx* out);
sfk_status sfk_ctx_destroy(sfk_ctx ctx);
const char* sfk_status_string(sfk_status s);
/* Last error message of the context (or of the calling thread if ctx is NULL). */
const char* sfk_last_error(sfk_ctx ctx);
/* Library version string. */
const char* sfk_version(void);

/* ------------------------------------------------------------------- tree */

/* Build the spatial index (the paper builds a k-d tree on the CPU and
 * uploads it, Section 3.2; here the tree is built on the device): bounding
 * box, space-filling curve keys (opts->curve), radix sort, leaf buckets of
 * 64 particles laid out as float4 in curve order, an implicit 64-ary
 * hierarchy of boxes over consecutive leaves. Results do not depend on the
 * curve beyond float32 summation order. With
 * opts->knn_k > 0 it also computes each particle's squared k-th nearest
 * neighbour distance (per-point bandwidth). d_h, if non-NULL, gives a
 * per-particle bandwidth instead (n floats, device, original order, > 0).
 * d_xyz is read during the call only (stream-ordered on hip_stream; the call
 * synchronises the stream before it returns). n = 0 gives an empty tree.
 * Errors: SFK_E_INVAL on n < 0, n >= 2^31 - 64, NULL pointers, a
 * non-finite coordinate, knn_k > 64 or knn_k >= n, a non-positive d_h,
 * key_bits outside 0..21, an unknown curve. */
sfk_status sfk_build_tree(sfk_ctx ctx, const float* d_xyz, int64_t n,
                          const float* d_h, const sfk_tree_opts* opts,
                          void* hip_stream, sfk_tree* out);
/* n particles, bbox = {xmin, ymin, zmin, xmax, ymax, zmax}, device bytes held. */
sfk_status sfk_tree_info(sfk_tree tree, int64_t* n, double bbox[6], size_t* device_bytes);
sfk_status sfk_tree_destroy(sfk_tree tree);

/* ------------------------------------------------------------- evaluation */

/* Evaluate one ROI into roi->d_out, stream-ordered on hip_stream (returns
 * once the work is enqueued; the grid is ready when the stream reaches it).
 * This is sfk_submit of one ROI on the caller's stream: the same kernels. */
sfk_status sfk_eval_roi(sfk_ctx ctx, sfk_tree tree, const sfk_roi* roi, void* hip_stream);

/* Size of the static device array that holds the workspace of
 * sfk_eval_roi_noalloc: one array per device the library runs on, held until
 * the process ends. */
#define SFK_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * sfk_eval_roi without any allocation: the same kernels and the same grid,
 * bitwise, stream-ordered on hip_stream (asynchronous), with the whole
 * workspace (descriptors, node coordinates, per-tile counts, offsets and leaf
 * slots, work items, partial sums, leaf lists) carved from the device's
 * static array of SFK_NOALLOC_SCRATCH_BYTES. The caller still owns roi->d_out.
 * Nothing starts at zero that must: each call's kernels clear what they use.
 * Limits: CLOUD-set, non-MBE ROIs (SFK_E_UNSUPPORTED otherwise); a ROI whose
 * per-tile arrays do not fit the array (about 1.5M tiles, e.g. 460^3 nodes
 * with 4x4x4 tiles) returns SFK_E_BUDGET before any launch. Smaller list
 * capacities than sfk_eval_roi's only make tiles walk the tree inside the
 * evaluation (same leaves, same order, same sums). A ROI that takes the
 * particle sweep (tile shape 7) needs 8 bytes per node of its 8^3-node tiles
 * and 8 bytes per 4096 particles of the tree; when that does not fit (about
 * 7.5M nodes) it takes the tile shape it would take without the sweep, and
 * its grid then equals sfk_eval_roi's within rounding, not bit for bit.
 * Concurrency: every call on a device shares that device's array. Calls of one
 * context are ordered (a call on another stream waits for the previous one);
 * calls from different contexts on one device that overlap in time race and
 * corrupt each other's results. Other errors as sfk_eval_roi. */
sfk_status sfk_eval_roi_noalloc(sfk_ctx ctx, sfk_tree tree, const sfk_roi* roi,
                                void* hip_stream);

/* Evaluate a batch of ROIs with uneven grids on one of the context's streams:
 * one persistent, work-stealing launch per group of ROIs that share the
 * kernel, bandwidth mode, tile shape and (for the particle sweep) node span,
 * the groups one after another. The descriptors are copied; the
 * d_out buffers must stay valid until the ticket completes. Returns with a
 * ticket without waiting for the batch to run, except when a free slot's
 * buffers must grow for the batch: replacing a workspace or staging buffer
 * first waits for that slot's previous batch, and the device allocation and
 * release themselves may synchronise the device. Batches that fit the slots'
 * buffers (every batch after a warm-up of the largest shape) never block.
 * SFK_E_BUDGET if the batch's workspace exceeds the budget.
 * A batch of one group replays the slot's captured
 * hipGraph (descriptor copy -> node coordinates -> tile range query -> work
 * plan -> leaf lists -> evaluation -> header readback), recaptured only when
 * the batch outgrows the graph's buffers. */
sfk_status sfk_submit(sfk_ctx ctx, sfk_tree tree, const sfk_roi* rois, int32_t n_rois,
                      sfk_ticket* out);
/* *done = 1 once the ticket's grids are written, never blocks. */
sfk_status sfk_poll(sfk_ctx ctx, sfk_ticket t, int32_t* done);
/* Block until done or timeout_us elapses (< 0: no timeout); SFK_E_NOT_READY on timeout. */
sfk_status sfk_wait(sfk_ctx ctx, sfk_ticket t, int64_t timeout_us);
/* Cancel a ticket that has not started on the device; SFK_E_NOT_READY if it is running. */
sfk_status sfk_cancel(sfk_ctx ctx, sfk_ticket t);

/* Tile shape used for tile-granular range queries and evaluation: one
 * wavefront owns tx*ty*tz grid nodes. 0 = chosen by the autotuner table. */
typedef struct {
  int32_t tile_shape;    /* 0 auto, 1 = 4x4x4, 2 = 4x4x2, 3 = 4x2x2, 4 = 2x2x2, 5 = 1x1x1
                            (a wavefront per tile, gathering), 6 = bricks of 16^3 nodes
                            (a workgroup per brick scattering particles into exact
                            integer node sums; uniform bandwidths only, others take 1),
                            7 = particle sweep (a workgroup per box of 4096 particles
                            scattering them once into the same integer node sums, so
                            its grids equal the bricks' bit for bit; uniform bandwidths
                            whose support spans at most 8 nodes per axis, others take
                            the default of their key without the sweep) */
  int32_t chunk_leaves;  /* leaves per work item (heavy tiles are split), 0 = 256 */
  int32_t persistent_waves_per_cu; /* 0 = automatic */
  int32_t list_capacity; /* leaf-list entries per batch, 0 = automatic; tiles whose
                            lists do not fit walk the tree inside the evaluation
                            kernel instead (same results, bitwise): one work item
                            per chunk while partial slots remain, else one per tile */
  int32_t disable_graphs; /* 1: batches on context streams use direct launches
                             instead of each slot's captured hipGraph */
  int32_t partial_capacity; /* partial-sum slots (chunks of split tiles) per batch,
                               0 = automatic (list_capacity / chunk_leaves when
                               list_capacity is set) */
} sfk_eval_opts;
sfk_status sfk_set_eval_opts(sfk_ctx ctx, const sfk_eval_opts* opts);
/* Time every tile shape on the sample ROIs and record the fastest per
 * (kernel, bandwidth mode, support-to-spacing bucket) for later batches. */
sfk_status sfk_autotune(sfk_ctx ctx, sfk_tree tree, const sfk_roi* sample, int32_t n);
/* The autotuner's table: up to cap (key, tile shape) pairs, *n_out = entries.
 * key = ((kernel * 4 + bandwidth mode) * 8 + support-in-spacings bucket) * 8
 * + particles-per-node bucket (uniform bandwidths: log2 of the particles
 * estimated in the box widened by the support, per node, plus 4, clamped to
 * 0..7; 0 for per-point bandwidths). */
sfk_status sfk_autotune_table(sfk_ctx ctx, int32_t* keys, int32_t* shapes, int32_t cap,
                              int32_t* n_out);
/* Tile shapes sfk_eval_opts.tile_shape can name (1..SFK_NUM_TILE_SHAPES). */
#define SFK_NUM_TILE_SHAPES 7
/* The times the last sfk_autotune measured: per key,
 * ms[i * SFK_NUM_TILE_SHAPES + s - 1] = the summed best-of-3 time of tile
 * shape s over that key's samples (1e30 for a shape the key cannot take).
 * *n_out = keys. */
sfk_status sfk_autotune_costs(sfk_ctx ctx, int32_t* keys, double* ms, int32_t cap,
                              int32_t* n_out);
/* Persist the table to a text file, with the device architecture (e.g.
 * gfx950) it was measured on; loading a table merges its entries, and a
 * table of another architecture is refused (SFK_E_UNSUPPORTED). SFK_E_INVAL
 * for unreadable or malformed files. */
sfk_status sfk_autotune_save(sfk_ctx ctx, const char* path);
sfk_status sfk_autotune_load(sfk_ctx ctx, const char* path);

/* -------------------------------------------------------------- profiling */

/* Device time of each pipeline phase, measured with HIP events recorded on
 * the stream each kernel is launched on (only while profiling is enabled). */
typedef struct {
  double tile_count_ms;  /* tile range query, count pass */
  double plan_ms;        /* work plan (prefix sums) */
  double tile_fill_ms;   /* tile range query, fill pass */
  double eval_ms;        /* evaluation kernel (the hot loop) */
  double build_ms;       /* tree build: bbox, keys, sort, leaves, boxes */
  double knn_ms;         /* k-NN bandwidth kernel */
  int64_t eval_launches;
  int64_t builds;
  int64_t last_total_leaves; /* candidate leaves of the last evaluated batch */
  int64_t last_items;        /* work items of the last evaluated batch */
} sfk_profile;

sfk_status sfk_profile_enable(sfk_ctx ctx, int32_t on);
/* Wait for the recorded events, add their durations into *out (totals since
 * the last reset) and optionally reset. */
sfk_status sfk_profile_read(sfk_ctx ctx, sfk_profile* out, int32_t reset);

/* ---------------------------------------------------------------- serving */

/* A request of the serving loop: it becomes visible at arrival_s seconds
 * after the loop starts. */
typedef struct {
  double arrival_s;
  sfk_roi roi;
} sfk_request;

typedef struct {
  int32_t mode;          /* 0 continuous batching, 1 one ROI per launch in FIFO order */
  int32_t n_slots;       /* batches in flight at once (each on its own stream), >= 1 */
  int32_t max_batch;     /* ROIs per batch, >= 1 */
  int32_t interleave;    /* 0: persistent evaluation grids, as sfk_submit uses; 1: grids of
                            one wavefront per tile, whose workgroups retire as they finish
                            so the kernels of requests on other streams interleave (tiles
                            and bricks; the particle sweep keeps its persistent grid) */
  double budget_bytes;   /* workspace + grid bytes admitted at once (0 = context budget) */
  double max_batch_work; /* continuous batching: a batch closes before the request that
                            would take its estimated useful pairs past this (a request
                            above it runs in a batch of its own, so light requests are not
                            held until a heavy batch-mate completes; they may still wait
                            for the CUs its kernel holds); 0 = 2e8, < 0 = no limit. The
                            estimate is the particles the tree's coarse boxes put in the
                            request's box (widened by the support) times the nodes one
                            support covers */
} sfk_serve_opts;

typedef struct {
  double arrival_s;   /* as requested */
  double admit_s;     /* when the request joined a launched batch */
  double done_s;      /* device completion observed by the host */
  double latency_ms;  /* done_s - arrival_s */
  int32_t batch;      /* batch index it ran in */
  int32_t status;     /* sfk_status of the request */
} sfk_request_result;

typedef struct {
  double wall_s;
  double p50_ms, p99_ms, max_ms;
  double evals_per_s;     /* useful (node, particle) pairs per second, if counted */
  int64_t n_batches;
  double mean_batch;      /* mean ROIs per batch */
  double mean_in_flight;  /* time-averaged batches in flight */
  int64_t budget_waits;   /* admissions deferred for memory */
} sfk_serve_summary;

/* Run the request loop over reqs (sorted by arrival) until every request is
 * done. Requests that arrive while others run are admitted as slots and
 * budget free up and run overlapped with them. */
sfk_status sfk_serve(sfk_ctx ctx, sfk_tree tree, const sfk_request* reqs, int64_t n,
                     const sfk_serve_opts* opts, sfk_request_result* h_results,
                     sfk_serve_summary* h_summary);

/* ------------------------------------------------- consumers of a grid */
/* These take a node grid in the layout sfk_eval_roi writes (res[0] * res[1]
 * * res[2] floats, x fastest) and the ROI whose nodes it holds; only
 * roi->lo, roi->hi and roi->res are read. Points are n x 3 float32 (AoS) on
 * the device. Interpolation is in double with a fixed operation order
 * (per axis f = ((p - lo)(res - 1)) / (hi - lo), cell floor(f) clamped to
 * [0, res - 2], t = f - cell clamped to [0, 1]; corner terms
 * ((wx wy) wz) value summed z-major, then y, then x), so threshold decisions
 * are reproducible. SFK_E_INVAL for a NULL pointer (unless n = 0), n < 0 or
 * invalid geometry (res < 2, lo >= hi, non-finite). */

/* Density at each point: trilinear interpolation of the surrounding grid
 * nodes (Section 3.1, after Eq. 8), rounded once to float; 0 for a point
 * outside the closed box. Stream-ordered, asynchronous. */
sfk_status sfk_sample_density(sfk_ctx ctx, const sfk_roi* roi, const float* d_grid,
                              const float* d_xyz, int64_t n, float* d_out, void* hip_stream);

/* Selection (Section 4.1: a density threshold, the region bounded by
 * the grid's iso-surface at that threshold, the points inside it): the
 * ascending indices of the points inside the closed box whose interpolated
 * density is >= iso. Writes the first min(count, cap) indices to d_idx
 * (int64, device) and the full count to *h_count; blocks on the stream. */
sfk_status sfk_select_points(sfk_ctx ctx, const sfk_roi* roi, const float* d_grid, double iso,
                             const float* d_xyz, int64_t n, int64_t* d_idx, int64_t cap,
                             int64_t* h_count, void* hip_stream);

/* Marching Cubes classification of the grid's (res - 1)^3 cells against iso
 * (Section 4.1): the case of a cell has bit dx + 2 dy + 4 dz set when
 * that corner's value is >= iso; a cell is active unless its case is 0 or
 * 255. Writes the first min(count, cap) active cells in ascending linear
 * cell index (x fastest over res - 1 cells per axis) to d_cells (int64) and
 * their cases to d_cases (uint8), the full count to *h_count; blocks. */
sfk_status sfk_iso_cells(sfk_ctx ctx, const sfk_roi* roi, const float* d_grid, double iso,
                         int64_t* d_cells, uint8_t* d_cases, int64_t cap, int64_t* h_count,
                         void* hip_stream);

/* The Marching Cubes iso-surface of the grid at iso (Section 4.1: the
 * selection volume is the region this surface bounds; Lorensen and Cline
 * 1987), as a triangle soup: 9 floats per triangle (three vertices x, y, z),
 * cell by cell in ascending linear cell index, each cell's triangles in its
 * case's order. The per-case triangles follow one rule computed from the
 * cube's faces (case bits as sfk_iso_cells; on a face with four crossed
 * edges the inside corners are cut off, so neighbouring cells agree and the
 * surface is closed where it does not meet the grid's boundary); normals
 * (v1 - v0) x (v2 - v0) point from values >= iso to values below. A vertex
 * on the edge from corner p (lower along the edge) to corner q sits at
 * x_p + t (x_q - x_p), t = (iso - f_p) / (f_q - f_p), in double, rounded once
 * to float. Writes the first min(count, cap) triangles to d_tris (device,
 * 9 * cap floats) and the count to *h_count; blocks on the stream. */
sfk_status sfk_iso_surface(sfk_ctx ctx, const sfk_roi* roi, const float* d_grid, double iso,
                           float* d_tris, int64_t cap, int64_t* h_count, void* hip_stream);

/* ------------------------------------------------- view cache (reuse) */
/* Recomputation policy of an interactive view (Section 6.3, limitations and
 * future work: recompute only when the scale changes by more than a
 * threshold, and evaluate the viewport plus a margin so that panning inside
 * it needs no new evaluation; Section 6.2: recompute once the user has moved
 * to a new scale).
 *
 * A view evaluates density on lattices of nodes o + g*s per axis (o = the
 * tree's bounding-box minimum, g an integer, s the spacing of the lattice),
 * cut into blocks of block^3 nodes. Block (bx, by, bz) of a lattice is the
 * ROI with lo_k = o_k + (b_k*block)*s, hi_k = o_k + (b_k*block + block - 1)*s
 * (double), res = block, CLOUD set, evaluated with the kernels of
 * sfk_eval_roi and one tile shape per lattice, so a cached block is bitwise
 * equal to a fresh sfk_eval_roi of that ROI. Blocks live in a device cache
 * of max_blocks blocks, evicted least recently used. A frame (a view box):
 *   1. wanted spacing s_w = (longest side of the box) / (res - 1); the cached
 *      lattice with the spacing closest to s_w in ratio is used if that ratio
 *      is within scale_threshold, else a lattice with s = s_w is created;
 *   2. every block holding a node within margin * (longest side) of the box
 *      is made present (only missing blocks are evaluated, in one batch);
 *   3. the lattice nodes g_lo..g_hi covering the box (g_lo = the largest
 *      node index at or below lo, g_hi = the smallest at or above hi) are
 *      copied into the caller's grid (x fastest).
 * The tree must outlive the view; frames of one view run in call order. */
typedef struct sfk_view_s* sfk_view;

typedef struct {
  int32_t kernel;          /* sfk_kernel */
  int32_t bw;              /* SFK_BW_FIXED, SFK_BW_PER_POINT, or SFK_BW_ROI_SCALED:
                              h_k = h0 * (res - 1) * s, fixed per lattice */
  int32_t norm;            /* sfk_norm */
  int32_t res;             /* wanted nodes across the box's longest side, >= 2 */
  float h[3];              /* FIXED: h per axis; ROI_SCALED: h0 in h[0] */
  int32_t block;           /* nodes per block edge: 8, 16, 32 or 64 (0 = 32) */
  double scale_threshold;  /* >= 1 (1: a new lattice whenever the spacing changes) */
  double margin;           /* >= 0, fraction of the box's longest side */
  int64_t max_blocks;      /* cache capacity in blocks, >= 1 */
} sfk_view_opts;

typedef struct {
  double lo[3], hi[3];       /* coordinates of the grid's first and last node */
  int64_t g0[3];             /* lattice index of the grid's first node */
  int32_t res[3];            /* nodes per axis of the grid */
  int32_t new_lattice;       /* 1 if the frame creates (created) a lattice */
  double spacing;            /* spacing s of the lattice */
  int64_t lattice_id;        /* lattices are numbered from 0 in creation order */
  int64_t blocks_needed;     /* blocks covering the box plus margin */
  int64_t blocks_evaluated;  /* of those, evaluated by this frame */
} sfk_view_frame_info;

/* Create a view of tree. The cache (max_blocks * block^3 floats) comes from
 * the context's allocator and counts against its budget (SFK_E_BUDGET).
 * SFK_E_INVAL: NULL pointers, kernel/norm out of range, bw MBE or out of
 * range, PER_POINT without a per-point bandwidth in the tree, non-positive
 * or non-finite h, res < 2, block not in {0, 8, 16, 32, 64},
 * scale_threshold < 1, margin < 0, max_blocks < 1, or a tree with no
 * particles. */
sfk_status sfk_view_create(sfk_ctx ctx, sfk_tree tree, const sfk_view_opts* opts,
                           sfk_view* out);
/* Waits for the view's last frame, then frees its cache. */
sfk_status sfk_view_destroy(sfk_view view);
/* One frame for the box [lo, hi] (hi > lo, finite). With d_out NULL only
 * *info is filled (what the frame would do; no device work, no state
 * change). Otherwise d_out (device, cap floats) receives the grid,
 * stream-ordered on hip_stream (asynchronous). SFK_E_INVAL if the grid needs
 * more than cap floats or more than 2^31 nodes; SFK_E_BUDGET if the box plus
 * margin needs more than max_blocks blocks. */
sfk_status sfk_view_frame(sfk_view view, const double lo[3], const double hi[3], float* d_out,
                          int64_t cap, sfk_view_frame_info* info, void* hip_stream);

/* ------------------------------------------- adaptive resolution (f4) */
/* Feature-aware refinement of a ROI grid (Section 6.3: a resolution that
 * adapts to the distribution so that fine structures in the region are not
 * missed at a fixed grid size).
 *
 * The base grid is evaluated into roi->d_out like sfk_eval_roi. Its cells
 * are grouped into bricks of `brick` cells per axis (the last brick of an
 * axis takes the cells that remain). A brick is refined when, over its
 * nodes, max - min > threshold * peak, both sides rounded to float32
 * (peak = the largest value of the base grid). A refined brick is the ROI
 * whose box spans the brick's corner nodes (their double coordinates as the
 * parent grid defines them) with 2*cells + 1 nodes per axis (half the
 * spacing), the same kernel, normalisation and bandwidth as the base (a
 * ROI-scaled bandwidth keeps the base ROI's h), evaluated like sfk_eval_roi
 * (bitwise the same as sfk_eval_roi of that ROI) into d_bricks. Refinement
 * repeats inside refined bricks, each split into bricks of `brick` of its
 * own cells, up to max_level levels. The list holds the bricks level by
 * level; within a level, by parent, then z, y, x. If a level's bricks do not
 * fit in the remaining capacity, refinement stops before that level
 * (complete = 0). Blocks on hip_stream between levels. */
typedef struct {
  int32_t level;       /* 1..max_level */
  int32_t parent;      /* index of the parent brick in the list, -1 = the base grid */
  int32_t cell0[3];    /* first cell of the brick in the parent grid */
  int32_t res[3];      /* nodes per axis of the brick's grid */
  double lo[3], hi[3]; /* box of the brick's grid */
  int64_t offset;      /* first float of the brick's grid in d_bricks */
} sfk_brick;

typedef struct {
  int32_t brick;       /* cells per brick edge, 2..64 */
  int32_t max_level;   /* 1..4 */
  float threshold;     /* > 0, relative to the base grid's peak */
  int32_t reserved;
} sfk_adaptive_opts;

typedef struct {
  int32_t n_bricks;    /* bricks listed in h_bricks */
  int32_t levels;      /* refinement levels evaluated */
  int32_t complete;    /* 0 if refinement stopped for lack of capacity */
  float peak;          /* largest value of the base grid */
  int64_t floats_used; /* of d_bricks */
} sfk_adaptive_result;

/* SFK_E_INVAL: NULL pointers, an invalid ROI, brick outside 2..64,
 * max_level outside 1..4, threshold not finite and > 0, cap_floats or
 * cap_bricks < 0. SFK_E_UNSUPPORTED: MBE or set = IN_ROI. */
sfk_status sfk_eval_adaptive(sfk_ctx ctx, sfk_tree tree, const sfk_roi* roi,
                             const sfk_adaptive_opts* opts, float* d_bricks, int64_t cap_floats,
                             sfk_brick* h_bricks, int32_t cap_bricks,
                             sfk_adaptive_result* h_result, void* hip_stream);

/* ----------------------------------------------------------- test exports */

/* Support sets S(n) of grid nodes [node_begin, node_end) of one ROI (CLOUD
 * set, non-MBE), as seen by the evaluation kernels: original particle
 * indices, ascending per node. h_offsets has node_end - node_begin + 1
 * entries; h_idx receives up to cap indices; *needed = total. If the total
 * exceeds cap only h_offsets and *needed are written. */
sfk_status sfk_debug_candidates(sfk_ctx ctx, sfk_tree tree, const sfk_roi* roi,
                                int64_t node_begin, int64_t node_end, int64_t* h_offsets,
                                int64_t* h_idx, int64_t cap, int64_t* needed);
/* Tests of the leaf-id checks: with bit 0 set, the count pass of every later
 * batch of this context stores ids outside the tree in the leaf slots past
 * the 64th of each tile; with bit 1, the fill pass stores them in the leaf
 * lists past the 64th entry of each tile. The fill pass (bit 0) and the
 * evaluation (bit 1) find them, read leaf 0 instead and flag the batch:
 * sfk_wait / sfk_poll of its ticket and its serving requests report
 * SFK_E_INTERNAL; a stream-ordered sfk_eval_roi reports it from the next
 * sfk_eval_roi of the context (which then does no work). 0 turns it off.
 * SFK_E_INVAL outside 0..3. */
sfk_status sfk_debug_poison(sfk_ctx ctx, int32_t bits);
/* Per-particle squared k-NN distance h_j^2 in original order (n floats). */
sfk_status sfk_debug_point_h2(sfk_ctx ctx, sfk_tree tree, float* h_h2);
/* The tree's particle order: h_perm[i] = original index of the i-th
 * particle in leaf (curve) order, n int32. */
sfk_status sfk_debug_tree_order(sfk_ctx ctx, sfk_tree tree, int32_t* h_perm);
/* Host-only (no device work): the sort key the tree build gives the cell
 * (x, y, z) of a 2^bits-per-axis lattice, for n cells given as uint32
 * triples; 3*bits-bit keys to h_keys. SFK_E_INVAL on NULL pointers, n < 0,
 * bits outside 1..21, an unknown curve or a coordinate >= 2^bits. */
sfk_status sfk_debug_curve_keys(int32_t curve, int32_t bits, const uint32_t* h_cells, int64_t n,
                                uint64_t* h_keys);
/* The tile range query of one ROI (CLOUD set, non-MBE) as the evaluation
 * uses it: the ROI is evaluated on the stream-ordered path into roi->d_out
 * (again with larger list capacities if its lists did not all fit), then
 * h_shape[3] = the tile shape, h_tile_cnt[t] = candidate leaves of tile t
 * (tiles x fastest over ceil(res / shape) tiles per axis; written if
 * *n_tiles <= tiles_cap), h_leaves = every tile's leaf list in tile order,
 * each ascending (written if *total <= cap). For the particle sweep
 * (shape 8x8x8) the tiles keep no lists (h_tile_cnt all 0) and h_leaves
 * holds the sweep's work items instead: the ascending indices of the boxes
 * of the hierarchy's first interior level (of the leaves when the tree has
 * at most 64) that pass the box test against the ROI's nodes, *total of
 * them. Blocks. */
sfk_status sfk_debug_tile_leaves(sfk_ctx ctx, sfk_tree tree, const sfk_roi* roi, int32_t* h_shape,
                                 int64_t* h_tile_cnt, int64_t tiles_cap, int32_t* h_leaves,
                                 int64_t cap, int64_t* n_tiles, int64_t* total);
/* Leaf boxes of the tree: h_boxes[6 i .. 6 i + 5] = lo xyz, hi xyz of leaf i
 * (leaf i holds particle slots 64 i .. 64 i + 63 in curve order). */
sfk_status sfk_debug_leaf_boxes(sfk_ctx ctx, sfk_tree tree, float* h_boxes);
/* Host-only (no device work): the Marching Cubes triangles sfk_iso_surface
 * uses for case cs (0..255): *n_tri triangles, 3 * n_tri edge ids in
 * h_edges (room for 15; edge ids as sfk_iso_surface describes: along x
 * dy + 2 dz, along y 4 + dx + 2 dz, along z 8 + dx + 2 dy). */
sfk_status sfk_debug_mc_case(int32_t cs, int8_t* h_edges, int32_t* n_tri);
/* Useful pairs E = sum_n #S(n) and pairs tested by the evaluation kernel
 * (tiles: listed leaves x 64 x nodes per tile; the particle sweep: listed
 * boxes x 4096 particles x the unrolled node span NM^3, an upper bound). */
sfk_status sfk_debug_eval_count(sfk_ctx ctx, sfk_tree tree, const sfk_roi* roi,
                                int64_t* useful_pairs, int64_t* tested_pairs);
/* Host-only: the tree's estimate of its particles in the closed box
 * [h_lo, h_hi] (3 doubles each, h_lo <= h_hi), as the runtime uses it to
 * choose tile shapes and to cap serving batches: the counts of the finest
 * host-held box level spread over a 32^3 lattice on the tree's bounding box
 * and summed (evenly within each cell). SFK_E_INVAL on a NULL or non-finite
 * argument or h_lo > h_hi. */
sfk_status sfk_debug_particle_estimate(sfk_ctx ctx, sfk_tree tree, const double* h_lo,
                                       const double* h_hi, double* particles);
/* Per-node support counts #S(n) (res product floats, device, x fastest). */
sfk_status sfk_debug_support_counts(sfk_ctx ctx, sfk_tree tree, const sfk_roi* roi,
                                    float* d_counts, void* hip_stream);

/* MBE stages of one ROI (Section 3.1). Host outputs, any may be NULL:
 * h_ell0[3] Eq. 1 lengths; *n_b particles in B; h_idx_b[n_b] their original
 * indices (ascending); h_pilot[M] pilot grid (Eq. 2); h_pden[n_b] pilot at
 * each particle (trilinear); *aveden (Eq. 5, mean); h_ell_j[n_b*3] adaptive
 * lengths (Eq. 6), in the order of h_idx_b. cap_b bounds the per-particle
 * outputs (SFK_E_INVAL if n_b > cap_b; *n_b is still written). The final
 * grid goes to roi->d_out. */
sfk_status sfk_debug_mbe(sfk_ctx ctx, sfk_tree tree, const sfk_roi* roi, float* h_ell0,
                         int64_t* n_b, int64_t* h_idx_b, float* h_pilot, float* h_pden,
                         double* aveden, float* h_ell_j, int64_t cap_b);

#ifdef __cplusplus
}
#endif
#endif /* SFKDE_H */
