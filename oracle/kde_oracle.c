/*
 * kde_oracle.c -- plain, slow, brute-force CPU reference for ROI kernel
 * density estimation (ScaleFree, arXiv 2601.20758, Section 3.1).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do. It shares no code, header or constant with the
 * HIP implementation.
 *
 * Conventions (the readings of the paper that every function below follows):
 *  - Grid nodes are vertex-centred on the closed box B: along axis k,
 *    x_i = lo + (i * (hi - lo)) / (res - 1) in double (Section 3.1 places
 *    nodes on a uniform grid over B and calls their distance the node
 *    spacing s_k = (hi - lo) / (res - 1)).
 *  - Linear node index x fastest: idx = x + y*res_x + z*res_x*res_y
 *    (Algorithm 2 and Algorithm 4 index the density buffer this way).
 *  - Support membership is decided in double on the float32 inputs by one
 *    fixed operation sequence (the "canonical predicate"), every operation
 *    rounded to double, no fused multiply-add:
 *        d_k = x_nk - p_k;  u_k = d_k * ih_k;
 *        u2  = (u_x*u_x + u_y*u_y) + u_z*u_z;
 *        member  <=>  u2 < c2
 *    with ih_k = (float)(1 / h_k) the float32 inverse bandwidth and c2 = 1
 *    for the Epanechnikov kernel (Eq. 4: zero for |x| >= 1, so the support
 *    boundary is excluded) and c2 = 9 for the Gaussian truncated at 3h.
 *    This is the per-axis scaled distance of Eq. 3 and Algorithm 2.
 *  - Kernel values are functions of that same u2.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -fPIC -shared.
 * Every loop over particles runs in index order inside one thread, so results
 * do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EPANECHNIKOV 0
#define ORC_GAUSS_TRUNC3 1
#define ORC_COUNT 2

/* ------------------------------------------------------------------------ */
/* Kernel normalisation constants.                                          */
/* ------------------------------------------------------------------------ */

/* Epanechnikov in 3D: 15 / (8 pi), the prefactor of Eq. 2 and Eq. 7. */
double orc_ck_epanechnikov(void) { return 15.0 / (8.0 * M_PI); }

/* Probability that a 3D standard normal vector has norm < 3, i.e.
 * P(chi^2_3 < 9) = erf(3/sqrt 2) - sqrt(2/pi) * 3 * exp(-9/2). */
double orc_p_chi2_3_below_9(void) {
  return erf(3.0 / sqrt(2.0)) - sqrt(2.0 / M_PI) * 3.0 * exp(-4.5);
}

/* Gaussian with sigma = h truncated at 3h and renormalised to unit mass:
 * 1 / ((2 pi)^{3/2} P(chi^2_3 < 9)). The paper uses only the Epanechnikov
 * kernel; the truncated Gaussian serves the per-point bandwidth workload. */
double orc_ck_gauss_trunc3(void) {
  return 1.0 / (pow(2.0 * M_PI, 1.5) * orc_p_chi2_3_below_9());
}

double orc_kernel_ck(int kernel) {
  if (kernel == ORC_EPANECHNIKOV) return orc_ck_epanechnikov();
  if (kernel == ORC_GAUSS_TRUNC3) return orc_ck_gauss_trunc3();
  return 1.0;
}

double orc_kernel_c2(int kernel) {
  return kernel == ORC_GAUSS_TRUNC3 ? 9.0 : 1.0;
}

/* Kernel profile of the squared scaled distance u2 (double). Eq. 4 for the
 * Epanechnikov kernel; exp(-u2/2) for the Gaussian; 1 for counting. */
double orc_kernel_value(int kernel, double u2) {
  if (kernel == ORC_EPANECHNIKOV) {
    double v = 1.0 - u2;
    return v > 0.0 ? v : 0.0;
  }
  if (kernel == ORC_GAUSS_TRUNC3) return exp(-0.5 * u2);
  return 1.0;
}

/* ------------------------------------------------------------------------ */
/* Grid geometry.                                                           */
/* ------------------------------------------------------------------------ */

double orc_node_coord(double lo, double hi, int res, int i) {
  return lo + ((double)i * (hi - lo)) / (double)(res - 1);
}

void orc_axis_coords(double lo, double hi, int res, double* out) {
  for (int i = 0; i < res; ++i) out[i] = orc_node_coord(lo, hi, res, i);
}

/* ------------------------------------------------------------------------ */
/* Canonical membership quantity: squared scaled distance in double.        */
/* ------------------------------------------------------------------------ */

double orc_u2(double xn, double yn, double zn, float px, float py, float pz,
              float ihx, float ihy, float ihz) {
  double ux = (xn - (double)px) * (double)ihx;
  double uy = (yn - (double)py) * (double)ihy;
  double uz = (zn - (double)pz) * (double)ihz;
  double sxy = ux * ux + uy * uy;
  return sxy + uz * uz;
}

/* ------------------------------------------------------------------------ */
/* Density at grid nodes (Eq. 2 with a uniform bandwidth, Eq. 7 with a      */
/* per-particle bandwidth).                                                 */
/*                                                                          */
/*  rho(n) = scale * sum_j [u2(n, j) < c2] * w_j * K(u2(n, j))              */
/*                                                                          */
/* pts      n x 3 float positions                                           */
/* ih_pp    n x 3 per-particle inverse bandwidths, or NULL -> ih_u          */
/* w_pp     n per-particle weights 1/(h_x h_y h_z), or NULL -> w_u          */
/* include  n flags (nonzero = particle takes part), or NULL -> all         */
/* nodes    node linear indices to evaluate (x fastest), count n_nodes      */
/* scale    C_K * nu (nu = 1/N or 1)                                        */
/* Threads of the OpenMP loops below (timing of the oracle on 1 thread and
 * on all host cores); no effect on any result. */
#include <omp.h>
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------ */
void orc_density_nodes(const float* pts, int64_t n, const float* ih_pp,
                       const double* w_pp, const float* ih_u, double w_u,
                       const uint8_t* include, int kernel, const double* lo,
                       const double* hi, const int* res, double scale,
                       const int64_t* nodes, int64_t n_nodes, double* out) {
  const double c2 = orc_kernel_c2(kernel);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t q = 0; q < n_nodes; ++q) {
    int64_t idx = nodes[q];
    int ix = (int)(idx % res[0]);
    int iy = (int)((idx / res[0]) % res[1]);
    int iz = (int)(idx / ((int64_t)res[0] * res[1]));
    double xn = orc_node_coord(lo[0], hi[0], res[0], ix);
    double yn = orc_node_coord(lo[1], hi[1], res[1], iy);
    double zn = orc_node_coord(lo[2], hi[2], res[2], iz);
    double sum = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      if (include && !include[j]) continue;
      const float* p = pts + 3 * j;
      float ihx, ihy, ihz;
      double w;
      if (ih_pp) {
        ihx = ih_pp[3 * j]; ihy = ih_pp[3 * j + 1]; ihz = ih_pp[3 * j + 2];
      } else {
        ihx = ih_u[0]; ihy = ih_u[1]; ihz = ih_u[2];
      }
      w = w_pp ? w_pp[j] : w_u;
      double u2 = orc_u2(xn, yn, zn, p[0], p[1], p[2], ihx, ihy, ihz);
      if (!(u2 < c2)) continue;
      if (kernel == ORC_COUNT)
        sum += 1.0;
      else
        sum += w * orc_kernel_value(kernel, u2);
    }
    out[q] = kernel == ORC_COUNT ? sum : scale * sum;
  }
}

/* Support set S(n) of each listed node: original particle indices in
 * increasing order. Two-call protocol: with idx == NULL only counts are
 * written (offsets[q+1] - offsets[q]); offsets has n_nodes + 1 entries. */
void orc_candidates(const float* pts, int64_t n, const float* ih_pp,
                    const float* ih_u, const uint8_t* include, int kernel,
                    const double* lo, const double* hi, const int* res,
                    const int64_t* nodes, int64_t n_nodes, int64_t* offsets,
                    int64_t* idx_out) {
  const double c2 = orc_kernel_c2(kernel);
  if (!idx_out) offsets[0] = 0;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t q = 0; q < n_nodes; ++q) {
    int64_t idx = nodes[q];
    int ix = (int)(idx % res[0]);
    int iy = (int)((idx / res[0]) % res[1]);
    int iz = (int)(idx / ((int64_t)res[0] * res[1]));
    double xn = orc_node_coord(lo[0], hi[0], res[0], ix);
    double yn = orc_node_coord(lo[1], hi[1], res[1], iy);
    double zn = orc_node_coord(lo[2], hi[2], res[2], iz);
    int64_t c = 0;
    int64_t base = idx_out ? offsets[q] : 0;
    for (int64_t j = 0; j < n; ++j) {
      if (include && !include[j]) continue;
      const float* p = pts + 3 * j;
      const float* ih = ih_pp ? ih_pp + 3 * j : ih_u;
      double u2 = orc_u2(xn, yn, zn, p[0], p[1], p[2], ih[0], ih[1], ih[2]);
      if (u2 < c2) {
        if (idx_out) idx_out[base + c] = j;
        ++c;
      }
    }
    if (!idx_out) offsets[q + 1] = c;
  }
  if (!idx_out)
    for (int64_t q = 0; q < n_nodes; ++q) offsets[q + 1] += offsets[q];
}

/* ------------------------------------------------------------------------ */
/* Per-point bandwidth from the k-th nearest neighbour.                     */
/* h_j^2 = k-th smallest canonical float32 squared distance from particle j */
/* to every other particle (self excluded by index; coincident particles    */
/* count). Canonical squared distance:                                      */
/*   d_k = fl(p_jk - p_ik); d2 = fl(fl(fl(dx*dx) + fl(dy*dy)) + fl(dz*dz)).  */
/* ------------------------------------------------------------------------ */

float orc_d2_f32(const float* a, const float* b) {
  volatile float dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  volatile float sx = dx * dx, sy = dy * dy, sz = dz * dz;
  volatile float sxy = sx + sy;
  volatile float s = sxy + sz;
  return s;
}

/* Returns 0 on success, -1 if n - 1 < k. Keeps the k smallest distances in
 * an ascending array (insertion), so the answer is its last entry. */
int orc_knn_h2(const float* pts, int64_t n, int k, const int64_t* queries,
               int64_t n_queries, float* out) {
  if (k < 1 || n - 1 < k) return -1;
#pragma omp parallel
  {
    float* a = (float*)malloc(sizeof(float) * (size_t)k);
#pragma omp for schedule(dynamic, 1)
    for (int64_t q = 0; q < n_queries; ++q) {
      int64_t j = queries[q];
      int m = 0; /* entries held, <= k */
      for (int64_t i = 0; i < n; ++i) {
        if (i == j) continue;
        float d = orc_d2_f32(pts + 3 * j, pts + 3 * i);
        if (m == k && !(d < a[k - 1])) continue;
        int p = m < k ? m++ : k - 1; /* slot freed at the end */
        while (p > 0 && a[p - 1] > d) {
          a[p] = a[p - 1];
          --p;
        }
        a[p] = d;
      }
      out[q] = a[k - 1];
    }
    free(a);
  }
  return 0;
}

/* Per-point parameters of a per-particle isotropic bandwidth h_j = sqrt(h2_j):
 * ih_j = (float)(1/h_j) on every axis and w_j = 1/h_j^3. A zero bandwidth
 * (>= k+1 coincident particles) has an empty support: ih = +inf makes every
 * scaled distance infinite or NaN, so the particle is never a member. */
void orc_point_params_from_h2(const float* h2, int64_t n, float* ih3, double* w) {
  for (int64_t j = 0; j < n; ++j) {
    double h = sqrt((double)h2[j]);
    if (h > 0.0) {
      float ih = (float)(1.0 / h);
      ih3[3 * j] = ih3[3 * j + 1] = ih3[3 * j + 2] = ih;
      w[j] = 1.0 / (h * h * h);
    } else {
      ih3[3 * j] = ih3[3 * j + 1] = ih3[3 * j + 2] = INFINITY;
      w[j] = 0.0;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* MBE (Section 3.1): initial smoothing length, pilot, ASL, final.          */
/* ------------------------------------------------------------------------ */

static int cmp_double(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

/* Percentile by linear interpolation between order statistics
 * (Hyndman-Fan type 7): with v sorted ascending and pos = (n-1) q,
 * P = v[floor(pos)] + (pos - floor(pos)) (v[floor(pos)+1] - v[floor(pos)]). */
double orc_percentile_sorted(const double* v, int64_t n, double q) {
  double pos = (double)(n - 1) * q;
  int64_t i = (int64_t)floor(pos);
  double f = pos - (double)i;
  if (i + 1 >= n) return v[n - 1];
  return v[i] + f * (v[i + 1] - v[i]);
}

double orc_percentile(const float* x, int64_t n, int stride, double q) {
  double* v = (double*)malloc(sizeof(double) * (size_t)n);
  for (int64_t i = 0; i < n; ++i) v[i] = (double)x[i * stride];
  qsort(v, (size_t)n, sizeof(double), cmp_double);
  double r = orc_percentile_sorted(v, n, q);
  free(v);
  return r;
}

/* Node spacing s_k of the ROI grid. */
double orc_spacing(double lo, double hi, int res) { return (hi - lo) / (double)(res - 1); }

/* Eq. 1 over the particles inside B (pts_b: n_b x 3):
 *   l_k = 2 (P80_k - P20_k) / ln(N_B),
 * natural logarithm; a non-positive or non-finite result (N_B < 2 or
 * P80 == P20) is replaced by the cap 5 s_k of Eq. 6. Rounded once to float. */
void orc_mbe_initial_ell(const float* pts_b, int64_t n_b, const double* lo,
                         const double* hi, const int* res, float* ell,
                         int* degenerate_flags) {
  *degenerate_flags = 0;
  for (int k = 0; k < 3; ++k) {
    double cap = 5.0 * orc_spacing(lo[k], hi[k], res[k]);
    double l = NAN;
    if (n_b >= 2) {
      double p20 = orc_percentile(pts_b + k, n_b, 3, 0.20);
      double p80 = orc_percentile(pts_b + k, n_b, 3, 0.80);
      l = 2.0 * (p80 - p20) / log((double)n_b);
    }
    if (!(l > 0.0) || !isfinite(l)) {
      l = cap;
      *degenerate_flags |= 1 << k;
    }
    ell[k] = (float)l;
  }
}

/* Trilinear interpolation of a node field (double, x fastest) at position p.
 * f = (p - lo) (res - 1) / (hi - lo); cell i = floor(f) clamped to
 * [0, res - 2]; t = f - i clamped to [0, 1]. */
double orc_trilinear(const double* grid, const double* lo, const double* hi,
                     const int* res, const float* p) {
  int i[3];
  double t[3];
  for (int k = 0; k < 3; ++k) {
    double f = ((double)p[k] - lo[k]) * (double)(res[k] - 1) / (hi[k] - lo[k]);
    int c = (int)floor(f);
    if (c < 0) c = 0;
    if (c > res[k] - 2) c = res[k] - 2;
    double tt = f - (double)c;
    if (tt < 0.0) tt = 0.0;
    if (tt > 1.0) tt = 1.0;
    i[k] = c;
    t[k] = tt;
  }
  double acc = 0.0;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        double wgt = (dx ? t[0] : 1.0 - t[0]) * (dy ? t[1] : 1.0 - t[1]) *
                     (dz ? t[2] : 1.0 - t[2]);
        int64_t idx = (int64_t)(i[0] + dx) +
                      (int64_t)res[0] * ((int64_t)(i[1] + dy) + (int64_t)res[1] * (i[2] + dz));
        acc += wgt * grid[idx];
      }
  return acc;
}

/* Adaptive smoothing length (Eqs. 5-6), given a pilot grid:
 *   pden_j = trilinear(pilot, r_j)                     (Section 3.1)
 *   aveDen = (1/N_B) sum_j pden_j                      (Eq. 5, read as a mean)
 *   l_kj   = min(l_k (aveDen / pden_j)^{1/3}, 5 s_k)   (Eq. 6)
 * pden_j <= 0 gives the cap. ell_j: n_b x 3 floats (rounded once). */
void orc_mbe_asl(const float* pts_b, int64_t n_b, const double* pilot,
                 const double* lo, const double* hi, const int* res,
                 const float* ell0, double* pden, double* aveden, float* ell_j) {
  double sum = 0.0;
  for (int64_t j = 0; j < n_b; ++j) {
    pden[j] = orc_trilinear(pilot, lo, hi, res, pts_b + 3 * j);
    sum += pden[j];
  }
  double ave = n_b > 0 ? sum / (double)n_b : 0.0;
  *aveden = ave;
  for (int64_t j = 0; j < n_b; ++j) {
    for (int k = 0; k < 3; ++k) {
      double cap = 5.0 * orc_spacing(lo[k], hi[k], res[k]);
      double l;
      if (pden[j] > 0.0) {
        l = (double)ell0[k] * cbrt(ave / pden[j]);
        if (l > cap) l = cap;
      } else {
        l = cap;
      }
      ell_j[3 * j + k] = (float)l;
    }
  }
}

/* Per-point parameters of an anisotropic per-particle smoothing length:
 * ih_k = (float)(1/l_k), w = 1/(l_x l_y l_z) in double. */
void orc_params_from_ell(const float* ell, int64_t n, float* ih3, double* w) {
  for (int64_t j = 0; j < n; ++j) {
    double lx = ell[3 * j], ly = ell[3 * j + 1], lz = ell[3 * j + 2];
    ih3[3 * j] = (float)(1.0 / lx);
    ih3[3 * j + 1] = (float)(1.0 / ly);
    ih3[3 * j + 2] = (float)(1.0 / lz);
    w[j] = 1.0 / (lx * ly * lz);
  }
}

/* ------------------------------------------------------------------------ */
/* Consumers of a density grid (Section 3.1, after Eq. 8: the density at any
 * position is the trilinear interpolation of the surrounding grid nodes;
 * Section 4.2 / selection: a density threshold, the Marching Cubes
 * iso-surface as selection volume, and the points inside it). Readings:
 * a position outside the closed box B has no surrounding nodes and density
 * 0; a point is selected when it lies in B and its interpolated density is
 * >= the threshold (the region the iso-surface bounds); the Marching Cubes
 * case of a cell has bit (dx + 2 dy + 4 dz) set when that corner's value is
 * >= the threshold, and a cell is active unless its case is 0 or 255. */

static int orc_in_closed_box(const double* lo, const double* hi, const float* p) {
  for (int k = 0; k < 3; ++k) {
    const double v = (double)p[k];
    if (!(v >= lo[k] && v <= hi[k])) return 0;
  }
  return 1;
}

/* out[j] = density at pts[j] (n x 3 floats), grid values in double. */
void orc_sample_points(const double* grid, const double* lo, const double* hi, const int* res,
                       const float* pts, int64_t n, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; ++j)
    out[j] = orc_in_closed_box(lo, hi, pts + 3 * j)
                 ? orc_trilinear(grid, lo, hi, res, pts + 3 * j)
                 : 0.0;
}

/* Ascending indices of the selected points; returns their count. */
int64_t orc_select_points(const double* grid, const double* lo, const double* hi,
                          const int* res, double iso, const float* pts, int64_t n,
                          int64_t* idx_out) {
  int64_t m = 0;
  for (int64_t j = 0; j < n; ++j) {
    if (!orc_in_closed_box(lo, hi, pts + 3 * j)) continue;
    if (orc_trilinear(grid, lo, hi, res, pts + 3 * j) >= iso) idx_out[m++] = j;
  }
  return m;
}

/* Active Marching Cubes cells in ascending linear cell index (x fastest over
 * (res - 1) cells per axis) and their cases; returns the count. */
int64_t orc_iso_cells(const double* grid, const int* res, double iso, int64_t* cells,
                      uint8_t* cases) {
  const int64_t cx = res[0] - 1, cy = res[1] - 1, cz = res[2] - 1;
  int64_t m = 0;
  for (int64_t k = 0; k < cz; ++k)
    for (int64_t j = 0; j < cy; ++j)
      for (int64_t i = 0; i < cx; ++i) {
        int c = 0;
        for (int b = 0; b < 8; ++b) {
          const int dx = b & 1, dy = (b >> 1) & 1, dz = (b >> 2) & 1;
          const double v =
              grid[(i + dx) + (int64_t)res[0] * ((j + dy) + (int64_t)res[1] * (k + dz))];
          if (v >= iso) c |= 1 << b;
        }
        if (c != 0 && c != 255) {
          cells[m] = i + cx * (j + cy * k);
          cases[m] = (uint8_t)c;
          ++m;
        }
      }
  return m;
}

/* ------------------------------------------------------------------------ */
/* Marching Cubes triangles (Section 4.1: the selection volume is the        */
/* iso-surface the grid's Marching Cubes extraction bounds; Lorensen and     */
/* Cline 1987). The per-case triangles are derived here from the cube's      */
/* faces rather than typed in as a table:                                     */
/*  - corner c = dx + 2 dy + 4 dz is inside when its value is >= iso;        */
/*  - edge ids: x edges dy + 2 dz, y edges 4 + dx + 2 dz, z edges            */
/*    8 + dx + 2 dy (the coordinates of the edge's lower corner);            */
/*  - face (k, v), k the normal axis and v its side, a = (k+1) mod 3,        */
/*    b = (k+2) mod 3: its corners in counterclockwise order seen from       */
/*    outside the cube, (a,b) = (0,0),(1,0),(1,1),(0,1) for v = 1 and        */
/*    (0,0),(0,1),(1,1),(1,0) for v = 0;                                      */
/*  - on each face every edge crossed from an inside to an outside corner    */
/*    (in the face's order) is joined to the first crossed edge met going    */
/*    backwards around the face: one segment on a face with two crossings,   */
/*    and on a face with four the inside corners are cut off (a rule that    */
/*    depends on the face alone, so the two cells sharing a face agree and   */
/*    the surface is closed);                                                 */
/*  - the segments form closed loops (each crossed edge leaves on one face   */
/*    and arrives on the other); loops start at their smallest edge, in      */
/*    ascending order. A loop v0 .. v(L-1) becomes the fan of triangles      */
/*    (v(s), v(s+i+1), v(s+i)), i = 1 .. L-2 (indices mod L), whose normals  */
/*    point from the inside to the outside; the apex s is the first vertex   */
/*    whose fan has no diagonal joining two edges of one cube face (such a   */
/*    diagonal would lie in the face and not match the neighbouring cell).   */
/* The vertex on edge (corner p, corner q), p the lower corner along the     */
/* edge's axis: t = (iso - f_p) / (f_q - f_p), coordinate                    */
/* x_p + t (x_q - x_p) along that axis and the node coordinates on the       */
/* other two, in double, rounded once to float.                              */
/* ------------------------------------------------------------------------ */

#define ORC_MC_MAXT 12
static int orc_mc_nt[256];
static signed char orc_mc_edges[256][3 * ORC_MC_MAXT];
static int orc_mc_built = 0;

static int orc_edge_of(int c0, int c1) {
  const int d = c0 ^ c1;
  const int lo = c0 < c1 ? c0 : c1;
  const int dx = lo & 1, dy = (lo >> 1) & 1, dz = (lo >> 2) & 1;
  if (d == 1) return dy + 2 * dz;
  if (d == 2) return 4 + dx + 2 * dz;
  return 8 + dx + 2 * dy;
}

/* Do cube edges e and f lie on a common face? An edge along axis k lies on
 * the faces normal to the other two axes at its own coordinates. */
static int orc_edges_share_face(int e, int f) {
  int fa[2][2], fb[2][2];
  int (*fs[2])[2] = {fa, fb};
  const int ed[2] = {e, f};
  for (int w = 0; w < 2; ++w) {
    const int ax = ed[w] / 4, r = ed[w] % 4;
    const int o1 = ax == 0 ? 1 : 0, o2 = ax == 2 ? 1 : 2;
    fs[w][0][0] = o1;
    fs[w][0][1] = r & 1;
    fs[w][1][0] = o2;
    fs[w][1][1] = r >> 1;
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      if (fa[i][0] == fb[j][0] && fa[i][1] == fb[j][1]) return 1;
  return 0;
}

static void orc_mc_build_case(int cs) {
  int succ[12];
  int crossed[12];
  for (int e = 0; e < 12; ++e) succ[e] = -1, crossed[e] = 0;
  for (int k = 0; k < 3; ++k)
    for (int v = 0; v < 2; ++v) {
      const int a = (k + 1) % 3, b = (k + 2) % 3;
      static const int up[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
      static const int dn[4][2] = {{0, 0}, {0, 1}, {1, 1}, {1, 0}};
      int q[4], ein[4], fe[4], cr[4];
      for (int i = 0; i < 4; ++i) {
        const int* ab = v ? up[i] : dn[i];
        q[i] = (v << k) | (ab[0] << a) | (ab[1] << b);
        ein[i] = (cs >> q[i]) & 1;
      }
      for (int i = 0; i < 4; ++i) {
        fe[i] = orc_edge_of(q[i], q[(i + 1) % 4]);
        cr[i] = ein[i] != ein[(i + 1) % 4];
        if (cr[i]) crossed[fe[i]] = 1;
      }
      for (int i = 0; i < 4; ++i) {
        if (!(ein[i] && !ein[(i + 1) % 4])) continue;  /* inside -> outside */
        for (int s = 1; s < 4; ++s) {
          const int j = (i + 4 - s) % 4;
          if (cr[j]) {
            succ[fe[i]] = fe[j];
            break;
          }
        }
      }
    }
  int seen[12] = {0}, nt = 0;
  for (int e = 0; e < 12; ++e) {
    if (!crossed[e] || seen[e]) continue;
    int loop[12], L = 0, x = e;
    do {
      seen[x] = 1;
      loop[L++] = x;
      x = succ[x];
    } while (x != e && x >= 0 && L < 12);
    int apex = 0;
    for (int st = 0; st < L; ++st) {
      int ok = 1;
      for (int i = 2; i + 1 < L; ++i)
        if (orc_edges_share_face(loop[st], loop[(st + i) % L])) ok = 0;
      if (ok) {
        apex = st;
        break;
      }
    }
    for (int i = 1; i + 1 < L; ++i) {
      orc_mc_edges[cs][3 * nt] = (signed char)loop[apex];
      orc_mc_edges[cs][3 * nt + 1] = (signed char)loop[(apex + i + 1) % L];
      orc_mc_edges[cs][3 * nt + 2] = (signed char)loop[(apex + i) % L];
      ++nt;
    }
  }
  orc_mc_nt[cs] = nt;
}

static void orc_mc_build(void) {
  if (orc_mc_built) return;
  for (int cs = 0; cs < 256; ++cs) orc_mc_build_case(cs);
  orc_mc_built = 1;
}

/* Triangles of one case: writes 3 * n edge ids and returns n. */
int orc_mc_case(int cs, int* edges) {
  orc_mc_build();
  for (int i = 0; i < 3 * orc_mc_nt[cs]; ++i) edges[i] = orc_mc_edges[cs][i];
  return orc_mc_nt[cs];
}

/* The iso-surface of the grid: triangles (9 floats each: three vertices)
 * cell by cell in ascending linear cell index, in the case's order. Writes
 * the first min(count, cap) and returns the count. */
int64_t orc_iso_surface(const double* grid, const double* lo, const double* hi, const int* res,
                        double iso, float* tris, int64_t cap) {
  orc_mc_build();
  const int64_t cx = res[0] - 1, cy = res[1] - 1, cz = res[2] - 1;
  int64_t m = 0;
  for (int64_t k = 0; k < cz; ++k)
    for (int64_t j = 0; j < cy; ++j)
      for (int64_t i = 0; i < cx; ++i) {
        int cs = 0;
        double f[8];
        for (int c = 0; c < 8; ++c) {
          const int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
          f[c] = grid[(i + dx) + (int64_t)res[0] * ((j + dy) + (int64_t)res[1] * (k + dz))];
          if (f[c] >= iso) cs |= 1 << c;
        }
        for (int t = 0; t < orc_mc_nt[cs]; ++t, ++m) {
          if (m >= cap) continue;
          for (int vtx = 0; vtx < 3; ++vtx) {
            const int e = orc_mc_edges[cs][3 * t + vtx];
            const int axis = e / 4, r = e % 4;
            int p;
            if (axis == 0) p = 2 * (r & 1) + 4 * (r >> 1);
            else if (axis == 1) p = (r & 1) + 4 * (r >> 1);
            else p = (r & 1) + 2 * (r >> 1);
            const int q = p | (1 << axis);
            const double tt = (iso - f[p]) / (f[q] - f[p]);
            const int64_t ci[3] = {i + (p & 1), j + ((p >> 1) & 1), k + ((p >> 2) & 1)};
            for (int d = 0; d < 3; ++d) {
              const double x0 = orc_node_coord(lo[d], hi[d], res[d], (int)ci[d]);
              double x = x0;
              if (d == axis) {
                const double x1 = orc_node_coord(lo[d], hi[d], res[d], (int)ci[d] + 1);
                x = x0 + tt * (x1 - x0);
              }
              tris[9 * m + 3 * vtx + d] = (float)x;
            }
          }
        }
      }
  return m;
}
