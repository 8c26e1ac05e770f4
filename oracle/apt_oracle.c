/*
 * apt_oracle.c -- TEST INFRASTRUCTURE ONLY: the CPU oracle.
 *
 * Plain definitions of what the spatial-statistics stage of the paper
 * computes, written for a reader to check against the paper by eye.  Build
 * with -O2 -ffp-contract=off (no fast-math): the distance expressions below
 * are evaluated exactly as written.  Nothing here is shared with, or called
 * by, the GPU library.
 *
 * The statistics (paper, Methods: "Descriptive, two-point spatial
 * statistics, and clustering"; Supplementary: "Customized user defined batch
 * processing queues"):
 *   - a target ("central") ion is an ion of species A whose distance to the
 *     specimen edge is at least d_srf (Methods: "Ion-to-edge distancing";
 *     the table of AM case-study tasks states the distance as a minimum);
 *   - neighbours are ions of species B other than the target itself; the
 *     edge filter applies to targets only;
 *   - kNN: the distances to each target's k-th nearest neighbours;
 *   - RDF: counts of target-neighbour pairs per radial bin of a rectangular
 *     transfer function r = [0, step, r_max];
 *   - null model: the same statistics on a random permutation of the labels
 *     (Supplementary: "Importance of high quality random number generators").
 * Precision (Supplementary: "Implementation details"): positions are FP32;
 * the RDF bin of a pair is decided on the FP64 squared distance of the two
 * stored FP32 positions, the kNN order on one fixed FP32 expression with the
 * original index as tie-break.
 */
#include "apt_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the OpenMP loops of the oracle use. */
int32_t orc_threads(void) {
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------- */
/* Distances                                                               */
/* ---------------------------------------------------------------------- */

/* FP32 squared distance: dx*dx, then two fused multiply-adds (dy, dz). */
float orc_d2f(const float* a, const float* b) {
    float dx = b[0] - a[0];
    float dy = b[1] - a[1];
    float dz = b[2] - a[2];
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

/* FP64 squared distance of the two stored positions: ((dx^2 + dy^2) + dz^2). */
double orc_D2(const float* a, const float* b) {
    double dx = (double)b[0] - (double)a[0];
    double dy = (double)b[1] - (double)a[1];
    double dz = (double)b[2] - (double)a[2];
    return ((dx * dx) + (dy * dy)) + (dz * dz);
}

/* ---------------------------------------------------------------------- */
/* Rectangular transfer function: bins [e_b, e_{b+1}), e_b = b*r_max/n     */
/* ---------------------------------------------------------------------- */

void orc_edges2(float r_max, int32_t n_bins, double* E2) {
    for (int32_t b = 0; b <= n_bins; ++b) {
        double e = ((double)b * (double)r_max) / (double)n_bins;
        E2[b] = e * e;
    }
}

int32_t orc_bin_of(double D2, const double* E2, int32_t n_bins) {
    if (!(D2 < E2[n_bins])) return n_bins;
    /* largest b with E2[b] <= D2 (E2[0] = 0 <= D2) */
    int32_t lo = 0, hi = n_bins; /* invariant: E2[lo] <= D2 < E2[hi] */
    while (hi - lo > 1) {
        int32_t mid = lo + (hi - lo) / 2;
        if (E2[mid] <= D2) lo = mid; else hi = mid;
    }
    return lo;
}

/* ---------------------------------------------------------------------- */
/* Eligibility                                                             */
/* ---------------------------------------------------------------------- */

static int is_species(uint8_t s, int32_t want) { return want == ORC_ANY || (int32_t)s == want; }

/* An ion with a NaN or infinite coordinate takes part in no pair, neither as
 * target (its row stays empty) nor as neighbour. */
static int finite3(const float* p) { return isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]); }

static int is_target(int64_t i, const uint8_t* lab, const float* d_bnd, int32_t A, float d_srf) {
    if (!is_species(lab[i], A)) return 0;
    if (d_bnd && !(d_bnd[i] >= d_srf)) return 0; /* inclusive; NaN is never eligible */
    return 1;
}

int64_t orc_select_targets(int64_t n, const uint8_t* lab, const float* d_bnd, int32_t A,
                           float d_srf, int64_t* out_ids) {
    int64_t t = 0;
    for (int64_t i = 0; i < n; ++i)
        if (is_target(i, lab, d_bnd, A, d_srf)) {
            if (out_ids) out_ids[t] = i;
            ++t;
        }
    return t;
}

/* ---------------------------------------------------------------------- */
/* RDF, brute force: every target against every neighbour                 */
/* ---------------------------------------------------------------------- */

void orc_rdf_brute(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n, int32_t A,
                   int32_t B, float d_srf, float r_max, int32_t n_bins, uint64_t* hist) {
    double* E2 = (double*)malloc(sizeof(double) * (size_t)(n_bins + 1));
    orc_edges2(r_max, n_bins, E2);
    memset(hist, 0, sizeof(uint64_t) * (size_t)n_bins);
    for (int64_t i = 0; i < n; ++i) {
        if (!is_target(i, lab, d_bnd, A, d_srf) || !finite3(xyz + 3 * i)) continue;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i || !is_species(lab[j], B) || !finite3(xyz + 3 * j)) continue;
            int32_t b = orc_bin_of(orc_D2(xyz + 3 * i, xyz + 3 * j), E2, n_bins);
            if (b < n_bins) hist[b]++;
        }
    }
    free(E2);
}

/* ---------------------------------------------------------------------- */
/* Uniform grid of the neighbour ions (oracle's own, counting sort)        */
/* ---------------------------------------------------------------------- */

typedef struct {
    double lo[3];
    double h;
    int64_t dim[3];
    int64_t* start; /* [ncell + 1] */
    int64_t* item;  /* neighbour indices, cell by cell, ascending within a cell */
    int64_t nitem;
} ogrid;

static int64_t ocell_axis(const ogrid* g, int a, double x) {
    double f = floor((x - g->lo[a]) / g->h);
    if (!(f >= 0)) return 0;
    if (f > (double)(g->dim[a] - 1)) return g->dim[a] - 1;
    return (int64_t)f;
}

static int pos_finite(double (*pos)(const void*, int64_t, int), const void* ctx, int64_t j) {
    return isfinite(pos(ctx, j, 0)) && isfinite(pos(ctx, j, 1)) && isfinite(pos(ctx, j, 2));
}

/* coords: position of ion i on axis a (pos(i, a)); h_min: smallest cell edge.
 * Only neighbours with finite positions enter the grid. */
static void ogrid_build(ogrid* g, int64_t n, const uint8_t* lab, int32_t B,
                        double (*pos)(const void*, int64_t, int), const void* ctx, double h_min) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int64_t nb = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (!is_species(lab[j], B) || !pos_finite(pos, ctx, j)) continue;
        ++nb;
        for (int a = 0; a < 3; ++a) {
            double v = pos(ctx, j, a);
            if (v < lo[a]) lo[a] = v;
            if (v > hi[a]) hi[a] = v;
        }
    }
    if (nb == 0)
        for (int a = 0; a < 3; ++a) { lo[a] = 0; hi[a] = 0; }
    double h = h_min;
    /* bounded table: at most ~8 cells per neighbour ion */
    for (;;) {
        double cells = 1;
        for (int a = 0; a < 3; ++a) cells *= floor((hi[a] - lo[a]) / h) + 1;
        if (cells <= 8.0 * (double)nb + 64.0) break;
        h *= 1.5;
    }
    int64_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
        g->lo[a] = lo[a];
        g->dim[a] = (int64_t)floor((hi[a] - lo[a]) / h) + 1;
        ncell *= g->dim[a];
    }
    g->h = h;
    g->start = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
    g->item = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nb > 0 ? nb : 1));
    g->nitem = nb;
    int64_t* cellof = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t j = 0; j < n; ++j) {
        if (!is_species(lab[j], B) || !pos_finite(pos, ctx, j)) { cellof[j] = -1; continue; }
        int64_t c[3];
        for (int a = 0; a < 3; ++a) c[a] = ocell_axis(g, a, pos(ctx, j, a));
        cellof[j] = (c[2] * g->dim[1] + c[1]) * g->dim[0] + c[0];
        g->start[cellof[j] + 1]++;
    }
    for (int64_t q = 0; q < ncell; ++q) g->start[q + 1] += g->start[q];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)ncell);
    memcpy(fill, g->start, sizeof(int64_t) * (size_t)ncell);
    for (int64_t j = 0; j < n; ++j)
        if (cellof[j] >= 0) g->item[fill[cellof[j]]++] = j;
    free(fill);
    free(cellof);
}

static void ogrid_free(ogrid* g) {
    free(g->start);
    free(g->item);
}

static double pos_plain(const void* ctx, int64_t j, int a) { return (double)((const float*)ctx)[3 * j + a]; }

/* ---------------------------------------------------------------------- */
/* RDF on the grid: cells of edge >= r_max, the 27 surrounding cells       */
/* ---------------------------------------------------------------------- */

void orc_rdf_grid(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n, int32_t A,
                  int32_t B, float d_srf, float r_max, int32_t n_bins, uint64_t* hist) {
    double* E2 = (double*)malloc(sizeof(double) * (size_t)(n_bins + 1));
    orc_edges2(r_max, n_bins, E2);
    ogrid g;
    ogrid_build(&g, n, lab, B, pos_plain, xyz, (double)r_max * (1.0 + 1e-6));
    memset(hist, 0, sizeof(uint64_t) * (size_t)n_bins);
#pragma omp parallel
    {
        /* one result buffer per thread, summed at the end */
        uint64_t* loc = (uint64_t*)calloc((size_t)n_bins, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            if (!is_target(i, lab, d_bnd, A, d_srf) || !finite3(xyz + 3 * i)) continue;
            const float* pi = xyz + 3 * i;
            int64_t c[3];
            for (int a = 0; a < 3; ++a) c[a] = ocell_axis(&g, a, (double)pi[a]);
            for (int64_t z = c[2] - 1; z <= c[2] + 1; ++z) {
                if (z < 0 || z >= g.dim[2]) continue;
                for (int64_t y = c[1] - 1; y <= c[1] + 1; ++y) {
                    if (y < 0 || y >= g.dim[1]) continue;
                    for (int64_t x = c[0] - 1; x <= c[0] + 1; ++x) {
                        if (x < 0 || x >= g.dim[0]) continue;
                        int64_t cell = (z * g.dim[1] + y) * g.dim[0] + x;
                        for (int64_t t = g.start[cell]; t < g.start[cell + 1]; ++t) {
                            int64_t j = g.item[t];
                            if (j == i) continue;
                            int32_t b = orc_bin_of(orc_D2(pi, xyz + 3 * j), E2, n_bins);
                            if (b < n_bins) loc[b]++;
                        }
                    }
                }
            }
        }
#pragma omp critical
        for (int32_t b = 0; b < n_bins; ++b) hist[b] += loc[b];
        free(loc);
    }
    ogrid_free(&g);
    free(E2);
}

/* ---------------------------------------------------------------------- */
/* kNN                                                                     */
/* ---------------------------------------------------------------------- */

/* Order key: FP32 squared distance bits (non-negative floats order like their
 * bit patterns), then the neighbour's original index. */
static uint64_t knn_key(float d2, int64_t j) {
    uint32_t bits;
    memcpy(&bits, &d2, sizeof bits);
    return ((uint64_t)bits << 32) | (uint64_t)(uint32_t)j;
}
static float key_d2(uint64_t key) {
    uint32_t bits = (uint32_t)(key >> 32);
    float f;
    memcpy(&f, &bits, sizeof f);
    return f;
}

/* Keep the k smallest keys seen so far, ascending (insertion). */
static void topk_insert(uint64_t* best, int32_t* cnt, int32_t k, uint64_t key) {
    if (*cnt == k && key >= best[k - 1]) return;
    int32_t p = *cnt < k ? (*cnt)++ : k - 1;
    while (p > 0 && best[p - 1] > key) {
        best[p] = best[p - 1];
        --p;
    }
    best[p] = key;
}

static void knn_emit(const float* xyz, int64_t i, int64_t row, const uint64_t* best, int32_t cnt,
                     int32_t k, int64_t* target_id, float* dist, int64_t* nbr_id, const double* KE2,
                     int32_t kb_nbins, uint64_t* knn_hist) {
    target_id[row] = i;
    for (int32_t m = 0; m < k; ++m) {
        if (m < cnt) {
            dist[row * k + m] = sqrtf(key_d2(best[m]));
            nbr_id[row * k + m] = (int64_t)(uint32_t)best[m];
        } else {
            dist[row * k + m] = INFINITY;
            nbr_id[row * k + m] = -1;
        }
    }
    if (knn_hist) {
        int32_t b = kb_nbins;
        if (cnt == k) b = orc_bin_of(orc_D2(xyz + 3 * i, xyz + 3 * (uint32_t)best[k - 1]), KE2, kb_nbins);
#pragma omp atomic
        knn_hist[b]++;
    }
}

static double* knn_hist_setup(float kb_rmax, int32_t kb_nbins, uint64_t* knn_hist) {
    if (!knn_hist) return NULL;
    double* KE2 = (double*)malloc(sizeof(double) * (size_t)(kb_nbins + 1));
    orc_edges2(kb_rmax, kb_nbins, KE2);
    memset(knn_hist, 0, sizeof(uint64_t) * (size_t)(kb_nbins + 1));
    return KE2;
}

int64_t orc_knn_brute(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n,
                      int32_t A, int32_t B, float d_srf, int32_t k, float r_knn_max,
                      int64_t* target_id, float* dist, int64_t* nbr_id, float kb_rmax,
                      int32_t kb_nbins, uint64_t* knn_hist) {
    double* KE2 = knn_hist_setup(kb_rmax, kb_nbins, knn_hist);
    float rk2 = r_knn_max * r_knn_max;
    uint64_t* best = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)k);
    int64_t row = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!is_target(i, lab, d_bnd, A, d_srf)) continue;
        int32_t cnt = 0;
        for (int64_t j = 0; j < n && finite3(xyz + 3 * i); ++j) {
            if (j == i || !is_species(lab[j], B) || !finite3(xyz + 3 * j)) continue;
            float d2 = orc_d2f(xyz + 3 * i, xyz + 3 * j);
            if (!(d2 <= rk2)) continue;
            topk_insert(best, &cnt, k, knn_key(d2, j));
        }
        knn_emit(xyz, i, row, best, cnt, k, target_id, dist, nbr_id, KE2, kb_nbins, knn_hist);
        ++row;
    }
    free(best);
    free(KE2);
    return row;
}

/* Grid kNN: examine cells in growing cubes around the target's cell; the
 * k-th key is final once its distance is below the distance from the target
 * to the outside of the examined cube. */
int64_t orc_knn_grid(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n,
                     int32_t A, int32_t B, float d_srf, int32_t k, float r_knn_max,
                     int64_t* target_id, float* dist, int64_t* nbr_id, float kb_rmax,
                     int32_t kb_nbins, uint64_t* knn_hist) {
    double* KE2 = knn_hist_setup(kb_rmax, kb_nbins, knn_hist);
    float rk2 = r_knn_max * r_knn_max;
    int64_t T = orc_select_targets(n, lab, d_bnd, A, d_srf, NULL);
    int64_t* tid = (int64_t*)malloc(sizeof(int64_t) * (size_t)(T > 0 ? T : 1));
    orc_select_targets(n, lab, d_bnd, A, d_srf, tid);
    int64_t nb = 0;
    for (int64_t j = 0; j < n; ++j) nb += is_species(lab[j], B) && finite3(xyz + 3 * j);
    /* cell edge ~ the spacing that holds a few neighbours per cell */
    double vol = 1.0;
    {
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int64_t j = 0; j < n; ++j)
            if (is_species(lab[j], B) && finite3(xyz + 3 * j))
                for (int a = 0; a < 3; ++a) {
                    if (xyz[3 * j + a] < lo[a]) lo[a] = xyz[3 * j + a];
                    if (xyz[3 * j + a] > hi[a]) hi[a] = xyz[3 * j + a];
                }
        for (int a = 0; a < 3; ++a) vol *= (nb > 0 ? hi[a] - lo[a] : 0.0) + 1e-3;
    }
    double h0 = cbrt(vol * (double)(k > 4 ? k : 4) / (double)(nb > 0 ? nb : 1));
    if (h0 < 1e-3) h0 = 1e-3;
    ogrid g;
    ogrid_build(&g, n, lab, B, pos_plain, xyz, h0);
#pragma omp parallel
    {
        uint64_t* best = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)k);
#pragma omp for schedule(dynamic, 64)
        for (int64_t row = 0; row < T; ++row) {
            int64_t i = tid[row];
            const float* pi = xyz + 3 * i;
            int64_t c[3];
            for (int a = 0; a < 3; ++a) c[a] = ocell_axis(&g, a, (double)pi[a]);
            int32_t cnt = 0;
            for (int64_t s = 0; finite3(pi); ++s) {
                /* cells on the surface of the cube of half-width s */
                for (int64_t z = c[2] - s; z <= c[2] + s; ++z) {
                    if (z < 0 || z >= g.dim[2]) continue;
                    for (int64_t y = c[1] - s; y <= c[1] + s; ++y) {
                        if (y < 0 || y >= g.dim[1]) continue;
                        for (int64_t x = c[0] - s; x <= c[0] + s; ++x) {
                            if (x < 0 || x >= g.dim[0]) continue;
                            int64_t ax = x - c[0], ay = y - c[1], az = z - c[2];
                            int64_t cheb = llabs(ax);
                            if (llabs(ay) > cheb) cheb = llabs(ay);
                            if (llabs(az) > cheb) cheb = llabs(az);
                            if (cheb != s) continue;
                            int64_t cell = (z * g.dim[1] + y) * g.dim[0] + x;
                            for (int64_t t = g.start[cell]; t < g.start[cell + 1]; ++t) {
                                int64_t j = g.item[t];
                                if (j == i) continue;
                                float d2 = orc_d2f(pi, xyz + 3 * j);
                                if (!(d2 <= rk2)) continue;
                                topk_insert(best, &cnt, k, knn_key(d2, j));
                            }
                        }
                    }
                }
                /* distance from the target to the outside of the examined cube;
                 * a side that reaches the edge of the grid has nothing beyond it */
                double cover = INFINITY;
                int whole = 1;
                for (int a = 0; a < 3; ++a) {
                    if (c[a] - s > 0) {
                        double w = (double)pi[a] - (g.lo[a] + (double)(c[a] - s) * g.h);
                        if (w < cover) cover = w;
                        whole = 0;
                    }
                    if (c[a] + s < g.dim[a] - 1) {
                        double w = (g.lo[a] + (double)(c[a] + s + 1) * g.h) - (double)pi[a];
                        if (w < cover) cover = w;
                        whole = 0;
                    }
                }
                if (whole) break;
                if (cover > 0 && (double)r_knn_max < cover * (1.0 - 1e-5)) break;
                if (cnt == k && cover > 0 && (double)key_d2(best[k - 1]) < cover * cover * (1.0 - 1e-5))
                    break;
            }
            knn_emit(xyz, i, row, best, cnt, k, target_id, dist, nbr_id, KE2, kb_nbins, knn_hist);
        }
        free(best);
    }
    ogrid_free(&g);
    free(tid);
    free(KE2);
    return T;
}

/* ---------------------------------------------------------------------- */
/* Null model: a random permutation of the labels                          */
/* ---------------------------------------------------------------------- */

/* i-th output (i = 0, 1, ...) of SplitMix64 started from state `seed`
 * (Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014): the state advances by the golden gamma, then is mixed. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

typedef struct {
    uint64_t key;
    int64_t idx;
} keyed;

static int keyed_cmp(const void* a, const void* b) {
    const keyed* x = (const keyed*)a;
    const keyed* y = (const keyed*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

/* pi = ascending order of the keys (ties by index); out[i] = lab[pi(i)]. */
void orc_permute_labels(const uint8_t* lab, int64_t n, uint64_t seed, uint8_t* out) {
    keyed* a = (keyed*)malloc(sizeof(keyed) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        a[i].key = orc_splitmix64(seed, (uint64_t)i);
        a[i].idx = i;
    }
    qsort(a, (size_t)n, sizeof(keyed), keyed_cmp);
    for (int64_t i = 0; i < n; ++i) out[i] = lab[a[i].idx];
    free(a);
}

/* ---------------------------------------------------------------------- */
/* Gaussian-smoothed RDF (FP64) and its adjoint                            */
/* ---------------------------------------------------------------------- */
/* Each pair adds to bin b the Gaussian mass (std sigma, centred on the pair
 * distance D) that falls in [e_b, e_{b+1}); only bins meeting
 * (D - 6 sigma, D + 6 sigma) and pairs with D < r_max + 6 sigma take part.
 * Coordinates are (x, y, s*z); d_bnd is not rescaled. */

static double Phi(double t) { return 0.5 * erfc(-t / M_SQRT2); }   /* lower tail */
static double Qtail(double t) { return 0.5 * erfc(t / M_SQRT2); }  /* upper tail */
static double phi(double t) { return exp(-0.5 * t * t) / sqrt(2.0 * M_PI); }

static double bin_mass(double lo, double hi) {
    /* P(lo <= Z < hi), Z standard normal, from the tail that does not cancel */
    if (lo >= 0) return Qtail(lo) - Qtail(hi);
    if (hi <= 0) return Phi(hi) - Phi(lo);
    return 1.0 - Qtail(hi) - Phi(lo);
}

typedef struct {
    const float* xyz;
    double s;
} scaled_ctx;

static double pos_scaled(const void* ctx, int64_t j, int a) {
    const scaled_ctx* c = (const scaled_ctx*)ctx;
    double v = (double)c->xyz[3 * j + a];
    return a == 2 ? c->s * v : v;
}

/* Calls visit(i, j, dX, dY, dZ, D, user) for every target i and neighbour j
 * with D < r_max + 6 sigma in scaled coordinates (serial, ascending i). */
typedef void (*pair_visitor)(int64_t i, int64_t j, double dX, double dY, double dZ, double D,
                             void* user);

static void smooth_pairs(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n,
                         int32_t A, int32_t B, float d_srf, double cut, double s,
                         pair_visitor visit, void* user) {
    scaled_ctx ctx = {xyz, s};
    ogrid g;
    ogrid_build(&g, n, lab, B, pos_scaled, &ctx, cut * (1.0 + 1e-6));
    for (int64_t i = 0; i < n; ++i) {
        if (!is_target(i, lab, d_bnd, A, d_srf) || !pos_finite(pos_scaled, &ctx, i)) continue;
        double P[3];
        int64_t c[3];
        for (int a = 0; a < 3; ++a) {
            P[a] = pos_scaled(&ctx, i, a);
            c[a] = ocell_axis(&g, a, P[a]);
        }
        for (int64_t z = c[2] - 1; z <= c[2] + 1; ++z) {
            if (z < 0 || z >= g.dim[2]) continue;
            for (int64_t y = c[1] - 1; y <= c[1] + 1; ++y) {
                if (y < 0 || y >= g.dim[1]) continue;
                for (int64_t x = c[0] - 1; x <= c[0] + 1; ++x) {
                    if (x < 0 || x >= g.dim[0]) continue;
                    int64_t cell = (z * g.dim[1] + y) * g.dim[0] + x;
                    for (int64_t t = g.start[cell]; t < g.start[cell + 1]; ++t) {
                        int64_t j = g.item[t];
                        if (j == i) continue;
                        double dX = pos_scaled(&ctx, j, 0) - P[0];
                        double dY = pos_scaled(&ctx, j, 1) - P[1];
                        double dZ = pos_scaled(&ctx, j, 2) - P[2];
                        double D = sqrt(((dX * dX) + (dY * dY)) + (dZ * dZ));
                        if (D < cut) visit(i, j, dX, dY, dZ, D, user);
                    }
                }
            }
        }
    }
    ogrid_free(&g);
}

typedef struct {
    const double* e;
    int32_t n_bins;
    double sigma;
    double* h;
    const double* grad_h;
    double* grad;
    double grad_s;
    double s;
    const float* xyz;
} smooth_state;

/* window of bins [*b0, *b1] that meet (D - 6 sigma, D + 6 sigma) */
static void window(const smooth_state* st, double D, int32_t* b0, int32_t* b1) {
    double w = 6.0 * st->sigma;
    *b0 = st->n_bins;
    *b1 = -1;
    for (int32_t b = 0; b < st->n_bins; ++b)
        if (st->e[b + 1] > D - w && st->e[b] < D + w) {
            if (b < *b0) *b0 = b;
            *b1 = b;
        }
}

static void visit_fwd(int64_t i, int64_t j, double dX, double dY, double dZ, double D, void* user) {
    (void)i; (void)j; (void)dX; (void)dY; (void)dZ;
    smooth_state* st = (smooth_state*)user;
    int32_t b0, b1;
    window(st, D, &b0, &b1);
    for (int32_t b = b0; b <= b1; ++b)
        st->h[b] += bin_mass((st->e[b] - D) / st->sigma, (st->e[b + 1] - D) / st->sigma);
}

static void visit_bwd(int64_t i, int64_t j, double dX, double dY, double dZ, double D, void* user) {
    smooth_state* st = (smooth_state*)user;
    if (D == 0.0) return;
    int32_t b0, b1;
    window(st, D, &b0, &b1);
    /* g = dL/dD = sum_b dL/dh_b * dw_b/dD, dw_b/dD = -(phi(c) - phi(a)) / sigma */
    double g = 0.0;
    for (int32_t b = b0; b <= b1; ++b) {
        double a = (st->e[b] - D) / st->sigma, c = (st->e[b + 1] - D) / st->sigma;
        g += st->grad_h[b] * (-(phi(c) - phi(a)) / st->sigma);
    }
    /* D = |p'_j - p'_i|; dD/dp'_j = u, dD/dp'_i = -u, u = (p'_j - p'_i)/D;
     * z' = s z, so dL/dz = s dL/dz' and dD/ds = s (z_j - z_i)^2 / D */
    double u[3] = {dX / D, dY / D, dZ / D};
    for (int a = 0; a < 3; ++a) {
        double f = a == 2 ? st->s : 1.0;
        st->grad[3 * j + a] += g * u[a] * f;
        st->grad[3 * i + a] -= g * u[a] * f;
    }
    double dz = (double)st->xyz[3 * j + 2] - (double)st->xyz[3 * i + 2];
    st->grad_s += g * st->s * dz * dz / D;
}

static double* bin_edges(float r_max, int32_t n_bins) {
    double* e = (double*)malloc(sizeof(double) * (size_t)(n_bins + 1));
    for (int32_t b = 0; b <= n_bins; ++b) e[b] = ((double)b * (double)r_max) / (double)n_bins;
    return e;
}

void orc_smooth_fwd(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n,
                    int32_t A, int32_t B, float d_srf, float r_max, int32_t n_bins, float sigma,
                    double s, double* h) {
    smooth_state st;
    memset(&st, 0, sizeof st);
    st.e = bin_edges(r_max, n_bins);
    st.n_bins = n_bins;
    st.sigma = (double)sigma;
    st.h = h;
    st.s = s;
    st.xyz = xyz;
    memset(h, 0, sizeof(double) * (size_t)n_bins);
    smooth_pairs(xyz, lab, d_bnd, n, A, B, d_srf, (double)r_max + 6.0 * (double)sigma, s, visit_fwd, &st);
    free((void*)st.e);
}

void orc_smooth_bwd(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n,
                    int32_t A, int32_t B, float d_srf, float r_max, int32_t n_bins, float sigma,
                    double s, const double* grad_h, double* grad_xyz, double* grad_s) {
    smooth_state st;
    memset(&st, 0, sizeof st);
    st.e = bin_edges(r_max, n_bins);
    st.n_bins = n_bins;
    st.sigma = (double)sigma;
    st.grad_h = grad_h;
    st.grad = grad_xyz;
    st.s = s;
    st.xyz = xyz;
    memset(grad_xyz, 0, sizeof(double) * 3 * (size_t)n);
    smooth_pairs(xyz, lab, d_bnd, n, A, B, d_srf, (double)r_max + 6.0 * (double)sigma, s, visit_bwd, &st);
    *grad_s = st.grad_s;
    free((void*)st.e);
}

/* Central finite differences of L = sum_b (h_b - t_b)^2 with respect to the
 * stored coordinates of a list of ions, step `step` (nm), given
 * resid[b] = h_b - t_b at the unperturbed positions.  Moving one ion changes
 * only the pairs it takes part in (as target and as neighbour), so with
 * c(P) = the smoothed counts of those pairs with the ion at P and
 * dp = c(P + step) - c(P), dm = c(P - step) - c(P):
 *   L(+) - L(-) = sum_b (dp_b - dm_b) (2 resid_b + dp_b + dm_b)
 * exactly; fd = that / (2 step).  Serial. */
static void ion_pairs_at(const smooth_state* st, const float* xyz, const uint8_t* lab, const float* d_bnd,
                         int32_t A, int32_t B, float d_srf, double cut, const ogrid* gB, const ogrid* gA,
                         const scaled_ctx* ctx, int64_t m, const double P[3], double* c) {
    const int as_target = is_target(m, lab, d_bnd, A, d_srf);
    const int as_nbr = is_species(lab[m], B);
    for (int role = 0; role < 2; ++role) {
        if (role == 0 && !as_target) continue;
        if (role == 1 && !as_nbr) continue;
        const ogrid* g = role == 0 ? gB : gA;
        int64_t cc[3];
        for (int a = 0; a < 3; ++a) cc[a] = ocell_axis(g, a, P[a]);
        for (int64_t z = cc[2] - 1; z <= cc[2] + 1; ++z) {
            if (z < 0 || z >= g->dim[2]) continue;
            for (int64_t y = cc[1] - 1; y <= cc[1] + 1; ++y) {
                if (y < 0 || y >= g->dim[1]) continue;
                for (int64_t x = cc[0] - 1; x <= cc[0] + 1; ++x) {
                    if (x < 0 || x >= g->dim[0]) continue;
                    int64_t cell = (z * g->dim[1] + y) * g->dim[0] + x;
                    for (int64_t t = g->start[cell]; t < g->start[cell + 1]; ++t) {
                        int64_t j = g->item[t];
                        if (j == m) continue;
                        if (role == 1 && !is_target(j, lab, d_bnd, A, d_srf)) continue;
                        double dX = pos_scaled(ctx, j, 0) - P[0];
                        double dY = pos_scaled(ctx, j, 1) - P[1];
                        double dZ = pos_scaled(ctx, j, 2) - P[2];
                        double D = sqrt(((dX * dX) + (dY * dY)) + (dZ * dZ));
                        if (!(D < cut)) continue;
                        int32_t b0, b1;
                        window(st, D, &b0, &b1);
                        for (int32_t b = b0; b <= b1; ++b)
                            c[b] += bin_mass((st->e[b] - D) / st->sigma, (st->e[b + 1] - D) / st->sigma);
                    }
                }
            }
        }
    }
    (void)xyz;
}

void orc_smooth_fd(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n, int32_t A, int32_t B,
                   float d_srf, float r_max, int32_t n_bins, float sigma, double s, const double* resid,
                   const int64_t* ions, int64_t n_ions, double step, double* fd) {
    smooth_state st;
    memset(&st, 0, sizeof st);
    st.e = bin_edges(r_max, n_bins);
    st.n_bins = n_bins;
    st.sigma = (double)sigma;
    const double cut = (double)r_max + 6.0 * (double)sigma;
    const double reach = cut * (1.0 + 1e-6) + 2.0 * step * (fabs(s) > 1.0 ? fabs(s) : 1.0);
    scaled_ctx ctx = {xyz, s};
    ogrid gB, gA;
    ogrid_build(&gB, n, lab, B, pos_scaled, &ctx, reach);
    ogrid_build(&gA, n, lab, A, pos_scaled, &ctx, reach);
    double* c0 = (double*)malloc(sizeof(double) * (size_t)n_bins);
    double* cp = (double*)malloc(sizeof(double) * (size_t)n_bins);
    double* cm = (double*)malloc(sizeof(double) * (size_t)n_bins);
    for (int64_t q = 0; q < n_ions; ++q) {
        const int64_t m = ions[q];
        for (int a = 0; a < 3; ++a) fd[3 * q + a] = 0.0;
        if (!finite3(xyz + 3 * m)) continue;
        double P0[3];
        for (int a = 0; a < 3; ++a) P0[a] = pos_scaled(&ctx, m, a);
        memset(c0, 0, sizeof(double) * (size_t)n_bins);
        ion_pairs_at(&st, xyz, lab, d_bnd, A, B, d_srf, cut, &gB, &gA, &ctx, m, P0, c0);
        for (int a = 0; a < 3; ++a) {
            double P[3];
            memset(cp, 0, sizeof(double) * (size_t)n_bins);
            memset(cm, 0, sizeof(double) * (size_t)n_bins);
            for (int sg = 0; sg < 2; ++sg) {
                for (int u = 0; u < 3; ++u) P[u] = P0[u];
                const double v = (double)xyz[3 * m + a] + (sg == 0 ? step : -step);
                P[a] = a == 2 ? s * v : v;
                ion_pairs_at(&st, xyz, lab, d_bnd, A, B, d_srf, cut, &gB, &gA, &ctx, m, P, sg == 0 ? cp : cm);
            }
            double dL = 0.0;
            for (int32_t b = 0; b < n_bins; ++b) {
                const double dp = cp[b] - c0[b], dm = cm[b] - c0[b];
                dL += (dp - dm) * (2.0 * resid[b] + dp + dm);
            }
            fd[3 * q + a] = dL / (2.0 * step);
        }
    }
    free(c0);
    free(cp);
    free(cm);
    ogrid_free(&gB);
    ogrid_free(&gA);
    free((void*)st.e);
}


/* Threads the OpenMP loops of the oracle use from now on (n >= 1). */
void orc_set_threads(int32_t n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ---------------------------------------------------------------------- */
/* Two-point statistics: the 3-D histogram of displacement vectors         */
/* ---------------------------------------------------------------------- */
/* RDF and kNN integrate the more general two-point statistic over
 * directions (paper, Methods: "Descriptive, two-point spatial statistics,
 * and clustering"; its serial sections are the spatial distribution maps).
 * Here: every ordered pair (target i, neighbour j != i) within R (the RDF's
 * rule: FP64 squared distance below R*R) adds one count to the cubic voxel
 * that holds its displacement v = p_j - p_i, each component the FP64
 * difference of the stored FP32 coordinates.  n voxels per axis cover
 * [-R, R); voxel m of an axis is [f_m, f_{m+1}) with the faces
 * f_m = ((2m - n) * R) / n in FP64; the flat index is (mz * n + my) * n + mx. */

void orc_sdm_faces(float R, int32_t n, double* F) {
    for (int32_t m = 0; m <= n; ++m) F[m] = ((double)(2 * m - n) * (double)R) / (double)n;
}

/* largest m in [0, n) with F[m] <= v (v in [F[0], F[n]) for a counted pair) */
static int32_t face_bin(double v, const double* F, int32_t n) {
    int32_t lo = 0, hi = n; /* F[lo] <= v < F[hi] */
    while (hi - lo > 1) {
        int32_t mid = lo + (hi - lo) / 2;
        if (F[mid] <= v) lo = mid; else hi = mid;
    }
    return lo;
}

static int64_t sdm_index(const float* pi, const float* pj, const double* F, int32_t n) {
    int64_t m[3];
    for (int a = 0; a < 3; ++a) m[a] = face_bin((double)pj[a] - (double)pi[a], F, n);
    return (m[2] * n + m[1]) * n + m[0];
}

void orc_sdm_brute(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n, int32_t A, int32_t B,
                   float d_srf, float R, int32_t n_vox, uint64_t* hist) {
    double E2[2];
    orc_edges2(R, 1, E2);
    double* F = (double*)malloc(sizeof(double) * (size_t)(n_vox + 1));
    orc_sdm_faces(R, n_vox, F);
    memset(hist, 0, sizeof(uint64_t) * (size_t)n_vox * (size_t)n_vox * (size_t)n_vox);
    for (int64_t i = 0; i < n; ++i) {
        if (!is_target(i, lab, d_bnd, A, d_srf) || !finite3(xyz + 3 * i)) continue;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i || !is_species(lab[j], B) || !finite3(xyz + 3 * j)) continue;
            if (!(orc_D2(xyz + 3 * i, xyz + 3 * j) < E2[1])) continue;
            hist[sdm_index(xyz + 3 * i, xyz + 3 * j, F, n_vox)]++;
        }
    }
    free(F);
}

void orc_sdm_grid(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n, int32_t A, int32_t B,
                  float d_srf, float R, int32_t n_vox, uint64_t* hist) {
    double E2[2];
    orc_edges2(R, 1, E2);
    double* F = (double*)malloc(sizeof(double) * (size_t)(n_vox + 1));
    orc_sdm_faces(R, n_vox, F);
    const size_t nv = (size_t)n_vox * (size_t)n_vox * (size_t)n_vox;
    ogrid g;
    ogrid_build(&g, n, lab, B, pos_plain, xyz, (double)R * (1.0 + 1e-6));
    memset(hist, 0, sizeof(uint64_t) * nv);
    /* targets in parallel; counts are added with atomic increments (integer
     * sums: the result does not depend on the order) */
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        if (!is_target(i, lab, d_bnd, A, d_srf) || !finite3(xyz + 3 * i)) continue;
        const float* pi = xyz + 3 * i;
        int64_t c[3];
        for (int a = 0; a < 3; ++a) c[a] = ocell_axis(&g, a, (double)pi[a]);
        for (int64_t z = c[2] - 1; z <= c[2] + 1; ++z) {
            if (z < 0 || z >= g.dim[2]) continue;
            for (int64_t y = c[1] - 1; y <= c[1] + 1; ++y) {
                if (y < 0 || y >= g.dim[1]) continue;
                for (int64_t x = c[0] - 1; x <= c[0] + 1; ++x) {
                    if (x < 0 || x >= g.dim[0]) continue;
                    int64_t cell = (z * g.dim[1] + y) * g.dim[0] + x;
                    for (int64_t t = g.start[cell]; t < g.start[cell + 1]; ++t) {
                        int64_t j = g.item[t];
                        if (j == i || !(orc_D2(pi, xyz + 3 * j) < E2[1])) continue;
                        int64_t v = sdm_index(pi, xyz + 3 * j, F, n_vox);
#pragma omp atomic
                        hist[v]++;
                    }
                }
            }
        }
    }
    ogrid_free(&g);
    free(F);
}

/* ------------------------------------------------------------------------
 * Maximum-separation clustering (paper, Methods: "Descriptive, two-point
 * spatial statistics, and clustering": the MS method, a DBScan variant with
 * the two parameters d_max and N_min; Supplementary, "Efficient batch
 * processing of spatial statistics": clusters that touch the edge of the
 * dataset are flagged as truncated).
 *
 * The vertices are the ions of species A.  Two of them are linked when both
 * positions are finite and their FP64 squared distance (orc_D2) is at most
 * d_max^2.  Clusters are the connected components; a component with at
 * least n_min ions is kept.  A component is found by a breadth-first search
 * started at its smallest index (indices are scanned upwards, so every
 * smaller vertex already belongs to another component), which is therefore
 * the component's name.
 * ------------------------------------------------------------------------ */

/* outputs from comp[i] (the component's smallest index, -1 off species) */
static void ms_outputs(const int64_t* comp, const float* d_bnd, int64_t n, int32_t n_min, float d_srf,
                       int64_t* label, int64_t* counts, uint64_t* size_hist, int32_t n_size_bins) {
    int64_t* size = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    uint8_t* trunc = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
    for (int64_t i = 0; i < n; ++i) {
        if (comp[i] < 0) continue;
        size[comp[i]]++;
        /* at the edge: the distance to the edge is not at least d_srf (NaN included) */
        if (d_bnd && !(d_bnd[i] >= d_srf)) trunc[comp[i]] = 1;
    }
    counts[0] = counts[1] = counts[2] = 0;
    if (size_hist) memset(size_hist, 0, sizeof(uint64_t) * (size_t)n_size_bins);
    for (int64_t i = 0; i < n; ++i) {
        label[i] = (comp[i] >= 0 && size[comp[i]] >= n_min) ? comp[i] : -1;
        if (comp[i] != i) continue;            /* one visit per component */
        const int64_t s = size[i];
        if (size_hist) size_hist[(s < n_size_bins ? s : n_size_bins) - 1]++;
        if (s >= n_min) {
            counts[0]++;
            counts[1] += trunc[i];
            counts[2] += s;
        }
    }
    free(size);
    free(trunc);
}

void orc_cluster_ms_brute(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n, int32_t A,
                          float d_max, int32_t n_min, float d_srf, int64_t* label, int64_t* counts,
                          uint64_t* size_hist, int32_t n_size_bins) {
    const double lim = (double)d_max * (double)d_max;
    int64_t* comp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t* queue = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) comp[i] = -1;
    for (int64_t i = 0; i < n; ++i) {
        if (!is_species(lab[i], A) || comp[i] >= 0) continue;
        int64_t head = 0, tail = 0;
        comp[i] = i;
        queue[tail++] = i;
        while (head < tail) {
            const int64_t u = queue[head++];
            if (!finite3(xyz + 3 * u)) continue;
            for (int64_t j = 0; j < n; ++j) {
                if (comp[j] >= 0 || !is_species(lab[j], A) || !finite3(xyz + 3 * j)) continue;
                if (orc_D2(xyz + 3 * u, xyz + 3 * j) <= lim) {
                    comp[j] = i;
                    queue[tail++] = j;
                }
            }
        }
    }
    ms_outputs(comp, d_bnd, n, n_min, d_srf, label, counts, size_hist, n_size_bins);
    free(queue);
    free(comp);
}

/* The same search with the candidates of a vertex taken from the 27 grid
 * cells around it (cell edge at least d_max). */
void orc_cluster_ms_grid(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n, int32_t A,
                         float d_max, int32_t n_min, float d_srf, int64_t* label, int64_t* counts,
                         uint64_t* size_hist, int32_t n_size_bins) {
    const double lim = (double)d_max * (double)d_max;
    ogrid g;
    ogrid_build(&g, n, lab, A, pos_plain, xyz, (double)d_max * (1.0 + 1e-6));
    int64_t* comp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t* queue = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) comp[i] = -1;
    for (int64_t i = 0; i < n; ++i) {
        if (!is_species(lab[i], A) || comp[i] >= 0) continue;
        int64_t head = 0, tail = 0;
        comp[i] = i;
        queue[tail++] = i;
        while (head < tail) {
            const int64_t u = queue[head++];
            const float* pu = xyz + 3 * u;
            if (!finite3(pu)) continue;
            int64_t c[3];
            for (int a = 0; a < 3; ++a) c[a] = ocell_axis(&g, a, (double)pu[a]);
            for (int64_t z = c[2] - 1; z <= c[2] + 1; ++z) {
                if (z < 0 || z >= g.dim[2]) continue;
                for (int64_t y = c[1] - 1; y <= c[1] + 1; ++y) {
                    if (y < 0 || y >= g.dim[1]) continue;
                    for (int64_t x = c[0] - 1; x <= c[0] + 1; ++x) {
                        if (x < 0 || x >= g.dim[0]) continue;
                        const int64_t cell = (z * g.dim[1] + y) * g.dim[0] + x;
                        for (int64_t t = g.start[cell]; t < g.start[cell + 1]; ++t) {
                            const int64_t j = g.item[t];
                            if (comp[j] >= 0 || orc_D2(pu, xyz + 3 * j) > lim) continue;
                            comp[j] = i;
                            queue[tail++] = j;
                        }
                    }
                }
            }
        }
    }
    ms_outputs(comp, d_bnd, n, n_min, d_srf, label, counts, size_hist, n_size_bins);
    ogrid_free(&g);
    free(queue);
    free(comp);
}

/* ------------------------------------------------------------------------
 * Ion-to-edge distancing (paper, Methods: "Ion-to-edge distancing";
 * Supplementary: "Triangle filtering methods for ion-to-edge distancing";
 * the benchmark table's "Surfacing" task with its probe distance d_prb).
 *
 * The distance of a point to a closed triangle is the smallest distance to
 * any point of it: the distance to the triangle's plane when the foot of the
 * perpendicular lies inside the triangle, else the smallest distance to its
 * three edges.  A triangle of zero area is its edges.  Arithmetic in FP64 on
 * the stored FP32 values.  d[i] is the smallest distance over the triangles,
 * rounded to FP32, when it is below d_prb, else +inf; NaN for an ion with a
 * non-finite position.  Triangles with a non-finite vertex are left out.
 * ------------------------------------------------------------------------ */
static void v3sub(const double* a, const double* b, double* r) {
    r[0] = a[0] - b[0];
    r[1] = a[1] - b[1];
    r[2] = a[2] - b[2];
}
static double v3dot(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void v3cross(const double* a, const double* b, double* r) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

/* squared distance of p to the segment [a, b] */
static double seg_d2(const double* p, const double* a, const double* b) {
    double ab[3], ap[3], q[3], pq[3];
    v3sub(b, a, ab);
    v3sub(p, a, ap);
    const double L = v3dot(ab, ab);
    double t = L > 0 ? v3dot(ap, ab) / L : 0.0;
    if (t < 0) t = 0;
    if (t > 1) t = 1;
    for (int k = 0; k < 3; ++k) q[k] = a[k] + t * ab[k];
    v3sub(p, q, pq);
    return v3dot(pq, pq);
}

/* squared distance of p to the closed triangle (v0, v1, v2) */
static double tri_d2(const double* p, const double* v0, const double* v1, const double* v2) {
    double best = seg_d2(p, v0, v1);
    double s = seg_d2(p, v1, v2);
    if (s < best) best = s;
    s = seg_d2(p, v2, v0);
    if (s < best) best = s;
    double e1[3], e2[3], nrm[3], w[3];
    v3sub(v1, v0, e1);
    v3sub(v2, v0, e2);
    v3cross(e1, e2, nrm);
    const double nn = v3dot(nrm, nrm);
    if (nn > 0) {
        v3sub(p, v0, w);
        const double h = v3dot(w, nrm);
        double f[3];
        for (int k = 0; k < 3; ++k) f[k] = p[k] - (h / nn) * nrm[k];   /* foot of the perpendicular */
        /* inside: on the inner side of all three edges */
        const double* V[3] = {v0, v1, v2};
        int inside = 1;
        for (int e = 0; e < 3; ++e) {
            double ed[3], fv[3], c[3];
            v3sub(V[(e + 1) % 3], V[e], ed);
            v3sub(f, V[e], fv);
            v3cross(ed, fv, c);
            if (v3dot(c, nrm) < 0) inside = 0;
        }
        if (inside) {
            const double h2 = h * h / nn;
            if (h2 < best) best = h2;
        }
    }
    return best;
}

static int tri_finite(const float* t) {
    for (int k = 0; k < 9; ++k)
        if (!isfinite(t[k])) return 0;
    return 1;
}

static float edge_result(const float* p, double best2, float d_prb) {
    if (!finite3(p)) return NAN;
    const double d = sqrt(best2);
    return d < (double)d_prb ? (float)d : INFINITY;
}

void orc_edge_brute(const float* xyz, int64_t n, const float* tri, int64_t n_tri, float d_prb, float* d) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        const double p[3] = {xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]};
        double best2 = INFINITY;
        for (int64_t t = 0; t < n_tri; ++t) {
            const float* T = tri + 9 * t;
            if (!tri_finite(T)) continue;
            const double v0[3] = {T[0], T[1], T[2]}, v1[3] = {T[3], T[4], T[5]}, v2[3] = {T[6], T[7], T[8]};
            const double s = tri_d2(p, v0, v1, v2);
            if (s < best2) best2 = s;
        }
        d[i] = edge_result(xyz + 3 * i, best2, d_prb);
    }
}

/* The same with the triangles binned into cubic cells of edge >= d_prb
 * (each in every cell its bounding box meets): only the triangles of the
 * cells that the cube [p - d_prb, p + d_prb] meets can lie within d_prb.
 * d_prb must be finite. */
typedef struct {
    double lo[3];
    double h;
    int64_t dim[3];
} tgrid;

/* cells [c0, c1] of the interval [x0, x1] on axis a, clamped to the grid;
 * 0 when the interval misses the grid */
static int tgrid_range(const tgrid* g, int a, double x0, double x1, int64_t* c0, int64_t* c1) {
    const double f0 = floor((x0 - g->lo[a]) / g->h), f1 = floor((x1 - g->lo[a]) / g->h);
    if (f1 < 0 || f0 > (double)(g->dim[a] - 1)) return 0;
    *c0 = f0 < 0 ? 0 : (int64_t)f0;
    *c1 = f1 > (double)(g->dim[a] - 1) ? g->dim[a] - 1 : (int64_t)f1;
    return 1;
}

/* the cell box of a triangle's vertices; 0 when it misses the grid */
static int tri_cells(const tgrid* g, const float* T, int64_t c0[3], int64_t c1[3]) {
    for (int a = 0; a < 3; ++a) {
        const double x0 = fmin(fmin(T[a], T[3 + a]), T[6 + a]), x1 = fmax(fmax(T[a], T[3 + a]), T[6 + a]);
        if (!tgrid_range(g, a, x0, x1, &c0[a], &c1[a])) return 0;
    }
    return 1;
}

void orc_edge_grid(const float* xyz, int64_t n, const float* tri, int64_t n_tri, float d_prb, float* d) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int64_t nv = 0;
    for (int64_t t = 0; t < n_tri; ++t) {
        if (!tri_finite(tri + 9 * t)) continue;
        ++nv;
        for (int k = 0; k < 9; ++k) {
            const double v = tri[9 * t + k];
            if (v < lo[k % 3]) lo[k % 3] = v;
            if (v > hi[k % 3]) hi[k % 3] = v;
        }
    }
    if (nv == 0) {
        for (int64_t i = 0; i < n; ++i) d[i] = edge_result(xyz + 3 * i, INFINITY, d_prb);
        return;
    }
    tgrid g;
    g.h = (double)d_prb;
    for (;;) {   /* bounded table: at most ~8 cells per triangle */
        double cells = 1;
        for (int a = 0; a < 3; ++a) cells *= floor((hi[a] - lo[a]) / g.h) + 1;
        if (cells <= 8.0 * (double)nv + 64.0) break;
        g.h *= 1.5;
    }
    int64_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = lo[a];
        g.dim[a] = (int64_t)floor((hi[a] - lo[a]) / g.h) + 1;
        ncell *= g.dim[a];
    }
    int64_t* start = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t c0[3], c1[3];
    for (int64_t t = 0; t < n_tri; ++t) {                    /* count */
        if (!tri_finite(tri + 9 * t) || !tri_cells(&g, tri + 9 * t, c0, c1)) continue;
        for (int64_t z = c0[2]; z <= c1[2]; ++z)
            for (int64_t y = c0[1]; y <= c1[1]; ++y)
                for (int64_t x = c0[0]; x <= c1[0]; ++x) start[(z * g.dim[1] + y) * g.dim[0] + x + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
    int64_t* item = (int64_t*)malloc(sizeof(int64_t) * (size_t)(start[ncell] > 0 ? start[ncell] : 1));
    int64_t* fill = (int64_t*)calloc((size_t)ncell, sizeof(int64_t));
    for (int64_t t = 0; t < n_tri; ++t) {                    /* fill */
        if (!tri_finite(tri + 9 * t) || !tri_cells(&g, tri + 9 * t, c0, c1)) continue;
        for (int64_t z = c0[2]; z <= c1[2]; ++z)
            for (int64_t y = c0[1]; y <= c1[1]; ++y)
                for (int64_t x = c0[0]; x <= c1[0]; ++x) {
                    const int64_t c = (z * g.dim[1] + y) * g.dim[0] + x;
                    item[start[c] + fill[c]++] = t;
                }
    }
    free(fill);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        const float* pi = xyz + 3 * i;
        double best2 = INFINITY;
        int64_t q0[3], q1[3];
        int ok = finite3(pi);
        for (int a = 0; ok && a < 3; ++a)
            ok = tgrid_range(&g, a, (double)pi[a] - (double)d_prb, (double)pi[a] + (double)d_prb, &q0[a], &q1[a]);
        if (ok) {
            const double p[3] = {pi[0], pi[1], pi[2]};
            for (int64_t z = q0[2]; z <= q1[2]; ++z)
                for (int64_t y = q0[1]; y <= q1[1]; ++y)
                    for (int64_t x = q0[0]; x <= q1[0]; ++x) {
                        const int64_t c = (z * g.dim[1] + y) * g.dim[0] + x;
                        for (int64_t k = start[c]; k < start[c + 1]; ++k) {
                            const float* T = tri + 9 * item[k];
                            const double v0[3] = {T[0], T[1], T[2]}, v1[3] = {T[3], T[4], T[5]},
                                         v2[3] = {T[6], T[7], T[8]};
                            const double s = tri_d2(p, v0, v1, v2);
                            if (s < best2) best2 = s;
                        }
                    }
        }
        d[i] = edge_result(pi, best2, d_prb);
    }
    free(item);
    free(start);
}
