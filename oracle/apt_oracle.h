/*
 * apt_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU reference for the spatial-statistics path (kNN and RDF
 * of target ions against neighbour ions, the label-randomised null model, a
 * Gaussian-smoothed RDF with its gradient, the two-point statistic, the
 * maximum-separation clustering and the ion-to-edge distancing).  Only the test-suite, the
 * smoke check and the benchmark's CPU baseline may call it; the GPU library
 * never includes, links or calls anything here, and this file shares no code
 * with it.  All pointers are host pointers.  Species 255 means "any species".
 */
#ifndef APT_ORACLE_H
#define APT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_ANY 255

/* Number of OpenMP threads the oracle's loops use. */
int32_t orc_threads(void);
void orc_set_threads(int32_t n);
void orc_sdm_faces(float R, int32_t n, double* F);
void orc_sdm_brute(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n, int32_t A, int32_t B,
                   float d_srf, float R, int32_t n_vox, uint64_t* hist);
void orc_sdm_grid(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n, int32_t A, int32_t B,
                  float d_srf, float R, int32_t n_vox, uint64_t* hist);

/* Maximum-separation clustering of the ions of species A: links at FP64
 * squared distance <= d_max^2, components of at least n_min ions kept.
 * label[n]: the smallest ion index of the ion's kept cluster, else -1;
 * counts[3]: kept clusters, kept clusters with an ion whose d_bnd is not
 * >= d_srf (0 without d_bnd), ions in kept clusters; size_hist[n_size_bins]
 * (may be NULL): every component by its size s, in bin min(s, n_size_bins)-1. */
void orc_cluster_ms_brute(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n, int32_t A,
                          float d_max, int32_t n_min, float d_srf, int64_t* label, int64_t* counts,
                          uint64_t* size_hist, int32_t n_size_bins);
void orc_cluster_ms_grid(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n, int32_t A,
                         float d_max, int32_t n_min, float d_srf, int64_t* label, int64_t* counts,
                         uint64_t* size_hist, int32_t n_size_bins);

/* Ion-to-edge distancing: d[i] = the FP64 distance of ion i to the closest
 * point of the closed triangles tri[n_tri][3][3], rounded to FP32, when
 * below d_prb, else +inf; NaN for a non-finite position; triangles with a
 * non-finite vertex are left out.  The grid form needs a finite d_prb. */
void orc_edge_brute(const float* xyz, int64_t n, const float* tri, int64_t n_tri, float d_prb, float* d);
void orc_edge_grid(const float* xyz, int64_t n, const float* tri, int64_t n_tri, float d_prb, float* d);

/* Canonical distances between two stored FP32 positions. */
float orc_d2f(const float* a, const float* b);   /* FP32, fixed evaluation order */
double orc_D2(const float* a, const float* b);   /* FP64, no fused operations   */

/* Squared bin edges E2[b] = e_b^2 with e_b = b * r_max / n_bins, b = 0..n_bins. */
void orc_edges2(float r_max, int32_t n_bins, double* E2);
/* b with E2[b] <= D2 < E2[b+1]; n_bins when D2 >= E2[n_bins]. */
int32_t orc_bin_of(double D2, const double* E2, int32_t n_bins);

/* Eligible targets in ascending index order; returns their count. */
int64_t orc_select_targets(int64_t n, const uint8_t* lab, const float* d_bnd, int32_t A,
                           float d_srf, int64_t* out_ids);

/* RDF: ordered-pair counts hist[n_bins] (overwritten). */
void orc_rdf_brute(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n, int32_t A,
                   int32_t B, float d_srf, float r_max, int32_t n_bins, uint64_t* hist);
void orc_rdf_grid(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n, int32_t A,
                  int32_t B, float d_srf, float r_max, int32_t n_bins, uint64_t* hist);

/* kNN: rows for the eligible targets in ascending index order.
 * target_id[T], dist[T][k] (+inf pad), nbr_id[T][k] (-1 pad).  knn_hist
 * (may be NULL) gets [kb_nbins + 1] counts of the k-th neighbour distance,
 * the last slot holding targets with no k-th neighbour inside the range.
 * Returns T.  r_knn_max = +inf for an unbounded search. */
int64_t orc_knn_brute(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n,
                      int32_t A, int32_t B, float d_srf, int32_t k, float r_knn_max,
                      int64_t* target_id, float* dist, int64_t* nbr_id, float kb_rmax,
                      int32_t kb_nbins, uint64_t* knn_hist);
int64_t orc_knn_grid(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n,
                     int32_t A, int32_t B, float d_srf, int32_t k, float r_knn_max,
                     int64_t* target_id, float* dist, int64_t* nbr_id, float kb_rmax,
                     int32_t kb_nbins, uint64_t* knn_hist);

/* Label randomisation: i-th SplitMix64 output for a seed, and the permuted labels. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t i);
void orc_permute_labels(const uint8_t* lab, int64_t n, uint64_t seed, uint8_t* out);

/* Gaussian-smoothed RDF (FP64) and its adjoint, coordinates (x, y, s*z). */
void orc_smooth_fwd(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n,
                    int32_t A, int32_t B, float d_srf, float r_max, int32_t n_bins, float sigma,
                    double s, double* h);
void orc_smooth_bwd(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n,
                    int32_t A, int32_t B, float d_srf, float r_max, int32_t n_bins, float sigma,
                    double s, const double* grad_h, double* grad_xyz, double* grad_s);
/* Central finite differences of L = sum_b (h_b - t_b)^2 (resid = h - t) with
 * respect to the coordinates of ions[0..n_ions), from the pairs each ion
 * takes part in; fd[n_ions][3]. */
void orc_smooth_fd(const float* xyz, const uint8_t* lab, const float* d_bnd, int64_t n, int32_t A, int32_t B,
                   float d_srf, float r_max, int32_t n_bins, float sigma, double s, const double* resid,
                   const int64_t* ions, int64_t n_ions, double step, double* fd);

#ifdef __cplusplus
}
#endif
#endif
