/*
 * apt_stat.h -- C ABI of the GPU spatial-statistics library (libaptstat.so).
 *
 * For every target ("central") ion of species A lying at least d_srf from
 * the specimen surface, the library computes the k nearest neighbours of
 * species B (distances and identities) and the radial-distribution pair
 * counts to B ions within r_max (paper, Methods: "Descriptive, two-point
 * spatial statistics, and clustering" and "Ion-to-edge distancing";
 * Supplementary: "Customized user defined batch processing queues").  Two
 * further forms sit beside it: label-randomised null replicates of many
 * species pairs in one launch (Supplementary: "Importance of high quality
 * random number generators"; Methods: "User-defined batch processing
 * queues"), and a Gaussian-smoothed RDF with its adjoint (an extension: not
 * in the paper).
 *
 * Conventions shared by every entry point
 *  - All data pointers are DEVICE pointers unless stated otherwise; the caller
 *    owns every input, output and workspace buffer.  The library never
 *    allocates device memory inside a call.
 *  - Calls are asynchronous on `stream` (a hipStream_t passed as void*,
 *    NULL = the null stream) and return as soon as the work is enqueued.
 *  - Outputs are overwritten, never accumulated.  Integer outputs are
 *    deterministic.
 *  - Host-detectable errors are returned immediately (before any GPU work)
 *    as an apt_status; apt_last_error() then gives a text.  Data-dependent
 *    errors are OR-ed into the device status word `*status` (int32, cleared
 *    by the call): APT_STATUS_NONFINITE, APT_STATUS_CAPACITY.
 *  - Positions: xyz[n][3] FP32 in nm, C-contiguous.  Labels: uint8, species
 *    0..254; APT_ANY (255) as a query species means "any species".
 *    d_bnd[n] FP32 distance to the specimen surface (nm), or NULL for no
 *    surface filter.  n < 2^32.
 *  - Target eligibility: lab[i] == A (or A == APT_ANY) and
 *    (d_bnd == NULL or d_bnd[i] >= d_srf); NaN is never eligible.
 *    Neighbours: lab[j] == B (or B == APT_ANY), j != i; neighbours are not
 *    filtered by d_bnd.
 *  - Distances: the RDF bin of a pair is decided on the FP64 squared distance
 *    ((dx*dx + dy*dy) + dz*dz) of the two stored FP32 positions (differences
 *    taken in FP64); the kNN order is the FP32 squared distance
 *    fmaf(dz,dz,fmaf(dy,dy,dx*dx)) with the neighbour index as tie-break.
 *  - Bins: [e_b, e_{b+1}) with e_b = b * r_max / n_bins (FP64), b < n_bins;
 *    a pair counts iff its distance is below r_max.  Counts are of ORDERED
 *    pairs (an A->A histogram counts each unordered pair twice).
 *  - uint64 outputs may be backed by int64 tensors (counts < 2^63).
 *  - A call may be issued from several host threads at once on different
 *    streams with different workspaces; calls that share a workspace must be
 *    ordered by the caller.
 */
#ifndef APT_STAT_H
#define APT_STAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    APT_OK = 0,
    APT_E_ARG = -1,          /* invalid argument                                   */
    APT_E_WORKSPACE = -2,    /* workspace NULL or smaller than apt_workspace_size  */
    APT_E_UNSUPPORTED = -3,  /* valid but outside the supported range              */
    APT_E_HIP = -4           /* a HIP runtime call or launch failed                */
} apt_status;

#define APT_ANY 255
#define APT_STATUS_NONFINITE 1 /* a target or neighbour of the call had a NaN or infinite coordinate
                                  (such ions take part in no pair) */
#define APT_STATUS_CAPACITY 2  /* more eligible targets than the kNN row capacity */

#define APT_MAX_BINS 65536     /* largest n_bins of any histogram */
#define APT_MAX_K 256          /* largest k */

typedef struct {
    const float* xyz;     /* [n][3] FP32, device                                 */
    const uint8_t* lab;   /* [n] species labels, device                          */
    const float* d_bnd;   /* [n] distance to the surface (nm), device, or NULL   */
    int64_t n;            /* number of ions, 0 <= n < 2^32                       */
} apt_cloud;

typedef struct {
    uint8_t target;       /* species A of the central ions (or APT_ANY)          */
    uint8_t neighbor;     /* species B of the neighbours (or APT_ANY)            */
    uint8_t pad[2];
    float d_srf;          /* minimum distance of a target to the surface (nm)    */
} apt_query;

typedef struct {
    float r_max;          /* upper edge of the last bin (nm), > 0, finite         */
    int32_t n_bins;       /* 1 <= n_bins <= APT_MAX_BINS                          */
} apt_bins;

/* Operation codes for apt_workspace_size. */
enum {
    APT_OP_RDF = 1,       /* apt_rdf                               */
    APT_OP_KNN = 2,       /* apt_knn                               */
    APT_OP_KNN_RDF = 3,   /* apt_knn_rdf                           */
    APT_OP_PERMUTE = 4,   /* apt_permute_labels                    */
    APT_OP_BATCHED = 5,   /* apt_rdf_batched (n_pairs, n_rep used) */
    APT_OP_SMOOTH = 6,    /* apt_rdf_smooth_fwd / _bwd             */
    APT_OP_SDM = 7,       /* apt_sdm                               */
    APT_OP_CLUSTER = 8    /* apt_cluster_ms                        */
};

/* Bytes of device workspace an operation needs for n ions (host only, no
 * GPU call).  Returns 0 for an unknown op or out-of-range sizes.  The
 * workspace must be 256-byte aligned (any hipMalloc / torch allocation is). */
size_t apt_workspace_size(int32_t op, int64_t n, int32_t n_pairs, int32_t n_rep);

/* RDF of one query (paper, Methods: "Descriptive, two-point spatial
 * statistics"; bins of a rectangular transfer function).
 *   hist[bins.n_bins] (uint64, device): ordered-pair counts, overwritten. */
apt_status apt_rdf(const apt_cloud* cloud, apt_query q, apt_bins bins, uint64_t* hist,
                   int32_t* status, void* ws, size_t ws_bytes, void* stream);

/* apt_rdf without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the call's scratch is a static device
 * array of 128 MiB (APT_NOALLOC_SCRATCH_BYTES) that each GPU the library runs
 * on holds from the library's load until the process ends.  Arguments,
 * results and errors as apt_rdf; clouds whose apt_rdf workspace exceeds the
 * array (about 1.5 million ions) return APT_E_UNSUPPORTED before any GPU
 * work.  The call allocates nothing (no hipMalloc, hipFree or allocating
 * library routine).  Every call on one GPU shares that GPU's array and
 * leaves its contents behind: calls that overlap on one GPU (concurrent
 * streams or host threads) race and must be ordered by the caller. */
#define APT_NOALLOC_SCRATCH_BYTES (128u << 20)
apt_status apt_rdf_noalloc(const apt_cloud* cloud, apt_query q, apt_bins bins, uint64_t* hist,
                           int32_t* status, void* stream);

/* kNN of one query (paper, Methods: kNN as the distribution of distances to
 * the k-th nearest neighbour of a given type).  Rows are for the eligible
 * targets in ascending ion index; the search radius is unbounded unless
 * r_knn_max is finite (neighbours with FP32 squared distance above
 * r_knn_max*r_knn_max are ignored).
 *   capacity           rows the output arrays hold (>= 0)
 *   target_id[cap]     int64 ion index of each row (ascending)
 *   dist[cap][k]       FP32 distances, ascending, +inf padding
 *   nbr_id[cap][k]     int64 neighbour indices, -1 padding
 *   knn_bins, knn_hist optional (knn_hist may be NULL): [knn_bins.n_bins + 1]
 *                      uint64 counts of targets per bin of their k-th
 *                      neighbour distance; the last slot counts targets
 *                      whose k-th neighbour is missing or >= knn_bins.r_max
 *   n_targets[1]       int64, device: number of eligible targets.  Rows
 *                      beyond `capacity` are dropped and APT_STATUS_CAPACITY
 *                      is set. */
apt_status apt_knn(const apt_cloud* cloud, apt_query q, int32_t k, float r_knn_max,
                   int64_t capacity, int64_t* target_id, float* dist, int64_t* nbr_id,
                   apt_bins knn_bins, uint64_t* knn_hist, int64_t* n_targets, int32_t* status,
                   void* ws, size_t ws_bytes, void* stream);

/* kNN and RDF of one query from a single neighbour enumeration (the paper's
 * batch queue evaluates several statistics per region of interest rather
 * than querying again: Supplementary, "Customized user defined batch
 * processing queues").  Arguments as apt_rdf and apt_knn; rdf_hist may not
 * be NULL. */
apt_status apt_knn_rdf(const apt_cloud* cloud, apt_query q, apt_bins rdf_bins, uint64_t* rdf_hist,
                       int32_t k, float r_knn_max, int64_t capacity, int64_t* target_id,
                       float* dist, int64_t* nbr_id, apt_bins knn_bins, uint64_t* knn_hist,
                       int64_t* n_targets, int32_t* status, void* ws, size_t ws_bytes,
                       void* stream);

/* Null model: out[i] = lab[pi(i)], pi = the ascending order of the keys
 * key(i) = i-th output (i = 0, 1, ...) of SplitMix64 started from state
 * `seed` (ties by index) -- a uniform random permutation of the labels
 * (paper, Suppl.: "Importance of high quality random number generators";
 * the paper's Mersenne-Twister stream is replaced by this counter-based
 * definition).  lab, out: [n] uint8, device, may not alias.  Workspace:
 * APT_OP_PERMUTE.  The same permutation defines the replicates of
 * apt_rdf_batched (seed of replicate r = seeds[r]). */
apt_status apt_permute_labels(const uint8_t* lab, int64_t n, uint64_t seed, uint8_t* out, int32_t* status,
                              void* ws, size_t ws_bytes, void* stream);

/* Speed knobs of apt_rdf_batched (results do not depend on them):
 *   cell_frac   grid cell edge as a fraction of rdf_bins.r_max, in (0, 4]
 *               (0 selects the default 0.5)
 *   rep_block   replicates permuted and evaluated per block, 1..64 (0 selects
 *               64; the workspace for n_rep may cap it lower)
 *   tile_reach  certified kNN reach of the 64-target tiles, as a multiple of
 *               the Poisson mean k-th neighbour distance, in [1, 4] (0 selects
 *               the default 1.3)
 *   tiles       0 automatic, 1 never use 64-target tiles */
typedef struct {
    float cell_frac;
    int32_t rep_block;
    float tile_reach;
    int32_t tiles;
} apt_batched_tuning;

/* Null-model replicates of several species pairs in one call (paper, Suppl.:
 * every statistic for randomised labels; Methods: "User-defined batch
 * processing queues").  For replicate r (0 <= r < n_rep) the labels are
 * apt_permute_labels(lab, seeds[r]); the outputs of (r, p) are DEFINED as
 * apt_knn_rdf's rdf_hist and knn_hist for query pairs[p] on those labels:
 *   pairs[n_pairs]   host array; concrete species (no APT_ANY), at most 16
 *                    pairs and 7 distinct species; each with its own d_srf
 *   seeds[n_rep]     host array
 *   rdf_hist         [n_rep][n_pairs][rdf_bins.n_bins] uint64 (n_bins <= 3072)
 *   knn_hist         [n_rep][n_pairs][knn_bins.n_bins + 1] uint64, or NULL;
 *                    k-th neighbour distance of every eligible target
 *   tuning           host pointer to an apt_batched_tuning, or NULL: the plan
 *                    is looked up in a process-wide cache keyed by the device,
 *                    n, the pairs, the bins and k; on a miss it is autotuned
 *                    first (timed trial launches of a few replicates on this
 *                    stream, which wait for the GPU; skipped, with the
 *                    defaults, while the stream is being captured), then
 *                    cached.  With NULL the launch sequence is also captured
 *                    once into a HIP graph, cached per call signature
 *                    (pointers, sizes, seeds), and replayed on later calls
 *                    with the same signature (not while the stream is being
 *                    captured or tracing is on)
 * Positions are binned once; replicates run in blocks of up to 64.
 * Workspace: apt_workspace_size(APT_OP_BATCHED, n, n_pairs, n_rep). */
apt_status apt_rdf_batched(const apt_cloud* cloud, const apt_query* pairs, int32_t n_pairs, const uint64_t* seeds,
                           int32_t n_rep, apt_bins rdf_bins, int32_t k, apt_bins knn_bins, uint64_t* rdf_hist,
                           uint64_t* knn_hist, const apt_batched_tuning* tuning, int32_t* status, void* ws,
                           size_t ws_bytes, void* stream);

/* The plan apt_rdf_batched(tuning = NULL) uses for these arguments
 * (want_knn_hist: whether knn_hist is non-NULL), if cached (host only, no
 * GPU work): *cached = 1 and *out filled (rep_block 0: as many as the
 * workspace holds), or *cached = 0.  apt_batched_plan_clear empties the plan
 * and graph caches (a later call tunes again). */
apt_status apt_batched_plan(const apt_cloud* cloud, const apt_query* pairs, int32_t n_pairs, apt_bins rdf_bins,
                            int32_t k, apt_bins knn_bins, int32_t want_knn_hist, apt_batched_tuning* out,
                            int32_t* cached);
apt_status apt_batched_plan_clear(void);

/* Two-point statistic of one query (paper, Methods: "Descriptive, two-point
 * spatial statistics, and clustering": the RDF and kNN integrate it over
 * directions; its sections through the target's plane are the spatial
 * distribution maps, computed in the paper with R = 2 nm and voxels of
 * 0.025 nm).  Every ordered pair (eligible target i, neighbour j != i)
 * within R (FP64 squared distance below R*R, the RDF's rule) adds one count
 * to the cubic voxel of its displacement v = p_j - p_i, each component the
 * FP64 difference of the stored FP32 coordinates.  n_vox voxels per axis
 * cover [-R, R): voxel m of an axis is [f_m, f_{m+1}), f_m = ((2m - n_vox)
 * R) / n_vox in FP64.
 *   R        ROI radius (nm), finite, > 0
 *   n_vox    voxels per axis, 1..512 (R = 2 nm with 0.025 nm voxels: 160)
 *   hist     [n_vox][n_vox][n_vox] uint64, device, overwritten; element
 *            (mz, my, mx), x fastest
 * Workspace: APT_OP_SDM. */
apt_status apt_sdm(const apt_cloud* cloud, apt_query q, float R, int32_t n_vox, uint64_t* hist, int32_t* status,
                   void* ws, size_t ws_bytes, void* stream);

/* Ion-to-edge distancing (paper, Methods: "Ion-to-edge distancing";
 * Supplementary: "Triangle filtering methods for ion-to-edge distancing";
 * its benchmark's "Surfacing" task with the probe distance d_prb).  For
 * every ion, the distance to the closest point of a given triangle hull
 * (closed triangles; a zero-area triangle is its edges), computed in FP64
 * on the stored FP32 values and rounded to FP32, when it is below d_prb;
 * +inf otherwise.  The result serves as cloud->d_bnd of the other calls
 * (an ion is a target when d >= d_srf: every ion at +inf is one for
 * d_srf <= d_prb).
 *   cloud        xyz and lab are read (lab only to bin the ions; any
 *                values); d_bnd is not
 *   tri          [n_tri][3][3] FP32, device: the vertices; triangles with a
 *                non-finite vertex are left out and set APT_STATUS_NONFINITE
 *   d_prb        > 0; +inf: exact for every ion (the search then spans the
 *                whole depth of the cloud: for large clouds give the largest
 *                distance that matters, e.g. the largest d_srf to be used)
 *   d            [n] FP32, device, overwritten; NaN for an ion with a
 *                non-finite position (APT_STATUS_NONFINITE)
 * Workspace: apt_edge_workspace_size(n, n_tri) bytes. */
size_t apt_edge_workspace_size(int64_t n, int64_t n_tri);
apt_status apt_edge_distance(const apt_cloud* cloud, const float* tri, int64_t n_tri, float d_prb, float* d,
                             int32_t* status, void* ws, size_t ws_bytes, void* stream);

/* Maximum-separation clustering (paper, Methods: "Descriptive, two-point
 * spatial statistics, and clustering": the MS method with its parameters
 * d_max and N_min; Supplementary, "Efficient batch processing of spatial
 * statistics": clusters that touch the dataset edge are flagged as
 * truncated).  The ions of `species` (APT_ANY: every ion) are the vertices;
 * two of them are linked when both positions are finite and their FP64
 * squared distance (differences of the stored FP32 coordinates) is at most
 * d_max^2.  Clusters are the connected components; those of at least n_min
 * ions are kept.  A cluster is named by its smallest ion index.
 *   d_max        > 0, finite (nm)
 *   n_min        >= 1
 *   d_srf        an ion whose cloud->d_bnd is not >= d_srf (NaN included)
 *                lies at the edge; not NaN; unused when cloud->d_bnd is NULL
 *   label        [n] int64, device, overwritten: for an ion of a kept
 *                cluster the smallest ion index of that cluster, else -1
 *   counts       [3] int64, device, overwritten: kept clusters, kept clusters
 *                with an ion at the edge (0 without d_bnd), ions in kept
 *                clusters
 *   size_hist    [n_size_bins] uint64, device, overwritten, or NULL: every
 *                cluster (kept or not) by its ion count s, in bin
 *                min(s, n_size_bins) - 1 (so any N_min's count follows)
 *   n_size_bins  1..65536 when size_hist is given
 * An ion of the species with a non-finite position is a cluster of its own
 * and sets APT_STATUS_NONFINITE.  Clouds of 2^31 ions or more return
 * APT_E_UNSUPPORTED.  Labels and counts do not depend on the order in which
 * the GPU links pairs.
 * Workspace: APT_OP_CLUSTER. */
apt_status apt_cluster_ms(const apt_cloud* cloud, uint8_t species, float d_max, int32_t n_min, float d_srf,
                          int64_t* label, int64_t* counts, uint64_t* size_hist, int32_t n_size_bins,
                          int32_t* status, void* ws, size_t ws_bytes, void* stream);

/* Gaussian-smoothed RDF, an extension (not in the paper) of the RDF's
 * rectangular transfer function (paper, Methods: "Descriptive, two-point
 * spatial statistics") that is differentiable in the positions and in a
 * scale factor s of the z axis (the reconstruction parameter to fit).
 * Positions are taken as (x, y, s*z); d_bnd is not rescaled.  Every ordered
 * pair (eligible target i of species A, neighbour j != i of species B) at
 * FP64 distance D < r_max + 6 sigma adds to each bin b whose interval meets
 * (D - 6 sigma, D + 6 sigma) the Gaussian mass
 *   w_b(D) = Phi((e_{b+1} - D) / sigma) - Phi((e_b - D) / sigma),
 * with e_b = b * r_max / n_bins and Phi the standard normal distribution
 * function (evaluated from the tail that does not cancel).
 *   sigma        > 0, at most (1020 bin widths) / 12
 *   z_scale      device double [1] (s), or NULL for s = 1
 *   h            [bins.n_bins] FP64, device, overwritten
 * bins.n_bins <= 4096.  Arithmetic after an FP32 culling test is FP64; the
 * result is reproducible bit for bit.  Targets and neighbours with a
 * non-finite (scaled) position take part in no pair and set
 * APT_STATUS_NONFINITE.
 * Workspace: APT_OP_SMOOTH. */
apt_status apt_rdf_smooth_fwd(const apt_cloud* cloud, apt_query q, apt_bins bins, float sigma, const double* z_scale,
                              double* h, int32_t* status, void* ws, size_t ws_bytes, void* stream);

/* Adjoint of apt_rdf_smooth_fwd: given grad_h = dL/dh [bins.n_bins] (FP64,
 * device), writes
 *   grad_xyz     [n][3] FP32, device, overwritten: dL/d(x, y, z) of every
 *                ion (0 for ions in no pair); accumulated in FP64
 *   grad_z_scale device double [1], dL/ds, or NULL to skip
 * with g = sum_b grad_h[b] dw_b/dD for each pair; a pair at D = 0 adds
 * nothing.  Pair lists are recomputed, not stored; each ion gathers its own
 * gradient over its pairs in both roles (no atomics), so the result is
 * reproducible bit for bit.  Arguments otherwise as the forward. */
apt_status apt_rdf_smooth_bwd(const apt_cloud* cloud, apt_query q, apt_bins bins, float sigma, const double* z_scale,
                              const double* grad_h, float* grad_xyz, double* grad_z_scale, int32_t* status, void* ws,
                              size_t ws_bytes, void* stream);

/* Number of eligible targets of a query, for sizing kNN outputs:
 * n_targets[1] (int64, device) is overwritten.  Workspace as APT_OP_KNN. */
apt_status apt_count_targets(const apt_cloud* cloud, apt_query q, int64_t* n_targets, void* ws,
                             size_t ws_bytes, void* stream);

/* Diagnostic, not part of any statistic: bins the cloud exactly as
 * apt_knn_rdf(q, bins, k, ...) would (k = 0: as apt_rdf), then sets
 * candidates[0] (uint64, device; overwritten) to the number of pair
 * evaluations of the kernel that counts the RDF: for the one-target-per-
 * wavefront pair kernel, the neighbour records its first enumeration visits,
 * summed over the eligible targets (the cell rows within bins.r_max, or
 * within the first kNN radius when k > 0 and that is larger, each row
 * trimmed to the x-range the sphere reaches); for the neighbour-major kernel
 * (dense neighbours), the records of each 64-record run times the targets
 * staged for it.  Divided by the in-range pair
 * count it gives the culling ratio of the grid (paper, Supplementary,
 * "Effectiveness of the spatial splitting").  Errors as
 * apt_knn_rdf; k < 0 or candidates NULL return APT_E_ARG.  Workspace as
 * APT_OP_KNN_RDF. */
apt_status apt_count_candidates(const apt_cloud* cloud, apt_query q, apt_bins bins, int32_t k,
                                uint64_t* candidates, int32_t* status, void* ws, size_t ws_bytes, void* stream);

/* Process-wide tuning of the plain entry points (host only; results do not
 * depend on it, only speed):
 *   tile_policy  0 automatic, 1 one target per wavefront, 2 64 targets per
 *                wavefront with LDS-staged neighbours and a register kNN list,
 *                3 one target per lane, each lane walking its own cells with a
 *                register kNN list, 4 the kNN one target per lane (register
 *                list within a certified radius) and the RDF one target per
 *                wavefront (2, 3 and 4 only when k <= 16 and n_bins <= 2048;
 *                4 also needs k >= 1)
 *   cell_occ     neighbours per grid cell aimed at with one target per
 *                wavefront (default 4)
 *   h_min_frac   smallest cell edge as a fraction of r_max (default 0.5)
 *   tile_occ     neighbours per grid cell aimed at with 64 targets per
 *                wavefront or one per lane (default 1; 0 selects the default)
 *   rdf_kernel   the RDF kernel of the dense-neighbour mode (tile_policy 4 or
 *                its automatic choice): 0 automatic, 1 neighbour-major (64
 *                neighbour records per wavefront against the targets in
 *                reach), 2 one target per wavefront
 * Out-of-range values (tile_policy outside 0..4, cell_occ or h_min_frac not
 * finite and > 0, tile_occ not finite and >= 0, rdf_kernel outside 0..2)
 * return APT_E_ARG and leave
 * the tuning unchanged.  apt_set_tuning(NULL) restores the defaults. */
typedef struct {
    int32_t tile_policy;
    float cell_occ;
    float h_min_frac;
    float tile_occ;
    int32_t rdf_kernel;
} apt_tuning;
apt_status apt_set_tuning(const apt_tuning* t);
apt_status apt_get_tuning(apt_tuning* t);

/* Tracing: while enabled, every call records HIP events on its stream
 * around its stages (on = 1) or around the one-target-per-wavefront pair
 * kernel and the neighbour-major RDF kernel only (on = 2: fewer events, each
 * of which the GPU executes as a command of its own); on = 0 disables it,
 * other values return APT_E_ARG.
 * apt_trace_read waits for the recorded events, returns the summed time
 * (ms) and number of launches of one stage ("binning" = bounding box to
 * sorted records, "pair" = the pair kernel, "tile" = the 64-target kernel
 * (and the per-lane kNN of mode 4), "nbr" = the neighbour-major RDF kernel,
 * "sdm" = the two-point statistic's kernel, "cluster" = the clustering's
 * union-find kernels, "edge" = the distancing's triangle grid and search,
 * "permute" and "partition" = the batched replicates' label permutation and
 * class split) and forgets that stage's records.  Host only; off by
 * default. */
apt_status apt_trace_enable(int32_t on);
apt_status apt_trace_read(const char* stage, double* ms_total, int64_t* launches);

/* Text of the last host-side error of the calling thread ("" if none). */
const char* apt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* APT_STAT_H */
