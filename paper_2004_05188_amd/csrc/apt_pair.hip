// Target-neighbour pair kernel: for each eligible target ion, every
// neighbour ion within the radius of interest, with the RDF counted into a
// per-wavefront LDS histogram and the k nearest neighbours selected exactly.
//
// This is the region-of-interest loop of the paper's spatial statistics
// (Supplementary: "Customized user defined batch processing queues": the
// spherical ROI around each central ion is inspected once and every queued
// statistic is evaluated on it; one result buffer per worker, merged at the
// end).  The mapping is GPU-first rather than the paper's thread-per-ROI:
//  * one wavefront per target; its 64 lanes walk the neighbours of the
//    stencil rows, flattened into one sequence so that short rows still fill
//    the wavefront, reading the cell-sorted SoA arrays coalesced;
//  * the stencil is culled per row of cells: only the x-range of cells that
//    the sphere of radius R meets in that row is read;
//  * RDF bins are decided in FP32 and re-decided in FP64 within a band around
//    every bin edge, which makes the counts equal to the FP64 definition;
//  * kNN: neighbours inside a search radius are collected into an LDS buffer
//    and sorted by (FP32 squared distance, index) keys; the radius grows
//    until at least k neighbours are inside it, so the result is exact and
//    the search unbounded;
//  * targets are processed in cell order and dealt out so that each XCD
//    (and its L2) works on one contiguous slab of space.
#include "apt_bin.hpp"
#include "apt_pairdev.hpp"

namespace apt {

size_t pair_lds_bytes(bool rdf, bool knn, int n_bins, bool hist_in_lds) {
    size_t b = 0;
    if (rdf && hist_in_lds) b += (size_t)kWavesPerBlock * (size_t)hist_stride(n_bins) * 4u;
    b = (b + 15) & ~size_t(15);
    if (knn) b += (size_t)kWavesPerBlock * kKnnCap * 8u;
    return b;
}

// Targets [t0, t1) of this XCD's share of a list of n_items (the eligible
// targets in cell order, or the straggler list when `list`), one per
// wavefront: RDF counts (rdf_on) and kNN rows (KNN).
template <int FLAGS, bool KNN>
__device__ __forceinline__ void pair_items(const PairArgs& a, const GridPlan& P, PairTask& T, bool list,
                                           bool rdf_on, uint32_t& since_flush, uint32_t flush_at) {
    constexpr bool LDS_HIST = (FLAGS & kRdfLds) != 0;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int l = lane_id();
    const uint32_t n_items = list ? *a.strag_count : P.nT;
    auto slot_of = [&](uint32_t s) { return list ? a.strag[s] : s; };

    // XCD-aware deal: XCD x takes the x-th eighth of the items in cell order
    // (the grid is a multiple of kXcd workgroups)
    const int xcd = blockIdx.x % kXcd;
    const int per_xcd = gridDim.x / kXcd;
    const uint32_t wx = (uint32_t)(blockIdx.x / kXcd) * kWavesPerBlock + (uint32_t)w;
    const uint32_t wstride = (uint32_t)per_xcd * kWavesPerBlock;
    const uint32_t t0 = (uint32_t)((uint64_t)n_items * (uint64_t)xcd / kXcd);
    const uint32_t t1 = (uint32_t)((uint64_t)n_items * (uint64_t)(xcd + 1) / kXcd);

    // target data of the next iteration is loaded one iteration ahead
    uint32_t s = t0 + wx;
    uint32_t n_rank = 0, n_i = 0;
    float n_px = 0.0f, n_py = 0.0f, n_pz = 0.0f;
    if (s < t1) {
        const uint32_t q = slot_of(s);
        n_rank = a.t_rank[q];
        n_i = a.t_id[q];
        n_px = a.tx[q];
        n_py = a.ty[q];
        n_pz = a.tz[q];
    }
    for (; s < t1; s += wstride) {
        const uint32_t rank = __builtin_amdgcn_readfirstlane(n_rank);
        const uint32_t i = __builtin_amdgcn_readfirstlane(n_i);
        const float px = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, n_px)));
        const float py = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, n_py)));
        const float pz = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, n_pz)));
        const uint32_t sn = s + wstride;
        if (sn < t1) {
            const uint32_t q = slot_of(sn);
            n_rank = a.t_rank[q];
            n_i = a.t_id[q];
            n_px = a.tx[q];
            n_py = a.ty[q];
            n_pz = a.tz[q];
        }
        uint32_t hits = 0;
        const int found = run_target<FLAGS, KNN>(P, T, px, py, pz, i, hits, rdf_on);
        if (KNN) {
            if ((int64_t)rank < a.capacity) {
                if (l == 0) a.target_id[rank] = (int64_t)i;
                for (int m = l; m < a.k; m += kWave) {
                    const size_t o = (size_t)rank * (size_t)a.k + (size_t)m;
                    if (m < found) {
                        const uint64_t key = T.kbuf[m];
                        a.dist[o] = sqrtf(u2f((uint32_t)(key >> 32)));
                        a.nbr_id[o] = (int64_t)(uint32_t)key;
                    } else {
                        a.dist[o] = INFINITY;
                        a.nbr_id[o] = -1;
                    }
                }
            }
            if (a.knn_hist && l == 0)
                atomicAdd((unsigned long long*)&a.knn_hist[kth_bin(found, a.k, T.kbuf, a.xyz, px, py, pz, a.KE2,
                                                                   a.kb_nbins, a.kb_inv_w64)],
                          1ull);
            wave_sync();
        }
        if (LDS_HIST) {
            // u32 LDS counters: flush before a further target could overflow them
            since_flush += wave_sum(hits);
            if (since_flush >= flush_at) {
                flush_hist(T.hist_l, a.hist, a.n_bins);
                since_flush = 0;
            }
        }
    }
}

// (at most 80 VGPRs, six wavefronts per SIMD: they hide more of the
// candidate loads' latency than the few registers spilled outside the
// candidate loop cost)
template <int FLAGS, bool KNN>
__global__ __launch_bounds__(kBlock, 6) void k_pair(PairArgs a) {
    constexpr bool LDS_HIST = (FLAGS & kRdfLds) != 0;
    constexpr bool RDF_T = (FLAGS & (kRdfLds | kRdfGlobal)) != 0;
    extern __shared__ __align__(16) uint8_t smem[];
    GridPlan P = *a.plan;
    refine_radii(P, a.occ, a.k);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (a.n_targets) *a.n_targets = (int64_t)P.nT;
        if (a.k > 0 && a.status && (int64_t)P.nT > a.capacity) atomicOr(a.status, APT_STATUS_CAPACITY);
    }
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int l = lane_id();
    PairTask T;
    T.bpos = a.bpos;
    T.cell_start = a.cell_start;
    T.n_bins = a.n_bins;
    T.r_enum = a.r_enum;
    T.thr2 = a.thr2;
    T.inv_w = a.inv_w;
    T.lo_b = a.delta_b;
    T.hi_b = 1.0f - a.delta_b;
    T.inv_w64 = a.inv_w64;
    T.E2 = a.E2;
    T.hist_l = reinterpret_cast<uint32_t*>(smem) + (size_t)w * hist_stride(a.n_bins);
    T.hist_g = a.hist;
    T.k = a.k;
    T.rk0 = P.rk0;
    T.rknn = a.rknn;
    T.rknn2 = a.rknn2;
    T.kbuf = nullptr;
    if (LDS_HIST)
        for (int b = l; b < a.n_bins; b += kWave) T.hist_l[b] = 0;
    if (KNN) {
        size_t off = LDS_HIST ? (size_t)kWavesPerBlock * hist_stride(a.n_bins) * 4u : 0;
        off = (off + 15) & ~size_t(15);
        T.kbuf = reinterpret_cast<uint64_t*>(smem + off) + (size_t)w * kKnnCap;
    }
    wave_sync();

    uint32_t since_flush = 0;      // hits counted into hist_l since its last flush (wave total)
    const uint32_t flush_at = P.nB >= 0x7FFFFFFFu ? 0u : 0xFFFFFFFFu - P.nB;
    if (P.tile_mode == 3) {
        // the neighbour-major kernel counts the RDF and the lane pass found
        // the kNN of most targets: the kNN of the targets it left in the list
        (void)RDF_T;
        if (KNN) pair_items<FLAGS, KNN>(a, P, T, true, false, since_flush, flush_at);
    } else {
        // In tile mode the tile pass already counted the RDF of every target
        // and left the targets whose kNN it could not certify in a list: this
        // pass finishes their kNN only.
        const bool list = P.tile_mode != 0;
        pair_items<FLAGS, KNN>(a, P, T, list, !list, since_flush, flush_at);
    }
    if (LDS_HIST) flush_hist(T.hist_l, a.hist, a.n_bins);
}

// Mode 3 with the RDF one target per wavefront (tuning): the RDF of every
// target, no kNN (the lane pass and k_pair do that).  Without the kNN state
// the loop fits 64 VGPRs: eight wavefronts per SIMD to hide the candidate
// loads' latency.
template <int FLAGS>
__global__ __launch_bounds__(kBlock, 8) void k_rdf_tgt(PairArgs a) {
    constexpr bool LDS_HIST = (FLAGS & kRdfLds) != 0;
    extern __shared__ __align__(16) uint8_t smem[];
    GridPlan P = *a.plan;
    if (P.tile_mode != 3 || P.rdf_nbr) return;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int l = lane_id();
    PairTask T;
    T.bpos = a.bpos;
    T.cell_start = a.cell_start;
    T.n_bins = a.n_bins;
    T.r_enum = a.r_enum;
    T.thr2 = a.thr2;
    T.inv_w = a.inv_w;
    T.lo_b = a.delta_b;
    T.hi_b = 1.0f - a.delta_b;
    T.inv_w64 = a.inv_w64;
    T.E2 = a.E2;
    T.hist_l = reinterpret_cast<uint32_t*>(smem) + (size_t)w * hist_stride(a.n_bins);
    T.hist_g = a.hist;
    T.k = 0;
    T.rk0 = 0.0f;
    T.rknn = INFINITY;
    T.rknn2 = INFINITY;
    T.kbuf = nullptr;
    if (LDS_HIST)
        for (int b = l; b < a.n_bins; b += kWave) T.hist_l[b] = 0;
    wave_sync();
    uint32_t since_flush = 0;
    const uint32_t flush_at = P.nB >= 0x7FFFFFFFu ? 0u : 0xFFFFFFFFu - P.nB;
    pair_items<FLAGS, false>(a, P, T, false, true, since_flush, flush_at);
    if (LDS_HIST) flush_hist(T.hist_l, a.hist, a.n_bins);
}

template __global__ void k_rdf_tgt<kRdfLds>(PairArgs);
template __global__ void k_rdf_tgt<kRdfLds | kSelf>(PairArgs);
template __global__ void k_rdf_tgt<kRdfGlobal>(PairArgs);
template __global__ void k_rdf_tgt<kRdfGlobal | kSelf>(PairArgs);

// Diagnostic: the neighbour records in the cell rows of the first
// enumeration of every eligible target in the one-target-per-wavefront
// kernel (radius r_enum, or the first kNN radius when that is larger),
// summed into *out.  One target per thread.
__global__ __launch_bounds__(kBlock) void k_count_candidates(const GridPlan* plan, const uint32_t* occ,
                                                             const uint32_t* cell_start, const float* tx,
                                                             const float* ty, const float* tz, float r_enum,
                                                             int32_t k, unsigned long long* out) {
    GridPlan P = *plan;
    if (P.tile_mode == 3 && P.rdf_nbr) return;   // counted by k_rdf_nbr<kCountEvals>
    refine_radii(P, occ, k);
    const float rk = P.rk0 * 1.000001f;
    const float R = (k > 0 && !(rk < r_enum)) ? rk : r_enum;
    const float Re = R + P.eps;
    const float R2 = Re * Re;
    unsigned long long acc = 0;
    for (uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x; t < P.nT; t += (uint64_t)gridDim.x * kBlock) {
        const float px = tx[t], py = ty[t], pz = tz[t];
        if (!(isfinite(px) && isfinite(py) && isfinite(pz))) continue;
        const int cy0 = cell_axis(P, 1, py - Re), cy1 = cell_axis(P, 1, py + Re);
        const int cz0 = cell_axis(P, 2, pz - Re), cz1 = cell_axis(P, 2, pz + Re);
        for (int cz = cz0; cz <= cz1; ++cz)
            for (int cy = cy0; cy <= cy1; ++cy) {
                uint32_t st, len;
                row_span(P, cell_start, cy, cz, px, py, pz, px, py, pz, R2, st, len);
                acc += len;
            }
    }
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, kWave);
    if (lane_id() == 0 && acc) atomicAdd(out, acc);
}

size_t tile_lds_bytes(bool rdf, int n_bins) {
    size_t b = rdf ? (size_t)kWavesPerBlock * (size_t)hist_stride(n_bins) * 4u : 0;
    b = (b + 15) & ~size_t(15);
    return b + (size_t)kWavesPerBlock * kStage * sizeof(float4);
}

// (at most 128 VGPRs: four wavefronts per SIMD against three, for a few spills)
template <int FLAGS, int KMAX>
__global__ __launch_bounds__(kBlock, 4) void k_pair_tile(PairArgs a) {
    constexpr bool LDS_HIST = (FLAGS & kRdfLds) != 0;
    GridPlan P = *a.plan;
    if (!P.tile_mode || (P.tile_mode == 3 && KMAX == 0)) return;
    refine_radii(P, a.occ, a.k);
    extern __shared__ __align__(16) uint8_t smem[];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int l = lane_id();
    PairTask T;
    T.bpos = a.bpos;
    T.cell_start = a.cell_start;
    T.n_bins = a.n_bins;
    T.r_enum = a.r_enum;
    T.thr2 = a.thr2;
    T.inv_w = a.inv_w;
    T.lo_b = a.delta_b;
    T.hi_b = 1.0f - a.delta_b;
    T.inv_w64 = a.inv_w64;
    T.E2 = a.E2;
    T.hist_l = reinterpret_cast<uint32_t*>(smem) + (size_t)w * hist_stride(a.n_bins);
    T.hist_g = a.hist;
    T.k = a.k;
    T.kbuf = nullptr;
    size_t off = LDS_HIST ? (size_t)kWavesPerBlock * hist_stride(a.n_bins) * 4u : 0;
    off = (off + 15) & ~size_t(15);
    float4* stage = reinterpret_cast<float4*>(smem + off) + (size_t)w * kStage;
    if (LDS_HIST)
        for (int b = l; b < a.n_bins; b += kWave) T.hist_l[b] = 0;
    wave_sync();
    const float Rk = KMAX > 0 ? fminf(P.rk_tile, a.rknn) : 0.0f;

    // XCD-aware work queue over tiles (cell order): each XCD takes one
    // eighth of them, its wavefronts take batches of consecutive tiles from
    // the XCD's counter, so the tiles in flight stay one compact region
    const uint32_t n_tiles = (P.nT + kWave - 1) / kWave;
    const int xcd = blockIdx.x % kXcd;
    const uint32_t g0 = (uint32_t)((uint64_t)n_tiles * (uint64_t)xcd / kXcd);
    const uint32_t g1 = (uint32_t)((uint64_t)n_tiles * (uint64_t)(xcd + 1) / kXcd);
    constexpr uint32_t kBatch = 4;
    uint32_t since_flush = 0;
    const uint32_t flush_at = P.nB >= 0x7FFFFFFFu / kWave ? 0u : 0xFFFFFFFFu - P.nB * kWave;
    for (;;) {
    uint32_t gb = 0;
    if (l == 0) gb = atomicAdd(a.work_q + kXcd + xcd, kBatch);
    gb = g0 + (uint32_t)__shfl((int)gb, 0, kWave);
    if (gb >= g1) break;
    const uint32_t ge = gb + kBatch < g1 ? gb + kBatch : g1;
    for (uint32_t g = gb; g < ge; ++g) {
        const uint32_t slot = g * kWave + (uint32_t)l;
        const bool valid = slot < P.nT;
        uint32_t rank = 0, i = 0;
        float px = 0.0f, py = 0.0f, pz = 0.0f;
        if (valid) {
            rank = a.t_rank[slot];
            i = a.t_id[slot];
            px = a.tx[slot];
            py = a.ty[slot];
            pz = a.tz[slot];
        }
        uint32_t hits = 0;
        TopK<KMAX> top;
        // mode 3: the kNN only (the one-per-wavefront pass counts the RDF)
        if (P.tile_mode >= 2) run_lane<FLAGS, KMAX>(P, T, valid, px, py, pz, i, Rk, top, hits, P.tile_mode == 2);
        else run_tile<FLAGS, KMAX>(P, T, valid, px, py, pz, i, Rk, stage, top, hits);
        if (KMAX > 0) {
            // certified: k keys within Rk, or the radius already is r_knn_max
            uint64_t kth = top.key[0];
#pragma unroll
            for (int q = 1; q < KMAX; ++q)
                if (q == a.k - 1) kth = top.key[q];
            const bool fin = isfinite(px) && isfinite(py) && isfinite(pz);
            const bool done = valid && (kth != ~0ull || Rk >= a.rknn || !fin);
            if (valid && !done) {
                const uint64_t m = __ballot(true);
                uint32_t base = 0;
                if (l == __builtin_ctzll(m)) base = atomicAdd(a.strag_count, (uint32_t)__popcll(m));
                base = __shfl(base, __builtin_ctzll(m), kWave);
                a.strag[base + __popcll(m & lanemask_lt())] = slot;
            }
            if (done) {
                int found = 0;
#pragma unroll
                for (int q = 0; q < KMAX; ++q) found += (q < a.k && top.key[q] != ~0ull);
                if ((int64_t)rank < a.capacity) {
                    a.target_id[rank] = (int64_t)i;
#pragma unroll
                    for (int q = 0; q < KMAX; ++q) {
                        if (q < a.k) {
                            const size_t o = (size_t)rank * (size_t)a.k + (size_t)q;
                            const uint64_t key = top.key[q];
                            if (q < found) {
                                a.dist[o] = sqrtf(u2f((uint32_t)(key >> 32)));
                                a.nbr_id[o] = (int64_t)(uint32_t)key;
                            } else {
                                a.dist[o] = INFINITY;
                                a.nbr_id[o] = -1;
                            }
                        }
                    }
                }
                if (a.knn_hist) {
                    int b = a.kb_nbins;
                    if (found == a.k) b = key_bin(kth, a.xyz, px, py, pz, a.KE2, a.kb_nbins, a.kb_inv_w64);
                    atomicAdd((unsigned long long*)&a.knn_hist[b], 1ull);
                }
            }
        }
        if (LDS_HIST) {
            since_flush += wave_sum(hits);
            if (since_flush >= flush_at) {
                flush_hist(T.hist_l, a.hist, a.n_bins);
                since_flush = 0;
            }
        }
    }
    }
    if (LDS_HIST) flush_hist(T.hist_l, a.hist, a.n_bins);
}

// ---------------------------------------------------- neighbour-major RDF --
// Mode 3 (neighbours dense enough that 64 consecutive records, a run of a
// few cells along one cell row, span little more than a cell): a wavefront
// holds 64 neighbour records, one per lane, and stages in LDS every target
// within r_max of their bounding box (targets are in plain cell order, with
// per-cell offsets); each staged target is then evaluated against all 64
// records at once.  The target's position is uniform across the wavefront,
// so a pair costs its distance, the comparison and, on a hit, the FP32 bin
// with the same FP64 re-decision band as the target-major kernels: no memory
// access per pair, and each record is read once per launch.
constexpr int kNbrList = 256;   // targets staged per wavefront per round

// (the LDS histogram has one more counter: pairs whose bin is n_bins, just
// beyond r_max, go there uncounted instead of taking a branch)
size_t nbr_lds_bytes(int n_bins, bool hist_in_lds) {
    size_t b = hist_in_lds ? (size_t)kWavesPerBlock * (size_t)hist_stride(n_bins + 1) * 4u : 0;
    b = (b + 15) & ~size_t(15);
    return b + (size_t)kWavesPerBlock * kNbrList * sizeof(float4);
}

// (at most 64 VGPRs: eight wavefronts per SIMD)
template <int FLAGS>
__global__ __launch_bounds__(kBlock, 8) void k_rdf_nbr(PairArgs a) {
    constexpr bool COUNT = (FLAGS & kCountEvals) != 0;
    constexpr bool LDS_HIST = !COUNT && (FLAGS & kRdfLds) != 0;
    const GridPlan P = *a.plan;
    if (P.tile_mode != 3 || !P.rdf_nbr) return;
    unsigned long long evals = 0;   // COUNT: pair evaluations (records x staged targets)
    extern __shared__ __align__(16) uint8_t smem[];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int l = lane_id();
    uint32_t* hist_l = reinterpret_cast<uint32_t*>(smem) + (size_t)w * hist_stride(a.n_bins + 1);
    size_t off = LDS_HIST ? (size_t)kWavesPerBlock * hist_stride(a.n_bins + 1) * 4u : 0;
    off = (off + 15) & ~size_t(15);
    float4* list = reinterpret_cast<float4*>(smem + off) + (size_t)w * kNbrList;
    if (LDS_HIST)
        for (int b = l; b <= a.n_bins; b += kWave) hist_l[b] = 0;
    wave_sync();

    const uint32_t nB = P.nB;
    const uint32_t n_chunks = (nB + kWave - 1) / kWave;
    // XCD-aware work queue over chunks (cell order): each XCD takes one
    // eighth of the chunks, and its wavefronts take batches of consecutive
    // chunks from the XCD's counter, so that the chunks in flight on an XCD
    // stay one compact region whose target rows its L2 keeps (a static deal
    // lets the wavefronts drift apart).  (workgroup b runs on XCD b mod 8)
    const int xcd = blockIdx.x % kXcd;
    const uint32_t c0 = (uint32_t)((uint64_t)n_chunks * (uint64_t)xcd / kXcd);
    const uint32_t c1 = (uint32_t)((uint64_t)n_chunks * (uint64_t)(xcd + 1) / kXcd);
    constexpr uint32_t kBatch = 16;
    const float Re = a.r_enum + P.eps;
    const float R2 = Re * Re;
    const float thr2 = a.thr2, inv_w = a.inv_w, lo_b = a.delta_b, hi_b = 1.0f - a.delta_b;
    const float half_band = 0.5f - a.delta_b;   // |fract - 1/2| beyond it: within delta_b of an edge
    uint32_t since_flush = 0;
    const uint32_t flush_at = 0xFFFFFFFFu - (uint32_t)(kWave * kNbrList);

    for (;;) {
    uint32_t cb = 0;
    if (l == 0) cb = atomicAdd(a.work_q + xcd, kBatch);
    cb = c0 + (uint32_t)__shfl((int)cb, 0, kWave);
    if (cb >= c1) break;
    const uint32_t ce = cb + kBatch < c1 ? cb + kBatch : c1;
    for (uint32_t c = cb; c < ce; ++c) {
        const uint32_t j = c * (uint32_t)kWave + (uint32_t)l;
        const bool valid = j < nB;
        const float4 rec = a.bpos[valid ? j : nB - 1];
        const bool fin0 = valid && isfinite(rec.x) && isfinite(rec.y) && isfinite(rec.z);
        // a run of 64 records may end one cell row and start the next, far
        // apart in x: each row's part is evaluated with its own bounding box
        const uint32_t crow = fin0 ? (uint32_t)cell_axis(P, 2, rec.z) * (uint32_t)P.dim[1] +
                                         (uint32_t)cell_axis(P, 1, rec.y)
                                   : 0xFFFFFFFFu;
        uint64_t todo = __ballot(fin0);
        while (todo) {
            const uint32_t row_sel = readlane(crow, __builtin_ctzll(todo));
            const bool fin = fin0 && crow == row_sel;
            todo &= ~__ballot(fin);
            // a box holding the part's records: its cells (one cell row; the
            // records are in cell order, so its first and last lanes hold its
            // lowest and highest x cell), widened by the FP32 margin of the
            // cells' assignment and bounds.  (Six lane reductions for the
            // exact box cost more VALU than the slightly larger box's extra
            // candidates.)
            const uint64_t pm = __ballot(fin);
            const int cxv = fin ? cell_axis(P, 0, rec.x) : 0;
            const int cxa = readlane(cxv, __builtin_ctzll(pm));
            const int cxb = readlane(cxv, 63 - __builtin_clzll(pm));
            const int cyr = (int)(row_sel % (uint32_t)P.dim[1]), czr = (int)(row_sel / (uint32_t)P.dim[1]);
            const float x0 = P.lo[0] + (float)cxa * P.h - P.eps, x1 = P.lo[0] + (float)(cxb + 1) * P.h + P.eps;
            const float y0 = P.lo[1] + (float)cyr * P.h - P.eps, y1 = P.lo[1] + (float)(cyr + 1) * P.h + P.eps;
            const float z0 = P.lo[2] + (float)czr * P.h - P.eps, z1 = P.lo[2] + (float)(czr + 1) * P.h + P.eps;
            const uint32_t n_rec = (uint32_t)__popcll(pm);
            // every staged target against the 64 records
            auto run = [&](int cnt) {
                if (COUNT) {
                    evals += (unsigned long long)cnt * n_rec;
                    return;
                }
                wave_sync();
#pragma unroll 4
                for (int t = 0; t < cnt; ++t) {
                    const float4 T = list[t];
                    const float dx = rec.x - T.x, dy = rec.y - T.y, dz = rec.z - T.z;
                    const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                    // (a target's pair with its own record lands in bin 0
                    // here and is taken off by k_nbr_self)
                    if (fin && d2 < thr2) {
                        const float tt = __builtin_amdgcn_sqrtf(d2) * inv_w;
                        int b = (int)tt;
                        if (LDS_HIST) {
                            // b == n_bins (beyond r_max) lands in the spare counter
                            if (__builtin_expect(fabsf(__builtin_amdgcn_fractf(tt) - 0.5f) > half_band, 0))
                                b = exact_bin(exact_D2(T.x, T.y, T.z, rec.x, rec.y, rec.z), a.E2, a.n_bins, a.inv_w64);
                            atomicAdd(&hist_l[b], 1u);
                        } else {
                            const float fr = tt - (float)b;
                            if (__builtin_expect(fr < lo_b || fr > hi_b, 0))
                                b = exact_bin(exact_D2(T.x, T.y, T.z, rec.x, rec.y, rec.z), a.E2, a.n_bins, a.inv_w64);
                            if (b < a.n_bins) atomicAdd((unsigned long long*)&a.hist[b], 1ull);
                        }
                    }
                }
                wave_sync();
                if (LDS_HIST) {
                    // at most cnt * 64 counts were added
                    since_flush += (uint32_t)cnt * n_rec;
                    if (since_flush >= flush_at) {
                        flush_hist(hist_l, a.hist, a.n_bins);
                        since_flush = 0;
                    }
                }
            };

            // target rows that the box grown by Re meets, each trimmed in x
            int cnt = 0;
            const int cy0 = cell_axis(P, 1, y0 - Re), cy1 = cell_axis(P, 1, y1 + Re);
            const int cz0 = cell_axis(P, 2, z0 - Re), cz1 = cell_axis(P, 2, z1 + Re);
            const int ny = cy1 - cy0 + 1, nz = cz1 - cz0 + 1;
            const int nrows = ny * nz;
            for (int rb = 0; rb < nrows; rb += kWave) {
                const int r = rb + l;
                uint32_t st = 0, len = 0;
                if (r < nrows)
                    row_span(P, a.t_cell_start, cy0 + r % ny, cz0 + r / ny, x0, y0, z0, x1, y1, z1, R2, st, len);
                const uint32_t inc = wave_incl_scan(len);
                const uint32_t tot = readlane(inc, kWave - 1);
                const uint32_t offr = inc - len;
                for (uint32_t b0 = 0; b0 < tot; b0 += kWave) {
                    // the target slot of lane v: the last row starting at or before v
                    const uint32_t v = b0 + (uint32_t)l;
                    const uint32_t lim = b0 + kWave < tot ? b0 + kWave : tot;
                    const int r0 = __popcll(__ballot(inc <= b0));
                    const int r1 = __popcll(__ballot(offr < lim)) - 1;
                    int row = r0;
                    for (int step = 32; step > 0; step >>= 1) {
                        if (step > r1 - r0) continue;            // uniform
                        const int cc = row + step;
                        const uint32_t oc = (uint32_t)__shfl((int)offr, cc < kWave ? cc : kWave - 1, kWave);
                        if (cc <= r1 && oc <= v) row = cc;
                    }
                    const uint32_t base = (uint32_t)__shfl((int)(st - offr), row, kWave);
                    bool keep = v < tot;
                    float tx = 0.0f, ty = 0.0f, tz = 0.0f;
                    if (keep) {
                        const uint32_t q = base + v;
                        tx = a.tx[q];
                        ty = a.ty[q];
                        tz = a.tz[q];
                        // exact cull against the records' box (a pair within
                        // r_max lies within r_max of the box)
                        const float ex = fmaxf(0.0f, fmaxf(x0 - tx, tx - x1));
                        const float ey = fmaxf(0.0f, fmaxf(y0 - ty, ty - y1));
                        const float ez = fmaxf(0.0f, fmaxf(z0 - tz, tz - z1));
                        keep = isfinite(tx) && isfinite(ty) && isfinite(tz) && ex * ex + ey * ey + ez * ez <= R2;
                    }
                    const uint64_t m = __ballot(keep);
                    if (keep) list[cnt + __popcll(m & lanemask_lt())] = make_float4(tx, ty, tz, 0.0f);
                    cnt += __popcll(m);
                    if (cnt > kNbrList - kWave) {
                        run(cnt);
                        cnt = 0;
                    }
                }
            }
            if (cnt > 0) run(cnt);
        }
    }
    }
    if (LDS_HIST) flush_hist(hist_l, a.hist, a.n_bins);
    if (COUNT && l == 0 && evals) atomicAdd((unsigned long long*)a.hist, evals);
}

template __global__ void k_rdf_nbr<kRdfLds>(PairArgs);
template __global__ void k_rdf_nbr<kRdfGlobal>(PairArgs);

__global__ __launch_bounds__(kBlock) void k_nbr_self(PairArgs a) {
    const GridPlan P = *a.plan;
    if (P.tile_mode != 3 || !P.rdf_nbr) return;
    uint32_t cnt = 0;
    for (uint32_t q = blockIdx.x * kBlock + threadIdx.x; q < P.nT; q += gridDim.x * kBlock) {
        if (!(isfinite(a.tx[q]) && isfinite(a.ty[q]) && isfinite(a.tz[q]))) continue;
        if (a.nbr_species == APT_ANY || (int)a.lab[a.t_id[q]] == a.nbr_species) ++cnt;
    }
    cnt = wave_sum(cnt);
    // (u64 arithmetic modulo 2^64: the order of this and the kernel's adds
    // does not matter)
    if (lane_id() == 0 && cnt) atomicAdd((unsigned long long*)a.hist, 0ull - (unsigned long long)cnt);
}
template __global__ void k_rdf_nbr<kRdfGlobal | kCountEvals>(PairArgs);

#define APT_TILE_INST(F, K) template __global__ void k_pair_tile<F, K>(PairArgs);
APT_TILE_INST(kRdfLds, 0)
APT_TILE_INST(kRdfLds | kSelf, 0)
APT_TILE_INST(kRdfLds, 4)
APT_TILE_INST(kRdfLds | kSelf, 4)
APT_TILE_INST(kRdfLds, 10)
APT_TILE_INST(kRdfLds | kSelf, 10)
APT_TILE_INST(kRdfLds, 16)
APT_TILE_INST(kRdfLds | kSelf, 16)
APT_TILE_INST(0, 4)
APT_TILE_INST(kSelf, 4)
APT_TILE_INST(0, 10)
APT_TILE_INST(kSelf, 10)
APT_TILE_INST(0, 16)
APT_TILE_INST(kSelf, 16)
#undef APT_TILE_INST

#define APT_PAIR_INST(F, K) template __global__ void k_pair<F, K>(PairArgs);
APT_PAIR_INST(kRdfLds, false)
APT_PAIR_INST(kRdfLds | kSelf, false)
APT_PAIR_INST(kRdfLds, true)
APT_PAIR_INST(kRdfLds | kSelf, true)
APT_PAIR_INST(kRdfGlobal, false)
APT_PAIR_INST(kRdfGlobal, true)
APT_PAIR_INST(kRdfGlobal | kSelf, false)
APT_PAIR_INST(kRdfGlobal | kSelf, true)
APT_PAIR_INST(0, true)
APT_PAIR_INST(kSelf, true)
#undef APT_PAIR_INST

}  // namespace apt
