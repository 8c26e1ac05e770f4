// Batched label-randomised replicates of many species pairs.
//
// The paper computes every spatial statistic for the original and for
// randomly reordered ion-type labels (Supplementary: "Importance of high
// quality random number generators") and machines off a queue of
// (statistic x ion-type pair) tasks per region of interest (Methods: "User-
// defined batch processing queues").  Here hundreds of replicates and all
// requested pairs run in few launches: positions are binned once; per
// replicate the binned ions are split by their permuted species into
// segments that stay in cell order (a stable partition, no re-sort); one
// pair launch then deals (replicate, pair, target) work to wavefronts in
// chunks through an atomic counter.  The result of (replicate r, pair p) is
// by definition the plain kNN/RDF of pair p on the labels of replicate r.
#include "apt_batched.hpp"
#include "apt_pairdev.hpp"

namespace apt {

size_t batched_lds_bytes(int n_bins) {
    size_t b = (size_t)kWavesPerBlock * (size_t)hist_stride(n_bins) * 4u;
    b = (b + 15) & ~size_t(15);
    return b + (size_t)kWavesPerBlock * kKnnCap * 8u;
}

// tiles: histogram + staging buffer (which later holds a straggler's kNN keys)
size_t batched_tile_lds_bytes(int n_bins) {
    static_assert(kStage * sizeof(float4) >= kKnnCap * sizeof(uint64_t), "key buffer inside the stage");
    size_t b = (size_t)kWavesPerBlock * (size_t)hist_stride(n_bins) * 4u;
    b = (b + 15) & ~size_t(15);
    return b + (size_t)kWavesPerBlock * kStage * sizeof(float4);
}

__device__ __forceinline__ int class_of(const PartArgs& a, int r, uint32_t id) {
    return a.slot[a.LR[(size_t)r * (size_t)a.n + id]];
}

// ---- 1. per-block class counts of the binned ions of each replicate
__global__ __launch_bounds__(kBlock) void k_bpart_count(PartArgs a) {
    const GridPlan P = *a.plan;
    const uint32_t* __restrict__ sid = a.vals[P.passes & 1];
    const int r = blockIdx.y;
    const int64_t beg = (int64_t)blockIdx.x * a.chunk;
    const int64_t end = beg + a.chunk < a.n ? beg + a.chunk : a.n;
    uint32_t c[kMaxClasses];
#pragma unroll
    for (int q = 0; q < kMaxClasses; ++q) c[q] = 0;
    for (int64_t p = beg + threadIdx.x; p < end; p += kBlock) {
        const int cls = class_of(a, r, sid[p]);
#pragma unroll
        for (int q = 0; q < kMaxClasses; ++q) c[q] += (cls == q);
    }
    __shared__ uint32_t s_c[kWavesPerBlock][kMaxClasses];
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < kMaxClasses; ++q) {
        const uint32_t t = wave_sum(c[q]);
        if (lane_id() == 0) s_c[w][q] = t;
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)a.C) {
        uint32_t t = 0;
        for (int v = 0; v < kWavesPerBlock; ++v) t += s_c[v][threadIdx.x];
        a.cnt[((size_t)r * a.C + threadIdx.x) * a.G + blockIdx.x] = t;
    }
}

// ---- 2. stable scatter of the binned ions into class segments
__global__ __launch_bounds__(kBlock) void k_bpart_scatter(PartArgs a) {
    const GridPlan P = *a.plan;
    const uint32_t* __restrict__ sid = a.vals[P.passes & 1];
    const uint32_t* __restrict__ skey = a.keys[P.passes & 1];
    const int r = blockIdx.y;
    const int w = threadIdx.x / kWave, l = lane_id();
    __shared__ uint32_t s_cnt[kMaxClasses][kPartItems][kWavesPerBlock];
    __shared__ uint32_t s_base[kMaxClasses][kPartItems][kWavesPerBlock];
    __shared__ uint32_t s_run[kMaxClasses];
    const int64_t beg = (int64_t)blockIdx.x * a.chunk;
    const int64_t end = beg + a.chunk < a.n ? beg + a.chunk : a.n;
    if (threadIdx.x < (unsigned)a.C) s_run[threadIdx.x] = a.cnt[((size_t)r * a.C + threadIdx.x) * a.G + blockIdx.x];
    __syncthreads();
    for (int64_t tile = beg; tile < end; tile += kPartTile) {
        int cls[kPartItems];
#pragma unroll
        for (int it = 0; it < kPartItems; ++it) {
            const int64_t p = tile + (int64_t)it * kBlock + threadIdx.x;
            cls[it] = p < end ? class_of(a, r, sid[p]) : -1;
            for (int q = 0; q < a.C; ++q) {
                const uint64_t m = __ballot(cls[it] == q);
                if (l == 0) s_cnt[q][it][w] = (uint32_t)__popcll(m);
            }
        }
        __syncthreads();
        if (w == 0) {
            // per class: exclusive scan over (item, wave) in index order
            for (int q = 0; q < a.C; ++q) {
                const uint32_t x = s_cnt[q][l / kWavesPerBlock][l % kWavesPerBlock];
                const uint32_t xs = wave_incl_scan(x);
                s_base[q][l / kWavesPerBlock][l % kWavesPerBlock] = xs - x + s_run[q];
                const uint32_t tot = readlane(xs, kWave - 1);
                wave_sync();
                if (l == 0) s_run[q] += tot;
                wave_sync();
            }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kPartItems; ++it) {
            const int64_t p = tile + (int64_t)it * kBlock + threadIdx.x;
            const int q = cls[it];
            // rank among this wave's items of the same class
            uint64_t m = 0;
            for (int qq = 0; qq < a.C; ++qq) {
                const uint64_t mq = __ballot(q == qq);
                if (q == qq) m = mq;
            }
            if (q >= 0) {
                const uint32_t dst = s_base[q][it][w] + (uint32_t)__popcll(m & lanemask_lt());
                a.Pp[dst] = a.S[p];
                a.Pcell[dst] = skey[p];
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ uint64_t seg_start(const uint32_t* cnt, int r, int C, int G, int q) {
    return cnt[((size_t)r * C + q) * G];
}
__device__ __forceinline__ uint64_t seg_end(const uint32_t* cnt, int r, int C, int G, int q, int64_t n) {
    return q + 1 < C ? (uint64_t)cnt[((size_t)r * C + q + 1) * G] : (uint64_t)(r + 1) * (uint64_t)n;
}

// ---- 3. cell offsets of every class segment (the "other" class needs none)
__global__ __launch_bounds__(kBlock) void k_bpart_cells(PartArgs a) {
    const GridPlan P = *a.plan;
    const int r = blockIdx.y;
    const uint32_t nc = P.n_cells;
    uint64_t sb[kMaxClasses + 1];
    for (int q = 0; q < a.C; ++q) sb[q] = seg_start(a.cnt, r, a.C, a.G, q);
    sb[a.C] = (uint64_t)(r + 1) * (uint64_t)a.n;
    const uint64_t r0 = (uint64_t)r * (uint64_t)a.n;
    for (uint64_t Q = r0 + (uint64_t)blockIdx.x * kBlock + threadIdx.x; Q < sb[a.C - 1];
         Q += (uint64_t)gridDim.x * kBlock) {
        int q = 0;
        while (Q >= sb[q + 1]) ++q;
        uint32_t* cs = a.CS + ((size_t)r * (a.C - 1) + q) * (size_t)a.cs_stride;
        const uint32_t c = a.Pcell[Q];
        const uint32_t c0 = Q == sb[q] ? 0u : a.Pcell[Q - 1] + 1u;
        for (uint32_t cc = c0; cc <= c; ++cc) cs[cc] = (uint32_t)Q;
        if (Q + 1 == sb[q + 1])
            for (uint32_t cc = c + 1; cc <= nc; ++cc) cs[cc] = (uint32_t)sb[q + 1];
    }
}

// classes with an empty segment: every offset is the segment start
__global__ __launch_bounds__(kBlock) void k_bpart_empty(PartArgs a) {
    const GridPlan P = *a.plan;
    const int r = blockIdx.y / (a.C - 1), q = blockIdx.y % (a.C - 1);
    const uint64_t s0 = seg_start(a.cnt, r, a.C, a.G, q), s1 = seg_end(a.cnt, r, a.C, a.G, q, a.n);
    if (s0 != s1) return;
    uint32_t* cs = a.CS + ((size_t)r * (a.C - 1) + q) * (size_t)a.cs_stride;
    for (uint32_t cc = blockIdx.x * kBlock + threadIdx.x; cc <= P.n_cells; cc += gridDim.x * kBlock)
        cs[cc] = (uint32_t)s0;
}

// Certified kNN radius of a tile: tile_reach (default 1.3) times the
// Poisson mean k-th distance (the first kNN radius rk0 is 1.15x that mean).
// Smaller radii stage fewer candidates, larger ones leave fewer targets to
// the exact one-by-one fallback; on the clustered needle 1.3x was fastest
// (1.0x took 3.4x its time, 1.15x 1.2x, 1.6x 1.14x, 2.0x 1.5x).
__device__ inline float tile_reach_rk0(const BatchPairArgs& a) { return a.tile_reach / 1.15f; }

// Cells that hold at least one ion (all ions are binned here), counted once
// per call: their volume is the specimen's, unlike the bounding box's (a
// needle fills less than half of its box).  *occ must be zero on entry.
__global__ __launch_bounds__(kBlock) void k_occupied(const GridPlan* plan, const uint32_t* cell_start,
                                                     uint32_t* occ) {
    const uint32_t nc = plan->n_cells;
    uint32_t c = 0;
    for (uint32_t q = blockIdx.x * kBlock + threadIdx.x; q < nc; q += gridDim.x * kBlock)
        c += cell_start[q + 1] > cell_start[q];
    c = wave_sum(c);
    if (lane_id() == 0 && c) atomicAdd(occ, c);
}

// volume the ions occupy: the occupied cells (never more than the box)
__device__ inline double batch_volume(const BatchPairArgs& a, const GridPlan& P) {
    double box = 1.0;
    for (int ax = 0; ax < 3; ++ax) box *= fmax((double)P.hi[ax] - (double)P.lo[ax], 1e-3);
    const double h = (double)P.h;
    const double v = (double)(*a.occ) * h * h * h;
    return v > 0.0 && v < box ? v : box;
}

// first kNN radius of a pair: 1.15 x the Poisson mean k-th distance at the
// neighbour class's density over the occupied volume
__device__ inline float batch_rk0(const GridPlan& P, double vol, uint64_t nb, int k) {
    const double rho = (double)(nb > 0 ? nb : 1) / vol;
    return (float)fmin(1.15 * cbrt(3.0 * ((double)k + 0.5) / (4.0 * M_PI * rho)), (double)P.r_all);
}

// Is pair p tiled (64 targets per wavefront)?  As in the plain path: targets
// at least as many as neighbours and dense enough that 64 of them fill no
// more than the cube of the search reach.  Class sizes are the same in
// every replicate (a permutation keeps them), so the choice is per pair.
__device__ inline bool batch_tiled(const BatchPairArgs& a, const GridPlan& P, int p) {
    if (!a.tile_ok) return false;
    const uint64_t na = seg_end(a.cnt, 0, a.C, a.G, a.pairs[p].a, a.n) - seg_start(a.cnt, 0, a.C, a.G, a.pairs[p].a);
    const uint64_t nb = seg_end(a.cnt, 0, a.C, a.G, a.pairs[p].b, a.n) - seg_start(a.cnt, 0, a.C, a.G, a.pairs[p].b);
    if (na < nb || na < 4096) return false;
    const double vol = batch_volume(a, P);
    const double rk_tile = (double)tile_reach_rk0(a) * (double)batch_rk0(P, vol, nb, a.k);
    const double R = fmax((double)a.r_enum, rk_tile);
    return 64.0 * vol / (double)na <= R * R * R;
}

// ---- 4. prefixes of the work over (replicate, pair): targets of the pairs
//         run one per wavefront, tiles of the tiled pairs
__global__ void k_batch_items(BatchPairArgs a) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const GridPlan P = *a.plan;
    bool tiled[kMaxPairs];
    for (int p = 0; p < a.n_pairs; ++p) tiled[p] = batch_tiled(a, P, p);
    uint64_t acc = 0, tacc = 0;
    for (int r = 0; r < a.R; ++r)
        for (int p = 0; p < a.n_pairs; ++p) {
            a.items[r * a.n_pairs + p] = acc;
            a.titems[r * a.n_pairs + p] = tacc;
            const int q = a.pairs[p].a;
            const uint64_t len = seg_end(a.cnt, r, a.C, a.G, q, a.n) - seg_start(a.cnt, r, a.C, a.G, q);
            if (tiled[p]) tacc += (len + kWave - 1) / kWave;
            else acc += len;
        }
    a.items[a.R * a.n_pairs] = acc;
    a.titems[a.R * a.n_pairs] = tacc;
    a.work[0] = 0;
    a.work[1] = 0;
}

// ---- 5. the pair launch over (replicate, pair, target)
constexpr uint64_t kChunk = 32;

__global__ __launch_bounds__(kBlock, 6) void k_pair_batched(BatchPairArgs a) {   // 6 waves per SIMD (<= 80 VGPRs)
    extern __shared__ __align__(16) uint8_t smem[];
    const GridPlan P = *a.plan;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int l = lane_id();
    PairTask T;
    T.n_bins = a.n_bins;
    T.r_enum = a.r_enum;
    T.thr2 = a.thr2;
    T.inv_w = a.inv_w;
    T.lo_b = a.delta_b;
    T.hi_b = 1.0f - a.delta_b;
    T.inv_w64 = a.inv_w64;
    T.E2 = a.E2;
    T.hist_l = reinterpret_cast<uint32_t*>(smem) + (size_t)w * hist_stride(a.n_bins);
    T.k = a.k;
    T.rknn = INFINITY;
    T.rknn2 = INFINITY;
    size_t off = ((size_t)kWavesPerBlock * hist_stride(a.n_bins) * 4u + 15) & ~size_t(15);
    T.kbuf = reinterpret_cast<uint64_t*>(smem + off) + (size_t)w * kKnnCap;
    for (int b = l; b < a.n_bins; b += kWave) T.hist_l[b] = 0;
    wave_sync();

    const int RP = a.R * a.n_pairs;
    const uint64_t total = a.items[RP];
    const double vol = batch_volume(a, P);
    int cur = -1;                     // (replicate, pair) of the LDS histogram contents
    uint32_t since_flush = 0;
    uint64_t seg_a0 = 0;
    const float* d_bnd = a.d_bnd;
    float d_srf = 0.0f;
    int rp = 0;
    for (;;) {
        uint64_t c0 = 0;
        if (l == 0) c0 = atomicAdd((unsigned long long*)a.work, (unsigned long long)kChunk);
        {
            // broadcast lane 0's chunk start as a wave-uniform value
            const uint64_t b = __shfl((unsigned long long)c0, 0, kWave);
            c0 = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32)) << 32) |
                 (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
        }
        if (c0 >= total) break;
        const uint64_t c1 = c0 + kChunk < total ? c0 + kChunk : total;
        // (replicate, pair) of the first item: last rp with items[rp] <= c0
        {
            int lo = 0, hi = RP;      // items[lo] <= c0 < items[hi]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (a.items[mid] <= c0) lo = mid; else hi = mid;
            }
            rp = lo;
        }
        for (uint64_t it = c0; it < c1; ++it) {
            while (it >= a.items[rp + 1]) ++rp;
            const int r = rp / a.n_pairs, p = rp % a.n_pairs;
            const BatchPair bp = a.pairs[p];
            if (rp != cur) {
                if (cur >= 0) {
                    const int rr = cur / a.n_pairs, pp = cur % a.n_pairs;
                    flush_hist(T.hist_l, a.rdf_hist + ((size_t)(a.rep0 + rr) * a.n_pairs + pp) * a.n_bins, a.n_bins);
                    since_flush = 0;
                }
                cur = rp;
                seg_a0 = seg_start(a.cnt, r, a.C, a.G, bp.a);
                const uint64_t b0 = seg_start(a.cnt, r, a.C, a.G, bp.b);
                const uint64_t b1 = seg_end(a.cnt, r, a.C, a.G, bp.b, a.n);
                T.bpos = a.Pp;
                T.cell_start = a.CS + ((size_t)r * (a.C - 1) + bp.b) * (size_t)a.cs_stride;
                T.rk0 = batch_rk0(P, vol, b1 - b0, a.k);
                T.hist_g = a.rdf_hist + ((size_t)(a.rep0 + r) * a.n_pairs + p) * a.n_bins;
                d_srf = bp.d_srf;
            }
            const uint64_t q = seg_a0 + (it - a.items[rp]);
            const float4 rec = a.Pp[q];
            const uint32_t i = __builtin_amdgcn_readfirstlane(__builtin_bit_cast(uint32_t, rec.w));
            if (d_bnd && !(d_bnd[i] >= d_srf)) continue;          // not an eligible target
            const float px = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, rec.x)));
            const float py = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, rec.y)));
            const float pz = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, rec.z)));
            uint32_t hits = 0;
            const int found = run_target<kRdfLds | kSelf, true>(P, T, px, py, pz, i, hits);
            if (a.knn_hist && l == 0) {
                const int b = kth_bin(found, a.k, T.kbuf, a.xyz, px, py, pz, a.KE2, a.kb_nbins, a.kb_inv_w64);
                atomicAdd((unsigned long long*)&a.knn_hist[((size_t)(a.rep0 + r) * a.n_pairs + p) *
                                                           (size_t)(a.kb_nbins + 1) + b],
                          1ull);
            }
            wave_sync();
            since_flush += wave_sum(hits);
            if (since_flush >= 0x7FFFFFFFu - (uint32_t)min((uint64_t)a.n, (uint64_t)0x7FFFFFFFu)) {
                flush_hist(T.hist_l, T.hist_g, a.n_bins);
                since_flush = 0;
            }
        }
    }
    if (cur >= 0) flush_hist(T.hist_l, T.hist_g, a.n_bins);
}

// ---- 6. the tiled pairs: 64 consecutive targets of a class segment per
//         wavefront (RDF and kNN from LDS-staged neighbours); a target whose
//         k-th neighbour lies beyond the tile's certified radius is finished
//         by the one-target-per-wavefront search right away (kNN only)
// (at most 128 VGPRs: four wavefronts per SIMD against three, for two small spills)
template <int KMAX>
__global__ __launch_bounds__(kBlock, 4) void k_pair_batched_tile(BatchPairArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    const GridPlan P = *a.plan;
    const int RP = a.R * a.n_pairs;
    const uint64_t total = a.titems[RP];
    if (total == 0) return;
    const double vol = batch_volume(a, P);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int l = lane_id();
    PairTask T;
    T.n_bins = a.n_bins;
    T.r_enum = a.r_enum;
    T.thr2 = a.thr2;
    T.inv_w = a.inv_w;
    T.lo_b = a.delta_b;
    T.hi_b = 1.0f - a.delta_b;
    T.inv_w64 = a.inv_w64;
    T.E2 = a.E2;
    T.hist_l = reinterpret_cast<uint32_t*>(smem) + (size_t)w * hist_stride(a.n_bins);
    T.k = a.k;
    T.rknn = INFINITY;
    T.rknn2 = INFINITY;
    size_t off = ((size_t)kWavesPerBlock * hist_stride(a.n_bins) * 4u + 15) & ~size_t(15);
    float4* stage = reinterpret_cast<float4*>(smem + off) + (size_t)w * kStage;
    T.kbuf = reinterpret_cast<uint64_t*>(stage);      // used only after the tile pass
    for (int b = l; b < a.n_bins; b += kWave) T.hist_l[b] = 0;
    wave_sync();

    int cur = -1;
    uint32_t since_flush = 0;
    uint64_t seg_a0 = 0, seg_len = 0;
    float d_srf = 0.0f, Rk = 0.0f;
    int rp = 0;
    for (;;) {
        uint64_t g = 0;
        if (l == 0) g = atomicAdd((unsigned long long*)&a.work[1], 1ull);
        {
            const uint64_t b = __shfl((unsigned long long)g, 0, kWave);
            g = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32)) << 32) |
                (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
        }
        if (g >= total) break;
        {
            int lo = 0, hi = RP;      // titems[lo] <= g < titems[hi]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (a.titems[mid] <= g) lo = mid; else hi = mid;
            }
            rp = lo;
        }
        const int r = rp / a.n_pairs, p = rp % a.n_pairs;
        const BatchPair bp = a.pairs[p];
        if (rp != cur) {
            if (cur >= 0) {
                flush_hist(T.hist_l, T.hist_g, a.n_bins);
                since_flush = 0;
            }
            cur = rp;
            seg_a0 = seg_start(a.cnt, r, a.C, a.G, bp.a);
            seg_len = seg_end(a.cnt, r, a.C, a.G, bp.a, a.n) - seg_a0;
            const uint64_t b0 = seg_start(a.cnt, r, a.C, a.G, bp.b);
            const uint64_t b1 = seg_end(a.cnt, r, a.C, a.G, bp.b, a.n);
            T.bpos = a.Pp;
            T.cell_start = a.CS + ((size_t)r * (a.C - 1) + bp.b) * (size_t)a.cs_stride;
            T.rk0 = batch_rk0(P, vol, b1 - b0, a.k);
            Rk = fminf(tile_reach_rk0(a) * T.rk0, P.r_all);
            T.hist_g = a.rdf_hist + ((size_t)(a.rep0 + r) * a.n_pairs + p) * a.n_bins;
            d_srf = bp.d_srf;
        }
        const uint64_t slot = (g - a.titems[rp]) * kWave + (uint64_t)l;
        bool valid = slot < seg_len;
        uint32_t i = 0;
        float px = 0.0f, py = 0.0f, pz = 0.0f;
        if (valid) {
            const float4 rec = a.Pp[seg_a0 + slot];
            i = __builtin_bit_cast(uint32_t, rec.w);
            px = rec.x;
            py = rec.y;
            pz = rec.z;
            valid = a.d_bnd == nullptr || a.d_bnd[i] >= d_srf;
        }
        uint32_t hits = 0;
        const uint64_t kth = run_tile_kth<kRdfLds | kSelf, KMAX>(P, T, valid, px, py, pz, i, Rk, a.k, stage, hits);
        const bool fin = isfinite(px) && isfinite(py) && isfinite(pz);
        const bool certified = valid && (kth != ~0ull || !fin);
        uint64_t* kh = a.knn_hist ? a.knn_hist + ((size_t)(a.rep0 + r) * a.n_pairs + p) * (size_t)(a.kb_nbins + 1)
                                  : nullptr;
        if (kh && certified) {
            int b = a.kb_nbins;
            if (kth != ~0ull) b = key_bin(kth, a.xyz, px, py, pz, a.KE2, a.kb_nbins, a.kb_inv_w64);
            atomicAdd((unsigned long long*)&kh[b], 1ull);
        }
        // the rest: one target at a time over the whole wavefront
        uint64_t rest = __ballot(valid && !certified);
        while (rest) {
            const int ln = __builtin_ctzll(rest);
            rest &= rest - 1;
            const uint32_t ti = (uint32_t)__builtin_amdgcn_readlane((int)i, ln);
            const float tx = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, px), ln));
            const float ty = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, py), ln));
            const float tz = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, pz), ln));
            uint32_t h2 = 0;
            wave_sync();
            const int found = run_target<kSelf, true>(P, T, tx, ty, tz, ti, h2, false);
            if (kh && l == 0) {
                const int b = kth_bin(found, a.k, T.kbuf, a.xyz, tx, ty, tz, a.KE2, a.kb_nbins, a.kb_inv_w64);
                atomicAdd((unsigned long long*)&kh[b], 1ull);
            }
            wave_sync();
        }
        since_flush += wave_sum(hits);
        if (since_flush >= 0x7FFFFFFFu - (uint32_t)min((uint64_t)a.n * kWave, (uint64_t)0x7FFFFFFFu)) {
            flush_hist(T.hist_l, T.hist_g, a.n_bins);
            since_flush = 0;
        }
    }
    if (cur >= 0) flush_hist(T.hist_l, T.hist_g, a.n_bins);
}

template __global__ void k_pair_batched_tile<4>(BatchPairArgs);
template __global__ void k_pair_batched_tile<10>(BatchPairArgs);
template __global__ void k_pair_batched_tile<16>(BatchPairArgs);

}  // namespace apt
