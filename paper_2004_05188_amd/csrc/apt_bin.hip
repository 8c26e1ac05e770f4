// Cell binning of a point cloud on the GPU: bounding box and counts, the
// device-side grid plan, stable compaction of targets and neighbours, an LSD
// radix sort on uniform-grid cell ids, and the gather into coalesced SoA
// arrays with per-cell start offsets.
//
// The paper splits the cloud into regions with one array per ion type
// (Methods: "Spatial splitting"; Supplementary: "Effectiveness of the
// spatial splitting for heterogeneous datasets") and accelerates constant-
// time point queries with a regular binning (Supplementary: "Details on
// efficient spatial indices").  Here the regions are the cells of one
// uniform grid over the neighbour species, sorted so that each row of cells
// along x is one contiguous range of memory.
#include "apt_bin.hpp"

namespace apt {

// ------------------------------------------------------------------------
// 1. counts and the bounding box of the targets and neighbours.  Block b
//    owns ions [b*chunk, (b+1)*chunk), striped over threads for coalesced
//    loads.
// ------------------------------------------------------------------------
constexpr int kCountItems = 8;

__global__ __launch_bounds__(kBlock) void k_count(CountArgs a) {
    if (a.do_init) init_body(a.init, blockIdx.x * kBlock + threadIdx.x, gridDim.x * kBlock);
    const int64_t beg = (int64_t)blockIdx.x * a.chunk;
    int64_t end = beg + a.chunk;
    if (end > a.n) end = a.n;
    uint32_t nt = 0, nb = 0;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int nf = 0;
    const double sd = a.zscale ? *a.zscale : 1.0;
    // kCountItems labels per thread in flight (one at a time leaves the
    // kernel latency-bound)
    for (int64_t i0 = beg + threadIdx.x; i0 < end; i0 += (int64_t)kBlock * kCountItems) {
        uint8_t lb[kCountItems];
#pragma unroll
        for (int u = 0; u < kCountItems; ++u) {
            const int64_t i = i0 + (int64_t)u * kBlock;
            lb[u] = i < end ? a.lab[i] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kCountItems; ++u) {
            const int64_t i = i0 + (int64_t)u * kBlock;
            if (i >= end) continue;
            bool isT, isB;
            select_ion(lb[u], a.d_bnd, i, a.A, a.B, a.d_srf, a.sel_union, &isT, &isB);
            nt += isT;
            nb += isB;
            // the box of the ions the call bins (targets and neighbours); the
            // others' positions are never read
            if (!(isT || isB)) continue;
            float p[3] = {a.xyz[3 * i], a.xyz[3 * i + 1], a.xyz[3 * i + 2]};
            if (a.zscale) p[2] = (float)((double)p[2] * sd);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (isfinite(p[c])) {
                    lo[c] = fminf(lo[c], p[c]);
                    hi[c] = fmaxf(hi[c], p[c]);
                } else {
                    nf = 1;
                }
            }
        }
    }
    // block reduction through LDS
    __shared__ float s_lo[3][kWavesPerBlock], s_hi[3][kWavesPerBlock];
    __shared__ uint32_t s_nt[kWavesPerBlock], s_nb[kWavesPerBlock];
    __shared__ int s_nf[kWavesPerBlock];
    nt = wave_sum(nt);
    nb = wave_sum(nb);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            lo[c] = fminf(lo[c], __shfl_xor(lo[c], d, kWave));
            hi[c] = fmaxf(hi[c], __shfl_xor(hi[c], d, kWave));
        }
    nf = __any(nf) ? 1 : 0;
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) {
        for (int c = 0; c < 3; ++c) { s_lo[c][w] = lo[c]; s_hi[c][w] = hi[c]; }
        s_nt[w] = nt;
        s_nb[w] = nb;
        s_nf[w] = nf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < kWavesPerBlock; ++v) {
            for (int c = 0; c < 3; ++c) {
                s_lo[c][0] = fminf(s_lo[c][0], s_lo[c][v]);
                s_hi[c][0] = fmaxf(s_hi[c][0], s_hi[c][v]);
            }
            s_nt[0] += s_nt[v];
            s_nb[0] += s_nb[v];
            s_nf[0] |= s_nf[v];
        }
        float* pb = a.part_bbox + 6 * blockIdx.x;
        for (int c = 0; c < 3; ++c) { pb[c] = s_lo[c][0]; pb[3 + c] = s_hi[c][0]; }
        a.part_cnt[2 * blockIdx.x] = s_nt[0];
        a.part_cnt[2 * blockIdx.x + 1] = s_nb[0];
        a.part_nf[blockIdx.x] = s_nf[0];
    }
}

// ------------------------------------------------------------------------
// 2. plan: reduce the block partials, scan the counts, choose the grid.
// ------------------------------------------------------------------------
__device__ uint32_t block_excl_scan_1024(uint32_t v, uint32_t* tmp, uint32_t* total) {
    // 1024 threads = 16 wavefronts
    const int w = threadIdx.x / kWave, l = lane_id();
    uint32_t inc = wave_incl_scan(v);
    if (l == kWave - 1) tmp[w] = inc;
    __syncthreads();
    if (w == 0) {
        uint32_t x = l < 16 ? tmp[l] : 0u;
        uint32_t xs = wave_incl_scan(x);
        if (l < 16) tmp[16 + l] = xs - x;
        if (l == 15) tmp[32] = xs;
    }
    __syncthreads();
    uint32_t r = inc - v + tmp[16 + w];
    *total = tmp[32];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(1024) void k_plan(PlanArgs a) {
    __shared__ uint32_t tmp[64];
    __shared__ float s_box[6][16];
    __shared__ int s_nf[16];
    const int t = threadIdx.x, w = t / kWave;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int nf = 0;
    // thread t owns partials [t*per, (t+1)*per)
    const int per = (a.G + 1023) / 1024;
    const int b0 = t * per;
    const int b1 = min(b0 + per, a.G);
    uint32_t ct = 0, cb = 0;
    for (int b = b0; b < b1; ++b) {
        const float* pb = a.part_bbox + 6 * b;
        for (int c = 0; c < 3; ++c) { lo[c] = fminf(lo[c], pb[c]); hi[c] = fmaxf(hi[c], pb[3 + c]); }
        nf |= a.part_nf[b];
        ct += a.part_cnt[2 * b];
        cb += a.part_cnt[2 * b + 1];
    }
    uint32_t totT, totB;
    uint32_t ot = block_excl_scan_1024(ct, tmp, &totT);
    uint32_t ob = block_excl_scan_1024(cb, tmp, &totB);
    for (int b = b0; b < b1; ++b) {
        a.part_off[2 * b] = ot;
        a.part_off[2 * b + 1] = ob;
        ot += a.part_cnt[2 * b];
        ob += a.part_cnt[2 * b + 1];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            lo[c] = fminf(lo[c], __shfl_xor(lo[c], d, kWave));
            hi[c] = fmaxf(hi[c], __shfl_xor(hi[c], d, kWave));
        }
    nf = __any(nf) ? 1 : 0;
    if (lane_id() == 0) {
        for (int c = 0; c < 3; ++c) { s_box[c][w] = lo[c]; s_box[3 + c][w] = hi[c]; }
        s_nf[w] = nf;
    }
    __syncthreads();
    if (t != 0) return;
    for (int v = 1; v < 16; ++v)
        for (int c = 0; c < 3; ++c) {
            s_box[c][0] = fminf(s_box[c][0], s_box[c][v]);
            s_box[3 + c][0] = fmaxf(s_box[3 + c][0], s_box[3 + c][v]);
            s_nf[0] |= s_nf[v];
        }
    GridPlan P;
    double ext[3];
    double amax = 0.0;
    for (int c = 0; c < 3; ++c) {
        float l = s_box[c][0], h = s_box[3 + c][0];
        if (!(l <= h)) { l = 0.0f; h = 0.0f; }    // no finite position at all
        P.lo[c] = l;
        P.hi[c] = h;
        ext[c] = (double)h - (double)l;          // exact-ish, never overflows in FP64
        amax = fmax(amax, fmax(fabs((double)l), fabs((double)h)));
    }
    const PlanParams& pp = a.pp;
    double vol = 1.0;
    for (int c = 0; c < 3; ++c) vol *= fmax(ext[c], 1e-3);
    const double rho = (double)(totB > 0 ? totB : 1) / vol;
    const double emax = fmax(ext[0], fmax(ext[1], ext[2]));
    // the Poisson mean k-th neighbour distance with a margin: the first kNN
    // search radius (clamped to the cloud's diagonal below)
    const double rk_raw = pp.k > 0 ? 1.15 * cbrt(3.0 * ((double)pp.k + 0.5) / (4.0 * M_PI * rho)) : 0.0;
    // 64 consecutive targets (cell order) per wavefront when the targets are at
    // least as dense as the neighbours; their kNN is certified within rk_tile
    // (one target per lane, mode 2, only when asked for: on the sparse needle
    // queries its lanes' serial walks were no faster than one target per
    // wavefront)
    if (pp.tile_policy == 1) P.tile_mode = 0;
    else if (pp.tile_policy == 2) P.tile_mode = pp.k <= 16 ? 1 : 0;
    else if (pp.tile_policy == 3) P.tile_mode = pp.k <= 16 ? 2 : 0;
    else if (pp.tile_policy == 4) P.tile_mode = (pp.k <= 16 && (pp.k >= 1 || pp.r_enum > 0.0f)) ? 3 : 0;
    else {
        // a tile pays when its 64 targets fill a region no larger than the
        // search reach, so that they share most of their candidates
        const double R = fmax((double)pp.r_enum, 1.6 / 1.15 * rk_raw);
        const double v64 = 64.0 * vol / (double)(totT > 0 ? totT : 1);
        P.tile_mode = (pp.k <= 16 && totT >= totB && totT >= 4096 && v64 <= R * R * R) ? 1 : 0;
        // neighbours so dense that 64 of them span well under r_max: the RDF
        // runs neighbour-major (64 records per wavefront against every target
        // within reach), and the kNN, whose radius is then well below r_max,
        // one target per lane among a few dozen records.  Only for 2^18
        // targets or more: with fewer, the per-lane kNN fills under four
        // wavefronts per SIMD and every neighbour chunk is still visited
        // (the 7.7e6-ion needle's 74 000 Sc targets against Al: 0.59 ms
        // against 0.40 ms one target per wavefront)
        const double a64 = cbrt(64.0 / rho);
        if (!P.tile_mode && pp.k <= 16 && pp.r_enum > 0.0f && a64 <= (double)pp.r_enum && totT >= (1u << 18) &&
            (pp.k == 0 || rk_raw <= 0.5 * (double)pp.r_enum))
            P.tile_mode = 3;
    }
    // cell edge: at least h_min, and large enough to hold ~occ neighbours
    // (tiles gather every candidate of their 64 targets: smaller cells pay;
    // in mode 3 the RDF enumeration sets the cell size)
    const bool tiles = P.tile_mode == 1 || P.tile_mode == 2;
    const double occ = (tiles && pp.tile_occ > 0.0f) ? (double)pp.tile_occ : (double)pp.occ;
    double h = fmax((double)pp.h_min, cbrt(occ / rho));
    if (totB == 0 || !(h > 0.0)) h = emax + 1.0;
    if (h < 1e-6 * (emax + 1.0)) h = 1e-6 * (emax + 1.0);
    if (h > 3.0e38) h = 3.0e38;
    for (;;) {
        // the cell count with the FP32 edge actually used
        const double hf = (double)(float)h;
        double cells = 1.0;
        for (int c = 0; c < 3; ++c) cells *= floor(ext[c] / hf) + 1.0;
        if (cells <= (double)pp.cell_cap || h >= 3.0e38) break;
        h = fmin(h * 1.25, 3.0e38);               // finite ext: terminates
    }
    // a smaller edge culls more candidates per target (on the 2e9-ion
    // needle the pair kernel took 10 % less time at 0.7x the edge); take it
    // for large neighbour sets (below 2^25 neighbours the finer grid's
    // binning cost more than it saved: +2 % on the 7.7e6-ion needle) when
    // its cell ids need no more radix passes (at 2e8 ions the extra pass
    // cost more).  Not in mode 3: there the neighbour-major RDF and the
    // binning of fewer cells gain more at the larger edge than the per-lane
    // kNN loses (2e9-ion needle, Sc -> any: 189 ms per step at 1.0 nm, 196
    // ms at 0.7 nm)
    if (pp.h_shrink > 0.0f && !tiles && P.tile_mode != 3 && totB >= (1u << 25) && h < 3.0e38) {
        const double h2 = fmax((double)pp.h_min * (double)pp.h_shrink, cbrt(occ / rho));
        if (h2 < h && h2 >= 1e-6 * (emax + 1.0)) {
            auto cells_of = [&](double hh) {
                const double hf = (double)(float)hh;
                double c = 1.0;
                for (int ax = 0; ax < 3; ++ax) c *= floor(ext[ax] / hf) + 1.0;
                return c;
            };
            // (both counts are at most cell_cap here: exact in u64)
            const double c1 = cells_of(h), c2 = cells_of(h2);
            if (c2 <= (double)pp.cell_cap &&
                sort_passes_for((uint64_t)c2 - 1u) == sort_passes_for((uint64_t)c1 - 1u))
                h = h2;
        }
    }
    P.h = (float)h;
    P.inv_h = (float)(1.0 / (double)P.h);
    uint64_t ncell = 1;
    for (int c = 0; c < 3; ++c) {
        P.dim[c] = (int32_t)(floor(ext[c] / (double)P.h) + 1.0);
        ncell *= (uint64_t)P.dim[c];
    }
    P.n_cells = (uint32_t)ncell;
    P.nT = totT;
    P.nB = totB;
    const uint32_t passes = (uint32_t)sort_passes_for(P.n_cells - 1u);
    P.passes = passes;
    P.bits = key_bits(P.n_cells - 1u);
    // targets in block-raster order when its keys fit 32 bits and need no
    // more passes than the largest cell id the workspace allows (the radix
    // passes launched for both sorts), else in cell order
    {
        const uint64_t nbx = ((uint64_t)P.dim[0] + 7) / 8, nby = ((uint64_t)P.dim[1] + 7) / 8,
                       nbz = ((uint64_t)P.dim[2] + 7) / 8;
        const uint64_t kmax = nbx * nby * nbz * 512u - 1u;
        const int cap_passes = sort_passes_for(pp.cell_cap - 1u);
        // (mode 3 looks targets up by cell: plain cell order)
        if (P.tile_mode != 3 && kmax <= 0xFFFFFFFFull && sort_passes_for(kmax) <= cap_passes) {
            P.tblock = 8;
            P.nbx = (int32_t)nbx;
            P.nby = (int32_t)nby;
            P.passes_T = (uint32_t)sort_passes_for(kmax);
            P.bits_T = key_bits(kmax);
        } else {
            P.tblock = 1;
            P.nbx = P.nby = 0;
            P.passes_T = passes;
            P.bits_T = P.bits;
        }
    }
    // (x - lo) * inv_h in FP32 misplaces a point by at most ~3 ulps of the
    // extent; cull with a margin well above that
    P.eps = (float)fmin(fmax(1e-5, 8.0 * 5.9604645e-8 * (emax + amax)), 3.0e38);
    const double hd = (double)P.h;
    const double diag = sqrt((ext[0] + hd) * (ext[0] + hd) + (ext[1] + hd) * (ext[1] + hd) +
                             (ext[2] + hd) * (ext[2] + hd));
    P.r_all = (float)fmin(diag + 2.0 * hd, 3.0e38);
    P.rk0 = pp.k > 0 ? (float)fmin(rk_raw, (double)P.r_all) : 0.0f;
    P.zscale = a.zscale ? (float)*a.zscale : 1.0f;
    P.nonfinite = s_nf[0];
    P.rk_tile = pp.k > 0 ? (float)fmin((P.tile_mode == 3 ? 1.3 : 1.6) / 1.15 * (double)P.rk0, (double)P.r_all)
                         : 0.0f;
    P.rdf_nbr = (P.tile_mode == 3 && pp.rdf_kernel != 2) ? 1 : 0;
    *a.plan = P;
    if (s_nf[0] && a.status) atomicOr(a.status, APT_STATUS_NONFINITE);
}

// ------------------------------------------------------------------------
// 3. stable compaction of target and neighbour indices
// ------------------------------------------------------------------------
constexpr int kCompactItems = 16;
constexpr int kCompactTile = kBlock * kCompactItems;

// The sort keys of the ions one tile of k_compact selected: targets
// [t0, t1) and neighbours [b0, b1) of the lists (contiguous: the compaction
// is stable), or every ion of [i0, i1) when the neighbours are all ions.
__device__ __forceinline__ void compact_keys(const CompactArgs& a, uint32_t t0, uint32_t t1, uint32_t b0, uint32_t b1,
                                              int64_t i0, int64_t i1) {
    const GridPlan P = *a.plan;
    const double sd = a.zscale ? *a.zscale : 1.0;
    constexpr int U = 4;   // list entries and positions in flight per thread
    // ion ids of list entries [j0, j0 + U * kBlock) of `list` (NULL: the
    // entries are the ions themselves), their positions, then f(j, id, x, y, z)
    auto run = [&](const uint32_t* list, int64_t j0, int64_t j1, auto&& f) {
        for (int64_t jb = j0 + threadIdx.x; jb < j1; jb += (int64_t)U * kBlock) {
            uint32_t id[U];
            float x[U], y[U], z[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t j = jb + (int64_t)u * kBlock;
                id[u] = j < j1 ? (list ? list[j] : (uint32_t)j) : 0u;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (jb + (int64_t)u * kBlock < j1) {
                    x[u] = a.xyz[3 * (size_t)id[u]];
                    y[u] = a.xyz[3 * (size_t)id[u] + 1];
                    z[u] = a.xyz[3 * (size_t)id[u] + 2];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t j = jb + (int64_t)u * kBlock;
                if (j < j1) {
                    const float zz = a.zscale ? (float)((double)z[u] * sd) : z[u];
                    f((uint32_t)j, id[u], x[u], y[u], zz);
                }
            }
        }
    };
    run(a.tid, t0, t1, [&](uint32_t j, uint32_t, float x, float y, float z) {
        a.tkeys[j] = target_key(P, x, y, z);
        a.tvals[j] = j;
    });
    float4* __restrict__ brec = rec_after(a.brec[0], a.brec[1], (int)P.passes, -1);
    auto bkey = [&](uint32_t j, uint32_t id, float x, float y, float z) {
        a.bkeys[j] = cell_id(P, x, y, z);
        brec[j] = make_float4(x, y, z, __builtin_bit_cast(float, id));
    };
    if (a.bsel) run(a.bsel, b0, b1, bkey);
    else run(nullptr, i0, i1, bkey);   // neighbours = every ion, in index order
}

// (at most 64 VGPRs: eight wavefronts per SIMD for the streaming reads)
__global__ __launch_bounds__(kBlock, 8) void k_compact(CompactArgs a) {
    __shared__ uint32_t s_cnt[2][kCompactItems][kWavesPerBlock];
    __shared__ uint32_t s_base[2][kCompactItems][kWavesPerBlock];
    __shared__ uint32_t s_run[2];
    const int w = threadIdx.x / kWave;
    const int64_t beg = (int64_t)blockIdx.x * a.chunk;
    int64_t end = beg + a.chunk;
    if (end > a.n) end = a.n;
    if (threadIdx.x == 0) {
        s_run[0] = a.part_off[2 * blockIdx.x];
        s_run[1] = a.part_off[2 * blockIdx.x + 1];
    }
    __syncthreads();
    for (int64_t tile = beg; tile < end; tile += kCompactTile) {
        uint64_t mt[kCompactItems], mb[kCompactItems];
#pragma unroll
        for (int it = 0; it < kCompactItems; ++it) {
            const int64_t i = tile + (int64_t)it * kBlock + threadIdx.x;
            bool isT = false, isB = false;
            if (i < end) {
                select_ion(a.lab[i], a.d_bnd, i, a.A, a.B, a.d_srf, a.sel_union, &isT, &isB);
                isB = isB && a.bsel != nullptr;
            }
            mt[it] = __ballot(isT);
            mb[it] = __ballot(isB);
            if (lane_id() == 0) {
                s_cnt[0][it][w] = __popcll(mt[it]);
                s_cnt[1][it][w] = __popcll(mb[it]);
            }
        }
        __syncthreads();
        if (threadIdx.x < kWave) {
            // exclusive scan over (item, wave) in index order, for both lists
            const int l = lane_id();
            for (int q = 0; q < 2; ++q) {
                uint32_t x = s_cnt[q][l / kWavesPerBlock][l % kWavesPerBlock];
                uint32_t xs = wave_incl_scan(x);
                s_base[q][l / kWavesPerBlock][l % kWavesPerBlock] = xs - x + s_run[q];
                uint32_t tot = readlane(xs, kWave - 1);
                wave_sync();
                if (l == 0) s_run[q] += tot;
            }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kCompactItems; ++it) {
            const int64_t i = tile + (int64_t)it * kBlock + threadIdx.x;
            const uint64_t bit = 1ull << lane_id();
            if (mt[it] & bit) a.tid[s_base[0][it][w] + __popcll(mt[it] & lanemask_lt())] = (uint32_t)i;
            if (mb[it] & bit) a.bsel[s_base[1][it][w] + __popcll(mb[it] & lanemask_lt())] = (uint32_t)i;
        }
        __syncthreads();   // the tile's list entries are visible to the whole workgroup
        if (a.tkeys) {
            const int64_t te = tile + kCompactTile < end ? tile + kCompactTile : end;
            compact_keys(a, s_base[0][0][0], s_run[0], s_base[1][0][0], s_run[1], tile, te);
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------------
// 4. cell keys
// ------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_keys(KeyArgs a) {
    const GridPlan P = *a.plan;
    const uint32_t n = a.count_is_T ? P.nT : P.nB;
    const double sd = a.zscale ? *a.zscale : 1.0;
    for (uint32_t j = blockIdx.x * kBlock + threadIdx.x; j < n; j += gridDim.x * kBlock) {
        const uint32_t id = a.src ? a.src[j] : j;
        float x = a.xyz[3 * (size_t)id], y = a.xyz[3 * (size_t)id + 1], z = a.xyz[3 * (size_t)id + 2];
        if (a.zscale) z = (float)((double)z * sd);
        a.keys[j] = a.count_is_T ? target_key(P, x, y, z) : cell_id(P, x, y, z);
        a.vals[j] = a.val_is_index ? j : id;
    }
}

// ------------------------------------------------------------------------
// 5. LSD radix sort of (cell id, value) pairs, kDigitBits per pass, stable.
//    Block b sorts its chunk tile by tile; digits of a tile are ranked
//    inside each wavefront with ballots, then placed through LDS so that
//    the global writes of one digit are contiguous.
// ------------------------------------------------------------------------
constexpr int kRsUp = 8;                     // keys per thread in flight in the upsweep
constexpr int kGatherItems = 4;              // random position reads per thread in flight
constexpr int kOrderItems = 2;               // the same for the (fewer) targets

__device__ __forceinline__ bool rs_active(const GridPlan& P, const SortArgs& a) {
    return (uint32_t)a.pass < (a.count_is_T ? P.passes_T : P.passes);
}

// The workgroup's sort, taken from the argument set with selects: indexing
// the array with a run-time value copies it to private memory, and every
// pointer read back from there becomes a flat one, whose loads the LDS waits
// of the ranking then also wait for.
__device__ __forceinline__ SortArgs sort_of(const SortSet& set, int q) {
    const SortArgs& s0 = set.s[0];
    const SortArgs& s1 = set.s[1];
    SortArgs a;
    a.plan = q ? s1.plan : s0.plan;
    a.count_is_T = q ? s1.count_is_T : s0.count_is_T;
    a.pass = q ? s1.pass : s0.pass;
    a.G = q ? s1.G : s0.G;
    a.keys[0] = q ? s1.keys[0] : s0.keys[0];
    a.keys[1] = q ? s1.keys[1] : s0.keys[1];
    a.vals[0] = q ? s1.vals[0] : s0.vals[0];
    a.vals[1] = q ? s1.vals[1] : s0.vals[1];
    a.counts = q ? s1.counts : s0.counts;
    a.totals = q ? s1.totals : s0.totals;
    a.rec[0] = q ? s1.rec[0] : s0.rec[0];
    a.rec[1] = q ? s1.rec[1] : s0.rec[1];
    return a;
}

template <typename T>
__device__ __forceinline__ T pick2(T p0, T p1, uint32_t bit) { return (bit & 1u) ? p1 : p0; }

// workgroup b of G sorts keys [b chunk, (b + 1) chunk): whole tiles
__device__ __forceinline__ void rs_chunk(uint32_t n, int G, uint32_t tile, uint32_t* chunk) {
    uint32_t c = (n + (uint32_t)G - 1u) / (uint32_t)G;
    *chunk = (c + tile - 1u) / tile * tile;
}

__global__ __launch_bounds__(kBlock) void k_rs_upsweep(SortSet set) {
    // sort 0 takes the first s[0].G workgroups, sort 1 the next s[1].G
    const uint32_t g0 = (uint32_t)set.s[0].G;
    const int q = blockIdx.x < g0 ? 0 : 1;
    if (q >= set.n) return;
    const SortArgs a = sort_of(set, q);
    const uint32_t bid = blockIdx.x - (q ? g0 : 0u);
    if (bid >= (uint32_t)a.G) return;
    const GridPlan P = *a.plan;
    if (!rs_active(P, a)) return;
    const uint32_t n = a.count_is_T ? P.nT : P.nB;
    const uint32_t* __restrict__ keys = pick2(a.keys[0], a.keys[1], (uint32_t)a.pass);
    __shared__ uint32_t s_h[kWavesPerBlock][kRadix];
    for (int i = threadIdx.x; i < kWavesPerBlock * kRadix; i += kBlock) (&s_h[0][0])[i] = 0;
    __syncthreads();
    uint32_t chunk;
    rs_chunk(n, a.G, (uint32_t)set.tile, &chunk);
    const uint64_t beg = (uint64_t)bid * chunk;
    uint64_t end = beg + chunk;
    if (end > n) end = n;
    const int w = threadIdx.x / kWave;
    uint32_t shift, mask;
    pass_digit(a.count_is_T ? P.bits_T : P.bits, a.count_is_T ? P.passes_T : P.passes, (uint32_t)a.pass, &shift,
               &mask);
    // kRsUp independent coalesced loads in flight per thread before the
    // LDS counts (one load at a time leaves the pass latency-bound)
    for (uint64_t i0 = beg + threadIdx.x; i0 < end; i0 += (uint64_t)kBlock * kRsUp) {
        uint32_t k[kRsUp];
#pragma unroll
        for (int u = 0; u < kRsUp; ++u) {
            const uint64_t i = i0 + (uint64_t)u * kBlock;
            k[u] = i < end ? keys[i] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kRsUp; ++u)
            if (i0 + (uint64_t)u * kBlock < end) atomicAdd(&s_h[w][(k[u] >> shift) & mask], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kRadix; d += kBlock) {
        uint32_t s = 0;
        for (int v = 0; v < kWavesPerBlock; ++v) s += s_h[v][d];
        a.counts[(size_t)d * a.G + bid] = s;
    }
}

// Row scan of the digit counts: workgroup d turns counts[d][0..G) into
// exclusive prefixes within the row and writes the row total to totals[d].
// The downsweep adds the digit bases (a scan of the kRadix totals).
__global__ __launch_bounds__(kBlock) void k_rs_scan(SortSet set) {
    const int q = blockIdx.x / kRadix;
    if (q >= set.n) return;
    const SortArgs a = sort_of(set, q);
    const GridPlan P = *a.plan;
    if (!rs_active(P, a)) return;
    __shared__ uint32_t s_w[kWavesPerBlock];
    const int d = blockIdx.x - q * kRadix, t = threadIdx.x, w = t / kWave, l = lane_id();
    const int G = a.G;
    const int per = (G + kBlock - 1) / kBlock;    // G <= 4096: at most 16 per thread
    uint32_t v[16];
    uint32_t sum = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int b = t * per + q;
        v[q] = (q < per && b < G) ? a.counts[(size_t)d * G + b] : 0u;
        sum += v[q];
    }
    const uint32_t inc = wave_incl_scan(sum);
    if (l == kWave - 1) s_w[w] = inc;
    __syncthreads();
    uint32_t run = inc - sum;
    for (int u = 0; u < w; ++u) run += s_w[u];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int b = t * per + q;
        if (q < per && b < G) a.counts[(size_t)d * G + b] = run;
        run += v[q];
    }
    if (t == kBlock - 1) a.totals[d] = run;
}

// LDS of one downsweep workgroup of BLOCK threads, ITEMS keys each
template <int BLOCK, int ITEMS>
struct DownLds {
    uint32_t key[BLOCK * ITEMS];
    float4 pay[BLOCK * ITEMS];           // values (as u32) or records
    uint32_t wcnt[BLOCK / kWave][kRadix];
    uint32_t lstart[kRadix];
    uint32_t tot[kRadix];
    uint32_t run[kRadix];
    uint32_t tmp[16];
};

// One workgroup's tiles: keys ranked by digit with ballots per wavefront,
// placed through LDS with their payload (a 4-byte value, or a 16-byte
// record) so that each digit's run leaves as one contiguous write.  The
// next tile's keys are loaded while this one is ranked and written; the
// payloads are loaded at the start of their own tile and wait in registers
// through the ranking (loading them a tile ahead too took the registers of
// three more keys per thread and was no faster).
template <class PAY, int BLOCK, int ITEMS>
__device__ __forceinline__ void downsweep_tiles(uint64_t beg, uint64_t end, uint32_t shift, uint32_t mask,
                                                const uint32_t* __restrict__ kin, uint32_t* __restrict__ kout,
                                                const PAY* __restrict__ pin, PAY* __restrict__ pout,
                                                DownLds<BLOCK, ITEMS>& S) {
    constexpr int kRsItems = ITEMS, kDsBlock = BLOCK, kDsWaves = BLOCK / kWave, kRsTile = BLOCK * ITEMS;
    const int t = threadIdx.x, w = t / kWave, l = lane_id();
    PAY* s_pay = reinterpret_cast<PAY*>(S.pay);
    uint32_t nkey[kRsItems];
    auto load_keys = [&](uint64_t tile) {
#pragma unroll
        for (int j = 0; j < kRsItems; ++j) {
            const uint64_t i = tile + (uint64_t)w * (kRsItems * kWave) + (uint64_t)j * kWave + l;
            nkey[j] = i < end ? kin[i] : 0u;
        }
    };
    if (beg < end) load_keys(beg);
    for (uint64_t tile = beg; tile < end; tile += kRsTile) {
        uint32_t key[kRsItems], pos[kRsItems];
        PAY pay[kRsItems];
        bool ok[kRsItems];
#pragma unroll
        for (int j = 0; j < kRsItems; ++j) {
            key[j] = nkey[j];
            const uint64_t i = tile + (uint64_t)w * (kRsItems * kWave) + (uint64_t)j * kWave + l;
            pay[j] = i < end ? pin[i] : PAY{};
        }
        if (tile + kRsTile < end) load_keys(tile + kRsTile);
        for (int i = t; i < kDsWaves * kRadix; i += kDsBlock) (&S.wcnt[0][0])[i] = 0;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kRsItems; ++j) {
            const uint64_t i = tile + (uint64_t)w * (kRsItems * kWave) + (uint64_t)j * kWave + l;
            ok[j] = i < end;
            const uint32_t d = (key[j] >> shift) & mask;
            uint64_t peers = __ballot(ok[j]);
#pragma unroll
            for (int bit = 0; bit < kDigitBits; ++bit) {
                const uint64_t b = __ballot((d >> bit) & 1u);
                peers &= ((d >> bit) & 1u) ? b : ~b;
            }
            const uint32_t before = S.wcnt[w][d];
            wave_sync();
            pos[j] = before + (uint32_t)__popcll(peers & lanemask_lt());
            if (ok[j] && (peers & lanemask_lt()) == 0) S.wcnt[w][d] = before + (uint32_t)__popcll(peers);
            wave_sync();
        }
        __syncthreads();
        // per-digit totals of the tile and wave prefixes
        uint32_t tot = 0;
        for (int d = t; d < kRadix; d += kDsBlock) {
            uint32_t acc = 0;
            for (int v = 0; v < kDsWaves; ++v) {
                const uint32_t c = S.wcnt[v][d];
                S.wcnt[v][d] = acc;
                acc += c;
            }
            S.tot[d] = acc;
            tot = acc;
        }
        // exclusive scan of the digit totals (thread t < kRadix: digit t)
        {
            uint32_t inc = wave_incl_scan(tot);
            if (l == kWave - 1) S.tmp[w] = inc;
            __syncthreads();
            uint32_t add = 0;
            for (int v = 0; v < w; ++v) add += S.tmp[v];
            if (t < kRadix) S.lstart[t] = inc - tot + add;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kRsItems; ++j) {
            if (ok[j]) {
                const uint32_t d = (key[j] >> shift) & mask;
                const uint32_t lp = S.lstart[d] + S.wcnt[w][d] + pos[j];
                S.key[lp] = key[j];
                s_pay[lp] = pay[j];
            }
        }
        __syncthreads();
        const uint32_t cnt = (uint32_t)((end - tile) < (uint64_t)kRsTile ? (end - tile) : kRsTile);
#pragma unroll
        for (int j = 0; j < kRsItems; ++j) {
            const uint32_t idx = (uint32_t)(j * kDsBlock + t);
            if (idx < cnt) {
                const uint32_t k = S.key[idx];
                const uint32_t d = (k >> shift) & mask;
                const uint32_t g = S.run[d] + (idx - S.lstart[d]);
                kout[g] = k;
                pout[g] = s_pay[idx];
            }
        }
        __syncthreads();
        for (int d = t; d < kRadix; d += kDsBlock) S.run[d] += S.tot[d];
        __syncthreads();
    }
}

template <int BLOCK, int ITEMS>
__device__ __forceinline__ void downsweep_body(const SortSet& set) {
    // sort 0 takes the first s[0].G workgroups, sort 1 the next s[1].G
    const uint32_t g0 = (uint32_t)set.s[0].G;
    const int q = blockIdx.x < g0 ? 0 : 1;
    if (q >= set.n) return;
    const SortArgs a = sort_of(set, q);
    const uint32_t bid = blockIdx.x - (q ? g0 : 0u);
    if (bid >= (uint32_t)a.G) return;
    const GridPlan P = *a.plan;
    if (!rs_active(P, a)) return;
    const uint32_t n = a.count_is_T ? P.nT : P.nB;
    const uint32_t* __restrict__ kin = pick2(a.keys[0], a.keys[1], (uint32_t)a.pass);
    uint32_t* __restrict__ kout = pick2(a.keys[0], a.keys[1], (uint32_t)a.pass + 1u);
    uint32_t shift, mask;
    pass_digit(a.count_is_T ? P.bits_T : P.bits, a.count_is_T ? P.passes_T : P.passes, (uint32_t)a.pass, &shift,
               &mask);

    __shared__ DownLds<BLOCK, ITEMS> S;

    uint32_t chunk;
    rs_chunk(n, a.G, (uint32_t)(BLOCK * ITEMS), &chunk);
    const uint64_t beg = (uint64_t)bid * chunk;
    uint64_t end = beg + chunk;
    if (end > n) end = n;
    const int t = threadIdx.x, w = t / kWave, l = lane_id();
    {
        // digit base = sum of the totals of the smaller digits (thread t < kRadix: digit t)
        const uint32_t tot_d = t < kRadix ? a.totals[t] : 0u;
        const uint32_t inc = wave_incl_scan(tot_d);
        if (l == kWave - 1) S.tmp[w] = inc;
        __syncthreads();
        uint32_t base = inc - tot_d;
        for (int v = 0; v < w; ++v) base += S.tmp[v];
        if (t < kRadix) S.run[t] = base + a.counts[(size_t)t * a.G + bid];
    }
    __syncthreads();
    if (a.rec[0]) {
        const int passes = a.count_is_T ? (int)P.passes_T : (int)P.passes;
        downsweep_tiles<float4>(beg, end, shift, mask, kin, kout, rec_after(a.rec[0], a.rec[1], passes, a.pass - 1),
                                rec_after(a.rec[0], a.rec[1], passes, a.pass), S);
    } else {
        downsweep_tiles<uint32_t>(beg, end, shift, mask, kin, kout, pick2(a.vals[0], a.vals[1], (uint32_t)a.pass),
                                  pick2(a.vals[0], a.vals[1], (uint32_t)a.pass + 1u), S);
    }
}

// (each kernel runs only with the tile its upsweep cut the chunks for)
__global__ __launch_bounds__(kDsLargeBlock) void k_rs_downsweep_large(SortSet set) {
    if (set.tile != kDsLargeBlock * kDsLargeItems) return;
    downsweep_body<kDsLargeBlock, kDsLargeItems>(set);
}

__global__ __launch_bounds__(kDsSmallBlock) void k_rs_downsweep_small(SortSet set) {
    if (set.tile != kDsSmallBlock * kDsSmallItems) return;
    downsweep_body<kDsSmallBlock, kDsSmallItems>(set);
}

// ------------------------------------------------------------------------
// 6. targets in cell order as SoA: rank, ion index, position
// ------------------------------------------------------------------------
__device__ __forceinline__ void take_order(const OrderArgs& a, uint32_t bid, uint32_t nblk) {
    const GridPlan P = *a.plan;
    const uint32_t* __restrict__ v = a.vals[P.passes_T & 1];
    const uint32_t* __restrict__ sk = a.keys[P.passes_T & 1];   // sorted target keys
    const uint64_t nT = P.nT, stride = (uint64_t)nblk * kBlock;
    uint32_t distinct = 0;
    uint32_t* tcs = P.tile_mode == 3 ? a.t_cell_start : nullptr;
    if (tcs && nT == 0)
        for (uint64_t c = (uint64_t)bid * kBlock + threadIdx.x; c <= P.n_cells; c += stride) tcs[c] = 0;
    // kOrderItems targets per thread in flight: the position reads are random
    for (uint64_t t0 = (uint64_t)bid * kBlock + threadIdx.x; t0 < nT; t0 += stride * kOrderItems) {
        uint32_t rank[kOrderItems], id[kOrderItems];
        float x[kOrderItems], y[kOrderItems], z[kOrderItems];
#pragma unroll
        for (int u = 0; u < kOrderItems; ++u) {
            const uint64_t t = t0 + (uint64_t)u * stride;
            rank[u] = t < nT ? v[t] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kOrderItems; ++u) id[u] = t0 + (uint64_t)u * stride < nT ? a.tid[rank[u]] : 0u;
#pragma unroll
        for (int u = 0; u < kOrderItems; ++u) {
            if (t0 + (uint64_t)u * stride < nT) {
                x[u] = a.xyz[3 * (size_t)id[u]];
                y[u] = a.xyz[3 * (size_t)id[u] + 1];
                z[u] = a.xyz[3 * (size_t)id[u] + 2];
            }
        }
#pragma unroll
        for (int u = 0; u < kOrderItems; ++u) {
            const uint64_t t = t0 + (uint64_t)u * stride;
            if (t < nT) {
                a.t_rank[t] = rank[u];
                a.t_id[t] = id[u];
                a.tx[t] = x[u];
                a.ty[t] = y[u];
                a.tz[t] = z[u];
                if (a.distinct) distinct += (t == 0 || sk[t] != sk[t - 1]) ? 1u : 0u;
            }
            if (tcs) {
                // plain cell order (the key is the cell id): target t starts
                // the cells (key[t-1], key[t]]; the last one also ends the
                // rest.  Long runs (sparse targets) are filled by the whole
                // wavefront, so that no lane writes millions of entries.
                uint32_t q0 = 0, q1 = 0;   // cells [q0, q1) take value t (then nT for the tail)
                uint32_t e0 = 0, e1 = 0;
                if (t < nT) {
                    const uint32_t c = sk[t];
                    q0 = t == 0 ? 0u : sk[t - 1] + 1u;
                    q1 = c + 1u;
                    if (t == nT - 1) {
                        e0 = c + 1u;
                        e1 = P.n_cells + 1u;
                    }
                }
                auto fill = [&](uint32_t f0, uint32_t f1, uint32_t val) {
                    if (f1 - f0 <= 32u) {
                        for (uint32_t q = f0; q < f1; ++q) tcs[q] = val;
                        f1 = f0;
                    }
                    // (lanes past the end of the loop are inactive: stride by
                    // the active lanes)
                    const uint64_t act = __ballot(true);
                    const uint32_t nact = (uint32_t)__popcll(act);
                    const uint32_t me = (uint32_t)__popcll(act & lanemask_lt());
                    uint64_t m = __ballot(f1 > f0);
                    while (m) {
                        const int ln = __builtin_ctzll(m);
                        m &= m - 1;
                        const uint32_t g0 = (uint32_t)__shfl((int)f0, ln, kWave);
                        const uint32_t g1 = (uint32_t)__shfl((int)f1, ln, kWave);
                        const uint32_t gv = (uint32_t)__shfl((int)val, ln, kWave);
                        for (uint32_t q = g0 + me; q < g1; q += nact) tcs[q] = gv;
                    }
                };
                fill(q0, q1, (uint32_t)t);
                fill(e0, e1, (uint32_t)nT);
            }
        }
    }
    if (a.distinct) {
        distinct = wave_sum(distinct);
        if (lane_id() == 0 && distinct) atomicAdd(a.distinct, distinct);
    }
}

// ------------------------------------------------------------------------
// 7. gather into 16-byte records (x, y, z, index) and cell start offsets
// ------------------------------------------------------------------------
__device__ __forceinline__ void gather(const GatherArgs& a, uint32_t bid, uint32_t nblk) {
    const GridPlan P = *a.plan;
    const uint32_t* __restrict__ key = a.keys[P.passes & 1];
    const uint32_t* __restrict__ val = a.vals[P.passes & 1];
    const uint32_t nB = P.nB, nc = P.n_cells;
    const double sd = a.zscale ? *a.zscale : 1.0;
    const uint32_t stride = nblk * kBlock;
    if (nB == 0) {
        for (uint32_t c = bid * kBlock + threadIdx.x; c <= nc; c += stride) a.cell_start[c] = 0;
        return;
    }
    const uint64_t st64 = stride;
    uint32_t distinct = 0;
    if (!a.xyz) {
        // the records are in place: cell offsets from the sorted keys only,
        // eight consecutive keys per thread (two 16-byte loads and the key
        // before them)
        constexpr uint32_t kRun = 8;
        const uint64_t n_runs = ((uint64_t)nB + kRun - 1) / kRun;
        // (every lane of a wavefront takes the same iterations: the long
        // runs of cells below are written by all of its lanes together)
        const uint64_t r_wave = (uint64_t)bid * kBlock + (threadIdx.x & ~(uint32_t)(kWave - 1));
        for (uint64_t rb = r_wave; rb < n_runs; rb += st64) {
            const uint64_t r = rb + (uint64_t)lane_id();
            const uint32_t p0 = r < n_runs ? (uint32_t)(r * kRun) : nB;
            uint32_t k[kRun];
            if (p0 + kRun <= nB) {
                const uint4 v0 = *reinterpret_cast<const uint4*>(key + p0);
                const uint4 v1 = *reinterpret_cast<const uint4*>(key + p0 + 4);
                k[0] = v0.x; k[1] = v0.y; k[2] = v0.z; k[3] = v0.w;
                k[4] = v1.x; k[5] = v1.y; k[6] = v1.z; k[7] = v1.w;
            } else {
#pragma unroll
                for (uint32_t u = 0; u < kRun; ++u) k[u] = p0 + u < nB ? key[p0 + u] : 0u;
            }
            uint32_t prev = (p0 == 0 || p0 >= nB) ? 0u : key[p0 - 1] + 1u;   // first cell this run may open
#pragma unroll
            for (uint32_t u = 0; u < kRun; ++u) {
                const uint32_t p = p0 + u;
                const bool in = p < nB;
                const uint32_t c = in ? k[u] : 0u;
                // cells [prev, c] start at record p; the last record also
                // closes cells (c, nc] at nB.  Runs of up to kShort cells are
                // written by their lane, longer ones (empty cells around the
                // specimen) by the whole wavefront, 64 consecutive cells per
                // store
                uint32_t q0 = prev, q1 = c, v = p;
                bool open = in && prev <= c;
                distinct += open ? 1u : 0u;   // the first record of its cell
                constexpr uint32_t kShort = 4;
                bool tail = in && p == nB - 1 && c < nc;
                if (open && c - prev < kShort) {
                    for (uint32_t q = prev; q <= c; ++q) a.cell_start[q] = p;
                    open = false;
                }
                if (tail && nc - c <= kShort) {
                    for (uint32_t q = c + 1; q <= nc; ++q) a.cell_start[q] = nB;
                    tail = false;
                }
                for (int pass = 0; pass < 2; ++pass) {
                    const bool mine = pass == 0 ? open : tail;
                    if (pass == 1) {
                        q0 = c + 1u;
                        q1 = nc;
                        v = nB;
                    }
                    uint64_t m = __ballot(mine);
                    while (m) {
                        const int s = __builtin_ctzll(m);
                        m &= m - 1;
                        const uint32_t s0 = (uint32_t)__shfl((int)q0, s, kWave);
                        const uint32_t s1 = (uint32_t)__shfl((int)q1, s, kWave);
                        const uint32_t sv = (uint32_t)__shfl((int)v, s, kWave);
                        for (uint32_t q = s0 + (uint32_t)lane_id(); q <= s1 && q >= s0; q += kWave)
                            a.cell_start[q] = sv;
                    }
                }
                if (in) prev = c + 1u;
            }
        }
    }
    // kGatherItems ions per thread in flight: the position reads are random
    for (uint64_t p0 = (uint64_t)bid * kBlock + threadIdx.x; a.xyz && p0 < nB; p0 += st64 * kGatherItems) {
        uint32_t id[kGatherItems];
        float x[kGatherItems], y[kGatherItems], z[kGatherItems];
#pragma unroll
        for (int u = 0; u < kGatherItems; ++u) id[u] = p0 + (uint64_t)u * st64 < nB ? val[p0 + (uint64_t)u * st64] : 0u;
#pragma unroll
        for (int u = 0; u < kGatherItems; ++u) {
            if (p0 + (uint64_t)u * st64 < nB) {
                x[u] = a.xyz[3 * (size_t)id[u]];
                y[u] = a.xyz[3 * (size_t)id[u] + 1];
                z[u] = a.xyz[3 * (size_t)id[u] + 2];
            }
        }
#pragma unroll
        for (int u = 0; u < kGatherItems; ++u) {
            const uint64_t pp = p0 + (uint64_t)u * st64;
            if (pp >= nB) continue;
            const uint32_t p = (uint32_t)pp;
            const float zz = a.zscale ? (float)((double)z[u] * sd) : z[u];
            a.bpos[p] = make_float4(x[u], y[u], zz, __builtin_bit_cast(float, id[u]));
            const uint32_t c = key[p];
            const uint32_t cprev = p == 0 ? 0u : key[p - 1] + 1u;
            for (uint32_t q = cprev; q <= c; ++q) a.cell_start[q] = p;
            distinct += cprev <= c ? 1u : 0u;   // the first record of its cell
            if (p == nB - 1)
                for (uint32_t q = c + 1; q <= nc; ++q) a.cell_start[q] = nB;
        }
    }
    if (a.distinct) {
        distinct = wave_sum(distinct);
        if (lane_id() == 0 && distinct) atomicAdd(a.distinct, distinct);
    }
}

__global__ __launch_bounds__(kBlock) void k_gather(GatherArgs a) { gather(a, blockIdx.x, gridDim.x); }

__global__ __launch_bounds__(kBlock) void k_order_gather(OrderArgs oa, GatherArgs ga, int32_t g_order) {
    if ((int32_t)blockIdx.x < g_order) take_order(oa, blockIdx.x, (uint32_t)g_order);
    else gather(ga, blockIdx.x - (uint32_t)g_order, gridDim.x - (uint32_t)g_order);
}


}  // namespace apt
