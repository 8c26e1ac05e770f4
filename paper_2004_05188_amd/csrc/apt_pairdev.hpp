// Device-side building blocks of the target-neighbour pair loop, shared by
// the plain kernel (apt_pair.hip) and the batched-replicate kernel
// (apt_batched.hip): the stencil enumeration, the exact kNN key sort and
// the per-target work (RDF counts and k nearest neighbours of one target).
#pragma once
#include "apt_pair.hpp"

namespace apt {

__device__ __forceinline__ uint32_t f2u(float f) { return __builtin_bit_cast(uint32_t, f); }
__device__ __forceinline__ float u2f(uint32_t u) { return __builtin_bit_cast(float, u); }

// Ascending sort of buf[0..c) by one wavefront; c <= kKnnCap.  Up to 64
// keys: each lane takes one key and counts the smaller ones (equal ones by
// position), broadcast lane by lane (no LDS round trips); beyond: a bitonic
// network over buf padded to a power of two with all-ones keys.
__device__ inline void wave_sort_keys(uint64_t* buf, int c) {
    const int l = lane_id();
    if (c <= kWave) {
        wave_sync();
        const uint64_t mine = l < c ? buf[l] : ~0ull;
        const uint32_t lo = (uint32_t)mine, hi = (uint32_t)(mine >> 32);
        int rank = 0;
        for (int j = 0; j < c; ++j) {
            const uint64_t kj = ((uint64_t)readlane(hi, j) << 32) | (uint64_t)readlane(lo, j);
            rank += (kj < mine || (kj == mine && j < l)) ? 1 : 0;
        }
        wave_sync();
        if (l < c) buf[rank] = mine;
        wave_sync();
        return;
    }
    int N = kWave;
    while (N < c) N <<= 1;
    for (int i = c + l; i < N; i += kWave) buf[i] = ~0ull;
    wave_sync();
    for (int size = 2; size <= N; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int p = l; p < (N >> 1); p += kWave) {
                const int i = ((p & ~(stride - 1)) << 1) | (p & (stride - 1));
                const int j = i + stride;
                const bool asc = (i & size) == 0;
                const uint64_t x = buf[i], y = buf[j];
                if ((x > y) == asc) {
                    buf[i] = y;
                    buf[j] = x;
                }
            }
            wave_sync();
        }
    }
}

// Visit the neighbours in the cell rows that a sphere of radius R around
// (px, py, pz) meets.  f(idx, x, y, z) is called by all 64 lanes per step,
// idx == kNone on lanes without a candidate.  kUnroll batches of 64
// candidates are located and their positions loaded before any is visited,
// so that several memory round trips overlap.
constexpr int kUnroll = 4;

// The i-th of L rows centre-out (middle of the range first, then
// alternately below and above; a permutation of [0, L)): enumerations that
// feed a k-smallest list visit rows in this order, so that the list fills
// with the nearest candidates early and later, farther candidates seldom
// change it; others keep raster order, which walks memory in sequence (the
// visiting order never changes a result).
__device__ __forceinline__ int centre_out(int i, int L) {
    return L / 2 + ((i & 1) ? -((i + 1) >> 1) : (i >> 1));
}

// Records [st, st + len) of the cell row (cy, cz) that can lie within R of
// the box [x0,x1] x [y0,y1] x [z0,z1] (R2 = (R + eps)^2): the row's cells
// trimmed to the x-range the sphere reaches at the row's distance from the
// box; len = 0 for a row beyond R.
__device__ __forceinline__ void row_span(const GridPlan& P, const uint32_t* __restrict__ cell_start, int cy, int cz,
                                         float x0, float y0, float z0, float x1, float y1, float z1, float R2,
                                         uint32_t& st, uint32_t& len) {
    const float ya = P.lo[1] + (float)cy * P.h - P.eps, yb = P.lo[1] + (float)(cy + 1) * P.h + P.eps;
    const float za = P.lo[2] + (float)cz * P.h - P.eps, zb = P.lo[2] + (float)(cz + 1) * P.h + P.eps;
    const float dy = fmaxf(0.0f, fmaxf(ya - y1, y0 - yb));
    const float dz = fmaxf(0.0f, fmaxf(za - z1, z0 - zb));
    const float d2 = dy * dy + dz * dz;
    st = 0;
    len = 0;
    if (d2 <= R2) {
        const float ex = sqrtf(R2 - d2) + P.eps;
        const int cx0 = cell_axis(P, 0, x0 - ex), cx1 = cell_axis(P, 0, x1 + ex);
        const uint32_t base = ((uint32_t)cz * (uint32_t)P.dim[1] + (uint32_t)cy) * (uint32_t)P.dim[0];
        st = cell_start[base + (uint32_t)cx0];
        len = cell_start[base + (uint32_t)cx1 + 1u] - st;
    }
}

template <class F>
__device__ __forceinline__ void enumerate_box(const GridPlan& P, const uint32_t* __restrict__ cell_start,
                                              const float4* __restrict__ bpos, float x0, float y0, float z0,
                                              float x1, float y1, float z1, float R, F&& f, bool centre = false) {
    // neighbours within R of the box [x0,x1] x [y0,y1] x [z0,z1]
    const int l = lane_id();
    const float Re = R + P.eps;
    const float R2 = Re * Re;
    const int cy0 = cell_axis(P, 1, y0 - Re), cy1 = cell_axis(P, 1, y1 + Re);
    const int cz0 = cell_axis(P, 2, z0 - Re), cz1 = cell_axis(P, 2, z1 + Re);
    const int ny = cy1 - cy0 + 1, nz = cz1 - cz0 + 1;
    const int nrows = ny * nz;
    for (int rb = 0; rb < nrows; rb += kWave) {
        const int r = rb + l;
        uint32_t st = 0, len = 0;
        if (r < nrows) {
            const int iz = r / ny, iy = r % ny;
            const int cz = cz0 + (centre ? centre_out(iz, nz) : iz), cy = cy0 + (centre ? centre_out(iy, ny) : iy);
            row_span(P, cell_start, cy, cz, x0, y0, z0, x1, y1, z1, R2, st, len);
        }
        const uint32_t inc = wave_incl_scan(len);
        const uint32_t tot = readlane(inc, kWave - 1);
        const uint32_t off = inc - len;
        for (uint32_t b0 = 0; b0 < tot; b0 += kWave * kUnroll) {
            uint32_t idx[kUnroll];
            float4 c[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint32_t b = b0 + (uint32_t)(kWave * u);
                const uint32_t v = b + (uint32_t)l;
                idx[u] = kNone;
                if (b < tot) {
                    const int r0 = __popcll(__ballot(inc <= b));   // first row ending after b
                    const uint32_t e0 = readlane(inc, r0);
                    if (e0 >= b + kWave) {
                        // the whole step lies in row r0
                        idx[u] = readlane(st, r0) + (v - (e0 - readlane(len, r0)));
                    } else {
                        // rows r0..r1 start before the step's end: each lane finds
                        // the last of them starting at or before its slot (binary
                        // lifting over the ascending row offsets, lane shuffles)
                        const uint32_t lim = b + kWave < tot ? b + kWave : tot;
                        const int r1 = __popcll(__ballot(off < lim)) - 1;
                        int row = r0;
                        for (int step = 32; step > 0; step >>= 1) {
                            if (step > r1 - r0) continue;            // uniform
                            const int c = row + step;
                            const uint32_t oc = (uint32_t)__shfl((int)off, c < kWave ? c : kWave - 1, kWave);
                            if (c <= r1 && oc <= v) row = c;
                        }
                        const uint32_t base = (uint32_t)__shfl((int)(st - off), row, kWave);
                        if (v < tot) idx[u] = base + v;
                    }
                }
            }
            // lanes without a candidate read record 0 (always present when tot > 0)
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) c[u] = bpos[idx[u] == kNone ? 0u : idx[u]];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
                if (b0 + (uint32_t)(kWave * u) < tot) f(idx[u] != kNone, c[u]);
        }
    }
}


template <class F>
__device__ __forceinline__ void enumerate(const GridPlan& P, const uint32_t* __restrict__ cell_start,
                                          const float4* __restrict__ bpos, float px, float py, float pz,
                                          float R, F&& f, bool centre = false) {
    enumerate_box(P, cell_start, bpos, px, py, pz, px, py, pz, R, f, centre);
}

// Everything one target needs besides its position and index.
struct PairTask {
    const float4* bpos;          // neighbour records, cell order
    const uint32_t* cell_start;  // [n_cells + 1] into bpos
    // RDF
    int n_bins;
    float r_enum, thr2, inv_w, lo_b, hi_b;
    double inv_w64;
    const double* E2;
    uint32_t* hist_l;            // per-wavefront LDS histogram (LDS variant)
    uint64_t* hist_g;            // global histogram (global variant)
    // kNN
    int k;
    float rk0, rknn, rknn2;
    uint64_t* kbuf;              // per-wavefront LDS key buffer [kKnnCap]
};

// RDF counts and kNN keys of one target.  Leaves the sorted keys in kbuf and
// returns how many of the k nearest were found; adds this lane's RDF counts
// to `hits`.
template <int FLAGS, bool KNN>
__device__ __forceinline__ int run_target(const GridPlan& P, const PairTask& T, float px, float py, float pz,
                                          uint32_t i, uint32_t& hits, bool rdf_on = true) {
    constexpr bool RDF_T = (FLAGS & (kRdfLds | kRdfGlobal)) != 0;
    const bool RDF = RDF_T && rdf_on;
    constexpr bool LDS_HIST = (FLAGS & kRdfLds) != 0;
    constexpr bool SELF = (FLAGS & kSelf) != 0;
    const int l = lane_id();
    const bool finite = isfinite(px) && isfinite(py) && isfinite(pz);
    auto dist2 = [&](float4 c) {
        const float dx = c.x - px, dy = c.y - py, dz = c.z - pz;
        return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    };
    auto cid = [](float4 c) { return __builtin_bit_cast(uint32_t, c.w); };

    // ---- RDF of one candidate: FP32 bin, FP64 re-decision near an edge
    auto rdf_one = [&](bool valid, float4 c, float d2) {
        bool ok = valid && d2 < T.thr2;
        if (SELF) ok = ok && !(d2 == 0.0f && cid(c) == i);     // the target itself
        const float t = __builtin_amdgcn_sqrtf(d2) * T.inv_w;
        int b = (int)t;
        const float fr = t - (float)b;
        if (ok) {
            if (__builtin_expect(fr < T.lo_b || fr > T.hi_b, 0))
                b = exact_bin(exact_D2(px, py, pz, c.x, c.y, c.z), T.E2, T.n_bins, T.inv_w64);
            if (b < T.n_bins) {
                if (LDS_HIST) atomicAdd(&T.hist_l[b], 1u);
                else atomicAdd((unsigned long long*)&T.hist_g[b], 1ull);
                ++hits;
            }
        }
    };

    // ---- kNN: keys of candidates in (rk2_prev, rk2] into the LDS buffer
    int cnt = 0;                        // keys in kbuf
    uint64_t thr_key = ~0ull;           // keys must be below this once the buffer was cut
    float rk = KNN ? fminf(T.rk0, T.rknn) : 0.0f;
    float rk2 = (KNN && rk >= T.rknn) ? T.rknn2 : rk * rk;
    float rk2_prev = -1.0f;
    auto knn_one = [&](bool valid, float4 c, float d2) {
        const uint32_t j = cid(c);
        bool q = valid && d2 <= rk2 && d2 > rk2_prev;
        if (SELF) q = q && j != i;
        const uint64_t key = ((uint64_t)f2u(d2) << 32) | (uint64_t)j;
        q = q && key < thr_key;
        uint64_t m = __ballot(q);
        if (m) {
            int nn = __popcll(m);
            // for small k the buffer is cut at 64 keys (once it holds k),
            // so that cuts and the final sort stay within one wavefront's
            // rank sort and later candidates meet the raised bar sooner
            if (cnt + nn > (T.k <= 32 ? kWave : kKnnCap) && cnt >= T.k) {
                // keep the k smallest keys, raise the bar to the k-th
                wave_sort_keys(T.kbuf, cnt);
                cnt = T.k;
                thr_key = T.kbuf[T.k - 1];
                q = q && key < thr_key;
                m = __ballot(q);
                nn = __popcll(m);
            }
            if (q) T.kbuf[cnt + __popcll(m & lanemask_lt())] = key;
            cnt += nn;
            wave_sync();
        }
    };

    if (finite) {
        if (RDF && (!KNN || rk * 1.000001f < T.r_enum)) {
            enumerate(P, T.cell_start, T.bpos, px, py, pz, T.r_enum,
                      [&](bool v, float4 c) { rdf_one(v, c, dist2(c)); });
            if (KNN)
                enumerate(P, T.cell_start, T.bpos, px, py, pz, rk * 1.000001f,
                          [&](bool v, float4 c) { knn_one(v, c, dist2(c)); }, true);
        } else if (RDF) {
            // the first kNN radius covers r_max: one enumeration for both
            enumerate(P, T.cell_start, T.bpos, px, py, pz, rk * 1.000001f, [&](bool v, float4 c) {
                const float d2 = dist2(c);
                rdf_one(v, c, d2);
                knn_one(v, c, d2);
            }, true);
        } else if (KNN) {
            enumerate(P, T.cell_start, T.bpos, px, py, pz, rk * 1.000001f,
                      [&](bool v, float4 c) { knn_one(v, c, dist2(c)); }, true);
        }
        if (KNN) {
            // grow the radius until k keys are certain (or everything was seen)
            while (cnt < T.k && rk < T.rknn && rk < P.r_all) {
                float g = cbrtf((float)(T.k + 1) / (float)(cnt + 1)) * 1.1f;
                g = fminf(fmaxf(g, 1.25f), 4.0f);
                rk2_prev = rk2;
                rk = fminf(rk * g, fminf(T.rknn, P.r_all));
                rk2 = rk >= T.rknn ? T.rknn2 : rk * rk;
                enumerate(P, T.cell_start, T.bpos, px, py, pz, rk * 1.000001f,
                          [&](bool v, float4 c) { knn_one(v, c, dist2(c)); }, true);
            }
        }
    }
    if (!KNN) return 0;
    wave_sort_keys(T.kbuf, cnt);
    (void)l;
    return cnt < T.k ? cnt : T.k;
}

// ---------------------------------------------------------------- tiles --
// 64 targets per wavefront, one per lane: the neighbour records within R of
// the targets' bounding box are staged through LDS in chunks, and every lane
// scans them for its own target, keeping its KMAX smallest kNN keys (FP32
// squared distance, index) in registers.  Used when targets are dense, so
// that the 64 targets of a tile are close together.
constexpr int kStage = 512;   // records per staging chunk (16 B each)

template <int KMAX>
struct TopK {
    uint64_t key[KMAX > 0 ? KMAX : 1];
};

// Returns this lane's number of kNN keys with d2 <= Rk^2 (0 when KMAX == 0).
template <int FLAGS, int KMAX>
__device__ __forceinline__ void run_tile(const GridPlan& P, const PairTask& T, bool valid, float px, float py,
                                         float pz, uint32_t i, float Rk, float4* stage, TopK<KMAX>& top,
                                         uint32_t& hits) {
    constexpr bool RDF = (FLAGS & (kRdfLds | kRdfGlobal)) != 0;
    constexpr bool LDS_HIST = (FLAGS & kRdfLds) != 0;
    constexpr bool SELF = (FLAGS & kSelf) != 0;
    const int l = lane_id();
#pragma unroll
    for (int m = 0; m < (KMAX > 0 ? KMAX : 1); ++m) top.key[m] = ~0ull;
    const bool fin = valid && isfinite(px) && isfinite(py) && isfinite(pz);
    float x0 = fin ? px : INFINITY, y0 = fin ? py : INFINITY, z0 = fin ? pz : INFINITY;
    float x1 = fin ? px : -INFINITY, y1 = fin ? py : -INFINITY, z1 = fin ? pz : -INFINITY;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        x0 = fminf(x0, __shfl_xor(x0, d, kWave));
        y0 = fminf(y0, __shfl_xor(y0, d, kWave));
        z0 = fminf(z0, __shfl_xor(z0, d, kWave));
        x1 = fmaxf(x1, __shfl_xor(x1, d, kWave));
        y1 = fmaxf(y1, __shfl_xor(y1, d, kWave));
        z1 = fmaxf(z1, __shfl_xor(z1, d, kWave));
    }
    if (!__any(fin)) return;
    const float rk2 = Rk * Rk;
    float R = 0.0f;
    if (RDF) R = T.r_enum;
    if (KMAX > 0) R = fmaxf(R, Rk * 1.000001f);

    auto scan = [&](int m) {
        wave_sync();
        for (int j = 0; j < m; ++j) {
            const float4 c = stage[j];
            const float dx = c.x - px, dy = c.y - py, dz = c.z - pz;
            const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            const uint32_t cj = __builtin_bit_cast(uint32_t, c.w);
            const bool me = fin && (!SELF || cj != i);
            if (RDF && me && d2 < T.thr2) {
                const float t = __builtin_amdgcn_sqrtf(d2) * T.inv_w;
                int b = (int)t;
                const float fr = t - (float)b;
                if (__builtin_expect(fr < T.lo_b || fr > T.hi_b, 0))
                    b = exact_bin(exact_D2(px, py, pz, c.x, c.y, c.z), T.E2, T.n_bins, T.inv_w64);
                if (b < T.n_bins) {
                    if (LDS_HIST) atomicAdd(&T.hist_l[b], 1u);
                    else atomicAdd((unsigned long long*)&T.hist_g[b], 1ull);
                    ++hits;
                }
            }
            if (KMAX > 0) {
                const uint64_t key = ((uint64_t)__builtin_bit_cast(uint32_t, d2) << 32) | (uint64_t)cj;
                if (me && d2 <= rk2 && key < top.key[KMAX - 1]) {
                    // insert, keeping the keys ascending
                    uint64_t x = key;
#pragma unroll
                    for (int q = 0; q < KMAX; ++q) {
                        const uint64_t lo = x < top.key[q] ? x : top.key[q];
                        const uint64_t hi = x < top.key[q] ? top.key[q] : x;
                        top.key[q] = lo;
                        x = hi;
                    }
                }
            }
        }
        wave_sync();
    };

    int m = 0;   // staged records
    enumerate_box(P, T.cell_start, T.bpos, x0, y0, z0, x1, y1, z1, R, [&](bool v, float4 c) {
        const uint64_t bal = __ballot(v);
        const int nn = __popcll(bal);
        if (m + nn > kStage) {
            scan(m);
            m = 0;
        }
        if (v) stage[m + __popcll(bal & lanemask_lt())] = c;
        m += nn;
    }, KMAX > 0);
    if (m > 0) scan(m);
    (void)l;
}

// One target per lane: each lane walks the cell rows within R of its own
// target (rows trimmed to the x-range the sphere reaches, as in
// enumerate_box) and reads the records one by one, kLaneU of them in flight;
// no staging, and no lane waits on a shared candidate list.  Same results as
// run_tile (same candidate set, order-free updates).  With rdf_on false only
// the kNN keys within Rk are taken (a small radius when the neighbours are
// dense: a few dozen records per lane).  Eight records in flight per lane
// (2e9-ion needle, 1.0 nm cells: 23.4 ms with four, 22.4 with eight, 34
// with two; sixteen spill).
constexpr int kLaneU = 8;

template <int FLAGS, int KMAX>
__device__ __forceinline__ void run_lane(const GridPlan& P, const PairTask& T, bool valid, float px, float py,
                                         float pz, uint32_t i, float Rk, TopK<KMAX>& top, uint32_t& hits,
                                         bool rdf_on = true) {
    constexpr bool RDF_T = (FLAGS & (kRdfLds | kRdfGlobal)) != 0;
    const bool RDF = RDF_T && rdf_on;
    constexpr bool LDS_HIST = (FLAGS & kRdfLds) != 0;
    constexpr bool SELF = (FLAGS & kSelf) != 0;
#pragma unroll
    for (int m = 0; m < (KMAX > 0 ? KMAX : 1); ++m) top.key[m] = ~0ull;
    const bool fin = valid && isfinite(px) && isfinite(py) && isfinite(pz);
    const float rk2 = Rk * Rk;
    float R = 0.0f;
    if (RDF) R = T.r_enum;
    if (KMAX > 0) R = fmaxf(R, Rk * 1.000001f);
    const float Re = R + P.eps;
    const float R2 = Re * Re;
    const int cy0 = cell_axis(P, 1, py - Re), cy1 = cell_axis(P, 1, py + Re);
    const int cz0 = cell_axis(P, 2, pz - Re), cz1 = cell_axis(P, 2, pz + Re);
    const int ny = cy1 - cy0 + 1, nz = cz1 - cz0 + 1;
    const int nrows = fin ? ny * nz : 0;
    int r = 0;                     // next row of this lane
    uint32_t j = 0, j1 = 0;        // records left in the current row
    for (;;) {
        // advance to the next row with records (rows beyond R are empty)
        while (j >= j1 && r < nrows) {
            const int cz = cz0 + centre_out(r / ny, nz), cy = cy0 + centre_out(r % ny, ny);
            ++r;
            uint32_t st, len;
            row_span(P, T.cell_start, cy, cz, px, py, pz, px, py, pz, R2, st, len);
            if (len) {
                j = st;
                j1 = st + len;
            }
        }
        if (j >= j1) break;
        float4 c[kLaneU];
#pragma unroll
        for (int u = 0; u < kLaneU; ++u) c[u] = T.bpos[j + (uint32_t)u < j1 ? j + (uint32_t)u : j];
#pragma unroll
        for (int u = 0; u < kLaneU; ++u) {
            if (j + (uint32_t)u >= j1) break;
            const float dx = c[u].x - px, dy = c[u].y - py, dz = c[u].z - pz;
            const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            const uint32_t cj = __builtin_bit_cast(uint32_t, c[u].w);
            const bool me = !SELF || cj != i;
            if (RDF && me && d2 < T.thr2) {
                const float t = __builtin_amdgcn_sqrtf(d2) * T.inv_w;
                int b = (int)t;
                const float fr = t - (float)b;
                if (__builtin_expect(fr < T.lo_b || fr > T.hi_b, 0))
                    b = exact_bin(exact_D2(px, py, pz, c[u].x, c[u].y, c[u].z), T.E2, T.n_bins, T.inv_w64);
                if (b < T.n_bins) {
                    if (LDS_HIST) atomicAdd(&T.hist_l[b], 1u);
                    else atomicAdd((unsigned long long*)&T.hist_g[b], 1ull);
                    ++hits;
                }
            }
            if (KMAX > 0) {
                const uint64_t key = ((uint64_t)__builtin_bit_cast(uint32_t, d2) << 32) | (uint64_t)cj;
                if (me && d2 <= rk2 && key < top.key[KMAX - 1]) {
                    uint64_t x = key;
#pragma unroll
                    for (int q = 0; q < KMAX; ++q) {
                        const uint64_t lo = x < top.key[q] ? x : top.key[q];
                        const uint64_t hi = x < top.key[q] ? top.key[q] : x;
                        top.key[q] = lo;
                        x = hi;
                    }
                }
            }
        }
        j += kLaneU;
    }
}

// As run_tile, for callers that need only each lane's k-th neighbour key
// (the k-th distance histogram).  The scan keeps the KMAX smallest FP32
// squared distances per lane with a min/max network (two instructions a
// slot, no keys); a second, smaller enumeration (radius: the largest k-th
// distance of the tile) then finds the k-th neighbour's index: the smallest
// index among the candidates at exactly that distance when the k-1 nearer
// ones are strictly nearer.  Returns the k-th key (FP32 d2 bits << 32 |
// index), or ~0 when it is not settled here: fewer than k neighbours within
// Rk, or the k-th distance shared by several of the k nearest (the caller
// finishes those targets exactly).
template <int FLAGS, int KMAX>
__device__ __forceinline__ uint64_t run_tile_kth(const GridPlan& P, const PairTask& T, bool valid, float px,
                                                 float py, float pz, uint32_t i, float Rk, int k, float4* stage,
                                                 uint32_t& hits) {
    constexpr bool RDF = (FLAGS & (kRdfLds | kRdfGlobal)) != 0;
    constexpr bool LDS_HIST = (FLAGS & kRdfLds) != 0;
    constexpr bool SELF = (FLAGS & kSelf) != 0;
    static_assert(KMAX > 0, "k-th key needs KMAX > 0");
    const bool fin = valid && isfinite(px) && isfinite(py) && isfinite(pz);
    float x0 = fin ? px : INFINITY, y0 = fin ? py : INFINITY, z0 = fin ? pz : INFINITY;
    float x1 = fin ? px : -INFINITY, y1 = fin ? py : -INFINITY, z1 = fin ? pz : -INFINITY;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        x0 = fminf(x0, __shfl_xor(x0, d, kWave));
        y0 = fminf(y0, __shfl_xor(y0, d, kWave));
        z0 = fminf(z0, __shfl_xor(z0, d, kWave));
        x1 = fmaxf(x1, __shfl_xor(x1, d, kWave));
        y1 = fmaxf(y1, __shfl_xor(y1, d, kWave));
        z1 = fmaxf(z1, __shfl_xor(z1, d, kWave));
    }
    if (!__any(fin)) return ~0ull;
    const float rk2 = Rk * Rk;
    const float R = RDF ? fmaxf(T.r_enum, Rk * 1.000001f) : Rk * 1.000001f;
    float top[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) top[q] = INFINITY;

    auto scan = [&](int m) {
        wave_sync();
        for (int j = 0; j < m; ++j) {
            const float4 c = stage[j];
            const float dx = c.x - px, dy = c.y - py, dz = c.z - pz;
            const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            const uint32_t cj = __builtin_bit_cast(uint32_t, c.w);
            const bool me = fin && (!SELF || cj != i);
            if (RDF && me && d2 < T.thr2) {
                const float t = __builtin_amdgcn_sqrtf(d2) * T.inv_w;
                int b = (int)t;
                const float fr = t - (float)b;
                if (__builtin_expect(fr < T.lo_b || fr > T.hi_b, 0))
                    b = exact_bin(exact_D2(px, py, pz, c.x, c.y, c.z), T.E2, T.n_bins, T.inv_w64);
                if (b < T.n_bins) {
                    if (LDS_HIST) atomicAdd(&T.hist_l[b], 1u);
                    else atomicAdd((unsigned long long*)&T.hist_g[b], 1ull);
                    ++hits;
                }
            }
            const bool in = me && d2 <= rk2;
            if (__ballot(in && d2 < top[KMAX - 1])) {
                float x = in ? d2 : INFINITY;
#pragma unroll
                for (int q = 0; q < KMAX; ++q) {
                    const float lo = fminf(x, top[q]);
                    x = fmaxf(x, top[q]);
                    top[q] = lo;
                }
            }
        }
        wave_sync();
    };
    int m = 0;
    auto stage_one = [&](auto&& sc) {
        return [&, sc](bool v, float4 c) {
            const uint64_t bal = __ballot(v);
            const int nn = __popcll(bal);
            if (m + nn > kStage) {
                sc(m);
                m = 0;
            }
            if (v) stage[m + __popcll(bal & lanemask_lt())] = c;
            m += nn;
        };
    };
    enumerate_box(P, T.cell_start, T.bpos, x0, y0, z0, x1, y1, z1, R, stage_one(scan), true);
    if (m > 0) scan(m);

    // the k-th distance and how many of the k nearest lie strictly nearer
    float tau = top[0];
#pragma unroll
    for (int q = 1; q < KMAX; ++q)
        if (q == k - 1) tau = top[q];
    int nearer = 0;
#pragma unroll
    for (int q = 0; q < KMAX; ++q) nearer += (q < k && top[q] < tau);
    bool settled = fin && tau <= rk2 && nearer == k - 1;
    // second pass: the smallest index at exactly the k-th distance
    float tmax = settled ? tau : 0.0f;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) tmax = fmaxf(tmax, __shfl_xor(tmax, d, kWave));
    uint32_t jk = 0xFFFFFFFFu;
    if (__any(settled)) {
        auto scan2 = [&](int mm) {
            wave_sync();
            for (int j = 0; j < mm; ++j) {
                const float4 c = stage[j];
                const float dx = c.x - px, dy = c.y - py, dz = c.z - pz;
                const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                const uint32_t cj = __builtin_bit_cast(uint32_t, c.w);
                const bool me = settled && (!SELF || cj != i);
                if (me && d2 == tau && cj < jk) jk = cj;
            }
            wave_sync();
        };
        m = 0;
        enumerate_box(P, T.cell_start, T.bpos, x0, y0, z0, x1, y1, z1, sqrtf(tmax) * 1.000001f, stage_one(scan2));
        if (m > 0) scan2(m);
    }
    settled = settled && jk != 0xFFFFFFFFu;
    return settled ? (((uint64_t)__builtin_bit_cast(uint32_t, tau) << 32) | (uint64_t)jk) : ~0ull;
}

// Flush a per-wavefront u32 LDS histogram into a global u64 histogram.
__device__ __forceinline__ void flush_hist(uint32_t* hist_l, uint64_t* hist_g, int n_bins) {
    for (int b = lane_id(); b < n_bins; b += kWave) {
        const uint32_t v = hist_l[b];
        if (v) atomicAdd((unsigned long long*)&hist_g[b], (unsigned long long)v);
        hist_l[b] = 0;
    }
    wave_sync();
}

// Bin of the distance of a kNN key (bits(d2f) << 32 | index) in the k-th
// distance histogram: the FP32 bin of the key's squared distance, exact
// away from the edges (the same band as the RDF's fast path: the FP32
// squared distance, root and scaling err by a few ulps); inside the band,
// the FP64 distance of the stored positions decides.
__device__ __forceinline__ int key_bin(uint64_t key, const float* xyz, float px, float py, float pz,
                                       const double* KE2, int kb_nbins, double kb_inv_w64) {
    const float t = __builtin_amdgcn_sqrtf(u2f((uint32_t)(key >> 32))) * (float)kb_inv_w64;
    if (!(t < (float)kb_nbins + 2.0f)) return kb_nbins;
    const float band = (float)fmin(0.25, fmax(1e-6 * kb_inv_w64, 4e-6 * (double)kb_nbins));
    const int bf = (int)t;
    const float fr = t - (float)bf;
    if (fr > band && fr < 1.0f - band) return bf < kb_nbins ? bf : kb_nbins;
    const uint32_t j = (uint32_t)key;
    return exact_bin(exact_D2(px, py, pz, xyz[3 * (size_t)j], xyz[3 * (size_t)j + 1], xyz[3 * (size_t)j + 2]),
                     KE2, kb_nbins, kb_inv_w64);
}

// Bin of the k-th neighbour's distance (kb_nbins when missing).
__device__ __forceinline__ int kth_bin(int found, int k, const uint64_t* kbuf, const float* xyz, float px,
                                       float py, float pz, const double* KE2, int kb_nbins, double kb_inv_w64) {
    if (found < k) return kb_nbins;
    return key_bin(kbuf[k - 1], xyz, px, py, pz, KE2, kb_nbins, kb_inv_w64);
}

}  // namespace apt
