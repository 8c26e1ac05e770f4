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
#include "apt_pair.hpp"

namespace apt {

size_t pair_lds_bytes(bool rdf, bool knn, int n_bins, bool hist_in_lds) {
    size_t b = 0;
    if (rdf && hist_in_lds) b += (size_t)kWavesPerBlock * (size_t)n_bins * 4u;
    b = (b + 15) & ~size_t(15);
    if (knn) b += (size_t)kWavesPerBlock * kKnnCap * 8u;
    return b;
}

__device__ __forceinline__ uint32_t f2u(float f) { return __builtin_bit_cast(uint32_t, f); }
__device__ __forceinline__ float u2f(uint32_t u) { return __builtin_bit_cast(float, u); }

// Ascending bitonic sort of buf[0..c) (padded to a power of two >= 64 with
// all-ones keys) by one wavefront; c <= kKnnCap.
__device__ void wave_sort_keys(uint64_t* buf, int c) {
    const int l = lane_id();
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

template <class F>
__device__ __forceinline__ void enumerate(const GridPlan& P, const uint32_t* __restrict__ cell_start,
                                          const float4* __restrict__ bpos, float px, float py, float pz,
                                          float R, F&& f) {
    const int l = lane_id();
    const float Re = R + P.eps;
    const float R2 = Re * Re;
    const int cy0 = cell_axis(P, 1, py - Re), cy1 = cell_axis(P, 1, py + Re);
    const int cz0 = cell_axis(P, 2, pz - Re), cz1 = cell_axis(P, 2, pz + Re);
    const int ny = cy1 - cy0 + 1;
    const int nrows = ny * (cz1 - cz0 + 1);
    for (int rb = 0; rb < nrows; rb += kWave) {
        const int r = rb + l;
        uint32_t st = 0, len = 0;
        if (r < nrows) {
            const int cz = cz0 + r / ny, cy = cy0 + r % ny;
            const float y0 = P.lo[1] + (float)cy * P.h - P.eps, y1 = P.lo[1] + (float)(cy + 1) * P.h + P.eps;
            const float z0 = P.lo[2] + (float)cz * P.h - P.eps, z1 = P.lo[2] + (float)(cz + 1) * P.h + P.eps;
            const float dy = fmaxf(0.0f, fmaxf(y0 - py, py - y1));
            const float dz = fmaxf(0.0f, fmaxf(z0 - pz, pz - z1));
            const float d2 = dy * dy + dz * dz;
            if (d2 <= R2) {
                const float ex = sqrtf(R2 - d2) + P.eps;
                const int cx0 = cell_axis(P, 0, px - ex), cx1 = cell_axis(P, 0, px + ex);
                const uint32_t base = ((uint32_t)cz * (uint32_t)P.dim[1] + (uint32_t)cy) * (uint32_t)P.dim[0];
                st = cell_start[base + (uint32_t)cx0];
                len = cell_start[base + (uint32_t)cx1 + 1u] - st;
            }
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
                        for (int rr = r0; rr < kWave; ++rr) {
                            const uint32_t o = readlane(off, rr);
                            if (o >= b + kWave || o >= tot) break;
                            const uint32_t s0 = readlane(st, rr), ln = readlane(len, rr);
                            if (v >= o && v < o + ln) idx[u] = s0 + (v - o);
                        }
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

template <int FLAGS, bool KNN>
__global__ __launch_bounds__(kBlock) void k_pair(PairArgs a) {
    constexpr bool RDF = (FLAGS & (kRdfLds | kRdfGlobal)) != 0;
    constexpr bool LDS_HIST = (FLAGS & kRdfLds) != 0;
    constexpr bool SELF = (FLAGS & kSelf) != 0;
    extern __shared__ __align__(16) uint8_t smem[];
    const GridPlan P = *a.plan;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int l = lane_id();
    uint32_t* hist_l = reinterpret_cast<uint32_t*>(smem) + (size_t)w * a.n_bins;
    if (LDS_HIST)
        for (int b = l; b < a.n_bins; b += kWave) hist_l[b] = 0;
    uint64_t* kbuf = nullptr;
    if (KNN) {
        size_t off = LDS_HIST ? (size_t)kWavesPerBlock * a.n_bins * 4u : 0;
        off = (off + 15) & ~size_t(15);
        kbuf = reinterpret_cast<uint64_t*>(smem + off) + (size_t)w * kKnnCap;
    }
    wave_sync();
    const float4* __restrict__ bpos = a.bpos;
    const float thr2 = a.thr2, inv_w = a.inv_w, lo_b = a.delta_b, hi_b = 1.0f - a.delta_b;
    const int n_bins = a.n_bins;

    // XCD-aware deal: XCD x takes the x-th eighth of the targets in cell order
    const int xcd = blockIdx.x % kXcd;
    const int per_xcd = gridDim.x / kXcd;
    const uint32_t wx = (uint32_t)(blockIdx.x / kXcd) * kWavesPerBlock + (uint32_t)w;
    const uint32_t wstride = (uint32_t)per_xcd * kWavesPerBlock;
    const uint32_t t0 = (uint32_t)((uint64_t)P.nT * (uint64_t)xcd / kXcd);
    const uint32_t t1 = (uint32_t)((uint64_t)P.nT * (uint64_t)(xcd + 1) / kXcd);
    uint32_t since_flush = 0;      // hits counted into hist_l since its last flush (wave total)
    const uint32_t flush_at = P.nB >= 0x7FFFFFFFu ? 0u : 0xFFFFFFFFu - P.nB;

    // target data of the next iteration is loaded one iteration ahead
    uint32_t s = t0 + wx;
    uint32_t n_rank = 0, n_i = 0;
    float n_px = 0.0f, n_py = 0.0f, n_pz = 0.0f;
    if (s < t1) {
        n_rank = a.t_rank[s];
        n_i = a.t_id[s];
        n_px = a.tx[s];
        n_py = a.ty[s];
        n_pz = a.tz[s];
    }
    for (; s < t1; s += wstride) {
        const uint32_t rank = __builtin_amdgcn_readfirstlane(n_rank);
        const uint32_t i = __builtin_amdgcn_readfirstlane(n_i);
        const float px = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, n_px)));
        const float py = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, n_py)));
        const float pz = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, n_pz)));
        const uint32_t sn = s + wstride;
        if (sn < t1) {
            n_rank = a.t_rank[sn];
            n_i = a.t_id[sn];
            n_px = a.tx[sn];
            n_py = a.ty[sn];
            n_pz = a.tz[sn];
        }
        const bool finite = isfinite(px) && isfinite(py) && isfinite(pz);
        uint32_t hits = 0;   // per lane

        auto dist2 = [&](const float4& c) {
            const float dx = c.x - px, dy = c.y - py, dz = c.z - pz;
            return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        };
        auto cid = [](const float4& c) { return __builtin_bit_cast(uint32_t, c.w); };

        // ---- RDF of one candidate: FP32 bin, FP64 re-decision near an edge
        auto rdf_one = [&](bool valid, const float4& c, float d2) {
            bool ok = valid && d2 < thr2;
            if (SELF) ok = ok && !(d2 == 0.0f && cid(c) == i);     // the target itself
            const float t = __builtin_amdgcn_sqrtf(d2) * inv_w;
            int b = (int)t;
            const float fr = t - (float)b;
            if (ok) {
                if (__builtin_expect(fr < lo_b || fr > hi_b, 0))
                    b = exact_bin(exact_D2(px, py, pz, c.x, c.y, c.z), a.E2, n_bins, a.inv_w64);
                if (b < n_bins) {
                    if (LDS_HIST) atomicAdd(&hist_l[b], 1u);
                    else atomicAdd((unsigned long long*)&a.hist[b], 1ull);
                    ++hits;
                }
            }
        };

        // ---- kNN: keys of candidates in (rk2_prev, rk2] into the LDS buffer
        int cnt = 0;                        // keys in kbuf
        uint64_t thr_key = ~0ull;           // keys must be below this once the buffer was cut
        float rk = KNN ? fminf(P.rk0, a.rknn) : 0.0f;
        float rk2 = (KNN && rk >= a.rknn) ? a.rknn2 : rk * rk;
        float rk2_prev = -1.0f;
        auto knn_one = [&](bool valid, const float4& c, float d2) {
            const uint32_t j = cid(c);
            bool q = valid && d2 <= rk2 && d2 > rk2_prev;
            if (SELF) q = q && j != i;
            const uint64_t key = ((uint64_t)f2u(d2) << 32) | (uint64_t)j;
            q = q && key < thr_key;
            uint64_t m = __ballot(q);
            if (m) {
                int nn = __popcll(m);
                if (cnt + nn > kKnnCap) {
                    // keep the k smallest keys, raise the bar to the k-th
                    wave_sort_keys(kbuf, cnt);
                    cnt = a.k;
                    thr_key = kbuf[a.k - 1];
                    q = q && key < thr_key;
                    m = __ballot(q);
                    nn = __popcll(m);
                }
                if (q) kbuf[cnt + __popcll(m & lanemask_lt())] = key;
                cnt += nn;
                wave_sync();
            }
        };

        if (finite) {
            if (RDF && (!KNN || rk * 1.000001f < a.r_enum)) {
                enumerate(P, a.cell_start, bpos, px, py, pz, a.r_enum,
                          [&](bool v, const float4& c) { rdf_one(v, c, dist2(c)); });
                if (KNN)
                    enumerate(P, a.cell_start, bpos, px, py, pz, rk * 1.000001f,
                              [&](bool v, const float4& c) { knn_one(v, c, dist2(c)); });
            } else if (RDF) {
                // the first kNN radius covers r_max: one enumeration for both
                enumerate(P, a.cell_start, bpos, px, py, pz, rk * 1.000001f, [&](bool v, const float4& c) {
                    const float d2 = dist2(c);
                    rdf_one(v, c, d2);
                    knn_one(v, c, d2);
                });
            } else if (KNN) {
                enumerate(P, a.cell_start, bpos, px, py, pz, rk * 1.000001f,
                          [&](bool v, const float4& c) { knn_one(v, c, dist2(c)); });
            }
            if (KNN) {
                // grow the radius until k keys are certain (or everything was seen)
                while (cnt < a.k && rk < a.rknn && rk < P.r_all) {
                    float g = cbrtf((float)(a.k + 1) / (float)(cnt + 1)) * 1.1f;
                    g = fminf(fmaxf(g, 1.25f), 4.0f);
                    rk2_prev = rk2;
                    rk = fminf(rk * g, fminf(a.rknn, P.r_all));
                    rk2 = rk >= a.rknn ? a.rknn2 : rk * rk;
                    enumerate(P, a.cell_start, bpos, px, py, pz, rk * 1.000001f,
                              [&](bool v, const float4& c) { knn_one(v, c, dist2(c)); });
                }
            }
        }

        if (KNN) {
            wave_sort_keys(kbuf, cnt);
            const int found = cnt < a.k ? cnt : a.k;
            if ((int64_t)rank < a.capacity) {
                if (l == 0) a.target_id[rank] = (int64_t)i;
                for (int m = l; m < a.k; m += kWave) {
                    const size_t o = (size_t)rank * (size_t)a.k + (size_t)m;
                    if (m < found) {
                        const uint64_t key = kbuf[m];
                        a.dist[o] = sqrtf(u2f((uint32_t)(key >> 32)));
                        a.nbr_id[o] = (int64_t)(uint32_t)key;
                    } else {
                        a.dist[o] = INFINITY;
                        a.nbr_id[o] = -1;
                    }
                }
            }
            if (a.knn_hist && l == 0) {
                int b = a.kb_nbins;
                if (found == a.k) {
                    const uint32_t j = (uint32_t)kbuf[a.k - 1];
                    b = exact_bin(exact_D2(px, py, pz, a.xyz[3 * (size_t)j], a.xyz[3 * (size_t)j + 1],
                                           a.xyz[3 * (size_t)j + 2]),
                                  a.KE2, a.kb_nbins, a.kb_inv_w64);
                }
                atomicAdd((unsigned long long*)&a.knn_hist[b], 1ull);
            }
            wave_sync();
        }
        if (LDS_HIST) {
            // u32 LDS counters: flush before a further target could overflow them
            since_flush += wave_sum(hits);
            if (since_flush >= flush_at) {
                for (int b = l; b < n_bins; b += kWave) {
                    const uint32_t v = hist_l[b];
                    if (v) atomicAdd((unsigned long long*)&a.hist[b], (unsigned long long)v);
                    hist_l[b] = 0;
                }
                since_flush = 0;
                wave_sync();
            }
        }
    }
    if (LDS_HIST) {
        for (int b = l; b < n_bins; b += kWave) {
            const uint32_t v = hist_l[b];
            if (v) atomicAdd((unsigned long long*)&a.hist[b], (unsigned long long)v);
        }
    }
}

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
