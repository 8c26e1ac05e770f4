// Label randomisation on the GPU: out[i] = lab[pi(i)] with pi the ascending
// order of the keys key(i) = i-th SplitMix64 output for the seed (ties by
// index), i.e. a uniform random permutation of the labels (paper, Suppl.:
// "Importance of high quality random number generators" -- the null model
// computes every statistic on randomly reordered ion-type labels).
//
// The permutation is the argsort of 64-bit keys, but no 64-bit radix sort is
// run: keys are dealt into buckets by their top bits (atomic counts, a scan,
// atomic placement), and each bucket -- a few dozen keys on average -- is
// sorted exactly by (key, index) in LDS by one wavefront.  Buckets are in
// key order, so the concatenated sorted buckets are the argsort.
#include "apt_perm.hpp"

namespace apt {

// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): the state advances by the
// golden gamma, then is mixed; this is the i-th output for state `seed`.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int perm_bucket_bits(int64_t n) {
    int b = 0;
    while (b < 26 && ((int64_t)32 << b) < n) ++b;   // about 32 keys per bucket
    return b;
}

// ---------------------------------------------------------- device scan --
// Exclusive scan of x[0..n) in place; part[] holds one value per block.
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t* x, int64_t n, int64_t chunk,
                                                       uint32_t* part) {
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = beg + chunk < n ? beg + chunk : n;
    uint32_t s = 0;
    for (int64_t i = beg + threadIdx.x; i < end; i += kBlock) s += x[i];
    __shared__ uint32_t sw[kWavesPerBlock];
    s = wave_sum(s);
    if (lane_id() == 0) sw[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kWavesPerBlock; ++w) t += sw[w];
        part[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(1024) void k_scan_parts(uint32_t* part, int G) {
    // G <= 1024
    __shared__ uint32_t tmp[16];
    const int t = threadIdx.x, w = t / kWave, l = lane_id();
    const uint32_t v = t < G ? part[t] : 0u;
    const uint32_t inc = wave_incl_scan(v);
    if (l == kWave - 1) tmp[w] = inc;
    __syncthreads();
    uint32_t base = 0;
    for (int u = 0; u < w; ++u) base += tmp[u];
    if (t < G) part[t] = base + inc - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(uint32_t* x, int64_t n, int64_t chunk,
                                                      const uint32_t* part) {
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = beg + chunk < n ? beg + chunk : n;
    __shared__ uint32_t sw[kWavesPerBlock];
    __shared__ uint32_t s_run;
    if (threadIdx.x == 0) s_run = part[blockIdx.x];
    __syncthreads();
    const int w = threadIdx.x / kWave;
    for (int64_t base = beg; base < end; base += kBlock) {
        const int64_t i = base + threadIdx.x;
        const uint32_t v = i < end ? x[i] : 0u;
        const uint32_t inc = wave_incl_scan(v);
        if (lane_id() == kWave - 1) sw[w] = inc;
        __syncthreads();
        uint32_t add = s_run;
        for (int u = 0; u < w; ++u) add += sw[u];
        if (i < end) x[i] = add + inc - v;
        __syncthreads();
        if (threadIdx.x == kBlock - 1) s_run = add + inc;
        __syncthreads();
    }
}

void device_excl_scan(uint32_t* x, int64_t n, uint32_t* part, hipStream_t st) {
    if (n <= 0) return;
    int G = (int)((n + 4095) / 4096);
    if (G > 1024) G = 1024;
    const int64_t chunk = (n + G - 1) / G;
    hipLaunchKernelGGL(k_scan_reduce, dim3(G), dim3(kBlock), 0, st, x, n, chunk, part);
    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(1024), 0, st, part, G);
    hipLaunchKernelGGL(k_scan_apply, dim3(G), dim3(kBlock), 0, st, x, n, chunk, part);
}

// ------------------------------------------------------------- buckets --
__global__ __launch_bounds__(kBlock) void k_perm_zero(PermArgs a) {
    const int64_t nb = (int64_t)1 << a.bits;
    for (int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x; b < nb * a.n_rep;
         b += (int64_t)gridDim.x * kBlock) {
        a.count[b] = 0;
        a.cursor[b] = 0;
    }
}

__global__ __launch_bounds__(kBlock) void k_perm_count(PermArgs a) {
    const int r = blockIdx.y;
    const uint64_t seed = a.seeds[r];
    const int64_t nb = (int64_t)1 << a.bits;
    uint32_t* cnt = a.count + (size_t)r * nb;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * kBlock) {
        const uint64_t key = splitmix64(seed, (uint64_t)i);
        const uint64_t b = a.bits ? key >> (64 - a.bits) : 0ull;
        atomicAdd(&cnt[b], 1u);
    }
}

__global__ __launch_bounds__(kBlock) void k_perm_place(PermArgs a) {
    const int r = blockIdx.y;
    const uint64_t seed = a.seeds[r];
    const int64_t nb = (int64_t)1 << a.bits;
    // count[] was scanned over all replicates at once: starts are global
    // positions, replicate r owning [r*n, (r+1)*n)
    const uint32_t* start = a.count + (size_t)r * nb;
    uint32_t* cur = a.cursor + (size_t)r * nb;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * kBlock) {
        const uint64_t key = splitmix64(seed, (uint64_t)i);
        const uint64_t b = a.bits ? key >> (64 - a.bits) : 0ull;
        const uint64_t slot = (uint64_t)start[b] + atomicAdd(&cur[b], 1u);
        a.ekey[slot] = key;
        a.eidx[slot] = (uint32_t)i;
    }
}

// sort (key, idx) pairs of one bucket ascending, in LDS, one wavefront
__device__ void wave_sort_pairs(uint64_t* k, uint32_t* v, int c, int N) {
    const int l = lane_id();
    for (int i = c + l; i < N; i += kWave) {
        k[i] = ~0ull;
        v[i] = 0xFFFFFFFFu;
    }
    wave_sync();
    for (int size = 2; size <= N; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int p = l; p < (N >> 1); p += kWave) {
                const int i = ((p & ~(stride - 1)) << 1) | (p & (stride - 1));
                const int j = i + stride;
                const bool asc = (i & size) == 0;
                const uint64_t ki = k[i], kj = k[j];
                const uint32_t vi = v[i], vj = v[j];
                const bool gt = ki > kj || (ki == kj && vi > vj);
                if (gt == asc) {
                    k[i] = kj;
                    k[j] = ki;
                    v[i] = vj;
                    v[j] = vi;
                }
            }
            wave_sync();
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_perm_sort(PermArgs a) {
    __shared__ uint64_t s_k[kWavesPerBlock][kPermCap];
    __shared__ uint32_t s_v[kWavesPerBlock][kPermCap];
    const int r = blockIdx.y;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int l = lane_id();
    const int64_t nb = (int64_t)1 << a.bits;
    const uint32_t* start = a.count + (size_t)r * nb;
    const uint64_t rbase = (uint64_t)r * (uint64_t)a.n;
    const uint8_t* lab = a.lab;
    uint8_t* out = a.out + (size_t)r * a.out_stride;
    for (int64_t b = (int64_t)blockIdx.x * kWavesPerBlock + w; b < nb; b += (int64_t)gridDim.x * kWavesPerBlock) {
        const uint64_t s0 = start[b];
        const uint64_t s1 = b + 1 < nb ? (uint64_t)start[b + 1] : rbase + (uint64_t)a.n;
        const int c = (int)(s1 - s0);
        if (c > kPermCap) {
            // probability below 1e-300 for random keys; reported, output invalid
            if (l == 0 && a.status) atomicOr(a.status, APT_STATUS_CAPACITY);
            continue;
        }
        for (int q = l; q < c; q += kWave) {
            s_k[w][q] = a.ekey[s0 + q];
            s_v[w][q] = a.eidx[s0 + q];
        }
        int N = 2;
        while (N < c) N <<= 1;
        wave_sort_pairs(s_k[w], s_v[w], c, N);
        for (int q = l; q < c; q += kWave) out[s0 - rbase + q] = lab[s_v[w][q]];
        wave_sync();
    }
}

// ------------------------------------------------ two-level form (LDS) --
// For n <= kPermLdsMax: coarse buckets by the top `bits` key bits (at most
// 2^13, about 2048 keys each), counted and filled with one global atomic per
// (workgroup, bucket); a coarse bucket is then split by the next six bits in
// LDS and every fine bucket (about 32 keys) ordered by one wavefront.  Only
// the indices travel through memory; keys are recomputed from them.

int perm_coarse_bits(int64_t n) {
    int b = 0;
    while (b < 13 && ((int64_t)2048 << b) < n) ++b;
    return b;
}

size_t perm_deal_lds_bytes(int coarse_bits) { return (size_t)2 * 4u << coarse_bits; }

__device__ __forceinline__ uint32_t coarse_of(uint64_t key, int bits) {
    return bits ? (uint32_t)(key >> (64 - bits)) : 0u;
}
__device__ __forceinline__ uint32_t fine_of(uint64_t key, int bits) {
    return (uint32_t)(key >> (64 - bits - kPermFineBits)) & ((1u << kPermFineBits) - 1u);
}

// block counts of the coarse buckets, added to count[r][b]
__global__ __launch_bounds__(kBlock) void k_permc_count(PermArgs a) {
    extern __shared__ uint32_t s_h[];
    const int r = blockIdx.y;
    const uint64_t seed = a.seeds[r];
    const int nb = 1 << a.bits;
    for (int b = threadIdx.x; b < nb; b += kBlock) s_h[b] = 0;
    __syncthreads();
    const int64_t beg = (int64_t)blockIdx.x * kPermChunk;
    const int64_t end = beg + kPermChunk < a.n ? beg + kPermChunk : a.n;
    for (int64_t i = beg + threadIdx.x; i < end; i += kBlock)
        atomicAdd(&s_h[coarse_of(splitmix64(seed, (uint64_t)i), a.bits)], 1u);
    __syncthreads();
    uint32_t* cnt = a.count + (size_t)r * nb;
    for (int b = threadIdx.x; b < nb; b += kBlock)
        if (s_h[b]) atomicAdd(&cnt[b], s_h[b]);
}

// indices into their coarse buckets (count[] now holds the global starts);
// the order inside a bucket is arbitrary: k_permc_sort orders it
__global__ __launch_bounds__(kBlock) void k_permc_place(PermArgs a) {
    extern __shared__ uint32_t s_mem[];
    const int nb = 1 << a.bits;
    uint32_t* s_h = s_mem;
    uint32_t* s_base = s_mem + nb;
    const int r = blockIdx.y;
    const uint64_t seed = a.seeds[r];
    for (int b = threadIdx.x; b < nb; b += kBlock) s_h[b] = 0;
    __syncthreads();
    const int64_t beg = (int64_t)blockIdx.x * kPermChunk;
    const int64_t end = beg + kPermChunk < a.n ? beg + kPermChunk : a.n;
    for (int64_t i = beg + threadIdx.x; i < end; i += kBlock)
        atomicAdd(&s_h[coarse_of(splitmix64(seed, (uint64_t)i), a.bits)], 1u);
    __syncthreads();
    const uint32_t* start = a.count + (size_t)r * nb;
    uint32_t* cur = a.cursor + (size_t)r * nb;
    for (int b = threadIdx.x; b < nb; b += kBlock) {
        const uint32_t h = s_h[b];
        s_base[b] = h ? start[b] + atomicAdd(&cur[b], h) : 0u;
        s_h[b] = 0;
    }
    __syncthreads();
    for (int64_t i = beg + threadIdx.x; i < end; i += kBlock) {
        const uint32_t b = coarse_of(splitmix64(seed, (uint64_t)i), a.bits);
        a.eidx[s_base[b] + atomicAdd(&s_h[b], 1u)] = (uint32_t)i;
    }
}

// one coarse bucket per workgroup: fine buckets in LDS, each ordered by
// (key, index) by one wavefront (ranks by counting for up to 64 keys, a
// bitonic sort beyond), labels gathered to their ranks
__global__ __launch_bounds__(kBlock) void k_permc_sort(PermArgs a) {
    constexpr int kItems = (kPermCoarseCap + kBlock - 1) / kBlock;
    constexpr int kFine = 1 << kPermFineBits;
    static_assert(kFine == kWave, "one wavefront scans the fine counts");
    __shared__ uint64_t s_k[kPermCoarseCap];
    __shared__ uint32_t s_v[kPermCoarseCap];
    __shared__ uint32_t s_fc[kFine], s_fo[kFine];
    __shared__ uint64_t w_k[kWavesPerBlock][kPermFineCap];
    __shared__ uint32_t w_v[kWavesPerBlock][kPermFineCap];
    const int r = blockIdx.y;
    const uint64_t seed = a.seeds[r];
    const int nb = 1 << a.bits;
    const int t = threadIdx.x, l = lane_id();
    const int w = __builtin_amdgcn_readfirstlane(t / kWave);
    const uint32_t* start = a.count + (size_t)r * nb;
    const uint64_t rbase = (uint64_t)r * (uint64_t)a.n;
    const uint8_t* lab = a.lab;
    uint8_t* out = a.out + (size_t)r * a.out_stride;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        const uint64_t s0 = start[b];
        const uint64_t s1 = b + 1 < nb ? (uint64_t)start[b + 1] : rbase + (uint64_t)a.n;
        const int c = (int)(s1 - s0);
        if (c > kPermCoarseCap) {
            // probability below 1e-100 for random keys; reported, output invalid
            if (t == 0 && a.status) atomicOr(a.status, APT_STATUS_CAPACITY);
            continue;
        }
        if (t < kFine) s_fc[t] = 0;
        __syncthreads();
        uint64_t kk[kItems];
        uint32_t vv[kItems];
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const int q = t + j * kBlock;
            vv[j] = q < c ? a.eidx[s0 + (uint64_t)q] : 0u;
        }
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            kk[j] = splitmix64(seed, (uint64_t)vv[j]);
            if (t + j * kBlock < c) atomicAdd(&s_fc[fine_of(kk[j], a.bits)], 1u);
        }
        __syncthreads();
        if (t < kFine) {
            // kFine == kWave: wavefront 0 scans the fine counts
            const uint32_t x = s_fc[t];
            const uint32_t ex = wave_incl_scan(x) - x;
            s_fo[t] = ex;
            s_fc[t] = ex;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            if (t + j * kBlock < c) {
                const uint32_t p = atomicAdd(&s_fc[fine_of(kk[j], a.bits)], 1u);
                s_k[p] = kk[j];
                s_v[p] = vv[j];
            }
        }
        __syncthreads();
        for (int f = w; f < kFine; f += kWavesPerBlock) {
            const int o0 = (int)s_fo[f];
            const int m = (f + 1 < kFine ? (int)s_fo[f + 1] : c) - o0;
            if (m > kPermFineCap) {
                if (l == 0 && a.status) atomicOr(a.status, APT_STATUS_CAPACITY);
                continue;
            }
            if (m == 0) continue;
            if (m <= kWave) {
                // lane q's rank among the m (key, index) pairs, the others
                // broadcast from their lanes: no sorting network, no LDS
                // round trips
                const uint64_t mk = l < m ? s_k[o0 + l] : ~0ull;
                const uint32_t mv = l < m ? s_v[o0 + l] : ~0u;
                const uint32_t mk_lo = (uint32_t)mk, mk_hi = (uint32_t)(mk >> 32);
                int rank = 0;
                for (int j = 0; j < m; ++j) {
                    const uint64_t kj = ((uint64_t)readlane(mk_hi, j) << 32) | (uint64_t)readlane(mk_lo, j);
                    const uint32_t vj = readlane(mv, j);
                    rank += (kj < mk || (kj == mk && vj < mv)) ? 1 : 0;
                }
                if (l < m) out[s0 - rbase + (uint64_t)(o0 + rank)] = lab[mv];
            } else {
                for (int q = l; q < m; q += kWave) {
                    w_k[w][q] = s_k[o0 + q];
                    w_v[w][q] = s_v[o0 + q];
                }
                int N = 2;
                while (N < m) N <<= 1;
                wave_sort_pairs(w_k[w], w_v[w], m, N);
                for (int q = l; q < m; q += kWave) out[s0 - rbase + (uint64_t)(o0 + q)] = lab[w_v[w][q]];
            }
            wave_sync();
        }
        __syncthreads();
    }
}

}  // namespace apt
