// Label permutation and device-wide scan (apt_perm.hip).
#pragma once
#include "apt_internal.hpp"

namespace apt {

constexpr int kPermCap = 512;   // keys one wavefront sorts per bucket
constexpr int kMaxRepPerLaunch = 64;

// Two-level form for n <= kPermLdsMax: keys dealt into at most 2^13 coarse
// buckets (<= 2048 keys on average) with block-aggregated counts, each coarse
// bucket then sorted by one workgroup in LDS.
constexpr int64_t kPermLdsMax = (int64_t)2048 << 13;
constexpr int kPermCoarseCap = 3584;   // keys of one coarse bucket in LDS
constexpr int kPermFineBits = 6;       // fine buckets per coarse bucket: 64
constexpr int kPermFineCap = 128;      // keys of one fine bucket a wavefront sorts
constexpr int kPermChunk = 65536;      // keys per workgroup when dealing

struct PermArgs {
    const uint8_t* lab;     // [n] labels, original order
    int64_t n;
    int32_t bits;           // bucket bits (2^bits buckets per replicate)
    int32_t n_rep;
    uint64_t seeds[kMaxRepPerLaunch];   // seed of each replicate of the launch
    uint32_t* count;        // [n_rep << bits]: counts, then global starts
    uint32_t* cursor;       // [n_rep << bits]
    uint64_t* ekey;         // [n_rep * n]
    uint32_t* eidx;         // [n_rep * n]
    uint8_t* out;           // out + r * out_stride: permuted labels of replicate r
    int64_t out_stride;
    int32_t* status;
};

int perm_bucket_bits(int64_t n);
int perm_coarse_bits(int64_t n);   // coarse bucket bits of the two-level form (n <= kPermLdsMax)
size_t perm_deal_lds_bytes(int coarse_bits);
void device_excl_scan(uint32_t* x, int64_t n, uint32_t* part, hipStream_t st);

__global__ void k_perm_zero(PermArgs a);
__global__ void k_perm_count(PermArgs a);
__global__ void k_perm_place(PermArgs a);
__global__ void k_perm_sort(PermArgs a);
__global__ void k_permc_count(PermArgs a);
__global__ void k_permc_place(PermArgs a);
__global__ void k_permc_sort(PermArgs a);

}  // namespace apt
