// Label permutation and device-wide scan (apt_perm.hip).
#pragma once
#include "apt_internal.hpp"

namespace apt {

constexpr int kPermCap = 512;   // keys one wavefront sorts per bucket
constexpr int kMaxRepPerLaunch = 64;

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
void device_excl_scan(uint32_t* x, int64_t n, uint32_t* part, hipStream_t st);

__global__ void k_perm_zero(PermArgs a);
__global__ void k_perm_count(PermArgs a);
__global__ void k_perm_place(PermArgs a);
__global__ void k_perm_sort(PermArgs a);

}  // namespace apt
