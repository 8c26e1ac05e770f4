// Host side of the C ABI: argument checks, workspace layout and the launch
// sequence of each entry point.  Nothing here allocates device memory.
#include <math.h>
#include <string.h>

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "apt_batched.hpp"
#include "apt_bin.hpp"
#include "apt_pair.hpp"
#include "apt_perm.hpp"
#include "apt_sdm.hpp"
#include "apt_cluster.hpp"
#include "apt_edge.hpp"
#include "apt_smooth.hpp"

namespace apt {

static thread_local std::string g_err;

static apt_status fail(apt_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

// ---------------------------------------------------------------- device --
struct DevInfo {
    int cus = 0;
};

static DevInfo device_info() {
    static std::mutex mu;
    static DevInfo cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return DevInfo{256};
    std::lock_guard<std::mutex> g(mu);
    if (cache[dev].cus == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cache[dev].cus = cus;
    }
    return cache[dev];
}

// ------------------------------------------------------------- tuning --
static std::mutex g_tune_mu;
static apt_tuning g_tune = {0, 4.0f, 0.5f, 1.0f, 0};

static apt_tuning tuning() {
    std::lock_guard<std::mutex> g(g_tune_mu);
    return g_tune;
}

// ------------------------------------------------------------ tracing --
struct TraceRec {
    std::string stage;
    hipEvent_t a, b;
    int dev;
};
static std::mutex g_trace_mu;
static std::vector<TraceRec> g_trace;
static std::atomic<int> g_trace_on{0};
// events are reused (creating two per stage per call costs host time that
// a fast call cannot hide); one free list per device
static std::map<int, std::vector<hipEvent_t>> g_event_pool;   // guarded by g_trace_mu

static hipEvent_t take_event(int dev) {
    {
        std::lock_guard<std::mutex> g(g_trace_mu);
        auto& v = g_event_pool[dev];
        if (!v.empty()) {
            hipEvent_t e = v.back();
            v.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct TraceSpan {
    hipEvent_t a = nullptr, b = nullptr;
    const char* stage;
    hipStream_t st;
    int dev = 0;
    TraceSpan(const char* s, hipStream_t stream) : stage(s), st(stream) {
        const int on = g_trace_on.load();
        if (!on || (on == 2 && strcmp(s, "pair") != 0 && strcmp(s, "nbr") != 0)) return;
        if (hipGetDevice(&dev) != hipSuccess) return;
        a = take_event(dev);
        b = take_event(dev);
        if (!a || !b) {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
            a = b = nullptr;
            return;
        }
        (void)hipEventRecord(a, st);
    }
    ~TraceSpan() {
        if (!a) return;
        (void)hipEventRecord(b, st);
        std::lock_guard<std::mutex> g(g_trace_mu);
        g_trace.push_back(TraceRec{stage, a, b, dev});
    }
};

// Grid of a one-target-per-wavefront kernel: exactly the workgroups that
// fit on the device at once, so that the static deal of targets runs in a
// single round (a second, partly filled round would leave CUs idle),
// rounded down to a multiple of the XCD count.
// The occupancy query is remembered per (device, kernel, LDS bytes): it
// costs host time on every call otherwise.
template <class K>
static int resident_grid(K kern, size_t lds) {
    static std::mutex mu;
    static std::map<std::tuple<int, const void*, size_t>, int> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const auto key = std::make_tuple(dev, reinterpret_cast<const void*>(kern), lds);
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, kBlock, lds) != hipSuccess || nb < 1) nb = 2;
    // the kernels deal items per XCD (workgroup b on XCD b mod 8, gridDim.x / 8
    // workgroups each): a multiple of kXcd covers every item exactly once
    int grid = device_info().cus * nb / kXcd * kXcd;
    if (grid < kXcd) grid = kXcd;
    std::lock_guard<std::mutex> g(mu);
    cache[key] = grid;
    return grid;
}

// LDS one workgroup may take
constexpr size_t kMaxLds = 64u * 1024u;

// ------------------------------------------------------------ sizing --
constexpr int kCountTile = 4096;

constexpr int kMaxCountBlocks = 2048;
static int count_blocks(int64_t n) {
    int64_t g = (n + kCountTile - 1) / kCountTile;
    if (g < 1) g = 1;
    if (g > kMaxCountBlocks) g = kMaxCountBlocks;
    return (int)g;
}
static int64_t count_chunk(int64_t n, int G) {
    int64_t c = (n + G - 1) / G;
    return (c + kCountTile - 1) / kCountTile * kCountTile;
}
static uint32_t cell_cap_for(int64_t n) {
    int64_t c = n / 2;
    if (c < 65536) c = 65536;
    if (c > 0xFFFFFF00ll) c = 0xFFFFFF00ll;
    return (uint32_t)c;
}
static int sort_passes_max(uint32_t cap) {
    return sort_passes_for(cap - 1u);
}
constexpr int kSortBlocks = 1024;   // most workgroups of a radix pass (the counts matrix is sized for it)
// Workgroups of a radix pass over at most n keys: fewer, fuller ones for
// small clouds (their fixed per-workgroup work dominates there; on the
// 7.7 M-ion needle 512 bin 2 % faster than 1024, on 2e8 ions 1024 win).
static int sort_blocks(int64_t n) { return n <= ((int64_t)1 << 25) ? 512 : kSortBlocks; }

// One radix pass of the sorts in `ss` (grid: their workgroups) over a cloud
// of n ions: upsweep, scan, and the downsweep whose tile suits the size.
static void launch_sort_pass(SortSet& ss, int grid, int64_t n, hipStream_t st) {
    const bool large = n > ((int64_t)1 << 25);
    ss.tile = large ? kDsLargeBlock * kDsLargeItems : kDsSmallBlock * kDsSmallItems;
    hipLaunchKernelGGL(k_rs_upsweep, dim3(grid), dim3(kBlock), 0, st, ss);
    hipLaunchKernelGGL(k_rs_scan, dim3(kRadix * ss.n), dim3(kBlock), 0, st, ss);
    if (large) hipLaunchKernelGGL(k_rs_downsweep_large, dim3(grid), dim3(kDsLargeBlock), 0, st, ss);
    else hipLaunchKernelGGL(k_rs_downsweep_small, dim3(grid), dim3(kDsSmallBlock), 0, st, ss);
}

// Workspace of the plain path (rdf / knn / knn_rdf).
struct PlainWs {
    GridPlan* plan;
    uint32_t* part_cnt;
    float* part_bbox;
    int32_t* part_nf;
    uint32_t* part_off;
    double* E2;
    double* KE2;
    uint32_t* tid;
    uint32_t* bsel;
    uint32_t* K[2];         // target sort keys and values (ping-pong)
    uint32_t* V[2];
    uint32_t* KB[2];        // neighbour sort keys (ping-pong)
    float4* brec2;          // the neighbour records' second buffer (the first is bpos)
    uint32_t* t_rank;
    uint32_t* t_id;
    float* tx;
    float* ty;
    float* tz;
    float4* bpos;
    uint32_t* cell_start;
    uint32_t* rs_counts;
    uint32_t* rs_totals;
    uint32_t* strag;
    uint32_t* strag_count;
    uint32_t* t_cell_start;
    size_t bytes;
};

static PlainWs carve_plain(void* base, int64_t n) {
    Carve c{reinterpret_cast<char*>(base)};
    PlainWs w;
    const size_t N = (size_t)(n > 0 ? n : 1);
    w.plan = c.take<GridPlan>(1);
    w.part_cnt = c.take<uint32_t>(2 * kMaxCountBlocks);
    w.part_bbox = c.take<float>(6 * kMaxCountBlocks);
    w.part_nf = c.take<int32_t>(kMaxCountBlocks);
    w.part_off = c.take<uint32_t>(2 * kMaxCountBlocks);
    w.E2 = c.take<double>(APT_MAX_BINS + 1);
    w.KE2 = c.take<double>(APT_MAX_BINS + 1);
    w.rs_counts = c.take<uint32_t>(2 * 256 * kSortBlocks);   // [sort][256][G]
    w.rs_totals = c.take<uint32_t>(2 * 256);
    w.tid = c.take<uint32_t>(N);
    w.bsel = c.take<uint32_t>(N);
    w.K[0] = c.take<uint32_t>(N);
    w.V[0] = c.take<uint32_t>(N);
    w.K[1] = c.take<uint32_t>(N);
    w.V[1] = c.take<uint32_t>(N);
    w.KB[0] = c.take<uint32_t>(N);
    w.KB[1] = c.take<uint32_t>(N);
    w.brec2 = c.take<float4>(N);
    w.t_rank = c.take<uint32_t>(N);
    w.t_id = c.take<uint32_t>(N);
    w.tx = c.take<float>(N);
    w.ty = c.take<float>(N);
    w.tz = c.take<float>(N);
    w.bpos = c.take<float4>(N);
    w.cell_start = c.take<uint32_t>((size_t)cell_cap_for(n) + 1);
    w.strag = c.take<uint32_t>(N);
    w.strag_count = c.take<uint32_t>(64);
    w.t_cell_start = c.take<uint32_t>((size_t)cell_cap_for(n) + 1);
    w.bytes = c.off;
    return w;
}

// Workspace of the label permutation for n ions and up to r replicates.
struct PermWs {
    uint32_t* count;
    uint32_t* cursor;
    uint32_t* part;
    uint64_t* ekey;
    uint32_t* eidx;
    size_t bytes;
};

// Up to kPermLdsMax labels the two-level form runs (coarse buckets, no key
// array); beyond, fine buckets of about 32 keys with keys and indices.
static bool perm_two_level(int64_t n) { return n <= kPermLdsMax; }

static PermWs carve_perm(void* base, int64_t n, int reps) {
    Carve c{reinterpret_cast<char*>(base)};
    PermWs w;
    const bool two = perm_two_level(n);
    const size_t nb = (size_t)1 << (two ? perm_coarse_bits(n) : perm_bucket_bits(n));
    const size_t N = (size_t)(n > 0 ? n : 1);
    w.count = c.take<uint32_t>(nb * reps);
    w.cursor = c.take<uint32_t>(nb * reps);
    w.part = c.take<uint32_t>(1024);
    w.ekey = two ? nullptr : c.take<uint64_t>(N * reps);
    w.eidx = c.take<uint32_t>(N * reps);
    w.bytes = c.off;
    return w;
}

// Permuted labels of `reps` replicates (seeds[r]) into out + r * out_stride.
static void run_permute(const uint8_t* lab, int64_t n, const uint64_t* seeds, int reps, uint8_t* out,
                        int64_t out_stride, const PermWs& w, int32_t* status, hipStream_t st) {
    for (int r0 = 0; r0 < reps; r0 += kMaxRepPerLaunch) {
        const int nr = reps - r0 < kMaxRepPerLaunch ? reps - r0 : kMaxRepPerLaunch;
        PermArgs pa{};
        const bool two = perm_two_level(n);
        pa.lab = lab;
        pa.n = n;
        pa.bits = two ? perm_coarse_bits(n) : perm_bucket_bits(n);
        pa.n_rep = nr;
        for (int r = 0; r < nr; ++r) pa.seeds[r] = seeds[r0 + r];
        pa.count = w.count;
        pa.cursor = w.cursor;
        pa.ekey = w.ekey;
        pa.eidx = w.eidx;
        pa.out = out + (size_t)r0 * out_stride;
        pa.out_stride = out_stride;
        pa.status = status;
        const int64_t nb = (int64_t)1 << pa.bits;
        const int cus = device_info().cus;
        if (two) {
            const int gd = n > 0 ? (int)((n + kPermChunk - 1) / kPermChunk) : 1;
            hipLaunchKernelGGL(k_perm_zero, dim3(cus * 4), dim3(kBlock), 0, st, pa);
            hipLaunchKernelGGL(k_permc_count, dim3(gd, nr), dim3(kBlock), perm_deal_lds_bytes(pa.bits) / 2, st, pa);
            device_excl_scan(w.count, nb * nr, w.part, st);
            hipLaunchKernelGGL(k_permc_place, dim3(gd, nr), dim3(kBlock), perm_deal_lds_bytes(pa.bits), st, pa);
            hipLaunchKernelGGL(k_permc_sort, dim3((unsigned)nb, nr), dim3(kBlock), 0, st, pa);
            continue;
        }
        int gx = (int)((n + kBlock * 4 - 1) / (kBlock * 4));
        if (gx > cus * 8) gx = cus * 8;
        if (gx < 1) gx = 1;
        hipLaunchKernelGGL(k_perm_zero, dim3(cus * 4), dim3(kBlock), 0, st, pa);
        hipLaunchKernelGGL(k_perm_count, dim3(gx, nr), dim3(kBlock), 0, st, pa);
        device_excl_scan(w.count, nb * nr, w.part, st);
        hipLaunchKernelGGL(k_perm_place, dim3(gx, nr), dim3(kBlock), 0, st, pa);
        int gs = (int)((nb + kWavesPerBlock - 1) / kWavesPerBlock);
        if (gs > cus * 8) gs = cus * 8;
        hipLaunchKernelGGL(k_perm_sort, dim3(gs, nr), dim3(kBlock), 0, st, pa);
    }
}

// Workspace of the batched replicates: the binning of all ions, and per
// block of R replicates their labels, permutation scratch, class segments
// and cell offsets.
constexpr int kMaxPartBlocks = 2048;
static int part_blocks(int64_t n) {
    int64_t g = (n + kPartTile - 1) / kPartTile;
    if (g < 1) g = 1;
    if (g > kMaxPartBlocks) g = kMaxPartBlocks;
    return (int)g;
}
static int batch_reps(int64_t n, int n_rep) {
    int64_t r = n_rep < kMaxRepPerLaunch ? n_rep : kMaxRepPerLaunch;
    const int64_t lim = (int64_t)0xFFFFFFFEll / (n > 0 ? n : 1);
    if (r > lim) r = lim;
    return (int)(r < 1 ? 1 : r);
}

struct BatchWs {
    PlainWs plain;    // plan, partials, edge tables, sort buffers, binned records
    PermWs perm;
    uint8_t* LR;
    uint32_t* cnt;
    float4* Pp;
    uint32_t* Pcell;
    uint32_t* CS;
    uint64_t* items;
    uint64_t* titems;
    uint64_t* work;
    size_t bytes;
};

static BatchWs carve_batched(void* base, int64_t n, int R) {
    BatchWs w;
    w.plain = carve_plain(base, n);
    char* b2 = base ? reinterpret_cast<char*>(base) + w.plain.bytes : nullptr;
    w.perm = carve_perm(b2, n, R);
    Carve c{b2 ? b2 + w.perm.bytes : nullptr};
    c.off = 0;
    const size_t N = (size_t)(n > 0 ? n : 1);
    w.LR = c.take<uint8_t>(N * R);
    w.cnt = c.take<uint32_t>((size_t)R * kMaxClasses * kMaxPartBlocks);
    w.Pp = c.take<float4>(N * R);
    w.Pcell = c.take<uint32_t>(N * R);
    w.CS = c.take<uint32_t>((size_t)R * (kMaxClasses - 1) * ((size_t)cell_cap_for(n) + 1));
    w.items = c.take<uint64_t>((size_t)R * kMaxPairs + 1);
    w.titems = c.take<uint64_t>((size_t)R * kMaxPairs + 1);
    w.work = c.take<uint64_t>(8);
    w.bytes = w.plain.bytes + w.perm.bytes + c.off;
    return w;
}

// ------------------------------------------------------------ checks --
static apt_status check_cloud(const apt_cloud* cl) {
    if (!cl) return fail(APT_E_ARG, "cloud is NULL");
    if (cl->n < 0) return fail(APT_E_ARG, "cloud->n is negative");
    if (cl->n >= (int64_t)0xFFFFFFFFll) return fail(APT_E_UNSUPPORTED, "cloud->n must be below 2^32 - 1");
    if (cl->n > 0 && (!cl->xyz || !cl->lab)) return fail(APT_E_ARG, "cloud->xyz or cloud->lab is NULL");
    return APT_OK;
}
static apt_status check_query(apt_query q) {
    if (isnan(q.d_srf)) return fail(APT_E_ARG, "query.d_srf is NaN");
    return APT_OK;
}
static apt_status check_bins(apt_bins b, const char* what) {
    if (!(b.r_max > 0.0f) || !isfinite(b.r_max))
        return fail(APT_E_ARG, std::string(what) + ".r_max must be finite and > 0");
    if (b.n_bins < 1 || b.n_bins > APT_MAX_BINS)
        return fail(APT_E_ARG, std::string(what) + ".n_bins must be in [1, 65536]");
    return APT_OK;
}
static apt_status check_ws(void* ws, size_t ws_bytes, size_t need) {
    if (!ws) return fail(APT_E_WORKSPACE, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(APT_E_WORKSPACE, "workspace is not 256-byte aligned");
    if (ws_bytes < need)
        return fail(APT_E_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes, got " +
                                         std::to_string(ws_bytes));
    return APT_OK;
}
static apt_status hip_check(const char* where) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(APT_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
    return APT_OK;
}

// ------------------------------------------------------- small kernels --
__global__ void k_init(InitArgs a) {
    init_body(a, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

struct FinishArgs {
    const GridPlan* plan;
    int64_t capacity;
    int64_t* n_targets;
    int32_t* status;
};
__global__ void k_finish(FinishArgs a) {
    const uint32_t nT = a.plan->nT;
    if (a.n_targets) *a.n_targets = (int64_t)nT;
    if (a.capacity >= 0 && (int64_t)nT > a.capacity && a.status) atomicOr(a.status, APT_STATUS_CAPACITY);
}

// The binning stage shared by the plain entry points.  Leaves in the
// workspace: plan, tid (eligible targets ascending), order (their ranks in
// cell order, with rank, index and position), neighbour SoA in cell order
// and cell_start.
// zscale (device, may be NULL) scales z before binning; sel_union makes
// targets and neighbours both the ions that take part in a pair in either
// role.
static apt_status run_binning(const apt_cloud* cl, apt_query q, const PlanParams& pp, const PlainWs& w,
                              int32_t* status, hipStream_t st, const double* zscale = nullptr,
                              int sel_union = 0, const InitArgs* init = nullptr) {
    const int64_t n = cl->n;
    const int G = count_blocks(n);
    const int64_t chunk = count_chunk(n, G);
    const int cus = device_info().cus;

    CountArgs ca{cl->xyz, cl->lab, cl->d_bnd, n, chunk, q.target, q.neighbor, q.d_srf, zscale,
                 w.part_cnt, w.part_bbox, w.part_nf, sel_union};
    if (init) {
        ca.init = *init;
        ca.do_init = 1;
    }
    hipLaunchKernelGGL(k_count, dim3(G), dim3(kBlock), 0, st, ca);
    PlanArgs pa{G, w.part_cnt, w.part_bbox, w.part_nf, w.part_off, pp, zscale, w.plan, status};
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, st, pa);
    const bool all_b = q.neighbor == APT_ANY;
    // the compaction writes both key lists (the plan is known by then)
    CompactArgs cm{cl->lab, cl->d_bnd, n, chunk, q.target, q.neighbor, q.d_srf, w.part_off, w.tid,
                   all_b ? nullptr : w.bsel, sel_union, w.plan, cl->xyz, zscale, w.K[0], w.V[0], w.KB[0],
                   {w.bpos, w.brec2}};
    hipLaunchKernelGGL(k_compact, dim3(G), dim3(kBlock), 0, st, cm);

    // both sorts share each pass's launches; target keys never need more
    // bytes than cell ids (the plan falls back to cell order when its
    // block-raster keys would)
    const int passes = sort_passes_max(pp.cell_cap);
    const int Gk = cus * 8;
    // the target sort on half the workgroups: targets are usually the rarer
    // species (on the needle's queries binning −2 to −5.5 %; a query whose
    // targets are the majority species bins ≈ 5 % slower)
    const int Gs = sort_blocks(n), GsT = Gs / 2;
    for (int p = 0; p < passes; ++p) {
        SortSet ss{};
        ss.s[0] = SortArgs{w.plan, 1, p, GsT, {w.K[0], w.K[1]}, {w.V[0], w.V[1]}, w.rs_counts, w.rs_totals};
        // the neighbours' 16-byte records travel with their keys: no random
        // position reads after the sort
        ss.s[1] = SortArgs{w.plan, 0, p, Gs, {w.KB[0], w.KB[1]}, {nullptr, nullptr},
                           w.rs_counts + (size_t)256 * kSortBlocks, w.rs_totals + 256, {w.bpos, w.brec2}};
        ss.n = 2;
        launch_sort_pass(ss, GsT + Gs, n, st);
    }
    // targets in cell order and the neighbour records, in one launch;
    // occupied cells (distinct sorted keys) feed the kNN radii
    const bool occ = pp.k > 0 && !zscale;
    OrderArgs oa{w.plan, cl->xyz, w.tid, {w.V[0], w.V[1]}, w.t_rank, w.t_id, w.tx, w.ty, w.tz,
                 {w.K[0], w.K[1]}, occ ? w.strag_count + 1 : nullptr, w.t_cell_start};
    GatherArgs ga{w.plan, nullptr, zscale, {w.KB[0], w.KB[1]}, {nullptr, nullptr}, w.bpos, w.cell_start,
                  occ ? w.strag_count + 2 : nullptr};
    // (up to 2^25 ions half the usual grid per half: more records per thread
    // beat more workgroups, −2 % on 7.5e6 records; beyond, the full grid:
    // at 2e9 records the half grid's fewer loads in flight cost 2 %)
    const int Go = n > ((int64_t)1 << 25) ? Gk : Gk / 2;
    hipLaunchKernelGGL(k_order_gather, dim3(2 * Go), dim3(kBlock), 0, st, oa, ga, Go);
    return hip_check("binning launch");
}

// The whole plain path.  rdf_hist / knn outputs may be absent.
// cand (diagnostic, device u64): bin as the call would, then count the RDF
// stencil's candidates into *cand instead of running the pair kernels.
static apt_status run_plain(const apt_cloud* cl, apt_query q, const apt_bins* rb, uint64_t* rdf_hist,
                            int32_t k, float r_knn_max, int64_t capacity, int64_t* target_id,
                            float* dist, int64_t* nbr_id, const apt_bins* kb, uint64_t* knn_hist,
                            int64_t* n_targets, int32_t* status, void* ws, size_t ws_bytes,
                            void* stream, uint64_t* cand = nullptr) {
    apt_status s;
    if ((s = check_cloud(cl)) != APT_OK) return s;
    if ((s = check_query(q)) != APT_OK) return s;
    if (!status) return fail(APT_E_ARG, "status is NULL");
    const bool do_rdf = rb != nullptr, do_knn = k > 0;
    if (do_rdf) {
        if ((s = check_bins(*rb, "rdf_bins")) != APT_OK) return s;
        if (!rdf_hist && !cand) return fail(APT_E_ARG, "rdf histogram output is NULL");
    }
    if (do_knn) {
        if (k > APT_MAX_K) return fail(APT_E_UNSUPPORTED, "k must be in [1, 256]");
        if (!(r_knn_max > 0.0f)) return fail(APT_E_ARG, "r_knn_max must be > 0 (or +inf)");
        if (capacity < 0) return fail(APT_E_ARG, "capacity is negative");
        if (!cand) {
            if (capacity > 0 && (!target_id || !dist || !nbr_id)) return fail(APT_E_ARG, "kNN row output is NULL");
            if (!n_targets) return fail(APT_E_ARG, "n_targets is NULL");
        }
        if (knn_hist && (s = check_bins(*kb, "knn_bins")) != APT_OK) return s;
    }
    PlainWs w = carve_plain(ws, cl->n);
    if ((s = check_ws(ws, ws_bytes, w.bytes)) != APT_OK) return s;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();

    InitArgs ia{status, cand ? cand : rdf_hist, cand ? 1 : (do_rdf ? rb->n_bins : 0), knn_hist,
                knn_hist ? kb->n_bins + 1 : 0, n_targets, w.strag_count,
                do_rdf ? w.E2 : nullptr, do_rdf ? rb->r_max : 0.0f, do_rdf ? rb->n_bins : 0,
                knn_hist ? w.KE2 : nullptr, knn_hist ? kb->r_max : 0.0f, knn_hist ? kb->n_bins : 0};
    ia.work_q = w.strag_count + 8;
    // (zeroed and filled by the binning's first kernel)

    const apt_tuning tu = tuning();
    const bool rdf_lds = do_rdf && pair_lds_bytes(true, do_knn, rb->n_bins, true) <= kMaxLds;
    const bool tile_fits = !do_rdf || tile_lds_bytes(true, rb->n_bins) <= kMaxLds;
    PlanParams pp;
    pp.h_min = do_rdf ? rb->r_max * tu.h_min_frac : 0.0f;
    pp.occ = tu.cell_occ;
    pp.tile_occ = tu.tile_occ;
    pp.k = do_knn ? k : 0;
    pp.cell_cap = cell_cap_for(cl->n);
    // tiles need an LDS histogram and at most 16 kNN keys per lane
    pp.tile_policy = (!tile_fits || (do_knn && k > 16)) ? 1 : tu.tile_policy;
    pp.r_enum = do_rdf ? rb->r_max : 0.0f;
    pp.h_shrink = 0.7f;
    pp.rdf_kernel = tu.rdf_kernel;
    {
        TraceSpan span("binning", st);
        if ((s = run_binning(cl, q, pp, w, status, st, nullptr, 0, &ia)) != APT_OK) return s;
    }
    if (cand) {
        hipLaunchKernelGGL(k_count_candidates, dim3(device_info().cus * 8), dim3(kBlock), 0, st, w.plan,
                           do_knn ? w.strag_count + 1 : nullptr, w.cell_start, w.tx, w.ty, w.tz, rb->r_max,
                           do_knn ? k : 0, reinterpret_cast<unsigned long long*>(cand));
        if (pp.tile_policy != 1) {
            // mode 3: the neighbour-major kernel's pair evaluations instead
            PairArgs ca{};
            ca.plan = w.plan;
            ca.tx = w.tx;
            ca.ty = w.ty;
            ca.tz = w.tz;
            ca.t_id = w.t_id;
            ca.bpos = w.bpos;
            ca.t_cell_start = w.t_cell_start;
            ca.work_q = w.strag_count + 8;
            ca.r_enum = (float)((double)rb->r_max * (1.0 + 4e-5));
            ca.hist = cand;
            ca.n_bins = 1;
            const size_t nl = nbr_lds_bytes(1, false);
            auto kern = k_rdf_nbr<kRdfGlobal | kCountEvals>;
            hipLaunchKernelGGL(kern, dim3(resident_grid(kern, nl)), dim3(kBlock), nl, st, ca);
        }
        return hip_check("candidate count launch");
    }

    PairArgs pa{};
    pa.plan = w.plan;
    pa.xyz = cl->xyz;
    pa.t_rank = w.t_rank;
    pa.t_id = w.t_id;
    pa.tx = w.tx;
    pa.ty = w.ty;
    pa.tz = w.tz;
    pa.bpos = w.bpos;
    pa.cell_start = w.cell_start;
    pa.self_possible = q.target == APT_ANY || q.neighbor == APT_ANY || q.target == q.neighbor;
    pa.lab = cl->lab;
    pa.nbr_species = q.neighbor;
    int n_bins = 1;
    bool in_lds = false;
    if (do_rdf) {
        n_bins = rb->n_bins;
        const double rmax = (double)rb->r_max;
        pa.n_bins = n_bins;
        // FP32 fast path: the bin of sqrt(d2f) is off from the FP64 bin only
        // within ~1e-4 bins of an edge (relative error of d2f, sqrt and the
        // scaling < 7 ulp); pairs within delta of an edge (at least 1e-6 nm)
        // are re-decided in FP64.
        const double w_bin = rmax / n_bins;
        double delta = fmax(1e-6, 2e-6 * rmax);
        double delta_b = fmax(delta / w_bin, 4e-6 * n_bins);
        if (delta_b > 0.25) delta_b = 0.25;
        pa.delta_b = (float)delta_b;
        pa.inv_w = (float)(n_bins / rmax);
        pa.inv_w64 = n_bins / rmax;
        pa.thr2 = (float)((rmax * (1.0 + 2e-5)) * (rmax * (1.0 + 2e-5)));
        pa.r_enum = (float)(rmax * (1.0 + 4e-5));
        pa.E2 = w.E2;
        pa.hist = rdf_hist;
        in_lds = rdf_lds;
        pa.hist_in_lds = in_lds ? 1 : 0;
    }
    if (do_knn) {
        pa.k = k;
        pa.rknn = r_knn_max;
        pa.rknn2 = r_knn_max * r_knn_max;
        pa.capacity = capacity;
        pa.target_id = target_id;
        pa.dist = dist;
        pa.nbr_id = nbr_id;
        pa.knn_hist = knn_hist;
        if (knn_hist) {
            pa.kb_nbins = kb->n_bins;
            pa.kb_inv_w64 = kb->n_bins / (double)kb->r_max;
            pa.KE2 = w.KE2;
        }
    }
    pa.strag = w.strag;
    pa.strag_count = w.strag_count;
    pa.t_cell_start = w.t_cell_start;
    pa.work_q = w.strag_count + 8;
    // the kNN radii from the occupied cells that the binning counted
    pa.occ = do_knn ? w.strag_count + 1 : nullptr;
    pa.n_targets = do_knn ? n_targets : nullptr;
    pa.status = status;
    const size_t lds = pair_lds_bytes(do_rdf, do_knn, n_bins, in_lds);
    if (pp.tile_policy != 1 && do_rdf) {
        // the RDF neighbour-major when the plan chooses mode 3 (exits otherwise)
        TraceSpan span("nbr", st);
        const bool self = pa.self_possible != 0;
        const size_t nl = nbr_lds_bytes(n_bins, in_lds);
        auto go = [&](auto kern) { hipLaunchKernelGGL(kern, dim3(resident_grid(kern, nl)), dim3(kBlock), nl, st, pa); };
        if (self)
            hipLaunchKernelGGL(k_nbr_self, dim3(std::max(1, device_info().cus * 2)), dim3(kBlock), 0, st, pa);
        if (in_lds) go(k_rdf_nbr<kRdfLds>);
        else go(k_rdf_nbr<kRdfGlobal>);
        if (tu.rdf_kernel == 2) {
            // (the tuning asks for the one-target-per-wavefront RDF in mode 3)
            const size_t tl = pair_lds_bytes(true, false, n_bins, in_lds);
            auto go2 = [&](auto kern) { hipLaunchKernelGGL(kern, dim3(resident_grid(kern, tl)), dim3(kBlock), tl, st, pa); };
            if (in_lds) self ? go2(k_rdf_tgt<kRdfLds | kSelf>) : go2(k_rdf_tgt<kRdfLds>);
            else self ? go2(k_rdf_tgt<kRdfGlobal | kSelf>) : go2(k_rdf_tgt<kRdfGlobal>);
        }
    }
    if (pp.tile_policy != 1) {
        // 64 targets per wavefront when the plan chooses it (exits otherwise)
        TraceSpan span("tile", st);
        const bool self = pa.self_possible != 0;
        const size_t tl = tile_lds_bytes(do_rdf, n_bins);
        auto go = [&](auto kern) { hipLaunchKernelGGL(kern, dim3(resident_grid(kern, tl)), dim3(kBlock), tl, st, pa); };
        const int km = !do_knn ? 0 : k <= 4 ? 4 : k <= 10 ? 10 : 16;
        if (do_rdf) {
            if (km == 0) self ? go(k_pair_tile<kRdfLds | kSelf, 0>) : go(k_pair_tile<kRdfLds, 0>);
            else if (km == 4) self ? go(k_pair_tile<kRdfLds | kSelf, 4>) : go(k_pair_tile<kRdfLds, 4>);
            else if (km == 10) self ? go(k_pair_tile<kRdfLds | kSelf, 10>) : go(k_pair_tile<kRdfLds, 10>);
            else self ? go(k_pair_tile<kRdfLds | kSelf, 16>) : go(k_pair_tile<kRdfLds, 16>);
        } else {
            if (km == 4) self ? go(k_pair_tile<kSelf, 4>) : go(k_pair_tile<0, 4>);
            else if (km == 10) self ? go(k_pair_tile<kSelf, 10>) : go(k_pair_tile<0, 10>);
            else self ? go(k_pair_tile<kSelf, 16>) : go(k_pair_tile<0, 16>);
        }
    }
    {
        TraceSpan span("pair", st);
        const bool self = pa.self_possible != 0;
        auto go = [&](auto kern) { hipLaunchKernelGGL(kern, dim3(resident_grid(kern, lds)), dim3(kBlock), lds, st, pa); };
        // RDF histograms in LDS unless there are too many bins
        if (do_rdf && !in_lds) {
            if (do_knn) self ? go(k_pair<kRdfGlobal | kSelf, true>) : go(k_pair<kRdfGlobal, true>);
            else self ? go(k_pair<kRdfGlobal | kSelf, false>) : go(k_pair<kRdfGlobal, false>);
        } else if (do_rdf && do_knn) {
            self ? go(k_pair<kRdfLds | kSelf, true>) : go(k_pair<kRdfLds, true>);
        } else if (do_rdf) {
            self ? go(k_pair<kRdfLds | kSelf, false>) : go(k_pair<kRdfLds, false>);
        } else {
            self ? go(k_pair<kSelf, true>) : go(k_pair<0, true>);
        }
    }
    return hip_check("pair launch");
}

// Argument checks of the batched path (no GPU work).
static apt_status check_batched(const apt_cloud* cl, const apt_query* pairs, int32_t n_pairs, const uint64_t* seeds,
                                int32_t n_rep, apt_bins rb, int32_t k, apt_bins kb, uint64_t* rdf_hist,
                                uint64_t* knn_hist, int32_t* status) {
    apt_status s;
    if ((s = check_cloud(cl)) != APT_OK) return s;
    if (!pairs || n_pairs < 1) return fail(APT_E_ARG, "pairs is NULL or n_pairs < 1");
    if (n_pairs > kMaxPairs) return fail(APT_E_UNSUPPORTED, "at most 16 pairs per call");
    if (!seeds || n_rep < 1) return fail(APT_E_ARG, "seeds is NULL or n_rep < 1");
    if ((s = check_bins(rb, "rdf_bins")) != APT_OK) return s;
    if (!rdf_hist) return fail(APT_E_ARG, "rdf_hist is NULL");
    if (k < 1) return fail(APT_E_ARG, "k must be >= 1");
    if (k > APT_MAX_K) return fail(APT_E_UNSUPPORTED, "k must be in [1, 256]");
    if (knn_hist && (s = check_bins(kb, "knn_bins")) != APT_OK) return s;
    if (!status) return fail(APT_E_ARG, "status is NULL");
    if (batched_lds_bytes(rb.n_bins) > kMaxLds)
        return fail(APT_E_UNSUPPORTED, "batched RDF supports at most 3072 bins");
    // the output histograms are zeroed and indexed with 32-bit counts
    const int64_t nh = (int64_t)n_rep * n_pairs * rb.n_bins;
    const int64_t nk = knn_hist ? (int64_t)n_rep * n_pairs * ((int64_t)kb.n_bins + 1) : 0;
    if (nh > (int64_t)INT32_MAX || nk > (int64_t)INT32_MAX)
        return fail(APT_E_UNSUPPORTED, "n_rep * n_pairs * bins must stay below 2^31 for each histogram");
    // species -> class; every species of the pairs gets one class
    uint8_t slot[256];
    int C = 0;
    int cls_of[256];
    for (int q = 0; q < 256; ++q) cls_of[q] = -1;
    for (int p = 0; p < n_pairs; ++p) {
        if (isnan(pairs[p].d_srf)) return fail(APT_E_ARG, "pair d_srf is NaN");
        for (int v = 0; v < 2; ++v) {
            const int sp = v ? pairs[p].neighbor : pairs[p].target;
            if (sp == APT_ANY) return fail(APT_E_UNSUPPORTED, "batched pairs name concrete species (not APT_ANY)");
            if (cls_of[sp] < 0) {
                if (C >= kMaxClasses - 1) return fail(APT_E_UNSUPPORTED, "at most 7 species over all pairs");
                cls_of[sp] = C++;
            }
        }
    }
    (void)slot;
    return APT_OK;
}

// The batched path with a resolved tuning.  mid (optional) is recorded on
// the stream once all ions are binned (the autotuner splits its trial
// times there).
static apt_status run_batched(const apt_cloud* cl, const apt_query* pairs, int32_t n_pairs, const uint64_t* seeds,
                              int32_t n_rep, apt_bins rb, int32_t k, apt_bins kb, uint64_t* rdf_hist,
                              uint64_t* knn_hist, int32_t* status, void* ws, size_t ws_bytes, void* stream,
                              const apt_batched_tuning& bt, hipEvent_t mid = nullptr) {
    apt_status s;
    if ((s = check_cloud(cl)) != APT_OK) return s;
    if (!pairs || n_pairs < 1) return fail(APT_E_ARG, "pairs is NULL or n_pairs < 1");
    if (n_pairs > kMaxPairs) return fail(APT_E_UNSUPPORTED, "at most 16 pairs per call");
    if (!seeds || n_rep < 1) return fail(APT_E_ARG, "seeds is NULL or n_rep < 1");
    if ((s = check_bins(rb, "rdf_bins")) != APT_OK) return s;
    if (!rdf_hist) return fail(APT_E_ARG, "rdf_hist is NULL");
    if (k < 1) return fail(APT_E_ARG, "k must be >= 1");
    if (k > APT_MAX_K) return fail(APT_E_UNSUPPORTED, "k must be in [1, 256]");
    if (knn_hist && (s = check_bins(kb, "knn_bins")) != APT_OK) return s;
    if (!status) return fail(APT_E_ARG, "status is NULL");
    if (batched_lds_bytes(rb.n_bins) > kMaxLds)
        return fail(APT_E_UNSUPPORTED, "batched RDF supports at most 3072 bins");
    // the output histograms are zeroed and indexed with 32-bit counts
    const int64_t nh = (int64_t)n_rep * n_pairs * rb.n_bins;
    const int64_t nk = knn_hist ? (int64_t)n_rep * n_pairs * ((int64_t)kb.n_bins + 1) : 0;
    if (nh > (int64_t)INT32_MAX || nk > (int64_t)INT32_MAX)
        return fail(APT_E_UNSUPPORTED, "n_rep * n_pairs * bins must stay below 2^31 for each histogram");
    // species -> class; every species of the pairs gets one class
    uint8_t slot[256];
    int C = 0;
    int cls_of[256];
    for (int q = 0; q < 256; ++q) cls_of[q] = -1;
    for (int p = 0; p < n_pairs; ++p) {
        if (isnan(pairs[p].d_srf)) return fail(APT_E_ARG, "pair d_srf is NaN");
        for (int v = 0; v < 2; ++v) {
            const int sp = v ? pairs[p].neighbor : pairs[p].target;
            if (sp == APT_ANY) return fail(APT_E_UNSUPPORTED, "batched pairs name concrete species (not APT_ANY)");
            if (cls_of[sp] < 0) {
                if (C >= kMaxClasses - 1) return fail(APT_E_UNSUPPORTED, "at most 7 species over all pairs");
                cls_of[sp] = C++;
            }
        }
    }
    const int Cn = C + 1;   // plus "other"
    for (int q = 0; q < 256; ++q) slot[q] = (uint8_t)(cls_of[q] >= 0 ? cls_of[q] : C);
    const int64_t n = cl->n;
    int R = batch_reps(n, n_rep);
    if (bt.rep_block > 0 && bt.rep_block < R) R = bt.rep_block;
    BatchWs w = carve_batched(ws, n, R);
    if ((s = check_ws(ws, ws_bytes, w.bytes)) != APT_OK) return s;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    const int cus = device_info().cus;

    // zero the outputs and the status word, edge tables
    InitArgs ia{status, rdf_hist, (int32_t)nh, knn_hist, (int32_t)nk, nullptr, nullptr,
                w.plain.E2, rb.r_max, rb.n_bins, knn_hist ? w.plain.KE2 : nullptr, kb.r_max, kb.n_bins};
    hipLaunchKernelGGL(k_init, dim3(cus * 4), dim3(256), 0, st, ia);

    // all ions binned once: records in cell order (w.plain.bpos), cell ids
    {
        TraceSpan span("binning", st);
        const PlainWs& pw = w.plain;
        const int G = count_blocks(n);
        const int64_t chunk = count_chunk(n, G);
        CountArgs ca{cl->xyz, cl->lab, nullptr, n, chunk, APT_ANY, APT_ANY, 0.0f, nullptr, pw.part_cnt, pw.part_bbox,
                     pw.part_nf};
        hipLaunchKernelGGL(k_count, dim3(G), dim3(kBlock), 0, st, ca);
        PlanParams pp{rb.r_max * bt.cell_frac, 4.0f, k, cell_cap_for(n), 1, rb.r_max};
        PlanArgs pa{G, pw.part_cnt, pw.part_bbox, pw.part_nf, pw.part_off, pp, nullptr, pw.plan, status};
        hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, st, pa);
        const int Gk = cus * 8;
        const int Gs = sort_blocks(n);
        KeyArgs kk{pw.plan, cl->xyz, nullptr, nullptr, 0, 0, pw.K[0], pw.V[0]};
        hipLaunchKernelGGL(k_keys, dim3(Gk), dim3(kBlock), 0, st, kk);
        for (int p = 0; p < sort_passes_max(pp.cell_cap); ++p) {
            SortSet ss{};
            ss.s[0] = SortArgs{pw.plan, 0, p, Gs, {pw.K[0], pw.K[1]}, {pw.V[0], pw.V[1]}, pw.rs_counts,
                               pw.rs_totals};
            ss.n = 1;
            launch_sort_pass(ss, Gs, n, st);
        }
        GatherArgs ga{pw.plan, cl->xyz, nullptr, {pw.K[0], pw.K[1]}, {pw.V[0], pw.V[1]}, pw.bpos, pw.cell_start,
                      nullptr};
        hipLaunchKernelGGL(k_gather, dim3(Gk), dim3(kBlock), 0, st, ga);
    }

    {
        // occupied cells of the all-ion grid (work[4] holds the count)
        InitArgs oa{nullptr, nullptr, 0, nullptr, 0, nullptr, reinterpret_cast<uint32_t*>(w.work + 4)};
        hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, st, oa);
        hipLaunchKernelGGL(k_occupied, dim3(cus * 4), dim3(kBlock), 0, st, w.plain.plan, w.plain.cell_start,
                           reinterpret_cast<uint32_t*>(w.work + 4));
    }
    if (mid) (void)hipEventRecord(mid, st);
    const int Gp = part_blocks(n);
    const int64_t pchunk = ((n + Gp - 1) / Gp + kPartTile - 1) / kPartTile * kPartTile;
    const size_t lds = batched_lds_bytes(rb.n_bins);
    const double w_bin = (double)rb.r_max / rb.n_bins;
    double delta_b = fmax(fmax(1e-6, 2e-6 * (double)rb.r_max) / w_bin, 4e-6 * rb.n_bins);
    if (delta_b > 0.25) delta_b = 0.25;
    for (int r0 = 0; r0 < n_rep; r0 += R) {
        const int nr = n_rep - r0 < R ? n_rep - r0 : R;
        {
            TraceSpan span("permute", st);
            run_permute(cl->lab, n, seeds + r0, nr, w.LR, n, w.perm, status, st);
        }
        PartArgs pa{};
        pa.plan = w.plain.plan;
        pa.S = w.plain.bpos;
        pa.keys[0] = w.plain.K[0];
        pa.keys[1] = w.plain.K[1];
        pa.vals[0] = w.plain.V[0];
        pa.vals[1] = w.plain.V[1];
        pa.LR = w.LR;
        pa.n = n;
        pa.chunk = pchunk;
        pa.G = Gp;
        pa.C = Cn;
        for (int q = 0; q < 256; ++q) pa.slot[q] = slot[q];
        pa.cnt = w.cnt;
        pa.Pp = w.Pp;
        pa.Pcell = w.Pcell;
        pa.CS = w.CS;
        pa.cs_stride = (int64_t)cell_cap_for(n) + 1;
        {
            TraceSpan span("partition", st);
            hipLaunchKernelGGL(k_bpart_count, dim3(Gp, nr), dim3(kBlock), 0, st, pa);
            device_excl_scan(w.cnt, (int64_t)nr * Cn * Gp, w.perm.part, st);
            hipLaunchKernelGGL(k_bpart_scatter, dim3(Gp, nr), dim3(kBlock), 0, st, pa);
            hipLaunchKernelGGL(k_bpart_cells, dim3(cus * 4, nr), dim3(kBlock), 0, st, pa);
            hipLaunchKernelGGL(k_bpart_empty, dim3(64, nr * (Cn - 1)), dim3(kBlock), 0, st, pa);
        }

        BatchPairArgs ba{};
        ba.plan = w.plain.plan;
        ba.xyz = cl->xyz;
        ba.d_bnd = cl->d_bnd;
        ba.Pp = w.Pp;
        ba.CS = w.CS;
        ba.cs_stride = pa.cs_stride;
        ba.cnt = w.cnt;
        ba.G = Gp;
        ba.C = Cn;
        ba.R = nr;
        ba.n_pairs = n_pairs;
        ba.n = n;
        ba.rep0 = r0;
        for (int p = 0; p < n_pairs; ++p) {
            ba.pairs[p].a = cls_of[pairs[p].target];
            ba.pairs[p].b = cls_of[pairs[p].neighbor];
            ba.pairs[p].d_srf = pairs[p].d_srf;
        }
        ba.items = w.items;
        ba.titems = w.titems;
        ba.work = w.work;
        ba.tile_ok = (k <= 16 && batched_tile_lds_bytes(rb.n_bins) <= kMaxLds && bt.tiles == 0) ? 1 : 0;
        ba.tile_reach = bt.tile_reach;
        ba.occ = reinterpret_cast<const uint32_t*>(w.work + 4);
        ba.n_bins = rb.n_bins;
        ba.r_enum = (float)((double)rb.r_max * (1.0 + 4e-5));
        ba.thr2 = (float)(((double)rb.r_max * (1.0 + 2e-5)) * ((double)rb.r_max * (1.0 + 2e-5)));
        ba.inv_w = (float)(rb.n_bins / (double)rb.r_max);
        ba.delta_b = (float)delta_b;
        ba.inv_w64 = rb.n_bins / (double)rb.r_max;
        ba.E2 = w.plain.E2;
        ba.rdf_hist = rdf_hist;
        ba.k = k;
        ba.kb_nbins = knn_hist ? kb.n_bins : 0;
        ba.kb_inv_w64 = knn_hist ? kb.n_bins / (double)kb.r_max : 0.0;
        ba.KE2 = w.plain.KE2;
        ba.knn_hist = knn_hist;
        hipLaunchKernelGGL(k_batch_items, dim3(1), dim3(64), 0, st, ba);
        {
            TraceSpan span2("pair", st);
            hipLaunchKernelGGL(k_pair_batched, dim3(cus * 8), dim3(kBlock), lds, st, ba);
        }
        if (ba.tile_ok) {
            TraceSpan span3("tile", st);
            const size_t tl = batched_tile_lds_bytes(rb.n_bins);
            auto go = [&](auto kern) {
                hipLaunchKernelGGL(kern, dim3(resident_grid(kern, tl)), dim3(kBlock), tl, st, ba);
            };
            if (k <= 4) go(k_pair_batched_tile<4>);
            else if (k <= 10) go(k_pair_batched_tile<10>);
            else go(k_pair_batched_tile<16>);
        }
    }
    return hip_check("batched launch");
}

// ------------------------------------------------- batched plans --
// apt_rdf_batched(tuning = NULL): the tuning comes from a process-wide plan
// cache keyed by what decides the best one (device, n, the pairs, bins, k,
// whether the k-th histogram is wanted), filled on a miss by timing trial
// launches; the launch sequence is captured once per call signature into a
// HIP graph and replayed.
static const apt_batched_tuning kBatchedDefaults = {0.5f, 0, 1.3f, 0};

static apt_status resolve_batched_tuning(const apt_batched_tuning* t, apt_batched_tuning* out) {
    apt_batched_tuning v = kBatchedDefaults;
    if (t) {
        if (!(t->cell_frac >= 0.0f && t->cell_frac <= 4.0f))
            return fail(APT_E_ARG, "tuning.cell_frac must be in (0, 4] (0: default)");
        if (t->rep_block < 0 || t->rep_block > kMaxRepPerLaunch)
            return fail(APT_E_ARG, "tuning.rep_block must be in [1, 64] (0: default)");
        if (!(t->tile_reach == 0.0f || (t->tile_reach >= 1.0f && t->tile_reach <= 4.0f)))
            return fail(APT_E_ARG, "tuning.tile_reach must be in [1, 4] (0: default)");
        if (t->tiles != 0 && t->tiles != 1) return fail(APT_E_ARG, "tuning.tiles must be 0 or 1");
        v = *t;
        if (v.cell_frac == 0.0f) v.cell_frac = kBatchedDefaults.cell_frac;
        if (v.tile_reach == 0.0f) v.tile_reach = kBatchedDefaults.tile_reach;
    }
    *out = v;
    return APT_OK;
}

template <class T>
static void key_put(std::string& k, const T& v) {
    k.append(reinterpret_cast<const char*>(&v), sizeof(T));
}

static std::string batched_plan_key(const apt_cloud* cl, const apt_query* pairs, int32_t n_pairs, apt_bins rb,
                                    int32_t k, apt_bins kb, bool want_knn) {
    std::string key;
    int dev = 0;
    (void)hipGetDevice(&dev);
    key_put(key, dev);
    key_put(key, cl->n);
    key_put(key, cl->d_bnd != nullptr);
    key_put(key, n_pairs);
    for (int p = 0; p < n_pairs; ++p) {
        key_put(key, pairs[p].target);
        key_put(key, pairs[p].neighbor);
        key_put(key, pairs[p].d_srf);
    }
    key_put(key, rb.r_max);
    key_put(key, rb.n_bins);
    key_put(key, k);
    key_put(key, want_knn);
    if (want_knn) {
        key_put(key, kb.r_max);
        key_put(key, kb.n_bins);
    }
    return key;
}

static std::mutex g_plan_mu;
static std::map<std::string, apt_batched_tuning> g_plans;

// Trial launches of a few replicates for a grid of cell edges and tile
// reaches, timed with events on the caller's stream; the score weights the
// per-replicate time by the call's replicate count.
static apt_status autotune_batched(const apt_cloud* cl, const apt_query* pairs, int32_t n_pairs, const uint64_t* seeds,
                                   int32_t n_rep, apt_bins rb, int32_t k, apt_bins kb, uint64_t* rdf_hist,
                                   uint64_t* knn_hist, int32_t* status, void* ws, size_t ws_bytes, void* stream,
                                   apt_batched_tuning* best) {
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int nt = n_rep < 4 ? n_rep : 4;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto& f : ev)
                if (f) (void)hipEventDestroy(f);
            return fail(APT_E_HIP, "autotune: hipEventCreate failed");
        }
    apt_batched_tuning base = kBatchedDefaults;
    base.rep_block = nt;
    apt_status s = run_batched(cl, pairs, n_pairs, seeds, nt, rb, k, kb, rdf_hist, knn_hist, status, ws, ws_bytes,
                               stream, base);                  // warm-up
    double best_score = INFINITY;
    *best = kBatchedDefaults;
    const float cells[] = {0.35f, 0.5f, 0.7f};
    const float reaches[] = {1.15f, 1.3f, 1.6f};
    for (float cf : cells) {
        for (float tr : reaches) {
            if (s != APT_OK) break;
            apt_batched_tuning t = base;
            t.cell_frac = cf;
            t.tile_reach = tr;
            (void)hipEventRecord(ev[0], st);
            s = run_batched(cl, pairs, n_pairs, seeds, nt, rb, k, kb, rdf_hist, knn_hist, status, ws, ws_bytes,
                            stream, t, ev[1]);
            (void)hipEventRecord(ev[2], st);
            if (s != APT_OK) break;
            float t_bin = 0.0f, t_rep = 0.0f;
            if (hipEventSynchronize(ev[2]) != hipSuccess || hipEventElapsedTime(&t_bin, ev[0], ev[1]) != hipSuccess ||
                hipEventElapsedTime(&t_rep, ev[1], ev[2]) != hipSuccess) {
                s = fail(APT_E_HIP, "autotune: event timing failed");
                break;
            }
            const double score = (double)t_bin + (double)t_rep * (double)n_rep / (double)nt;
            if (score < best_score) {
                best_score = score;
                *best = t;
            }
        }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    best->rep_block = 0;      // as many replicates per block as the workspace holds
    return s;
}

struct GraphEntry {
    std::string key;
    hipGraph_t graph;
    hipGraphExec_t exec;
};
static std::mutex g_graph_mu;
static std::vector<GraphEntry> g_graphs;     // most recent last
constexpr size_t kMaxGraphs = 8;

static void drop_graph(GraphEntry& e) {
    (void)hipGraphExecDestroy(e.exec);
    (void)hipGraphDestroy(e.graph);
}

// A stream of the library's own per device to capture on (a capture does
// not run anything; the graph is launched on the caller's stream, which may
// be the null stream).  Default priority.
static hipStream_t capture_stream() {
    static std::mutex mu;
    static std::map<int, hipStream_t> streams;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> g(mu);
    auto it = streams.find(dev);
    if (it != streams.end()) return it->second;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    streams[dev] = s;
    return s;
}

// ------------------------------------------------- two-point statistic --
static apt_status run_sdm(const apt_cloud* cl, apt_query q, float R, int32_t n_vox, uint64_t* hist, int32_t* status,
                          void* ws, size_t ws_bytes, void* stream) {
    apt_status s;
    if ((s = check_cloud(cl)) != APT_OK) return s;
    if ((s = check_query(q)) != APT_OK) return s;
    if (!(R > 0.0f) || !isfinite(R)) return fail(APT_E_ARG, "R must be finite and > 0");
    if (n_vox < 1 || n_vox > kSdmMaxVox) return fail(APT_E_ARG, "n_vox must be in [1, 512]");
    if (!hist) return fail(APT_E_ARG, "hist is NULL");
    if (!status) return fail(APT_E_ARG, "status is NULL");
    PlainWs w = carve_plain(ws, cl->n);
    if ((s = check_ws(ws, ws_bytes, w.bytes)) != APT_OK) return s;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    const int64_t nv = (int64_t)n_vox * n_vox * n_vox;
    InitArgs ia{status, hist, (int32_t)nv, nullptr, 0, nullptr, w.strag_count};
    const apt_tuning tu = tuning();
    const double Rd = (double)R;
    PlanParams pp;
    pp.h_min = R * tu.h_min_frac;
    pp.occ = tu.cell_occ;
    pp.tile_occ = tu.tile_occ;
    pp.k = 0;
    pp.cell_cap = cell_cap_for(cl->n);
    pp.tile_policy = 1;                        // one target per wavefront
    pp.r_enum = (float)(Rd * (1.0 + 4e-5));
    pp.h_shrink = 0.7f;
    {
        TraceSpan span("binning", st);
        if ((s = run_binning(cl, q, pp, w, status, st, nullptr, 0, &ia)) != APT_OK) return s;
    }
    hipLaunchKernelGGL(k_sdm_faces, dim3(1), dim3(kBlock), 0, st, w.E2, R, n_vox);
    SdmArgs a{};
    a.plan = w.plan;
    a.t_id = w.t_id;
    a.tx = w.tx;
    a.ty = w.ty;
    a.tz = w.tz;
    a.bpos = w.bpos;
    a.cell_start = w.cell_start;
    a.self_possible = q.target == APT_ANY || q.neighbor == APT_ANY || q.target == q.neighbor;
    a.R = R;
    a.r_enum = pp.r_enum;
    a.in2 = (float)((Rd * (1.0 - 2e-5)) * (Rd * (1.0 - 2e-5)));
    a.out2 = (float)((Rd * (1.0 + 2e-5)) * (Rd * (1.0 + 2e-5)));
    a.R2 = Rd * Rd;
    a.n_vox = n_vox;
    a.inv_w = (float)((double)n_vox / (2.0 * Rd));
    // the FP32 voxel coordinate errs by < 2e-7 * n_vox voxels (difference,
    // offset and scaling each rounded once): decide in FP64 within 16 ulps
    a.band = (float)fmin(0.25, fmax(1e-4, 16.0 * 5.9604645e-8 * (double)n_vox));
    a.F = w.E2;
    a.hist = hist;
    {
        TraceSpan span("sdm", st);
        hipLaunchKernelGGL(k_sdm, dim3(resident_grid(k_sdm, 0)), dim3(kBlock), 0, st, a);
    }
    return hip_check("two-point statistic launch");
}

// Workspace of the smoothed RDF: the plain binning, the edges and the
// per-wavefront partial results.
constexpr size_t kSmoothPart = (size_t)1 << 21;
struct SmoothWs {
    PlainWs plain;
    double* E;
    double* part;
    size_t bytes;
};
static SmoothWs carve_smooth(void* base, int64_t n) {
    SmoothWs w;
    w.plain = carve_plain(base, n);
    Carve c{base ? reinterpret_cast<char*>(base) + w.plain.bytes : nullptr};
    w.E = c.take<double>(kSmoothMaxBins + 1);
    w.part = c.take<double>(kSmoothPart);
    w.bytes = w.plain.bytes + c.off;
    return w;
}

// Forward (bwd == false: h) or adjoint (grad_h -> grad_xyz, grad_s).
static apt_status run_smooth(bool bwd, const apt_cloud* cl, apt_query q, apt_bins rb, float sigma,
                             const double* zscale, double* h, const double* grad_h, float* grad_xyz,
                             double* grad_s, int32_t* status, void* ws, size_t ws_bytes, void* stream) {
    apt_status s;
    if ((s = check_cloud(cl)) != APT_OK) return s;
    if ((s = check_query(q)) != APT_OK) return s;
    if ((s = check_bins(rb, "bins")) != APT_OK) return s;
    if (rb.n_bins > kSmoothMaxBins) return fail(APT_E_UNSUPPORTED, "smoothed RDF supports at most 4096 bins");
    if (!(sigma > 0.0f) || !isfinite(sigma)) return fail(APT_E_ARG, "sigma must be finite and > 0");
    if (!status) return fail(APT_E_ARG, "status is NULL");
    if (!bwd && !h) return fail(APT_E_ARG, "h is NULL");
    if (bwd && !grad_h) return fail(APT_E_ARG, "grad_h is NULL");
    if (bwd && cl->n > 0 && !grad_xyz) return fail(APT_E_ARG, "grad_xyz is NULL");
    const double sig = (double)sigma;
    const double w6 = 6.0 * sig;
    const double cut = (double)rb.r_max + 6.0 * sig;
    const double width = (double)rb.r_max / rb.n_bins;
    const double mw = floor(2.0 * w6 / width) + 3.0;     // most bins one window meets, with a margin
    if (!(mw + 1.0 <= (double)kSmoothTerms))             // its edges are buffered
        return fail(APT_E_UNSUPPORTED, "sigma spans more than 1020 bins (12 sigma / bin width)");
    if (!((float)(cut * (1.0 + 2e-5)) < 1e30f)) return fail(APT_E_ARG, "r_max + 6 sigma is too large");
    SmoothWs w = carve_smooth(ws, cl->n);
    if ((s = check_ws(ws, ws_bytes, w.bytes)) != APT_OK) return s;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    const int cus = device_info().cus;

    InitArgs ia{status, nullptr, 0, nullptr, 0, nullptr, nullptr};
    hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, st, ia);
    hipLaunchKernelGGL(k_smooth_edges, dim3(16), dim3(256), 0, st, w.E, rb.r_max, rb.n_bins);
    if (bwd && cl->n > 0) hipLaunchKernelGGL(k_fill_f32, dim3(cus * 4), dim3(256), 0, st, grad_xyz, 3 * cl->n);

    const apt_tuning tu = tuning();
    const float r_pre = (float)(cut * (1.0 + 2e-5));
    PlanParams pp;
    pp.h_min = r_pre * tu.h_min_frac;
    pp.occ = tu.cell_occ;
    pp.tile_occ = 0.0f;
    pp.k = 0;
    pp.cell_cap = cell_cap_for(cl->n);
    pp.tile_policy = 1;
    pp.r_enum = r_pre;
    {
        TraceSpan span("binning", st);
        if ((s = run_binning(cl, q, pp, w.plain, status, st, zscale, bwd ? 1 : 0)) != APT_OK) return s;
    }
    SmoothArgs sa{};
    sa.plan = w.plain.plan;
    sa.xyz = cl->xyz;
    sa.lab = cl->lab;
    sa.d_bnd = cl->d_bnd;
    sa.zscale = zscale;
    sa.t_id = w.plain.t_id;
    sa.bpos = w.plain.bpos;
    sa.cell_start = w.plain.cell_start;
    sa.A = q.target;
    sa.B = q.neighbor;
    sa.d_srf = q.d_srf;
    sa.uni = bwd ? 1 : 0;
    sa.n_bins = rb.n_bins;
    sa.hcap = (int)fmin(64.0, floor((double)kSmoothTerms / (mw + 1.0)));
    sa.r_pre = r_pre;
    sa.sigma = sig;
    sa.cut = cut;
    sa.w6 = w6;
    sa.inv_width = rb.n_bins / (double)rb.r_max;
    sa.E = w.E;
    sa.grad_h = grad_h;
    sa.part = w.part;
    sa.grad_xyz = grad_xyz;
    if (!bwd) {
        int W = (int)(kSmoothPart / (size_t)rb.n_bins);
        if (W > kSmoothWaves) W = kSmoothWaves;
        sa.W = W;
        TraceSpan span("smooth", st);
        hipLaunchKernelGGL(k_smooth_fwd, dim3(W), dim3(kWave), smooth_lds_bytes(true, rb.n_bins), st, sa);
        SmoothReduceArgs ra{w.part, W, rb.n_bins, h};
        hipLaunchKernelGGL(k_smooth_reduce, dim3((rb.n_bins + kWave - 1) / kWave), dim3(kWave * kReduceGroups), 0,
                           st, ra);
    } else {
        sa.W = kSmoothWaves;
        TraceSpan span("smooth", st);
        hipLaunchKernelGGL(k_smooth_bwd, dim3(kSmoothWaves), dim3(kWave), smooth_lds_bytes(false, rb.n_bins), st,
                           sa);
        if (grad_s) {
            SmoothReduceArgs ra{w.part, kSmoothWaves, 1, grad_s};
            hipLaunchKernelGGL(k_smooth_reduce, dim3(1), dim3(kWave * kReduceGroups), 0, st, ra);
        }
    }
    return hip_check("smoothed RDF launch");
}

// ------------------------------------------------------ static scratch --
// The workspace of apt_rdf_noalloc: one array per device, held from the
// library's load until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol): its device address, taken once per device with that device
// current, is what the launches receive.
constexpr size_t kStaticScratchBytes = (size_t)APT_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64];

static apt_status static_scratch(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return fail(APT_E_HIP, "hipGetDevice failed");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(APT_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return APT_OK;
}

}  // namespace apt

using namespace apt;

extern "C" {

const char* apt_last_error(void) { return g_err.c_str(); }

apt_status apt_set_tuning(const apt_tuning* t) {
    apt_tuning v = {0, 4.0f, 0.5f, 1.0f, 0};
    if (t) {
        if (t->rdf_kernel < 0 || t->rdf_kernel > 2) return fail(APT_E_ARG, "rdf_kernel must be 0, 1 or 2");
        if (t->tile_policy < 0 || t->tile_policy > 4) return fail(APT_E_ARG, "tile_policy must be 0, 1, 2, 3 or 4");
        if (!(t->cell_occ > 0.0f) || !(t->h_min_frac > 0.0f) || !isfinite(t->cell_occ) || !isfinite(t->h_min_frac))
            return fail(APT_E_ARG, "cell_occ and h_min_frac must be finite and > 0");
        if (!(t->tile_occ >= 0.0f) || !isfinite(t->tile_occ))
            return fail(APT_E_ARG, "tile_occ must be finite and >= 0");
        v = *t;
        if (v.tile_occ == 0.0f) v.tile_occ = 1.0f;
    }
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune = v;
    return APT_OK;
}

apt_status apt_get_tuning(apt_tuning* t) {
    if (!t) return fail(APT_E_ARG, "apt_get_tuning: NULL");
    *t = tuning();
    return APT_OK;
}

apt_status apt_trace_enable(int32_t on) {
    if (on < 0 || on > 2) return fail(APT_E_ARG, "apt_trace_enable: on must be 0, 1 or 2");
    g_trace_on.store(on);
    return APT_OK;
}

apt_status apt_trace_read(const char* stage, double* ms_total, int64_t* launches) {
    if (!stage || !ms_total || !launches) return fail(APT_E_ARG, "apt_trace_read: NULL argument");
    std::vector<TraceRec> mine;
    {
        std::lock_guard<std::mutex> g(g_trace_mu);
        std::vector<TraceRec> rest;
        for (auto& r : g_trace) (r.stage == stage ? mine : rest).push_back(r);
        g_trace.swap(rest);
    }
    double tot = 0.0;
    apt_status s = APT_OK;
    for (auto& r : mine) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
            s = fail(APT_E_HIP, "apt_trace_read: event wait failed");
        tot += ms;
    }
    {
        // back to the free lists (both events have completed)
        std::lock_guard<std::mutex> g(g_trace_mu);
        for (auto& r : mine) {
            g_event_pool[r.dev].push_back(r.a);
            g_event_pool[r.dev].push_back(r.b);
        }
    }
    *ms_total = tot;
    *launches = (int64_t)mine.size();
    return s;
}

size_t apt_workspace_size(int32_t op, int64_t n, int32_t n_pairs, int32_t n_rep) {
    (void)n_pairs;
    (void)n_rep;
    if (n < 0 || n >= (int64_t)0xFFFFFFFFll) return 0;
    switch (op) {
        case APT_OP_RDF:
        case APT_OP_KNN:
        case APT_OP_KNN_RDF:
            return carve_plain(nullptr, n).bytes;
        case APT_OP_PERMUTE:
            return carve_perm(nullptr, n, 1).bytes;
        case APT_OP_BATCHED:
            if (n_rep < 1) return 0;
            return carve_batched(nullptr, n, batch_reps(n, n_rep)).bytes;
        case APT_OP_SMOOTH:
            return carve_smooth(nullptr, n).bytes;
        case APT_OP_SDM:
        case APT_OP_CLUSTER:
            return carve_plain(nullptr, n).bytes;
        default:
            return 0;
    }
}

apt_status apt_permute_labels(const uint8_t* lab, int64_t n, uint64_t seed, uint8_t* out, int32_t* status,
                              void* ws, size_t ws_bytes, void* stream) {
    if (n < 0) return fail(APT_E_ARG, "n is negative");
    if (n >= (int64_t)0xFFFFFFFFll) return fail(APT_E_UNSUPPORTED, "n must be below 2^32 - 1");
    if (n > 0 && (!lab || !out)) return fail(APT_E_ARG, "lab or out is NULL");
    if (!status) return fail(APT_E_ARG, "status is NULL");
    PermWs w = carve_perm(ws, n, 1);
    apt_status s;
    if ((s = check_ws(ws, ws_bytes, w.bytes)) != APT_OK) return s;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    InitArgs ia{status, nullptr, 0, nullptr, 0, nullptr, nullptr};
    hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, st, ia);
    if (n > 0) run_permute(lab, n, &seed, 1, out, n, w, status, st);
    return hip_check("permute launch");
}

apt_status apt_rdf_batched(const apt_cloud* cloud, const apt_query* pairs, int32_t n_pairs, const uint64_t* seeds,
                           int32_t n_rep, apt_bins rdf_bins, int32_t k, apt_bins knn_bins, uint64_t* rdf_hist,
                           uint64_t* knn_hist, const apt_batched_tuning* tuning, int32_t* status, void* ws,
                           size_t ws_bytes, void* stream) {
    apt_batched_tuning bt;
    apt_status s;
    if (tuning) {
        if ((s = resolve_batched_tuning(tuning, &bt)) != APT_OK) return s;
        return run_batched(cloud, pairs, n_pairs, seeds, n_rep, rdf_bins, k, knn_bins, rdf_hist, knn_hist, status,
                           ws, ws_bytes, stream, bt);
    }
    // arguments first (the plan key reads them; the autotuner's trials must
    // not be the first to reject them)
    if ((s = check_batched(cloud, pairs, n_pairs, seeds, n_rep, rdf_bins, k, knn_bins, rdf_hist, knn_hist,
                           status)) != APT_OK)
        return s;
    if ((s = check_ws(ws, ws_bytes, carve_batched(nullptr, cloud->n, batch_reps(cloud->n, n_rep)).bytes)) != APT_OK)
        return s;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (st && hipStreamIsCapturing(st, &cap) != hipSuccess) cap = hipStreamCaptureStatusNone;
    const bool capturing = cap != hipStreamCaptureStatusNone;
    const std::string pkey = batched_plan_key(cloud, pairs, n_pairs, rdf_bins, k, knn_bins, knn_hist != nullptr);
    bool have = false;
    {
        std::lock_guard<std::mutex> g(g_plan_mu);
        auto it = g_plans.find(pkey);
        if (it != g_plans.end()) {
            bt = it->second;
            have = true;
        }
    }
    if (!have) {
        if (capturing) {
            // no timing inside a capture: the defaults, not cached
            return run_batched(cloud, pairs, n_pairs, seeds, n_rep, rdf_bins, k, knn_bins, rdf_hist, knn_hist,
                               status, ws, ws_bytes, stream, kBatchedDefaults);
        }
        if ((s = autotune_batched(cloud, pairs, n_pairs, seeds, n_rep, rdf_bins, k, knn_bins, rdf_hist, knn_hist,
                                  status, ws, ws_bytes, stream, &bt)) != APT_OK)
            return s;
        std::lock_guard<std::mutex> g(g_plan_mu);
        g_plans[pkey] = bt;
    }
    if (capturing || g_trace_on.load() != 0)
        return run_batched(cloud, pairs, n_pairs, seeds, n_rep, rdf_bins, k, knn_bins, rdf_hist, knn_hist, status,
                           ws, ws_bytes, stream, bt);
    // the launch sequence as a graph, per call signature
    std::string gkey = pkey;
    key_put(gkey, n_rep);
    for (int r = 0; r < n_rep; ++r) key_put(gkey, seeds[r]);
    key_put(gkey, cloud->xyz);
    key_put(gkey, cloud->lab);
    key_put(gkey, cloud->d_bnd);
    key_put(gkey, rdf_hist);
    key_put(gkey, knn_hist);
    key_put(gkey, status);
    key_put(gkey, ws);
    key_put(gkey, ws_bytes);
    {
        std::lock_guard<std::mutex> g(g_graph_mu);
        for (auto& e : g_graphs)
            if (e.key == gkey) {
                if (hipGraphLaunch(e.exec, st) != hipSuccess) return fail(APT_E_HIP, "hipGraphLaunch failed");
                return APT_OK;
            }
    }
    hipStream_t cs = capture_stream();
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool ok = cs && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        s = run_batched(cloud, pairs, n_pairs, seeds, n_rep, rdf_bins, k, knn_bins, rdf_hist, knn_hist, status, ws,
                        ws_bytes, cs, bt);
        ok = hipStreamEndCapture(cs, &graph) == hipSuccess && graph != nullptr;
        if (s != APT_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return s;
        }
        ok = ok && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
    }
    (void)hipGetLastError();
    if (!ok) {
        // no graph: the same sequence launched directly
        if (graph) (void)hipGraphDestroy(graph);
        return run_batched(cloud, pairs, n_pairs, seeds, n_rep, rdf_bins, k, knn_bins, rdf_hist, knn_hist, status,
                           ws, ws_bytes, stream, bt);
    }
    if (hipGraphLaunch(exec, st) != hipSuccess) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        return fail(APT_E_HIP, "hipGraphLaunch failed");
    }
    std::lock_guard<std::mutex> g(g_graph_mu);
    if (g_graphs.size() >= kMaxGraphs) {
        drop_graph(g_graphs.front());
        g_graphs.erase(g_graphs.begin());
    }
    g_graphs.push_back(GraphEntry{gkey, graph, exec});
    return APT_OK;
}

apt_status apt_batched_plan(const apt_cloud* cloud, const apt_query* pairs, int32_t n_pairs, apt_bins rdf_bins,
                            int32_t k, apt_bins knn_bins, int32_t want_knn_hist, apt_batched_tuning* out,
                            int32_t* cached) {
    if (!cloud || !pairs || n_pairs < 1 || n_pairs > kMaxPairs || !out || !cached)
        return fail(APT_E_ARG, "apt_batched_plan: NULL or out-of-range argument");
    const std::string key = batched_plan_key(cloud, pairs, n_pairs, rdf_bins, k, knn_bins, want_knn_hist != 0);
    std::lock_guard<std::mutex> g(g_plan_mu);
    auto it = g_plans.find(key);
    *cached = it != g_plans.end() ? 1 : 0;
    if (*cached) *out = it->second;
    return APT_OK;
}

apt_status apt_batched_plan_clear(void) {
    {
        std::lock_guard<std::mutex> g(g_plan_mu);
        g_plans.clear();
    }
    std::lock_guard<std::mutex> g(g_graph_mu);
    for (auto& e : g_graphs) drop_graph(e);
    g_graphs.clear();
    return APT_OK;
}

apt_status apt_sdm(const apt_cloud* cloud, apt_query q, float R, int32_t n_vox, uint64_t* hist, int32_t* status,
                   void* ws, size_t ws_bytes, void* stream) {
    return run_sdm(cloud, q, R, n_vox, hist, status, ws, ws_bytes, stream);
}

// ------------------------------------------------- ion-to-edge distance --
// The plain binning (every ion a neighbour, no targets) puts the ions in cell
// order; the triangle arrays follow it in the workspace.
struct EdgeWs {
    PlainWs plain;
    TriPlan* tp;
    float4* tc;
    uint32_t piece_cap;
    float4* pc;
    uint32_t* ptri;
    uint32_t* pcell;
    uint32_t* tcnt;
    uint32_t* tstart;
    uint32_t* tblk;
    uint32_t* torder;
    float4* tsorted;
    size_t bytes;
};

// pieces the triangles may be cut into: four per triangle and a fixed reserve
static uint32_t edge_piece_cap(int64_t n_tri) { return (uint32_t)std::min<int64_t>(4 * n_tri + 65536, 0xF0000000ll); }

static EdgeWs carve_edge(void* base, int64_t n, int64_t n_tri) {
    EdgeWs w;
    w.plain = carve_plain(base, n);
    Carve c{reinterpret_cast<char*>(base), w.plain.bytes};
    const size_t T = (size_t)(n_tri > 0 ? n_tri : 1);
    w.piece_cap = edge_piece_cap(n_tri);
    const size_t PC = w.piece_cap;
    w.tp = c.take<TriPlan>(1);
    w.tc = c.take<float4>(T);
    w.pc = c.take<float4>(PC);
    w.ptri = c.take<uint32_t>(PC);
    w.pcell = c.take<uint32_t>(PC);
    w.tcnt = c.take<uint32_t>(kTriCells);
    w.tstart = c.take<uint32_t>((size_t)kTriCells + 1);
    w.tblk = c.take<uint32_t>(kTriScanBlocks);
    w.torder = c.take<uint32_t>(PC);
    w.tsorted = c.take<float4>(PC);
    w.bytes = c.off;
    return w;
}

size_t apt_edge_workspace_size(int64_t n, int64_t n_tri) {
    if (n < 0 || n >= (int64_t)0xFFFFFFFFll || n_tri < 0 || n_tri >= (int64_t)0xFFFFFFFFll) return 0;
    return carve_edge(nullptr, n, n_tri).bytes;
}

apt_status apt_edge_distance(const apt_cloud* cloud, const float* tri, int64_t n_tri, float d_prb, float* d,
                             int32_t* status, void* ws, size_t ws_bytes, void* stream) {
    apt_status s;
    if ((s = check_cloud(cloud)) != APT_OK) return s;
    if (n_tri < 0) return fail(APT_E_ARG, "n_tri is negative");
    if (n_tri >= (int64_t)0xFFFFFFFFll) return fail(APT_E_UNSUPPORTED, "n_tri must be below 2^32 - 1");
    if (n_tri > 0 && !tri) return fail(APT_E_ARG, "tri is NULL");
    if (!(d_prb > 0.0f)) return fail(APT_E_ARG, "d_prb must be > 0 (+inf: no probe limit)");
    if (cloud->n > 0 && !d) return fail(APT_E_ARG, "d is NULL");
    if (!status) return fail(APT_E_ARG, "status is NULL");
    EdgeWs w = carve_edge(ws, cloud->n, n_tri);
    if ((s = check_ws(ws, ws_bytes, w.bytes)) != APT_OK) return s;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    apt_cloud cl = *cloud;
    cl.d_bnd = nullptr;
    apt_query q{};
    q.target = 254;                            // no targets: the ions are binned as neighbours only
    q.neighbor = APT_ANY;
    q.d_srf = 0.0f;
    InitArgs ia{status, nullptr, 0, nullptr, 0, nullptr, w.plain.strag_count};
    const apt_tuning tu = tuning();
    PlanParams pp;
    pp.h_min = tu.h_min_frac;                  // about 0.5 nm: the lanes of a wavefront stay close
    pp.occ = tu.cell_occ;
    pp.tile_occ = tu.tile_occ;
    pp.k = 0;
    pp.cell_cap = cell_cap_for(cl.n);
    pp.tile_policy = 1;
    pp.r_enum = 1.0f;
    pp.h_shrink = 0.7f;
    EdgeArgs a{};
    a.plan = w.plain.plan;
    a.bpos = w.plain.bpos;
    a.tp = w.tp;
    a.tri = tri;
    a.n_tri = (uint32_t)n_tri;
    a.d_prb = d_prb;
    a.piece_cap = w.piece_cap;
    a.tc = w.tc;
    a.pc = w.pc;
    a.ptri = w.ptri;
    a.pcell = w.pcell;
    a.tcnt = w.tcnt;
    a.tstart = w.tstart;
    a.tblk = w.tblk;
    a.torder = w.torder;
    a.tsorted = w.tsorted;
    a.d_out = d;
    a.n = cl.n;
    a.status = status;
    {
        TraceSpan span("binning", st);
        if ((s = run_binning(&cl, q, pp, w.plain, status, st, nullptr, 0, &ia)) != APT_OK) return s;
    }
    const int gn = (int)std::min<int64_t>(std::max<int64_t>((cl.n + kBlock - 1) / kBlock, 1), 8192);
    const int gt = (int)std::min<int64_t>(std::max<int64_t>((n_tri + kBlock - 1) / kBlock, 1), 4096);
    {
        TraceSpan span("edge", st);
        hipLaunchKernelGGL(k_edge_zero, dim3(gn), dim3(kBlock), 0, st, a);
        hipLaunchKernelGGL(k_edge_prep, dim3(gt), dim3(kBlock), 0, st, a);
        hipLaunchKernelGGL(k_edge_plan, dim3(1), dim3(64), 0, st, a);
        hipLaunchKernelGGL(k_edge_measure, dim3(gt), dim3(kBlock), 0, st, a);
        hipLaunchKernelGGL(k_edge_plan_pieces, dim3(1), dim3(64), 0, st, a);
        hipLaunchKernelGGL(k_edge_pieces, dim3(gt), dim3(kBlock), 0, st, a);
        hipLaunchKernelGGL(k_edge_clear, dim3(1024), dim3(kBlock), 0, st, a);
        hipLaunchKernelGGL(k_edge_count, dim3(4096), dim3(kBlock), 0, st, a);
        hipLaunchKernelGGL(k_edge_scan_blocks, dim3(kTriScanBlocks), dim3(kBlock), 0, st, a);
        hipLaunchKernelGGL(k_edge_scan_add, dim3(kTriScanBlocks), dim3(kBlock), 0, st, a);
        hipLaunchKernelGGL(k_edge_fill, dim3(4096), dim3(kBlock), 0, st, a);
        hipLaunchKernelGGL(k_edge_dist, dim3(gn), dim3(kBlock), 0, st, a);
    }
    return hip_check("edge distance launch");
}

// ------------------------------------------------ maximum separation --
// The species' ions are binned as the targets and neighbours of one query
// (no surface filter: every ion of the species is a vertex); the union-find
// forest and the cluster sizes live in the radix sort's key arrays, which
// the binning no longer needs once it has finished.
apt_status apt_cluster_ms(const apt_cloud* cloud, uint8_t species, float d_max, int32_t n_min, float d_srf,
                          int64_t* label, int64_t* counts, uint64_t* size_hist, int32_t n_size_bins,
                          int32_t* status, void* ws, size_t ws_bytes, void* stream) {
    apt_status s;
    if ((s = check_cloud(cloud)) != APT_OK) return s;
    if (cloud->n >= ((int64_t)1 << 31)) return fail(APT_E_UNSUPPORTED, "clustering needs fewer than 2^31 ions");
    if (!(d_max > 0.0f) || !isfinite(d_max)) return fail(APT_E_ARG, "d_max must be finite and > 0");
    if (n_min < 1) return fail(APT_E_ARG, "n_min must be >= 1");
    if (isnan(d_srf)) return fail(APT_E_ARG, "d_srf is NaN");
    if (size_hist && (n_size_bins < 1 || n_size_bins > APT_MAX_BINS))
        return fail(APT_E_ARG, "n_size_bins must be in [1, 65536]");
    if (!counts || !status) return fail(APT_E_ARG, "counts or status is NULL");
    if (cloud->n > 0 && !label) return fail(APT_E_ARG, "label is NULL");
    PlainWs w = carve_plain(ws, cloud->n);
    if ((s = check_ws(ws, ws_bytes, w.bytes)) != APT_OK) return s;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    apt_cloud cl = *cloud;
    cl.d_bnd = nullptr;                        // every ion of the species is a vertex
    apt_query q{};
    q.target = species;
    q.neighbor = species;
    q.d_srf = 0.0f;
    InitArgs ia{status, size_hist, size_hist ? n_size_bins : 0, reinterpret_cast<uint64_t*>(counts), 3, nullptr,
                w.strag_count};
    const apt_tuning tu = tuning();
    const double dm = (double)d_max;
    PlanParams pp;
    pp.h_min = d_max * tu.h_min_frac;
    pp.occ = tu.cell_occ;
    pp.tile_occ = tu.tile_occ;
    pp.k = 0;
    pp.cell_cap = cell_cap_for(cl.n);
    pp.tile_policy = 1;                        // one target per wavefront
    pp.r_enum = (float)(dm * (1.0 + 4e-5));
    pp.h_shrink = 0.7f;
    {
        TraceSpan span("binning", st);
        if ((s = run_binning(&cl, q, pp, w, status, st, nullptr, 0, &ia)) != APT_OK) return s;
    }
    if (cl.n == 0) return hip_check("clustering launch");
    const uint32_t n = (uint32_t)cl.n;
    uint32_t* parent = w.K[0];
    uint32_t* size = w.K[1];
    const int g = (int)std::min<int64_t>(((int64_t)n + kBlock - 1) / kBlock, 8192);
    ClusterLinkArgs la{};
    la.plan = w.plan;
    la.t_id = w.t_id;
    la.tx = w.tx;
    la.ty = w.ty;
    la.tz = w.tz;
    la.bpos = w.bpos;
    la.cell_start = w.cell_start;
    la.r_enum = pp.r_enum;
    la.in2 = (float)((dm * (1.0 - 2e-5)) * (dm * (1.0 - 2e-5)));
    la.out2 = (float)((dm * (1.0 + 2e-5)) * (dm * (1.0 + 2e-5)));
    la.lim2 = dm * dm;
    la.parent = parent;
    ClusterOutArgs oa{};
    oa.lab = cl.lab;
    oa.d_bnd = cloud->d_bnd;
    oa.d_srf = d_srf;
    oa.A = species;
    oa.n = n;
    oa.n_min = n_min;
    oa.parent = parent;
    oa.size = size;
    oa.label = label;
    oa.counts = reinterpret_cast<unsigned long long*>(counts);
    oa.size_hist = size_hist;
    oa.n_size_bins = size_hist ? n_size_bins : 0;
    {
        TraceSpan span("cluster", st);
        hipLaunchKernelGGL(k_ms_init, dim3(g), dim3(kBlock), 0, st, parent, size, n);
        hipLaunchKernelGGL(k_ms_link, dim3(resident_grid(k_ms_link, 0)), dim3(kBlock), 0, st, la);
        hipLaunchKernelGGL(k_ms_roots, dim3(g), dim3(kBlock), 0, st, oa);
        hipLaunchKernelGGL(k_ms_final, dim3(g), dim3(kBlock), 0, st, oa);
    }
    return hip_check("clustering launch");
}

apt_status apt_count_targets(const apt_cloud* cloud, apt_query q, int64_t* n_targets, void* ws, size_t ws_bytes,
                             void* stream) {
    apt_status s;
    if ((s = check_cloud(cloud)) != APT_OK) return s;
    if ((s = check_query(q)) != APT_OK) return s;
    if (!n_targets) return fail(APT_E_ARG, "n_targets is NULL");
    PlainWs w = carve_plain(ws, cloud->n);
    if ((s = check_ws(ws, ws_bytes, w.bytes)) != APT_OK) return s;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    const int G = count_blocks(cloud->n);
    CountArgs ca{cloud->xyz, cloud->lab, cloud->d_bnd, cloud->n, count_chunk(cloud->n, G), q.target, q.neighbor,
                 q.d_srf, nullptr, w.part_cnt, w.part_bbox, w.part_nf};
    hipLaunchKernelGGL(k_count, dim3(G), dim3(kBlock), 0, st, ca);
    PlanParams pp{1.0f, 4.0f, 0, cell_cap_for(cloud->n), 1, 0.0f};
    PlanArgs pa{G, w.part_cnt, w.part_bbox, w.part_nf, w.part_off, pp, nullptr, w.plan, nullptr};
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, st, pa);
    FinishArgs fa{w.plan, -1, n_targets, nullptr};
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1), 0, st, fa);
    return hip_check("count launch");
}

apt_status apt_rdf(const apt_cloud* cloud, apt_query q, apt_bins bins, uint64_t* hist, int32_t* status,
                   void* ws, size_t ws_bytes, void* stream) {
    return run_plain(cloud, q, &bins, hist, 0, INFINITY, 0, nullptr, nullptr, nullptr, nullptr, nullptr,
                     nullptr, status, ws, ws_bytes, stream);
}

apt_status apt_rdf_noalloc(const apt_cloud* cloud, apt_query q, apt_bins bins, uint64_t* hist, int32_t* status,
                           void* stream) {
    apt_status s;
    if ((s = check_cloud(cloud)) != APT_OK) return s;
    const size_t need = carve_plain(nullptr, cloud->n).bytes;
    if (need > kStaticScratchBytes)
        return fail(APT_E_UNSUPPORTED, "apt_rdf_noalloc: " + std::to_string(cloud->n) + " ions need " +
                                           std::to_string(need) + " bytes of scratch; the static scratch holds " +
                                           std::to_string(kStaticScratchBytes));
    void* ws = nullptr;
    if ((s = static_scratch(&ws)) != APT_OK) return s;
    return run_plain(cloud, q, &bins, hist, 0, INFINITY, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                     status, ws, kStaticScratchBytes, stream);
}

apt_status apt_knn(const apt_cloud* cloud, apt_query q, int32_t k, float r_knn_max, int64_t capacity,
                   int64_t* target_id, float* dist, int64_t* nbr_id, apt_bins knn_bins, uint64_t* knn_hist,
                   int64_t* n_targets, int32_t* status, void* ws, size_t ws_bytes, void* stream) {
    if (k < 1) return fail(APT_E_ARG, "k must be >= 1");
    return run_plain(cloud, q, nullptr, nullptr, k, r_knn_max, capacity, target_id, dist, nbr_id, &knn_bins,
                     knn_hist, n_targets, status, ws, ws_bytes, stream);
}

apt_status apt_knn_rdf(const apt_cloud* cloud, apt_query q, apt_bins rdf_bins, uint64_t* rdf_hist, int32_t k,
                       float r_knn_max, int64_t capacity, int64_t* target_id, float* dist, int64_t* nbr_id,
                       apt_bins knn_bins, uint64_t* knn_hist, int64_t* n_targets, int32_t* status, void* ws,
                       size_t ws_bytes, void* stream) {
    if (k < 1) return fail(APT_E_ARG, "k must be >= 1");
    return run_plain(cloud, q, &rdf_bins, rdf_hist, k, r_knn_max, capacity, target_id, dist, nbr_id,
                     &knn_bins, knn_hist, n_targets, status, ws, ws_bytes, stream);
}

apt_status apt_count_candidates(const apt_cloud* cloud, apt_query q, apt_bins bins, int32_t k,
                                uint64_t* candidates, int32_t* status, void* ws, size_t ws_bytes, void* stream) {
    if (k < 0) return fail(APT_E_ARG, "k must be >= 0");
    if (!candidates) return fail(APT_E_ARG, "candidates is NULL");
    return run_plain(cloud, q, &bins, nullptr, k, INFINITY, 0, nullptr, nullptr, nullptr, nullptr, nullptr,
                     nullptr, status, ws, ws_bytes, stream, candidates);
}

apt_status apt_rdf_smooth_fwd(const apt_cloud* cloud, apt_query q, apt_bins bins, float sigma, const double* z_scale,
                              double* h, int32_t* status, void* ws, size_t ws_bytes, void* stream) {
    return run_smooth(false, cloud, q, bins, sigma, z_scale, h, nullptr, nullptr, nullptr, status, ws, ws_bytes,
                      stream);
}

apt_status apt_rdf_smooth_bwd(const apt_cloud* cloud, apt_query q, apt_bins bins, float sigma, const double* z_scale,
                              const double* grad_h, float* grad_xyz, double* grad_z_scale, int32_t* status, void* ws,
                              size_t ws_bytes, void* stream) {
    return run_smooth(true, cloud, q, bins, sigma, z_scale, nullptr, grad_h, grad_xyz, grad_z_scale, status, ws,
                      ws_bytes, stream);
}

}  // extern "C"
