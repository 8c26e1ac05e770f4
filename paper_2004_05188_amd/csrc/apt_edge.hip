// Ion-to-edge distancing (paper, Methods: "Ion-to-edge distancing";
// Supplementary: "Triangle filtering methods for ion-to-edge distancing").
//
// The paper filters the candidate triangles of each ion with a coarse
// distance map and an R-tree.  Here every triangle is covered by pieces (the
// m x m sub-triangles of a barycentric subdivision, m from the triangle's
// size) that are binned once by their centroid into a uniform grid over the
// ions' bounding box.  A piece lies within its radius of its centroid, so a
// cell at Chebyshev ring q from an ion's cell holds only pieces at least
// (q - 1) h - r_piece away, and the distance to a piece bounds the distance
// to its triangle from above: the exact distance is always taken to the
// whole triangle.  The pieces keep long slivers (a hull's cap fans) from
// widening every ion's search.  Ions are taken in the cell order of their
// own binning, one per lane, so that the lanes of a wavefront search
// neighbouring cells.  Each lane walks the rings around its cell, nearest
// first, and stops when the next ring cannot hold a piece closer than the
// best distance found or the probe distance d_prb; slabs, rows, cells and
// pieces whose FP32 lower bound already reaches that distance are skipped.
// The distance itself is FP64 on the stored FP32 values: the plane distance
// when the perpendicular's foot lies inside the triangle (all three
// barycentric weights of the foot, in dot-product form, non-negative), else
// the nearest of the three edges.
#include "apt_edge.hpp"

namespace apt {

// the accumulators of the triangle sizes, and NaN for every ion (the ions
// with a finite position are overwritten by k_edge_dist)
__global__ __launch_bounds__(kBlock) void k_edge_zero(EdgeArgs a) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.tp->rmax_bits = 0u;
        a.tp->n_valid = 0u;
        a.tp->r_sum = 0.0;
        for (int j = 0; j < kPieceSizes; ++j) a.tp->pieces_at[j] = 0ull;
        a.tp->piece_ctr = 0u;
        a.tp->piece_rmax_bits = 0u;
        a.tp->piece_cap = a.piece_cap;
    }
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * kBlock)
        a.d_out[i] = __builtin_nanf("");
}

// FP32 radius of the points q[0..2] about their centroid c, widened for its
// own rounding (the triangle is the vertices' hull, so it lies within it)
__device__ __forceinline__ float4 centroid_radius(const float* q) {
    const float cx = ((q[0] + q[3]) + q[6]) / 3.0f;
    const float cy = ((q[1] + q[4]) + q[7]) / 3.0f;
    const float cz = ((q[2] + q[5]) + q[8]) / 3.0f;
    float r2 = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float dx = q[3 * k] - cx, dy = q[3 * k + 1] - cy, dz = q[3 * k + 2] - cz;
        r2 = fmaxf(r2, dx * dx + dy * dy + dz * dz);
    }
    return make_float4(cx, cy, cz, sqrtf(r2) * 1.00001f + 1e-6f);
}

__global__ __launch_bounds__(kBlock) void k_edge_prep(EdgeArgs a) {
    uint32_t nv = 0;
    float rm = 0.0f;
    double rs = 0.0;
    for (uint32_t t = blockIdx.x * kBlock + threadIdx.x; t < a.n_tri; t += gridDim.x * kBlock) {
        const float* T = a.tri + 9 * (size_t)t;
        float v[9];
        bool ok = true;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            v[k] = T[k];
            ok = ok && isfinite(v[k]);
        }
        if (!ok) {
            a.tc[t] = make_float4(0.0f, 0.0f, 0.0f, -1.0f);
            atomicOr(a.status, APT_STATUS_NONFINITE);
            continue;
        }
        const float4 c = centroid_radius(v);
        a.tc[t] = c;
        ++nv;
        rm = fmaxf(rm, c.w);
        rs += (double)c.w;
    }
    nv = wave_sum(nv);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        rm = fmaxf(rm, __shfl_xor(rm, d, kWave));
        rs += __shfl_xor(rs, d, kWave);
    }
    if (lane_id() == 0 && nv) {
        atomicAdd(&a.tp->n_valid, nv);
        atomicMax(&a.tp->rmax_bits, __float_as_uint(rm));
        atomicAdd(&a.tp->r_sum, rs);
    }
}

// the triangle grid: over the ions' bounding box, cells about twice the
// mean triangle radius (and at least a third of the probe distance, so that
// a probe needs few rings), at most kTriCells of them
__global__ void k_edge_plan(EdgeArgs a) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const GridPlan P = *a.plan;
    TriPlan& T = *a.tp;
    T.r_max = __uint_as_float(T.rmax_bits);
    double ext[3], vol = 1.0, amax = 0.0;
    for (int c = 0; c < 3; ++c) {
        const float l = P.nB > 0 ? P.lo[c] : 0.0f, hh = P.nB > 0 ? P.hi[c] : 0.0f;
        T.lo[c] = l;
        ext[c] = (double)hh - (double)l;
        vol *= fmax(ext[c], 1e-3);
        amax = fmax(amax, fmax(fabs((double)l), fabs((double)hh)));
    }
    double h = T.n_valid ? 2.0 * T.r_sum / (double)T.n_valid : 1.0;
    if (isfinite(a.d_prb)) h = fmax(h, (double)a.d_prb / 3.0);
    h = fmax(h, cbrt(vol / (double)kTriCells) * 1.0001);
    h = fmax(h, 1e-3);
    for (;;) {
        double cells = 1.0;
        for (int c = 0; c < 3; ++c) cells *= floor(ext[c] / h) + 1.0;
        if (cells <= (double)kTriCells) break;
        h *= 1.1;
    }
    uint32_t nc = 1;
    for (int c = 0; c < 3; ++c) {
        T.dim[c] = (int32_t)floor(ext[c] / h) + 1;
        nc *= (uint32_t)T.dim[c];
    }
    T.n_cells = nc;
    T.h = (float)h;
    T.inv_h = (float)(1.0 / h);
    T.rho = (float)(0.5 * h);
    // cell indices, centroids and piece vertices are FP32: each may sit a
    // few roundings away from the exact value
    T.slack = (float)(1e-5 * (amax + h) + 1e-6);
    T.prb2 = isfinite(a.d_prb) ? (double)a.d_prb * (double)a.d_prb : INFINITY;
}

__device__ __forceinline__ float piece_rho(const TriPlan& T, int j) {
    return j < kPieceSizes - 1 ? T.rho * (float)(1u << j) : T.r_max;
}
__device__ __forceinline__ uint32_t pieces_per_side(float r, float rho) {
    const float m = ceilf(r / rho);
    return m < 1.0f ? 1u : (m > 4096.0f ? 4096u : (uint32_t)m);
}

// pieces the triangles would take for each candidate piece radius
__global__ __launch_bounds__(kBlock) void k_edge_measure(EdgeArgs a) {
    const TriPlan T = *a.tp;
    unsigned long long acc[kPieceSizes];
#pragma unroll
    for (int j = 0; j < kPieceSizes; ++j) acc[j] = 0ull;
    for (uint32_t t = blockIdx.x * kBlock + threadIdx.x; t < a.n_tri; t += gridDim.x * kBlock) {
        const float r = a.tc[t].w;
        if (r < 0.0f) continue;
#pragma unroll
        for (int j = 0; j < kPieceSizes; ++j) {
            const unsigned long long m = pieces_per_side(r, piece_rho(T, j));
            acc[j] += m * m;
        }
    }
#pragma unroll
    for (int j = 0; j < kPieceSizes; ++j) {
        unsigned long long v = acc[j];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, d, kWave);
            const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), d, kWave);
            v += ((unsigned long long)hi << 32) | lo;
        }
        if (lane_id() == 0 && v) atomicAdd(&a.tp->pieces_at[j], v);
    }
}

// the smallest piece radius whose pieces fit the workspace (the last
// candidate, one piece per triangle, always does)
__global__ void k_edge_plan_pieces(EdgeArgs a) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    TriPlan& T = *a.tp;
    int j = 0;
    while (j < kPieceSizes - 1 && T.pieces_at[j] > (unsigned long long)T.piece_cap) ++j;
    T.rho = piece_rho(T, j);
    T.n_pieces = (uint32_t)T.pieces_at[j];
}

// grid point (i, k) of the m x m subdivision: a + (i/m)(b - a) + (k/m)(c - a)
__device__ __forceinline__ void sub_point(const float* v, uint32_t i, uint32_t k, float inv_m, float* q) {
    const float u = (float)i * inv_m, w = (float)k * inv_m;
#pragma unroll
    for (int c = 0; c < 3; ++c) q[c] = v[c] + u * (v[3 + c] - v[c]) + w * (v[6 + c] - v[c]);
}

__global__ __launch_bounds__(kBlock) void k_edge_pieces(EdgeArgs a) {
    const TriPlan T = *a.tp;
    float rmax = 0.0f;
    for (uint32_t t = blockIdx.x * kBlock + threadIdx.x; t < a.n_tri; t += gridDim.x * kBlock) {
        const float4 tc = a.tc[t];
        if (tc.w < 0.0f) continue;
        const uint32_t m = pieces_per_side(tc.w, T.rho);
        const uint32_t base = atomicAdd(&a.tp->piece_ctr, m * m);
        if (m == 1u) {
            a.pc[base] = tc;
            a.ptri[base] = t;
            rmax = fmaxf(rmax, tc.w);
            continue;
        }
        float v[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) v[k] = a.tri[9 * (size_t)t + k];
        const float inv_m = 1.0f / (float)m;
        uint32_t out = base;
        // rows of the subdivision: m - r upward and m - r - 1 downward pieces
        for (uint32_t r = 0; r < m; ++r) {
            for (uint32_t i = 0; i + r < m; ++i) {
                float q[9];
                sub_point(v, i, r, inv_m, q);
                sub_point(v, i + 1, r, inv_m, q + 3);
                sub_point(v, i, r + 1, inv_m, q + 6);
                float4 c = centroid_radius(q);
                c.w += T.slack;
                a.pc[out] = c;
                a.ptri[out] = t;
                rmax = fmaxf(rmax, c.w);
                ++out;
                if (i + r + 1 < m) {
                    sub_point(v, i + 1, r, inv_m, q);
                    sub_point(v, i + 1, r + 1, inv_m, q + 3);
                    sub_point(v, i, r + 1, inv_m, q + 6);
                    c = centroid_radius(q);
                    c.w += T.slack;
                    a.pc[out] = c;
                    a.ptri[out] = t;
                    rmax = fmaxf(rmax, c.w);
                    ++out;
                }
            }
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) rmax = fmaxf(rmax, __shfl_xor(rmax, d, kWave));
    if (lane_id() == 0 && rmax > 0.0f) atomicMax(&a.tp->piece_rmax_bits, __float_as_uint(rmax));
}

__global__ __launch_bounds__(kBlock) void k_edge_clear(EdgeArgs a) {
    const uint32_t nc = a.tp->n_cells;
    for (uint32_t c = blockIdx.x * kBlock + threadIdx.x; c < nc; c += gridDim.x * kBlock) a.tcnt[c] = 0u;
}

__device__ __forceinline__ int edge_axis(const TriPlan& T, int c, float x) {
    const float f = floorf((x - T.lo[c]) * T.inv_h);
    if (!(f >= 0.0f)) return 0;
    const int m = (int)fminf(f, (float)(T.dim[c] - 1));
    return m;
}

__global__ __launch_bounds__(kBlock) void k_edge_count(EdgeArgs a) {
    const TriPlan T = *a.tp;
    for (uint32_t p = blockIdx.x * kBlock + threadIdx.x; p < T.n_pieces; p += gridDim.x * kBlock) {
        const float4 c = a.pc[p];
        const uint32_t cell = ((uint32_t)edge_axis(T, 2, c.z) * (uint32_t)T.dim[1] + (uint32_t)edge_axis(T, 1, c.y)) *
                                  (uint32_t)T.dim[0] + (uint32_t)edge_axis(T, 0, c.x);
        a.pcell[p] = cell;
        atomicAdd(a.tcnt + cell, 1u);
    }
}

// exclusive offsets of the cell counts: each block scans its tile of
// kTriScanTile cells and leaves the tile's sum; the second kernel adds the
// sums of the tiles before it
__global__ __launch_bounds__(kBlock) void k_edge_scan_blocks(EdgeArgs a) {
    const uint32_t nc = a.tp->n_cells;
    const uint32_t base = blockIdx.x * (uint32_t)kTriScanTile;
    if (base >= nc) return;
    __shared__ uint32_t s_w[kWavesPerBlock];
    constexpr int per = kTriScanTile / kBlock;   // 16 consecutive cells per thread
    const uint32_t c0 = base + threadIdx.x * per;
    uint32_t v[per], sum = 0;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        v[k] = c0 + k < nc ? a.tcnt[c0 + k] : 0u;
        sum += v[k];
    }
    const uint32_t inc = wave_incl_scan(sum);
    const int w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) s_w[w] = inc;
    __syncthreads();
    uint32_t run = inc - sum;
    for (int u = 0; u < w; ++u) run += s_w[u];
#pragma unroll
    for (int k = 0; k < per; ++k) {
        if (c0 + k < nc) a.tstart[c0 + k] = run;
        run += v[k];
    }
    if (threadIdx.x == kBlock - 1) a.tblk[blockIdx.x] = run;
}

__global__ __launch_bounds__(kBlock) void k_edge_scan_add(EdgeArgs a) {
    const uint32_t nc = a.tp->n_cells;
    const uint32_t base = blockIdx.x * (uint32_t)kTriScanTile;
    if (base >= nc) return;
    __shared__ uint32_t s_off;
    if (threadIdx.x < kWave) {
        uint32_t s = 0;
        for (uint32_t b = lane_id(); b < blockIdx.x; b += kWave) s += a.tblk[b];
        s = wave_sum(s);
        if (lane_id() == 0) s_off = s;
    }
    __syncthreads();
    const uint32_t off = s_off;
    const uint32_t end = base + kTriScanTile < nc ? base + kTriScanTile : nc;
    for (uint32_t c = base + threadIdx.x; c < end; c += kBlock) a.tstart[c] += off;
    if (end == nc && threadIdx.x == 0) a.tstart[nc] = off + a.tblk[blockIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_edge_fill(EdgeArgs a) {
    const uint32_t np = a.tp->n_pieces;
    for (uint32_t p = blockIdx.x * kBlock + threadIdx.x; p < np; p += gridDim.x * kBlock) {
        const uint32_t cell = a.pcell[p];
        const uint32_t pos = a.tstart[cell] + atomicSub(a.tcnt + cell, 1u) - 1u;
        a.torder[pos] = a.ptri[p];
        a.tsorted[pos] = a.pc[p];
    }
}

// squared distance of p to the segment [u, u + e] (FP64)
__device__ __forceinline__ double seg_dist2(double px, double py, double pz, double ux, double uy, double uz,
                                            double ex, double ey, double ez) {
#pragma clang fp contract(off)
    const double wx = px - ux, wy = py - uy, wz = pz - uz;
    const double ee = ex * ex + ey * ey + ez * ez;
    double t = ee > 0.0 ? (wx * ex + wy * ey + wz * ez) / ee : 0.0;
    t = fmin(fmax(t, 0.0), 1.0);
    const double qx = wx - t * ex, qy = wy - t * ey, qz = wz - t * ez;
    return qx * qx + qy * qy + qz * qz;
}

// squared distance of p to the closed triangle T (FP64 on the FP32 vertices)
__device__ __forceinline__ double tri_dist2(double px, double py, double pz, const float* __restrict__ T) {
#pragma clang fp contract(off)
    const double ax = T[0], ay = T[1], az = T[2];
    const double bx = T[3], by = T[4], bz = T[5];
    const double cx = T[6], cy = T[7], cz = T[8];
    const double e1x = bx - ax, e1y = by - ay, e1z = bz - az;   // b - a
    const double e2x = cx - ax, e2y = cy - ay, e2z = cz - az;   // c - a
    const double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
    const double nn = nx * nx + ny * ny + nz * nz;
    const double wx = px - ax, wy = py - ay, wz = pz - az;
    if (nn > 0.0) {
        // barycentric weights of the foot of the perpendicular, scaled by nn
        const double d1 = e1x * wx + e1y * wy + e1z * wz, d2 = e2x * wx + e2y * wy + e2z * wz;
        const double bpx = px - bx, bpy = py - by, bpz = pz - bz;
        const double d3 = e1x * bpx + e1y * bpy + e1z * bpz, d4 = e2x * bpx + e2y * bpy + e2z * bpz;
        const double cpx = px - cx, cpy = py - cy, cpz = pz - cz;
        const double d5 = e1x * cpx + e1y * cpy + e1z * cpz, d6 = e2x * cpx + e2y * cpy + e2z * cpz;
        const double wa = d3 * d6 - d5 * d4, wb = d5 * d2 - d1 * d6, wc = d1 * d4 - d3 * d2;
        if (wa >= 0.0 && wb >= 0.0 && wc >= 0.0) {
            const double hgt = wx * nx + wy * ny + wz * nz;
            return hgt * hgt / nn;
        }
    }
    double d = seg_dist2(px, py, pz, ax, ay, az, e1x, e1y, e1z);
    d = fmin(d, seg_dist2(px, py, pz, bx, by, bz, cx - bx, cy - by, cz - bz));
    d = fmin(d, seg_dist2(px, py, pz, ax, ay, az, e2x, e2y, e2z));
    return d;
}

// FP32 gap (nm) between a coordinate and cell m's interval on axis c
__device__ __forceinline__ float axis_gap(const TriPlan& T, int c, float p, int m) {
    const float l = T.lo[c] + (float)m * T.h, u = l + T.h;
    return fmaxf(fmaxf(l - p, p - u), 0.0f);
}

__global__ __launch_bounds__(kBlock) void k_edge_dist(EdgeArgs a) {
    const GridPlan P = *a.plan;
    const TriPlan T = *a.tp;
    const float skip = __uint_as_float(T.piece_rmax_bits) + T.slack;   // a cell's pieces reach this far out
    for (uint32_t p = blockIdx.x * kBlock + threadIdx.x; p < P.nB; p += gridDim.x * kBlock) {
        const float4 r = a.bpos[p];
        const uint32_t idx = __builtin_bit_cast(uint32_t, r.w);
        if (!(isfinite(r.x) && isfinite(r.y) && isfinite(r.z))) {
            a.d_out[idx] = __builtin_nanf("");
            continue;
        }
        double best2 = T.prb2;
        // a gap g (FP32, nm) is beyond reach when g - skip >= the best distance
        auto beyond = [&](float g) {
            const float s = g * 0.99999f - skip;
            return s > 0.0f && (double)s * (double)s >= best2;
        };
        if (T.n_pieces > 0) {
            const double px = r.x, py = r.y, pz = r.z;
            const int cx = edge_axis(T, 0, r.x), cy = edge_axis(T, 1, r.y), cz = edge_axis(T, 2, r.z);
            for (int q = 0;; ++q) {
                if (beyond((float)(q - 1) * T.h)) break;
                if (cx - q < 0 && cy - q < 0 && cz - q < 0 && cx + q >= T.dim[0] && cy + q >= T.dim[1] &&
                    cz + q >= T.dim[2])
                    break;                           // every cell has been visited
                for (int dz = -q; dz <= q; ++dz) {
                    const int z = cz + dz;
                    if (z < 0 || z >= T.dim[2]) continue;
                    const float gz = axis_gap(T, 2, r.z, z);
                    if (beyond(gz)) continue;
                    for (int dy = -q; dy <= q; ++dy) {
                        const int y = cy + dy;
                        if (y < 0 || y >= T.dim[1]) continue;
                        const float gy = axis_gap(T, 1, r.y, y);
                        const float gyz = sqrtf(gy * gy + gz * gz);
                        if (beyond(gyz)) continue;
                        const bool full = q == 0 || dz == -q || dz == q || dy == -q || dy == q;
                        const int step = full ? 1 : 2 * q;
                        for (int x = cx - q; x <= cx + q; x += step) {
                            if (x < 0 || x >= T.dim[0]) continue;
                            const float gx = axis_gap(T, 0, r.x, x);
                            if (beyond(sqrtf(gx * gx + gyz * gyz))) continue;
                            const uint32_t cell = ((uint32_t)z * (uint32_t)T.dim[1] + (uint32_t)y) *
                                                      (uint32_t)T.dim[0] + (uint32_t)x;
                            const uint32_t k1 = a.tstart[cell + 1];
                            for (uint32_t k = a.tstart[cell]; k < k1; ++k) {
                                const float4 c = a.tsorted[k];
                                const float ddx = r.x - c.x, ddy = r.y - c.y, ddz = r.z - c.z;
                                const float lbt = sqrtf(ddx * ddx + ddy * ddy + ddz * ddz) * 0.99999f -
                                                  c.w - T.slack;
                                if (lbt > 0.0f && (double)lbt * (double)lbt >= best2) continue;
                                const double d2 = tri_dist2(px, py, pz, a.tri + 9 * (size_t)a.torder[k]);
                                best2 = fmin(best2, d2);
                            }
                        }
                    }
                }
            }
        }
        const double d = sqrt(best2);
        a.d_out[idx] = (d < (double)a.d_prb) ? (float)d : __builtin_inff();
    }
}

}  // namespace apt
