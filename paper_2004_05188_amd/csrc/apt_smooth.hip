// Gaussian-smoothed RDF (forward) and its adjoint: an extension of the
// paper's rectangular-transfer-function RDF (Methods: "Descriptive,
// two-point spatial statistics") that is differentiable in the positions
// and in a scale factor of the z axis.
//
// Bin b of a pair at distance D receives w_b(D) = Phi((e_{b+1}-D)/sigma) -
// Phi((e_b-D)/sigma), evaluated through the tail of the normal distribution
// that does not cancel; only bins meeting (D - 6 sigma, D + 6 sigma) and
// pairs with D < r_max + 6 sigma count.  dw_b/dD = -(phi(t_{b+1}) -
// phi(t_b)) / sigma.
//
// Both kernels assign ions to wavefronts statically and sum in a fixed
// order, so results are reproducible bit for bit:
//  * forward: one wavefront per target; its pairs are collected, then the
//    Gaussian tail at each (pair, bin edge) is computed on its own lane, and
//    the bin terms (differences of adjacent edges) are added pair by pair to
//    the wavefront's FP64 LDS histogram; a reduction kernel sums the
//    per-wavefront rows in a fixed order (consecutive row ranges in row
//    order, then the range sums in range order);
//  * adjoint: pair lists are recomputed, not stored.  Every ion that takes
//    part in a pair (target or neighbour) gathers the derivative of L with
//    respect to its own position over its pairs in both roles, so no two
//    wavefronts write the same output and no atomics are needed.
#include "apt_pairdev.hpp"
#include "apt_smooth.hpp"

#pragma clang fp contract(off)

namespace apt {

size_t smooth_lds_bytes(bool fwd, int n_bins) {
    size_t b = (size_t)kSmoothTerms * 8u + (size_t)kWave * (5u * 8u + 4u);
    if (fwd) b += (size_t)n_bins * 8u;
    return b;
}

__global__ void k_smooth_edges(double* E, float r_max, int n_bins) {
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b <= n_bins; b += gridDim.x * blockDim.x)
        E[b] = ((double)b * (double)r_max) / (double)n_bins;
}

__global__ void k_fill_f32(float* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

// Bins [b0, b1] that meet (D - 6 sigma, D + 6 sigma); D < r_max + 6 sigma
// guarantees that the range is not empty.
__device__ __forceinline__ void smooth_window(const SmoothArgs& a, double D, int* b0, int* b1) {
    const int nb = a.n_bins;
    const double lo = D - a.w6, hi = D + a.w6;
    int g = (int)floor(lo * a.inv_width);
    g = g < 0 ? 0 : (g > nb - 1 ? nb - 1 : g);
    while (g > 0 && a.E[g] > lo) --g;
    while (g < nb - 1 && !(a.E[g + 1] > lo)) ++g;
    int h = (int)floor(hi * a.inv_width);
    h = h < 0 ? 0 : (h > nb - 1 ? nb - 1 : h);
    while (h < nb - 1 && a.E[h + 1] < hi) ++h;
    while (h > 0 && !(a.E[h] < hi)) --h;
    *b0 = g;
    *b1 = h;
}

__device__ __forceinline__ bool smooth_is_target(const SmoothArgs& a, uint32_t i) {
    const uint8_t l = a.lab[i];
    return (a.A == APT_ANY || l == a.A) && (a.d_bnd == nullptr || a.d_bnd[i] >= a.d_srf);
}
__device__ __forceinline__ bool smooth_is_nbr(const SmoothArgs& a, uint32_t i) {
    return a.B == APT_ANY || a.lab[i] == a.B;
}

template <bool BWD>
__device__ __forceinline__ void smooth_body(const SmoothArgs& a) {
    extern __shared__ __align__(16) uint8_t smem[];
    double* s_term = reinterpret_cast<double*>(smem);   // [kSmoothTerms] per-(pair, bin) terms
    double* s_D = s_term + kSmoothTerms;                // [64] buffered pairs: distance,
    double* s_dx = s_D + kWave;                         //   scaled displacement (candidate - ion),
    double* s_dy = s_dx + kWave;
    double* s_dz = s_dy + kWave;
    double* s_zz = s_dz + kWave;                        //   unscaled z difference,
    int* s_mul = reinterpret_cast<int*>(s_zz + kWave);  //   roles: count | (ion is the target) << 8
    double* s_hist = reinterpret_cast<double*>(s_mul + kWave);   // forward: [n_bins]

    const GridPlan P = *a.plan;
    const int l = lane_id();
    const double s = a.zscale ? *a.zscale : 1.0;
    const float rp = a.r_pre + P.eps;
    const float rp2 = rp * rp;
    if (!BWD) {
        for (int b = l; b < a.n_bins; b += kWave) s_hist[b] = 0.0;
        wave_sync();
    }
    double gs = 0.0;   // adjoint: this lane's share of dL/ds

    for (uint32_t t = blockIdx.x; t < P.nT; t += (uint32_t)a.W) {
        const uint32_t m = a.t_id[t];
        const float xm = a.xyz[3 * (size_t)m], ym = a.xyz[3 * (size_t)m + 1], zm = a.xyz[3 * (size_t)m + 2];
        const double Xm = (double)xm, Ym = (double)ym, Zm = s * (double)zm;
        const float pz = (float)Zm;
        const bool mT = BWD ? smooth_is_target(a, m) : true;
        const bool mB = BWD ? smooth_is_nbr(a, m) : false;
        double gx = 0.0, gy = 0.0, gz = 0.0;
        int nh = 0;   // buffered pairs (wave-uniform)

        auto flush = [&]() {
            wave_sync();
            // per pair: its window's bins b0 .. b0 + mh - 1 and their mh + 1
            // edges; the Gaussian tail (forward) or density (adjoint) is
            // evaluated once per edge, on its own lane, and shared by the
            // two bins that meet there
            int b0 = 0, mh = 0, me = 0;
            if (l < nh) {
                int b1;
                smooth_window(a, s_D[l], &b0, &b1);
                mh = b1 - b0 + 1;
                me = mh + 1;
            }
            const uint32_t inc = wave_incl_scan((uint32_t)me);
            const uint32_t tot = readlane(inc, kWave - 1);
            const uint32_t off = inc - (uint32_t)me;
            for (uint32_t c0 = 0; c0 < tot; c0 += kWave) {
                const uint32_t v = c0 + (uint32_t)l;
                int h = -1, ev = 0;
                const int r0 = __popcll(__ballot(inc <= c0));   // first pair ending after c0
                for (int rr = r0; rr < nh; ++rr) {
                    const uint32_t o = readlane(off, rr);
                    if (o >= c0 + kWave) break;
                    const uint32_t ln = (uint32_t)readlane(me, rr);
                    if (v >= o && v < o + ln) {
                        h = rr;
                        ev = readlane(b0, rr) + (int)(v - o);
                    }
                }
                if (h >= 0) {
                    const double t = (a.E[ev] - s_D[h]) / a.sigma;
                    if (!BWD) {
                        // the tail 0.5 erfc(|t| / sqrt 2) > 0, negated when t < 0
                        const double u = 0.5 * erfc(fabs(t) / M_SQRT2);
                        s_term[v] = t >= 0.0 ? u : -u;
                    } else {
                        s_term[v] = exp(-0.5 * t * t) / sqrt(2.0 * M_PI);
                    }
                }
            }
            wave_sync();
            if (!BWD) {
                // pair by pair (windows of different pairs overlap)
                for (int h = 0; h < nh; ++h) {
                    const uint32_t o = readlane(off, h);
                    const int ln = readlane(mh, h), bb = readlane(b0, h);
                    for (int q = l; q < ln; q += kWave) {
                        // bin mass from the tails at its edges: both edges above
                        // D, both below, or D inside the bin (an edge exactly at
                        // D falls to the last case with the same value)
                        const double slo = s_term[o + q], shi = s_term[o + q + 1];
                        const double vlo = fabs(slo), vhi = fabs(shi);
                        s_hist[bb + q] += slo > 0.0 ? vlo - vhi : (shi < 0.0 ? vhi - vlo : (1.0 - vhi) - vlo);
                    }
                    wave_sync();
                }
            } else if (l < nh) {
                double g = 0.0;
                for (int q = 0; q < mh; ++q) {
                    const double plo = s_term[off + (uint32_t)q], phi = s_term[off + (uint32_t)q + 1];
                    g += a.grad_h[b0 + q] * (-(phi - plo) / a.sigma);
                }
                const double D = s_D[l];
                if (D != 0.0) {
                    const int mul = s_mul[l];
                    const double cnt = (double)(mul & 0xff);
                    gx -= cnt * (g * (s_dx[l] / D));
                    gy -= cnt * (g * (s_dy[l] / D));
                    gz -= cnt * ((g * (s_dz[l] / D)) * s);
                    if (mul >> 8) {
                        const double zz = s_zz[l];
                        gs += g * s * zz * zz / D;
                    }
                }
            }
            wave_sync();
            nh = 0;
        };

        enumerate(P, a.cell_start, a.bpos, xm, ym, pz, a.r_pre, [&](bool valid, float4 c) {
            const uint32_t o = __builtin_bit_cast(uint32_t, c.w);
            bool hit = false;
            double D = 0.0, dX = 0.0, dY = 0.0, dZ = 0.0, zz = 0.0;
            int mul = 0;
            if (valid && o != m) {
                const float fx = c.x - xm, fy = c.y - ym, fz = c.z - pz;
                if (fx * fx + fy * fy + fz * fz < rp2) {
                    int t1 = 1, t2 = 0;
                    if (BWD) {
                        t1 = (mT && smooth_is_nbr(a, o)) ? 1 : 0;
                        t2 = (mB && smooth_is_target(a, o)) ? 1 : 0;
                    }
                    if (t1 + t2 > 0) {
                        const float zo = a.xyz[3 * (size_t)o + 2];
                        dX = (double)c.x - Xm;
                        dY = (double)c.y - Ym;
                        dZ = s * (double)zo - Zm;
                        D = sqrt((dX * dX + dY * dY) + dZ * dZ);
                        hit = D < a.cut;
                        mul = (t1 + t2) | (t1 << 8);
                        zz = (double)zo - (double)zm;
                    }
                }
            }
            uint64_t bal = __ballot(hit);
            while (bal) {
                const int room = a.hcap - nh;
                const bool mine = (bal >> l) & 1ull;
                const int rank = __popcll(bal & lanemask_lt());
                const uint64_t take = __ballot(mine && rank < room);
                if ((take >> l) & 1ull) {
                    const int slot = nh + rank;
                    s_D[slot] = D;
                    if (BWD) {
                        s_dx[slot] = dX;
                        s_dy[slot] = dY;
                        s_dz[slot] = dZ;
                        s_zz[slot] = zz;
                        s_mul[slot] = mul;
                    }
                }
                nh += __popcll(take);
                bal &= ~take;
                if (nh == a.hcap) flush();
            }
        });
        if (nh > 0) flush();

        if (BWD) {
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) {
                gx += __shfl_xor(gx, d, kWave);
                gy += __shfl_xor(gy, d, kWave);
                gz += __shfl_xor(gz, d, kWave);
            }
            if (l == 0) {
                a.grad_xyz[3 * (size_t)m] = (float)gx;
                a.grad_xyz[3 * (size_t)m + 1] = (float)gy;
                a.grad_xyz[3 * (size_t)m + 2] = (float)gz;
            }
        }
    }

    if (!BWD) {
        wave_sync();
        double* row = a.part + (size_t)blockIdx.x * (size_t)a.n_bins;
        for (int b = l; b < a.n_bins; b += kWave) row[b] = s_hist[b];
    } else {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) gs += __shfl_xor(gs, d, kWave);
        if (l == 0) a.part[blockIdx.x] = gs;
    }
}

__global__ __launch_bounds__(kWave) void k_smooth_fwd(SmoothArgs a) { smooth_body<false>(a); }
__global__ __launch_bounds__(kWave) void k_smooth_bwd(SmoothArgs a) { smooth_body<true>(a); }

// out[b] = sum over the W per-wavefront rows of part[w][b], in a fixed
// order: kReduceGroups consecutive row ranges, each summed in row order,
// then the range sums in range order (the same result on every run).
// Workgroup: 64 bins x kReduceGroups ranges; grid: ceil(n_bins / 64).
__global__ __launch_bounds__(kWave * kReduceGroups) void k_smooth_reduce(SmoothReduceArgs a) {
    __shared__ double s_p[kReduceGroups][kWave];
    const int tb = threadIdx.x % kWave, g = threadIdx.x / kWave;
    const int b = blockIdx.x * kWave + tb;
    const int w0 = (int)((int64_t)a.W * g / kReduceGroups), w1 = (int)((int64_t)a.W * (g + 1) / kReduceGroups);
    double acc = 0.0;
    if (b < a.n_bins) {
        const double* col = a.part + (size_t)b;
        int w = w0;
        for (; w + 8 <= w1; w += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = col[(size_t)(w + u) * (size_t)a.n_bins];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += v[u];
        }
        for (; w < w1; ++w) acc += col[(size_t)w * (size_t)a.n_bins];
    }
    s_p[g][tb] = acc;
    __syncthreads();
    if (g == 0 && b < a.n_bins) {
        double t = 0.0;
        for (int q = 0; q < kReduceGroups; ++q) t += s_p[q][tb];
        a.out[b] = t;
    }
}

}  // namespace apt
