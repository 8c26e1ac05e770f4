/*
 * Seeded synthetic atom-probe point clouds (input generator only).
 *
 * This module makes inputs for both the oracle and the GPU library and
 * holds none of the spatial-statistics arithmetic.  Every random draw is a
 * pure function of (seed, stream, ion index), so any index range can be
 * regenerated on its own and the output does not depend on thread count.
 *
 * Shapes (the paper's synthetic specimens, Methods: Case studies,
 * "Benchmarking all functionality with synthetic datasets"): a box, or a
 * conical frustum with its axis along +z (z in [0, H], radius R0 at z = 0
 * and R1 at z = H).  Ions are i.i.d. uniform in the shape, exactly n of
 * them.  Spherical solute clusters stand in for the Al3Sc precipitates:
 * an ion whose noise-free position lies within r_c of a cluster centre is
 * Sc with probability p_c_sc and Al otherwise; other ions draw Sc / Si / Al
 * from the matrix probabilities.  Gaussian positional noise is applied after
 * labelling, and the distance to the specimen surface is computed from the
 * noisy position (negative outside the shape).
 *
 * Labels: 0 = Al, 1 = Sc, 2 = Si.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SYN_BOX 0
#define SYN_FRUSTUM 1

#define LAB_AL 0
#define LAB_SC 1
#define LAB_SI 2

typedef struct {
    int32_t shape;       /* SYN_BOX or SYN_FRUSTUM */
    int32_t pad0;
    double L[3];         /* box sides, box = [0,L0) x [0,L1) x [0,L2) */
    double H, R0, R1;    /* frustum */
    int64_t n;           /* number of ions */
    uint64_t seed;
    double p_m_sc;       /* matrix: P(Sc) */
    double p_m_si;       /* matrix: P(Si) */
    double p_c_sc;       /* inside a cluster: P(Sc), else Al */
    int64_t n_clusters;
    double r_c;          /* cluster radius */
    double noise;        /* positional noise sigma per axis */
} synth_params;

/* ---- counter-based random numbers --------------------------------------- */
static inline uint64_t mix64(uint64_t z) {
    z ^= z >> 30; z *= 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 27; z *= 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return z;
}
static inline uint64_t rnd(uint64_t seed, uint64_t stream, uint64_t i) {
    return mix64(mix64(seed * 0x9E3779B97F4A7C15ULL + stream * 0x632BE59BD9B4E019ULL) +
                 i * 0xD1B54A32D192ED03ULL);
}
/* uniform in [0, 1) with 53 random bits */
static inline double u01(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }
/* uniform in (0, 1] */
static inline double u01_open0(uint64_t r) { return ((double)(r >> 11) + 1.0) * 0x1.0p-53; }

enum { ST_POS0 = 0, ST_POS1, ST_POS2, ST_LAB, ST_N0, ST_N1, ST_N2, ST_N3, ST_CENTRE };

static double frustum_surface_distance(const synth_params* p, double x, double y, double z) {
    double rho = sqrt(x * x + y * y);
    double Rz = p->R0 + (p->R1 - p->R0) * z / p->H;
    double cosa = p->H / sqrt(p->H * p->H + (p->R0 - p->R1) * (p->R0 - p->R1));
    double d = (Rz - rho) * cosa;
    if (z < d) d = z;
    if (p->H - z < d) d = p->H - z;
    return d;
}

static double box_surface_distance(const synth_params* p, double x, double y, double z) {
    double d = x;
    if (p->L[0] - x < d) d = p->L[0] - x;
    if (y < d) d = y;
    if (p->L[1] - y < d) d = p->L[1] - y;
    if (z < d) d = z;
    if (p->L[2] - z < d) d = p->L[2] - z;
    return d;
}

double synth_surface_distance(const synth_params* p, double x, double y, double z) {
    return p->shape == SYN_FRUSTUM ? frustum_surface_distance(p, x, y, z)
                                   : box_surface_distance(p, x, y, z);
}

double synth_volume(const synth_params* p) {
    if (p->shape == SYN_FRUSTUM)
        return M_PI * p->H * (p->R0 * p->R0 + p->R0 * p->R1 + p->R1 * p->R1) / 3.0;
    return p->L[0] * p->L[1] * p->L[2];
}

/* Uniform point in the shape from three uniforms. */
static void sample_shape(const synth_params* p, double u0, double u1, double u2,
                         double* x, double* y, double* z) {
    if (p->shape == SYN_FRUSTUM) {
        /* z by inverting the cumulative cross-section area (proportional to R(z)^2) */
        double r;
        if (fabs(p->R1 - p->R0) < 1e-12 * p->R0) {
            r = p->R0;
            *z = u2 * p->H;
        } else {
            double a3 = p->R0 * p->R0 * p->R0, b3 = p->R1 * p->R1 * p->R1;
            r = cbrt(a3 + u2 * (b3 - a3));
            *z = (r - p->R0) * p->H / (p->R1 - p->R0);
            if (*z < 0) *z = 0;
            if (*z > p->H) *z = p->H;
        }
        double rho = r * sqrt(u0);
        double th = 2.0 * M_PI * u1;
        *x = rho * cos(th);
        *y = rho * sin(th);
    } else {
        *x = u0 * p->L[0];
        *y = u1 * p->L[1];
        *z = u2 * p->L[2];
    }
}

/* Cluster centres: uniform in the shape eroded by r_c (overlaps allowed). */
int synth_centres(const synth_params* p, double* c) {
    for (int64_t m = 0; m < p->n_clusters; ++m) {
        for (uint64_t att = 0;; ++att) {
            uint64_t base = ((uint64_t)m << 20) + att * 3;
            double u0 = u01(rnd(p->seed, ST_CENTRE, base));
            double u1 = u01(rnd(p->seed, ST_CENTRE, base + 1));
            double u2 = u01(rnd(p->seed, ST_CENTRE, base + 2));
            double x, y, z;
            sample_shape(p, u0, u1, u2, &x, &y, &z);
            if (synth_surface_distance(p, x, y, z) >= p->r_c) {
                c[3 * m] = x; c[3 * m + 1] = y; c[3 * m + 2] = z;
                break;
            }
            if (att > (1u << 18)) return -1;
        }
    }
    return 0;
}

/* Uniform hash grid over the cluster centres, cell edge >= r_c. */
typedef struct {
    double lo[3], h;
    int64_t dim[3];
    int64_t* start; /* [ncell + 1] */
    int64_t* item;  /* [n_clusters] */
} cgrid;

static int cgrid_build(cgrid* g, const double* c, int64_t m, double r_c) {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < m; ++i)
        for (int a = 0; a < 3; ++a) {
            if (c[3 * i + a] < lo[a]) lo[a] = c[3 * i + a];
            if (c[3 * i + a] > hi[a]) hi[a] = c[3 * i + a];
        }
    double h = r_c > 0 ? r_c : 1.0;
    /* keep the table small: at most ~4 cells per centre plus a floor */
    for (;;) {
        double cells = 1;
        for (int a = 0; a < 3; ++a) cells *= floor((hi[a] - lo[a]) / h) + 1;
        if (cells <= 4.0 * (double)m + 4096.0) break;
        h *= 1.25;
    }
    int64_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
        g->lo[a] = lo[a];
        g->dim[a] = (int64_t)floor((hi[a] - lo[a]) / h) + 1;
        ncell *= g->dim[a];
    }
    g->h = h;
    g->start = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
    g->item = (int64_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    if (!g->start || !g->item) return -1;
    int64_t* cell = (int64_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < m; ++i) {
        int64_t ci[3];
        for (int a = 0; a < 3; ++a) {
            ci[a] = (int64_t)floor((c[3 * i + a] - g->lo[a]) / h);
            if (ci[a] < 0) ci[a] = 0;
            if (ci[a] >= g->dim[a]) ci[a] = g->dim[a] - 1;
        }
        cell[i] = (ci[2] * g->dim[1] + ci[1]) * g->dim[0] + ci[0];
        g->start[cell[i] + 1]++;
    }
    for (int64_t q = 0; q < ncell; ++q) g->start[q + 1] += g->start[q];
    int64_t* fill = (int64_t*)malloc((size_t)ncell * sizeof(int64_t));
    memcpy(fill, g->start, (size_t)ncell * sizeof(int64_t));
    for (int64_t i = 0; i < m; ++i) g->item[fill[cell[i]]++] = i;
    free(fill);
    free(cell);
    return 0;
}

static int in_any_cluster(const cgrid* g, const double* c, double r_c, double x, double y, double z) {
    double q[3] = {x, y, z};
    int64_t lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = (int64_t)floor((q[a] - r_c - g->lo[a]) / g->h);
        hi[a] = (int64_t)floor((q[a] + r_c - g->lo[a]) / g->h);
        if (lo[a] < 0) lo[a] = 0;
        if (hi[a] >= g->dim[a]) hi[a] = g->dim[a] - 1;
        if (lo[a] > hi[a]) return 0;
    }
    double r2 = r_c * r_c;
    for (int64_t cz = lo[2]; cz <= hi[2]; ++cz)
        for (int64_t cy = lo[1]; cy <= hi[1]; ++cy)
            for (int64_t cx = lo[0]; cx <= hi[0]; ++cx) {
                int64_t cell = (cz * g->dim[1] + cy) * g->dim[0] + cx;
                for (int64_t t = g->start[cell]; t < g->start[cell + 1]; ++t) {
                    const double* cc = c + 3 * g->item[t];
                    double dx = x - cc[0], dy = y - cc[1], dz = z - cc[2];
                    if (dx * dx + dy * dy + dz * dz < r2) return 1;
                }
            }
    return 0;
}

/*
 * Generate ions [i0, i1) into xyz[(i1-i0)][3], lab[(i1-i0)], d_bnd[(i1-i0)]
 * (any output may be NULL).  centres: [n_clusters][3] from synth_centres.
 * Returns 0 on success.
 */
int synth_generate(const synth_params* p, const double* centres, int64_t i0, int64_t i1,
                   float* xyz, uint8_t* lab, float* d_bnd) {
    cgrid g;
    memset(&g, 0, sizeof g);
    int have_cl = p->n_clusters > 0 && p->r_c > 0 && centres;
    if (have_cl && cgrid_build(&g, centres, p->n_clusters, p->r_c) != 0) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = i0; i < i1; ++i) {
        uint64_t ui = (uint64_t)i;
        double x, y, z;
        sample_shape(p, u01(rnd(p->seed, ST_POS0, ui)), u01(rnd(p->seed, ST_POS1, ui)),
                     u01(rnd(p->seed, ST_POS2, ui)), &x, &y, &z);
        double ul = u01(rnd(p->seed, ST_LAB, ui));
        uint8_t s;
        if (have_cl && in_any_cluster(&g, centres, p->r_c, x, y, z)) {
            s = ul < p->p_c_sc ? LAB_SC : LAB_AL;
        } else {
            s = ul < p->p_m_sc ? LAB_SC : (ul < p->p_m_sc + p->p_m_si ? LAB_SI : LAB_AL);
        }
        if (p->noise > 0) {
            /* Box-Muller: two pairs of uniforms -> four normals, three used */
            double a1 = u01_open0(rnd(p->seed, ST_N0, ui)), b1 = u01(rnd(p->seed, ST_N1, ui));
            double a2 = u01_open0(rnd(p->seed, ST_N2, ui)), b2 = u01(rnd(p->seed, ST_N3, ui));
            double m1 = sqrt(-2.0 * log(a1)), m2 = sqrt(-2.0 * log(a2));
            x += p->noise * m1 * cos(2.0 * M_PI * b1);
            y += p->noise * m1 * sin(2.0 * M_PI * b1);
            z += p->noise * m2 * cos(2.0 * M_PI * b2);
        }
        int64_t o = i - i0;
        float fx = (float)x, fy = (float)y, fz = (float)z;
        if (xyz) { xyz[3 * o] = fx; xyz[3 * o + 1] = fy; xyz[3 * o + 2] = fz; }
        if (lab) lab[o] = s;
        if (d_bnd) d_bnd[o] = (float)synth_surface_distance(p, (double)fx, (double)fy, (double)fz);
    }
    free(g.start);
    free(g.item);
    return 0;
}
