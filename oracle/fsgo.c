/*
 * fsgo.c -- CPU oracle for the FastSimilarityGraph hot path.
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT: only the tests, the smoke
 * check and the benchmark's CPU-baseline leg load it.  Plain C99 + OpenMP,
 * FP64 throughout, no blocking, fusion or reordering beyond the paper's own
 * definitions.  See fsgo.h for the conventions.
 */
#include "fsgo.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC 2011).  One round maps (c0,c1,c2,c3) with key      */
/* (k0,k1) to (hi(M1*c2)^c1^k0, lo(M1*c2), hi(M0*c0)^c3^k1, lo(M0*c0)); the */
/* key is advanced by the Weyl constants between rounds.                    */
/* ------------------------------------------------------------------------ */
static const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PHILOX_M1 = 0xCA5A826395121157ULL;
static const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ULL; /* golden ratio */
static const uint64_t PHILOX_W1 = 0xBB67AE8584CAA73BULL; /* sqrt(3) - 1 */

static void mul_hi_lo(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void fsgo_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mul_hi_lo(PHILOX_M0, c0, &hi0, &lo0);
        mul_hi_lo(PHILOX_M1, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double fsgo_uniform(uint64_t seed, uint64_t i, uint64_t l, uint32_t level) {
    uint64_t ctr[4] = {i, l, (uint64_t)(level / 4u), 0};
    uint64_t key[2] = {seed, 0};
    uint64_t out[4];
    fsgo_philox4x64_10(ctr, key, out);
    uint64_t word = out[level % 4u];
    return (double)(word >> 11) * (1.0 / 9007199254740992.0); /* 2^-53 */
}

void fsgo_philox_batch(const uint64_t* ctrs, int64_t m, const uint64_t key[2], uint64_t* out) {
    for (int64_t t = 0; t < m; ++t) fsgo_philox4x64_10(ctrs + 4 * t, key, out + 4 * t);
}

/* ------------------------------------------------------------------------ */
/* Tree and kernel                                                          */
/* ------------------------------------------------------------------------ */
int64_t fsgo_split(int64_t a, int64_t b) { return a + (b - a) / 2; }

/* The three kernels of Section 2.1: Gaussian exp(-gamma ||x-y||_2^2), exponential
 * exp(-gamma ||x-y||_2) and Laplacian exp(-gamma ||x-y||_1), each from the
 * coordinate differences in FP64. */
double fsgo_kernel(const float* x, const float* y, int32_t d, int32_t kind, double gamma) {
    double dist2 = 0.0, dist1 = 0.0;
    for (int32_t t = 0; t < d; ++t) {
        double diff = (double)x[t] - (double)y[t];
        dist2 += diff * diff;
        dist1 += fabs(diff);
    }
    if (kind == FSGO_EXPONENTIAL) return exp(-gamma * sqrt(dist2));
    if (kind == FSGO_LAPLACIAN) return exp(-gamma * dist1);
    return exp(-gamma * dist2);
}

/* r[j] = k(x_i, x_j) for every j, with r[i] = 0 (no self loop). */
static void kernel_row(const float* X, int64_t n, int32_t d, int32_t kind, double gamma, int64_t i, double* r) {
    const float* xi = X + (size_t)i * (size_t)d;
    for (int64_t j = 0; j < n; ++j)
        r[j] = (j == i) ? 0.0 : fsgo_kernel(xi, X + (size_t)j * (size_t)d, d, kind, gamma);
}

/* Mass of the index range [a,b) of a kernel row: the KDE g_[a,b] of eq. (1). */
static double range_mass(const double* r, int64_t a, int64_t b) {
    double s = 0.0;
    for (int64_t j = a; j < b; ++j) s += r[j];
    return s;
}

static int valid_kind(int32_t kind) {
    return kind == FSGO_GAUSSIAN || kind == FSGO_EXPONENTIAL || kind == FSGO_LAPLACIAN;
}

static int valid_common(int64_t n, int32_t d, int32_t kind, double gamma) {
    return n >= 1 && d >= 1 && valid_kind(kind) && isfinite(gamma) && gamma > 0.0;
}

int fsgo_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Degrees: g_[1,n](x_i) without the self term (Algorithm 2, the KDE after  */
/* the sampling loop).                                                      */
/* ------------------------------------------------------------------------ */
int fsgo_degrees(const float* X, int64_t n, int32_t d, int32_t kind, double gamma, double* deg) {
    if (!X || !deg || !valid_common(n, d, kind, gamma)) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        const float* xi = X + (size_t)i * (size_t)d;
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j)
            if (j != i) s += fsgo_kernel(xi, X + (size_t)j * (size_t)d, d, kind, gamma);
        deg[i] = s;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Segmented KDE                                                            */
/* ------------------------------------------------------------------------ */
int fsgo_kde_segmented(const float* Q, int64_t nq, const float* X, int64_t nx, int32_t d,
                       int32_t kind, double gamma, int64_t n_seg, const int64_t* q_ptr, const int32_t* q_idx,
                       const int32_t* lo, const int32_t* mid, const int32_t* hi,
                       const int32_t* self_idx, double* out_left, double* out_right) {
    if (!Q || !X || !q_ptr || !q_idx || !lo || !mid || !hi || !out_left || !out_right) return -1;
    if (nq < 1 || nx < 1 || d < 1 || !valid_kind(kind) || !isfinite(gamma) || gamma <= 0.0 || n_seg < 0) return -1;
    for (int64_t s = 0; s < n_seg; ++s) {
        if (!(0 <= lo[s] && lo[s] <= mid[s] && mid[s] <= hi[s] && hi[s] <= nx)) return -1;
        if (q_ptr[s] > q_ptr[s + 1] || q_ptr[s] < 0) return -1;
    }
    if (n_seg == 0) return 0;
    int64_t e_begin = q_ptr[0], e_end = q_ptr[n_seg];
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t e = e_begin; e < e_end; ++e) {
        /* the segment holding entry e: the last s with q_ptr[s] <= e */
        int64_t s_lo = 0, s_hi = n_seg - 1;
        while (s_lo < s_hi) {
            int64_t s_mid = s_lo + (s_hi - s_lo + 1) / 2;
            if (q_ptr[s_mid] <= e) s_lo = s_mid; else s_hi = s_mid - 1;
        }
        int64_t s = s_lo;
        int64_t qi = q_idx[e];
        int64_t self = self_idx ? (int64_t)self_idx[e] : -1;
        if (qi < 0 || qi >= nq) { out_left[e] = NAN; out_right[e] = NAN; continue; }
        const float* q = Q + (size_t)qi * (size_t)d;
        double left = 0.0, right = 0.0;
        for (int64_t j = lo[s]; j < mid[s]; ++j)
            if (j != self) left += fsgo_kernel(q, X + (size_t)j * (size_t)d, d, kind, gamma);
        for (int64_t j = mid[s]; j < hi[s]; ++j)
            if (j != self) right += fsgo_kernel(q, X + (size_t)j * (size_t)d, d, kind, gamma);
        out_left[e] = left;
        out_right[e] = right;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sampling: Algorithm 1 for one query, followed down the tree one level at  */
/* a time.  Level-batching (Section 4.2) regroups queries but leaves every  */
/* decision a function of the query's own node masses and uniform, so one   */
/* query at a time gives the same result.                                   */
/* ------------------------------------------------------------------------ */
static int32_t descend(const double* r, int64_t n, uint64_t seed, int64_t i, int64_t l,
                       double* min_margin) {
    int64_t a = 0, b = n;
    uint32_t level = 0;
    double margin = INFINITY;
    while (b - a > 1) {
        int64_t mid = fsgo_split(a, b);
        double mL = range_mass(r, a, mid);
        double mR = range_mass(r, mid, b);
        double t = mL + mR;
        double u = fsgo_uniform(seed, (uint64_t)i, (uint64_t)l, level);
        int go_left = (u * t < mL);
        if (go_left && mL == 0.0) go_left = 0;  /* never enter a child of zero mass */
        if (!go_left && mR == 0.0) go_left = 1;
        double m = fabs(u - mL / t);
        if (m < margin) margin = m;
        if (go_left) b = mid; else a = mid;
        ++level;
    }
    if (min_margin) *min_margin = margin;
    return (int32_t)a;
}

int fsgo_sample_rows(const float* X, int64_t n, int32_t d, int32_t kind, double gamma, int32_t L,
                     uint64_t seed, const int32_t* rows, int64_t n_rows, int32_t* nbr,
                     double* deg, double* margin) {
    if (!X || !nbr || !valid_common(n, d, kind, gamma) || L < 1 || n_rows < 0) return -1;
    if (!rows && n_rows != n) return -1;
    if (n > 2147483647LL) return -1;
    int failed = 0;
#pragma omp parallel
    {
        double* r = (double*)malloc((size_t)n * sizeof(double));
        if (!r) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t t = 0; t < n_rows; ++t) {
            if (!r) continue;
            int64_t i = rows ? (int64_t)rows[t] : t;
            if (i < 0 || i >= n) {
                for (int32_t l = 0; l < L; ++l) nbr[t * L + l] = -2;
                continue;
            }
            kernel_row(X, n, d, kind, gamma, i, r);
            double deg_i = range_mass(r, 0, n);
            if (deg) deg[t] = deg_i;
            for (int32_t l = 0; l < L; ++l) {
                double m = INFINITY;
                int32_t y = -1;
                if (deg_i > 0.0) y = descend(r, n, seed, i, l, &m);
                nbr[t * L + l] = y;
                if (margin) margin[t * L + l] = m;
            }
        }
        free(r);
    }
    return failed ? -2 : 0;
}

int fsgo_path_probability(const float* X, int64_t n, int32_t d, int32_t kind, double gamma, int64_t i,
                          int64_t j, double* prob) {
    if (!X || !prob || !valid_common(n, d, kind, gamma) || i < 0 || i >= n || j < 0 || j >= n)
        return -1;
    double* r = (double*)malloc((size_t)n * sizeof(double));
    if (!r) return -2;
    kernel_row(X, n, d, kind, gamma, i, r);
    double p = 1.0;
    int64_t a = 0, b = n;
    while (b - a > 1) {
        int64_t mid = fsgo_split(a, b);
        double m_parent = range_mass(r, a, b);
        if (j < mid) {
            p *= (m_parent > 0.0) ? range_mass(r, a, mid) / m_parent : 0.0;
            b = mid;
        } else {
            p *= (m_parent > 0.0) ? range_mass(r, mid, b) / m_parent : 0.0;
            a = mid;
        }
    }
    free(r);
    *prob = p;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Reweighting and CSR (Algorithm 2, the loop over the sampled edges).      */
/* ------------------------------------------------------------------------ */
typedef struct { int32_t row, col; } entry_t;

static int cmp_entry(const void* pa, const void* pb) {
    const entry_t* a = (const entry_t*)pa;
    const entry_t* b = (const entry_t*)pb;
    if (a->row != b->row) return a->row < b->row ? -1 : 1;
    if (a->col != b->col) return a->col < b->col ? -1 : 1;
    return 0;
}

int fsgo_build_csr(const float* X, int64_t n, int32_t d, int32_t kind, double gamma, int32_t L,
                   const int32_t* nbr, const double* deg_in, int64_t* row_ptr, int32_t* col,
                   double* w, int64_t cap, int64_t* nnz) {
    if (!X || !nbr || !row_ptr || !nnz || !valid_common(n, d, kind, gamma) || L < 1 || cap < 0)
        return -1;
    if (cap > 0 && (!col || !w)) return -1;
    int64_t n_samples = n * (int64_t)L;
    for (int64_t s = 0; s < n_samples; ++s)
        if (nbr[s] < -1 || nbr[s] >= n || nbr[s] == s / L) return -1;

    double* deg = NULL;
    if (!deg_in) {
        deg = (double*)malloc((size_t)n * sizeof(double));
        if (!deg) return -2;
        fsgo_degrees(X, n, d, kind, gamma, deg);
        deg_in = deg;
    }
    /* Each sampled edge {i, y} as the two directed entries (i,y) and (y,i). */
    entry_t* ent = (entry_t*)malloc((size_t)(2 * n_samples + 1) * sizeof(entry_t));
    if (!ent) { free(deg); return -2; }
    int64_t m = 0;
    for (int64_t s = 0; s < n_samples; ++s) {
        int32_t i = (int32_t)(s / L), y = nbr[s];
        if (y < 0) continue;
        ent[m].row = i; ent[m].col = y; ++m;
        ent[m].row = y; ent[m].col = i; ++m;
    }
    qsort(ent, (size_t)m, sizeof(entry_t), cmp_entry);
    /* E is a set: keep one copy of each directed entry. */
    int64_t u = 0;
    for (int64_t k = 0; k < m; ++k)
        if (k == 0 || cmp_entry(&ent[k], &ent[k - 1]) != 0) ent[u++] = ent[k];
    *nnz = u;
    if (u > cap) { free(ent); free(deg); return -3; }

    for (int64_t r = 0; r <= n; ++r) row_ptr[r] = 0;
    for (int64_t k = 0; k < u; ++k) row_ptr[ent[k].row + 1] += 1;
    for (int64_t r = 0; r < n; ++r) row_ptr[r + 1] += row_ptr[r];

    for (int64_t k = 0; k < u; ++k) {
        int64_t i = ent[k].row, j = ent[k].col;
        double kij = fsgo_kernel(X + (size_t)i * (size_t)d, X + (size_t)j * (size_t)d, d, kind, gamma);
        double p_i = fmin((double)L * kij / deg_in[i], 1.0);
        double p_j = fmin((double)L * kij / deg_in[j], 1.0);
        double p_hat = p_i + p_j - p_i * p_j;
        col[k] = (int32_t)j;
        w[k] = kij / p_hat;
    }
    free(ent);
    free(deg);
    return 0;
}
