/*
 * fsgo -- CPU oracle for the FastSimilarityGraph hot path (Macgregor & Sun,
 * "A Fast Similarity Graph Construction via Kernel Density Estimation",
 * NeurIPS 2023).
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load this
 * library.  It shares no code, header, table or constant with the GPU
 * library: it is a plain, slow, obviously correct FP64 restatement of the
 * paper's definitions, written so that a reader can check each function
 * against the paper by eye.
 *
 * Conventions (every reading of the paper is listed in the design notes):
 *  - points are FP32, row-major n x d; every value is promoted exactly to FP64;
 *  - kernel k(x,y) = exp(-gamma * ||x - y||^2), difference form, FP64
 *    (Section 2.1, Gaussian kernel; gamma = 1/sigma^2 in the paper's
 *    notation, 1/(2 sigma^2) in the workload descriptions); the other two
 *    kernels Section 2.1 names put ||x - y||_2 (exponential) or ||x - y||_1
 *    (Laplacian) in the exponent, with the same scale gamma;
 *  - the self term j == i is excluded from every mass and degree (the
 *    similarity graph of Section 2.1 has no self loops);
 *  - the partition tree is over index order; node [a,b) splits at
 *    mid = a + floor((b-a)/2), i.e. |X1| = floor(|X|/2) (Section 4.1);
 *  - uniforms come from Philox4x64-10 (Salmon et al., SC'11):
 *    key = (seed, 0), counter = (i, l, floor(level/4), 0),
 *    u = (word[level mod 4] >> 11) * 2^-53, in [0,1);
 *  - a sample at node [a,b) goes left iff u * (mL + mR) < mL, and never
 *    enters a child of zero mass (Algorithm 1, the branch on r);
 *  - indices are 0-based; nodes are half-open [a,b).
 * Return codes: 0 ok, -1 invalid argument, -2 out of memory, -3 capacity.
 */
#ifndef FSGO_H
#define FSGO_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* Kernel kinds (Section 2.1). */
#define FSGO_GAUSSIAN 0    /* exp(-gamma ||x - y||_2^2) */
#define FSGO_EXPONENTIAL 1 /* exp(-gamma ||x - y||_2)   */
#define FSGO_LAPLACIAN 2   /* exp(-gamma ||x - y||_1)   */

/* Philox4x64 with 10 rounds: out = philox(ctr, key).  (Salmon et al. 2011) */
void fsgo_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* out[4t..4t+3] = philox(ctrs[4t..4t+3], key) for t < m. */
void fsgo_philox_batch(const uint64_t* ctrs, int64_t m, const uint64_t key[2], uint64_t* out);

/* The uniform drawn for sample l of point i at tree level `level` (Algorithm 1,
 * one fresh r per recursion step). */
double fsgo_uniform(uint64_t seed, uint64_t i, uint64_t l, uint32_t level);

/* Split point of node [a,b): the left child holds floor((b-a)/2) points (Section 4.1). */
int64_t fsgo_split(int64_t a, int64_t b);

/* Kernel `kind` between two FP32 points, evaluated in FP64 from the
 * coordinate differences (Section 2.1).  Every function below takes the
 * kernel kind beside gamma; -1 for an unknown kind. */
double fsgo_kernel(const float* x, const float* y, int32_t d, int32_t kind, double gamma);

/* deg[i] = sum_{j != i} k(x_i, x_j)  (the KDE g_[1,n](x_i) of Algorithm 2
 * with the self term removed). */
int fsgo_degrees(const float* X, int64_t n, int32_t d, int32_t kind, double gamma, double* deg);

/* Segmented KDE (the KDE problem of Section 2.2 restricted to index ranges):
 * for segment s and every entry e in [q_ptr[s], q_ptr[s+1]):
 *   out_left[e]  = sum_{j in [lo[s], mid[s]), j != self_idx[e]} k(Q[q_idx[e]], X[j])
 *   out_right[e] = sum_{j in [mid[s], hi[s]), j != self_idx[e]} k(Q[q_idx[e]], X[j])
 * self_idx may be NULL (nothing excluded). */
int fsgo_kde_segmented(const float* Q, int64_t nq, const float* X, int64_t nx, int32_t d,
                       int32_t kind, double gamma, int64_t n_seg, const int64_t* q_ptr, const int32_t* q_idx,
                       const int32_t* lo, const int32_t* mid, const int32_t* hi,
                       const int32_t* self_idx, double* out_left, double* out_right);

/* Algorithm 1 run L times from the root for the listed rows (rows == NULL:
 * every row, n_rows must equal n).  For row r = rows[t] and sample l:
 *   nbr[t*L + l]    = the sampled neighbour y_{r,l}, or -1 when deg_r == 0;
 *   margin[t*L + l] = min over the levels of |u - mL/(mL+mR)| (may be NULL);
 *   deg[t]          = deg_r (may be NULL). */
int fsgo_sample_rows(const float* X, int64_t n, int32_t d, int32_t kind, double gamma, int32_t L,
                     uint64_t seed, const int32_t* rows, int64_t n_rows, int32_t* nbr,
                     double* deg, double* margin);

/* Probability that the descent from point i ends at leaf j, as the product
 * of the branch probabilities along the path (the product in the proof of
 * Lemma 1).  With an exact KDE it equals k(x_i,x_j)/deg_i. */
int fsgo_path_probability(const float* X, int64_t n, int32_t d, int32_t kind, double gamma, int64_t i,
                          int64_t j, double* prob);

/* Algorithm 2 after the sampling loop: the set of undirected edges
 * {i, nbr[i*L+l]} (nbr == -1 skipped), each with weight k/p_hat where
 *   p_i = min(L k/deg_i, 1), p_j = min(L k/deg_j, 1), p_hat = p_i + p_j - p_i p_j,
 * written as a symmetric CSR (each edge in both rows, columns ascending).
 * deg may be NULL (then computed here).  cap bounds col/w; *nnz receives 2|E|. */
int fsgo_build_csr(const float* X, int64_t n, int32_t d, int32_t kind, double gamma, int32_t L,
                   const int32_t* nbr, const double* deg, int64_t* row_ptr, int32_t* col,
                   double* w, int64_t cap, int64_t* nnz);

/* Number of OpenMP threads the oracle uses. */
int fsgo_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
