// vlbm_observables.hip -- observables of the convergence study and the quantile
// diagnostics (gfx950): strong pathwise error (eq:strongError), cell-averaged
// differences of statistic fields (eq:mean, eq:std), the mean of per-cell
// one-point W1 values (eq:w1disc), empirical quantiles of sorted sample stores
// (eq:empcdf) and the quantile width ratio (eq:widthratio).
//
// Every reduction here runs in a fixed order (strided per-thread sums, then a
// fixed tree in LDS), so results do not depend on scheduling: two runs on the
// same data give the same bits.
#include "../../include/vlbm.h"
#include "vlbm_device.h"

namespace vlbm {

static constexpr int RED_THREADS = 1024;

// Fixed-order block sum of one value per thread (blockDim.x == NT).
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *lds)
{
    lds[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    return lds[0];
}

// ---------------------------------------------------------------------------
// Two-stage reductions over fields of common-grid cells (up to the 12.8 M nodes
// of the largest level).  Stage 1: block b reduces the contiguous range
// [b * RED_CHUNK, (b + 1) * RED_CHUNK) -- each thread a strided sum, then a fixed
// tree in LDS -- into partials[b].  Stage 2: one block sums the partials the
// same way and divides by the element count.  The order depends on n only, so
// equal inputs give equal bits, and the work is spread over n / RED_CHUNK
// blocks instead of one compute unit.
// ---------------------------------------------------------------------------
static constexpr int RED_CHUNK = 1024;      // elements per stage-1 block
static constexpr int PART_THREADS = 256;    // threads per stage-1 block

long long reduction_partials(long long n) { return (n + RED_CHUNK - 1) / RED_CHUNK; }

// partials[b] = sum over the block's range of |x_i - y_i| (|x_i| if y is null)
__global__ void __launch_bounds__(PART_THREADS) abs_partial_kernel(const double *__restrict__ x,
                                                                   const double *__restrict__ y,
                                                                   long long n, double *__restrict__ partials)
{
    __shared__ double lds[PART_THREADS];
    const long long i0 = (long long)blockIdx.x * RED_CHUNK;
    double s = 0.0;
    for (int k = threadIdx.x; k < RED_CHUNK; k += PART_THREADS) {
        const long long i = i0 + k;
        if (i < n)
            s += fabs(y ? x[i] - y[i] : x[i]);
    }
    const double tot = block_sum<PART_THREADS>(s, lds);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = tot;
}

// One-point W1 of eq:w1disc per cell from two sorted stores [m][ncell]:
// w1_cell[c] = (1/m) sum_k |a_(k) - b_(k)| (if w1_cell is not null), and the
// block's sum of these values into partials[b] (if partials is not null).
__global__ void __launch_bounds__(PART_THREADS) w1_partial_kernel(const double *__restrict__ a,
                                                                  const double *__restrict__ b,
                                                                  long long ncell, int m,
                                                                  double *__restrict__ w1_cell,
                                                                  double *__restrict__ partials)
{
    __shared__ double lds[PART_THREADS];
    const long long c0 = (long long)blockIdx.x * RED_CHUNK;
    double s = 0.0;
    for (int k = threadIdx.x; k < RED_CHUNK; k += PART_THREADS) {
        const long long c = c0 + k;
        if (c < ncell) {
            double w = 0.0;
            for (int q = 0; q < m; ++q)
                w += fabs(a[(size_t)q * ncell + c] - b[(size_t)q * ncell + c]);
            w = w / (double)m;
            if (w1_cell)
                w1_cell[c] = w;
            s += w;
        }
    }
    if (!partials)
        return;
    const double tot = block_sum<PART_THREADS>(s, lds);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = tot;
}

// out[0] = (sum of the np values in partials) / n, in a fixed order.
__global__ void __launch_bounds__(RED_THREADS) finish_mean_kernel(const double *__restrict__ partials,
                                                                  long long np, long long n, double *out)
{
    __shared__ double lds[RED_THREADS];
    double s = 0.0;
    for (long long i = threadIdx.x; i < np; i += RED_THREADS)
        s += partials[i];
    const double tot = block_sum<RED_THREADS>(s, lds);
    if (threadIdx.x == 0)
        out[0] = tot / (double)n;
}

// Relative L1 difference of realization m (eq:strongError): block m reduces
// sum_k |a[m][k] - b[m][k]| and sum_k |b[m][k]| over the common-grid cells.
__global__ void __launch_bounds__(256) strong_error_kernel(const double *__restrict__ a,
                                                           const double *__restrict__ b,
                                                           long long ncell, double *per_real)
{
    __shared__ double lds[256];
    const size_t base = (size_t)blockIdx.x * (size_t)ncell;
    double num = 0.0, den = 0.0;
    for (long long k = threadIdx.x; k < ncell; k += 256) {
        const double bv = b[base + k];
        num += fabs(a[base + k] - bv);
        den += fabs(bv);
    }
    const double tn = block_sum<256>(num, lds);
    __syncthreads();
    const double td = block_sum<256>(den, lds);
    if (threadIdx.x == 0)
        per_real[blockIdx.x] = tn / td;
}

struct QuantileArgs {
    int n_q;
    int k[VLBM_MAX_QUANTILES]; // 0-based order-statistic index of each quantile
};

// p_alpha of eq:empcdf from a sorted store [m][ncell]: the order statistic
// ceil(alpha m) (1-based), i.e. row k = ceil(alpha m) - 1.
__global__ void __launch_bounds__(256) quantile_kernel(const double *__restrict__ sorted, long long ncell,
                                                       QuantileArgs qa, double *__restrict__ out)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell)
        return;
    for (int q = 0; q < qa.n_q; ++q)
        out[(size_t)q * (size_t)ncell + c] = sorted[(size_t)qa.k[q] * (size_t)ncell + c];
}

// Q of eq:widthratio from the order statistics of p5, p16, p84, p95.
__global__ void __launch_bounds__(256) width_ratio_kernel(const double *__restrict__ sorted, long long ncell,
                                                          int k5, int k16, int k84, int k95, double *__restrict__ q)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell)
        return;
    const double p5 = sorted[(size_t)k5 * ncell + c], p16 = sorted[(size_t)k16 * ncell + c];
    const double p84 = sorted[(size_t)k84 * ncell + c], p95 = sorted[(size_t)k95 * ncell + c];
    q[c] = (p95 - p5) / (p84 - p16);
}

// ---------------------------------------------------------------------------
// Two-point Wasserstein distance (eq:w2).  One workgroup per ordered pair of
// subsampled cells (k, k'): the coarse law has the M points
// P_i = (a[i][c_k], a[i][c_k']), the fine law Q_j = (b[j][c_k], b[j][c_k']), and
// W = min over permutations s of (1/M) sum_i |P_i - Q_s(i)| (Euclidean cost).
// Solved exactly by shortest augmenting paths with row / column potentials
// (Hungarian method): row i is inserted by growing a Dijkstra tree over the
// columns on reduced costs C(i0, j) - u(i0) - v(j) until an unmatched column is
// reached, then the path is flipped.  Columns are owned by threads (their
// potential, tentative distance, predecessor and tree flag stay in registers);
// row potentials, the matching and the points sit in LDS.  The argmin over
// columns breaks ties by the smallest column index, so every run gives the
// same assignment.  Costs are recomputed from the points, sqrt(dx^2 + dy^2).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int subsample_index(int k, int n, int n_pd) { return (2 * k + 1) * n / (2 * n_pd); }

template <int NT, int MAXC>
__global__ void __launch_bounds__(NT) w12_kernel(const double *__restrict__ a, const double *__restrict__ b,
                                                 int ncx, int ncy, int m, int n_pd, double *__restrict__ w_pair)
{
    extern __shared__ double lds_dyn[];
    double *px = lds_dyn, *py = px + m, *u = py + m; // u[0..m]: row potentials (row 0 unused)
    __shared__ double red_v[NT / 64];
    __shared__ int red_j[NT / 64];
    __shared__ int s_j1;
    int *pm = (int *)(u + m + 1); // pm[j] = row matched to column j (1-based rows, 0 = none)
    int *way = pm + m + 1;        // predecessor column of each column in the tree
    const int pair = blockIdx.x, npts = n_pd * n_pd;
    const int k1 = pair / npts, k2 = pair % npts;
    const size_t ncell = (size_t)ncx * (size_t)ncy;
    const size_t c1 = (size_t)subsample_index(k1 / n_pd, ncy, n_pd) * ncx + subsample_index(k1 % n_pd, ncx, n_pd);
    const size_t c2 = (size_t)subsample_index(k2 / n_pd, ncy, n_pd) * ncx + subsample_index(k2 % n_pd, ncx, n_pd);
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;

    // columns owned by this thread: j = 1 + t + c * NT
    double qx[MAXC], qy[MAXC], v[MAXC], minv[MAXC];
    bool used[MAXC];
#pragma unroll
    for (int c = 0; c < MAXC; ++c) {
        const int j = 1 + t + c * NT;
        qx[c] = qy[c] = v[c] = 0.0;
        if (j <= m) {
            qx[c] = b[(size_t)(j - 1) * ncell + c1];
            qy[c] = b[(size_t)(j - 1) * ncell + c2];
        }
    }
    for (int i = t; i < m; i += NT) {
        px[i] = a[(size_t)i * ncell + c1];
        py[i] = a[(size_t)i * ncell + c2];
    }
    for (int j = t; j <= m; j += NT) {
        u[j] = 0.0;
        pm[j] = 0;
    }
    __syncthreads();

    bool failed = false; // non-finite samples: no valid augmenting column (uniform)
    for (int row = 1; row <= m && !failed; ++row) {
        if (t == 0)
            pm[0] = row;
#pragma unroll
        for (int c = 0; c < MAXC; ++c) {
            minv[c] = INFINITY;
            used[c] = false;
        }
        int j0 = 0;
        __syncthreads();
        // the tree gains one matched column per pass, so a row needs at most row passes
        for (int pass = 0;; ++pass) {
            // column j0 joins the tree (column 0 is the virtual start)
#pragma unroll
            for (int c = 0; c < MAXC; ++c)
                if (1 + t + c * NT == j0)
                    used[c] = true;
            const int i0 = pm[j0];
            const double ux = px[i0 - 1], uy = py[i0 - 1], ui = u[i0];
            double best = INFINITY;
            int bj = 0x7fffffff;
#pragma unroll
            for (int c = 0; c < MAXC; ++c) {
                const int j = 1 + t + c * NT;
                if (j <= m && !used[c]) {
                    const double dx = ux - qx[c], dy = uy - qy[c];
                    const double cur = (sqrt(dx * dx + dy * dy) - ui) - v[c];
                    if (cur < minv[c]) {
                        minv[c] = cur;
                        way[j] = j0;
                    }
                    if (minv[c] < best) { // columns of a thread ascend: ties keep the smaller j
                        best = minv[c];
                        bj = j;
                    }
                }
            }
            // block argmin, ties -> smallest column
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const double ob = __shfl_xor(best, o, 64);
                const int oj = __shfl_xor(bj, o, 64);
                if (ob < best || (ob == best && oj < bj)) {
                    best = ob;
                    bj = oj;
                }
            }
            if (NT > 64) {
                if (lane == 0) {
                    red_v[wv] = best;
                    red_j[wv] = bj;
                }
                __syncthreads();
                best = red_v[0];
                bj = red_j[0];
#pragma unroll
                for (int w = 1; w < NT / 64; ++w)
                    if (red_v[w] < best || (red_v[w] == best && red_j[w] < bj)) {
                        best = red_v[w];
                        bj = red_j[w];
                    }
            }
            const double delta = best;
            const int j1 = bj;
            if (j1 < 1 || j1 > m || pass > m) { // only with NaN / infinite samples
                failed = true;
                break;
            }
            // potentials: tree columns and their rows move by delta, the others' distances drop
            if (t == 0) {
                u[pm[0]] += delta; // the virtual column 0 is always in the tree
                s_j1 = j1;
            }
#pragma unroll
            for (int c = 0; c < MAXC; ++c) {
                const int j = 1 + t + c * NT;
                if (j <= m) {
                    if (used[c]) {
                        u[pm[j]] += delta;
                        v[c] -= delta;
                    } else {
                        minv[c] -= delta;
                    }
                }
            }
            __syncthreads();
            j0 = s_j1;
            const bool reached_free = pm[j0] == 0;
            // every thread has read pm[j0] before thread 0 flips the path (which
            // rewrites pm) or any thread starts the next pass
            __syncthreads();
            if (reached_free)
                break;
        }
        if (failed)
            break;
        // flip the augmenting path back to the virtual column
        if (t == 0) {
            int j = j0;
            while (j != 0) {
                const int jp = way[j];
                pm[j] = pm[jp];
                j = jp;
            }
        }
        __syncthreads();
    }
    if (failed) {
        if (t == 0)
            w_pair[pair] = NAN;
        return;
    }
    // matched cost in row order: row i is matched to the column whose pm is i
    int *col_of = way; // reuse: col_of[i] for rows 1..m
    for (int j = 1 + t; j <= m; j += NT)
        col_of[pm[j]] = j;
    __syncthreads();
    if (t == 0) {
        double tot = 0.0;
        for (int i = 1; i <= m; ++i) {
            const int j = col_of[i];
            if (j < 1 || j > m) { // not a permutation: never read memory with it
                tot = NAN;
                break;
            }
            const double dx = px[i - 1] - b[(size_t)(j - 1) * ncell + c1];
            const double dy = py[i - 1] - b[(size_t)(j - 1) * ncell + c2];
            tot += sqrt(dx * dx + dy * dy);
        }
        w_pair[pair] = tot / (double)m;
    }
}

// 0-based index of the empirical quantile at pct percent of m samples:
// ceil(pct m / 100) - 1, in exact integer arithmetic.
__host__ __device__ inline int quantile_row(int pct, int m) { return (int)(((long long)pct * m + 99) / 100) - 1; }

// ---------------------------------------------------------------------------
// Launchers (called by the C ABI in vlbm_api.hip after argument validation).
// ---------------------------------------------------------------------------
// Workspace of the stage-1 partial sums: `partials` holds at least
// reduction_partials(n) doubles (caller-provided or the static workspace).
void launch_mean_abs_diff(const double *x, const double *y, long long n, double *out, double *partials,
                          hipStream_t st)
{
    const long long np = reduction_partials(n);
    abs_partial_kernel<<<(unsigned)np, PART_THREADS, 0, st>>>(x, y, n, partials);
    finish_mean_kernel<<<1, RED_THREADS, 0, st>>>(partials, np, n, out);
}

void launch_w1(const double *a, const double *b, long long ncell, int m, double *w1_cell, double *w1_mean,
               double *partials, hipStream_t st)
{
    const long long np = reduction_partials(ncell);
    w1_partial_kernel<<<(unsigned)np, PART_THREADS, 0, st>>>(a, b, ncell, m, w1_cell, w1_mean ? partials : nullptr);
    if (w1_mean)
        finish_mean_kernel<<<1, RED_THREADS, 0, st>>>(partials, np, ncell, w1_mean);
}

void launch_strong_error(const double *a, const double *b, long long ncell, int m, double *per_real,
                         double *out, hipStream_t st)
{
    strong_error_kernel<<<m, 256, 0, st>>>(a, b, ncell, per_real);
    finish_mean_kernel<<<1, RED_THREADS, 0, st>>>(per_real, m, m, out);
}

void launch_quantiles(const double *sorted, long long ncell, int m, const int *pct, int n_q, double *out,
                      hipStream_t st)
{
    QuantileArgs qa{};
    qa.n_q = n_q;
    for (int q = 0; q < n_q; ++q)
        qa.k[q] = quantile_row(pct[q], m);
    quantile_kernel<<<(unsigned)((ncell + 255) / 256), 256, 0, st>>>(sorted, ncell, qa, out);
}

// LDS bytes of one two-point workgroup: points (2m), row potentials (m+1),
// matching and predecessors (2 (m+1) ints)
size_t w12_lds_bytes(int m) { return (size_t)(3 * m + 1) * sizeof(double) + (size_t)2 * (m + 1) * sizeof(int); }

void launch_w12(const double *a, const double *b, int ncx, int ncy, int m, int n_pd, double *w_pair,
                double *w_mean, hipStream_t st)
{
    const unsigned P = (unsigned)(n_pd * n_pd) * (unsigned)(n_pd * n_pd);
    const size_t lds = w12_lds_bytes(m);
    if (m <= 256)
        w12_kernel<64, 4><<<P, 64, lds, st>>>(a, b, ncx, ncy, m, n_pd, w_pair);
    else
        w12_kernel<256, 4><<<P, 256, lds, st>>>(a, b, ncx, ncy, m, n_pd, w_pair);
    if (w_mean)
        finish_mean_kernel<<<1, RED_THREADS, 0, st>>>(w_pair, (long long)P, (long long)P, w_mean);
}

void launch_width_ratio(const double *sorted, long long ncell, int m, double *q, hipStream_t st)
{
    width_ratio_kernel<<<(unsigned)((ncell + 255) / 256), 256, 0, st>>>(
        sorted, ncell, quantile_row(5, m), quantile_row(16, m), quantile_row(84, m), quantile_row(95, m), q);
}

} // namespace vlbm
