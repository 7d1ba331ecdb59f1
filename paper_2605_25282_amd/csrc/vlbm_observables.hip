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

// out[0] = (1/n) sum_i |x_i - y_i|  (y == nullptr: (1/n) sum_i |x_i|).
// One block: statistics fields are small next to the ensemble state.
__global__ void __launch_bounds__(RED_THREADS) mean_abs_diff_kernel(const double *__restrict__ x,
                                                                    const double *__restrict__ y,
                                                                    long long n, double *out)
{
    __shared__ double lds[RED_THREADS];
    double s = 0.0;
    for (long long i = threadIdx.x; i < n; i += RED_THREADS)
        s += fabs(y ? x[i] - y[i] : x[i]);
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

// 0-based index of the empirical quantile at pct percent of m samples:
// ceil(pct m / 100) - 1, in exact integer arithmetic.
__host__ __device__ inline int quantile_row(int pct, int m) { return (int)(((long long)pct * m + 99) / 100) - 1; }

// ---------------------------------------------------------------------------
// Launchers (called by the C ABI in vlbm_api.hip after argument validation).
// ---------------------------------------------------------------------------
void launch_mean_abs_diff(const double *x, const double *y, long long n, double *out, hipStream_t st)
{
    mean_abs_diff_kernel<<<1, RED_THREADS, 0, st>>>(x, y, n, out);
}

void launch_strong_error(const double *a, const double *b, long long ncell, int m, double *per_real,
                         double *out, hipStream_t st)
{
    strong_error_kernel<<<m, 256, 0, st>>>(a, b, ncell, per_real);
    mean_abs_diff_kernel<<<1, RED_THREADS, 0, st>>>(per_real, nullptr, m, out);
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

void launch_width_ratio(const double *sorted, long long ncell, int m, double *q, hipStream_t st)
{
    width_ratio_kernel<<<(unsigned)((ncell + 255) / 256), 256, 0, st>>>(
        sorted, ncell, quantile_row(5, m), quantile_row(16, m), quantile_row(84, m), quantile_row(95, m), q);
}

} // namespace vlbm
