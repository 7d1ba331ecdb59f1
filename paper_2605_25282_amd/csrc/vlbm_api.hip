// vlbm_api.hip -- host side of the C ABI declared in include/vlbm.h.
//
// The host validates every argument before enqueueing anything, owns the
// per-ensemble control ring (time, step count, kinetic speed, wave-speed
// maximum, latched status per realization) and sequences the kernels of
// vlbm_kernels.hip on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/vlbm.h"
#include "vlbm_device.h"

namespace vlbm {
template <int PREC> __global__ void init_macro_kernel(PhysArgs, LevelArgs, const double *, Ctl);
template <int PREC> __global__ void equilibrium_kernel(PhysArgs, LevelArgs, Ctl, int);
template <int PREC> __global__ void step_ref_kernel(PhysArgs, LevelArgs, Ctl, int, double);
template <int PREC> __global__ void step_march_kernel(PhysArgs, MultiLevel, Ctl, int, double);
template <int PREC> __global__ void moments_kernel(PhysArgs, LevelArgs, Ctl, int, double *, double *, double *);
template <int PREC> __global__ void get_state_kernel(LevelArgs, Ctl, int, double *);
template <int PREC> __global__ void set_macro_kernel(PhysArgs, LevelArgs, Ctl, const double *);
template <int PREC> __global__ void set_state_kernel(PhysArgs, LevelArgs, Ctl, const double *);
template <int PREC>
__global__ void stats_accumulate_kernel(PhysArgs, LevelArgs, Ctl, int, int, double *, long long, double *, long long);
__global__ void stats_finalize_kernel(const double *, long long, long long, double *, double *);
template <int CPB> __global__ void sort_samples_kernel(double *, long long, int, int);
long long reduction_partials(long long n);
void launch_mean_abs_diff(const double *x, const double *y, long long n, double *out, double *partials,
                          hipStream_t st);
void launch_w1(const double *a, const double *b, long long ncell, int m, double *w1_cell, double *w1_mean,
               double *partials, hipStream_t st);
void launch_strong_error(const double *a, const double *b, long long ncell, int m, double *per_real,
                         double *out, hipStream_t st);
void launch_quantiles(const double *sorted, long long ncell, int m, const int *pct, int n_q, double *out,
                      hipStream_t st);
void launch_width_ratio(const double *sorted, long long ncell, int m, double *q, hipStream_t st);
void launch_w12(const double *a, const double *b, int ncx, int ncy, int m, int n_pd, double *w_pair,
                double *w_mean, hipStream_t st);
} // namespace vlbm

using namespace vlbm;

namespace {

thread_local std::string g_err = "no error";

vlbm_status fail(vlbm_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(VLBM_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

#define LAUNCH_CHECK(what)                                                              \
    do {                                                                                \
        hipError_t e_ = hipGetLastError();                                              \
        if (e_ != hipSuccess)                                                           \
            return fail(VLBM_ERR_HIP, "%s launch failed: %s", what, hipGetErrorString(e_)); \
    } while (0)

// Bytes of the per-ensemble control block: the three-launch ring of time, kinetic
// speed, step count and wave-speed maximum, the status words, and the nine
// counters of the dynamic work dealing.
size_t ctl_block_bytes(int nr)
{
    return (size_t)3 * nr * (sizeof(double) * 2 + sizeof(long long) + sizeof(unsigned long long)) +
           (size_t)nr * sizeof(int) + 9 * sizeof(unsigned);
}

// Bytes of one state buffer: R x ny row blocks, each of nstrip strip blocks
// that hold 64 element positions of all 20 planes (FP64: 160 B per position;
// mixed: 8 FP64 and 12 FP32 planes, 112 B per position).
size_t state_bytes(int prec, int bc, int nx, int ny, int R)
{
    const size_t slots = (size_t)SLOTS * (size_t)strip_count(nx, bc == VLBM_BC_PERIODIC);
    return (size_t)R * (size_t)ny * slots * (prec == VLBM_FP64 ? 160u : 112u);
}

vlbm_status check_params(const vlbm_params *p)
{
    if (!p)
        return fail(VLBM_ERR_ARG, "params is NULL");
    if (!(p->gamma > 1.0) || !std::isfinite(p->gamma))
        return fail(VLBM_ERR_ARG, "gamma must be > 1 (got %g)", p->gamma);
    if (!(p->alpha >= 0.0 && p->alpha < 1.0))
        return fail(VLBM_ERR_ARG, "alpha must lie in [0, 1) (got %g)", p->alpha);
    if (!(p->kappa >= 1.0) || !std::isfinite(p->kappa))
        return fail(VLBM_ERR_ARG, "kappa must be >= 1 (got %g)", p->kappa);
    if (!(p->rlmp_relax >= 0.0) || !std::isfinite(p->rlmp_relax))
        return fail(VLBM_ERR_ARG, "rlmp_relax must be >= 0 (got %g)", p->rlmp_relax);
    if (!(p->pos_eps >= 0.0 && p->pos_eps < 1.0))
        return fail(VLBM_ERR_ARG, "pos_eps must lie in [0, 1) (got %g)", p->pos_eps);
    if (!(p->rho_amb > 0.0) || !(p->p_amb > 0.0) || !(p->rho_jet > 0.0) || !(p->r_jet >= 0.0) ||
        !std::isfinite(p->v_jet) || !std::isfinite(p->kl_amp) || !std::isfinite(p->rho_amb) ||
        !std::isfinite(p->p_amb) || !std::isfinite(p->rho_jet) || !std::isfinite(p->r_jet))
        return fail(VLBM_ERR_ARG, "jet constants must be finite with rho_amb, p_amb, rho_jet > 0, r_jet >= 0");
    if (p->kl_modes < 0 || p->kl_modes > 64)
        return fail(VLBM_ERR_ARG, "kl_modes must lie in [0, 64] (got %d)", p->kl_modes);
    if (p->kl_decay < 0 || p->kl_decay > 16)
        return fail(VLBM_ERR_ARG, "kl_decay must lie in [0, 16] (got %d)", p->kl_decay);
    if (p->bc < VLBM_BC_JET || p->bc > VLBM_BC_NEUMANN)
        return fail(VLBM_ERR_ARG, "unknown bc %d", p->bc);
    if (p->limiter < VLBM_LIMITER_RLMP || p->limiter > VLBM_THETA_ONE)
        return fail(VLBM_ERR_ARG, "unknown limiter %d", p->limiter);
    if (p->precision != VLBM_FP64 && p->precision != VLBM_MIXED)
        return fail(VLBM_ERR_ARG, "unknown precision %d", p->precision);
    if (p->reserved != 0)
        return fail(VLBM_ERR_ARG, "reserved must be 0");
    return VLBM_OK;
}

vlbm_status check_grid(int precision, int bc, int nx, int ny, int R)
{
    if (nx < 3 || ny < 3)
        return fail(VLBM_ERR_SIZE, "a level needs nx, ny >= 3 (got %d x %d)", nx, ny);
    if (R < 1 || R > 65535)
        return fail(VLBM_ERR_SIZE, "n_real must lie in [1, 65535] (got %d)", R);
    if ((ny + 3) / 4 > 65535)
        return fail(VLBM_ERR_SIZE, "ny = %d exceeds the launch grid", ny);
    // kernels address a realization's state with 32-bit byte offsets
    const double per_real = (double)state_bytes(precision, bc, nx, ny, 1);
    if (per_real >= 4294967296.0)
        return fail(VLBM_ERR_SIZE, "one realization of a %d x %d level needs %.0f bytes (limit 4 GiB)", nx, ny, per_real);
    if ((double)nx * (double)ny * (double)R * 20.0 > 9.0e15)
        return fail(VLBM_ERR_SIZE, "level too large");
    return VLBM_OK;
}

PhysArgs phys_args(const vlbm_params &p)
{
    return PhysArgs{p.gamma, p.alpha, p.kappa, p.rlmp_relax, p.pos_eps, p.rho_amb, p.p_amb, p.rho_jet,
                    p.v_jet, p.r_jet, p.kl_amp, p.kl_modes, p.kl_decay, p.bc, p.limiter};
}

dim3 node_grid(const LevelArgs &L) { return dim3((L.nx + 63) / 64, (L.ny + 3) / 4, L.R); }

} // namespace

struct vlbm_ensemble {
    vlbm_params p;
    std::vector<LevelArgs> levels;
    int n_real = 0;
    hipStream_t stream = nullptr;
    void *ctl_mem = nullptr;
    double *coeffs_dev = nullptr;
    Ctl ctl{};
    long long n_launch = 0; // launches since the last (re)initialisation: ring phase = n % 3
    int kernel = VLBM_KERNEL_MARCH;
    int chunk_rows = 0;     // 0 = automatic
    int n_cu = 256;         // compute units of the device
    int march_blocks_per_cu[3] = {4, 2, 1}; // resident blocks per CU for 1, 2, 4 waves per block
    int waves_per_block = 4; // wavefronts per block of the marching kernel (1, 2 or 4)
    int item_order = 0;      // 0 strip fastest, 1 realization fastest
    int dealing = 1;         // 0 static round-robin, 1 per-XCD work queues (default)
    std::vector<int> level_chunk; // per-level chunk override (0 = from chunk_rows / model)
    // hipGraph of GRAPH_STEPS consecutive steps (ring phases 0,1,2,...), captured on
    // an internal stream and replayed on the ensemble's stream
    bool use_graph = true;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph = nullptr;
    double graph_t_final = 0.0;
};

static constexpr int GRAPH_STEPS = 30; // a multiple of 3 (the control ring's period)

namespace {
// Process-wide cache of tuned configurations, keyed by the whole launch
// (precision, boundary mode, limiter, realizations and every level's shape):
// the chunk height of each level, waves per block and item order.
typedef std::vector<long long> TuneKey;
struct TuneChoice {
    std::vector<int> chunks;
    int waves_per_block = 4;
    int item_order = 0;
    int dealing = 1;
};
std::map<TuneKey, TuneChoice> g_tune_cache;
std::mutex g_tune_mu;

TuneKey tune_key(const vlbm_ensemble *e)
{
    TuneKey k{e->p.precision, e->p.bc, e->p.limiter, e->n_real, (long long)e->levels.size()};
    for (const LevelArgs &L : e->levels) {
        k.push_back(L.nx);
        k.push_back(L.ny);
    }
    return k;
}

int wpb_index(int wpb) { return wpb == 1 ? 0 : (wpb == 2 ? 1 : 2); }
} // namespace

namespace {

int phase_of(const vlbm_ensemble *e) { return (int)(e->n_launch % 3); }

// Strips of the marching kernel = column strips of the state layout; lane 62 of
// the last strip carries the last column of a bounded level of 60 q + 1 columns.
int strips_of(const vlbm_ensemble *e, const LevelArgs &L, int *lane62)
{
    const bool periodic = e->p.bc == VLBM_BC_PERIODIC;
    *lane62 = (!periodic && (L.nx - 1) % STRIP == 0) ? 1 : 0;
    return L.nstrip;
}

// Resident wavefronts of the marching kernel (one per SIMD at its register use).
long long resident_waves(const vlbm_ensemble *e)
{
    const int wpb = e->waves_per_block;
    return (long long)e->n_cu * e->march_blocks_per_cu[wpb_index(wpb)] * wpb;
}

// Default chunk height: the even split of the rows nearest 64 (short items keep
// neighbouring strips in step and let the work queues balance finely), split
// further while there are fewer than eight items per resident wave; rows >= 16.
int model_chunk(const vlbm_ensemble *e, const LevelArgs &L, int nstrip)
{
    const long long target = 8LL * resident_waves(e);
    const long long per_chunk = (long long)L.R * nstrip;
    int nch = std::max(1, (L.ny + 32) / 64);
    while ((long long)nch * per_chunk < target && (L.ny + nch) / (nch + 1) >= 16)
        ++nch;
    int chunk = (L.ny + nch - 1) / nch;
    return chunk < 16 ? std::min(16, L.ny) : chunk;
}

MarchArgs march_args(const vlbm_ensemble *e, int level)
{
    const LevelArgs &L = e->levels[level];
    MarchArgs ma{};
    ma.nstrip = strips_of(e, L, &ma.lane62_last);
    int chunk = e->level_chunk.empty() ? 0 : e->level_chunk[level];
    if (chunk <= 0)
        chunk = e->chunk_rows;
    if (chunk <= 0)
        chunk = model_chunk(e, L, ma.nstrip);
    if (chunk > L.ny)
        chunk = L.ny;
    ma.chunk = chunk;
    ma.nchunk = (L.ny + chunk - 1) / chunk;
    ma.order = e->item_order;
    return ma;
}

// One launch over levels [l0, l1): concatenated work items, grid sized to the
// resident capacity, XCD-aware block numbering.
MultiLevel multi_level(const vlbm_ensemble *e, int l0, int l1, unsigned *grid)
{
    MultiLevel ml{};
    ml.nlev = l1 - l0;
    ml.item_off[0] = 0;
    for (int i = 0; i < ml.nlev; ++i) {
        ml.L[i] = e->levels[l0 + i];
        ml.ma[i] = march_args(e, l0 + i);
        ml.item_off[i + 1] = ml.item_off[i] + (long long)ml.L[i].R * ml.ma[i].nstrip * ml.ma[i].nchunk;
    }
    const int wpb = e->waves_per_block;
    ml.wpb = wpb;
    ml.dynamic = e->dealing;
    long long blocks = (ml.item_off[ml.nlev] + wpb - 1) / wpb;
    const long long resident = resident_waves(e) / wpb;
    if (blocks > resident)
        blocks = resident;
    if (blocks < 1)
        blocks = 1;
    ml.nblocks = (int)blocks;
    ml.per_xcd = (ml.nblocks + 7) / 8;
    *grid = (unsigned)(8 * ml.per_xcd);
    return ml;
}

// Enqueue one step of levels [l0, l1) on stream st.
vlbm_status launch_step(vlbm_ensemble *e, const PhysArgs &ph, int l0, int l1, int phase, double t_final,
                        hipStream_t st)
{
    if (e->kernel == VLBM_KERNEL_REFERENCE) {
        for (int l = l0; l < l1; ++l) {
            const LevelArgs &L = e->levels[l];
            if (e->p.precision == VLBM_FP64)
                step_ref_kernel<0><<<node_grid(L), 256, 0, st>>>(ph, L, e->ctl, phase, t_final);
            else
                step_ref_kernel<1><<<node_grid(L), 256, 0, st>>>(ph, L, e->ctl, phase, t_final);
        }
    } else {
        unsigned grid = 0;
        const MultiLevel ml = multi_level(e, l0, l1, &grid);
        const unsigned threads = 64u * (unsigned)ml.wpb;
        if (e->p.precision == VLBM_FP64)
            step_march_kernel<0><<<grid, threads, 0, st>>>(ph, ml, e->ctl, phase, t_final);
        else
            step_march_kernel<1><<<grid, threads, 0, st>>>(ph, ml, e->ctl, phase, t_final);
    }
    LAUNCH_CHECK("step");
    return VLBM_OK;
}

vlbm_status check_level(const vlbm_ensemble *e, int level)
{
    if (!e)
        return fail(VLBM_ERR_ARG, "ensemble is NULL");
    if (level < 0 || level >= (int)e->levels.size())
        return fail(VLBM_ERR_ARG, "level %d out of range [0, %zu)", level, e->levels.size());
    return VLBM_OK;
}

// Read the control slot holding the current state into host vectors.
vlbm_status read_ctl(const vlbm_ensemble *e, std::vector<double> &t, std::vector<long long> &steps,
                     std::vector<double> &a, std::vector<int> &status)
{
    const int nr = e->ctl.nr, ph = phase_of(e);
    t.resize(nr);
    steps.resize(nr);
    a.resize(nr);
    status.resize(nr);
    HIP_TRY(hipMemcpyAsync(t.data(), e->ctl.t + (size_t)ph * nr, nr * sizeof(double), hipMemcpyDeviceToHost, e->stream));
    HIP_TRY(hipMemcpyAsync(steps.data(), e->ctl.steps + (size_t)ph * nr, nr * sizeof(long long), hipMemcpyDeviceToHost, e->stream));
    HIP_TRY(hipMemcpyAsync(a.data(), e->ctl.a_last + (size_t)ph * nr, nr * sizeof(double), hipMemcpyDeviceToHost, e->stream));
    HIP_TRY(hipMemcpyAsync(status.data(), e->ctl.status, nr * sizeof(int), hipMemcpyDeviceToHost, e->stream));
    HIP_TRY(hipStreamSynchronize(e->stream));
    return VLBM_OK;
}

} // namespace

extern "C" {

const char *vlbm_last_error(void) { return g_err.c_str(); }

vlbm_status vlbm_kl_coefficients(uint64_t seed, int64_t first, int32_t count, int32_t modes, double *out)
{
    if (!out)
        return fail(VLBM_ERR_ARG, "out is NULL");
    if (first < 0 || count < 0 || modes < 0 || modes > 64)
        return fail(VLBM_ERR_ARG, "need first >= 0, count >= 0 and 0 <= modes <= 64");
    // SplitMix64 (Steele, Lea & Flood 2014) in counter mode: draw n of the stream
    // seeded with `seed` is the mixing function applied to seed + (n + 1) G.
    const uint64_t G = 0x9E3779B97F4A7C15ull;
    const uint64_t per = 2ull * (uint64_t)modes;
    for (int64_t k = 0; k < count; ++k)
        for (uint64_t c = 0; c < per; ++c) {
            const uint64_t n = ((uint64_t)first + (uint64_t)k) * per + c;
            uint64_t z = seed + (n + 1ull) * G;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z = z ^ (z >> 31);
            const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0); // top 53 bits, [0, 1)
            out[k * (int64_t)per + (int64_t)c] = 2.0 * u - 1.0;
        }
    return VLBM_OK;
}

vlbm_status vlbm_state_bytes(const vlbm_params *p, int32_t nx, int32_t ny, int32_t n_real, size_t *bytes)
{
    vlbm_status rc = check_params(p);
    if (rc != VLBM_OK)
        return rc;
    if ((rc = check_grid(p->precision, p->bc, nx, ny, n_real)) != VLBM_OK)
        return rc;
    if (!bytes)
        return fail(VLBM_ERR_ARG, "bytes is NULL");
    *bytes = state_bytes(p->precision, p->bc, nx, ny, n_real);
    return VLBM_OK;
}

vlbm_status vlbm_init_ensemble(const vlbm_params *p, const vlbm_level *levels, int32_t n_levels,
                               const double *coeffs, int32_t n_real, void *hip_stream,
                               vlbm_ensemble **out)
{
    vlbm_status rc = check_params(p);
    if (rc != VLBM_OK)
        return rc;
    if (!out)
        return fail(VLBM_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!levels || n_levels < 1 || n_levels > MAX_LEVELS)
        return fail(VLBM_ERR_ARG, "need 1..%d levels (got %d)", MAX_LEVELS, n_levels);
    if (p->bc == VLBM_BC_JET && !coeffs && p->kl_modes > 0)
        return fail(VLBM_ERR_ARG, "coeffs is NULL for the jet problem");
    for (int l = 0; l < n_levels; ++l) {
        const vlbm_level &L = levels[l];
        if ((rc = check_grid(p->precision, p->bc, L.nx, L.ny, n_real)) != VLBM_OK)
            return rc;
        if (!(L.dx > 0.0) || !std::isfinite(L.dx) || !std::isfinite(L.y_min))
            return fail(VLBM_ERR_ARG, "level %d: dx must be finite and > 0", l);
        for (int b = 0; b < 2; ++b)
            if (!L.state[b] || ((uintptr_t)L.state[b] & 255))
                return fail(VLBM_ERR_ARG, "level %d: state[%d] must be a non-NULL 256-byte aligned device pointer", l, b);
    }
    if (coeffs)
        for (long long k = 0; k < (long long)n_real * 2 * p->kl_modes; ++k)
            if (!(coeffs[k] >= -1.0 && coeffs[k] <= 1.0))
                return fail(VLBM_ERR_ARG, "coeffs[%lld] = %g outside [-1, 1]", k, coeffs[k]);
    if ((long long)n_real * n_levels > 1 << 24)
        return fail(VLBM_ERR_SIZE, "too many realizations");

    vlbm_ensemble *e = new vlbm_ensemble();
    e->p = *p;
    e->n_real = n_real;
    e->stream = (hipStream_t)hip_stream;
    const int nr = n_real * n_levels;
    for (int l = 0; l < n_levels; ++l) {
        LevelArgs L{levels[l].nx, levels[l].ny, n_real, strip_count(levels[l].nx, p->bc == VLBM_BC_PERIODIC),
                    l * n_real, levels[l].dx, levels[l].y_min, {levels[l].state[0], levels[l].state[1]}};
        e->levels.push_back(L);
    }
    const size_t ctl_bytes = ctl_block_bytes(nr);
    hipError_t he = hipMalloc(&e->ctl_mem, ctl_bytes);
    if (he != hipSuccess) {
        delete e;
        return fail(VLBM_ERR_HIP, "hipMalloc(control) failed: %s", hipGetErrorString(he));
    }
    char *c = (char *)e->ctl_mem;
    e->ctl.t = (double *)c;
    c += 3 * nr * sizeof(double);
    e->ctl.a_last = (double *)c;
    c += 3 * nr * sizeof(double);
    e->ctl.steps = (long long *)c;
    c += 3 * nr * sizeof(long long);
    e->ctl.amax = (unsigned long long *)c;
    c += 3 * nr * sizeof(unsigned long long);
    e->ctl.status = (int *)c;
    c += nr * sizeof(int);
    e->ctl.work = (unsigned *)c;
    e->ctl.nr = nr;
    const size_t ncoef = (size_t)n_real * 2 * p->kl_modes;
    if (ncoef > 0) {
        he = hipMalloc(&e->coeffs_dev, ncoef * sizeof(double));
        if (he == hipSuccess && coeffs)
            he = hipMemcpyAsync(e->coeffs_dev, coeffs, ncoef * sizeof(double), hipMemcpyHostToDevice, e->stream);
        if (he == hipSuccess && !coeffs)
            he = hipMemsetAsync(e->coeffs_dev, 0, ncoef * sizeof(double), e->stream);
    }
    if (he == hipSuccess)
        he = hipMemsetAsync(e->ctl_mem, 0, ctl_bytes, e->stream);
    if (he != hipSuccess) {
        vlbm_destroy(e);
        return fail(VLBM_ERR_HIP, "initialisation copy failed: %s", hipGetErrorString(he));
    }
    {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess &&
            prop.multiProcessorCount > 0)
            e->n_cu = prop.multiProcessorCount;
        for (int i = 0; i < 3; ++i) {
            const int threads = 64 << i;
            int occ = 0;
            hipError_t oe = p->precision == VLBM_FP64
                                ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, step_march_kernel<0>, threads, 0)
                                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, step_march_kernel<1>, threads, 0);
            if (oe == hipSuccess && occ > 0)
                e->march_blocks_per_cu[i] = occ;
        }
    }
    const PhysArgs ph = phys_args(*p);
    for (const LevelArgs &L : e->levels) {
        if (p->precision == VLBM_FP64) {
            init_macro_kernel<0><<<node_grid(L), 256, 0, e->stream>>>(ph, L, e->coeffs_dev, e->ctl);
            equilibrium_kernel<0><<<node_grid(L), 256, 0, e->stream>>>(ph, L, e->ctl, 0);
        } else {
            init_macro_kernel<1><<<node_grid(L), 256, 0, e->stream>>>(ph, L, e->coeffs_dev, e->ctl);
            equilibrium_kernel<1><<<node_grid(L), 256, 0, e->stream>>>(ph, L, e->ctl, 0);
        }
        hipError_t le = hipGetLastError();
        if (le != hipSuccess) {
            vlbm_destroy(e);
            return fail(VLBM_ERR_HIP, "init launch failed: %s", hipGetErrorString(le));
        }
    }
    // A configuration tuned earlier in this process for the same launch.
    e->level_chunk.assign(e->levels.size(), 0);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(tune_key(e));
        if (it != g_tune_cache.end()) {
            e->level_chunk = it->second.chunks;
            e->waves_per_block = it->second.waves_per_block;
            e->item_order = it->second.item_order;
            e->dealing = it->second.dealing;
        }
    }
    // The host coefficient array may be released once this call returns.
    he = hipStreamSynchronize(e->stream);
    if (he != hipSuccess) {
        vlbm_destroy(e);
        return fail(VLBM_ERR_HIP, "init failed: %s", hipGetErrorString(he));
    }
    *out = e;
    return VLBM_OK;
}

namespace {
// Re-base the control ring so that slot 0 is current (n_launch = 0), with the
// realizations of `level` at the given time, step count and last kinetic speed
// (HOST arrays [R]; NULL = zeros), their status cleared and their wave-speed
// maximum zeroed for the kernel that loads the state to accumulate.  Other
// levels keep their clock and buffers (their step counts are kept).
vlbm_status rebase_ring(vlbm_ensemble *e, int level, const double *t_lvl, const int64_t *steps_lvl,
                        const double *a_lvl)
{
    std::vector<double> t, a;
    std::vector<long long> steps;
    std::vector<int> status;
    vlbm_status rc = read_ctl(e, t, steps, a, status);
    if (rc != VLBM_OK)
        return rc;
    const LevelArgs &L = e->levels[level];
    const int nr = e->ctl.nr, ph = phase_of(e);
    std::vector<unsigned long long> amax(nr, 0ull);
    HIP_TRY(hipMemcpyAsync(amax.data(), e->ctl.amax + (size_t)ph * nr, nr * sizeof(unsigned long long), hipMemcpyDeviceToHost, e->stream));
    HIP_TRY(hipStreamSynchronize(e->stream));
    for (int m = 0; m < L.R; ++m) {
        t[L.ctl_off + m] = t_lvl ? t_lvl[m] : 0.0;
        steps[L.ctl_off + m] = steps_lvl ? (long long)steps_lvl[m] : 0;
        a[L.ctl_off + m] = a_lvl ? a_lvl[m] : 0.0;
        status[L.ctl_off + m] = 0;
        amax[L.ctl_off + m] = 0ull;
    }
    HIP_TRY(hipMemsetAsync(e->ctl_mem, 0, ctl_block_bytes(nr), e->stream));
    HIP_TRY(hipMemcpyAsync(e->ctl.t, t.data(), nr * sizeof(double), hipMemcpyHostToDevice, e->stream));
    HIP_TRY(hipMemcpyAsync(e->ctl.steps, steps.data(), nr * sizeof(long long), hipMemcpyHostToDevice, e->stream));
    HIP_TRY(hipMemcpyAsync(e->ctl.a_last, a.data(), nr * sizeof(double), hipMemcpyHostToDevice, e->stream));
    HIP_TRY(hipMemcpyAsync(e->ctl.amax, amax.data(), nr * sizeof(unsigned long long), hipMemcpyHostToDevice, e->stream));
    HIP_TRY(hipMemcpyAsync(e->ctl.status, status.data(), nr * sizeof(int), hipMemcpyHostToDevice, e->stream));
    e->n_launch = 0;
    return VLBM_OK;
}
} // namespace

vlbm_status vlbm_set_macroscopic(vlbm_ensemble *e, int32_t level, const double *u)
{
    vlbm_status rc = check_level(e, level);
    if (rc != VLBM_OK)
        return rc;
    if (!u)
        return fail(VLBM_ERR_ARG, "u is NULL");
    if ((rc = rebase_ring(e, level, nullptr, nullptr, nullptr)) != VLBM_OK)
        return rc;
    const LevelArgs &L = e->levels[level];
    const PhysArgs ph_args = phys_args(e->p);
    if (e->p.precision == VLBM_FP64) {
        set_macro_kernel<0><<<node_grid(L), 256, 0, e->stream>>>(ph_args, L, e->ctl, u);
        equilibrium_kernel<0><<<node_grid(L), 256, 0, e->stream>>>(ph_args, L, e->ctl, 0);
    } else {
        set_macro_kernel<1><<<node_grid(L), 256, 0, e->stream>>>(ph_args, L, e->ctl, u);
        equilibrium_kernel<1><<<node_grid(L), 256, 0, e->stream>>>(ph_args, L, e->ctl, 0);
    }
    LAUNCH_CHECK("set_macroscopic");
    HIP_TRY(hipStreamSynchronize(e->stream));
    return VLBM_OK;
}

vlbm_status vlbm_set_state(vlbm_ensemble *e, int32_t level, const double *state, const double *t,
                           const int64_t *steps, const double *a_last)
{
    vlbm_status rc = check_level(e, level);
    if (rc != VLBM_OK)
        return rc;
    if (!state || !t || !steps)
        return fail(VLBM_ERR_ARG, "state, t and steps must be non-NULL");
    const LevelArgs &L = e->levels[level];
    for (int m = 0; m < L.R; ++m) {
        if (!std::isfinite(t[m]) || t[m] < 0.0 || steps[m] < 0)
            return fail(VLBM_ERR_ARG, "realization %d: t must be finite and >= 0, steps >= 0", m);
        if (a_last && !(a_last[m] >= 0.0 && std::isfinite(a_last[m])))
            return fail(VLBM_ERR_ARG, "realization %d: a_last must be finite and >= 0", m);
    }
    if ((rc = rebase_ring(e, level, t, steps, a_last)) != VLBM_OK)
        return rc;
    const PhysArgs ph_args = phys_args(e->p);
    if (e->p.precision == VLBM_FP64)
        set_state_kernel<0><<<node_grid(L), 256, 0, e->stream>>>(ph_args, L, e->ctl, state);
    else
        set_state_kernel<1><<<node_grid(L), 256, 0, e->stream>>>(ph_args, L, e->ctl, state);
    LAUNCH_CHECK("set_state");
    HIP_TRY(hipStreamSynchronize(e->stream));
    return VLBM_OK;
}

namespace {
void drop_graph(vlbm_ensemble *e)
{
    if (e->graph) {
        (void)hipGraphExecDestroy(e->graph);
        e->graph = nullptr;
    }
}

// Capture GRAPH_STEPS steps (phases 0..GRAPH_STEPS-1 mod 3) into e->graph.
vlbm_status capture_graph(vlbm_ensemble *e, double t_final)
{
    drop_graph(e);
    if (!e->cap_stream)
        HIP_TRY(hipStreamCreateWithFlags(&e->cap_stream, hipStreamNonBlocking));
    const PhysArgs ph = phys_args(e->p);
    HIP_TRY(hipStreamBeginCapture(e->cap_stream, hipStreamCaptureModeThreadLocal));
    vlbm_status rc = VLBM_OK;
    for (int s = 0; s < GRAPH_STEPS && rc == VLBM_OK; ++s)
        rc = launch_step(e, ph, 0, (int)e->levels.size(), s % 3, t_final, e->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t he = hipStreamEndCapture(e->cap_stream, &g);
    if (rc != VLBM_OK) {
        if (g)
            (void)hipGraphDestroy(g);
        return rc;
    }
    if (he != hipSuccess)
        return fail(VLBM_ERR_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(he));
    he = hipGraphInstantiate(&e->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (he != hipSuccess) {
        e->graph = nullptr;
        return fail(VLBM_ERR_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(he));
    }
    e->graph_t_final = t_final;
    return VLBM_OK;
}
} // namespace

vlbm_status vlbm_step(vlbm_ensemble *e, double t_final, int32_t n_steps, int32_t *all_done)
{
    if (!e)
        return fail(VLBM_ERR_ARG, "ensemble is NULL");
    if (!std::isfinite(t_final))
        return fail(VLBM_ERR_ARG, "t_final must be finite");
    if (n_steps < 0)
        return fail(VLBM_ERR_ARG, "n_steps must be >= 0");
    const PhysArgs ph = phys_args(e->p);
    int left = n_steps;
    auto eager = [&](int n) -> vlbm_status {
        for (int s = 0; s < n; ++s) {
            vlbm_status rc = launch_step(e, ph, 0, (int)e->levels.size(), phase_of(e), t_final, e->stream);
            if (rc != VLBM_OK)
                return rc;
            e->n_launch++;
        }
        return VLBM_OK;
    };
    if (e->use_graph && left >= GRAPH_STEPS + 2) {
        // align the ring phase to 0, then replay whole graphs
        const int lead = (int)((3 - e->n_launch % 3) % 3);
        vlbm_status rc = eager(lead);
        if (rc != VLBM_OK)
            return rc;
        left -= lead;
        if (!e->graph || e->graph_t_final != t_final) {
            rc = capture_graph(e, t_final);
            if (rc != VLBM_OK)
                return rc;
        }
        while (left >= GRAPH_STEPS) {
            HIP_TRY(hipGraphLaunch(e->graph, e->stream));
            e->n_launch += GRAPH_STEPS;
            left -= GRAPH_STEPS;
        }
    }
    {
        vlbm_status rc = eager(left);
        if (rc != VLBM_OK)
            return rc;
    }
    if (all_done) {
        std::vector<double> t, a;
        std::vector<long long> steps;
        std::vector<int> status;
        vlbm_status rc = read_ctl(e, t, steps, a, status);
        if (rc != VLBM_OK)
            return rc;
        int done = 1;
        for (int k = 0; k < e->ctl.nr; ++k) {
            if (status[k] & STATUS_NONFINITE)
                return fail(VLBM_ERR_NONFINITE, "realization %d of level %d produced a non-finite value",
                            k % e->n_real, k / e->n_real);
            if (status[k] & STATUS_NONPOSITIVE)
                return fail(VLBM_ERR_NONPOSITIVE, "realization %d of level %d produced rho <= 0 or p <= 0",
                            k % e->n_real, k / e->n_real);
            if (!(t[k] >= t_final))
                done = 0;
        }
        *all_done = done;
    }
    return VLBM_OK;
}

vlbm_status vlbm_times(const vlbm_ensemble *e, int32_t level, double *t_out, int64_t *steps_out,
                       double *a_out, int32_t *status_out)
{
    vlbm_status rc = check_level(e, level);
    if (rc != VLBM_OK)
        return rc;
    std::vector<double> t, a;
    std::vector<long long> steps;
    std::vector<int> status;
    if ((rc = read_ctl(e, t, steps, a, status)) != VLBM_OK)
        return rc;
    const LevelArgs &L = e->levels[level];
    for (int m = 0; m < L.R; ++m) {
        const int k = L.ctl_off + m;
        if (t_out)
            t_out[m] = t[k];
        if (steps_out)
            steps_out[m] = steps[k];
        if (a_out)
            a_out[m] = a[k];
        if (status_out)
            status_out[m] = (status[k] & STATUS_NONFINITE) ? VLBM_ERR_NONFINITE
                            : (status[k] & STATUS_NONPOSITIVE) ? VLBM_ERR_NONPOSITIVE : VLBM_OK;
    }
    return VLBM_OK;
}

vlbm_status vlbm_get_state(const vlbm_ensemble *e, int32_t level, double *out)
{
    vlbm_status rc = check_level(e, level);
    if (rc != VLBM_OK)
        return rc;
    if (!out)
        return fail(VLBM_ERR_ARG, "out is NULL");
    const LevelArgs &L = e->levels[level];
    if (e->p.precision == VLBM_FP64)
        get_state_kernel<0><<<node_grid(L), 256, 0, e->stream>>>(L, e->ctl, phase_of(e), out);
    else
        get_state_kernel<1><<<node_grid(L), 256, 0, e->stream>>>(L, e->ctl, phase_of(e), out);
    LAUNCH_CHECK("get_state");
    return VLBM_OK;
}

vlbm_status vlbm_moments(const vlbm_ensemble *e, int32_t level, double *rho, double *speed, double *p)
{
    vlbm_status rc = check_level(e, level);
    if (rc != VLBM_OK)
        return rc;
    if (!rho && !speed && !p)
        return VLBM_OK;
    const LevelArgs &L = e->levels[level];
    const PhysArgs ph = phys_args(e->p);
    if (e->p.precision == VLBM_FP64)
        moments_kernel<0><<<node_grid(L), 256, 0, e->stream>>>(ph, L, e->ctl, phase_of(e), rho, speed, p);
    else
        moments_kernel<1><<<node_grid(L), 256, 0, e->stream>>>(ph, L, e->ctl, phase_of(e), rho, speed, p);
    LAUNCH_CHECK("moments");
    return VLBM_OK;
}

vlbm_status vlbm_ensemble_stats(const vlbm_ensemble *e, int32_t level, int32_t r, double *acc, int64_t acc_cells,
                                int64_t n_prev, double *samples, int64_t sample_rows, int64_t m_offset)
{
    vlbm_status rc = check_level(e, level);
    if (rc != VLBM_OK)
        return rc;
    const LevelArgs &L = e->levels[level];
    if (r < 1 || L.nx % r || L.ny % r)
        return fail(VLBM_ERR_ARG, "restriction factor %d must divide %d x %d", r, L.nx, L.ny);
    const long long ncell = (long long)(L.nx / r) * (L.ny / r);
    if (!acc)
        return fail(VLBM_ERR_ARG, "acc is NULL");
    if (acc_cells != ncell)
        return fail(VLBM_ERR_SIZE, "acc holds %lld cells per field, the %d x %d level restricted by %d has %lld",
                    (long long)acc_cells, L.nx, L.ny, r, ncell);
    if (n_prev < 0 || m_offset < 0)
        return fail(VLBM_ERR_ARG, "n_prev and m_offset must be >= 0");
    if (samples && m_offset + L.R > sample_rows)
        return fail(VLBM_ERR_SIZE, "sample store of %lld rows cannot take rows %lld .. %lld",
                    (long long)sample_rows, (long long)m_offset, (long long)(m_offset + L.R - 1));
    const PhysArgs ph = phys_args(e->p);
    const dim3 grid((unsigned)((ncell + 255) / 256));
    if (e->p.precision == VLBM_FP64)
        stats_accumulate_kernel<0><<<grid, 256, 0, e->stream>>>(ph, L, e->ctl, phase_of(e), r, acc, n_prev, samples, m_offset);
    else
        stats_accumulate_kernel<1><<<grid, 256, 0, e->stream>>>(ph, L, e->ctl, phase_of(e), r, acc, n_prev, samples, m_offset);
    LAUNCH_CHECK("ensemble_stats");
    return VLBM_OK;
}

vlbm_status vlbm_stats_finalize(const double *acc, int64_t n_cells, int64_t n_total, double *mean,
                                double *std_out, void *hip_stream)
{
    if (!acc)
        return fail(VLBM_ERR_ARG, "acc is NULL");
    if (n_cells < 1 || n_total < 1)
        return fail(VLBM_ERR_ARG, "n_cells and n_total must be >= 1");
    if (!mean && !std_out)
        return VLBM_OK;
    stats_finalize_kernel<<<(unsigned)((n_cells + 255) / 256), 256, 0, (hipStream_t)hip_stream>>>(
        acc, n_cells, n_total, mean, std_out);
    LAUNCH_CHECK("stats_finalize");
    return VLBM_OK;
}

vlbm_status vlbm_sort_samples(double *samples, int64_t n_cells, int32_t m, void *hip_stream)
{
    if (!samples)
        return fail(VLBM_ERR_ARG, "samples is NULL");
    if (n_cells < 1 || m < 1 || m > 4096)
        return fail(VLBM_ERR_SIZE, "need n_cells >= 1 and 1 <= m <= 4096 (got %lld, %d)", (long long)n_cells, m);
    int mp = 1;
    while (mp < m)
        mp <<= 1;
    if (mp < 2)
        mp = 2;
    hipStream_t st = (hipStream_t)hip_stream;
    if (mp <= 256) {
        sort_samples_kernel<16><<<(unsigned)((n_cells + 15) / 16), 256, 16 * mp * sizeof(double), st>>>(samples, n_cells, m, mp);
    } else if (mp <= 1024) {
        sort_samples_kernel<4><<<(unsigned)((n_cells + 3) / 4), 256, 4 * mp * sizeof(double), st>>>(samples, n_cells, m, mp);
    } else {
        sort_samples_kernel<1><<<(unsigned)n_cells, 256, mp * sizeof(double), st>>>(samples, n_cells, m, mp);
    }
    LAUNCH_CHECK("sort_samples");
    return VLBM_OK;
}

namespace {
// Stage-1 partial sums of a two-stage reduction: stream-ordered device memory,
// released on the same stream once the reduction has consumed it.
struct StreamScratch {
    double *p = nullptr;
    hipStream_t st = nullptr;
    ~StreamScratch()
    {
        if (p)
            (void)hipFreeAsync(p, st);
    }
};

vlbm_status check_w1_args(const double *a, const double *b, int64_t n_cells, int32_t m)
{
    if (!a || !b)
        return fail(VLBM_ERR_ARG, "sample stores must be non-NULL");
    if (n_cells < 1 || m < 1)
        return fail(VLBM_ERR_SIZE, "need n_cells >= 1 and m >= 1 (got %lld, %d)", (long long)n_cells, m);
    return VLBM_OK;
}
} // namespace

vlbm_status vlbm_w1(const double *a, const double *b, int64_t n_cells, int32_t m, double *w1_cell,
                    double *w1_mean, void *hip_stream)
{
    vlbm_status rc = check_w1_args(a, b, n_cells, m);
    if (rc != VLBM_OK)
        return rc;
    if (!w1_cell && !w1_mean)
        return VLBM_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    StreamScratch ws;
    ws.st = st;
    if (w1_mean)
        HIP_TRY(hipMallocAsync((void **)&ws.p, (size_t)reduction_partials(n_cells) * sizeof(double), st));
    launch_w1(a, b, n_cells, m, w1_cell, w1_mean, ws.p, st);
    LAUNCH_CHECK("w1");
    return VLBM_OK;
}

} // extern "C"

// Workspace of vlbm_w1_noalloc: the stage-1 partial sums of the W_{1,1}
// average, in a file-scope device array (one copy per device, held until the
// process ends).  Host code never passes the array's name to a kernel: its
// device address is looked up once per device and kept in g_noalloc_ptr.
static __device__ __align__(256) double scratch[VLBM_W1_NOALLOC_MAX_PARTIALS];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
double *g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};
std::mutex g_noalloc_mu;

// Device address of the current device's copy of the workspace (looked up on
// the first call made with that device current).
vlbm_status noalloc_scratch(double **out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(VLBM_ERR_ARG, "device ordinal %d outside [0, %d)", dev, NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t he = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (he != hipSuccess || !ptr)
            return fail(VLBM_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev,
                        hipGetErrorString(he));
        g_noalloc_ptr[dev] = (double *)ptr;
    }
    *out = g_noalloc_ptr[dev];
    return VLBM_OK;
}
} // namespace

extern "C" {

vlbm_status vlbm_w1_noalloc(const double *a, const double *b, int64_t n_cells, int32_t m, double *w1_cell,
                            double *w1_mean, void *hip_stream)
{
    vlbm_status rc = check_w1_args(a, b, n_cells, m);
    if (rc != VLBM_OK)
        return rc;
    if (w1_mean && reduction_partials(n_cells) > VLBM_W1_NOALLOC_MAX_PARTIALS)
        return fail(VLBM_ERR_SIZE, "vlbm_w1_noalloc: n_cells = %lld needs %lld partial sums, the fixed "
                    "workspace holds %d (at most %lld cells with w1_mean)", (long long)n_cells,
                    reduction_partials(n_cells), VLBM_W1_NOALLOC_MAX_PARTIALS,
                    (long long)VLBM_W1_NOALLOC_MAX_PARTIALS * 1024LL);
    if (!w1_cell && !w1_mean)
        return VLBM_OK;
    double *ws = nullptr;
    if (w1_mean) {
        rc = noalloc_scratch(&ws);
        if (rc != VLBM_OK)
            return rc;
    }
    // every partial the second stage reads is written by the first, so the
    // workspace needs no clearing between calls
    launch_w1(a, b, n_cells, m, w1_cell, w1_mean, ws, (hipStream_t)hip_stream);
    LAUNCH_CHECK("w1_noalloc");
    return VLBM_OK;
}

vlbm_status vlbm_strong_error(const double *a, const double *b, int64_t n_cells, int32_t m, double *per_real,
                              double *out, void *hip_stream)
{
    if (!a || !b || !per_real || !out)
        return fail(VLBM_ERR_ARG, "a, b, per_real and out must be non-NULL");
    if (n_cells < 1 || m < 1 || m > 1 << 24)
        return fail(VLBM_ERR_SIZE, "need n_cells >= 1 and 1 <= m <= 2^24");
    launch_strong_error(a, b, n_cells, m, per_real, out, (hipStream_t)hip_stream);
    LAUNCH_CHECK("strong_error");
    return VLBM_OK;
}

vlbm_status vlbm_mean_abs_diff(const double *x, const double *y, int64_t n, double *out, void *hip_stream)
{
    if (!x || !out)
        return fail(VLBM_ERR_ARG, "x and out must be non-NULL");
    if (n < 1)
        return fail(VLBM_ERR_SIZE, "need n >= 1");
    hipStream_t st = (hipStream_t)hip_stream;
    StreamScratch ws;
    ws.st = st;
    HIP_TRY(hipMallocAsync((void **)&ws.p, (size_t)reduction_partials(n) * sizeof(double), st));
    launch_mean_abs_diff(x, y, n, out, ws.p, st);
    LAUNCH_CHECK("mean_abs_diff");
    return VLBM_OK;
}

vlbm_status vlbm_quantiles(const double *sorted, int64_t n_cells, int32_t m, const int32_t *pct, int32_t n_q,
                           double *out, void *hip_stream)
{
    if (!sorted || !pct || !out)
        return fail(VLBM_ERR_ARG, "sorted, pct and out must be non-NULL");
    if (n_cells < 1 || m < 1)
        return fail(VLBM_ERR_SIZE, "need n_cells >= 1 and m >= 1");
    if (n_q < 1 || n_q > VLBM_MAX_QUANTILES)
        return fail(VLBM_ERR_ARG, "n_q must lie in [1, %d] (got %d)", VLBM_MAX_QUANTILES, n_q);
    for (int q = 0; q < n_q; ++q)
        if (pct[q] < 1 || pct[q] > 100)
            return fail(VLBM_ERR_ARG, "pct[%d] = %d outside [1, 100]", q, pct[q]);
    launch_quantiles(sorted, n_cells, m, pct, n_q, out, (hipStream_t)hip_stream);
    LAUNCH_CHECK("quantiles");
    return VLBM_OK;
}

vlbm_status vlbm_width_ratio(const double *sorted, int64_t n_cells, int32_t m, double *q, void *hip_stream)
{
    if (!sorted || !q)
        return fail(VLBM_ERR_ARG, "sorted and q must be non-NULL");
    if (n_cells < 1 || m < 1)
        return fail(VLBM_ERR_SIZE, "need n_cells >= 1 and m >= 1");
    launch_width_ratio(sorted, n_cells, m, q, (hipStream_t)hip_stream);
    LAUNCH_CHECK("width_ratio");
    return VLBM_OK;
}

vlbm_status vlbm_w12(const double *a, const double *b, int32_t ncx, int32_t ncy, int32_t m, int32_t n_pd,
                     double *w_pair, double *w_mean, void *hip_stream)
{
    if (!a || !b || !w_pair)
        return fail(VLBM_ERR_ARG, "a, b and w_pair must be non-NULL");
    if (ncx < 1 || ncy < 1 || m < 1 || m > VLBM_W12_MAX_SAMPLES)
        return fail(VLBM_ERR_SIZE, "need ncx, ncy >= 1 and 1 <= m <= %d (got %d x %d, m = %d)",
                    VLBM_W12_MAX_SAMPLES, ncx, ncy, m);
    if (n_pd < 1 || n_pd > ncx || n_pd > ncy || n_pd > 200)
        return fail(VLBM_ERR_ARG, "n_pd must lie in [1, min(ncx, ncy, 200)] (got %d)", n_pd);
    launch_w12(a, b, ncx, ncy, m, n_pd, w_pair, w_mean, (hipStream_t)hip_stream);
    LAUNCH_CHECK("w12");
    return VLBM_OK;
}

vlbm_status vlbm_rate_fit(const double *errors, const double *dx, int32_t n, double *rate, double *intercept)
{
    if (!errors || !dx || !rate)
        return fail(VLBM_ERR_ARG, "errors, dx and rate must be non-NULL");
    if (n < 2)
        return fail(VLBM_ERR_SIZE, "need at least two points (got %d)", n);
    double sx = 0.0, sy = 0.0;
    for (int i = 0; i < n; ++i) {
        if (!(errors[i] > 0.0) || !(dx[i] > 0.0) || !std::isfinite(errors[i]) || !std::isfinite(dx[i]))
            return fail(VLBM_ERR_ARG, "errors and mesh widths must be finite and > 0 (point %d)", i);
        sx += std::log(dx[i]);
        sy += std::log(errors[i]);
    }
    const double mx = sx / n, my = sy / n;
    double sxx = 0.0, sxy = 0.0;
    for (int i = 0; i < n; ++i) {
        const double u = std::log(dx[i]) - mx;
        sxx += u * u;
        sxy += u * (std::log(errors[i]) - my);
    }
    if (!(sxx > 0.0))
        return fail(VLBM_ERR_ARG, "the mesh widths must not all be equal");
    *rate = sxy / sxx;
    if (intercept)
        *intercept = my - *rate * mx;
    return VLBM_OK;
}

vlbm_status vlbm_tune(vlbm_ensemble *e, int32_t kernel, int32_t chunk_rows)
{
    if (!e)
        return fail(VLBM_ERR_ARG, "ensemble is NULL");
    const bool no_graph = (kernel & VLBM_KERNEL_NO_GRAPH) != 0;
    kernel &= ~VLBM_KERNEL_NO_GRAPH;
    if (kernel != VLBM_KERNEL_REFERENCE && kernel != VLBM_KERNEL_MARCH)
        return fail(VLBM_ERR_ARG, "unknown kernel %d", kernel);
    if (chunk_rows != 0 && (chunk_rows < 4 || chunk_rows > 65536))
        return fail(VLBM_ERR_ARG, "chunk_rows must be 0 or lie in [4, 65536] (got %d)", chunk_rows);
    e->kernel = kernel;
    e->chunk_rows = chunk_rows;
    e->use_graph = !no_graph;
    std::fill(e->level_chunk.begin(), e->level_chunk.end(), 0);
    e->waves_per_block = 4;
    e->item_order = 0;
    e->dealing = 1;
    drop_graph(e);
    return VLBM_OK;
}

vlbm_status vlbm_set_tuning(vlbm_ensemble *e, const int32_t *chunks, int32_t waves_per_block, int32_t item_order,
                            int32_t dealing)
{
    if (!e)
        return fail(VLBM_ERR_ARG, "ensemble is NULL");
    if (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4)
        return fail(VLBM_ERR_ARG, "waves_per_block must be 1, 2 or 4 (got %d)", waves_per_block);
    if (item_order != 0 && item_order != 1)
        return fail(VLBM_ERR_ARG, "item_order must be 0 or 1 (got %d)", item_order);
    if (dealing != 0 && dealing != 1)
        return fail(VLBM_ERR_ARG, "dealing must be 0 or 1 (got %d)", dealing);
    if (chunks)
        for (size_t l = 0; l < e->levels.size(); ++l)
            if (chunks[l] != 0 && (chunks[l] < 4 || chunks[l] > 65536))
                return fail(VLBM_ERR_ARG, "chunks[%zu] must be 0 or lie in [4, 65536] (got %d)", l, chunks[l]);
    for (size_t l = 0; l < e->levels.size(); ++l)
        e->level_chunk[l] = chunks ? chunks[l] : 0;
    e->waves_per_block = waves_per_block;
    e->item_order = item_order;
    e->dealing = dealing;
    drop_graph(e);
    return VLBM_OK;
}

vlbm_status vlbm_get_tuning(const vlbm_ensemble *e, int32_t *chunks, int32_t *waves_per_block, int32_t *item_order,
                            int32_t *dealing)
{
    if (!e)
        return fail(VLBM_ERR_ARG, "ensemble is NULL");
    if (chunks)
        for (size_t l = 0; l < e->levels.size(); ++l)
            chunks[l] = march_args(e, (int)l).chunk;
    if (waves_per_block)
        *waves_per_block = e->waves_per_block;
    if (item_order)
        *item_order = e->item_order;
    if (dealing)
        *dealing = e->dealing;
    return VLBM_OK;
}

namespace {
// Work models of one launch: every work item costs its rows plus the 4-row
// prologue of the march.  Static round-robin dealing: item i goes to wave
// i mod W and the launch lasts as long as the most loaded wave.  Work queues:
// the work spreads evenly and the launch lasts the average load plus at most one
// item (the last ones handed out).
double dealing_model(const vlbm_ensemble *e, const std::vector<int> &chunks, int dealing)
{
    const long long W = resident_waves(e);
    std::vector<double> load((size_t)W, 0.0);
    long long i = 0;
    for (size_t l = 0; l < e->levels.size(); ++l) {
        const LevelArgs &L = e->levels[l];
        int lane62 = 0;
        const int nstrip = strips_of(e, L, &lane62);
        const int chunk = std::min(chunks[l], L.ny);
        const int nchunk = (L.ny + chunk - 1) / chunk;
        const long long per_real = (long long)nstrip * nchunk;
        const long long n = (long long)L.R * per_real;
        for (long long k = 0; k < n; ++k, ++i) {
            const long long rem = e->item_order == 0 ? k % per_real : k / L.R;
            const int ch = (int)(rem / nstrip);
            const int rows = std::min(chunk, L.ny - ch * chunk);
            load[(size_t)(i % W)] += rows + 4;
        }
    }
    if (dealing == 0)
        return *std::max_element(load.begin(), load.end());
    double total = 0.0;
    for (double x : load)
        total += x;
    int longest = 0;
    for (size_t l = 0; l < e->levels.size(); ++l)
        longest = std::max(longest, std::min(chunks[l], e->levels[l].ny));
    return total / (double)W + longest + 4;
}

// Candidate chunk tuples: for every common target height h (the distinct heights
// ny_l / n of all levels), each level takes the height of its even split closest
// above h; tuples are ranked by the dealing model and the best `keep` returned.
std::vector<std::vector<int>> chunk_candidates(const vlbm_ensemble *e, size_t keep, int dealing)
{
    std::vector<int> targets;
    if (dealing == 1) {
        // work queues: the model cannot see how short items keep neighbouring
        // strips in step, so a ladder of common heights is timed instead
        for (int h : {32, 48, 64, 96, 128, 192, 256, 384})
            targets.push_back(h);
        keep = std::max(keep, targets.size());
    } else {
        for (const LevelArgs &L : e->levels)
            for (int n = 1; n <= std::min(L.ny, 256); ++n) {
                const int h = std::max(4, (L.ny + n - 1) / n);
                if (std::find(targets.begin(), targets.end(), h) == targets.end())
                    targets.push_back(h);
            }
    }
    std::vector<std::pair<double, std::vector<int>>> ranked;
    for (int h : targets) {
        std::vector<int> t;
        for (const LevelArgs &L : e->levels) {
            const int n = std::max(1, L.ny / h);
            t.push_back(std::min(L.ny, std::max(4, (L.ny + n - 1) / n)));
        }
        bool seen = false;
        for (auto &r : ranked)
            seen = seen || r.second == t;
        if (!seen)
            ranked.push_back({dealing_model(e, t, dealing), t});
    }
    std::stable_sort(ranked.begin(), ranked.end(),
                     [](const std::pair<double, std::vector<int>> &a, const std::pair<double, std::vector<int>> &b) {
                         return a.first < b.first;
                     });
    std::vector<std::vector<int>> out;
    for (size_t k = 0; k < ranked.size() && out.size() < keep; ++k)
        out.push_back(ranked[k].second);
    return out;
}
} // namespace

vlbm_status vlbm_autotune(vlbm_ensemble *e, double t_final, int32_t steps_per_candidate, int32_t *chunks_out)
{
    if (!e)
        return fail(VLBM_ERR_ARG, "ensemble is NULL");
    if (!std::isfinite(t_final))
        return fail(VLBM_ERR_ARG, "t_final must be finite");
    if (steps_per_candidate < 1 || steps_per_candidate > 1000)
        return fail(VLBM_ERR_ARG, "steps_per_candidate must lie in [1, 1000]");
    const int nlev = (int)e->levels.size();
    auto report = [&]() {
        if (chunks_out)
            for (int l = 0; l < nlev; ++l)
                chunks_out[l] = e->kernel == VLBM_KERNEL_MARCH ? march_args(e, l).chunk : 0;
    };
    if (e->kernel != VLBM_KERNEL_MARCH) {
        report();
        return VLBM_OK;
    }
    drop_graph(e);
    // A configuration is (chunk height per level, waves per block, item order,
    // dealing), timed on steps_per_candidate live steps of the whole launch (all
    // levels, as vlbm_step runs them).  Search: chunk tuples under the work
    // queues and under the static dealing, each ranked by its model, then the
    // block size and the item order around the fastest.
    std::vector<int> dflt(nlev);
    e->waves_per_block = 4;
    e->item_order = 0;
    e->dealing = 1;
    for (int l = 0; l < nlev; ++l) {
        int lane62 = 0;
        dflt[l] = model_chunk(e, e->levels[l], strips_of(e, e->levels[l], &lane62));
    }
    std::vector<std::vector<int>> dyn_tuples = chunk_candidates(e, 5, 1);
    if (std::find(dyn_tuples.begin(), dyn_tuples.end(), dflt) == dyn_tuples.end())
        dyn_tuples.push_back(dflt);
    const std::vector<std::vector<int>> static_tuples = chunk_candidates(e, 2, 0);

    hipEvent_t ev[2];
    HIP_TRY(hipEventCreate(&ev[0]));
    HIP_TRY(hipEventCreate(&ev[1]));
    const PhysArgs ph = phys_args(e->p);
    vlbm_status rc = VLBM_OK;
    bool all_done = false;
    // time the current configuration: average launch time, or < 0 if the
    // ensemble finished (or failed) before it could be timed
    auto time_config = [&]() -> double {
        if (all_done || rc != VLBM_OK)
            return -1.0;
        if (hipEventRecord(ev[0], e->stream) != hipSuccess) {
            rc = fail(VLBM_ERR_HIP, "hipEventRecord failed");
            return -1.0;
        }
        for (int s = 0; s < steps_per_candidate && rc == VLBM_OK; ++s) {
            rc = launch_step(e, ph, 0, nlev, phase_of(e), t_final, e->stream);
            if (rc == VLBM_OK)
                e->n_launch++;
        }
        if (rc != VLBM_OK)
            return -1.0;
        if (hipEventRecord(ev[1], e->stream) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess) {
            rc = fail(VLBM_ERR_HIP, "event synchronisation failed");
            return -1.0;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
        std::vector<double> t, a;
        std::vector<long long> st;
        std::vector<int> status;
        if ((rc = read_ctl(e, t, st, a, status)) != VLBM_OK)
            return -1.0;
        bool done = true;
        for (double x : t)
            done = done && x >= t_final;
        if (done) { // the last launches may have had nothing left to do
            all_done = true;
            return -1.0;
        }
        return (double)ms / steps_per_candidate;
    };
    TuneChoice best;
    best.chunks = dflt;
    best.dealing = 1;
    double best_ms = 1e300;
    auto consider = [&](const std::vector<int> &chunks, int wpb, int order, int dealing) {
        e->level_chunk = chunks;
        e->waves_per_block = wpb;
        e->item_order = order;
        e->dealing = dealing;
        const double ms = time_config();
        if (ms > 0.0 && ms < best_ms) {
            best_ms = ms;
            best.chunks = chunks;
            best.waves_per_block = wpb;
            best.item_order = order;
            best.dealing = dealing;
        }
    };
    for (const auto &t : dyn_tuples)
        consider(t, 4, 0, 1);
    for (const auto &t : static_tuples)
        consider(t, 4, 0, 0);
    const std::vector<int> best_chunks = best.chunks;
    const int best_dealing = best.dealing;
    consider(best_chunks, 2, 0, best_dealing);
    consider(best_chunks, 1, 0, best_dealing);
    consider(best_chunks, best.waves_per_block, 1, best_dealing);
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    e->level_chunk = best.chunks;
    e->waves_per_block = best.waves_per_block;
    e->item_order = best.item_order;
    e->dealing = best.dealing;
    if (rc != VLBM_OK)
        return rc;
    if (best_ms < 1e300) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[tune_key(e)] = best;
    }
    report();
    return VLBM_OK;
}

vlbm_status vlbm_destroy(vlbm_ensemble *e)
{
    if (!e)
        return VLBM_OK;
    (void)hipStreamSynchronize(e->stream);
    drop_graph(e);
    if (e->cap_stream)
        (void)hipStreamDestroy(e->cap_stream);
    if (e->ctl_mem)
        (void)hipFree(e->ctl_mem);
    if (e->coeffs_dev)
        (void)hipFree(e->coeffs_dev);
    delete e;
    return VLBM_OK;
}

} // extern "C"
