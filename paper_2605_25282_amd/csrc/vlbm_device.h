// vlbm_device.h -- device-side building blocks of the VLBM ensemble library
// (gfx950).  Internal header of the HIP library; not part of the public ABI.
//
// Floating-point contract: this library is compiled with -ffp-contract=off and
// without fast-math, and every expression below is written so that its
// operation order is fixed.  The blended update with the limiter amplifies a
// one-ulp difference by roughly 1.5 per step at Mach 2000 (Sec. 2.2 setup), so
// the FP64 path is written to be bitwise reproducible: correctly rounded
// division and square root, correctly rounded cos/sin for the inlet profile,
// no reassociation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vlbm {

// ---------------------------------------------------------------------------
// Scheme parameters resolved for one time step.
// ---------------------------------------------------------------------------
struct Phys {
    double gamma;      // heat-capacity ratio (eq:eos)
    double alpha;      // rest-population weight (eq:maxwellians5)
    double w;          // (1 - alpha) / 4, weight of M_1..M_4
    double h;          // 1 / (2 a), a = kinetic speed of the step
    double rlmp_relax; // relaxation of the local density bounds
    double pos_eps;    // internal-energy floor (fraction of the low-order value)
    double inv_w;      // 1 / w
    bool w_pow2;       // w is a power of two: x / w == x * inv_w exactly
};

// ---------------------------------------------------------------------------
// Pointwise physics (eq:eos, eq:fluxF, eq:fluxG, eq:maxwellians12-34)
// ---------------------------------------------------------------------------

// D2Q5 Maxwellians M_1..M_4 of the state u: M[k][v], k = 0..3.
__device__ __forceinline__ void maxwellians(const Phys &P, const double u[4], double M[4][4])
{
    const double rho = u[0], m1 = u[1], m2 = u[2], E = u[3];
    const double v1 = m1 / rho;
    const double v2 = m2 / rho;
    const double p = (P.gamma - 1.0) * (E - 0.5 * rho * (v1 * v1 + v2 * v2));
    const double f[4] = {m1, m1 * v1 + p, m1 * v2, (E + p) * v1};
    const double g[4] = {m2, m2 * v1, m2 * v2 + p, (E + p) * v2};
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const double wu = P.w * u[v];
        M[0][v] = wu + P.h * f[v];
        M[1][v] = wu - P.h * f[v];
        M[2][v] = wu + P.h * g[v];
        M[3][v] = wu - P.h * g[v];
    }
}

// Largest characteristic speed max(|v1|,|v2|) + c of the state u; *bad is set
// when rho <= 0, p <= 0 or a value is not finite.
// (Written without branches: every lane evaluates the same instructions.)
__device__ __forceinline__ double wave_speed(double gamma, const double u[4], int *bad)
{
    const double rho = u[0];
    const double v1 = u[1] / rho;
    const double v2 = u[2] / rho;
    const double p = (gamma - 1.0) * (u[3] - 0.5 * rho * (v1 * v1 + v2 * v2));
    const bool ok = rho > 0.0 && p > 0.0 && isfinite(rho) && isfinite(p);
    const double c = sqrt(gamma * p / rho);
    *bad |= ok ? 0 : 1;
    return ok ? fmax(fabs(v1), fabs(v2)) + c : 0.0;
}

// Relaxed local density bounds and low-order internal energy of a cell whose
// low-order state is L, from the densities of its four bar states M_k/w
// (M1w = M_1 of the west neighbour, ...) and, if alpha > 0, its own density.
__device__ __forceinline__ void cell_bounds(const Phys &P, const double L[4], double m1w_rho,
                                            double m2e_rho, double m3s_rho, double m4n_rho,
                                            double rho_c, double *rmin_out, double *rmax_out,
                                            double *rhoe_out)
{
    // Division by w > 0 is monotone, so the largest (smallest) bar density
    // max_k M_k/w equals (max_k M_k)/w bit for bit: two divisions, not four.
    // When w is a power of two (alpha = 0: w = 1/4) the division is an exact
    // scaling and the product with 1/w is the same number.
    const double mx = fmax(fmax(m1w_rho, m2e_rho), fmax(m3s_rho, m4n_rho));
    const double mn = fmin(fmin(m1w_rho, m2e_rho), fmin(m3s_rho, m4n_rho));
    double rmax, rmin;
    if (P.w_pow2) {
        rmax = mx * P.inv_w;
        rmin = mn * P.inv_w;
    } else {
        rmax = mx / P.w;
        rmin = mn / P.w;
    }
    if (P.alpha > 0.0) {
        rmax = fmax(rmax, rho_c);
        rmin = fmin(rmin, rho_c);
    }
    const double delta = P.rlmp_relax * (rmax - rmin);
    *rmax_out = rmax + delta;
    *rmin_out = fmax(rmin - delta, 0.5 * rmin);
    *rhoe_out = L[3] - 0.5 * (L[1] * L[1] + L[2] * L[2]) / L[0];
}

// Maxwellian M_4 alone (the only one a node contributes to the low-order
// state of the node below it), same operation order as maxwellians().
__device__ __forceinline__ void maxwellian4(const Phys &P, const double u[4], double M4[4])
{
    const double rho = u[0], m1 = u[1], m2 = u[2], E = u[3];
    const double v1 = m1 / rho;
    const double v2 = m2 / rho;
    const double p = (P.gamma - 1.0) * (E - 0.5 * rho * (v1 * v1 + v2 * v2));
    const double g[4] = {m2, m2 * v1, m2 * v2 + p, (E + p) * v2};
#pragma unroll
    for (int v = 0; v < 4; ++v)
        M4[v] = P.w * u[v] - P.h * g[v];
}

// Largest theta in [0,1] keeping L + theta*D inside [rmin, rmax] in density and
// above pos_eps * rhoeL in internal energy (the quadratic
// Q = rho E - |m|^2/2 - eps rhoeL rho has the sign of the constraint for rho > 0).
// In two parts: side_main takes the density bound and evaluates the quadratic
// at it (selects, no branches); only where Q is negative there does side_root
// solve the quadratic for its root.  A caller that needs several sides can
// evaluate all their main parts in one stretch of straight-line code and then
// take the (rarely needed) roots, so the independent divisions interleave.
struct SideTheta {
    double th, c0, c1, c2; // density-bounded theta, coefficients of Q(theta)
    bool ok;               // rhoeL > 0 (otherwise theta = 0)
    bool root;             // Q(th) < 0: the root of Q bounds theta
};
__device__ __forceinline__ SideTheta side_main(const Phys &P, const double L[4], double rmin, double rmax,
                                               double rhoeL, const double D[4])
{
    const bool dpos = D[0] > 0.0, dneg = D[0] < 0.0;
    const double num = dpos ? rmax - L[0] : rmin - L[0];
    const double quot = num / D[0];
    double th = (dpos || dneg) ? quot : 1.0;
    th = fmin(fmax(th, 0.0), 1.0);

    const bool ok = rhoeL > 0.0;
    const double eps = P.pos_eps;
    const double c2 = D[0] * D[3] - 0.5 * (D[1] * D[1] + D[2] * D[2]);
    const double c1 = L[0] * D[3] + D[0] * L[3] - (L[1] * D[1] + L[2] * D[2]) - eps * rhoeL * D[0];
    const double c0 = (1.0 - eps) * L[0] * rhoeL;
    const double q = c0 + th * (c1 + th * c2);
    return SideTheta{th, c0, c1, c2, ok, ok && !(q >= 0.0)};
}
// theta bounded by the smallest positive root of Q (only meaningful when s.root)
__device__ __forceinline__ double side_root(const SideTheta &s)
{
    double disc = s.c1 * s.c1 - 4.0 * s.c2 * s.c0;
    disc = disc < 0.0 ? 0.0 : disc;
    const double sq = sqrt(disc);
    const bool c1neg = s.c1 < 0.0;
    const double rn = c1neg ? 2.0 * s.c0 : s.c1 + sq;
    const double rd = c1neg ? sq - s.c1 : -2.0 * s.c2;
    const double rq = rn / rd;
    const double r = (c1neg || s.c2 < 0.0) ? rq : 0.0;
    return fmin(fmax(r, 0.0), s.th);
}
// the limited theta of one side from its two parts
__device__ __forceinline__ double side_value(const SideTheta &s, double root)
{
    return s.ok ? (s.root ? root : s.th) : 0.0;
}
__device__ __forceinline__ double side_theta(const Phys &P, const double L[4], double rmin,
                                             double rmax, double rhoeL, const double D[4])
{
    const SideTheta s = side_main(P, L, rmin, rmax, rhoeL, D);
    double root = s.th;
    if (s.root)
        root = side_root(s);
    return side_value(s, root);
}

// ---------------------------------------------------------------------------
// Correctly rounded cos / sin (inlet profile, eq:karhunenExp).
// Double-double arithmetic (Dekker 1971; Knuth's TwoSum), Cody-Waite reduction
// by pi/2 split into three doubles, Taylor series of degree 27 on |r| <= pi/4.
// The double-double result carries ~100 correct bits, so rounding it once to
// double gives the correctly rounded value except in cases closer than
// ~2^-100 to a rounding boundary.
// ---------------------------------------------------------------------------
struct dd {
    double hi, lo;
};
__device__ __forceinline__ dd dd_two_sum(double a, double b)
{
    const double s = a + b;
    const double bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ dd dd_fast_two_sum(double a, double b)
{
    const double s = a + b;
    return {s, b - (s - a)};
}
__device__ __forceinline__ dd dd_two_prod(double a, double b)
{
    const double p = a * b;
    return {p, __builtin_fma(a, b, -p)};
}
__device__ __forceinline__ dd dd_add(dd a, dd b)
{
    dd s = dd_two_sum(a.hi, b.hi);
    const dd t = dd_two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = dd_fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return dd_fast_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd dd_mul(dd a, dd b)
{
    dd p = dd_two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return dd_fast_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ dd dd_div_d(dd a, double b)
{
    const double q1 = a.hi / b;
    const dd p = dd_two_prod(q1, b);
    dd r = dd_two_sum(a.hi, -p.hi);
    r.lo -= p.lo;
    r.lo += a.lo;
    const double q2 = (r.hi + r.lo) / b;
    return dd_fast_two_sum(q1, q2);
}

// sin and cos of x (|x| < 2^20), correctly rounded to double.
__device__ inline void cr_sincos(double x, double *s_out, double *c_out)
{
    const double pio2_1 = 0x1.921fb54442d18p+0;    // pi/2 = pio2_1 + pio2_2 + pio2_3 + O(2^-164)
    const double pio2_2 = 0x1.1a62633145c07p-54;
    const double pio2_3 = -0x1.f1976b7ed8fbcp-110;
    const double n = rint(x * 0x1.45f306dc9c883p-1); // x * 2/pi
    const dd p1 = dd_two_prod(n, pio2_1);
    dd r = dd_two_sum(x, -p1.hi);
    r.lo -= p1.lo;
    r = dd_fast_two_sum(r.hi, r.lo);
    const dd p2 = dd_two_prod(n, pio2_2);
    r = dd_add(r, dd{-p2.hi, -p2.lo});
    r = dd_add(r, dd{-n * pio2_3, 0.0});
    // Taylor coefficients 1/k!, k = 0..27, in double-double.
    dd cs[14], cc[14];
    dd f = {1.0, 0.0};
    cc[0] = f;
    for (int k = 1; k < 28; ++k) {
        f = dd_div_d(f, (double)k);
        if (k & 1)
            cs[k >> 1] = ((k >> 1) & 1) ? dd{-f.hi, -f.lo} : f;
        else
            cc[k >> 1] = ((k >> 1) & 1) ? dd{-f.hi, -f.lo} : f;
    }
    const dd r2 = dd_mul(r, r);
    dd ts = cs[13], tc = cc[13];
    for (int k = 12; k >= 0; --k) {
        ts = dd_add(dd_mul(ts, r2), cs[k]);
        tc = dd_add(dd_mul(tc, r2), cc[k]);
    }
    const dd sr = dd_mul(ts, r), cr = tc;
    const int q = ((int)n) & 3;
    dd s, c;
    if (q == 0) { s = sr; c = cr; }
    else if (q == 1) { s = cr; c = dd{-sr.hi, -sr.lo}; }
    else if (q == 2) { s = dd{-sr.hi, -sr.lo}; c = dd{-cr.hi, -cr.lo}; }
    else { s = dd{-cr.hi, -cr.lo}; c = sr; }
    *s_out = s.hi + s.lo;
    *c_out = c.hi + c.lo;
}

// ---------------------------------------------------------------------------
// Per-realization control block, ring-buffered over three launches: launch n
// reads slot n%3, writes slot (n+1)%3 and clears the maximum of slot (n+2)%3.
// ---------------------------------------------------------------------------
struct Ctl {
    double *t;              // [3][NR] time
    long long *steps;       // [3][NR] step count
    double *a_last;         // [3][NR] kinetic speed of the last step
    unsigned long long *amax; // [3][NR] max wave speed of the state (bits of a double >= 0)
    int *status;            // [NR] latched failure bits (1 nonpositive, 2 nonfinite)
    unsigned *work;         // [9] dynamic dealing: next item of each XCD's range, then
                            // the count of wavefronts that have left (reset to 0 by the last)
    int nr;                 // NR = number of (level, realization) pairs
};

enum { STATUS_NONPOSITIVE = 1, STATUS_NONFINITE = 2 };

// Bit pattern of a non-negative double, monotone in its value.
__device__ __forceinline__ unsigned long long ordered_bits(double x)
{
    return (unsigned long long)__double_as_longlong(x);
}

// Block-wide max of v (every thread passes its value), then one atomicMax.
template <int NT>
__device__ __forceinline__ void block_atomic_max(double v, unsigned long long *dst)
{
    __shared__ double red[NT / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = fmax(v, __shfl_xor(v, o, 64));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
        red[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
#pragma unroll
        for (int k = 1; k < NT / 64; ++k)
            m = fmax(m, red[k]);
        atomicMax(dst, ordered_bits(m));
    }
}

// Time-step control shared by every block of one realization: kinetic speed
// a = kappa*2*max/(1-alpha), dt = dx/a, shortened near t_final exactly as the
// oracle does (reading R9).
struct StepCtl {
    double a, t_new;
    bool active;
};
__device__ __forceinline__ StepCtl step_control(double t, double amax, double kappa, double alpha,
                                                double dx, double t_final)
{
    StepCtl c;
    c.active = t < t_final;
    double a = kappa * 2.0 * amax / (1.0 - alpha);
    double dt = dx / a;
    if (t + dt >= t_final) {
        dt = t_final - t;
        a = dx / dt;
        c.t_new = t_final;
    } else if (t + 2.0 * dt > t_final) {
        dt = 0.5 * (t_final - t);
        a = dx / dt;
        c.t_new = t + dt;
    } else {
        c.t_new = t + dt;
    }
    c.a = a;
    return c;
}

// ---------------------------------------------------------------------------
// State access.  FP64: double [4 var][5 slot][R][ny][nx].  Mixed: the var 0..2
// planes as float (same index), padded to 256 B, then the var 3 planes as double.
// ---------------------------------------------------------------------------
// State layout of one level buffer, both precisions: realization-major, then
// row-major, and within a row one contiguous block of `pitch` bytes holding the
// rows of all 20 planes (v, s) of that mesh row.  A wave marching over the rows
// of one realization therefore touches two compact address windows per row
// (input and output buffer) instead of 40 planes far apart, and all of a
// realization's state lies within 4 GiB of its first byte, so kernels address
// it with one 64-bit base and 32-bit offsets.
// Within a row block the columns are grouped by the step kernel's strips:
// strip q (columns 60q .. 60q+59, the last strip also column 60q+60 when that
// is the last column of a bounded level) owns element slots 0..63 of a strip
// block, and the row block is its nstrip strip blocks one after another.  A
// strip block holds all 20 planes of its 64 slots, each plane one run of 64
// elements, so the wave of a strip reads and writes whole 128-byte lines (the
// unused slots take whatever its halo lanes hold) and every plane sits at a
// compile-time offset within the block:
//   FP64:  double [5 slot][4 var][64]                 10240 B per strip block
//   mixed: double u[4 var][64], double E[4 slot][64],
//          float q[4 slot][3 var][64] (rho, rho v1, rho v2)   7168 B
// A column's "slot index" is 64 q + (i - 60 q); its byte offset within the
// row block is q * (strip block) + (i - 60 q) * (element size).
static constexpr int STRIP = 60;   // output columns per strip
static constexpr int SLOTS = 64;   // element slots per strip block and plane

// Raw buffer resources of the step kernel: 64-bit base, no stride, bound
// num_records, 32-bit data format (the descriptor word of untyped gfx9
// buffers).  Accesses whose lane offset exceeds num_records are dropped
// (stores) or read as 0 (loads).  Stores carry the non-temporal hint.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
static constexpr int BUF_FORMAT_WORD = 0x00020000;
static constexpr int BUF_NT = 2;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const char *row, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)row, (short)0, (int)bytes, BUF_FORMAT_WORD);
}
// A plane offset (a compile-time constant) is split into the instruction's
// 12-bit immediate (added to the lane offset) and a multiple of 4096 in the
// scalar offset, so no register holds it.
__device__ __forceinline__ int buf_voff(unsigned lane_off, unsigned plane_off) { return (int)(lane_off + (plane_off & 4095u)); }
__device__ __forceinline__ int buf_soff(unsigned plane_off) { return (int)(plane_off & ~4095u); }

// Strips per row: ceil(nx / 60), except that a bounded level whose last column
// is 60 q + 60 lets the last strip's lane 62 carry it (that column is a copy of
// its left neighbour, which the same wave computes).
__host__ __device__ inline int strip_count(int nx, bool periodic)
{
    if (!periodic && (nx - 1) % STRIP == 0)
        return (nx - 1) / STRIP;
    return (nx + STRIP - 1) / STRIP;
}

// slot index of column i (64 * strip + position in the strip)
__device__ __forceinline__ unsigned col_slot(int i, int nstrip)
{
    const int q = min(i / STRIP, nstrip - 1);
    return (unsigned)(SLOTS * q + (i - STRIP * q));
}

struct StateFP64 {
    char *p;
    int ny, nstrip;
    unsigned pitch; // bytes per row block
    static constexpr unsigned BLOCK = 20u * SLOTS * 8u; // bytes per strip block (160 B per slot)
    __device__ static __forceinline__ StateFP64 make(void *b, int ny, int nstrip)
    {
        return StateFP64{(char *)b, ny, nstrip, BLOCK * (unsigned)nstrip};
    }
    __device__ static __forceinline__ unsigned esize(int, int) { return 8u; }
    // byte offset of plane (v, s) within a strip block
    __device__ static __forceinline__ unsigned poff(int v, int s) { return (unsigned)(s * 4 + v) * SLOTS * 8u; }
    // byte offset of slot index `slot` within a row block, for the element size of plane (v, s)
    __device__ static __forceinline__ unsigned lane_off(unsigned slot, int, int)
    {
        return (slot / SLOTS) * BLOCK + (slot % SLOTS) * 8u;
    }
    // first byte of realization m
    __device__ __forceinline__ char *real_base(int m) const { return p + (size_t)m * (size_t)ny * pitch; }
    __device__ __forceinline__ size_t at(int v, int s, int m, int j, int i) const
    {
        return ((size_t)m * (size_t)ny + (size_t)j) * pitch + lane_off(col_slot(i, nstrip), v, s) + poff(v, s);
    }
    __device__ __forceinline__ double ld(int v, int s, int m, int j, int i) const { return *(const double *)(p + at(v, s, m, j, i)); }
    __device__ __forceinline__ void st(int v, int s, int m, int j, int i, double x) const { *(double *)(p + at(v, s, m, j, i)) = x; }
    // value a store of x in variable v reads back as
    __device__ static __forceinline__ double stored(int, double x) { return x; }
    // Raw element bits for prefetching: the conversion to double happens at the
    // point of use, so a load in flight is not waited for at the loop back-edge.
    __device__ static __forceinline__ double decode(int, int, unsigned long long r) { return __longlong_as_double((long long)r); }
    // Buffer forms used by the step kernel: `rsrc` covers one row block, lane_off
    // is the lane's byte offset within it, plane_off the plane's offset within a
    // strip block.
    __device__ static __forceinline__ unsigned long long ldbuf(__amdgpu_buffer_rsrc_t rsrc, int, int, unsigned lane_off,
                                                               unsigned plane_off)
    {
        const u32x2 r = __builtin_amdgcn_raw_buffer_load_b64(rsrc, buf_voff(lane_off, plane_off), buf_soff(plane_off), 0);
        return ((unsigned long long)r.y << 32) | r.x;
    }
    __device__ static __forceinline__ void stbuf(__amdgpu_buffer_rsrc_t rsrc, int, int, unsigned lane_off,
                                                 unsigned plane_off, double x)
    {
        const unsigned long long b = (unsigned long long)__double_as_longlong(x);
        const u32x2 d = {(unsigned)(b & 0xffffffffull), (unsigned)(b >> 32)};
        __builtin_amdgcn_raw_buffer_store_b64(d, rsrc, buf_voff(lane_off, plane_off), buf_soff(plane_off), BUF_NT);
    }
};

struct StateMixed {
    char *p;
    int ny, nstrip;
    unsigned pitch;
    static constexpr unsigned BLOCK = 8u * SLOTS * 8u + 12u * SLOTS * 4u; // 7168 B per strip block (112 B per slot)
    __device__ static __forceinline__ StateMixed make(void *b, int ny, int nstrip)
    {
        return StateMixed{(char *)b, ny, nstrip, BLOCK * (unsigned)nstrip};
    }
    __device__ static __forceinline__ bool is_f32(int v, int s) { return s > 0 && v < 3; }
    __device__ static __forceinline__ unsigned esize(int v, int s) { return is_f32(v, s) ? 4u : 8u; }
    __device__ static __forceinline__ unsigned poff(int v, int s)
    {
        if (is_f32(v, s))
            return 8u * SLOTS * 8u + (unsigned)((s - 1) * 3 + v) * SLOTS * 4u;
        return (unsigned)(s == 0 ? v : 3 + s) * SLOTS * 8u;
    }
    __device__ static __forceinline__ unsigned lane_off(unsigned slot, int v, int s)
    {
        return (slot / SLOTS) * BLOCK + (slot % SLOTS) * esize(v, s);
    }
    __device__ __forceinline__ char *real_base(int m) const { return p + (size_t)m * (size_t)ny * pitch; }
    __device__ __forceinline__ size_t at(int v, int s, int m, int j, int i) const
    {
        return ((size_t)m * (size_t)ny + (size_t)j) * pitch + lane_off(col_slot(i, nstrip), v, s) + poff(v, s);
    }
    __device__ __forceinline__ double ld(int v, int s, int m, int j, int i) const
    {
        const char *q = p + at(v, s, m, j, i);
        return is_f32(v, s) ? (double)*(const float *)q : *(const double *)q;
    }
    __device__ __forceinline__ void st(int v, int s, int m, int j, int i, double x) const
    {
        char *q = p + at(v, s, m, j, i);
        if (is_f32(v, s))
            *(float *)q = (float)x;
        else
            *(double *)q = x;
    }
    // the macroscopic slot is FP64, so a stored u reads back unchanged
    __device__ static __forceinline__ double stored(int, double x) { return x; }
    __device__ static __forceinline__ double decode(int v, int s, unsigned long long r)
    {
        if (is_f32(v, s))
            return (double)__uint_as_float((unsigned int)r);
        return __longlong_as_double((long long)r);
    }
    __device__ static __forceinline__ unsigned long long ldbuf(__amdgpu_buffer_rsrc_t rsrc, int v, int s, unsigned lane_off,
                                                               unsigned plane_off)
    {
        if (is_f32(v, s))
            return (unsigned long long)__builtin_amdgcn_raw_buffer_load_b32(rsrc, buf_voff(lane_off, plane_off),
                                                                            buf_soff(plane_off), 0);
        const u32x2 r = __builtin_amdgcn_raw_buffer_load_b64(rsrc, buf_voff(lane_off, plane_off), buf_soff(plane_off), 0);
        return ((unsigned long long)r.y << 32) | r.x;
    }
    __device__ static __forceinline__ void stbuf(__amdgpu_buffer_rsrc_t rsrc, int v, int s, unsigned lane_off,
                                                 unsigned plane_off, double x)
    {
        if (is_f32(v, s)) {
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint((float)x), rsrc, buf_voff(lane_off, plane_off),
                                                  buf_soff(plane_off), BUF_NT);
            return;
        }
        const unsigned long long b = (unsigned long long)__double_as_longlong(x);
        const u32x2 d = {(unsigned)(b & 0xffffffffull), (unsigned)(b >> 32)};
        __builtin_amdgcn_raw_buffer_store_b64(d, rsrc, buf_voff(lane_off, plane_off), buf_soff(plane_off), BUF_NT);
    }
};

// Launch arguments of one mesh level and of the physics (plain values).
struct LevelArgs {
    int nx, ny, R;   // nodes incl. layers, realizations
    int nstrip;      // column strips of the state layout (strip_count)
    int ctl_off;     // index of realization 0 of this level in the control arrays
    double dx, y_min;
    void *buf[2];    // ping-pong state buffers
};

struct PhysArgs {
    double gamma, alpha, kappa, rlmp_relax, pos_eps;
    double rho_amb, p_amb, rho_jet, v_jet, r_jet, kl_amp;
    int kl_modes, kl_decay, bc, limiter;
};


// Scheme parameters of one step of a realization whose kinetic speed is a.
__device__ __forceinline__ Phys make_phys(const PhysArgs &ph, double a)
{
    Phys P;
    P.gamma = ph.gamma;
    P.alpha = ph.alpha;
    P.w = (1.0 - ph.alpha) / 4.0;
    P.h = 1.0 / (2.0 * a);
    P.rlmp_relax = ph.rlmp_relax;
    P.pos_eps = ph.pos_eps;
    P.inv_w = 1.0 / P.w;
    int e;
    P.w_pow2 = frexp(P.w, &e) == 0.5;
    return P;
}

enum { BC_JET = 0, BC_PERIODIC = 1, BC_NEUMANN = 2 };
enum { LIM_RLMP = 0, LIM_ZERO = 1, LIM_ONE = 2 };

template <int PREC> struct StateOf;
template <> struct StateOf<0> {
    typedef StateFP64 type;
    __device__ static type make(void *b, int ny, int nstrip) { return StateFP64::make(b, ny, nstrip); }
};
template <> struct StateOf<1> {
    typedef StateMixed type;
    __device__ static type make(void *b, int ny, int nstrip) { return StateMixed::make(b, ny, nstrip); }
};

// Work decomposition of the marching step kernel for one level.
struct MarchArgs {
    int nstrip;      // column strips per realization (the layout's strips)
    int chunk;       // rows per work item
    int nchunk;      // row chunks per realization
    int lane62_last; // 1: lane 62 of the last strip writes the copy column nx-1
    int order;       // work-item order: 0 strip fastest (consecutive items are
                     // neighbouring strips of one realization), 1 realization
                     // fastest (consecutive items are one tile of consecutive
                     // realizations)
};

// All mesh levels advanced by one launch: work items are concatenated level by
// level (realization, row chunk, strip within a level).
static constexpr int MAX_LEVELS = 8;
struct MultiLevel {
    int nlev;
    int wpb;                       // wavefronts per block (1, 2 or 4)
    int dynamic;                   // 0: static round-robin dealing; 1: per-XCD work queues
    int nblocks;                   // logical blocks (wpb waves each) of the grid
    int per_xcd;                   // logical blocks per XCD slot
    long long item_off[MAX_LEVELS + 1];
    LevelArgs L[MAX_LEVELS];
    MarchArgs ma[MAX_LEVELS];
};

// Node kinds of reading R8: 0 interior, 1 Dirichlet inlet layer, 2 copy layer.
__device__ __forceinline__ int node_kind(int bc, int nx, int ny, int i, int j)
{
    if (bc == BC_PERIODIC)
        return 0;
    if (bc == BC_JET && i == 0)
        return 1;
    if (i == 0 || i == nx - 1 || j == 0 || j == ny - 1)
        return 2;
    return 0;
}

} // namespace vlbm
