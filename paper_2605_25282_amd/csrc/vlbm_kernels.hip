// vlbm_kernels.hip -- HIP kernels (gfx950) of the VLBM ensemble library:
// initial datum, the fused stream-collide step, moments and statistics.
//
// Work decomposition: one mesh level per launch; blockIdx.z selects the
// realization, (blockIdx.x, blockIdx.y) a tile of nodes.  Within a
// realization every block re-derives the same kinetic speed and time step from
// the ring-buffered control block, so no grid-wide synchronisation is needed.
#include "vlbm_device.h"

namespace vlbm {

// ---------------------------------------------------------------------------
// Initial datum (eq:u0_def): macroscopic state and its wave-speed maximum.
// ---------------------------------------------------------------------------
template <int PREC>
__global__ void __launch_bounds__(256) init_macro_kernel(PhysArgs ph, LevelArgs L,
                                                         const double *__restrict__ coeffs, Ctl ctl)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int m = blockIdx.z;
    const size_t plane = (size_t)L.nx * L.ny;
    auto S = StateOf<PREC>::make(L.buf[0], L.ny, L.nstrip);
    double s = 0.0;
    if (i < L.nx && j < L.ny) {
        double u[4];
        const double y = L.y_min + (j + 0.5) * L.dx;
        if (i == 0 && ph.bc == BC_JET) {
            // eq:rho_inlet_def with eq:karhunenExp (ybar = y / r_jet, W = cos^2(pi ybar / 2))
            double rho = ph.rho_amb;
            if (!(fabs(y) > ph.r_jet)) {
                const double yb = y / ph.r_jet;
                const double *c = coeffs + (size_t)m * 2 * ph.kl_modes;
                double sum = 0.0;
                for (int k = 1; k <= ph.kl_modes; ++k) {
                    double kp = 1.0;
                    for (int q = 0; q < ph.kl_decay; ++q)
                        kp *= (double)k;
                    const double amp = 1.0 / kp;
                    double sk, ck;
                    cr_sincos(k * M_PI * yb, &sk, &ck);
                    sum += amp * (c[2 * (k - 1)] * ck + c[2 * (k - 1) + 1] * sk);
                }
                double sw, W;
                cr_sincos(0.5 * M_PI * yb, &sw, &W);
                W = W * W;
                rho = ph.rho_jet * (1.0 + ph.kl_amp * sum * W);
            }
            const double v1 = (fabs(y) <= ph.r_jet) ? ph.v_jet : 0.0;
            u[0] = rho;
            u[1] = rho * v1;
            u[2] = 0.0;
            u[3] = ph.p_amb / (ph.gamma - 1.0) + 0.5 * rho * (v1 * v1);
        } else {
            u[0] = ph.rho_amb;
            u[1] = 0.0;
            u[2] = 0.0;
            u[3] = ph.p_amb / (ph.gamma - 1.0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v)
            S.st(v, 0, m, j, i, u[v]);
        int bad = 0;
        s = wave_speed(ph.gamma, u, &bad);
        if (bad)
            atomicOr(&ctl.status[L.ctl_off + m], STATUS_NONPOSITIVE);
    }
    block_atomic_max<256>(s, &ctl.amax[L.ctl_off + m]);
}

// Populations at equilibrium for the kinetic speed of slot 0 of the control
// ring: u_k = M_k(u; a_0), a_0 = kappa * 2 * max / (1 - alpha) (reading R7).
template <int PREC>
__global__ void __launch_bounds__(256) equilibrium_kernel(PhysArgs ph, LevelArgs L, Ctl ctl, int buf)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int m = blockIdx.z;
    if (i >= L.nx || j >= L.ny)
        return;
    const size_t plane = (size_t)L.nx * L.ny;
    auto S = StateOf<PREC>::make(L.buf[buf], L.ny, L.nstrip);
    const double amax = __longlong_as_double((long long)ctl.amax[L.ctl_off + m]);
    const double a = ph.kappa * 2.0 * amax / (1.0 - ph.alpha);
    const Phys P = make_phys(ph, a);
    double u[4], M[4][4];
#pragma unroll
    for (int v = 0; v < 4; ++v)
        u[v] = S.ld(v, 0, m, j, i);
    maxwellians(P, u, M);
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            S.st(v, 1 + k, m, j, i, M[k][v]);
}

// ---------------------------------------------------------------------------
// Fused stream-collide step (eq:vlbm1 - eq:vlbm5), reference form: one thread
// per output node, every intermediate recomputed from global memory.
// ---------------------------------------------------------------------------
template <class St>
struct NodeAccess {
    St S;
    int m, nx, ny, bc;
    __device__ __forceinline__ int wx(int i) const { return bc == BC_PERIODIC ? (i < 0 ? i + nx : (i >= nx ? i - nx : i)) : i; }
    __device__ __forceinline__ int wy(int j) const { return bc == BC_PERIODIC ? (j < 0 ? j + ny : (j >= ny ? j - ny : j)) : j; }
    __device__ __forceinline__ void load_u(int i, int j, double u[4]) const
    {
#pragma unroll
        for (int v = 0; v < 4; ++v)
            u[v] = S.ld(v, 0, m, j, i);
    }
    __device__ __forceinline__ void load_pop(int k, int i, int j, double q[4]) const
    {
#pragma unroll
        for (int v = 0; v < 4; ++v)
            q[v] = S.ld(v, 1 + k, m, j, i);
    }
};

// Low-order state and bounds of interior cell (i, j).
template <class Acc>
__device__ __forceinline__ void low_order(const Phys &P, const Acc &A, int i, int j, double L[4],
                                          double *rmin, double *rmax, double *rhoe)
{
    double u[4], M[4][4];
    double M1w[4], M2e[4], M3s[4], M4n[4];
    A.load_u(A.wx(i - 1), j, u);
    maxwellians(P, u, M);
#pragma unroll
    for (int v = 0; v < 4; ++v) M1w[v] = M[0][v];
    A.load_u(A.wx(i + 1), j, u);
    maxwellians(P, u, M);
#pragma unroll
    for (int v = 0; v < 4; ++v) M2e[v] = M[1][v];
    A.load_u(i, A.wy(j - 1), u);
    maxwellians(P, u, M);
#pragma unroll
    for (int v = 0; v < 4; ++v) M3s[v] = M[2][v];
    A.load_u(i, A.wy(j + 1), u);
    maxwellians(P, u, M);
#pragma unroll
    for (int v = 0; v < 4; ++v) M4n[v] = M[3][v];
    A.load_u(i, j, u);
#pragma unroll
    for (int v = 0; v < 4; ++v)
        L[v] = P.alpha * u[v] + M1w[v] + M2e[v] + M3s[v] + M4n[v];
    cell_bounds(P, L, M1w[0], M2e[0], M3s[0], M4n[0], u[0], rmin, rmax, rhoe);
}

// New state (20 values) of interior node (i, j).
template <class Acc>
__device__ __forceinline__ void update_node(const Phys &P, const Acc &A, int lim, int i, int j,
                                            double out[5][4])
{
    const int im = A.wx(i - 1), ip = A.wx(i + 1), jm = A.wy(j - 1), jp = A.wy(j + 1);
    double u[4], M[4][4], q[4];
    // Maxwellians and non-equilibrium parts at the node and its 4 neighbours.
    double Mc[4][4], Nc[4][4];
    A.load_u(i, j, u);
    maxwellians(P, u, Mc);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        A.load_pop(k, i, j, q);
#pragma unroll
        for (int v = 0; v < 4; ++v)
            Nc[k][v] = Mc[k][v] - q[v];
    }
    double Mw[4], Nw[4], Me[4], Ne[4], Ms[4], Ns[4], Mn[4], Nn[4];
    A.load_u(im, j, u);
    maxwellians(P, u, M);
    A.load_pop(0, im, j, q);
#pragma unroll
    for (int v = 0; v < 4; ++v) { Mw[v] = M[0][v]; Nw[v] = M[0][v] - q[v]; }
    A.load_u(ip, j, u);
    maxwellians(P, u, M);
    A.load_pop(1, ip, j, q);
#pragma unroll
    for (int v = 0; v < 4; ++v) { Me[v] = M[1][v]; Ne[v] = M[1][v] - q[v]; }
    A.load_u(i, jm, u);
    maxwellians(P, u, M);
    A.load_pop(2, i, jm, q);
#pragma unroll
    for (int v = 0; v < 4; ++v) { Ms[v] = M[2][v]; Ns[v] = M[2][v] - q[v]; }
    A.load_u(i, jp, u);
    maxwellians(P, u, M);
    A.load_pop(3, i, jp, q);
#pragma unroll
    for (int v = 0; v < 4; ++v) { Mn[v] = M[3][v]; Nn[v] = M[3][v] - q[v]; }

    double txm, txp, tym, typ;
    if (lim == LIM_ZERO) {
        txm = txp = tym = typ = 0.0;
    } else if (lim == LIM_ONE) {
        txm = txp = tym = typ = 1.0;
    } else {
        double Lc[4], rminc, rmaxc, rhoec;
        low_order(P, A, i, j, Lc, &rminc, &rmaxc, &rhoec);
        // For each face: A_f = N_out(upstream) - N_in(downstream); the node is
        // downstream (sigma = +1) of its west/south faces and upstream
        // (sigma = -1) of its east/north faces.  A neighbour contributes its
        // own one-sided bound only if the scheme updates it (reading R8).
        double Af[4], Dn[4], Dc[4], Ln[4], rminn, rmaxn, rhoen;
        // west face (im,j)-(i,j)
        for (int v = 0; v < 4; ++v) { Af[v] = Nw[v] - Nc[1][v]; Dn[v] = -4.0 * Af[v]; Dc[v] = 4.0 * Af[v]; }
        txm = 1.0;
        if (node_kind(A.bc, A.nx, A.ny, im, j) == 0) {
            low_order(P, A, im, j, Ln, &rminn, &rmaxn, &rhoen);
            txm = fmin(txm, side_theta(P, Ln, rminn, rmaxn, rhoen, Dn));
        }
        txm = fmin(txm, side_theta(P, Lc, rminc, rmaxc, rhoec, Dc));
        // east face (i,j)-(ip,j)
        for (int v = 0; v < 4; ++v) { Af[v] = Nc[0][v] - Ne[v]; Dc[v] = -4.0 * Af[v]; Dn[v] = 4.0 * Af[v]; }
        txp = 1.0;
        txp = fmin(txp, side_theta(P, Lc, rminc, rmaxc, rhoec, Dc));
        if (node_kind(A.bc, A.nx, A.ny, ip, j) == 0) {
            low_order(P, A, ip, j, Ln, &rminn, &rmaxn, &rhoen);
            txp = fmin(txp, side_theta(P, Ln, rminn, rmaxn, rhoen, Dn));
        }
        // south face (i,jm)-(i,j)
        for (int v = 0; v < 4; ++v) { Af[v] = Ns[v] - Nc[3][v]; Dn[v] = -4.0 * Af[v]; Dc[v] = 4.0 * Af[v]; }
        tym = 1.0;
        if (node_kind(A.bc, A.nx, A.ny, i, jm) == 0) {
            low_order(P, A, i, jm, Ln, &rminn, &rmaxn, &rhoen);
            tym = fmin(tym, side_theta(P, Ln, rminn, rmaxn, rhoen, Dn));
        }
        tym = fmin(tym, side_theta(P, Lc, rminc, rmaxc, rhoec, Dc));
        // north face (i,j)-(i,jp)
        for (int v = 0; v < 4; ++v) { Af[v] = Nc[2][v] - Nn[v]; Dc[v] = -4.0 * Af[v]; Dn[v] = 4.0 * Af[v]; }
        typ = 1.0;
        typ = fmin(typ, side_theta(P, Lc, rminc, rmaxc, rhoec, Dc));
        if (node_kind(A.bc, A.nx, A.ny, i, jp) == 0) {
            low_order(P, A, i, jp, Ln, &rminn, &rmaxn, &rhoen);
            typ = fmin(typ, side_theta(P, Ln, rminn, rmaxn, rhoen, Dn));
        }
    }
    A.load_u(i, j, u);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const double u1 = Mw[v] + txm * Nw[v];
        const double u2 = Me[v] + txp * Ne[v];
        const double u3 = Ms[v] + tym * Ns[v];
        const double u4 = Mn[v] + typ * Nn[v];
        const double corr = P.alpha * u[v] - txm * Nc[1][v] - txp * Nc[0][v] - tym * Nc[3][v] - typ * Nc[2][v];
        out[1][v] = u1;
        out[2][v] = u2;
        out[3][v] = u3;
        out[4][v] = u4;
        out[0][v] = (u1 + u2 + u3 + u4) + corr;
    }
}

template <int PREC>
__global__ void __launch_bounds__(256) step_ref_kernel(PhysArgs ph, LevelArgs L, Ctl ctl, int phase,
                                                       double t_final)
{
    const int m = blockIdx.z;
    const int cm = L.ctl_off + m;
    const int r0 = phase, r1 = (phase + 1) % 3, r2 = (phase + 2) % 3;
    const int nr = ctl.nr;
    const double t = ctl.t[r0 * nr + cm];
    const long long s = ctl.steps[r0 * nr + cm];
    const double amax = __longlong_as_double((long long)ctl.amax[r0 * nr + cm]);
    const StepCtl sc = step_control(t, amax, ph.kappa, ph.alpha, L.dx, t_final);
    const bool lead = blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0;
    if (!sc.active) {
        if (lead) {
            ctl.t[r1 * nr + cm] = t;
            ctl.steps[r1 * nr + cm] = s;
            ctl.a_last[r1 * nr + cm] = ctl.a_last[r0 * nr + cm];
            ctl.amax[r1 * nr + cm] = ctl.amax[r0 * nr + cm];
            ctl.amax[r2 * nr + cm] = 0ull;
        }
        return;
    }
    if (lead) {
        ctl.t[r1 * nr + cm] = sc.t_new;
        ctl.steps[r1 * nr + cm] = s + 1;
        ctl.a_last[r1 * nr + cm] = sc.a;
        ctl.amax[r2 * nr + cm] = 0ull;
    }
    const Phys P = make_phys(ph, sc.a);
    const size_t plane = (size_t)L.nx * L.ny;
    auto Sin = StateOf<PREC>::make(L.buf[s & 1], L.ny, L.nstrip);
    auto Sout = StateOf<PREC>::make(L.buf[(s + 1) & 1], L.ny, L.nstrip);
    typedef typename StateOf<PREC>::type St;
    NodeAccess<St> A{Sin, m, L.nx, L.ny, ph.bc};

    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    double wmax = 0.0;
    if (i < L.nx && j < L.ny) {
        double out[5][4];
        const int kind = node_kind(ph.bc, L.nx, L.ny, i, j);
        if (kind == 1) {
            double u[4], M[4][4];
            A.load_u(i, j, u);
            maxwellians(P, u, M);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                out[0][v] = u[v];
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    out[1 + k][v] = M[k][v];
            }
        } else {
            const int is = kind == 2 ? min(max(i, 1), L.nx - 2) : i;
            const int js = kind == 2 ? min(max(j, 1), L.ny - 2) : j;
            update_node(P, A, ph.limiter, is, js, out);
        }
#pragma unroll
        for (int sl = 0; sl < 5; ++sl)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                Sout.st(v, sl, m, j, i, out[sl][v]);
        // Admissibility of the stored state and its wave speed (next a_n).
        double us[4];
#pragma unroll
        for (int v = 0; v < 4; ++v)
            us[v] = Sout.ld(v, 0, m, j, i);
        int bad = 0;
        wmax = wave_speed(ph.gamma, us, &bad);
        const bool finite = isfinite(us[0]) && isfinite(us[1]) && isfinite(us[2]) && isfinite(us[3]);
        if (!finite)
            atomicOr(&ctl.status[cm], STATUS_NONFINITE);
        else if (bad)
            atomicOr(&ctl.status[cm], STATUS_NONPOSITIVE);
    }
    block_atomic_max<256>(wmax, &ctl.amax[r1 * nr + cm]);
}

// ---------------------------------------------------------------------------
// Moments and state export
// ---------------------------------------------------------------------------
template <int PREC>
__global__ void __launch_bounds__(256) moments_kernel(PhysArgs ph, LevelArgs L, Ctl ctl, int phase,
                                                      double *rho_o, double *speed_o, double *p_o)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int m = blockIdx.z;
    if (i >= L.nx || j >= L.ny)
        return;
    const long long s = ctl.steps[phase * ctl.nr + L.ctl_off + m];
    const size_t plane = (size_t)L.nx * L.ny;
    auto S = StateOf<PREC>::make(L.buf[s & 1], L.ny, L.nstrip);
    const size_t n = (size_t)j * L.nx + i;
    const double rho = S.ld(0, 0, m, j, i), m1 = S.ld(1, 0, m, j, i), m2 = S.ld(2, 0, m, j, i), E = S.ld(3, 0, m, j, i);
    const double v1 = m1 / rho;
    const double v2 = m2 / rho;
    const size_t o = (size_t)m * plane + n;
    if (rho_o)
        rho_o[o] = rho;
    if (speed_o)
        speed_o[o] = sqrt(v1 * v1 + v2 * v2);
    if (p_o)
        p_o[o] = (ph.gamma - 1.0) * (E - 0.5 * rho * (v1 * v1 + v2 * v2));
}

template <int PREC>
__global__ void __launch_bounds__(256) get_state_kernel(LevelArgs L, Ctl ctl, int phase, double *out)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int m = blockIdx.z;
    if (i >= L.nx || j >= L.ny)
        return;
    const long long s = ctl.steps[phase * ctl.nr + L.ctl_off + m];
    const size_t plane = (size_t)L.nx * L.ny;
    auto S = StateOf<PREC>::make(L.buf[s & 1], L.ny, L.nstrip);
    const size_t n = (size_t)j * L.nx + i;
    for (int v = 0; v < 4; ++v)
        for (int sl = 0; sl < 5; ++sl)
            out[((size_t)(v * 5 + sl) * L.R + m) * plane + n] = S.ld(v, sl, m, j, i);
}

// Load a macroscopic field [4][R][ny][nx] into slot 0 of buffer 0 and record
// its wave-speed maximum.
template <int PREC>
__global__ void __launch_bounds__(256) set_macro_kernel(PhysArgs ph, LevelArgs L, Ctl ctl,
                                                        const double *__restrict__ u_in)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int m = blockIdx.z;
    const size_t plane = (size_t)L.nx * L.ny;
    auto S = StateOf<PREC>::make(L.buf[0], L.ny, L.nstrip);
    double s = 0.0;
    if (i < L.nx && j < L.ny) {
        const size_t n = (size_t)j * L.nx + i;
        double u[4];
        for (int v = 0; v < 4; ++v) {
            u[v] = u_in[((size_t)v * L.R + m) * plane + n];
            S.st(v, 0, m, j, i, u[v]);
            u[v] = S.ld(v, 0, m, j, i);
        }
        int bad = 0;
        s = wave_speed(ph.gamma, u, &bad);
        if (bad)
            atomicOr(&ctl.status[L.ctl_off + m], STATUS_NONPOSITIVE);
    }
    block_atomic_max<256>(s, &ctl.amax[L.ctl_off + m]);
}

// Load a full state (20 values per node, layout [4 var][5 slot][R][ny][nx]) into
// the buffer each realization's step count selects (slot 0 of the control ring
// is current), and record the wave-speed maximum of the stored macroscopic
// state: the kinetic speed of the next step, as the step kernel's epilogue
// would have recorded it.
template <int PREC>
__global__ void __launch_bounds__(256) set_state_kernel(PhysArgs ph, LevelArgs L, Ctl ctl,
                                                        const double *__restrict__ in)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int m = blockIdx.z;
    const size_t plane = (size_t)L.nx * L.ny;
    const long long s = ctl.steps[L.ctl_off + m];
    auto S = StateOf<PREC>::make(L.buf[s & 1], L.ny, L.nstrip);
    double w = 0.0;
    if (i < L.nx && j < L.ny) {
        const size_t n = (size_t)j * L.nx + i;
        for (int v = 0; v < 4; ++v)
            for (int sl = 0; sl < 5; ++sl)
                S.st(v, sl, m, j, i, in[((size_t)(v * 5 + sl) * L.R + m) * plane + n]);
        double u[4];
        for (int v = 0; v < 4; ++v)
            u[v] = S.ld(v, 0, m, j, i);
        int bad = 0;
        w = wave_speed(ph.gamma, u, &bad);
        const bool fin = isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]) && isfinite(u[3]);
        if (!fin)
            atomicOr(&ctl.status[L.ctl_off + m], STATUS_NONFINITE);
        else if (bad)
            atomicOr(&ctl.status[L.ctl_off + m], STATUS_NONPOSITIVE);
    }
    block_atomic_max<256>(w, &ctl.amax[L.ctl_off + m]);
}

// ---------------------------------------------------------------------------
// Statistics (Sec. 3.2, 3.4)
// ---------------------------------------------------------------------------

// One thread per coarse cell: restrict the moments of every realization of the
// batch (r x r average), two-pass batch mean and M2, pairwise merge into acc,
// scatter the restricted density into the sample store.
template <int PREC>
__global__ void __launch_bounds__(256) stats_accumulate_kernel(PhysArgs ph, LevelArgs L, Ctl ctl,
                                                               int phase, int r, double *acc,
                                                               long long n_prev, double *samples,
                                                               long long m_offset)
{
    const int ncx = L.nx / r, ncy = L.ny / r;
    const long long ncell = (long long)ncx * ncy;
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= ncell)
        return;
    const int ci = (int)(cell % ncx), cj = (int)(cell / ncx);
    const size_t plane = (size_t)L.nx * L.ny;
    const double inv = 1.0 / (double)(r * r);
    double sum[3] = {0.0, 0.0, 0.0};
    for (int pass = 0; pass < 2; ++pass) {
        double mean[3], m2[3] = {0.0, 0.0, 0.0};
        for (int f = 0; f < 3; ++f)
            mean[f] = sum[f] / (double)L.R;
        for (int m = 0; m < L.R; ++m) {
            const long long s = ctl.steps[phase * ctl.nr + L.ctl_off + m];
            auto S = StateOf<PREC>::make(L.buf[s & 1], L.ny, L.nstrip);
            double blk[3] = {0.0, 0.0, 0.0};
            for (int dj = 0; dj < r; ++dj)
                for (int di = 0; di < r; ++di) {
                    const int jj = cj * r + dj, ii = ci * r + di;
                    const double rho = S.ld(0, 0, m, jj, ii), m1 = S.ld(1, 0, m, jj, ii),
                                 m2v = S.ld(2, 0, m, jj, ii), E = S.ld(3, 0, m, jj, ii);
                    const double v1 = m1 / rho, v2 = m2v / rho;
                    blk[0] += rho;
                    blk[1] += sqrt(v1 * v1 + v2 * v2);
                    blk[2] += (ph.gamma - 1.0) * (E - 0.5 * rho * (v1 * v1 + v2 * v2));
                }
            for (int f = 0; f < 3; ++f)
                blk[f] *= inv;
            if (pass == 0) {
                for (int f = 0; f < 3; ++f)
                    sum[f] += blk[f];
                if (samples)
                    samples[(size_t)(m_offset + m) * ncell + cell] = blk[0];
            } else {
                for (int f = 0; f < 3; ++f) {
                    const double d = blk[f] - mean[f];
                    m2[f] += d * d;
                }
            }
        }
        if (pass == 1) {
            for (int f = 0; f < 3; ++f) {
                double *am = acc + (size_t)(2 * f) * ncell, *aq = acc + (size_t)(2 * f + 1) * ncell;
                if (n_prev == 0) {
                    am[cell] = mean[f];
                    aq[cell] = m2[f];
                } else {
                    const double na = (double)n_prev, nb = (double)L.R, n = na + nb;
                    const double d = mean[f] - am[cell];
                    am[cell] = am[cell] + d * (nb / n);
                    aq[cell] = aq[cell] + m2[f] + d * d * (na * nb / n);
                }
            }
        }
    }
}

__global__ void __launch_bounds__(256) stats_finalize_kernel(const double *__restrict__ acc,
                                                             long long ncell, long long n,
                                                             double *mean, double *sd)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell)
        return;
    for (int f = 0; f < 3; ++f) {
        if (mean)
            mean[(size_t)f * ncell + c] = acc[(size_t)(2 * f) * ncell + c];
        if (sd)
            sd[(size_t)f * ncell + c] = sqrt(acc[(size_t)(2 * f + 1) * ncell + c] / (double)n);
    }
}

// Per-cell ascending sort of a [m][ncell] store: one block per group of
// CPB cells, LDS bitonic network over the padded power-of-two length.
template <int CPB>
__global__ void __launch_bounds__(256) sort_samples_kernel(double *samples, long long ncell, int m, int mp)
{
    extern __shared__ double sh[];   // [CPB][mp]
    const long long c0 = (long long)blockIdx.x * CPB;
    for (int idx = threadIdx.x; idx < CPB * mp; idx += blockDim.x) {
        const int c = idx % CPB, k = idx / CPB;
        double v = __builtin_huge_val();
        if (k < m && c0 + c < ncell)
            v = samples[(size_t)k * ncell + c0 + c];
        sh[c * mp + k] = v;
    }
    __syncthreads();
    const int half = mp >> 1;
    for (int size = 2; size <= mp; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int idx = threadIdx.x; idx < CPB * half; idx += blockDim.x) {
                const int c = idx / half, t = idx % half;
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool up = ((lo & size) == 0);
                double *col = sh + c * mp;
                const double a = col[lo], b = col[hi];
                if ((a > b) == up) {
                    col[lo] = b;
                    col[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    for (int idx = threadIdx.x; idx < CPB * mp; idx += blockDim.x) {
        const int c = idx % CPB, k = idx / CPB;
        if (k < m && c0 + c < ncell)
            samples[(size_t)k * ncell + c0 + c] = sh[c * mp + k];
    }
}

// Explicit instantiations.
template __global__ void init_macro_kernel<0>(PhysArgs, LevelArgs, const double *, Ctl);
template __global__ void init_macro_kernel<1>(PhysArgs, LevelArgs, const double *, Ctl);
template __global__ void equilibrium_kernel<0>(PhysArgs, LevelArgs, Ctl, int);
template __global__ void equilibrium_kernel<1>(PhysArgs, LevelArgs, Ctl, int);
template __global__ void step_ref_kernel<0>(PhysArgs, LevelArgs, Ctl, int, double);
template __global__ void step_ref_kernel<1>(PhysArgs, LevelArgs, Ctl, int, double);
template __global__ void moments_kernel<0>(PhysArgs, LevelArgs, Ctl, int, double *, double *, double *);
template __global__ void moments_kernel<1>(PhysArgs, LevelArgs, Ctl, int, double *, double *, double *);
template __global__ void get_state_kernel<0>(LevelArgs, Ctl, int, double *);
template __global__ void get_state_kernel<1>(LevelArgs, Ctl, int, double *);
template __global__ void set_macro_kernel<0>(PhysArgs, LevelArgs, Ctl, const double *);
template __global__ void set_macro_kernel<1>(PhysArgs, LevelArgs, Ctl, const double *);
template __global__ void set_state_kernel<0>(PhysArgs, LevelArgs, Ctl, const double *);
template __global__ void set_state_kernel<1>(PhysArgs, LevelArgs, Ctl, const double *);
template __global__ void stats_accumulate_kernel<0>(PhysArgs, LevelArgs, Ctl, int, int, double *, long long, double *, long long);
template __global__ void stats_accumulate_kernel<1>(PhysArgs, LevelArgs, Ctl, int, int, double *, long long, double *, long long);
template __global__ void sort_samples_kernel<1>(double *, long long, int, int);
template __global__ void sort_samples_kernel<4>(double *, long long, int, int);
template __global__ void sort_samples_kernel<16>(double *, long long, int, int);

} // namespace vlbm
