// vlbm_step_march.hip -- fused stream-collide step (eq:vlbm1 - eq:vlbm5) for
// gfx950, register-resident row marching.
//
// Decomposition.  One wavefront owns a strip of 64 consecutive columns of one
// realization and one chunk of rows; lanes 2..61 produce the strip's 60
// output columns, lanes 0, 1, 62, 63 are the halo the radius-2 stencil needs.
// The wave marches up its rows.  Iteration k reads the macroscopic row k and
// the population row k-1 (both prefetched one iteration ahead) and
//   S1  computes the Maxwellians M(k)                      (eq:maxwellians12-34)
//   S2  forms the low-order state and density bounds of row k-1, its
//       non-equilibrium parts N(k-1) = M(k-1) - u_k(k-1) and the blending
//       parameter of every x-face of row k-1
//   S3  forms the blending parameter of the y-faces between rows k-2 and k-1
//       and writes row k-2 (eq:vlbm1-5).
// Every quantity of a node is computed once; x-neighbours are exchanged with
// cross-lane shuffles, y-neighbours live in a three-row register ring.  Each
// value of the state is read from HBM once (plus the 4-column and 4-row halos)
// and written once: 320 B per FP64 node update.
//
// Every arithmetic expression has the operand order of the reference form in
// vlbm_kernels.hip (and of the oracle), so the result is bitwise identical.
//
// Boundary layers (Dirichlet inlet column, zero-gradient copy columns and
// rows) are produced by the wave that owns the copied interior node.  Blocks
// are renumbered so that consecutive work lands on one XCD (shared L2 for the
// halo re-reads).
#include "vlbm_device.h"

namespace vlbm {

struct MarchArgs {
    int nstrip;     // column strips per realization
    int chunk;      // rows per work item
    int nchunk;     // row chunks per realization
    int nblocks;    // logical blocks (4 waves each)
    int per_xcd;    // logical blocks per XCD slot
    int lane62_last; // 1: lane 62 of the last strip writes the copy column nx-1
};

static constexpr int STRIP = 60;

__device__ __forceinline__ double from_left(double x) { return __shfl_up(x, 1, 64); }
__device__ __forceinline__ double from_right(double x) { return __shfl_down(x, 1, 64); }
__device__ __forceinline__ int from_left_i(int x) { return __shfl_up(x, 1, 64); }
__device__ __forceinline__ int from_right_i(int x) { return __shfl_down(x, 1, 64); }

template <int PREC>
__global__ void __launch_bounds__(256, 1)
step_march_kernel(PhysArgs ph, LevelArgs L, Ctl ctl, int phase, double t_final, MarchArgs ma)
{
    const int b = blockIdx.x;
    const int lb = (b & 7) * ma.per_xcd + (b >> 3);
    if (lb >= ma.nblocks)
        return;
    const int lane = threadIdx.x & 63;
    const long long gw = (long long)lb * 4 + (threadIdx.x >> 6);
    const long long per_real = (long long)ma.nstrip * ma.nchunk;
    if (gw >= per_real * L.R)
        return;
    const int m = (int)(gw / per_real);
    const int rem = (int)(gw % per_real);
    const int chunk = rem / ma.nstrip, strip = rem % ma.nstrip;

    // ---- time-step control (identical in every wave of the realization) ----
    const int cm = L.ctl_off + m, nr = ctl.nr;
    const int r0 = phase, r1 = (phase + 1) % 3, r2 = (phase + 2) % 3;
    const double t = ctl.t[r0 * nr + cm];
    const long long s = ctl.steps[r0 * nr + cm];
    const double amax = __longlong_as_double((long long)ctl.amax[r0 * nr + cm]);
    const StepCtl sc = step_control(t, amax, ph.kappa, ph.alpha, L.dx, t_final);
    const bool lead = strip == 0 && chunk == 0 && lane == 0;
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
    const Phys P{ph.gamma, ph.alpha, (1.0 - ph.alpha) / 4.0, 1.0 / (2.0 * sc.a), ph.rlmp_relax, ph.pos_eps};
    const int nx = L.nx, ny = L.ny, bc = ph.bc, lim = ph.limiter;
    const bool periodic = bc == BC_PERIODIC;
    const size_t plane = (size_t)nx * ny;
    const auto Sin = StateOf<PREC>::make(L.buf[s & 1], plane, L.R);
    const auto Sout = StateOf<PREC>::make(L.buf[(s + 1) & 1], plane, L.R);

    // ---- geometry of this lane ----
    const int c = strip * STRIP - 2 + lane; // column
    const int cx = periodic ? ((c % nx) + nx) % nx : min(max(c, 0), nx - 1);
    bool out_lane = lane >= 2 && lane <= 61 && c < nx;
    if (!periodic && ma.lane62_last && strip == ma.nstrip - 1) {
        if (lane == 62 && c == nx - 1)
            out_lane = true;
        if (lane == 2 && c == nx - 1)
            out_lane = false;
    }
    const int kind_col_interior = periodic ? 1 : (c >= 1 && c <= nx - 2); // column is interior
    const bool inlet_col = bc == BC_JET && c == 0;
    // copy columns: take the result of the neighbouring lane
    const bool copy_from_right = !periodic && c == 0 && bc == BC_NEUMANN;
    const bool copy_from_left = !periodic && c == nx - 1;
    const bool wave_copy = !periodic && (strip == ma.nstrip - 1 || (strip == 0 && bc == BC_NEUMANN));
    const bool inlet_wave = bc == BC_JET && strip == 0;
    const int y0 = chunk * ma.chunk, y1 = min(ny, y0 + ma.chunk);

    auto row_of = [&](int j) { return periodic ? ((j % ny) + ny) % ny : min(max(j, 0), ny - 1); };
    auto interior = [&](int j) -> bool {
        if (periodic)
            return true;
        return kind_col_interior && j >= 1 && j <= ny - 2;
    };

    // ---- register ring ----
    double U0[4], U1[4], U2[4];       // macroscopic rows k, k-1, k-2
    double MA[4][4], MB[4][4];        // Maxwellians of rows k, k-1
    double MC[3][4];                  // M_1..M_3 of row k-2
    double NB[4][4], NC[4][4];        // non-equilibrium parts of rows k-1, k-2
    double LB[4], LC[4];              // low-order states of rows k-1, k-2
    double bB[3], bC[3];              // (rho_min', rho_max', rho e_L) of rows k-1, k-2
    double txB = 0.0, txC = 0.0;      // theta of the east x-face, rows k-1, k-2
    double tyD = 0.0;                 // theta of the y-face between rows k-3 and k-2
    double o3D[4];                    // streamed population 3 leaving row k-3
    double Un[4], Pn[4][4];           // prefetch: U(k+1), populations of row k
    double wmax = 0.0;
    int bad = 0;

#pragma unroll
    for (int v = 0; v < 4; ++v) {
        U1[v] = U2[v] = LB[v] = LC[v] = o3D[v] = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            MB[q][v] = NB[q][v] = NC[q][v] = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q)
            MC[q][v] = 0.0;
    }
    bB[0] = bB[1] = bB[2] = bC[0] = bC[1] = bC[2] = 0.0;

    const int k_first = y0 - 2, k_last = y1 + 1;
    {
        const size_t n0 = (size_t)row_of(k_first) * nx + cx;
#pragma unroll
        for (int v = 0; v < 4; ++v)
            Un[v] = Sin.ld(v, 0, m, n0);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                Pn[q][v] = 0.0;
    }

    for (int k = k_first; k <= k_last; ++k) {
        double Pc[4][4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            U0[v] = Un[v];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                Pc[q][v] = Pn[q][v];
        }
        // prefetch the next rows
        if (k < k_last) {
            const size_t nu = (size_t)row_of(k + 1) * nx + cx;
#pragma unroll
            for (int v = 0; v < 4; ++v)
                Un[v] = Sin.ld(v, 0, m, nu);
        }
        if (k >= y0 - 1 && k <= y1) { // population row k is used (as row k-1) next iteration
            const size_t np = (size_t)row_of(k) * nx + cx;
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    Pn[q][v] = Sin.ld(v, 1 + q, m, np);
        }

        // S1: Maxwellians of row k
        maxwellians(P, U0, MA);

        // S2: row k-1
        const int jB = k - 1;
        double M1w[4], M2e[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            M1w[v] = from_left(MB[0][v]);
            M2e[v] = from_right(MB[1][v]);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v)
            LB[v] = P.alpha * U1[v] + M1w[v] + M2e[v] + MC[2][v] + MA[3][v];
        cell_bounds(P, LB, M1w[0], M2e[0], MC[2][0], MA[3][0], U1[0], &bB[0], &bB[1], &bB[2]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                NB[q][v] = MB[q][v] - Pc[q][v];
        {
            // x-face between this column and the next, row k-1
            double Lr[4], br[3], N2r[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                Lr[v] = from_right(LB[v]);
                N2r[v] = from_right(NB[1][v]);
            }
#pragma unroll
            for (int q = 0; q < 3; ++q)
                br[q] = from_right(bB[q]);
            const bool in1 = interior(jB);
            const int in2 = from_right_i((int)in1);
            double th = 0.0;
            if (in1 || in2) {
                if (lim == LIM_ZERO) {
                    th = 0.0;
                } else if (lim == LIM_ONE) {
                    th = 1.0;
                } else {
                    double Dup[4], Ddn[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const double A = NB[0][v] - N2r[v];
                        Dup[v] = -4.0 * A;
                        Ddn[v] = 4.0 * A;
                    }
                    th = 1.0;
                    if (in1)
                        th = fmin(th, side_theta(P, LB, bB[0], bB[1], bB[2], Dup));
                    if (in2)
                        th = fmin(th, side_theta(P, Lr, br[0], br[1], br[2], Ddn));
                }
            }
            txB = th;
        }

        // S3: row r = k-2
        const int r = k - 2;
        double tyC = 0.0;
        {
            const bool in1 = interior(r), in2 = interior(r + 1);
            if (in1 || in2) {
                if (lim == LIM_ZERO) {
                    tyC = 0.0;
                } else if (lim == LIM_ONE) {
                    tyC = 1.0;
                } else {
                    double Dup[4], Ddn[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const double A = NC[2][v] - NB[3][v];
                        Dup[v] = -4.0 * A;
                        Ddn[v] = 4.0 * A;
                    }
                    tyC = 1.0;
                    if (in1)
                        tyC = fmin(tyC, side_theta(P, LC, bC[0], bC[1], bC[2], Dup));
                    if (in2)
                        tyC = fmin(tyC, side_theta(P, LB, bB[0], bB[1], bB[2], Ddn));
                }
            }
        }
        const double txw = from_left(txC);
        double R[5][4], o3C[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double out1 = MC[0][v] + txC * NC[0][v];
            const double out2 = MC[1][v] + txw * NC[1][v];
            o3C[v] = MC[2][v] + tyC * NC[2][v];
            const double u4 = MB[3][v] + tyC * NB[3][v];
            const double corr = P.alpha * U2[v] - txw * NC[1][v] - txC * NC[0][v] - tyD * NC[3][v] - tyC * NC[2][v];
            const double u1 = from_left(out1);
            const double u2 = from_right(out2);
            const double u3 = o3D[v];
            R[1][v] = u1;
            R[2][v] = u2;
            R[3][v] = u3;
            R[4][v] = u4;
            R[0][v] = (u1 + u2 + u3 + u4) + corr;
        }
        // copy columns take the result of the adjacent (interior) column
        if (wave_copy) {
#pragma unroll
            for (int sl = 0; sl < 5; ++sl)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const double fl = from_left(R[sl][v]);
                    const double fr = from_right(R[sl][v]);
                    if (copy_from_left)
                        R[sl][v] = fl;
                    else if (copy_from_right)
                        R[sl][v] = fr;
                }
        }
        // Dirichlet inlet column (eq:inletBC): u kept, populations at equilibrium for a_n
        if (inlet_wave) {
            double Mi[4][4];
            maxwellians(P, U2, Mi);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                R[0][v] = inlet_col ? U2[v] : R[0][v];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    R[1 + q][v] = inlet_col ? Mi[q][v] : R[1 + q][v];
            }
        }
        // ---- store row r ----
        if (out_lane && r >= y0 && r < y1) {
            const bool copy_row = !periodic && (r == 0 || r == ny - 1);
            if (inlet_col || !copy_row) {
                const size_t n = (size_t)r * nx + c;
#pragma unroll
                for (int sl = 0; sl < 5; ++sl)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        Sout.st(v, sl, m, n, R[sl][v]);
                double us[4];
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    us[v] = Sout.stored(v, R[0][v]);
                int b2 = 0;
                wmax = fmax(wmax, wave_speed(ph.gamma, us, &b2));
                const bool fin = isfinite(us[0]) && isfinite(us[1]) && isfinite(us[2]) && isfinite(us[3]);
                bad |= !fin ? STATUS_NONFINITE : (b2 ? STATUS_NONPOSITIVE : 0);
                // zero-gradient rows copy the adjacent interior row (not the inlet corners)
                if (!periodic && !inlet_col && (r == 1 || r == ny - 2)) {
                    if (r == 1) {
                        const size_t n2 = (size_t)c;
#pragma unroll
                        for (int sl = 0; sl < 5; ++sl)
#pragma unroll
                            for (int v = 0; v < 4; ++v)
                                Sout.st(v, sl, m, n2, R[sl][v]);
                    }
                    if (r == ny - 2) {
                        const size_t n2 = (size_t)(ny - 1) * nx + c;
#pragma unroll
                        for (int sl = 0; sl < 5; ++sl)
#pragma unroll
                            for (int v = 0; v < 4; ++v)
                                Sout.st(v, sl, m, n2, R[sl][v]);
                    }
                }
            }
        }

        // ---- rotate the ring ----
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            U2[v] = U1[v];
            U1[v] = U0[v];
#pragma unroll
            for (int q = 0; q < 3; ++q)
                MC[q][v] = MB[q][v];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                MB[q][v] = MA[q][v];
                NC[q][v] = NB[q][v];
            }
            LC[v] = LB[v];
            o3D[v] = o3C[v];
        }
        bC[0] = bB[0];
        bC[1] = bB[1];
        bC[2] = bB[2];
        txC = txB;
        tyD = tyC;
    }

    // ---- wave-speed maximum (next a_n) and latched status ----
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        wmax = fmax(wmax, __shfl_xor(wmax, o, 64));
        bad |= __shfl_xor(bad, o, 64);
    }
    if (lane == 0) {
        atomicMax(&ctl.amax[r1 * nr + cm], ordered_bits(wmax));
        if (bad)
            atomicOr(&ctl.status[cm], bad & STATUS_NONFINITE ? STATUS_NONFINITE : STATUS_NONPOSITIVE);
    }
}

template __global__ void step_march_kernel<0>(PhysArgs, LevelArgs, Ctl, int, double, MarchArgs);
template __global__ void step_march_kernel<1>(PhysArgs, LevelArgs, Ctl, int, double, MarchArgs);

} // namespace vlbm
