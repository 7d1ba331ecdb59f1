// vlbm_step_march.hip -- fused stream-collide step (eq:vlbm1 - eq:vlbm5) for
// gfx950, register-resident row marching.
//
// Decomposition.  One wavefront owns a strip of 64 consecutive columns of one
// realization and one chunk of rows; lanes 2..61 produce the strip's 60
// output columns, lanes 0, 1, 62, 63 are the halo the radius-2 stencil needs.
// The wave marches up its rows.  Iteration k reads the macroscopic row k and
// the population row k-1 (both prefetched two iterations ahead) and
//   - forms the Maxwellians (eq:maxwellians12-34) of row k, which serve as
//     M_4 of the low-order state of row k-1 now and as the Maxwellians of
//     row k in the next iteration,
//   - forms the non-equilibrium parts N = M - u_k of row k-1, its low-order
//     state, density bounds and the blending parameter of its east x-face,
//   - forms the blending parameter of the y-face between rows k-2 and k-1,
//   - finishes row k-2 (u_4 and u of eq:vlbm4-5) and
//   - writes u_1..u_3 of row k-1 (eq:vlbm1-3), which no longer depend on
//     anything unknown, keeping only the partial sums of eq:vlbm5.
// Only four 4-vectors per node (partial sum, partial correction, N_3, M_3),
// the low-order state and the Maxwellians of the newest row travel to the
// next iteration.  x-neighbours are exchanged with DPP lane shifts.  Each
// value of the state is read from memory once (plus the 2-column and 2-row
// halos of the stencil; the halo lanes read a neighbouring strip only where
// the stencil uses it) and written once, each store instruction covering the
// whole 64-element run of one plane in the strip's block (see the layout in
// vlbm_device.h): 320 B per FP64 node update.  Loads and stores go through
// raw buffer resources of one row block, so an address is a scalar base, one
// loop-invariant lane offset and the plane's compile-time offset; stores and
// the limiter's side conditions are lane-uniform or selects, so the loop has
// few branches.
//
// Every arithmetic expression has the operand order of the reference form in
// vlbm_kernels.hip (and of the oracle), so the result is bitwise identical.
//
// Boundary layers (Dirichlet inlet column, zero-gradient copy columns and
// rows) are produced by the wave that owns the copied interior node.
//
// Work items (realization, row chunk, strip) of every mesh level are ordered
// strip-fastest (or realization-fastest, a tuning choice) and given to a
// persistent grid of blocks of 1, 2 or 4 wavefronts sized to the resident
// capacity of the chip, either through per-XCD work queues (the default) or
// round-robin; both keep neighbouring strips on one XCD's L2.
#include "vlbm_device.h"

namespace vlbm {

// Minimum resident blocks per CU the register allocation is held to (1 leaves
// the full 512-entry register file to one wave per SIMD).
#ifndef VLBM_MARCH_MIN_BLOCKS
#define VLBM_MARCH_MIN_BLOCKS 1
#endif

// Lane exchange along the strip: lane i receives the value of lane i-1
// (from_left) or lane i+1 (from_right).  DPP wavefront shifts by one lane
// (a VALU operand modifier, no LDS round trip) into a fresh register; the end
// lanes receive 0 (bound control), which only halo lanes ever read, so the
// shifted value needs no copy of the source first.
__device__ __forceinline__ int dpp_left_i(int x) { return __builtin_amdgcn_mov_dpp(x, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ int dpp_right_i(int x) { return __builtin_amdgcn_mov_dpp(x, 0x130, 0xf, 0xf, true); }
__device__ __forceinline__ double from_left(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = dpp_left_i((int)(b & 0xffffffffll)), hi = dpp_left_i((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double from_right(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = dpp_right_i((int)(b & 0xffffffffll)), hi = dpp_right_i((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ int from_left_i(int x) { return dpp_left_i(x); }
__device__ __forceinline__ int from_right_i(int x) { return dpp_right_i(x); }

template <int PREC>
__device__ __forceinline__ void march_item(const PhysArgs &ph, const LevelArgs &L, const MarchArgs &ma,
                                           const Ctl &ctl, int phase, double t_final, long long item, int lane)
{
    int m, rem;
    if (ma.order == 0) { // strip fastest
        const long long per_real = (long long)ma.nstrip * ma.nchunk;
        m = (int)(item / per_real);
        rem = (int)(item % per_real);
    } else { // realization fastest
        m = (int)(item % L.R);
        rem = (int)(item / L.R);
    }
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
    const Phys P = make_phys(ph, sc.a);
    const int nx = L.nx, ny = L.ny, bc = ph.bc, lim = ph.limiter;
    const bool periodic = bc == BC_PERIODIC;
    typedef typename StateOf<PREC>::type St;
    const St Sin = StateOf<PREC>::make(L.buf[s & 1], ny, L.nstrip);
    const St Sout = StateOf<PREC>::make(L.buf[(s + 1) & 1], ny, L.nstrip);
    // Wave-uniform base of this realization in the input and output buffers;
    // a row of a plane sits at a 32-bit byte offset from it (a realization's
    // state is below 4 GiB), so every access is one scalar base plus the
    // lane's column offset.
    const char *const inb = Sin.real_base(m);
    char *const outb = Sout.real_base(m);
    const unsigned pitch = Sin.pitch;

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
    // interior node: every node of a periodic level, else rows 1..ny-2 of an
    // interior column (one unsigned compare on the row)
    const bool col_int = periodic || kind_col_interior;
    const unsigned int_rows = periodic ? 0xffffffffu : (unsigned)max(ny - 2, 0);
    auto interior = [&](int j) -> bool { return col_int && (unsigned)(j - (periodic ? 0 : 1)) < int_rows; };
    // Slot indices of this lane.  Loads read the slot of the clamped (or
    // wrapped) column cx.  Stores cover the strip's 64 slots with all lanes --
    // lane l writes slot (l - 2) mod 64, so lanes 2..61 (and lane 62 when it
    // carries the last column) land on their columns and the halo lanes fill
    // the unused slots -- and every store instruction writes whole lines.
    const unsigned slot_in = col_slot(cx, L.nstrip);
    const unsigned slot_out = (unsigned)(SLOTS * strip + ((lane - 2) & (SLOTS - 1)));
    // The halo lanes need the macroscopic state (radius-2 stencil) but only two
    // population values: u_1 of lane 1 (the west face of the strip) and u_2 of
    // lane 62 (its east face).  For the other population planes a halo lane reads
    // the slot of the nearest output column instead, a line the wave reads anyway,
    // so the neighbouring strips' lines are fetched for 8 of the 20 planes only.
    // Whatever a halo lane computes from those values never reaches an output lane.
    const unsigned slot_inner = (unsigned)__shfl((int)slot_in, lane < 2 ? 2 : 61, 64);
    const bool halo_lane = lane < 2 || lane > 61;
    unsigned slot_pop[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bool needed = !halo_lane || (q == 0 && lane == 1) || (q == 1 && lane == 62);
        slot_pop[q] = needed ? slot_in : slot_inner;
    }
    // Byte offsets of the lane within a row block, in the two element sizes
    // (v = 3 is an FP64 plane in every slot, v = 0 of a population slot the
    // FP32 one of the mixed layout).
    unsigned o_in = St::lane_off(slot_in, 3, 0), o_pop8[4], o_pop4[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        o_pop8[q] = St::lane_off(slot_pop[q], 3, 1 + q);
        o_pop4[q] = St::lane_off(slot_pop[q], 0, 1 + q);
    }
    auto col_in = [&](int v, int sl) -> unsigned {
        return sl == 0 ? o_in : (St::esize(v, sl) == 8u ? o_pop8[sl - 1] : o_pop4[sl - 1]);
    };
    // The inlet column's lane stores its scheme values into the strip's last
    // (padding) slot, which the halo lanes fill with scratch values anyway; its
    // Dirichlet values go to its own slot.  So every scheme store is one store
    // by all lanes, with no branch on the lane.
    const unsigned slot_scheme = inlet_col ? (unsigned)(SLOTS * strip + SLOTS - 1) : slot_out;
    auto col_out = [&](int v, int sl) -> unsigned { return St::lane_off(slot_out, v, sl); };
    unsigned o_sch8 = St::lane_off(slot_scheme, 3, 1), o_sch4 = St::lane_off(slot_scheme, 0, 1);
    auto col_scheme = [&](int v, int sl) -> unsigned { return St::esize(v, sl) == 8u ? o_sch8 : o_sch4; };
    // The offsets are re-declared live in every iteration (an empty asm), so the
    // constant plane offsets are added where the loads and stores are and fold
    // into their immediate fields, instead of being hoisted into one register
    // per plane.
    auto pin_offsets = [&]() {
        asm volatile("" : "+v"(o_in), "+v"(o_pop8[0]), "+v"(o_pop8[1]), "+v"(o_pop8[2]), "+v"(o_pop8[3]), "+v"(o_sch8));
        if constexpr (PREC == 1)
            asm volatile("" : "+v"(o_pop4[0]), "+v"(o_pop4[1]), "+v"(o_pop4[2]), "+v"(o_pop4[3]), "+v"(o_sch4));
    };
    double wmax = 0.0;
    int bad = 0;
    // Every access goes through a buffer resource of one row block (uniform, in
    // scalar registers): the lane's byte offset within the row block is the
    // vector offset, the plane's offset within a strip block a constant.
    auto out_row = [&](int j) { return row_rsrc(outb + (size_t)((unsigned)j * pitch), pitch); };
    auto in_row = [&](int j) { return row_rsrc(inb + (size_t)((unsigned)j * pitch), pitch); };
    auto store_slot = [&](int sl, int j, const double x[4]) {
        const __amdgpu_buffer_rsrc_t rj = out_row(j);
#pragma unroll
        for (int v = 0; v < 4; ++v)
            St::stbuf(rj, v, sl, col_scheme(v, sl), St::poff(v, sl), x[v]);
    };
    auto store_inlet = [&](int sl, int j, const double x[4]) {
        const __amdgpu_buffer_rsrc_t rj = out_row(j);
#pragma unroll
        for (int v = 0; v < 4; ++v)
            St::stbuf(rj, v, sl, col_out(v, sl), St::poff(v, sl), x[v]);
    };
    // wave-speed maximum and admissibility of a stored state, for the lanes in `mask`
    auto account = [&](const double u[4], bool mask) {
        double us[4];
#pragma unroll
        for (int v = 0; v < 4; ++v)
            us[v] = Sout.stored(v, u[v]);
        int b2 = 0;
        const double ws = wave_speed(ph.gamma, us, &b2);
        const bool fin = isfinite(us[0]) && isfinite(us[1]) && isfinite(us[2]) && isfinite(us[3]);
        wmax = fmax(wmax, mask ? ws : 0.0);
        bad |= !mask ? 0 : (!fin ? STATUS_NONFINITE : (b2 ? STATUS_NONPOSITIVE : 0));
    };
    auto shuffle_copy = [&](double x[4]) {
        if (wave_copy) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double fl = from_left(x[v]);
                const double fr = from_right(x[v]);
                x[v] = copy_from_left ? fl : (copy_from_right ? fr : x[v]);
            }
        }
    };
    // Row j of the chunk is stored by the wave (the same condition for every
    // lane); it is duplicated into the zero-gradient rows 0 / ny-1 when it is
    // the adjacent interior row.  The stored values of the output lanes but the
    // inlet's (written on its own) enter the wave-speed maximum and the
    // admissibility check.
    const int w_lo = periodic ? y0 : max(y0, 1), w_hi = periodic ? y1 : min(y1, ny - 1);
    const unsigned w_span = (unsigned)max(w_hi - w_lo, 0);
    auto row_written = [&](int j) { return (unsigned)(j - w_lo) < w_span; };
    const bool scheme_lane = out_lane && !inlet_col;
    // (a level with ny = 3 duplicates its single interior row into both)
    const int dup_lo_row = periodic ? -1 : 1, dup_hi_row = periodic ? -1 : ny - 2;
    auto dup_lo = [&](int j) { return j == dup_lo_row; };
    auto dup_hi = [&](int j) { return j == dup_hi_row; };

    // ---- register ring ----
    // Row k-2, finished in iteration k: (u1+u2)+u3, the correction without its
    // north-face term, N_3 and M_3, the low-order state and its bounds.
    double U1[4], MC[4][4]; // row k-1 and its Maxwellians (formed in iteration k-1)
    double pC[4], cC[4], N3C[4], M3C[4], LC[4], bC[3];
    // Prefetch ring, two rows deep: buffer X_k holds the macroscopic row k and the
    // population row k-1 used by iteration k; it is refilled with X_{k+2} as soon
    // as it has been read.  Loads are unconditional (rows clamped to the chunk's
    // range; the surplus ones re-read rows just fetched), so at least the 20 loads
    // of X_{k+1} are always issued after those of X_k and the wait for X_k never
    // has to wait for the stores of the previous iteration.
    double UA[4], UB[4];
    unsigned long long PA[4][4], PB[4][4]; // raw element bits

#pragma unroll
    for (int v = 0; v < 4; ++v) {
        U1[v] = (v == 0 || v == 3) ? 1.0 : 0.0; // placeholder row before the first load
        pC[v] = cC[v] = N3C[v] = M3C[v] = LC[v] = 0.0;
    }
    bC[0] = bC[1] = bC[2] = 0.0;
    maxwellians(P, U1, MC);

    const int k_first = y0 - 2, k_last = y1 + 1;
    // population row needed by iteration k is k-1; rows below y0-1 or above y1
    // never reach a stored value
    // (a bounded level clamps to [0, ny-1]; the bounds are folded once)
    const int p_lo = max(y0 - 1, 0), p_hi = min(y1, ny - 1), u_hi = min(k_last, ny - 1);
    auto prow = [&](int k) { return periodic ? row_of(min(max(k - 1, y0 - 1), y1)) : min(max(k - 1, p_lo), p_hi); };
    auto urow = [&](int k) { return periodic ? row_of(min(k, k_last)) : min(max(k, 0), u_hi); };
    auto load_x = [&](int k, double (&Ux)[4], unsigned long long (&Px)[4][4]) {
        const int ju = urow(k), jp = prow(k);
        const __amdgpu_buffer_rsrc_t ru = in_row(ju), rp = in_row(jp);
#pragma unroll
        for (int v = 0; v < 4; ++v)
            Ux[v] = St::decode(v, 0, St::ldbuf(ru, v, 0, col_in(v, 0), St::poff(v, 0)));
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                Px[q][v] = St::ldbuf(rp, v, 1 + q, col_in(v, 1 + q), St::poff(v, 1 + q));
    };
    // an even number of iterations (a leading one on rows that are never stored
    // when chunk + 4 is odd), so the two buffers alternate without a join
    const int k_start = k_first - ((k_last - k_first + 1) & 1);
    load_x(k_start, UA, PA);
    load_x(k_start + 1, UB, PB);

    auto iteration = [&](int k, double (&Ux)[4], unsigned long long (&Px)[4][4]) __attribute__((always_inline)) {
        pin_offsets();
        double U0[4];
#pragma unroll
        for (int v = 0; v < 4; ++v)
            U0[v] = Ux[v];
        // Row k-1: non-equilibrium parts (its populations arrived).
        double MB[4][4], NB[4][4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                MB[q][v] = MC[q][v];
                NB[q][v] = MB[q][v] - St::decode(v, 1 + q, Px[q][v]);
            }
        load_x(k + 2, Ux, Px);
        // Row k: Maxwellians, M_4 for the low-order state of row k-1 now, all
        // four for the next iteration.
        double MN[4][4];
        maxwellians(P, U0, MN);

        // Low-order state and bounds of row k-1.
        const int jB = k - 1;
        double LB[4], bB[3];
        {
            const double *M4n = MN[3]; // row k
            double M1w[4], M2e[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                M1w[v] = from_left(MB[0][v]);
                M2e[v] = from_right(MB[1][v]);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v)
                LB[v] = P.alpha * U1[v] + M1w[v] + M2e[v] + M3C[v] + M4n[v];
            cell_bounds(P, LB, M1w[0], M2e[0], M3C[0], M4n[0], U1[0], &bB[0], &bB[1], &bB[2]);
        }
        // Blending parameters of the two faces this iteration settles: the east
        // x-face of row k-1 and the y-face between rows k-2 and k-1, each the
        // smallest theta its interior sides admit.  The main parts of all four
        // sides are straight-line code evaluated on every lane (the results of
        // sides that are not interior are never selected), so their divisions
        // interleave; the root of the energy quadratic follows where a lane
        // needs it.
        const int r = k - 2;
        double txB, tyC;
        {
            double Lr[4], br[3], N2r[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                Lr[v] = from_right(LB[v]);
                N2r[v] = from_right(NB[1][v]);
            }
#pragma unroll
            for (int q = 0; q < 3; ++q)
                br[q] = from_right(bB[q]);
            const bool inx1 = interior(jB);
            const bool inx2 = from_right_i((int)inx1) != 0;
            const bool iny1 = interior(r), iny2 = inx1;
            double Dxu[4], Dxd[4], Dyu[4], Dyd[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double A = NB[0][v] - N2r[v];
                Dxu[v] = -4.0 * A;
                Dxd[v] = 4.0 * A;
                const double B = N3C[v] - NB[3][v];
                Dyu[v] = -4.0 * B;
                Dyd[v] = 4.0 * B;
            }
            const SideTheta sd[4] = {side_main(P, LB, bB[0], bB[1], bB[2], Dxu),
                                     side_main(P, Lr, br[0], br[1], br[2], Dxd),
                                     side_main(P, LC, bC[0], bC[1], bC[2], Dyu),
                                     side_main(P, LB, bB[0], bB[1], bB[2], Dyd)};
            const bool use[4] = {inx1, inx2, iny1, iny2};
            bool need[4];
            double root[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                need[i] = use[i] && sd[i].root;
                root[i] = sd[i].th;
            }
            // one branch on all four (it depends on every side's main part, so
            // none of them is deferred past another side's root)
            if (need[0] || need[1] || need[2] || need[3]) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (need[i])
                        root[i] = side_root(sd[i]);
            }
            double th[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                th[i] = side_value(sd[i], root[i]);
            auto face = [&](bool in1, bool in2, double t1, double t2) {
                double t = 1.0;
                t = in1 ? fmin(t, t1) : t;
                t = in2 ? fmin(t, t2) : t;
                const double mode = lim == LIM_ZERO ? 0.0 : (lim == LIM_ONE ? 1.0 : t);
                return (in1 || in2) ? mode : 0.0;
            };
            txB = face(inx1, inx2, th[0], th[1]);
            tyC = face(iny1, iny2, th[2], th[3]);
        }

        // Finish row k-2 (eq:vlbm4 and eq:vlbm5): u_4 and the macroscopic state.
        {
            double u4[4], u0[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                u4[v] = MB[3][v] + tyC * NB[3][v];
                u0[v] = (pC[v] + u4[v]) + (cC[v] - tyC * N3C[v]);
            }
            shuffle_copy(u4);
            shuffle_copy(u0);
            // (outside the store branch, so its divisions join the straight-line code)
            account(u0, scheme_lane && row_written(r));
            if (row_written(r)) {
                store_slot(0, r, u0);
                store_slot(4, r, u4);
                if (dup_lo(r)) {
                    store_slot(0, 0, u0);
                    store_slot(4, 0, u4);
                }
                if (dup_hi(r)) {
                    store_slot(0, ny - 1, u0);
                    store_slot(4, ny - 1, u4);
                }
            }
        }
        // Row k-1: populations u_1..u_3 (eq:vlbm1-3) are final; keep the partial
        // sums of eq:vlbm5 for the next iteration.
        const double txw = from_left(txB);
        double pB[4], cB[4];
        {
            double u1[4], u2[4], u3[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double out1 = MB[0][v] + txB * NB[0][v];
                const double out2 = MB[1][v] + txw * NB[1][v];
                u1[v] = from_left(out1);
                u2[v] = from_right(out2);
                u3[v] = M3C[v] + tyC * N3C[v];
                pB[v] = (u1[v] + u2[v]) + u3[v];
                cB[v] = ((P.alpha * U1[v] - txw * NB[1][v]) - txB * NB[0][v]) - tyC * NB[3][v];
            }
            shuffle_copy(u1);
            shuffle_copy(u2);
            shuffle_copy(u3);
            if (row_written(jB)) {
                store_slot(1, jB, u1);
                store_slot(2, jB, u2);
                store_slot(3, jB, u3);
                if (dup_lo(jB)) {
                    store_slot(1, 0, u1);
                    store_slot(2, 0, u2);
                    store_slot(3, 0, u3);
                }
                if (dup_hi(jB)) {
                    store_slot(1, ny - 1, u1);
                    store_slot(2, ny - 1, u2);
                    store_slot(3, ny - 1, u3);
                }
            }
            // Dirichlet inlet column (eq:inletBC): u kept, populations at
            // equilibrium for this step's kinetic speed.
            if (inlet_wave && jB >= y0 && jB < y1) {
                if (out_lane && inlet_col) {
                    store_inlet(0, jB, U1);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        store_inlet(1 + q, jB, MB[q]);
                }
                account(U1, out_lane && inlet_col);
            }
        }

        // ---- rotate the ring ----
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            U1[v] = U0[v];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                MC[q][v] = MN[q][v];
            pC[v] = pB[v];
            cC[v] = cB[v];
            N3C[v] = NB[2][v];
            M3C[v] = MB[2][v];
            LC[v] = LB[v];
        }
        bC[0] = bB[0];
        bC[1] = bB[1];
        bC[2] = bB[2];
    };

    for (int k = k_start; k <= k_last; k += 2) {
        iteration(k, UA, PA);
        iteration(k + 1, UB, PB);
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

template <int PREC>
__global__ void __launch_bounds__(256, VLBM_MARCH_MIN_BLOCKS)
step_march_kernel(PhysArgs ph, MultiLevel ml, Ctl ctl, int phase, double t_final)
{
    const int b = blockIdx.x;
    const int lb = (b & 7) * ml.per_xcd + (b >> 3);
    const int lane = threadIdx.x & 63;
    const long long n_items = ml.item_off[ml.nlev];
    const long long grid_waves = (long long)ml.nblocks * ml.wpb;
    // the wave index is uniform across the wave: keep it (and everything derived
    // from it: work item, realization, plane bases, time control) in scalar registers
    const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    // Static dealing: item i goes to wavefront i mod W.  Dynamic dealing: the
    // items are split into 8 contiguous ranges, one per XCD (blocks are
    // dispatched round-robin over the XCDs, so block b runs on XCD b mod 8 and
    // neighbouring strips stay on one L2); every wavefront takes the next item of
    // its XCD's range from a counter and, once that range is exhausted, of the
    // following XCDs' ranges in turn, so the last items go to whichever
    // wavefronts are free.  Each wavefront then counts itself out and the last
    // one resets the counters for the next launch (no wavefront of this launch
    // pulls any more by then, and the next launch starts after this one ended).
    const bool dyn = ml.dynamic != 0;
    if (!dyn && lb >= ml.nblocks)
        return;
    const int x0 = b & 7;
    int r = 0; // ranges visited: XCD (x0 + r) mod 8
    auto range_lo = [&](int k) -> long long { return n_items * ((x0 + k) & 7) / 8; };
    auto range_hi = [&](int k) -> long long { return n_items * (((x0 + k) & 7) + 1) / 8; };
    // next item of the current range, moving on through the ranges; n_items when all are done
    auto pull = [&]() -> long long {
        for (; r < 8; ++r) {
            unsigned k = 0;
            if (lane == 0)
                k = atomicAdd(ctl.work + ((x0 + r) & 7), 1u);
            const long long it = range_lo(r) + (long long)(unsigned)__builtin_amdgcn_readfirstlane((int)k);
            if (it < range_hi(r))
                return it;
        }
        return n_items;
    };
    long long item = dyn ? pull() : (long long)lb * ml.wpb + wid;
    int l = 0;
    while (item < n_items) {
        if (dyn)
            l = 0;
        while (item >= ml.item_off[l + 1])
            ++l;
        march_item<PREC>(ph, ml.L[l], ml.ma[l], ctl, phase, t_final, item - ml.item_off[l], lane);
        item = dyn ? pull() : item + grid_waves;
    }
    if (dyn && lane == 0) {
        const unsigned waves = gridDim.x * (blockDim.x >> 6);
        if (atomicAdd(ctl.work + 8, 1u) == waves - 1) {
#pragma unroll
            for (int k = 0; k < 9; ++k)
                atomicExch(ctl.work + k, 0u);
        }
    }
}

template __global__ void step_march_kernel<0>(PhysArgs, MultiLevel, Ctl, int, double);
template __global__ void step_march_kernel<1>(PhysArgs, MultiLevel, Ctl, int, double);

} // namespace vlbm
