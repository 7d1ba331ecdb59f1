/*
 * vlbm_oracle.c -- plain FP64 CPU oracle for the probabilistic vectorial
 * lattice Boltzmann method (VLBM, D2Q5) of Simonis & Wissocq, "Computing
 * statistical solutions of a Mach 2000 astrophysical jet".
 *
 * TEST INFRASTRUCTURE.  This library exists to check the HIP implementation.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no source, header, constant table or helper
 * with the HIP library, and the HIP library never calls it.
 *
 * Style: one realization at a time, one node at a time, every quantity of the
 * scheme materialised in its own array, no blocking, fusion or reordering
 * beyond what the paper's formulas state.  Build with
 *     gcc -O2 -std=gnu99 -ffp-contract=off -fPIC -shared ... -lquadmath -lm
 * (no fast-math: the Mach-2000 pressure recovery cancels about six digits).
 *
 * Readings of points the paper leaves open:
 *   R1  alpha is a run-time parameter in [0,1) (eq:maxwellians5).
 *   R2  kinetic speed a_n = kappa * 2 * max_nodes(max(|v1|,|v2|) + c) / (1-alpha):
 *       the Bouchut condition for D2Q5 (eigenvalues of dM_k/du = w I +- A/(2a)
 *       non-negative) with a safety factor kappa >= 1 (Sec. 2.1, Sec. 2.3 CFL).
 *   R3  the blending parameter theta and the relaxed-local-maximum-principle
 *       (RLMP) limiter are defined in a cited work that is not available; this
 *       oracle uses per-face convex limiting of the low-order (theta = 0)
 *       update: relaxed local density bounds over the bar states plus an
 *       internal-energy floor.  Parity with the paper's own theta: UNPINNED.
 *   R7  initial populations are at equilibrium, u_k = M_k(u_0; a_0).
 *   R8  cell-centred nodes; column i = 0 is the Dirichlet inlet layer, the
 *       last column and the first/last rows are zero-gradient copy layers that
 *       take the full nodal state (u and u_1..u_4) of the nearest interior
 *       node after the interior update.  A layer node has no low-order update
 *       of its own, so it imposes no limiter constraint: the theta of a face
 *       is the minimum of the one-sided values of the adjacent nodes that the
 *       scheme updates.  (Forcing theta = 0 on layer faces instead breaks the
 *       exact preservation of uniform states next to a wall whenever a_n
 *       changes between steps.)
 *   R9  the time step dt = dx/a_n is shortened so that t lands exactly on
 *       t_final, taking a = dx/dt (larger than the Bouchut bound, hence still
 *       admissible).  When less than two full steps remain, the remainder is
 *       halved first, so the final steps never use more than twice the
 *       Bouchut speed (a nearly vanishing last step would otherwise replace
 *       every state by the mean of its neighbours).
 *
 * State layout of one realization (this file only):
 *     st[((s*4 + v)*ny + j)*nx + i]
 * slot s = 0 is the macroscopic state u, s = 1..4 the populations u_1..u_4;
 * variable v = 0..3 is (rho, rho v1, rho v2, E).  u_5 is never stored: the
 * scheme of eq:vlbm1-eq:vlbm5 eliminates it (Sec. 2.1).
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double gamma;      /* heat-capacity ratio of eq:eos                         */
    double alpha;      /* rest-population weight of eq:maxwellians5, in [0,1)   */
    double kappa;      /* safety factor on the Bouchut kinetic speed (R2)       */
    double rlmp_relax; /* relaxation of the local density bounds (R3)           */
    double pos_eps;    /* internal-energy floor, fraction of the low-order value */
    double rho_amb, p_amb, rho_jet, v_jet, r_jet; /* jet constants, Sec. 2.2 */
    double kl_amp;      /* A of eq:karhunenExp                                */
    int32_t kl_modes;   /* K of eq:karhunenExp                                */
    int32_t kl_decay;   /* p of eq:karhunenExp (a non-negative integer)       */
    int32_t bc;         /* ORC_BC_JET, ORC_BC_PERIODIC, ORC_BC_NEUMANN        */
    int32_t theta_mode; /* ORC_THETA_LIMITER, _ZERO, _ONE, _GIVEN             */
    int32_t storage;    /* ORC_STORE_FP64, ORC_STORE_MIXED                    */
} orc_params;

typedef struct {
    int32_t nx, ny;
    double dx;    /* mesh width, equal in x and y */
    double y_min; /* lower domain edge; node j sits at y_min + (j + 1/2) dx */
} orc_grid;

enum { ORC_BC_JET = 0, ORC_BC_PERIODIC = 1, ORC_BC_NEUMANN = 2 };
enum { ORC_THETA_LIMITER = 0, ORC_THETA_ZERO = 1, ORC_THETA_ONE = 2, ORC_THETA_GIVEN = 3 };
enum { ORC_OK = 0, ORC_ERR_ARG = -1, ORC_ERR_NONPOSITIVE = -4, ORC_ERR_NONFINITE = -5 };
/* Storage of the state between steps.  ORC_STORE_MIXED is the mixed-precision
 * variant (not in the paper): the rho, rho v1, rho v2 components of the
 * populations u_1..u_4 are held in binary32; the macroscopic u and the energy
 * populations stay binary64, and all arithmetic is binary64. */
enum { ORC_STORE_FP64 = 0, ORC_STORE_MIXED = 1 };

#define ST(st, s, v, j, i) (st)[((size_t)((s) * 4 + (v)) * (size_t)G->ny + (size_t)(j)) * (size_t)G->nx + (size_t)(i)]

/* ------------------------------------------------------------------------ */
/* Pointwise physics                                                         */
/* ------------------------------------------------------------------------ */

/* Ideal-gas pressure, eq:eos: p = (gamma-1)(E - rho (v1^2 + v2^2)/2). */
double orc_pressure(const orc_params *P, const double *u)
{
    const double rho = u[0];
    const double v1 = u[1] / rho;
    const double v2 = u[2] / rho;
    return (P->gamma - 1.0) * (u[3] - 0.5 * rho * (v1 * v1 + v2 * v2));
}

/* Euler fluxes f(u), g(u) of eq:fluxF and eq:fluxG, with rho v1 and rho v2
 * taken directly from the conserved momenta. */
void orc_fluxes(const orc_params *P, const double *u, double *f, double *g)
{
    const double rho = u[0], m1 = u[1], m2 = u[2], E = u[3];
    const double v1 = m1 / rho;
    const double v2 = m2 / rho;
    const double p = (P->gamma - 1.0) * (E - 0.5 * rho * (v1 * v1 + v2 * v2));
    f[0] = m1;
    f[1] = m1 * v1 + p;
    f[2] = m1 * v2;
    f[3] = (E + p) * v1;
    g[0] = m2;
    g[1] = m2 * v1;
    g[2] = m2 * v2 + p;
    g[3] = (E + p) * v2;
}

/* D2Q5 Maxwellians of eq:maxwellians12 and eq:maxwellians34 for kinetic
 * speed a.  M[k][v], k = 0..3 stands for M_1..M_4.  (M_5 = alpha u is never
 * needed explicitly.) */
void orc_maxwellians(const orc_params *P, double a, const double *u, double *M)
{
    double f[4], g[4];
    orc_fluxes(P, u, f, g);
    const double w = (1.0 - P->alpha) / 4.0;
    const double h = 1.0 / (2.0 * a);
    for (int v = 0; v < 4; ++v) {
        const double wu = w * u[v];
        M[0 * 4 + v] = wu + h * f[v];
        M[1 * 4 + v] = wu - h * f[v];
        M[2 * 4 + v] = wu + h * g[v];
        M[3 * 4 + v] = wu - h * g[v];
    }
}

/* Largest characteristic speed of the two flux Jacobians at u:
 * max(|v1|, |v2|) + c with c = sqrt(gamma p / rho).  Sets *bad when the
 * state is not admissible (rho <= 0, p <= 0 or not finite). */
double orc_wave_speed(const orc_params *P, const double *u, int *bad)
{
    const double rho = u[0];
    const double v1 = u[1] / rho;
    const double v2 = u[2] / rho;
    const double p = (P->gamma - 1.0) * (u[3] - 0.5 * rho * (v1 * v1 + v2 * v2));
    if (!(rho > 0.0) || !(p > 0.0) || !isfinite(rho) || !isfinite(p)) {
        *bad = 1;
        return 0.0;
    }
    const double c = sqrt(P->gamma * p / rho);
    return fmax(fabs(v1), fabs(v2)) + c;
}

/* ------------------------------------------------------------------------ */
/* Stochastic inlet and initial datum (Sec. 2.2, Sec. 2.3)                   */
/* ------------------------------------------------------------------------ */

/* Correctly rounded cosine and sine of a double: evaluated in binary128 and
 * rounded once to binary64.  The inlet profile feeds a scheme that amplifies
 * one-ulp differences (one ulp in one inlet density grows to a 1e-12 .. 6e-11
 * relative difference of the state within 50 steps of the Mach-2000 jet,
 * depending on alpha), so it is defined with correctly rounded elementary
 * functions rather than with whatever accuracy a particular libm offers. */
static double cr_cos(double x) { return (double)cosq((__float128)x); }
static double cr_sin(double x) { return (double)sinq((__float128)x); }

/* Inlet density of eq:rho_inlet_def with the Karhunen-Loeve perturbation of
 * eq:karhunenExp.  coef[2(k-1)] = Y_k, coef[2(k-1)+1] = Z_k, k = 1..K.
 * The modes are functions of the normalised coordinate ybar = y / r_jet and
 * the window is W(ybar) = cos^2(pi ybar / 2) (readings R4, R5).  The decay
 * k^(-p) uses the integer exponent p of the paper (p = 2). */
double orc_inlet_density(const orc_params *P, double y, const double *coef)
{
    if (fabs(y) > P->r_jet)
        return P->rho_amb;
    const double yb = y / P->r_jet;
    double s = 0.0;
    for (int k = 1; k <= P->kl_modes; ++k) {
        const double Yk = coef[2 * (k - 1)];
        const double Zk = coef[2 * (k - 1) + 1];
        double kp = 1.0;
        for (int q = 0; q < P->kl_decay; ++q)
            kp *= (double)k;
        const double amp = 1.0 / kp;
        s += amp * (Yk * cr_cos(k * M_PI * yb) + Zk * cr_sin(k * M_PI * yb));
    }
    double W = cr_cos(0.5 * M_PI * yb);
    W = W * W;
    return P->rho_jet * (1.0 + P->kl_amp * s * W);
}

/* Inlet state u_inlet = (rho, rho v1, 0, E) of Sec. 2.2: step velocity
 * profile, pressure p_amb, E from eq:eos. */
void orc_inlet_state(const orc_params *P, double y, const double *coef, double *u)
{
    const double rho = orc_inlet_density(P, y, coef);
    const double v1 = (fabs(y) <= P->r_jet) ? P->v_jet : 0.0;
    u[0] = rho;
    u[1] = rho * v1;
    u[2] = 0.0;
    u[3] = P->p_amb / (P->gamma - 1.0) + 0.5 * rho * (v1 * v1);
}

/* Quiescent ambient state u_amb of eq:u0_def. */
static void ambient_state(const orc_params *P, double *u)
{
    u[0] = P->rho_amb;
    u[1] = 0.0;
    u[2] = 0.0;
    u[3] = P->p_amb / (P->gamma - 1.0);
}

/* Kinetic speed a of the Bouchut condition (reading R2), max over every node
 * of the grid including boundary layers.  Returns a <= 0 if some node is not
 * admissible. */
double orc_kinetic_speed(const orc_params *P, const orc_grid *G, const double *st)
{
    double smax = 0.0;
    int bad = 0;
    for (int j = 0; j < G->ny; ++j)
        for (int i = 0; i < G->nx; ++i) {
            double u[4];
            for (int v = 0; v < 4; ++v)
                u[v] = ST(st, 0, v, j, i);
            const double s = orc_wave_speed(P, u, &bad);
            if (s > smax)
                smax = s;
        }
    if (bad)
        return -1.0;
    return P->kappa * 2.0 * smax / (1.0 - P->alpha);
}

/* Round the stored populations to the storage precision (ORC_STORE_MIXED). */
static void store_round(const orc_params *P, const orc_grid *G, double *st)
{
    if (P->storage != ORC_STORE_MIXED)
        return;
    for (int s = 1; s <= 4; ++s)
        for (int v = 0; v < 3; ++v)
            for (int j = 0; j < G->ny; ++j)
                for (int i = 0; i < G->nx; ++i)
                    ST(st, s, v, j, i) = (double)(float)ST(st, s, v, j, i);
}

/* Populations at equilibrium with the macroscopic state, u_k = M_k(u; a)
 * (reading R7). */
void orc_fill_equilibrium(const orc_params *P, const orc_grid *G, double a, double *st)
{
    for (int j = 0; j < G->ny; ++j)
        for (int i = 0; i < G->nx; ++i) {
            double u[4], M[16];
            for (int v = 0; v < 4; ++v)
                u[v] = ST(st, 0, v, j, i);
            orc_maxwellians(P, a, u, M);
            for (int k = 0; k < 4; ++k)
                for (int v = 0; v < 4; ++v)
                    ST(st, 1 + k, v, j, i) = M[k * 4 + v];
        }
    store_round(P, G, st);
}

/* Initial datum of eq:u0_def for one realization: u_inlet on column 0,
 * u_amb elsewhere, populations at equilibrium for the initial kinetic speed. */
int orc_init(const orc_params *P, const orc_grid *G, const double *coef, double *st)
{
    if (G->nx < 3 || G->ny < 3 || !(G->dx > 0.0))
        return ORC_ERR_ARG;
    for (int j = 0; j < G->ny; ++j) {
        const double y = G->y_min + (j + 0.5) * G->dx;
        for (int i = 0; i < G->nx; ++i) {
            double u[4];
            if (i == 0 && P->bc == ORC_BC_JET)
                orc_inlet_state(P, y, coef, u);
            else
                ambient_state(P, u);
            for (int v = 0; v < 4; ++v)
                ST(st, 0, v, j, i) = u[v];
        }
    }
    const double a0 = orc_kinetic_speed(P, G, st);
    if (!(a0 > 0.0))
        return ORC_ERR_NONPOSITIVE;
    orc_fill_equilibrium(P, G, a0, st);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Limiter (reading R3)                                                      */
/* ------------------------------------------------------------------------ */

/* Largest theta in [0,1] such that the candidate state L + theta*D keeps
 *   (i)  its density inside [rmin, rmax], and
 *   (ii) its internal energy rho e = E - |m|^2/(2 rho) >= eps * rhoeL,
 * where L is the low-order state of the cell, D = 4 sigma A_f its share of the
 * antidiffusive face flux and rhoeL = rho e(L).  Both feasible sets are
 * intervals containing 0: (i) is linear in theta, (ii) is a superlevel set of
 * a concave function.  (ii) is written as the quadratic
 *   Q(theta) = rho(theta) E(theta) - |m(theta)|^2/2 - eps rhoeL rho(theta)
 * which has the sign of rho e - eps rhoeL while rho > 0. */
double orc_side_theta(const orc_params *P, const double *L, double rmin, double rmax,
                      double rhoeL, const double *D)
{
    double th = 1.0;
    if (D[0] > 0.0)
        th = (rmax - L[0]) / D[0];
    else if (D[0] < 0.0)
        th = (rmin - L[0]) / D[0];
    th = fmin(fmax(th, 0.0), 1.0);

    if (!(rhoeL > 0.0))
        return 0.0;
    const double eps = P->pos_eps;
    const double c2 = D[0] * D[3] - 0.5 * (D[1] * D[1] + D[2] * D[2]);
    const double c1 = L[0] * D[3] + D[0] * L[3] - (L[1] * D[1] + L[2] * D[2]) - eps * rhoeL * D[0];
    const double c0 = (1.0 - eps) * L[0] * rhoeL;
    const double q = c0 + th * (c1 + th * c2);
    if (q >= 0.0)
        return th;
    /* Q(0) = c0 > 0 > Q(th): the first root in (0, th), by the cancellation-free
     * form of the quadratic formula. */
    double disc = c1 * c1 - 4.0 * c2 * c0;
    if (disc < 0.0)
        disc = 0.0;
    const double sq = sqrt(disc);
    double r;
    if (c1 < 0.0)
        r = 2.0 * c0 / (sq - c1);
    else if (c2 < 0.0)
        r = (c1 + sq) / (-2.0 * c2);
    else
        r = 0.0;
    return fmin(fmax(r, 0.0), th);
}

/* ------------------------------------------------------------------------ */
/* One stream-collide step, eq:vlbm1 - eq:vlbm5                              */
/* ------------------------------------------------------------------------ */

/* Node kinds: 0 interior (updated by the scheme), 1 Dirichlet inlet layer,
 * 2 zero-gradient copy layer (reading R8). */
static int node_kind(const orc_params *P, const orc_grid *G, int i, int j)
{
    if (P->bc == ORC_BC_PERIODIC)
        return 0;
    if (P->bc == ORC_BC_JET && i == 0)
        return 1;
    if (i == 0 || i == G->nx - 1 || j == 0 || j == G->ny - 1)
        return 2;
    return 0;
}

static int wrap(int i, int n) { return (i % n + n) % n; }
static int clampi(int i, int lo, int hi) { return i < lo ? lo : (i > hi ? hi : i); }

/*
 * Advance one realization by one time step with kinetic speed a.
 *
 * st, st_new   : states in the layout above (distinct buffers).
 * theta_x_in/theta_y_in : per-face blending parameters, used only when
 *                theta_mode == ORC_THETA_GIVEN.  theta_x[j*nx + i] belongs to
 *                the face between nodes (i,j) and (i+1,j); theta_y[j*nx + i]
 *                to the face between (i,j) and (i,j+1).  Faces between two
 *                boundary-layer nodes are never used (theta = 0 there).
 * theta_x_out/theta_y_out : if non-NULL, receive the theta actually used.
 * bounds_out   : if non-NULL, [3][ny][nx] receives, per interior cell, the
 *                relaxed density bounds rho_min', rho_max' and rho e of the
 *                low-order state (zero elsewhere).
 * Returns ORC_OK, ORC_ERR_NONPOSITIVE or ORC_ERR_NONFINITE (the step is
 * completed either way).
 */
int orc_step(const orc_params *P, const orc_grid *G, double a, const double *st, double *st_new,
             const double *theta_x_in, const double *theta_y_in, double *theta_x_out,
             double *theta_y_out, double *bounds_out)
{
    const int nx = G->nx, ny = G->ny;
    const size_t nn = (size_t)nx * (size_t)ny;
    if (nx < 3 || ny < 3 || !(a > 0.0))
        return ORC_ERR_ARG;
    const double alpha = P->alpha;
    const double w = (1.0 - alpha) / 4.0;
    const int periodic = (P->bc == ORC_BC_PERIODIC);

    /* Per-node Maxwellians M_k(u^n) and non-equilibrium parts N_k = M_k - u_k. */
    double *M = malloc(nn * 16 * sizeof(double));
    double *N = malloc(nn * 16 * sizeof(double));
    /* Per-cell low-order state, relaxed density bounds, low-order rho e. */
    double *UL = calloc(nn * 4, sizeof(double));
    double *RMIN = calloc(nn, sizeof(double));
    double *RMAX = calloc(nn, sizeof(double));
    double *RHOEL = calloc(nn, sizeof(double));
    double *TX = calloc(nn, sizeof(double));
    double *TY = calloc(nn, sizeof(double));
    if (!M || !N || !UL || !RMIN || !RMAX || !RHOEL || !TX || !TY) {
        free(M); free(N); free(UL); free(RMIN); free(RMAX); free(RHOEL); free(TX); free(TY);
        return ORC_ERR_ARG;
    }
#define NODE(i, j) ((size_t)(j) * (size_t)nx + (size_t)(i))

    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double u[4];
            for (int v = 0; v < 4; ++v)
                u[v] = ST(st, 0, v, j, i);
            double *Mn = M + NODE(i, j) * 16;
            orc_maxwellians(P, a, u, Mn);
            for (int k = 0; k < 4; ++k)
                for (int v = 0; v < 4; ++v)
                    N[NODE(i, j) * 16 + k * 4 + v] = Mn[k * 4 + v] - ST(st, 1 + k, v, j, i);
        }

    /* Low-order state (the theta = 0 update of eq:vlbm5) and its bar states
     * M_k(neighbour)/w, whose densities bound the limited update. */
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            if (node_kind(P, G, i, j) != 0)
                continue;
            const int im = periodic ? wrap(i - 1, nx) : i - 1;
            const int ip = periodic ? wrap(i + 1, nx) : i + 1;
            const int jm = periodic ? wrap(j - 1, ny) : j - 1;
            const int jp = periodic ? wrap(j + 1, ny) : j + 1;
            const double *M1 = M + NODE(im, j) * 16 + 0 * 4;
            const double *M2 = M + NODE(ip, j) * 16 + 1 * 4;
            const double *M3 = M + NODE(i, jm) * 16 + 2 * 4;
            const double *M4 = M + NODE(i, jp) * 16 + 3 * 4;
            double *L = UL + NODE(i, j) * 4;
            for (int v = 0; v < 4; ++v)
                L[v] = alpha * ST(st, 0, v, j, i) + M1[v] + M2[v] + M3[v] + M4[v];
            const double b1 = M1[0] / w, b2 = M2[0] / w, b3 = M3[0] / w, b4 = M4[0] / w;
            double rmax = fmax(fmax(b1, b2), fmax(b3, b4));
            double rmin = fmin(fmin(b1, b2), fmin(b3, b4));
            if (alpha > 0.0) {
                rmax = fmax(rmax, ST(st, 0, 0, j, i));
                rmin = fmin(rmin, ST(st, 0, 0, j, i));
            }
            const double delta = P->rlmp_relax * (rmax - rmin);
            RMAX[NODE(i, j)] = rmax + delta;
            RMIN[NODE(i, j)] = fmax(rmin - delta, 0.5 * rmin);
            RHOEL[NODE(i, j)] = L[3] - 0.5 * (L[1] * L[1] + L[2] * L[2]) / L[0];
        }

    /* Blending parameter per face. */
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            /* x-face between (i,j) and (i+1,j) */
            if (periodic || i + 1 < nx) {
                const int i2 = periodic ? wrap(i + 1, nx) : i + 1;
                const int in1 = node_kind(P, G, i, j) == 0, in2 = node_kind(P, G, i2, j) == 0;
                double th = 0.0;
                if (in1 || in2) {
                    if (P->theta_mode == ORC_THETA_ZERO)
                        th = 0.0;
                    else if (P->theta_mode == ORC_THETA_ONE)
                        th = 1.0;
                    else if (P->theta_mode == ORC_THETA_GIVEN)
                        th = theta_x_in[NODE(i, j)];
                    else {
                        double A[4], Dup[4], Ddn[4];
                        for (int v = 0; v < 4; ++v) {
                            A[v] = N[NODE(i, j) * 16 + 0 * 4 + v] - N[NODE(i2, j) * 16 + 1 * 4 + v];
                            Dup[v] = -4.0 * A[v];
                            Ddn[v] = 4.0 * A[v];
                        }
                        th = 1.0;
                        if (in1)
                            th = fmin(th, orc_side_theta(P, UL + NODE(i, j) * 4, RMIN[NODE(i, j)],
                                                         RMAX[NODE(i, j)], RHOEL[NODE(i, j)], Dup));
                        if (in2)
                            th = fmin(th, orc_side_theta(P, UL + NODE(i2, j) * 4, RMIN[NODE(i2, j)],
                                                         RMAX[NODE(i2, j)], RHOEL[NODE(i2, j)], Ddn));
                    }
                }
                TX[NODE(i, j)] = th;
            }
            /* y-face between (i,j) and (i,j+1) */
            if (periodic || j + 1 < ny) {
                const int j2 = periodic ? wrap(j + 1, ny) : j + 1;
                const int in1 = node_kind(P, G, i, j) == 0, in2 = node_kind(P, G, i, j2) == 0;
                double th = 0.0;
                if (in1 || in2) {
                    if (P->theta_mode == ORC_THETA_ZERO)
                        th = 0.0;
                    else if (P->theta_mode == ORC_THETA_ONE)
                        th = 1.0;
                    else if (P->theta_mode == ORC_THETA_GIVEN)
                        th = theta_y_in[NODE(i, j)];
                    else {
                        double A[4], Dup[4], Ddn[4];
                        for (int v = 0; v < 4; ++v) {
                            A[v] = N[NODE(i, j) * 16 + 2 * 4 + v] - N[NODE(i, j2) * 16 + 3 * 4 + v];
                            Dup[v] = -4.0 * A[v];
                            Ddn[v] = 4.0 * A[v];
                        }
                        th = 1.0;
                        if (in1)
                            th = fmin(th, orc_side_theta(P, UL + NODE(i, j) * 4, RMIN[NODE(i, j)],
                                                         RMAX[NODE(i, j)], RHOEL[NODE(i, j)], Dup));
                        if (in2)
                            th = fmin(th, orc_side_theta(P, UL + NODE(i, j2) * 4, RMIN[NODE(i, j2)],
                                                         RMAX[NODE(i, j2)], RHOEL[NODE(i, j2)], Ddn));
                    }
                }
                TY[NODE(i, j)] = th;
            }
        }

    /* Interior update, eq:vlbm1 - eq:vlbm5. */
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            if (node_kind(P, G, i, j) != 0)
                continue;
            const int im = periodic ? wrap(i - 1, nx) : i - 1;
            const int ip = periodic ? wrap(i + 1, nx) : i + 1;
            const int jm = periodic ? wrap(j - 1, ny) : j - 1;
            const int jp = periodic ? wrap(j + 1, ny) : j + 1;
            const double txm = TX[NODE(im, j)]; /* theta_{i-1/2,j} */
            const double txp = TX[NODE(i, j)];  /* theta_{i+1/2,j} */
            const double tym = TY[NODE(i, jm)]; /* theta_{i,j-1/2} */
            const double typ = TY[NODE(i, j)];  /* theta_{i,j+1/2} */
            const double *Mw = M + NODE(im, j) * 16, *Nw = N + NODE(im, j) * 16;
            const double *Me = M + NODE(ip, j) * 16, *Ne = N + NODE(ip, j) * 16;
            const double *Ms = M + NODE(i, jm) * 16, *Ns = N + NODE(i, jm) * 16;
            const double *Mn = M + NODE(i, jp) * 16, *Nn = N + NODE(i, jp) * 16;
            const double *Nc = N + NODE(i, j) * 16;
            for (int v = 0; v < 4; ++v) {
                const double u1 = Mw[0 * 4 + v] + txm * Nw[0 * 4 + v]; /* eq:vlbm1 */
                const double u2 = Me[1 * 4 + v] + txp * Ne[1 * 4 + v]; /* eq:vlbm2 */
                const double u3 = Ms[2 * 4 + v] + tym * Ns[2 * 4 + v]; /* eq:vlbm3 */
                const double u4 = Mn[3 * 4 + v] + typ * Nn[3 * 4 + v]; /* eq:vlbm4 */
                const double corr = alpha * ST(st, 0, v, j, i) - txm * Nc[1 * 4 + v] - txp * Nc[0 * 4 + v] -
                                    tym * Nc[3 * 4 + v] - typ * Nc[2 * 4 + v];
                ST(st_new, 1, v, j, i) = u1;
                ST(st_new, 2, v, j, i) = u2;
                ST(st_new, 3, v, j, i) = u3;
                ST(st_new, 4, v, j, i) = u4;
                ST(st_new, 0, v, j, i) = (u1 + u2 + u3 + u4) + corr; /* eq:vlbm5 */
            }
        }

    /* Boundary layers (reading R8): Dirichlet inlet keeps u_inlet with
     * equilibrium populations (eq:inletBC); copy layers take the new state of
     * the nearest interior node (eq:outletBC, eq:transverseBC). */
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const int kind = node_kind(P, G, i, j);
            if (kind == 1) {
                double u[4], Mi[16];
                for (int v = 0; v < 4; ++v) {
                    u[v] = ST(st, 0, v, j, i);
                    ST(st_new, 0, v, j, i) = u[v];
                }
                orc_maxwellians(P, a, u, Mi);
                for (int k = 0; k < 4; ++k)
                    for (int v = 0; v < 4; ++v)
                        ST(st_new, 1 + k, v, j, i) = Mi[k * 4 + v];
            } else if (kind == 2) {
                const int is = clampi(i, 1, nx - 2), js = clampi(j, 1, ny - 2);
                for (int s = 0; s < 5; ++s)
                    for (int v = 0; v < 4; ++v)
                        ST(st_new, s, v, j, i) = ST(st_new, s, v, js, is);
            }
        }

    store_round(P, G, st_new);

    /* Admissibility of the new state. */
    int status = ORC_OK;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const double rho = ST(st_new, 0, 0, j, i);
            const double m1 = ST(st_new, 0, 1, j, i), m2 = ST(st_new, 0, 2, j, i);
            const double E = ST(st_new, 0, 3, j, i);
            if (!isfinite(rho) || !isfinite(m1) || !isfinite(m2) || !isfinite(E)) {
                status = ORC_ERR_NONFINITE;
                continue;
            }
            const double rhoe = E - 0.5 * (m1 * m1 + m2 * m2) / rho;
            if ((!(rho > 0.0) || !(rhoe > 0.0)) && status == ORC_OK)
                status = ORC_ERR_NONPOSITIVE;
        }

    if (theta_x_out)
        memcpy(theta_x_out, TX, nn * sizeof(double));
    if (theta_y_out)
        memcpy(theta_y_out, TY, nn * sizeof(double));
    if (bounds_out) {
        memcpy(bounds_out, RMIN, nn * sizeof(double));
        memcpy(bounds_out + nn, RMAX, nn * sizeof(double));
        memcpy(bounds_out + 2 * nn, RHOEL, nn * sizeof(double));
    }
#undef NODE
    free(M); free(N); free(UL); free(RMIN); free(RMAX); free(RHOEL); free(TX); free(TY);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Time loop (Sec. 2.3: dt = dx / a_n, a_n re-evaluated every step)          */
/* ------------------------------------------------------------------------ */

/*
 * Advance one realization from time *t until t_final, taking at most
 * max_steps steps.  On entry st holds the state at *t; on return the state
 * at the new *t, *steps is incremented by the steps taken and *a_last holds
 * the kinetic speed of the last step.  The final steps are shortened to land
 * on t_final exactly (reading R9).
 */
int orc_run(const orc_params *P, const orc_grid *G, double t_final, int64_t max_steps, double *st,
            double *t, int64_t *steps, double *a_last)
{
    const size_t n = (size_t)20 * (size_t)G->nx * (size_t)G->ny;
    double *tmp = malloc(n * sizeof(double));
    if (!tmp)
        return ORC_ERR_ARG;
    int status = ORC_OK;
    for (int64_t s = 0; s < max_steps && *t < t_final; ++s) {
        double a = orc_kinetic_speed(P, G, st);
        if (!(a > 0.0)) {
            status = ORC_ERR_NONPOSITIVE;
            break;
        }
        double dt = G->dx / a;
        double t_new;
        if (*t + dt >= t_final) {
            dt = t_final - *t;
            a = G->dx / dt;
            t_new = t_final;
        } else if (*t + 2.0 * dt > t_final) {
            dt = 0.5 * (t_final - *t);
            a = G->dx / dt;
            t_new = *t + dt;
        } else {
            t_new = *t + dt;
        }
        status = orc_step(P, G, a, st, tmp, NULL, NULL, NULL, NULL, NULL);
        memcpy(st, tmp, n * sizeof(double));
        *t = t_new;
        *steps += 1;
        if (a_last)
            *a_last = a;
        if (status != ORC_OK)
            break;
    }
    free(tmp);
    return status;
}
