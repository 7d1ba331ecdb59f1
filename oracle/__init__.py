"""Plain FP64 CPU oracle for the probabilistic VLBM Mach-2000 jet ensemble.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library (``paper_2605_25282_amd``) and never imports it.

The stepping arithmetic lives in ``vlbm_oracle.c`` (one realization at a time,
one node at a time, FP64, no fast-math).  The ensemble statistics of Sec. 3.2
and Sec. 3.4 of the paper (restriction, mean, population standard deviation,
one-point Wasserstein-1) are written below with numpy, each one the plain
definition it cites.

State layout used by this package for one realization: a float64 array of
shape (20, ny, nx); row ``s*4 + v`` is variable v (rho, rho v1, rho v2, E) of
slot s (0 = macroscopic u, 1..4 = populations u_1..u_4).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vlbm_oracle.c")
# ORACLE_LIB names another build of vlbm_oracle.c to load (the sanitizer test
# runs the oracle from an AddressSanitizer / UBSan build this way)
_LIB = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "libvlbm_oracle.so")

BC = {"jet": 0, "periodic": 1, "neumann": 2}
THETA = {"limiter": 0, "zero": 1, "one": 2, "given": 3}
STORAGE = {"fp64": 0, "mixed": 1}
OK, ERR_ARG, ERR_NONPOSITIVE, ERR_NONFINITE = 0, -1, -4, -5


def build(force: bool = True) -> str:
    """Compile vlbm_oracle.c with gcc (FP64, contraction off, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=gnu99", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
             "-shared", _SRC, "-o", tmp, "-lquadmath", "-lm"],
            check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("alpha", ctypes.c_double),
                ("kappa", ctypes.c_double), ("rlmp_relax", ctypes.c_double),
                ("pos_eps", ctypes.c_double), ("rho_amb", ctypes.c_double),
                ("p_amb", ctypes.c_double), ("rho_jet", ctypes.c_double),
                ("v_jet", ctypes.c_double), ("r_jet", ctypes.c_double),
                ("kl_amp", ctypes.c_double), ("kl_modes", ctypes.c_int32),
                ("kl_decay", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("theta_mode", ctypes.c_int32), ("storage", ctypes.c_int32)]


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("dx", ctypes.c_double), ("y_min", ctypes.c_double)]


@dataclass
class Params:
    """Physical and numerical parameters (Sec. 2.1-2.3 of the paper)."""
    gamma: float = 5.0 / 3.0
    # weight of the rest population M_5 = alpha u (eq:maxwellians5; the paper
    # leaves it free): the standard D2Q5 weights, 1/3 at rest and 1/6 per
    # moving direction.  With alpha = 0 every update draws on the four
    # neighbours only and the even and odd sublattices decouple.
    alpha: float = 1.0 / 3.0
    kappa: float = 1.0
    rlmp_relax: float = 0.1
    pos_eps: float = 1e-2
    rho_amb: float = 0.5
    p_amb: float = 0.4127
    rho_jet: float = 5.0
    v_jet: float = 800.0
    r_jet: float = 0.05
    kl_amp: float = 0.1
    kl_decay: int = 2
    kl_modes: int = 10
    bc: str = "jet"
    theta_mode: str = "limiter"
    storage: str = "fp64"

    def c(self) -> _Params:
        return _Params(self.gamma, self.alpha, self.kappa, self.rlmp_relax, self.pos_eps,
                       self.rho_amb, self.p_amb, self.rho_jet, self.v_jet, self.r_jet,
                       self.kl_amp, self.kl_modes, self.kl_decay, BC[self.bc],
                       THETA[self.theta_mode], STORAGE[self.storage])


@dataclass
class Grid:
    """Cell-centred uniform grid: node (i, j) at x = (i+1/2) dx, y = y_min + (j+1/2) dx."""
    nx: int
    ny: int
    dx: float
    y_min: float = 0.0

    def c(self) -> _Grid:
        return _Grid(self.nx, self.ny, self.dx, self.y_min)

    def y(self) -> np.ndarray:
        return self.y_min + (np.arange(self.ny) + 0.5) * self.dx


_lib_handle = None
_dp = ctypes.POINTER(ctypes.c_double)


def _lib():
    global _lib_handle
    if _lib_handle is None:
        path = _LIB if os.path.exists(_LIB) else build(force=False)
        lib = ctypes.CDLL(path)
        P, G = ctypes.POINTER(_Params), ctypes.POINTER(_Grid)
        lib.orc_pressure.argtypes = [P, _dp]
        lib.orc_pressure.restype = ctypes.c_double
        lib.orc_fluxes.argtypes = [P, _dp, _dp, _dp]
        lib.orc_maxwellians.argtypes = [P, ctypes.c_double, _dp, _dp]
        lib.orc_wave_speed.argtypes = [P, _dp, ctypes.POINTER(ctypes.c_int)]
        lib.orc_wave_speed.restype = ctypes.c_double
        lib.orc_inlet_density.argtypes = [P, ctypes.c_double, _dp]
        lib.orc_inlet_density.restype = ctypes.c_double
        lib.orc_inlet_state.argtypes = [P, ctypes.c_double, _dp, _dp]
        lib.orc_kinetic_speed.argtypes = [P, G, _dp]
        lib.orc_kinetic_speed.restype = ctypes.c_double
        lib.orc_fill_equilibrium.argtypes = [P, G, ctypes.c_double, _dp]
        lib.orc_init.argtypes = [P, G, _dp, _dp]
        lib.orc_init.restype = ctypes.c_int
        lib.orc_side_theta.argtypes = [P, _dp, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, _dp]
        lib.orc_side_theta.restype = ctypes.c_double
        lib.orc_step.argtypes = [P, G, ctypes.c_double, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        lib.orc_step.restype = ctypes.c_int
        lib.orc_run.argtypes = [P, G, ctypes.c_double, ctypes.c_int64, _dp,
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(ctypes.c_double)]
        lib.orc_run.restype = ctypes.c_int
        _lib_handle = lib
    return _lib_handle


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _vec(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


# --------------------------------------------------------------------------
# Pointwise physics (eq:eos, eq:fluxF, eq:fluxG, eq:maxwellians12-5)
# --------------------------------------------------------------------------

def pressure(p: Params, u) -> float:
    return _lib().orc_pressure(ctypes.byref(p.c()), _ptr(_vec(u)))


def fluxes(p: Params, u):
    f, g = np.zeros(4), np.zeros(4)
    _lib().orc_fluxes(ctypes.byref(p.c()), _ptr(_vec(u)), _ptr(f), _ptr(g))
    return f, g


def maxwellians(p: Params, a: float, u) -> np.ndarray:
    """Return M[k][v], k = 0..3 for M_1..M_4."""
    M = np.zeros(16)
    _lib().orc_maxwellians(ctypes.byref(p.c()), a, _ptr(_vec(u)), _ptr(M))
    return M.reshape(4, 4)


def wave_speed(p: Params, u) -> tuple[float, bool]:
    bad = ctypes.c_int(0)
    s = _lib().orc_wave_speed(ctypes.byref(p.c()), _ptr(_vec(u)), ctypes.byref(bad))
    return s, bool(bad.value)


def inlet_density(p: Params, y: float, coef) -> float:
    return _lib().orc_inlet_density(ctypes.byref(p.c()), float(y), _ptr(_vec(coef)))


def inlet_state(p: Params, y: float, coef) -> np.ndarray:
    u = np.zeros(4)
    _lib().orc_inlet_state(ctypes.byref(p.c()), float(y), _ptr(_vec(coef)), _ptr(u))
    return u


def side_theta(p: Params, L, rmin, rmax, rhoeL, D) -> float:
    return _lib().orc_side_theta(ctypes.byref(p.c()), _ptr(_vec(L)), rmin, rmax, rhoeL,
                                 _ptr(_vec(D)))


# --------------------------------------------------------------------------
# Whole-grid operations on one realization
# --------------------------------------------------------------------------

def init(p: Params, g: Grid, coef) -> np.ndarray:
    """Initial datum of eq:u0_def with equilibrium populations."""
    st = np.zeros((20, g.ny, g.nx))
    rc = _lib().orc_init(ctypes.byref(p.c()), ctypes.byref(g.c()), _ptr(_vec(coef)), _ptr(st))
    if rc != OK:
        raise RuntimeError(f"orc_init failed: {rc}")
    return st


def kinetic_speed(p: Params, g: Grid, st: np.ndarray) -> float:
    return _lib().orc_kinetic_speed(ctypes.byref(p.c()), ctypes.byref(g.c()), _ptr(st))


def fill_equilibrium(p: Params, g: Grid, a: float, st: np.ndarray) -> None:
    _lib().orc_fill_equilibrium(ctypes.byref(p.c()), ctypes.byref(g.c()), a, _ptr(st))


def from_macroscopic(p: Params, g: Grid, u: np.ndarray) -> np.ndarray:
    """State with macroscopic field u (4, ny, nx) and equilibrium populations."""
    st = np.zeros((20, g.ny, g.nx))
    st[0:4] = u
    a = kinetic_speed(p, g, st)
    if not a > 0:
        raise ValueError("state not admissible")
    fill_equilibrium(p, g, a, st)
    return st


def step(p: Params, g: Grid, a: float, st: np.ndarray, theta_x=None, theta_y=None,
         diagnostics: bool = False):
    """One stream-collide step (eq:vlbm1-eq:vlbm5) with kinetic speed a.

    Returns (new_state, status) or, with diagnostics, (new_state, status,
    theta_x, theta_y, bounds) where bounds = (rho_min', rho_max', rho e_L)."""
    new = np.zeros_like(st)
    tx_in = None if theta_x is None else _vec(theta_x)
    ty_in = None if theta_y is None else _vec(theta_y)
    tx = np.zeros((g.ny, g.nx)) if diagnostics else None
    ty = np.zeros((g.ny, g.nx)) if diagnostics else None
    bd = np.zeros((3, g.ny, g.nx)) if diagnostics else None
    rc = _lib().orc_step(ctypes.byref(p.c()), ctypes.byref(g.c()), a, _ptr(st), _ptr(new),
                         _ptr(tx_in), _ptr(ty_in), _ptr(tx), _ptr(ty), _ptr(bd))
    if rc == ERR_ARG:
        raise ValueError("orc_step: bad arguments")
    if diagnostics:
        return new, rc, tx, ty, bd
    return new, rc


def run(p: Params, g: Grid, st: np.ndarray, t_final: float, max_steps: int = 1 << 40,
        t: float = 0.0):
    """Time loop of Sec. 2.3 (dt = dx / a_n).  Returns (state, t, steps, a_last, status)."""
    st = np.ascontiguousarray(st.copy())
    tt, ss, al = ctypes.c_double(t), ctypes.c_int64(0), ctypes.c_double(0.0)
    rc = _lib().orc_run(ctypes.byref(p.c()), ctypes.byref(g.c()), t_final, int(max_steps),
                        _ptr(st), ctypes.byref(tt), ctypes.byref(ss), ctypes.byref(al))
    return st, tt.value, ss.value, al.value, rc


def run_ensemble(p: Params, g: Grid, coefs: np.ndarray, t_final: float,
                 max_steps: int = 1 << 40, threads: int | None = None):
    """Independent realizations (one per row of coefs), each from eq:u0_def.

    The C loop releases the GIL, so realizations run concurrently on
    ``threads`` host threads.  Returns (states [M,20,ny,nx], t [M], steps [M],
    status [M])."""
    coefs = np.asarray(coefs, dtype=np.float64)
    M = coefs.shape[0]
    threads = threads or min(M, os.cpu_count() or 1)

    def one(m):
        st0 = init(p, g, coefs[m])
        return run(p, g, st0, t_final, max_steps)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(one, range(M)))
    states = np.stack([r[0] for r in res])
    return (states, np.array([r[1] for r in res]), np.array([r[2] for r in res]),
            np.array([r[4] for r in res]))


# --------------------------------------------------------------------------
# Ensemble statistics (Sec. 3.2 restriction, Sec. 3.4 observables)
# --------------------------------------------------------------------------

def moments(p: Params, u: np.ndarray):
    """Density, speed |v| and pressure (eq:eos) of macroscopic fields u[..., 4 vars, ny, nx]
    given as the leading 4 rows of the last three axes."""
    rho, m1, m2, E = u[..., 0, :, :], u[..., 1, :, :], u[..., 2, :, :], u[..., 3, :, :]
    v1 = m1 / rho
    v2 = m2 / rho
    pr = (p.gamma - 1.0) * (E - 0.5 * rho * (v1 * v1 + v2 * v2))
    speed = np.sqrt(v1 * v1 + v2 * v2)
    return rho, speed, pr


def restrict(field: np.ndarray, r: int) -> np.ndarray:
    """Conservative restriction of Sec. 3.2: each coarse cell is the average of
    the r x r fine nodes it contains (last two axes are y, x)."""
    *lead, ny, nx = field.shape
    if ny % r or nx % r:
        raise ValueError("grid not divisible by the restriction factor")
    blocks = field.reshape(*lead, ny // r, r, nx // r, r)
    return blocks.sum(axis=(-3, -1)) / (r * r)


def ensemble_mean(samples: np.ndarray) -> np.ndarray:
    """E_M of eq:mean: (1/M) sum over the realization axis 0."""
    return samples.sum(axis=0) / samples.shape[0]


def ensemble_std(samples: np.ndarray) -> np.ndarray:
    """Square root of the population variance used in eq:std (divide by M)."""
    mean = ensemble_mean(samples)
    return np.sqrt(((samples - mean) ** 2).sum(axis=0) / samples.shape[0])


def w1(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Per-cell one-point Wasserstein-1 of eq:w1disc between two equal-size
    empirical laws (realization axis 0): mean absolute difference of the
    ascending order statistics."""
    if a.shape != b.shape:
        raise ValueError("equal ensemble sizes and grids required")
    return np.abs(np.sort(a, axis=0) - np.sort(b, axis=0)).sum(axis=0) / a.shape[0]


# ---------------------------------------------------------------------------
# Observables of the convergence study (Sec. 3.3-3.4) and the centreline
# quantile diagnostics (Sec. 4, eq:empcdf, eq:widthratio).
# ---------------------------------------------------------------------------

def strong_error(coarse: np.ndarray, fine_r: np.ndarray) -> float:
    """E_strong of eq:strongError.  coarse[m], fine_r[m]: density of realization m
    on the common grid (the finer member already restricted); the relative L1
    difference of each realization, averaged over the M realizations.  The cell
    area of the L1 norms cancels in the ratio."""
    if coarse.shape != fine_r.shape:
        raise ValueError("same realizations and grid required")
    M = coarse.shape[0]
    total = 0.0
    for m in range(M):
        num = np.abs(coarse[m] - fine_r[m]).sum()
        den = np.abs(fine_r[m]).sum()
        total += num / den
    return total / M


def cell_mean_abs_diff(x: np.ndarray, y: np.ndarray) -> float:
    """(1/N_x) sum_k |x_k - y_k| over the cells of the common grid: eq:mean when
    x, y are the two ensemble-mean fields, eq:std when they are the two
    standard-deviation fields."""
    if x.shape != y.shape:
        raise ValueError("same grid required")
    return float(np.abs(x - y).sum() / x.size)


def w11(a: np.ndarray, b: np.ndarray) -> float:
    """W_{1,1} of eq:w1disc: the per-cell one-point W1 averaged over the cells."""
    d = w1(a, b)
    return float(d.sum() / d.size)


def empirical_quantile(samples: np.ndarray, pct: int) -> np.ndarray:
    """p_alpha of eq:empcdf, alpha = pct / 100 (integer percent in 1..100), per
    cell (axis 0 = realizations): the smallest xi with hat F(xi) >= alpha.
    hat F jumps only at sample values, so the infimum is a sample value; the
    test hat F(xi) >= alpha is made exactly as 100 * #{x_m <= xi} >= pct * M,
    with #{x_m <= s} counted by binary search in the sorted samples."""
    if not 1 <= pct <= 100:
        raise ValueError("pct must lie in 1..100")
    M = samples.shape[0]
    flat = samples.reshape(M, -1)
    out = np.empty(flat.shape[1])
    for c in range(flat.shape[1]):
        s = np.sort(flat[:, c])
        count = np.searchsorted(s, s, side="right")  # #{x_m <= s_(j)} for every j
        j = int(np.argmax(100 * count >= pct * M))     # first j meeting the test
        out[c] = s[j]
    return out.reshape(samples.shape[1:])


def width_ratio(samples: np.ndarray) -> np.ndarray:
    """Q of eq:widthratio: (p95 - p5) / (p84 - p16) per cell."""
    return (empirical_quantile(samples, 95) - empirical_quantile(samples, 5)) / \
        (empirical_quantile(samples, 84) - empirical_quantile(samples, 16))


def rate_fit(errors, dx) -> tuple[float, float]:
    """(r, c) of eq:ratefit: least-squares line log E = r log dx + c."""
    x = np.log(np.asarray(dx, dtype=np.float64))
    y = np.log(np.asarray(errors, dtype=np.float64))
    xm, ym = x.mean(), y.mean()
    r = float(((x - xm) * (y - ym)).sum() / ((x - xm) ** 2).sum())
    return r, float(ym - r * xm)


def cauchy_pairs(L: int):
    """eq:cauchy: (coarser level, finer level, level whose mesh width the error
    is associated with) for l = 1..L: levels l-1 and l, mesh width of l-1."""
    return [(l - 1, l, l - 1) for l in range(1, L + 1)]


def reference_pairs(L: int):
    """eq:ref: level l against the finest level L for l = 0..L-1, mesh width of l."""
    return [(l, L, l) for l in range(L)]


def subsample_indices(n: int, n_pd: int) -> np.ndarray:
    """Cell indices of the n_pd-point subsample of one direction of the common
    grid (Sec. 3.4, two-point construction): the cells containing the centres
    of n_pd equal intervals, floor((2k + 1) n / (2 n_pd)), k = 0..n_pd-1."""
    if not 1 <= n_pd <= n:
        raise ValueError("need 1 <= n_pd <= n")
    k = np.arange(n_pd)
    return (2 * k + 1) * n // (2 * n_pd)


def w1_2d(p: np.ndarray, q: np.ndarray) -> float:
    """First Wasserstein distance with Euclidean ground cost between two
    empirical laws of M points each in R^2 (rows of p and q), computed exactly
    as the optimal assignment (an LP whose optimum is a permutation)."""
    from scipy.optimize import linear_sum_assignment
    if p.shape != q.shape or p.shape[1] != 2:
        raise ValueError("two (M, 2) point sets required")
    cost = np.sqrt((p[:, None, 0] - q[None, :, 0]) ** 2 + (p[:, None, 1] - q[None, :, 1]) ** 2)
    rows, cols = linear_sum_assignment(cost)
    total = 0.0
    for i, j in zip(rows, cols):
        total += cost[i, j]
    return total / p.shape[0]


def w12(a: np.ndarray, b: np.ndarray, n_pd: int = 10):
    """W_{1,2} of eq:w2.  a, b: (M, ncy, ncx) density samples of the coarse and
    the restricted fine ensemble on the common grid.  Subsample n_pd points per
    direction (n_pd^2 cells), form for every ordered pair of retained cells
    (k, k') the joint law of (rho(x_k), rho(x_k')) over the ensemble, and average
    the 2-D W1 of the two laws over the P = n_pd^4 pairs.  Returns (mean,
    per-pair values in pair order k * n_pd^2 + k', cells in row-major order)."""
    M, ncy, ncx = a.shape
    jy, ix = subsample_indices(ncy, n_pd), subsample_indices(ncx, n_pd)
    cells = [(j, i) for j in jy for i in ix]
    vals = []
    for (j1, i1) in cells:
        for (j2, i2) in cells:
            p = np.stack([a[:, j1, i1], a[:, j2, i2]], axis=1)
            q = np.stack([b[:, j1, i1], b[:, j2, i2]], axis=1)
            vals.append(w1_2d(p, q))
    vals = np.array(vals)
    return float(vals.sum() / vals.size), vals
