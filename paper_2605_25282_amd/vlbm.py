"""Python binding of the C ABI in include/vlbm.h (libvlbm_hip.so, gfx950).

Argument marshalling only: every step of the method runs in the HIP kernels of
the library.  PyTorch provides device memory (``torch.empty(..., device="cuda")``)
and the HIP stream (``torch.cuda.current_stream().cuda_stream``).  Importing this
module does not need a GPU; loading the library fails loudly if it was not
built (see ``paper_2605_25282_amd.build``).
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvlbm_hip.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "vlbm.h")

OK, ERR_ARG, ERR_HIP, ERR_SIZE, ERR_NONPOSITIVE, ERR_NONFINITE, ERR_STATE = 0, -1, -2, -3, -4, -5, -6
BC = {"jet": 0, "periodic": 1, "neumann": 2}
LIMITER = {"limiter": 0, "zero": 1, "one": 2}
PRECISION = {"fp64": 0, "mixed": 1}


class VlbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"vlbm error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    """vlbm_params of include/vlbm.h, with the Mach-2000 jet defaults (Sec. 2.2)."""
    _fields_ = [("gamma", ctypes.c_double), ("alpha", ctypes.c_double),
                ("kappa", ctypes.c_double), ("rlmp_relax", ctypes.c_double),
                ("pos_eps", ctypes.c_double), ("rho_amb", ctypes.c_double),
                ("p_amb", ctypes.c_double), ("rho_jet", ctypes.c_double),
                ("v_jet", ctypes.c_double), ("r_jet", ctypes.c_double),
                ("kl_amp", ctypes.c_double), ("kl_modes", ctypes.c_int32),
                ("kl_decay", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("limiter", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    @classmethod
    def jet(cls, **kw) -> "Params":
        d = dict(gamma=5.0 / 3.0, alpha=1.0 / 3.0, kappa=1.0, rlmp_relax=0.1, pos_eps=1e-2,
                 rho_amb=0.5, p_amb=0.4127, rho_jet=5.0, v_jet=800.0, r_jet=0.05, kl_amp=0.1,
                 kl_modes=10, kl_decay=2, bc="jet", limiter="limiter", precision="fp64")
        d.update(kw)
        d["bc"] = BC[d["bc"]] if isinstance(d["bc"], str) else d["bc"]
        d["limiter"] = LIMITER[d["limiter"]] if isinstance(d["limiter"], str) else d["limiter"]
        d["precision"] = (PRECISION[d["precision"]] if isinstance(d["precision"], str)
                          else d["precision"])
        return cls(**d, reserved=0)


class Level(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("dx", ctypes.c_double),
                ("y_min", ctypes.c_double), ("state", ctypes.c_void_p * 2)]


_lib = None
_VP = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)


def header_functions() -> list[str]:
    """Names of the functions declared in include/vlbm.h."""
    txt = open(HEADER_PATH).read()
    return sorted(set(re.findall(r"^\s*(?:vlbm_status|const char \*)\s*(vlbm_\w+)\(", txt, re.M)))


def lib():
    """Load libvlbm_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2605_25282_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(Params)
        i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "vlbm_last_error": ([], ctypes.c_char_p),
            "vlbm_state_bytes": ([P, i32, i32, i32, ctypes.POINTER(ctypes.c_size_t)], i32),
            "vlbm_init_ensemble": ([P, ctypes.POINTER(Level), i32, _DP, i32, _VP,
                                    ctypes.POINTER(_VP)], i32),
            "vlbm_set_macroscopic": ([_VP, i32, _VP], i32),
            "vlbm_set_state": ([_VP, i32, _VP, _DP, ctypes.POINTER(i64), _DP], i32),
            "vlbm_step": ([_VP, dbl, i32, ctypes.POINTER(i32)], i32),
            "vlbm_times": ([_VP, i32, _DP, ctypes.POINTER(i64), _DP, ctypes.POINTER(i32)], i32),
            "vlbm_get_state": ([_VP, i32, _VP], i32),
            "vlbm_moments": ([_VP, i32, _VP, _VP, _VP], i32),
            "vlbm_ensemble_stats": ([_VP, i32, i32, _VP, i64, i64, _VP, i64, i64], i32),
            "vlbm_kl_coefficients": ([ctypes.c_uint64, i64, i32, i32, _DP], i32),
            "vlbm_stats_finalize": ([_VP, i64, i64, _VP, _VP, _VP], i32),
            "vlbm_sort_samples": ([_VP, i64, i32, _VP], i32),
            "vlbm_w1": ([_VP, _VP, i64, i32, _VP, _VP, _VP], i32),
            "vlbm_w1_noalloc": ([_VP, _VP, i64, i32, _VP, _VP, _VP], i32),
            "vlbm_strong_error": ([_VP, _VP, i64, i32, _VP, _VP, _VP], i32),
            "vlbm_mean_abs_diff": ([_VP, _VP, i64, _VP, _VP], i32),
            "vlbm_quantiles": ([_VP, i64, i32, ctypes.POINTER(i32), i32, _VP, _VP], i32),
            "vlbm_width_ratio": ([_VP, i64, i32, _VP, _VP], i32),
            "vlbm_rate_fit": ([_DP, _DP, i32, _DP, _DP], i32),
            "vlbm_w12": ([_VP, _VP, i32, i32, i32, i32, _VP, _VP, _VP], i32),
            "vlbm_tune": ([_VP, i32, i32], i32),
            "vlbm_set_tuning": ([_VP, ctypes.POINTER(i32), i32, i32, i32], i32),
            "vlbm_get_tuning": ([_VP, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                 ctypes.POINTER(i32)], i32),
            "vlbm_autotune": ([_VP, dbl, i32, ctypes.POINTER(i32)], i32),
            "vlbm_destroy": ([_VP], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def last_error() -> str:
    return lib().vlbm_last_error().decode()


def _check(rc: int) -> None:
    if rc != OK:
        raise VlbmError(rc, last_error())


def _ptr(t) -> _VP:
    """Device pointer of a torch tensor (or None)."""
    return None if t is None else _VP(t.data_ptr())


def _f64(t, numel: int, name: str) -> _VP:
    """Device pointer of a contiguous float64 CUDA tensor holding at least numel
    values (None passes through); anything else raises before the call."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name}: expected a CUDA tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name}: expected float64, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name}: needs {numel} values, tensor holds {t.numel()}")
    return _VP(t.data_ptr())


def _stream(stream=None) -> _VP:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return _VP(s.cuda_stream)


def vlbm_state_bytes(p: Params, nx: int, ny: int, n_real: int) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().vlbm_state_bytes(ctypes.byref(p), nx, ny, n_real, ctypes.byref(out)))
    return out.value


def vlbm_init_ensemble(p: Params, levels: list[Level], coeffs: np.ndarray | None, n_real: int,
                       stream=None) -> _VP:
    arr = (Level * len(levels))(*levels)
    c = None
    if coeffs is not None:
        coeffs = np.ascontiguousarray(coeffs, dtype=np.float64)
        c = coeffs.ctypes.data_as(_DP)
    h = _VP()
    _check(lib().vlbm_init_ensemble(ctypes.byref(p), arr, len(levels), c, n_real,
                                    _stream(stream), ctypes.byref(h)))
    return h


def vlbm_set_macroscopic(h, level: int, u) -> None:
    _check(lib().vlbm_set_macroscopic(h, level, _ptr(u)))


def vlbm_set_state(h, level: int, state, t, steps, a_last=None) -> None:
    tt = np.ascontiguousarray(t, dtype=np.float64)
    ss = np.ascontiguousarray(steps, dtype=np.int64)
    aa = None if a_last is None else np.ascontiguousarray(a_last, dtype=np.float64)
    _check(lib().vlbm_set_state(h, level, _ptr(state), tt.ctypes.data_as(_DP),
                                ss.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                None if aa is None else aa.ctypes.data_as(_DP)))


def vlbm_step(h, t_final: float, n_steps: int, want_done: bool = True):
    done = ctypes.c_int32(0)
    _check(lib().vlbm_step(h, t_final, n_steps, ctypes.byref(done) if want_done else None))
    return bool(done.value) if want_done else None


def vlbm_times(h, level: int, n_real: int):
    t = np.zeros(n_real)
    s = np.zeros(n_real, dtype=np.int64)
    a = np.zeros(n_real)
    st = np.zeros(n_real, dtype=np.int32)
    _check(lib().vlbm_times(h, level, t.ctypes.data_as(_DP),
                            s.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            a.ctypes.data_as(_DP),
                            st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return t, s, a, st


def vlbm_get_state(h, level: int, out) -> None:
    _check(lib().vlbm_get_state(h, level, _ptr(out)))


def vlbm_moments(h, level: int, rho=None, speed=None, p=None) -> None:
    _check(lib().vlbm_moments(h, level, _ptr(rho), _ptr(speed), _ptr(p)))


def vlbm_ensemble_stats(h, level: int, r: int, acc, n_prev: int, samples=None,
                        m_offset: int = 0) -> None:
    """acc: float64 [3][2][n_cells]; samples: float64 [rows][n_cells] (rows >=
    m_offset + n_real), n_cells = (nx/r)(ny/r) of the level."""
    if acc is None or acc.dim() < 1 or acc.numel() % 6:
        raise ValueError("acc must be a float64 tensor of 6 * n_cells values")
    cells = acc.numel() // 6
    rows = 0
    if samples is not None:
        if samples.numel() % cells:
            raise ValueError("samples must hold whole rows of n_cells values")
        rows = samples.numel() // cells
    _check(lib().vlbm_ensemble_stats(h, level, r, _f64(acc, 6 * cells, "acc"), cells, n_prev,
                                     _f64(samples, rows * cells, "samples"), rows, m_offset))


def vlbm_stats_finalize(acc, n_cells: int, n_total: int, mean=None, std=None, stream=None) -> None:
    """acc: float64 [3][2][n_cells] of n_total realizations; mean, std: float64
    [3][n_cells] (either may be None)."""
    _check(lib().vlbm_stats_finalize(_f64(acc, 6 * n_cells, "acc"), n_cells, n_total,
                                     _f64(mean, 3 * n_cells, "mean"), _f64(std, 3 * n_cells, "std"),
                                     _stream(stream)))


def vlbm_kl_coefficients(seed: int, first: int, count: int, modes: int = 10) -> np.ndarray:
    """KL coefficients of realizations first .. first+count-1, shape (count, 2 modes)."""
    out = np.zeros((count, 2 * modes))
    _check(lib().vlbm_kl_coefficients(seed & 0xFFFFFFFFFFFFFFFF, first, count, modes,
                                      out.ctypes.data_as(_DP)))
    return out


def vlbm_sort_samples(samples, n_cells: int, m: int, stream=None) -> None:
    _check(lib().vlbm_sort_samples(_f64(samples, n_cells * m, "samples"), n_cells, m, _stream(stream)))


def vlbm_w1(a, b, n_cells: int, m: int, w1_cell=None, w1_mean=None, stream=None) -> None:
    _check(lib().vlbm_w1(_f64(a, n_cells * m, "a"), _f64(b, n_cells * m, "b"), n_cells, m,
                         _f64(w1_cell, n_cells, "w1_cell"), _f64(w1_mean, 1, "w1_mean"),
                         _stream(stream)))


def vlbm_w1_noalloc(a, b, n_cells: int, m: int, w1_cell=None, w1_mean=None, stream=None) -> None:
    """vlbm_w1 with the library's fixed per-device workspace (no device allocation)."""
    _check(lib().vlbm_w1_noalloc(_f64(a, n_cells * m, "a"), _f64(b, n_cells * m, "b"), n_cells, m,
                                 _f64(w1_cell, n_cells, "w1_cell"), _f64(w1_mean, 1, "w1_mean"),
                                 _stream(stream)))


def vlbm_strong_error(a, b, n_cells: int, m: int, per_real, out, stream=None) -> None:
    _check(lib().vlbm_strong_error(_f64(a, n_cells * m, "a"), _f64(b, n_cells * m, "b"), n_cells, m,
                                   _f64(per_real, m, "per_real"), _f64(out, 1, "out"), _stream(stream)))


def vlbm_mean_abs_diff(x, y, n: int, out, stream=None) -> None:
    _check(lib().vlbm_mean_abs_diff(_f64(x, n, "x"), _f64(y, n, "y"), n, _f64(out, 1, "out"),
                                    _stream(stream)))


def vlbm_quantiles(sorted_samples, n_cells: int, m: int, pct, out, stream=None) -> None:
    pc = (ctypes.c_int32 * len(pct))(*[int(x) for x in pct])
    _check(lib().vlbm_quantiles(_f64(sorted_samples, n_cells * m, "sorted"), n_cells, m, pc, len(pct),
                                _f64(out, len(pct) * n_cells, "out"), _stream(stream)))


def vlbm_width_ratio(sorted_samples, n_cells: int, m: int, q, stream=None) -> None:
    _check(lib().vlbm_width_ratio(_f64(sorted_samples, n_cells * m, "sorted"), n_cells, m,
                                  _f64(q, n_cells, "q"), _stream(stream)))


def vlbm_w12(a, b, ncx: int, ncy: int, m: int, n_pd: int, w_pair, w_mean=None, stream=None) -> None:
    cells = ncx * ncy
    _check(lib().vlbm_w12(_f64(a, cells * m, "a"), _f64(b, cells * m, "b"), ncx, ncy, m, n_pd,
                          _f64(w_pair, n_pd ** 4, "w_pair"), _f64(w_mean, 1, "w_mean"), _stream(stream)))


def vlbm_rate_fit(errors, dx) -> tuple[float, float]:
    e = np.ascontiguousarray(errors, dtype=np.float64)
    d = np.ascontiguousarray(dx, dtype=np.float64)
    if e.shape != d.shape:
        raise ValueError("errors and dx must have the same length")
    r, c = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(lib().vlbm_rate_fit(e.ctypes.data_as(_DP), d.ctypes.data_as(_DP), len(e),
                               ctypes.byref(r), ctypes.byref(c)))
    return r.value, c.value


KERNEL = {"reference": 0, "march": 1, "reference-eager": 0x100, "march-eager": 0x101}


def vlbm_tune(h, kernel: str | int = "march", chunk_rows: int = 0) -> None:
    k = KERNEL[kernel] if isinstance(kernel, str) else kernel
    _check(lib().vlbm_tune(h, k, chunk_rows))


def vlbm_set_tuning(h, chunks, waves_per_block: int = 4, item_order: int = 0, dealing: int = 0) -> None:
    """chunks: rows per work item of every level (0 = default), or None for all defaults."""
    c = None if chunks is None else (ctypes.c_int32 * len(chunks))(*[int(x) for x in chunks])
    _check(lib().vlbm_set_tuning(h, c, waves_per_block, item_order, dealing))


def vlbm_get_tuning(h, n_levels: int) -> tuple[list[int], int, int, int]:
    """(chunk height of every level, waves per block, item order, dealing) in use."""
    c = (ctypes.c_int32 * n_levels)()
    w, o, d = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib().vlbm_get_tuning(h, c, ctypes.byref(w), ctypes.byref(o), ctypes.byref(d)))
    return list(c), w.value, o.value, d.value


def vlbm_autotune(h, t_final: float, steps_per_candidate: int, n_levels: int) -> list[int]:
    out = (ctypes.c_int32 * n_levels)()
    _check(lib().vlbm_autotune(h, t_final, steps_per_candidate, out))
    return list(out)


def vlbm_destroy(h) -> None:
    _check(lib().vlbm_destroy(h))


class Ensemble:
    """Convenience owner of the device buffers of one ensemble (torch tensors).

    levels: list of (nx, ny, dx, y_min).  The state buffers are allocated here
    with torch and handed to the library; everything else is a direct call of
    the C ABI."""

    def __init__(self, params: Params, levels, coeffs, n_real: int, stream=None):
        import torch
        self.params, self.n_real = params, n_real
        self.shapes = [(int(nx), int(ny)) for (nx, ny, _, _) in levels]
        self.buffers = []
        lv = []
        for (nx, ny, dx, y_min) in levels:
            nbytes = vlbm_state_bytes(params, int(nx), int(ny), n_real)
            bufs = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(2)]
            self.buffers.append(bufs)
            lv.append(Level(int(nx), int(ny), float(dx), float(y_min),
                            (_VP * 2)(bufs[0].data_ptr(), bufs[1].data_ptr())))
        self.h = vlbm_init_ensemble(params, lv, coeffs, n_real, stream)

    def close(self) -> None:
        if self.h is not None:
            vlbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tune(self, kernel: str | int = "march", chunk_rows: int = 0) -> None:
        vlbm_tune(self.h, kernel, chunk_rows)

    def autotune(self, t_final: float, steps_per_candidate: int = 4) -> list[int]:
        return vlbm_autotune(self.h, t_final, steps_per_candidate, len(self.shapes))

    def set_tuning(self, chunks=None, waves_per_block: int = 4, item_order: int = 0, dealing: int = 0) -> None:
        vlbm_set_tuning(self.h, chunks, waves_per_block, item_order, dealing)

    def get_tuning(self) -> tuple[list[int], int, int, int]:
        return vlbm_get_tuning(self.h, len(self.shapes))

    def step(self, t_final: float, n_steps: int, want_done: bool = True):
        return vlbm_step(self.h, t_final, n_steps, want_done)

    def run(self, t_final: float, chunk: int = 64, max_steps: int = 1 << 30) -> int:
        """Step until every realization has reached t_final; returns launches made."""
        n = 0
        while n < max_steps:
            k = min(chunk, max_steps - n)
            done = self.step(t_final, k)
            n += k
            if done:
                break
        return n

    def times(self, level: int = 0):
        return vlbm_times(self.h, level, self.n_real)

    def state(self, level: int = 0):
        """Current state as a float64 tensor [4 var][5 slot][R][ny][nx]."""
        import torch
        nx, ny = self.shapes[level]
        out = torch.empty((4, 5, self.n_real, ny, nx), dtype=torch.float64, device="cuda")
        vlbm_get_state(self.h, level, out)
        return out

    def set_macroscopic(self, level: int, u) -> None:
        vlbm_set_macroscopic(self.h, level, u)

    def set_state(self, level: int, state, t, steps, a_last=None) -> None:
        vlbm_set_state(self.h, level, state, t, steps, a_last)

    def moments(self, level: int = 0):
        import torch
        nx, ny = self.shapes[level]
        out = [torch.empty((self.n_real, ny, nx), dtype=torch.float64, device="cuda")
               for _ in range(3)]
        vlbm_moments(self.h, level, *out)
        return out
