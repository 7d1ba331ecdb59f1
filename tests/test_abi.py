"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/vlbm.h declares, and rejects invalid arguments before
touching the device."""
import ctypes

import numpy as np
import pytest

from paper_2605_25282_amd import vlbm


@pytest.fixture(scope="module")
def lib():
    return vlbm.lib()


def test_header_declares_the_boundary():
    names = vlbm.header_functions()
    for required in ("vlbm_init_ensemble", "vlbm_step", "vlbm_moments", "vlbm_ensemble_stats",
                     "vlbm_last_error", "vlbm_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in vlbm.header_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_wraps_every_declared_function(lib):
    """The Python binding carries every declared function under the same name
    (with the signature table entry the loader sets), so a caller never reaches
    an unwrapped entry point; vlbm_last_error is wrapped as last_error."""
    import inspect
    src = inspect.getsource(vlbm.lib)
    for n in vlbm.header_functions():
        assert f'"{n}"' in src, f"{n} has no signature entry"
        if n != "vlbm_last_error":
            assert callable(getattr(vlbm, n, None)), f"{n} has no wrapper"


def _slots(nx, periodic=False):
    """Element slots of a plane row: 64 per strip of 60 columns (a bounded level
    of 60 q + 1 columns keeps q strips, the last one carrying 61 columns)."""
    q = (nx - 1) // 60 if (not periodic and (nx - 1) % 60 == 0) else -(-nx // 60)
    return 64 * q


def test_state_bytes(lib):
    p = vlbm.Params.jet()
    assert _slots(128) == 192 and _slots(121) == 128 and _slots(121, True) == 192 and _slots(640) == 704
    assert vlbm.vlbm_state_bytes(p, 128, 64, 8) == 8 * 64 * _slots(128) * 160
    assert vlbm.vlbm_state_bytes(p, 121, 37, 3) == 3 * 37 * _slots(121) * 160
    pp = vlbm.Params.jet(bc="periodic", kl_modes=0)
    assert vlbm.vlbm_state_bytes(pp, 121, 37, 3) == 3 * 37 * _slots(121, True) * 160
    pm = vlbm.Params.jet(precision="mixed")
    # 8 FP64 planes (u, E of the populations) and 12 FP32 planes: 112 B per slot
    assert vlbm.vlbm_state_bytes(pm, 128, 64, 8) == 8 * 64 * _slots(128) * (8 * 8 + 12 * 4)


@pytest.mark.parametrize("field,value", [("gamma", 1.0), ("alpha", 1.0), ("alpha", -0.1),
                                         ("kappa", 0.5), ("pos_eps", 1.0), ("rho_amb", 0.0),
                                         ("kl_modes", 65), ("kl_decay", -1), ("bc", 7),
                                         ("limiter", 9), ("precision", 3), ("reserved", 1)])
def test_invalid_params_rejected(lib, field, value):
    p = vlbm.Params.jet()
    setattr(p, field, value)
    with pytest.raises(vlbm.VlbmError) as ei:
        vlbm.vlbm_state_bytes(p, 16, 16, 1)
    assert ei.value.code == vlbm.ERR_ARG
    assert field.split("_")[0] in vlbm.last_error() or field == "reserved" or "jet constants" in vlbm.last_error()


@pytest.mark.parametrize("nx,ny,R", [(2, 16, 1), (16, 2, 1), (16, 16, 0), (16, 16, 70000)])
def test_invalid_sizes_rejected(lib, nx, ny, R):
    with pytest.raises(vlbm.VlbmError) as ei:
        vlbm.vlbm_state_bytes(vlbm.Params.jet(), nx, ny, R)
    assert ei.value.code == vlbm.ERR_SIZE


def test_realization_state_limit(lib):
    """Kernels address one realization's state with 32-bit byte offsets: a level
    whose realization needs 4 GiB or more is refused up front; the mixed layout
    (112 B per node instead of 160) admits larger levels."""
    with pytest.raises(vlbm.VlbmError) as ei:
        vlbm.vlbm_state_bytes(vlbm.Params.jet(), 6000, 5000, 1)
    assert ei.value.code == vlbm.ERR_SIZE and "4 GiB" in vlbm.last_error()
    assert vlbm.vlbm_state_bytes(vlbm.Params.jet(precision="mixed"), 6000, 5000, 1) == 112 * _slots(6000) * 5000
    # the largest configuration of the study (5056 x 2528) fits in FP64
    assert vlbm.vlbm_state_bytes(vlbm.Params.jet(), 5056, 2528, 2) == 2 * 160 * _slots(5056) * 2528


def test_init_rejects_before_any_device_work(lib):
    """Validation happens before any HIP call, so these run without a GPU."""
    p = vlbm.Params.jet()
    lv = vlbm.Level(16, 16, 0.1, 0.0, (ctypes.c_void_p * 2)(None, None))
    coefs = np.zeros((1, 20))
    with pytest.raises(vlbm.VlbmError) as ei:
        vlbm.vlbm_init_ensemble(p, [lv], coefs, 1, stream=type("S", (), {"cuda_stream": 0})())
    assert ei.value.code == vlbm.ERR_ARG and "state" in vlbm.last_error()
    lv = vlbm.Level(16, 16, 0.1, 0.0, (ctypes.c_void_p * 2)(4096, 8192))
    bad = np.full((1, 20), 1.5)
    with pytest.raises(vlbm.VlbmError) as ei:
        vlbm.vlbm_init_ensemble(p, [lv], bad, 1, stream=type("S", (), {"cuda_stream": 0})())
    assert ei.value.code == vlbm.ERR_ARG and "outside" in vlbm.last_error()
    lv = vlbm.Level(16, 16, -0.1, 0.0, (ctypes.c_void_p * 2)(4096, 8192))
    with pytest.raises(vlbm.VlbmError):
        vlbm.vlbm_init_ensemble(p, [lv], coefs, 1, stream=type("S", (), {"cuda_stream": 0})())


def test_null_handles_rejected(lib):
    assert lib.vlbm_step(None, 1.0, 1, None) == vlbm.ERR_ARG
    assert lib.vlbm_set_state(None, 0, None, None, None, None) == vlbm.ERR_ARG
    assert lib.vlbm_moments(None, 0, None, None, None) == vlbm.ERR_ARG
    assert lib.vlbm_ensemble_stats(None, 0, 1, None, 0, 0, None, 0, 0) == vlbm.ERR_ARG
    assert lib.vlbm_sort_samples(None, 1, 1, None) == vlbm.ERR_ARG
    assert lib.vlbm_w1(None, None, 1, 1, None, None, None) == vlbm.ERR_ARG
    assert lib.vlbm_stats_finalize(None, 1, 1, None, None, None) == vlbm.ERR_ARG
    assert lib.vlbm_destroy(None) == vlbm.OK


def test_rate_fit_reproduces_the_printed_tables(lib):
    """The library's eq:ratefit (host arithmetic) reproduces every rate printed in
    Tables 1-7 from the printed per-pair errors, and equals the oracle's fit."""
    import os
    import oracle as O
    golden = os.path.join(os.path.dirname(__file__), "golden", "convergence_tables.txt")
    blocks = {}
    for line in open(golden):
        if line.startswith("#") or not line.strip():
            continue
        t, proto, kind, a_, b_, *vals = line.split()
        pairs, rates = blocks.setdefault((t, proto), ([], None))
        if kind == "pair":
            pairs.append((int(a_), [float(v) for v in vals]))
        else:
            blocks[(t, proto)] = (pairs, [float(v) for v in vals])
    n = 0
    for (t, proto), (pairs, rates) in blocks.items():
        dx = [2.5 / nx for nx, _ in pairs]
        for k in range(5):
            errs = [v[k] for _, v in pairs]
            r, c = vlbm.vlbm_rate_fit(errs, dx)
            assert abs(r - rates[k]) <= 1.5e-3, (t, proto, k, r, rates[k])
            ro, co = O.rate_fit(errs, dx)
            assert r == pytest.approx(ro, rel=1e-14, abs=1e-15) and c == pytest.approx(co, rel=1e-14)
            n += 1
    assert n == 70


def test_rate_fit_rejects_bad_input(lib):
    for errs, dx in [([1.0], [0.1]), ([1.0, -1.0], [0.1, 0.05]), ([1.0, 2.0], [0.1, 0.1]),
                     ([1.0, float("nan")], [0.1, 0.05]), ([1.0, 2.0], [0.0, 0.05])]:
        with pytest.raises(vlbm.VlbmError):
            vlbm.vlbm_rate_fit(errs, dx)


def test_observable_entry_points_validate_before_launch(lib):
    """Bad arguments are refused before anything touches a device."""
    fake = ctypes.c_void_p(4096)
    i32 = ctypes.c_int32
    assert lib.vlbm_strong_error(None, fake, 10, 2, fake, fake, None) == vlbm.ERR_ARG
    assert lib.vlbm_strong_error(fake, fake, 10, 2, None, fake, None) == vlbm.ERR_ARG
    assert lib.vlbm_strong_error(fake, fake, 0, 2, fake, fake, None) == vlbm.ERR_SIZE
    assert lib.vlbm_mean_abs_diff(None, None, 10, fake, None) == vlbm.ERR_ARG
    assert lib.vlbm_mean_abs_diff(fake, None, 0, fake, None) == vlbm.ERR_SIZE
    pct = (i32 * 3)(5, 50, 101)
    assert lib.vlbm_quantiles(fake, 10, 4, pct, 3, fake, None) == vlbm.ERR_ARG
    assert "101" in vlbm.last_error()
    pct = (i32 * 9)(*([50] * 9))
    assert lib.vlbm_quantiles(fake, 10, 4, pct, 9, fake, None) == vlbm.ERR_ARG
    assert lib.vlbm_quantiles(fake, 0, 4, pct, 1, fake, None) == vlbm.ERR_SIZE
    assert lib.vlbm_width_ratio(fake, 10, 0, fake, None) == vlbm.ERR_SIZE
    assert lib.vlbm_w1(fake, fake, 0, 4, None, fake, None) == vlbm.ERR_SIZE
    assert lib.vlbm_w1(fake, fake, 10, 0, fake, fake, None) == vlbm.ERR_SIZE
    assert lib.vlbm_w1_noalloc(None, fake, 10, 4, fake, fake, None) == vlbm.ERR_ARG
    assert lib.vlbm_w1_noalloc(fake, fake, 0, 4, None, fake, None) == vlbm.ERR_SIZE
    # the fixed workspace holds VLBM_W1_NOALLOC_MAX_PARTIALS partial sums of 1024 cells
    limit = 16384 * 1024
    assert lib.vlbm_w1_noalloc(fake, fake, limit + 1, 4, None, fake, None) == vlbm.ERR_SIZE
    assert "16384" in vlbm.last_error()
    assert lib.vlbm_w12(None, fake, 10, 10, 4, 3, fake, None, None) == vlbm.ERR_ARG
    assert lib.vlbm_w12(fake, fake, 10, 10, 4, 3, None, None, None) == vlbm.ERR_ARG
    assert lib.vlbm_w12(fake, fake, 10, 10, 1025, 3, fake, None, None) == vlbm.ERR_SIZE
    assert lib.vlbm_w12(fake, fake, 10, 10, 0, 3, fake, None, None) == vlbm.ERR_SIZE
    assert lib.vlbm_w12(fake, fake, 10, 2, 4, 3, fake, None, None) == vlbm.ERR_ARG  # n_pd > ncy
    assert lib.vlbm_w12(fake, fake, 10, 10, 4, 0, fake, None, None) == vlbm.ERR_ARG


# SplitMix64 test vector: the first five outputs of the generator seeded with
# 1234567, as published with the reference implementation of Steele, Lea and
# Flood's generator (the splitmix64.c that accompanies xoshiro).
_SPLITMIX64_1234567 = [6457827717110365317, 3203168211198807973, 9817491932198370423,
                       4593380528125082431, 16408922859458223821]


def test_kl_coefficients_follow_the_published_generator(lib):
    """vlbm_kl_coefficients draws coefficient c of realization m from output
    m * 2K + c of SplitMix64: its first values for seed 1234567 are the published
    outputs mapped to [-1, 1) by their top 53 bits."""
    got = vlbm.vlbm_kl_coefficients(1234567, 0, 1, modes=3)[0]
    want = [2.0 * ((z >> 11) / 2.0 ** 53) - 1.0 for z in _SPLITMIX64_1234567]
    assert list(got[:5]) == want
    # output n of realization m sits at column n - m * 2K
    got2 = vlbm.vlbm_kl_coefficients(1234567, 1, 1, modes=2)[0]
    assert got2[0] == want[4]


def test_kl_coefficients_nested_and_equal_to_the_input_generator(lib):
    """(seed, m) fixes realization m's draw whatever the batch (Sec. 3.1's nested
    sample sets), and the library's draws are those of the seeded input module."""
    from paper_2605_25282_amd import inputs
    full = vlbm.vlbm_kl_coefficients(inputs.DEFAULT_SEED, 0, 40)
    part = vlbm.vlbm_kl_coefficients(inputs.DEFAULT_SEED, 17, 9)
    assert np.array_equal(full[17:26], part)
    assert np.array_equal(full, inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, 40))
    assert np.all(full >= -1.0) and np.all(full < 1.0)
    assert lib.vlbm_kl_coefficients(1, 0, 1, 65, ctypes.cast(ctypes.c_void_p(4096), ctypes.POINTER(ctypes.c_double))) == vlbm.ERR_ARG
    assert lib.vlbm_kl_coefficients(1, -1, 1, 2, None) == vlbm.ERR_ARG


def test_binding_refuses_tensors_that_do_not_fit():
    """The binding checks dtype, device, contiguity and size before it hands a
    pointer to the library (a float32 or short buffer would otherwise be written
    out of bounds by the device)."""
    torch = pytest.importorskip("torch")
    with pytest.raises(TypeError):
        vlbm._f64(torch.zeros(10, dtype=torch.float64), 10, "x")  # host tensor
    if torch.cuda.is_available():
        with pytest.raises(TypeError):
            vlbm._f64(torch.zeros(10, dtype=torch.float32, device="cuda"), 10, "x")
        with pytest.raises(ValueError):
            vlbm._f64(torch.zeros(9, dtype=torch.float64, device="cuda"), 10, "x")
        with pytest.raises(ValueError):
            vlbm._f64(torch.zeros((4, 4), dtype=torch.float64, device="cuda").t(), 16, "x")
