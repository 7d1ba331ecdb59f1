"""GPU parity at the study's full configuration sizes, in the launch
configuration the benchmark uses (one persistent launch per step over all
levels, graph replays), on realizations the oracle recomputes one by one, plus
the batch-streamed statistics used for ensembles larger than one batch.

FP64 bar: per (variable, slot) plane, max |gpu - oracle| / max |oracle| <=
1e-11 (the path is bitwise, so the observed difference is 0)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O
from paper_2605_25282_amd import inputs, vlbm

TOL = 1e-11


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    vlbm.lib()
    yield
    torch.cuda.synchronize()


def _plane_err(mine, ref):
    worst = 0.0
    for k in range(20):
        d = np.abs(mine[k] - ref[k]).max()
        den = np.abs(ref[k]).max()
        if den == 0.0:
            den = np.abs(ref[(k // 4) * 4 + 3]).max()
        worst = max(worst, d / den)
    return worst


def _picked(ens, level, picks):
    """Realizations `picks` of a level in the oracle's layout (20, ny, nx)."""
    st = ens.state(level)
    out = {}
    for m in picks:
        s = st[:, :, m].cpu().numpy()
        out[m] = s.transpose(1, 0, 2, 3).reshape(20, s.shape[2], s.shape[3])
    del st
    torch.cuda.empty_cache()
    return out


def _oracle(p, grid, coefs, steps, picks):
    sub = np.stack([coefs[m] for m in picks])
    states, t, n, status = O.run_ensemble(p, grid, sub, 1e30, max_steps=steps, threads=len(picks))
    assert np.all(status == O.OK) and np.all(n == steps)
    return {m: states[i] for i, m in enumerate(picks)}


def test_three_levels_full_size():
    """320 x 160, 640 x 320 and 1280 x 640 with 128 realizations each (same seeds),
    40 steps of one launch per step (graph replays); first and last realization
    of every level against the oracle."""
    R, steps = 128, 40
    shapes = [(320, 160), (640, 320), (1280, 640)]
    levels = [(nx, ny, 1.0 / nx, -0.25) for nx, ny in shapes]
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, R)
    ens = vlbm.Ensemble(vlbm.Params.jet(), levels, coefs, R)
    ens.step(1e30, steps)
    picks = (0, R - 1)
    got = {}
    for l in range(3):
        t, s, a, status = ens.times(l)
        assert np.all(s == steps) and np.all(status == 0)
        got[l] = _picked(ens, l, picks)
    ens.close()
    p = O.Params()
    for l, (nx, ny, dx, y0) in enumerate(levels):
        ref = _oracle(p, O.Grid(nx, ny, dx, y0), coefs, steps, picks)
        for m in picks:
            assert _plane_err(got[l][m], ref[m]) <= TOL, (l, m)


def test_jet1280_mixed_full_ensemble():
    """1280 x 640 with 256 realizations in mixed storage, 30 steps; first and last
    realization against the oracle's mixed storage mode."""
    w = inputs.WORKLOADS["jet1280"]
    steps = 30
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, w.m)
    ens = vlbm.Ensemble(vlbm.Params.jet(precision="mixed"), [(w.nx, w.ny, w.dx, w.y_min)], coefs, w.m)
    ens.step(1e30, steps)
    picks = (0, w.m - 1)
    got = _picked(ens, 0, picks)
    ens.close()
    ref = _oracle(O.Params(storage="mixed"), O.Grid(w.nx, w.ny, w.dx, w.y_min), coefs, steps, picks)
    for m in picks:
        assert _plane_err(got[m], ref[m]) <= TOL, m


def test_largest_level_two_realizations():
    """5056 x 2528 (12.8 M nodes, the study's finest level): a realization's
    state is 2.2 GB, so realization 1 starts beyond 4 GiB of the buffer; 4 steps
    of both against the oracle."""
    w = inputs.WORKLOADS["jet5056"]
    R, steps = 2, 4
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, R)
    ens = vlbm.Ensemble(vlbm.Params.jet(), [(w.nx, w.ny, w.dx, w.y_min)], coefs, R)
    assert vlbm.vlbm_state_bytes(vlbm.Params.jet(), w.nx, w.ny, 1) > 2 ** 31
    ens.step(1e30, steps)
    got = _picked(ens, 0, (0, 1))
    ens.close()
    ref = _oracle(O.Params(), O.Grid(w.nx, w.ny, w.dx, w.y_min), coefs, steps, (0, 1))
    for m in (0, 1):
        assert _plane_err(got[m], ref[m]) <= TOL, m


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_headline_pair_against_the_oracle(precision):
    """The benchmark's launch: the 5056x2528 level and its 2528x1264 partner on
    the same seeds, both advanced by one launch per step (graph replays), in
    either storage; 2 realizations, 4 steps, every plane of both levels against
    the oracle in the same storage (the mixed path rounds the same planes to
    binary32 at the same points, so it is bitwise too)."""
    fine = inputs.WORKLOADS["jet5056"]
    works = [(fine.nx // 2, fine.ny // 2), (fine.nx, fine.ny)]
    levels = [(nx, ny, 1.0 / nx, -0.25) for nx, ny in works]
    R, steps = 2, 4
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, R)
    ens = vlbm.Ensemble(vlbm.Params.jet(precision=precision), levels, coefs, R)
    ens.step(1e30, steps)
    got = [_picked(ens, l, (0, 1)) for l in range(2)]
    ens.close()
    for l, (nx, ny, dx, y_min) in enumerate(levels):
        ref = _oracle(O.Params(storage=precision), O.Grid(nx, ny, dx, y_min), coefs, steps, (0, 1))
        for m in (0, 1):
            assert _plane_err(got[l][m], ref[m]) <= TOL, (precision, l, m)


@pytest.mark.parametrize("precision,decomposition", [("fp64", ([33, 32], 4, 0, 1)),
                                                      ("mixed", ([64, 64], 4, 0, 1))])
def test_headline_batch_sampled_against_the_oracle(precision, decomposition):
    """The benchmark's whole launch: a batch of 45 realizations of the
    5056x2528 + 2528x1264 pair (about 250 GB of state in FP64) at the
    decomposition the default line tuned to, 4 steps; the density, speed and
    pressure of realizations 0, 22 and 44 (the last one beyond 96 GB into the
    fine level's buffer) of both levels equal the oracle's bit for bit."""
    fine = inputs.WORKLOADS["jet5056"]
    works = [(fine.nx // 2, fine.ny // 2), (fine.nx, fine.ny)]
    levels = [(nx, ny, 1.0 / nx, -0.25) for nx, ny in works]
    R, steps, picks = 45, 4, (0, 22, 44)
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, R)
    torch.cuda.empty_cache()  # the batch takes most of HBM: start from an empty cache
    ens = vlbm.Ensemble(vlbm.Params.jet(precision=precision), levels, coefs, R)
    ens.set_tuning(*decomposition)
    ens.step(1e30, steps)
    got = []
    for l in range(2):
        t, s, a, status = ens.times(l)
        assert np.all(s == steps) and np.all(status == 0)
        mom = ens.moments(l)
        got.append({m: [f[m].cpu().numpy() for f in mom] for m in picks})
        del mom
    ens.close()
    del ens
    torch.cuda.empty_cache()
    p = O.Params(storage=precision)
    for l, (nx, ny, dx, y_min) in enumerate(levels):
        ref = _oracle(p, O.Grid(nx, ny, dx, y_min), coefs, steps, picks)
        for m in picks:
            want = O.moments(p, ref[m][0:4])
            for f in range(3):
                assert np.array_equal(got[l][m][f], want[f]), (precision, l, m, f)


def test_headline_pair_is_independent_of_the_decomposition():
    """The benchmark's 5056x2528 + 2528x1264 pair (8 realizations here), 30
    steps of one launch per step under the work-queue dealing with the default
    items, the static round-robin dealing with 632-row items, and the work
    queues with the tuned 33 / 32-row items on blocks of one wavefront: the
    states of both levels are equal bit for bit (compared on the device)."""
    fine = inputs.WORKLOADS["jet5056"]
    works = [(fine.nx // 2, fine.ny // 2), (fine.nx, fine.ny)]
    levels = [(nx, ny, 1.0 / nx, -0.25) for nx, ny in works]
    R, steps = 8, 30
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, R)
    ref = None
    for chunks, wpb, order, deal in ((None, 4, 0, 1), ([632, 632], 4, 0, 0), ([33, 32], 1, 0, 1)):
        ens = vlbm.Ensemble(vlbm.Params.jet(), levels, coefs, R)
        ens.set_tuning(chunks, wpb, order, deal)
        ens.step(1e30, steps)
        for l in range(2):
            t, s, a, status = ens.times(l)
            assert np.all(s == steps) and np.all(status == 0)
        states = [ens.state(l) for l in range(2)]
        ens.close()
        del ens
        if ref is None:
            ref = states
        else:
            for l in range(2):
                assert torch.equal(states[l], ref[l]), (chunks, wpb, order, deal, l)
        del states
        torch.cuda.empty_cache()


def test_batched_statistics_equal_one_batch():
    """An ensemble streamed in two batches (accumulators merged with n_prev,
    samples scattered at m_offset) gives the statistics of the whole ensemble
    run at once: the same sample store bit for bit, mean and std within 1e-12."""
    w = inputs.WORKLOADS["jet128"]
    M, r = 16, 2
    level = [(w.nx, w.ny, w.dx, w.y_min)]
    ncell = (w.nx // r) * (w.ny // r)
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, M)

    def run(first, count):
        e = vlbm.Ensemble(vlbm.Params.jet(), level, coefs[first:first + count], count)
        e.run(w.t_final, chunk=64)
        return e

    acc1 = torch.empty((3, 2, ncell), dtype=torch.float64, device="cuda")
    smp1 = torch.empty((M, ncell), dtype=torch.float64, device="cuda")
    e = run(0, M)
    vlbm.vlbm_ensemble_stats(e.h, 0, r, acc1, 0, smp1, 0)
    e.close()
    acc2 = torch.empty_like(acc1)
    smp2 = torch.full_like(smp1, -1.0)
    for first in (0, M // 2):
        e = run(first, M // 2)
        vlbm.vlbm_ensemble_stats(e.h, 0, r, acc2, first, smp2, first)
        e.close()
    out = []
    for acc in (acc1, acc2):
        mean = torch.empty((3, ncell), dtype=torch.float64, device="cuda")
        std = torch.empty_like(mean)
        vlbm.vlbm_stats_finalize(acc, ncell, M, mean, std)
        out.append((mean.cpu().numpy(), std.cpu().numpy()))
    torch.cuda.synchronize()
    assert np.array_equal(smp1.cpu().numpy(), smp2.cpu().numpy())
    for f in range(3):
        assert np.allclose(out[1][0][f], out[0][0][f], rtol=1e-12, atol=0)
        assert np.allclose(out[1][1][f], out[0][1][f], rtol=1e-10, atol=1e-14 * np.abs(out[0][0][f]).max())
    # and both equal the oracle's statistics of the restricted samples
    samples = smp1.cpu().numpy().reshape(M, w.ny // r, w.nx // r)
    assert np.allclose(out[0][0][0], O.ensemble_mean(samples).ravel(), rtol=1e-12, atol=0)
