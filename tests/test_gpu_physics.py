"""The jet as the paper describes it (Sec. 2.2 and Sec. 4), on the HIP path:
qualitative numbers the paper prints, checked on seeded ensembles.

* The bow shock advances at the empirical jet-head velocity 666.7 (tracked on
  the axis; tolerance 10%, the paper gives no error bar).
* Upstream of the head the laminar core carries the inlet randomness without
  amplifying it: on the axis the ensemble mean density is the injected 5 and
  the standard deviation the inlet measure's A rho_jet (sum_k k^-4 / 3)^(1/2)
  = 0.30 (tolerance for 32 realizations: 25%).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2605_25282_amd import inputs, vlbm

V_HEAD = 666.7
SIGMA_AXIS = 0.1 * 5.0 * np.sqrt(sum(k ** -4.0 for k in range(1, 11)) / 3.0)


@pytest.fixture(scope="module")
def axis_profiles():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = inputs.WORKLOADS["jet640"]
    M = 32
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, M)
    ens = vlbm.Ensemble(vlbm.Params.jet(), [(w.nx, w.ny, w.dx, w.y_min)], coefs, M)
    out = {}
    for t in (4e-4, 1e-3):
        ens.run(t, chunk=120)
        tt, s, a, status = ens.times(0)
        assert np.all(status == 0) and np.all(tt == t)
        rho = torch.empty((M, w.ny, w.nx), dtype=torch.float64, device="cuda")
        vlbm.vlbm_moments(ens.h, 0, rho, None, None)
        r = rho.cpu().numpy()
        out[t] = 0.5 * (r[:, w.ny // 2 - 1, :] + r[:, w.ny // 2, :])  # rows at y = -dx/2, +dx/2
    ens.close()
    return w, out


def test_bow_shock_moves_at_the_jet_head_velocity(axis_profiles):
    w, prof = axis_profiles

    def head(t):  # mean over realizations of the last axis node behind the bow shock
        a = prof[t]
        return np.mean([(np.nonzero(a[m] > 2.0 * 0.5)[0].max() + 0.5) * w.dx for m in range(a.shape[0])])

    v = (head(1e-3) - head(4e-4)) / (1e-3 - 4e-4)
    assert abs(v / V_HEAD - 1.0) < 0.10, v


def test_laminar_core_carries_the_inlet_randomness(axis_profiles):
    w, prof = axis_profiles
    assert SIGMA_AXIS == pytest.approx(0.30, abs=0.005)
    a = prof[1e-3]
    i0, i1 = int(0.02 / w.dx), int(0.3 / w.dx)
    mean = a[:, i0:i1].mean(axis=0)
    std = a[:, i0:i1].std(axis=0)
    assert np.all(np.abs(mean / 5.0 - 1.0) < 0.06), mean.min()
    assert np.all(np.abs(std / SIGMA_AXIS - 1.0) < 0.25), (std.min(), std.max())


def test_centerline_quantile_diagnostics_paper_geometry():
    """Sec. 4 on the paper's domain at 1000x800 with 64 realizations to
    t = 0.0035, through the library's statistics, sort, quantile and
    width-ratio kernels, on the row next to the axis.  The paper (4000x3200,
    M = 1000) reports a laminar core with std ~0.30 and mean ~5, the leading
    fringe at x ~ 2.27 where the width ratio Q grows far beyond its Gaussian
    1.654, a Gaussian Q (median ~1.67) inside the mixing region and positively
    skewed bands there (median (p95 - mean)/(mean - p5) ~ 1.4; 1.2 at this
    resolution, 1.45 at 2000x1600).  Bounds allow for the coarser grid and the
    64 samples."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = inputs.PAPER_GRIDS["paper1000"]
    M, t_final = 64, 0.0035
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, M)
    ens = vlbm.Ensemble(vlbm.Params.jet(), [(w.nx, w.ny, w.dx, w.y_min)], coefs, M)
    ens.run(t_final, chunk=240)
    t, s, a, status = ens.times(0)
    assert np.all(status == 0) and np.all(t == t_final)
    ncell = w.nx * w.ny
    acc = torch.empty((3, 2, ncell), dtype=torch.float64, device="cuda")
    smp = torch.empty((M, ncell), dtype=torch.float64, device="cuda")
    vlbm.vlbm_ensemble_stats(ens.h, 0, 1, acc, 0, smp, 0)
    ens.close()
    mean = torch.empty((3, ncell), dtype=torch.float64, device="cuda")
    std = torch.empty_like(mean)
    vlbm.vlbm_stats_finalize(acc, ncell, M, mean, std)
    j = w.ny // 2
    row = smp[:, j * w.nx:(j + 1) * w.nx].contiguous()
    vlbm.vlbm_sort_samples(row, w.nx, M)
    qs = torch.empty((5, w.nx), dtype=torch.float64, device="cuda")
    vlbm.vlbm_quantiles(row, w.nx, M, [5, 16, 50, 84, 95], qs)
    q = torch.empty(w.nx, dtype=torch.float64, device="cuda")
    vlbm.vlbm_width_ratio(row, w.nx, M, q)
    torch.cuda.synchronize()
    mu = mean[0, j * w.nx:(j + 1) * w.nx].cpu().numpy()
    sd = std[0, j * w.nx:(j + 1) * w.nx].cpu().numpy()
    p5, p16, p50, p84, p95 = qs.cpu().numpy()
    Q = q.cpu().numpy()
    x = (np.arange(w.nx) + 0.5) * w.dx
    core = (x > 0.2) & (x < 0.8)
    assert abs(sd[core].mean() / SIGMA_AXIS - 1.0) < 0.25
    assert abs(mu[core].mean() / 5.0 - 1.0) < 0.1
    i_f = int(np.nonzero(p95 > 1.0)[0].max())  # twice the ambient density
    assert 2.15 < x[i_f] < 2.40, x[i_f]
    near = Q[max(i_f - 20, 0):i_f + 21]
    assert np.nanmax(near[np.isfinite(near)]) > 10.0
    mix = (sd > 1.0) & (p16 > 1.0)
    assert mix.sum() > 100
    assert 1.45 < np.median(Q[mix]) < 1.90
    assert np.median((p95[mix] - mu[mix]) / (mu[mix] - p5[mix])) > 1.0
