"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Bar (FP64): per (variable, slot) plane, max |gpu - oracle| / max |oracle| <= 1e-11
after the stated number of steps; the path is designed to be bitwise
reproducible, so the tests also report the exact maximum difference.  The
statistics are compared at 1e-3 relative (sums over cells of |difference| over
sums of |reference|), and sort/W1 on seeded synthetic stores bit for bit / to
rounding.  Every input is seeded; nothing the oracle consumes comes from the GPU.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O
from paper_2605_25282_amd import inputs, vlbm

TOL = 1e-11


def _to_oracle(gpu_state, m):
    """[4 var][5 slot][R][ny][nx] -> oracle layout (20, ny, nx) for realization m."""
    s = gpu_state[:, :, m]
    return s.transpose(1, 0, 2, 3).reshape(20, s.shape[2], s.shape[3])


def _plane_err(mine, ref):
    """Relative error per (slot, var) plane (reading of the 1e-11 bar)."""
    worst = 0.0
    for s in range(5):
        for v in range(4):
            d = np.abs(mine[s * 4 + v] - ref[s * 4 + v]).max()
            den = np.abs(ref[s * 4 + v]).max()
            if den == 0.0:
                den = np.abs(ref[s * 4 + 3]).max()
            worst = max(worst, d / den)
    return worst


def _grid(name):
    w = inputs.WORKLOADS[name]
    return w, O.Grid(w.nx, w.ny, w.dx, w.y_min)


def _oracle_runs(p, g, coefs, t_final, max_steps, ms):
    out = {}
    for m in ms:
        out[m] = O.run(p, g, O.init(p, g, coefs[m]), t_final, max_steps=max_steps)
    return out


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    vlbm.lib()
    yield
    torch.cuda.synchronize()


def test_init_bitwise():
    """Initial datum (eq:u0_def, correctly rounded inlet profile) and equilibrium
    populations are bit-identical to the oracle's."""
    w, g = _grid("jet128")
    R = 8
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, R)
    ens = vlbm.Ensemble(vlbm.Params.jet(), [(w.nx, w.ny, w.dx, w.y_min)], coefs, R)
    st = ens.state(0).cpu().numpy()
    ens.close()
    p = O.Params()
    for m in range(R):
        ref = O.init(p, g, coefs[m])
        assert np.array_equal(_to_oracle(st, m), ref), f"realization {m}"


@pytest.mark.parametrize("alpha", [0.0, 1.0 / 3.0])
def test_jet_50_steps(alpha):
    """The headline parity case: 128 x 64 jet, 8 realizations, exactly 50 steps."""
    w, g = _grid("jet128")
    R, steps = 8, 50
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, R)
    ens = vlbm.Ensemble(vlbm.Params.jet(alpha=alpha), [(w.nx, w.ny, w.dx, w.y_min)], coefs, R)
    ens.step(1e30, steps)
    st = ens.state(0).cpu().numpy()
    t, s, a, status = ens.times(0)
    ens.close()
    assert np.all(s == steps) and np.all(status == 0)
    p = O.Params(alpha=alpha)
    ref = _oracle_runs(p, g, coefs, 1e30, steps, range(R))
    worst, maxdiff = 0.0, 0.0
    for m in range(R):
        r_st, r_t, r_n, r_a, rc = ref[m]
        assert rc == O.OK and r_n == steps
        mine = _to_oracle(st, m)
        worst = max(worst, _plane_err(mine, r_st))
        maxdiff = max(maxdiff, np.abs(mine - r_st).max())
        assert t[m] == r_t and a[m] == r_a
    print(f"alpha={alpha}: worst plane rel err {worst:.3e}, max abs diff {maxdiff:.3e}")
    assert worst <= TOL


def test_jet_to_t_final():
    """A full run to t = 1e-4: identical step counts, final times and states."""
    w, g = _grid("jet128")
    R = 8
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 100, R)
    ens = vlbm.Ensemble(vlbm.Params.jet(), [(w.nx, w.ny, w.dx, w.y_min)], coefs, R)
    ens.run(w.t_final, chunk=16)
    st = ens.state(0).cpu().numpy()
    t, s, a, status = ens.times(0)
    ens.close()
    ref = _oracle_runs(O.Params(), g, coefs, w.t_final, 1 << 30, range(R))
    for m in range(R):
        r_st, r_t, r_n, r_a, rc = ref[m]
        assert s[m] == r_n and t[m] == r_t == w.t_final and a[m] == r_a
        assert _plane_err(_to_oracle(st, m), r_st) <= TOL


def _prim(rho, v1, v2, p, gamma):
    return np.stack([rho, rho * v1, rho * v2, p / (gamma - 1.0) + 0.5 * rho * (v1 * v1 + v2 * v2)])


@pytest.mark.parametrize("bc,lim", [("periodic", "limiter"), ("periodic", "zero"), ("periodic", "one"),
                                    ("neumann", "limiter")])
def test_verification_modes(bc, lim):
    """Other boundary/theta modes on a loaded smooth or shock-tube state, 30 steps."""
    nx, ny, R, gamma = 70, 37, 3, 1.4
    dx = 1.0 / nx
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    u = np.zeros((4, R, ny, nx))
    for m in range(R):
        if bc == "periodic":
            rho = 1.3 + 0.3 * np.sin(2 * np.pi * (x / nx + m / 7.0)) * np.cos(2 * np.pi * y / ny)
            v1 = 0.5 * np.cos(2 * np.pi * y / ny)
            v2 = 0.3 * np.sin(2 * np.pi * x / nx)
            pr = 1.0 + 0.2 * np.cos(2 * np.pi * (x / nx + y / ny))
        else:
            left = x < nx // 2 + m
            rho = np.where(left, 1.0, 0.125)
            v1 = np.zeros_like(rho)
            v2 = np.zeros_like(rho)
            pr = np.where(left, 1.0, 0.1)
        u[:, m] = _prim(rho, v1, v2, pr, gamma)
    prm = vlbm.Params.jet(gamma=gamma, bc=bc, limiter=lim, kl_modes=0)
    ens = vlbm.Ensemble(prm, [(nx, ny, dx, 0.0)], None, R)
    ens.set_macroscopic(0, torch.tensor(u, device="cuda"))
    ens.step(1e30, 30)
    st = ens.state(0).cpu().numpy()
    ens.close()
    p = O.Params(gamma=gamma, bc=bc, theta_mode=lim, kl_modes=0)
    g = O.Grid(nx, ny, dx, 0.0)
    for m in range(R):
        ref, _, n, _, rc = O.run(p, g, O.from_macroscopic(p, g, u[:, m]), 1e30, max_steps=30)
        assert n == 30
        assert _plane_err(_to_oracle(st, m), ref) <= TOL


def test_moments_bitwise():
    w, g = _grid("jet128")
    R = 4
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, R)
    ens = vlbm.Ensemble(vlbm.Params.jet(), [(w.nx, w.ny, w.dx, w.y_min)], coefs, R)
    ens.step(1e30, 12)
    rho, speed, pr = [t.cpu().numpy() for t in ens.moments(0)]
    ens.close()
    p = O.Params()
    for m in range(R):
        ref, *_ = O.run(p, g, O.init(p, g, coefs[m]), 1e30, max_steps=12)
        r, s, q = O.moments(p, ref[0:4])
        assert np.array_equal(rho[m], r) and np.array_equal(speed[m], s) and np.array_equal(pr[m], q)


def _rel_l1(a, b):
    return np.abs(a - b).sum() / np.abs(b).sum()


def test_two_level_statistics():
    """Mean, std (r = 1 and r = 2) and the one-point W1 between a fine and a coarse
    level restricted to the coarse grid, against the oracle's own runs."""
    R = 8
    fine, coarse = (128, 64), (64, 32)
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, R)
    t_final = 1e-4
    levels = [(nx, ny, 1.0 / nx, -0.25) for (nx, ny) in (coarse, fine)]
    ens = vlbm.Ensemble(vlbm.Params.jet(), levels, coefs, R)
    ens.run(t_final, chunk=16)
    ncell = coarse[0] * coarse[1]
    accs, samples = [], []
    for lvl, r in ((0, 1), (1, 2)):
        acc = torch.empty((3, 2, ncell), dtype=torch.float64, device="cuda")
        smp = torch.empty((R, ncell), dtype=torch.float64, device="cuda")
        vlbm.vlbm_ensemble_stats(ens.h, lvl, r, acc, 0, smp, 0)
        accs.append(acc)
        samples.append(smp)
    mean = torch.empty((3, ncell), dtype=torch.float64, device="cuda")
    std = torch.empty_like(mean)
    vlbm.vlbm_stats_finalize(accs[1], ncell, R, mean, std)
    for smp in samples:
        vlbm.vlbm_sort_samples(smp, ncell, R)
    w1c = torch.empty(ncell, dtype=torch.float64, device="cuda")
    w1m = torch.empty(1, dtype=torch.float64, device="cuda")
    vlbm.vlbm_w1(samples[0], samples[1], ncell, R, w1c, w1m)
    torch.cuda.synchronize()
    mean, std, w1c, w1m = mean.cpu().numpy(), std.cpu().numpy(), w1c.cpu().numpy(), w1m.item()
    ens.close()
    # oracle
    p = O.Params()
    fields = {}
    for (nx, ny), r in ((coarse, 1), (fine, 2)):
        g = O.Grid(nx, ny, 1.0 / nx, -0.25)
        st = np.stack([O.run(p, g, O.init(p, g, coefs[m]), t_final)[0] for m in range(R)])
        rho, sp, pr = O.moments(p, st[:, 0:4])
        fields[r] = [O.restrict(f, r) for f in (rho, sp, pr)]
    for f in range(3):
        assert _rel_l1(mean[f], O.ensemble_mean(fields[2][f]).ravel()) <= 1e-12
        assert _rel_l1(std[f], O.ensemble_std(fields[2][f]).ravel()) <= 1e-9
    ref_w1 = O.w1(fields[1][0], fields[2][0]).ravel()
    assert _rel_l1(w1c, ref_w1) <= 1e-12
    assert w1m == pytest.approx(ref_w1.mean(), rel=1e-12)


@pytest.mark.parametrize("m,ncell", [(1, 5), (7, 300), (64, 1000), (100, 333), (1000, 77), (4096, 3)])
def test_sort_and_w1_synthetic(m, ncell):
    a = inputs.random_fields(1000 + m, (m, ncell))
    b = inputs.random_fields(2000 + m, (m, ncell))
    ta, tb = torch.tensor(a, device="cuda"), torch.tensor(b, device="cuda")
    vlbm.vlbm_sort_samples(ta, ncell, m)
    vlbm.vlbm_sort_samples(tb, ncell, m)
    w1c = torch.empty(ncell, dtype=torch.float64, device="cuda")
    vlbm.vlbm_w1(ta, tb, ncell, m, w1c, None)
    torch.cuda.synchronize()
    assert np.array_equal(ta.cpu().numpy(), np.sort(a, axis=0))
    assert np.allclose(w1c.cpu().numpy(), O.w1(a, b), rtol=1e-12, atol=0)


def test_nonpositive_state_is_reported():
    """A loaded state with negative pressure latches the realization's status and
    vlbm_step reports VLBM_ERR_NONPOSITIVE; the other realization is unaffected."""
    nx, ny, R, gamma = 16, 16, 2, 1.4
    one = np.ones((ny, nx))
    u = np.zeros((4, R, ny, nx))
    u[:, 0] = _prim(one, 0 * one, 0 * one, one, gamma)
    bad = one.copy()
    bad[5, 7] = -1.0
    u[:, 1] = _prim(one, 0 * one, 0 * one, bad, gamma)
    ens = vlbm.Ensemble(vlbm.Params.jet(gamma=gamma, bc="neumann", kl_modes=0), [(nx, ny, 0.1, 0.0)], None, R)
    ens.set_macroscopic(0, torch.tensor(u, device="cuda"))
    with pytest.raises(vlbm.VlbmError) as ei:
        ens.step(1.0, 3)
    assert ei.value.code == vlbm.ERR_NONPOSITIVE
    t, s, a, status = ens.times(0)
    ens.close()
    assert status[0] == 0 and status[1] == vlbm.ERR_NONPOSITIVE


def test_jet640_sampled_realizations():
    """Full-size 640 x 320 ensemble of 64 realizations in one launch configuration,
    50 steps; three realizations recomputed by the oracle."""
    w, g = _grid("jet640")
    steps = 50
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, w.m)
    ens = vlbm.Ensemble(vlbm.Params.jet(), [(w.nx, w.ny, w.dx, w.y_min)], coefs, w.m)
    ens.step(1e30, steps)
    st = ens.state(0)
    picks = (0, 37, w.m - 1)
    mine = {m: st[:, :, m].cpu().numpy() for m in picks}
    ens.close()
    del st
    ref = _oracle_runs(O.Params(), g, coefs, 1e30, steps, picks)
    for m in picks:
        s = mine[m]
        assert _plane_err(s.transpose(1, 0, 2, 3).reshape(20, w.ny, w.nx), ref[m][0]) <= TOL


def _loaded_state(bc, nx, ny, R, gamma):
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    u = np.zeros((4, R, ny, nx))
    for m in range(R):
        if bc == "periodic":
            rho = 1.3 + 0.3 * np.sin(2 * np.pi * (x / nx + m / 7.0)) * np.cos(2 * np.pi * y / ny)
            v1 = 0.5 * np.cos(2 * np.pi * y / ny)
            v2 = 0.3 * np.sin(2 * np.pi * x / nx)
            pr = 1.0 + 0.2 * np.cos(2 * np.pi * (x / nx + y / ny))
        else:
            left = (x + y // 3) < nx // 2 + m
            rho = np.where(left, 1.0, 0.125)
            v1 = np.where(left, 0.3, -0.2)
            v2 = 0.1 * np.sin(2 * np.pi * x / nx)
            pr = np.where(left, 1.0, 0.1)
        u[:, m] = _prim(rho, v1, v2, pr, gamma)
    return u


@pytest.mark.parametrize("bc,nx,ny,chunk", [
    ("jet", 128, 64, 0), ("jet", 121, 37, 16), ("jet", 181, 50, 7), ("jet", 61, 19, 4),
    ("jet", 3, 3, 4), ("jet", 64, 5, 0), ("neumann", 61, 33, 8), ("neumann", 122, 29, 5),
    ("periodic", 70, 37, 16), ("periodic", 121, 20, 6), ("neumann", 3, 4, 4)])
def test_march_kernel_equals_reference(bc, nx, ny, chunk):
    """The marching kernel (strips of 60 output columns, register ring over rows) and the
    reference kernel give bit-identical states, including grids where the last column
    falls on a strip edge, ragged row chunks and 3-node levels."""
    R, steps, gamma = 3, 25, (5.0 / 3.0 if bc == "jet" else 1.4)
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, R)
    out = {}
    for kern in ("reference", "march"):
        prm = vlbm.Params.jet(bc=bc, gamma=gamma) if bc == "jet" else \
            vlbm.Params.jet(bc=bc, gamma=gamma, kl_modes=0)
        y_min = -0.5 * ny / nx
        ens = vlbm.Ensemble(prm, [(nx, ny, 1.0 / nx, y_min)], coefs if bc == "jet" else None, R)
        ens.tune(kern, chunk)
        if bc != "jet":
            ens.set_macroscopic(0, torch.tensor(_loaded_state(bc, nx, ny, R, gamma), device="cuda"))
        ens.step(1e30, steps)
        out[kern] = (ens.state(0).cpu().numpy(), ens.times(0))
        ens.close()
    assert np.array_equal(out["reference"][0], out["march"][0])
    for a, b in zip(out["reference"][1], out["march"][1]):
        assert np.array_equal(a, b)


def test_march_kernel_equals_reference_jet640():
    """Full-size 640 x 320 x 64 ensemble, 30 steps, default decomposition."""
    w = inputs.WORKLOADS["jet640"]
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, w.m)
    res = {}
    for kern in ("reference", "march"):
        ens = vlbm.Ensemble(vlbm.Params.jet(), [(w.nx, w.ny, w.dx, w.y_min)], coefs, w.m)
        ens.tune(kern, 0)
        ens.step(1e30, 30)
        st = ens.state(0)
        res[kern] = (st.sum(dim=(2, 3, 4)).cpu().numpy(), st[:, :, ::9].cpu().numpy())
        ens.close()
        del st
    assert np.array_equal(res["reference"][0], res["march"][0])
    assert np.array_equal(res["reference"][1], res["march"][1])


def test_autotune_is_result_neutral_and_cached():
    """Tuning runs live steps with several decompositions; the ensemble must end
    bit-identical to an untuned one, and the choice must be reused by a new ensemble."""
    w = inputs.WORKLOADS["jet128"]
    R = 8
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, R)
    a = vlbm.Ensemble(vlbm.Params.jet(), [(w.nx, w.ny, w.dx, w.y_min)], coefs, R)
    chunks = a.autotune(1e30, steps_per_candidate=2)
    assert len(chunks) == 1 and 4 <= chunks[0] <= w.ny
    tuned = a.get_tuning()
    assert tuned[0] == chunks and tuned[1] in (1, 2, 4) and tuned[2] in (0, 1) and tuned[3] in (0, 1)
    n_tune = int(a.times(0)[1][0])
    a.step(1e30, 40 - n_tune)
    b = vlbm.Ensemble(vlbm.Params.jet(), [(w.nx, w.ny, w.dx, w.y_min)], coefs, R)
    b.tune("reference", 0)
    b.step(1e30, 40)
    sa, sb = a.state(0).cpu().numpy(), b.state(0).cpu().numpy()
    assert np.array_equal(sa, sb)
    c = vlbm.Ensemble(vlbm.Params.jet(), [(w.nx, w.ny, w.dx, w.y_min)], coefs, R)
    assert c.get_tuning() == tuned  # the cached choice
    c.step(1e30, 40)
    assert np.array_equal(c.state(0).cpu().numpy(), sa)
    for e in (a, b, c):
        e.close()


def test_every_decomposition_is_bitwise_equal():
    """Two levels in one launch under every decomposition the tuner can pick --
    uneven chunk heights, 1, 2 or 4 wavefronts per block, strip-fastest or
    realization-fastest items -- give the same states bit for bit, and
    vlbm_get_tuning reports what vlbm_set_tuning set."""
    R = 5
    levels = _three_levels(64)[:2]
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, R)
    ref = None
    for chunks, wpb, order, deal in (([0, 0], 4, 0, 0), ([7, 13], 4, 0, 0), ([7, 13], 2, 0, 0),
                                     ([7, 13], 1, 0, 0), ([5, 64], 4, 1, 0), ([9, 4], 2, 1, 0),
                                     ([32, 11], 1, 1, 0), ([0, 0], 4, 0, 1), ([7, 13], 2, 1, 1),
                                     ([5, 4], 1, 0, 1), ([64, 64], 4, 1, 1)):
        e = vlbm.Ensemble(vlbm.Params.jet(), levels, coefs, R)
        e.set_tuning(chunks, wpb, order, deal)
        got_chunks, got_wpb, got_order, got_deal = e.get_tuning()
        assert (got_wpb, got_order, got_deal) == (wpb, order, deal)
        assert all(g == (min(c, ny) if c else g) for g, c, (_, ny, _, _) in zip(got_chunks, chunks, levels))
        e.step(1e30, 45)
        st = [e.state(l).cpu().numpy() for l in range(2)]
        clocks = [e.times(l)[:2] for l in range(2)]
        e.close()
        if ref is None:
            ref = (st, clocks)
            continue
        for l in range(2):
            assert np.array_equal(st[l], ref[0][l]), (chunks, wpb, order, deal, l)
            assert np.array_equal(clocks[l][0], ref[1][l][0]) and np.array_equal(clocks[l][1], ref[1][l][1])
    e = vlbm.Ensemble(vlbm.Params.jet(), levels, coefs, R)
    for bad in ((None, 3, 0, 0), (None, 4, 2, 0), ([2, 0], 4, 0, 0), (None, 4, 0, 2)):
        with pytest.raises(vlbm.VlbmError):
            e.set_tuning(*bad)
    e.close()


def _three_levels(nx0):
    return [(nx0 << k, (nx0 << k) // 2, 1.0 / (nx0 << k), -0.25) for k in range(3)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replay_equals_eager(precision):
    """Step runs long enough to be replayed from captured hipGraphs (a ragged lead to
    re-align the control ring, whole 30-step graphs, an eager tail, repeated calls with
    host reads in between) end bit-identical to eager launches of the marching and the
    reference kernel, on three levels stepped by one launch per step."""
    R = 5
    levels = _three_levels(48)
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 7, R)
    res = {}
    for kern in ("march", "march-eager", "reference-eager"):
        ens = vlbm.Ensemble(vlbm.Params.jet(precision=precision), levels, coefs, R)
        ens.tune(kern, 0)
        hist = []
        for n in (1, 64, 33, 95):
            ens.step(1e30, n)
            hist.append(ens.times(1))
        res[kern] = ([ens.state(l).cpu().numpy() for l in range(3)], hist)
        ens.close()
    for kern in ("march-eager", "reference-eager"):
        for l in range(3):
            assert np.array_equal(res["march"][0][l], res[kern][0][l]), (kern, l)
        for ha, hb in zip(res["march"][1], res[kern][1]):
            for a, b in zip(ha, hb):
                assert np.array_equal(a, b)
    assert np.all(res["march"][1][-1][1] == 193)


def test_graph_replays_past_t_final():
    """Replays that run past t_final leave finished realizations untouched: the run
    ends at the same step counts, times and states as an eager run to t_final."""
    R = 4
    levels = _three_levels(32)
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 50, R)
    t_final = 4e-4  # 24, 51 and 124 steps on the three levels
    out = {}
    for kern in ("march", "march-eager"):
        ens = vlbm.Ensemble(vlbm.Params.jet(), levels, coefs, R)
        ens.tune(kern, 0)
        done = ens.step(t_final, 600)
        assert done
        out[kern] = [(ens.state(l).cpu().numpy(), ens.times(l)) for l in range(3)]
        ens.close()
    for l in range(3):
        assert np.array_equal(out["march"][l][0], out["march-eager"][l][0])
        for a, b in zip(out["march"][l][1], out["march-eager"][l][1]):
            assert np.array_equal(a, b)
        assert np.all(out["march"][l][1][0] == t_final)


def test_multilevel_single_launch_matches_oracle():
    """Three nested levels (48 x 24, 96 x 48, 192 x 96) advanced together, one launch
    per step and graph replays, each against the oracle run of that level alone."""
    R, steps = 3, 40
    levels = _three_levels(48)
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, R)
    ens = vlbm.Ensemble(vlbm.Params.jet(), levels, coefs, R)
    ens.step(1e30, steps)
    got = [(ens.state(l).cpu().numpy(), ens.times(l)) for l in range(3)]
    ens.close()
    p = O.Params()
    for l, (nx, ny, dx, y_min) in enumerate(levels):
        g = O.Grid(nx, ny, dx, y_min)
        st, (t, s, a, status) = got[l]
        assert np.all(s == steps) and np.all(status == 0)
        for m in range(R):
            r_st, r_t, r_n, r_a, rc = O.run(p, g, O.init(p, g, coefs[m]), 1e30, max_steps=steps)
            assert rc == O.OK and r_n == steps and t[m] == r_t and a[m] == r_a
            assert _plane_err(_to_oracle(st, m), r_st) <= TOL, (l, m)


@pytest.mark.parametrize("alpha", [0.0, 1.0 / 3.0])
def test_mixed_precision_matches_mixed_oracle(alpha):
    """Mixed storage (populations' rho, rho v in FP32; u and E populations FP64;
    all arithmetic FP64) against the oracle's mixed storage mode, 50 steps."""
    w, g = _grid("jet128")
    R, steps = 8, 50
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, R)
    ens = vlbm.Ensemble(vlbm.Params.jet(alpha=alpha, precision="mixed"),
                        [(w.nx, w.ny, w.dx, w.y_min)], coefs, R)
    ens.step(1e30, steps)
    st = ens.state(0).cpu().numpy()
    ens.close()
    p = O.Params(alpha=alpha, storage="mixed")
    worst = 0.0
    for m in range(R):
        ref, _, n, _, rc = O.run(p, g, O.init(p, g, coefs[m]), 1e30, max_steps=steps)
        assert rc == O.OK and n == steps
        worst = max(worst, _plane_err(_to_oracle(st, m), ref))
    print(f"mixed alpha={alpha}: worst plane rel err {worst:.3e}")
    assert worst <= TOL


@pytest.mark.parametrize("bc,nx,ny,chunk", [("jet", 128, 64, 0), ("jet", 121, 37, 16),
                                            ("neumann", 61, 33, 8), ("periodic", 70, 37, 16)])
def test_mixed_march_equals_reference(bc, nx, ny, chunk):
    R, steps, gamma = 3, 25, (5.0 / 3.0 if bc == "jet" else 1.4)
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, R)
    out = {}
    for kern in ("reference", "march"):
        kw = dict(bc=bc, gamma=gamma, precision="mixed")
        if bc != "jet":
            kw["kl_modes"] = 0
        ens = vlbm.Ensemble(vlbm.Params.jet(**kw), [(nx, ny, 1.0 / nx, -0.5 * ny / nx)],
                            coefs if bc == "jet" else None, R)
        ens.tune(kern, chunk)
        if bc != "jet":
            ens.set_macroscopic(0, torch.tensor(_loaded_state(bc, nx, ny, R, gamma), device="cuda"))
        ens.step(1e30, steps)
        out[kern] = ens.state(0).cpu().numpy()
        ens.close()
    assert np.array_equal(out["reference"], out["march"])


def test_mixed_vs_fp64_statistics_gpu():
    """The mixed variant's ensemble statistics against the FP64 run on the GPU at the
    final time of the 128 x 64 workload: mean/std (rel. L1) and W1 / mean density."""
    w = inputs.WORKLOADS["jet128"]
    R = w.m
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, R)
    ncell = w.nx * w.ny
    res = {}
    for prec in ("fp64", "mixed"):
        ens = vlbm.Ensemble(vlbm.Params.jet(precision=prec), [(w.nx, w.ny, w.dx, w.y_min)], coefs, R)
        ens.run(w.t_final, chunk=16)
        acc = torch.empty((3, 2, ncell), dtype=torch.float64, device="cuda")
        smp = torch.empty((R, ncell), dtype=torch.float64, device="cuda")
        vlbm.vlbm_ensemble_stats(ens.h, 0, 1, acc, 0, smp, 0)
        mean = torch.empty((3, ncell), dtype=torch.float64, device="cuda")
        std = torch.empty_like(mean)
        vlbm.vlbm_stats_finalize(acc, ncell, R, mean, std)
        vlbm.vlbm_sort_samples(smp, ncell, R)
        res[prec] = (mean, std, smp)
        ens.close()
    w1c = torch.empty(ncell, dtype=torch.float64, device="cuda")
    w1m = torch.empty(1, dtype=torch.float64, device="cuda")
    vlbm.vlbm_w1(res["fp64"][2], res["mixed"][2], ncell, R, w1c, w1m)
    torch.cuda.synchronize()
    m64, s64 = res["fp64"][0].cpu().numpy(), res["fp64"][1].cpu().numpy()
    mmx, smx = res["mixed"][0].cpu().numpy(), res["mixed"][1].cpu().numpy()
    em = _rel_l1(mmx, m64)
    es = _rel_l1(smx, s64)
    ew = w1m.item() / m64[0].mean()
    print(f"mixed vs fp64: mean {em:.3e}, std {es:.3e}, W1/mean(rho) {ew:.3e}")
    assert em < 1e-3 and es < 1e-3 and ew < 1e-3


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_checkpoint_resume_is_bitwise(precision):
    """Save every level's state and clock after 33 steps (vlbm_get_state,
    vlbm_times), restore them into a fresh ensemble (vlbm_set_state) and step
    on: after 70 steps in all, states, times and step counts equal those of an
    uninterrupted run bit for bit (two levels, one launch per step, graph
    replays on both sides)."""
    R = 5
    levels = _three_levels(48)[:2]
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 3, R)
    prm = vlbm.Params.jet(precision=precision)
    ref = vlbm.Ensemble(prm, levels, coefs, R)
    ref.step(1e30, 70)
    want = [(ref.state(l).cpu().numpy(), ref.times(l)) for l in range(2)]
    ref.close()
    a = vlbm.Ensemble(prm, levels, coefs, R)
    a.step(1e30, 33)
    saved = [(a.state(l), a.times(l)) for l in range(2)]
    a.close()
    b = vlbm.Ensemble(prm, levels, np.zeros_like(coefs), R)  # a different initial datum
    for l, (st, (t, s, al, status)) in enumerate(saved):
        assert np.all(s == 33) and np.all(status == 0)
        b.set_state(l, st, t, s, al)
    b.step(1e30, 37)
    for l in range(2):
        got = b.state(l).cpu().numpy()
        assert np.array_equal(got, want[l][0]), l
        for x, y in zip(b.times(l)[:3], want[l][1][:3]):
            assert np.array_equal(x, y)
    b.close()


def _jet640_stats(precision, t_final, first_seed=0, ulp=None):
    """Restricted (2 x 2) mean/std of (rho, |v|, p) and sorted restricted density
    samples of the 640 x 320, 64-realization workload at t_final; ulp = (variable,
    direction) moves the inlet column's macroscopic variable by one ulp first."""
    w = inputs.WORKLOADS["jet640"]
    R = w.m
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, first_seed, R)
    ncell = (w.nx // 2) * (w.ny // 2)
    ens = vlbm.Ensemble(vlbm.Params.jet(precision=precision), [(w.nx, w.ny, w.dx, w.y_min)], coefs, R)
    if ulp is not None:
        var, sign = ulp
        st = ens.state(0)
        col = st[var, 0, :, :, 0]
        st[var, 0, :, :, 0] = torch.nextafter(col, torch.full_like(col, sign * float("inf")))
        t, s, a, _ = ens.times(0)
        ens.set_state(0, st, t, s, a)
        del st
    ens.run(t_final, chunk=240)
    t, _, _, status = ens.times(0)
    assert np.all(status == 0) and np.all(t == t_final)
    acc = torch.empty((3, 2, ncell), dtype=torch.float64, device="cuda")
    smp = torch.empty((R, ncell), dtype=torch.float64, device="cuda")
    vlbm.vlbm_ensemble_stats(ens.h, 0, 2, acc, 0, smp, 0)
    mean = torch.empty((3, ncell), dtype=torch.float64, device="cuda")
    std = torch.empty_like(mean)
    vlbm.vlbm_stats_finalize(acc, ncell, R, mean, std)
    vlbm.vlbm_sort_samples(smp, ncell, R)
    ens.close()
    return mean.cpu().numpy(), std.cpu().numpy(), smp


def _stat_errors(ref, other):
    """W1 / mean density (eq:w1disc), and the largest rel. L1 error of the mean
    and of the std fields (eq:mean, eq:std) of `other` against `ref`."""
    m0, s0, smp0 = ref
    m1, s1, smp1 = other
    nc = m0.shape[1]
    w1c = torch.empty(nc, dtype=torch.float64, device="cuda")
    w1m = torch.zeros(1, dtype=torch.float64, device="cuda")
    vlbm.vlbm_w1(smp0, smp1, nc, smp0.shape[0], w1c, w1m)
    torch.cuda.synchronize()
    return (w1m.item() / m0[0].mean(), max(_rel_l1(m1[f], m0[f]) for f in range(3)),
            max(_rel_l1(s1[f], s0[f]) for f in range(3)))


def test_mixed_vs_fp64_at_final_time_is_at_the_roundoff_floor():
    """The benchmark workload (640 x 320, 64 realizations) at its final time
    t = 1e-3, after the bow shock and the shear-layer instability have
    developed.  There the trajectories decorrelate under any perturbation of
    round-off size: an FP64 ensemble whose inlet density is moved by one ulp
    differs from the unperturbed one by about 4e-3 of the mean density in W1,
    four times the 1e-3 of a literal bar.  The mixed variant is held to that
    floor instead: its W1, mean and std errors against the FP64 ensemble (same
    seeds) are at most 1.5 times the larger of the two one-ulp perturbations'
    (measured about 1.2), and below the difference between two independent
    seed sets (the sampling noise of 64 realizations)."""
    t_final = inputs.WORKLOADS["jet640"].t_final
    ref = _jet640_stats("fp64", t_final)
    mixed = _stat_errors(ref, _jet640_stats("mixed", t_final))
    floors = [_stat_errors(ref, _jet640_stats("fp64", t_final, ulp=(0, sign))) for sign in (1, -1)]
    noise = _stat_errors(ref, _jet640_stats("fp64", t_final, first_seed=64))
    floor = [max(f[k] for f in floors) for k in range(3)]
    names = ("W1/mean(rho)", "mean rel L1", "std rel L1")
    for k, name in enumerate(names):
        print(f"t=1e-3 {name}: mixed {mixed[k]:.3e}, one-ulp floor {floor[k]:.3e} "
              f"(ratio {mixed[k] / floor[k]:.2f}), independent seeds {noise[k]:.3e}")
    assert floor[0] > 1e-3  # round-off alone already exceeds the literal 1e-3 bar
    for k in range(3):
        assert mixed[k] <= 1.5 * floor[k], names[k]
        assert mixed[k] < noise[k], names[k]
