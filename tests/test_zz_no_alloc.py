"""The allocation-free W1 entry point (vlbm_w1_noalloc) against vlbm_w1, through
the C ABI: the per-cell one-point W1 of eq:w1disc and its average W_{1,1} must
be the same bits, on two calls in a row, the second on a smaller input (the
fixed workspace keeps the first call's partial sums, none of which the second
may read), and inputs beyond the workspace are refused before any launch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2605_25282_amd import vlbm


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    vlbm.lib()
    yield
    torch.cuda.synchronize()


def _sorted_pair(n_cells, m, seed):
    """Two seeded sorted sample stores [m][n_cells] (float64, on the GPU)."""
    g = np.random.default_rng(seed)
    a = np.sort(g.gamma(2.0, 1.5, size=(m, n_cells)), axis=0)
    b = np.sort(a + g.normal(0.0, 0.3, size=(m, n_cells)), axis=0)
    return torch.tensor(a, device="cuda"), torch.tensor(b, device="cuda"), a, b


def _both(a, b, n_cells, m):
    dev = dict(dtype=torch.float64, device="cuda")
    out = {}
    for name, fn in (("alloc", vlbm.vlbm_w1), ("noalloc", vlbm.vlbm_w1_noalloc)):
        cell = torch.full((n_cells,), -1.0, **dev)
        mean = torch.full((1,), -1.0, **dev)
        fn(a, b, n_cells, m, cell, mean)
        torch.cuda.synchronize()
        out[name] = (cell.cpu().numpy(), float(mean.item()))
    return out


def test_noalloc_equals_w1_on_two_calls_second_smaller():
    for n_cells, m, seed in ((1_000_003, 8, 1), (5_001, 4, 2)):
        print(f"vlbm_w1_noalloc: n_cells={n_cells} m={m} seed={seed}", flush=True)
        a, b, ha, hb = _sorted_pair(n_cells, m, seed)
        out = _both(a, b, n_cells, m)
        cell_a, mean_a = out["alloc"]
        cell_n, mean_n = out["noalloc"]
        assert np.array_equal(cell_a, cell_n)
        assert mean_a == mean_n
        # and both are the definition of eq:w1disc
        ref = np.abs(ha - hb).mean(axis=0)
        assert np.abs(cell_n - ref).max() <= 1e-12 * np.abs(ref).max()
        assert mean_n == pytest.approx(ref.mean(), rel=1e-12, abs=0.0)


def test_noalloc_per_cell_only_and_size_limit():
    n_cells, m = 2_048, 3
    a, b, ha, hb = _sorted_pair(n_cells, m, 3)
    cell = torch.empty(n_cells, dtype=torch.float64, device="cuda")
    vlbm.vlbm_w1_noalloc(a, b, n_cells, m, cell, None)
    torch.cuda.synchronize()
    assert np.abs(cell.cpu().numpy() - np.abs(ha - hb).mean(axis=0)).max() <= 1e-12
    # one cell past the workspace: refused (the per-cell values alone need no workspace)
    big = 16384 * 1024 + 1
    x = torch.zeros(big, dtype=torch.float64, device="cuda")
    mean = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(vlbm.VlbmError) as ei:
        vlbm.vlbm_w1_noalloc(x, x, big, 1, None, mean)
    assert ei.value.code == vlbm.ERR_SIZE
    cell_big = torch.full((big,), -1.0, dtype=torch.float64, device="cuda")
    vlbm.vlbm_w1_noalloc(x, x, big, 1, cell_big, None)
    torch.cuda.synchronize()
    assert float(cell_big.abs().max()) == 0.0
