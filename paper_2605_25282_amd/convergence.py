"""Convergence study over the mesh levels of one ensemble (Sec. 3.2-3.4).

Composes C-ABI calls only: every level's moments are restricted on the device
to the common (coarsest) grid (`vlbm_ensemble_stats`), giving its ensemble mean
and standard deviation fields and the restricted density of every realization;
the observables of each compared pair -- W_{1,1} (eq:w1disc), W_{1,2} (eq:w2),
E_mean (eq:mean), E_std (eq:std), E_strong (eq:strongError) -- come from
`vlbm_w1`, `vlbm_w12`, `vlbm_mean_abs_diff` and `vlbm_strong_error`, the pairs
from the Cauchy
(eq:cauchy) and reference (eq:ref) protocols, and the rates from
`vlbm_rate_fit` (eq:ratefit).  This module only chooses pairs and allocates
buffers.
"""
from __future__ import annotations

from dataclasses import dataclass, field

from . import vlbm

OBSERVABLES = ("W11", "W12", "E_mean", "E_std", "E_strong")


def cauchy_pairs(L: int):
    """(coarser level, finer level, level of the associated mesh width), l = 1..L."""
    return [(l - 1, l, l - 1) for l in range(1, L + 1)]


def reference_pairs(L: int):
    return [(l, L, l) for l in range(L)]


@dataclass
class LevelStats:
    """Statistics of one level on the common grid (device tensors)."""
    mean: object      # [3][n_cells]: rho, |v|, p
    std: object       # [3][n_cells]
    samples: object   # [M][n_cells] restricted density per realization
    sorted: object    # the same, each cell's column sorted


@dataclass
class Study:
    dx: list
    n_cells: int
    m: int
    errors: dict = field(default_factory=dict)  # (protocol, observable) -> [errors per pair]
    pairs: dict = field(default_factory=dict)   # protocol -> [(coarse, fine, dx level)]
    rates: dict = field(default_factory=dict)   # (protocol, observable) -> rate


def level_stats(ens, level: int, r: int, stream=None) -> LevelStats:
    """Restrict level `level` by r x r blocks to the common grid and form its
    statistics (one pass over the ensemble's state, no host copy)."""
    import torch
    nx, ny = ens.shapes[level]
    n_cells = (nx // r) * (ny // r)
    M = ens.n_real
    acc = torch.empty((3, 2, n_cells), dtype=torch.float64, device="cuda")
    samples = torch.empty((M, n_cells), dtype=torch.float64, device="cuda")
    vlbm.vlbm_ensemble_stats(ens.h, level, r, acc, 0, samples, 0)
    mean = torch.empty((3, n_cells), dtype=torch.float64, device="cuda")
    std = torch.empty_like(mean)
    vlbm.vlbm_stats_finalize(acc, n_cells, M, mean, std, stream)
    srt = samples.clone()
    vlbm.vlbm_sort_samples(srt, n_cells, M, stream)
    return LevelStats(mean, std, samples, srt)


def pair_errors(a: LevelStats, b: LevelStats, ncx: int, ncy: int, m: int, n_pd: int,
                stream=None) -> dict:
    """The five observables between a coarser member a and a finer member b."""
    import torch
    n_cells = ncx * ncy
    out = torch.zeros(5, dtype=torch.float64, device="cuda")
    w1c = torch.empty(n_cells, dtype=torch.float64, device="cuda")
    per = torch.empty(m, dtype=torch.float64, device="cuda")
    w2p = torch.empty(n_pd ** 4, dtype=torch.float64, device="cuda")
    vlbm.vlbm_w1(a.sorted, b.sorted, n_cells, m, w1c, out[0:1], stream)
    vlbm.vlbm_w12(a.samples, b.samples, ncx, ncy, m, n_pd, w2p, out[1:2], stream)
    vlbm.vlbm_mean_abs_diff(a.mean[0], b.mean[0], n_cells, out[2:3], stream)
    vlbm.vlbm_mean_abs_diff(a.std[0], b.std[0], n_cells, out[3:4], stream)
    vlbm.vlbm_strong_error(a.samples, b.samples, n_cells, m, per, out[4:5], stream)
    vals = out.cpu().tolist()
    return dict(zip(OBSERVABLES, vals))


def study(ens, dx, n_pd: int = 10, stream=None) -> Study:
    """Cauchy and reference tables and rates over all levels of `ens` (levels
    ordered coarse to fine, each a refinement of level 0 by an integer factor);
    n_pd subsampled points per direction for W_{1,2} (the paper uses 10)."""
    L = len(ens.shapes) - 1
    nx0, ny0 = ens.shapes[0]
    stats = []
    for l, (nx, ny) in enumerate(ens.shapes):
        r = nx // nx0
        if r * nx0 != nx or r * ny0 != ny:
            raise ValueError(f"level {l} ({nx} x {ny}) is not a refinement of level 0")
        stats.append(level_stats(ens, l, r, stream))
    n_cells, m = nx0 * ny0, ens.n_real
    st = Study(dx=list(dx), n_cells=n_cells, m=m)
    for proto, pairs in (("cauchy", cauchy_pairs(L)), ("reference", reference_pairs(L))):
        st.pairs[proto] = pairs
        errs = [pair_errors(stats[c], stats[f], nx0, ny0, m, n_pd, stream) for c, f, _ in pairs]
        for obs in OBSERVABLES:
            st.errors[(proto, obs)] = [e[obs] for e in errs]
            if len(pairs) >= 2:
                st.rates[(proto, obs)] = vlbm.vlbm_rate_fit(st.errors[(proto, obs)],
                                                            [dx[w] for _, _, w in pairs])[0]
    return st
