"""The throughput workload at full size -- N = 200 bosons, M = 5 orbitals
(dim 70,058,751), seed 2 -- against the oracle.

Every apply path the benchmark times (reduced map, reduced chained, paper
map, paper chained, table-free) at the benchmark's launch shape, on one
seeded sample of 100,000 rows plus the first two and the last two tiles
(the last one ragged: 63 rows): relative infinity-norm <= 1e-12 with the
oracle's maximum as the scale (Eq. Haction).  The tables behind the table
paths, bit-exact on 10,000 seeded rows plus the same edge tiles: the hashing
table, the single-jump map, and the double-jump map of each form (Sec. IV;
the reduced form keeps the true double jumps of each valid removal pair).
"""

import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_helpers import TILE, rel_inf, sampled_tables

pytestmark = pytest.mark.gpu

N, M, SEED = 200, 5, 2
TOL = 1e-12
PATHS = {  # name: (form, double-jump map); None = table-free
    "reduced_map": ("reduced", True),
    "reduced_chained": ("reduced", False),
    "paper_map": ("paper", True),
    "paper_chained": ("paper", False),
    "direct": (None, False),
}


def edge_rows(D):
    tiles = (D + TILE - 1) // TILE
    return np.concatenate([np.arange(2 * TILE), np.arange((tiles - 2) * TILE, D)])


@pytest.fixture(scope="module")
def workload(oracle_native):
    C, h, g = W.random_instance(N, M, SEED)
    D = C.size
    rng = np.random.default_rng(2026)
    rows = np.unique(np.concatenate([rng.integers(0, D, 100_000), edge_rows(D)]))
    print(f"[headline] oracle H.C on {rows.size} rows", flush=True)
    ref = oracle_native.apply_h(N, M, h, g, C, rows)
    return C, h, g, rows, ref


@pytest.mark.parametrize("path", list(PATHS))
def test_apply_path_sampled_rows(mc, workload, path):
    C, h, g, rows, ref = workload
    form, has_map = PATHS[path]
    hd, gd, Cd = (torch.from_numpy(x).cuda() for x in (h, g, C))
    HC = torch.empty_like(Cd)
    if form is None:
        mc.apply_H_direct(hd, gd, Cd, N, M, out=HC)
        tab = None
    else:
        tab = mc.build_tables(N, M, double_jumps=has_map, form=form)
        mc.apply_H(hd, gd, Cd, tab, out=HC)
    got = HC[torch.from_numpy(rows).cuda()].cpu().numpy()
    err = rel_inf(got, ref)
    print(f"[headline] {path}: rel err {err:.2e} on {rows.size} rows", flush=True)
    assert err <= TOL
    del tab, HC, Cd
    torch.cuda.empty_cache()


@pytest.mark.parametrize("form", ["reduced", "paper"])
def test_tables_sampled_rows_bit_exact(mc, oracle_native, form):
    tab = mc.build_tables(N, M, form=form)
    D = tab.dim
    rng = np.random.default_rng(77)
    rows = np.unique(np.concatenate([rng.integers(0, D, 10_000), edge_rows(D)]))
    occ, t1, t2 = sampled_tables(tab, rows)
    assert np.array_equal(occ, oracle_native.occ_rows(N, M, rows))
    assert np.array_equal(t1, oracle_native.t1_rows(N, M, rows))
    off, ent = (oracle_native.t2r_rows if form == "reduced" else oracle_native.t2_rows)(N, M, rows)
    for i in range(rows.size):
        assert np.array_equal(t2[i], ent[off[i]:off[i + 1]]), (form, int(rows[i]))
    del tab
    torch.cuda.empty_cache()
