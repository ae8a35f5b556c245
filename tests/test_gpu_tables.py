"""GPU tables vs the oracle, bit-exact: occupations (hashing table), single
and double jump maps, batch hash/unhash and the double-jump lookup."""

import numpy as np
import pytest
import torch

from tests.gpu_helpers import tiled_t2_check_and_rows

pytestmark = pytest.mark.gpu

CASES = [(1, 1), (3, 1), (1, 4), (2, 2), (3, 5), (4, 5), (10, 5), (7, 4), (5, 7), (6, 8),
         (12, 6), (20, 3), (2, 9), (3, 10), (300, 2), (256, 3)]


@pytest.mark.parametrize("N,M", CASES)
def test_tables_match_oracle(mc, oracle_native, N, M):
    tab = mc.build_tables(N, M)
    torch.cuda.synchronize()
    D = tab.dim
    assert D == oracle_native.dim(N, M)
    occ = tab.occupations()
    assert np.array_equal(occ, oracle_native.occ_rows(N, M))
    assert np.array_equal(tab.single_jumps(), oracle_native.t1_rows(N, M))
    rows = np.arange(D)
    got = tiled_t2_check_and_rows(tab, rows)
    off, ent = oracle_native.t2_rows(N, M)
    for g in rows:
        assert np.array_equal(got[g], ent[off[g]:off[g + 1]]), g
    # padding rows of the last tile are empty everywhere
    o = tab.occ.cpu().numpy().reshape(tab.tiles, M, 64)
    pad = tab.tiles * 64 - D
    if pad:
        assert np.all(o[-1, :, 64 - pad:] == 0)
        t1 = tab.t1.cpu().numpy().reshape(tab.tiles, M, M, 64)
        assert np.all(t1[-1, :, :, 64 - pad:] == -1)
    compact = int(mc.tables_size(N, M).t2_compact_entries)
    assert sum(len(x) for x in got) == compact


@pytest.mark.parametrize("N,M", CASES)
def test_reduced_tables_match_oracle(mc, oracle_native, N, M):
    """Reduced double-jump map (true double jumps only) vs the oracle's rows."""
    tab = mc.build_tables(N, M, form="reduced")
    torch.cuda.synchronize()
    rows = np.arange(tab.dim)
    got = tiled_t2_check_and_rows(tab, rows)
    off, ent = oracle_native.t2r_rows(N, M)
    for g in rows:
        assert np.array_equal(got[g], ent[off[g]:off[g + 1]]), g
    assert sum(len(x) for x in got) == int(mc.tables_size(N, M).t2r_compact_entries)
    # the single-jump map does not depend on the form
    assert np.array_equal(tab.single_jumps(), oracle_native.t1_rows(N, M))


def test_lookup_rejects_reduced_form(mc):
    tab = mc.build_tables(6, 4, form="reduced")
    q = torch.zeros((1, 5), dtype=torch.int64, device="cuda")
    with pytest.raises(mc.MCError):
        mc.t2_lookup(q, tab)


@pytest.mark.parametrize("N,M", [(10, 5), (5, 7), (300, 2), (2, 9)])
def test_lookup_matches_oracle(mc, oracle_native, N, M):
    tab = mc.build_tables(N, M)
    D = tab.dim
    rng = np.random.default_rng(N * 100 + M)
    Q = 4000
    q = np.stack([rng.integers(0, D, Q), rng.integers(0, M, Q), rng.integers(0, M, Q),
                  rng.integers(0, M, Q), rng.integers(0, M, Q)], axis=1).astype(np.int64)
    # out-of-range queries give -1
    q[:3] = [[D, 0, 0, 0, 0], [0, M, 0, 0, 0], [-1, 0, 0, 0, 0]]
    got = mc.t2_lookup(torch.from_numpy(q).cuda(), tab).cpu().numpy()
    assert np.all(got[:3] == -1)
    occ = oracle_native.occ_rows(N, M, q[3:, 0])
    for (g, k, s, qq, l), n, v in zip(q[3:], occ, got[3:]):
        a, b = min(k, s), max(k, s)
        ok = (n[a] >= 2) if a == b else (n[a] >= 1 and n[b] >= 1)
        if not ok:
            assert v == -1
            continue
        m = n.copy()
        m[a] -= 1
        m[b] -= 1
        m[qq] += 1
        m[l] += 1
        assert v == oracle_native.hash_occ(m, N)


@pytest.mark.parametrize("N,M", [(10, 5), (200, 5), (50, 6), (300, 2), (4, 12)])
def test_hash_unhash_batch(mc, oracle_native, N, M):
    tab = mc.build_tables(N, M, double_jumps=False)
    D = tab.dim
    rng = np.random.default_rng(5)
    idx = np.concatenate([rng.integers(0, D, 5000), [0, D - 1, D, -1]]).astype(np.int64)
    occ = mc.unhash_batch(torch.from_numpy(idx).cuda(), tab).cpu().numpy()
    ref = oracle_native.occ_rows(N, M, idx[:-2])
    assert np.array_equal(occ[:-2], ref)
    assert np.all(occ[-2:] == -1)
    back = mc.hash_batch(torch.from_numpy(ref.astype(np.int32)).cuda(), tab).cpu().numpy()
    assert np.array_equal(back, idx[:-2])
    bad = ref[:2].copy()
    bad[0, 0] += 1          # wrong particle number
    bad[1, 0] = -1          # negative occupation
    assert np.all(mc.hash_batch(torch.from_numpy(bad.astype(np.int32)).cuda(), tab).cpu().numpy() == -1)


def test_large_space_sampled_rows(mc, oracle_native):
    """N = 200, M = 5 (dim 70,058,751): sampled rows, bit-exact."""
    N, M = 200, 5
    tab = mc.build_tables(N, M)
    D = tab.dim
    assert tab.t2_required >= int(mc.tables_size(N, M).t2_compact_entries)
    rng = np.random.default_rng(11)
    rows = np.unique(np.concatenate([rng.integers(0, D, 300), np.arange(64), D - 1 - np.arange(70)]))
    occ_t = tab.occ.view(torch.uint8)
    # occupations / single jumps of the sampled rows
    tiles, lanes = rows // 64, rows % 64
    o = occ_t.reshape(tab.tiles, M, 64)[torch.from_numpy(tiles).cuda(), :, torch.from_numpy(lanes).cuda()]
    assert np.array_equal(o.cpu().numpy().astype(np.int64), oracle_native.occ_rows(N, M, rows))
    t1 = tab.t1.reshape(tab.tiles, M, M, 64)[torch.from_numpy(tiles).cuda(), :, :, torch.from_numpy(lanes).cuda()]
    assert np.array_equal(t1.cpu().numpy(), oracle_native.t1_rows(N, M, rows))
    # double jumps through the lookup: every (k <= s, q, l) of each row
    ks = [(k, s) for k in range(M) for s in range(k, M)]
    q = np.array([[g, k, s, a, b] for g in rows for (k, s) in ks for a in range(M) for b in range(M)],
                 dtype=np.int64)
    got = mc.t2_lookup(torch.from_numpy(q).cuda(), tab).cpu().numpy()
    off, ent = oracle_native.t2_rows(N, M, rows)
    occ = oracle_native.occ_rows(N, M, rows)
    per = len(ks) * M * M
    for i, g in enumerate(rows):
        mine = got[i * per:(i + 1) * per].reshape(len(ks), M * M)
        keep = [j for j, (k, s) in enumerate(ks)
                if ((occ[i][k] >= 2) if k == s else (occ[i][k] >= 1 and occ[i][s] >= 1))]
        assert np.array_equal(mine[keep].reshape(-1), ent[off[i]:off[i + 1]])
        drop = [j for j in range(len(ks)) if j not in keep]
        assert np.all(mine[drop] == -1)
    del tab
    torch.cuda.empty_cache()
