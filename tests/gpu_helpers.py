"""Helpers for GPU parity tests: host-side remapping of the tiled tables and
the relative infinity-norm used as the floating-point bar."""

import numpy as np

TILE = 64
# two evaluations of the same sums in different orders (paths that group
# the terms differently) agree to this relative infinity-norm
ORDER_TOL = 1e-14


def rel_inf(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.max(np.abs(b)) if b.size else 0.0
    if den == 0.0:
        return float(np.max(np.abs(a - b))) if a.size else 0.0
    return float(np.max(np.abs(a - b)) / den)


def pair_list(M):
    return [(k, s) for k in range(M) for s in range(k, M)]


def pair_valid(occ, k, s):
    """occ: (R, M) array -> bool (R,)"""
    if k == s:
        return occ[:, k] >= 2
    return (occ[:, k] >= 1) & (occ[:, s] >= 1)


def pair_slots(M, k, s, form):
    """Slots of removal pair (k, s) in a double-jump block of the given form."""
    if form == "paper":
        return M * M
    return M * (M - 1) // 2 if k == s else (M - 1) * (M - 2) // 2


def tiled_t2_check_and_rows(tables, rows):
    """Reads the tiled double-jump map back and returns, for each requested
    row, its entries in the per-row layout of the tables' form (valid removal
    pairs in lexicographic order; M*M slots each in the paper form, the true
    double jumps in the reduced form).  Also asserts the layout invariants:
    pair mask = union of valid pairs over the tile, offsets consistent with
    the mask, and -1 padding for rows that cannot lose a pair."""
    M, D = tables.M, tables.dim
    form = tables.form
    slots = np.array([pair_slots(M, k, s, form) for k, s in pair_list(M)], dtype=np.int64)
    P = M * (M + 1) // 2
    W = (P + 63) // 64
    occ = tables.occupations()
    t2 = tables.t2.cpu().numpy()
    off = tables.t2_off.cpu().numpy()
    pm_words = tables.pmask.cpu().numpy().view(np.uint64).reshape(tables.tiles, W)
    bits = np.zeros((tables.tiles, P), dtype=bool)
    for p in range(P):
        bits[:, p] = (pm_words[:, p // 64] >> np.uint64(p % 64)) & np.uint64(1) == 1
    # mask is exactly the union over the tile's rows
    occ_pad = np.zeros((tables.tiles * TILE, M), dtype=np.int64)
    occ_pad[:D] = occ
    for p, (k, s) in enumerate(pair_list(M)):
        v = pair_valid(occ_pad, k, s).reshape(tables.tiles, TILE).any(axis=1)
        assert np.array_equal(v, bits[:, p]), ("pair mask", p)
    counts = (bits * slots[None, :]).sum(axis=1).astype(np.int64) * TILE
    assert off[0] == 0 and np.array_equal(np.diff(off), counts), "t2 offsets"
    assert tables.t2_required == off[-1]
    # start of each pair's block within its tile (in slots)
    start = np.cumsum(bits * slots[None, :], axis=1) - bits * slots[None, :]
    out = []
    for g in np.asarray(rows, dtype=np.int64):
        tile, lane = divmod(int(g), TILE)
        ent = []
        for p, (k, s) in enumerate(pair_list(M)):
            if not bits[tile, p]:
                continue
            base = off[tile] + start[tile, p] * TILE + lane
            blk = t2[base + np.arange(slots[p]) * TILE]
            n = occ[g]
            ok = (n[k] >= 2) if k == s else (n[k] >= 1 and n[s] >= 1)
            if ok:
                ent.append(blk)
            else:
                assert np.all(blk == -1), ("padding", g, p)
        out.append(np.concatenate(ent) if ent else np.zeros(0, np.int32))
    return out


def sampled_tables(tables, rows):
    """Occupations, single-jump rows and double-jump rows (per-row layout of
    the tables' form, as returned by the oracle) of the given rows only,
    gathered on the device: the tiled double-jump map is never copied whole.
    Also asserts that the tile's blocks of removal pairs a row cannot lose
    hold -1."""
    import torch

    M = tables.M
    P = M * (M + 1) // 2
    W = (P + 63) // 64
    rows = np.asarray(rows, dtype=np.int64)
    tiles, lanes = rows // TILE, rows % TILE
    dev = tables.t1.device
    ti, la = torch.from_numpy(tiles).to(dev), torch.from_numpy(lanes).to(dev)
    occ_t = tables.occ if tables.occ.dtype == torch.uint8 else tables.occ.view(torch.int16)
    o = occ_t.reshape(tables.tiles, M, TILE)[ti, :, la].cpu().numpy().astype(np.int64)
    if tables.occ.dtype != torch.uint8:
        o &= 0xFFFF
    t1 = tables.t1.reshape(tables.tiles, M, M, TILE)[ti, :, :, la].cpu().numpy()
    if tables.t2 is None:
        return o, t1, None
    slots = np.array([pair_slots(M, k, s, tables.form) for k, s in pair_list(M)], dtype=np.int64)
    pm_words = tables.pmask.reshape(tables.tiles, W)[ti].cpu().numpy().view(np.uint64)
    off = tables.t2_off[ti].cpu().numpy()
    idx, owner, valid_flag = [], [], []
    for r in range(rows.size):
        base = off[r]
        for p, (k, s) in enumerate(pair_list(M)):
            if not (int(pm_words[r, p // 64]) >> (p % 64)) & 1:
                continue
            blk = base + lanes[r] + np.arange(slots[p]) * TILE
            n = o[r]
            ok = (n[k] >= 2) if k == s else (n[k] >= 1 and n[s] >= 1)
            idx.append(blk)
            owner.append(np.full(slots[p], r))
            valid_flag.append(np.full(slots[p], ok))
            base += slots[p] * TILE
    idx = np.concatenate(idx)
    owner = np.concatenate(owner)
    valid_flag = np.concatenate(valid_flag)
    ent = tables.t2[torch.from_numpy(idx).to(dev)].cpu().numpy()
    assert np.all(ent[~valid_flag] == -1), "padding of removal pairs a row cannot lose"
    counts = np.bincount(owner[valid_flag], minlength=rows.size)
    per_row = np.split(ent[valid_flag], np.cumsum(counts)[:-1])
    return o, t1, per_row
