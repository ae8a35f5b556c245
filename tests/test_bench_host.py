"""bench.py's host-side contract (CPU only): one GPU, byte models."""

import math
import os
import subprocess
import sys

from tests.conftest import ROOT


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_byte_models():
    sys.path.insert(0, ROOT)
    import bench
    N, M = 200, 5
    D = math.comb(N + M - 1, N)
    nc2 = math.comb(N - 2 + M - 1, N - 2)
    paper = bench.algorithmic_bytes(N, M, "paper_map")
    assert paper["t2"] == 4 * 25 * 15 * nc2            # M^2 slots per removal pair
    assert abs(paper["total"] - 111.156e9) < 1e6
    red = bench.algorithmic_bytes(N, M, "reduced_map")
    assert red["t2"] == 4 * 110 * nc2                  # true double jumps of a full row
    chained = bench.algorithmic_bytes(N, M, "reduced_chained")
    assert chained["t2"] == 0 and chained["offsets"] == 0
    assert chained["total"] == 4 * 25 * D + 5 * D + 32 * D
    direct = bench.algorithmic_bytes(N, M, "direct")
    assert direct["total"] == 32 * D                   # no table: C in, HC out
    assert set(bench.PATHS) == set(bench.KERNELS)


def test_counter_records_follow_their_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench
    assert set(bench.KERNEL_SOURCES) == set(bench.PATHS)
    for p in bench.PATHS:
        assert len(bench.kernel_source_hash(p)) == 16
    # a table-free source change leaves the table paths' records valid
    assert "mc_direct.h" not in bench.KERNEL_SOURCES["reduced_map"]


def test_stream_byte_model_counts_full_tiles():
    """Full tiles read the anchor columns only; other tiles every
    single-jump column and their whole double-jump block."""
    import types

    import torch
    sys.path.insert(0, ROOT)
    import bench
    import paper_2005_13679_amd as mc
    M = 5
    slots, cols = mc.apply_stream_columns(M, "reduced")
    ndbl = slots - M * (M - 1)
    # tile 0 full; tile 1 misses pair 14; tile 2 has a short block
    blocks = [ndbl * 64, (ndbl - 1) * 64, (ndbl - 3) * 64]
    off = torch.tensor([0] + list(torch.tensor(blocks).cumsum(0)), dtype=torch.int64)
    full_mask = (1 << 15) - 1
    pmask = torch.tensor([full_mask, full_mask & ~(1 << 14), full_mask], dtype=torch.int64)
    tab = types.SimpleNamespace(M=M, dim=3 * 64 - 5, tiles=3, t2_off=off, pmask=pmask,
                                occ=torch.zeros(3 * 64 * M, dtype=torch.uint8), form="reduced")
    B = bench.stream_bytes(mc, tab)
    assert B["full_tiles"] == 1 and B["anchor_columns"] == 54
    assert B["table_columns_read"] == 4 * 64 * (54 + 2 * 20) + 4 * (blocks[1] + blocks[2])
    assert B["total"] == (B["table_columns_read"] + 3 * 64 * M + 8 * (3 + 4)
                          + 32 * tab.dim)
