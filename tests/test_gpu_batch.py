"""Batched persistent H.C, segmented Lanczos operations, graph capture and
the schedule autotuner."""

import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_helpers import rel_inf

pytestmark = pytest.mark.gpu

# (N, M, double-jump map, form)
SHAPES = [(8, 3, True, "paper"), (12, 4, False, "paper"), (3, 8, True, "paper"),
          (10, 5, False, "paper"), (9, 5, True, "paper"), (1, 6, False, "paper"),
          (20, 3, False, "paper"), (6, 7, True, "paper"), (2, 2, True, "paper"),
          (15, 6, False, "paper"), (8, 8, False, "paper"), (5, 7, False, "paper"),
          (4, 8, True, "paper"), (11, 5, True, "reduced"), (9, 4, False, "reduced"),
          (6, 8, False, "reduced"), (5, 7, True, "reduced"), (2, 2, True, "reduced"),
          (3, 1, False, "reduced"), (12, 6, False, "reduced"),
          # table-free instances (descriptors with sizes only)
          (7, 5, False, "direct"), (10, 3, False, "direct"), (4, 8, False, "direct"),
          (14, 6, False, "direct"), (1, 2, False, "direct"), (9, 7, False, "direct")]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.fixture(scope="module")
def small_batch(mc):
    from paper_2005_13679_amd.batch import Batch
    insts, host = [], []
    for i, (N, M, t2, form) in enumerate(SHAPES):
        C, h, g = W.random_instance(N, M, 100 + i)
        if form == "direct":
            tab = mc.DirectSpace(N, M)
        else:
            tab = mc.build_tables(N, M, double_jumps=t2, form=form)
        insts.append((tab, dev(h), dev(g)))
        host.append((N, M, C, h, g))
    return insts, host


def batch_vector(b, vecs):
    x = b.vector()
    for i, v in enumerate(vecs):
        b.segment(x, i).copy_(dev(v))
    return x


def test_batched_apply_equals_plain_and_oracle(mc, oracle_native, small_batch):
    from paper_2005_13679_amd.batch import Batch
    insts, host = small_batch
    b = Batch(insts)
    C = batch_vector(b, [x[2] for x in host])
    HC = b.apply_H(C, b.vector())
    for i, ((tab, hd, gd), (N, M, Ch, h, g)) in enumerate(zip(insts, host)):
        plain = mc.apply_H(hd, gd, b.segment(C, i).contiguous(), tab)
        assert torch.equal(b.segment(HC, i), plain), (N, M)
        assert rel_inf(plain.cpu().numpy(), oracle_native.apply_h(N, M, h, g, Ch)) <= 1e-12


def test_every_schedule_gives_identical_results(mc, small_batch):
    from paper_2005_13679_amd.autotune import CANDIDATES
    from paper_2005_13679_amd.batch import Batch
    insts, host = small_batch
    ref = None
    # plus thresholds that send every / some instances to launches of their own
    extra = [{"blocks_per_cu": 2, "order": 3, "solo_tiles": 1},
             {"blocks_per_cu": 1, "order": 0, "solo_tiles": 3},
             {"blocks_per_cu": 2, "order": 1, "solo_tiles": 0}]
    for sched in CANDIDATES + extra:
        b = Batch(insts, sched)
        C = batch_vector(b, [x[2] for x in host])
        out = b.apply_H(C, b.vector())
        if ref is None:
            ref = out
        else:
            assert torch.equal(out, ref), sched


def test_segmented_vector_ops(mc, small_batch):
    from paper_2005_13679_amd.batch import Batch
    insts, host = small_batch
    b = Batch(insts)
    rng = np.random.default_rng(1)
    xs = [rng.standard_normal(t.dim) + 1j * rng.standard_normal(t.dim) for t, _, _ in insts]
    ys = [rng.standard_normal(t.dim) + 1j * rng.standard_normal(t.dim) for t, _, _ in insts]
    x, y = batch_vector(b, xs), batch_vector(b, ys)
    d = torch.empty(b.count, dtype=torch.complex128, device=b.device)
    b.dot(x, y, d)
    for i in range(b.count):
        assert abs(d[i].item() - np.vdot(xs[i], ys[i])) <= 1e-12 * np.sum(np.abs(xs[i]) * np.abs(ys[i]))
    beta = torch.empty(b.count, dtype=torch.float64, device=b.device)
    z = b.vector()
    b.normalize(x, z, beta)
    for i in range(b.count):
        assert abs(beta[i].item() - np.linalg.norm(xs[i])) <= 1e-12 * np.linalg.norm(xs[i])
        assert np.allclose(b.segment(z, i).cpu().numpy(), xs[i] / np.linalg.norm(xs[i]), atol=1e-14)
    alpha = d.clone()
    w = x.clone()
    b.lanczos_orth(w, y, z, alpha, beta)
    for i in range(b.count):
        ref = xs[i] - alpha[i].real.item() * ys[i] - beta[i].item() * (xs[i] / np.linalg.norm(xs[i]))
        assert np.allclose(b.segment(w, i).cpu().numpy(), ref, atol=1e-12)


def test_graph_replays_match_eager_and_plain(mc, small_batch):
    from paper_2005_13679_amd.batch import Batch, BatchedLanczos, plain_lanczos
    insts, host = small_batch
    b = Batch(insts)
    rng = np.random.default_rng(2)
    v0s = [W.random_coefficients(rng, t.dim) for t, _, _ in insts]
    v0 = batch_vector(b, v0s)
    steps = 12
    eager = BatchedLanczos(b, steps, graph=False)
    a_e, b_e = eager.run(v0)
    lz = BatchedLanczos(b, steps, graph=True)
    for rep in range(3):
        # unrelated eager work between replays
        junk = torch.randn(1 << 20, device=b.device).sum().item()
        assert np.isfinite(junk)
        a_g, b_g = lz.run(v0)
        assert np.array_equal(a_g, a_e) and np.array_equal(b_g, b_e), rep
    for i, (tab, hd, gd) in enumerate(insts):
        n = min(steps, tab.dim)
        a_p, b_p = plain_lanczos(tab, hd, gd, dev(v0s[i]), steps)
        a_p = a_p.real.cpu().numpy()
        b_p = b_p.cpu().numpy()
        # the recurrence amplifies rounding differences once the Krylov space
        # is exhausted (tiny dimensions); compare the steps before that
        k = min(n - 1, steps)
        assert np.allclose(a_g[:k, i], a_p[:k], rtol=1e-10, atol=1e-10), i
        assert np.allclose(b_g[:k, i], b_p[:k], rtol=1e-10, atol=1e-10), i


def test_autotuner_caches(mc, small_batch, tmp_path):
    from paper_2005_13679_amd import autotune
    insts, _ = small_batch
    path = str(tmp_path / "tune.json")
    r1 = autotune.tune(insts, cache_path=path, candidates=autotune.CANDIDATES[:3], reps=1)
    assert not r1["cached"] and r1["schedule"] in autotune.CANDIDATES[:3]
    r2 = autotune.tune(insts, cache_path=path)
    assert r2["cached"] and r2["schedule"] == r1["schedule"]


def test_table_free_batch_of_large_instances(mc, oracle_native):
    """Table-free instances, some large enough for launches of their own
    (N = 40, M = 8: dim 62,891,499 is the largest draw of the 64-instance
    workload), against the plain table-free apply; sampled rows vs the oracle."""
    from paper_2005_13679_amd.batch import Batch
    shapes = [(40, 8), (30, 6), (12, 7), (25, 4), (8, 3)]
    insts, host = [], []
    for i, (N, M) in enumerate(shapes):
        _, h, g = W.random_instance(1, M, 500 + i)
        insts.append((mc.DirectSpace(N, M), dev(h), dev(g)))
        host.append((N, M, h, g))
    b = Batch(insts, {"blocks_per_cu": 2, "order": 3, "solo_tiles": 16384})
    rng = np.random.default_rng(77)
    C = b.vector()
    C.copy_(torch.complex(torch.randn(b.length, dtype=torch.float64, device="cuda"),
                          torch.randn(b.length, dtype=torch.float64, device="cuda")))
    HC = b.apply_H(C, b.vector())
    for i, ((sp, hd, gd), (N, M, h, g)) in enumerate(zip(insts, host)):
        Ci = b.segment(C, i).contiguous()
        plain = mc.apply_H(hd, gd, Ci, sp)
        assert torch.equal(b.segment(HC, i), plain), (N, M)
        rows = np.unique(np.concatenate([rng.integers(0, sp.dim, 300), [0, sp.dim - 1]]))
        ref = oracle_native.apply_h(N, M, h, g, Ci.cpu().numpy(), rows)
        assert rel_inf(plain[torch.from_numpy(rows).cuda()].cpu().numpy(), ref) <= 1e-12
    del b, C, HC
    torch.cuda.empty_cache()


def test_batch_rejects_unsupported(mc):
    from paper_2005_13679_amd.batch import Batch
    tab = mc.build_tables(300, 2)   # N > 255: 16-bit occupations
    with pytest.raises(mc.MCError):
        Batch([(tab, np.eye(2), np.zeros((2, 2, 2, 2)))])


def test_batched_lanczos_convenience(mc, small_batch):
    insts, _ = small_batch
    a1, b1 = mc.batched_lanczos(insts, steps=6, seed=3)
    a2, b2 = mc.batched_lanczos(insts, steps=6, seed=3, graph=False)
    assert a1.shape == (6, len(insts)) and np.array_equal(a1, a2) and np.array_equal(b1, b2)
