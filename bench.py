"""Throughput of the bosonic H.C apply on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large_random|small_random]

A step is one H.C apply (Eq. Haction) through the jump maps on the workload
N = 200 bosons, M = 5 orbitals (dim 70,058,751), complex128 coefficients;
inputs and tables are resident in HBM before timing starts.  The timed path
is the case-split sum over the reduced double-jump map by default
(--path), the other paths are timed beside it.  Prints one JSON
line with applies/s, the HBM roofline of the apply kernel (algorithmic bytes
per apply / mean kernel time from HIP events on the launch stream) and the
CPU oracle timed on a bounded sample of rows on this host.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "large_random": dict(N=200, M=5, seed=2),
    "small_random": dict(N=10, M=5, seed=0),
    "autograd_size": dict(N=50, M=6, seed=3),
}


# How the apply runs: (table form, double-jump map present)
PATHS = {
    "reduced_map": ("reduced", True),      # case-split sum, reduced double-jump map
    "reduced_chained": ("reduced", False),  # case-split sum, true double jumps chained
    "paper_map": ("paper", True),          # the paper's sum and double-jump map
    "paper_chained": ("paper", False),     # the paper's sum, every slot chained
    "direct": (None, False),               # case-split sum, no table: targets in closed form
}
# dominant kernel of each path (the one the roofline and profiles refer to)
KERNELS = {
    "reduced_map": "k_apply_split<5, uint8, false, MAP=true>",
    "reduced_chained": "k_apply_split<5, uint8, false, MAP=false>",
    "paper_map": "k_apply<5, uint8, false>",
    "paper_chained": "k_apply_chained<5, uint8, false>",
    "direct": "k_apply_direct<5, false>",
}


def algorithmic_bytes(N: int, M: int, path: str = "reduced_map") -> dict:
    """Bytes one apply must move, each structure once: dense single-jump map
    (M^2 D int32), the double-jump rows of the path's form (paper: M^2 slots
    per valid removal pair, M^2 * M(M+1)/2 * N_c(N-2, M) entries; reduced: the
    true double jumps, [M * M(M-1)/2 + M(M-1)/2 * (M-1)(M-2)/2] * N_c(N-2, M)
    entries; none when chained), per-row offsets (D+1 int64, with a map),
    occupations (M D uint8), coefficients in and out (16 D each).  The
    table-free path reads no table: coefficients in and out only."""
    form, has_map = PATHS[path]
    D = math.comb(N + M - 1, N)
    if form is None:
        parts = {"coefficients_in": 16 * D, "coefficients_out": 16 * D}
        parts["total"] = sum(parts.values())
        return parts
    nc2 = math.comb(N - 2 + M - 1, N - 2) if N >= 2 else 0
    if form == "paper":
        per_row = M * M * (M * (M + 1) // 2)
    else:
        per_row = M * (M * (M - 1) // 2) + (M * (M - 1) // 2) * ((M - 1) * (M - 2) // 2)
    parts = {
        "t1": 4 * M * M * D,
        "t2": 4 * per_row * nc2 if has_map else 0,
        "offsets": 8 * (D + 1) if has_map else 0,
        "occupations": M * D * (1 if N <= 255 else 2),
        "coefficients_in": 16 * D,
        "coefficients_out": 16 * D,
    }
    parts["total"] = sum(parts.values())
    return parts


def stream_bytes(mc, tab) -> dict:
    """Bytes the apply kernel must move, each once, through the double-jump
    map of `tab` (either form, tiled layout): on a tile where every removal
    pair occurs and the double-jump block is complete, only the class
    anchors' table columns (mc.apply_stream_columns: the other jumps' targets
    follow from the anchors' by index arithmetic along runs); on the other
    tiles every single-jump column and the tile's whole double-jump block;
    plus the occupations, the tile masks and offsets, and the coefficients
    in and out."""
    import torch
    M, D, tiles = tab.M, tab.dim, tab.tiles
    slots, cols = mc.apply_stream_columns(M, tab.form)
    nsing = M * (M - 1)
    P = M * (M + 1) // 2
    W = (P + 63) // 64
    off = tab.t2_off[: tiles + 1]
    blk = off[1:] - off[:-1]
    full = blk == (slots - nsing) * 64
    pm = tab.pmask[: tiles * W].reshape(tiles, W)
    for w in range(W):
        bits = min(64, P - 64 * w)
        want = -1 if bits == 64 else (1 << bits) - 1
        full &= pm[:, w] == want
    nfull = int(full.sum().item()) if 2 <= M <= 5 else 0
    partial_blk = int(blk.sum().item()) - (int(blk[full].sum().item()) if nfull else 0)
    table = 4 * 64 * (nfull * cols + (tiles - nfull) * nsing) + 4 * partial_blk
    parts = {
        "table_columns_read": table,
        "occupations": tab.occ.numel() * tab.occ.element_size(),
        "tile_masks_offsets": 8 * (tiles * W + tiles + 1),
        "coefficients_in": 16 * D,
        "coefficients_out": 16 * D,
        "full_tiles": nfull,
        "tiles": tiles,
        "anchor_columns": cols,
        "slots": slots,
    }
    parts["total"] = sum(v for k, v in parts.items()
                         if k not in ("full_tiles", "tiles", "anchor_columns", "slots"))
    del torch
    return parts


# what the counters show limits each path's apply kernel (the HBM roofline is
# the one that bounds the byte model; these kernels stop short of it)
LIMITERS = {
    "reduced_map": "texture data path (98 % busy, 36 % of it waiting on L1 misses of the anchor "
                   "gathers) and vector ALU (2,550 instructions per tile, about 68 % of the "
                   "cycles): 195 vector memory reads per tile; HBM-side traffic 27.1 GB per apply "
                   "at 3.4 TB/s (rocprofv3 FETCH_SIZE)",
    "reduced_chained": "coefficient gathers through L1/TA (chained second hops)",
    "paper_map": "vector ALU (the paper's 395 slots of arithmetic per row on 131 gathered "
                 "targets) and the anchor gathers",
    "paper_chained": "coefficient gathers through L1/TA (chained second hops)",
    "direct": "vector ALU (closed-form targets and amplitudes) and coefficient gathers",
}
TARGET_FRAC = 0.60   # of HBM peak on the path's byte model, N = 200, M = 5
FP64_PEAK_TFLOPS = 78.6


def rho_models(N: int, M: int) -> dict:
    """Algorithmic work of the Gram-matrix density matrices: rho1 over the
    configurations of N-1 particles (M columns), rho2 over those of N-2
    (P = M(M+1)/2 columns); flops = 8 per complex product over the unique
    (upper-triangle) Gram entries.  Bytes: the table-free kernels read C
    (16 D); through the maps they also read the occupations (M D), the
    single jumps out of orbital 0 (4 (M-1) per intermediate) and, for rho2,
    the (0,0) block of the paper-form double-jump map (4 M(M-1)/2 per
    intermediate)."""
    D = math.comb(N + M - 1, N)
    D1 = math.comb(N - 1 + M - 1, N - 1) if N >= 1 else 0
    D2 = math.comb(N - 2 + M - 1, N - 2) if N >= 2 else 0
    P = M * (M + 1) // 2
    return {
        "rho1": {"flops": 8 * D1 * (M * (M + 1) // 2), "bytes_direct": 16 * D,
                 "bytes_maps": 16 * D + M * D + 4 * (M - 1) * D1},
        "rho2": {"flops": 8 * D2 * (P * (P + 1) // 2), "bytes_direct": 16 * D,
                 "bytes_maps": 16 * D + M * D + 4 * (M - 1) * D2 + 4 * (M * (M - 1) // 2) * D2},
    }


# sources each path's apply kernel is built from
KERNEL_SOURCES = {
    "reduced_map": ("mc_ops.hip", "mc_internal.h", "mc_apply.h", "mc_split.h"),
    "reduced_chained": ("mc_ops.hip", "mc_internal.h", "mc_apply.h", "mc_split.h"),
    "paper_map": ("mc_ops.hip", "mc_internal.h", "mc_apply.h", "mc_split.h"),
    "paper_chained": ("mc_ops.hip", "mc_internal.h", "mc_apply.h"),
    "direct": ("mc_ops.hip", "mc_internal.h", "mc_apply.h", "mc_split.h", "mc_direct.h"),
}


def kernel_source_hash(path: str = "reduced_map") -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[path]:
        with open(os.path.join(ROOT, "paper_2005_13679_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(N: int, M: int, path_name: str):
    """HBM bytes per apply from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"{path_name}_N{N}_M{M}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_source_hash(path_name):
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(N, M, h, g, C, budget_s: float = 15.0) -> dict:
    """The oracle (plain C, OpenMP over rows) on a seeded sample of rows, scaled
    to whole applies per second."""
    from oracle import native
    native.build(force=False)
    D = C.size
    rng = np.random.default_rng(12345)
    pilot = rng.integers(0, D, 2000)
    t0 = time.perf_counter()
    native.apply_h(N, M, h, g, C, pilot)
    rate = len(pilot) / (time.perf_counter() - t0)
    n = int(min(D, max(2000, rate * budget_s)))
    rows = rng.integers(0, D, n)
    t0 = time.perf_counter()
    native.apply_h(N, M, h, g, C, rows)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": (n / dt) / D,
        "unit": "applies/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{n} seeded random rows of the {D}-row apply in {dt:.1f} s "
                  f"({n / dt:.0f} rows/s), scaled by rows",
    }


def make_apply(mc, name, N, M, dev, hd, gd, Cd, HC):
    """(apply closure, tables or None) of one path."""
    form, has_map = PATHS[name]
    if form is None:
        return (lambda: mc.apply_H_direct(hd, gd, Cd, N, M, out=HC)), None
    tab = mc.build_tables(N, M, dev, double_jumps=has_map, form=form)
    return (lambda: mc.apply_H(hd, gd, Cd, tab, out=HC)), tab


def _median_ms(fn, reps, stream):
    import torch
    times = []
    for _ in range(reps):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record(stream)
        fn()
        e.record(stream)
        torch.cuda.synchronize()
        times.append(s.elapsed_time(e))
    times.sort()
    return times[len(times) // 2]


def autograd_leg(dev) -> dict:
    """E = <C|H C> forward + backward (dC, dh, dg) vs one plain apply, N=50, M=6."""
    import torch
    import paper_2005_13679_amd as mc
    import workloads as W
    N, M = 50, 6
    C, h, g = W.random_instance(N, M, 3)
    Cd, hd, gd = (torch.from_numpy(x).to(dev) for x in (C, h, g))
    HC = torch.empty_like(Cd)
    stream = torch.cuda.current_stream(dev)
    Cg, hg, gg = (x.clone().requires_grad_(True) for x in (Cd, hd, gd))

    def with_tables(form):
        tab = mc.build_tables(N, M, dev, form=form)
        mc.apply_H(hd, gd, Cd, tab, out=HC)
        plain = _median_ms(lambda: mc.apply_H(hd, gd, Cd, tab, out=HC), 10, stream)

        def fwd_bwd():
            for x in (Cg, hg, gg):
                x.grad = None
            mc.energy(Cg, hg, gg, tab).real.backward()

        fwd_bwd()
        full = _median_ms(fwd_bwd, 5, stream)
        rho2 = _median_ms(lambda: mc.rho2(Cd, tab), 5, stream)
        rho1 = _median_ms(lambda: mc.rho1(Cd, tab), 5, stream)
        del tab
        torch.cuda.empty_cache()
        return plain, full, rho1, rho2

    plain, full, rho1, rho2 = with_tables("paper")
    plain_r, full_r, rho1_r, rho2_r = with_tables("reduced")
    rm = rho_models(N, M)
    # the same with no table
    sp = mc.DirectSpace(N, M, dev)
    mc.apply_H(hd, gd, Cd, sp, out=HC)
    plain_d = _median_ms(lambda: mc.apply_H(hd, gd, Cd, sp, out=HC), 10, stream)

    def fwd_bwd_d():
        for x in (Cg, hg, gg):
            x.grad = None
        mc.energy(Cg, hg, gg, sp).real.backward()

    fwd_bwd_d()
    full_d = _median_ms(fwd_bwd_d, 5, stream)
    rho2_d = _median_ms(lambda: mc.rho2(Cd, sp), 5, stream)
    rho1_d = _median_ms(lambda: mc.rho1(Cd, sp), 5, stream)
    def roof(name, ms, via):
        f = rm[name]["flops"] / (ms * 1e-3) / 1e12
        b = rm[name][f"bytes_{via}"] / (ms * 1e-3) / 1e9
        return {"bound": "alu", "achieved": f, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": f / FP64_PEAK_TFLOPS, "algorithmic_GB_per_s": b,
                "frac_of_hbm_peak": b / HBM_PEAK_GBS}

    return {"workload": f"N={N}, M={M}, dim {C.size}", "plain_apply_ms": plain,
            "energy_fwd_bwd_ms": full, "ratio_fwd_bwd_over_apply": full / plain,
            "rho1_ms": rho1, "rho2_ms": rho2,
            "rho1_roofline": roof("rho1", rho1, "maps"), "rho2_roofline": roof("rho2", rho2, "maps"),
            "reduced_tables": {"plain_apply_ms": plain_r, "energy_fwd_bwd_ms": full_r,
                               "ratio_fwd_bwd_over_apply": full_r / plain_r,
                               "rho1_ms": rho1_r, "rho2_ms": rho2_r},
            "table_free": {"plain_apply_ms": plain_d, "energy_fwd_bwd_ms": full_d,
                           "ratio_fwd_bwd_over_apply": full_d / plain_d,
                           "rho1_ms": rho1_d, "rho2_ms": rho2_d,
                           "rho1_roofline": roof("rho1", rho1_d, "direct"),
                           "rho2_roofline": roof("rho2", rho2_d, "direct")}}


def sil_leg(dev, N: int = 200, M: int = 5, dt: float = 1e-5, tol: float = 1e-10) -> dict:
    """One Short Iterative Lanczos step exp(-i H dt) C on the throughput
    workload (reduced tables), adaptive Krylov dimension up to 16."""
    import torch
    import paper_2005_13679_amd as mc
    import workloads as W
    C, h, g = W.random_instance(N, M, 2)
    tab = mc.build_tables(N, M, dev, form="reduced")
    hd, gd, Cd = (torch.from_numpy(x).to(dev) for x in (h, g, C))
    st = mc.SILStepper(tab, hd, gd, kmax=16)
    out = torch.empty_like(Cd)
    st.step(Cd, dt, tol=tol, out=out)       # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out, m, err = st.step(Cd, dt, tol=tol, out=out)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    res = {"workload": f"N={N}, M={M}, dim {C.size}, reduced tables", "dt": dt, "tol": tol,
           "krylov_dim": m, "error_estimate": err, "step_ms": sec * 1e3,
           "ms_per_krylov_vector": sec * 1e3 / max(m, 1)}
    del st, tab
    torch.cuda.empty_cache()
    # the same step with no table
    st = mc.SILStepper(mc.DirectSpace(N, M, dev), hd, gd, kmax=16)
    out2 = torch.empty_like(Cd)
    st.step(Cd, dt, tol=tol, out=out2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out2, m2, _ = st.step(Cd, dt, tol=tol, out=out2)
    torch.cuda.synchronize()
    sec2 = time.perf_counter() - t0
    diff = float(torch.max(torch.abs(out - out2)) / torch.max(torch.abs(out)))
    res["table_free"] = {"krylov_dim": m2, "step_ms": sec2 * 1e3,
                         "rel_diff_vs_tables": diff}
    del st, out, out2, Cd
    torch.cuda.empty_cache()
    return res


def hbm_reference(dev, gib: float = 8.0) -> dict:
    """Achievable streaming rates on this GPU, for reading the roofline
    fractions: a device-to-device copy and a read-only reduction of `gib` GiB
    (torch's own kernels; context, not part of the path)."""
    import torch
    n = int(gib * (1 << 30)) // 8
    src = torch.ones(n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream(dev)
    dst.copy_(src)
    copy_ms = _median_ms(lambda: dst.copy_(src), 5, stream)
    src.sum()
    read_ms = _median_ms(lambda: src.sum(), 5, stream)
    del src, dst
    torch.cuda.empty_cache()
    nbytes = n * 8
    return {"copy_GB_per_s": 2 * nbytes / (copy_ms * 1e-3) / 1e9,
            "read_GB_per_s": nbytes / (read_ms * 1e-3) / 1e9, "size_GiB": gib}


def lieb_liniger_leg(dev) -> dict:
    """Plane-wave Lieb-Liniger ring (Sec. VI; momentum-conserving g): H.C at
    N=40, M=7 (dim 9,366,819) through each path, and the Lanczos ground state
    of N=20, M=7 (dim 230,230), gamma = 1, with the sparse apply."""
    import torch
    import paper_2005_13679_amd as mc
    from paper_2005_13679_amd import lanczos
    import workloads as W
    res = {}
    N, M = 40, 7
    h = torch.from_numpy(W.lieb_liniger_h(M)).to(dev)
    g = torch.from_numpy(W.lieb_liniger_g(M, 1.0 * N)).to(dev)
    C = torch.from_numpy(W.random_coefficients(np.random.default_rng(1), W.fock_dim(N, M))).to(dev)
    out = torch.empty_like(C)
    stream = torch.cuda.current_stream(dev)
    for name, form, maps, fn in (("paper_map", "paper", True, mc.apply_H),
                                 ("reduced_map", "reduced", True, mc.apply_H),
                                 ("sparse_reduced_map", "reduced", True, mc.apply_H_sparse),
                                 ("sparse_chained", "reduced", False, mc.apply_H_sparse)):
        tab = mc.build_tables(N, M, dev, double_jumps=maps, form=form)
        fn(h, g, C, tab, out=out)
        res[f"apply_ms_{name}"] = _median_ms(lambda: [fn(h, g, C, tab, out=out) for _ in range(10)],
                                              3, stream) / 10
        del tab
        torch.cuda.empty_cache()
    res["apply_workload"] = f"N={N}, M={M}, dim {C.numel()}, c = gamma N / L, gamma = 1"
    N, M = 20, 7
    h = torch.from_numpy(W.lieb_liniger_h(M)).to(dev)
    g = torch.from_numpy(W.lieb_liniger_g(M, 1.0 * N)).to(dev)
    tab = mc.build_tables(N, M, dev, form="reduced")
    v0 = torch.from_numpy(W.random_coefficients(np.random.default_rng(2), tab.dim)).to(dev)
    t0 = time.perf_counter()
    e0, a, b, it = lanczos.ground_state(h, g, tab, v0, sparse=True)
    torch.cuda.synchronize()
    res["lanczos"] = {"workload": f"N={N}, M={M}, dim {tab.dim}, gamma = 1", "E0": e0,
                      "iterations": int(it), "seconds": time.perf_counter() - t0}
    del tab
    torch.cuda.empty_cache()
    return res


def batched_leg(dev, steps: int = 50, table_free: bool = False) -> dict:
    """64 seeded instances (N ~ U{8..40}, M ~ U{3..8}): 50 Lanczos steps for all
    of them in one captured graph (autotuned schedule) vs the same steps per
    instance with the single-instance calls.  Tables in the reduced form
    (double-jump maps within a 40 GB budget, the rest chained), or no table
    at all (table_free)."""
    import torch
    import paper_2005_13679_amd as mc
    from paper_2005_13679_amd import autotune
    from paper_2005_13679_amd.batch import Batch, BatchedLanczos, choose_double_jumps, plain_lanczos
    import workloads as W
    draws = W.batch_draws(64, 4)
    use_t2 = ([False] * len(draws) if table_free
              else choose_double_jumps(draws, budget_bytes=40e9, form="reduced"))
    insts = []
    for i, ((N, M), t2) in enumerate(zip(draws, use_t2)):
        _, h, g = W.random_instance(1, M, 1000 + i)
        if table_free:
            tab = mc.DirectSpace(N, M, dev)
        else:
            tab = mc.build_tables(N, M, dev, double_jumps=t2, form="reduced")
        insts.append((tab, torch.from_numpy(h).to(dev), torch.from_numpy(g).to(dev)))
    total_dim = sum(t.dim for t, _, _ in insts)
    print(f"[bench] batched: {len(insts)} instances, total dim {total_dim}; autotuning",
          file=sys.stderr, flush=True)
    import tempfile
    tuned = autotune.tune(insts, cache_path=os.path.join(tempfile.gettempdir(), "mc_autotune_cache.json"),
                          reps=2)
    print(f"[bench] batched: schedule {tuned['schedule']}", file=sys.stderr, flush=True)
    b = Batch(insts, tuned["schedule"])
    apply_ms = autotune.time_schedule(insts, tuned["schedule"], reps=3)
    rng = np.random.default_rng(9)
    v0 = b.vector()
    for i, (t, _, _) in enumerate(insts):
        b.segment(v0, i).copy_(torch.from_numpy(W.random_coefficients(rng, t.dim)).to(dev))
    print(f"[bench] batched: one apply {apply_ms:.1f} ms; capturing {steps} Lanczos steps",
          file=sys.stderr, flush=True)
    lz = BatchedLanczos(b, steps, graph=True)
    a_b, be_b = lz.run(v0)                       # warm replay
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a_b, be_b = lz.run(v0)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    print(f"[bench] batched: graph replay {t_batch:.2f} s; per-instance plain runs",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    worst = 0.0
    for i, (t, hd, gd) in enumerate(insts):
        if i % 16 == 0:
            print(f"[bench] batched: plain instance {i}/{len(insts)}", file=sys.stderr, flush=True)
        a_p, b_p = plain_lanczos(t, hd, gd, b.segment(v0, i).contiguous(), steps)
        torch.cuda.synchronize()
        k = min(steps, t.dim - 1, 8)
        a_p = a_p.real.cpu().numpy()
        if k > 0:
            worst = max(worst, float(np.max(np.abs(a_p[:k] - a_b[:k, i]) / np.maximum(1.0, np.abs(a_p[:k])))))
    t_plain = time.perf_counter() - t0
    out = {"instances": len(insts), "total_dim": int(total_dim),
           "table_form": "none (table-free)" if table_free else "reduced",
           "table_bytes": int(sum(sum(t.nbytes().values()) for t, _, _ in insts)),
           "with_double_jump_map": int(sum(use_t2)), "steps": steps,
           "schedule": tuned["schedule"], "schedule_cached": tuned["cached"],
           "batched_apply_ms": apply_ms,
           "batched_graph_s": t_batch, "plain_eager_s": t_plain,
           "batched_instance_applies_per_s": len(insts) * steps / t_batch,
           "plain_instance_applies_per_s": len(insts) * steps / t_plain,
           "speedup": t_plain / t_batch, "max_rel_alpha_diff_first_steps": worst}
    del lz, b, insts
    torch.cuda.empty_cache()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large_random", choices=sorted(WORKLOADS))
    ap.add_argument("--path", default="reduced_map", choices=sorted(PATHS),
                    help="table form and double-jump source of the timed apply")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--extras", action="store_true", help="also time rho1/rho2 passes")
    ap.add_argument("--quick", action="store_true",
                    help="skip the other apply paths and the autograd and batched legs")
    ap.add_argument("--only", default=None,
                    choices=["autograd", "lieb_liniger", "sil", "batched", "batched_table_free"],
                    help="run one secondary leg alone and print its JSON (for profiling)")
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="run one elementwise copy of this size first (HBM counter scale)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "path is a design, not a build", file=sys.stderr)
        return 2

    import torch
    import paper_2005_13679_amd as mc
    import workloads as W

    if args.only:
        dev = torch.device("cuda", 0)
        torch.cuda.set_device(dev)
        legs = {"autograd": autograd_leg, "lieb_liniger": lieb_liniger_leg, "sil": sil_leg,
                "batched": batched_leg,
                "batched_table_free": lambda d: batched_leg(d, table_free=True)}
        print(f"[bench] leg {args.only}", file=sys.stderr, flush=True)
        print(json.dumps({args.only: legs[args.only](dev)}), flush=True)
        return 0

    wl = WORKLOADS[args.workload]
    N, M, seed = wl["N"], wl["M"], wl["seed"]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    print(f"[bench] workload {args.workload} N={N} M={M}: drawing inputs", file=sys.stderr, flush=True)
    C, h, g = W.random_instance(N, M, seed)
    D = C.size
    form, has_map = PATHS[args.path]
    Cd = torch.from_numpy(C).to(dev)
    hd = torch.from_numpy(h).to(dev)
    gd = torch.from_numpy(g).to(dev)
    HC = torch.empty_like(Cd)
    t0 = time.perf_counter()
    apply, tab = make_apply(mc, args.path, N, M, dev, hd, gd, Cd, HC)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    tab_bytes = tab.nbytes() if tab is not None else {}
    print(f"[bench] tables built in {build_s:.2f} s ({sum(tab_bytes.values()) / 1e9:.2f} GB)",
          file=sys.stderr, flush=True)

    if args.copy_calibration_gib > 0:
        n = int(args.copy_calibration_gib * (1 << 30)) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)   # reads and writes n * 8 bytes
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        apply()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(args.steps):
        apply()
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / args.steps
    print(f"[bench] {args.steps} applies ({args.path}): {ms:.3f} ms each", file=sys.stderr, flush=True)

    B = algorithmic_bytes(N, M, args.path)
    if has_map:
        B = stream_bytes(mc, tab)
    achieved = B["total"] / (ms * 1e-3) / 1e9
    traffic = measured_traffic(N, M, args.path)
    out = {
        "metric": f"H.C applies/s (N={N}, M={M}, complex128) with HBM GB/s",
        "value": 1e3 / ms,
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: N={N} bosons, M={M} orbitals, dim {D}, "
                               "complex128 C, random Hermitian h, symmetric g",
                   "N": N, "M": M, "dim": D, "path": args.path, "table_form": form,
                   "double_jump_map": has_map, "parallelism": "single GPU"},
        "roofline": {
            "kernel": KERNELS[args.path].replace("<5", f"<{M}"),
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_frac": (traffic / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS) if traffic else None,
            "target_frac": TARGET_FRAC,
            "meets_target": achieved / HBM_PEAK_GBS >= TARGET_FRAC,
            "limiter": LIMITERS[args.path],
        },
        "algorithmic_bytes_per_apply": B["total"],
        "algorithmic_bytes_parts": B,
        # the same apply against structure-once models of whole tables (the
        # kernel reads less; context only, not the roofline)
        "byte_models": {
            name: {"bytes": b, "equivalent_GB_per_s": b / (ms * 1e-3) / 1e9,
                   "equivalent_frac_of_peak": b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
            for name, b in (("reduced_tables_once", algorithmic_bytes(N, M, "reduced_map")["total"]),
                            ("paper_tables_once", algorithmic_bytes(N, M, "paper_map")["total"]))
        } if has_map else None,
        "table_build_s": build_s,
        "table_bytes": tab_bytes,
    }

    if args.extras and tab is not None:
        extras = {}
        for name, fn in (("rho1", lambda: mc.rho1(Cd, tab)), ("rho2", lambda: mc.rho2(Cd, tab))):
            fn()
            torch.cuda.synchronize()
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record(stream)
            fn()
            e.record(stream)
            torch.cuda.synchronize()
            extras[f"{name}_ms"] = s.elapsed_time(e)
        out["extras"] = extras

    if not args.quick:
        del apply, tab
        torch.cuda.empty_cache()
        others = {}
        for name, (f2, m2) in PATHS.items():
            if name == args.path:
                continue
            print(f"[bench] path {name}", file=sys.stderr, flush=True)
            ap2, t2 = make_apply(mc, name, N, M, dev, hd, gd, Cd, HC)
            for _ in range(2):
                ap2()
            ms2 = _median_ms(lambda: [ap2() for _ in range(5)], 3, stream) / 5
            B2 = (stream_bytes(mc, t2) if m2 else algorithmic_bytes(N, M, name))["total"]
            others[name] = {"ms_per_apply": ms2, "applies_per_s": 1e3 / ms2,
                            "algorithmic_bytes": B2, "GB_per_s": B2 / (ms2 * 1e-3) / 1e9,
                            "frac_of_hbm_peak": B2 / (ms2 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                            "table_bytes": sum(t2.nbytes().values()) if t2 is not None else 0,
                            "kernel": KERNELS[name].replace("<5", f"<{M}")}
            del ap2, t2
            torch.cuda.empty_cache()
        out["other_paths"] = others
        print("[bench] HBM streaming reference", file=sys.stderr, flush=True)
        out["hbm_reference"] = hbm_reference(dev)
        print("[bench] autograd leg (N=50, M=6)", file=sys.stderr, flush=True)
        out["autograd_vs_plain"] = autograd_leg(dev)
        print("[bench] Lieb-Liniger leg (sparse apply, Lanczos)", file=sys.stderr, flush=True)
        out["lieb_liniger"] = lieb_liniger_leg(dev)
        print("[bench] SIL propagation leg (N=200, M=5)", file=sys.stderr, flush=True)
        out["sil_step"] = sil_leg(dev)
        print("[bench] batched leg (64 instances, 50 Lanczos steps)", file=sys.stderr, flush=True)
        out["batched_vs_plain"] = batched_leg(dev)
        print("[bench] batched leg, table-free instances", file=sys.stderr, flush=True)
        out["batched_vs_plain_table_free"] = batched_leg(dev, table_free=True)

    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a row sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(N, M, h, g, C)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
