"""The oracle's pins catch plausible mistakes (CPU only).

Each case copies oracle/mc_oracle.c to a temporary directory, plants one
mistake by text substitution, compiles it with gcc, swaps it in for the
oracle library, and runs the cheap pins.  Every planted mistake must make at
least one pin fail; the unmodified copy must pass them all.
"""

import ctypes
import os
import subprocess

import numpy as np
import pytest

import workloads as W
from oracle import combinatorics as cb
from oracle import dense
from tests.conftest import ROOT, golden

SRC = os.path.join(ROOT, "oracle", "mc_oracle.c")

MUTATIONS = {
    "drop_interaction_half": ("double amp = 0.5 * sqrt(amp2);", "double amp = sqrt(amp2);"),
    "transpose_h": ("double hr = h[2 * (k * M + l)], hi = h[2 * (k * M + l) + 1];",
                    "double hr = h[2 * (l * M + k)], hi = h[2 * (l * M + k) + 1];"),
    "creation_amplitude_off_by_one": ("    n[j] += 1;\n    return (double)n[j];",
                                      "    n[j] += 1;\n    return (double)(n[j] > 1 ? n[j] - 1 : 1);"),
    "total_cost_particle_count_off_by_one": ("            ++i;\n            index += orc_nc(i, orb);",
                                             "            index += orc_nc(i, orb);\n            ++i;"),
    "unhash_bisection_keeps_lower_bound": ("            if (orc_hash(N, M, n) <= beta) lo = mid;",
                                           "            if (orc_hash(N, M, n) < beta) lo = mid;"),
    "rho_missing_conjugate": ("double ar = C[2 * gamma], ai = -C[2 * gamma + 1];   /* conj(C_gamma) */",
                              "double ar = C[2 * gamma], ai = C[2 * gamma + 1];"),
    # counts only (the row writer keeps the right rule, so rows get shorter
    # than their lengths, never longer)
    "same_orbital_removal_one_particle": ("            if (k == s) { if (n[k] >= 2) ++p; }",
                                          "            if (k == s) { if (n[k] >= 1) ++p; }"),
    "reduced_map_wrong_creation_order": (
        "for (int32_t l = q; l < M; ++l) {\n                        if (q == k",
        "for (int32_t l = 0; l <= q; ++l) {\n                        if (q == k"),
    "reduced_map_keeps_shared_orbital": (
        "                        if (q == k || q == s || l == k || l == s) continue;",
        "                        if (q == k || l == s) continue;"),
    "unhash_remainder_dropped": ("    n[0] = left;\n    return 0;",
                                 "    return 0;"),
}


def build_variant(tmp_path, name, old, new):
    text = open(SRC).read()
    if old is not None:
        assert text.count(old) == 1, f"mutation {name} does not match the oracle source"
        text = text.replace(old, new)
    src = tmp_path / f"{name}.c"
    src.write_text(text)
    lib = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", str(lib),
                           str(src), "-lm"])
    return str(lib)


def pin_checks(native):
    """Cheap pins; returns the names of those that fail."""
    failed = []

    def check(name, fn):
        try:
            fn()
        except AssertionError:
            failed.append(name)

    def worked_example():
        ex = golden("hash_worked_example.json")
        assert native.hash_occ(ex["occupation"], ex["N"]) == ex["index"]
        assert list(native.unhash(ex["index"], ex["N"], ex["M"])) == ex["occupation"]

    def bijection():
        N, M = 4, 4
        occ = np.array(list(cb.compositions(N, M)), dtype=np.int32)
        idx = native.hash_rows(occ, N)
        assert sorted(idx) == list(range(cb.dim(N, M)))
        assert np.array_equal(native.occ_rows(N, M, idx), occ)

    def dense_bruteforce():
        for N, M, seed in ((3, 3, 1), (2, 4, 2)):
            C, h, g = W.random_instance(N, M, seed)
            H = dense.hamiltonian(N, M, h, g)
            assert np.allclose(native.apply_h(N, M, h, g, C), H @ C, atol=1e-12)

    def single_particle():
        M = 5
        C, h, g = W.random_instance(1, M, 3)
        hn = h + 0.5j * np.triu(np.ones((M, M)), 1)
        assert np.allclose(native.apply_h(1, M, hn, g, C), hn @ C, atol=1e-13)

    def pair_counting():
        N, M = 6, 3
        C, _, _ = W.random_instance(N, M, 2)
        d = np.eye(M)
        g = 0.5 * (np.einsum("kl,sq->ksql", d, d) + np.einsum("kq,sl->ksql", d, d))
        assert np.allclose(native.apply_h(N, M, np.zeros((M, M)), g, C), 0.5 * N * (N - 1) * C,
                           atol=1e-12)

    def rho_invariants():
        N, M = 4, 3
        C, h, g = W.random_instance(N, M, 5)
        r1 = native.rho1(N, M, C)
        r2 = native.rho2(N, M, C)
        assert abs(np.trace(r1) - N) < 1e-12
        assert np.allclose(r1, r1.conj().T, atol=1e-13)
        E1 = np.vdot(C, native.apply_h(N, M, h, g, C))
        assert abs(E1 - (np.sum(h * r1) + 0.5 * np.sum(g * r2))) < 1e-12

    def jump_counts():
        ex = golden("double_jump_example.json")
        N, M = ex["N"], ex["M"]
        lens = native.t2_row_lengths(N, M)
        assert lens.sum() == M * M * (M * (M + 1) // 2) * cb.nc(N - 2, M)
        off, ent = native.t2_rows(N, M)
        assert len(ent) == lens.sum()

    def reduced_map():
        N, M = 5, 4
        occ = native.occ_rows(N, M)
        off, ent = native.t2r_rows(N, M)
        per = M * (M * (M - 1) // 2) + (M * (M - 1) // 2) * ((M - 1) * (M - 2) // 2)
        assert off[-1] == per * cb.nc(N - 2, M)
        for gam in range(occ.shape[0]):
            n = occ[gam]
            want = []
            for k in range(M):
                for s in range(k, M):
                    if not (n[k] >= 2 if k == s else (n[k] >= 1 and n[s] >= 1)):
                        continue
                    for q in range(M):
                        for l in range(q, M):
                            if q in (k, s) or l in (k, s):
                                continue
                            m = n.copy()
                            m[k] -= 1
                            m[s] -= 1
                            m[q] += 1
                            m[l] += 1
                            want.append(cb.index_of(list(m)))
            assert list(ent[off[gam]:off[gam + 1]]) == want

    for name, fn in [("worked_example", worked_example), ("reduced_map", reduced_map), ("bijection", bijection),
                     ("dense_bruteforce", dense_bruteforce), ("single_particle", single_particle),
                     ("pair_counting", pair_counting), ("rho_invariants", rho_invariants),
                     ("jump_counts", jump_counts)]:
        check(name, fn)
    return failed


def load_into(native, path):
    lib = ctypes.CDLL(path)
    i32, i64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.orc_nc.argtypes = [i64, i64]
    lib.orc_nc.restype = i64
    lib.orc_hash.argtypes = [i32, i32, p]
    lib.orc_hash.restype = i64
    lib.orc_unhash.argtypes = [i32, i32, i64, p]
    lib.orc_unhash.restype = ctypes.c_int
    lib.orc_apply_h_rows.argtypes = [i32, i32, p, p, p, p, i64, p]
    lib.orc_rho1.argtypes = [i32, i32, p, p]
    lib.orc_rho2.argtypes = [i32, i32, p, p]
    lib.orc_rho2_elements.argtypes = [i32, i32, p, p, i64, p]
    lib.orc_occ_rows.argtypes = [i32, i32, p, i64, p]
    lib.orc_t1_rows.argtypes = [i32, i32, p, i64, p]
    lib.orc_t2_row_lengths.argtypes = [i32, i32, p, i64, p]
    lib.orc_t2_rows.argtypes = [i32, i32, p, i64, p, p]
    lib.orc_t2r_row_lengths.argtypes = [i32, i32, p, i64, p]
    lib.orc_t2r_rows.argtypes = [i32, i32, p, i64, p, p]
    lib.orc_hash_rows.argtypes = [i32, i32, p, i64, p]
    return lib


@pytest.fixture
def swap_oracle(monkeypatch):
    from oracle import native

    def swap(path):
        monkeypatch.setattr(native, "_lib", load_into(native, path))
        return native
    return swap


def test_unmodified_copy_passes(tmp_path, swap_oracle):
    native = swap_oracle(build_variant(tmp_path, "clean", None, None))
    assert pin_checks(native) == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(tmp_path, swap_oracle, name):
    old, new = MUTATIONS[name]
    native = swap_oracle(build_variant(tmp_path, name, old, new))
    failed = pin_checks(native)
    assert failed, f"mutation {name} was not caught by any pin"
