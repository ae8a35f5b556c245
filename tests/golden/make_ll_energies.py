"""Writes ll_energies.json: ground-state energies of the plane-wave
Lieb-Liniger Hamiltonian (Sec. VI) from the oracle alone -- oracle H.C,
oracle Lanczos with full reorthogonalisation, and the Bethe-ansatz solver.

    python tests/golden/make_ll_energies.py

N = 20 bosons on a ring of length L = 1, plane waves with momenta
2*pi*n, n = -(M-1)/2 .. (M-1)/2, M in {1, 3, 5, 7}; contact strength
c = gamma * N / L for gamma in {0.1, 1, 10}.  The start vector is seeded.
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import bethe, native  # noqa: E402
from oracle.lanczos import lanczos_ground  # noqa: E402


def main():
    N, L = 20, 1.0
    out = {"what": "oracle Lanczos and Bethe-ansatz ground-state energies of the plane-wave "
                   "Lieb-Liniger Hamiltonian, N = 20, L = 1",
           "script": "tests/golden/make_ll_energies.py", "N": N, "L": L, "runs": []}
    for gamma in (0.1, 1.0, 10.0):
        c = gamma * N / L
        e_ba = bethe.ground_energy(N, c, L)
        for M in (1, 3, 5, 7):
            h = W.lieb_liniger_h(M, L)
            g = W.lieb_liniger_g(M, c, L)
            D = native.dim(N, M)
            v0 = W.random_coefficients(np.random.default_rng(1000 + M), D)
            t0 = time.time()
            e0, a, b, it = lanczos_ground(lambda v: native.apply_h(N, M, h, g, v), v0,
                                          max_iter=min(D, 400), tol=1e-13, res_tol=1e-10)
            out["runs"].append({"gamma": gamma, "c": c, "M": M, "dim": D, "E0": float(e0),
                                "E_bethe": e_ba, "iterations": int(it)})
            print(f"gamma={gamma} M={M} D={D} E0={e0:.12f} E_BA={e_ba:.12f} it={it} "
                  f"({time.time() - t0:.0f} s)", flush=True)
    with open(os.path.join(HERE, "ll_energies.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
