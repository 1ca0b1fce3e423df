"""Write the dense-oracle eigenvalues of the 64-atom cell to this folder.

    python tests/golden/make_config2_eigenvalues.py

The cell is the seeded 64-atom cubic cell (a = 20.5 bohr, Gamma, 25 Ry,
18,277 plane waves, grid 72^3, 256 projectors).  Its dense Hamiltonian
(5.3 GB complex128) is built by the CPU oracle row block by row block and
its lowest 128 eigenvalues are taken by LAPACK's MRRR driver through
``oracle.eigh_lowest``.  Nothing here touches the GPU library: the file
written is the oracle's, and the GPU tests of the full-size float64 and mixed
precision solves compare with it.  Takes several minutes on 8 cores and
about 16 GB of memory.

The iterative-diagonalization appendix defines the wanted result: the lowest
N solutions of H psi = eps psi (S = 1 here) in the plane-wave basis.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_0906_2569_amd import pwgen  # noqa: E402

OUT = os.path.join(HERE, "config2_eigenvalues.txt")


def main():
    p = pwgen.config2()
    t0 = time.perf_counter()
    h = oracle.dense_h_of(p)
    t1 = time.perf_counter()
    herm = float(np.abs(h - h.conj().T).max())
    w, _ = oracle.eigh_lowest(h, p.nb)
    t2 = time.perf_counter()
    with open(OUT, "w") as f:
        f.write("# lowest 128 eigenvalues (Ha, ascending) of the dense plane-wave Hamiltonian of the\n")
        f.write("# seeded 64-atom cell: a = 20.5 bohr, Gamma, ecutwfc 25 Ry, npw 18277, grid 72^3,\n")
        f.write("# 256 s/p projectors, diagonal D ~ U[0.5, 2] Ry; seed 20090602 (pwgen.config2).\n")
        f.write("# Written by tests/golden/make_config2_eigenvalues.py from the CPU float64 oracle\n")
        f.write(f"# (dense H built in {t1 - t0:.0f} s, max |H - H^H| = {herm:.2e}, eigh in {t2 - t1:.0f} s).\n")
        for x in w:
            f.write(f"{x:.17e}\n")
    print(f"wrote {OUT}: {len(w)} eigenvalues, [{w[0]:.12f}, {w[-1]:.12f}] Ha; "
          f"H {t1 - t0:.0f} s, eigh {t2 - t1:.0f} s")


if __name__ == "__main__":
    main()
