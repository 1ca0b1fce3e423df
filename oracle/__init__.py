"""CPU FP64 oracle (test infrastructure only; never called by the product path).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.
"""
from .dense import (kinetic, dft_matrix, vtilde_table, vtilde_lookup, dense_d, h_rows,
                    dense_h, dense_h_of, hpsi, hpsi_rows_of, hpsi_brute, h_diag,
                    eigh_lowest, davidson, reduced_eigh, secular_roots, kato_temple, density, scf_norm2,
                    pcg, dense_s, dense_s_of, eigh_lowest_gen)
