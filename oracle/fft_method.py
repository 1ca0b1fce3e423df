"""CPU FFT-method float64 H.psi: the fair CPU throughput baseline.

TEST INFRASTRUCTURE ONLY, and not the oracle's definition (that is
``dense.py``, which applies the explicit H_GG').  This module computes the
same product the way a CPU plane-wave code does -- scatter of the sphere
onto the FFT box, inverse 3D FFT, V(r) psi(r) in real space, forward FFT,
gather, kinetic diagonal, and the projector term as two BLAS products -- so
that the benchmark can time a CPU method of the same algorithmic order as
the GPU path beside the O(npw^2) dense oracle.  The CPU tests check it
against ``dense.py``.

Conventions as in ``dense.py``: psi(r_j) = sum_G psi_G exp(+i G.r_j)
(unscaled), (f)_G = (1/N) sum_j f(r_j) exp(-i G.r_j).  Uses scipy.fft with
every host core.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft


def _dense_blocks(nbeta, blk_off, dmat):
    """Block-diagonal D from the flat column-major blocks (entry (i, j) of a
    block at offset i + j*nh)."""
    d = np.zeros((nbeta, nbeta), dtype=np.complex128)
    flat = np.asarray(dmat, dtype=np.complex128).ravel()
    pos = 0
    for b in range(len(blk_off) - 1):
        o0, o1 = int(blk_off[b]), int(blk_off[b + 1])
        nh = o1 - o0
        for j in range(nh):
            d[o0:o1, o0 + j] = flat[pos + j * nh:pos + (j + 1) * nh]
        pos += nh * nh
    return d


def hpsi(miller, kpg, vloc_r, beta, blk_off, dmat, psi, workers=None):
    """H.psi for bands psi [nb][npw] by 3D FFTs and BLAS, in complex128."""
    workers = workers or os.cpu_count() or 1
    v = np.asarray(vloc_r, dtype=np.float64)
    n3, n2, n1 = v.shape
    n = n1 * n2 * n3
    m = np.asarray(miller, dtype=np.int64)
    i1, i2, i3 = m[:, 0] % n1, m[:, 1] % n2, m[:, 2] % n3
    kin = 0.5 * np.sum(np.asarray(kpg) ** 2, axis=1)
    psi = np.asarray(psi, dtype=np.complex128)
    out = kin[None, :] * psi
    box = np.zeros((n3, n2, n1), dtype=np.complex128)
    for b in range(psi.shape[0]):
        box[...] = 0.0
        box[i3, i2, i1] = psi[b]
        r = scipy.fft.ifftn(box, workers=workers, overwrite_x=True) * n
        r *= v
        f = scipy.fft.fftn(r, workers=workers, overwrite_x=True)
        out[b] += f[i3, i2, i1] / n
    beta = np.asarray(beta, dtype=np.complex128)
    if beta.shape[0]:
        d = _dense_blocks(beta.shape[0], blk_off, dmat)
        becp = np.conj(beta) @ psi.T                     # <beta_j|psi_b>   [nbeta][nb]
        out += (beta.T @ (d @ becp)).T                   # sum_ij beta_i D_ij <beta_j|psi>
    return out
