"""CPU FP64 dense oracle for plane-wave H.psi and the block Davidson iteration.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
``cpu_baseline`` leg of the benchmark may import this module; the product
path never calls it.  It shares no code with the GPU library: no FFT, no
blocking, no fusion -- each function is the plain definition, written out in
NumPy/SciPy in float64 / complex128.

Hamiltonian in a plane-wave basis (Hartree atomic units), following the
Kohn-Sham equation of the self-consistency appendix (kinetic -hbar^2/2m
nabla^2 plus a potential), the separable projector form of the
pseudopotential (beta projectors, Sec. 3 and the SCF appendix's <psi|beta>
notation) and the plane-wave / FFT-grid representation of the parallelization
section:

    H_{GG'} = 1/2 |k+G|^2 delta_{GG'}                               (kinetic)
            + Vt((m_G - m_G') mod n)                                (local)
            + sum_I sum_{ij in I} beta_i(G) D^I_{ij} conj(beta_j(G'))  (nonlocal)

with Vt(dm) = (1/N) sum_j V(r_j) exp(-2 pi i sum_d dm_d j_d / n_d), the
discrete Fourier coefficient of the real potential sampled on the grid.
The forward transform convention is psi(r_j) = sum_G psi_G exp(+i G.r_j)
(unscaled); the Bloch factor exp(ik.r) commutes with V(r) and is not applied.

The Davidson routine follows the iterative-diagonalization appendix (block
Davidson: residuals g = (H - eps S) psi, corrections D g with the diagonal
preconditioner, reduced problem on span{psi, dpsi}, Ritz update, optional
expanding basis up to a fixed size), with S = 1.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg


# ----------------------------------------------------------------------------
# H.psi pieces
# ----------------------------------------------------------------------------

def kinetic(kpg: np.ndarray) -> np.ndarray:
    """Kinetic diagonal T_G = |k+G|^2 / 2 (Ha), from Cartesian k+G in bohr^-1."""
    kpg = np.asarray(kpg, dtype=np.float64)
    return 0.5 * np.sum(kpg * kpg, axis=1)


def dft_matrix(n: int, sign: int) -> np.ndarray:
    """Plain DFT matrix F[m, j] = exp(sign * 2 pi i m j / n)."""
    m = np.arange(n)
    return np.exp(sign * 2j * math.pi * np.outer(m, m) / n)


def vtilde_table(vloc_r: np.ndarray) -> np.ndarray:
    """Vt(dm) for every dm mod n, as a [n3][n2][n1] complex table.

    Direct discrete Fourier sums (three explicit DFT matrices, O(n^4)); no FFT.
    ``vloc_r`` is [n3][n2][n1] (x fastest).
    """
    v = np.asarray(vloc_r, dtype=np.float64)
    n3, n2, n1 = v.shape
    f1, f2, f3 = dft_matrix(n1, -1), dft_matrix(n2, -1), dft_matrix(n3, -1)
    t = np.einsum("mj,abj->abm", f1, v.astype(np.complex128))   # over j1
    t = np.einsum("mj,ajc->amc", f2, t)                          # over j2
    t = np.einsum("mj,jbc->mbc", f3, t)                          # over j3
    return t / float(n1 * n2 * n3)


def vtilde_lookup(vt: np.ndarray, dm: np.ndarray) -> np.ndarray:
    """Vt at integer offsets dm[..., 3] (h, k, l), wrapped mod the grid."""
    n3, n2, n1 = vt.shape
    return vt[dm[..., 2] % n3, dm[..., 1] % n2, dm[..., 0] % n1]


def dense_d(nbeta: int, blk_off, dmat) -> np.ndarray:
    """Block-diagonal D (nbeta x nbeta) from concatenated col-major blocks."""
    d = np.zeros((nbeta, nbeta), dtype=np.complex128)
    pos = 0
    for i in range(len(blk_off) - 1):
        o0, o1 = int(blk_off[i]), int(blk_off[i + 1])
        nh = o1 - o0
        d[o0:o1, o0:o1] = np.asarray(dmat[pos:pos + nh * nh]).reshape(nh, nh).T
        pos += nh * nh
    return d


def h_rows(miller, kpg, vloc_r, beta, blk_off, dmat, rows, vt=None) -> np.ndarray:
    """Rows ``rows`` of the dense Hamiltonian, shape [len(rows)][npw]."""
    miller = np.asarray(miller, dtype=np.int64)
    rows = np.asarray(rows, dtype=np.int64)
    if vt is None:
        vt = vtilde_table(vloc_r)
    dm = miller[rows][:, None, :] - miller[None, :, :]
    h = vtilde_lookup(vt, dm).astype(np.complex128)
    t = kinetic(kpg)
    h[np.arange(len(rows)), rows] += t[rows]
    beta = np.asarray(beta, dtype=np.complex128)
    if beta.shape[0] > 0:
        d = dense_d(beta.shape[0], blk_off, dmat)
        # sum_ij beta_i(G) D_ij conj(beta_j(G'))   (beta stored [nbeta][npw])
        h += (beta[:, rows].T @ d) @ np.conj(beta)
    return h


def dense_h(miller, kpg, vloc_r, beta, blk_off, dmat) -> np.ndarray:
    """The full dense npw x npw Hamiltonian."""
    npw = np.asarray(miller).shape[0]
    vt = vtilde_table(vloc_r)
    out = np.empty((npw, npw), dtype=np.complex128)
    step = 2048
    for r0 in range(0, npw, step):
        rows = np.arange(r0, min(npw, r0 + step))
        out[r0:r0 + len(rows)] = h_rows(miller, kpg, vloc_r, beta, blk_off, dmat, rows, vt=vt)
    return out


def dense_h_of(p) -> np.ndarray:
    """dense_h for a generated problem object."""
    return dense_h(p.miller, p.kpg, p.vloc_r, p.beta, p.blk_off, p.dmat)


def dense_s(npw, beta, blk_off, qmat) -> np.ndarray:
    """Overlap S = 1 + sum_I sum_ij beta_i q^I_ij beta_j^H of the ultrasoft form
    (the generalized problem H psi = eps S psi of the iterative-diagonalization
    appendix); q blocks laid out as the D blocks.  qmat None: S = 1."""
    s = np.eye(npw, dtype=np.complex128)
    beta = np.asarray(beta, dtype=np.complex128)
    if qmat is not None and beta.shape[0] > 0:
        q = dense_d(beta.shape[0], blk_off, qmat)
        s += beta.T @ q @ np.conj(beta)
    return s


def dense_s_of(p) -> np.ndarray:
    return dense_s(p.npw, p.beta, p.blk_off, getattr(p, "qmat", None))


def eigh_lowest_gen(h: np.ndarray, s: np.ndarray, nb: int):
    """Lowest nb solutions of H c = eps S c (S positive definite), ascending;
    eigenvectors S-orthonormal, as [nb][npw]."""
    w, v = scipy.linalg.eigh(h, s, subset_by_index=[0, nb - 1])
    return w, v.T.copy()


def hpsi(h: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """H.psi for bands stored [nb][npw]: (H psi_b)_G = sum_G' H_GG' psi_b(G')."""
    return np.asarray(psi) @ h.T


def hpsi_rows_of(p, psi, rows) -> np.ndarray:
    """(H psi)[:, rows] computed from explicit rows of H (for large cells)."""
    hr = h_rows(p.miller, p.kpg, p.vloc_r, p.beta, p.blk_off, p.dmat, rows)
    return np.asarray(psi) @ hr.T


def hpsi_brute(miller, kpg, vloc_r, beta, blk_off, dmat, psi) -> np.ndarray:
    """H.psi through real space by explicit sums (no H matrix, no FFT).

    psi(r_j) = sum_G psi_G exp(+2 pi i m_G.j/n); (V psi)(r) = V(r) psi(r);
    (V psi)_G = (1/N) sum_j exp(-2 pi i m_G.j/n) (V psi)(r_j); the projector
    term sum_ij beta_i D_ij <beta_j|psi> reads D from the flat block list
    itself (it does not go through dense_d).  For tiny cells.
    """
    miller = np.asarray(miller, dtype=np.int64)
    v = np.asarray(vloc_r, dtype=np.float64)
    n3, n2, n1 = v.shape
    j3, j2, j1 = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    frac = np.stack([j1.ravel() / n1, j2.ravel() / n2, j3.ravel() / n3], axis=1)
    phase = np.exp(2j * math.pi * (miller @ frac.T))           # [npw][N]
    psi = np.asarray(psi, dtype=np.complex128)
    out = np.empty_like(psi)
    t = kinetic(kpg)
    vflat = v.ravel()
    beta = np.asarray(beta, dtype=np.complex128)
    dflat = np.asarray(dmat, dtype=np.complex128).ravel()
    for b in range(psi.shape[0]):
        pr = psi[b] @ phase                                     # psi(r_j)
        vg = (np.conj(phase) @ (vflat * pr)) / vflat.size       # (V psi)_G
        acc = t * psi[b] + vg
        # nonlocal term walked block by block straight from the flat input:
        # block I starts at sum_{J<I} nh_J^2, and its element (i, j) (row i,
        # column j, column-major) sits at i + j*nh inside the block
        pos = 0
        for blk in range(len(blk_off) - 1):
            o0, o1 = int(blk_off[blk]), int(blk_off[blk + 1])
            nh = o1 - o0
            for j in range(nh):
                proj = np.vdot(beta[o0 + j], psi[b])              # <beta_j|psi>
                for i in range(nh):
                    dij = dflat[pos + i + j * nh]
                    if dij != 0:
                        acc = acc + beta[o0 + i] * dij * proj
            pos += nh * nh
        out[b] = acc
    return out


def h_diag(miller, kpg, vloc_r, beta, blk_off, dmat) -> np.ndarray:
    """Exact diagonal <k+G|H|k+G> (used by the Davidson preconditioner)."""
    v = np.asarray(vloc_r, dtype=np.float64)
    diag = kinetic(kpg) + float(np.mean(v))         # Vt(0) = mean of V(r)
    beta = np.asarray(beta, dtype=np.complex128)
    if beta.shape[0]:
        d = dense_d(beta.shape[0], blk_off, dmat)
        diag = diag + np.real(np.einsum("ig,ij,jg->g", beta, d, np.conj(beta)))
    return diag


# ----------------------------------------------------------------------------
# output density and scf norm (self-consistency appendix)
# ----------------------------------------------------------------------------

def density(miller, nr, psi, w, omega) -> np.ndarray:
    """rho(r_j) = (1/omega) sum_b w_b |psi_b(r_j)|^2 on the grid, [n3][n2][n1].

    psi_b(r_j) = sum_G psi_b(G) exp(+2 pi i m_G.j / n) by explicit phase sums
    (no FFT); the output-density equation of the self-consistency appendix
    with occupation weights w_b.  For small cells.
    """
    miller = np.asarray(miller, dtype=np.int64)
    n1, n2, n3 = (int(x) for x in nr)
    j3, j2, j1 = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    frac = np.stack([j1.ravel() / n1, j2.ravel() / n2, j3.ravel() / n3], axis=1)
    phase = np.exp(2j * math.pi * (miller @ frac.T))            # [npw][N]
    psi = np.asarray(psi, dtype=np.complex128)
    rho = np.zeros(n1 * n2 * n3)
    for b in range(psi.shape[0]):
        pr = psi[b] @ phase
        rho += float(w[b]) * (pr.real ** 2 + pr.imag ** 2)
    return (rho / omega).reshape(n3, n2, n1)


def scf_norm2(drho, bvec, omega) -> float:
    """Squared scf norm 4 pi omega sum_{G != 0} |drho(G)|^2 / |G|^2.

    drho(G) = (1/N) sum_j drho(r_j) exp(-i G.r_j) by three explicit DFT
    matrices (no FFT); G = sum_d m_d b_d with b_d = bvec[d] and the grid index
    i_d -> m_d = i_d for i_d <= n_d/2, else i_d - n_d.  The Hartree-energy
    form of the self-consistency error estimate of the self-consistency
    appendix, in Hartree units (e^2 = 1).
    """
    d = np.asarray(drho, dtype=np.float64)
    n3, n2, n1 = d.shape
    f1, f2, f3 = dft_matrix(n1, -1), dft_matrix(n2, -1), dft_matrix(n3, -1)
    t = np.einsum("mj,abj->abm", f1, d.astype(np.complex128))
    t = np.einsum("mj,ajc->amc", f2, t)
    t = np.einsum("mj,jbc->mbc", f3, t)
    c = t / float(n1 * n2 * n3)
    b = np.asarray(bvec, dtype=np.float64).reshape(3, 3)
    total = 0.0
    for i3 in range(n3):
        m3 = i3 if i3 <= n3 // 2 else i3 - n3
        for i2 in range(n2):
            m2 = i2 if i2 <= n2 // 2 else i2 - n2
            for i1 in range(n1):
                m1 = i1 if i1 <= n1 // 2 else i1 - n1
                if m1 == 0 and m2 == 0 and m3 == 0:
                    continue
                g = m1 * b[0] + m2 * b[1] + m3 * b[2]
                total += abs(c[i3, i2, i1]) ** 2 / float(g @ g)
    return 4.0 * math.pi * omega * total


# ----------------------------------------------------------------------------
# spectra
# ----------------------------------------------------------------------------

def eigh_lowest(h: np.ndarray, nb: int):
    """Lowest nb eigenpairs of the dense Hermitian H (ascending)."""
    w, v = scipy.linalg.eigh(h, subset_by_index=[0, nb - 1], driver="evr")
    return w, v.T.copy()          # eigenvectors as [nb][npw]


def davidson(h: np.ndarray, psi0: np.ndarray, nb: int, hdiag: np.ndarray | None = None,
             ndim: int = 2, tol_resid: float = 1e-6, tol_deig: float = 5e-9,
             max_iter: int = 200, precond_floor: float = 0.2):
    """Block Davidson on a dense H, in the order the appendix states it.

    1. orthonormalise the trial orbitals and take eps_i = <psi_i|H|psi_i>;
    2. residuals g_i = (H - eps_i) psi_i;
    3. corrections dpsi_i = g_i / (H_GG - eps_i) for unconverged i (the
       diagonal approximation of (H - eps)^-1, with the denominator replaced
       by its smooth maximum with a floor tau so it stays positive);
    4. reduced problem sum_k (H_jk - eps S_jk) c_k = 0 on the basis phi
       (directions in which the overlap is numerically singular are dropped);
    5. psi_i = sum_j c^(i)_j phi_j; eps_i = <psi_i|H|psi_i>; iterate, growing the
       basis with new corrections until ndim*nb, then restarting from psi
       (with H psi applied afresh).
    Returns (eps, psi [nb][npw], iterations, residual norms).
    """
    psi = np.asarray(psi0, dtype=np.complex128).copy()
    if hdiag is None:
        hdiag = np.real(np.diag(h))
    # step 1: orthonormalise (Cholesky of the overlap) and Rayleigh quotients
    s = np.conj(psi) @ psi.T
    lo = np.linalg.cholesky(s)                # s = L L^H
    psi = np.linalg.solve(np.conj(lo), psi)   # rows: conj(L)^-1 psi -> orthonormal
    hpsi_ = hpsi(h, psi)
    eps = np.real(np.einsum("bg,bg->b", np.conj(psi), hpsi_))
    phi = psi.copy()
    hphi = hpsi_.copy()
    eps_prev = np.full(nb, np.inf)
    it = 0
    rn = None
    while True:
        g = hpsi_ - eps[:, None] * psi                       # step 2
        rn = np.linalg.norm(g, axis=1)
        conv = (rn <= tol_resid) & (np.abs(eps - eps_prev) <= tol_deig)
        if conv.all() or it >= max_iter:
            break
        todo = np.nonzero(~conv)[0]
        x = hdiag[None, :] - eps[todo, None]                 # step 3
        # smooth maximum of x and the floor tau: x far above tau, >= tau/2
        den = 0.5 * (x + precond_floor + np.sqrt((x - precond_floor) ** 2 + precond_floor ** 2))
        dpsi = g[todo] / den
        dpsi /= np.linalg.norm(dpsi, axis=1, keepdims=True)
        if phi.shape[0] + len(todo) > ndim * nb:             # restart from Ritz vectors
            # H psi is recomputed rather than carried over: rotating H phi by the
            # Ritz coefficients multiplies its rounding error by their norm,
            # which compounds over restarts when the basis is ill-conditioned
            phi, hphi = psi.copy(), hpsi(h, psi)
        phi = np.concatenate([phi, dpsi], axis=0)
        hphi = np.concatenate([hphi, hpsi(h, dpsi)], axis=0)
        hred = np.conj(phi) @ hphi.T                         # step 4
        sred = np.conj(phi) @ phi.T
        hred = 0.5 * (hred + np.conj(hred.T))
        sred = 0.5 * (sred + np.conj(sred.T))
        w, c = reduced_eigh(hred, sred, nb)
        eps_prev = eps
        psi = c.T @ phi                                      # step 5
        hpsi_ = c.T @ hphi
        eps = np.real(np.einsum("bg,bg->b", np.conj(psi), hpsi_))
        it += 1
    return eps, psi, it, rn


def pcg(h: np.ndarray, psi0: np.ndarray, nb: int, kin: np.ndarray, tol_resid: float = 1e-6,
        tol_deig: float = 5e-9, max_iter: int = 400, precond_floor: float = 0.2):
    """Band-by-band preconditioned conjugate gradient (the iterative-
    diagonalization appendix, "Conjugate-Gradient"), S = 1, on a dense H.

    Band i minimizes <y|H~|y> - lambda(<y|S~|y> - 1) with H~ = PHP, S~ = PSP,
    y = P^-1 psi, orthogonal to the bands already found; written here in the
    psi variables (P g and P h of the appendix are the vectors kept):
      lambda = <y|S~H~|y> / <y|S~^2|y> = Re <psi|P^2|H psi> / <psi|P^2|psi>,
      P g = P^2 (H - lambda) psi, made orthogonal to psi_j (j < i);
      P h = P g + gamma P h_prev, gamma = Re <g - g_prev|S~|g> / <g_prev|S~|g_prev>
            (Polak-Ribiere; <g|S~|g'> = <P g|P g'>), P h made orthogonal to psi;
      n = P h / ||P h||;  psi <- psi cos(theta) + n sin(theta),
      theta = (1/2) atan(a / (eps - b)), a = 2 Re <psi|H|n>, b = <n|H|n>,
      eps = <psi|H|psi>, taking of the two stationary angles theta and
      theta + pi/2 the one with the lower energy.
    P^2 is kinetic-only: P^2(G) = 1 / smax(T_G, tau), the smooth maximum of
    T_G = |k+G|^2/2 and tau (the appendix's 2m / (hbar^2 |k+G|^2) up to a
    constant factor, which the iteration does not see, kept finite at k+G = 0).
    Band i stops when ||H psi - eps psi|| <= tol_resid and |d eps| <= tol_deig,
    or after max_iter iterations.  Returns (eps, psi [nb][npw], iterations per band).
    """
    x = kin
    p2 = 1.0 / (0.5 * (x + precond_floor + np.sqrt((x - precond_floor) ** 2 + precond_floor ** 2)))
    npw = h.shape[0]
    out = np.zeros((nb, npw), dtype=np.complex128)
    eps_out = np.zeros(nb)
    iters = []
    for i in range(nb):
        psi = np.asarray(psi0[i], dtype=np.complex128).copy()
        for _ in range(2):                                   # orthonormalize to the bands found
            psi -= out[:i].T @ (np.conj(out[:i]) @ psi)
        psi /= np.linalg.norm(psi)
        hpsi_ = h @ psi
        eps = float(np.real(np.vdot(psi, hpsi_)))
        g_prev = d_prev = None
        gg_prev = 0.0
        it = 0
        while True:
            lam = float(np.real(np.vdot(psi, p2 * hpsi_)) / np.real(np.vdot(psi, p2 * psi)))
            g = p2 * (hpsi_ - lam * psi)
            g -= out[:i].T @ (np.conj(out[:i]) @ g)
            gg = float(np.real(np.vdot(g, g)))
            if g_prev is None:
                d = g.copy()
            else:
                gamma = float(np.real(np.vdot(g - g_prev, g))) / gg_prev
                d = g + gamma * d_prev
            d -= psi * np.vdot(psi, d)
            n = d / np.linalg.norm(d)
            hn = h @ n
            a = 2.0 * float(np.real(np.vdot(psi, hn)))
            b = float(np.real(np.vdot(n, hn)))
            theta = 0.5 * math.atan(a / (eps - b)) if eps != b else math.pi / 4
            def energy(t):
                return eps * math.cos(t) ** 2 + b * math.sin(t) ** 2 + a * math.sin(t) * math.cos(t)
            if energy(theta + 0.5 * math.pi) < energy(theta):
                theta += 0.5 * math.pi
            psi = psi * math.cos(theta) + n * math.sin(theta)
            hpsi_ = hpsi_ * math.cos(theta) + hn * math.sin(theta)
            eps_new = float(np.real(np.vdot(psi, hpsi_)))
            it += 1
            r = float(np.linalg.norm(hpsi_ - eps_new * psi))
            done = r <= tol_resid and abs(eps_new - eps) <= tol_deig
            eps = eps_new
            g_prev, d_prev, gg_prev = g, d, gg
            if done or it >= max_iter:
                break
        out[i] = psi
        eps_out[i] = eps
        iters.append(it)
    return eps_out, out, iters


def reduced_eigh(hred: np.ndarray, sred: np.ndarray, nev: int, drop: float = 1e-10):
    """Lowest nev solutions of hred c = w sred c on the numerically independent
    part of the basis.

    The overlap is diagonalized, directions with eigenvalue below
    ``drop * max eigenvalue`` are discarded (corrections that fell inside the
    span of the basis), and the standard problem is solved on the rest.
    Returns (w, c) with c sred-orthonormal, shape [n][nev].
    """
    sig, u = np.linalg.eigh(sred)
    keep = sig > drop * sig.max()
    if keep.sum() < nev:
        raise np.linalg.LinAlgError("reduced basis has rank < nev")
    q = u[:, keep] / np.sqrt(sig[keep])[None, :]
    a = np.conj(q.T) @ hred @ q
    a = 0.5 * (a + np.conj(a.T))
    w, y = np.linalg.eigh(a)
    return w[:nev], q @ y[:, :nev]


def secular_roots(t: np.ndarray, beta: np.ndarray, d: float, count: int, tol: float = 1e-15):
    """Lowest ``count`` eigenvalues of diag(t) + d |beta><beta| (d > 0).

    Textbook rank-one update: each distinct pole p with multiplicity k keeps
    k - 1 eigenvalues equal to p; the others are the roots of
    f(lam) = 1 - d sum_p W_p / (lam - p), one in each interval between
    consecutive poles and one above the last (W_p = sum over the pole of
    |beta_G|^2).  Roots are found by plain bisection in float64.
    """
    assert d > 0
    t = np.asarray(t, dtype=np.float64)
    w = np.abs(np.asarray(beta)) ** 2
    order = np.argsort(t, kind="stable")
    t, w = t[order], w[order]
    poles, weights, mult = [], [], []
    i = 0
    while i < len(t):
        j = i
        while j + 1 < len(t) and abs(t[j + 1] - t[i]) <= 1e-12 * max(1.0, abs(t[i])):
            j += 1
        poles.append(t[i])
        weights.append(w[i:j + 1].sum())
        mult.append(j - i + 1)
        i = j + 1
    poles = np.array(poles)
    weights = np.array(weights)
    vals = []
    for p, k in zip(poles, mult):
        vals.extend([p] * (k - 1))

    def f(lam):
        return 1.0 - d * np.sum(weights / (lam - poles))

    upper = poles[-1] + d * weights.sum() + 1.0
    for idx in range(len(poles)):
        lo_ = poles[idx]
        hi_ = poles[idx + 1] if idx + 1 < len(poles) else upper
        a_, b_ = lo_, hi_
        for _ in range(200):
            mid = 0.5 * (a_ + b_)
            if mid <= a_ or mid >= b_:
                break
            if f(mid) < 0:
                a_ = mid
            else:
                b_ = mid
            if b_ - a_ <= tol * max(1.0, abs(mid)):
                break
        vals.append(0.5 * (a_ + b_))
        if len(vals) >= count + len(t):
            break
    vals = np.sort(np.array(vals))
    return vals[:count]


def kato_temple(theta: np.ndarray, resid: np.ndarray):
    """A-posteriori bounds for Ritz pairs (theta_i, residual norm r_i).

    Returns (bauer_fike, kato_temple): an exact eigenvalue lies within r_i of
    theta_i, and for an isolated Ritz value |theta_i - lambda_i| <=
    r_i^2 / delta_i with delta_i the distance from theta_i to the nearest
    other spectral interval [theta_j - r_j, theta_j + r_j].  Where the
    intervals overlap, the Kato-Temple value is +inf.
    """
    theta = np.asarray(theta, dtype=np.float64)
    r = np.asarray(resid, dtype=np.float64)
    kt = np.full_like(theta, np.inf)
    for i in range(len(theta)):
        others = [abs(theta[j] - theta[i]) - r[j] for j in range(len(theta)) if j != i]
        if not others:
            continue
        delta = min(others)
        if delta > r[i]:
            kt[i] = r[i] ** 2 / delta
    return r.copy(), kt
