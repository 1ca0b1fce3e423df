"""Pins of the CPU oracle against what the mathematics fixes (no GPU).

Each test pins part of the oracle to something other than itself: a closed
form, a textbook reduction, an independent route (explicit real-space sums,
the generator's own V(G) coefficients) or an invariant of the Hamiltonian.
"""
import math

import numpy as np
import pytest

import oracle
from paper_0906_2569_amd import pwgen


def _free(a=10.0, ecut=15.0, nr=(30, 30, 30), natoms=8, nb=16, seed=1, **kw):
    return pwgen.make_cell(a, ecut, natoms, nb, seed, nr=nr, with_vloc=False, with_beta=False, **kw)


def test_sphere_sizes():
    # counts of {m : |G_m|^2 <= ecut} for the workloads' cells
    assert pwgen.sphere(10.0, 15.0)[0].shape[0] == 949
    assert pwgen.sphere(20.5, 25.0)[0].shape[0] == 18277
    m, _, _ = pwgen.sphere(41.0, 30.0)
    assert m.shape[0] == 191471
    assert pwgen.min_grid(m) == (144, 144, 144)


def test_free_electron_closed_form():
    # V = 0, beta = 0: eigenvalues are |G|^2/2 = (2 pi/a)^2 |m|^2 / 2 exactly.
    p = _free()
    h = oracle.dense_h_of(p)
    w, _ = oracle.eigh_lowest(h, 16)
    unit = 2.0 * math.pi ** 2 / 100.0          # (2 pi / 10)^2 / 2 = 0.19739208802...
    expect = np.array([0.0] + [unit] * 6 + [2 * unit] * 9)
    assert abs(unit - 0.19739208802178717) < 1e-15
    np.testing.assert_allclose(w, expect, atol=1e-13)
    # the 12-fold |m|^2 = 2 shell is complete in the sphere
    w2, _ = oracle.eigh_lowest(h, 19)
    np.testing.assert_allclose(w2[7:19], 2 * unit, atol=1e-13)


def test_free_electron_shifted_k():
    # k = (1/4, 1/4, 0) b: eigenvalues are |k+G|^2/2 for the sorted sphere
    a = 10.0
    p = pwgen.make_cell(a, 10.0, 0, 8, 3, kfrac=(0.25, 0.25, 0.0), with_vloc=False, with_beta=False)
    h = oracle.dense_h_of(p)
    w, _ = oracle.eigh_lowest(h, 8)
    b = 2 * math.pi / a
    # hand-enumerated lowest |k+G|^2 (units b^2): (1/4,1/4,0)->1/8 (x1: m=0),
    # m=(-1,0,0),(0,-1,0) -> 9/16+1/16=5/8 (x2), m=(-1,-1,0) -> 9/8 (x1),
    # m=(0,0,+-1) -> 1/8+1 = 9/8 (x2)
    expect = 0.5 * b * b * np.array([1 / 8, 5 / 8, 5 / 8, 9 / 8, 9 / 8, 9 / 8])
    np.testing.assert_allclose(w[:6], expect, atol=1e-13)


def test_vtilde_equals_generator_coefficients():
    # The generator defines V(G) and builds V(r) by its own inverse transform;
    # the oracle's direct DFT of V(r) must give those coefficients back, and
    # zero outside their support.  A flipped sign gives conj(V(G)) != V(G).
    p = pwgen.config1()
    vt = oracle.vtilde_table(p.vloc_r)
    got = oracle.vtilde_lookup(vt, p.vg_miller.astype(np.int64))
    np.testing.assert_allclose(got, p.vg_coef, atol=1e-15, rtol=0)
    assert np.abs(p.vg_coef.imag).max() > 1e-3          # really complex
    mask = np.ones(vt.shape, dtype=bool)
    n3, n2, n1 = vt.shape
    vm = p.vg_miller
    mask[vm[:, 2] % n3, vm[:, 1] % n2, vm[:, 0] % n1] = False
    assert np.abs(vt[mask]).max() < 1e-15


def test_single_plane_wave_gives_v_of_g_difference():
    # psi = e_{G0}: (H psi)_G = T_G0 delta + V(G - G0), with V from the generator.
    p = pwgen.config1(with_beta=False)
    h = oracle.dense_h_of(p)
    vdict = {tuple(m): c for m, c in zip(p.vg_miller.tolist(), p.vg_coef)}
    t = oracle.kinetic(p.kpg)
    rng = np.random.default_rng(0)
    for g0 in rng.choice(p.npw, 5, replace=False):
        e = np.zeros((1, p.npw), dtype=np.complex128)
        e[0, g0] = 1.0
        out = oracle.hpsi(h, e)[0]
        expect = np.array([vdict.get(tuple(m), 0.0) for m in (p.miller - p.miller[g0]).tolist()])
        expect[g0] += t[g0]
        np.testing.assert_allclose(out, expect, atol=1e-14, rtol=0)


@pytest.mark.parametrize("seed,a,ecut,kfrac,nr", [
    (11, 5.0, 6.0, (0, 0, 0), None),
    (12, 4.0, 8.0, (0.25, 0.25, 0.0), None),
    (13, 6.0, 4.0, (0.1, -0.3, 0.2), (15, 16, 18)),
    (14, 5.5, 5.0, (0, 0, 0), (12, 10, 9)),   # grid below the no-alias bound: still exact mod n
])
def test_dense_equals_real_space_brute_force(seed, a, ecut, kfrac, nr):
    p = pwgen.tiny_cell(seed, a=a, ecut_ry=ecut, natoms=2, nb=3, kfrac=kfrac, nr=nr)
    h = oracle.dense_h_of(p)
    ref = oracle.hpsi_brute(p.miller, p.kpg, p.vloc_r, p.beta, p.blk_off, p.dmat, p.psi0)
    got = oracle.hpsi(h, p.psi0)
    np.testing.assert_allclose(got, ref, atol=1e-12, rtol=0)


def test_hermitian():
    p = pwgen.config1()
    h = oracle.dense_h_of(p)
    assert np.abs(h - h.conj().T).max() <= 1e-15 * np.abs(h).max() * 10
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, p.npw)) + 1j * rng.standard_normal((2, p.npw))
    hx = oracle.hpsi(h, x)
    lhs = np.vdot(x[0], hx[1])
    rhs = np.conj(np.vdot(x[1], hx[0]))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_constant_potential_shifts_spectrum():
    p = pwgen.config1()
    c = 0.37
    h0 = oracle.dense_h(p.miller, p.kpg, np.zeros_like(p.vloc_r), p.beta, p.blk_off, p.dmat)
    h1 = oracle.dense_h(p.miller, p.kpg, np.full_like(p.vloc_r, c), p.beta, p.blk_off, p.dmat)
    w0, _ = oracle.eigh_lowest(h0, 16)
    w1, _ = oracle.eigh_lowest(h1, 16)
    np.testing.assert_allclose(w1, w0 + c, atol=1e-13)


def test_rank_one_secular_equation():
    # V = 0, a single projector with D = d: textbook secular equation.
    p = pwgen.config1(with_vloc=False)
    beta = p.beta[:1]
    for d in (0.25, 1.0):
        h = oracle.dense_h(p.miller, p.kpg, np.zeros_like(p.vloc_r), beta,
                           np.array([0, 1], dtype=np.int32), np.array([d], dtype=np.complex128))
        w, _ = oracle.eigh_lowest(h, 20)
        ref = oracle.secular_roots(oracle.kinetic(p.kpg), beta[0], d, 20)
        np.testing.assert_allclose(w, ref, atol=1e-12)
        assert abs(w[0]) > 1e-4                       # the projector really moved the bottom


def test_nonlocal_acting_on_its_projector():
    # V = 0, one normalised projector beta with D = d:  H beta = T beta + d beta.
    p = pwgen.config1(with_vloc=False)
    beta = p.beta[1:2]                                 # a p-projector (complex, odd)
    d = 0.8
    h = oracle.dense_h(p.miller, p.kpg, np.zeros_like(p.vloc_r), beta,
                       np.array([0, 1], dtype=np.int32), np.array([d], dtype=np.complex128))
    out = oracle.hpsi(h, beta)[0]
    np.testing.assert_allclose(out, oracle.kinetic(p.kpg) * beta[0] + d * beta[0], atol=1e-14)


def test_time_reversal_pair():
    # real V(r) and real diagonal D: eps_n(k) = eps_n(-k)
    streams = np.random.SeedSequence(77).spawn(4)
    pa = pwgen.make_cell(7.0, 8.0, 3, 8, None, kfrac=(0.25, 0.25, 0.0), streams=streams)
    pb = pwgen.make_cell(7.0, 8.0, 3, 8, None, kfrac=(-0.25, -0.25, 0.0), streams=streams)
    wa, _ = oracle.eigh_lowest(oracle.dense_h_of(pa), 8)
    wb, _ = oracle.eigh_lowest(oracle.dense_h_of(pb), 8)
    np.testing.assert_allclose(wa, wb, atol=1e-12)


def test_grid_translation_invariance():
    # translating V(r) by a grid vector and every atom by the same vector is a
    # unitary (diagonal phase) change of basis: the spectrum is unchanged.
    streams = np.random.SeedSequence(78).spawn(4)
    p = pwgen.make_cell(6.0, 8.0, 3, 8, None, kfrac=(0.1, 0.2, 0.3), streams=streams)
    n1, n2, n3 = p.nr
    shift = np.array([3, 1, 2])                     # grid steps along x, y, z
    v2 = np.roll(p.vloc_r, shift=(shift[2], shift[1], shift[0]), axis=(0, 1, 2))
    tvec = p.a * shift / np.array([n1, n2, n3])
    beta2 = p.beta * np.exp(-1j * (p.kpg @ tvec))[None, :]
    h1 = oracle.dense_h_of(p)
    h2 = oracle.dense_h(p.miller, p.kpg, v2, beta2, p.blk_off, p.dmat)
    w1, _ = oracle.eigh_lowest(h1, 8)
    w2, _ = oracle.eigh_lowest(h2, 8)
    np.testing.assert_allclose(w1, w2, atol=1e-12)
    assert np.abs(h1 - h2).max() > 1e-3               # the matrices themselves differ


def test_h_diag_matches_dense_diagonal():
    p = pwgen.config1()
    h = oracle.dense_h_of(p)
    hd = oracle.h_diag(p.miller, p.kpg, p.vloc_r, p.beta, p.blk_off, p.dmat)
    np.testing.assert_allclose(hd, np.real(np.diag(h)), atol=1e-14)


@pytest.mark.parametrize("ndim", [2, 3, 4])
def test_davidson_converges_to_dense_spectrum(ndim):
    p = pwgen.config1()
    h = oracle.dense_h_of(p)
    w, _ = oracle.eigh_lowest(h, p.nb)
    # the 2N form (restart every iteration) converges slowly for the top band,
    # whose gap to band nb+1 is small: there only the eigenvalues are checked
    eps, psi, it, rn = oracle.davidson(h, p.psi0, p.nb, ndim=ndim, max_iter=400)
    if ndim > 2:
        assert rn.max() <= 1e-6
        assert 3 < it < 400
    np.testing.assert_allclose(eps, w, atol=5e-9)
    # Ritz values bound the exact ones from above (Courant-Fischer)
    assert np.all(eps >= w - 1e-12)
    # orthonormal output
    np.testing.assert_allclose(np.conj(psi) @ psi.T, np.eye(p.nb), atol=1e-12)


def test_a_posteriori_bounds_hold():
    p = pwgen.config1()
    h = oracle.dense_h_of(p)
    w, v = oracle.eigh_lowest(h, 20)
    rng = np.random.default_rng(5)
    x = v[:8] + 1e-4 * (rng.standard_normal(v[:8].shape) + 1j * rng.standard_normal(v[:8].shape))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    hx = oracle.hpsi(h, x)
    theta = np.real(np.einsum("bg,bg->b", np.conj(x), hx))
    r = np.linalg.norm(hx - theta[:, None] * x, axis=1)
    bf, kt = oracle.kato_temple(theta, r)
    assert np.all(np.abs(theta - w[:8]) <= bf + 1e-14)
    finite = np.isfinite(kt)
    assert finite.any()
    assert np.all(np.abs(theta - w[:8])[finite] <= kt[finite] * (1 + 1e-6) + 1e-15)


def test_davidson_projectors_only():
    # V = 0: near-dependent corrections; the reduced problem drops them and
    # H psi is re-applied at restarts, so the iteration still converges
    p = pwgen.config1(with_vloc=False)
    h = oracle.dense_h_of(p)
    w, _ = oracle.eigh_lowest(h, p.nb)
    eps, psi, it, rn = oracle.davidson(h, p.psi0, p.nb, ndim=4, max_iter=400)
    assert rn.max() <= 1e-6
    np.testing.assert_allclose(eps, w, atol=5e-9)


def test_reduced_eigh_drops_dependent_directions():
    rng = np.random.default_rng(4)
    n = 12
    x = rng.standard_normal((n, 30)) + 1j * rng.standard_normal((n, 30))
    x[7] = x[2] + 1e-14 * x[5]              # dependent basis vector
    a = rng.standard_normal((30, 30)) + 1j * rng.standard_normal((30, 30))
    a = a + a.conj().T
    hred = np.conj(x) @ a @ x.T
    sred = np.conj(x) @ x.T
    w, c = oracle.reduced_eigh(hred, sred, 5)
    # same Ritz values as the basis without the duplicate
    keep = [i for i in range(n) if i != 7]
    w2 = scipy_eigh(hred[np.ix_(keep, keep)], sred[np.ix_(keep, keep)])[:5]
    np.testing.assert_allclose(w, w2, atol=1e-9)


def scipy_eigh(h, s):
    import scipy.linalg
    return scipy.linalg.eigh(h, s, eigvals_only=True)


def _random_unitary(rng, n):
    z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))[None, :]


def test_projector_rotation_invariance_pins_d_layout():
    # Rotating one atom's projectors, beta' = beta U (beta' as npw x nh columns),
    # with D' = U^H D U leaves sum_ij beta_i D_ij beta_j^H, hence H, unchanged.
    # D' is complex and not diagonal; reading its column-major block transposed
    # gives conj(D') and breaks the identity.  Both routes to H.psi are pinned:
    # the dense matrix and the real-space brute force.
    p = pwgen.tiny_cell(91, a=6.0, ecut_ry=8.0, natoms=3, nb=4, kfrac=(0.1, 0.2, -0.3))
    rng = np.random.default_rng(91)
    p.dmat = pwgen.hermitian_blocks(rng, p.blk_off)
    h0 = oracle.dense_h_of(p)
    atom = 1
    o0, o1 = int(p.blk_off[atom]), int(p.blk_off[atom + 1])
    nh = o1 - o0
    u = _random_unitary(rng, nh)
    beta2 = p.beta.copy()
    beta2[o0:o1] = (p.beta[o0:o1].T @ u).T
    d_blk = p.dmat[o0 * nh:(o0 + nh) * nh].reshape(nh, nh).T     # col-major block (nh = 4 for all atoms)
    assert np.abs(d_blk - np.conj(d_blk.T)).max() < 1e-15
    assert np.abs(d_blk - d_blk.T).max() > 1e-2                    # really complex off-diagonal
    d2 = np.conj(u.T) @ d_blk @ u
    dmat2 = p.dmat.copy()
    dmat2[o0 * nh:(o0 + nh) * nh] = d2.T.ravel()                   # write back column-major
    h1 = oracle.dense_h(p.miller, p.kpg, p.vloc_r, beta2, p.blk_off, dmat2)
    np.testing.assert_allclose(h1, h0, atol=1e-13, rtol=0)
    # the transposed reading is not invariant (the test can fail)
    dmat_t = p.dmat.copy()
    dmat_t[o0 * nh:(o0 + nh) * nh] = d2.ravel()
    h_bad = oracle.dense_h(p.miller, p.kpg, p.vloc_r, beta2, p.blk_off, dmat_t)
    assert np.abs(h_bad - h0).max() > 1e-3
    # brute-force route reads the flat blocks itself
    ref = oracle.hpsi(h0, p.psi0)
    got = oracle.hpsi_brute(p.miller, p.kpg, p.vloc_r, beta2, p.blk_off, dmat2, p.psi0)
    np.testing.assert_allclose(got, ref, atol=1e-12, rtol=0)


def test_general_d_on_orthonormal_projectors():
    # V = 0, one atom at Gamma: its s, px, py, pz projectors are orthonormal on
    # the inversion-symmetric sphere, so H beta_k = T beta_k + sum_i beta_i D_ik
    # for a general Hermitian D (column k of D, not row k).
    p = pwgen.make_cell(10.0, 15.0, 1, 4, 5, nr=(30, 30, 30), with_vloc=False)
    gram = np.conj(p.beta) @ p.beta.T
    np.testing.assert_allclose(gram, np.eye(4), atol=1e-14)
    rng = np.random.default_rng(5)
    dmat = pwgen.hermitian_blocks(rng, p.blk_off)
    d = dmat.reshape(4, 4).T                                        # d[i, k] = D_ik
    h = oracle.dense_h(p.miller, p.kpg, p.vloc_r, p.beta, p.blk_off, dmat)
    out = oracle.hpsi(h, p.beta)
    t = oracle.kinetic(p.kpg)
    expect = t[None, :] * p.beta + d.T @ p.beta                     # row k: sum_i D_ik beta_i
    np.testing.assert_allclose(out, expect, atol=1e-14)
    out_b = oracle.hpsi_brute(p.miller, p.kpg, p.vloc_r, p.beta, p.blk_off, dmat, p.beta)
    np.testing.assert_allclose(out_b, expect, atol=1e-13)


def test_cpu_fft_method_baseline_matches_dense():
    # the timed CPU FFT-method baseline computes the oracle's product
    from oracle import fft_method
    p = pwgen.tiny_cell(95, a=7.0, ecut_ry=9.0, natoms=3, nb=5, kfrac=(0.25, -0.25, 0.0), nr=(36, 30, 40))
    p.dmat = pwgen.hermitian_blocks(np.random.default_rng(95), p.blk_off)
    ref = oracle.hpsi(oracle.dense_h_of(p), p.psi0)
    got = fft_method.hpsi(p.miller, p.kpg, p.vloc_r, p.beta, p.blk_off, p.dmat, p.psi0)
    np.testing.assert_allclose(got, ref, atol=1e-12, rtol=0)


def test_density_charge_equals_weighted_norms():
    # (omega/N) sum_j rho(r_j) = sum_b w_b ||psi_b||^2 (Parseval on a grid that
    # holds the sphere without aliasing)
    p = pwgen.tiny_cell(96, a=6.0, ecut_ry=8.0, natoms=2, nb=4, kfrac=(0.25, 0.0, -0.25), nr=(20, 18, 24))
    w = np.array([2.0, 1.5, 0.5, 0.25])
    omega = p.a ** 3
    rho = oracle.density(p.miller, p.nr, p.psi0 * np.array([1, 2, 3, 4])[:, None], w, omega)
    n = np.prod(p.nr)
    assert abs(rho.sum() * omega / n - float(np.sum(w * np.array([1, 4, 9, 16])))) <= 1e-12
    assert rho.min() >= 0.0


def test_density_of_plane_waves_closed_form():
    # one plane wave: uniform w/omega; two plane waves a e^{iG1 r} + b e^{iG2 r}:
    # (|a|^2 + |b|^2 + 2 Re(a conj(b) e^{i(G1-G2).r})) / omega
    p = pwgen.tiny_cell(97, a=5.0, ecut_ry=6.0, natoms=1, nb=1, nr=(12, 10, 15))
    omega = p.a ** 3
    g1, g2 = 3, 7
    psi = np.zeros((2, p.npw), dtype=np.complex128)
    psi[0, g1] = 0.8 - 0.6j
    a, b = 0.3 + 0.4j, -0.5 + 0.2j
    psi[1, g1], psi[1, g2] = a, b
    rho1 = oracle.density(p.miller, p.nr, psi[:1], [1.7], omega)
    np.testing.assert_allclose(rho1, 1.7 / omega, rtol=1e-13)
    rho2 = oracle.density(p.miller, p.nr, psi[1:], [1.0], omega)
    n1, n2, n3 = p.nr
    j3, j2, j1 = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    dm = p.miller[g1] - p.miller[g2]
    ph = np.exp(2j * math.pi * (dm[0] * j1 / n1 + dm[1] * j2 / n2 + dm[2] * j3 / n3))
    expect = (abs(a) ** 2 + abs(b) ** 2 + 2 * np.real(a * np.conj(b) * ph)) / omega
    np.testing.assert_allclose(rho2, expect, atol=1e-15)


@pytest.mark.parametrize("m0", [(1, 0, 0), (0, 2, 1), (-2, 1, 3)])
def test_scf_norm_of_a_cosine(m0):
    # drho(r) = c cos(G0.r) has coefficients c/2 at +-G0:
    # ||drho||^2 = 4 pi omega 2 (c/2)^2 / |G0|^2 = 2 pi omega c^2 / |G0|^2
    nr = (12, 10, 15)
    bvec = np.array([[0.7, 0.1, 0.0], [0.0, 0.9, 0.2], [0.1, 0.0, 0.8]])
    omega = (2 * math.pi) ** 3 / abs(np.linalg.det(bvec))
    n1, n2, n3 = nr
    j3, j2, j1 = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    c = 0.37
    d = c * np.cos(2 * math.pi * (m0[0] * j1 / n1 + m0[1] * j2 / n2 + m0[2] * j3 / n3))
    g0 = m0[0] * bvec[0] + m0[1] * bvec[1] + m0[2] * bvec[2]
    got = oracle.scf_norm2(d, bvec, omega)
    assert abs(got - 2 * math.pi * omega * c * c / float(g0 @ g0)) <= 1e-12 * got
    # a constant has no G != 0 component; the norm is quadratic
    assert abs(oracle.scf_norm2(d + 5.0, bvec, omega) - got) <= 1e-12 * got
    assert abs(oracle.scf_norm2(3.0 * d, bvec, omega) - 9.0 * got) <= 1e-12 * got


def test_pcg_converges_to_dense_spectrum():
    # band-by-band preconditioned CG: the lowest nb eigenvalues of the dense H
    p = pwgen.config1()
    h = oracle.dense_h_of(p)
    w, _ = oracle.eigh_lowest(h, 8)
    eps, psi, iters = oracle.pcg(h, p.psi0[:8], 8, oracle.kinetic(p.kpg), max_iter=600)
    print("pcg iterations per band", iters)
    np.testing.assert_allclose(eps, w, atol=5e-9)
    np.testing.assert_allclose(np.conj(psi) @ psi.T, np.eye(8), atol=1e-10)
    assert max(iters) < 600
    # the returned vectors are eigenvectors: residuals at the tolerance
    r = np.linalg.norm(psi @ h.T - eps[:, None] * psi, axis=1)
    assert r.max() <= 1e-6


def test_ultrasoft_single_plane_wave_projector_closed_form():
    # V = 0 and one projector that is a single plane wave e_G0, with D = d and
    # q: H and S are diagonal; the generalized eigenvalues are T_G for G != G0
    # and (T_G0 + d) / (1 + q) at G0
    p = pwgen.make_cell(10.0, 15.0, 0, 8, 7, nr=(30, 30, 30), with_vloc=False, with_beta=False)
    g0 = 40
    beta = np.zeros((1, p.npw), dtype=np.complex128)
    beta[0, g0] = np.exp(0.7j)
    d, q = 0.9, 0.6
    blk = np.array([0, 1], dtype=np.int32)
    h = oracle.dense_h(p.miller, p.kpg, p.vloc_r, beta, blk, np.array([d], dtype=np.complex128))
    s = oracle.dense_s(p.npw, beta, blk, np.array([q], dtype=np.complex128))
    t = oracle.kinetic(p.kpg)
    expect = np.sort(np.concatenate([np.delete(t, g0), [(t[g0] + d) / (1 + q)]]))[:30]
    w, v = oracle.eigh_lowest_gen(h, s, 30)
    np.testing.assert_allclose(w, expect, atol=1e-12)
    np.testing.assert_allclose(np.conj(v) @ s @ v.T, np.eye(30), atol=1e-12)


def test_ultrasoft_rotation_invariance_and_q_zero():
    # beta' = beta U, q' = U^H q U leaves S unchanged (a transposed reading of the
    # q blocks fails); q = 0 gives S = 1
    p = pwgen.tiny_cell(98, a=6.0, ecut_ry=8.0, natoms=2, nb=4)
    rng = np.random.default_rng(98)
    qmat = pwgen.hermitian_blocks(rng, p.blk_off, scale=0.2)
    s0 = oracle.dense_s(p.npw, p.beta, p.blk_off, qmat)
    u = _random_unitary(rng, 4)
    beta2 = p.beta.copy()
    beta2[4:8] = (p.beta[4:8].T @ u).T
    qb = qmat[16:32].reshape(4, 4).T
    q2 = qmat.copy()
    q2[16:32] = (np.conj(u.T) @ qb @ u).T.ravel()
    np.testing.assert_allclose(oracle.dense_s(p.npw, beta2, p.blk_off, q2), s0, atol=1e-14)
    assert np.abs(s0 - np.eye(p.npw)).max() > 1e-3
    np.testing.assert_allclose(oracle.dense_s(p.npw, p.beta, p.blk_off, np.zeros_like(qmat)), np.eye(p.npw))


def test_gamma_cell_is_real_in_real_space():
    # with the -i of the p projectors, beta(-G) = conj(beta(G)) and
    # H(-G, -G') = conj(H(G, G')): H maps real functions to real functions, so
    # the half sphere carries them; diagonal D leaves H unchanged by the phase
    g = pwgen.gamma_cell(10.0, 15.0, 8, 4, 31, nr=(30, 30, 30))
    mir = pwgen.mirror_index(g.full.miller)
    np.testing.assert_allclose(g.full.beta[:, mir], np.conj(g.full.beta), atol=1e-15)
    h = oracle.dense_h_of(g.full)
    np.testing.assert_allclose(h[np.ix_(mir, mir)], np.conj(h), atol=1e-14)
    ref = pwgen.make_cell(10.0, 15.0, 8, 4, 31, nr=(30, 30, 30))
    np.testing.assert_allclose(h, oracle.dense_h_of(ref), atol=1e-14)
    hp = oracle.hpsi(h, g.full.psi0)
    np.testing.assert_allclose(hp[:, mir], np.conj(hp), atol=1e-14)
    assert len(g.half) == (g.full.npw + 1) // 2 and g.half[0] == np.nonzero((g.full.miller == 0).all(1))[0][0]


def test_gamma_ultrasoft_overlap_needs_real_q():
    # at Gamma S = 1 + beta q beta^H maps real-space-real functions to real
    # ones, S(-G, -G') = conj(S(G, G')), exactly when the q blocks are real:
    # the half sphere then carries S psi too.  A q block with an imaginary
    # part breaks the symmetry (the Gamma plan refuses such blocks).
    g = pwgen.gamma_cell(10.0, 15.0, 8, 4, 32, nr=(30, 30, 30))
    mir = pwgen.mirror_index(g.full.miller)
    q = pwgen.hermitian_blocks(np.random.default_rng(32), g.full.blk_off, scale=0.1)
    assert np.abs(q.imag).max() > 1e-3
    s_real = oracle.dense_s(g.full.npw, g.full.beta, g.full.blk_off, np.ascontiguousarray(q.real + 0j))
    np.testing.assert_allclose(s_real[np.ix_(mir, mir)], np.conj(s_real), atol=1e-14)
    sp = g.full.psi0 @ s_real.T
    np.testing.assert_allclose(sp[:, mir], np.conj(sp), atol=1e-14)
    s_cplx = oracle.dense_s(g.full.npw, g.full.beta, g.full.blk_off, q)
    assert np.abs(s_cplx[np.ix_(mir, mir)] - np.conj(s_cplx)).max() > 1e-4
