"""Gamma-point real-wavefunction path (half sphere, two bands per transform, real
products) on the GPU, against the dense oracle on the whole sphere."""
import numpy as np
import pytest

import oracle
from paper_0906_2569_amd import pwgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL_EIG = 5e-9


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0906_2569_amd import pwdft
    return pwdft.Context(0)


def _rel(got, ref):
    return (np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)).max()


def _gdot(a, b):
    """full-sphere inner products <a_i|b_j> of half-sphere real functions"""
    return 2 * np.real(np.conj(a) @ b.T) - np.outer(a[:, 0].real, b[:, 0].real)


def _hpsi(ctx, g, psi, prec=0, ld=None, **kw):
    from paper_0906_2569_amd import pwdft
    plan = pwdft.Plan(ctx, g, precision=max(prec, 0), nb_max=psi.shape[0], ndim_max=0, gamma=1, **kw)
    try:
        ld = ld or g.npw
        x = torch.zeros((psi.shape[0], ld), dtype=torch.complex128, device="cuda")
        x[:, :g.npw] = torch.from_numpy(psi).cuda()
        y = plan.hpsi(x, prec=prec)
        torch.cuda.synchronize()
        return y[:, :g.npw].cpu().numpy(), plan.info()
    finally:
        plan.close()


@pytest.mark.parametrize("nb,ld", [(16, None), (15, None), (1, 480), (7, 481)])
def test_gamma_hpsi_against_dense(ctx, nb, ld):
    g = pwgen.gamma_cell(10.0, 15.0, 8, 16, 21, nr=(30, 30, 30))
    h = oracle.dense_h_of(g.full)
    psi = g.psi0[:nb]
    got, info = _hpsi(ctx, g, psi, ld=ld)
    ref = oracle.hpsi(h, g.expand(psi))[:, g.half]
    assert _rel(got, ref) <= 1e-11
    assert np.abs(got[:, 0].imag).max() == 0.0            # H psi(0) is real


def test_gamma_hpsi_mixed(ctx):
    g = pwgen.gamma_cell(10.0, 15.0, 8, 16, 22, nr=(30, 30, 30))
    h = oracle.dense_h_of(g.full)
    got, _ = _hpsi(ctx, g, g.psi0, prec=1)
    ref = oracle.hpsi(h, g.expand(g.psi0))[:, g.half]
    err = _rel(got, ref)
    assert 1e-9 < err <= 2e-6


@pytest.mark.parametrize("plane_mode,chunked", [(1, False), (0, True), (1, True)])
def test_gamma_plane_forms_and_chunks(ctx, plane_mode, chunked):
    g = pwgen.gamma_cell(7.0, 9.0, 3, 11, 23, nr=(36, 30, 40))
    h = oracle.dense_h_of(g.full)
    kw = {"plane_mode": plane_mode}
    if chunked:
        _, i0 = _hpsi(ctx, g, g.psi0[:1], plane_mode=plane_mode)
        n1, n2, n3 = g.nr
        per = 16 * n3 * ((i0["nsticks"] + 3) // 4 * 4) + (16 * n3 * n2 * i0["ncols"] if plane_mode == 1 else 0)
        kw["fft_ws_bytes"] = 2 * per + 100
    got, info = _hpsi(ctx, g, g.psi0, **kw)
    if chunked:
        assert info["band_chunk"] == 2     # pairs per chunk: 11 bands = 6 pairs in 3 chunks, the last band alone
    ref = oracle.hpsi(h, g.expand(g.psi0))[:, g.half]
    assert _rel(got, ref) <= 1e-11


def test_gamma_half_sphere_checks(ctx):
    from paper_0906_2569_amd import pwdft
    g = pwgen.gamma_cell(10.0, 15.0, 8, 4, 24, nr=(30, 30, 30))
    bad = pwgen.GammaProblem(full=g.full, half=g.half, miller=g.full.miller, kpg=g.full.kpg, beta=g.full.beta,
                             psi0=g.full.psi0)
    with pytest.raises(pwdft.PwError) as ei:          # the whole sphere: G and -G both listed
        pwdft.Plan(ctx, bad, precision=0, nb_max=4, ndim_max=0, gamma=1)
    assert ei.value.status == pwdft.PW_EINVAL


def _solve(ctx, g, precision=0, ndim=4, **kw):
    from paper_0906_2569_amd import pwdft
    plan = pwdft.Plan(ctx, g, precision=precision, nb_max=g.nb, ndim_max=ndim, gamma=1)
    try:
        x = torch.from_numpy(g.psi0).cuda()
        st, eig, resid, stats = plan.davidson(x, opts=pwdft.default_opts(ndim=ndim, max_iter=400, **kw))
        torch.cuda.synchronize()
        return st, eig.cpu().numpy(), resid.cpu().numpy(), x.cpu().numpy(), stats.asdict()
    finally:
        plan.close()


@pytest.mark.parametrize("precision,ndim,lock,sub32", [(0, 4, 1, 1), (0, 2, 1, 1), (1, 4, 1, 1), (1, 4, 1, 2),
                                                       (0, 3, 0, 1)])
def test_gamma_davidson_against_dense(ctx, precision, ndim, lock, sub32):
    g = pwgen.gamma_cell(10.0, 15.0, 8, 16, 25, nr=(30, 30, 30))
    h = oracle.dense_h_of(g.full)
    w, _ = oracle.eigh_lowest(h, g.nb)
    st, eig, resid, psi, stats = _solve(ctx, g, precision, ndim, lock=lock, sub32=sub32)
    print("gamma Davidson", precision, ndim, lock, stats, "max err", np.abs(eig - w).max())
    assert st == 0
    np.testing.assert_allclose(eig, w, atol=TOL_EIG, rtol=0)
    np.testing.assert_allclose(_gdot(psi, psi), np.eye(g.nb), atol=1e-10)
    full = g.expand(psi)
    r = np.linalg.norm(oracle.hpsi(h, full) - eig[:, None] * full, axis=1)
    np.testing.assert_allclose(resid, r, rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("precision,ndim", [(0, 3), (1, 2)])
def test_gamma_config2_solve_against_golden(ctx, precision, ndim):
    # the 64-atom cell at Gamma (diagonal D: the -i of the p projectors leaves
    # H unchanged) against the golden dense-oracle eigenvalues; mixed: the
    # float32 stage with float32 real Ritz rotations
    import os
    g = pwgen.gamma_cell(20.5, 25.0, 64, 128, pwgen.SEED_BASE + 2, nr=(72, 72, 72))
    w = np.loadtxt(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config2_eigenvalues.txt"))
    st, eig, resid, psi, stats = _solve(ctx, g, precision, ndim, sub32=2)
    print("gamma config-2 solve", stats, "max err", np.abs(eig - w).max())
    assert st == 0
    np.testing.assert_allclose(eig, w, atol=TOL_EIG, rtol=0)


@pytest.mark.parametrize("n3", [80, 144])
def test_gamma_group_z_passes_float64(ctx, n3):
    # float64 Gamma columns of n3 = 16 LS points beyond the quad form take the
    # 16-lane-group z passes (band pairs packed as a + i b)
    g = pwgen.gamma_cell(10.0, 15.0, 8, 15, 23, nr=(30, 30, n3))
    h = oracle.dense_h_of(g.full)
    got, _ = _hpsi(ctx, g, g.psi0)
    ref = oracle.hpsi(h, g.expand(g.psi0))[:, g.half]
    assert _rel(got, ref) <= 1e-11
    assert np.abs(got[:, 0].imag).max() == 0.0


@pytest.mark.parametrize("nb", [16, 7])
def test_gamma_pcg_against_dense(ctx, nb):
    # band-by-band CG on the half sphere: real whole-sphere inner products
    # (2 sum - G = 0 term) in every step and in the projections on the bands found
    from paper_0906_2569_amd import pwdft
    g = pwgen.gamma_cell(10.0, 15.0, 8, 16, 26, nr=(30, 30, 30))
    h = oracle.dense_h_of(g.full)
    w, _ = oracle.eigh_lowest(h, nb)
    plan = pwdft.Plan(ctx, g, precision=0, nb_max=nb, ndim_max=2, gamma=1)
    try:
        x = torch.from_numpy(np.ascontiguousarray(g.psi0[:nb])).cuda()
        st, eig, resid, stats = plan.pcg(x)
        torch.cuda.synchronize()
        eig, resid, psi = eig.cpu().numpy(), resid.cpu().numpy(), x.cpu().numpy()
    finally:
        plan.close()
    print("gamma CG", nb, stats.asdict(), "max err", np.abs(eig - w).max())
    assert st == 0 and stats.nconv == nb
    np.testing.assert_allclose(eig, w, atol=TOL_EIG, rtol=0)
    np.testing.assert_allclose(_gdot(psi, psi), np.eye(nb), atol=1e-10)
    assert np.abs(psi[:, 0].imag).max() == 0.0
    full = g.expand(psi)
    r = np.linalg.norm(oracle.hpsi(h, full) - eig[:, None] * full, axis=1)
    np.testing.assert_allclose(resid, r, rtol=1e-6, atol=1e-12)


def _gamma_us(seed, general=False):
    # a Gamma cell with ultrasoft q blocks: diagonal ones, or small real
    # symmetric ones (real-space-real projectors need real q at Gamma)
    g = pwgen.gamma_cell(10.0, 15.0, 8, 16, seed, nr=(30, 30, 30))
    if general:
        q = pwgen.hermitian_blocks(np.random.default_rng(seed), g.full.blk_off, scale=0.1)
        g.full.qmat = np.ascontiguousarray(q.real.astype(np.complex128))
    else:
        g.full.qmat = pwgen.ultrasoft_q(g.full, seed)
    return g


@pytest.mark.parametrize("prec,general", [(0, False), (0, True), (1, True)])
def test_gamma_spsi_against_dense(ctx, prec, general):
    from paper_0906_2569_amd import pwdft
    g = _gamma_us(28, general)
    s = oracle.dense_s_of(g.full)
    plan = pwdft.Plan(ctx, g, precision=prec, nb_max=g.nb, ndim_max=0, gamma=1)
    try:
        got = plan.spsi(torch.from_numpy(np.ascontiguousarray(g.psi0)).cuda(), prec=prec).cpu().numpy()
    finally:
        plan.close()
    ref = (g.expand(g.psi0) @ s.T)[:, g.half]
    assert _rel(got, ref) <= (1e-11 if prec == 0 else 2e-6)
    assert np.abs(got[:, 0].imag).max() == 0.0


@pytest.mark.parametrize("precision,lock,general", [(0, 1, False), (0, 0, True), (1, 1, True)])
def test_gamma_generalized_davidson_against_dense(ctx, precision, lock, general):
    g = _gamma_us(29, general)
    h, s = oracle.dense_h_of(g.full), oracle.dense_s_of(g.full)
    w, _ = oracle.eigh_lowest_gen(h, s, g.nb)
    st, eig, resid, psi, stats = _solve(ctx, g, precision, 2, lock=lock, sub32=1)
    print("gamma generalized Davidson", precision, lock, general, stats, "max err", np.abs(eig - w).max())
    assert st == 0
    np.testing.assert_allclose(eig, w, atol=TOL_EIG, rtol=0)
    full = g.expand(psi)
    np.testing.assert_allclose(np.real(np.conj(full) @ s @ full.T), np.eye(g.nb), atol=1e-10)
    r = np.linalg.norm(full @ h.T - eig[:, None] * (full @ s.T), axis=1)
    np.testing.assert_allclose(resid, r, rtol=1e-6, atol=1e-12)


def test_gamma_generalized_pcg_against_dense(ctx):
    from paper_0906_2569_amd import pwdft
    g = _gamma_us(30, True)
    h, s = oracle.dense_h_of(g.full), oracle.dense_s_of(g.full)
    nb = 8
    w, _ = oracle.eigh_lowest_gen(h, s, nb)
    plan = pwdft.Plan(ctx, g, precision=0, nb_max=nb, ndim_max=2, gamma=1)
    try:
        x = torch.from_numpy(np.ascontiguousarray(g.psi0[:nb])).cuda()
        st, eig, resid, stats = plan.pcg(x)
        torch.cuda.synchronize()
        eig, psi = eig.cpu().numpy(), x.cpu().numpy()
    finally:
        plan.close()
    print("gamma generalized CG", stats.asdict(), "max err", np.abs(eig - w).max())
    assert st == 0
    np.testing.assert_allclose(eig, w, atol=TOL_EIG, rtol=0)
    full = g.expand(psi)
    np.testing.assert_allclose(np.real(np.conj(full) @ s @ full.T), np.eye(nb), atol=1e-10)


def test_gamma_refuses_complex_q(ctx):
    # q blocks with an imaginary part cannot belong to real-space-real
    # projectors: the Gamma plan is refused, as for complex D
    from paper_0906_2569_amd import pwdft
    g = _gamma_us(31, True)
    q = pwgen.hermitian_blocks(np.random.default_rng(31), g.full.blk_off, scale=0.1)
    assert np.abs(q.imag).max() > 1e-3
    g.full.qmat = q
    with pytest.raises(pwdft.PwError) as ei:
        pwdft.Plan(ctx, g, precision=0, nb_max=g.nb, ndim_max=0, gamma=1)
    assert ei.value.status == pwdft.PW_EINVAL
