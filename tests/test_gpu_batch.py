"""Batched H.psi and Davidson (independent cells and k-points) against the
same problems run alone and against the dense FP64 oracle."""
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


def _problems():
    # mixed sizes, grids (register and LDS plane passes) and k-points; the
    # last two are the +-k pair of one cell (time-reversal twins)
    ps = [pwgen.config1(),
          pwgen.tiny_cell(51, a=6.0, ecut_ry=8.0, natoms=2, nb=6, kfrac=(0.25, 0.25, 0.0)),
          pwgen.tiny_cell(52, a=7.0, ecut_ry=9.0, natoms=4, nb=8, kfrac=(0.1, -0.2, 0.3), nr=(36, 30, 40)),
          pwgen.tiny_cell(53, a=8.0, ecut_ry=10.0, natoms=3, nb=10, kfrac=(0.0, 0.0, 0.0), nr=(36, 36, 36))]
    ss = np.random.SeedSequence(54).spawn(4)
    for kf in ((0.25, 0.25, 0.0), (-0.25, -0.25, 0.0)):
        ps.append(pwgen.make_cell(6.5, 9.0, 3, 8, None, kfrac=kf, streams=ss))
    return ps


@pytest.fixture(scope="module")
def batch(ctx):
    from paper_0906_2569_amd import pwdft
    ps = _problems()
    plans = [pwdft.Plan(ctx, p, precision=pwdft.PW_MIXED, nb_max=p.nb, ndim_max=3) for p in ps]
    yield ps, plans
    for pl in plans:
        pl.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_hpsi_batched_equals_alone(ctx, batch, prec):
    from paper_0906_2569_amd import pwdft
    ps, plans = batch
    xs = [torch.from_numpy(p.psi0).cuda() for p in ps]
    alone = []
    for pl, x in zip(plans, xs):
        y = torch.empty_like(x)
        pl.hpsi(x, y, prec=prec)
        alone.append(y)
    outs = [torch.full_like(x, complex(float("nan"), 0.0)) for x in xs]
    pwdft.hpsi_batched(ctx, plans, xs, outs, prec=prec, nstreams=3)
    torch.cuda.synchronize()
    for a, b in zip(alone, outs):
        assert torch.equal(a, b)          # same kernels, same plan: bit for bit
    if prec == 0:
        h = oracle.dense_h_of(ps[0])
        ref = oracle.hpsi(h, ps[0].psi0)
        got = outs[0].cpu().numpy()
        assert (np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)).max() <= 1e-11


@pytest.mark.parametrize("nworkers", [1, 4])
def test_davidson_batched_against_alone_and_dense(ctx, batch, nworkers):
    from paper_0906_2569_amd import pwdft
    ps, plans = batch
    opts = pwdft.default_opts(ndim=3)
    xs = [torch.from_numpy(p.psi0).cuda() for p in ps]
    st, sts, eigs, res, stats = pwdft.davidson_batched(ctx, plans, xs, opts=opts, nworkers=nworkers)
    assert st == 0 and all(s == 0 for s in sts)
    for p, pl, x, e, r in zip(ps, plans, xs, eigs, res):
        w, _ = oracle.eigh_lowest(oracle.dense_h_of(p), p.nb)
        np.testing.assert_allclose(e.cpu().numpy(), w, atol=TOL_EIG, rtol=0)
        assert r.max().item() <= 1e-6
        xa = torch.from_numpy(p.psi0).cuda()
        st1, e1, r1, _ = pl.davidson(xa, opts=opts)
        torch.cuda.synchronize()
        assert st1 == 0
        np.testing.assert_allclose(e.cpu().numpy(), e1.cpu().numpy(), atol=1e-10, rtol=0)
    # time-reversal twins (+k, -k of one cell): identical spectra
    np.testing.assert_allclose(eigs[-1].cpu().numpy(), eigs[-2].cpu().numpy(), atol=2 * TOL_EIG)


def test_batched_argument_errors(ctx, batch):
    from paper_0906_2569_amd import pwdft
    ps, plans = batch
    xs = [torch.from_numpy(p.psi0).cuda() for p in ps[:2]]
    with pytest.raises(pwdft.PwError) as ei:
        pwdft.davidson_batched(ctx, [plans[0], plans[0]], [xs[0], xs[0].clone()])
    assert ei.value.status == pwdft.PW_EINVAL
    with pytest.raises(pwdft.PwError) as ei:
        pwdft.hpsi_batched(ctx, [plans[1], plans[1]], [xs[1], xs[1]], [torch.empty_like(xs[1])] * 2)
    assert ei.value.status == pwdft.PW_EINVAL
    pwdft.hpsi_batched(ctx, [], [], [])   # empty batch is a no-op


def test_batched_not_converged_status(ctx, batch):
    from paper_0906_2569_amd import pwdft
    ps, plans = batch
    xs = [torch.from_numpy(p.psi0).cuda() for p in ps[:3]]
    st, sts, eigs, res, stats = pwdft.davidson_batched(ctx, plans[:3], xs,
                                                       opts=pwdft.default_opts(max_iter=1), nworkers=2)
    assert st == pwdft.PW_ENOTCONV and all(s == pwdft.PW_ENOTCONV for s in sts)
    for p, e in zip(ps, eigs):
        w, _ = oracle.eigh_lowest(oracle.dense_h_of(p), p.nb)
        assert np.all(e.cpu().numpy() >= w - 1e-10)   # Ritz values bound the eigenvalues from above


def test_concurrent_cooperative_eigensolver(ctx):
    # reduced problems of 64..512 rows use the multi-workgroup
    # tridiagonalization; several of them running at once (other kernels
    # sharing the compute units) must give the same results as one at a time
    from paper_0906_2569_amd import pwdft
    ps = [pwgen.serving_request(i, ecut_ry=12.0, max_atoms=24, min_atoms=8) for i in range(1, 5)]
    assert all(2 * p.nb >= 64 for p in ps)
    opts = pwdft.default_opts(ndim=2)
    plans = [pwdft.Plan(ctx, p, precision=pwdft.PW_MIXED, nb_max=p.nb, ndim_max=2) for p in ps]
    try:
        alone = []
        for pl, p in zip(plans, ps):
            x = torch.from_numpy(p.psi0).cuda()
            st, e, _, _ = pl.davidson(x, opts=opts)
            torch.cuda.synchronize()
            assert st == 0
            alone.append(e.cpu().numpy())
        for _ in range(2):
            xs = [torch.from_numpy(p.psi0).cuda() for p in ps]
            st, sts, eigs, res, stats = pwdft.davidson_batched(ctx, plans, xs, opts=opts, nworkers=4)
            assert st == 0 and all(s == 0 for s in sts)
            for e, ea in zip(eigs, alone):
                np.testing.assert_allclose(e.cpu().numpy(), ea, atol=1e-10, rtol=0)
    finally:
        for pl in plans:
            pl.close()
