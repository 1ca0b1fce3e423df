"""hpsi_apply captured once in a HIP graph and replayed: every replay equals the
eager call on the same input, bit for bit (same kernels, no atomics)."""
import numpy as np
import pytest

import oracle
from paper_0906_2569_amd import pwgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0906_2569_amd import pwdft
    return pwdft.Context(0)


def _random_block(rng, nb, npw):
    x = rng.standard_normal((nb, npw)) + 1j * rng.standard_normal((nb, npw))
    return x / np.linalg.norm(x, axis=1, keepdims=True)


@pytest.mark.parametrize("cfg,prec", [("config1", 0), ("config1", 1), ("config2", 0)])
def test_hpsi_graph_replays_equal_eager(ctx, cfg, prec):
    from paper_0906_2569_amd import pwdft
    p = getattr(pwgen, cfg)()
    nb = min(p.nb, 32)
    plan = pwdft.Plan(ctx, p, precision=prec, nb_max=nb, ndim_max=0)
    try:
        rng = np.random.default_rng(20090607)
        x = torch.from_numpy(_random_block(rng, nb, p.npw)).cuda()
        y = torch.empty_like(x)
        g = plan.hpsi_graph(x, y, prec=prec)
        for rep in range(4):
            # eager work between replays: a new input written in place, and the
            # eager product of the same input into another buffer
            x.copy_(torch.from_numpy(_random_block(rng, nb, p.npw)))
            ref = plan.hpsi(x.clone(), prec=prec)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(y, ref), f"{cfg} prec {prec} replay {rep}"
        if cfg == "config1" and prec == 0:
            # and the replayed product is H psi (float64 against the dense oracle)
            want = oracle.hpsi(oracle.dense_h_of(p), x.cpu().numpy())
            err = np.linalg.norm(y.cpu().numpy() - want, axis=1) / np.linalg.norm(want, axis=1)
            assert err.max() <= 1e-11
    finally:
        plan.close()


def test_graph_of_gamma_and_mixed_plans(ctx):
    # the C-ABI capture holds the side-stream projector products and their join
    from paper_0906_2569_amd import pwdft
    g = pwgen.gamma_cell(10.0, 15.0, 8, 16, 26, nr=(30, 30, 30))
    plan = pwdft.Plan(ctx, g, precision=1, nb_max=g.nb, ndim_max=0, gamma=1, nl_overlap=1)
    try:
        x = torch.from_numpy(g.psi0).cuda()
        y = torch.empty_like(x)
        graph = plan.hpsi_graph(x, y, prec=1)
        for rep in range(3):
            x.mul_(0.5 + rep)
            ref = plan.hpsi(x.clone(), prec=1)
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(y, ref), rep
        graph.close()
    finally:
        plan.close()


@pytest.mark.parametrize("gamma", [0, 1])
def test_graph_replays_after_set_potential(ctx, gamma):
    # a captured H.psi reads the plan's potential buffers: after
    # pw_plan_set_potential its replays give the product with the new V(r),
    # equal to the eager call (full sphere and Gamma plans)
    import dataclasses
    from paper_0906_2569_amd import pwdft
    if gamma:
        g = pwgen.gamma_cell(10.0, 15.0, 8, 16, 27, nr=(30, 30, 30))
        p, x0, full = g, g.psi0, g.full
    else:
        p = pwgen.config1()
        x0, full = p.psi0, p
    v2 = np.ascontiguousarray(full.vloc_r * 0.5 + 0.02)
    plan = pwdft.Plan(ctx, p, precision=0, nb_max=p.nb, ndim_max=0, gamma=gamma)
    try:
        x = torch.from_numpy(np.ascontiguousarray(x0)).cuda()
        y = torch.empty_like(x)
        gr = plan.hpsi_graph(x, y, prec=0)
        gr.replay()
        torch.cuda.synchronize()
        old = y.clone()
        plan.set_potential(torch.from_numpy(v2).cuda())
        for _ in range(2):
            ref = plan.hpsi(x.clone(), prec=0)
            torch.cuda.synchronize()
            gr.replay()
            torch.cuda.synchronize()
            assert torch.equal(y, ref)
        assert not torch.equal(y, old)
        h2 = oracle.dense_h_of(dataclasses.replace(full, vloc_r=v2))
        want = oracle.hpsi(h2, full.psi0)
        got = y.cpu().numpy()
        if gamma:
            want = want[:, g.half]
        err = np.linalg.norm(got - want, axis=1) / np.linalg.norm(want, axis=1)
        assert err.max() <= 1e-11
    finally:
        plan.close()
