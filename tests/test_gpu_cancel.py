"""Cancelling solves (pw_cancel, pw_server_cancel) through the C ABI.  Every
solve here is bounded by max_iter, so a cancel that failed would still end."""
import threading
import time

import numpy as np
import pytest

from paper_0906_2569_amd import pwgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0906_2569_amd import pwdft
    return pwdft.Context(0)


def _never_converging(pwdft):
    # tolerance 0: the solve runs until max_iter (about 20 s at most here)
    return pwdft.default_opts(ndim=4, max_iter=20000, tol_resid=0.0, tol_deig=0.0)


def _run_in_thread(fn):
    box = {}

    def target():
        try:
            box["ret"] = fn()
        except Exception as e:   # the binding raises PwError for PW_ECANCELLED
            box["err"] = e
    t = threading.Thread(target=target)
    t.start()
    return t, box


def test_cancel_running_davidson(ctx):
    from paper_0906_2569_amd import pwdft
    p = pwgen.config1()
    plan = pwdft.Plan(ctx, p, precision=0, nb_max=p.nb, ndim_max=4)
    try:
        x = torch.from_numpy(p.psi0).cuda()
        eig = torch.empty(p.nb, dtype=torch.float64, device="cuda")
        res = torch.empty_like(eig)
        t0 = time.perf_counter()
        th, box = _run_in_thread(lambda: plan.davidson(x, eig, res, opts=_never_converging(pwdft)))
        time.sleep(0.5)
        plan.cancel()
        th.join(timeout=60)
        assert not th.is_alive()
        dt = time.perf_counter() - t0
        assert isinstance(box.get("err"), pwdft.PwError) and box["err"].status == pwdft.PW_ECANCELLED, box
        assert dt < 15.0
        # the outputs are the current Ritz pairs: finite, orthonormal vectors
        torch.cuda.synchronize()
        assert np.all(np.isfinite(eig.cpu().numpy())) and np.all(np.isfinite(res.cpu().numpy()))
        psi = x.cpu().numpy()
        np.testing.assert_allclose(np.conj(psi) @ psi.T, np.eye(p.nb), atol=1e-10)
        # the flag does not carry over: the next solve converges normally
        x.copy_(torch.from_numpy(p.psi0))
        st, _, _, stats = plan.davidson(x, opts=pwdft.default_opts(ndim=4))
        assert st == 0
    finally:
        plan.close()


def test_cancel_before_start_and_pcg(ctx):
    from paper_0906_2569_amd import pwdft
    p = pwgen.config1()
    plan = pwdft.Plan(ctx, p, precision=0, nb_max=p.nb, ndim_max=4)
    try:
        x = torch.from_numpy(p.psi0).cuda()
        plan.cancel()                      # no solve running: the next one stops at its first check
        with pytest.raises(pwdft.PwError) as ei:
            plan.davidson(x, opts=_never_converging(pwdft))
        assert ei.value.status == pwdft.PW_ECANCELLED
        x.copy_(torch.from_numpy(p.psi0))
        th, box = _run_in_thread(lambda: plan.pcg(x, max_iter=20000, tol_resid=0.0, tol_deig=0.0))
        time.sleep(0.5)
        plan.cancel()
        th.join(timeout=60)
        assert not th.is_alive()
        assert isinstance(box.get("err"), pwdft.PwError) and box["err"].status == pwdft.PW_ECANCELLED, box
    finally:
        plan.close()


def test_server_cancel_queued_and_running(ctx):
    from paper_0906_2569_amd import pwdft
    srv = pwdft.Server(ctx, nworkers=1, precision=pwdft.PW_FP64)
    try:
        p = pwgen.config1()
        q = pwgen.tiny_cell(51, a=6.0, ecut_ry=8.0, natoms=2, nb=6)
        xa = torch.from_numpy(p.psi0).cuda()
        xb = torch.from_numpy(q.psi0).cuda()
        ta, _, _ = srv.submit(p, xa, opts=_never_converging(pwdft))
        tb, _, _ = srv.submit(q, xb, opts=pwdft.default_opts(ndim=4))
        time.sleep(0.5)
        srv.cancel(tb)                     # still queued behind the running request
        with pytest.raises(pwdft.PwError) as eb:
            srv.wait(tb)
        assert eb.value.status == pwdft.PW_ECANCELLED
        srv.cancel(ta)                     # running
        with pytest.raises(pwdft.PwError) as ea:
            srv.wait(ta)
        assert ea.value.status == pwdft.PW_ECANCELLED
        # the server keeps serving
        xc = torch.from_numpy(q.psi0).cuda()
        tc, _, _ = srv.submit(q, xc, opts=pwdft.default_opts(ndim=4))
        st, stats, times = srv.wait(tc)
        assert st == 0
    finally:
        srv.close()
