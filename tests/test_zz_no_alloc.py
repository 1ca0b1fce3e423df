"""The allocation-free reduced eigensolver against the allocating one, through the C ABI."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0906_2569_amd import pwdft
    return pwdft.Context(0)


def _pair(rng, n):
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    h = (x + x.conj().T) / 2
    y = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    s = y @ y.conj().T / n + np.eye(n)
    return h, s


def _run(ctx, h, s, nev, noalloc):
    from paper_0906_2569_amd import pwdft
    hd = torch.from_numpy(np.ascontiguousarray(h.T)).cuda()
    sd = torch.from_numpy(np.ascontiguousarray(s.T)).cuda()
    w, c, dbg = pwdft.reduced_eigh(ctx, hd, sd, nev, debug=True, noalloc=noalloc)
    torch.cuda.synchronize()
    return w.cpu().numpy(), c.cpu().numpy().T, dbg.cpu().numpy()


def test_noalloc_matches_allocating_entry_point(ctx):
    # two calls in a row, the second smaller: the static workspace keeps the
    # first call's contents, and the second must not depend on them
    for n, nev, seed in ((256, 128, 1), (200, 90, 2), (70, 35, 3)):
        rng = np.random.default_rng(seed)
        h, s = _pair(rng, n)
        w0, c0, t0 = _run(ctx, h, s, nev, noalloc=False)
        w1, c1, t1 = _run(ctx, h, s, nev, noalloc=True)
        tol = 1e-12 * n
        np.testing.assert_allclose(w1, w0, atol=tol, rtol=0)
        # the tridiagonal: d (n values) and e (n - 1 values)
        np.testing.assert_allclose(t1[:2 * n - 1], t0[:2 * n - 1], atol=tol, rtol=0)
        # eigenvectors agree up to a phase per column (the spectrum of random
        # matrices has no degeneracy); S-orthonormal, small residuals
        ph = np.sum(np.conj(c0) * (s @ c1), axis=0)
        np.testing.assert_allclose(np.abs(ph), 1.0, atol=1e-9)
        np.testing.assert_allclose(c1, c0 * ph[None, :], atol=1e-9)
        r = np.linalg.norm(h @ c1 - (s @ c1) * w1[None, :], axis=0).max()
        assert r <= 1e-10 * n
        print(f"n={n}: max |w_noalloc - w| = {np.abs(w1 - w0).max():.2e}, bitwise equal: "
              f"{np.array_equal(w1, w0) and np.array_equal(c1, c0)}")


def test_noalloc_rejects_sizes_beyond_its_workspace(ctx):
    from paper_0906_2569_amd import pwdft
    rng = np.random.default_rng(4)
    h, s = _pair(rng, 257)
    with pytest.raises(pwdft.PwError) as ei:
        _run(ctx, h, s, 10, noalloc=True)
    assert ei.value.status == pwdft.PW_EINVAL
    assert "256" in str(ei.value)
