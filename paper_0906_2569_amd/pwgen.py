"""Seeded synthetic inputs for the plane-wave H.psi / Davidson path.

This module only draws inputs: cells, the G-sphere (Miller indices and
Cartesian k+G), a real local potential on the FFT grid, Gaussian s/p
projectors, diagonal D blocks and random trial wavefunctions.  It holds none
of the method's arithmetic (no kinetic energy, no products with H, no
eigen-solves), so both the GPU path and the CPU oracle can consume it.

Conventions (Hartree atomic units; cut-offs are given in Ry):
  * cubic cell of edge ``a`` bohr; reciprocal vectors b_i = (2 pi / a) e_i;
    G = (2 pi / a) m for integer Miller m = (h, k, l).
  * the wavefunction sphere is {m : |k + G_m|^2 <= ecut_ry}, |q|^2 in
    bohr^-2 equals the kinetic energy in Ry (the boundary of the sphere is
    inclusive).  Order: ascending |k+G|^2, ties broken lexicographically on
    (h, k, l).
  * V(r) is stored as a real array ``[n3][n2][n1]`` (x fastest) and is the
    Fourier series V(r_j) = sum_m V(m) exp(+2 pi i m.j/n) of Hermitian
    coefficients V(-m) = conj(V(m)), V(0) = 0, supported on |G|^2 <= 4 ecut.
  * arrays of bands / projectors are column-major ``[ncol][npw]`` (the
    coefficients of one band are contiguous), complex128.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

RY_TO_HA = 0.5
SIGMA_V = 2.0        # bohr^-1, width of the Gaussian decay of V(G)
SIGMA_BETA = 2.0     # bohr^-1, radial width of the s/p projectors
V_RMS_HA = 0.5       # realised rms of V(r) over the grid points
NPROJ_PER_ATOM = 4   # s, px, py, pz


@dataclass
class Problem:
    """One plane-wave eigenproblem (one cell at one k-point)."""
    a: float                      # cubic cell edge, bohr
    ecut_ry: float                # wavefunction cut-off, Ry
    kpt: np.ndarray               # Cartesian k, bohr^-1, shape (3,)
    miller: np.ndarray            # int32 [npw][3]
    kpg: np.ndarray               # float64 [npw][3], k+G in bohr^-1
    nr: tuple                     # (n1, n2, n3)
    vloc_r: np.ndarray            # float64 [n3][n2][n1], Ha
    vg_miller: np.ndarray         # int32 [nv][3] support of V(G)
    vg_coef: np.ndarray           # complex128 [nv] V(G) in Ha (after rescale)
    tau: np.ndarray               # float64 [natoms][3] Cartesian positions, bohr
    beta: np.ndarray              # complex128 [nbeta][npw]
    blk_off: np.ndarray           # int32 [natoms+1] projector offsets
    dmat: np.ndarray              # complex128, concatenated nh x nh blocks (col-major), Ha
    nb: int                       # number of bands wanted
    psi0: np.ndarray              # complex128 [nb][npw] trial wavefunctions
    name: str = ""
    meta: dict = field(default_factory=dict)
    qmat: np.ndarray | None = None  # complex128 augmentation blocks q (col-major, like dmat); None: S = 1

    @property
    def npw(self) -> int:
        return int(self.miller.shape[0])

    @property
    def nbeta(self) -> int:
        return int(self.beta.shape[0])

    @property
    def natoms(self) -> int:
        return int(self.tau.shape[0])


# ----------------------------------------------------------------------------
# geometry helpers
# ----------------------------------------------------------------------------

def smooth_235(nmin: int) -> int:
    """Smallest integer >= nmin whose only prime factors are 2, 3 and 5."""
    n = max(1, int(nmin))
    while True:
        m = n
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        if m == 1:
            return n
        n += 1


def sphere(a: float, ecut_ry: float, kfrac=(0.0, 0.0, 0.0)):
    """Miller indices and k+G of the sphere |k+G|^2 <= ecut_ry, sorted.

    ``kfrac`` is k in crystal coordinates (units of b_i).  Returns
    (miller int32 [npw][3], kpg float64 [npw][3], kcart float64 [3]).
    """
    b = 2.0 * math.pi / a
    kfrac = np.asarray(kfrac, dtype=np.float64)
    kcart = b * kfrac
    gmax = math.sqrt(ecut_ry)
    mmax = int(math.ceil(gmax / b + np.abs(kfrac).max() + 1))
    r = np.arange(-mmax, mmax + 1)
    h, k, l = np.meshgrid(r, r, r, indexing="ij")
    m = np.stack([h.ravel(), k.ravel(), l.ravel()], axis=1)
    q = kcart[None, :] + b * m
    q2 = np.einsum("ij,ij->i", q, q)
    sel = q2 <= ecut_ry
    m, q, q2 = m[sel], q[sel], q2[sel]
    order = np.lexsort((m[:, 2], m[:, 1], m[:, 0], q2))
    return m[order].astype(np.int32), q[order].astype(np.float64), kcart


def min_grid(miller: np.ndarray) -> tuple:
    """Per-axis smallest {2,3,5}-smooth n with n >= 4*max|m|+1 (no aliasing)."""
    hmax = np.abs(miller).max(axis=0)
    return tuple(int(smooth_235(4 * int(h) + 1)) for h in hmax)


# ----------------------------------------------------------------------------
# random draws
# ----------------------------------------------------------------------------

def _vloc(rng, a, ecut_ry, nr):
    """Hermitian Gaussian-decaying random V(G) on |G|^2 <= 4 ecut and its V(r)."""
    b = 2.0 * math.pi / a
    gmax2 = 4.0 * ecut_ry
    mmax = int(math.ceil(math.sqrt(gmax2) / b))
    r = np.arange(-mmax, mmax + 1)
    h, k, l = np.meshgrid(r, r, r, indexing="ij")
    m = np.stack([h.ravel(), k.ravel(), l.ravel()], axis=1)
    g2 = (b * b) * np.einsum("ij,ij->i", m, m).astype(np.float64)
    keep = g2 <= gmax2
    # half space G > 0 (lexicographic on h, k, l)
    pos = (m[:, 0] > 0) | ((m[:, 0] == 0) & (m[:, 1] > 0)) | \
          ((m[:, 0] == 0) & (m[:, 1] == 0) & (m[:, 2] > 0))
    half = m[keep & pos]
    g2h = (b * b) * np.einsum("ij,ij->i", half, half).astype(np.float64)
    order = np.lexsort((half[:, 2], half[:, 1], half[:, 0]))
    half, g2h = half[order], g2h[order]
    xi = rng.standard_normal((half.shape[0], 2))
    coef = np.exp(-g2h / (2.0 * SIGMA_V ** 2)) * (xi[:, 0] + 1j * xi[:, 1]) / math.sqrt(2.0)
    n1, n2, n3 = nr
    vgrid = np.zeros((n3, n2, n1), dtype=np.complex128)
    vgrid[half[:, 2] % n3, half[:, 1] % n2, half[:, 0] % n1] = coef
    vgrid[(-half[:, 2]) % n3, (-half[:, 1]) % n2, (-half[:, 0]) % n1] = np.conj(coef)
    vr = np.fft.ifftn(vgrid) * (n1 * n2 * n3)
    vr = np.ascontiguousarray(vr.real)
    rms = math.sqrt(float(np.mean(vr * vr)))
    scale = V_RMS_HA / rms
    vr *= scale
    coef = coef * scale
    vm = np.concatenate([half, -half], axis=0).astype(np.int32)
    vc = np.concatenate([coef, np.conj(coef)])
    return vr, vm, vc


def _projectors(kpg, tau):
    """Gaussian-radial s and Cartesian p projectors, each normalised on the sphere."""
    q2 = np.einsum("ij,ij->i", kpg, kpg)
    g = np.exp(-q2 / (2.0 * SIGMA_BETA ** 2))
    out = []
    for t in tau:
        sf = np.exp(-1j * (kpg @ t))
        shapes = [g, kpg[:, 0] / SIGMA_BETA * g, kpg[:, 1] / SIGMA_BETA * g,
                  kpg[:, 2] / SIGMA_BETA * g]
        for s in shapes:
            v = s * sf
            nrm = math.sqrt(float(np.vdot(v, v).real))
            out.append(v / nrm if nrm > 0 else v)
    return np.ascontiguousarray(np.array(out, dtype=np.complex128).reshape(len(out), -1))


def random_psi(rng, nb, npw):
    """Complex-normal trial wavefunctions, each band normalised to 1."""
    z = rng.standard_normal((nb, npw, 2))
    psi = (z[..., 0] + 1j * z[..., 1]) / math.sqrt(2.0)
    psi /= np.linalg.norm(psi, axis=1, keepdims=True)
    return np.ascontiguousarray(psi)


def hermitian_blocks(rng, blk_off, scale=0.5):
    """Random complex Hermitian D blocks (one per atom), concatenated column-major.

    Block I is nh x nh with nh = blk_off[I+1] - blk_off[I]; entry (i, j) of a
    block is stored at offset i + j*nh inside it.  Diagonal U[0.25, 1] Ha,
    off-diagonal complex normal times ``scale``/2, Hermitian by construction.
    """
    out = []
    for i in range(len(blk_off) - 1):
        nh = int(blk_off[i + 1] - blk_off[i])
        z = rng.standard_normal((nh, nh)) + 1j * rng.standard_normal((nh, nh))
        a = 0.25 * scale * (z + np.conj(z.T))
        a[np.diag_indices(nh)] = rng.uniform(0.25, 1.0, size=nh)
        out.append(np.ascontiguousarray(a.T).ravel())     # column-major
    return np.concatenate(out) if out else np.zeros((0,), dtype=np.complex128)


def ultrasoft_q(problem, seed, lo=0.1, hi=0.5):
    """Diagonal augmentation blocks q (one per atom, U[lo, hi] on the diagonal,
    concatenated column-major like dmat), drawn from their own stream, so that
    S = 1 + sum_I beta_I q_I beta_I^H is Hermitian and positive definite."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), 77])))
    blocks = []
    for i in range(len(problem.blk_off) - 1):
        nh = int(problem.blk_off[i + 1] - problem.blk_off[i])
        blocks.append(np.diag(rng.uniform(lo, hi, size=nh)).astype(np.complex128).T.ravel())
    return np.concatenate(blocks) if blocks else np.zeros((0,), dtype=np.complex128)


def make_cell(a, ecut_ry, natoms, nb, seed, kfrac=(0.0, 0.0, 0.0), nr=None,
              name="", with_vloc=True, with_beta=True, streams=None):
    """Build one seeded problem.

    Sub-streams of ``SeedSequence(seed)`` are used in the fixed order
    positions, V(G), D, psi.  ``streams`` may pass already-spawned sequences
    (used when several k-points share one cell).
    """
    if streams is None:
        streams = np.random.SeedSequence(seed).spawn(4)
    rng_pos, rng_v, rng_d, rng_psi = (np.random.Generator(np.random.PCG64(s)) for s in streams)
    miller, kpg, kcart = sphere(a, ecut_ry, kfrac)
    if nr is None:
        nr = min_grid(miller)
    nr = tuple(int(x) for x in nr)
    npw = miller.shape[0]
    tau = rng_pos.random((natoms, 3)) * a
    if with_vloc:
        vr, vm, vc = _vloc(rng_v, a, ecut_ry, nr)
    else:
        vr = np.zeros((nr[2], nr[1], nr[0]))
        vm = np.zeros((0, 3), dtype=np.int32)
        vc = np.zeros((0,), dtype=np.complex128)
    if with_beta and natoms > 0:
        beta = _projectors(kpg, tau)
        dvals = rng_d.uniform(0.5, 2.0, size=(natoms, NPROJ_PER_ATOM)) * RY_TO_HA
        blocks = []
        for i in range(natoms):
            blk = np.diag(dvals[i]).astype(np.complex128)
            blocks.append(blk.T.ravel())   # col-major
        dmat = np.concatenate(blocks)
        blk_off = (np.arange(natoms + 1) * NPROJ_PER_ATOM).astype(np.int32)
    else:
        beta = np.zeros((0, npw), dtype=np.complex128)
        dmat = np.zeros((0,), dtype=np.complex128)
        blk_off = np.zeros((1,), dtype=np.int32)
    psi0 = random_psi(rng_psi, nb, npw)
    return Problem(a=float(a), ecut_ry=float(ecut_ry), kpt=kcart, miller=miller, kpg=kpg,
                   nr=nr, vloc_r=vr, vg_miller=vm, vg_coef=vc, tau=tau, beta=beta,
                   blk_off=blk_off, dmat=dmat, nb=int(nb), psi0=psi0, name=name,
                   meta={"seed": seed, "natoms": natoms, "kfrac": tuple(kfrac)})


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------

SEED_BASE = 20090600


def config1(**kw):
    """a = 10 bohr, Gamma, 15 Ry (npw 949), grid 30^3, 8 atoms, 32 beta, 16 bands."""
    return make_cell(10.0, 15.0, 8, 16, SEED_BASE + 1, nr=(30, 30, 30),
                     name="cfg1_a10_15Ry_nb16", **kw)


def config2(**kw):
    """a = 20.5 bohr, Gamma, 25 Ry (npw 18277), grid 72^3, 64 atoms, 256 beta, 128 bands."""
    return make_cell(20.5, 25.0, 64, 128, SEED_BASE + 2, nr=(72, 72, 72),
                     name="cfg2_a20.5_25Ry_nb128", **kw)


def config3(**kw):
    """Identical inputs to config2 (same seed); run in mixed precision."""
    p = make_cell(20.5, 25.0, 64, 128, SEED_BASE + 2, nr=(72, 72, 72),
                  name="cfg3_a20.5_25Ry_nb128_mixed", **kw)
    return p


KPTS_2x2x1 = ((0.25, 0.25, 0.0), (-0.25, -0.25, 0.0), (0.25, -0.25, 0.0), (-0.25, 0.25, 0.0))


def config4_cells(ncells=32, ecut_ry=25.0, seed=SEED_BASE + 4):
    """Parameters of the batched workload: (a, natoms) per cell."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    a = rng.uniform(10.0, 20.0, size=ncells)
    nat = rng.integers(8, 65, size=ncells)
    return [(float(a[i]), int(nat[i])) for i in range(ncells)]


def config4(ncells=32, ecut_ry=25.0, seed=SEED_BASE + 4, kpts=KPTS_2x2x1):
    """32 cells x 4 k-points (shifted 2x2x1 set, crystal (+-1/4, +-1/4, 0)).

    The k-points of one cell share its positions, V and D (same sub-streams);
    psi is drawn per k-point.
    """
    cells = config4_cells(ncells, ecut_ry, seed)
    root = np.random.SeedSequence(seed).spawn(ncells)
    out = []
    for ic, (a, nat) in enumerate(cells):
        base = root[ic].spawn(3 + len(kpts))
        for ik, kf in enumerate(kpts):
            streams = [base[0], base[1], base[2], base[3 + ik]]
            out.append(make_cell(a, ecut_ry, nat, 2 * nat, None, kfrac=kf,
                                 name=f"cfg4_c{ic}_k{ik}", streams=streams))
    return out


def serving_request(idx, seed=SEED_BASE + 5, ecut_ry=30.0, max_atoms=512, min_atoms=8):
    """One request of the served workload: log-uniform atom count, constant density."""
    ss = np.random.SeedSequence([seed, idx]).spawn(5)
    rng = np.random.Generator(np.random.PCG64(ss[4]))
    u = rng.random()
    natoms = int(round(min_atoms * (max_atoms / min_atoms) ** u))
    a = 41.0 * (natoms / 512.0) ** (1.0 / 3.0)
    t = rng.uniform(0.0, 0.5)
    return make_cell(a, ecut_ry, natoms, 2 * natoms, None, kfrac=(t, 0.0, 0.0),
                     name=f"req{idx}_nat{natoms}", streams=ss[:4])


def tiny_cell(seed, a=5.0, ecut_ry=6.0, natoms=2, nb=4, kfrac=(0.0, 0.0, 0.0), nr=None, **kw):
    """Small cells for brute-force checks (npw ~ 10-100)."""
    return make_cell(a, ecut_ry, natoms, nb, seed, kfrac=kfrac, nr=nr, name=f"tiny{seed}", **kw)


def config5_largest(nb=1024, **kw):
    """The largest served request at Gamma: a = 41 bohr, 30 Ry (npw 191471),
    grid 144^3, 512 atoms, 2048 beta, 1024 bands (fewer with ``nb``: the
    first nb bands of the same draw)."""
    return make_cell(41.0, 30.0, 512, nb, SEED_BASE + 5, name=f"cfg5_a41_30Ry_nat512_nb{nb}", **kw)


CONFIGS = {1: config1, 2: config2, 3: config3}


# ----------------------------------------------------------------------------
# Gamma point, real wavefunctions: half-sphere storage
# ----------------------------------------------------------------------------

def half_sphere_index(miller: np.ndarray) -> np.ndarray:
    """Indices of the half sphere in a full Gamma sphere: G = 0 first, then the
    G > 0 (lexicographic on (h, k, l)) in the sphere's order.  Their mirrors -G
    make up the rest of the sphere."""
    m = np.asarray(miller)
    zero = np.nonzero((m == 0).all(axis=1))[0]
    assert len(zero) == 1, "the Gamma sphere holds G = 0 once"
    pos = (m[:, 0] > 0) | ((m[:, 0] == 0) & (m[:, 1] > 0)) | ((m[:, 0] == 0) & (m[:, 1] == 0) & (m[:, 2] > 0))
    return np.concatenate([zero, np.nonzero(pos)[0]])


def mirror_index(miller: np.ndarray) -> np.ndarray:
    """For each G of the sphere, the index of -G."""
    m = np.asarray(miller)
    key = {tuple(x): i for i, x in enumerate(m.tolist())}
    return np.array([key[(-x[0], -x[1], -x[2])] for x in m.tolist()], dtype=np.int64)


@dataclass
class GammaProblem:
    """A Gamma-point cell in two forms: `full` (the complex problem on the whole
    sphere, its projectors real in real space) and the half-sphere arrays the
    real-wavefunction path takes (`miller`, `kpg`, `beta`, `psi0`, indices into
    the full sphere in `half`)."""
    full: Problem
    half: np.ndarray
    miller: np.ndarray
    kpg: np.ndarray
    beta: np.ndarray
    psi0: np.ndarray

    def __getattr__(self, name):     # everything else as in the full problem
        return getattr(self.full, name)

    @property
    def npw(self) -> int:
        return int(self.miller.shape[0])

    def expand(self, x_half: np.ndarray) -> np.ndarray:
        """Full-sphere coefficients of real functions given on the half sphere:
        f(-G) = conj(f(G))."""
        x_half = np.atleast_2d(x_half)
        out = np.zeros((x_half.shape[0], self.full.npw), dtype=np.complex128)
        out[:, self.half] = x_half
        mir = mirror_index(self.full.miller)
        out[:, mir[self.half]] = np.conj(x_half)
        return out


def gamma_cell(a, ecut_ry, natoms, nb, seed, nr=None, name="", with_vloc=True, with_beta=True):
    """A Gamma-point cell for the real-wavefunction path.  As make_cell, with
    the p projectors multiplied by -i (the (-i)^l factor of the structure
    factor form), so that every projector is real in real space:
    beta(-G) = conj(beta(G)).  The trial block is real in real space (its
    half-sphere coefficients, with psi(0) real, and their mirrors)."""
    p = make_cell(a, ecut_ry, natoms, nb, seed, nr=nr, name=name or f"gamma{seed}",
                  with_vloc=with_vloc, with_beta=with_beta)
    if p.nbeta:
        beta = p.beta.copy()
        for j in range(p.nbeta):
            if j % NPROJ_PER_ATOM != 0:
                beta[j] *= -1j
        p.beta = beta
    half = half_sphere_index(p.miller)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed or 0), 78])))
    z = rng.standard_normal((nb, len(half), 2))
    ph = (z[..., 0] + 1j * z[..., 1]) / math.sqrt(2.0)
    ph[:, 0] = ph[:, 0].real
    g = GammaProblem(full=p, half=half, miller=np.ascontiguousarray(p.miller[half]),
                     kpg=np.ascontiguousarray(p.kpg[half]), beta=np.ascontiguousarray(p.beta[:, half]),
                     psi0=None)
    full_psi = g.expand(ph)
    full_psi /= np.linalg.norm(full_psi, axis=1, keepdims=True)
    p.psi0 = full_psi
    g.psi0 = np.ascontiguousarray(full_psi[:, half])
    return g
