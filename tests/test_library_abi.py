"""The C-ABI library loads and exports every symbol include/pwdft.h declares (no GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_0906_2569_amd", "libpwdft.so")
HDR = os.path.join(ROOT, "include", "pwdft.h")


def declared():
    text = open(HDR).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_0906_2569_amd import build
        build.build()
    lib = ctypes.CDLL(LIB)
    lib.pw_footprint_bytes.restype = ctypes.c_size_t
    return lib


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("hpsi_apply", "davidson_solve", "pw_plan_create", "pw_ctx_create", "pw_reduced_eigh"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for n in declared():
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if " T " in l)
    assert set(declared()) <= exported


def test_binding_lists_every_export():
    from paper_0906_2569_amd import pwdft
    assert sorted(pwdft.EXPORTS) == declared()


def test_host_side_validation_without_gpu(lib):
    # pw_footprint_bytes validates on the host only: a grid below 4*max|m|+1
    # is rejected (0 bytes), a valid one gives a positive footprint
    import numpy as np
    from paper_0906_2569_amd import pwdft, pwgen
    pwdft.load(LIB)
    p = pwgen.config1()
    s = pwdft.Problem()
    miller = np.ascontiguousarray(p.miller, dtype=np.int32)
    kpg = np.ascontiguousarray(p.kpg)
    blk = np.ascontiguousarray(p.blk_off, dtype=np.int32)
    dmat = np.ascontiguousarray(p.dmat)
    s.npw = p.npw
    s.miller = miller.ctypes.data
    s.kpg = kpg.ctypes.data
    s.vloc_r = 1            # never dereferenced on the host
    s.nbeta = p.nbeta
    s.beta = 1
    s.ld_beta = p.npw
    s.nblk = len(blk) - 1
    s.blk_off = blk.ctypes.data
    s.dmat = dmat.ctypes.data
    o = pwdft.PlanOpts(pwdft.PW_FP64, 16, 4)
    for n, ok in ((30, True), (25, True), (24, False), (16, False)):
        s.nr[0] = s.nr[1] = s.nr[2] = n
        fp = lib.pw_footprint_bytes(ctypes.byref(s), ctypes.byref(o))
        assert (fp > 0) == ok, n
    s.nr[0] = s.nr[1] = s.nr[2] = 30
    s.ld_beta = p.npw - 1
    assert lib.pw_footprint_bytes(ctypes.byref(s), ctypes.byref(o)) == 0
    s.ld_beta = p.npw
    s.nr[0] = 49          # 7^2: not a 2,3,5-smooth FFT length
    assert lib.pw_footprint_bytes(ctypes.byref(s), ctypes.byref(o)) == 0


def test_davidson_option_defaults_and_layout(lib):
    # the C defaults land in the binding's fields one for one: a field order
    # or padding that differed between include/pwdft.h and the binding would
    # put them in the wrong places
    from paper_0906_2569_amd import pwdft
    pwdft.load(LIB)
    o = pwdft.DavOpts()
    ctypes.memset(ctypes.byref(o), 0x7F, ctypes.sizeof(o))
    lib.pw_david_opts_default(ctypes.byref(o))
    assert ctypes.sizeof(o) == 56
    assert (o.ndim, o.max_iter, o.lock, o.sub32) == (2, 200, 1, 1)
    assert (o.tol_resid, o.tol_deig, o.precond_floor, o.ladder_switch) == (1e-6, 5e-9, 0.2, 3e-4)
    assert not o.history


def test_cg_and_server_option_defaults_and_layout(lib):
    from paper_0906_2569_amd import pwdft
    pwdft.load(LIB)
    c = pwdft.CgOpts()
    ctypes.memset(ctypes.byref(c), 0x7F, ctypes.sizeof(c))
    lib.pw_cg_opts_default(ctypes.byref(c))
    assert ctypes.sizeof(c) == 32
    assert (c.max_iter, c.tol_resid, c.tol_deig, c.precond_floor) == (400, 1e-6, 5e-9, 0.2)
    s = pwdft.ServerOpts()
    ctypes.memset(ctypes.byref(s), 0x7F, ctypes.sizeof(s))
    lib.pw_server_opts_default(ctypes.byref(s))
    assert ctypes.sizeof(s) == 24
    assert (s.nworkers, s.mem_budget, s.precision, s.gamma) == (4, 0, pwdft.PW_MIXED, 0)
