"""Python binding of libpwdft (ctypes; argument marshalling only).

Every computation runs in the HIP library; torch tensors provide device
memory and streams.  Loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpwdft.so")

PW_OK, PW_ENOTCONV = 0, 1
PW_EINVAL, PW_ENOMEM, PW_EDEVICE, PW_EBREAKDOWN, PW_ENAN, PW_ECANCELLED = -1, -2, -3, -4, -5, -6
PW_FP64, PW_MIXED = 0, 1
STATUS_NAMES = {0: "PW_OK", 1: "PW_ENOTCONV", -1: "PW_EINVAL", -2: "PW_ENOMEM", -3: "PW_EDEVICE",
                -4: "PW_EBREAKDOWN", -5: "PW_ENAN", -6: "PW_ECANCELLED"}

# every symbol include/pwdft.h declares
EXPORTS = ["pw_last_error", "pw_ctx_create", "pw_ctx_destroy", "pw_david_opts_default",
           "pw_footprint_bytes", "pw_plan_create", "pw_plan_destroy", "pw_plan_info",
           "pw_plan_set_potential", "hpsi_apply", "davidson_solve", "hpsi_apply_batched", "davidson_solve_batched",
           "pw_reduced_eigh", "pw_reduced_eigh_noalloc", "pw_density", "pw_scf_norm", "pcg_solve", "pw_cg_opts_default", "spsi_apply", "pw_cancel", "pw_hpsi_graph_create",
           "pw_graph_launch", "pw_graph_destroy", "pw_server_cancel", "pw_profile_enable", "pw_server_opts_default", "pw_server_create",
           "pw_server_submit", "pw_server_wait", "pw_server_poll", "pw_server_clock", "pw_server_destroy",
           "pw_server_info", "pw_profile_count", "pw_profile_name", "pw_profile_read", "pw_profile_only"]


class PwError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Problem(C.Structure):
    _fields_ = [("npw", C.c_int32), ("miller", C.c_void_p), ("kpg", C.c_void_p),
                ("nr", C.c_int32 * 3), ("vloc_r", C.c_void_p), ("nbeta", C.c_int32),
                ("beta", C.c_void_p), ("ld_beta", C.c_int32), ("nblk", C.c_int32),
                ("blk_off", C.c_void_p), ("dmat", C.c_void_p), ("qmat", C.c_void_p)]


class PlanOpts(C.Structure):
    _fields_ = [("precision", C.c_int), ("nb_max", C.c_int32), ("ndim_max", C.c_int32),
                ("plane_mode", C.c_int32), ("fft_ws_bytes", C.c_size_t), ("nl_overlap", C.c_int32),
                ("density", C.c_int32), ("gamma", C.c_int32)]


class DavOpts(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("max_iter", C.c_int32), ("tol_resid", C.c_double),
                ("tol_deig", C.c_double), ("precond_floor", C.c_double),
                ("ladder_switch", C.c_double), ("history", C.POINTER(C.c_double)), ("lock", C.c_int32),
                ("sub32", C.c_int32)]


class CgOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("tol_resid", C.c_double), ("tol_deig", C.c_double),
                ("precond_floor", C.c_double)]


class CgStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("max_band_iters", C.c_int32), ("nconv", C.c_int32),
                ("max_resid", C.c_double)]

    def asdict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerOpts(C.Structure):
    _fields_ = [("nworkers", C.c_int32), ("mem_budget", C.c_size_t), ("precision", C.c_int), ("gamma", C.c_int32)]


class DavStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("n_hpsi_fp32", C.c_int32),
                ("n_hpsi_fp64", C.c_int32), ("nconv", C.c_int32), ("iters_fp32", C.c_int32),
                ("fresh_starts", C.c_int32), ("nlocked", C.c_int32), ("max_resid", C.c_double)]

    def asdict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Load libpwdft.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_0906_2569_amd.build`")
    lib = C.CDLL(path)
    lib.pw_last_error.restype = C.c_char_p
    lib.pw_ctx_create.argtypes = [C.c_int, C.POINTER(C.c_void_p)]
    lib.pw_ctx_destroy.argtypes = [C.c_void_p]
    lib.pw_david_opts_default.argtypes = [C.POINTER(DavOpts)]
    lib.pw_david_opts_default.restype = None
    lib.pw_footprint_bytes.argtypes = [C.POINTER(Problem), C.POINTER(PlanOpts)]
    lib.pw_footprint_bytes.restype = C.c_size_t
    lib.pw_plan_create.argtypes = [C.c_void_p, C.POINTER(Problem), C.POINTER(PlanOpts), C.POINTER(C.c_void_p)]
    lib.pw_plan_destroy.argtypes = [C.c_void_p]
    lib.pw_plan_info.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
    lib.pw_plan_set_potential.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    lib.hpsi_apply.argtypes = [C.c_void_p, C.c_int, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                               C.c_int32, C.c_void_p]
    lib.spsi_apply.argtypes = lib.hpsi_apply.argtypes
    lib.pw_cancel.argtypes = [C.c_void_p]
    lib.pw_hpsi_graph_create.argtypes = [C.c_void_p, C.c_int, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                                         C.c_int32, C.POINTER(C.c_void_p)]
    lib.pw_graph_launch.argtypes = [C.c_void_p, C.c_void_p]
    lib.pw_graph_destroy.argtypes = [C.c_void_p]
    lib.pw_server_cancel.argtypes = [C.c_void_p, C.c_int64]
    lib.davidson_solve.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                                   C.c_void_p, C.POINTER(DavOpts), C.POINTER(DavStats), C.c_void_p]
    P = C.POINTER
    lib.hpsi_apply_batched.argtypes = [C.c_void_p, C.c_int32, P(C.c_void_p), C.c_int, P(C.c_int32),
                                       P(C.c_void_p), P(C.c_int32), P(C.c_void_p), P(C.c_int32), C.c_int32,
                                       C.c_void_p]
    lib.davidson_solve_batched.argtypes = [C.c_void_p, C.c_int32, P(C.c_void_p), P(C.c_int32), P(C.c_void_p),
                                           P(C.c_int32), P(C.c_void_p), P(C.c_void_p), P(DavOpts), P(DavStats),
                                           P(C.c_int), C.c_int32, C.c_void_p]
    lib.pw_server_opts_default.argtypes = [P(ServerOpts)]
    lib.pw_server_opts_default.restype = None
    lib.pw_server_create.argtypes = [C.c_void_p, P(ServerOpts), P(C.c_void_p)]
    lib.pw_server_submit.argtypes = [C.c_void_p, P(Problem), C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                                     C.c_void_p, P(DavOpts), P(C.c_int64)]
    lib.pw_server_wait.argtypes = [C.c_void_p, C.c_int64, P(DavStats), P(C.c_double)]
    lib.pw_server_poll.argtypes = [C.c_void_p, C.c_int64, P(C.c_int32)]
    lib.pw_server_info.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
    lib.pw_server_clock.argtypes = [C.c_void_p]
    lib.pw_server_clock.restype = C.c_double
    lib.pw_server_destroy.argtypes = [C.c_void_p]
    lib.pw_reduced_eigh.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                    C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
    lib.pw_reduced_eigh_noalloc.argtypes = lib.pw_reduced_eigh.argtypes
    lib.pw_cg_opts_default.argtypes = [P(CgOpts)]
    lib.pw_cg_opts_default.restype = None
    lib.pcg_solve.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, P(CgOpts),
                              P(CgStats), C.c_void_p]
    lib.pw_density.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_double, C.c_int32,
                               C.c_void_p, C.c_void_p]
    lib.pw_scf_norm.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.c_double,
                                C.POINTER(C.c_double), C.c_void_p]
    lib.pw_profile_enable.argtypes = [C.c_int]
    lib.pw_profile_only.argtypes = [C.c_int32]
    lib.pw_profile_count.restype = C.c_int32
    lib.pw_profile_name.argtypes = [C.c_int32]
    lib.pw_profile_name.restype = C.c_char_p
    lib.pw_profile_read.argtypes = [C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    for name in ("pw_ctx_create", "pw_ctx_destroy", "pw_plan_create", "pw_plan_destroy",
                 "pw_plan_info", "pw_plan_set_potential", "hpsi_apply", "spsi_apply", "davidson_solve",
                 "pw_cancel",
                 "pw_hpsi_graph_create", "pw_graph_launch", "pw_graph_destroy", "pw_server_cancel", "hpsi_apply_batched", "davidson_solve_batched",
                 "pw_reduced_eigh", "pw_reduced_eigh_noalloc", "pw_density", "pw_scf_norm", "pcg_solve",
                 "pw_profile_enable", "pw_profile_only", "pw_profile_read", "pw_server_create",
                 "pw_server_submit", "pw_server_wait", "pw_server_poll", "pw_server_destroy",
                 "pw_server_info"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(st):
    if st != PW_OK:
        raise PwError(st, load().pw_last_error().decode())
    return st


def default_opts(**kw) -> DavOpts:
    o = DavOpts()
    load().pw_david_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Context:
    def __init__(self, device: int = 0):
        self.lib = load()
        self.h = C.c_void_p()
        self._children = weakref.WeakSet()
        _check(self.lib.pw_ctx_create(device, C.byref(self.h)))
        self.device = device

    def _adopt(self, obj):
        """Track a plan or server of this context: they are closed before it."""
        self._children.add(obj)

    def close(self):
        if self.h:
            # plans and servers hold the context; close them first (a garbage
            # cycle may finalize the context before them)
            for obj in list(self._children):
                obj.close()
            self.lib.pw_ctx_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _problem_struct(p, dev):
    """Marshal a generated problem into the C struct; returns (struct, keepalive)."""
    import torch
    miller = np.ascontiguousarray(p.miller, dtype=np.int32)
    kpg = np.ascontiguousarray(p.kpg, dtype=np.float64)
    vr = torch.from_numpy(np.ascontiguousarray(p.vloc_r, dtype=np.float64)).to(dev)
    beta = torch.from_numpy(np.ascontiguousarray(p.beta, dtype=np.complex128)).to(dev)
    blk = np.ascontiguousarray(p.blk_off, dtype=np.int32)
    dmat = np.ascontiguousarray(p.dmat, dtype=np.complex128)
    s = Problem()
    s.npw = miller.shape[0]
    s.miller = miller.ctypes.data
    s.kpg = kpg.ctypes.data
    s.nr[0], s.nr[1], s.nr[2] = (int(x) for x in p.nr)
    s.vloc_r = vr.data_ptr()
    s.nbeta = beta.shape[0]
    s.beta = beta.data_ptr() if beta.shape[0] else None
    s.ld_beta = s.npw
    s.nblk = len(blk) - 1
    s.blk_off = blk.ctypes.data
    s.dmat = dmat.ctypes.data if dmat.size else None
    qm = getattr(p, "qmat", None)
    qmat = np.ascontiguousarray(qm, dtype=np.complex128) if qm is not None else None
    s.qmat = qmat.ctypes.data if (qmat is not None and qmat.size) else None
    return s, (miller, kpg, vr, beta, blk, dmat, qmat)


def footprint_bytes(p, precision=PW_FP64, nb_max=None, ndim_max=4, device=0, plane_mode=0,
                    fft_ws_bytes=0) -> int:
    import torch
    s, keep = _problem_struct(p, torch.device("cuda", device))
    o = PlanOpts(precision, nb_max or p.nb, ndim_max, plane_mode, fft_ws_bytes)
    return int(load().pw_footprint_bytes(C.byref(s), C.byref(o)))


def profile_enable(on=True):
    _check(load().pw_profile_enable(1 if on else 0))


def profile_only(name):
    """Reset and time only the kernel class `name` (None: every class)."""
    lib = load()
    k = -1
    if name is not None:
        names = [lib.pw_profile_name(i).decode() for i in range(lib.pw_profile_count())]
        k = names.index(name)
    _check(lib.pw_profile_only(k))


def profile_read():
    """{kernel class: (launches, total ms, algorithmic units)} since profile_enable()."""
    lib = load()
    out = {}
    for k in range(lib.pw_profile_count()):
        n, ms, u = C.c_int64(), C.c_double(), C.c_double()
        _check(lib.pw_profile_read(k, C.byref(n), C.byref(ms), C.byref(u)))
        out[lib.pw_profile_name(k).decode()] = (int(n.value), float(ms.value), float(u.value))
    return out


def _ptrs(tensors):
    return (C.c_void_p * len(tensors))(*[C.c_void_p(t.data_ptr()) for t in tensors])


def _ints(vals):
    return (C.c_int32 * len(vals))(*[int(v) for v in vals])


def hpsi_batched(ctx, plans, psis, outs, prec=PW_FP64, nstreams=0, stream=None):
    """outs[i] = H_i psis[i] for every plan (asynchronous, worker streams of ctx)."""
    n = len(plans)
    assert len(psis) == n and len(outs) == n
    hs = (C.c_void_p * n)(*[p.h.value for p in plans])
    _check(ctx.lib.hpsi_apply_batched(ctx.h, n, hs, prec, _ints([x.shape[0] for x in psis]), _ptrs(psis),
                                      _ints([x.stride(0) for x in psis]), _ptrs(outs),
                                      _ints([y.stride(0) for y in outs]), nstreams, _stream_ptr(stream)))


def davidson_batched(ctx, plans, psis, opts=None, nworkers=0, stream=None):
    """Davidson on every (plan, psi) pair; returns (status, per-item status, eig list, resid list, stats list)."""
    import torch
    n = len(plans)
    eigs = [torch.empty(x.shape[0], dtype=torch.float64, device=x.device) for x in psis]
    res = [torch.empty(x.shape[0], dtype=torch.float64, device=x.device) for x in psis]
    stats = (DavStats * n)()
    status = (C.c_int * n)()
    opts = opts or default_opts()
    hs = (C.c_void_p * n)(*[p.h.value for p in plans])
    st = ctx.lib.davidson_solve_batched(ctx.h, n, hs, _ints([x.shape[0] for x in psis]), _ptrs(psis),
                                        _ints([x.stride(0) for x in psis]), _ptrs(eigs), _ptrs(res),
                                        C.byref(opts), stats, status, nworkers, _stream_ptr(stream))
    if st not in (PW_OK, PW_ENOTCONV):
        _check(st)
    return st, list(status), eigs, res, [stats[i] for i in range(n)]


def reduced_eigh(ctx, h, s, nev, debug=False, stream=None, noalloc=False):
    """Lowest nev eigenpairs of h c = w s c (torch complex128 n x n on the device).

    The matrices are read column-major: pass the transpose-free torch tensors
    of the matrices as [col][row] (i.e. ``m.T.contiguous()`` of a row-major
    NumPy-style matrix).  Returns (w, C[nev][n], tridiag or None).
    """
    import torch
    n = h.shape[0]
    w = torch.empty(nev, dtype=torch.float64, device=h.device)
    c = torch.empty((nev, n), dtype=torch.complex128, device=h.device)
    dbg = torch.empty(2 * n, dtype=torch.float64, device=h.device) if debug else None
    fn = load().pw_reduced_eigh_noalloc if noalloc else load().pw_reduced_eigh
    _check(fn(ctx.h, n, nev, C.c_void_p(h.data_ptr()), C.c_void_p(s.data_ptr()), n,
                                  C.c_void_p(w.data_ptr()), C.c_void_p(c.data_ptr()), n,
                                  C.c_void_p(dbg.data_ptr()) if debug else None, _stream_ptr(stream)))
    return w, c, dbg


class Plan:
    """A problem's maps, operator copies and workspace on one device."""

    def __init__(self, ctx: Context, p, precision=PW_FP64, nb_max=None, ndim_max=4, plane_mode=0,
                 fft_ws_bytes=0, nl_overlap=0, density=0, gamma=0):
        import torch
        self.ctx = ctx
        self.lib = ctx.lib
        self.dev = torch.device("cuda", ctx.device)
        s, keep = _problem_struct(p, self.dev)
        self.opts = PlanOpts(precision, int(nb_max or p.nb), int(ndim_max), int(plane_mode), int(fft_ws_bytes),
                             int(nl_overlap), int(density), int(gamma))
        self.h = C.c_void_p()
        _check(self.lib.pw_plan_create(ctx.h, C.byref(s), C.byref(self.opts), C.byref(self.h)))
        ctx._adopt(self)
        del keep
        self.npw = int(s.npw)
        self.nr = tuple(int(x) for x in p.nr)
        self.precision = precision

    def info(self):
        out = (C.c_int64 * 8)()
        _check(self.lib.pw_plan_info(self.h, out))
        keys = ["npw", "nsticks", "ncols", "N", "nbeta", "band_chunk", "plane64", "plane32"]
        d = dict(zip(keys, list(out)))
        # plane pass form: 0 register kernel, 1 three kernels, 2 lane-group kernel, 3 generic LDS kernel
        d["split_plane64"] = int(d["plane64"] == 1)
        d["split_plane32"] = int(d["plane32"] == 1)
        return d

    def set_potential(self, vloc_r, stream=None):
        """Replace V_loc(r) (float64 [n3][n2][n1] on the device) for the next H.psi and solves."""
        assert vloc_r.dtype.is_floating_point and vloc_r.element_size() == 8 and vloc_r.is_contiguous()
        assert vloc_r.numel() == self.nr[0] * self.nr[1] * self.nr[2]
        _check(self.lib.pw_plan_set_potential(self.h, C.c_void_p(vloc_r.data_ptr()), _stream_ptr(stream)))

    def hpsi(self, psi, out=None, prec=PW_FP64, stream=None):
        """out = H psi for psi [nb][>=npw] complex128 on the device."""
        import torch
        assert psi.dtype == torch.complex128 and psi.is_cuda and psi.dim() == 2
        assert psi.stride(1) == 1
        if out is None:
            out = torch.empty_like(psi)
        _check(self.lib.hpsi_apply(self.h, prec, psi.shape[0], C.c_void_p(psi.data_ptr()), psi.stride(0),
                                   C.c_void_p(out.data_ptr()), out.stride(0), _stream_ptr(stream)))
        return out

    def spsi(self, psi, out=None, prec=PW_FP64, stream=None):
        """out = S psi (the ultrasoft overlap; psi itself for norm-conserving problems)."""
        import torch
        assert psi.dtype == torch.complex128 and psi.is_cuda and psi.dim() == 2 and psi.stride(1) == 1
        if out is None:
            out = torch.empty_like(psi)
        _check(self.lib.spsi_apply(self.h, prec, psi.shape[0], C.c_void_p(psi.data_ptr()), psi.stride(0),
                                   C.c_void_p(out.data_ptr()), out.stride(0), _stream_ptr(stream)))
        return out

    def hpsi_graph(self, psi, out, prec=PW_FP64):
        """A captured hpsi_apply for these buffers (pw_hpsi_graph_create): its
        replay() relaunches out = H psi on the current torch stream.  psi and
        out must stay allocated, in place, while the graph is used; their
        contents may change between replays."""
        assert psi.shape == out.shape and psi.stride(1) == 1 and out.stride(1) == 1
        h = C.c_void_p()
        _check(self.lib.pw_hpsi_graph_create(self.h, prec, psi.shape[0], C.c_void_p(psi.data_ptr()), psi.stride(0),
                                             C.c_void_p(out.data_ptr()), out.stride(0), C.byref(h)))
        return HpsiGraph(self, h, (psi, out))

    def cancel(self):
        """Stop the solve running on this plan (from another thread): it returns PW_ECANCELLED."""
        _check(self.lib.pw_cancel(self.h))

    def davidson(self, psi, eig=None, resid=None, opts=None, stream=None, history=None):
        """In-place block Davidson on psi [nb][>=npw]; returns (status, eig, resid, stats).

        history: optional float64 numpy array of >= 2*max_iter entries that
        receives (max residual norm, Ritz rotation growth) per iteration."""
        import torch
        nb = psi.shape[0]
        if eig is None:
            eig = torch.empty(nb, dtype=torch.float64, device=psi.device)
        if resid is None:
            resid = torch.empty(nb, dtype=torch.float64, device=psi.device)
        opts = opts or default_opts()
        if history is not None:
            assert history.dtype == np.float64 and history.flags.c_contiguous
            assert history.size >= 2 * opts.max_iter
            opts.history = history.ctypes.data_as(C.POINTER(C.c_double))
        stats = DavStats()
        st = self.lib.davidson_solve(self.h, nb, C.c_void_p(psi.data_ptr()), psi.stride(0),
                                     C.c_void_p(eig.data_ptr()), C.c_void_p(resid.data_ptr()),
                                     C.byref(opts), C.byref(stats), _stream_ptr(stream))
        if st not in (PW_OK, PW_ENOTCONV):
            _check(st)
        return st, eig, resid, stats

    def pcg(self, psi, eig=None, resid=None, opts=None, stream=None, **kw):
        """In-place band-by-band conjugate gradient on psi [nb][>=npw]; returns (status, eig, resid, stats)."""
        import torch
        nb = psi.shape[0]
        if eig is None:
            eig = torch.empty(nb, dtype=torch.float64, device=psi.device)
        if resid is None:
            resid = torch.empty(nb, dtype=torch.float64, device=psi.device)
        if opts is None:
            opts = CgOpts()
            self.lib.pw_cg_opts_default(C.byref(opts))
            for k, v in kw.items():
                setattr(opts, k, v)
        stats = CgStats()
        st = self.lib.pcg_solve(self.h, nb, C.c_void_p(psi.data_ptr()), psi.stride(0), C.c_void_p(eig.data_ptr()),
                                C.c_void_p(resid.data_ptr()), C.byref(opts), C.byref(stats), _stream_ptr(stream))
        if st not in (PW_OK, PW_ENOTCONV):
            _check(st)
        return st, eig, resid, stats

    def density(self, psi, w, omega, rho=None, accumulate=False, stream=None):
        """rho (+)= (1/omega) sum_b w_b |psi_b(r)|^2 on the plan's grid; returns rho
        (torch float64 [n3][n2][n1]).  Needs a plan created with density=1."""
        import torch
        assert psi.dtype == torch.complex128 and psi.stride(1) == 1
        w = torch.as_tensor(w, dtype=torch.float64, device=psi.device).contiguous()
        if rho is None:
            rho = torch.empty((self.nr[2], self.nr[1], self.nr[0]), dtype=torch.float64, device=psi.device)
        _check(self.lib.pw_density(self.h, psi.shape[0], C.c_void_p(psi.data_ptr()), psi.stride(0),
                                   C.c_void_p(w.data_ptr()), float(omega), 1 if accumulate else 0,
                                   C.c_void_p(rho.data_ptr()), _stream_ptr(stream)))
        return rho

    def scf_norm2(self, rho_out, rho_in, bvec, omega, stream=None):
        """4 pi omega sum_{G != 0} |drho(G)|^2 / |G|^2 of drho = rho_out - rho_in (device grids);
        bvec: 3x3 reciprocal vectors (rows, bohr^-1)."""
        bv = (C.c_double * 9)(*[float(x) for x in np.asarray(bvec, dtype=np.float64).ravel()])
        out = C.c_double()
        _check(self.lib.pw_scf_norm(self.h, C.c_void_p(rho_out.data_ptr()), C.c_void_p(rho_in.data_ptr()), bv,
                                    float(omega), C.byref(out), _stream_ptr(stream)))
        return float(out.value)

    def close(self):
        if self.h:
            self.lib.pw_plan_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HpsiGraph:
    """hpsi_apply captured in a HIP graph (see Plan.hpsi_graph)."""

    def __init__(self, plan, h, keep):
        self.plan, self.lib, self.h, self._keep = plan, plan.lib, h, keep

    def replay(self, stream=None):
        _check(self.lib.pw_graph_launch(self.h, _stream_ptr(stream)))

    def close(self):
        if self.h:
            self.lib.pw_graph_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop of the library (see pw_server_* in include/pwdft.h)."""

    def __init__(self, ctx: Context, nworkers=4, mem_budget=0, precision=PW_MIXED, gamma=0):
        self.ctx, self.lib = ctx, ctx.lib
        o = ServerOpts()
        self.lib.pw_server_opts_default(C.byref(o))
        o.nworkers, o.mem_budget, o.precision = int(nworkers), int(mem_budget), int(precision)
        o.gamma = int(gamma)
        self.h = C.c_void_p()
        self._keep = {}
        _check(self.lib.pw_server_create(ctx.h, C.byref(o), C.byref(self.h)))
        ctx._adopt(self)

    def clock(self) -> float:
        return float(self.lib.pw_server_clock(self.h))

    def info(self):
        """Requests served, pool bytes, peak pool use, allocations outside the pool."""
        out = (C.c_int64 * 4)()
        _check(self.lib.pw_server_info(self.h, out))
        return dict(zip(["served", "pool_bytes", "pool_peak", "pool_fallbacks"], list(out)))

    def submit(self, p, psi, opts=None):
        """Enqueue problem p with trial block psi (torch [nb][npw] on the device, solved in place);
        returns (ticket, eig, resid)."""
        import torch
        s, keep = _problem_struct(p, psi.device)
        eig = torch.empty(psi.shape[0], dtype=torch.float64, device=psi.device)
        res = torch.empty_like(eig)
        opts = opts or default_opts()
        # the worker reads psi, V and beta on its own stream: their uploads
        # (on torch's stream) must be complete before the request is submitted
        torch.cuda.current_stream(psi.device).synchronize()
        t = C.c_int64()
        _check(self.lib.pw_server_submit(self.h, C.byref(s), psi.shape[0], C.c_void_p(psi.data_ptr()),
                                         psi.stride(0), C.c_void_p(eig.data_ptr()), C.c_void_p(res.data_ptr()),
                                         C.byref(opts), C.byref(t)))
        self._keep[t.value] = (s, keep, psi, eig, res, opts)
        return t.value, eig, res

    def wait(self, ticket):
        """Block until done; returns (status, stats dict, (t_submit, t_start, t_end))."""
        st = DavStats()
        times = (C.c_double * 3)()
        rc = self.lib.pw_server_wait(self.h, ticket, C.byref(st), times)
        self._keep.pop(ticket, None)
        if rc not in (PW_OK, PW_ENOTCONV):
            _check(rc)
        return rc, st.asdict(), (times[0], times[1], times[2])

    def cancel(self, ticket):
        _check(self.lib.pw_server_cancel(self.h, ticket))

    def close(self):
        if self.h:
            self.lib.pw_server_destroy(self.h)
            self.h = C.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
