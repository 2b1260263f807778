"""Thin ctypes binding of libdisco (include/disco.h).

Argument marshalling only: every step runs in the HIP library.  Device
buffers are torch tensors on the GPU (complex128 unless stated); the context
issues its work on torch's current stream.  The binding raises when the
library has not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdisco.so")

OK, EINVAL, ENOMEM, EHIP, ENOCONV, EBREAKDOWN, ESTATE = 0, -1, -2, -3, -4, -5, -6
F64, F32, BF16 = 0, 1, 2
HOST, DEVICE = 0, 1
G_1, G_5, G_X, G_Y, G_Z = 0, 1, 2, 3, 4
G_TILDE = 8  # added to a loop code: the loop of gamma_4 Gamma^+ gamma_4
EPI_DOTAUX, EPI_NORM, EPI_DOTIN, EPI_DOTAUXIN = 2, 4, 8, 16
CGNR_F64, BICGSTAB_DC, FGMRES_NN, BICGSTAB_RU = 0, 1, 2, 3
K_STENCIL = 0
K_NN = 2
K_STENCIL_F64, K_STENCIL_F32, K_STENCIL_BF16 = 10, 11, 12
K_MFMA = 1
OPT_GRAPHS, OPT_STAGE, OPT_EO, OPT_TILE_Y, OPT_TILE_T, OPT_NARROW = 1, 2, 3, 4, 5, 6
K_STENCIL_EO_F64, K_STENCIL_EO_F32, K_STENCIL_EO_BF16 = 13, 14, 15


class DiscoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libdisco error %d: %s" % (code, msg))
        self.code = code


class SolverParams(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("inner_prec", ctypes.c_int), ("inner_tol", ctypes.c_double), ("rhs_block", ctypes.c_int),
                ("fallback", ctypes.c_int), ("check_every", ctypes.c_int), ("restart", ctypes.c_int),
                ("net", ctypes.c_void_p)]


class SolverStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_iters", ctypes.c_int), ("fallback_used", ctypes.c_int),
                ("converged", ctypes.c_int), ("true_rel_residual", ctypes.c_double)]


class TrainParams(ctypes.Structure):
    _fields_ = [("npairs", ctypes.c_int), ("nsnap", ctypes.c_int), ("snap_iters", ctypes.c_int * 8),
                ("batch", ctypes.c_int), ("steps", ctypes.c_int), ("lr", ctypes.c_double),
                ("seed", ctypes.c_ulonglong)]


class TrainStats(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_int), ("steps", ctypes.c_int), ("first_loss", ctypes.c_double),
                ("final_loss", ctypes.c_double), ("gen_seconds", ctypes.c_double), ("train_seconds", ctypes.c_double)]


_lib = None

P, I, D, LL = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
_SIGS = {
    "disco_create": ([P, P, I, P], I),
    "disco_destroy": ([P], I),
    "disco_set_stream": ([P, P], I),
    "disco_last_error": ([P], ctypes.c_char_p),
    "disco_gauge_set": ([P, P, I], I),
    "disco_clover_setup": ([P, D, D], I),
    "disco_clover_get": ([P, P], I),
    "disco_domains_create": ([P, P, I, P], I),
    "disco_domains_destroy": ([P], I),
    "disco_dirac_apply": ([P, I, I, I, P, P], I),
    "disco_dirac_block_apply": ([P, P, I, I, I, P, P], I),
    "disco_dirac_apply_noalloc": ([P, I, I, I, P, P], I),
    "disco_native_bytes": ([P, I, I], LL),
    "disco_to_native": ([P, I, I, P, P], I),
    "disco_from_native": ([P, I, I, P, P], I),
    "disco_dirac_apply_native": ([P, P, I, I, I, P, P], I),
    "disco_dirac_eo_apply": ([P, P, I, I, I, D, D, D, I, P, P, P, P, P], I),
    "disco_solve_multi_rhs": ([P, P, ctypes.POINTER(SolverParams), I, P, P, ctypes.POINTER(SolverStats)], I),
    "disco_profile_enable": ([P, I], I),
    "disco_profile_reset": ([P], I),
    "disco_profile_get": ([P, I, ctypes.POINTER(LL), ctypes.POINTER(D), ctypes.POINTER(D)], I),
}
_SIGS.update({
    "disco_ape_smear": ([P, I, D], I),
    "disco_smeared_get": ([P, P], I),
    "disco_laplace_apply": ([P, I, P, P], I),
    "disco_laplace_eigvecs": ([P, I, D, P, P], I),
    "disco_laplace_eigvecs_slices": ([P, I, D, P, I, P, P], I),
    "disco_perambulator": ([P, P, I, I, P, P, I, P], I),
    "disco_loops": ([P, P, I, I, P, P, I, P], I),
    "disco_loops_distill": ([P, P, P, I, P, P, I, ctypes.POINTER(SolverParams), P, P, ctypes.POINTER(SolverStats)], I),
    "disco_last_solves": ([P], LL),
    "disco_perambulators_tt": ([P, P, P, I, ctypes.c_ulonglong, ctypes.POINTER(SolverParams), P,
                                ctypes.POINTER(SolverStats)], I),
    "disco_profile_stride": ([P, I], I),
    "disco_set_option": ([P, I, I], I),
    "disco_get_option": ([P, I, ctypes.POINTER(I)], I),
    "disco_autotune": ([P, P, I, ctypes.POINTER(I), P], I),
    "disco_correlator": ([P, P, P, P, P, I, I, P, I, I, P, P, P, P], I),
    "disco_slab_sets": ([I, I, ctypes.POINTER(I), P], I),
    "disco_loops_slab": ([P, P, I, P, P, I, I, ctypes.POINTER(SolverParams), P, P, ctypes.POINTER(SolverStats)], I),
    "disco_slab_sets_open": ([I, I, ctypes.POINTER(I), P], I),
    "disco_loops_slab_open": ([P, P, I, P, P, I, I, ctypes.POINTER(SolverParams), P, P, ctypes.POINTER(SolverStats)],
                              I),
    "disco_nr_splice": ([P, P, P, I, I, P], I),
    "disco_profile_weights": ([P, ctypes.c_long, D, P], I),
    "disco_perambulators_all": ([P, P, I, ctypes.c_ulonglong, ctypes.POINTER(SolverParams), P,
                                 ctypes.POINTER(SolverStats)], I),
    "disco_connected": ([P, P, I, I, P, P, I, P, I, P], I),
    "disco_effective_mass": ([P, I, P], I),
    "disco_net_create": ([P, I, ctypes.c_ulonglong, P], I),
    "disco_net_destroy": ([P], I),
    "disco_net_refresh": ([P], I),
    "disco_net_weights_count": ([P], LL),
    "disco_net_set_weights": ([P, P, I], I),
    "disco_net_get_weights": ([P, P, I], I),
    "disco_net_apply": ([P, I, P, P], I),
    "disco_net_backward": ([P, I, P, P, P, P], I),
    "disco_net_train": ([P, ctypes.POINTER(TrainParams), ctypes.POINTER(TrainStats)], I),
})
_OPTIONAL = {}


def lib():
    """Load libdisco.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libdisco.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        h = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in list(_SIGS.items()) + list(_OPTIONAL.items()):
            fn = getattr(h, name, None)
            if fn is None:
                if name in _SIGS:
                    raise ImportError("libdisco.so lacks %s" % name)
                continue
            fn.argtypes = args
            fn.restype = res
        _lib = h
    return _lib


def exported_symbols():
    return list(_SIGS) + list(_OPTIONAL)


def _torch():
    import torch
    return torch


def _dptr(t):
    if t is None:
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a GPU torch tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Domains:
    def __init__(self, ctx: "Context", cut):
        cut = np.ascontiguousarray(np.asarray(cut, dtype=np.uint8))
        self.ctx = ctx
        self.cut = cut
        h = ctypes.c_void_p()
        ctx._chk(lib().disco_domains_create(ctx.h, cut.ctypes.data_as(P), cut.shape[1], ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            lib().disco_domains_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Net:
    """The gauge-covariant network (learned preconditioner) on a context's gauge field."""

    def __init__(self, ctx: "Context", channels: int = 16, seed: int = 1):
        self.ctx = ctx
        h = ctypes.c_void_p()
        ctx._chk(lib().disco_net_create(ctx.h, int(channels), ctypes.c_ulonglong(seed), ctypes.byref(h)))
        self.h = h
        self.nw = int(lib().disco_net_weights_count(h))

    def close(self):
        if getattr(self, "h", None):
            lib().disco_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def refresh(self):
        """Re-tabulate the transporters after the context's gauge field changed."""
        self.ctx._chk(lib().disco_net_refresh(self.h))

    def get_weights(self) -> np.ndarray:
        w = np.empty(self.nw, dtype=np.float32)
        self.ctx._chk(lib().disco_net_get_weights(self.h, w.ctypes.data_as(P), HOST))
        return w

    def set_weights(self, w):
        w = np.ascontiguousarray(np.asarray(w, dtype=np.float32))
        if w.size != self.nw:
            raise ValueError("expected %d weights" % self.nw)
        self.ctx._chk(lib().disco_net_set_weights(self.h, w.ctypes.data_as(P), HOST))

    def apply(self, x):
        out = _torch().empty_like(x)
        self.ctx._chk(lib().disco_net_apply(self.h, x.shape[0], _dptr(x), _dptr(out)))
        return out

    def backward(self, x, grad_out, want_grad_in=True):
        torch = _torch()
        gw = torch.empty(self.nw, dtype=torch.float32, device=x.device)
        gi = torch.empty_like(x) if want_grad_in else None
        self.ctx._chk(lib().disco_net_backward(self.h, x.shape[0], _dptr(x), _dptr(grad_out), _dptr(gw), _dptr(gi)))
        return gw, gi

    def train(self, npairs, snap_iters=(0, 8, 32, 96), batch=4, steps=100, lr=1e-3, seed=1):
        tp = TrainParams()
        tp.npairs = int(npairs)
        tp.nsnap = len(snap_iters)
        for k, v in enumerate(snap_iters):
            tp.snap_iters[k] = int(v)
        tp.batch = int(batch)
        tp.steps = int(steps)
        tp.lr = float(lr)
        tp.seed = int(seed)
        ts = TrainStats()
        self.ctx._chk(lib().disco_net_train(self.h, ctypes.byref(tp), ctypes.byref(ts)))
        return ts


class Context:
    """A libdisco context for one lattice on one GPU."""

    def __init__(self, dims, bc=(1, 1, 1, -1), device: int = 0):
        torch = _torch()
        self.dims = tuple(int(d) for d in dims)
        self.bc = tuple(int(b) for b in bc)
        self.V = int(np.prod(self.dims))
        self.Vs = self.V // self.dims[3]
        self.device = device
        d = (ctypes.c_int * 4)(*self.dims)
        b = (ctypes.c_int * 4)(*self.bc)
        h = ctypes.c_void_p()
        rc = lib().disco_create(d, b, device, ctypes.byref(h))
        if rc != OK:
            raise DiscoError(rc, "disco_create failed")
        self.h = h
        self.sync_stream()

    # -- plumbing
    def _chk(self, rc):
        if rc != OK:
            raise DiscoError(rc, lib().disco_last_error(self.h).decode())
        return rc

    def sync_stream(self):
        torch = _torch()
        s = torch.cuda.current_stream(self.device).cuda_stream
        self._chk(lib().disco_set_stream(self.h, ctypes.c_void_p(s)))

    def close(self):
        if getattr(self, "h", None):
            lib().disco_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dev(self, a, dtype=None):
        """numpy -> GPU torch tensor (complex128 by default)."""
        torch = _torch()
        t = torch.from_numpy(np.ascontiguousarray(a))
        if dtype is not None:
            t = t.to(dtype)
        return t.to("cuda:%d" % self.device)

    def empty_spinors(self, n):
        torch = _torch()
        return torch.empty((n, self.V, 4, 3), dtype=torch.complex128, device="cuda:%d" % self.device)

    # -- setup
    def gauge_set(self, U):
        U = np.ascontiguousarray(U, dtype=np.complex128)
        self._chk(lib().disco_gauge_set(self.h, U.ctypes.data_as(P), HOST))

    def gauge_set_device(self, U_t):
        self._chk(lib().disco_gauge_set(self.h, _dptr(U_t), DEVICE))

    def clover_setup(self, kappa, csw):
        self._chk(lib().disco_clover_setup(self.h, float(kappa), float(csw)))

    def clover_get(self):
        torch = _torch()
        A = torch.empty((self.V, 12, 12), dtype=torch.complex128, device="cuda:%d" % self.device)
        self._chk(lib().disco_clover_get(self.h, _dptr(A)))
        return A

    def domains(self, cut) -> Domains:
        return Domains(self, cut)

    # -- operators
    def dirac_apply(self, psi, prec=F64, dagger=False, out=None):
        n = psi.shape[0]
        out = self.empty_spinors(n) if out is None else out
        self._chk(lib().disco_dirac_apply(self.h, prec, int(dagger), n, _dptr(psi), _dptr(out)))
        return out

    def dirac_apply_noalloc(self, psi, prec=F64, dagger=False, out=None):
        """As dirac_apply, through the entry point that allocates no device memory."""
        n = psi.shape[0]
        out = self.empty_spinors(n) if out is None else out
        self._chk(lib().disco_dirac_apply_noalloc(self.h, prec, int(dagger), n, _dptr(psi), _dptr(out)))
        return out

    def dirac_block_apply(self, dom: Domains, psi, prec=F64, dagger=False, out=None):
        n = psi.shape[0]
        out = self.empty_spinors(n) if out is None else out
        self._chk(lib().disco_dirac_block_apply(self.h, dom.h, prec, int(dagger), n, _dptr(psi), _dptr(out)))
        return out

    def native_bytes(self, prec, n):
        return int(lib().disco_native_bytes(self.h, prec, n))

    def to_native(self, prec, psi):
        torch = _torch()
        n = psi.shape[0]
        out = torch.empty(self.native_bytes(prec, n), dtype=torch.uint8, device=psi.device)
        self._chk(lib().disco_to_native(self.h, prec, n, _dptr(psi), _dptr(out)))
        return out

    def from_native(self, prec, nat, n):
        out = self.empty_spinors(n)
        self._chk(lib().disco_from_native(self.h, prec, n, _dptr(nat), _dptr(out)))
        return out

    def dirac_apply_native(self, dom, prec, nat_in, nat_out, n, dagger=False):
        self._chk(lib().disco_dirac_apply_native(self.h, None if dom is None else dom.h, prec, int(dagger), n,
                                                 _dptr(nat_in), _dptr(nat_out)))

    def dirac_eo_apply(self, psi, parity, ca, cg, cb, prec=F64, dom: Domains | None = None, aux=None, aux2=None,
                       epi=0):
        """The even-odd piece out = ca aux + A^-1 (cg aux + cb H psi) at the sites of
        `parity` (zero elsewhere), as the solver launches it; returns (out, sums)
        with sums [n][4] complex (None when epi = 0)."""
        n = psi.shape[0]
        out = self.empty_spinors(n)
        sums = np.zeros((n, 4), dtype=np.complex128) if epi else None
        self._chk(lib().disco_dirac_eo_apply(self.h, None if dom is None else dom.h, prec, int(parity), n,
                                             float(ca), float(cg), float(cb), int(epi), _dptr(psi), _dptr(aux),
                                             _dptr(aux2), _dptr(out),
                                             None if sums is None else sums.ctypes.data_as(P)))
        return out, sums

    # -- solver
    @staticmethod
    def params(method=BICGSTAB_DC, tol=1e-10, max_iter=0, inner_prec=F32, inner_tol=0.0, rhs_block=0,
               fallback=1, check_every=0, restart=0, net=None) -> SolverParams:
        p = SolverParams(method, tol, max_iter, inner_prec, inner_tol, rhs_block, fallback, check_every, restart,
                         None if net is None else net.h.value)
        p._net = net  # keep the network alive while the parameters are in use
        return p

    def solve_multi_rhs(self, b, params: SolverParams, dom: Domains | None = None, x=None, allow_noconv=False):
        n = b.shape[0]
        x = self.empty_spinors(n) if x is None else x
        stats = (SolverStats * max(1, n))()
        rc = lib().disco_solve_multi_rhs(self.h, None if dom is None else dom.h, ctypes.byref(params), n,
                                         _dptr(b), _dptr(x), stats)
        if rc == ENOCONV and allow_noconv:
            pass
        else:
            self._chk(rc)
        return x, [stats[i] for i in range(n)]

    # -- distillation
    def ape_smear(self, steps, alpha):
        self._chk(lib().disco_ape_smear(self.h, int(steps), float(alpha)))

    def smeared_get(self):
        torch = _torch()
        out = torch.empty((self.V, 4, 3, 3), dtype=torch.complex128, device="cuda:%d" % self.device)
        self._chk(lib().disco_smeared_get(self.h, _dptr(out)))
        return out

    def laplace_apply(self, y):
        torch = _torch()
        out = torch.empty_like(y)
        self._chk(lib().disco_laplace_apply(self.h, y.shape[0], _dptr(y), _dptr(out)))
        return out

    def laplace_eigvecs(self, nv, tol=1e-12):
        torch = _torch()
        T = self.dims[3]
        Vev = torch.empty((T, nv, self.Vs, 3), dtype=torch.complex128, device="cuda:%d" % self.device)
        lam = np.empty((T, nv), dtype=np.float64)
        self._chk(lib().disco_laplace_eigvecs(self.h, int(nv), float(tol), _dptr(Vev), lam.ctypes.data_as(P)))
        return Vev, lam

    def laplace_eigvecs_slices(self, nv, tsel, tol=1e-12):
        """Eigenpairs on the timeslices tsel only: ([len(tsel)][nv][Vs][3], [len(tsel)][nv])."""
        torch = _torch()
        ts = np.ascontiguousarray(np.asarray(tsel, dtype=np.int32))
        Vev = torch.empty((len(ts), nv, self.Vs, 3), dtype=torch.complex128, device="cuda:%d" % self.device)
        lam = np.empty((len(ts), nv), dtype=np.float64)
        self._chk(lib().disco_laplace_eigvecs_slices(self.h, int(nv), float(tol), ts.ctypes.data_as(P), len(ts),
                                                     _dptr(Vev), lam.ctypes.data_as(P)))
        return Vev, lam

    def perambulator(self, Vev, X, t_snk):
        torch = _torch()
        nv = Vev.shape[1]
        t = np.ascontiguousarray(np.asarray(t_snk, dtype=np.int32))
        tau = torch.empty((len(t), nv, 4, X.shape[0]), dtype=torch.complex128, device=X.device)
        self._chk(lib().disco_perambulator(self.h, _dptr(Vev), nv, X.shape[0], _dptr(X), t.ctypes.data_as(P),
                                           len(t), _dptr(tau)))
        return tau

    def loops(self, tau_tt, gammas, w=None):
        torch = _torch()
        T, nv = tau_tt.shape[0], tau_tt.shape[1]
        g = np.ascontiguousarray(np.asarray(gammas, dtype=np.int32))
        L = torch.empty((len(g), T), dtype=torch.complex128, device=tau_tt.device)
        self._chk(lib().disco_loops(self.h, _dptr(tau_tt), T, nv, _dptr(w), g.ctypes.data_as(P), len(g), _dptr(L)))
        return L

    def loops_distill(self, Vev, gammas, params: SolverParams, dom: Domains | None = None, w=None, want_tau=False):
        torch = _torch()
        T, nv = Vev.shape[0], Vev.shape[1]
        g = np.ascontiguousarray(np.asarray(gammas, dtype=np.int32))
        L = torch.empty((len(g), T), dtype=torch.complex128, device=Vev.device)
        tau = torch.empty((T, nv, 4, nv, 4), dtype=torch.complex128, device=Vev.device) if want_tau else None
        agg = SolverStats()
        self._chk(lib().disco_loops_distill(self.h, None if dom is None else dom.h, _dptr(Vev), nv, _dptr(w),
                                            g.ctypes.data_as(P), len(g), ctypes.byref(params), _dptr(L), _dptr(tau),
                                            ctypes.byref(agg)))
        return L, tau, agg

    def slab_sets(self, delta, open_time=False):
        T = self.dims[3]
        n = I()
        m = (ctypes.c_ulonglong * T)()
        fn = lib().disco_slab_sets_open if open_time else lib().disco_slab_sets
        rc = fn(T, int(delta), ctypes.byref(n), ctypes.cast(m, P))
        if rc != OK:
            raise DiscoError(rc, "bad slab width %r" % (delta,))
        return [int(m[k]) for k in range(n.value)]

    def loops_slab(self, Vev, gammas, delta, params: SolverParams, w=None, want_tau=False, open_time=False):
        torch = _torch()
        T, nv = Vev.shape[0], Vev.shape[1]
        g = np.ascontiguousarray(np.asarray(gammas, dtype=np.int32))
        L = torch.empty((len(g), T), dtype=torch.complex128, device=Vev.device)
        tau = torch.empty((T, nv, 4, nv, 4), dtype=torch.complex128, device=Vev.device) if want_tau else None
        agg = SolverStats()
        fn = lib().disco_loops_slab_open if open_time else lib().disco_loops_slab
        self._chk(fn(self.h, _dptr(Vev), nv, _dptr(w), g.ctypes.data_as(P), len(g), int(delta),
                     ctypes.byref(params), _dptr(L), _dptr(tau), ctypes.byref(agg)))
        return L, tau, agg

    @staticmethod
    def nr_splice(Cc, dC, deltas):
        """C^NR spliced by separation from host arrays: Cc [T], dC [len(deltas)][T]."""
        Cc = np.ascontiguousarray(np.asarray(Cc, dtype=np.complex128))
        dC = np.ascontiguousarray(np.asarray(dC, dtype=np.complex128))
        dl = np.ascontiguousarray(np.asarray(deltas, dtype=np.int32))
        out = np.empty_like(Cc)
        rc = lib().disco_nr_splice(Cc.ctypes.data_as(P), dC.ctypes.data_as(P), dl.ctypes.data_as(P), len(dl),
                                   len(Cc), out.ctypes.data_as(P))
        if rc != OK:
            raise DiscoError(rc, "bad splice arguments")
        return out

    def perambulators_all(self, Vev, params: SolverParams, tmask=0):
        torch = _torch()
        T, nv = Vev.shape[0], Vev.shape[1]
        tau = torch.zeros((T, T, nv, 4, nv, 4), dtype=torch.complex128, device=Vev.device)
        agg = SolverStats()
        self._chk(lib().disco_perambulators_all(self.h, _dptr(Vev), nv, int(tmask), ctypes.byref(params), _dptr(tau),
                                                ctypes.byref(agg)))
        return tau, agg

    def connected(self, tau_all, gammas, w=None, y0s=None):
        torch = _torch()
        T, nv = tau_all.shape[0], tau_all.shape[2]
        g = np.ascontiguousarray(np.asarray(gammas, dtype=np.int32))
        y = None if y0s is None else np.ascontiguousarray(np.asarray(y0s, dtype=np.int32))
        C = torch.empty((len(g), T), dtype=torch.complex128, device=tau_all.device)
        self._chk(lib().disco_connected(self.h, _dptr(tau_all), T, nv, _dptr(w), g.ctypes.data_as(P), len(g),
                                        None if y is None else y.ctypes.data_as(P), 0 if y is None else len(y),
                                        _dptr(C)))
        return C

    @staticmethod
    def effective_mass(C):
        C = np.ascontiguousarray(np.asarray(C, dtype=np.float64))
        m = np.empty(len(C) - 1, dtype=np.float64)
        rc = lib().disco_effective_mass(C.ctypes.data_as(P), len(C), m.ctypes.data_as(P))
        if rc != OK:
            raise DiscoError(rc, "effective mass needs at least two values")
        return m

    @staticmethod
    def profile_weights(lam, omega):
        lam = np.ascontiguousarray(np.asarray(lam, dtype=np.float64))
        w = np.empty_like(lam)
        rc = lib().disco_profile_weights(lam.ctypes.data_as(P), lam.size, float(omega), w.ctypes.data_as(P))
        if rc != OK:
            raise DiscoError(rc, "bad profile width %r" % (omega,))
        return w

    def perambulators_tt(self, Vev, tmask, params: SolverParams, tau, dom: Domains | None = None):
        agg = SolverStats()
        self._chk(lib().disco_perambulators_tt(self.h, None if dom is None else dom.h, _dptr(Vev), Vev.shape[1],
                                               int(tmask), ctypes.byref(params), _dptr(tau), ctypes.byref(agg)))
        return agg

    def set_option(self, option, value):
        self._chk(lib().disco_set_option(self.h, int(option), int(value)))

    def get_option(self, option):
        v = I()
        self._chk(lib().disco_get_option(self.h, int(option), ctypes.byref(v)))
        return v.value

    def autotune(self, inner_prec=F32, dom: Domains | None = None):
        best = ctypes.c_int(0)
        cost = np.zeros(4, dtype=np.float64)
        self._chk(lib().disco_autotune(self.h, None if dom is None else dom.h, int(inner_prec), ctypes.byref(best),
                                       cost.ctypes.data_as(P)))
        return best.value, {k: c for k, c in zip((8, 16, 32, 64), cost) if c > 0}

    def last_solves(self):
        return int(lib().disco_last_solves(self.h))

    def correlator(self, L_full, Lt_full, L_blk, Lt_blk, y0s=None, vev_mode=1):
        torch = _torch()
        ncfg, T = L_full.shape
        y = None if y0s is None else np.ascontiguousarray(np.asarray(y0s, dtype=np.int32))
        mk = lambda *s: torch.empty(s, dtype=torch.complex128, device=L_full.device)
        C, Cf, dC, four = mk(T), mk(T), mk(T), mk(4, T)
        self._chk(lib().disco_correlator(self.h, _dptr(L_full), _dptr(Lt_full), _dptr(L_blk), _dptr(Lt_blk), ncfg, T,
                                         None if y is None else y.ctypes.data_as(P), 0 if y is None else len(y),
                                         int(vev_mode), _dptr(C), _dptr(Cf), _dptr(dC), _dptr(four)))
        return C, Cf, dC, four

    # -- profiling
    def profile_enable(self, on=True):
        self._chk(lib().disco_profile_enable(self.h, int(on)))

    def profile_stride(self, stride):
        self._chk(lib().disco_profile_stride(self.h, int(stride)))

    def profile_reset(self):
        self._chk(lib().disco_profile_reset(self.h))

    def profile_get(self, kernel=K_STENCIL):
        n = LL()
        ms = D()
        by = D()
        self._chk(lib().disco_profile_get(self.h, kernel, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
        return n.value, ms.value, by.value
