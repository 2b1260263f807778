"""Plain FP64 CPU reference ("the oracle") for the subtraction method's hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import this
package.  The GPU library never imports it, and it shares no code with the GPU
library; the only thing both sides take from elsewhere is the seeded input
arrays made by ``synth``.

What is computed, and where the paper defines it (sections/equations of
"Subtraction method for disconnected diagrams in full QCD"):

  clover, dirac, cgnr     Wilson-clover D and its solves (C core in oracle.c;
                          Methodology and the action named in Results).
  dirac(cut=...)          D_Lambda: D restricted to the fields inside each
                          domain, Dirichlet faces (Domain decomposition
                          subsection, block-matrix equation).
  ape_smear, laplace,     distillation eigenvectors of the gauge-covariant 3-D
  laplace_eigvecs         Laplacian on APE-smeared links (Analysis with
                          standard distillation; Gaussian-profiled section).
  sources, perambulator,  distillation: sources v_i(t) (x) e_alpha, their
  loops                   solutions projected as V^+ D^-1 V, and the quark
                          loop L_Gamma(x0) = sum_x Tr[Gamma D^-1(x,x)] in its
                          distillation form with diagonal elementals
                          Gamma_ab |g(lambda_i)|^2 delta_ij (Methodology,
                          equation Cdisc and the loop definition under it;
                          elementals equation of the Gaussian-profiled section).
  correlator              VEV-subtracted disconnected correlator (equation
                          Cdisc), the completely factorised one, the
                          subtracted one (equation subtracted_correlator), and
                          the four terms of equations corr1-corr4, averaged
                          over source times y0.

Conventions: site s = x + Lx(y + Ly(z + Lz t)); links U[s][mu][a][b];
spinors [s][spin][colour]; Euclidean hermitian chiral gamma basis with
gamma_5 = diag(1,1,-1,-1); boundary phase of the time hop given by bc[3].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib_handle = None

# gamma codes shared by name with the library's loop channels; G_TILDE added to a
# code asks for Gamma~ = gamma_0 Gamma^+ gamma_0 (gamma_0 the time gamma)
G_1, G_5, G_X, G_Y, G_Z = 0, 1, 2, 3, 4
G_TILDE = 8


def build(force: bool = False) -> str:
    """Compile the C core with gcc (plain loops, OpenMP over sites)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _lib():
    global _lib_handle
    if _lib_handle is None:
        build()
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        lib.orc_clover.argtypes = [P, P, D, D, P]
        lib.orc_dirac.argtypes = [P, P, P, P, D, P, I, I, P, P]
        lib.orc_cgnr.argtypes = [P, P, P, P, D, P, I, P, P, D, I, P, P]
        lib.orc_cgnr.restype = I
        lib.orc_gamma.argtypes = [I, P]
        lib.orc_set_threads.argtypes = [I]
        lib.orc_set_threads.restype = I
        _lib_handle = lib
    return _lib_handle


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims(dims):
    return np.ascontiguousarray(np.asarray(dims, dtype=np.int32))


def gamma(mu: int) -> np.ndarray:
    """gamma_{mu+1} for mu = 0..3 (x,y,z,t) and gamma_5 for mu = 4."""
    out = np.zeros((4, 4), dtype=np.complex128)
    _lib().orc_gamma(mu, _ptr(out))
    return out


def channel_matrix(code: int) -> np.ndarray:
    """Dirac matrix Gamma of a loop channel: 1, gamma_5, gamma_1, gamma_2, gamma_3,
    or Gamma~ of one of them when the code carries G_TILDE."""
    if code & G_TILDE:
        return tilde(channel_matrix(code & ~G_TILDE))
    if code == G_1:
        return np.eye(4, dtype=np.complex128)
    if code == G_5:
        return gamma(4)
    return gamma(code - 2)


def tilde(gm: np.ndarray) -> np.ndarray:
    """Gamma-tilde = gamma_0 Gamma^+ gamma_0, with gamma_0 the time gamma
    (Methodology, definition under equation Cdisc)."""
    g0 = gamma(3)
    return g0 @ gm.conj().T @ g0


# --------------------------------------------------------------------------
# operator
# --------------------------------------------------------------------------

def clover(U: np.ndarray, dims, kappa: float, csw: float) -> np.ndarray:
    """A(x) = 1 + i csw kappa sum_{mu<nu} sigma_mu_nu Fhat_mu_nu(x): [V][12][12]."""
    U = np.ascontiguousarray(U, dtype=np.complex128)
    V = int(np.prod(dims))
    A = np.zeros((V, 12, 12), dtype=np.complex128)
    _lib().orc_clover(_ptr(_dims(dims)), _ptr(U), kappa, csw, _ptr(A))
    return A


def _cut_arg(cut, dims):
    if cut is None:
        return None, max(dims)
    c = np.ascontiguousarray(np.asarray(cut, dtype=np.uint8))
    return c, c.shape[1]


def set_threads(n: int) -> int:
    """Timing helper: OpenMP threads of later oracle calls (n > 0); returns the
    previous maximum."""
    return _lib().orc_set_threads(int(n))


def dirac(U, A, dims, bc, kappa, psi, cut=None, dagger=False) -> np.ndarray:
    """D psi (or D_Lambda psi when cut masks are given; D^+ with dagger)."""
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    lib = _lib()
    c, lmax = _cut_arg(cut, dims)
    d = _dims(dims)
    b = _dims(bc)
    if psi.ndim == 4:
        return np.stack([dirac(U, A, dims, bc, kappa, p, cut, dagger) for p in psi])
    out = np.empty_like(psi)
    lib.orc_dirac(_ptr(d), _ptr(b), _ptr(np.ascontiguousarray(U)), _ptr(np.ascontiguousarray(A)),
                  kappa, None if c is None else _ptr(c), lmax, int(dagger), _ptr(psi), _ptr(out))
    return out


def cgnr(U, A, dims, bc, kappa, b, cut=None, tol=1e-12, maxit=100000):
    """Solve D x = b (or D_Lambda x = b) by CGNR to true relative residual tol.
    Returns (x, iterations, true relative residual)."""
    b = np.ascontiguousarray(b, dtype=np.complex128)
    x = np.zeros_like(b)
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0)
    c, lmax = _cut_arg(cut, dims)
    st = _lib().orc_cgnr(_ptr(_dims(dims)), _ptr(_dims(bc)), _ptr(np.ascontiguousarray(U)),
                         _ptr(np.ascontiguousarray(A)), kappa, None if c is None else _ptr(c), lmax,
                         _ptr(b), _ptr(x), tol, maxit, ctypes.byref(it), ctypes.byref(rr))
    if st != 0:
        raise RuntimeError("oracle CGNR did not converge: %d iterations, residual %g" % (it.value, rr.value))
    return x, it.value, rr.value


def dense_dirac(U, A, dims, bc, kappa, cut=None, dagger=False) -> np.ndarray:
    """The operator as a dense (12V x 12V) matrix, column j = D e_j (tiny lattices only)."""
    V = int(np.prod(dims))
    n = 12 * V
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros((V, 4, 3), dtype=np.complex128)
    flat = e.reshape(-1)
    for j in range(n):
        flat[j] = 1
        M[:, j] = dirac(U, A, dims, bc, kappa, e, cut, dagger).reshape(-1)
        flat[j] = 0
    return M


# --------------------------------------------------------------------------
# even-odd pieces (the Schur factorisation of D on the even sites; a standard
# technique the paper does not use, checked here because the production solver
# inverts D through it; D^-1 itself is unchanged)
# --------------------------------------------------------------------------

def site_parity(dims) -> np.ndarray:
    """(x + y + z + t) mod 2 for every site s = x + Lx(y + Ly(z + Lz t))."""
    Lx, Ly, Lz, Lt = dims
    s = np.arange(Lx * Ly * Lz * Lt)
    return (s % Lx + (s // Lx) % Ly + (s // (Lx * Ly)) % Lz + s // (Lx * Ly * Lz)) % 2


def site_apply(M: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """Site-local 12x12 matrices M [V][12][12] on spinors [..][V][4][3]."""
    sh = psi.shape
    flat = psi.reshape(sh[:-2] + (12,))
    return np.matmul(M, flat[..., None])[..., 0].reshape(sh)


def eo_piece(U, A, dims, bc, kappa, parity, ca, cg, cb, psi, aux=None, cut=None, Ainv=None) -> np.ndarray:
    """out(x) = ca aux(x) + A(x)^-1 [cg aux(x) + cb (H psi_{1-p})(x)] at the sites x
    of parity p, zero at the others, with psi_{1-p} = psi on the sites of the
    other parity only and H the hopping sum of D = A - kappa H (with D_Lambda's
    hops when cut is given).  A is site-local and psi_{1-p} vanishes at the
    sites of parity p, so there H psi_{1-p} = -(D psi_{1-p}) / kappa.  With the
    coefficients of the solver these are the pieces of
    M = 1 - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe, of its source
    A_ee^-1 (b_e + kappa H_eo A_oo^-1 b_o) and of the odd reconstruction
    A_oo^-1 (b_o + kappa H_oe x_e).  Ainv: A^-1 per site when already at hand."""
    par = site_parity(dims)
    on = par == parity
    pin = np.where((par == 1 - parity)[:, None, None], psi, 0)
    h = -dirac(U, A, dims, bc, kappa, pin, cut)[..., on, :, :] / kappa
    a = np.zeros_like(psi) if aux is None else aux
    Ai = (np.linalg.inv(A) if Ainv is None else Ainv)[on]
    out = np.zeros_like(psi)
    out[..., on, :, :] = ca * a[..., on, :, :] + site_apply(Ai, cg * a[..., on, :, :] + cb * h)
    return out


# --------------------------------------------------------------------------
# gauge utilities (numpy): coordinates, shifts, gauge transformations
# --------------------------------------------------------------------------

def _lat(a: np.ndarray, dims) -> np.ndarray:
    """View a per-site array [V, ...] as [Lt, Lz, Ly, Lx, ...]."""
    Lx, Ly, Lz, Lt = dims
    return a.reshape((Lt, Lz, Ly, Lx) + a.shape[1:])


_AX = {0: 3, 1: 2, 2: 1, 3: 0}  # direction mu -> axis in the [t,z,y,x] view


def shift(a_lat: np.ndarray, mu: int, step: int) -> np.ndarray:
    """f(x + step*mu) as a field of x (periodic)."""
    return np.roll(a_lat, -step, axis=_AX[mu])


def gauge_transform(U, dims, Om) -> np.ndarray:
    """U_mu(x) -> Om(x) U_mu(x) Om(x+mu)^+."""
    Ul = _lat(U, dims)
    Ol = _lat(Om, dims)
    out = np.empty_like(Ul)
    for mu in range(4):
        Of = shift(Ol, mu, 1)
        out[..., mu, :, :] = Ol @ Ul[..., mu, :, :] @ np.conj(np.swapaxes(Of, -1, -2))
    return out.reshape(U.shape)


# --------------------------------------------------------------------------
# APE smearing and the 3-D covariant Laplacian (distillation set-up)
# --------------------------------------------------------------------------

def su3_project(M: np.ndarray) -> np.ndarray:
    """Gauge-covariant projection to SU(3): polar factor W = M (M^+M)^{-1/2},
    then W / det(W)^{1/3} with the principal cube root."""
    H = np.conj(np.swapaxes(M, -1, -2)) @ M
    w, v = np.linalg.eigh(H)
    isq = np.einsum("...ij,...j,...kj->...ik", v, 1.0 / np.sqrt(w), np.conj(v))
    W = M @ isq
    det = np.linalg.det(W)
    return W / (det ** (1.0 / 3.0))[..., None, None]


def ape_smear(U, dims, alpha: float, steps: int) -> np.ndarray:
    """APE smearing of the spatial links (all links updated together per step):
    U_k <- P[(1-alpha) U_k + (alpha/4) sum of the four spatial staples].
    Time links are left unchanged.  The smeared links feed the Laplacian only
    (distillation sources are built on APE-smeared links)."""
    cur = np.array(_lat(U, dims), copy=True)
    for _ in range(steps):
        new = cur.copy()
        for k in range(3):
            S = np.zeros_like(cur[..., k, :, :])
            Uk = cur[..., k, :, :]
            for j in range(3):
                if j == k:
                    continue
                Uj = cur[..., j, :, :]
                dag = lambda m: np.conj(np.swapaxes(m, -1, -2))
                # up staple: U_j(x) U_k(x+j) U_j(x+k)^+
                S += Uj @ shift(Uk, j, 1) @ dag(shift(Uj, k, 1))
                # down staple: U_j(x-j)^+ U_k(x-j) U_j(x-j+k)
                Ujm = shift(Uj, j, -1)
                S += dag(Ujm) @ shift(Uk, j, -1) @ shift(shift(Uj, j, -1), k, 1)
            new[..., k, :, :] = su3_project((1 - alpha) * Uk + (alpha / 4.0) * S)
        cur = new
    return cur.reshape(U.shape)


def laplace(Us, dims, psi) -> np.ndarray:
    """-Delta psi(x) = sum_{k=1..3} [2 psi(x) - U_k(x) psi(x+k) - U_k(x-k)^+ psi(x-k)]
    on colour vectors psi [V][3] (acts within each timeslice)."""
    Ul = _lat(Us, dims)
    pl = _lat(psi, dims)
    out = np.zeros_like(pl)
    for k in range(3):
        Uk = Ul[..., k, :, :]
        out += 2 * pl
        out -= np.einsum("...ab,...b->...a", Uk, shift(pl, k, 1))
        Ub = shift(Uk, k, -1)
        out -= np.einsum("...ba,...b->...a", np.conj(Ub), shift(pl, k, -1))
    return out.reshape(psi.shape)


def laplace_dense_timeslice(Us, dims, t: int) -> np.ndarray:
    """Dense matrix of -Delta on timeslice t, index (xvec, colour), xvec = x + Lx(y + Ly z)."""
    Lx, Ly, Lz, Lt = dims
    Vs = Lx * Ly * Lz
    n = 3 * Vs
    V = Vs * Lt
    M = np.empty((n, n), dtype=np.complex128)
    # apply to all unit vectors on the slice at once, in chunks
    for j0 in range(0, n, 192):
        j1 = min(n, j0 + 192)
        cols = []
        for j in range(j0, j1):
            e = np.zeros((V, 3), dtype=np.complex128)
            e[t * Vs + j // 3, j % 3] = 1
            cols.append(e)
        for jj, e in enumerate(cols):
            M[:, j0 + jj] = laplace(Us, dims, e)[t * Vs:(t + 1) * Vs].reshape(-1)
    return M


def laplace_eigvecs(Us, dims, nv: int):
    """Lowest nv eigenpairs of -Delta on every timeslice, ascending.
    Returns (V [T][nv][Vs][3], lam [T][nv]).  Dense eigh (LAPACK) per slice for
    small slices, ARPACK (scipy eigsh) otherwise; eigenvector phases arbitrary."""
    Lx, Ly, Lz, Lt = dims
    Vs = Lx * Ly * Lz
    n = 3 * Vs
    vecs = np.empty((Lt, nv, Vs, 3), dtype=np.complex128)
    lam = np.empty((Lt, nv))
    if n <= 1600:
        for t in range(Lt):
            w, v = np.linalg.eigh(laplace_dense_timeslice(Us, dims, t))
            lam[t] = w[:nv]
            vecs[t] = v[:, :nv].T.reshape(nv, Vs, 3)
        return vecs, lam
    import scipy.sparse.linalg as sla
    V = Vs * Lt
    for t in range(Lt):
        def mv(y, t=t):
            e = np.zeros((V, 3), dtype=np.complex128)
            e[t * Vs:(t + 1) * Vs] = y.reshape(Vs, 3)
            return laplace(Us, dims, e)[t * Vs:(t + 1) * Vs].reshape(-1)
        op = sla.LinearOperator((n, n), matvec=mv, dtype=np.complex128)
        w, v = sla.eigsh(op, k=nv, which="SA", tol=1e-13)
        o = np.argsort(w)
        lam[t] = w[o]
        vecs[t] = v[:, o].T.reshape(nv, Vs, 3)
    return vecs, lam


# --------------------------------------------------------------------------
# distillation: sources, perambulators, loops
# --------------------------------------------------------------------------

def source(Vt, dims, t: int, i: int, alpha: int) -> np.ndarray:
    """eta(x) = delta_{x4,t} v_i(t; xvec) (x) e_alpha: spinor [V][4][3]."""
    Lx, Ly, Lz, Lt = dims
    Vs = Lx * Ly * Lz
    eta = np.zeros((Lt * Vs, 4, 3), dtype=np.complex128)
    eta[t * Vs:(t + 1) * Vs, alpha, :] = Vt[t, i]
    return eta


def project(Vt, dims, X, t: int) -> np.ndarray:
    """tau[j][beta][r] = sum_{xvec,c} conj(v_j(t;xvec)_c) X_r(t,xvec)_{beta,c}
    for solutions X [n][V][4][3]: the sink side of V^+ D^-1 V at timeslice t."""
    Lx, Ly, Lz, Lt = dims
    Vs = Lx * Ly * Lz
    slab = X[:, t * Vs:(t + 1) * Vs]            # [n][Vs][4][3]
    return np.einsum("jxc,rxbc->jbr", np.conj(Vt[t]), slab)


def perambulator_tt(U, A, dims, bc, kappa, Vt, t: int, cut=None, tol=1e-13):
    """tau(t,t)[j][beta][i][alpha] = V(t)^+ D^-1 V(t) (or with D_Lambda)."""
    nv = Vt.shape[1]
    tau = np.empty((nv, 4, nv, 4), dtype=np.complex128)
    for i in range(nv):
        X = []
        for a in range(4):
            x, _, _ = cgnr(U, A, dims, bc, kappa, source(Vt, dims, t, i, a), cut, tol)
            X.append(x)
        tau[:, :, i, :] = project(Vt, dims, np.stack(X), t)
    return tau


def loop_from_tau(tau_tt: np.ndarray, gm: np.ndarray, w=None) -> complex:
    """L = sum_i w_i sum_{ab} Gamma_ab tau(t,t)[i][b][i][a]: the trace of the
    diagonal elementals Gamma (x) diag(w) against the perambulator."""
    nv = tau_tt.shape[0]
    if w is None:
        w = np.ones(nv)
    s = 0j
    for i in range(nv):
        s += w[i] * np.trace(gm @ tau_tt[i, :, i, :])
    return s


def loops(tau_all: np.ndarray, codes, w=None) -> np.ndarray:
    """Loop table L[g][t] from perambulators tau_all [T][nv][4][nv][4]."""
    T = tau_all.shape[0]
    out = np.empty((len(codes), T), dtype=np.complex128)
    for gi, c in enumerate(codes):
        gm = channel_matrix(c)
        for t in range(T):
            out[gi, t] = loop_from_tau(tau_all[t], gm, None if w is None else w[t])
    return out


def point_loops(Dinv: np.ndarray, dims, gm: np.ndarray) -> np.ndarray:
    """L(t) = sum_xvec Tr[Gamma D^-1(x,x)] from a dense inverse (tiny lattices)."""
    Lx, Ly, Lz, Lt = dims
    Vs = Lx * Ly * Lz
    V = Vs * Lt
    G = Dinv.reshape(V, 4, 3, V, 4, 3)
    out = np.zeros(Lt, dtype=np.complex128)
    for s in range(V):
        blk = G[s, :, :, s, :, :]                 # [a][c][b][c']
        spin = np.einsum("acbc->ab", blk)         # colour trace
        out[s // Vs] += np.trace(gm @ spin)
    return out


# --------------------------------------------------------------------------
# correlators
# --------------------------------------------------------------------------

def _cov(La, Lb, y0s, vev_mode):
    """C(dt) = mean_{y0} [ mean_c La(y0+dt) Lb(y0) - VEV ] for La, Lb [ncfg][T]."""
    ncfg, T = La.shape
    C = np.zeros(T, dtype=np.complex128)
    for dt in range(T):
        acc = 0j
        for y0 in y0s:
            x0 = (y0 + dt) % T
            two = np.mean(La[:, x0] * Lb[:, y0])
            if vev_mode == 0:
                vev = np.mean(La[:, x0]) * np.mean(Lb[:, y0])
            else:
                vev = np.mean(La) * np.mean(Lb)
            acc += two - vev
        C[dt] = acc / len(y0s)
    return C


def correlator(L_full, Lt_full, L_blk, Lt_blk, y0s=None, vev_mode=1):
    """Full C^(d), completely factorised C^(d)_{L0,L1}, subtracted
    dC = C^(d) - C^(d)_{L0,L1}, and the four terms of equations corr1-corr4
    (block-block, block-delta, delta-block, delta-delta) with
    delta L = L - L_Lambda.  Inputs [ncfg][T]; vev_mode 0 = per-timeslice
    means, 1 = means over configurations and timeslices."""
    L_full = np.atleast_2d(L_full)
    Lt_full = np.atleast_2d(Lt_full)
    L_blk = np.atleast_2d(L_blk)
    Lt_blk = np.atleast_2d(Lt_blk)
    T = L_full.shape[1]
    if y0s is None:
        y0s = list(range(T))
    C_full = _cov(L_full, Lt_full, y0s, vev_mode)
    C_fact = _cov(L_blk, Lt_blk, y0s, vev_mode)
    dL, dLt = L_full - L_blk, Lt_full - Lt_blk
    four = np.stack([
        C_fact,
        _cov(L_blk, dLt, y0s, vev_mode),
        _cov(dL, Lt_blk, y0s, vev_mode),
        _cov(dL, dLt, y0s, vev_mode),
    ])
    return C_full, C_fact, C_full - C_fact, four


# --------------------------------------------------------------------------
# the paper's region schedule and Gaussian profiles
# --------------------------------------------------------------------------

def slab_cut(dims, x0: int, delta: int, open_time: bool = False) -> np.ndarray:
    """Cut masks of the partition whose region around operator time x0 is the
    temporal slab {t : |t - x0| <= h} (mod T), h = (delta-1)/2, over all space
    (Domain decomposition subsection): faces after x0+h and after x0-h-1.
    With open_time (the open boundary in time of the paper's ensemble, read as
    one more cut): the face between T-1 and 0 is cut and the slab is clipped
    at the boundaries instead of wrapping."""
    T = dims[3]
    h = (delta - 1) // 2
    cut = np.zeros((4, max(dims)), dtype=np.uint8)
    if open_time:
        cut[3, T - 1] = 1
        if x0 + h < T - 1:
            cut[3, x0 + h] = 1
        if x0 - h - 1 >= 0:
            cut[3, x0 - h - 1] = 1
        return cut
    cut[3, (x0 + h) % T] = 1
    cut[3, (x0 - h - 1) % T] = 1
    return cut


def open_time_cut(dims) -> np.ndarray:
    """Cut masks of the open time boundary alone: the full operator of an
    ensemble with open boundary conditions in time."""
    cut = np.zeros((4, max(dims)), dtype=np.uint8)
    cut[3, dims[3] - 1] = 1
    return cut


def slab_loops(U, A, dims, bc, kappa, Vt, delta: int, codes, w=None, tol=1e-13, open_time=False):
    """L[g][x0]: the loop of D_Lambda(x0)^-1 at x0 for every operator time x0,
    each solved on its own (no multi-site packing)."""
    T = dims[3]
    nv = Vt.shape[1]
    tau = np.empty((T, nv, 4, nv, 4), dtype=np.complex128)
    for x0 in range(T):
        tau[x0] = perambulator_tt(U, A, dims, bc, kappa, Vt, x0, slab_cut(dims, x0, delta, open_time), tol)
    return loops(tau, codes, w), tau


def nr_splice(Cc, dC_by_delta, deltas) -> np.ndarray:
    """The noise-reduced estimator spliced by separation (Results, analysis with
    standard distillation): C^NR(dt) = C^(c)(dt) + dC_Delta(dt), Delta the widest
    of the given slab widths that is smaller than dt; NaN where none is."""
    T = len(Cc)
    out = np.full(T, np.nan + 0j, dtype=np.complex128)
    for dt in range(T):
        below = [k for k, d in enumerate(deltas) if d < dt]
        if below:
            k = max(below, key=lambda q: deltas[q])
            out[dt] = Cc[dt] + dC_by_delta[k][dt]
    return out


def profile_weights(lam, omega: float) -> np.ndarray:
    """|g_k(lambda)|^2 for the Gaussian profile g_k(lambda) =
    exp(-lambda^2 / (2 (0.8 omega_k)^2)) (Gaussian-profiled subsection)."""
    lam = np.asarray(lam, dtype=np.float64)
    g = np.exp(-lam ** 2 / (2.0 * (0.8 * omega) ** 2))
    return np.abs(g) ** 2


# --------------------------------------------------------------------------
# connected contraction (equation Cfull)
# --------------------------------------------------------------------------

def perambulator_all(U, A, dims, bc, kappa, Vt, ts: int, tol=1e-13) -> np.ndarray:
    """tau[tk][j][beta][i][alpha] = V(tk)^+ D^-1 V(ts) for every sink tk."""
    T = dims[3]
    nv = Vt.shape[1]
    tau = np.empty((T, nv, 4, nv, 4), dtype=np.complex128)
    for i in range(nv):
        X = []
        for a in range(4):
            x, _, _ = cgnr(U, A, dims, bc, kappa, source(Vt, dims, ts, i, a), None, tol)
            X.append(x)
        X = np.stack(X)
        for tk in range(T):
            tau[tk, :, :, i, :] = project(Vt, dims, X, tk)
    return tau


def connected(tau_all, codes, w=None, y0s=None) -> np.ndarray:
    """C[g][dt] = -(1/|Y|) sum_{y0} Tr[Phi_G(x0) tau(x0,y0) Phi_Gt(y0) tau(y0,x0)],
    x0 = y0+dt mod T, Phi_G(t) = Gamma (x) diag(w(t)), Gamma~ = g4 Gamma^+ g4,
    with both directions taken from direct solves (tau_all[ts][tk] =
    V(tk)^+ D^-1 V(ts)): the sink-to-source perambulator tau(y0,x0) comes from
    the sources at x0, not from gamma_5-hermiticity."""
    T = tau_all.shape[0]
    nv = tau_all.shape[2]
    y0s = list(range(T)) if y0s is None else list(y0s)
    g4 = gamma(3)
    out = np.zeros((len(codes), T), dtype=np.complex128)
    for gi, c in enumerate(codes):
        G = channel_matrix(c)
        Gt = g4 @ np.conj(G.T) @ g4
        for dt in range(T):
            acc = 0j
            for y0 in y0s:
                x0 = (y0 + dt) % T
                wx = np.ones(nv) if w is None else w[x0]
                wy = np.ones(nv) if w is None else w[y0]
                Phi_x = np.kron(np.diag(wx), G)      # index j*4 + beta
                Phi_y = np.kron(np.diag(wy), Gt)
                fwd = tau_all[y0, x0].reshape(4 * nv, 4 * nv)   # tau(x0, y0)
                bwd = tau_all[x0, y0].reshape(4 * nv, 4 * nv)   # tau(y0, x0)
                acc += np.trace(Phi_x @ fwd @ Phi_y @ bwd)
            out[gi, dt] = -acc / len(y0s)
    return out
