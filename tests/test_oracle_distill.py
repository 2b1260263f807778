"""Pins of the oracle's distillation chain: APE smearing, the covariant
Laplacian and its eigenvectors, perambulators, loops and correlators."""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from lattice_fixtures import abelian_flux_field, unit_field, coords, momenta

BC = (1, 1, 1, -1)
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_su3_projection_polar_factor():
    """For M = W P with W in SU(3) and P hermitian positive, the projection returns W."""
    W = synth.random_su3(5, 1)
    rng = np.random.default_rng(2)
    Z = rng.standard_normal((5, 3, 3)) + 1j * rng.standard_normal((5, 3, 3))
    P = Z @ np.conj(np.swapaxes(Z, 1, 2)) + 0.5 * np.eye(3)
    out = oracle.su3_project(W @ P)
    assert np.abs(out - W).max() < 1e-13


def test_ape_unit_field_and_constant_flux_are_fixed_points():
    """U = 1 is unchanged; a constant abelian flux in a spatial plane is also
    unchanged, because every staple sum equals U_k times a positive diagonal."""
    dims = (4, 4, 4, 2)
    U1 = unit_field(dims)
    assert np.abs(oracle.ape_smear(U1, dims, 0.5, 3) - U1).max() < 1e-14
    U, _ = abelian_flux_field(dims, 0, 1, 1)
    S = oracle.ape_smear(U, dims, 0.5, 2)
    assert np.abs(S - U).max() < 1e-13


def test_ape_changes_rough_links_covariantly():
    dims = (4, 4, 2, 2)
    U = synth.gauge_field(dims, 0.5, 3)
    S = oracle.ape_smear(U, dims, 0.5, 2)
    # smeared spatial links are SU(3), time links untouched
    Sk = S[:, :3]
    assert np.abs(Sk @ np.conj(np.swapaxes(Sk, -1, -2)) - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(Sk) - 1).max() < 1e-13
    assert np.abs(S[:, 3] - U[:, 3]).max() == 0
    assert np.abs(S[:, :3] - U[:, :3]).max() > 1e-2
    # smearing reduces roughness: mean plaquette-free measure |Re tr U|/3 moves towards 1 (smoother)
    V = int(np.prod(dims))
    Om = synth.random_su3(V, 4)
    S2 = oracle.ape_smear(oracle.gauge_transform(U, dims, Om), dims, 0.5, 2)
    assert np.abs(S2 - oracle.gauge_transform(S, dims, Om)).max() < 1e-12


def test_laplacian_free_spectrum():
    """U = 1: eigenvalues 4 sum_k sin^2(p_k/2), p_k = 2 pi n/L_k, each three-fold (colour)."""
    dims = (4, 2, 3, 2)
    M = oracle.laplace_dense_timeslice(unit_field(dims), dims, 1)
    ev = np.sort(np.linalg.eigvalsh(M))
    ps = [2 * np.pi * np.arange(L) / L for L in dims[:3]]
    ref = sorted(4 * (np.sin(a / 2) ** 2 + np.sin(b / 2) ** 2 + np.sin(c / 2) ** 2)
                 for a in ps[0] for b in ps[1] for c in ps[2] for _ in range(3))
    assert np.abs(ev - np.array(ref)).max() < 1e-13


def test_laplacian_hermitian_gauge_invariant_spectrum():
    dims = (4, 4, 2, 2)
    U = synth.gauge_field(dims, 0.6, 7)
    M = oracle.laplace_dense_timeslice(U, dims, 0)
    assert np.abs(M - M.conj().T).max() < 1e-15
    ev = np.linalg.eigvalsh(M)
    assert ev.min() > -1e-12
    V = int(np.prod(dims))
    Om = synth.random_su3(V, 8)
    ev2 = np.linalg.eigvalsh(oracle.laplace_dense_timeslice(oracle.gauge_transform(U, dims, Om), dims, 0))
    assert np.abs(ev - ev2).max() < 1e-12


def test_eigvecs_dense_and_arpack_agree():
    dims = (4, 4, 4, 2)
    Us = oracle.ape_smear(synth.gauge_field(dims, 0.4, 9), dims, 0.5, 1)
    V1, l1 = oracle.laplace_eigvecs(Us, dims, 6)
    # residual and orthonormality of the dense path
    Vs = 64
    for t in range(2):
        for i in range(6):
            e = np.zeros((Vs * 2, 3), dtype=np.complex128)
            e[t * Vs:(t + 1) * Vs] = V1[t, i]
            r = oracle.laplace(Us, dims, e)[t * Vs:(t + 1) * Vs] - l1[t, i] * V1[t, i]
            assert np.abs(r).max() < 1e-12
        G = np.einsum("ixc,jxc->ij", np.conj(V1[t]), V1[t])
        assert np.abs(G - np.eye(6)).max() < 1e-13
    # the ARPACK path (forced) gives the same eigenvalues and projector
    import scipy.sparse.linalg as sla
    for t in range(2):
        def mv(y, t=t):
            e = np.zeros((Vs * 2, 3), dtype=np.complex128)
            e[t * Vs:(t + 1) * Vs] = y.reshape(Vs, 3)
            return oracle.laplace(Us, dims, e)[t * Vs:(t + 1) * Vs].reshape(-1)
        op = sla.LinearOperator((192, 192), matvec=mv, dtype=np.complex128)
        w, v = sla.eigsh(op, k=6, which="SA", tol=1e-13)
        o = np.argsort(w)
        assert np.abs(w[o] - l1[t]).max() < 1e-10
        P1 = V1[t].reshape(6, -1).T @ np.conj(V1[t].reshape(6, -1))
        P2 = v[:, o] @ np.conj(v[:, o]).T
        assert np.abs(P1 - P2).max() < 1e-8


def _plane_wave_basis(dims, ks, colours):
    Lx, Ly, Lz, Lt = dims
    Vs = Lx * Ly * Lz
    X = coords(dims)[:Vs, :3]
    vecs = []
    for k in ks:
        ph = np.exp(1j * (X @ np.asarray(k))) / np.sqrt(Vs)
        for c in colours:
            v = np.zeros((Vs, 3), dtype=np.complex128)
            v[:, c] = ph
            vecs.append(v)
    return np.broadcast_to(np.stack(vecs), (Lt,) + np.stack(vecs).shape).copy()


def test_free_field_loops_closed_form():
    """U = 1, plane-wave distillation vectors: tau(t,t) = (1/Lt) sum_p4 D(k,p4)^-1 (x) 1,
    hence L_Gamma(t) = sum_(k,c) (1/Lt) sum_p4 Tr[Gamma D(k,p4)^-1]."""
    dims = (4, 4, 4, 4)
    kappa = 0.1
    U = unit_field(dims)
    A = oracle.clover(U, dims, kappa, 1.0)
    ks = [(0.0, 0.0, 0.0), (2 * np.pi / 4, 0.0, 2 * np.pi * 3 / 4)]
    Vt = _plane_wave_basis(dims, ks, [0, 2])
    nv = Vt.shape[1]
    g = [oracle.gamma(m) for m in range(4)]
    p4s = momenta(dims, BC)[3]
    codes = [oracle.G_1, oracle.G_5, oracle.G_X, oracle.G_Y, oracle.G_Z]
    t = 2
    tau = oracle.perambulator_tt(U, A, dims, BC, kappa, Vt, t)
    Lv = [oracle.loop_from_tau(tau, oracle.channel_matrix(c)) for c in codes]
    for ci, c in enumerate(codes):
        gm = oracle.channel_matrix(c)
        ref = 0j
        for k in ks:
            for p4 in p4s:
                p = list(k) + [p4]
                M = 1 - 2 * kappa * sum(np.cos(p))
                S = (M * np.eye(4) - 2j * kappa * sum(g[m] * np.sin(p[m]) for m in range(4))) / (
                    M ** 2 + 4 * kappa ** 2 * sum(np.sin(p) ** 2))
                ref += 2 * np.trace(gm @ S) / len(p4s)   # two colours per momentum
        assert abs(Lv[ci] - ref) < 1e-11, (c, Lv[ci], ref)
    # off-diagonal (k, c) blocks vanish
    blk = tau.reshape(nv, 4, nv, 4)
    for i in range(nv):
        for j in range(nv):
            if i != j:
                assert np.abs(blk[j, :, i, :]).max() < 1e-11


def test_kappa_zero_loops():
    """kappa = 0: D = 1, tau = V^+ V = 1, so L_1 = 4 Nv and the other channels vanish."""
    dims = (2, 2, 2, 4)
    U = synth.gauge_field(dims, 0.5, 1)
    A = oracle.clover(U, dims, 0.0, 1.0)
    Vt, _ = oracle.laplace_eigvecs(U, dims, 5)
    tau = np.stack([oracle.perambulator_tt(U, A, dims, BC, 0.0, Vt, t) for t in range(4)])
    L = oracle.loops(tau, [oracle.G_1, oracle.G_5, oracle.G_X, oracle.G_Y, oracle.G_Z])
    assert np.abs(L[0] - 20).max() < 1e-12
    assert np.abs(L[1:]).max() < 1e-12


@pytest.fixture(scope="module")
def tiny_setup():
    dims = (2, 2, 2, 4)
    U = synth.gauge_field(dims, 0.5, 61)
    kappa = 0.12
    A = oracle.clover(U, dims, kappa, 1.0)
    D = oracle.dense_dirac(U, A, dims, BC, kappa)
    return dims, U, A, kappa, D


def test_full_eigenbasis_distillation_equals_point_loop(tiny_setup):
    """Nv = 3 Vs: V V^+ = 1 on the timeslice, so the distillation loop equals
    the point loop sum_x Tr[Gamma D^-1(x,x)] of the Methodology definition."""
    dims, U, A, kappa, D = tiny_setup
    Dinv = np.linalg.inv(D)
    Vt, _ = oracle.laplace_eigvecs(U, dims, 24)
    tau = np.stack([oracle.perambulator_tt(U, A, dims, BC, kappa, Vt, t) for t in range(4)])
    codes = [oracle.G_1, oracle.G_5, oracle.G_X, oracle.G_Y, oracle.G_Z]
    L = oracle.loops(tau, codes)
    for ci, c in enumerate(codes):
        ref = oracle.point_loops(Dinv, dims, oracle.channel_matrix(c))
        assert np.abs(L[ci] - ref).max() < 1e-11


def test_loop_reality_and_tau_g5_hermiticity(tiny_setup):
    """gamma_5-hermiticity: tau(t,t)^+ = g5 tau g5, so L_1, L_g5 are real and
    L_gi imaginary on every configuration."""
    dims, U, A, kappa, D = tiny_setup
    Vt, _ = oracle.laplace_eigvecs(U, dims, 3)
    tau = oracle.perambulator_tt(U, A, dims, BC, kappa, Vt, 1)
    M = tau.reshape(12, 12)
    G5 = np.kron(np.eye(3), oracle.gamma(4))
    assert np.abs(M.conj().T - G5 @ M @ G5).max() < 1e-12
    L = [oracle.loop_from_tau(tau, oracle.channel_matrix(c)) for c in range(5)]
    assert abs(L[0].imag) < 1e-12 and abs(L[1].imag) < 1e-12
    for c in (2, 3, 4):
        assert abs(L[c].real) < 1e-12


def test_loops_gauge_invariant():
    """Loops built from eigenvectors recomputed on the transformed field are unchanged."""
    dims = (2, 2, 2, 4)
    U = synth.gauge_field(dims, 0.5, 71)
    kappa = 0.12
    V = int(np.prod(dims))
    Om = synth.random_su3(V, 72)
    codes = [oracle.G_1, oracle.G_5, oracle.G_X]
    out = []
    for UU in (U, oracle.gauge_transform(U, dims, Om)):
        A = oracle.clover(UU, dims, kappa, 1.3)
        Us = oracle.ape_smear(UU, dims, 0.5, 1)
        Vt, _ = oracle.laplace_eigvecs(Us, dims, 4)
        tau = np.stack([oracle.perambulator_tt(UU, A, dims, BC, kappa, Vt, t) for t in range(4)])
        out.append(oracle.loops(tau, codes))
    assert np.abs(out[0] - out[1]).max() < 1e-11


def test_block_loops_single_domain_equal_full(tiny_setup):
    dims, U, A, kappa, D = tiny_setup
    Vt, _ = oracle.laplace_eigvecs(U, dims, 2)
    cut = np.zeros((4, 4), dtype=np.uint8)
    a = oracle.perambulator_tt(U, A, dims, BC, kappa, Vt, 0)
    b = oracle.perambulator_tt(U, A, dims, BC, kappa, Vt, 0, cut=cut)
    assert np.abs(a - b).max() < 1e-11


def test_correlator_hand_example():
    g = json.load(open(os.path.join(GOLD, "correlator_hand_example.json")))
    L = np.array(g["L"], dtype=np.complex128)
    for mode, key in ((0, "C_vev_per_timeslice"), (1, "C_vev_translation_averaged")):
        C, Cf, dC, four = oracle.correlator(L, L, L, L, vev_mode=mode)
        assert np.abs(C - np.array(g[key])).max() < 1e-15
        assert np.abs(dC).max() == 0


def test_correlator_four_terms_sum_and_shift_invariance():
    rng = np.random.default_rng(5)
    ncfg, T = 7, 6
    Lf = rng.standard_normal((ncfg, T)) + 1j * rng.standard_normal((ncfg, T))
    Ltf = rng.standard_normal((ncfg, T))
    Lb = Lf + 0.1 * rng.standard_normal((ncfg, T))
    Ltb = Ltf + 0.1 * rng.standard_normal((ncfg, T))
    for mode in (0, 1):
        C, Cf, dC, four = oracle.correlator(Lf, Ltf, Lb, Ltb, vev_mode=mode)
        assert np.abs(four.sum(axis=0) - C).max() < 1e-13
        assert np.abs(dC - (four[1] + four[2] + four[3])).max() < 1e-13
        C2, _, _, _ = oracle.correlator(Lf + 3.0, Ltf - 2.0, Lb, Ltb, vev_mode=mode)
        assert np.abs(C2 - C).max() < 1e-12
    # a subset of source times averages only those
    C, _, _, _ = oracle.correlator(Lf, Ltf, Lb, Ltb, y0s=[2], vev_mode=0)
    ref = np.mean(Lf[:, 3] * Ltf[:, 2]) - np.mean(Lf[:, 3]) * np.mean(Ltf[:, 2])
    assert abs(C[1] - ref) < 1e-14


def _diag_phase_field(dims, spread, seed):
    """Diagonal SU(3) links diag(e^{i a}, e^{i b}, e^{-i(a+b)}) with Gaussian phases
    (a U(1) x U(1) embedding): staples, their sums and the projection act entry by
    entry, so one APE step has a closed form per colour."""
    V = int(np.prod(dims))
    rng = np.random.default_rng(seed)
    ph = spread * rng.standard_normal((V, 4, 2))
    ph = np.concatenate([ph, -ph.sum(axis=2, keepdims=True)], axis=2)   # [V][mu][c]
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    for c in range(3):
        U[:, :, c, c] = np.exp(1j * ph[:, :, c])
    return U, ph


def _ape_step_diag_closed_form(ph, dims, alpha):
    """One APE step on a diagonal phase field, written entry by entry with explicit
    site arithmetic: m_c = (1 - alpha) e^{i phi_k,c(x)} + (alpha/4) sum over the four
    spatial staples of e^{i (staple phase)}, polar factor m_c/|m_c|, then division by
    the principal cube root of the determinant.  Returns the new phases [V][mu][c]."""
    Lx, Ly, Lz, Lt = dims
    L = (Lx, Ly, Lz, Lt)

    def idx(x):
        return x[0] + Lx * (x[1] + Ly * (x[2] + Lz * x[3]))

    def step(x, mu, d):
        y = list(x)
        y[mu] = (y[mu] + d) % L[mu]
        return y

    V = int(np.prod(dims))
    out = ph.copy()
    for s in range(V):
        x = [s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)]
        for k in range(3):
            w = np.empty(3, dtype=np.complex128)
            for c in range(3):
                m = (1 - alpha) * np.exp(1j * ph[s, k, c])
                for j in range(3):
                    if j == k:
                        continue
                    # forward staple U_j(x) U_k(x+j) U_j(x+k)^+
                    up = ph[s, j, c] + ph[idx(step(x, j, 1)), k, c] - ph[idx(step(x, k, 1)), j, c]
                    # backward staple U_j(x-j)^+ U_k(x-j) U_j(x-j+k)
                    xm = step(x, j, -1)
                    dn = -ph[idx(xm), j, c] + ph[idx(xm), k, c] + ph[idx(step(xm, k, 1)), j, c]
                    m += (alpha / 4.0) * (np.exp(1j * up) + np.exp(1j * dn))
                w[c] = m / abs(m)
            theta = np.angle(np.prod(w))               # principal argument in (-pi, pi]
            out[s, k] = np.angle(w) - theta / 3.0
    return out


@pytest.mark.parametrize("alpha", [0.5, 0.8])
def test_ape_closed_form_on_diagonal_phase_links(alpha):
    """On diagonal (abelian) links with random phases the staple sum is no longer a
    positive multiple of U, so the result fixes the weighting (1 - alpha) U +
    (alpha/4) S, the staple paths and the determinant fix; two steps check that a
    sweep updates every link from the previous sweep."""
    dims = (4, 4, 4, 2)
    U, ph = _diag_phase_field(dims, 0.6, 21)
    S1 = oracle.ape_smear(U, dims, alpha, 1)
    S2 = oracle.ape_smear(U, dims, alpha, 2)
    p1 = _ape_step_diag_closed_form(ph, dims, alpha)
    p2 = _ape_step_diag_closed_form(p1, dims, alpha)
    for S, p in ((S1, p1), (S2, p2)):
        ref = np.zeros_like(U)
        for c in range(3):
            ref[:, :3, c, c] = np.exp(1j * p[:, :3, c])
        ref[:, 3] = U[:, 3]
        assert np.abs(S - ref).max() < 1e-13
    # the smearing moved the links by far more than the tolerance
    assert np.abs(S1 - U).max() > 1e-1
