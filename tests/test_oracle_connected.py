"""Pins of the oracle's connected contraction: with a complete eigenbasis the
distillation contraction is the point-to-point one of a dense inverse, and the
two directions of the perambulator obey gamma_5-hermiticity."""
import numpy as np

import oracle
import synth

BC = (1, 1, 1, -1)


def test_complete_basis_equals_point_contraction():
    dims = (2, 2, 1, 4)
    kappa, csw = 0.12, 1.0
    U = synth.gauge_field(dims, 0.5, 101)
    A = oracle.clover(U, dims, kappa, csw)
    Lx, Ly, Lz, Lt = dims
    Vs = Lx * Ly * Lz
    nv = 3 * Vs
    Vt, _ = oracle.laplace_eigvecs(oracle.ape_smear(U, dims, 0.5, 1), dims, nv)
    tau = np.stack([oracle.perambulator_all(U, A, dims, BC, kappa, Vt, ts, tol=1e-14) for ts in range(Lt)])
    codes = [oracle.G_1, oracle.G_5, oracle.G_X, oracle.G_Z]
    C = oracle.connected(tau, codes)
    Dinv = np.linalg.inv(oracle.dense_dirac(U, A, dims, BC, kappa)).reshape(Lt, Vs, 12, Lt, Vs, 12)
    g4 = oracle.gamma(3)
    for gi, c in enumerate(codes):
        G = oracle.channel_matrix(c)
        Gt = g4 @ np.conj(G.T) @ g4
        Gk, Gtk = np.kron(G, np.eye(3)), np.kron(Gt, np.eye(3))  # spin*3 + colour
        for dt in range(Lt):
            ref = 0j
            for y0 in range(Lt):
                x0 = (y0 + dt) % Lt
                tot = 0j
                for xs in range(Vs):
                    for ys in range(Vs):
                        tot += np.trace(Gk @ Dinv[x0, xs, :, y0, ys, :] @ Gtk @ Dinv[y0, ys, :, x0, xs, :])
                ref += tot
            ref = -ref / Lt
            assert abs(C[gi, dt] - ref) <= 1e-10 * max(1.0, abs(ref))


def test_gamma5_hermiticity_of_perambulators():
    dims = (2, 2, 2, 4)
    kappa, csw = 0.13, 1.2
    U = synth.gauge_field(dims, 0.4, 102)
    A = oracle.clover(U, dims, kappa, csw)
    Vt, _ = oracle.laplace_eigvecs(oracle.ape_smear(U, dims, 0.5, 1), dims, 3)
    tau = np.stack([oracle.perambulator_all(U, A, dims, BC, kappa, Vt, ts, tol=1e-14) for ts in range(4)])
    g5 = np.diag([1.0, 1.0, -1.0, -1.0])
    G5 = np.kron(np.eye(3), g5)
    for x0 in range(4):
        for y0 in range(4):
            fwd = tau[y0, x0].reshape(12, 12)
            bwd = tau[x0, y0].reshape(12, 12)
            assert np.abs(bwd - G5 @ np.conj(fwd.T) @ G5).max() < 1e-11


def test_pseudoscalar_connected_correlator_is_a_sum_of_squares():
    """For Gamma = gamma_5 (Gamma-tilde = gamma_4 gamma_5 gamma_4 = -gamma_5) the
    fermion-loop sign and gamma_5-hermiticity make the connected contraction
    C(dt) = (1/|Y|) sum_{y0} sum_{j,beta,i,alpha} w_j(x0) w_i(y0) |tau(x0,y0)[j,beta,i,alpha]|^2,
    real and non-negative.  A dropped sign, or Gamma in place of Gamma-tilde on
    the source side, gives the negative of this."""
    dims = (2, 2, 2, 4)
    kappa, csw = 0.13, 1.2
    U = synth.gauge_field(dims, 0.4, 103)
    A = oracle.clover(U, dims, kappa, csw)
    nv = 3
    Vt, _ = oracle.laplace_eigvecs(oracle.ape_smear(U, dims, 0.5, 1), dims, nv)
    T = dims[3]
    tau = np.stack([oracle.perambulator_all(U, A, dims, BC, kappa, Vt, ts, tol=1e-14) for ts in range(T)])
    rng = np.random.default_rng(5)
    w = rng.uniform(0.2, 1.5, size=(T, nv))
    for wt in (None, w):
        C = oracle.connected(tau, [oracle.G_5], w=wt)[0]
        for dt in range(T):
            ref = 0.0
            for y0 in range(T):
                x0 = (y0 + dt) % T
                a = np.abs(tau[y0, x0]) ** 2                     # [j][beta][i][alpha]
                wx = np.ones(nv) if wt is None else wt[x0]
                wy = np.ones(nv) if wt is None else wt[y0]
                ref += np.einsum("j,jbia,i->", wx, a, wy)
            ref /= T
            assert ref > 0
            assert abs(C[dt] - ref) <= 1e-11 * ref
