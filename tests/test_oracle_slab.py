"""Pins of the oracle's region schedule (centred temporal slabs) and of the
Gaussian distillation profiles."""
import numpy as np
import pytest

import oracle
import synth

BC = (1, 1, 1, -1)


def _slab_sites(dims, x0, delta):
    Lx, Ly, Lz, Lt = dims
    Vs = Lx * Ly * Lz
    h = (delta - 1) // 2
    ts = [(x0 + k) % Lt for k in range(-h, h + 1)]
    return ts, np.concatenate([np.arange(t * Vs, (t + 1) * Vs) for t in ts])


@pytest.mark.parametrize("delta", [1, 3])
def test_slab_loops_equal_principal_submatrix_inverse(delta):
    """D_Lambda(x0)^-1 at (x0, x0) is the inverse of the principal submatrix of
    the dense D on the slab sites (taken by slicing, with no cut masks), so
    the slab loops follow from a brute-force dense inverse."""
    dims = (2, 2, 2, 6)
    kappa, csw = 0.13, 1.1
    U = synth.gauge_field(dims, 0.5, 81)
    A = oracle.clover(U, dims, kappa, csw)
    Us = oracle.ape_smear(U, dims, 0.5, 1)
    Vt, _ = oracle.laplace_eigvecs(Us, dims, 2)
    codes = [oracle.G_1, oracle.G_5, oracle.G_X]
    L, _ = oracle.slab_loops(U, A, dims, BC, kappa, Vt, delta, codes, tol=1e-14)
    Dd = oracle.dense_dirac(U, A, dims, BC, kappa)
    Lx, Ly, Lz, Lt = dims
    Vs = Lx * Ly * Lz
    nv = Vt.shape[1]
    for x0 in range(Lt):
        ts, sites = _slab_sites(dims, x0, delta)
        idx = (sites[:, None] * 12 + np.arange(12)[None, :]).ravel()
        inv = np.linalg.inv(Dd[np.ix_(idx, idx)])
        # position of timeslice x0 inside the slab
        k0 = ts.index(x0)
        blk = inv.reshape(len(ts), Vs, 4, 3, len(ts), Vs, 4, 3)[k0, :, :, :, k0]
        tau = np.einsum("jxc,xbcyad,iyd->jbia", np.conj(Vt[x0]), blk, Vt[x0])
        for gi, c in enumerate(codes):
            ref = oracle.loop_from_tau(tau, oracle.channel_matrix(c))
            assert abs(L[gi, x0] - ref) <= 1e-11 * max(1.0, abs(ref))


def test_slab_loops_gauge_invariant():
    dims = (2, 2, 2, 6)
    kappa, csw = 0.12, 1.0
    U = synth.gauge_field(dims, 0.5, 82)
    V = int(np.prod(dims))
    Om = synth.random_su3(V, 83)
    Ug = oracle.gauge_transform(U, dims, Om)
    codes = [oracle.G_1, oracle.G_5]
    out = []
    for W in (U, Ug):
        A = oracle.clover(W, dims, kappa, csw)
        Vt, _ = oracle.laplace_eigvecs(oracle.ape_smear(W, dims, 0.5, 1), dims, 2)
        L, _ = oracle.slab_loops(W, A, dims, BC, kappa, Vt, 3, codes, tol=1e-14)
        out.append(L)
    assert np.abs(out[0] - out[1]).max() < 1e-10 * np.abs(out[0]).max()


def test_profile_weights_closed_form():
    w = oracle.profile_weights([0.0, 0.8 * 0.129, 2 * 0.8 * 0.05], 0.129)
    assert w[0] == 1.0
    assert abs(w[1] - np.exp(-1.0)) < 1e-15
    w2 = oracle.profile_weights([2 * 0.8 * 0.05], 0.05)
    assert abs(w2[0] - np.exp(-4.0)) < 1e-15
    # a very wide profile is standard distillation
    assert np.abs(oracle.profile_weights(np.linspace(0, 2, 7), 1e8) - 1.0).max() < 1e-15
