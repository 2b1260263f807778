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


def test_open_time_cut_removes_exactly_the_wrap_hops():
    """The open time boundary as a cut: the dense operator with the face between
    T-1 and 0 cut equals the dense D with every entry coupling timeslice T-1
    and timeslice 0 set to zero (and nothing else changed)."""
    dims = (2, 2, 2, 4)
    kappa, csw = 0.13, 1.2
    U = synth.gauge_field(dims, 0.5, 84)
    A = oracle.clover(U, dims, kappa, csw)
    D = oracle.dense_dirac(U, A, dims, BC, kappa)
    Do = oracle.dense_dirac(U, A, dims, BC, kappa, oracle.open_time_cut(dims))
    Vs, T = 8, dims[3]
    t_of = np.repeat(np.arange(T), Vs * 12)
    wrap = ((t_of[:, None] == T - 1) & (t_of[None, :] == 0)) | ((t_of[:, None] == 0) & (t_of[None, :] == T - 1))
    assert np.abs(D[wrap]).max() > 0.01
    assert np.array_equal(Do, np.where(wrap, 0, D))


@pytest.mark.parametrize("delta", [1, 3])
def test_open_time_slab_loops_equal_clipped_submatrix_inverse(delta):
    """With the open time boundary the slab of x0 is clipped at t = 0 and T-1:
    its loops are those of the inverse of the principal submatrix of the dense
    open-boundary operator on the clipped slab's sites."""
    dims = (2, 2, 2, 6)
    kappa, csw = 0.13, 1.1
    U = synth.gauge_field(dims, 0.5, 85)
    A = oracle.clover(U, dims, kappa, csw)
    Vt, _ = oracle.laplace_eigvecs(oracle.ape_smear(U, dims, 0.5, 1), dims, 2)
    codes = [oracle.G_1, oracle.G_5, oracle.G_X]
    L, _ = oracle.slab_loops(U, A, dims, BC, kappa, Vt, delta, codes, tol=1e-14, open_time=True)
    Do = oracle.dense_dirac(U, A, dims, BC, kappa, oracle.open_time_cut(dims))
    Vs, Lt = 8, dims[3]
    h = (delta - 1) // 2
    for x0 in range(Lt):
        ts = [t for t in range(x0 - h, x0 + h + 1) if 0 <= t < Lt]
        sites = np.concatenate([np.arange(t * Vs, (t + 1) * Vs) for t in ts])
        idx = (sites[:, None] * 12 + np.arange(12)[None, :]).ravel()
        inv = np.linalg.inv(Do[np.ix_(idx, idx)])
        k0 = ts.index(x0)
        blk = inv.reshape(len(ts), Vs, 4, 3, len(ts), Vs, 4, 3)[k0, :, :, :, k0]
        tau = np.einsum("jxc,xbcyad,iyd->jbia", np.conj(Vt[x0]), blk, Vt[x0])
        for gi, c in enumerate(codes):
            ref = oracle.loop_from_tau(tau, oracle.channel_matrix(c))
            assert abs(L[gi, x0] - ref) <= 1e-11 * max(1.0, abs(ref))


def test_nr_splice_takes_the_papers_widths():
    """The splice rule (the widest width below the separation) reproduces the
    paper's choice of block size per source-sink distance."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "nr_splice_widths.json")))
    widths = g["widths"]
    T = 48
    Cc = np.zeros(T, dtype=np.complex128)
    dC = np.array([np.full(T, 1000.0 * w) for w in widths], dtype=np.complex128)   # tags each width
    out = oracle.nr_splice(Cc, dC, widths)
    for dt, w in g["width_at_separation"].items():
        assert out[int(dt)] == 1000.0 * w, (dt, w)
    assert np.isnan(out[:8]).all()       # no block is narrower than separations up to 7
    # and it is C^(c) + dC of that width
    rng = np.random.default_rng(3)
    Cc = rng.standard_normal(T) + 1j * rng.standard_normal(T)
    dC = rng.standard_normal((4, T)) + 1j * rng.standard_normal((4, T))
    out = oracle.nr_splice(Cc, dC, widths)
    assert out[10] == Cc[10] + dC[1][10] and out[30] == Cc[30] + dC[3][30]
