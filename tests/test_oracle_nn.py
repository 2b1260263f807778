"""Pins of the oracle's gauge-covariant network (the learned preconditioner):
closed forms, the Wilson hopping term, covariance, the path order, and
finite-difference gradients."""
import numpy as np
import pytest

import oracle
import synth
from oracle import nn

DIMS = (3, 3, 3, 4)


def _unit_links(dims):
    V = int(np.prod(dims))
    return np.broadcast_to(np.eye(3, dtype=np.complex128), (V, 4, 3, 3)).copy()


def _rand_layer(rng, co, ci):
    return rng.standard_normal((nn.NOFF, co, ci, 4, 4)) + 1j * rng.standard_normal((nn.NOFF, co, ci, 4, 4))


def _site(dims, x, y, z, t):
    Lx, Ly, Lz, Lt = dims
    return x + Lx * (y + Ly * (z + Lz * t))


@pytest.mark.parametrize("bc", [(1, 1, 1, 1), (1, 1, 1, -1)])
def test_free_field_plane_wave(bc):
    """U = 1: a layer is a translation-invariant convolution, so a plane wave
    e^{ipx} u maps to (sum_d W[d] e^{ip.d}) u e^{ipx}; antiperiodic time shifts
    p_t by pi/L_t.  Pins the direction of every one of the 81 offsets."""
    dims = DIMS
    rng = np.random.default_rng(3)
    W = _rand_layer(rng, 1, 1)
    T = nn.transports(_unit_links(dims), dims, bc)
    n = (1, 2, 1, 3)
    p = [2 * np.pi * n[mu] / dims[mu] for mu in range(4)]
    if bc[3] < 0:
        p[3] = (2 * np.pi * n[3] + np.pi) / dims[3]
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t)).reshape(-1)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    psi = phase[:, None, None] * u[None]
    out = nn.layer_forward(T, dims, W, psi[None])[0]
    What = sum(W[k, 0, 0] * np.exp(1j * np.dot(p, d)) for k, d in enumerate(nn.OFFSETS))
    ref = phase[:, None, None] * (What @ u)[None]
    assert np.abs(out - ref).max() < 1e-12 * np.abs(ref).max()


def _wilson_weights(kappa, co=1, ci=1, o=0, i=0):
    """delta weights that make a layer the Wilson operator 1 - kappa H."""
    W = np.zeros((nn.NOFF, co, ci, 4, 4), dtype=np.complex128)
    W[40, o, i] = np.eye(4)
    for mu in range(4):
        g = oracle.gamma(mu)
        e = [0, 0, 0, 0]
        e[mu] = 1
        W[nn.offset_index(e), o, i] = -kappa * (np.eye(4) - g)
        e[mu] = -1
        W[nn.offset_index(e), o, i] = -kappa * (np.eye(4) + g)
    return W


@pytest.mark.parametrize("bc", [(1, 1, 1, -1), (1, 1, 1, 1)])
def test_delta_weights_give_wilson_operator(bc):
    """Nearest-neighbour delta weights reproduce the Wilson hopping term: the
    layer equals the C oracle's D at c_sw = 0 (A = 1)."""
    dims = DIMS
    kappa = 0.13
    U = synth.gauge_field(dims, 0.5, 4)
    A = oracle.clover(U, dims, kappa, 0.0)
    T = nn.transports(U, dims, bc)
    psi = synth.random_spinor(int(np.prod(dims)), 1, 5)[0]
    out = nn.layer_forward(T, dims, _wilson_weights(kappa), psi[None])[0]
    ref = oracle.dirac(U, A, dims, bc, kappa, psi)
    assert np.abs(out - ref).max() < 1e-13 * np.abs(ref).max()


def test_three_layers_compose():
    """Channel routing through 1 -> C -> C -> 1: identity, Wilson, Wilson in
    channel 1 (other channels zero) give D_W^2."""
    dims = DIMS
    kappa = 0.11
    bc = (1, 1, 1, -1)
    C = 3
    U = synth.gauge_field(dims, 0.4, 6)
    A = oracle.clover(U, dims, kappa, 0.0)
    T = nn.transports(U, dims, bc)
    W1 = np.zeros((nn.NOFF, C, 1, 4, 4), dtype=np.complex128)
    W1[40, 1, 0] = np.eye(4)
    W2 = _wilson_weights(kappa, C, C, 2, 1)
    W3 = _wilson_weights(kappa, 1, C, 0, 2)
    psi = synth.random_spinor(int(np.prod(dims)), 1, 7)[0]
    out = nn.apply(T, dims, [W1, W2, W3], psi)
    ref = oracle.dirac(U, A, dims, bc, kappa, oracle.dirac(U, A, dims, bc, kappa, psi))
    assert np.abs(out - ref).max() < 1e-13 * np.abs(ref).max()


def test_gauge_covariance():
    """N[U^Om](Om r) = Om N[U](r) for random weights and a random transform."""
    dims = DIMS
    bc = (1, 1, 1, -1)
    V = int(np.prod(dims))
    rng = np.random.default_rng(8)
    C = 2
    Ws = [_rand_layer(rng, C, 1), _rand_layer(rng, C, C), _rand_layer(rng, 1, C)]
    U = synth.gauge_field(dims, 0.6, 9)
    Om = synth.random_su3(V, 10)
    r = synth.random_spinor(V, 1, 11)[0]
    out = nn.apply(nn.transports(U, dims, bc), dims, Ws, r)
    Ug = oracle.gauge_transform(U, dims, Om)
    rg = np.einsum("xab,xsb->xsa", Om, r)
    outg = nn.apply(nn.transports(Ug, dims, bc), dims, Ws, rg)
    ref = np.einsum("xab,xsb->xsa", Om, out)
    assert np.abs(outg - ref).max() < 1e-11 * np.abs(ref).max()


def test_axis_ordered_path():
    """The transporter of d = (+1, +1, 0, 0) takes the x hop first: with unit
    links except U_y(x0 + x^) = R, a source at x0 + d reaches x0 as R psi (the
    y-first path would see only unit links)."""
    dims = DIMS
    U = _unit_links(dims)
    R = synth.random_su3(1, 12)[0]
    x0 = (0, 1, 2, 1)
    U[_site(dims, x0[0] + 1, x0[1], x0[2], x0[3]), 1] = R
    T = nn.transports(U, dims, (1, 1, 1, 1))
    W = np.zeros((nn.NOFF, 1, 1, 4, 4), dtype=np.complex128)
    W[nn.offset_index((1, 1, 0, 0)), 0, 0] = np.eye(4)
    V = int(np.prod(dims))
    psi = np.zeros((V, 4, 3), dtype=np.complex128)
    u = synth.random_spinor(1, 1, 13)[0, 0]
    psi[_site(dims, x0[0] + 1, x0[1] + 1, x0[2], x0[3])] = u
    out = nn.layer_forward(T, dims, W, psi[None])[0]
    s0 = _site(dims, *x0)
    assert np.abs(out[s0] - u @ R.T).max() < 1e-14
    # the y-first path from x0 would pass U_y(x0) = 1 and U_x(x0 + y^) = 1
    assert np.abs(out[s0] - u).max() > 0.1
    # every other site sees only unit links or no source
    mask = np.ones(V, dtype=bool)
    mask[s0] = False
    assert np.abs(out[mask]).max() < 1e-15


def test_boundary_phase_on_diagonal_path():
    """A diagonal offset whose t hop crosses the wrap picks up bc[3] once."""
    dims = DIMS
    U = _unit_links(dims)
    T_anti = nn.transports(U, dims, (1, 1, 1, -1))
    Lx, Ly, Lz, Lt = dims
    k = nn.offset_index((1, 0, -1, 1))
    for s in range(int(np.prod(dims))):
        t = s // (Lx * Ly * Lz)
        expect = -1.0 if t == Lt - 1 else 1.0
        assert np.abs(T_anti[k, s] - expect * np.eye(3)).max() < 1e-15


def test_gradients_finite_difference():
    """dL/dRe W and dL/dIm W against central differences of the loss, for
    entries of all three layers (so the input gradients of layers 2 and 3
    are exercised too)."""
    dims = (2, 3, 2, 3)
    bc = (1, 1, 1, -1)
    V = int(np.prod(dims))
    rng = np.random.default_rng(14)
    C = 2
    Ws = [0.3 * _rand_layer(rng, C, 1), 0.05 * _rand_layer(rng, C, C), 0.05 * _rand_layer(rng, 1, C)]
    U = synth.gauge_field(dims, 0.7, 15)
    T = nn.transports(U, dims, bc)
    R = synth.random_spinor(V, 2, 16)
    E = synth.random_spinor(V, 2, 17)
    loss, G = nn.loss_and_grad(T, dims, Ws, R, E)
    h = 1e-6
    for li in range(3):
        for _ in range(4):
            idx = tuple(int(rng.integers(0, s)) for s in Ws[li].shape)
            for unit, part in ((1.0, np.real), (1j, np.imag)):
                Wp = [w.copy() for w in Ws]
                Wm = [w.copy() for w in Ws]
                Wp[li][idx] += unit * h
                Wm[li][idx] -= unit * h
                lp, _ = nn.loss_and_grad(T, dims, Wp, R, E)
                lm, _ = nn.loss_and_grad(T, dims, Wm, R, E)
                fd = (lp - lm) / (2 * h)
                assert abs(fd - part(G[li][idx])) < 1e-6 * max(1.0, abs(fd)), (li, idx, fd, G[li][idx])


def test_linear_and_pack_roundtrip():
    dims = (2, 2, 3, 2)
    bc = (1, 1, 1, -1)
    V = int(np.prod(dims))
    Ws = nn.init_weights(2, 18)
    flat = nn.pack_weights(Ws)
    assert flat.size == 2 * nn.NOFF * 16 * (2 + 4 + 2)
    back = nn.unpack_weights(flat, 2)
    assert all(np.array_equal(a, b) for a, b in zip(Ws, back))
    T = nn.transports(synth.gauge_field(dims, 0.5, 19), dims, bc)
    r1, r2 = synth.random_spinor(V, 2, 20)
    a, b = 0.7 - 0.2j, -1.3 + 0.4j
    lhs = nn.apply(T, dims, Ws, a * r1 + b * r2)
    rhs = a * nn.apply(T, dims, Ws, r1) + b * nn.apply(T, dims, Ws, r2)
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()
