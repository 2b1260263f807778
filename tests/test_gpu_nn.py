"""GPU parity of the learned preconditioner.

The network's forward and backward kernels (BF16 activations and transported
inputs, BF16 weights on the matrix cores, FP32 accumulation) against the
oracle's FP64 network; training on solver-generated pairs; FGMRES with the
trained network judged by the oracle's FP64 true residual; and the gain of
the trained network over the untrained one at equal cost per iteration.

Tolerance: every product on the matrix cores takes BF16 operands (relative
rounding error <= 2^-9 each, RMS ~1.1e-3), summed in FP32.  Through three
layers the relative L2 error of the output stays at a few 1e-3; the tests
allow 1.5e-2 (forward) and 3e-2 (gradients, one more rounded operand)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import nn

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)
DIMS = (4, 4, 4, 4)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def disco():
    import paper_2609_37049_amd as d
    d.lib()
    return d


@pytest.fixture(scope="module")
def small(disco):
    U = synth.gauge_field(DIMS, 0.4, 31)
    ctx = disco.Context(DIMS, BC)
    ctx.gauge_set(U)
    ctx.clover_setup(0.12, 1.0)
    T = nn.transports(U, DIMS, BC)
    return ctx, U, T


def _rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def test_forward_matches_oracle(disco, small):
    ctx, U, T = small
    _say("net forward 4^4, random weights")
    Ws = nn.init_weights(16, 3)
    net = disco.Net(ctx, 16, 1)
    net.set_weights(nn.pack_weights(Ws))
    r = synth.random_spinor(ctx.V, 2, 32)
    out = net.apply(ctx.dev(r)).cpu().numpy()
    for p in range(2):
        ref = nn.apply(T, DIMS, Ws, r[p])
        err = _rel(out[p], ref)
        _say("  rhs %d: rel L2 error %.2e" % (p, err))
        assert err < 1.5e-2


def test_delta_weights_give_wilson_squared(disco, small):
    """Layers identity -> Wilson -> Wilson (channel 1 and 2) make the network
    D_W^2 (c_sw = 0), compared with the C oracle's operator."""
    ctx, U, T = small
    kappa = 0.125
    C = 16
    W1 = np.zeros((nn.NOFF, C, 1, 4, 4), dtype=np.complex128)
    W1[40, 1, 0] = np.eye(4)
    W2 = np.zeros((nn.NOFF, C, C, 4, 4), dtype=np.complex128)
    W3 = np.zeros((nn.NOFF, 1, C, 4, 4), dtype=np.complex128)
    for W, o, i in ((W2, 2, 1), (W3, 0, 2)):
        W[40, o, i] = np.eye(4)
        for mu in range(4):
            g = oracle.gamma(mu)
            e = [0, 0, 0, 0]
            e[mu] = 1
            W[nn.offset_index(e), o, i] = -kappa * (np.eye(4) - g)
            e[mu] = -1
            W[nn.offset_index(e), o, i] = -kappa * (np.eye(4) + g)
    net = disco.Net(ctx, 16, 1)
    net.set_weights(nn.pack_weights([W1, W2, W3]))
    r = synth.random_spinor(ctx.V, 1, 33)
    out = net.apply(ctx.dev(r)).cpu().numpy()[0]
    A = oracle.clover(U, DIMS, kappa, 0.0)
    ref = oracle.dirac(U, A, DIMS, BC, kappa, oracle.dirac(U, A, DIMS, BC, kappa, r[0]))
    err = _rel(out, ref)
    _say("net = D_W^2: rel L2 error %.2e" % err)
    assert err < 1e-2


def test_backward_matches_oracle(disco, small):
    ctx, U, T = small
    _say("net backward 4^4, random weights")
    Ws = nn.init_weights(16, 4)
    net = disco.Net(ctx, 16, 1)
    net.set_weights(nn.pack_weights(Ws))
    n = 2
    r = synth.random_spinor(ctx.V, n, 34)
    go = synth.random_spinor(ctx.V, n, 35)
    gw, gi = net.backward(ctx.dev(r), ctx.dev(go))
    gw = nn.unpack_weights(gw.cpu().numpy(), 16)
    gi = gi.cpu().numpy()
    G = [np.zeros_like(W) for W in Ws]
    for p in range(n):
        acts = nn.forward(T, DIMS, Ws, r[p])
        g = go[p][None]
        for li in (2, 1, 0):
            GW, g = nn.layer_backward(T, DIMS, Ws[li], acts[li], g)
            G[li] += GW
        e = _rel(gi[p], g[0])
        _say("  grad_in rhs %d: rel L2 error %.2e" % (p, e))
        assert e < 3e-2
    for li in range(3):
        e = _rel(gw[li], G[li])
        _say("  grad_w layer %d: rel L2 error %.2e" % (li, e))
        assert e < 3e-2


@pytest.fixture(scope="module")
def medium(disco):
    dims = (8, 8, 8, 8)
    U = synth.gauge_field(dims, 0.3, 41)
    ctx = disco.Context(dims, BC)
    ctx.gauge_set(U)
    ctx.clover_setup(0.12, 1.0)
    A = oracle.clover(U, dims, 0.12, 1.0)
    return dims, ctx, U, A


@pytest.fixture(scope="module")
def trained(disco, medium):
    dims, ctx, U, A = medium
    _say("training the network on 8^4 (32 pairs, 80 steps)")
    net = disco.Net(ctx, 16, 7)
    st = net.train(32, snap_iters=(0, 8, 24, 64), batch=4, steps=80, lr=2e-3, seed=5)
    _say("  loss %.4f -> %.4f (pairs %d, gen %.2f s, train %.2f s)" % (st.first_loss, st.final_loss, st.pairs,
                                                                       st.gen_seconds, st.train_seconds))
    return net, st


def test_training_lowers_loss(trained):
    net, st = trained
    assert st.pairs == 32 and st.steps == 80
    assert np.isfinite(st.final_loss)
    assert st.final_loss < 0.8 * st.first_loss


def _true_res(U, A, dims, kappa, b, x, cut=None):
    r = b - oracle.dirac(U, A, dims, BC, kappa, x, cut)
    return np.linalg.norm(r) / np.linalg.norm(b)


@pytest.mark.parametrize("tol", [1e-10, 1e-12])
def test_fgmres_nn_converges(disco, medium, trained, tol):
    dims, ctx, U, A = medium
    net, _ = trained
    b = synth.random_spinor(ctx.V, 3, 42)
    P = ctx.params(method=disco.FGMRES_NN, tol=tol, net=net, restart=16, rhs_block=3)
    x, st = ctx.solve_multi_rhs(ctx.dev(b), P)
    x = x.cpu().numpy()
    for k in range(3):
        res = _true_res(U, A, dims, 0.12, b[k], x[k])
        _say("  fgmres-nn tol %.0e rhs %d: %d Arnoldi steps, %d cycles, reported %.2e, oracle %.2e, fallback %d" %
             (tol, k, st[k].iters, st[k].outer_iters, st[k].true_rel_residual, res, st[k].fallback_used))
        assert st[k].converged
        assert res <= tol * 1.05
        assert abs(res - st[k].true_rel_residual) <= max(1e-2 * res, 2e-15)


def test_fgmres_nn_block_operator(disco, medium, trained):
    """D_Lambda solves with the (full-lattice) network as preconditioner: the
    flexible outer iteration still converges on the restricted system."""
    dims, ctx, U, A = medium
    net, _ = trained
    cut = synth.tiling_cuts(dims, (4, 4, 4, 4))
    dom = ctx.domains(cut)
    b = synth.random_spinor(ctx.V, 2, 43)
    P = ctx.params(method=disco.FGMRES_NN, tol=1e-10, net=net, rhs_block=2)
    x, st = ctx.solve_multi_rhs(ctx.dev(b), P, dom)
    x = x.cpu().numpy()
    for k in range(2):
        res = _true_res(U, A, dims, 0.12, b[k], x[k], cut)
        _say("  fgmres-nn block rhs %d: %d steps, oracle residual %.2e" % (k, st[k].iters, res))
        assert res <= 1.05e-10


def test_fgmres_nn_fallback(disco, medium):
    """A network that returns zero makes every FGMRES cycle stall; the FP64
    CGNR fallback then finishes the solve and the FP64 residual judges it."""
    dims, ctx, U, A = medium
    dead = disco.Net(ctx, 16, 1)
    dead.set_weights(np.zeros(dead.nw, dtype=np.float32))
    b = synth.random_spinor(ctx.V, 1, 44)
    P = ctx.params(method=disco.FGMRES_NN, tol=1e-10, net=dead, fallback=1)
    x, st = ctx.solve_multi_rhs(ctx.dev(b), P)
    res = _true_res(U, A, dims, 0.12, b[0], x.cpu().numpy()[0])
    _say("  fallback: used %d, oracle residual %.2e" % (st[0].fallback_used, res))
    assert st[0].fallback_used == 1
    assert res <= 1.05e-10
    P0 = ctx.params(method=disco.FGMRES_NN, tol=1e-10, net=dead, fallback=0)
    with pytest.raises(disco.DiscoError):
        ctx.solve_multi_rhs(ctx.dev(b), P0)


def test_gain_of_trained_network(disco, medium, trained):
    """Same FGMRES(16), same cost per step: the trained network against the
    untrained one (identity through channel 0 plus noise, i.e. essentially
    unpreconditioned FGMRES).  The gain is the ratio of Arnoldi steps."""
    dims, ctx, U, A = medium
    net, _ = trained
    fresh = disco.Net(ctx, 16, 7)
    b = ctx.dev(synth.random_spinor(ctx.V, 4, 45))
    steps = {}
    for name, m in (("trained", net), ("untrained", fresh)):
        P = ctx.params(method=disco.FGMRES_NN, tol=1e-10, net=m, restart=16, rhs_block=4)
        x, st = ctx.solve_multi_rhs(b, P)
        steps[name] = st[0].iters
        assert all(s.converged for s in st)
    _say("  Arnoldi steps to 1e-10: trained %d, untrained %d (gain %.2fx)" %
         (steps["trained"], steps["untrained"], steps["untrained"] / max(1, steps["trained"])))
    assert steps["trained"] < steps["untrained"]


def test_training_over_ensembles_generalises(disco):
    """Pairs from two seeded ensembles (training continues across gauge fields
    with the transporters re-tabulated), evaluated on a held-out ensemble:
    the trained network still beats the untrained one there."""
    dims = (8, 8, 8, 8)
    kappa, csw = 0.12, 1.0
    ctx = disco.Context(dims, BC)
    net = None
    for seed in (71, 72):
        ctx.gauge_set(synth.gauge_field(dims, 0.3, seed))
        ctx.clover_setup(kappa, csw)
        if net is None:
            net = disco.Net(ctx, 16, 9)
        else:
            net.refresh()
        st = net.train(32, snap_iters=(0, 8, 24, 64), batch=4, steps=60, lr=2e-3, seed=seed)
        _say("  ensemble %d: loss %.4f -> %.4f" % (seed, st.first_loss, st.final_loss))
    ctx.gauge_set(synth.gauge_field(dims, 0.3, 73))
    ctx.clover_setup(kappa, csw)
    net.refresh()
    fresh = disco.Net(ctx, 16, 9)
    b = ctx.dev(synth.random_spinor(ctx.V, 2, 74))
    steps = {}
    for name, m in (("trained", net), ("untrained", fresh)):
        P = ctx.params(method=disco.FGMRES_NN, tol=1e-10, net=m, rhs_block=2)
        _, st = ctx.solve_multi_rhs(b, P)
        assert all(s.converged for s in st)
        steps[name] = st[0].iters
    _say("  held-out ensemble: trained %d, untrained %d Arnoldi steps" % (steps["trained"], steps["untrained"]))
    assert steps["trained"] < steps["untrained"]


# ---- at the size the benchmark runs the network (16^3 x 32)
FULL = (16, 16, 16, 32)


def _wilson_squared_weights(kappa, C=16):
    W1 = np.zeros((nn.NOFF, C, 1, 4, 4), dtype=np.complex128)
    W1[40, 1, 0] = np.eye(4)
    W2 = np.zeros((nn.NOFF, C, C, 4, 4), dtype=np.complex128)
    W3 = np.zeros((nn.NOFF, 1, C, 4, 4), dtype=np.complex128)
    for W, o, i in ((W2, 2, 1), (W3, 0, 2)):
        W[40, o, i] = np.eye(4)
        for mu in range(4):
            g = oracle.gamma(mu)
            e = [0, 0, 0, 0]
            e[mu] = 1
            W[nn.offset_index(e), o, i] = -kappa * (np.eye(4) - g)
            e[mu] = -1
            W[nn.offset_index(e), o, i] = -kappa * (np.eye(4) + g)
    return [W1, W2, W3]


def test_delta_weights_give_wilson_squared_full_size(disco):
    """The network with delta weights is D_W^2 (c_sw = 0) on the full 16^3 x 32
    lattice of the benchmark, compared with the C oracle's operator applied
    twice to the same two right-hand sides (8 per launch as in the solver)."""
    kappa = 0.125
    U = synth.gauge_field(FULL, 0.25, 2)
    ctx = disco.Context(FULL, BC)
    ctx.gauge_set(U)
    ctx.clover_setup(kappa, 0.0)
    net = disco.Net(ctx, 16, 1)
    net.set_weights(nn.pack_weights(_wilson_squared_weights(kappa)))
    r = synth.random_spinor(ctx.V, 8, 34)
    out = net.apply(ctx.dev(r)).cpu().numpy()
    A = oracle.clover(U, FULL, kappa, 0.0)
    for p in (0, 7):
        ref = oracle.dirac(U, A, FULL, BC, kappa, oracle.dirac(U, A, FULL, BC, kappa, r[p]))
        err = _rel(out[p], ref)
        _say("net = D_W^2 at 16^3x32, rhs %d: rel L2 error %.2e" % (p, err))
        assert err < 1e-2
    net.close()


def test_gauge_covariance_full_size(disco):
    """With random weights on the full 16^3 x 32 lattice: N[U^g](g r) = g N[U](r)
    for a random SU(3) transform g, to the BF16 accuracy of two applications
    (each within 1.5e-2 of the exact network)."""
    U = synth.gauge_field(FULL, 0.25, 2)
    V = int(np.prod(FULL))
    Om = synth.random_su3(V, 35)
    ctx = disco.Context(FULL, BC)
    ctx.gauge_set(U)
    ctx.clover_setup(0.125, 1.5)
    net = disco.Net(ctx, 16, 1)
    net.set_weights(nn.pack_weights(nn.init_weights(16, 36)))
    r = synth.random_spinor(V, 2, 37)
    out = net.apply(ctx.dev(r)).cpu().numpy()
    ctx.gauge_set(oracle.gauge_transform(U, FULL, Om))
    net.refresh()
    rg = np.einsum("xab,pxsb->pxsa", Om, r)
    outg = net.apply(ctx.dev(rg)).cpu().numpy()
    for p in range(2):
        ref = np.einsum("xab,xsb->xsa", Om, out[p])
        err = _rel(outg[p], ref)
        _say("gauge covariance at 16^3x32, rhs %d: rel L2 difference %.2e" % (p, err))
        assert err < 3e-2
    net.close()
