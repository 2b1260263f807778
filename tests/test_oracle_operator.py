"""Pins of the oracle's operator against what the mathematics fixes.

Each test checks the CPU oracle against something other than itself: the
gamma algebra, closed forms on gauge fields with a known answer, operator
identities, and dense LAPACK linear algebra.  A dropped term, a wrong sign or
index, or a transposed operand in the oracle fails at least one of them.
"""
import numpy as np
import pytest

import oracle
import synth
from lattice_fixtures import abelian_flux_field, unit_field, coords, momenta

BC = (1, 1, 1, -1)


def test_gamma_algebra():
    g = [oracle.gamma(m) for m in range(5)]
    for a in range(4):
        assert np.allclose(g[a], g[a].conj().T)
        for b in range(4):
            assert np.allclose(g[a] @ g[b] + g[b] @ g[a], 2 * np.eye(4) * (a == b), atol=1e-15)
    # chiral basis: gamma_5 diagonal, +1 on the upper two spins
    assert np.allclose(g[4], np.diag([1, 1, -1, -1]))
    # time gamma is the off-diagonal identity
    assert np.allclose(g[3], np.block([[np.zeros((2, 2)), np.eye(2)], [np.eye(2), np.zeros((2, 2))]]))


def test_clover_unit_field_is_identity():
    dims = (2, 2, 2, 4)
    A = oracle.clover(unit_field(dims), dims, 0.13, 1.7)
    assert np.abs(A - np.eye(12)[None]).max() < 1e-15


@pytest.mark.parametrize("mu,nu", [(0, 1), (0, 3), (1, 2), (2, 3)])
def test_clover_constant_abelian_flux(mu, nu):
    """Constant flux theta through every (mu,nu) plaquette: each leaf is
    exp(i theta H), so Fhat = i sin(theta H) and
    A = 1 - csw kappa sigma_mu_nu (x) sin(theta H) (closed form)."""
    dims = (4, 4, 4, 4)
    U, theta = abelian_flux_field(dims, mu, nu, 1)
    kappa, csw = 0.12, 1.3
    A = oracle.clover(U, dims, kappa, csw)
    g = [oracle.gamma(m) for m in range(4)]
    sig = 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])
    Fh = np.diag(np.sin(theta * np.array([1.0, -1.0, 0.0])))
    expect = np.eye(12) - csw * kappa * np.kron(sig, Fh)
    assert np.abs(A - expect[None]).max() < 1e-14


def test_clover_hermitian_commutes_g5_covariant():
    dims = (4, 2, 2, 4)
    U = synth.gauge_field(dims, 0.6, 11)
    A = oracle.clover(U, dims, 0.11, 1.4)
    assert np.abs(A - np.conj(np.swapaxes(A, 1, 2))).max() < 1e-15
    G5 = np.kron(oracle.gamma(4), np.eye(3))
    assert np.abs(A @ G5 - G5 @ A).max() < 1e-15
    V = int(np.prod(dims))
    Om = synth.random_su3(V, 12)
    A2 = oracle.clover(oracle.gauge_transform(U, dims, Om), dims, 0.11, 1.4)
    Ob = np.einsum("ab,sij->saibj", np.eye(4), Om).reshape(V, 12, 12)
    assert np.abs(A2 - Ob @ A @ np.conj(np.swapaxes(Ob, 1, 2))).max() < 1e-13


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 4, 2, 6)])
def test_free_field_plane_waves(dims):
    """U = 1: D e^{ipx} u = [1 - 2 kappa sum cos p + 2 i kappa sum gamma sin p] e^{ipx} u,
    with time momenta (2 pi n + pi)/L_t for the antiperiodic direction."""
    kappa = 0.11
    U = unit_field(dims)
    A = oracle.clover(U, dims, kappa, 1.0)
    X = coords(dims)
    g = [oracle.gamma(m) for m in range(4)]
    rng = np.random.default_rng(3)
    moms = momenta(dims, BC)
    for trial in range(4):
        p = [moms[m][rng.integers(len(moms[m]))] for m in range(4)]
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        ph = np.exp(1j * (X @ np.array(p)))
        psi = ph[:, None, None] * u[None]
        M = (1 - 2 * kappa * sum(np.cos(p))) * np.eye(4) + 2j * kappa * sum(g[m] * np.sin(p[m]) for m in range(4))
        expect = ph[:, None, None] * (M @ u)[None]
        out = oracle.dirac(U, A, dims, BC, kappa, psi)
        assert np.abs(out - expect).max() < 1e-13


def test_g5_hermiticity_dense():
    """D^+ = g5 D g5 as a property of the dense matrix (not of the dagger flag)."""
    dims = (2, 2, 2, 4)
    U = synth.gauge_field(dims, 0.6, 5)
    A = oracle.clover(U, dims, 0.11, 1.3)
    D = oracle.dense_dirac(U, A, dims, BC, 0.11)
    G5 = np.kron(np.eye(32), np.kron(oracle.gamma(4), np.eye(3)))
    assert np.abs(D.conj().T - G5 @ D @ G5).max() < 1e-14
    Dd = oracle.dense_dirac(U, A, dims, BC, 0.11, dagger=True)
    assert np.abs(Dd - D.conj().T).max() < 1e-14


def test_gauge_covariance_of_D():
    dims = (4, 2, 4, 2)
    U = synth.gauge_field(dims, 0.5, 7)
    kappa, csw = 0.12, 1.2
    A = oracle.clover(U, dims, kappa, csw)
    V = int(np.prod(dims))
    Om = synth.random_su3(V, 8)
    U2 = oracle.gauge_transform(U, dims, Om)
    A2 = oracle.clover(U2, dims, kappa, csw)
    psi = synth.random_spinor(V, 1, 9)[0]
    lhs = oracle.dirac(U2, A2, dims, BC, kappa, np.einsum("sij,saj->sai", Om, psi))
    rhs = np.einsum("sij,saj->sai", Om, oracle.dirac(U, A, dims, BC, kappa, psi))
    assert np.abs(lhs - rhs).max() < 1e-13


def _domain_ids(dims, cut):
    """Label of the domain of each site, from the cut masks (test helper)."""
    ids = []
    for mu in range(4):
        L = dims[mu]
        lab, cur = [], 0
        for x in range(L):
            lab.append(cur)
            if cut[mu, x] and x != L - 1:
                cur += 1
        # a domain that wraps around (no cut at the wrap face) joins the first
        if not cut[mu, L - 1]:
            last = lab[-1]
            lab = [0 if v == last else v for v in lab]
        ids.append(lab)
    X = coords(dims)
    key = [ids[0][x[0]] + 100 * (ids[1][x[1]] + 100 * (ids[2][x[2]] + 100 * ids[3][x[3]])) for x in X]
    return np.asarray(key)


def test_block_operator_single_domain_equals_D():
    dims = (2, 2, 4, 4)
    U = synth.gauge_field(dims, 0.5, 21)
    A = oracle.clover(U, dims, 0.12, 1.0)
    psi = synth.random_spinor(64, 1, 22)[0]
    cut = np.zeros((4, 4), dtype=np.uint8)
    assert np.abs(oracle.dirac(U, A, dims, BC, 0.12, psi, cut) - oracle.dirac(U, A, dims, BC, 0.12, psi)).max() == 0


@pytest.mark.parametrize("block", [(2, 2, 2, 2), (4, 2, 2, 2), (2, 2, 2, 4), (1, 1, 1, 1)])
def test_block_operator_is_principal_submatrix(block):
    """D_Lambda equals D on pairs of sites in the same domain and is zero
    between domains (block-diagonal principal submatrices)."""
    dims = (4, 2, 2, 4)
    U = synth.gauge_field(dims, 0.5, 31)
    kappa = 0.12
    A = oracle.clover(U, dims, kappa, 1.1)
    cut = synth.tiling_cuts(dims, block)
    D = oracle.dense_dirac(U, A, dims, BC, kappa)
    Db = oracle.dense_dirac(U, A, dims, BC, kappa, cut=cut)
    dom = np.repeat(_domain_ids(dims, cut), 12)
    same = dom[:, None] == dom[None, :]
    assert np.abs(Db[same] - D[same]).max() == 0
    assert np.abs(Db[~same]).max() == 0
    if block == (1, 1, 1, 1):
        # every hop removed: the operator is the clover term alone
        assert np.abs(Db - _blockdiag(A)).max() < 1e-15


def _blockdiag(A):
    V = A.shape[0]
    M = np.zeros((12 * V, 12 * V), dtype=np.complex128)
    for s in range(V):
        M[12 * s:12 * s + 12, 12 * s:12 * s + 12] = A[s]
    return M


def test_offset_tiling_gives_uneven_domains():
    dims = (24, 24, 24, 48)
    cut = synth.offset_tiling_cuts(dims, (6, 6, 8, 12))
    ext = []
    for mu in range(4):
        c = np.flatnonzero(cut[mu, :dims[mu]])
        ext.append(list(np.diff(np.concatenate([[-1], c]))))
    assert ext[0] == [3, 6, 6, 6, 3] and ext[2] == [4, 8, 8, 4] and ext[3] == [6, 12, 12, 12, 6]


def test_cgnr_against_dense_lu():
    dims = (2, 2, 2, 4)
    U = synth.gauge_field(dims, 0.6, 41)
    kappa = 0.12
    A = oracle.clover(U, dims, kappa, 1.2)
    D = oracle.dense_dirac(U, A, dims, BC, kappa)
    b = synth.random_spinor(32, 1, 42)[0]
    x, it, rr = oracle.cgnr(U, A, dims, BC, kappa, b, tol=1e-13)
    xd = np.linalg.solve(D, b.reshape(-1)).reshape(b.shape)
    assert rr <= 1e-13
    assert np.abs(x - xd).max() / np.abs(xd).max() < 1e-11


def test_free_field_propagator_closed_form():
    """U = 1: D^-1(p) = [M - 2 i kappa sum gamma sin p] / [M^2 + 4 kappa^2 sum sin^2 p],
    M = 1 - 2 kappa sum cos p; compared on a plane-wave source."""
    dims = (4, 4, 4, 4)
    kappa = 0.1
    U = unit_field(dims)
    A = oracle.clover(U, dims, kappa, 1.0)
    X = coords(dims)
    g = [oracle.gamma(m) for m in range(4)]
    moms = momenta(dims, BC)
    p = [moms[0][1], moms[1][0], moms[2][3], moms[3][2]]
    u = np.zeros((4, 3), dtype=np.complex128)
    u[1, 2] = 1
    ph = np.exp(1j * (X @ np.array(p)))
    b = ph[:, None, None] * u[None]
    x, _, _ = oracle.cgnr(U, A, dims, BC, kappa, b, tol=1e-13)
    M = 1 - 2 * kappa * sum(np.cos(p))
    S = (M * np.eye(4) - 2j * kappa * sum(g[m] * np.sin(p[m]) for m in range(4))) / (M ** 2 + 4 * kappa ** 2 * sum(np.sin(p) ** 2))
    expect = ph[:, None, None] * (S @ u)[None]
    assert np.abs(x - expect).max() < 1e-12


def test_schur_factorisation_of_propagator():
    """(D^-1)_{LL} = D_L^-1 + D_L^-1 D_dL (D^-1)_{L*L*} D_dL* D_L^-1 with D_L the
    Dirichlet-restricted operator (factorisation equation, read as the block
    inverse), on a temporal slab partition."""
    dims = (2, 2, 2, 4)
    U = synth.gauge_field(dims, 0.6, 51)
    kappa = 0.12
    A = oracle.clover(U, dims, kappa, 1.1)
    cut = synth.tiling_cuts(dims, (2, 2, 2, 2))
    cut[:3] = 0  # temporal slabs only: t in {0,1} and {2,3}
    D = oracle.dense_dirac(U, A, dims, BC, kappa)
    Db = oracle.dense_dirac(U, A, dims, BC, kappa, cut=cut)
    t = coords(dims)[:, 3]
    inL = np.repeat(t < 2, 12)
    L, Ls = np.flatnonzero(inL), np.flatnonzero(~inL)
    Dinv = np.linalg.inv(D)
    DLinv = np.linalg.inv(Db[np.ix_(L, L)])
    rhs = DLinv + DLinv @ D[np.ix_(L, Ls)] @ Dinv[np.ix_(Ls, Ls)] @ D[np.ix_(Ls, L)] @ DLinv
    assert np.abs(Dinv[np.ix_(L, L)] - rhs).max() < 1e-12
    # the restricted operator really is the principal submatrix
    assert np.abs(Db[np.ix_(L, L)] - D[np.ix_(L, L)]).max() == 0


def test_oracle_thread_count_does_not_change_results():
    """The timing helper that runs the oracle on one thread changes no
    arithmetic: D psi is the same bit for bit (sites are independent)."""
    import numpy as np
    import oracle
    import synth
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.3, 1)
    A = oracle.clover(U, dims, 0.12, 1.0)
    rng = np.random.default_rng(3)
    psi = rng.standard_normal((256, 4, 3)) + 1j * rng.standard_normal((256, 4, 3))
    y_all = oracle.dirac(U, A, dims, (1, 1, 1, -1), 0.12, psi)
    old = oracle.set_threads(1)
    try:
        assert old >= 1
        y_one = oracle.dirac(U, A, dims, (1, 1, 1, -1), 0.12, psi)
    finally:
        assert oracle.set_threads(old) == 1
    assert np.array_equal(y_all, y_one)


@pytest.mark.parametrize("with_cut", [False, True])
def test_even_odd_pieces_solve_the_dense_system(with_cut):
    """The oracle's even-odd pieces, composed as the solver composes them, solve
    D x = b (or D_Lambda x = b): x_e from the dense Schur complement
    M = 1 - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe on the source
    A_ee^-1 (b_e + kappa H_eo A_oo^-1 b_o), x_o = A_oo^-1 (b_o + kappa H_oe x_e),
    against a dense LU solve of the whole operator."""
    dims = (2, 2, 2, 4)
    kappa, csw = 0.13, 1.4
    U = synth.gauge_field(dims, 0.5, 61)
    A = oracle.clover(U, dims, kappa, csw)
    cut = None
    if with_cut:
        cut = np.zeros((4, 4), dtype=np.uint8)
        cut[3, 1] = cut[0, 1] = 1
    V = int(np.prod(dims))
    par = oracle.site_parity(dims)
    ev = np.flatnonzero(par == 0)
    b = synth.random_spinor(V, 1, 62)[0]
    piece = lambda p, ca, cg, cb, psi, aux=None: oracle.eo_piece(U, A, dims, BC, kappa, p, ca, cg, cb, psi, aux, cut)
    zero = np.zeros_like(b)
    u_o = piece(1, 0.0, 1.0, 0.0, zero, b)
    rhat = piece(0, 0.0, 1.0, kappa, u_o, b)

    def M(v):
        return piece(0, 1.0, 0.0, -kappa * kappa, piece(1, 0.0, 0.0, 1.0, v), v)
    # dense M on the even sites
    n = 12 * len(ev)
    Md = np.empty((n, n), dtype=np.complex128)
    for j in range(n):
        e = np.zeros_like(b)
        e[ev[j // 12], (j % 12) // 3, j % 3] = 1
        Md[:, j] = M(e)[ev].reshape(-1)
    xe = np.zeros_like(b)
    xe[ev] = np.linalg.solve(Md, rhat[ev].reshape(-1)).reshape(len(ev), 4, 3)
    x = xe + piece(1, 0.0, 1.0, kappa, xe, b)
    D = oracle.dense_dirac(U, A, dims, BC, kappa, cut)
    ref = np.linalg.solve(D, b.reshape(-1)).reshape(V, 4, 3)
    assert np.abs(x - ref).max() < 1e-12 * np.abs(ref).max()
    # and the pieces vanish off their parity
    assert np.abs(rhat[par == 1]).max() == 0 and np.abs(u_o[par == 0]).max() == 0
