"""GPU parity of the even-odd stencil launches, element by element, against the
oracle's even-odd pieces on the same inputs.

The solvers invert D (and D_Lambda) through the Schur complement of the even
sites, M = 1 - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe, so every production solve
runs these launches: the two halves of M (the second with the fused
reductions of the BiCGStab iteration), the even-odd source and the odd
reconstruction.  They are checked here at the solver's launch shapes (1 to 64
right-hand sides per launch, LDS staging of links and A^-1 on and off, FP64,
FP32 and BF16 storage, full and domain-restricted operator) and at the
benchmark's lattices, 16^3 x 32 and 24^3 x 48, with 64 right-hand sides per
launch.  Inputs are rounded to the storage precision before both sides see
them, so the differences are the kernel's arithmetic and its output rounding:
  FP64  1e-13 of max|ref|;
  FP32  2e-6  (FP32 arithmetic over the eight hops and the 6x6 blocks);
  BF16  4e-3  (the output is rounded to BF16: unit roundoff 2^-8 = 3.9e-3).
The fused sums are formed in the arithmetic precision before that rounding,
so they are held to 1e-12 (FP64) and 2e-5 (FP32 arithmetic) of |a| |b|.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)
TOL = {0: 1e-13, 1: 2e-6, 2: 4e-3}
SUM_TOL = {0: 1e-12, 1: 2e-5, 2: 2e-5}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def disco():
    import paper_2609_37049_amd as d
    d.lib()
    return d


def _pieces(disco, kappa):
    """(name, parity, ca, cg, cb, epi): the launches of the even-odd solvers."""
    all4 = disco.EPI_DOTAUX | disco.EPI_NORM | disco.EPI_DOTIN | disco.EPI_DOTAUXIN
    return [
        ("hop A_oo^-1 H_oe", 1, 0.0, 0.0, 1.0, 0),
        ("Schur 1 - k^2 A_ee^-1 H_eo (.) with <rh, v>", 0, 1.0, 0.0, -kappa * kappa, disco.EPI_DOTAUX),
        ("Schur with the four sums", 0, 1.0, 0.0, -kappa * kappa, all4),
        ("Schur with norm and <t, s>", 0, 1.0, 0.0, -kappa * kappa, disco.EPI_NORM | disco.EPI_DOTIN),
        ("source A_ee^-1 (r_e + k H_eo u_o)", 0, 0.0, 1.0, kappa, 0),
        ("reconstruction A_oo^-1 (r_o + k H_oe e_e)", 1, 0.0, 1.0, kappa, 0),
    ]


def _round(t, prec, disco):
    """Round a complex128 torch tensor to the storage precision (in place of a copy)."""
    import torch
    if prec == disco.F32:
        return t.to(torch.complex64).to(torch.complex128)
    if prec == disco.BF16:
        re = t.real.to(torch.float32).to(torch.bfloat16).to(torch.float64)
        im = t.imag.to(torch.float32).to(torch.bfloat16).to(torch.float64)
        return torch.complex(re, im)
    return t


def _check_pieces(disco, ctx, U, A, Ainv, dims, kappa, cut, dom, prec, n, seed, lanes, tag, production_only=False):
    V = ctx.V
    psi = _round(synth.random_spinor_device(V, n, seed), prec, disco)
    aux = _round(synth.random_spinor_device(V, n, seed + 1), prec, disco)
    aux2 = _round(synth.random_spinor_device(V, n, seed + 2), prec, disco)
    psi_h = psi[lanes].cpu().numpy()
    aux_h = aux[lanes].cpu().numpy()
    aux2_h = aux2[lanes].cpu().numpy()
    par = oracle.site_parity(dims)
    worst = {}
    refs_by_coef = {}
    for name, p, ca, cg, cb, epi in _pieces(disco, kappa):
        if production_only and epi == disco.EPI_NORM | disco.EPI_DOTIN:
            continue   # an epilogue the even-odd solvers do not launch
        out_t, sums = ctx.dirac_eo_apply(psi, p, ca, cg, cb, prec, dom, aux, aux2, epi)
        out = out_t[lanes].cpu().numpy()
        del out_t
        key = (p, ca, cg, cb)
        if key not in refs_by_coef:
            refs_by_coef[key] = oracle.eo_piece(U, A, dims, BC, kappa, p, ca, cg, cb, psi_h, aux_h, cut, Ainv)
        ref = refs_by_coef[key]
        err = np.abs(out - ref).max() / np.abs(ref).max()
        worst[name] = err
        assert err < TOL[prec], (tag, name, err)
        assert np.abs(out[:, par != p]).max() == 0, (tag, name, "written off its parity")
        if epi:
            on = (par == p)[None, :, None, None]
            ax = np.where(on, aux_h, 0)
            a2 = np.where(on, aux2_h, 0)
            refs = {disco.EPI_DOTAUX: (0, np.einsum("rsac,rsac->r", a2.conj(), ref)),
                    disco.EPI_NORM: (1, np.einsum("rsac,rsac->r", ref.conj(), ref)),
                    disco.EPI_DOTIN: (2, np.einsum("rsac,rsac->r", ref.conj(), ax)),
                    disco.EPI_DOTAUXIN: (3, np.einsum("rsac,rsac->r", a2.conj(), ax))}
            nrm = lambda z: np.sqrt(np.einsum("rsac,rsac->r", z.conj(), z).real)
            scale = {0: nrm(a2) * nrm(ref), 1: nrm(ref) ** 2, 2: nrm(ref) * nrm(ax), 3: nrm(a2) * nrm(ax)}
            for bit, (slot, rv) in refs.items():
                got = sums[lanes, slot]
                if epi & bit:
                    e = np.abs(got - rv) / scale[slot]
                    assert e.max() < SUM_TOL[prec], (tag, name, slot, e.max())
                else:
                    assert np.abs(got).max() == 0
    _say("  %s: %s" % (tag, ", ".join("%s %.1e" % (k.split(" ")[0], v) for k, v in worst.items())))


SMALL = (6, 6, 6, 4)   # 432 sites per parity: a ragged last block for 1, 3 and 8 right-hand sides
SHAPES = [(0, 1, 0), (0, 3, 0), (0, 64, 0), (1, 1, 0), (1, 8, 0), (1, 8, 1), (1, 64, 0), (1, 64, 1),
          (2, 3, 0), (2, 8, 1), (2, 64, 0), (2, 64, 1)]


@pytest.fixture(scope="module")
def small(disco):
    dims, kappa, csw = SMALL, 0.13, 1.4
    U = synth.gauge_field(dims, 0.5, 81)
    ctx = disco.Context(dims, BC)
    ctx.gauge_set(U)
    ctx.clover_setup(kappa, csw)
    A = oracle.clover(U, dims, kappa, csw)
    cut = synth.offset_tiling_cuts(dims, (4, 4, 2, 2))
    return dims, kappa, U, A, np.linalg.inv(A), ctx, cut, ctx.domains(cut)


@pytest.mark.parametrize("prec,n,stage", SHAPES)
@pytest.mark.parametrize("masked", [False, True])
def test_even_odd_pieces_small(disco, small, prec, n, stage, masked):
    dims, kappa, U, A, Ainv, ctx, cut, dom = small
    _say("even-odd pieces", dims, "prec", prec, "n", n, "stage", stage, "masked", masked)
    ctx.set_option(disco.OPT_STAGE, stage)
    try:
        _check_pieces(disco, ctx, U, A, Ainv, dims, kappa, cut if masked else None, dom if masked else None,
                      prec, n, 900 + 7 * n + prec, list(range(n)), "small n=%d" % n)
    finally:
        ctx.set_option(disco.OPT_STAGE, -1)


def test_even_odd_rejects_what_it_does_not_launch(disco, small):
    dims, kappa, U, A, Ainv, ctx, cut, dom = small
    psi = synth.random_spinor_device(ctx.V, 2, 5)
    with pytest.raises(disco.DiscoError) as e:
        ctx.dirac_eo_apply(psi, 0, 1.0, 0.0, 1.0, disco.F32, None, None, None, 0)   # ca needs aux
    assert e.value.code == disco.EINVAL
    with pytest.raises(disco.DiscoError) as e:
        ctx.dirac_eo_apply(psi, 2, 0.0, 0.0, 1.0, disco.F32)
    assert e.value.code == disco.EINVAL
    with pytest.raises(disco.DiscoError) as e:
        ctx.dirac_eo_apply(psi, 0, 1.0, 0.0, 1.0, disco.F32, None, psi, psi, disco.EPI_NORM)  # not a solver epilogue
    assert e.value.code == disco.EINVAL
    odd = disco.Context((4, 4, 4, 3), BC)
    odd.gauge_set(synth.gauge_field((4, 4, 4, 3), 0.3, 3))
    odd.clover_setup(0.12, 1.0)
    with pytest.raises(disco.DiscoError) as e:
        odd.dirac_eo_apply(synth.random_spinor_device(odd.V, 1, 6), 0, 0.0, 0.0, 1.0, disco.F64)
    assert e.value.code == disco.EINVAL


def _bench_lattice(disco, name):
    pre = synth.PRESETS[name]
    U = synth.gauge_field(pre.dims, pre.eps, pre.seed)
    ctx = disco.Context(pre.dims, BC)
    ctx.gauge_set(U)
    ctx.clover_setup(pre.kappa, pre.csw)
    A = oracle.clover(U, pre.dims, pre.kappa, pre.csw)
    return pre, U, A, np.linalg.inv(A), ctx


@pytest.mark.timeout(900)
def test_even_odd_pieces_16x16x16x32_all_lanes(disco):
    """The precision workload's lattice with the solver's 64-wide block: every
    lane of every piece, D and D_Lambda (4^3 x 8 domains)."""
    pre, U, A, Ainv, ctx = _bench_lattice(disco, "prec_16x16x16x32")
    cut = synth.tiling_cuts(pre.dims, pre.block)
    dom = ctx.domains(cut)
    for prec in (disco.BF16, disco.F32):
        for masked in (False, True):
            _say("even-odd pieces 16x16x16x32, 64 rhs, prec", prec, "masked", masked)
            _check_pieces(disco, ctx, U, A, Ainv, pre.dims, pre.kappa, cut if masked else None,
                          dom if masked else None, prec, 64, 300 + prec, list(range(64)),
                          "16x16x16x32 prec %d masked %d" % (prec, masked), production_only=True)


@pytest.mark.timeout(900)
def test_even_odd_pieces_24x24x24x48_sampled_lanes(disco):
    """The batching workload's lattice (half-lattice vectors of 1 GB at 64 BF16
    right-hand sides, beyond the Infinity Cache) in the solver's 64-wide launch:
    every site of a sample of lanes, D and D_Lambda on the uneven 6x6x8x12
    tiling with edge remainders."""
    pre, U, A, Ainv, ctx = _bench_lattice(disco, "batch_24x24x24x48")
    cut = synth.offset_tiling_cuts(pre.dims, pre.block)
    dom = ctx.domains(cut)
    lanes = [0, 1, 31, 32, 63]
    for prec in (disco.BF16, disco.F32):
        for masked in (False, True):
            _say("even-odd pieces 24x24x24x48, 64 rhs, prec", prec, "masked", masked)
            _check_pieces(disco, ctx, U, A, Ainv, pre.dims, pre.kappa, cut if masked else None,
                          dom if masked else None, prec, 64, 400 + prec, lanes,
                          "24x24x24x48 prec %d masked %d" % (prec, masked), production_only=True)
