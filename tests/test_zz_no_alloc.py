"""The entry point that allocates no device memory, disco_dirac_apply_noalloc,
against disco_dirac_apply through the C ABI: same kernels, so the results are
identical bit for bit, on two calls in a row (the second with fewer right-hand
sides and a smaller lattice), in every storage precision, and sizes beyond its
fixed scratch are refused with a clear error."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def disco():
    import paper_2609_37049_amd as d
    d.lib()
    return d


def _ctx(disco, dims, seed):
    ctx = disco.Context(dims, BC)
    ctx.gauge_set(synth.gauge_field(dims, 0.4, seed))
    ctx.clover_setup(0.124, 1.3)
    return ctx


def test_noalloc_apply_equals_apply(disco):
    big = _ctx(disco, (8, 8, 8, 16), 91)       # 8192 sites: more right-hand sides than one launch
    small = _ctx(disco, (4, 4, 6, 4), 92)      # a second, smaller call after it
    for prec in (disco.F64, disco.F32, disco.BF16):
        for ctx, n, seed in ((big, 70, 93), (small, 3, 94)):
            _say("noalloc apply", ctx.dims, "prec", prec, "nrhs", n)
            psi = ctx.dev(synth.random_spinor(ctx.V, n, seed + prec))
            for dag in (False, True):
                ref = ctx.dirac_apply(psi, prec, dag).cpu().numpy()
                got = ctx.dirac_apply_noalloc(psi, prec, dag).cpu().numpy()
                assert np.array_equal(got, ref), (ctx.dims, prec, n, dag)


def test_noalloc_refuses_what_does_not_fit(disco):
    # 32^3 x 64 in FP64: one right-hand side needs 2 x 403 MB, beyond the 256 MiB scratch
    ctx = disco.Context((32, 32, 32, 64), BC)
    psi = ctx.empty_spinors(1)
    with pytest.raises(disco.DiscoError) as e:
        ctx.dirac_apply_noalloc(psi, disco.F64)
    assert e.value.code == disco.EINVAL and "scratch" in str(e.value)
