"""GPU parity of the clover term and the clover-Wilson operator (paper
Section 2, Eq. (1)) against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from paper_2112_00501_amd import cloversap as cs
from paper_2112_00501_amd import synth
from tests.gpu_helpers import TOL_D, TOL_D_SITE, Case, rel, site_err

pytestmark = pytest.mark.gpu

PRECS = [cs.F64, cs.F32, cs.F16, cs.BF16]


@pytest.fixture(scope="module")
def cfg1():
    return Case((8, 8, 8, 8), 0.3, 0.13, 1.0, 1001)


@pytest.fixture(scope="module")
def wide():
    # four blocks in every direction: the +mu and -mu neighbour blocks differ
    return Case((16, 16, 16, 16), 0.25, 0.137, 1.1, 17)


@pytest.fixture(scope="module")
def ragged():
    # one block in x (the periodic neighbour is the block itself), odd block counts
    return Case((4, 8, 12, 8), 0.3, 0.1355, 1.1, 7)


def test_clover_term_matches_oracle(cfg1, ragged):
    for c in (cfg1, ragged):
        T = c.op.clover.export()
        torch.cuda.synchronize()
        assert np.abs(T.cpu().numpy() - c.T).max() < 1e-14


@pytest.mark.parametrize("dagger", [False, True])
@pytest.mark.parametrize("prec", PRECS)
def test_dslash_parity(cfg1, ragged, wide, prec, dagger):
    for c in (cfg1, ragged, wide):
        psi = synth.source(c.dims, 2001)
        fin = c.to_dev(psi, prec)
        fout = c.lat.new_field(prec)
        (c.op.apply_Ddag if dagger else c.op.apply_D)(fout, fin, prec)
        got = c.to_host(fout, prec)
        ref = (oracle.apply_Ddag if dagger else oracle.apply_D)(c.dims, c.U, c.T, c.kappa, psi)
        err, serr = rel(got, ref), site_err(got, ref)
        print(f"dims={c.dims} prec={prec} dagger={dagger} rel.err={err:.3e} site.err={serr:.3e}")
        assert err <= TOL_D[prec]
        assert serr <= TOL_D_SITE[prec]


def test_dslash_batched_equals_single(cfg1):
    c = cfg1
    psis = synth.source(c.dims, 5, nrhs=3)
    for prec in (cs.F64, cs.F32):
        fin = c.to_dev(psis, prec)
        fout = c.lat.new_field(prec, 3)
        c.op.apply_D(fout, fin, prec, nrhs=3)
        got = c.to_host(fout, prec, 3)
        for r in range(3):
            f1 = c.to_dev(psis[r], prec)
            o1 = c.lat.new_field(prec)
            c.op.apply_D(o1, f1, prec)
            assert np.array_equal(c.to_host(o1, prec), got[r])
