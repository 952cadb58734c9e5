"""GPU parity with antiperiodic boundary conditions in time (fermion fields
with psi(x + L_t e_t) = -psi(x), the usual choice; the paper states none),
through the C ABI's lattice flag, against the oracle, which takes the
boundary condition through its links (U_t negated on the last time slice;
pinned against the free-field spectrum and the periodic operator on the CPU).
Lattices with two and four blocks in time, so that the hop across the
boundary joins the same or a different pair of blocks than the interior
hops."""
import numpy as np
import pytest
import torch

import oracle
from oracle import mg
from paper_2112_00501_amd import cloversap as cs
from paper_2112_00501_amd import synth
from tests.gpu_helpers import TOL_D, TOL_D_SITE, Case, rel, site_err
from tests.test_gpu_mg import dense_from_stencil
from tests.test_gpu_sap import TOL_SAP, TOL_SAP_SITE

pytestmark = pytest.mark.gpu

BDIM = (4, 4, 4, 4)


@pytest.fixture(scope="module")
def ap8():
    return Case((8, 8, 8, 8), 0.3, 0.13, 1.0, 1001, antiperiodic_t=True)


@pytest.fixture(scope="module")
def ap16():
    return Case((8, 8, 8, 16), 0.25, 0.137, 1.1, 19, antiperiodic_t=True)


@pytest.mark.parametrize("dagger", [False, True])
@pytest.mark.parametrize("prec", [cs.F64, cs.F32, cs.F16, cs.BF16])
def test_dslash_antiperiodic(ap8, ap16, prec, dagger):
    for c in (ap8, ap16):
        psi = synth.source(c.dims, 2101)
        fout = c.lat.new_field(prec)
        (c.op.apply_Ddag if dagger else c.op.apply_D)(fout, c.to_dev(psi, prec), prec)
        got = c.to_host(fout, prec)
        fn = oracle.apply_Ddag if dagger else oracle.apply_D
        ref = fn(c.dims, c.Uo, c.T, c.kappa, psi)
        err, serr = rel(got, ref), site_err(got, ref)
        periodic = rel(got, fn(c.dims, c.U, c.T, c.kappa, psi))
        print(f"dims={c.dims} prec={prec} dagger={dagger} rel.err={err:.3e} site.err={serr:.3e} "
              f"vs periodic {periodic:.3e}")
        assert err <= TOL_D[prec]
        assert serr <= TOL_D_SITE[prec]
        assert periodic > 1e-2  # the flag changes the operator


@pytest.mark.parametrize("prec,lanes", [(cs.F64, 1), (cs.F32, 1), (cs.F32, 2), (cs.F16, 1), (cs.F16, 2),
                                        (cs.BF16, 1), (cs.BF16, 2)])
def test_sap_antiperiodic(ap8, ap16, prec, lanes):
    for c in (ap8, ap16):
        b = synth.source(c.dims, 2102)
        x0 = 0.3 * synth.source(c.dims, 2103)
        for zero in (True, False):
            ref = oracle.sap(c.dims, BDIM, c.Uo, c.T, c.kappa, 2, 4, b, x0=None if zero else x0)
            xd = c.lat.new_field(prec) if zero else c.to_dev(x0, prec)
            c.op.sap_smooth_cfg(xd, c.to_dev(b, prec), prec, 1, cs.LaunchConfig(1, 0, lanes), n_cy=2, n_mr=4,
                                x0_is_zero=zero)
            got = c.to_host(xd, prec)
            err, serr = rel(got, ref), site_err(got, ref)
            print(f"dims={c.dims} prec={prec} lanes={lanes} from_zero={zero} rel.err={err:.3e} site.err={serr:.3e}")
            assert err <= TOL_SAP[prec]
            assert serr <= TOL_SAP_SITE[prec]


@pytest.mark.parametrize("inner", [cs.F64, cs.F32, cs.BF16])
def test_gcr_antiperiodic_oracle_residual(ap16, inner):
    c = ap16
    b = synth.source(c.dims, 2104)
    bd = c.to_dev(b, cs.F64)
    xd = c.lat.new_field(cs.F64).zero_()
    st, stats = c.op.gcr_solve(xd, bd, cs.SolverParams(inner_prec=inner,
                                                       basis_prec=cs.F64 if inner == cs.F64 else cs.F32))
    x = c.to_host(xd, cs.F64)
    r = oracle.residual_norm(c.dims, c.Uo, c.kappa, c.csw, b, x) / np.linalg.norm(b)
    rp = oracle.residual_norm(c.dims, c.U, c.kappa, c.csw, b, x) / np.linalg.norm(b)
    print(f"inner={inner} iterations={stats[0]['iters']} oracle relres={r:.3e} (periodic operator: {rp:.3e})")
    assert st == 0 and r <= 1e-10
    assert rp > 1e-4


def test_force_antiperiodic(ap8):
    c = ap8
    x, y = synth.source(c.dims, 2105), synth.source(c.dims, 2106)
    g, _ = c.op.force(c.to_dev(x, cs.F64), c.to_dev(y, cs.F64))
    torch.cuda.synchronize()
    gh, gc = oracle.force(c.dims, c.Uo, c.kappa, c.csw, x, y)
    err = rel(g.cpu().numpy(), gh + gc)
    print(f"antiperiodic force rel.err={err:.3e}")
    assert err < 1e-12


def test_multigrid_antiperiodic(ap8):
    """P and the coarse operator D_c (whose +t and -t faces of the two
    aggregates in time differ by the boundary sign) against the oracle's."""
    c, nv = ap8, 4
    etas = [synth.source(c.dims, 6200 + i) for i in range(nv)]
    etas_d = c.lat.import_field(torch.from_numpy(np.stack(etas)).cuda(), cs.F32)
    prm = cs.MgParams(nv=nv, n_cy_setup=4, n_mr=4, n_adapt=0, n_coarse=20, n_cy_post=2, tol_coarse=0.0)
    m = cs.Multigrid(c.op, etas_d, prm)
    P, Dc = m.export()
    torch.cuda.synchronize()
    P_or, Dc_or, aggs, _ = mg.setup(c.dims, BDIM, c.Uo, c.T, c.kappa, etas, n_cy_setup=4, n_mr=4, n_adapt=0)
    Pg = c.lat.export_field(P, cs.F32, nv).cpu().numpy().reshape(nv, -1, 4, 3)
    errP = rel(Pg, P_or)
    errD = rel(dense_from_stencil(Dc, c.dims), Dc_or)
    print(f"antiperiodic multigrid: P rel.err={errP:.3e} D_c rel.err={errD:.3e}")
    assert errP < 1e-5 and errD < 1e-5
    # the MG-preconditioned solve reaches the antiperiodic system's solution
    b = synth.source(c.dims, 2107)
    xd = c.lat.new_field(cs.F64).zero_()
    st, stats = m.gcr_solve(xd, c.to_dev(b, cs.F64), cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32))
    x = c.to_host(xd, cs.F64)
    r = oracle.residual_norm(c.dims, c.Uo, c.kappa, c.csw, b, x) / np.linalg.norm(b)
    print(f"antiperiodic MG-FGCR: {stats['iters']} iterations, oracle relres {r:.3e}")
    assert st == 0 and r <= 1e-10
