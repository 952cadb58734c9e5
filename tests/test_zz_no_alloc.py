"""The allocation-free force entry point (cs_force_noalloc) against cs_force,
through the C ABI: the same kernels on a fixed workspace, so the results are
identical bit for bit.  Two calls in a row, the second on a smaller lattice
(the workspace keeps the first call's contents, which must not leak into the
second), then a lattice too large for the workspace, which is refused."""
import numpy as np
import pytest
import torch

import oracle
from paper_2112_00501_amd import cloversap as cs
from paper_2112_00501_amd import synth
from tests.gpu_helpers import rel

pytestmark = pytest.mark.gpu


def _case(dims, seed):
    U = synth.gauge_field(dims, 0.3, seed)
    lat = cs.Lattice(dims)
    op = cs.Operator(lat, torch.from_numpy(U).cuda(), 0.1355, 1.0)
    x = synth.source(dims, seed + 1)
    y = synth.source(dims, seed + 2)
    xd = lat.import_field(torch.from_numpy(x).cuda(), cs.F64)
    yd = lat.import_field(torch.from_numpy(y).cuda(), cs.F64)
    return U, lat, op, x, y, xd, yd


def _both(op, lat, xd, yd):
    V = lat.volume
    g_ref, G_ref = op.force(xd, yd, want_lie=True, want_grad=True)
    g = torch.full((V, 4, 8), float("nan"), dtype=torch.float64, device="cuda")
    G = torch.full((V, 4, 3, 3), float("nan"), dtype=torch.complex128, device="cuda")
    op.force_noalloc(xd, yd, g_lie=g, grad_U=G)
    torch.cuda.synchronize()
    return g_ref.cpu().numpy(), G_ref.cpu().numpy(), g.cpu().numpy(), G.cpu().numpy()


def test_noalloc_force_equals_force_on_two_calls():
    # first call: 16^3 x 32 (131,072 sites, most of the workspace)
    U1, lat1, op1, x1, y1, xd1, yd1 = _case((16, 16, 16, 32), 41)
    g_ref, G_ref, g, G = _both(op1, lat1, xd1, yd1)
    print(f"16^3x32: max |g - g_ref| = {np.abs(g - g_ref).max():.3e}")
    assert np.array_equal(g, g_ref)
    assert np.array_equal(G, G_ref)
    # second call, smaller lattice: 8^4, also against the oracle
    dims = (8, 8, 8, 8)
    U2, lat2, op2, x2, y2, xd2, yd2 = _case(dims, 43)
    g_ref, G_ref, g, G = _both(op2, lat2, xd2, yd2)
    assert np.array_equal(g, g_ref)
    assert np.array_equal(G, G_ref)
    gh, gc = oracle.force(dims, U2, 0.1355, 1.0, x2, y2)
    err = rel(g, gh + gc)
    print(f"8^4: noalloc force vs oracle rel.err={err:.3e}")
    assert err < 1e-12
    # only the g_lie output, on the larger lattice again
    g3 = torch.zeros((lat1.volume, 4, 8), dtype=torch.float64, device="cuda")
    op1.force_noalloc(xd1, yd1, g_lie=g3)
    torch.cuda.synchronize()
    g_ref1, _ = op1.force(xd1, yd1, want_lie=True, want_grad=False)
    assert np.array_equal(g3.cpu().numpy(), g_ref1.cpu().numpy())


def test_noalloc_force_refuses_a_lattice_beyond_the_workspace():
    dims = (16, 16, 16, 40)  # 163,840 sites x 864 bytes > 128 MiB
    lat = cs.Lattice(dims)
    U = np.zeros((lat.volume, 4, 3, 3), np.complex128)
    U[:, :, [0, 1, 2], [0, 1, 2]] = 1.0
    op = cs.Operator(lat, torch.from_numpy(U).cuda(), 0.13, 1.0)
    xd = lat.new_field(cs.F64).zero_()
    g = torch.zeros((lat.volume, 4, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(cs.CloverSapError) as e:
        op.force_noalloc(xd, xd, g_lie=g)
    assert e.value.status == -1
    assert "workspace" in str(e.value)
