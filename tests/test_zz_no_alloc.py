"""hfr_residual_noalloc (no device allocation; its element shares live in a
static device array) against hfr_residual, through the C ABI: identical h,
g and R_im on two calls in a row, the second on a smaller mesh, and a mesh
too large for the array refused before any launch."""
import ctypes

import numpy as np
import pytest
import torch

import fr_inputs as fi
import oracle
from oracle import residual as ores
import paper_2401_16632_amd as hp
from tests.cases import c1_desc, cylinder_desc, cylinder_state_at
from tests.gpu_util import dev, host, soa

pytestmark = pytest.mark.gpu


def _inputs(desc, p, mask, uinf, cyl, efr=False):
    om = oracle.QuadMesh(desc, p, implicit_mask=mask, uinf=uinf)
    hm = hp.Mesh(desc, p, implicit_mask=mask, uinf=uinf, efr=efr)
    if cyl:
        u = cylinder_state_at(om.x, om.y, seed=3, amp=0.02)
    else:
        u = fi.perturb_state(fi.isentropic_vortex(om.x, om.y), 0.01, 11)
    ntp = hm.Ntp
    uhat = fi.perturb_state(np.ones((ntp, 4)) * u.mean(axis=(0, 1, 2)), 0.01, 5)
    ustar = fi.perturb_state(u[om.imp_elems], 0.005, 6)
    return hm, u, uhat, ustar


def _both(hm, u, uhat, ustar, a):
    lib = hp.load_library()
    ni, nt = 4 * hm.Nim * hm.Np, 4 * hm.Ntp
    z = lambda n: torch.zeros(max(1, n), dtype=torch.float64, device="cuda")
    ud, uh, us = dev(soa(u)), dev(uhat), dev(soa(ustar))
    s = hp.Solver(hm)
    h1, g1, r1 = z(ni), z(nt), z(ni)
    s.residual(ud, uh, us, a, h=h1, g=g1, R_im=r1)
    h2, g2, r2 = z(ni), z(nt), z(ni)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.hfr_residual_noalloc(hm.handle, ptr(ud), ptr(uh), ptr(us), float(a),
                                  ptr(h2), ptr(g2), ptr(r2), st)
    assert rc == 0, lib.fr_last_error()
    torch.cuda.synchronize()
    s.close()
    return (host(h1), host(g1), host(r1)), (host(h2), host(g2), host(r2))


@pytest.mark.parametrize("efr", [False, True])
def test_noalloc_matches_hfr_residual_on_two_calls(efr):
    uinf = tuple(fi.freestream_state(0.2))
    d, mask = cylinder_desc(n_theta=32, n_r=16, n_implicit_rings=4)
    big = _inputs(d, 4, mask, uinf, True, efr)
    d2, mask2 = c1_desc(n=6)
    small = _inputs(d2, 2, mask2, (1.0, 1.0, 0.0, 40.0), False, efr)
    print(f"noalloc: cylinder 32x16 p=4 then vortex 6x6 p=2, efr={efr}", flush=True)
    for case, a in ((big, 1e-3), (small, 0.05)):
        ref, got = _both(*case, a)
        for x, y in zip(ref, got):
            assert np.array_equal(x, y)


def test_noalloc_refuses_a_mesh_beyond_its_array():
    # 132 x 132 quads at p = 4, all implicit: 17424 * 80 doubles > 2^20
    d = fi.periodic_quad_mesh(132, 132)
    hm = hp.Mesh(d, 4, implicit_mask=np.ones(132 * 132, bool),
                 uinf=(1.0, 1.0, 0.0, 40.0))
    lib = hp.load_library()
    t = torch.zeros(4, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(t.data_ptr())
    rc = lib.hfr_residual_noalloc(hm.handle, p, p, p, 0.1, p, p, None, None)
    assert rc == -1 and "scratch array" in lib.fr_last_error().decode()
