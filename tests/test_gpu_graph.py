"""Graph form of the Newton iteration (hfr_opts.iteration_graph): the
elimination, assembly, preconditioner set-up, first chunk of the trace solve
and the checks of the next iterate are recorded once per chunk length and
stage arguments and replayed.  The replays run the eager queue's kernels in
its order, so every stage matches the eager solver bit for bit; eager work
and host waits sit between the replays (every Newton iteration reads its
norms back).  Rebinding the workspace drops the graphs."""
import ctypes

import numpy as np
import pytest
import torch

import fr_inputs as fi
import paper_2401_16632_amd as hp
from tests.cases import c1_desc, cylinder_desc, cylinder_state_at
from tests.gpu_util import dev, host, soa

pytestmark = pytest.mark.gpu

UINF = tuple(fi.freestream_state(0.2))


def _cylinder(p=3, efr=False):
    d, mask = cylinder_desc(n_theta=24, n_r=8, n_implicit_rings=3)
    mesh = hp.Mesh(d, p, implicit_mask=mask, uinf=UINF, efr=efr)
    x = mesh.maps()["sol_xy"].reshape(mesh.Ne, p + 1, p + 1, 2)
    u = cylinder_state_at(x[..., 0], x[..., 1], seed=3, amp=0.02)
    es = mesh.maps()["es"].reshape(8, 24)
    dt = 2.0 * 0.5 * (es[2].max() + es[3].min()) / (6.0 * (2 * p + 1))   # local CFL rule
    return mesh, u, dt


def _run(mesh, solver, u, dt, n=3):
    stp = hp.ImexStepper(mesh, solver)
    ud = dev(soa(u))
    out, replays = [], 0
    for _ in range(n):
        un, stats = stp.step(ud, dt)
        ud = un.clone()
        out.append(host(ud).copy())
        replays += sum(s["graph_replays"] for s in stats)
    return out, replays


@pytest.mark.parametrize("case", ["cyl_p3_fp64", "cyl_p3_fp32", "cyl_p4_fp32", "cyl_p3_efr",
                                  "c1_p2_fp32", "cyl_p4_fp32_forcing", "cyl_p3_efr_forcing"])
def test_graph_replays_match_eager_bit_for_bit(case):
    if case.startswith("c1"):
        d, mask = c1_desc()
        mesh = hp.Mesh(d, 2, implicit_mask=mask, uinf=(1.0, 1.0, 0.0, 40.0))
        x = mesh.maps()["sol_xy"].reshape(mesh.Ne, 3, 3, 2)
        u, dt = fi.isentropic_vortex(x[..., 0], x[..., 1]), 0.01
    else:
        p = 4 if "p4" in case else 3
        mesh, u, dt = _cylinder(p, efr="efr" in case)
    prec = "fp64" if "fp64" in case or "efr" in case else "fp32"
    print("graph case:", case, flush=True)
    # forcing: the Krylov tolerance of each solve comes from the device's
    # Newton norms, which the replays read as the eager queue does
    fc = 1e-3 if case.endswith("forcing") else 0.0
    a, r0 = _run(mesh, hp.Solver(mesh, precision=prec, precond=prec, forcing=fc), u, dt)
    b, r1 = _run(mesh, hp.Solver(mesh, precision=prec, precond=prec, graph=True,
                                 forcing=fc), u, dt)
    assert r0 == 0 and r1 > 0, (r0, r1)
    for k, (x, y) in enumerate(zip(a, b)):
        assert np.isfinite(x).all()
        assert np.array_equal(x, y), (k, float(np.abs(x - y).max()))


def test_rebinding_the_workspace_drops_the_graphs():
    mesh, u, dt = _cylinder(3)
    ref, _ = _run(mesh, hp.Solver(mesh, precision="fp32", precond="fp32"), u, dt, n=2)
    s = hp.Solver(mesh, precision="fp32", precond="fp32", workspace="torch", graph=True)
    a, ra = _run(mesh, s, u, dt, n=2)
    lib = hp.load_library()
    ws2 = torch.empty(s.workspace_bytes + 1024, dtype=torch.uint8, device="cuda")
    assert lib.hfr_solver_bind_workspace(s.handle, ctypes.c_void_p(ws2.data_ptr()),
                                         ctypes.c_size_t(ws2.numel())) == 0
    old = s.workspace
    s.workspace = ws2
    del old
    torch.cuda.synchronize()
    b, rb = _run(mesh, s, u, dt, n=2)
    assert ra > 0 and rb > 0
    for x, y, z in zip(ref, a, b):
        assert np.array_equal(x, y) and np.array_equal(x, z)
