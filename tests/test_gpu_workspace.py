"""Caller-owned solver workspace (hfr_solver_bind_workspace): the solver runs
in device memory the caller allocated (a PyTorch tensor) and gives the same
stages, bit for bit, as with the memory the library allocates; unbound,
short or misaligned workspaces are refused."""
import ctypes

import numpy as np
import pytest
import torch

import fr_inputs as fi
import paper_2401_16632_amd as hp
from paper_2401_16632_amd import _abi
from tests.cases import cylinder_desc, cylinder_state_at
from tests.gpu_util import dev, host, soa

pytestmark = pytest.mark.gpu

UINF = tuple(fi.freestream_state(0.2))


def _case(p=3):
    d, mask = cylinder_desc(n_theta=24, n_r=8, n_implicit_rings=3)
    mesh = hp.Mesh(d, p, implicit_mask=mask, uinf=UINF)
    x = mesh.maps()["sol_xy"].reshape(mesh.Ne, p + 1, p + 1, 2)
    u = cylinder_state_at(x[..., 0], x[..., 1], seed=3, amp=0.02)
    return mesh, u


def _steps(mesh, solver, u, dt, n=2):
    stp = hp.ImexStepper(mesh, solver)
    ud = dev(soa(u))
    out = []
    for _ in range(n):
        un, _ = stp.step(ud, dt)
        ud = un.clone()
        out.append(host(ud).copy())
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_caller_workspace_gives_the_same_stages(precision):
    mesh, u = _case()
    es = mesh.maps()["es"].reshape(8, 24)
    dt = 2.0 * 0.5 * (es[2].max() + es[3].min()) / (6.0 * 7)   # local CFL rule
    a = _steps(mesh, hp.Solver(mesh, precision=precision, precond=precision), u, dt)
    s = hp.Solver(mesh, precision=precision, precond=precision, workspace="torch")
    assert s.workspace is not None and s.workspace.numel() >= s.workspace_bytes
    b = _steps(mesh, s, u, dt)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    # bound again to a fresh buffer: the same stages
    lib = hp.load_library()
    ws2 = torch.empty(s.workspace_bytes + 1024, dtype=torch.uint8, device="cuda")
    rc = lib.hfr_solver_bind_workspace(s.handle, ctypes.c_void_p(ws2.data_ptr()),
                                       ctypes.c_size_t(ws2.numel()))
    assert rc == 0, lib.fr_last_error()
    s.workspace = ws2
    c = _steps(mesh, s, u, dt)
    for x, y in zip(a, c):
        assert np.array_equal(x, y)


def test_unbound_short_or_misaligned_workspace_is_refused():
    mesh, u = _case(p=2)
    lib = hp.load_library()
    o = _abi.HfrOpts()
    o.precision, o.precond, o.gmres_restart, o.gmres_max_iters = 0, 0, 30, 100
    o.gmres_rtol, o.newton_max_iters, o.newton_tol = 1e-10, 10, 1e-12
    o.caller_workspace = 1
    ws = ctypes.c_size_t()
    h = ctypes.c_void_p()
    assert lib.hfr_solver_create(mesh.handle, ctypes.byref(o), ctypes.byref(ws),
                                 ctypes.byref(h)) == 0
    try:
        n = 4 * mesh.Nim * mesh.Np
        t = torch.zeros(max(n, 4 * mesh.Ntp, 4 * mesh.Ne * mesh.Np), dtype=torch.float64,
                        device="cuda")
        p = ctypes.c_void_p(t.data_ptr())
        rc = lib.hfr_residual(h, p, p, p, 0.1, None, None, None, None)
        assert rc == -1 and "not bound" in lib.fr_last_error().decode()
        buf = torch.empty(ws.value + 512, dtype=torch.uint8, device="cuda")
        base = buf.data_ptr()
        assert lib.hfr_solver_bind_workspace(h, ctypes.c_void_p(base),
                                             ctypes.c_size_t(ws.value - 1)) == -1
        assert lib.hfr_solver_bind_workspace(h, ctypes.c_void_p(base + 8),
                                             ctypes.c_size_t(ws.value)) == -1
        assert lib.hfr_solver_bind_workspace(h, ctypes.c_void_p(base),
                                             ctypes.c_size_t(ws.value)) == 0
        assert lib.hfr_residual(h, p, p, p, 0.1, None, None, None, None) == 0
        torch.cuda.synchronize()
    finally:
        lib.hfr_solver_destroy(h)
    # a library-owned solver refuses a binding
    s = hp.Solver(mesh)
    assert lib.hfr_solver_bind_workspace(s.handle, ctypes.c_void_p(base),
                                         ctypes.c_size_t(ws.value)) == -1
