"""Damped Newton (hfr_opts.newton_damping): on a stretched cylinder whose
impulsive first stage sits at local CFL ~40 at the wall, a full Newton step
leaves the admissible states (non-finite residual) in the oracle and on the
GPU alike; with the step halved until the residual is finite both converge
to the same stage."""
import ctypes

import numpy as np
import pytest
import torch

import fr_inputs as fi
import oracle
from oracle import newton as onw, residual as ores, imex as oimex
import paper_2401_16632_amd as hp
from paper_2401_16632_amd import _abi
from tests.gpu_util import dev, host, soa, unsoa, rel_err

pytestmark = pytest.mark.gpu

UINF = fi.freestream_state(0.2)


@pytest.fixture(scope="module")
def case():
    nt, nr, ratio, J, p = 24, 26, 1.209, 20, 3
    d = fi.cylinder_ogrid(nt, nr, first=1e-4, ratio=ratio)
    m0 = oracle.QuadMesh(d, p, uinf=UINF)
    es = m0.Es.reshape(nr, nt)
    cut = 0.5 * (es[J - 1].max() + es[J].min())
    dt = 2.0 * cut / (6.0 * (2 * p + 1))
    om = oracle.QuadMesh(d, p, es_cutoff=cut, uinf=UINF)
    P = p + 1
    u = fi.perturb_state(np.broadcast_to(UINF, (om.Ne, P, P, 4)).copy(), 1e-3, 2)
    ph = oracle.Euler()
    tab = oimex.himex2c()
    u1 = u.copy()
    u1[om.exp_elems] += dt * tab.Abar[1, 0] * ores.fr_residual(om, ph, u)[om.exp_elems]
    with pytest.raises(Exception):
        onw.solve_stage(om, ph, u1, u[om.imp_elems], dt * tab.A[0, 0], tol=1e-12)
    u_im, uhat, _ = onw.solve_stage(om, ph, u1, u[om.imp_elems], dt * tab.A[0, 0],
                                    tol=1e-12, damping=True, maxit=40)
    mesh = hp.Mesh(d, p, es_cutoff=cut, uinf=tuple(UINF))
    return mesh, om, u, dt, u_im, uhat


def _first_stage(mesh, u, dt, **kw):
    s = hp.Solver(mesh, rtol=1e-10, newton_tol=1e-12, max_iters=3000, newton_max_iters=40,
                  **kw)
    stp = hp.ImexStepper(mesh, s, "HIMEX2C")
    ud = dev(soa(u))
    lib = hp.load_library()
    st = _abi.ImexState(ud.data_ptr(), stp.u.data_ptr(), stp.uhat.data_ptr(),
                        stp.R_im.data_ptr(), stp.R_ex.data_ptr())
    ns = _abi.HfrNewtonStats()
    rc = 0
    for stage in (0, 1):
        rc = lib.imex_stage(mesh.handle, s.handle, ctypes.byref(stp.tab), stage, float(dt),
                            ctypes.byref(st), ctypes.byref(ns), None)
        if rc:
            break
    torch.cuda.synchronize()
    return rc, stp, ns


def test_full_steps_fail_like_the_oracle(case):
    mesh, om, u, dt, _, _ = case
    print("damping case: 24x26 cylinder p=3, full steps", flush=True)
    rc, _, _ = _first_stage(mesh, u, dt)
    assert rc == -6                                  # FR_E_NONFINITE


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_damped_stage_matches_damped_oracle(case, precision):
    mesh, om, u, dt, u_im, uhat = case
    print(f"damping case: 24x26 cylinder p=3, damped, {precision}", flush=True)
    rc, stp, ns = _first_stage(mesh, u, dt, damping=True, precision=precision,
                               precond=precision)
    assert rc == 0, hp.load_library().fr_last_error()
    ug = unsoa(host(stp.u), mesh.Ne, om.P)
    tol = 1e-11 if precision == "fp64" else 1e-8
    assert rel_err(ug[om.imp_elems], u_im) <= tol
    assert rel_err(host(stp.uhat), uhat) <= tol
