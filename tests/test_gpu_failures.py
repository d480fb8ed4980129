"""Failure paths of the implicit stage through the C ABI: a non-finite state
returns FR_E_NONFINITE, a Newton iteration cap FR_E_NOT_CONVERGED (with the
documented state: u_n untouched), a Krylov iteration cap FR_E_NOT_CONVERGED
from hfr_trace_solve with its statistics.  Every condition is data the host
sets up; every kernel runs to its normal end."""
import numpy as np
import pytest
import torch

import fr_inputs as fi
import paper_2401_16632_amd as hp
from tests.cases import c1_desc
from tests.gpu_util import dev, host, soa

pytestmark = pytest.mark.gpu


def _case():
    d, mask = c1_desc()
    mesh = hp.Mesh(d, 2, implicit_mask=mask, uinf=(1.0, 1.0, 0.0, 40.0))
    x = mesh.maps()["sol_xy"].reshape(mesh.Ne, 3, 3, 2)
    u = fi.isentropic_vortex(x[..., 0], x[..., 1])
    return mesh, u


def test_nonfinite_state_is_reported():
    mesh, u = _case()
    u = u.copy()
    k = int(mesh.maps()["implicit_elems"][3])
    u[k, 1, 1, 0] = np.nan
    s = hp.Solver(mesh)
    stp = hp.ImexStepper(mesh, s)
    print("nonfinite case: c1 p=2, NaN in implicit element", k, flush=True)
    with pytest.raises(hp.HfrError, match="FR_E_NONFINITE"):
        stp.step(dev(soa(u)), 0.01)
    torch.cuda.synchronize()


def test_newton_cap_leaves_u_n_untouched():
    mesh, u = _case()
    s = hp.Solver(mesh, newton_max_iters=1, newton_tol=1e-18)
    stp = hp.ImexStepper(mesh, s)
    un = dev(soa(u))
    before = host(un).copy()
    print("newton cap case: c1 p=2, 1 iteration, tol 1e-18", flush=True)
    with pytest.raises(hp.HfrError, match="FR_E_NOT_CONVERGED"):
        stp.step(un, 0.01)
    torch.cuda.synchronize()
    assert np.array_equal(host(un), before)
    # the stage buffer holds a finite Newton iterate
    assert np.isfinite(host(stp.u)).all()


def test_krylov_cap_through_trace_solve():
    mesh, u = _case()
    from oracle import residual as ores
    import oracle
    d, mask = c1_desc()
    om = oracle.QuadMesh(d, 2, implicit_mask=mask, uinf=(1.0, 1.0, 0.0, 40.0))
    u = fi.perturb_state(fi.isentropic_vortex(om.x, om.y), 0.01, 3)
    uhat = ores.trace_average(om, u)
    ustar = fi.perturb_state(u[om.imp_elems], 0.005, 4)
    s = hp.Solver(mesh, max_iters=2, restart=30, rtol=1e-14)
    s.assemble_condense(dev(soa(u)), dev(uhat), dev(soa(ustar)), 0.05)
    duh = torch.zeros(4 * mesh.Ntp, dtype=torch.float64, device="cuda")
    print("krylov cap case: c1 p=2, 2 iterations, rtol 1e-14", flush=True)
    with pytest.raises(hp.HfrError, match="FR_E_NOT_CONVERGED"):
        s.trace_solve(duh)
    st = s.trace_solve(duh, allow_unconverged=True)
    assert st["iterations"] == 2 and 0.0 < st["rel_residual"] < 1.0
    assert np.isfinite(host(duh)).all()
