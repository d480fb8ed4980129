"""The condensation of the next Newton iteration queued behind the checks of
the current iterate and skipped on the device when they pass (the blocked
elimination kernel, fused with the linearisation in FP32, after a gated fill
in FP64).  Event timers switch the queuing off, so the same steps with and
without timers must give the same states bit for bit, with the queued
launches actually taken (a Newton solve of several iterations after the
first one)."""
import numpy as np
import pytest

import fr_inputs as fi
import paper_2401_16632_amd as hp
from tests.cases import cylinder_desc, cylinder_state_at
from tests.gpu_util import dev, host, soa

pytestmark = pytest.mark.gpu

UINF = tuple(fi.freestream_state(0.2))


def _case(p):
    d, mask = cylinder_desc(n_theta=24, n_r=8, n_implicit_rings=3)
    mesh = hp.Mesh(d, p, implicit_mask=mask, uinf=UINF)
    x = mesh.maps()["sol_xy"].reshape(mesh.Ne, p + 1, p + 1, 2)
    u = cylinder_state_at(x[..., 0], x[..., 1], seed=3, amp=0.02)
    es = mesh.maps()["es"].reshape(8, 24)
    dt = 2.0 * 0.5 * (es[2].max() + es[3].min()) / (6.0 * (2 * p + 1))
    return mesh, u, dt


def _run(mesh, solver, u, dt, timed, n=3):
    if timed:
        solver.timing(True)
    stp = hp.ImexStepper(mesh, solver)
    ud = dev(soa(u))
    out, its, queued = [], [], 0
    for _ in range(n):
        un, stats = stp.step(ud, dt)
        ud = un.clone()
        out.append(host(ud).copy())
        its.append([s["newton_iters"] for s in stats])
        queued += sum(s["queued_linearisations"] for s in stats)
    return out, its, queued


@pytest.mark.parametrize("p,precision,forcing", [(4, "fp32", 0.0), (4, "fp32", 1e-3),
                                                  (4, "fp64", 0.0), (2, "fp32", 0.0)])
def test_queued_condensation_matches_unqueued(p, precision, forcing):
    print("queued condensation case:", p, precision, forcing, flush=True)
    mesh, u, dt = _case(p)
    kw = dict(precision=precision, precond=precision, condense="blocked", forcing=forcing)
    a, ia, qa = _run(mesh, hp.Solver(mesh, **kw), u, dt, timed=False)
    b, ib, qb = _run(mesh, hp.Solver(mesh, **kw), u, dt, timed=True)
    assert ia == ib, (ia, ib)
    assert qa > 0 and qb == 0, (qa, qb)
    for k, (x, y) in enumerate(zip(a, b)):
        assert np.isfinite(x).all()
        assert np.array_equal(x, y), (k, float(np.abs(x - y).max()))
