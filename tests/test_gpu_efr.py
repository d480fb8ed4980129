"""GPU parity of the interior-embedded (EFR) trace against the oracle on
the same seeded inputs: nodal transmission residual, condensed node-block
system, trace solve and recovery, block-Jacobi node blocks, and whole IMEX
steps in FP64 and with FP32 condensation."""
import numpy as np
import pytest
import torch

import fr_inputs as fi
import oracle
from oracle import efr, newton as onw, imex as oimex
import paper_2401_16632_amd as hp
from tests.cases import c1_desc, cylinder_desc, cylinder_state_at
from tests.gpu_util import dev, host, soa, unsoa, rel_err

pytestmark = pytest.mark.gpu

UINF_CYL = tuple(fi.freestream_state(0.2))


class EPair:
    def __init__(self, desc, p, mask, uinf):
        self.om = oracle.QuadMesh(desc, p, implicit_mask=mask, uinf=uinf)
        self.tr = efr.EfrTrace(self.om)
        self.hm = hp.Mesh(desc, p, implicit_mask=mask, uinf=uinf, efr=True)
        self.p, self.P = p, p + 1
        self.ph = oracle.Euler()


def _build(name):
    if name.startswith("c1"):
        d, mask = c1_desc() if name == "c1_p2" else c1_desc(n=6, perturb=0.2, seed=4)
        p = 2 if name == "c1_p2" else 3
        pr = EPair(d, p, mask, (1.0, 1.0, 0.0, 40.0))
        u = fi.perturb_state(fi.isentropic_vortex(pr.om.x, pr.om.y), 0.01, 11)
    else:
        d, mask = cylinder_desc(n_theta=24, n_r=8, n_implicit_rings=3)
        pr = EPair(d, 3, mask, UINF_CYL)
        u = cylinder_state_at(pr.om.x, pr.om.y, seed=3, amp=0.02)
    return pr, u


def _inputs(pr, u, seed=5):
    U = fi.perturb_state(efr.node_average(pr.om, pr.tr, u), 0.005, seed)
    ustar = fi.perturb_state(u[pr.om.imp_elems], 0.005, seed + 1)
    return U, ustar


@pytest.mark.parametrize("name", ["c1_p2", "c1_p3", "cyl_p3"])
def test_efr_residual(name):
    pr, u = _build(name)
    om, hm = pr.om, pr.hm
    U, ustar = _inputs(pr, u)
    a = 0.037
    R_o, g_o = efr.efr_residual(om, pr.tr, pr.ph, u, U)
    h_o = u[om.imp_elems] - ustar - a * R_o
    s = hp.Solver(hm)
    h = torch.zeros(4 * hm.Nim * hm.Np, dtype=torch.float64, device="cuda")
    g = torch.zeros(4 * hm.Ntp, dtype=torch.float64, device="cuda")
    R = torch.zeros_like(h)
    s.residual(dev(soa(u)), dev(U), dev(soa(ustar)), a, h=h, g=g, R_im=R)
    torch.cuda.synchronize()
    sc = max(1.0, np.abs(R_o).max())
    assert np.abs(unsoa(host(R), hm.Nim, pr.P) - R_o).max() <= 1e-12 * sc
    assert np.abs(unsoa(host(h), hm.Nim, pr.P) - h_o).max() <= 1e-12 * sc
    assert np.abs(host(g).reshape(-1, 4) - g_o).max() <= 1e-12 * max(1.0, np.abs(g_o).max())


@pytest.mark.parametrize("name", ["c1_p2", "c1_p3", "cyl_p3"])
def test_efr_condense_solve_recover(name):
    pr, u = _build(name)
    om, hm = pr.om, pr.hm
    U, ustar = _inputs(pr, u)
    # a_ii dt of a stage at the local-CFL time step on the cylinder
    a = 0.05 if name != "cyl_p3" else 0.3 * _cfl_dt(pr)
    sysd = efr.condense(om, pr.tr, pr.ph, u, U, ustar, a)
    s = hp.Solver(hm, rtol=1e-12, max_iters=3000, restart=60)
    s.assemble_condense(dev(soa(u)), dev(U), dev(soa(ustar)), a)
    N = 4 * hm.Ntp
    t = torch.zeros(N, dtype=torch.float64, device="cuda")
    s.get_system(t=t)
    x = np.random.default_rng(0).normal(size=N)
    y = torch.zeros(N, dtype=torch.float64, device="cuda")
    s.matvec(dev(x), y)
    torch.cuda.synchronize()
    Lx = sysd["L"] @ x
    assert np.abs(host(y) - Lx).max() <= 1e-11 * max(1, np.abs(Lx).max())
    assert np.abs(host(t) - sysd["t"]).max() <= 1e-11 * max(1, np.abs(sysd["t"]).max())
    duh = torch.zeros(N, dtype=torch.float64, device="cuda")
    st = s.trace_solve(duh, allow_unconverged=True)
    dU_o = onw.trace_solve(sysd["L"], sysd["t"])
    res_o = np.linalg.norm(sysd["t"] - sysd["L"] @ host(duh)) / np.linalg.norm(sysd["t"])
    assert st["rel_residual"] <= 1e-11 and res_o <= 1e-10, (st, res_o)
    du = torch.zeros(4 * hm.Nim * hm.Np, dtype=torch.float64, device="cuda")
    s.recover(dev(dU_o), du)
    torch.cuda.synchronize()
    du_o = efr.recover(sysd, dU_o).reshape(hm.Nim, pr.P, pr.P, 4)
    assert np.abs(unsoa(host(du), hm.Nim, pr.P) - du_o).max() <= 1e-11 * max(1e-300, np.abs(du_o).max())


@pytest.mark.parametrize("precision,precond,tol", [("fp64", "fp64", 1e-13),
                                                   ("fp32", "fp32", 1e-6)])
def test_efr_node_block_jacobi(precision, precond, tol):
    pr, u = _build("c1_p2")
    U, ustar = _inputs(pr, u)
    sysd = efr.condense(pr.om, pr.tr, pr.ph, u, U, ustar, 0.05)
    s = hp.Solver(pr.hm, precision=precision, precond=precond)
    s.assemble_condense(dev(soa(u)), dev(U), dev(soa(ustar)), 0.05)
    X = s.get_preconditioner().cpu().numpy()
    L = sysd["L"].tocsr()
    assert X.shape == (pr.tr.Nn, 4, 4)
    for a in range(pr.tr.Nn):
        D = L[4 * a:4 * a + 4, 4 * a:4 * a + 4].toarray()
        err = np.abs(X[a] @ D - np.eye(4)).max()
        assert err <= tol * 4 * np.abs(X[a]).max() * np.abs(D).max(), (a, err)


def _cfl_dt(pr, lam=6.0, rings=3, n_theta=24):
    """Time step of the local-CFL rule (CFL = 1 between the last implicit
    and the first explicit ring)."""
    es = pr.om.Es.reshape(-1, n_theta)
    cut = 0.5 * (es[rings - 1].max() + es[rings].min())
    return 2.0 * cut / (lam * (2 * pr.p + 1))


def _run_steps(pr, u0, dt, nsteps, precision="fp64", precond="fp64"):
    s = hp.Solver(pr.hm, precision=precision, precond=precond, rtol=1e-12,
                  newton_tol=1e-13, max_iters=3000)
    stp = hp.ImexStepper(pr.hm, s, "HIMEX2C")
    ud = dev(soa(u0))
    uo = u0.copy()
    errs = []
    for _ in range(nsteps):
        un, _ = stp.step(ud, dt)
        ud = un.clone()
        uo, _ = oimex.imex_step(pr.om, pr.ph, oimex.himex2c(), uo, dt,
                                tol=1e-13, trace=pr.tr)
        errs.append(rel_err(unsoa(host(ud), pr.hm.Ne, pr.P), uo))
    return errs


def test_efr_imex_steps_fp64_c1():
    pr, _ = _build("c1_p2")
    u0 = fi.isentropic_vortex(pr.om.x, pr.om.y)
    errs = _run_steps(pr, u0, 0.01, 5)
    assert max(errs) <= 1e-11, errs


def test_efr_imex_steps_fp32_condensation():
    pr, _ = _build("c1_p2")
    u0 = fi.isentropic_vortex(pr.om.x, pr.om.y)
    errs = _run_steps(pr, u0, 0.01, 3, precision="fp32", precond="fp32")
    assert max(errs) <= 1e-8, errs


def test_efr_imex_step_cylinder():
    pr, u = _build("cyl_p3")
    errs = _run_steps(pr, u, _cfl_dt(pr), 2)
    assert max(errs) <= 1e-11, errs
