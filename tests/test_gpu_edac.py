"""GPU parity of the EDAC physics (Appendix A, inviscid, with the hybridized
stabilisation given for it) against the oracle on the same seeded inputs:
explicit and hybridized residuals, element blocks, the condensed system,
trace solve and recovery, and IMEX steps (FP64 and FP32 condensation, the
HFR and the interior-embedded trace)."""
import numpy as np
import pytest
import torch

import fr_inputs as fi
import oracle
from oracle import residual as ores, newton as onw, imex as oimex, efr
import paper_2401_16632_amd as hp
from tests.cases import c1_desc, cylinder_desc
from tests.gpu_util import dev, host, soa, unsoa, rel_err

pytestmark = pytest.mark.gpu

UINF = tuple(fi.edac_freestream())


class EPair:
    def __init__(self, desc, p, mask, theta, efr_trace=False):
        self.om = oracle.QuadMesh(desc, p, implicit_mask=mask, uinf=UINF)
        self.hm = hp.Mesh(desc, p, implicit_mask=mask, uinf=UINF, physics="edac",
                          theta=theta, efr=efr_trace)
        self.p, self.P, self.theta = p, p + 1, theta
        self.ph = oracle.EDAC(theta)
        self.tr = efr.EfrTrace(self.om) if efr_trace else None


def _build(name, efr_trace=False):
    if name.startswith("cyl"):
        d, mask = cylinder_desc(n_theta=24, n_r=8, n_implicit_rings=3)
        pr = EPair(d, 3, mask, 50.0, efr_trace)
        rng = np.random.default_rng(3)
        base = np.broadcast_to(np.asarray(UINF), pr.om.x.shape + (4,))
        u = base + 0.02 * rng.uniform(-1.0, 1.0, size=base.shape)
    else:
        d, mask = c1_desc() if name == "c1_p2" else c1_desc(n=6, perturb=0.2, seed=4)
        pr = EPair(d, 2 if name == "c1_p2" else 3, mask, 20.0, efr_trace)
        u = fi.perturb_state(fi.edac_vortex(pr.om.x, pr.om.y), 0.01, 11)
    return pr, u


def _stage_inputs(pr, u, seed=5):
    om = pr.om
    uhat = ores.trace_average(om, u)
    uhat = uhat + 0.005 * np.random.default_rng(seed).uniform(-1, 1, size=uhat.shape)
    ustar = fi.perturb_state(u[om.imp_elems], 0.005, seed + 1)
    return uhat, ustar


def _cfl_dt(pr, rings=3, n_theta=24):
    lam = 1.5 + np.sqrt(0.25 + pr.theta)
    es = pr.om.Es.reshape(-1, n_theta)
    cut = 0.5 * (es[rings - 1].max() + es[rings].min())
    return 2.0 * cut / (lam * (2 * pr.p + 1))


@pytest.mark.parametrize("name", ["c1_p2", "pert_p3", "cyl_p3"])
def test_edac_explicit_rhs(name):
    pr, u = _build(name)
    om, hm = pr.om, pr.hm
    R_o = ores.fr_residual(om, pr.ph, u)[om.exp_elems]
    R = torch.zeros(4 * hm.Nex * hm.Np, dtype=torch.float64, device="cuda")
    hm.explicit_rhs(dev(soa(u)), R)
    torch.cuda.synchronize()
    assert np.abs(unsoa(host(R), hm.Nex, pr.P) - R_o).max() <= 1e-12 * max(1.0, np.abs(R_o).max())


@pytest.mark.parametrize("name", ["c1_p2", "pert_p3", "cyl_p3"])
def test_edac_hfr_residual(name):
    pr, u = _build(name)
    om, hm = pr.om, pr.hm
    uhat, ustar = _stage_inputs(pr, u)
    a = 0.037
    R_o, g_o = ores.hfr_residual(om, pr.ph, u, uhat)
    h_o = u[om.imp_elems] - ustar - a * R_o
    s = hp.Solver(hm)
    h = torch.zeros(4 * hm.Nim * hm.Np, dtype=torch.float64, device="cuda")
    g = torch.zeros(4 * hm.Ntp, dtype=torch.float64, device="cuda")
    R = torch.zeros_like(h)
    s.residual(dev(soa(u)), dev(uhat), dev(soa(ustar)), a, h=h, g=g, R_im=R)
    torch.cuda.synchronize()
    sc = max(1.0, np.abs(R_o).max())
    assert np.abs(unsoa(host(R), hm.Nim, pr.P) - R_o).max() <= 1e-12 * sc
    assert np.abs(unsoa(host(h), hm.Nim, pr.P) - h_o).max() <= 1e-12 * sc
    assert np.abs(host(g).reshape(-1, 4) - g_o).max() <= 1e-12 * max(1.0, np.abs(g_o).max())


@pytest.mark.parametrize("name", ["c1_p2", "cyl_p3"])
def test_edac_element_blocks(name):
    """Analytic element blocks against the oracle's complex-step ones."""
    pr, u = _build(name)
    om, hm = pr.om, pr.hm
    uhat, ustar = _stage_inputs(pr, u)
    a = 0.05
    outer = ores.implicit_outer(om, u, uhat)
    A, B, C, D = onw.element_blocks(om, pr.ph, u[om.imp_elems], outer, a)
    s = hp.Solver(hm, keep_blocks=True)
    s.assemble_condense(dev(soa(u)), dev(uhat), dev(soa(ustar)), a)
    n, m = s.n, s.m
    blk = torch.zeros(hm.Nim * (n + m) ** 2, dtype=torch.float64, device="cuda")
    s.get_blocks(blk)
    torch.cuda.synchronize()
    G = host(blk).reshape(hm.Nim, n + m, n + m)
    sc = max(1.0, np.abs(A).max())
    assert np.abs(G[:, :n, :n] - A).max() <= 1e-11 * sc
    for k in range(hm.Nim):
        loc, _ = onw.trace_index(om, k, 4)
        Gk = G[k]
        assert np.abs(Gk[:n, n + loc] - B[k][:, loc]).max() <= 1e-11 * sc
        assert np.abs(Gk[n + loc, :n] - C[k][loc, :]).max() <= 1e-11 * max(1, np.abs(C).max())
        assert np.abs(Gk[np.ix_(n + loc, n + loc)] - D[k][np.ix_(loc, loc)]).max() <= \
            1e-11 * max(1, np.abs(D).max())


@pytest.mark.parametrize("name", ["c1_p2", "cyl_p3"])
def test_edac_condense_solve_recover(name):
    pr, u = _build(name)
    om, hm = pr.om, pr.hm
    uhat, ustar = _stage_inputs(pr, u)
    a = 0.05 if name != "cyl_p3" else 0.3 * _cfl_dt(pr)
    sysd = onw.condense(om, pr.ph, u, uhat, ustar, a)
    s = hp.Solver(hm, rtol=1e-12, max_iters=3000, restart=60)
    s.assemble_condense(dev(soa(u)), dev(uhat), dev(soa(ustar)), a)
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
    res_o = np.linalg.norm(sysd["t"] - sysd["L"] @ host(duh)) / np.linalg.norm(sysd["t"])
    assert st["rel_residual"] <= 1e-11 and res_o <= 1e-10, (st, res_o)
    duh_o = onw.trace_solve(sysd["L"], sysd["t"])
    du = torch.zeros(4 * hm.Nim * hm.Np, dtype=torch.float64, device="cuda")
    s.recover(dev(duh_o), du)
    torch.cuda.synchronize()
    du_o = onw.recover(sysd, duh_o).reshape(hm.Nim, pr.P, pr.P, 4)
    assert np.abs(unsoa(host(du), hm.Nim, pr.P) - du_o).max() <= 1e-11 * max(1e-300, np.abs(du_o).max())


def _run_steps(pr, u0, dt, nsteps, precision="fp64"):
    s = hp.Solver(pr.hm, precision=precision, precond=precision, rtol=1e-12,
                  newton_tol=1e-13, max_iters=3000)
    stp = hp.ImexStepper(pr.hm, s, "HIMEX2C")
    ud, uo = dev(soa(u0)), u0.copy()
    errs = []
    for _ in range(nsteps):
        un, _ = stp.step(ud, dt)
        ud = un.clone()
        uo, _ = oimex.imex_step(pr.om, pr.ph, oimex.himex2c(), uo, dt, tol=1e-13,
                                trace=pr.tr)
        errs.append(rel_err(unsoa(host(ud), pr.hm.Ne, pr.P), uo))
    return errs


def test_edac_imex_steps_fp64_c1():
    pr, u = _build("c1_p2")
    errs = _run_steps(pr, u, 0.01, 5)
    assert max(errs) <= 1e-11, errs


def test_edac_imex_steps_fp32_condensation():
    pr, u = _build("c1_p2")
    errs = _run_steps(pr, u, 0.01, 3, precision="fp32")
    assert max(errs) <= 1e-8, errs


def test_edac_imex_steps_cylinder():
    pr, u = _build("cyl_p3")
    errs = _run_steps(pr, u, _cfl_dt(pr), 2)
    assert max(errs) <= 1e-11, errs


def test_edac_efr_imex_steps():
    pr, u = _build("pert_p3", efr_trace=True)
    errs = _run_steps(pr, u, 0.01, 2)
    assert max(errs) <= 1e-11, errs


def test_edac_rejects_bad_theta():
    d, mask = c1_desc(n=3)
    for bad in (0.0, -1.0, float("inf")):
        with pytest.raises(hp.HfrError):
            hp.Mesh(d, 2, implicit_mask=mask, uinf=UINF, physics="edac", theta=bad)
