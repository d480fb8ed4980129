"""GPU parity of every entry point of the C ABI against the CPU oracle on
the same seeded inputs (elementwise; tolerances derived from FP64 rounding
of the operations involved)."""
import numpy as np
import pytest
import torch

import fr_inputs as fi
import oracle
from oracle import residual as ores, newton as onw, imex as oimex
import paper_2401_16632_amd as hp
from tests.cases import c1_desc, cylinder_desc, cylinder_state_at
from tests.gpu_util import Pair, dev, host, soa, unsoa, rel_err

pytestmark = pytest.mark.gpu

UINF_CYL = tuple(fi.freestream_state(0.2))


def _pairs():
    d1, m1 = c1_desc()
    d2, m2 = c1_desc(n=6, perturb=0.2, seed=4)
    d3, m3 = cylinder_desc(n_theta=24, n_r=8, n_implicit_rings=3)
    return {
        "c1_p2": (d1, 2, m1, "vortex"),
        "pert_p3": (d2, 3, m2, "vortex"),
        "cyl_p3": (d3, 3, m3, "cyl"),
        "cyl_p4": (d3, 4, m3, "cyl"),
        "c1_p1": (d1, 1, m1, "vortex"),
        "c1_p5": (d1, 5, m1, "vortex"),
    }


def _build(name):
    d, p, mask, kind = _pairs()[name]
    uinf = UINF_CYL if kind == "cyl" else (1.0, 1.0, 0.0, 40.0)
    pr = Pair(d, p, mask, uinf=uinf)
    om = pr.om
    if kind == "vortex":
        u = fi.perturb_state(fi.isentropic_vortex(om.x, om.y), 0.01, 11)
    else:
        u = cylinder_state_at(om.x, om.y, seed=3, amp=0.02)
    return pr, u


@pytest.mark.parametrize("name", ["c1_p2", "pert_p3", "cyl_p3", "cyl_p4"])
def test_explicit_rhs(name):
    pr, u = _build(name)
    om, hm = pr.om, pr.hm
    R_o = ores.fr_residual(om, pr.ph, u)[om.exp_elems]
    ud = dev(soa(u))
    R = torch.zeros(4 * hm.Nex * hm.Np, dtype=torch.float64, device="cuda")
    hm.explicit_rhs(ud, R)
    torch.cuda.synchronize()
    R_g = unsoa(host(R), hm.Nex, pr.P)
    scale = max(1.0, np.abs(R_o).max())
    assert np.abs(R_g - R_o).max() <= 1e-12 * scale


def _stage_inputs(pr, u, seed=5):
    om = pr.om
    uhat = fi.perturb_state(ores.trace_average(om, u), 0.005, seed)
    ustar = fi.perturb_state(u[om.imp_elems], 0.005, seed + 1)
    return uhat, ustar


@pytest.mark.parametrize("name", ["c1_p2", "pert_p3", "cyl_p3"])
def test_hfr_residual(name):
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
    P = pr.P
    sc = max(1.0, np.abs(R_o).max())
    assert np.abs(unsoa(host(R), hm.Nim, P) - R_o).max() <= 1e-12 * sc
    assert np.abs(unsoa(host(h), hm.Nim, P) - h_o).max() <= 1e-12 * sc
    assert np.abs(host(g).reshape(-1, 4) - g_o).max() <= 1e-12 * max(1.0, np.abs(g_o).max())


@pytest.mark.parametrize("name", ["c1_p2", "cyl_p3", "c1_p1"])
def test_element_blocks_match_oracle_derivatives(name):
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
        assert np.abs(Gk[np.ix_(n + loc, n + loc)] - D[k][np.ix_(loc, loc)]).max() <= 1e-11 * max(1, np.abs(D).max())


@pytest.mark.parametrize("name,precision", [("c1_p2", "fp64"), ("cyl_p3", "fp64"),
                                            ("c1_p2", "fp32"), ("cyl_p4", "fp64"),
                                            ("cyl_p4", "fp32"), ("c1_p1", "fp64"),
                                            ("c1_p1", "fp32"), ("c1_p5", "fp64"),
                                            ("c1_p5", "fp32")])
def test_element_factorisation(name, precision):
    """Each element's swept tableau: A^-1, -A^-1 B, C A^-1 (pivot-permuted)
    and the Schur complement D - C A^-1 B, checked with NumPy on the GPU's
    own (oracle-verified) element blocks."""
    pr, u = _build(name)
    hm = pr.hm
    uhat, ustar = _stage_inputs(pr, u)
    s = hp.Solver(hm, precision=precision, precond=precision, keep_blocks=True)
    s.assemble_condense(dev(soa(u)), dev(uhat), dev(soa(ustar)), 0.05)
    n, m = s.n, s.m
    blk = torch.zeros(hm.Nim * (n + m) ** 2, dtype=torch.float64, device="cuda")
    s.get_blocks(blk)
    F, piv = s.get_factors()
    torch.cuda.synchronize()
    G = host(blk).reshape(hm.Nim, n + m, n + m)
    F = F.double().cpu().numpy()
    piv = piv.cpu().numpy().astype(np.int64)
    tol = 1e-10 if precision == "fp64" else 2e-4
    for k in range(hm.Nim):
        p = piv[k]
        assert sorted(p.tolist()) == list(range(n)), k
        A, B, C, D = G[k, :n, :n], G[k, :n, n:], G[k, n:, :n], G[k, n:, n:]
        Ai = np.linalg.inv(A)
        X = Ai @ B
        W = C @ Ai
        S = D - C @ X
        T = F[k]
        for got, ref in ((T[:n, :n][p, :], Ai[:, p]), (T[:n, n:][p, :], -X),
                         (T[n:, :n], W[:, p]), (T[n:, n:], S)):
            err = np.abs(got - ref).max()
            assert err <= tol * max(1.0, np.abs(ref).max()), (k, err)


@pytest.mark.parametrize("name,precision,precond,tol", [
    ("c1_p2", "fp64", "fp64", 1e-13), ("cyl_p3", "fp64", "fp64", 1e-13),
    ("cyl_p3", "fp32", "fp32", 1e-6), ("cyl_p3", "fp32", "bf16", 1e-2),
    ("cyl_p4", "fp64", "fp64", 1e-13), ("cyl_p4", "fp32", "fp32", 1e-6),
    ("c1_p5", "fp64", "fp64", 1e-13), ("c1_p5", "fp32", "bf16", 1e-2)])
def test_block_jacobi_inverse(name, precision, precond, tol):
    """The preconditioner blocks invert the oracle's diagonal face blocks of
    L: backward error |X D - I| / (bs |X| |D|) within a few units of the
    coarsest precision involved (L stored in FP32 in the FP32 form, the
    inverse rounded to FP32 or BF16)."""
    pr, u = _build(name)
    om, hm = pr.om, pr.hm
    uhat, ustar = _stage_inputs(pr, u)
    a = 0.05
    sysd = onw.condense(om, pr.ph, u, uhat, ustar, a)
    s = hp.Solver(hm, precision=precision, precond=precond)
    s.assemble_condense(dev(soa(u)), dev(uhat), dev(soa(ustar)), a)
    X = s.get_preconditioner().cpu().numpy()
    L = sysd["L"].tocsr()
    bs = 4 * pr.P
    for F in range(X.shape[0]):
        D = L[F * bs:(F + 1) * bs, F * bs:(F + 1) * bs].toarray()
        err = np.abs(X[F] @ D - np.eye(bs)).max()
        assert err <= tol * bs * np.abs(X[F]).max() * np.abs(D).max(), (F, err)


def _cfl_dt(pr, lam=6.0, rings=3, n_theta=24):
    """Time step of the local-CFL rule (CFL = 1 between the last implicit
    and the first explicit ring)."""
    es = pr.om.Es.reshape(-1, n_theta)
    cut = 0.5 * (es[rings - 1].max() + es[rings].min())
    return 2.0 * cut / (lam * (2 * pr.p + 1))


@pytest.mark.parametrize("name,passes", [("c1_p2", 1), ("pert_p3", 1), ("cyl_p3", 1),
                                         ("c1_p2", 2), ("cyl_p3", 2), ("c1_p1", 1),
                                         ("cyl_p4", 1), ("c1_p5", 1)])
def test_condense_solve_recover(name, passes):
    """Condensed system against the oracle's, the trace solve to 1e-12 with
    one and with two Gram-Schmidt passes per Arnoldi step, and recovery;
    p = 1 to 5 cover every face block size of the product kernel (8 to 24)."""
    pr, u = _build(name)
    om, hm = pr.om, pr.hm
    uhat, ustar = _stage_inputs(pr, u)
    # a_ii dt of a stage at the local-CFL time step on the cylinder (block
    # Jacobi GMRES stalls near local CFL ~ 1e3, far outside the method's
    # operating range); 0.05 on the vortex meshes
    a = 0.3 * _cfl_dt(pr) if name.startswith("cyl") else 0.05
    sysd = onw.condense(om, pr.ph, u, uhat, ustar, a)
    s = hp.Solver(hm, rtol=1e-12, max_iters=3000, restart=60, cgs_passes=passes)
    s.assemble_condense(dev(soa(u)), dev(uhat), dev(soa(ustar)), a)
    N = 4 * hm.Ntp
    t = torch.zeros(N, dtype=torch.float64, device="cuda")
    s.get_system(t=t)
    rng = np.random.default_rng(0)
    x = rng.normal(size=N)
    y = torch.zeros(N, dtype=torch.float64, device="cuda")
    s.matvec(dev(x), y)
    torch.cuda.synchronize()
    Lx = sysd["L"] @ x
    assert np.abs(host(y) - Lx).max() <= 1e-11 * max(1, np.abs(Lx).max())
    assert np.abs(host(t) - sysd["t"]).max() <= 1e-11 * max(1, np.abs(sysd["t"]).max())
    # the product the Krylov solver runs, L D^-1 x, with the solver's own
    # block inverses (checked against the oracle's blocks elsewhere)
    X = s.get_preconditioner().cpu().numpy()
    bs = X.shape[1]
    s.product(dev(x), y)
    torch.cuda.synchronize()
    LDx = sysd["L"] @ np.einsum("fab,fb->fa", X, x.reshape(-1, bs)).ravel()
    assert np.abs(host(y) - LDx).max() <= 1e-11 * max(1, np.abs(LDx).max())
    duh = torch.zeros(N, dtype=torch.float64, device="cuda")
    st = s.trace_solve(duh, allow_unconverged=True)
    duh_o = onw.trace_solve(sysd["L"], sysd["t"])
    # the GPU solution solves the oracle's trace system (relative residual)
    res_o = np.linalg.norm(sysd["t"] - sysd["L"] @ host(duh)) / np.linalg.norm(sysd["t"])
    assert st["rel_residual"] <= 1e-11 and res_o <= 1e-10, (st, res_o)
    assert np.abs(host(duh) - duh_o).max() <= 1e-6 * max(1e-300, np.abs(duh_o).max())
    du = torch.zeros(4 * hm.Nim * hm.Np, dtype=torch.float64, device="cuda")
    s.recover(dev(duh_o), du)
    torch.cuda.synchronize()
    du_o = onw.recover(sysd, duh_o).reshape(hm.Nim, pr.P, pr.P, 4)
    assert np.abs(unsoa(host(du), hm.Nim, pr.P) - du_o).max() <= 1e-11 * max(1e-300, np.abs(du_o).max())


@pytest.mark.parametrize("name", ["c1_p1", "c1_p2", "cyl_p4", "c1_p5"])
def test_trace_solve_fp32_form(name):
    """FP32 form (tableaux, trace matrix and preconditioner in FP32) at the
    face block sizes 8, 12, 20 and 24: the Arnoldi steps use the FP32
    preconditioned matrix, while the final residual is formed in FP64 from
    the unpreconditioned FP32 matrix by a separate kernel, so it must reach
    the GMRES tolerance; the solution agrees with the oracle's FP64 trace
    solution to the accuracy of an FP32 condensation (1e-3 relative)."""
    pr, u = _build(name)
    om, hm = pr.om, pr.hm
    uhat, ustar = _stage_inputs(pr, u)
    a = 0.3 * _cfl_dt(pr) if name.startswith("cyl") else 0.05
    sysd = onw.condense(om, pr.ph, u, uhat, ustar, a)
    s = hp.Solver(hm, precision="fp32", precond="fp32", rtol=1e-12, max_iters=3000,
                  restart=60)
    s.assemble_condense(dev(soa(u)), dev(uhat), dev(soa(ustar)), a)
    N = 4 * hm.Ntp
    duh = torch.zeros(N, dtype=torch.float64, device="cuda")
    st = s.trace_solve(duh, allow_unconverged=True)
    assert st["rel_residual"] <= 1e-11, st
    duh_o = onw.trace_solve(sysd["L"], sysd["t"])
    assert np.abs(host(duh) - duh_o).max() <= 1e-3 * np.abs(duh_o).max()


def _run_steps(pr, u0, dt, nsteps, precision="fp64", precond="fp64",
               tab="HIMEX2C", tol=1e-13, cgs_passes=1):
    om, hm = pr.om, pr.hm
    s = hp.Solver(hm, precision=precision, precond=precond, rtol=1e-12,
                  newton_tol=tol, max_iters=3000, cgs_passes=cgs_passes)
    stp = hp.ImexStepper(hm, s, tab)
    ud = dev(soa(u0))
    uo = u0.copy()
    errs, its = [], []
    for _ in range(nsteps):
        un, stats = stp.step(ud, dt)
        ud = un.clone()
        uo, _ = oimex.imex_step(om, pr.ph, oimex.TABLEAUS[tab](), uo, dt, tol=1e-13)
        ug = unsoa(host(ud), hm.Ne, pr.P)
        errs.append(rel_err(ug, uo))
        its.append([st["newton_iters"] for st in stats])
    return errs, its


def test_imex_steps_fp64_c1():
    """The FP64 GPU path matches the oracle within 1e-11 (relative, per
    conserved variable) after every one of 10 steps of the vortex case."""
    pr, _ = _build("c1_p2")
    u0 = fi.isentropic_vortex(pr.om.x, pr.om.y)
    errs, its = _run_steps(pr, u0, 0.01, 10)
    assert max(errs) <= 1e-11, errs


def test_imex_steps_fp64_cylinder_two_passes():
    """The Newton path with two Gram-Schmidt passes per Arnoldi step matches
    the oracle as the default single pass does."""
    pr, u = _build("cyl_p3")
    errs, _ = _run_steps(pr, u, _cfl_dt(pr), 2, cgs_passes=2)
    assert max(errs) <= 1e-11, errs


def test_solver_rejects_bad_options():
    pr, _ = _build("c1_p1")
    for kw in (dict(cgs_passes=3), dict(cgs_passes=-1), dict(jacobian_lag=-1),
               dict(restart=0), dict(forcing=-1e-3), dict(forcing=1.0),
               dict(rtol=1e-6, forcing=1e-7)):
        with pytest.raises(hp.HfrError):
            hp.Solver(pr.hm, **kw)


def test_imex_steps_fp64_cylinder_ars():
    pr, u = _build("cyl_p3")
    errs, _ = _run_steps(pr, u, _cfl_dt(pr), 2, tab="ARS222")
    assert max(errs) <= 1e-11, errs


def test_imex_steps_fp64_cylinder_p4():
    pr, u = _build("cyl_p4")
    errs, _ = _run_steps(pr, u, _cfl_dt(pr), 2)
    assert max(errs) <= 1e-11, errs


@pytest.mark.parametrize("pc", ["fp32", "bf16"])
def test_imex_steps_fp32_condensation(pc):
    """FP32 element LU / Schur products with FP64 residuals and Newton: the
    converged step still matches the FP64 oracle within 1e-8."""
    pr, _ = _build("c1_p2")
    u0 = fi.isentropic_vortex(pr.om.x, pr.om.y)
    errs, its = _run_steps(pr, u0, 0.01, 3, precision="fp32", precond=pc)
    assert max(errs) <= 1e-8, errs


def test_all_explicit_and_all_implicit_meshes():
    d, _ = c1_desc(n=4)
    for mask in (np.zeros(16, bool), np.ones(16, bool)):
        pr = Pair(d, 2, mask)
        u0 = fi.isentropic_vortex(pr.om.x, pr.om.y)
        errs, _ = _run_steps(pr, u0, 0.02, 1)
        assert max(errs) <= 1e-11, errs


def test_timing_categories():
    """Selected timer categories record their kernels only; all categories
    record every phase; the stage result does not depend on timing."""
    pr, _ = _build("c1_p2")
    u0 = fi.isentropic_vortex(pr.om.x, pr.om.y)
    s = hp.Solver(pr.hm, rtol=1e-12, newton_tol=1e-13, max_iters=3000)
    stp = hp.ImexStepper(pr.hm, s, "HIMEX2C")
    s.timing(only=["condense"])
    a, _ = stp.step(dev(soa(u0)), 0.01)
    a = host(a)
    t = s.timing(False)
    assert t["condense"][1] > 0 and t["condense"][0] > 0
    assert all(v[1] == 0 for k, v in t.items() if k != "condense"), t
    s.timing(True)
    b, _ = stp.step(dev(soa(u0)), 0.01)
    b = host(b)
    t = s.timing(False)
    assert all(t[k][1] > 0 for k in ("residual", "condense", "fill", "trace_solve", "recover")), t
    assert np.array_equal(a, b)
    lib = hp.load_library()
    assert lib.hfr_timing(s.handle, 7, None, None) != 0      # neither 0, 1 nor a selection


_ORACLE_STEPS = {}


@pytest.mark.parametrize("name,pc", [("cyl_p4", "fp32"), ("cyl_p4", "bf16"),
                                     ("c1_p5", "fp32"), ("c1_p5", "bf16")])
def test_imex_steps_fp32_condensation_high_order(name, pc):
    """The precision form at p = 4 (the 24x8 cylinder at the local-CFL time
    step) and p = 5 (the vortex case): FP32 element tableaux with an FP32 or
    a BF16 block-Jacobi preconditioner, FP64 residuals, Newton and Arnoldi;
    two IMEX steps match the FP64 oracle within 1e-8 after each step."""
    pr, u = _build(name)
    if name.startswith("c1"):
        u = fi.isentropic_vortex(pr.om.x, pr.om.y)
        dt = 0.01
    else:
        dt = _cfl_dt(pr)
    hm = pr.hm
    if name not in _ORACLE_STEPS:
        uo, seq = u.copy(), []
        for _ in range(2):
            uo, _ = oimex.imex_step(pr.om, pr.ph, oimex.himex2c(), uo, dt, tol=1e-13)
            seq.append(uo)
        _ORACLE_STEPS[name] = seq
    s = hp.Solver(hm, precision="fp32", precond=pc, rtol=1e-10, newton_tol=1e-13,
                  max_iters=3000)
    stp = hp.ImexStepper(hm, s, "HIMEX2C")
    ud = dev(soa(u))
    for k in range(2):
        un, stats = stp.step(ud, dt)
        ud = un.clone()
        err = rel_err(unsoa(host(ud), hm.Ne, pr.P), _ORACLE_STEPS[name][k])
        assert err <= 1e-8, (k, err, stats)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 1e-8)])
def test_imex_steps_with_forcing(precision, tol):
    """Inexact Newton (hfr_opts.gmres_forcing_max): the trace solves of a
    stage stop at the device's forcing term instead of the fixed tolerance.
    Two IMEX steps of the 24x8 p = 4 cylinder at the local-CFL time step
    match the oracle as without it, with fewer Krylov iterations."""
    pr, u = _build("cyl_p4")
    dt = _cfl_dt(pr)
    hm = pr.hm
    if "cyl_p4" not in _ORACLE_STEPS:
        uo, seq = u.copy(), []
        for _ in range(2):
            uo, _ = oimex.imex_step(pr.om, pr.ph, oimex.himex2c(), uo, dt, tol=1e-13)
            seq.append(uo)
        _ORACLE_STEPS["cyl_p4"] = seq
    its = {}
    for forcing in (0.0, 1e-3):
        print("forcing case:", precision, forcing, flush=True)
        s = hp.Solver(hm, precision=precision, precond=precision, rtol=1e-10,
                      newton_tol=1e-13, max_iters=3000, forcing=forcing)
        stp = hp.ImexStepper(hm, s, "HIMEX2C")
        ud = dev(soa(u))
        its[forcing] = 0
        for k in range(2):
            un, stats = stp.step(ud, dt)
            ud = un.clone()
            its[forcing] += sum(st["gmres_iters"] for st in stats)
            err = rel_err(unsoa(host(ud), hm.Ne, pr.P), _ORACLE_STEPS["cyl_p4"][k])
            assert err <= tol, (forcing, k, err, stats)
        s.close()
    assert its[1e-3] < its[0.0], its


_ORACLE_STEPS_B = {}


@pytest.mark.parametrize("name", ["c1_p1", "c1_p2", "cyl_p3", "cyl_p4", "c1_p5"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("kernel", ["blocked", "blocked_w8"])
def test_blocked_condensation_steps(name, precision, kernel):
    """The element elimination in panels of 16 exchanges with the update of
    the rest of the tableau on matrix-core tiles (every padded block count
    p = 1 to 5, four or eight waves per element): two IMEX steps against
    the oracle, 1e-11 in FP64 and 1e-8 with FP32 tableaux."""
    pr, u = _build(name)
    if name.startswith("c1"):
        u = fi.isentropic_vortex(pr.om.x, pr.om.y)
        dt = 0.01
    else:
        dt = _cfl_dt(pr)
    hm = pr.hm
    if name not in _ORACLE_STEPS_B:
        uo, seq = u.copy(), []
        for _ in range(2):
            uo, _ = oimex.imex_step(pr.om, pr.ph, oimex.himex2c(), uo, dt, tol=1e-13)
            seq.append(uo)
        _ORACLE_STEPS_B[name] = seq
    s = hp.Solver(hm, precision=precision, precond=precision, rtol=1e-10,
                  newton_tol=1e-13, max_iters=3000, condense=kernel)
    assert s.condense_choice()[0] == kernel
    stp = hp.ImexStepper(hm, s, "HIMEX2C")
    ud = dev(soa(u))
    print("blocked steps:", name, precision, kernel, flush=True)
    tol = 1e-11 if precision == "fp64" else 1e-8
    for k in range(2):
        un, stats = stp.step(ud, dt)
        ud = un.clone()
        err = rel_err(unsoa(host(ud), hm.Ne, pr.P), _ORACLE_STEPS_B[name][k])
        assert err <= tol, (k, err, stats)


def test_condense_autotuner_choice():
    """With the automatic choice the solver times the three condensation
    kernels on its first linearisation, keeps the fastest, and a second
    solver of the same order and precision reuses the choice; the step
    still matches the oracle."""
    pr, u = _build("cyl_p3")
    dt = _cfl_dt(pr)
    s = hp.Solver(pr.hm, precision="fp32", precond="fp32", rtol=1e-10, newton_tol=1e-13,
                  max_iters=3000)
    assert s.condense_choice()[0] == "auto"
    stp = hp.ImexStepper(pr.hm, s, "HIMEX2C")
    un, _ = stp.step(dev(soa(u)), dt)
    name, ms = s.condense_choice()
    assert name in ("sweep", "blocked", "blocked_w8"), name
    assert all(v > 0 for v in ms.values()), ms
    assert ms[name] == min(ms.values())
    uo, _ = oimex.imex_step(pr.om, pr.ph, oimex.himex2c(), u, dt, tol=1e-13)
    assert rel_err(unsoa(host(un), pr.hm.Ne, pr.P), uo) <= 1e-8
    s2 = hp.Solver(pr.hm, precision="fp32", precond="fp32")
    hp.ImexStepper(pr.hm, s2, "HIMEX2C").step(dev(soa(u)), dt)
    assert s2.condense_choice() == (name, ms)


@pytest.mark.parametrize("name,precision", [("cyl_p4", "fp32"), ("cyl_p4", "fp64"),
                                            ("c1_p5", "fp32")])
def test_compact_factors_after_newton(name, precision):
    """The compact element layout of the Newton path (blocked elimination,
    face blocks of 20 and 24 rows) as hfr_get_factors documents it: the
    Schur complement D - C A^-1 B as 4 x 4 column-major face sub-blocks at
    the start of the slot, then -A^-1 B (n x m, column-major, row p_k
    holding unknown k), checked with NumPy on the element blocks of the same
    (last) linearisation of an IMEX step."""
    pr, u = _build(name)
    hm = pr.hm
    dt = _cfl_dt(pr) if name.startswith("cyl") else 0.01
    s = hp.Solver(hm, precision=precision, precond=precision, keep_blocks=True,
                  condense="blocked", rtol=1e-10, newton_tol=1e-13, max_iters=3000)
    stp = hp.ImexStepper(hm, s, "HIMEX2C")
    stp.step(dev(soa(u)), dt)
    n, m = s.n, s.m
    bs, k2 = m // 4, (n + m) ** 2
    blk = torch.zeros(hm.Nim * k2, dtype=torch.float64, device="cuda")
    s.get_blocks(blk)
    F, piv = s.get_factors()
    torch.cuda.synchronize()
    G = host(blk).reshape(hm.Nim, n + m, n + m)
    raw = F.transpose(1, 2).reshape(hm.Nim, k2).double().cpu().numpy()   # slot order
    piv = piv.cpu().numpy().astype(np.int64)
    tol = 1e-10 if precision == "fp64" else 2e-4
    for k in range(hm.Nim):
        A, B, C, D = G[k, :n, :n], G[k, :n, n:], G[k, n:, :n], G[k, n:, n:]
        X = np.linalg.solve(A, B)
        S = D - C @ X
        scale = max(1.0, np.abs(S).max())
        for lr in range(4):
            for lc in range(4):
                o = (4 * lc + lr) * bs * bs
                sub = raw[k, o:o + bs * bs].reshape(bs, bs).T
                ref = S[lr * bs:(lr + 1) * bs, lc * bs:(lc + 1) * bs]
                err = np.abs(sub - ref).max()
                assert err <= tol * scale, (k, lr, lc, err)
        o = 16 * bs * bs
        Xc = raw[k, o:o + n * m].reshape(m, n).T
        err = np.abs(Xc[piv[k], :] + X).max()
        assert err <= tol * max(1.0, np.abs(X).max()), (k, err)


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-8), ("fp64", 1e-11)])
def test_compact_newton_restarts_match_oracle(precision, tol):
    """The compact Newton path forms only L D^-1; a Krylov cycle that ends
    short of its target restarts from the true residual t - L x summed from
    the element Schur sub-blocks.  With a restart length of 3 every solve
    restarts several times; two IMEX steps of the 24x8 p = 4 cylinder still
    match the oracle."""
    pr, u = _build("cyl_p4")
    dt = _cfl_dt(pr)
    hm = pr.hm
    if "cyl_p4" not in _ORACLE_STEPS:
        uo, seq = u.copy(), []
        for _ in range(2):
            uo, _ = oimex.imex_step(pr.om, pr.ph, oimex.himex2c(), uo, dt, tol=1e-13)
            seq.append(uo)
        _ORACLE_STEPS["cyl_p4"] = seq
    s = hp.Solver(hm, precision=precision, precond=precision, restart=3, rtol=1e-10,
                  newton_tol=1e-13, max_iters=3000, condense="blocked")
    stp = hp.ImexStepper(hm, s, "HIMEX2C")
    ud = dev(soa(u))
    for k in range(2):
        un, stats = stp.step(ud, dt)
        ud = un.clone()
        assert all(st["gmres_iters"] > 3 * st["newton_iters"] for st in stats), stats
        err = rel_err(unsoa(host(ud), hm.Ne, pr.P), _ORACLE_STEPS["cyl_p4"][k])
        assert err <= tol, (k, err, stats)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_matvec_after_compact_newton(precision):
    """After a Newton stage of the compact path (which forms only L D^-1),
    hfr_trace_matvec forms L and returns L x: it equals the Krylov product
    L D^-1 applied to D x, with D the inverse of each returned diagonal
    block inverse."""
    pr, u = _build("cyl_p4")
    hm = pr.hm
    s = hp.Solver(hm, precision=precision, precond=precision, condense="blocked")
    stp = hp.ImexStepper(hm, s, "HIMEX2C")
    stp.step(dev(soa(u)), _cfl_dt(pr))
    nt = 4 * hm.Ntp
    rng = np.random.default_rng(7)
    x = rng.standard_normal(nt)
    Dinv = s.get_preconditioner().cpu().numpy()
    bs = Dinv.shape[1]
    w = np.concatenate([np.linalg.solve(Dinv[f], x[f * bs:(f + 1) * bs])
                        for f in range(Dinv.shape[0])])
    y1 = torch.zeros(nt, dtype=torch.float64, device="cuda")
    y2 = torch.zeros(nt, dtype=torch.float64, device="cuda")
    s.matvec(dev(x), y1)
    s.product(dev(w), y2)
    torch.cuda.synchronize()
    a, b = host(y1), host(y2)
    tol = 1e-10 if precision == "fp64" else 1e-4
    assert np.abs(a - b).max() <= tol * np.abs(b).max(), float(np.abs(a - b).max())
