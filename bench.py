#!/usr/bin/env python
"""Benchmark of the hybridized IMEX hot path on one MI355X.

A step is one IMEX step (alg:imex): three explicit FR residuals and two
hybridized implicit stages, each solved by Newton with element-block
condensation, a GMRES trace solve and local recovery.  The metric is the
implicit-stage throughput: implicit DOF (N_im * Np * 4) per second of
implicit-stage wall time (from the stage's entry to R_i ready: u*, the
initial trace, every Newton iteration and R_i), averaged over the timed
stages, for the FP32 condensation form with an FP32 block-Jacobi
preconditioner (``value``), next to the same form with a BF16
preconditioner and the FP64 form on the same workload.

Prints ONE JSON line.  Only one GPU is supported.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"hbm_gbs": 8000.0, "fp64_tflops": 78.6, "fp32_tflops": 157.3}
MACH = 0.2
WAVE = 1.0 + 1.0 / MACH          # |v| + c of the free stream (|v| = 1)
THETA = 100.0                    # EDAC 1/M^2 of the airfoil case (M = 0.1)
WAVE_EDAC = 1.5 + math.sqrt(0.25 + THETA)   # EDAC wave speed of the stream


def cylinder_workload(name):
    import fr_inputs as fi
    if name == "c2":
        n_theta, n_r, p, first, ratio = 128, 64, 3, 1e-4, 1.15
    elif name in ("c3", "c3_small"):
        # p = 4 with the outer radius of c2; c3_small is a 64x20 mesh of the
        # same radii that the CPU oracle solves within a test
        n_theta, n_r = (256, 128) if name == "c3" else (64, 20)
        p, first = 4, 1e-4
        gap = first * (1.15 ** 64 - 1.0) / 0.15
        ratio = fi.ogrid_ratio_for_outer(n_r, first, gap)
    else:
        raise ValueError(name)
    d = fi.cylinder_ogrid(n_theta, n_r, first=first, ratio=ratio)
    return d, p, n_theta, n_r, first, ratio


def c5_instances(seed=5, count=64, p=3):
    """The batch of independent cylinders: quads per instance log-uniform in
    [2e3, 2e4] with n_theta = 2 n_r, wall-normal ratio U[1.1, 1.25], first
    cell 1e-4 D, p = 3; each instance's implicit rings and time step by the
    local-CFL rule with IF ~ 0.2 of its own rings."""
    import fr_inputs as fi
    rng = np.random.default_rng(seed)
    specs = []
    for _ in range(count):
        nq = float(np.exp(rng.uniform(np.log(2e3), np.log(2e4))))
        nr = max(6, int(round(np.sqrt(nq / 2.0))))
        specs.append((2 * nr, nr, 1e-4, float(rng.uniform(1.1, 1.25))))
    descs = [fi.cylinder_ogrid(nt, nr, first=first, ratio=ratio)
             for nt, nr, first, ratio in specs]
    return descs, specs, p


def describe(name):
    if name == "c5":
        descs, specs, p = c5_instances()
        nq = sum(nt * nr for nt, nr, _, _ in specs)
        return (f"2D Euler (viscous terms not built), batch of {len(specs)} independent "
                f"cylinder O-grids ({nq} quads, 2e3..2e4 each), p={p}, ratio 1.1..1.25, "
                f"implicit = local CFL > 1 per instance (IF ~ 0.2), own time step each, "
                f"one launch per kernel for all, HIMEX2C pair")
    d, p, nt, nr, first, ratio = cylinder_workload(name)
    return (f"2D Euler (viscous terms not built), circular cylinder O-grid "
            f"{nt}x{nr} quads, p={p}, first cell {first:g} D, ratio {ratio:.4f}, "
            f"Mach {MACH}, implicit = local CFL > 1 (IF ~ 0.2), HIMEX2C pair")


def build_batch(hp, if_target=0.2, seed=2):
    """The independent-cylinder batch as one mesh with per-instance time
    steps (the stage calls then take dt = 1)."""
    import fr_inputs as fi
    descs, specs, p = c5_instances()
    uinf = fi.freestream_state(MACH)
    masks, dts = [], []
    for d, (nt, nr, first, ratio) in zip(descs, specs):
        probe = hp.Mesh(d, p, uinf=uinf, host_only=True)
        es = probe.maps()["es"].reshape(nr, nt)
        J = max(1, int(round(if_target * nr)))
        cut = 0.5 * (es[J - 1].max() + es[J].min())
        masks.append(es.ravel() <= cut)
        dts.append(2.0 * cut / (WAVE * (2 * p + 1)))
    batch = fi.concat_meshes(descs)
    mesh = hp.Mesh(batch, p, implicit_mask=np.concatenate(masks), uinf=uinf)
    mesh.set_instance_dt(dts)
    P = p + 1
    u = fi.perturb_state(np.broadcast_to(uinf, (mesh.Ne, P, P, 4)).copy(), 1e-3, seed)
    return mesh, hp.soa_from_elements(u).ravel(), 1.0, None


def build_case(hp, name, if_target=0.2, seed=2, efr=False, physics="euler"):
    """Mesh, partition (CFL rule), time step and initial state; ``efr``
    selects the interior-embedded trace, ``physics`` the Euler or the EDAC
    equations (free stream P = 0, |v| = 1, seeded 1e-3 additive noise)."""
    import fr_inputs as fi
    if name == "c5":
        return build_batch(hp, if_target, seed)
    d, p, nt, nr, first, ratio = cylinder_workload(name)
    edac = physics == "edac"
    uinf = fi.edac_freestream() if edac else fi.freestream_state(MACH)
    probe = hp.Mesh(d, p, uinf=uinf, host_only=True)
    es = probe.maps()["es"].reshape(nr, nt)
    J = max(1, int(round(if_target * nr)))
    es_cut = 0.5 * (es[J - 1].max() + es[J].min())
    # local CFL_k = dt * lambda * (2p+1) / (2 E_s,k); implicit iff CFL_k > 1
    dt = 2.0 * es_cut / ((WAVE_EDAC if edac else WAVE) * (2 * p + 1))
    mesh = hp.Mesh(d, p, es_cutoff=es_cut, uinf=uinf, efr=efr, physics=physics,
                   theta=THETA)
    xy = mesh.maps()["sol_xy"]
    P = p + 1
    u = np.broadcast_to(uinf, (mesh.Ne, P, P, 4)).copy()
    if edac:
        u = u + 1e-3 * np.random.default_rng(seed).uniform(-1.0, 1.0, size=u.shape)
    else:
        u = fi.perturb_state(u, 1e-3, seed)
    return mesh, hp.soa_from_elements(u).ravel(), dt, xy


def condense_flops(n, m):
    """Algorithmic FLOPs of one element condensation: LU of A (2n^3/3),
    A^-1 [B r] (2n^2 m + 2n^2), C X (2 n m^2 + 2 n m), D - C X (m^2)."""
    return 2 * n ** 3 / 3 + 2 * n * n * m + 2 * n * m * m + 2 * n * n + 2 * n * m + m * m


CONDENSE = "auto"
DAMPING = False
# inexact Newton: ceiling of the per-solve Krylov tolerance (hfr_opts.
# gmres_forcing_max); the same policy in every form
FORCING = 1e-3


def run_form(hp, torch, mesh, u0, dt, precision, precond, steps, warmup,
             newton_tol, graph=False):
    """graph: Newton iterations replayed as recorded graphs; the timed region
    then runs without any event timer (timers select the eager queue)."""
    solver = hp.Solver(mesh, precision=precision, precond=precond,
                       restart=30, max_iters=400, rtol=1e-6,
                       newton_max_iters=30, newton_tol=newton_tol,
                       condense=CONDENSE, damping=DAMPING, graph=graph,
                       forcing=FORCING)
    stp = hp.ImexStepper(mesh, solver, "HIMEX2C")
    ud = torch.from_numpy(u0).cuda()
    u = ud.clone()
    for _ in range(warmup):
        un, _ = stp.step(u, dt)
        u = un.clone()
    torch.cuda.synchronize()
    # timed region: no event timers (with them the solver queues no
    # linearisation ahead of its Newton test, and each adds event records)
    impl_ms, newton, gmres, queued, replays = [], [], [], [], 0
    t0 = time.perf_counter()
    for _ in range(steps):
        un, stats = stp.step(u, dt)
        u = un.clone()
        for s in stats:
            impl_ms.append(s["implicit_ms"])
            newton.append(s["newton_iters"])
            gmres.append(s["gmres_iters"])
            queued.append(s["queued_linearisations"])
            replays += s["graph_replays"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = u.cpu().numpy()

    def timed_pass(only):
        if only is None:
            solver.timing(True)
        else:
            solver.timing(only=only)
        uu = u.clone()
        for _ in range(min(3, steps)):
            un, _ = stp.step(uu, dt)
            uu = un.clone()
        torch.cuda.synchronize()
        return solver.timing(False)
    # the bandwidth-bound kernels, each timed alone (events around its own
    # launches only): explicit residual (K2) and the Arnoldi product (K8)
    hbm = {k: timed_pass([k]) [k] for k in ("explicit", "spmv")}
    # the roofline kernel (the condensation) alone, events around its launches
    timers = timed_pass(["condense"]) if not graph else None
    # phase breakdown from a separate, fully instrumented pass
    phases = timed_pass(None)
    choice, cand = solver.condense_choice()
    res = dict(wall_s=wall, impl_ms=impl_ms, newton=newton, gmres=gmres, queued=queued,
               graph_replays=replays,
               timers=timers, phases=phases, hbm=hbm, state=out,
               workspace=solver.workspace_bytes,
               condense=dict(kernel=choice, candidates_ms=cand))
    solver.close()
    return res


def first_stage(hp, torch, mesh, u0, dt, precision, precond, newton_tol):
    """State and trace after the first implicit stage of a step (stages 0
    and 1 of imex_stage), for the comparison with the oracle."""
    import ctypes
    from paper_2401_16632_amd import _abi
    solver = hp.Solver(mesh, precision=precision, precond=precond, restart=30,
                       max_iters=3000, rtol=1e-10, newton_max_iters=30,
                       newton_tol=newton_tol, forcing=FORCING)
    stp = hp.ImexStepper(mesh, solver, "HIMEX2C")
    ud = torch.from_numpy(u0).cuda()
    lib = hp.load_library()
    st = _abi.ImexState(ud.data_ptr(), stp.u.data_ptr(), stp.uhat.data_ptr(),
                        stp.R_im.data_ptr(), stp.R_ex.data_ptr())
    ns = _abi.HfrNewtonStats()
    for stage in (0, 1):
        rc = lib.imex_stage(mesh.handle, solver.handle, ctypes.byref(stp.tab), stage,
                            float(dt), ctypes.byref(st), ctypes.byref(ns), None)
        if rc != 0:
            raise RuntimeError(lib.fr_last_error().decode())
    torch.cuda.synchronize()
    out = stp.u.cpu().numpy(), stp.uhat.cpu().numpy()
    solver.close()
    return out


def measured_traffic(workload, kernel):
    """HBM bytes per launch of the condensation kernel from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE runs scaled by a
    plain copy of known size), or None when the kernel sources have changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hbm_counters_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for ln in open(path):
        if ":" in ln and not ln.startswith(" "):
            k, v = ln.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("condense_kernel", "").find(kernel) < 0:
        return None
    h = hashlib.sha256()
    for f in ("kernels_condense.hip", "internal.h", "euler.h", "wave_ops.h"):
        with open(os.path.join(ROOT, "paper_2401_16632_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != vals.get("condense_source_sha256"):
        return None
    return float(vals["condense_traffic_bytes_per_launch"])


CK_KERNEL = {"sweep": "k_condense_sweep", "blocked": "k_condense_blocked",
             "blocked_w8": "k_condense_blocked"}


def roofline(form, mesh, timers, precision, workload="c2", phases=None, ck="sweep"):
    """Roofline of the kernel with the largest share of the stage (from the
    instrumented pass when given), measured by the events of the timed
    region when that kernel was timed there."""
    n, m = 4 * mesh.Np, 16 * mesh.P
    share = phases if phases is not None else timers
    cand = {k: share[k][0] for k in ("condense", "spmv", "explicit")}
    dom = max(cand, key=cand.get)
    src = timers if timers[dom][1] > 0 else share
    cms, ccnt = src["condense"]
    sms, scnt = src["spmv"]
    ems, ecnt = src["explicit"]
    if dom == "condense":
        # the element elimination and the Schur complement from C's
        # structure (one launch per linearisation with the blocked kernel,
        # which ends with the lift; the sweep is followed by its own lift
        # launch, timed together)
        fl = condense_flops(n, m) * mesh.Nim
        avg = cms / max(1, ccnt) * 1e-3
        pk = PEAK["fp32_tflops"] if precision == "fp32" else PEAK["fp64_tflops"]
        ach = fl / avg / 1e12
        kname = CK_KERNEL.get(ck, "k_condense_sweep")
        traffic = (measured_traffic(workload, f"{kname}<{mesh.P}, float")
                   if precision == "fp32" else None)
        label = (f"{kname} (elimination + Schur lift)" if kname == "k_condense_blocked"
                 else f"condense ({kname} + k_schur_lift)")
        return dict(kernel=label,
                    bound="mfma" if kname == "k_condense_blocked" else "alu",
                    achieved=ach, peak=pk,
                    unit="TFLOP/s", frac=ach / pk, traffic=traffic,
                    launches=ccnt, avg_ms=avg * 1e3,
                    algorithmic_per_launch=fl)
    if dom == "spmv":
        bs = 4 * mesh.P
        nnzb = mesh_blocks(mesh)
        vb = 8 if precision == "fp64" else 4
        by = nnzb * bs * bs * vb + 2 * 4 * mesh.Ntp * 8
        avg = sms / max(1, scnt) * 1e-3
        ach = by / avg / 1e9
        return dict(kernel="spmv", bound="hbm", achieved=ach,
                    peak=PEAK["hbm_gbs"], unit="GB/s", frac=ach / PEAK["hbm_gbs"],
                    traffic=None, launches=scnt, avg_ms=avg * 1e3,
                    algorithmic_per_launch=by)
    by = explicit_bytes(mesh)
    avg = ems / max(1, ecnt) * 1e-3
    ach = by / avg / 1e9
    return dict(kernel="explicit_rhs", bound="hbm", achieved=ach,
                peak=PEAK["hbm_gbs"], unit="GB/s", frac=ach / PEAK["hbm_gbs"],
                traffic=None, launches=ecnt, avg_ms=avg * 1e3,
                algorithmic_per_launch=by)


def mesh_blocks(mesh):
    """Number of face blocks of the trace matrix (self + the other trace
    faces of the two elements sharing each trace face)."""
    mp = mesh.maps()
    fk = mp["face_kind"]
    fe = mp["face_elem"]
    trace = fk == 2
    per_elem = np.zeros(mesh.Ne, np.int64)
    for s in range(2):
        e = fe[trace, s]
        np.add.at(per_elem, e, 1)
    return int(sum(per_elem[fe[f, 0]] + per_elem[fe[f, 1]] - 1
                   for f in np.nonzero(trace)[0]))


def explicit_bytes(mesh):
    """Per launch: read u and write R of every explicit element (4 Np FP64
    each), its 4 vertices (64 B) and its 4 face records (32 B each)."""
    return mesh.Nex * (2 * 4 * mesh.Np * 8 + 64 + 4 * 32)


# form: (tableau precision, preconditioner storage, Newton iterations as
# replayed graphs)
FORMS = {"fp32": ("fp32", "fp32", False), "fp32_bf16": ("fp32", "bf16", False),
         "fp32_graph": ("fp32", "fp32", True),
         "fp64": ("fp64", "fp64", False)}


def oracle_first_stage(name, threads):
    """The oracle (never tuned) on a bounded sample: the first implicit
    stage of step 1 of workload ``name`` (Newton to 1e-12 with exact element
    Jacobians, condensation and a sparse direct trace solve), with the BLAS
    thread pool limited to ``threads``.  Returns (seconds, Newton
    iterations, implicit DOF, oracle mesh, u_im, uhat)."""
    import fr_inputs as fi
    import oracle
    from oracle import newton as onw, residual as ores, imex as oimex
    from threadpoolctl import threadpool_limits
    d, p, nt, nr, first, ratio = cylinder_workload(name)
    uinf = fi.freestream_state(MACH)
    m0 = oracle.QuadMesh(d, p, uinf=uinf)
    es = m0.Es.reshape(nr, nt)
    J = max(1, int(round(0.2 * nr)))
    es_cut = 0.5 * (es[J - 1].max() + es[J].min())
    dt = 2.0 * es_cut / (WAVE * (2 * p + 1))
    om = oracle.QuadMesh(d, p, es_cutoff=es_cut, uinf=uinf)
    P = p + 1
    u = fi.perturb_state(np.broadcast_to(uinf, (om.Ne, P, P, 4)).copy(), 1e-3, 2)
    ph = oracle.Euler()
    tab = oimex.himex2c()
    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        u1 = u.copy()
        u1[om.exp_elems] += dt * tab.Abar[1, 0] * ores.fr_residual(om, ph, u)[om.exp_elems]
        u_im, uhat, its = onw.solve_stage(om, ph, u1, u[om.imp_elems], dt * tab.A[0, 0],
                                          tol=1e-12, maxit=30)
        el = time.perf_counter() - t0
    return el, its, om.Nim * P * P * 4, om, u_im, uhat


def oracle_leg(hp, torch, name, forms):
    """cpu_baseline (the oracle on one host core and on all of them) and the
    error of every GPU form against the oracle on the same stage."""
    ncpu = os.cpu_count() or 1
    el1, its, dof, om, u_im, uhat = oracle_first_stage(name, 1)
    eln, _, _, _, _, _ = oracle_first_stage(name, ncpu)
    d, p, nt, nr, first, ratio = cylinder_workload(name)
    base = dict(value=dof / eln, unit="implicit-stage DOF/s", cores=ncpu,
                kind="oracle", value_1core=dof / el1,
                sample=(f"first implicit stage of step 1 of the {nt}x{nr} p={p} cylinder "
                        f"of the benchmark's radii, CFL rule and seed ({om.Nim} implicit "
                        f"elements, Newton to 1e-12 in {its} iterations): "
                        f"{eln:.1f} s with {ncpu} BLAS threads, {el1:.1f} s with one"))
    mesh, u0, dt, _ = build_case(hp, name)
    errs = {}
    for f in forms:
        if FORMS[f][2]:                  # the graph form repeats an eager form
            continue
        ug, uh = first_stage(hp, torch, mesh, u0, dt, *FORMS[f][:2], 1e-12)
        ue = ug.reshape(4, mesh.Ne, mesh.Np)[:, om.imp_elems]
        uo = hp.soa_from_elements(u_im)
        num = np.abs(ue - uo).max(axis=(1, 2))
        errs[f] = float((num / np.abs(uo).max(axis=(1, 2))).max())
        ht = np.abs(uh.reshape(-1, 4) - uhat).max(axis=0) / np.abs(uhat).max(axis=0)
        errs[f + "_trace"] = float(ht.max())
    errs["sample"] = (f"first implicit stage, {nt}x{nr} p={p} cylinder, Newton to 1e-12 "
                      f"on both sides; max over conserved variables of "
                      f"|u - u_oracle|_inf / |u_oracle|_inf over the implicit elements "
                      f"(and over the trace)")
    mesh.close()
    return base, errs


def filter_rate(torch, mesh, u0, reps=20, replays=20):
    """Modal filter (Appendix B, airfoil parameters) on the whole state.
    Launches are captured in a HIP graph (reps per graph) so that host
    launch cost stays out of the figure; the time per launch is the event
    time of the replays divided by the launches.  A plain device copy of the
    same bytes, timed the same way, shows what HBM reaches at this size."""
    u = torch.from_numpy(u0).cuda()
    dst = torch.empty_like(u)
    prm = dict(alpha=100.0, s=1.0, eta_c=3.0, kappa=1.0)

    def per_launch(fn):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(3):
                fn()
        torch.cuda.current_stream().wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(reps):
                fn()
        g.replay()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(replays):
            g.replay()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) * 1e3 / (reps * replays)

    us = per_launch(lambda: mesh.modal_filter(u, **prm))
    copy_us = per_launch(lambda: dst.copy_(u))
    nbytes = 2 * 8 * 4 * mesh.Ne * mesh.Np
    return {"us_per_launch": us, "algorithmic_bytes": nbytes,
            "achieved_GBps": nbytes / us * 1e-3,
            "frac_of_hbm": nbytes / us * 1e-3 / PEAK["hbm_gbs"],
            "same_size_copy_us": copy_us}


def copy_calibration(nbytes, reps=5):
    """A plain device copy of known size (read nbytes, write nbytes), the
    reference for the HBM traffic counters."""
    import torch
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 4, "reps": reps}))


def hbm_kernels(mesh, res, precision):
    """Bandwidth of the explicit residual (K2) and of the Arnoldi product
    (K8, the trace SpMV) from the passes that time each alone: algorithmic
    bytes per launch over the average launch time."""
    out = {}
    ms, cnt = res["hbm"]["explicit"]
    if cnt:
        by = explicit_bytes(mesh)
        gbs = by / (ms / cnt * 1e-3) / 1e9
        out["explicit_rhs"] = dict(bytes_per_launch=by, avg_us=ms / cnt * 1e3,
                                   achieved_GBps=gbs, frac=gbs / PEAK["hbm_gbs"],
                                   launches=cnt)
    ms, cnt = res["hbm"]["spmv"]
    if cnt:
        bs = 4 * mesh.P
        vb = 8 if precision == "fp64" else 4
        by = mesh_blocks(mesh) * bs * bs * vb + 2 * 4 * mesh.Ntp * 8
        gbs = by / (ms / cnt * 1e-3) / 1e9
        out["trace_spmv"] = dict(bytes_per_launch=by, avg_us=ms / cnt * 1e3,
                                 achieved_GBps=gbs, frac=gbs / PEAK["hbm_gbs"],
                                 launches=cnt)
    return out


def form_summary(mesh, rr, precision):
    dof = mesh.Nim * mesh.Np * 4
    return {
        "implicit_dof_per_s": dof / (np.mean(rr["impl_ms"]) * 1e-3),
        "implicit_ms_per_stage": float(np.mean(rr["impl_ms"])),
        "newton_iters_per_stage": float(np.mean(rr["newton"])),
        "gmres_iters_per_stage": float(np.mean(rr["gmres"])),
        "queued_linearisations_per_stage": float(np.mean(rr["queued"])),
        "hbm_kernels": hbm_kernels(mesh, rr, precision),
        "phase_ms_instrumented_pass": {k: v[0] for k, v in rr["phases"].items()},
        "phase_launches_instrumented_pass": {k: v[1] for k, v in rr["phases"].items()},
        "workspace_bytes": rr["workspace"],
        "condense_kernel": rr["condense"],
    }


def rel_diff(a, b):
    a, b = a.reshape(4, -1), b.reshape(4, -1)
    return float((np.abs(a - b).max(axis=1) /
                  np.maximum(np.abs(b).max(axis=1), 1e-300)).max())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3", choices=["c2", "c3", "c3_small", "c5"])
    ap.add_argument("--forms", default="fp32,fp32_bf16,fp64,fp32_graph")
    ap.add_argument("--no-efr", action="store_true",
                    help="skip the interior-embedded trace forms")
    ap.add_argument("--newton-tol", type=float, default=1e-10)
    ap.add_argument("--forcing", type=float, default=1e-3,
                    help="ceiling of the Krylov tolerance inside Newton (0: every "
                         "solve to 1e-6)")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (cpu_baseline and error_vs_oracle)")
    ap.add_argument("--oracle-workload", default="c3_small",
                    choices=["c3_small", "c2", "c3"])
    ap.add_argument("--no-edac", action="store_true",
                    help="skip the EDAC forms")
    ap.add_argument("--no-filter", action="store_true",
                    help="skip the modal-filter measurement")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter reference)")
    ap.add_argument("--condense", default="auto", choices=["auto", "sweep", "blocked", "blocked_w8"],
                    help="element elimination kernel inside Newton")
    args = ap.parse_args()
    global CONDENSE, DAMPING, FORCING
    CONDENSE = args.condense
    FORCING = args.forcing
    # the batch's most stretched instances start impulsively at local CFL
    # ~50 at the wall: Newton needs the admissible-step damping there
    DAMPING = args.workload == "c5"
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2401_16632_amd as hp
    hp.load_library()
    mesh, u0, dt, _ = build_case(hp, args.workload)
    forms = args.forms.split(",")
    for f in forms:
        if f not in FORMS:
            raise SystemExit(f"unknown form {f}")
    results = {}
    for f in forms:
        results[f] = run_form(hp, torch, mesh, u0, dt, *FORMS[f][:2], args.steps,
                              args.warmup, args.newton_tol, graph=FORMS[f][2])
        r = results[f]
        print(f"# form {f}: wall {r['wall_s']:.3f} s, implicit ms/stage "
              f"{np.mean(r['impl_ms']):.3f}, newton {np.mean(r['newton']):.2f}, "
              f"gmres/stage {np.mean(r['gmres']):.1f}", file=sys.stderr, flush=True)
    dof = mesh.Nim * mesh.Np * 4
    main_form = "fp32" if "fp32" in results else forms[0]
    r = results[main_form]
    stage_s = np.mean(r["impl_ms"]) * 1e-3
    prec = FORMS[main_form][0]
    line = {
        "metric": "Implicit-stage DOF/s, FP32-MFMA batched vs FP64 hybridized, at matched error",
        "value": dof / stage_s,
        "unit": "implicit-stage DOF/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["wall_s"] * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": describe(args.workload),
                   "n_elems": mesh.Ne, "n_implicit": mesh.Nim,
                   "implicit_dof": dof, "dt": dt,
                   "newton_tol": args.newton_tol,
                   "krylov_tolerance": (f"inexact Newton, per-solve relative tolerance "
                                        f"in [1e-6, {args.forcing:g}] from the quadratic "
                                        f"model of the next residual" if args.forcing > 0
                                        else "1e-6 every solve"),
                   "form": main_form,
                   "stage_timer": "imex_stage entry (queued work drained) to R_i ready"},
        "roofline": roofline(main_form, mesh, r["timers"], prec, args.workload,
                             r["phases"], r["condense"]["kernel"]),
    }
    for f, rr in results.items():
        line[f"{f}_form"] = form_summary(mesh, rr, FORMS[f][0])
        if FORMS[f][2]:
            line[f"{f}_form"]["graph_replays_per_stage"] = (rr["graph_replays"] /
                                                            len(rr["impl_ms"]))
    if "fp32_graph" in results and "fp32" in results:
        line["fp32_graph_equals_fp32"] = bool(np.array_equal(results["fp32_graph"]["state"],
                                                             results["fp32"]["state"]))
    if "fp64" in results:
        for f in results:
            if f != "fp64":
                line[f"{f}_vs_fp64_rel_err"] = rel_diff(results[f]["state"],
                                                        results["fp64"]["state"])
                line[f"speedup_{f}_over_fp64"] = (np.mean(results["fp64"]["impl_ms"]) /
                                                  np.mean(results[f]["impl_ms"]))
    for f in results:
        results[f]["state"] = None
    if args.workload == "c5":
        args.no_efr = args.no_edac = True
        line["config"]["instances"] = 64
    if not args.no_efr:
        # the same workload with the interior-embedded trace (EFR)
        mesh_e, u0e, dte, _ = build_case(hp, args.workload, efr=True)
        efr_states = {}
        for f in ("fp32", "fp64"):
            rr = run_form(hp, torch, mesh_e, u0e, dte, *FORMS[f][:2], args.steps,
                          args.warmup, args.newton_tol)
            efr_states[f] = rr["state"]
            line[f"efr_{f}_form"] = form_summary(mesh_e, rr, f)
            line[f"efr_{f}_form"]["trace_unknowns"] = 4 * mesh_e.Ntp
            print(f"# efr form {f}: implicit ms/stage {np.mean(rr['impl_ms']):.3f}, "
                  f"gmres/stage {np.mean(rr['gmres']):.1f}", file=sys.stderr, flush=True)
        line["efr_fp32_vs_fp64_rel_err"] = rel_diff(efr_states["fp32"], efr_states["fp64"])
        line["hfr_trace_unknowns"] = 4 * mesh.Ntp
        mesh_e.close()
    if not args.no_edac:
        # the same O-grid and partition with the EDAC equations (theta = 100)
        mesh_d, u0d, dtd, _ = build_case(hp, args.workload, physics="edac")
        edac_states = {}
        for f in ("fp32", "fp64"):
            rr = run_form(hp, torch, mesh_d, u0d, dtd, *FORMS[f][:2], args.steps,
                          args.warmup, args.newton_tol)
            edac_states[f] = rr["state"]
            line[f"edac_{f}_form"] = form_summary(mesh_d, rr, f)
            line[f"edac_{f}_form"].update(theta=THETA, dt=dtd)
            print(f"# edac form {f}: implicit ms/stage {np.mean(rr['impl_ms']):.3f}, "
                  f"gmres/stage {np.mean(rr['gmres']):.1f}", file=sys.stderr, flush=True)
        line["edac_fp32_vs_fp64_rel_err"] = rel_diff(edac_states["fp32"], edac_states["fp64"])
        mesh_d.close()
    if not args.no_filter:
        line["modal_filter"] = filter_rate(torch, mesh, u0)
    mesh.close()
    if not args.no_cpu_baseline:
        print("# oracle leg", file=sys.stderr, flush=True)
        base, errs = oracle_leg(hp, torch, args.oracle_workload, forms)
        line["cpu_baseline"] = base
        line["error_vs_oracle"] = errs
    print(json.dumps(line))


if __name__ == "__main__":
    main()
