#!/usr/bin/env python
"""Benchmark of the hybridized IMEX hot path on one MI355X.

A step is one IMEX step (alg:imex): three explicit FR residuals and two
hybridized implicit stages, each solved by Newton with element-block
condensation, a GMRES trace solve and local recovery.  The metric is the
implicit-stage throughput: implicit DOF (N_im * Np * 4) per second of
implicit-stage wall time, averaged over the timed stages, for the FP32
condensation form (``value``) next to the FP64 form on the same workload.

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
    elif name == "c3":
        n_theta, n_r, p, first = 256, 128, 4, 1e-4
        gap = first * (1.15 ** 64 - 1.0) / 0.15      # same outer radius as c2
        ratio = fi.ogrid_ratio_for_outer(n_r, first, gap)
    else:
        raise ValueError(name)
    d = fi.cylinder_ogrid(n_theta, n_r, first=first, ratio=ratio)
    return d, p, n_theta, n_r, first, ratio


def describe(name):
    d, p, nt, nr, first, ratio = cylinder_workload(name)
    return (f"2D Euler, circular cylinder O-grid {nt}x{nr} quads, p={p}, "
            f"first cell {first:g} D, ratio {ratio:.4f}, Mach {MACH}, "
            f"implicit = local CFL > 1 (IF ~ 0.2), HIMEX2C pair")


def build_case(hp, name, if_target=0.2, seed=2, efr=False, physics="euler"):
    """Mesh, partition (CFL rule), time step and initial state; ``efr``
    selects the interior-embedded trace, ``physics`` the Euler or the EDAC
    equations (free stream P = 0, |v| = 1, seeded 1e-3 additive noise)."""
    import fr_inputs as fi
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


def run_form(hp, torch, mesh, u0, dt, precision, precond, steps, warmup,
             newton_tol):
    solver = hp.Solver(mesh, precision=precision, precond=precond,
                       restart=30, max_iters=400, rtol=1e-6,
                       newton_max_iters=30, newton_tol=newton_tol)
    stp = hp.ImexStepper(mesh, solver, "HIMEX2C")
    ud = torch.from_numpy(u0).cuda()
    u = ud.clone()
    for _ in range(warmup):
        un, _ = stp.step(u, dt)
        u = un.clone()
    torch.cuda.synchronize()
    # timed region: only the condensation sweep (the roofline kernel) is
    # bracketed by events; every timed launch adds two event records
    solver.timing(only=["condense"])
    impl_ms, newton, gmres = [], [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        un, stats = stp.step(u, dt)
        u = un.clone()
        for s in stats:
            impl_ms.append(s["implicit_ms"])
            newton.append(s["newton_iters"])
            gmres.append(s["gmres_iters"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    timers = solver.timing(False)
    out = u.cpu().numpy()
    # phase breakdown from a separate, fully instrumented pass
    solver.timing(True)
    uu = u.clone()
    for _ in range(min(3, steps)):
        un, _ = stp.step(uu, dt)
        uu = un.clone()
    torch.cuda.synchronize()
    phases = solver.timing(False)
    res = dict(wall_s=wall, impl_ms=impl_ms, newton=newton, gmres=gmres,
               timers=timers, phases=phases, state=out, nblocks=None,
               workspace=solver.workspace_bytes)
    solver.close()
    return res


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


def roofline(form, mesh, timers, precision, workload="c2", phases=None):
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
        fl = condense_flops(n, m) * mesh.Nim
        avg = cms / max(1, ccnt) * 1e-3
        pk = PEAK["fp32_tflops"] if precision == "fp32" else PEAK["fp64_tflops"]
        ach = fl / avg / 1e12
        traffic = (measured_traffic(workload, f"k_condense_sweep<{mesh.P}, float")
                   if precision == "fp32" else None)
        return dict(kernel="condense", bound="alu", achieved=ach, peak=pk,
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


def cpu_baseline(name):
    """The oracle timed on a bounded sample of the same workload: the first
    implicit stage of step 1 (Newton to 1e-10 with exact element Jacobians,
    condensation and a sparse direct trace solve), single-threaded."""
    import fr_inputs as fi
    import oracle
    from oracle import newton as onw, imex as oimex
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
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        _, _, its = onw.solve_stage(om, ph, u, u[om.imp_elems], dt * tab.A[0, 0],
                                    tol=1e-10, maxit=30)
        el = time.perf_counter() - t0
    dof = om.Nim * P * P * 4
    return dict(value=dof / el, unit="implicit-stage DOF/s", cores=1,
                kind="oracle",
                sample=(f"first implicit stage of step 1 on the full workload "
                        f"({om.Nim} implicit elements, Newton to 1e-10 in {its} "
                        f"iterations), {el:.1f} s single-threaded NumPy/SciPy"))


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=["c2", "c3"])
    ap.add_argument("--forms", default="fp32,fp64")
    ap.add_argument("--no-efr", action="store_true",
                    help="skip the interior-embedded trace forms")
    ap.add_argument("--newton-tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-edac", action="store_true",
                    help="skip the EDAC forms")
    ap.add_argument("--no-filter", action="store_true",
                    help="skip the modal-filter measurement")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter reference)")
    args = ap.parse_args()
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
    results = {}
    for f in forms:
        pc = "fp32" if f == "fp32" else "fp64"
        results[f] = run_form(hp, torch, mesh, u0, dt, f, pc, args.steps,
                              args.warmup, args.newton_tol)
        r = results[f]
        print(f"# form {f}: wall {r['wall_s']:.3f} s, implicit ms/stage "
              f"{np.mean(r['impl_ms']):.3f}, newton {np.mean(r['newton']):.2f}, "
              f"gmres/stage {np.mean(r['gmres']):.1f}", file=sys.stderr, flush=True)
    dof = mesh.Nim * mesh.Np * 4
    main_form = "fp32" if "fp32" in results else forms[0]
    r = results[main_form]
    stage_s = np.mean(r["impl_ms"]) * 1e-3
    value = dof / stage_s
    line = {
        "metric": "Implicit-stage DOF/s, FP32-MFMA batched vs FP64 hybridized, at matched error",
        "value": value,
        "unit": "implicit-stage DOF/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["wall_s"] * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if main_form == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": describe(args.workload),
                   "n_elems": mesh.Ne, "n_implicit": mesh.Nim,
                   "implicit_dof": dof, "dt": dt,
                   "newton_tol": args.newton_tol,
                   "form": main_form},
        "roofline": roofline(main_form, mesh, r["timers"], main_form, args.workload,
                             r["phases"]),
    }
    for f, rr in results.items():
        line[f"{f}_form"] = {
            "implicit_dof_per_s": dof / (np.mean(rr["impl_ms"]) * 1e-3),
            "implicit_ms_per_stage": float(np.mean(rr["impl_ms"])),
            "newton_iters_per_stage": float(np.mean(rr["newton"])),
            "gmres_iters_per_stage": float(np.mean(rr["gmres"])),
            "phase_ms_instrumented_pass": {k: v[0] for k, v in rr["phases"].items()},
            "phase_launches_instrumented_pass": {k: v[1] for k, v in rr["phases"].items()},
            "workspace_bytes": rr["workspace"],
        }
    if "fp32" in results and "fp64" in results:
        a, b = results["fp32"]["state"], results["fp64"]["state"]
        a = a.reshape(4, -1)
        b = b.reshape(4, -1)
        line["fp32_vs_fp64_rel_err"] = float(
            (np.abs(a - b).max(axis=1) / np.abs(b).max(axis=1)).max())
        line["speedup_fp32_over_fp64"] = (
            np.mean(results["fp64"]["impl_ms"]) / np.mean(results["fp32"]["impl_ms"]))
    if not args.no_efr:
        # the same workload with the interior-embedded trace (EFR)
        mesh_e, u0e, dte, _ = build_case(hp, args.workload, efr=True)
        dof_e = mesh_e.Nim * mesh_e.Np * 4
        efr_states = {}
        for f in forms:
            pc = "fp32" if f == "fp32" else "fp64"
            rr = run_form(hp, torch, mesh_e, u0e, dte, f, pc, args.steps,
                          args.warmup, args.newton_tol)
            efr_states[f] = rr["state"]
            line[f"efr_{f}_form"] = {
                "implicit_dof_per_s": dof_e / (np.mean(rr["impl_ms"]) * 1e-3),
                "implicit_ms_per_stage": float(np.mean(rr["impl_ms"])),
                "newton_iters_per_stage": float(np.mean(rr["newton"])),
                "gmres_iters_per_stage": float(np.mean(rr["gmres"])),
                "trace_unknowns": 4 * mesh_e.Ntp,
                "phase_ms_instrumented_pass": {k: v[0] for k, v in rr["phases"].items()},
            }
            print(f"# efr form {f}: implicit ms/stage {np.mean(rr['impl_ms']):.3f}, "
                  f"gmres/stage {np.mean(rr['gmres']):.1f}", file=sys.stderr, flush=True)
        if "fp32" in efr_states and "fp64" in efr_states:
            a, b = efr_states["fp32"].reshape(4, -1), efr_states["fp64"].reshape(4, -1)
            line["efr_fp32_vs_fp64_rel_err"] = float(
                (np.abs(a - b).max(axis=1) / np.abs(b).max(axis=1)).max())
        line["hfr_trace_unknowns"] = 4 * mesh.Ntp
    if not args.no_edac:
        # the same O-grid and partition with the EDAC equations (theta = 100)
        mesh_d, u0d, dtd, _ = build_case(hp, args.workload, physics="edac")
        edac_states = {}
        for f in forms:
            pc = "fp32" if f == "fp32" else "fp64"
            rr = run_form(hp, torch, mesh_d, u0d, dtd, f, pc, args.steps,
                          args.warmup, args.newton_tol)
            edac_states[f] = rr["state"]
            line[f"edac_{f}_form"] = {
                "implicit_dof_per_s": mesh_d.Nim * mesh_d.Np * 4 / (np.mean(rr["impl_ms"]) * 1e-3),
                "implicit_ms_per_stage": float(np.mean(rr["impl_ms"])),
                "newton_iters_per_stage": float(np.mean(rr["newton"])),
                "gmres_iters_per_stage": float(np.mean(rr["gmres"])),
                "theta": THETA, "dt": dtd,
            }
            print(f"# edac form {f}: implicit ms/stage {np.mean(rr['impl_ms']):.3f}, "
                  f"gmres/stage {np.mean(rr['gmres']):.1f}", file=sys.stderr, flush=True)
        if "fp32" in edac_states and "fp64" in edac_states:
            a, b = edac_states["fp32"].reshape(4, -1), edac_states["fp64"].reshape(4, -1)
            line["edac_fp32_vs_fp64_rel_err"] = float(
                (np.abs(a - b).max(axis=1) / np.maximum(np.abs(b).max(axis=1), 1e-300)).max())
    if not args.no_filter:
        line["modal_filter"] = filter_rate(torch, mesh, u0)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
