"""Python binding of the C ABI (marshalling and host-side shape checks)."""
import ctypes

import numpy as np
import torch

from . import _abi

_LIB = None


def load_library():
    """Load the built HIP library; raises if it is missing (no fallback)."""
    global _LIB
    if _LIB is None:
        _LIB = _abi.load()
    return _LIB


class HfrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_abi.STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(st):
    if st != _abi.FR_OK:
        raise HfrError(st, load_library().fr_last_error().decode())


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t, numel, name):
    """Device pointer of a contiguous float64 CUDA tensor of ``numel``."""
    if numel == 0:
        return None if t is None else ctypes.c_void_p(t.data_ptr())
    if t is None:
        raise ValueError(f"{name} is required")
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} entries, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _opt(t, numel, name):
    return None if t is None else _dev(t, numel, name)


def soa_from_elements(u):
    """(Ne, P, P, 4) element-major array -> (4, Ne, P*P) SoA layout."""
    Ne, P, _, nv = u.shape
    return np.ascontiguousarray(np.transpose(u, (3, 0, 1, 2)).reshape(nv, Ne, P * P))


def elements_from_soa(a, P):
    nv, Ne, _ = a.shape
    return np.ascontiguousarray(np.transpose(a.reshape(nv, Ne, P, P), (1, 2, 3, 0)))


TABLEAU_IDS = {"HIMEX2C": 0, "ARS222": 1}


def tableau(name="HIMEX2C"):
    """The library's additive pair of that name (imex_tableau_get)."""
    if name not in TABLEAU_IDS:
        raise ValueError(f"unknown tableau {name}")
    tab = _abi.ImexTableau()
    _check(load_library().imex_tableau_get(TABLEAU_IDS[name], ctypes.byref(tab)))
    return tab


class Mesh:
    """fr_mesh_create over a mesh description dict (see fr_inputs)."""

    def __init__(self, desc, order, implicit_mask=None, es_cutoff=-1.0,
                 gamma=1.4, uinf=(1.0, 0.0, 0.0, 1.0), host_only=False,
                 efr=False, physics="euler", theta=100.0):
        lib = load_library()
        self._keep = []

        def arr(x, dt):
            a = np.ascontiguousarray(np.asarray(x), dtype=dt)
            self._keep.append(a)
            return a
        xy = arr(desc["node_xy"], np.float64)
        en = arr(desc["elem_nodes"], np.int32)
        d = _abi.FrMeshDesc()
        d.n_nodes = xy.shape[0]
        d.node_xy = xy.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if desc.get("node_topo") is not None:
            tp = arr(desc["node_topo"], np.int32)
            d.node_topo = tp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.n_elems = en.shape[0]
        d.elem_nodes = en.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        if desc.get("elem_face_bc") is not None:
            bc = arr(desc["elem_face_bc"], np.int8)
            d.elem_face_bc = bc.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
        d.order = int(order)
        if implicit_mask is not None:
            mk = arr(implicit_mask, np.uint8)
            if mk.shape[0] != en.shape[0]:
                raise ValueError("implicit_mask length != number of elements")
            d.implicit_mask = mk.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        d.es_cutoff = float(es_cutoff)
        d.gamma = float(gamma)
        for v in range(4):
            d.uinf[v] = float(uinf[v])
        d.flags = (1 if host_only else 0) | (2 if efr else 0)
        kinds = {"euler": 0, "edac": 1}
        if physics not in kinds:
            raise ValueError(f"unknown physics {physics!r}")
        d.physics = kinds[physics]
        d.theta = float(theta)
        if desc.get("elem_instance") is not None:
            inst = arr(desc["elem_instance"], np.int32)
            d.elem_instance = inst.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            d.n_instances = int(desc["n_instances"])
        h = ctypes.c_void_p()
        _check(lib.fr_mesh_create(ctypes.byref(d), ctypes.byref(h)))
        self._keep = []
        self.handle = h
        info = _abi.FrMeshInfo()
        _check(lib.fr_mesh_get_info(h, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in info._fields_}
        self.P = order + 1
        self.Np = self.P * self.P
        self.Ne = self.info["n_elems"]
        self.Nim = self.info["n_implicit"]
        self.Nex = self.info["n_explicit"]
        self.Ntp = self.info["n_trace_points"]
        self.Ntf = self.info["n_trace_faces"]
        self.efr = bool(self.info["efr"])
        self._maps = None

    def set_instance_dt(self, dt):
        """Per-instance time steps (fr_mesh_set_instance_dt)."""
        a = np.ascontiguousarray(np.asarray(dt, np.float64))
        if a.shape != (self.info["n_instances"],):
            raise ValueError("one time step per instance")
        _check(load_library().fr_mesh_set_instance_dt(
            self.handle, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def maps(self):
        if self._maps is None:
            lib = load_library()
            Nf, P = self.info["n_faces"], self.P
            out = dict(face_elem=np.zeros((Nf, 2), np.int32),
                       face_local=np.zeros((Nf, 2), np.int32),
                       face_kind=np.zeros(Nf, np.int32),
                       trace_map=np.zeros((self.Nim, 4, P), np.int32),
                       implicit_elems=np.zeros(self.Nim, np.int32),
                       explicit_elems=np.zeros(self.Nex, np.int32),
                       es=np.zeros(self.Ne, np.float64),
                       sol_xy=np.zeros((self.Ne, self.Np, 2), np.float64))
            ptr = lambda a: ctypes.c_void_p(a.ctypes.data) if a.size else None
            _check(lib.fr_mesh_get_maps(self.handle, *[ptr(out[k]) for k in
                   ("face_elem", "face_local", "face_kind", "trace_map",
                    "implicit_elems", "explicit_elems", "es", "sol_xy")]))
            self._maps = out
        return self._maps

    def explicit_rhs(self, u, R_ex, stream=None):
        lib = load_library()
        _check(lib.fr_explicit_rhs(self.handle, _dev(u, 4 * self.Ne * self.Np, "u"),
                                   _dev(R_ex, 4 * self.Nex * self.Np, "R_ex"),
                                   _stream(stream)))

    def modal_filter(self, u, alpha=100.0, s=1.0, eta_c=3.0, kappa=1.0,
                     stream=None):
        """Filter the flat SoA float64 state u in place (Appendix B)."""
        lib = load_library()
        prm = _abi.FrFilterParams(float(alpha), float(s), float(eta_c),
                                  float(kappa))
        _check(lib.fr_modal_filter(self.handle, ctypes.byref(prm),
                                   _dev(u, 4 * self.Ne * self.Np, "u"),
                                   _stream(stream)))

    def close(self):
        if getattr(self, "handle", None):
            load_library().fr_mesh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_PREC = {"fp64": 0, "fp32": 1}
_PC = {"fp64": 0, "fp32": 1, "bf16": 2}


class Solver:
    """hfr_solver_create and the per-call entry points of the implicit stage."""

    def __init__(self, mesh, precision="fp64", precond="fp64", restart=30,
                 max_iters=600, rtol=1e-10, newton_max_iters=25,
                 newton_tol=1e-13, keep_blocks=False, jacobian_lag=0,
                 cgs_passes=1, workspace=None, condense="auto", damping=False,
                 graph=False, forcing=0.0):
        """workspace: None (the library allocates its working memory) or
        "torch" (a uint8 CUDA tensor allocated here and bound with
        hfr_solver_bind_workspace; kept as self.workspace).  forcing:
        hfr_opts.gmres_forcing_max (0: every solve inside Newton to rtol)."""
        lib = load_library()
        self.mesh = mesh
        o = _abi.HfrOpts()
        o.precision = _PREC[precision]
        o.precond = _PC[precond]
        o.gmres_restart = restart
        o.gmres_max_iters = max_iters
        o.gmres_rtol = rtol
        o.newton_max_iters = newton_max_iters
        o.newton_tol = newton_tol
        o.keep_blocks = 1 if keep_blocks else 0
        o.jacobian_lag = int(jacobian_lag)
        o.gmres_cgs_passes = int(cgs_passes)
        if workspace not in (None, "torch"):
            raise ValueError("workspace must be None or 'torch'")
        o.caller_workspace = 1 if workspace == "torch" else 0
        ck = {"auto": 0, "sweep": 1, "blocked": 2, "blocked_w8": 3}
        if condense not in ck:
            raise ValueError(f"condense must be one of {sorted(ck)}")
        o.condense_kernel = ck[condense]
        o.newton_damping = 1 if damping else 0
        o.iteration_graph = 1 if graph else 0
        o.gmres_forcing_max = float(forcing)
        self.opts = o
        self.workspace = None
        ws = ctypes.c_size_t()
        h = ctypes.c_void_p()
        _check(lib.hfr_solver_create(mesh.handle, ctypes.byref(o),
                                     ctypes.byref(ws), ctypes.byref(h)))
        self.handle = h
        self.workspace_bytes = ws.value
        if workspace == "torch":
            # torch's caching allocator hands out 512-byte aligned blocks
            self.workspace = torch.empty(max(256, ws.value), dtype=torch.uint8,
                                         device="cuda")
            _check(lib.hfr_solver_bind_workspace(
                h, ctypes.c_void_p(self.workspace.data_ptr()),
                ctypes.c_size_t(self.workspace.numel())))
        m = mesh
        self.n = 4 * m.Np
        self.m = 16 * m.P

    def _sizes(self):
        m = self.mesh
        return 4 * m.Ne * m.Np, 4 * m.Ntp, 4 * m.Nim * m.Np

    def residual(self, u, uhat, ustar, aii_dt, h=None, g=None, R_im=None,
                 stream=None):
        nu, nt, ni = self._sizes()
        _check(load_library().hfr_residual(
            self.handle, _dev(u, nu, "u"), _dev(uhat, nt, "uhat"),
            _dev(ustar, ni, "ustar"), float(aii_dt), _opt(h, ni, "h"),
            _opt(g, nt, "g"), _opt(R_im, ni, "R_im"), _stream(stream)))

    def assemble_condense(self, u, uhat, ustar, aii_dt, stream=None):
        nu, nt, ni = self._sizes()
        _check(load_library().hfr_assemble_condense(
            self.handle, _dev(u, nu, "u"), _dev(uhat, nt, "uhat"),
            _dev(ustar, ni, "ustar"), float(aii_dt), _stream(stream)))

    def trace_solve(self, duhat, stream=None, allow_unconverged=False):
        _, nt, _ = self._sizes()
        st = _abi.HfrSolveStats()
        rc = load_library().hfr_trace_solve(self.handle, _dev(duhat, nt, "duhat"),
                                            ctypes.byref(st), _stream(stream))
        if not (allow_unconverged and rc == -5):
            _check(rc)
        return dict(iterations=st.iterations, restarts=st.restarts,
                    rel_residual=st.rel_residual)

    def recover(self, duhat, du, stream=None):
        _, nt, ni = self._sizes()
        _check(load_library().hfr_recover(self.handle, _dev(duhat, nt, "duhat"),
                                          _dev(du, ni, "du"), _stream(stream)))

    def matvec(self, x, y, stream=None):
        _, nt, _ = self._sizes()
        _check(load_library().hfr_trace_matvec(self.handle, _dev(x, nt, "x"),
                                               _dev(y, nt, "y"), _stream(stream)))

    def product(self, x, y, stream=None):
        """y = L D^-1 x, the product the Krylov solver runs."""
        _, nt, _ = self._sizes()
        _check(load_library().hfr_trace_product(self.handle, _dev(x, nt, "x"),
                                                _dev(y, nt, "y"), _stream(stream)))

    def get_system(self, t=None, h=None, g=None, stream=None):
        _, nt, ni = self._sizes()
        _check(load_library().hfr_get_system(self.handle, _opt(t, nt, "t"),
                                             _opt(h, ni, "h"), _opt(g, nt, "g"),
                                             _stream(stream)))

    def get_blocks(self, out, stream=None):
        k = self.n + self.m
        _check(load_library().hfr_get_blocks(
            self.handle, _dev(out, self.mesh.Nim * k * k, "blocks"),
            _stream(stream)))

    def get_factors(self, stream=None):
        """Swept element tableaux (Nim, n+m, n+m) indexed [element, row,
        column] and the pivot rows (Nim, n) of the n exchanges."""
        m = self.mesh
        k = self.n + self.m
        dt = torch.float64 if self.opts.precision == 0 else torch.float32
        f = torch.zeros(m.Nim * k * k, dtype=dt, device="cuda")
        pv = torch.zeros(m.Nim * self.n, dtype=torch.int32, device="cuda")
        _check(load_library().hfr_get_factors(
            self.handle, ctypes.c_void_p(f.data_ptr()),
            ctypes.c_void_p(pv.data_ptr()), _stream(stream)))
        # stored column-major per element
        return f.view(m.Nim, k, k).transpose(1, 2), pv.view(m.Nim, self.n)

    def get_preconditioner(self, stream=None):
        """Block-Jacobi inverses (block rows, bs, bs) indexed [row block, row,
        column], as float64 (BF16 blocks are widened)."""
        m = self.mesh
        # block rows: trace faces of 4(p+1) unknowns (HFR) or trace nodes of
        # 4 unknowns (EFR)
        bs = 4 if m.efr else 4 * m.P
        ntf = m.Ntp if m.efr else m.Ntp // m.P
        pc = self.opts.precond
        dt = {0: torch.float64, 1: torch.float32, 2: torch.int16}[pc]
        d = torch.zeros(ntf * bs * bs, dtype=dt, device="cuda")
        _check(load_library().hfr_get_preconditioner(
            self.handle, ctypes.c_void_p(d.data_ptr()), _stream(stream)))
        if pc == 2:
            d = ((d.to(torch.int32) & 0xFFFF) << 16).view(torch.float32)
        return d.double().view(ntf, bs, bs).transpose(1, 2)

    def timing(self, enable=None, only=None):
        """Start (True) / stop (False) the kernel timers, or with ``only`` (a
        list of timer names) start those alone; returns the accumulated
        {name: (ms, launches)} after a device sync."""
        ms = (ctypes.c_double * len(_abi.TIMERS))()
        cnt = (ctypes.c_int64 * len(_abi.TIMERS))()
        if only is not None:
            en = _abi.TIMING_SELECT
            for name in only:
                en |= 1 << _abi.TIMERS.index(name)
        else:
            en = -1 if enable is None else (1 if enable else 0)
        _check(load_library().hfr_timing(self.handle, en, ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(_abi.TIMERS)}

    def condense_choice(self):
        """(kernel name, candidate ms) of the condensation kernel in use."""
        k = ctypes.c_int32()
        ms = (ctypes.c_double * 3)()
        _check(load_library().hfr_condense_choice(self.handle, ctypes.byref(k), ms))
        names = {0: "auto", 1: "sweep", 2: "blocked", 3: "blocked_w8"}
        return names[k.value], dict(zip(("sweep", "blocked", "blocked_w8"), list(ms)))

    def close(self):
        if getattr(self, "handle", None):
            load_library().hfr_solver_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ImexStepper:
    """Device buffers and the stage sequence of one IMEX step (imex_stage)."""

    def __init__(self, mesh, solver, name="HIMEX2C", device="cuda"):
        self.mesh, self.solver = mesh, solver
        self.tab = tableau(name)
        s = self.tab.s
        m = mesh
        f64 = dict(dtype=torch.float64, device=device)
        self.u = torch.zeros(4 * m.Ne * m.Np, **f64)
        self.uhat = torch.zeros(max(1, 4 * m.Ntp), **f64)
        self.R_im = torch.zeros(max(1, s * 4 * m.Nim * m.Np), **f64)
        self.R_ex = torch.zeros(max(1, (s + 1) * 4 * m.Nex * m.Np), **f64)
        self.stats = []

    def step(self, u_n, dt, stream=None, filter=None):
        """Advance u_n (flat SoA float64 CUDA tensor) by dt; returns the new
        state tensor (a view of an internal buffer) and per-stage stats.
        filter: None, or keyword arguments of Mesh.modal_filter applied to
        u_{n+1} after the last stage."""
        lib = load_library()
        m = self.mesh
        _dev(u_n, 4 * m.Ne * m.Np, "u_n")
        st = _abi.ImexState()
        st.u_n = u_n.data_ptr()
        st.u = self.u.data_ptr()
        st.uhat = self.uhat.data_ptr()
        st.R_im = self.R_im.data_ptr()
        st.R_ex = self.R_ex.data_ptr()
        stats = []
        solver = self.solver.handle if self.solver is not None else None
        for i in range(self.tab.s + 2):
            ns = _abi.HfrNewtonStats()
            _check(lib.imex_stage(m.handle, solver, ctypes.byref(self.tab), i,
                                  float(dt), ctypes.byref(st), ctypes.byref(ns),
                                  _stream(stream)))
            if 1 <= i <= self.tab.s:
                stats.append(dict(newton_iters=ns.newton_iters,
                                  gmres_iters=ns.gmres_iters,
                                  residual=ns.residual,
                                  implicit_ms=ns.implicit_ms,
                                  graph_replays=ns.graph_replays,
                                  queued_linearisations=ns.queued_linearisations))
        if filter is not None:
            m.modal_filter(self.u, stream=stream, **filter)
        self.stats = stats
        return self.u, stats
