"""Newton solve of one implicit stage by static condensation.

Section 3.1 (stage system eq:9oind, eq:23nffsd), Section 3.2 (Newton block
system, condensed trace system L du_hat = t with L = D - C A^-1 B and
t = s - C A^-1 r, local back-substitution eq:localproblems, element-by-element
assembly eq:assembly / eq:assembly2, element blocks eq:elemA and
eq:elemsystemB).

Readings taken where the paper is silent or inconsistent:
  * h = u - u* - a_ii dt R(u, u_hat) with R = du/dt (the printed A and B
    blocks carry inconsistent signs); A, B, C, D are the exact derivatives of
    h and of the element shares g^(k) of the transmission residual, taken by
    the complex step (derivative of an analytic function to round-off).
  * r = -h, s = -g (so the Newton update is u += du, u_hat += du_hat).
  * The trace system is solved directly (the paper does not name its global
    solver); the converged stage is then the discrete solution to round-off.
  * Stop when max(|h|_inf, |g|_inf) <= tol * max(1, |u*|_inf).

Element-local vector order: u_k flattened from [j, i, v]; trace-side vector
from [face, q, v], restricted to the element's trace faces.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .residual import (hfr_local, assemble_trace, implicit_outer, trace_average,
                       hfr_residual)

CSTEP = 1e-30


class NewtonError(RuntimeError):
    pass


def element_blocks(mesh, phys, u_im, outer, aii_dt):
    """A_k = dh_k/du_k, B_k = dh_k/d(outer), C^k = dg^(k)/du_k,
    D^k = dg^(k)/d(outer) for every implicit element, full local size
    (n = P*P*nv columns of u, M = 4*P*nv columns of the outer states).
    Entries belonging to non-trace faces are removed by ``trace_index``."""
    E, P, _, nv = u_im.shape
    n = P * P * nv
    M = 4 * P * nv
    A = np.zeros((E, n, n))
    B = np.zeros((E, n, M))
    C = np.zeros((E, M, n))
    D = np.zeros((E, M, M))
    uc = u_im.astype(np.complex128)
    oc = outer.astype(np.complex128)
    for col in range(n):
        j, i, v = np.unravel_index(col, (P, P, nv))
        up = uc.copy()
        up[:, j, i, v] += 1j * CSTEP
        R, gk = hfr_local(mesh, phys, up, oc)
        A[:, :, col] = -aii_dt * (R.imag / CSTEP).reshape(E, n)
        A[:, col, col] += 1.0
        C[:, :, col] = (gk.imag / CSTEP).reshape(E, M)
    for col in range(M):
        f, q, v = np.unravel_index(col, (4, P, nv))
        op = oc.copy()
        op[:, f, q, v] += 1j * CSTEP
        R, gk = hfr_local(mesh, phys, uc, op)
        B[:, :, col] = -aii_dt * (R.imag / CSTEP).reshape(E, n)
        D[:, :, col] = (gk.imag / CSTEP).reshape(E, M)
    return A, B, C, D


def trace_index(mesh, k, nv):
    """(local columns, global trace unknowns) of implicit element k."""
    tm = mesh.trace_map[k]                     # (4, P)
    loc, glob = [], []
    for f in range(4):
        for q in range(mesh.P):
            if tm[f, q] >= 0:
                for v in range(nv):
                    loc.append((f * mesh.P + q) * nv + v)
                    glob.append(tm[f, q] * nv + v)
    return np.array(loc, np.int64), np.array(glob, np.int64)


def condense(mesh, phys, u_all, uhat, ustar_im, aii_dt):
    """Residuals, element blocks and the assembled condensed system.

    Returns a dict with h (Nim, n), g (Ntp*nv,), the per-element factors
    needed for recovery (X_B = A^-1 B, X_r = A^-1 r), L (sparse CSR) and t."""
    nv = phys.nv
    im = mesh.imp_elems
    u_im = u_all[im]
    E, P = len(im), mesh.P
    n = P * P * nv
    outer = implicit_outer(mesh, u_all, uhat)
    R, gk = hfr_local(mesh, phys, u_im, outer)
    h = (u_im - ustar_im - aii_dt * R).reshape(E, n)
    g = assemble_trace(mesh, gk).reshape(-1)
    A, B, C, D = element_blocks(mesh, phys, u_im, outer, aii_dt)
    r = -h
    sk = -gk.reshape(E, -1)
    Nt = mesh.Ntp * nv
    rows, cols, vals = [], [], []
    t = np.zeros(Nt)
    XB, Xr, idx = [], [], []
    for k in range(E):
        loc, glob = trace_index(mesh, k, nv)
        Bk = B[k][:, loc]
        Ck = C[k][loc, :]
        Dk = D[k][np.ix_(loc, loc)]
        xb = np.linalg.solve(A[k], Bk)
        xr = np.linalg.solve(A[k], r[k])
        Lk = Dk - Ck @ xb
        tk = sk[k][loc] - Ck @ xr
        rr, cc = np.meshgrid(glob, glob, indexing="ij")
        rows.append(rr.ravel())
        cols.append(cc.ravel())
        vals.append(Lk.ravel())
        np.add.at(t, glob, tk)
        XB.append(xb)
        Xr.append(xr)
        idx.append(glob)
    if Nt:
        L = sp.coo_matrix((np.concatenate(vals),
                           (np.concatenate(rows), np.concatenate(cols))),
                          shape=(Nt, Nt)).tocsr()
    else:
        L = sp.csr_matrix((0, 0))
    return dict(h=h, g=g, A=A, B=B, C=C, D=D, XB=XB, Xr=Xr, idx=idx, L=L,
                t=t, R=R)


def trace_solve(L, t):
    """Direct solve of the condensed trace system L du_hat = t."""
    if L.shape[0] == 0:
        return np.zeros(0)
    return spla.spsolve(L.tocsc(), t)


def recover(sysd, duhat):
    """Local back-substitution (eq:localproblems):
    du_k = A_k^-1 (r_k - B_k du_hat_k) = X_r - X_B du_hat_k."""
    return np.stack([xr - xb @ duhat[gi] for xr, xb, gi in
                     zip(sysd["Xr"], sysd["XB"], sysd["idx"])])


def solve_stage(mesh, phys, u_all, ustar_im, aii_dt, uhat0=None, tol=1e-13,
                maxit=25, history=None, damping=False):
    """Newton iteration for (u_im, u_hat) of one implicit stage.

    u_all: full state whose explicit part is the explicit stage value (used
    at Upsilon faces) and whose implicit part is the initial guess.  The
    initial trace is the average of the two sides' interpolated states.
    With ``damping`` an update after which the stage residual is not
    finite is halved, up to seven times (a globalisation of Newton: it
    changes the path, not the root).  Returns (u_im, uhat, iterations)."""
    nv = phys.nv
    u_all = u_all.copy()
    im = mesh.imp_elems
    P = mesh.P
    uhat = trace_average(mesh, u_all) if uhat0 is None else uhat0.copy()
    scale = max(1.0, float(np.max(np.abs(ustar_im))) if ustar_im.size else 1.0)
    for it in range(maxit + 1):
        sysd = condense(mesh, phys, u_all, uhat, ustar_im, aii_dt)
        res = max(np.max(np.abs(sysd["h"]), initial=0.0),
                  np.max(np.abs(sysd["g"]), initial=0.0))
        if history is not None:
            history.append(res)
        if not np.isfinite(res):
            raise NewtonError("non-finite residual")
        if res <= tol * scale:
            return u_all[im], uhat, it
        if it == maxit:
            break
        duhat = trace_solve(sysd["L"], sysd["t"])
        du = recover(sysd, duhat).reshape(len(im), P, P, nv)
        duhat = duhat.reshape(-1, nv)
        base_u, base_h = u_all[im].copy(), uhat
        th = 1.0
        for _ in range(8 if damping else 1):
            u_all[im] = base_u + th * du
            uhat = base_h + th * duhat
            if not damping:
                break
            with np.errstate(invalid="ignore", divide="ignore"):
                R, g = hfr_residual(mesh, phys, u_all, uhat)
            if np.all(np.isfinite(R)) and np.all(np.isfinite(g)):
                break
            th *= 0.5
    raise NewtonError(f"Newton did not converge (residual {res:.3e})")


def dense_full_system(mesh, phys, u_all, uhat, ustar_im, aii_dt):
    """Brute-force check object: the unhybridized dense Newton system
    [A B; C D] [du; du_hat] = [r; s] assembled over all implicit elements and
    all trace unknowns (small meshes only)."""
    nv = phys.nv
    sysd = condense(mesh, phys, u_all, uhat, ustar_im, aii_dt)
    E = len(mesh.imp_elems)
    n = mesh.P * mesh.P * nv
    Nt = mesh.Ntp * nv
    K = np.zeros((E * n + Nt, E * n + Nt))
    rhs = np.zeros(E * n + Nt)
    for k in range(E):
        loc, glob = trace_index(mesh, k, nv)
        K[k * n:(k + 1) * n, k * n:(k + 1) * n] = sysd["A"][k]
        K[k * n:(k + 1) * n, E * n + glob] += sysd["B"][k][:, loc]
        K[E * n + glob, k * n:(k + 1) * n] += sysd["C"][k][loc, :]
        K[np.ix_(E * n + glob, E * n + glob)] += sysd["D"][k][np.ix_(loc, loc)]
        rhs[k * n:(k + 1) * n] = -sysd["h"][k]
    rhs[E * n:] = -sysd["g"]
    return K, rhs, sysd
