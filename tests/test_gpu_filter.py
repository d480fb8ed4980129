"""GPU parity of the modal filter (Appendix B) against the oracle: every
order, parameter sets that damp, cut and leave modes alone, ragged tiles,
the full 128x64 p=3 cylinder on sampled elements, filtered IMEX steps, and
the parameter checks of the entry point."""
import numpy as np
import pytest
import torch

import fr_inputs as fi
import oracle
from oracle import imex as oimex, modal_filter as omf
from oracle.operators import RefOps
import paper_2401_16632_amd as hp
from tests.cases import c1_desc
from tests.gpu_util import Pair, dev, host, soa, unsoa

pytestmark = pytest.mark.gpu

PARAMS = [dict(alpha=100.0, s=1.0, eta_c=3.0, kappa=1.0),   # airfoil run
          dict(alpha=36.0, s=2.0, eta_c=2.0, kappa=0.5),
          dict(alpha=5.0, s=1.0, eta_c=0.0, kappa=1.0),
          dict(alpha=8.0, s=1.5, eta_c=1.5, kappa=2.0),
          dict(alpha=100.0, s=1.0, eta_c=11.0, kappa=1.0)]  # identity


def _oracle(om, u, prm):
    return omf.apply(om, u, prm["alpha"], prm["s"], prm["eta_c"], prm["kappa"])


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("k", range(len(PARAMS)))
def test_filter_matches_oracle(p, k):
    """4 Ne = 324 columns: several tiles with a ragged last one at every
    order; FP64 throughout, so the bar is a few rounding errors of the
    Np-term sums."""
    prm = PARAMS[k]
    d, mask = c1_desc(n=9, perturb=0.2, seed=7)
    pr = Pair(d, p, mask)
    u = fi.perturb_state(fi.isentropic_vortex(pr.om.x, pr.om.y), 0.05, 13 + p)
    ud = dev(soa(u))
    pr.hm.modal_filter(ud, **prm)
    torch.cuda.synchronize()
    got = unsoa(host(ud), pr.hm.Ne, pr.P)
    ref = _oracle(pr.om, u, prm)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    if k == len(PARAMS) - 1:
        assert np.abs(got - u).max() <= 1e-13 * np.abs(u).max()


def test_filter_full_cylinder_sampled():
    """The 128x64 p=3 cylinder of the benchmark: 128 sampled elements against
    the oracle's filter matrix, and every element's cell mean conserved up
    to rounding (the mean mode is never damped)."""
    import bench
    mesh, u0, dt, xy = bench.build_case(hp, "c2")
    P = mesh.P
    ops = RefOps(P - 1)
    prm = PARAMS[0]
    rng = np.random.default_rng(3)
    b = u0.reshape(4, mesh.Ne, P * P) * (1.0 + 0.05 * rng.standard_normal((4, mesh.Ne, P * P)))
    ud = dev(b)
    mesh.modal_filter(ud, **prm)
    torch.cuda.synchronize()
    a = host(ud).reshape(4, mesh.Ne, P * P)
    F = omf.filter_matrix(ops, prm["alpha"], prm["s"], prm["eta_c"], prm["kappa"])
    sample = rng.choice(mesh.Ne, 128, replace=False)
    ref = np.einsum("pq,veq->vep", F, b[:, sample, :])
    assert np.abs(a[:, sample, :] - ref).max() <= 1e-13 * np.abs(ref).max()
    W = np.outer(ops.w, ops.w).ravel()
    assert np.abs(a @ W - b @ W).max() <= 1e-13 * np.abs(b @ W).max()


def test_filtered_imex_steps():
    """Three HIMEX2C steps of the p=3 vortex case, each followed by the
    filter, against the oracle's step and filter."""
    d, mask = c1_desc(n=6, perturb=0.2, seed=4)
    pr = Pair(d, 3, mask)
    prm = dict(alpha=10.0, s=1.0, eta_c=2.0, kappa=1.0)
    u0 = fi.isentropic_vortex(pr.om.x, pr.om.y)
    s = hp.Solver(pr.hm, rtol=1e-12, newton_tol=1e-13, max_iters=3000)
    stp = hp.ImexStepper(pr.hm, s, "HIMEX2C")
    ud, uo = dev(soa(u0)), u0.copy()
    for _ in range(3):
        un, _ = stp.step(ud, 0.01, filter=prm)
        ud = un.clone()
        uo, _ = oimex.imex_step(pr.om, pr.ph, oimex.TABLEAUS["HIMEX2C"](), uo,
                                0.01, tol=1e-13)
        uo = _oracle(pr.om, uo, prm)
        ug = unsoa(host(ud), pr.hm.Ne, pr.P)
        assert np.abs(ug - uo).max() <= 1e-11 * np.abs(uo).max()


def test_filter_rejects_bad_parameters():
    d, mask = c1_desc(n=3)
    pr = Pair(d, 2, mask)
    u = torch.zeros(4 * pr.hm.Ne * pr.hm.Np, dtype=torch.float64, device="cuda")
    for bad in (dict(alpha=-1.0), dict(s=0.0), dict(kappa=-0.5),
                dict(alpha=float("nan"))):
        with pytest.raises(hp.HfrError):
            pr.hm.modal_filter(u, **bad)
