"""Several independent meshes in one (fr_mesh_desc.elem_instance), each
with its own time step (fr_mesh_set_instance_dt): every kernel runs once
per stage over all instances, and each instance's IMEX steps match the
oracle run on that instance alone with its own time step."""
import numpy as np
import pytest

import fr_inputs as fi
import oracle
from oracle import imex as oimex
import paper_2401_16632_amd as hp
from tests.gpu_util import dev, host, soa, unsoa, rel_err

pytestmark = pytest.mark.gpu

UINF = tuple(fi.freestream_state(0.2))
SPECS = [  # n_theta, n_r, first cell, ratio, implicit rings
    (16, 6, 2e-3, 1.25, 2),
    (24, 8, 1e-3, 1.20, 3),
    (12, 5, 3e-3, 1.15, 2),
]


def _instances(p):
    descs, masks, dts = [], [], []
    for nt, nr, first, ratio, rings in SPECS:
        d = fi.cylinder_ogrid(nt, nr, first=first, ratio=ratio)
        ring = np.arange(nt * nr) // nt
        om = oracle.QuadMesh(d, p, uinf=UINF)
        es = om.Es.reshape(nr, nt)
        cut = 0.5 * (es[rings - 1].max() + es[rings].min())
        descs.append(d)
        masks.append(ring < rings)
        dts.append(2.0 * cut / (6.0 * (2 * p + 1)))   # local CFL rule
    return descs, masks, dts


@pytest.mark.parametrize("p,precision", [(2, "fp64"), (3, "fp64"), (3, "fp32")])
def test_instances_match_separate_oracle_runs(p, precision):
    descs, masks, dts = _instances(p)
    batch = fi.concat_meshes(descs)
    mask = np.concatenate(masks)
    hm = hp.Mesh(batch, p, implicit_mask=mask, uinf=UINF)
    assert hm.info["n_instances"] == len(descs)
    hm.set_instance_dt(dts)
    P = p + 1
    us, oms = [], []
    for i, (d, mk) in enumerate(zip(descs, masks)):
        om = oracle.QuadMesh(d, p, implicit_mask=mk, uinf=UINF)
        u = np.broadcast_to(np.asarray(UINF), (om.Ne, P, P, 4)).copy()
        us.append(fi.perturb_state(u, 1e-3, 10 + i))
        oms.append(om)
    s = hp.Solver(hm, precision=precision, precond=precision, rtol=1e-10,
                  newton_tol=1e-13, max_iters=3000)
    stp = hp.ImexStepper(hm, s, "HIMEX2C")
    ud = dev(soa(np.concatenate(us)))
    ref = [u.copy() for u in us]
    tol = 1e-11 if precision == "fp64" else 1e-8
    print(f"batch: {len(descs)} cylinders p={p} {precision}", flush=True)
    for step in range(2):
        un, _ = stp.step(ud, 1.0)             # every instance by its own dt
        ud = un.clone()
        ug = unsoa(host(ud), hm.Ne, P)
        off = 0
        for i, om in enumerate(oms):
            ref[i], _ = oimex.imex_step(om, oracle.Euler(), oimex.himex2c(), ref[i], dts[i],
                                        tol=1e-13)
            err = rel_err(ug[off:off + om.Ne], ref[i])
            assert err <= tol, (step, i, err)
            off += om.Ne
