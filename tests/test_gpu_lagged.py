"""Lagged Jacobian (factor reuse across Newton iterations and stages, the
paper's Jacobian update policy): the converged steps are unchanged, only the
Newton iteration count grows."""
import numpy as np
import pytest

import fr_inputs as fi
from oracle import imex as oimex
import paper_2401_16632_amd as hp
from tests.cases import c1_desc
from tests.gpu_util import Pair, dev, host, soa, unsoa, rel_err

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("lag,precision", [(1, "fp64"), (100, "fp64"), (100, "fp32")])
def test_lagged_jacobian_steps_match_oracle(lag, precision):
    d, mask = c1_desc()
    pr = Pair(d, 2, mask)
    om, hm = pr.om, pr.hm
    u0 = fi.isentropic_vortex(om.x, om.y)
    s = hp.Solver(hm, precision=precision, precond=precision, rtol=1e-12,
                  newton_tol=1e-13, newton_max_iters=80, max_iters=3000,
                  jacobian_lag=lag)
    stp = hp.ImexStepper(hm, s, "HIMEX2C")
    ud = dev(soa(u0))
    uo = u0.copy()
    iters = []
    for _ in range(4):
        un, stats = stp.step(ud, 0.01)
        ud = un.clone()
        uo, _ = oimex.imex_step(om, pr.ph, oimex.himex2c(), uo, 0.01, tol=1e-13)
        iters += [st["newton_iters"] for st in stats]
        err = rel_err(unsoa(host(ud), hm.Ne, pr.P), uo)
        assert err <= (1e-11 if precision == "fp64" else 1e-9), (err, iters)
