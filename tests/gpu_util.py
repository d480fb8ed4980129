"""Helpers of the GPU parity tests: build the oracle and the HIP objects from
the same seeded inputs and move arrays between their layouts."""
import numpy as np
import torch

import oracle
import paper_2401_16632_amd as hp


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).cuda()


def host(t):
    return t.detach().cpu().numpy()


def soa(u):          # (E,P,P,4) -> flat [4][E][Np]
    return hp.soa_from_elements(u).ravel()


def unsoa(flat, E, P):
    return hp.elements_from_soa(np.asarray(flat).reshape(4, E, P * P), P)


class Pair:
    """Oracle mesh + HIP mesh of one description."""

    def __init__(self, desc, p, mask, uinf=(1.0, 1.0, 0.0, 40.0)):
        self.om = oracle.QuadMesh(desc, p, implicit_mask=mask, uinf=uinf)
        self.hm = hp.Mesh(desc, p, implicit_mask=mask, uinf=uinf)
        self.p, self.P = p, p + 1
        self.ph = oracle.Euler()


def rel_err(a, b):
    """max over variables of |a_v - b_v|_inf / |b_v|_inf."""
    a = np.asarray(a).reshape(-1, 4)
    b = np.asarray(b).reshape(-1, 4)
    num = np.abs(a - b).max(axis=0)
    den = np.maximum(np.abs(b).max(axis=0), 1e-300)
    return float((num / den).max())
