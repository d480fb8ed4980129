"""Additive IMEX Runge-Kutta pairs for the element-partitioned step.

The implicit part is the two-stage, second-order SDIRK tableau of Section
3.1 (gamma = 1 - sqrt(2)/2).  Its explicit partner (padded form of
table:butcherimex, c_bar = [0 c]) has rows (gamma, 0, 0) and
(delta, 1 - delta, 0) with delta = 1 - 1/(2 gamma); the default pair uses
b_bar = [0 b] so the interface fluxes cancel over a step, the ARS222 pair
uses b_bar = (delta, 1 - delta, 0).
"""
import math


def _sdirk2():
    g = 1.0 - math.sqrt(0.5)
    return g, [[g, 0.0], [1.0 - g, g]], [1.0 - g, g]


def pair(name):
    g, A, b = _sdirk2()
    d = 1.0 - 1.0 / (2.0 * g)
    Abar = [[0.0, 0.0, 0.0], [g, 0.0, 0.0], [d, 1.0 - d, 0.0]]
    if name == "HIMEX2C":
        bbar = [0.0, b[0], b[1]]
    elif name == "ARS222":
        bbar = [d, 1.0 - d, 0.0]
    else:
        raise ValueError(f"unknown tableau {name}")
    return dict(name=name, s=2, A=A, b=b, Abar=Abar, bbar=bbar)
