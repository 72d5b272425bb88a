"""Checks of a Riemann-problem solution against the values the paper prints
(Section "Riemann Problem"; tests/golden/riemann_problem.txt), shared by the
oracle test and the GPU test."""

import numpy as np


def check_riemann(x, h, G):
    """Plateau mean over [-80, -20] (between the rarefaction tail, near
    (u* - c*) t = -123, and the dispersive shock) and the highest wave in x > 0."""
    hs_closed = (np.sqrt(G["h_L"]) + np.sqrt(G["h_R"])) ** 2 / 4.0
    d0 = abs(G["h_L"] - G["h_R"])
    am_closed = d0 - d0 * d0 / 12.0
    plateau = h[(x >= -80.0) & (x <= -20.0)].mean()
    hm = h[x > 0].max()
    # the printed values are the closed forms rounded
    assert abs(hs_closed - G["h_star"]) <= 0.005 and abs(am_closed - G["a_plus"]) <= 5e-4
    assert abs(1.0 + G["a_plus"] - G["h_max"]) <= 0.01
    assert abs(plateau - hs_closed) <= 0.005 * hs_closed, (plateau, hs_closed)
    assert abs(hm - (1.0 + am_closed)) <= 0.02 * (1.0 + am_closed), (hm, 1.0 + am_closed)
    return plateau, hm
