"""Pins of the ideal-fluid Riemann solution used as a test reference: the
shock satisfies both jump conditions, the fan matches the plateau at its
tail, and the similarity profile is continuous across the fan."""
import math

import numpy as np

from paper_1208_0961_amd import hydro
from paper_1208_0961_amd import workload as W


def test_jump_conditions_and_continuity():
    eL = 3 * W.gluon_density(0.40) * 0.40
    eR = 3 * W.gluon_density(0.32) * 0.32
    R = hydro.Riemann(eL, eR)
    r1, r2 = R.jump_residual()
    assert abs(r1) < 1e-13 and abs(r2) < 1e-13
    # fan tail meets the plateau, fan head meets the left state
    e_tail, v_tail = R.state(R.tail - 1e-12)
    assert abs(e_tail / R.es - 1) < 1e-9 and abs(v_tail - R.vs) < 1e-9
    e_head, v_head = R.state(R.head + 1e-12)
    assert abs(e_head / eL - 1) < 1e-9 and abs(v_head) < 1e-9
    # inside the fan the flow obeys the similarity relation xi = (v - cs)/(1 - v cs)
    for xi in np.linspace(R.head + 1e-3, R.tail - 1e-3, 7):
        e, v = R.state(xi)
        assert abs((v - hydro.CS) / (1 - v * hydro.CS) - xi) < 1e-12
    # the shock is supersonic relative to the state ahead, subsonic behind
    assert hydro.CS < R.shock < 1.0
    vrel = (R.shock - R.vs) / (1 - R.shock * R.vs)
    assert vrel < hydro.CS


def test_paper_cross_section_units():
    """sigma = 10 GeV^-2 (Sec. 5) is 0.3894 fm^2 with hbar c = 0.19733 GeV fm."""
    sigma_fm2 = 10.0 * W.HBARC ** 2
    assert abs(sigma_fm2 - 0.38938) < 1e-4
