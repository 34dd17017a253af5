"""Whole-run pin: at large cross section the kinetic Riemann evolution
approaches the ideal-fluid (e = 3p) solution (the paper's Sec. 5 benchmark;
its Fig. 2 and Fig. 3 show the shock and the approach to an ideal fluid as
sigma grows).  Geometry of the 1-D tube (10 x 1 x 1 fm, T = 0.40 / 0.32 GeV)
with 4 x 4 transverse cells so that cells hold ~34 / ~17 test particles,
r_test = 400 (N = 40 834), observed at t = 4 fm/c."""
import numpy as np
import pytest

from paper_1208_0961_amd import hydro
from paper_1208_0961_amd import workload as W


def _evolve(orc, sigma, dt, tend=4.0, seed=1):
    w = W.Workload("riemann-hydro", (10.0, 1.0, 1.0), (100, 4, 4), 400.0, sigma, dt,
                   0.40, 0.32, seed=seed)
    st = orc.State(*W.riemann_state(w, seed=seed))
    p = orc.make_params(**w.params())
    orc.run(p, st, 0, int(round(tend / dt)), nthreads=8)
    return orc.observe(p, st)


@pytest.mark.slow
def test_riemann_approaches_ideal_hydro(orc):
    eL = 3 * W.gluon_density(0.40) * 0.40
    eR = 3 * W.gluon_density(0.32) * 0.32
    R = hydro.Riemann(eL, eR)
    tend = 4.0
    # 0.5 fm bins, each the mean of the exact profile over the bin
    sub = (np.arange(20)[:, None] + (np.arange(50)[None, :] + 0.5) / 50) * 0.5
    want = np.array([[R.profiles((x - 5.0) / tend)[0] for x in row] for row in sub]).mean(1)
    xs = (np.arange(100) + 0.5) * 0.1
    plateau = (xs > 3.6) & (xs < 7.0)         # between fan tail (3.26) and shock (7.58)
    l1 = {}
    for sigma, dt in ((0.4, 0.005), (1.6, 0.005), (4.0, 0.002)):
        T00, T0x = _evolve(orc, sigma, dt, tend)
        l1[sigma] = np.abs(T00.reshape(20, 5).mean(1) - want).mean()
        if sigma == 4.0:
            t00s, t0xs = R.profiles(0.0)      # plateau values 10.890, 2.741
            assert abs(T00[plateau].mean() / t00s - 1) < 0.03
            assert abs(T0x[plateau].mean() / t0xs - 1) < 0.03
    assert l1[0.4] > l1[1.6] > l1[4.0], l1
