"""The N-version verification problem (the paper's verification section,
Table 2).  The published gold-standard activation times are not available,
so the checks are parity with the oracle on the coarsest grid and
self-convergence of the activation times along the P1-P8 diagonal under
refinement (0.5, 0.2, 0.1 mm at dt 0.005 ms)."""
import numpy as np
import pytest

from oracle import orc
from paper_2510_12011_amd import inputs, nversion as nv

pytestmark = pytest.mark.gpu


def _sim(spec):
    from paper_2510_12011_amd import sim
    print(f"[case] {spec.name} n={spec.mesh.n_nodes}", flush=True)
    return sim.from_spec(spec)


def test_nversion_coarse_matches_oracle():
    """dx = 0.5 mm, the first 30 ms: activation times equal the oracle's
    within one time step at every node activated by then (the same nodes)."""
    steps = 6000
    spec = inputs.nversion(0.5, steps)
    s = _sim(spec)
    s.run(steps)
    lat_g, _ = s.times()
    o = orc.Oracle(spec)
    o.steps(steps)
    lat_o = o.state.lat
    assert np.array_equal(np.isfinite(lat_g), np.isfinite(lat_o))
    fin = np.isfinite(lat_o)
    assert fin.sum() > 100
    assert abs(lat_g[fin] - lat_o[fin]).max() <= spec.dt * (1 + 1e-9)


def test_nversion_self_convergence():
    """Every grid activates the whole cuboid; the activation times along the
    diagonal move less from 0.2 to 0.1 mm than from 0.5 to 0.2 mm, and at P8
    they decrease monotonically with refinement (coarse P1 grids conduct
    slower)."""
    prof = {}
    for h in (0.5, 0.2, 0.1):
        spec = inputs.nversion(h, 60000)
        s = _sim(spec)
        t, steps, lat = nv.run_to_activation(s, spec)
        assert np.isfinite(lat).all(), h
        prof[h] = t
        print(f"  dx {h}: {steps} steps, activation P1 {t[0]:.3f} ms, P8 {t[-1]:.3f} ms", flush=True)
    d1 = np.abs(prof[0.5] - prof[0.2]).max()
    d2 = np.abs(prof[0.2] - prof[0.1]).max()
    print(f"  max diagonal difference 0.5-0.2: {d1:.3f} ms, 0.2-0.1: {d2:.3f} ms", flush=True)
    assert d2 < d1
    assert prof[0.5][-1] > prof[0.2][-1] > prof[0.1][-1]
