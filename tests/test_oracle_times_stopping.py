"""Pins of the oracle's output times, PCG iterates, stopping rules and timed
stimuli against what the paper and the mathematics fix (CPU only).

* LAT / LRT ("Software functionality": activation when V first becomes
  positive; repolarisation when V returns below -70 mV while falling): a
  uniform stimulus over the whole mesh reduces every node to the single-cell
  operator split, so each node's times are the single cell's, at the step
  time t^{k+1} of the step that produced the crossing.
* Algorithm 1: the j-th Jacobi-PCG iterate minimises the A-norm error over
  x0 + span{(D^-1 A)^i z0, i < j} (a dense least-energy problem, solved here
  with numpy, not by a CG recurrence).
* Stopping (the two relative modes): the returned x is the first iterate
  x_j, j >= 1 (Algorithm 1 tests after each update), whose dense residual
  D^-1 (b - A x_j) passes the test against ||D^-1 b|| (relative to the
  right-hand side) or against ||z0|| (relative to the initial residual).
* Stimuli as (nodes, start, duration, intensity), overlapping ones adding
  ("Software functionality"): with no ionic current the summed theta-scheme
  rows give 1^T M (V^{k+1} - V^k) = (dt / Cm) 1^T M I_stim^k at every step.
"""
import numpy as np
import pytest

from oracle import orc
from paper_2510_12011_amd import inputs


def _single_cell_times(params, dt, ist, n_steps, cm):
    """Single-cell operator split V <- V + dt (I_stim/Cm - I_ion/Cm) and the
    step times of its first V > 0 and its first later V < -70 while falling,
    with the values on both sides of each crossing (for the margin)."""
    V, u = orc.ionic_init("ms", 1, params)
    lat = lrt = np.inf
    lat_pair = lrt_pair = None
    for k in range(n_steps):
        iion = orc.ionic_step("ms", V, u, dt, params)
        Vn = V + dt * (ist(k) / cm - iion)
        t1 = (k + 1) * dt
        if np.isinf(lat) and Vn[0] > 0.0:
            lat, lat_pair = t1, (V[0], Vn[0])
        elif np.isfinite(lat) and np.isinf(lrt) and Vn[0] < -70.0 and Vn[0] < V[0]:
            lrt, lrt_pair = t1, (V[0], Vn[0])
        V = Vn
    return lat, lrt, lat_pair, lrt_pair


def test_uniform_stimulus_activation_and_repolarisation_times():
    """Every node's LAT and LRT equal the single cell's crossing step times
    exactly (no interpolation; t^{k+1} of the step whose new V crosses).
    A t^k / t^{k+1} slip, another activation threshold or another
    repolarisation level all change these times.  (At the first step after
    activation with V < -70 mV, V is necessarily falling -- the value before
    it was above -70 -- so the falling condition adds nothing to a single
    beat.)"""
    dt, n_steps = 0.05, 5000                      # 250 ms: past repolarisation
    params = np.array(inputs.ATRIUM_MS_PARAMS)
    sp = inputs.small_box(nx=4, ny=3, nz=3, ionic="ms", n_steps=n_steps, dt=dt)
    sp.ionic_params = inputs.ATRIUM_MS_PARAMS
    sp.stimuli = [inputs.Stimulus(np.arange(sp.mesh.n_nodes, dtype=np.int32), 0.0, 1.0, 0.5)]
    sp.rtol = 1e-13
    o = orc.Oracle(sp)
    o.steps(n_steps)
    k_end = int(round(1.0 / dt))
    lat, lrt, lat_pair, lrt_pair = _single_cell_times(
        params, dt, lambda k: 0.5 if k < k_end else 0.0, n_steps, sp.cm)
    assert np.isfinite(lat) and np.isfinite(lrt) and lrt > lat + 50.0
    # the crossings are clear of the uniform-state rounding (<= 1e-9 mV)
    assert lat_pair[0] < -1e-6 and lat_pair[1] > 1e-6
    assert lrt_pair[0] > -70.0 + 1e-6 and lrt_pair[1] < -70.0 - 1e-6
    assert (o.state.lat == lat).all(), (np.unique(o.state.lat), lat)
    assert (o.state.lrt == lrt).all(), (np.unique(o.state.lrt), lrt)


def _small_system(seed=0):
    sp = inputs.small_box(nx=5, ny=4, nz=3, jitter=0.2, seed=seed)
    m = orc.assemble_spec(sp)
    A = sp.chi * sp.cm * m.M + sp.theta * sp.dt * m.K
    Ad = m.dense("M") * sp.chi * sp.cm + m.dense("K") * sp.theta * sp.dt
    return m, A, Ad


def test_pcg_iterates_minimise_energy_over_krylov_space():
    """Iterate j of Jacobi-PCG (Algorithm 1) is x0 + V y with V a basis of the
    preconditioned Krylov space K_j(D^-1 A, z0) and y solving the Galerkin
    system V^T A V y = V^T r0: the unique minimiser of ||x - x*||_A there.
    Pins alpha, beta, the preconditioner and the update order, independently
    of any CG recurrence."""
    m, A, Ad = _small_system()
    rng = np.random.default_rng(1)
    n = m.n
    b = Ad @ rng.normal(size=n)
    x0 = rng.normal(size=n)
    dinv = 1.0 / np.diag(Ad)
    r0 = b - Ad @ x0
    xs = np.linalg.solve(Ad, b)
    basis = [dinv * r0]
    for j in range(1, 7):
        Q, _ = np.linalg.qr(np.stack(basis, axis=1))
        y = np.linalg.solve(Q.T @ Ad @ Q, Q.T @ r0)
        x_ref = x0 + Q @ y
        x_j, it, _ = orc.pcg(m, A, b, x0, atol=0.0, rtol=1e-30, rel_mode=1, max_iter=j)
        assert it == -1                                  # stopped by the cap at j
        err = np.linalg.norm(x_j - x_ref) / np.linalg.norm(x_ref)
        assert err <= 1e-10, (j, err)
        # A-optimality: no other point of the space is closer in the A-norm
        e_j = (x_j - xs) @ Ad @ (x_j - xs)
        for _ in range(3):
            xp = x_j + Q @ rng.normal(scale=1e-3, size=Q.shape[1])
            assert (xp - xs) @ Ad @ (xp - xs) > e_j
        basis.append(dinv * (Ad @ basis[-1]))


@pytest.mark.parametrize("rel_mode", [0, 1])
def test_stopping_rule_returns_first_passing_iterate(rel_mode):
    """With rel_mode 1 the solve stops at the first iterate x_j (j >= 1) whose
    dense ||D^-1 (b - A x_j)|| <= rtol ||D^-1 b||; with rel_mode 0 against
    ||z0||.
    The start is close to the solution, so ||z0|| << ||D^-1 b|| and the two
    modes stop at different iterates; rtol sits halfway (geometrically)
    between two consecutive iterates' residuals, so the crossing is clear."""
    m, A, Ad = _small_system(seed=2)
    rng = np.random.default_rng(3)
    n = m.n
    xs = rng.normal(size=n)
    b = Ad @ xs
    x0 = xs + 1e-3 * rng.normal(size=n)
    dinv = 1.0 / np.diag(Ad)
    zn = []
    iterates = [x0]
    for j in range(1, 16):
        x_j, it, _ = orc.pcg(m, A, b, x0, atol=0.0, rtol=1e-30, rel_mode=1, max_iter=j)
        iterates.append(x_j)
    for x in iterates:
        zn.append(np.linalg.norm(dinv * (b - Ad @ x)))
    zn = np.array(zn)
    ref = np.linalg.norm(dinv * b) if rel_mode == 1 else zn[0]
    target = 5 if rel_mode == 0 else 2
    assert zn[target] < zn[target - 1]
    rtol = np.sqrt(zn[target] * zn[target - 1]) / ref
    expect = 1 + int(np.argmax(zn[1:] <= rtol * ref))
    assert (zn[1:expect] > rtol * ref * (1 + 1e-6)).all() and zn[expect] < rtol * ref * (1 - 1e-6)
    x, it, znorm = orc.pcg(m, A, b, x0, atol=0.0, rtol=rtol, rel_mode=rel_mode, max_iter=1000)
    assert it == expect, (it, expect, zn[:expect + 2] / ref, rtol)
    np.testing.assert_array_equal(x, iterates[expect])
    assert znorm == pytest.approx(zn[expect], rel=1e-8)


def test_stopping_modes_differ_after_good_start():
    """A start near the solution: relative to ||z0|| asks for the same
    reduction again (several iterations), relative to ||D^-1 b|| is met after
    the first update (the test follows the update, as in Algorithm 1; only
    the absolute and rounding-floor tests can accept x0 untouched)."""
    m, A, Ad = _small_system(seed=4)
    rng = np.random.default_rng(5)
    xs = rng.normal(size=m.n)
    b = Ad @ xs
    x0 = xs + 1e-9 * rng.normal(size=m.n)
    _, it_init, _ = orc.pcg(m, A, b, x0, rtol=1e-6, rel_mode=0)
    _, it_rhs, _ = orc.pcg(m, A, b, x0, rtol=1e-6, rel_mode=1)
    assert it_rhs == 1 and it_init >= 3
    _, it_floor, _ = orc.pcg(m, A, b, xs, rtol=1e-6, rel_mode=1)
    assert it_floor == 0                         # at the rounding floor


def test_two_overlapping_stimuli_charge_balance_per_step():
    """Two stimuli with overlapping node sets, the second starting at 0.5 ms:
    with no ionic current each step's charge change 1^T M (V^{k+1} - V^k)
    equals (dt / Cm) 1^T M I_stim^k with I_stim^k the sum of the stimuli
    active at step k (round(start/dt) <= k < round((start + duration)/dt)).
    A start that is ignored, an inclusive end, or stimuli that replace
    instead of adding each break it at some step."""
    sp = inputs.small_box(nx=6, ny=5, nz=4, ionic="ms", n_steps=200)
    sp.ionic = "none"
    sp.rtol = 1e-14
    s1 = inputs.box_corner_nodes(sp.mesh, 0.6)
    s2 = inputs.box_corner_nodes(sp.mesh, 0.4, 1.0, 0.8)
    assert np.intersect1d(s1, s2).size > 0 and np.setdiff1d(s2, s1).size > 0
    sp.stimuli = [inputs.Stimulus(s1, 0.0, 1.0, 0.5), inputs.Stimulus(s2, 0.5, 1.0, 0.3)]
    o = orc.Oracle(sp)
    m = o.mats
    ones = np.ones(m.n)
    seen = set()
    for k in range(200):
        ist = np.zeros(m.n)
        if k < 100:
            ist[s1] += 0.5
        if 50 <= k < 150:
            ist[s2] += 0.3
        rhs = sp.dt / sp.cm * (ones @ orc.spmv(m, m.M, ist))
        V0 = o.state.V.copy()
        o.steps(1)
        lhs = ones @ orc.spmv(m, m.M, o.state.V - V0)
        assert lhs == pytest.approx(rhs, rel=1e-10, abs=1e-12), k
        seen.add(round(rhs, 12))
    assert len(seen) == 4          # both alone, both together, neither
