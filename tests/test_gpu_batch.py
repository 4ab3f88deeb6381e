"""Batched form: several unstructured ellipsoidal shells (each with its own
conductivity scale and stimulus site) advanced as one block-diagonal system
with per-instance CG scalars.

* every instance against the FP64 oracle run on its own (bar of the
  mixed-precision form: V relative L2 <= 1e-5 at every snapshot, activation
  times within one time step);
* the batch against each instance run alone through the same solver
  (bitwise identical: instances share no arithmetic);
* graph-replayed steps against kernel-by-kernel steps (bitwise, every
  snapshot, with eager work between the replays);
* the autotuner's choices and forced lanes-per-row layouts against the
  default (FP32 summation order only);
* the persistent iteration (one launch runs every instance's iterations,
  instance-local barriers) against the oracle and the default path, also
  replayed as graphs.
"""
import numpy as np
import pytest

from oracle import orc
from paper_2510_12011_amd import inputs

pytestmark = pytest.mark.gpu

V_REL_L2 = 1e-5
STEPS, EVERY = 400, 100


@pytest.fixture(scope="module")
def bspec():
    # small shells (semi-axes 4-6 mm, wall 1-1.5 mm: spacing ~0.3 mm)
    b = inputs.batch_shells(n_inst=5, total_nodes=25_000, n_min=2_500, n_max=9_000, seed=7,
                            n_steps=STEPS, axes_mm=(4.0, 6.0), wall_mm=(1.0, 1.5))
    print(f"[batch] {b.name}: sizes {[i.mesh.n_nodes for i in b.instances]}", flush=True)
    return b


def _rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _split(v, ptr):
    return [v[..., ptr[k]:ptr[k + 1]] for k in range(len(ptr) - 1)]


@pytest.fixture(scope="module")
def batch_run(bspec):
    from paper_2510_12011_amd import sim
    print("[case] batched run, kernel by kernel", flush=True)
    s = sim.batch_from_spec(bspec)
    v, st = s.run(STEPS, EVERY)
    lat, _ = s.times()
    its = s.instance_iterations(STEPS)
    return dict(v=v, status=st, lat=lat, its=its, stats=s.stats())


def test_instances_match_oracle(bspec, batch_run):
    assert batch_run["status"] == 0
    ptr = bspec.node_ptr()
    vs = _split(batch_run["v"], ptr)
    lats = _split(batch_run["lat"], ptr)
    for k in range(len(bspec.instances)):
        spec = bspec.instance_spec(k)
        print(f"[case] oracle instance {k} n={spec.mesh.n_nodes}", flush=True)
        o = orc.Oracle(spec)
        v_or, _ = o.steps(STEPS, out_every=EVERY)
        errs = [_rel_l2(a, b) for a, b in zip(vs[k], v_or)]
        print(f"  instance {k}: V rel L2 max {max(errs):.2e}", flush=True)
        assert max(errs) <= V_REL_L2, errs
        fa, fb = np.isfinite(lats[k]), np.isfinite(o.state.lat)
        assert (fa != fb).sum() <= max(2, 1e-4 * fa.size)
        both = fa & fb
        assert both.sum() > 0
        assert abs(lats[k][both] - o.state.lat[both]).max() <= spec.dt * (1 + 1e-9)


def test_per_instance_iterations(bspec, batch_run):
    its = batch_run["its"]
    assert its.shape == (STEPS, len(bspec.instances))
    assert (its >= 0).all()
    # instances differ in size and conductivity: their counts are not all equal
    assert len(np.unique(its.mean(axis=0))) > 1
    print(f"  mean iterations per instance {np.round(its.mean(axis=0), 2)}", flush=True)


def test_batch_equals_individual_runs(bspec, batch_run):
    from paper_2510_12011_amd import sim
    ptr = bspec.node_ptr()
    vs = _split(batch_run["v"], ptr)
    for k in range(len(bspec.instances)):
        print(f"[case] instance {k} alone", flush=True)
        s = sim.batch_of_one(bspec.instance_spec(k))
        v, st = s.run(STEPS, EVERY)
        assert st == 0
        assert np.array_equal(v, vs[k]), np.abs(v - vs[k]).max()
        assert np.array_equal(s.instance_iterations(STEPS)[:, 0], batch_run["its"][:, k])


def test_graph_replay_matches_eager(bspec, batch_run):
    from paper_2510_12011_amd import sim
    print("[case] batched run, graph replay", flush=True)
    s = sim.batch_from_spec(bspec)
    s.set_tuning(graph=True)
    snaps = []
    for _ in range(STEPS // EVERY):
        v, st = s.run(EVERY, EVERY)   # replays separated by host copies
        assert st == 0
        snaps.append(v[0])
    for a, b in zip(snaps, batch_run["v"]):
        assert np.array_equal(a, b), np.abs(a - b).max()


@pytest.mark.parametrize("fmt,lpr", [("sell", 2), ("sell", 4), ("sell4", 1), ("csr", 4),
                                     ("csr", 8), ("csr", 16)])
def test_lanes_per_row_layouts(bspec, batch_run, fmt, lpr):
    from paper_2510_12011_amd import sim
    print(f"[case] {fmt}, lanes per row {lpr}", flush=True)
    s = sim.batch_from_spec(bspec)
    s.set_tuning(fmt=fmt)
    s.set_tuning(lanes_per_row=lpr, tiles_per_group=2)
    v, st = s.run(STEPS, EVERY)
    assert st == 0
    errs = [_rel_l2(a, b) for a, b in zip(v, batch_run["v"])]
    print(f"  lanes per row {lpr}: V rel L2 vs default {max(errs):.2e}", flush=True)
    assert max(errs) <= V_REL_L2


def test_autotune_installs_fastest(bspec, batch_run):
    from paper_2510_12011_amd import sim
    print("[case] autotune", flush=True)
    s = sim.batch_from_spec(bspec)
    rep = s.autotune(reps=10)
    cands = rep["candidates"]
    assert len(cands) >= 18
    assert rep["seconds"] == min(c[3] for c in cands)
    assert (rep["fmt"], rep["lanes_per_row"], rep["tiles_per_group"]) in [c[:3] for c in cands]
    print(f"  chose {rep['fmt']}, lanes/row {rep['lanes_per_row']}, tiles/group "
          f"{rep['tiles_per_group']}: {rep['seconds'] * 1e6:.1f} us", flush=True)
    v, st = s.run(STEPS, EVERY)
    assert st == 0
    errs = [_rel_l2(a, b) for a, b in zip(v, batch_run["v"])]
    assert max(errs) <= V_REL_L2


def test_batch_converges_relative_to_initial_residual(bspec):
    """Per-instance stopping relative to ||z0|| at 1e-10 (see the mixed-form
    test of the same name): every instance converges every step and matches
    its oracle run."""
    from paper_2510_12011_amd import sim
    import copy
    b = copy.copy(bspec)
    b.instances = bspec.instances[:2]
    b.rel_mode, b.rtol = 0, 1e-10
    print("[case] batch of 2, rtol 1e-10 of ||z0||", flush=True)
    s = sim.batch_from_spec(b)
    v, st = s.run(200, 100)
    its = s.instance_iterations(200)
    assert st == 0 and (its >= 0).all() and its.max() < 100
    ptr = b.node_ptr()
    for k in range(2):
        o = orc.Oracle(b.instance_spec(k))
        v_or, _ = o.steps(200, out_every=100)
        errs = [_rel_l2(a, c) for a, c in zip(_split(v, ptr)[k], v_or)]
        assert max(errs) <= V_REL_L2, errs


@pytest.mark.parametrize("graph", [False, True])
def test_persistent_iteration(bspec, batch_run, graph):
    """The persistent launch against the oracle (the mixed-precision bar) and
    against the five-launch iteration (same scalars and stopping decisions,
    so the same iteration counts; V within FP32 summation-order effects)."""
    from paper_2510_12011_amd import sim
    print(f"[case] batched run, persistent iteration, graph={graph}", flush=True)
    s = sim.batch_from_spec(bspec)
    s.set_tuning(persistent=True, graph=graph)
    v, st = s.run(STEPS, EVERY)
    assert st == 0
    lat, _ = s.times()
    its = s.instance_iterations(STEPS)
    ptr = bspec.node_ptr()
    vs, lats = _split(v, ptr), _split(lat, ptr)
    ref = _split(batch_run["v"], ptr)
    diff = max(_rel_l2(a, b) for k in range(len(ptr) - 1) for a, b in zip(vs[k], ref[k]))
    print(f"  persistent vs five-launch: V rel L2 max {diff:.2e}, iteration counts equal on "
          f"{(its == batch_run['its']).mean():.3f} of the solves", flush=True)
    assert diff <= 1e-9
    assert abs(its.astype(int) - batch_run["its"]).max() <= 1
    for k in (0, len(bspec.instances) - 1):
        spec = bspec.instance_spec(k)
        o = orc.Oracle(spec)
        v_or, _ = o.steps(STEPS, out_every=EVERY)
        assert max(_rel_l2(a, b) for a, b in zip(vs[k], v_or)) <= V_REL_L2
        fin = np.isfinite(o.state.lat) & np.isfinite(lats[k])
        assert abs(lats[k][fin] - o.state.lat[fin]).max() <= spec.dt * (1 + 1e-9)
