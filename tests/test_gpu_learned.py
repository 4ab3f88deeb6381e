"""Learned warm start: recorded features against the oracle, solutions
unchanged by the warm start (same tolerance), and the gain of a network
trained on the GPU over the previous-step warm start on held-out stimulus
sites (REL_RHS 1e-8 for every comparison: equal accuracy)."""
import numpy as np
import pytest

from oracle import orc
from paper_2510_12011_amd import inputs

pytestmark = pytest.mark.gpu


def _sim(spec, precision="fp64", prepare=True):
    from paper_2510_12011_amd import sim
    print(f"[case] {spec.name} n={spec.mesh.n_nodes} {precision}", flush=True)
    return sim.from_spec(spec, precision=precision, prepare=prepare)


def _rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_recorder_features_match_oracle():
    import torch
    from paper_2510_12011_amd import _lib as L, learn
    spec = inputs.small_box(nx=8, ny=6, nz=5, ionic="tt", n_steps=250, stim_extent=0.5)
    spec.rtol, spec.rel_mode = 1e-12, 1
    s = _sim(spec)
    s.run(250)
    n = spec.mesh.n_nodes
    X = torch.empty((n, 4), dtype=torch.float32, device="cuda:0")
    dV = torch.empty(n, dtype=torch.float32, device="cuda:0")
    s._check(L.lib().mdx_set_recorder(s._h, learn._p(X), learn._p(dV)))
    s.run(1)
    s._check(L.lib().mdx_set_recorder(s._h, None, None))
    order = np.zeros(n, np.int32)
    import ctypes as C
    s._check(L.lib().mdx_get_node_order(s._h, order.ctypes.data_as(C.c_void_p)))
    Xg = np.zeros((n, 4))
    Xg[order] = X.cpu().numpy()
    dVg = np.zeros(n)
    dVg[order] = dV.cpu().numpy()
    # oracle: same 250 steps, then the features of step 250 and its increment
    o = orc.Oracle(spec)
    o.steps(250)
    V, Vp, u = o.state.V.copy(), o.state.Vprev.copy(), o.state.u.copy()
    iion = orc.ionic_step("tt", V, u, spec.dt)           # u advanced on a copy
    kv = orc.spmv(o.mats, o.mats.K, Vp)                   # neighbour aggregate of V^{n-1}
    kd = o.mats.dense("K").diagonal()
    ref = np.stack([V, V - Vp, -iion, kv / kd], axis=1)    # the 2 ms stimulus ended at step 200
    o.steps(1)
    dref = o.state.V - V
    for c in range(4):
        scale = abs(ref[:, c]).max()
        np.testing.assert_allclose(Xg[:, c], ref[:, c], rtol=0, atol=1e-5 * scale + 1e-6)
    np.testing.assert_allclose(dVg, dref, rtol=0, atol=1e-5 * abs(dref).max())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_untrained_network_leaves_solution_unchanged(precision):
    """Any network only changes the starting point: with an untrained one
    (mostly falling back to V^k) the run still matches the oracle."""
    from paper_2510_12011_amd import learn, _lib as L
    spec = inputs.tiny_cube(n=12, n_steps=300)
    spec.rtol, spec.rel_mode = 1e-8, 1
    s = _sim(spec, precision)
    learn.install(s, learn.init_params(1), np.array([-60, 0, 0, 0, 30, 1, 10, 1, 0.5]))
    s.set_solver(spec.atol, spec.rtol, 1, spec.max_iter, L.MDX_WS_MLP,
                 1 if precision == "mixed" else 0, 50)
    v_gpu, st = s.run(300, 100)
    assert st == 0
    o = orc.Oracle(spec)
    v_or, _ = o.steps(300, out_every=100)
    err = max(_rel_l2(a, b) for a, b in zip(v_gpu, v_or))
    print(f"  untrained MLP warm start: V rel L2 {err:.2e}, fallbacks {s.stats()['fallbacks']}",
          flush=True)
    assert err <= 1e-5


def _shell_spec(mesh, site, n_steps):
    return inputs.shell_run(mesh=mesh, ionic="tt", dt=0.02, n_steps=n_steps, site_seed=site)


def test_trained_network_saves_iterations():
    """Train on 3 recorded trajectories of a ~100k-node shell (ten
    Tusscher-Panfilov, dt 0.02 ms, 40 ms each, random endocardial sites), then
    on a held-out site compare CG iterations per step with the previous-step
    warm start (the yardstick) and the extrapolation 2V^k - V^{k-1}."""
    from paper_2510_12011_amd import learn, _lib as L
    import torch
    mesh = inputs.ellipsoid_shell(n_nodes=100_000, seed=1000)
    steps = 2000
    Xs, Ds = [], []
    for site in (1, 2, 3):
        s = _sim(_shell_spec(mesh, site, steps))
        X, dV = learn.record(s, steps, every=10, seed=site)
        Xs.append(X)
        Ds.append(dV)
        trainer = s
    X, dV = torch.cat(Xs), torch.cat(Ds)
    print(f"  {X.shape[0]} samples", flush=True)
    params, norm, hist = learn.fit(trainer, X, dV, epochs=8, batch=4096, lr=2e-3,
                                   log=lambda m: print("  " + m, flush=True))
    assert hist[-1] < hist[0]
    res = {}
    for ws, name in ((L.MDX_WS_PREV, "prev"), (L.MDX_WS_EXTRAP, "extrap"), (L.MDX_WS_MLP, "mlp")):
        spec = _shell_spec(mesh, 101, steps)
        s = _sim(spec)
        if ws == L.MDX_WS_MLP:
            learn.install(s, params, norm)
        s.set_solver(0.0, 1e-8, 1, 1000, ws, 0, 50)
        el, it, fb = learn.timed_run(s, steps)
        res[name] = (float(it.mean()), el, fb)
        print(f"  {name}: mean iterations {it.mean():.2f}, {el:.3f} s, fallbacks {fb}", flush=True)
    assert res["mlp"][0] < res["prev"][0]
