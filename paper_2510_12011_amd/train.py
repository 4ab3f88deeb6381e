"""Training of the learned warm start's network for the ellipsoidal-shell
workload, on the GPU with the library's own kernels (a set-up step, run once
before benchmarks; its result is the weights file the benchmark loads).

    python -m paper_2510_12011_amd.train [--sites 20] [--steps 20000] [--out FILE]

Protocol: trajectories of the plain FP64 solver (extrapolated warm start,
REL_RHS 1e-8) on the ~1.2M-node shell (mesh seed 1000), ten
Tusscher-Panfilov cells, dt 0.02 ms, from rest with the stimulus at random
endocardial sites (seeds 1..sites), each `steps` long (20,000 = 400 ms: the
wave's spread, the plateau and repolarisation); every 10th step records the
nodes whose increment exceeds 0.02 mV and 5% of the others, at most `cap`
per recorded step; then Adam on the mean-squared error of the standardised
departure from the extrapolation (learn.fit).  Sites 101..105 are held out
for evaluation.
"""
from __future__ import annotations

import argparse
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "weights", "shell_tt_dt0.02.npz")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sites", type=int, default=20)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--cap", type=int, default=1500)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--out", default=DEFAULT_OUT)
    a = ap.parse_args()
    from . import inputs, learn, sim
    t0 = time.perf_counter()
    mesh = inputs.ellipsoid_shell(n_nodes=1_200_000, seed=1000)
    print(f"[train] shell {mesh.n_nodes} nodes, meshed in {time.perf_counter() - t0:.1f} s",
          flush=True)
    Xs, Ds = [], []
    trainer = None
    for site in range(1, a.sites + 1):
        t1 = time.perf_counter()
        spec = inputs.shell_run(mesh=mesh, ionic="tt", dt=0.02, n_steps=a.steps, site_seed=site)
        s = sim.from_spec(spec)
        X, dV = learn.record(s, a.steps, every=10, seed=site, cap=a.cap)
        Xs.append(X)
        Ds.append(dV)
        it = s.stats()["cg_iters_total"] / max(1, s.stats()["steps"])
        if trainer is not None:
            trainer.close()
        trainer = s
        print(f"[train] site {site}: {X.shape[0]} samples, {a.steps} steps "
              f"({it:.2f} CG iterations/step) in {time.perf_counter() - t1:.1f} s", flush=True)
    X, dV = learn.concat(Xs), learn.concat(Ds)
    del Xs, Ds
    t1 = time.perf_counter()
    params, norm, hist = learn.fit(trainer, X, dV, epochs=a.epochs, batch=8192, lr=2e-3,
                                   log=lambda m: print("[train] " + m, flush=True))
    print(f"[train] {X.shape[0]} samples, loss {hist[0]:.4f} -> {hist[-1]:.4f}, "
          f"fit in {time.perf_counter() - t1:.1f} s", flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    learn.save(a.out, params, norm, n_nodes=mesh.n_nodes, mesh_seed=1000, dt=0.02,
               sites=a.sites, steps=a.steps, samples=int(X.shape[0]), epochs=a.epochs,
               loss_first=hist[0], loss_last=hist[-1])
    print(f"[train] wrote {a.out} ({time.perf_counter() - t0:.0f} s in all)", flush=True)


if __name__ == "__main__":
    main()
