"""Writes the stored oracle results that the long-window GPU parity tests
compare against.  Calls only the CPU oracle (oracle/) on the seeded inputs
(paper_2510_12011_amd.inputs); nothing here touches the GPU path.

    python tests/golden/make_golden.py [slab_h0.1 | slab_h0.05_prefix |
                                        shell_prefix | cohort4] [--threads N]

Each file holds, for a seeded sample of nodes (ids in `nodes`, original
numbering): the activation times LAT (ms, +inf where not reached) and V at
the end of the window, plus the run's settings.  The windows contain the
wavefront, where iteration counts and errors differ most from the rest
phase:
  slab_h0.1          the 442,401-node ten Tusscher-Panfilov slab, dt 0.01 ms,
                     its full 10,000 steps (100 ms), REL_INITIAL 1e-10
  slab_h0.05_prefix  the 3,449,001-node slab, first 5,000 steps (50 ms),
                     REL_RHS 1e-8 (the precision form's settings)
  shell_prefix       the 1.26M-node ellipsoidal shell, held-out site 101,
                     dt 0.02 ms, first 2,500 steps (50 ms), REL_RHS 1e-10 (a
                     tolerance at which runs from different starting guesses
                     agree far inside the 1e-5 bar)
  cohort4            the four smallest instances (by node target) of the
                     64-shell batched cohort, Mitchell-Schaeffer, dt 0.01 ms,
                     their full 5,000 steps
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import orc  # noqa: E402
from paper_2510_12011_amd import inputs  # noqa: E402

SAMPLE = 32768


def sample_nodes(n, seed, k=SAMPLE):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=min(k, n), replace=False)).astype(np.int64)


def run(spec, steps, seed):
    o = orc.Oracle(spec)
    t0 = time.perf_counter()
    _, iters = o.steps(steps)
    el = time.perf_counter() - t0
    nodes = sample_nodes(spec.mesh.n_nodes, seed)
    st = o.state
    print(f"{spec.name}: {steps} steps in {el:.0f} s, mean iterations {iters.mean():.2f}, "
          f"activated {np.isfinite(st.lat).sum()} of {spec.mesh.n_nodes}", flush=True)
    return dict(nodes=nodes, lat=st.lat[nodes].copy(), V=st.V[nodes].copy(),
                n_nodes=np.int64(spec.mesh.n_nodes), steps=np.int64(steps),
                iters=iters.astype(np.int32), n_activated=np.int64(np.isfinite(st.lat).sum()))


def slab_h01():
    return {"slab": run(inputs.slab(h=0.1), 10000, 1)}


def slab_h005_prefix():
    return {"slab": run(inputs.slab_precision(h=0.05, precision="fp64"), 5000, 2)}


def shell_prefix():
    spec = inputs.shell_run(ionic="tt", dt=0.02, n_steps=2500, site_seed=101, rtol=1e-10)
    return {"shell": run(spec, 2500, 3)}


def cohort4():
    t = inputs.cohort_targets()
    small = [int(i) for i in np.argsort(t)[:4]]
    b = inputs.batch_shells(only=small)
    out = {}
    for k, i in enumerate(small):
        r = run(b.instance_spec(k), 5000, 10 + i)
        r["instance"] = np.int64(i)
        out[f"inst{i}"] = r
    return out


JOBS = {"slab_h0.1": slab_h01, "slab_h0.05_prefix": slab_h005_prefix,
        "shell_prefix": shell_prefix, "cohort4": cohort4}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("jobs", nargs="*", default=list(JOBS))
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    if a.threads:
        orc.lib().orc_set_threads(a.threads)
    for name in a.jobs:
        res = JOBS[name]()
        flat = {f"{grp}/{k}": v for grp, d in res.items() for k, v in d.items()}
        np.savez_compressed(os.path.join(HERE, f"{name}.npz"), **flat)
        print(f"wrote {name}.npz", flush=True)


if __name__ == "__main__":
    main()
