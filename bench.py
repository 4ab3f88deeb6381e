"""Benchmark of the monodomain hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload learned]

A step is one time step of the whole hot path (ionic update, fused RHS and
initial residual, warm start, Jacobi-PCG to tolerance, activation times) on
the workload's synthetic mesh.  W untimed steps run first, the state is reset
to rest, then exactly K steps are timed between device synchronisations.  The
value is DOF*steps/s = n_nodes * K / seconds.

Workloads: learned (default: the learned warm start + mixed precision
against plain FP64 PCG on a 1.2M-node shell at equal accuracy), slab (plain
FP64, 442,401 nodes), precision / precision_fp64 (3.45M-node slab), batched
(64 shells, 12M nodes), tiny, nversion (the N-version verification problem at
0.5 / 0.2 / 0.1 mm, each run to full activation), surface / surface_mixed (the
atrial surface stand-in: 655,362-node closed triangle surface), batched_surface
(16 closed triangle surfaces advanced together).

Also reported, as one JSON line:
  roofline      the dominant kernel (PCG SpMV with fused p.q): algorithmic
                bytes per launch (12 B per structural nonzero + 16 B per row)
                over its mean duration, measured with HIP events attached to
                every dispatch of that kernel in the timed region, against
                8 TB/s; beside it a measured triad ceiling (c = a + 1.5 b
                over 1 GiB arrays)
  cpu_baseline  the CPU oracle (plain FP64 C, OpenMP) timed on this host on a
                bounded prefix of the same workload, and on one thread over a
                shorter prefix
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("DOF·steps/s at equal accuracy, learned+FP32 vs plain FP64 PCG; "
          "SpMV HBM GB/s")
HBM_PEAK_GBS = 8000.0
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "learned_shell_1.26M_hbm_traffic.md")
SLAB_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "precision_slab_3.45M_hbm_traffic.md")


def measured_traffic(profile, kernel, source):
    """HBM bytes per launch of `kernel` from a committed counter summary,
    or None if the summary is missing or the kernel's source file changed
    since the counters were taken (its recorded sha256 differs)."""
    import hashlib
    import re
    try:
        text = open(profile).read()
        src = open(os.path.join(ROOT, source), "rb").read()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch %s: (\S+)" % re.escape(kernel), text)
    h = re.search(r"source_sha256 %s: (\w+)" % re.escape(source), text)
    if not m or not h or hashlib.sha256(src).hexdigest() != h.group(1):
        return None
    return float(m.group(1))


def workload(name):
    """(spec, description, precision) of a named workload."""
    from paper_2510_12011_amd import inputs
    if name == "slab":
        return (inputs.slab(h=0.1),
                "slab 20x7x3 mm, h=0.1 mm Kuhn tets (442,401 nodes), ten Tusscher-Panfilov, "
                "plain FP64, rtol 1e-10 of ||z0||", "fp64")
    if name in ("precision", "precision_fp64"):
        prec = "mixed" if name == "precision" else "fp64"
        return (inputs.slab_precision(h=0.05, precision=prec),
                f"slab 20x7x3 mm, h=0.05 mm Kuhn tets (3,449,001 nodes), ten Tusscher-Panfilov, "
                f"{'mixed FP32/FP64' if prec == 'mixed' else 'plain FP64'}, rtol 1e-8 of ||D^-1 b||",
                prec)
    if name == "tiny":
        return (inputs.tiny_cube(), "unit cube 20^3 hexes, Mitchell-Schaeffer, plain FP64", "fp64")
    if name in ("surface", "surface_mixed"):
        prec = "mixed" if name == "surface_mixed" else "fp64"
        return (inputs.atrium_surface(),
                "atrial surface stand-in: closed ellipsoidal triangle surface 40x33x30 mm "
                "(655,362 nodes, 1,310,720 P1 triangles), classic two-variable Mitchell-Schaeffer with the "
                "paper's atrial parameters, isotropic 0.4 S/m, dt 0.01 ms, apex stimulus, "
                f"{'mixed FP32/FP64' if prec == 'mixed' else 'plain FP64'}, atol 1e-5 and "
                "rtol 1e-5 of ||D^-1 b||", prec)
    if name == "surface_crn":
        return (inputs.atrium_surface(ionic="crn"),
                "atrial surface stand-in: closed ellipsoidal triangle surface 40x33x30 mm "
                "(655,362 nodes, 1,310,720 P1 triangles), Courtemanche-Ramirez-Nattel atrial "
                "cell, isotropic 0.4 S/m, dt 0.01 ms, apex stimulus, plain FP64, atol 1e-5 and "
                "rtol 1e-5 of ||D^-1 b||", "fp64")
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(spec, steps, threads=None):
    from oracle import orc
    if threads:
        orc.lib().orc_set_threads(threads)
    o = orc.Oracle(spec)
    t0 = time.perf_counter()
    _, it = o.steps(steps)
    dt = time.perf_counter() - t0
    cores = orc.threads()
    # the single-core figure, on a shorter prefix of the same run
    s1 = max(1, steps // 8)
    orc.lib().orc_set_threads(1)
    o1 = orc.Oracle(spec, mats=o.mats)
    t0 = time.perf_counter()
    o1.steps(s1)
    dt1 = time.perf_counter() - t0
    orc.lib().orc_set_threads(cores)
    return {"value": spec.mesh.n_nodes * steps / dt, "unit": "DOF*steps/s",
            "cores": cores, "kind": "oracle",
            "sample": f"first {steps} steps from rest of the same workload "
                      f"(mean {float(np.mean(it)):.1f} CG iterations/step), setup excluded",
            "single_core": {"value": spec.mesh.n_nodes * s1 / dt1, "unit": "DOF*steps/s",
                            "sample": f"first {s1} steps from rest, one thread"}}


def triad_ceiling(mib=1024, reps=5):
    """Achievable HBM rate: c = a + 1.5 b over three 1 GiB FP32 arrays (12
    bytes per element moved), timed with events; the reference beside the
    8 TB/s specification peak."""
    import torch
    n = mib * 262144
    a = torch.rand(n, dtype=torch.float32, device="cuda:0")
    b = torch.rand_like(a)
    c = torch.empty_like(a)
    for _ in range(2):
        torch.add(a, b, alpha=1.5, out=c)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.add(a, b, alpha=1.5, out=c)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del a, b, c
    torch.cuda.empty_cache()
    return 12.0 * n / sec / 1e9


WEIGHTS = os.path.join(ROOT, "paper_2510_12011_amd", "weights", "shell_tt_dt0.02.npz")
CHECKPOINT_MS = 20.0
HELD_OUT = (101, 102, 103, 104, 105)
ACCURACY_BAR = 1e-5          # V relative L2 against the tight reference


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def shell_network(args, mesh, spec):
    """The learned warm start's network: the weights the training protocol
    (paper_2510_12011_amd/train.py: 20 sites x 400 ms) wrote for this mesh,
    else a short training here (printed as such)."""
    from paper_2510_12011_amd import learn, sim
    if os.path.exists(WEIGHTS):
        params, norm, meta = learn.load(WEIGHTS)
        if int(meta.get("n_nodes", -1)) == mesh.n_nodes:
            print(f"[bench] network: {os.path.relpath(WEIGHTS, ROOT)} (trained on "
                  f"{meta['sites']} sites x {meta['steps']} steps, {meta['samples']} samples, "
                  f"loss {meta['loss_first']:.4f} -> {meta['loss_last']:.4f})", flush=True)
            return params, norm, dict(meta, source="weights file")
    import torch
    t0 = time.perf_counter()
    Xs, Ds = [], []
    for site in range(1, args.train_sites + 1):
        s = sim.from_spec(spec(site, args.train_steps))
        X, dV = learn.record(s, args.train_steps, every=10, seed=site, cap=20000)
        Xs.append(X)
        Ds.append(dV)
        trainer = s
    X, dV = learn.concat(Xs), learn.concat(Ds)
    params, norm, hist = learn.fit(trainer, X, dV, epochs=args.train_epochs, batch=8192, lr=2e-3)
    print(f"[bench] network: no weights file for this mesh, trained here on {args.train_sites} "
          f"sites x {args.train_steps} steps in {time.perf_counter() - t0:.1f} s", flush=True)
    return params, norm, dict(sites=args.train_sites, steps=args.train_steps,
                              samples=int(X.shape[0]), loss_first=hist[0], loss_last=hist[-1],
                              source="trained in the benchmark")


def learned_workload(args):
    """The learned form (the headline): one ~1.2M-node ellipsoidal shell, ten
    Tusscher-Panfilov, dt 0.02 ms, stopping on ||D^-1 r|| relative to
    ||D^-1 b||.  The network (trained on the GPU by the library's kernels on
    20 trajectories of the plain solver, paper_2510_12011_amd/train.py)
    predicts the departure from the extrapolation 2V^k - V^{k-1}.

    Window: each held-out stimulus site is pre-run by plain FP64 PCG from rest
    to 20 ms, when the wavefront is inside the shell, and checkpointed; every
    timed run starts from that checkpoint (W untimed steps, the checkpoint
    restored, then K timed steps), so all of them time the same wavefront
    steps.  On site 101:
      * learned warm start + mixed precision (the value),
      * plain FP64 PCG with the paper's extrapolated warm start,
      * the other warm start x precision pairs,
    at the workload's tolerance 1e-8, and the first two and extrapolated +
    mixed again at 3e-9 ("equal accuracy": every run's V and activation times
    measured against plain FP64 at 1e-12 from the same checkpoint, the bar
    being 1e-5 and one dt); sites 102-105 repeat the three 3e-9 runs.  Also:
    the roofline of the iteration's SpMV on this shell (its FP32 matrix can
    stay in the Infinity Cache) and on the 3.45M-node slab (HBM-bound), and
    the CPU oracle on the same window."""
    import torch
    from oracle import orc
    from paper_2510_12011_amd import _lib as L, inputs, learn, sim
    t0 = time.perf_counter()
    mesh = inputs.ellipsoid_shell(n_nodes=1_200_000, seed=1000)
    n = mesh.n_nodes

    def spec(site, steps):
        return inputs.shell_run(mesh=mesh, ionic="tt", dt=0.02, n_steps=steps, site_seed=site)

    params, norm, net = shell_network(args, mesh, spec)
    k0 = int(round(CHECKPOINT_MS / 0.02))
    held = HELD_OUT[:max(1, min(args.sites, len(HELD_OUT)))]
    ckpt = {}
    for site in held:
        s = sim.from_spec(spec(site, k0), precision="fp64")
        s.set_solver(0.0, 1e-10, 1, 1000, L.MDX_WS_EXTRAP, 0, 50)
        s.run(k0)
        ckpt[site] = s.get_state()
        act = int(np.isfinite(ckpt[site]["lat"]).sum())
        print(f"[bench] site {site}: checkpoint at {CHECKPOINT_MS:g} ms, {act} of {n} nodes "
              f"activated", flush=True)
        s.close()
    print(f"[bench] shell {n} nodes; set-up {time.perf_counter() - t0:.1f} s", flush=True)

    ctxs = {}

    def context(precision, ws):
        key = (precision, ws)
        if key not in ctxs:
            s = sim.from_spec(spec(held[0], k0 + args.steps), precision=precision)
            if precision == "fp64" and args.iter_scheme is not None:
                s.set_tuning(iter_scheme=args.iter_scheme)
            if ws == L.MDX_WS_MLP:
                learn.install(s, params, norm)
            ctxs[key] = s
        return ctxs[key]

    def restore(s, c):
        s.set_state(c["V"], c["Vprev"], c["u"], c["lat"], c["lrt"], c["step"])

    def timed(precision, ws, rtol, site=held[0], profile=False):
        s = context(precision, ws)
        s.set_solver(0.0, rtol, 1, 1000, ws, sim.PRECISION[precision], 50)
        c = ckpt[site]
        if args.warmup:
            restore(s, c)
            s.run(args.warmup)
        restore(s, c)
        s.set_profiling(args.profile_every if profile else 0)
        st0 = s.stats()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, status = s.run(args.steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        st1 = s.stats()
        s.set_profiling(0)
        it = s.iterations(args.steps)
        state = s.get_state()
        st = {k: st1[k] - st0[k] for k in ("spmv_timed", "spmv_seconds", "spmv_bytes",
                                           "fallbacks")}
        st["nnz"] = st1["nnz"]
        name = {L.MDX_WS_MLP: "MLP", L.MDX_WS_EXTRAP: "extrapolated", L.MDX_WS_PREV: "previous"}[ws]
        print(f"[bench] site {site} {precision} warm start {name}, rtol {rtol:g}: {args.steps} "
              f"steps in {el:.3f} s, mean CG iterations {it.mean():.2f}, fallbacks "
              f"{st['fallbacks']}, status {status}", flush=True)
        return dict(seconds=el, iters=float(it.mean()), iters_p95=float(np.percentile(it, 95)),
                    stats=st, V=state["V"], lat=state["lat"], rate=n * args.steps / el)

    eq = 3e-9
    runs = {
        "learned_mixed_1e-8": timed("mixed", L.MDX_WS_MLP, 1e-8),
        "plain_fp64_1e-8": timed("fp64", L.MDX_WS_EXTRAP, 1e-8),
        "plain_fp64_prev_1e-8": timed("fp64", L.MDX_WS_PREV, 1e-8),
        "learned_fp64_1e-8": timed("fp64", L.MDX_WS_MLP, 1e-8),
        "extrap_mixed_1e-8": timed("mixed", L.MDX_WS_EXTRAP, 1e-8),
        "prev_mixed_1e-8": timed("mixed", L.MDX_WS_PREV, 1e-8),
        "learned_mixed_3e-9": timed("mixed", L.MDX_WS_MLP, eq, profile=True),
        "plain_fp64_3e-9": timed("fp64", L.MDX_WS_EXTRAP, eq),
        "extrap_mixed_3e-9": timed("mixed", L.MDX_WS_EXTRAP, eq),
    }
    tight = {held[0]: timed("fp64", L.MDX_WS_EXTRAP, 1e-12)}

    def accuracy(r, ref):
        e = float(np.linalg.norm(r["V"] - ref["V"]) / np.linalg.norm(ref["V"]))
        fa, fb = np.isfinite(r["lat"]), np.isfinite(ref["lat"])
        both = fa & fb
        lat = float(np.abs(r["lat"][both] - ref["lat"][both]).max()) if both.any() else 0.0
        return e, lat, int((fa != fb).sum())

    summary = {}
    for key, r in runs.items():
        e, lat, mism = accuracy(r, tight[held[0]])
        r.update(V_rel_l2=e, lat_max_diff_ms=lat, lat_mismatch=mism)
        summary[key] = {"dof_steps_per_s": r["rate"], "mean_cg_iters": r["iters"],
                        "p95_cg_iters": r["iters_p95"], "V_rel_l2": e, "lat_max_diff_ms": lat,
                        "lat_activation_mismatch": mism}
        print(f"[bench] {key}: {r['rate']:.3e} DOF*steps/s, V rel L2 {e:.2e}, LAT max diff "
              f"{lat:g} ms", flush=True)
    # the other held-out sites: the three runs at equal accuracy
    sites = {held[0]: {k: runs[k] for k in ("learned_mixed_3e-9", "plain_fp64_3e-9",
                                                "extrap_mixed_3e-9")}}
    for site in held[1:]:
        sites[site] = {"learned_mixed_3e-9": timed("mixed", L.MDX_WS_MLP, eq, site),
                       "plain_fp64_3e-9": timed("fp64", L.MDX_WS_EXTRAP, eq, site),
                       "extrap_mixed_3e-9": timed("mixed", L.MDX_WS_EXTRAP, eq, site)}
        tight[site] = timed("fp64", L.MDX_WS_EXTRAP, 1e-12, site)
        for r in sites[site].values():
            e, lat, mism = accuracy(r, tight[site])
            r.update(V_rel_l2=e, lat_max_diff_ms=lat, lat_mismatch=mism)

    def agg(key):
        rs = [sites[st][key] for st in held]
        return (n * args.steps * len(rs) / sum(r["seconds"] for r in rs),
                float(np.mean([r["iters"] for r in rs])), max(r["V_rel_l2"] for r in rs),
                max(r["lat_max_diff_ms"] for r in rs), sum(r["lat_mismatch"] for r in rs))

    five = {k: agg(k) for k in ("learned_mixed_3e-9", "plain_fp64_3e-9", "extrap_mixed_3e-9")}
    for k, v in five.items():
        print(f"[bench] {len(held)} held-out sites, {k}: {v[0]:.3e} DOF*steps/s, mean CG iterations "
              f"{v[1]:.2f}, worst V rel L2 {v[2]:.2e}, worst LAT diff {v[3]:g} ms", flush=True)
    lrn = runs["learned_mixed_3e-9"]
    plain = runs["plain_fp64_3e-9"]
    ok = all(r["V_rel_l2"] <= ACCURACY_BAR and r["lat_max_diff_ms"] <= 0.02 + 1e-12
             and r["lat_mismatch"] == 0 for st in held for r in sites[st].values())
    if not ok:
        print("[bench] WARNING: a run at 3e-9 missed the accuracy bar (1e-5, one dt): "
              "the speed-ups below are not at equal accuracy", flush=True)
    value = lrn["rate"]
    st = lrn["stats"]
    launches = max(1, st["spmv_timed"])
    spmv_avg = st["spmv_seconds"] / launches
    bytes_avg = st["spmv_bytes"] / launches
    achieved = bytes_avg / spmv_avg / 1e9
    desc = (f"learned form: ellipsoidal shell {n} nodes (Kuhn-split curvilinear grid), ten "
            f"Tusscher-Panfilov, dt 0.02 ms; per-node MLP warm start correcting the "
            f"extrapolation (BF16 MFMA, trained on the GPU) + mixed FP32/FP64 PCG vs plain FP64 "
            f"PCG (extrapolated warm start), both to rtol 3e-9 of ||D^-1 b|| (equal accuracy vs "
            f"FP64 at 1e-12), held-out site 101, window from a checkpoint at "
            f"{CHECKPOINT_MS:g} ms (wavefront inside the shell)")
    out = {
        "metric": METRIC, "value": value, "unit": "DOF*steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * lrn["seconds"] / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64+bf16", "data": "synthetic",
        "config": {"workload": desc, "n_nodes": n, "nnz": st["nnz"], "dt_ms": 0.02,
                   "rtol": eq, "window_start_ms": CHECKPOINT_MS,
                   "plain_fp64_dof_steps_per_s": plain["rate"],
                   "speedup_vs_plain_fp64": value / plain["rate"],
                   "speedup_vs_extrapolated_mixed": value / runs["extrap_mixed_3e-9"]["rate"],
                   "mean_cg_iters_learned": lrn["iters"], "mean_cg_iters_plain": plain["iters"],
                   "V_rel_l2_learned": lrn["V_rel_l2"], "V_rel_l2_plain": plain["V_rel_l2"],
                   "lat_max_diff_ms_learned": lrn["lat_max_diff_ms"],
                   "equal_accuracy": bool(ok),
                   "held_out_sites": len(held),
                   "five_sites_speedup_vs_plain_fp64":
                       five["learned_mixed_3e-9"][0] / five["plain_fp64_3e-9"][0],
                   "five_sites_speedup_vs_extrapolated_mixed":
                       five["learned_mixed_3e-9"][0] / five["extrap_mixed_3e-9"][0],
                   "five_sites_mean_cg_iters_learned": five["learned_mixed_3e-9"][1],
                   "five_sites_mean_cg_iters_extrapolated": five["extrap_mixed_3e-9"][1],
                   "accuracy_reference": "plain FP64 PCG at rtol 1e-12 from the same checkpoint",
                   "runs": summary, "fallbacks": int(st["fallbacks"]),
                   "train_sites": int(net["sites"]), "train_steps": int(net["steps"]),
                   "network": net["source"]},
        "roofline": {"bound": "hbm", "kernel": "k_cg_spmv32", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(TRAFFIC_PROFILE, "k_cg_spmv32",
                                                 "paper_2510_12011_amd/csrc/mdx_mixed.hip"),
                     "traffic_source": os.path.relpath(TRAFFIC_PROFILE, ROOT),
                     "bytes_per_launch": bytes_avg,
                     "avg_launch_us": 1e6 * spmv_avg, "launches_timed": st["spmv_timed"],
                     "sampled_every_n_steps": args.profile_every,
                     "cache_resident": bool(6 * st["nnz"] < 256e6)},
    }
    for s in ctxs.values():
        s.close()
    out["roofline_hbm"] = slab_roofline()
    tri = triad_ceiling()
    out["roofline"]["triad_GBs"] = tri
    out["roofline"]["frac_of_triad"] = achieved / tri
    out["roofline_hbm"]["triad_GBs"] = tri
    out["roofline_hbm"]["frac_of_triad"] = out["roofline_hbm"]["achieved"] / tri
    print(f"[bench] triad ceiling {tri:.0f} GB/s", flush=True)
    if not args.no_cpu:
        print(f"[bench] cpu baseline: oracle, {args.cpu_steps} steps of the same window",
              flush=True)
        sp = spec(held[0], k0 + args.cpu_steps)
        sp.rtol = eq
        out["cpu_baseline"] = cpu_baseline_window(sp, ckpt[held[0]], args.cpu_steps)
        out["config"]["cpu_single_core_dof_steps_per_s"] = out["cpu_baseline"]["single_core"]["value"]
        out["config"]["cpu_model"] = out["cpu_baseline"]["cpu_model"]
    print(json.dumps(out), flush=True)


def cpu_baseline_window(spec, state, steps):
    """The CPU oracle (all host cores) from the checkpoint state over `steps`
    steps of the benchmark's window, and on one thread over a quarter of
    them; setup excluded."""
    from oracle import orc
    o = orc.Oracle(spec)

    def start(o):
        o.state = orc.State(state["V"].copy(), state["Vprev"].copy(), state["u"].copy(),
                            state["lat"].copy(), state["lrt"].copy(), int(state["step"]))

    start(o)
    t0 = time.perf_counter()
    _, it = o.steps(steps)
    dt = time.perf_counter() - t0
    cores = orc.threads()
    s1 = max(1, steps // 4)
    orc.lib().orc_set_threads(1)
    o1 = orc.Oracle(spec, mats=o.mats)
    start(o1)
    t0 = time.perf_counter()
    o1.steps(s1)
    dt1 = time.perf_counter() - t0
    orc.lib().orc_set_threads(cores)
    model = cpu_model()
    n = spec.mesh.n_nodes
    return {"value": n * steps / dt, "unit": "DOF*steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} steps of the benchmark's window (from the checkpoint at "
                      f"{CHECKPOINT_MS:g} ms, mean {float(np.mean(it)):.1f} CG iterations/step, "
                      f"rtol {spec.rtol:g}), setup excluded; {model}; one thread: "
                      f"{n * s1 / dt1:.3e} DOF*steps/s over {s1} steps",
            "cpu_model": model,
            "single_core": {"value": n * s1 / dt1, "unit": "DOF*steps/s",
                            "sample": f"{s1} steps of the same window, one thread"}}


def slab_roofline(steps=60):
    """The iteration's FP32 SpMV on the 3.45M-node slab (its 306 MB matrix is
    larger than the Infinity Cache: every product streams it from HBM):
    events on every launch over `steps` steps after as many untimed ones."""
    from paper_2510_12011_amd import inputs, sim
    spec = inputs.slab_precision(h=0.05, precision="mixed")
    s = sim.from_spec(spec, precision="mixed")
    s.run(steps)
    s.set_profiling(1)
    st0 = s.stats()
    s.run(steps)
    st = s.stats()
    s.close()
    timed = st["spmv_timed"] - st0["spmv_timed"]
    sec = st["spmv_seconds"] - st0["spmv_seconds"]
    by = st["spmv_bytes"] - st0["spmv_bytes"]
    work = st["spmv_work"] - st0["spmv_work"]
    avg, bpl = sec / max(1, timed), by / max(1, work)
    achieved = by / sec / 1e9
    print(f"[bench] slab 3.45M: k_cg_spmv32 {1e6 * avg:.1f} us per launch, "
          f"{achieved:.0f} GB/s ({achieved / HBM_PEAK_GBS:.3f} of peak)", flush=True)
    return {"bound": "hbm", "kernel": "k_cg_spmv32",
            "workload": "slab 20x7x3 mm, h=0.05 mm (3,449,001 nodes, 51,020,601 nnz), mixed "
                        "FP32/FP64 PCG, ten Tusscher-Panfilov",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(SLAB_TRAFFIC_PROFILE, "k_cg_spmv32",
                                        "paper_2510_12011_amd/csrc/mdx_mixed.hip"),
            "traffic_source": os.path.relpath(SLAB_TRAFFIC_PROFILE, ROOT),
            "bytes_per_launch": bpl, "avg_launch_us": 1e6 * avg, "launches_timed": timed,
            "launches_with_product": work, "cache_resident": False}


def nversion_workload(args):
    """The N-version verification problem (dt 0.005 ms) at 0.5, 0.2 and 0.1 mm,
    each run from rest until every node has activated; activation times along
    the P1-P8 diagonal.  The value is the 0.1 mm run's DOF*steps/s."""
    import torch
    from paper_2510_12011_amd import inputs, nversion as nv, sim
    table, rate, n, steps01, el01 = {}, None, 0, 0, 0.0
    for h in (0.5, 0.2, 0.1):
        spec = inputs.nversion(h, 60000)
        s = sim.from_spec(spec)
        s.set_profiling(args.profile_every)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t, steps, _ = nv.run_to_activation(s, spec)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        table[f"{h:g}"] = {"P1_ms": float(t[0]), "P8_ms": float(t[-1]), "steps": steps,
                           "diagonal_ms": [round(float(v), 3) for v in t],
                           "mean_cg_iters": s.stats()["cg_iters_total"] / steps}
        print(f"[bench] dx {h}: {spec.mesh.n_nodes} nodes, {steps} steps in {el:.2f} s, "
              f"activation P1 {t[0]:.3f} ms, P8 {t[-1]:.3f} ms", flush=True)
        if h == 0.1:
            n, steps01, el01 = spec.mesh.n_nodes, steps, el
            rate = n * steps / el
            st = s.stats()
    launches = max(1, st["spmv_timed"])
    spmv_avg = st["spmv_seconds"] / launches
    bytes_avg = st["spmv_bytes"] / launches
    achieved = bytes_avg / spmv_avg / 1e9
    out = {
        "metric": METRIC, "value": rate, "unit": "DOF*steps/s", "n_gpus": 1, "steps": steps01,
        "warmup": 0, "ms_per_step": 1e3 * el01 / steps01, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "N-version problem (20x7x3 mm cuboid, TTP06, Table 2 sigma, "
                               "50 uA/mm^3 corner stimulus, dt 0.005 ms), dx 0.1 mm run from "
                               "rest to full activation; activation times along P1-P8 at "
                               "dx 0.5, 0.2, 0.1 mm",
                   "n_nodes": n, "activation": table},
        "roofline": {"bound": "hbm", "kernel": "k_spmv_dot", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "bytes_per_launch": bytes_avg,
                     "avg_launch_us": 1e6 * spmv_avg, "launches_timed": st["spmv_timed"],
                     "sampled_every_n_steps": args.profile_every,
                     "cache_resident": bool(10 * st["nnz"] < 256e6)},
    }
    print(json.dumps(out), flush=True)


def batched_workload(args):
    """The batched form: 64 unstructured ellipsoidal shells (about 12M
    nodes), Mitchell-Schaeffer, mixed precision, one block-diagonal solve per
    step with per-instance CG scalars, steps replayed as HIP graphs, SpMV
    layout chosen by the autotuner.  The cohort is meshed before torch or the
    library is loaded (its worker pool forks this process)."""
    from paper_2510_12011_amd import inputs
    t0 = time.perf_counter()
    surf = args.workload == "batched_surface"
    if surf:
        # a cohort of atrial-surface stand-ins: 16 closed ellipsoidal surfaces
        # of 163,842 or 655,362 nodes (7,536,672 in all), semi-axes 20-40 mm
        b = inputs.batch_surfaces(n_inst=16, levels=(7, 8), seed=0, n_steps=args.steps,
                                  axes_mm=(20.0, 40.0), stim_radius=2.0)
    else:
        b = inputs.batch_shells(n_inst=args.instances, total_nodes=args.total_nodes, seed=0,
                                workers=min(16, os.cpu_count() or 1),
                                progress=lambda k, m: print(f"[bench] meshed {k} of {m}",
                                                            flush=True))
    n = b.n_nodes
    sizes = [i.mesh.n_nodes for i in b.instances]
    print(f"[bench] {len(sizes)} {'surfaces' if surf else 'shells'}, {n} nodes "
          f"({min(sizes)}..{max(sizes)}), meshed in "
          f"{time.perf_counter() - t0:.1f} s", flush=True)
    import torch
    from paper_2510_12011_amd import sim
    t0 = time.perf_counter()
    s = sim.batch_from_spec(b)
    print(f"[bench] assembled and prepared in {time.perf_counter() - t0:.1f} s", flush=True)
    rep = s.autotune(reps=10)
    print(f"[bench] autotune: {rep['fmt']}, {rep['lanes_per_row']} lanes/row, "
          f"{rep['tiles_per_group']} tiles/group, {rep['seconds'] * 1e6:.1f} us", flush=True)
    for c in rep["candidates"]:
        print(f"[bench]   candidate {c[0]:4s} lanes/row {c[1]:2d} tiles/group {c[2]}: "
              f"{c[3] * 1e6:8.1f} us, {rep['bytes'] / c[3] / 1e9:7.1f} GB/s", flush=True)
    def install():
        s.set_tuning(fmt=rep["fmt"])
        s.set_tuning(lanes_per_row=rep["lanes_per_row"], tiles_per_group=rep["tiles_per_group"],
                     graph=not args.no_graph)
        if args.persistent:
            s.set_tuning(persistent=True)
    if args.warmup:
        install()
        s.run(args.warmup)
        s.prepare(b.dt)           # back to rest (also resets the layout choice)
    install()
    s.set_profiling(args.profile_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, status = s.run(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = s.stats()
    its = s.instance_iterations(args.steps)
    print(f"[bench] {args.steps} steps in {elapsed:.3f} s, mean CG iterations per instance "
          f"{its.mean():.2f} (max {its.max()}), status {status}", flush=True)
    launches = st["spmv_timed"]
    # the persistent iteration has no separate SpMV launches to time
    spmv_avg = st["spmv_seconds"] / launches if launches else None
    bytes_avg = st["spmv_bytes"] / launches if launches else None
    achieved = bytes_avg / spmv_avg / 1e9 if launches else None
    desc = (f"batched form: {len(sizes)} unstructured ellipsoidal shells (Delaunay, "
            f"{min(sizes)}..{max(sizes)} nodes, {n} total), Mitchell-Schaeffer, sigma scaled "
            f"U(0.5,1.5), random endocardial sites, mixed FP32/FP64, rtol 1e-8 of ||D^-1 b||, "
            f"per-instance CG, HIP-graph steps"
            f"{', persistent iteration kernel' if args.persistent else ''}")
    if surf:
        desc = (f"batched form: {len(sizes)} closed ellipsoidal triangle surfaces (atrial "
                f"stand-ins, {min(sizes)}..{max(sizes)} nodes, {n} total), Mitchell-Schaeffer "
                f"with the paper's atrial parameters, 0.4 S/m scaled U(0.5,1.5), random sites, "
                f"mixed FP32/FP64, rtol 1e-8 of ||D^-1 b||, per-instance CG, HIP-graph steps")
    out = {
        "metric": METRIC, "value": n * args.steps / elapsed, "unit": "DOF*steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": desc, "n_nodes": n, "n_instances": len(sizes),
                   "nnz": st["nnz"], "dt_ms": b.dt, "rtol": b.rtol,
                   "spmv_format": rep["fmt"], "lanes_per_row": rep["lanes_per_row"],
                   "tiles_per_group": rep["tiles_per_group"], "graph": not args.no_graph,
                   "persistent": bool(args.persistent),
                   "mean_cg_iters": float(its.mean()), "max_cg_iters": int(its.max())},
        "roofline": {"bound": "hbm",
                     "kernel": {"sell": "k_b_spmv", "csr": "k_b_spmv_csr", "sell4": "k_b_spmv_v4",
                                "sell4nt": "k_b_spmv_v4"}[rep["fmt"]],
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if launches else None, "traffic": None,
                     "bytes_per_launch": bytes_avg,
                     "avg_launch_us": 1e6 * spmv_avg if launches else None,
                     "launches_timed": st["spmv_timed"],
                     "sampled_every_n_steps": args.profile_every, "cache_resident": False},
    }
    if not args.no_cpu:
        from oracle import orc
        small = np.argsort(sizes)[:4]
        t_cpu, dof = 0.0, 0
        for k in small:
            o = orc.Oracle(b.instance_spec(int(k)))
            t1 = time.perf_counter()
            o.steps(args.cpu_steps)
            t_cpu += time.perf_counter() - t1
            dof += sizes[k] * args.cpu_steps
        out["cpu_baseline"] = {"value": dof / t_cpu, "unit": "DOF*steps/s", "cores": orc.threads(),
                               "kind": "oracle",
                               "sample": f"the 4 smallest instances, first {args.cpu_steps} steps "
                                         f"from rest each, setup excluded"}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: learned 3000, slab 10000, batched 1000, "
                         "precision 2000, tiny 500, surface 5000; nversion runs to full "
                         "activation)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps before the timed region (default: 0 learned, 10 batched, "
                         "100 otherwise)")
    ap.add_argument("--workload", default="learned",
                    choices=["learned", "slab", "precision", "precision_fp64", "batched", "tiny",
                             "nversion", "surface", "surface_mixed", "surface_crn",
                             "batched_surface"])
    ap.add_argument("--cpu-steps", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-every", type=int, default=10)
    ap.add_argument("--instances", type=int, default=64, help="batched workload")
    ap.add_argument("--total-nodes", type=int, default=12_000_000, help="batched workload")
    ap.add_argument("--no-graph", action="store_true", help="batched workload")
    ap.add_argument("--iter-scheme", type=int, choices=[0, 1], default=None,
                    help="FP64 PCG iteration in three kernels (0, the library's default) or "
                         "two (1): single-mesh workloads and the learned workload's FP64 runs")
    ap.add_argument("--persistent", action="store_true",
                    help="batched workload: CG iterations in one persistent launch")
    ap.add_argument("--copy-check", type=int, default=0, metavar="MIB",
                    help="after the run, copy a MIB-MiB device buffer 3 times (a kernel of known "
                         "traffic for scaling hardware byte counters)")
    ap.add_argument("--sites", type=int, default=5,
                    help="learned workload: held-out stimulus sites timed (1-5)")
    ap.add_argument("--train-sites", type=int, default=8, help="learned workload")
    ap.add_argument("--train-steps", type=int, default=2000, help="learned workload")
    ap.add_argument("--train-epochs", type=int, default=10, help="learned workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: a simulation runs on one GPU; the sharded "
              "multi-GPU path is a design, not code (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    if args.steps is None:
        args.steps = {"learned": 3000, "slab": 10000, "batched": 1000, "precision": 2000,
                      "precision_fp64": 2000, "tiny": 500, "nversion": 0, "surface": 5000,
                      "surface_mixed": 5000, "surface_crn": 5000, "batched_surface": 2000}[args.workload]
    if args.warmup is None:
        args.warmup = {"learned": 0, "batched": 10, "batched_surface": 10}.get(args.workload, 100)
    if args.workload in ("batched", "batched_surface"):
        batched_workload(args)
    elif args.workload == "nversion":
        nversion_workload(args)
    elif args.workload == "learned":
        learned_workload(args)
    else:
        single_workload(args)
    if args.copy_check:
        copy_check(args.copy_check)


def copy_check(mib):
    """Device-to-device copies of a known size: each reads and writes
    mib MiB, so a byte counter's reading on them gives its scale."""
    import torch
    a = torch.ones(mib * 262144, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"[bench] copy check: 3 copies of {mib} MiB ({mib * 1048576} bytes read and written each)",
          flush=True)


def single_workload(args):
    import torch
    from paper_2510_12011_amd import sim

    spec, desc, prec = workload(args.workload)
    n = spec.mesh.n_nodes
    print(f"[bench] workload {args.workload}: {n} nodes, {spec.mesh.n_tets} elements, {prec}",
          flush=True)
    s = sim.from_spec(spec, precision=prec)
    if args.iter_scheme is not None:
        s.set_tuning(iter_scheme=args.iter_scheme)
    st = s.stats()
    if args.warmup:
        s.run(args.warmup)
        s.prepare(spec.dt)          # back to rest; timing starts from t = 0
    # HIP events on the SpMV launches of every 10th step of the timed region
    # (events on every launch would slow the step loop by ~15%)
    s.set_profiling(args.profile_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, status = s.run(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = s.stats()
    iters = s.iterations(args.steps)
    print(f"[bench] {args.steps} steps in {elapsed:.3f} s, mean CG iterations "
          f"{iters.mean():.2f}, status {status}", flush=True)

    value = n * args.steps / elapsed
    nnz = st["nnz"]
    # dominant kernel: the PCG launch carrying q = A p.  Its algorithmic bytes
    # (summed by the library over the launches that did the product): per
    # structural nonzero the value and column (12 B FP64, 8 B FP32), per row p
    # read once and q written once (16 B FP64, 8 B FP32)
    launches = max(1, st["spmv_timed"])
    spmv_avg = st["spmv_seconds"] / launches
    bytes_avg = st["spmv_bytes"] / launches
    achieved = bytes_avg / spmv_avg / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": desc, "n_nodes": n, "nnz": nnz, "n_elements": spec.mesh.n_tets,
                   "dt_ms": spec.dt, "rtol": spec.rtol,
                   "stopping": "relative to ||z0||" if spec.rel_mode == 0 else "relative to ||D^-1 b||",
                   "warm_start": "2V^k - V^(k-1)", "mean_cg_iters": float(iters.mean()),
                   "max_cg_iters": int(iters.max()),
                   "iteration_kernels": 2 if prec != "fp64" or args.iter_scheme == 1 else 3},
        "roofline": {"bound": "hbm",
                     "kernel": ("k_cg_spmv" if args.iter_scheme == 1 else "k_spmv_dot")
                     if prec == "fp64" else "k_cg_spmv32",
                     "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "bytes_per_launch": bytes_avg,
                     "avg_launch_us": 1e6 * spmv_avg, "launches_timed": st["spmv_timed"],
                     "sampled_every_n_steps": args.profile_every,
                     "launches_with_product": st["spmv_work"],
                     "cache_resident": bool((12 if prec == "fp64" else 8) * nnz < 256e6)},
    }
    tri = triad_ceiling()
    out["roofline"]["triad_GBs"] = tri
    out["roofline"]["frac_of_triad"] = achieved / tri
    if not args.no_cpu:
        print(f"[bench] cpu baseline: oracle, {args.cpu_steps} steps", flush=True)
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
