"""Python front end of the monodomain library (thin: marshalling only).

PyTorch provides the device memory (the persistent workspace and the setup
scratch are ``torch.uint8`` tensors on the device) and the HIP stream (the
current torch stream of that device).  Every step of the method runs in the
HIP kernels of ``libmonox.so``.

The call sequence mirrors the paper's API ("Best Practices" section):
device, ionic model with editable parameters, mesh with unit conversion,
per-region conductivities, stimuli, then solve with tolerances and a save
interval.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


IONIC = {"none": L.MDX_IONIC_NONE, "ms": L.MDX_IONIC_MS, "tt": L.MDX_IONIC_TT,
         "crn": L.MDX_IONIC_CRN}
# theta of the integration schemes the paper tabulates
THETA = {"forward_euler": 0.0, "crank_nicolson": 0.5, "galerkin": 2.0 / 3.0, "backward_euler": 1.0}

PRECISION = {"fp64": L.MDX_PREC_FP64, "mixed": L.MDX_PREC_MIXED,
             "mixed_gates32": L.MDX_PREC_MIXED_GATES32}


class Simulation:
    """One monodomain simulation on one GPU (one mdx_ctx)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self._torch = torch
        self.device = device
        torch.cuda.set_device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        self._check(L.lib().mdx_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream)),
                    ctx=None)
        self._h = h
        self._ws = None
        self.n = 0
        self.nstates = 0
        self.kind = "none"

    # -- plumbing -------------------------------------------------------
    def _check(self, status, ctx="self"):
        if status < 0:
            msg = (L.lib().mdx_last_error(self._h).decode() if ctx is not None else
                   "context creation failed")
            raise L.MdxError(status, msg)
        return status

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.lib().mdx_destroy(self._h)
            self._h = C.c_void_p()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- problem statement ----------------------------------------------
    def set_mesh(self, xyz, tets, region=None, fibre=None, unit_conversion=1.0):
        """Tetrahedra ([m, 4] ids) or, given [m, 3] ids, a triangle surface
        mesh in 3D; region and fibre are per element."""
        xyz = np.ascontiguousarray(xyz, np.float64)
        tets = np.ascontiguousarray(tets, np.int32)
        if tets.ndim != 2 or tets.shape[1] not in (3, 4):
            raise ValueError("elements must be an [m, 4] (tetrahedra) or [m, 3] (triangles) array")
        region = None if region is None else np.ascontiguousarray(region, np.int32)
        fibre = None if fibre is None else np.ascontiguousarray(fibre, np.float64)
        fn = L.lib().mdx_set_surface_mesh if tets.shape[1] == 3 else L.lib().mdx_set_mesh
        self._check(fn(self._h, xyz.shape[0], _ptr(xyz), unit_conversion, tets.shape[0],
                       _ptr(tets), _ptr(region), _ptr(fibre)))
        self.n = xyz.shape[0]

    def set_mesh_batch(self, node_ptr, xyz, tets, region=None, fibre=None, unit_conversion=1.0):
        """Several meshes as one batched context: instance i owns the nodes
        [node_ptr[i], node_ptr[i+1]) of the concatenated arrays."""
        ptr = np.ascontiguousarray(node_ptr, np.int64)
        xyz = np.ascontiguousarray(xyz, np.float64)
        tets = np.ascontiguousarray(tets, np.int32)
        if tets.ndim != 2 or tets.shape[1] not in (3, 4):
            raise ValueError("elements must be an [m, 4] (tetrahedra) or [m, 3] (triangles) array")
        region = None if region is None else np.ascontiguousarray(region, np.int32)
        fibre = None if fibre is None else np.ascontiguousarray(fibre, np.float64)
        fn = (L.lib().mdx_set_surface_mesh_batch if tets.shape[1] == 3
              else L.lib().mdx_set_mesh_batch)
        self._check(fn(self._h, ptr.shape[0] - 1, _ptr(ptr), xyz.shape[0], _ptr(xyz),
                       unit_conversion, tets.shape[0], _ptr(tets), _ptr(region), _ptr(fibre)))
        self.n = xyz.shape[0]
        self.node_ptr = ptr

    def add_conductivity(self, region_ids, il, it):
        ids = np.ascontiguousarray(np.atleast_1d(region_ids), np.int32)
        self._check(L.lib().mdx_add_conductivity(self._h, ids.shape[0], _ptr(ids), il, it))

    def add_conductivity_ie(self, region_ids, il, it, el, et):
        """Intra- (il, it) and extracellular (el, et) conductivities; the
        library combines them per direction."""
        ids = np.ascontiguousarray(np.atleast_1d(region_ids), np.int32)
        self._check(L.lib().mdx_add_conductivity_ie(self._h, ids.shape[0], _ptr(ids), il, it,
                                                    el, et))

    def set_tissue(self, chi, cm, theta=0.5):
        """theta: a number in [0, 1] or a scheme name of THETA."""
        theta = THETA[theta] if isinstance(theta, str) else theta
        self._check(L.lib().mdx_set_tissue(self._h, chi, cm, theta))

    def set_mass_lumping(self, lumped: bool):
        self._check(L.lib().mdx_set_mass_lumping(self._h, int(bool(lumped))))

    def set_ionic(self, kind: str, params=None):
        k = IONIC[kind]
        p = None if params is None else np.ascontiguousarray(params, np.float64)
        self._check(L.lib().mdx_set_ionic(self._h, k, 0 if p is None else p.shape[0], _ptr(p)))
        self.kind = kind
        self.nstates = L.lib().mdx_ionic_nstates(k)

    def add_stimulus(self, nodes, start, duration, intensity):
        idx = np.ascontiguousarray(nodes, np.int32)
        self._check(L.lib().mdx_add_stimulus(self._h, idx.shape[0], _ptr(idx), start, duration,
                                             intensity))

    def set_solver(self, atol=0.0, rtol=1e-10, rel_mode=0, max_iter=1000, warm_start=1,
                   precision=0, rr_interval=50):
        o = L.SolverOpts(atol, rtol, rel_mode, max_iter, warm_start, precision, rr_interval, 0)
        self._check(L.lib().mdx_set_solver(self._h, C.byref(o)))

    # -- device memory and setup ----------------------------------------
    def workspace_size(self):
        a, b = C.c_size_t(), C.c_size_t()
        self._check(L.lib().mdx_workspace_size(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def _alloc(self, nbytes):
        t = self._torch.empty(nbytes + 256, dtype=self._torch.uint8, device=f"cuda:{self.device}")
        off = (-t.data_ptr()) % 256
        return t, off

    def prepare(self, dt):
        pb, sb = self.workspace_size()
        ws, off = self._alloc(pb)
        self._check(L.lib().mdx_bind_workspace(self._h, C.c_void_p(ws.data_ptr() + off), pb))
        self._ws = ws
        scratch, soff = self._alloc(sb)
        self._check(L.lib().mdx_prepare(self._h, dt, C.c_void_p(scratch.data_ptr() + soff), sb))
        del scratch
        self.dt = dt

    # -- stepping and results --------------------------------------------
    def run(self, n_steps, out_every=0):
        """Advance n_steps; returns snapshots [n_steps // out_every, n] and the status."""
        n_out = n_steps // out_every if out_every > 0 else 0
        v_out = np.zeros((max(n_out, 1), self.n)) if n_out else None
        st = self._check(L.lib().mdx_run(self._h, n_steps, out_every, _ptr(v_out)))
        return (v_out[:n_out] if n_out else np.zeros((0, self.n))), st

    def times(self):
        lat, lrt = np.zeros(self.n), np.zeros(self.n)
        self._check(L.lib().mdx_get_times(self._h, _ptr(lat), _ptr(lrt)))
        return lat, lrt

    def apd(self):
        """Action potential duration per node, LRT - LAT (ms; inf where the
        node has not activated and repolarised)."""
        apd = np.zeros(self.n)
        self._check(L.lib().mdx_get_apd(self._h, _ptr(apd)))
        return apd

    def iterations(self, n):
        it = np.zeros(n, np.int32)
        self._check(L.lib().mdx_get_iterations(self._h, n, _ptr(it)))
        return it

    def stats(self):
        s = L.Stats()
        self._check(L.lib().mdx_get_stats(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in L.Stats._fields_}

    def set_tuning(self, max_groups=None, iter_scheme=None, lanes_per_row=None,
                   tiles_per_group=None, graph=None, fmt=None, nontemporal=None,
                   compact_columns=None, spmv_max_groups=None, persistent=None):
        """fmt: 'sell', 'csr', 'sell4' or 'sell4nt' (batched iteration SpMV
        storage), set before lanes_per_row; compact_columns: 16-bit column
        offsets in the single-mesh per-step kernels (default on)."""
        f = None if fmt is None else {"sell": 0, "csr": 1, "sell4": 2, "sell4nt": 3}[fmt]
        for key, v in ((L.MDX_TUNE_MAX_GROUPS, max_groups), (L.MDX_TUNE_ITER_SCHEME, iter_scheme),
                       (L.MDX_TUNE_SPMV_MAX_GROUPS, spmv_max_groups),
                       (L.MDX_TUNE_PERSISTENT, None if persistent is None else int(bool(persistent))),
                       (L.MDX_TUNE_FORMAT, f), (L.MDX_TUNE_NONTEMPORAL, nontemporal),
                       (L.MDX_TUNE_COMPACT_COLUMNS,
                        None if compact_columns is None else int(bool(compact_columns))),
                       (L.MDX_TUNE_LANES_PER_ROW, lanes_per_row),
                       (L.MDX_TUNE_TILES_PER_GROUP, tiles_per_group),
                       (L.MDX_TUNE_GRAPH, None if graph is None else int(bool(graph)))):
            if v is not None:
                self._check(L.lib().mdx_set_tuning(self._h, key, int(v)))

    def instance_iterations(self, n):
        """Batched context: PCG iterations [n steps, n_inst] (-1: not converged)."""
        k = self.node_ptr.shape[0] - 1
        it = np.zeros((n, k), np.int32)
        self._check(L.lib().mdx_get_instance_iterations(self._h, n, _ptr(it)))
        return it

    def autotune(self, reps=20):
        """Batched context: time the SpMV variants, install the fastest."""
        r = L.TuneReport()
        self._check(L.lib().mdx_autotune(self._h, int(reps), C.byref(r)))
        fmts = ("sell", "csr", "sell4", "sell4nt")
        cands = [(fmts[r.cand_format[i]], r.cand_lanes_per_row[i], r.cand_tiles_per_group[i],
                  r.cand_seconds[i]) for i in range(r.n_candidates)]
        return dict(fmt=fmts[r.format], lanes_per_row=r.lanes_per_row,
                    tiles_per_group=r.tiles_per_group, seconds=r.seconds, bytes=r.bytes,
                    candidates=cands)

    def set_profiling(self, every_n=1):
        """Time the SpMV launches of every every_n-th step (0: off)."""
        self._check(L.lib().mdx_set_profiling(self._h, int(every_n)))

    def get_state(self):
        V, Vp = np.zeros(self.n), np.zeros(self.n)
        u = np.zeros((self.nstates, self.n))
        lat, lrt = np.zeros(self.n), np.zeros(self.n)
        k = C.c_int64()
        self._check(L.lib().mdx_get_state(self._h, _ptr(V), _ptr(Vp),
                                          _ptr(u) if self.nstates else None, _ptr(lat),
                                          _ptr(lrt), C.byref(k)))
        return dict(V=V, Vprev=Vp, u=u, lat=lat, lrt=lrt, step=k.value)

    def set_state(self, V, Vprev, u=None, lat=None, lrt=None, step=0):
        f = lambda a: None if a is None else np.ascontiguousarray(a, np.float64)
        V, Vprev, u, lat, lrt = f(V), f(Vprev), f(u), f(lat), f(lrt)
        self._check(L.lib().mdx_set_state(self._h, _ptr(V), _ptr(Vprev), _ptr(u), _ptr(lat),
                                          _ptr(lrt), step))

    def matrix(self, which):
        """(rows, cols, vals) in original numbering; which in 'M', 'K', 'A'."""
        w = {"M": L.MDX_MAT_M, "K": L.MDX_MAT_K, "A": L.MDX_MAT_A}[which]
        nnz = C.c_int64()
        self._check(L.lib().mdx_get_matrix(self._h, w, C.byref(nnz), None, None, None))
        rows = np.zeros(nnz.value, np.int32)
        cols = np.zeros(nnz.value, np.int32)
        vals = np.zeros(nnz.value)
        self._check(L.lib().mdx_get_matrix(self._h, w, C.byref(nnz), _ptr(rows), _ptr(cols),
                                           _ptr(vals)))
        return rows, cols, vals

    def solve(self, b, x0):
        """One PCG solve of A x = b (the library's FP64 iteration, the solver
        options' tolerances); returns (x, iterations or -1)."""
        b = np.ascontiguousarray(b, np.float64)
        x0 = np.ascontiguousarray(x0, np.float64)
        x = np.empty_like(b)
        it = C.c_int32(0)
        self._check(L.lib().mdx_solve(self._h, _ptr(b), _ptr(x0), _ptr(x), C.byref(it)))
        return x, it.value

    def spmv(self, which, x):
        w = {"M": L.MDX_MAT_M, "K": L.MDX_MAT_K, "A": L.MDX_MAT_A}[which]
        x = np.ascontiguousarray(x, np.float64)
        y = np.zeros(self.n)
        self._check(L.lib().mdx_spmv(self._h, w, _ptr(x), _ptr(y)))
        return y

    def ionic_step(self, dt, V, u):
        """One ionic update of independent cells on device tensors (float64):
        V [n], u [nstates, n] updated in place; returns I_ion/Cm [n]."""
        torch = self._torch
        n = V.shape[0]
        iion = torch.empty(n, dtype=torch.float64, device=V.device)
        self._check(L.lib().mdx_ionic_step(self._h, dt, n, _dptr(V),
                                           _dptr(u) if self.nstates else None, _dptr(iion)))
        return iion


def from_spec(spec, device: int = 0, ionic_params=None, prepare=True,
              precision: str | None = None) -> Simulation:
    """Build a Simulation from an inputs.RunSpec (precision: 'fp64' or
    'mixed'; default: the spec's)."""
    sim = Simulation(device)
    m = spec.mesh
    sim.set_mesh(m.xyz, m.tets, m.region, m.fibre)
    sim.add_conductivity(np.unique(m.region), spec.sigma_l, spec.sigma_t)
    for ids, il, it, el, et in getattr(spec, "ie_regions", []):
        sim.add_conductivity_ie(ids, il, it, el, et)
    sim.set_tissue(spec.chi, spec.cm, spec.theta)
    if getattr(spec, "lumped_mass", False):
        sim.set_mass_lumping(True)
    if ionic_params is None:
        ionic_params = getattr(spec, "ionic_params", None)
    sim.set_ionic(spec.ionic, ionic_params)
    for s in spec.stimuli:
        sim.add_stimulus(s.nodes, s.start, s.duration, s.intensity)
    prec = precision if precision is not None else getattr(spec, "precision", "fp64")
    sim.set_solver(spec.atol, spec.rtol, spec.rel_mode, spec.max_iter, spec.warm_start,
                   PRECISION[prec], getattr(spec, "rr_interval", 50))
    if prepare:
        sim.prepare(spec.dt)
    return sim


def batch_from_spec(bspec, device: int = 0, ionic_params=None, prepare=True) -> Simulation:
    """Build a batched Simulation from an inputs.BatchSpec: the instances'
    meshes concatenated, instance k's elements tagged region k with its own
    conductivities, its stimuli moved to the concatenated numbering."""
    sim = Simulation(device)
    ptr = bspec.node_ptr()
    inst = bspec.instances
    xyz = np.concatenate([i.mesh.xyz for i in inst])
    tets = np.concatenate([i.mesh.tets + ptr[k] for k, i in enumerate(inst)]).astype(np.int32)
    region = np.concatenate([np.full(i.mesh.n_tets, k, np.int32) for k, i in enumerate(inst)])
    fibre = (None if any(i.mesh.fibre is None for i in inst) else
             np.concatenate([i.mesh.fibre for i in inst]))
    sim.set_mesh_batch(ptr, xyz, tets, region, fibre)
    for k, i in enumerate(inst):
        sim.add_conductivity([k], i.sigma_l, i.sigma_t)
    sim.set_tissue(bspec.chi, bspec.cm, bspec.theta)
    if ionic_params is None:
        ionic_params = getattr(bspec, "ionic_params", None)
    sim.set_ionic(bspec.ionic, ionic_params)
    for k, i in enumerate(inst):
        for s in i.stimuli:
            sim.add_stimulus(np.asarray(s.nodes) + ptr[k], s.start, s.duration, s.intensity)
    sim.set_solver(bspec.atol, bspec.rtol, bspec.rel_mode, bspec.max_iter, bspec.warm_start,
                   PRECISION[bspec.precision], bspec.rr_interval)
    if prepare:
        sim.prepare(bspec.dt)
    return sim


def batch_of_one(spec, device: int = 0, ionic_params=None, prepare=True) -> Simulation:
    """A single RunSpec as a batched context of one instance (same solver as
    a batch, for comparing a batch member with its stand-alone run)."""
    from .inputs import BatchSpec, Instance
    b = BatchSpec(name=spec.name, instances=[Instance(spec.mesh, spec.sigma_l, spec.sigma_t,
                                                      spec.stimuli)],
                  chi=spec.chi, cm=spec.cm, theta=spec.theta, ionic=spec.ionic, dt=spec.dt,
                  n_steps=spec.n_steps, rtol=spec.rtol, atol=spec.atol, rel_mode=spec.rel_mode,
                  max_iter=spec.max_iter, warm_start=spec.warm_start,
                  precision=spec.precision if spec.precision != "fp64" else "mixed",
                  rr_interval=spec.rr_interval)
    return batch_from_spec(b, device, ionic_params, prepare)
