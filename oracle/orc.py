"""Python access to the CPU oracle (``orc.c``).  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It compiles ``orc.c`` with gcc into ``liborc.so`` beside
this file and wraps its entry points with ctypes.  Everything here is plain
FP64 on the host; nothing here touches a GPU or the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import time
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB = os.path.join(_HERE, "liborc.so")

IONIC_KIND = {"none": 0, "ms": 1, "tt": 2, "crn": 3}


def build(force: bool = True) -> str:
    """Compile orc.c -> liborc.so (plain gcc, IEEE FP64, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i64, i32, f64 = C.c_int64, C.c_int, C.c_double
        L.orc_pattern.restype = i64
        L.orc_pattern.argtypes = [i64, i64, P, P, P, i64]
        L.orc_element.restype = f64
        L.orc_element.argtypes = [P, P, P, P, P, f64, f64, P, P]
        L.orc_assemble.restype = i64
        L.orc_assemble.argtypes = [i64, P, i64, P, P, P, P, P, P, P, P]
        L.orc_pattern_elems.restype = i64
        L.orc_pattern_elems.argtypes = [i64, i64, C.c_int, P, P, P, i64]
        L.orc_element_tri.restype = f64
        L.orc_element_tri.argtypes = [P, P, P, P, f64, f64, P, P]
        L.orc_assemble_tri.restype = i64
        L.orc_assemble_tri.argtypes = [i64, P, i64, P, P, P, P, P, P, P, P]
        L.orc_spmv.restype = None
        L.orc_spmv.argtypes = [i64, P, P, P, P, P]
        L.orc_pcg.restype = i32
        L.orc_pcg.argtypes = [i64, P, P, P, P, P, f64, f64, i32, i32, P]
        L.orc_ionic_nstates.restype = i32
        L.orc_ionic_nstates.argtypes = [i32]
        L.orc_ionic_nparams.restype = i32
        L.orc_ionic_nparams.argtypes = [i32]
        L.orc_ionic_defaults.restype = None
        L.orc_ionic_defaults.argtypes = [i32, P]
        L.orc_ionic_init.restype = None
        L.orc_ionic_init.argtypes = [i32, P, i64, P, P]
        L.orc_ionic_step.restype = None
        L.orc_ionic_step.argtypes = [i32, P, i64, f64, P, P, P]
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [i32]
        L.orc_get_threads.restype = i32
        L.orc_get_threads.argtypes = []
        L.orc_steps.restype = i32
        L.orc_steps.argtypes = [i64, P, P, P, P, P, i32, P, i32, P, P, P, P, P,
                                P, P, P, P, P, i64, i64, i64, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------------------
# assembly
# ---------------------------------------------------------------------------
def element(pts, fibre=None, sl=1.0, st=1.0):
    """Element mass and stiffness of one tet: (Me[4,4], Ke[4,4], det J)."""
    pts = _c(pts, np.float64).reshape(4, 3)
    fib = None if fibre is None else _c(fibre, np.float64)
    Me = np.zeros(16)
    Ke = np.zeros(16)
    det = lib().orc_element(_p(pts[0]), _p(pts[1]), _p(pts[2]), _p(pts[3]), _p(fib),
                            float(sl), float(st), _p(Me), _p(Ke))
    return Me.reshape(4, 4), Ke.reshape(4, 4), det


def element_tri(pts, fibre=None, sl=1.0, st=1.0):
    """Element mass and stiffness of one surface triangle in 3D:
    (Me[3,3], Ke[3,3], det of the metric E^T E)."""
    pts = _c(pts, np.float64).reshape(3, 3)
    fib = None if fibre is None else _c(fibre, np.float64)
    Me = np.zeros(9)
    Ke = np.zeros(9)
    det = lib().orc_element_tri(_p(pts[0]), _p(pts[1]), _p(pts[2]), _p(fib),
                                float(sl), float(st), _p(Me), _p(Ke))
    return Me.reshape(3, 3), Ke.reshape(3, 3), det


def pattern(n, elems):
    """CSR pattern of an element mesh ([m, 4] tetrahedra or [m, 3]
    surface triangles): row i holds every node sharing an element with i."""
    elems = _c(elems, np.int32)
    npe = elems.shape[1]
    row_ptr = np.zeros(n + 1, np.int64)
    nnz = lib().orc_pattern_elems(n, elems.shape[0], npe, _p(elems), _p(row_ptr), None, 0)
    col = np.zeros(nnz, np.int32)
    lib().orc_pattern_elems(n, elems.shape[0], npe, _p(elems), _p(row_ptr), _p(col), nnz)
    return row_ptr, col


@dataclass
class Matrices:
    row_ptr: np.ndarray
    col: np.ndarray
    M: np.ndarray
    K: np.ndarray

    @property
    def n(self):
        return self.row_ptr.shape[0] - 1

    def dense(self, which):
        v = self.M if which == "M" else self.K
        D = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        D[rows, self.col] = v
        return D


def assemble(xyz, tets, fibre, sl, st):
    """Global consistent mass M and stiffness K (CSR, sorted columns) of a
    tetrahedral mesh ([m, 4]) or a triangle surface mesh ([m, 3])."""
    xyz = _c(xyz, np.float64)
    tets = _c(tets, np.int32)
    n, m = xyz.shape[0], tets.shape[0]
    sl = _c(np.broadcast_to(sl, (m,)), np.float64)
    st = _c(np.broadcast_to(st, (m,)), np.float64)
    fib = None if fibre is None else _c(fibre, np.float64)
    row_ptr, col = pattern(n, tets)
    M = np.zeros(col.shape[0])
    K = np.zeros(col.shape[0])
    fn = lib().orc_assemble_tri if tets.shape[1] == 3 else lib().orc_assemble
    rc = fn(n, _p(xyz), m, _p(tets), _p(fib), _p(sl), _p(st),
            _p(row_ptr), _p(col), _p(M), _p(K))
    if rc != 0:
        raise ValueError(f"degenerate element {-rc - 1}")
    return Matrices(row_ptr, col, M, K)


def series_conductivity(s_i, s_e):
    """Monodomain conductivity of intra- and extracellular conductivities in
    one direction: the two in series, s_i s_e / (s_i + s_e) (reproduces
    Table 2's values from the intra/extra pairs)."""
    return s_i * s_e / (s_i + s_e)


def assemble_spec(spec):
    sl, st = spec.sigma_per_tet()
    sl, st = sl.copy(), st.copy()
    for ids, il, it, el, et in getattr(spec, "ie_regions", []):
        sel = np.isin(spec.mesh.region, np.atleast_1d(ids))
        sl[sel] = series_conductivity(il, el)
        st[sel] = series_conductivity(it, et)
    mats = assemble(spec.mesh.xyz, spec.mesh.tets, spec.mesh.fibre, sl, st)
    return lumped(mats) if getattr(spec, "lumped_mass", False) else mats


def lumped(mats: Matrices) -> Matrices:
    """The same matrices with M replaced by its row-sum lumping: each row's
    entries summed onto its diagonal, the rest zero (same pattern)."""
    rows = np.repeat(np.arange(mats.n), np.diff(mats.row_ptr))
    sums = np.bincount(rows, weights=mats.M, minlength=mats.n)
    M = np.where(mats.col == rows, sums[rows], 0.0)
    return Matrices(mats.row_ptr, mats.col, M, mats.K)


def spmv(mats: Matrices, val, x):
    x = _c(x, np.float64)
    y = np.zeros(mats.n)
    lib().orc_spmv(mats.n, _p(mats.row_ptr), _p(mats.col), _p(_c(val, np.float64)),
                   _p(x), _p(y))
    return y


def pcg(mats: Matrices, Aval, b, x0, atol=0.0, rtol=1e-10, rel_mode=0, max_iter=1000):
    x = _c(x0, np.float64).copy()
    zn = C.c_double(0.0)
    it = lib().orc_pcg(mats.n, _p(mats.row_ptr), _p(mats.col), _p(_c(Aval, np.float64)),
                       _p(_c(b, np.float64)), _p(x), atol, rtol, rel_mode, max_iter,
                       C.byref(zn))
    return x, it, zn.value


# ---------------------------------------------------------------------------
# ionic models
# ---------------------------------------------------------------------------
def ionic_defaults(kind: str):
    k = IONIC_KIND[kind]
    p = np.zeros(max(1, lib().orc_ionic_nparams(k)))
    lib().orc_ionic_defaults(k, _p(p))
    return p[:lib().orc_ionic_nparams(k)]


def ionic_nstates(kind: str) -> int:
    return lib().orc_ionic_nstates(IONIC_KIND[kind])


def ionic_init(kind: str, n: int, params=None):
    k = IONIC_KIND[kind]
    params = ionic_defaults(kind) if params is None else _c(params, np.float64)
    V = np.zeros(n)
    u = np.zeros(max(1, ionic_nstates(kind)) * n)
    lib().orc_ionic_init(k, _p(params), n, _p(V), _p(u))
    return V, u[:ionic_nstates(kind) * n].reshape(ionic_nstates(kind), n)


def ionic_step(kind: str, V, u, dt, params=None):
    """Advance states in place by one step from V; returns I_ion / Cm (mV/ms)."""
    k = IONIC_KIND[kind]
    params = ionic_defaults(kind) if params is None else _c(params, np.float64)
    V = _c(V, np.float64)
    n = V.shape[0]
    assert u.flags.c_contiguous and u.dtype == np.float64
    iion = np.zeros(n)
    lib().orc_ionic_step(k, _p(params), n, float(dt), _p(V), _p(u), _p(iion))
    return iion


# ---------------------------------------------------------------------------
# time stepping
# ---------------------------------------------------------------------------
@dataclass
class State:
    V: np.ndarray
    Vprev: np.ndarray
    u: np.ndarray
    lat: np.ndarray
    lrt: np.ndarray
    k: int = 0

    def copy(self):
        return State(self.V.copy(), self.Vprev.copy(), self.u.copy(), self.lat.copy(),
                     self.lrt.copy(), self.k)


class Oracle:
    """A monodomain run on the CPU: assembled matrices plus state."""

    def __init__(self, spec, ionic_params=None, mats: Matrices | None = None):
        self.spec = spec
        self.mats = assemble_spec(spec) if mats is None else mats
        self.kind = spec.ionic
        if ionic_params is None:
            ionic_params = getattr(spec, "ionic_params", None)
        self.params = (ionic_defaults(self.kind) if ionic_params is None
                       else _c(ionic_params, np.float64))
        n = spec.mesh.n_nodes
        V, u = ionic_init(self.kind, n, self.params)
        self.state = State(V, V.copy(), np.ascontiguousarray(u), np.full(n, np.inf),
                           np.full(n, np.inf), 0)
        st = spec.stimuli
        self.stim_off = np.zeros(len(st) + 1, np.int64)
        for i, s in enumerate(st):
            self.stim_off[i + 1] = self.stim_off[i] + len(s.nodes)
        self.stim_idx = (np.concatenate([s.nodes for s in st]).astype(np.int32)
                         if st else np.zeros(1, np.int32))
        self.stim_par = (np.array([[s.start, s.duration, s.intensity] for s in st],
                                  np.float64).ravel() if st else np.zeros(3))

    def steps(self, n_steps, out_every=0, extra_src=None, tissue=None):
        """Advance n_steps; returns (snapshots [n_out, n], iters [n_steps])."""
        sp, m, s = self.spec, self.mats, self.state
        n = m.n
        tissue = np.array(tissue if tissue is not None else
                          [sp.chi, sp.cm, sp.theta, sp.dt], np.float64)
        solver = np.array([sp.atol, sp.rtol], np.float64)
        isolver = np.array([sp.rel_mode, sp.max_iter, sp.warm_start], np.int32)
        n_out = n_steps // out_every if out_every > 0 else 0
        v_out = np.zeros((max(n_out, 1), n))
        iters = np.zeros(n_steps, np.int32)
        src = None if extra_src is None else _c(extra_src, np.float64)
        rc = lib().orc_steps(n, _p(m.row_ptr), _p(m.col), _p(m.M), _p(m.K), _p(tissue),
                             IONIC_KIND[self.kind], _p(self.params), len(sp.stimuli),
                             _p(self.stim_off), _p(self.stim_idx), _p(self.stim_par),
                             _p(solver), _p(isolver), _p(s.V), _p(s.Vprev), _p(s.u),
                             _p(s.lat), _p(s.lrt), s.k, n_steps, out_every, _p(v_out),
                             _p(iters), _p(src))
        s.k += n_steps
        self.last_rc = rc
        return v_out[:n_out], iters


def timed_steps(spec, n_steps, threads=None):
    """Wall time of n_steps of the oracle's step loop (setup excluded)."""
    if threads is not None:
        lib().orc_set_threads(int(threads))
    o = Oracle(spec)
    t0 = time.perf_counter()
    _, iters = o.steps(n_steps)
    return time.perf_counter() - t0, iters


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return lib().orc_get_threads()
