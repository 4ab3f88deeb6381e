"""Seeded synthetic inputs: meshes, fibres, stimulus sites and run parameters.

This module builds the arrays a monodomain simulation is given (vertex
coordinates, tetrahedra, fibre directions, stimulus node sets and the scalar
parameters of the problem statement in the paper's "Software functionality"
section).  It holds none of the method's arithmetic: no element matrices, no
ionic model, no solver.  Both the HIP path and the CPU oracle are fed from here.

Units follow the paper's Table 1: mm, ms, mV, uA/mm^2, uF/mm^2, 1/mm, S/m.

Meshes
------
* ``kuhn_box``: a structured box of nx*ny*nz hexahedra, each split into the six
  Kuhn (Freudenthal) tetrahedra that share the main diagonal of the hex; the
  split is conforming, so neighbouring hexes agree on their shared faces.
  Node numbering runs z fastest, then y, then x.
* ``ellipsoid_shell``: a truncated ellipsoidal shell (ventricle-like) meshed by
  Delaunay tetrahedralisation of a jittered lattice, with helical fibres.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# unit conversions (problem statements quote cm-based values)
# ---------------------------------------------------------------------------
PER_CM_TO_PER_MM = 0.1          # chi: 1400 /cm -> 140 /mm
UF_PER_CM2_TO_PER_MM2 = 0.01    # Cm: 1 uF/cm^2 -> 0.01 uF/mm^2
UA_PER_CM2_TO_PER_MM2 = 0.01    # I_stim: 50 uA/cm^2 -> 0.5 uA/mm^2


@dataclass
class Mesh:
    """A P1 tetrahedral mesh in mm.

    xyz     float64 [n, 3]  vertex coordinates (possibly jittered)
    tets    int32   [m, 4]  vertex ids, 0-based, positively oriented
    grid    float64 [n, 3]  unjittered coordinates (stimulus regions are
                            selected on these), equal to xyz if no jitter
    fibre   float64 [m, 3]  per-element fibre direction or None (isotropic)
    region  int32   [m]     element region tag
    """
    xyz: np.ndarray
    tets: np.ndarray
    grid: np.ndarray
    fibre: np.ndarray | None
    region: np.ndarray
    shape: tuple = ()

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])


def _node_id(i, j, k, ny, nz):
    return (i * (ny + 1) + j) * (nz + 1) + k


def kuhn_box(nx: int, ny: int, nz: int, lx: float, ly: float, lz: float,
             jitter: float = 0.0, seed: int = 0,
             fibre: tuple | None = None) -> Mesh:
    """Structured Kuhn-split box [0,lx]x[0,ly]x[0,lz] with nx*ny*nz hexes.

    ``jitter`` is the amplitude, as a fraction of the grid spacing along each
    axis, of a uniform per-coordinate perturbation applied only to nodes that
    lie on no boundary face (so the boundary, and the total volume, are
    unchanged).  Draws come from ``numpy.random.default_rng(seed)``.
    """
    hx, hy, hz = lx / nx, ly / ny, lz / nz
    ii, jj, kk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1),
                             np.arange(nz + 1), indexing="ij")
    grid = np.stack([ii.ravel() * hx, jj.ravel() * hy, kk.ravel() * hz],
                    axis=1).astype(np.float64)
    xyz = grid.copy()
    if jitter > 0.0:
        interior = ((ii > 0) & (ii < nx) & (jj > 0) & (jj < ny)
                    & (kk > 0) & (kk < nz)).ravel()
        rng = np.random.default_rng(seed)
        d = rng.uniform(-1.0, 1.0, size=(int(interior.sum()), 3))
        xyz[interior] += d * (jitter * np.array([hx, hy, hz]))

    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz),
                             indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    unit = np.eye(3, dtype=np.int64)
    tets = []
    for perm in itertools.permutations(range(3)):
        offs = [np.zeros(3, np.int64)]
        for ax in perm:
            offs.append(offs[-1] + unit[ax])
        # orientation of this permutation's tet on the unit cube
        e = np.array([offs[1], offs[2], offs[3]], dtype=np.float64)
        if np.linalg.det(e) < 0:
            offs[2], offs[3] = offs[3], offs[2]
        cols = [_node_id(ci + o[0], cj + o[1], ck + o[2], ny, nz) for o in offs]
        tets.append(np.stack(cols, axis=1))
    # interleave so the six tets of one hex are adjacent in memory
    tets = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    m = tets.shape[0]
    fib = None
    if fibre is not None:
        fib = np.tile(np.asarray(fibre, np.float64), (m, 1))
    return Mesh(xyz=xyz, tets=tets, grid=grid, fibre=fib,
                region=np.zeros(m, np.int32), shape=(nx, ny, nz))


def box_corner_nodes(mesh: Mesh, ex: float, ey: float | None = None,
                     ez: float | None = None, tol: float = 1e-9) -> np.ndarray:
    """Ids of the nodes whose unjittered coordinates satisfy x<=ex, y<=ey, z<=ez."""
    ey = ex if ey is None else ey
    ez = ex if ez is None else ez
    g = mesh.grid
    sel = (g[:, 0] <= ex + tol) & (g[:, 1] <= ey + tol) & (g[:, 2] <= ez + tol)
    return np.nonzero(sel)[0].astype(np.int32)


# ---------------------------------------------------------------------------
# run descriptions
# ---------------------------------------------------------------------------
@dataclass
class Stimulus:
    nodes: np.ndarray          # int32 node ids
    start: float               # ms
    duration: float            # ms
    intensity: float           # uA/mm^2


@dataclass
class RunSpec:
    """Everything a monodomain run is given, in the paper's units."""
    name: str
    mesh: Mesh
    sigma_l: float             # S/m, along the fibre
    sigma_t: float             # S/m, across the fibre
    chi: float                 # 1/mm
    cm: float                  # uF/mm^2
    theta: float
    ionic: str                 # "ms" | "tt"
    dt: float                  # ms
    n_steps: int
    stimuli: list = field(default_factory=list)
    rtol: float = 1e-10
    atol: float = 0.0
    rel_mode: int = 0          # 0: relative to the initial residual; 1: to D^-1 b
    max_iter: int = 1000
    warm_start: int = 1        # 0: previous step; 1: 2V^k - V^{k-1}
    out_every: int = 100       # snapshot interval in steps
    precision: str = "fp64"    # "fp64" | "mixed"
    rr_interval: int = 50      # mixed: residual replacement interval

    def sigma_per_tet(self):
        m = self.mesh.n_tets
        return (np.full(m, self.sigma_l, np.float64),
                np.full(m, self.sigma_t, np.float64))


def tiny_cube(n: int = 20, jitter: float = 0.05, seed: int = 0,
              n_steps: int = 500, stim_extent: float = 0.5) -> RunSpec:
    """Unit cube, n^3 hexes -> 6n^3 tets, isotropic sigma 0.1 S/m,
    two-variable Mitchell-Schaeffer cell model, corner stimulus
    50 uA/cm^2 for 2 ms, dt 0.01 ms, relative tolerance 1e-10."""
    mesh = kuhn_box(n, n, n, 1.0, 1.0, 1.0, jitter=jitter, seed=seed)
    stim = Stimulus(box_corner_nodes(mesh, stim_extent), 0.0, 2.0,
                    50.0 * UA_PER_CM2_TO_PER_MM2)
    return RunSpec(name=f"tiny_cube_{n}", mesh=mesh, sigma_l=0.1, sigma_t=0.1,
                   chi=1400 * PER_CM_TO_PER_MM, cm=1.0 * UF_PER_CM2_TO_PER_MM2,
                   theta=0.5, ionic="ms", dt=0.01, n_steps=n_steps,
                   stimuli=[stim], rtol=1e-10)


def slab(h: float = 0.1, n_steps: int = 10000, ionic: str = "tt",
         rtol: float = 1e-10, rel_mode: int = 0) -> RunSpec:
    """20 x 7 x 3 mm cuboid, structured grid of spacing h split into Kuhn
    tets, fibres along x, sigma_l 0.17 / sigma_t 0.019 S/m, ten Tusscher-type
    cell model, 1.5 mm corner cube stimulated at 50 uA/cm^2 for 2 ms, dt 0.01 ms."""
    nx, ny, nz = int(round(20 / h)), int(round(7 / h)), int(round(3 / h))
    mesh = kuhn_box(nx, ny, nz, 20.0, 7.0, 3.0, fibre=(1.0, 0.0, 0.0))
    stim = Stimulus(box_corner_nodes(mesh, 1.5), 0.0, 2.0,
                    50.0 * UA_PER_CM2_TO_PER_MM2)
    return RunSpec(name=f"slab_h{h:g}", mesh=mesh, sigma_l=0.17, sigma_t=0.019,
                   chi=1400 * PER_CM_TO_PER_MM, cm=1.0 * UF_PER_CM2_TO_PER_MM2,
                   theta=0.5, ionic=ionic, dt=0.01, n_steps=n_steps,
                   stimuli=[stim], rtol=rtol, rel_mode=rel_mode)


def small_box(nx=6, ny=5, nz=4, lx=1.2, ly=1.0, lz=0.8, jitter=0.05, seed=3,
              fibre=(0.6, 0.8, 0.0), ionic="ms", n_steps=50, theta=0.5,
              sigma_l=0.17, sigma_t=0.019, stim_extent=0.4, rtol=1e-10,
              dt=0.01) -> RunSpec:
    """A few-hundred-node anisotropic box for fast tests."""
    mesh = kuhn_box(nx, ny, nz, lx, ly, lz, jitter=jitter, seed=seed, fibre=fibre)
    stim = Stimulus(box_corner_nodes(mesh, stim_extent), 0.0, 2.0,
                    50.0 * UA_PER_CM2_TO_PER_MM2)
    return RunSpec(name=f"box_{nx}x{ny}x{nz}", mesh=mesh, sigma_l=sigma_l,
                   sigma_t=sigma_t, chi=140.0, cm=0.01, theta=theta, ionic=ionic,
                   dt=dt, n_steps=n_steps, stimuli=[stim], rtol=rtol)


def slab_precision(h: float = 0.05, n_steps: int = 10000, precision: str = "mixed") -> RunSpec:
    """The slab at h (default 0.05 mm: 401 x 141 x 61 = 3,449,001 nodes) for the
    mixed-precision form: relative tolerance 1e-8 against ||D^-1 b||, FP64
    residual replacement every 50 iterations and at convergence."""
    sp = slab(h=h, n_steps=n_steps, rtol=1e-8, rel_mode=1)
    sp.precision = precision
    sp.name = f"slab_h{h:g}_{precision}"
    return sp
