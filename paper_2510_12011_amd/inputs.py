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
* ``ellipsoid_shell``: a truncated ellipsoidal shell (ventricle-like) built
  as a curvilinear hexahedral grid split into Kuhn tets, with helical fibres.
* ``shell_cap``: a truncated ellipsoidal shell meshed as unstructured tets
  (Delaunay tetrahedralisation of a jittered lattice), with helical fibres;
  ``batch_shells`` draws a seeded cohort of them for the batched form.
* ``icosphere`` / ``ellipsoid_surface``: closed triangle surface meshes (the
  icosahedron refined by edge midpoints, pushed onto the unit sphere, then
  scaled to an ellipsoid), the stand-in for the paper's left-atrium surface
  meshes (``atrium_surface``).
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
    """A P1 mesh in mm: tetrahedra, or triangles of a surface in 3D.

    xyz     float64 [n, 3]  vertex coordinates (possibly jittered)
    tets    int32   [m, 4]  vertex ids, 0-based, positively oriented; or
                    [m, 3]  the vertex ids of surface triangles
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
    # regions given intra- and extracellular conductivities instead:
    # entries (region ids, il, it, el, et) in S/m, applied after sigma_l/t
    ie_regions: list = field(default_factory=list)
    lumped_mass: bool = False  # M lumped (row sums on the diagonal)
    ionic_params: tuple | None = None   # the cell model's parameters (None: defaults)

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


def nversion(h: float = 0.1, n_steps: int = 40000) -> RunSpec:
    """The N-version verification problem as the paper states it (its
    verification section and Table 2): the 20 x 7 x 3 mm cuboid with fibres
    along x, Kuhn tets of spacing h (0.5, 0.2 or 0.1 mm), no jitter,
    sigma_l / sigma_t 0.1334177 / 0.0173515 S/m, chi 140 /mm, Cm
    0.01 uF/mm^2, ten Tusscher-Panfilov, dt 0.005 ms.  The volumetric
    stimulus of 50 uA/mm^3 is chi * I_stim, so I_stim = 50/140 uA/mm^2, on the
    1.5 mm corner cube at P1 = (0, 0, 0) for 2 ms.  Solver as the slab's
    (rtol 1e-10 of ||z0||)."""
    nx, ny, nz = int(round(20 / h)), int(round(7 / h)), int(round(3 / h))
    mesh = kuhn_box(nx, ny, nz, 20.0, 7.0, 3.0, fibre=(1.0, 0.0, 0.0))
    chi = 140.0
    stim = Stimulus(box_corner_nodes(mesh, 1.5), 0.0, 2.0, 50.0 / chi)
    return RunSpec(name=f"nversion_h{h:g}", mesh=mesh, sigma_l=0.1334177, sigma_t=0.0173515,
                   chi=chi, cm=0.01, theta=0.5, ionic="tt", dt=0.005, n_steps=n_steps,
                   stimuli=[stim], rtol=1e-10, rel_mode=0)


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


# ---------------------------------------------------------------------------
# ellipsoidal shells (ventricle-like)
# ---------------------------------------------------------------------------
def ellipsoid_shell(a: float = 35.0, b: float = 30.0, c: float = 45.0, wall: float = 9.0,
                    n_nodes: int = 200_000, theta0_deg: float = 12.0,
                    fibre_endo_deg: float = 60.0, fibre_epi_deg: float = -60.0,
                    seed: int = 0, jitter: float = 0.1) -> Mesh:
    """Truncated ellipsoidal shell: epicardial semi-axes (a, b, c) in mm
    (c along z, the long axis), wall thickness `wall`, cut at the equatorial
    plane z = 0 and open at the apex (polar angle < theta0).

    Built as a curvilinear hexahedral grid in (depth, polar angle, azimuth)
    -- azimuth periodic -- split into Kuhn tets, with a seeded interior jitter
    of `jitter` of the local spacing in the polar and azimuthal directions.
    Grid counts are chosen for about `n_nodes` nodes with cells of similar
    size in all three directions.  Fibres: helical angle varying linearly
    through the wall from `fibre_endo_deg` (endocardium) to `fibre_epi_deg`
    (epicardium), measured from the circumferential direction towards the
    long axis.  Region tag 0 everywhere; grid holds the unjittered
    coordinates."""
    th0, th1 = np.deg2rad(theta0_deg), np.pi / 2
    rm = (a + b + c) / 3.0                         # mean epicardial radius
    r_in = 1.0 - wall / rm                         # inner surface as a radial fraction
    # cell counts: depth n_r, polar n_t, azimuth n_p (periodic)
    len_t = (th1 - th0) * (rm - 0.5 * wall)
    len_p = 2 * np.pi * (rm - 0.5 * wall) * np.sin(0.5 * (th0 + th1))
    h = (wall * len_t * len_p / n_nodes) ** (1.0 / 3.0)
    n_r = max(2, int(round(wall / h)))
    n_t = max(4, int(round(len_t / h)))
    n_p = max(8, int(round(len_p / h)))
    rr = np.linspace(r_in, 1.0, n_r + 1)
    tt = np.linspace(th0, th1, n_t + 1)
    pp = np.arange(n_p) * (2 * np.pi / n_p)
    R, TT, PP = np.meshgrid(rr, tt, pp, indexing="ij")
    rng = np.random.default_rng(seed)
    if jitter > 0:
        inner = (np.arange(n_t + 1) > 0) & (np.arange(n_t + 1) < n_t)
        dt_, dp_ = (th1 - th0) / n_t, 2 * np.pi / n_p
        jt = rng.uniform(-1, 1, TT.shape) * jitter * dt_
        jp = rng.uniform(-1, 1, PP.shape) * jitter * dp_
        TT = TT + jt * inner[None, :, None]
        PP = PP + jp
    def to_xyz(R, TT, PP):
        return np.stack([a * R * np.sin(TT) * np.cos(PP), b * R * np.sin(TT) * np.sin(PP),
                         c * R * np.cos(TT)], axis=-1)
    xyz = to_xyz(R, TT, PP).reshape(-1, 3)
    Rg, Tg, Pg = np.meshgrid(rr, tt, pp, indexing="ij")
    grid = to_xyz(Rg, Tg, Pg).reshape(-1, 3)

    def nid(i, j, k):
        return (i * (n_t + 1) + j) * n_p + (k % n_p)

    ci, cj, ck = np.meshgrid(np.arange(n_r), np.arange(n_t), np.arange(n_p), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    unit = np.eye(3, dtype=np.int64)
    tets = []
    for perm in itertools.permutations(range(3)):
        offs = [np.zeros(3, np.int64)]
        for ax in perm:
            offs.append(offs[-1] + unit[ax])
        cols = [nid(ci + o[0], cj + o[1], ck + o[2]) for o in offs]
        tets.append(np.stack(cols, axis=1))
    tets = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int64)
    # orient positively
    p = xyz[tets]
    det = np.einsum("ij,ij->i", p[:, 1] - p[:, 0], np.cross(p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]))
    flip = det < 0
    tets[flip, 2], tets[flip, 3] = tets[flip, 3].copy(), tets[flip, 2].copy()
    tets = tets.astype(np.int32)
    # helical fibres at element centroids (in the unjittered parametrisation)
    cen_r = rr[ci][:, None].repeat(6, axis=1).ravel() + 0.5 * (rr[1] - rr[0])
    cen_t = tt[cj][:, None].repeat(6, axis=1).ravel() + 0.5 * (tt[1] - tt[0])
    cen_p = pp[ck][:, None].repeat(6, axis=1).ravel() + np.pi / n_p
    depth = (cen_r - r_in) / (1.0 - r_in)                 # 0 endo .. 1 epi
    alpha = np.deg2rad(fibre_endo_deg + (fibre_epi_deg - fibre_endo_deg) * depth)
    e_p = np.stack([-a * np.sin(cen_p), b * np.cos(cen_p), np.zeros_like(cen_p)], axis=1)
    e_t = np.stack([a * np.cos(cen_t) * np.cos(cen_p), b * np.cos(cen_t) * np.sin(cen_p),
                    -c * np.sin(cen_t)], axis=1)
    e_p /= np.linalg.norm(e_p, axis=1, keepdims=True)
    e_t /= np.linalg.norm(e_t, axis=1, keepdims=True)
    fib = np.cos(alpha)[:, None] * e_p + np.sin(alpha)[:, None] * e_t
    fib /= np.linalg.norm(fib, axis=1, keepdims=True)
    mesh = Mesh(xyz=xyz, tets=tets, grid=grid, fibre=fib, region=np.zeros(tets.shape[0], np.int32),
                shape=(n_r, n_t, n_p))
    mesh.r_frac = np.repeat(rr, (n_t + 1) * n_p)        # per-node radial fraction
    mesh.r_in = r_in
    return mesh


def endocardial_site(mesh: Mesh, seed: int, radius: float = 1.5) -> np.ndarray:
    """Nodes within `radius` mm of a random endocardial node (seeded)."""
    if hasattr(mesh, "endo"):
        endo = np.nonzero(mesh.endo)[0]
    else:
        endo = np.nonzero(np.isclose(mesh.r_frac, mesh.r_in))[0]
    rng = np.random.default_rng(seed)
    centre = mesh.grid[endo[rng.integers(endo.shape[0])]]
    d = np.linalg.norm(mesh.grid - centre, axis=1)
    return np.nonzero(d <= radius)[0].astype(np.int32)


def shell_run(n_nodes: int = 1_200_000, ionic: str = "tt", dt: float = 0.02, n_steps: int = 20000,
              site_seed: int = 1, mesh_seed: int = 1000, sigma_scale: float = 1.0,
              rtol: float = 1e-8, rel_mode: int = 1, mesh: Mesh | None = None) -> RunSpec:
    """Ventricle-like shell run: sigma (0.17, 0.019) S/m times sigma_scale,
    chi 140/mm, Cm 0.01 uF/mm^2, 0.5 uA/mm^2 for 2 ms at a random endocardial
    site; relative tolerance 1e-8 of ||D^-1 b||."""
    if mesh is None:
        mesh = ellipsoid_shell(n_nodes=n_nodes, seed=mesh_seed)
    stim = Stimulus(endocardial_site(mesh, site_seed), 0.0, 2.0, 50.0 * UA_PER_CM2_TO_PER_MM2)
    return RunSpec(name=f"shell_{mesh.n_nodes}_site{site_seed}", mesh=mesh,
                   sigma_l=0.17 * sigma_scale, sigma_t=0.019 * sigma_scale, chi=140.0, cm=0.01,
                   theta=0.5, ionic=ionic, dt=dt, n_steps=n_steps, stimuli=[stim], rtol=rtol,
                   rel_mode=rel_mode)


# ---------------------------------------------------------------------------
# unstructured shells and the batched cohort
# ---------------------------------------------------------------------------
def _cap_map(P, a, b, c, wall, rd, r_in):
    """Parametric cylinder (disk of radius rd, height wall) -> ellipsoidal
    cap shell.  The disk radius maps linearly to the polar angle (0 at the
    apex, pi/2 at the equator), height to the radial fraction."""
    u, v = P[..., 0] / rd, P[..., 1] / rd
    rho = np.hypot(u, v)
    f = 0.5 * np.pi * np.sinc(0.5 * rho)          # sin(pi rho / 2) / rho, smooth at 0
    R = r_in + (1.0 - r_in) * (P[..., 2] / wall)
    return np.stack([a * R * f * u, b * R * f * v, c * R * np.cos(0.5 * np.pi * rho)], axis=-1)


def shell_cap(a: float = 35.0, b: float = 30.0, c: float = 45.0, wall: float = 9.0,
              n_nodes: int = 100_000, seed: int = 0, jitter: float = 0.25,
              fibre_endo_deg: float = 60.0, fibre_epi_deg: float = -60.0,
              q_min: float = 0.05) -> Mesh:
    """Truncated ellipsoidal shell (apex to the equatorial plane z = 0),
    epicardial semi-axes (a, b, c) mm with c along z, wall thickness `wall`,
    meshed with unstructured P1 tets.

    A cubic lattice of about `n_nodes` points fills a parametric cylinder
    (disk x wall depth); every coordinate is jittered by up to `jitter` of the
    spacing (seeded); the points are Delaunay-tetrahedralised
    (scipy.spatial.Delaunay, i.e. Qhull), tets of normalised quality
    6 sqrt(2) vol / l_rms^3 below `q_min` (slivers) are dropped with any node
    they leave unused, and the cylinder is mapped onto the shell (disk radius
    to polar angle, depth to the radial fraction).  Fibres: helical angle
    linear in depth from `fibre_endo_deg` (endocardium) to `fibre_epi_deg`
    (epicardium), from the circumferential direction towards the long axis,
    at element centroids.  mesh.endo marks the endocardial lattice layer."""
    from scipy.spatial import Delaunay
    rm = (a + b + c) / 3.0
    r_in = 1.0 - wall / rm
    rd = 0.5 * np.pi * rm
    h = (np.pi * rd * rd * wall / n_nodes) ** (1.0 / 3.0)
    for _ in range(3):   # match the lattice count to n_nodes
        nz = max(2, int(round(wall / h)))
        nd = int(np.ceil(rd / h))
        xs = np.arange(-nd, nd + 1) * h
        cnt = int(((xs[:, None] ** 2 + xs[None, :] ** 2) <= rd * rd).sum()) * (nz + 1)
        h *= (cnt / n_nodes) ** (1.0 / 3.0)
    nz = max(2, int(round(wall / h)))
    hz = wall / nz
    nd = int(np.ceil(rd / h))
    xs = np.arange(-nd, nd + 1) * h
    X, Y, Z = np.meshgrid(xs, xs, np.arange(nz + 1) * hz, indexing="ij")
    keep = (X * X + Y * Y) <= rd * rd
    grid_p = np.stack([X[keep], Y[keep], Z[keep]], axis=1)
    layer = np.rint(grid_p[:, 2] / hz).astype(np.int64)
    rng = np.random.default_rng(seed)
    P = grid_p + rng.uniform(-jitter, jitter, grid_p.shape) * np.array([h, h, hz])
    tets = Delaunay(P).simplices.astype(np.int64)
    e = P[tets]
    vol = np.einsum("ij,ij->i", e[:, 1] - e[:, 0], np.cross(e[:, 2] - e[:, 0], e[:, 3] - e[:, 0])) / 6.0
    l2 = sum(((e[:, i] - e[:, j]) ** 2).sum(1) for i in range(4) for j in range(i + 1, 4)) / 6.0
    q = 6.0 * np.sqrt(2.0) * np.abs(vol) / l2 ** 1.5
    tets = tets[q >= q_min]
    used = np.zeros(P.shape[0], bool)
    used[tets.ravel()] = True
    new_id = np.cumsum(used) - 1
    tets = new_id[tets]
    P, grid_p, layer = P[used], grid_p[used], layer[used]
    xyz = _cap_map(P, a, b, c, wall, rd, r_in)
    grid = _cap_map(grid_p, a, b, c, wall, rd, r_in)
    # orient positively in physical space
    e = xyz[tets]
    det = np.einsum("ij,ij->i", e[:, 1] - e[:, 0], np.cross(e[:, 2] - e[:, 0], e[:, 3] - e[:, 0]))
    flip = det < 0
    tets[flip, 2], tets[flip, 3] = tets[flip, 3].copy(), tets[flip, 2].copy()
    # fibres at parametric centroids
    cen = P[tets].mean(axis=1)
    rho = np.hypot(cen[:, 0], cen[:, 1]) / rd
    th, ph = 0.5 * np.pi * rho, np.arctan2(cen[:, 1], cen[:, 0])
    depth = np.clip(cen[:, 2] / wall, 0.0, 1.0)
    alpha = np.deg2rad(fibre_endo_deg + (fibre_epi_deg - fibre_endo_deg) * depth)
    e_p = np.stack([-a * np.sin(ph), b * np.cos(ph), np.zeros_like(ph)], axis=1)
    e_t = np.stack([a * np.cos(th) * np.cos(ph), b * np.cos(th) * np.sin(ph), -c * np.sin(th)],
                   axis=1)
    e_p /= np.linalg.norm(e_p, axis=1, keepdims=True)
    e_t /= np.linalg.norm(e_t, axis=1, keepdims=True)
    fib = np.cos(alpha)[:, None] * e_p + np.sin(alpha)[:, None] * e_t
    fib /= np.linalg.norm(fib, axis=1, keepdims=True)
    mesh = Mesh(xyz=xyz, tets=tets.astype(np.int32), grid=grid, fibre=fib,
                region=np.zeros(tets.shape[0], np.int32), shape=(nz, nd))
    mesh.endo = layer == 0
    return mesh


@dataclass
class Instance:
    """One member of a batch: its own mesh, conductivities and stimuli."""
    mesh: Mesh
    sigma_l: float
    sigma_t: float
    stimuli: list


@dataclass
class BatchSpec:
    """Independent monodomain problems advanced together (batched form)."""
    name: str
    instances: list
    chi: float
    cm: float
    theta: float
    ionic: str
    dt: float
    n_steps: int
    rtol: float = 1e-8
    atol: float = 0.0
    rel_mode: int = 1
    max_iter: int = 1000
    warm_start: int = 1
    precision: str = "mixed"
    rr_interval: int = 50
    ionic_params: tuple | None = None   # the cell model's parameters (None: defaults)

    @property
    def n_nodes(self) -> int:
        return sum(i.mesh.n_nodes for i in self.instances)

    def node_ptr(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum([i.mesh.n_nodes for i in self.instances])]).astype(
            np.int64)

    def instance_spec(self, k: int) -> RunSpec:
        """Instance k as a stand-alone run."""
        it = self.instances[k]
        return RunSpec(name=f"{self.name}_inst{k}", mesh=it.mesh, sigma_l=it.sigma_l,
                       sigma_t=it.sigma_t, chi=self.chi, cm=self.cm, theta=self.theta,
                       ionic=self.ionic, dt=self.dt, n_steps=self.n_steps, stimuli=it.stimuli,
                       rtol=self.rtol, atol=self.atol, rel_mode=self.rel_mode,
                       max_iter=self.max_iter, warm_start=self.warm_start,
                       precision=self.precision, rr_interval=self.rr_interval,
                       ionic_params=self.ionic_params)


def _cap_job(args):
    return shell_cap(**args)


def _gpu_may_be_live() -> bool:
    """True when this process may already hold a GPU context: torch has
    initialised its device runtime, or a profiler's preloaded library (which
    initialises the GPU before the program starts) is in the environment.
    Such a process is never forked; the meshes are then built serially."""
    import os
    import sys
    pre = os.environ.get("LD_PRELOAD", "")
    if "rocprof" in pre or any(k.startswith("ROCPROF") for k in os.environ):
        return True
    torch = sys.modules.get("torch")
    try:
        return bool(torch is not None and torch.cuda.is_initialized())
    except Exception:
        return True


def cohort_targets(n_inst: int = 64, total_nodes: int = 12_000_000, seed: int = 0,
                   n_min: int = 50_000, n_max: int = 400_000) -> np.ndarray:
    """Node targets of batch_shells' instances (the same draws)."""
    rng = np.random.default_rng(seed)
    rng.uniform(0.0, 1.0, (n_inst, 3))
    rng.uniform(0.0, 1.0, n_inst)
    n = np.exp(rng.uniform(np.log(n_min), np.log(n_max), n_inst))
    for _ in range(20):
        n = np.clip(n * (total_nodes / n.sum()), n_min, n_max)
    return n


def batch_shells(n_inst: int = 64, total_nodes: int = 12_000_000, seed: int = 0,
                 n_min: int = 50_000, n_max: int = 400_000, n_steps: int = 5000,
                 dt: float = 0.01, ionic: str = "ms", workers: int = 1,
                 axes_mm: tuple = (25.0, 45.0), wall_mm: tuple = (6.0, 12.0),
                 stim_radius: float = 1.5, only=None, progress=None) -> BatchSpec:
    """A seeded cohort of unstructured ellipsoidal shells: semi-axes
    U(axes_mm) (default 25-45 mm, the longest along z), wall U(wall_mm)
    (default 6-12 mm), node targets log-uniform in [n_min, n_max] rescaled to
    sum to about total_nodes (and clipped to the range), sigma (0.17, 0.019)
    S/m times U(0.5, 1.5), stimulus 0.5 uA/mm^2 for 2 ms on the nodes within
    stim_radius mm of a random endocardial node; Mitchell-Schaeffer cells,
    chi 140/mm, Cm 0.01 uF/mm^2, theta 0.5, relative tolerance 1e-8 of
    ||D^-1 b||, mixed precision.  only: indices of the instances to mesh and
    keep (in that order; every draw of the full cohort is still made, so each
    kept instance is the one the full cohort holds).  progress(done, total),
    if given, is called after each mesh built in this process."""
    rng = np.random.default_rng(seed)
    axes = np.sort(rng.uniform(axes_mm[0], axes_mm[1], (n_inst, 3)), axis=1)
    walls = rng.uniform(wall_mm[0], wall_mm[1], n_inst)
    n = np.exp(rng.uniform(np.log(n_min), np.log(n_max), n_inst))
    for _ in range(20):
        n = np.clip(n * (total_nodes / n.sum()), n_min, n_max)
    scale = rng.uniform(0.5, 1.5, n_inst)
    sites = rng.integers(0, 2 ** 31 - 1, n_inst)
    jobs = [dict(a=float(axes[i, 0]), b=float(axes[i, 1]), c=float(axes[i, 2]),
                 wall=float(walls[i]), n_nodes=int(n[i]), seed=int(seed * 1000 + i))
            for i in range(n_inst)]
    keep = list(range(n_inst)) if only is None else [int(i) for i in only]
    jobs = [jobs[i] for i in keep]
    if workers > 1 and not _gpu_may_be_live():
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            meshes = pool.map(_cap_job, jobs, chunksize=1)
    else:
        meshes = []
        for j in jobs:
            meshes.append(shell_cap(**j))
            if progress:
                progress(len(meshes), len(jobs))
    inst = []
    for i, m in zip(keep, meshes):
        stim = Stimulus(endocardial_site(m, int(sites[i]), stim_radius), 0.0, 2.0,
                        50.0 * UA_PER_CM2_TO_PER_MM2)
        inst.append(Instance(mesh=m, sigma_l=0.17 * scale[i], sigma_t=0.019 * scale[i],
                             stimuli=[stim]))
    return BatchSpec(name=f"shells{n_inst}_{sum(m.n_nodes for m in meshes)}", instances=inst,
                     chi=140.0, cm=0.01, theta=0.5, ionic=ionic, dt=dt, n_steps=n_steps)


# ---------------------------------------------------------------------------
# closed triangle surfaces (the atrial surface workload)
# ---------------------------------------------------------------------------
def icosphere(level: int):
    """Unit-sphere triangulation: the regular icosahedron (12 vertices, 20
    faces) with every triangle split into four at its edge midpoints
    ``level`` times, each new vertex pushed onto the sphere.  Returns
    (xyz [10*4^level + 2, 3], tris [20*4^level, 3] int32), faces oriented
    outwards."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    xyz = np.array([(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
                    (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
                    (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)], np.float64)
    xyz /= np.linalg.norm(xyz, axis=1, keepdims=True)
    tris = np.array([(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
                     (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
                     (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
                     (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)], np.int64)
    for _ in range(level):
        n = xyz.shape[0]
        a, b, c = tris[:, 0], tris[:, 1], tris[:, 2]
        e = np.stack([np.concatenate([a, b, c]), np.concatenate([b, c, a])], axis=1)
        key = np.minimum(e[:, 0], e[:, 1]) * n + np.maximum(e[:, 0], e[:, 1])
        uk, inv = np.unique(key, return_inverse=True)
        lo, hi = uk // n, uk % n
        mid = xyz[lo] + xyz[hi]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        xyz = np.concatenate([xyz, mid])
        m_ab, m_bc, m_ca = (n + inv).reshape(3, -1)
        tris = np.concatenate([np.stack([a, m_ab, m_ca], 1), np.stack([b, m_bc, m_ab], 1),
                               np.stack([c, m_ca, m_bc], 1), np.stack([m_ab, m_bc, m_ca], 1)])
    # orient outwards: (x1 - x0) x (x2 - x0) along the centroid
    p = xyz[tris]
    nrm = np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])
    flip = np.einsum("ij,ij->i", nrm, p.mean(axis=1)) < 0
    tris[flip, 1], tris[flip, 2] = tris[flip, 2].copy(), tris[flip, 1].copy()
    return xyz, tris.astype(np.int32)


def ellipsoid_surface(level: int, axes=(40.0, 33.0, 30.0), fibres: bool = True) -> Mesh:
    """Closed ellipsoidal surface (semi-axes in mm) from ``icosphere(level)``;
    fibres (if asked) along z x c for each triangle's centroid c, which the
    solver projects onto the triangle's plane."""
    u, tris = icosphere(level)
    xyz = u * np.asarray(axes, np.float64)
    fib = None
    if fibres:
        cen = xyz[tris].mean(axis=1)
        fib = np.stack([-cen[:, 1], cen[:, 0], np.zeros(cen.shape[0])], axis=1)
    return Mesh(xyz=xyz, tets=tris, grid=xyz.copy(), fibre=fib,
                region=np.zeros(tris.shape[0], np.int32), shape=(level,))


# parameters of the paper's left-atrium example ("Best Practices" section),
# applied to the classic two-variable Mitchell-Schaeffer model (the paper
# calls its cell model a modified one without giving the modification):
# tau_in, tau_out, tau_open, tau_close, u_gate (its u_crit, 0.1 there too, is
# the same threshold here), v_rest, v_amp
ATRIUM_MS_PARAMS = (0.15, 1.5, 105.0, 185.0, 0.1, -80.0, 100.0)


def atrium_surface(level: int = 8, n_steps: int = 5000, axes=(40.0, 33.0, 30.0),
                   radius: float = 2.0, ionic: str = "ms") -> RunSpec:
    """Left-atrium-like surface workload, after the paper's atrium example
    ("Best Practices" section; its surface timings are in "Performance
    measurements"): a closed ellipsoidal triangle surface (level 8: 655,362
    nodes, close to the 660,557-node atrial mesh it reports), isotropic
    0.4 S/m, dt 0.01 ms, a 50 uA/cm^2 stimulus for 2 ms on the nodes within
    ``radius`` mm of the +x apex, absolute and relative tolerance 1e-5
    (relative to ||D^-1 b||).  Cell model: the classic two-variable
    Mitchell-Schaeffer with the atrial parameters above (``ionic="ms"``) or
    the Courtemanche-Ramirez-Nattel atrial model (``"crn"``), the other
    atrial model the paper names."""
    mesh = ellipsoid_surface(level, axes, fibres=False)
    apex = np.array([axes[0], 0.0, 0.0])
    nodes = np.flatnonzero(np.linalg.norm(mesh.xyz - apex, axis=1) <= radius).astype(np.int32)
    stim = Stimulus(nodes, 0.0, 2.0, 50.0 * UA_PER_CM2_TO_PER_MM2)
    return RunSpec(name=f"atrium_surface_{mesh.n_nodes}", mesh=mesh, sigma_l=0.4, sigma_t=0.4,
                   chi=1400 * PER_CM_TO_PER_MM, cm=1.0 * UF_PER_CM2_TO_PER_MM2, theta=0.5,
                   ionic=ionic, dt=0.01, n_steps=n_steps, stimuli=[stim], rtol=1e-5, atol=1e-5,
                   rel_mode=1, max_iter=100,
                   ionic_params=ATRIUM_MS_PARAMS if ionic == "ms" else None)


def small_surface(level: int = 4, n_steps: int = 400, anisotropic: bool = True,
                  ionic: str = "ms") -> RunSpec:
    """A small ellipsoidal surface for parity runs (level 4: 2,562 nodes,
    semi-axes 8 x 6.6 x 6 mm), tangent-projected azimuthal fibres with 0.4 /
    0.1 S/m if ``anisotropic``, dt 0.01 ms; Mitchell-Schaeffer with the atrial
    parameters or (``ionic="crn"``) the Courtemanche-Ramirez-Nattel model."""
    axes = (8.0, 6.6, 6.0)
    mesh = ellipsoid_surface(level, axes, fibres=anisotropic)
    apex = np.array([axes[0], 0.0, 0.0])
    nodes = np.flatnonzero(np.linalg.norm(mesh.xyz - apex, axis=1) <= 1.2).astype(np.int32)
    stim = Stimulus(nodes, 0.0, 2.0, 50.0 * UA_PER_CM2_TO_PER_MM2)
    return RunSpec(name=f"small_surface_{mesh.n_nodes}", mesh=mesh, sigma_l=0.4,
                   sigma_t=0.1 if anisotropic else 0.4, chi=1400 * PER_CM_TO_PER_MM,
                   cm=1.0 * UF_PER_CM2_TO_PER_MM2, theta=0.5, ionic=ionic, dt=0.01,
                   n_steps=n_steps, stimuli=[stim], rtol=1e-10,
                   ionic_params=ATRIUM_MS_PARAMS if ionic == "ms" else None)


def batch_surfaces(n_inst: int = 4, levels=(3, 4), seed: int = 0, n_steps: int = 400,
                   axes_mm: tuple = (6.0, 9.0), stim_radius: float = 1.2,
                   precision: str = "mixed") -> BatchSpec:
    """A seeded cohort of closed ellipsoidal triangle surfaces (the paper's
    batch of atrial surfaces, in small): refinement level drawn from
    ``levels``, semi-axes U(axes_mm) sorted ascending, isotropic 0.4 S/m times
    U(0.5, 1.5), stimulus 0.5 uA/mm^2 for 2 ms on the nodes within
    stim_radius mm of a random node; the atrial Mitchell-Schaeffer
    parameters, dt 0.01 ms, rtol 1e-8 of ||D^-1 b||."""
    rng = np.random.default_rng(seed)
    inst = []
    for _ in range(n_inst):
        level = int(rng.choice(levels))
        axes = tuple(np.sort(rng.uniform(axes_mm[0], axes_mm[1], 3)))
        mesh = ellipsoid_surface(level, axes, fibres=False)
        c = mesh.xyz[rng.integers(mesh.n_nodes)]
        nodes = np.flatnonzero(np.linalg.norm(mesh.xyz - c, axis=1) <= stim_radius)
        sig = 0.4 * rng.uniform(0.5, 1.5)
        inst.append(Instance(mesh=mesh, sigma_l=sig, sigma_t=sig,
                             stimuli=[Stimulus(nodes.astype(np.int32), 0.0, 2.0,
                                               50.0 * UA_PER_CM2_TO_PER_MM2)]))
    return BatchSpec(name=f"batch_surfaces_{n_inst}", instances=inst,
                     chi=1400 * PER_CM_TO_PER_MM, cm=1.0 * UF_PER_CM2_TO_PER_MM2, theta=0.5,
                     ionic="ms", dt=0.01, n_steps=n_steps, rtol=1e-8, precision=precision,
                     ionic_params=ATRIUM_MS_PARAMS)
