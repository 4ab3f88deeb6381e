"""Pins of the oracle's surface-triangle assembly (P1 triangles in 3D).

Every expected value here comes from outside the oracle: hand-computed
element matrices of the unit right triangle, invariance under rigid motions,
the exactness of P1 elements for linear functions, and the spectrum of the
Laplace-Beltrami operator on a sphere (eigenvalues l (l + 1) / R^2 with
multiplicity 2 l + 1).
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import orc
from paper_2510_12011_amd import inputs

UNIT = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])


def _rotation(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    return q if np.linalg.det(q) > 0 else -q


def test_unit_right_triangle_isotropic():
    # textbook P1 matrices of the triangle (0,0), (1,0), (0,1): area 1/2,
    # gradients (-1,-1), (1,0), (0,1)
    Me, Ke, det = orc.element_tri(UNIT)
    assert det == pytest.approx(1.0)
    np.testing.assert_allclose(Me, np.array([[2, 1, 1], [1, 2, 1], [1, 1, 2]]) / 24.0, atol=1e-15)
    np.testing.assert_allclose(Ke, 0.5 * np.array([[2, -1, -1], [-1, 1, 0], [-1, 0, 1]]),
                               atol=1e-15)


def test_unit_right_triangle_anisotropic():
    # fibre along x, sigma = diag(2, 0.5): K_ab = 1/2 (2 gx_a gx_b + 0.5 gy_a gy_b)
    _, Ke, _ = orc.element_tri(UNIT, fibre=[1.0, 0.0, 0.0], sl=2.0, st=0.5)
    np.testing.assert_allclose(Ke, [[1.25, -1.0, -0.25], [-1.0, 1.0, 0.0], [-0.25, 0.0, 0.25]],
                               atol=1e-15)
    # a fibre with a component normal to the triangle acts through its projection
    _, Kp, _ = orc.element_tri(UNIT, fibre=[3.0, 0.0, -5.0], sl=2.0, st=0.5)
    np.testing.assert_allclose(Kp, Ke, atol=1e-14)
    # a fibre normal to the triangle leaves it isotropic (transverse value)
    _, Kn, _ = orc.element_tri(UNIT, fibre=[0.0, 0.0, 1.0], sl=2.0, st=0.5)
    _, Ki, _ = orc.element_tri(UNIT, sl=0.5, st=0.5)
    np.testing.assert_allclose(Kn, Ki, atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_rigid_motion_invariance(seed):
    rng = np.random.default_rng(100 + seed)
    tri = rng.uniform(-1, 1, (3, 3))
    fib = rng.standard_normal(3)
    Q = _rotation(seed)
    shift = rng.uniform(-5, 5, 3)
    Me, Ke, _ = orc.element_tri(tri, fibre=fib, sl=1.7, st=0.3)
    Me2, Ke2, _ = orc.element_tri(tri @ Q.T + shift, fibre=Q @ fib, sl=1.7, st=0.3)
    np.testing.assert_allclose(Me2, Me, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(Ke2, Ke, rtol=1e-10, atol=1e-12)
    # relabelling the vertices permutes rows and columns
    perm = [2, 0, 1]
    Me3, Ke3, _ = orc.element_tri(tri[perm], fibre=fib, sl=1.7, st=0.3)
    np.testing.assert_allclose(Ke3, Ke[np.ix_(perm, perm)], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(Me3, Me[np.ix_(perm, perm)], rtol=1e-12, atol=1e-15)


def _planar_patch(seed, nx=7, ny=5, lx=2.0, ly=1.5):
    """A jittered nx*ny rectangle split into triangles, rotated into 3D."""
    rng = np.random.default_rng(seed)
    xs, ys = np.meshgrid(np.linspace(0, lx, nx + 1), np.linspace(0, ly, ny + 1), indexing="ij")
    P = np.stack([xs.ravel(), ys.ravel(), np.zeros(xs.size)], axis=1)
    inner = (xs.ravel() > 0) & (xs.ravel() < lx) & (ys.ravel() > 0) & (ys.ravel() < ly)
    P[inner, :2] += rng.uniform(-0.2, 0.2, (inner.sum(), 2)) * [lx / nx, ly / ny]
    tris = []
    for i in range(nx):
        for j in range(ny):
            a, b = i * (ny + 1) + j, (i + 1) * (ny + 1) + j
            tris += [(a, b, b + 1), (a, b + 1, a + 1)]
    Q = _rotation(seed + 7)
    return P @ Q.T + np.array([0.3, -1.0, 2.0]), np.array(tris, np.int32), Q, lx * ly


@pytest.mark.parametrize("seed", [0, 1])
def test_planar_patch_linear_exactness(seed):
    xyz, tris, Q, area = _planar_patch(seed)
    d = Q @ np.array([np.cos(0.4), np.sin(0.4), 0.0])        # in-plane fibre
    e = Q @ np.array([-np.sin(0.4), np.cos(0.4), 0.0])       # in-plane, across it
    nrm = Q @ np.array([0.0, 0.0, 1.0])
    sl, st = 0.9, 0.2
    fib = np.tile(d + 0.7 * nrm, (tris.shape[0], 1))        # projection is d
    mats = orc.assemble(xyz, tris, fib, sl, st)
    K, M = mats.dense("K"), mats.dense("M")
    n = xyz.shape[0]
    assert M.sum() == pytest.approx(area, rel=1e-12)
    np.testing.assert_allclose(K @ np.ones(n), 0.0, atol=1e-12)
    np.testing.assert_allclose(K, K.T, atol=1e-14)
    c = np.array([0.7, -1.3, 0.4])
    u = xyz @ c
    # energy of a linear function: area * (sl (c.d)^2 + st (c.e)^2); the
    # normal component of c is invisible to the surface gradient
    assert u @ K @ u == pytest.approx(area * (sl * (c @ d) ** 2 + st * (c @ e) ** 2), rel=1e-11)
    # M 1 is the lumped area per node; 1^T M u integrates u exactly
    assert np.ones(n) @ M @ u == pytest.approx(area * (c @ _centroid(xyz, tris)), rel=1e-11)


def _centroid(xyz, tris):
    p = xyz[tris]
    a = 0.5 * np.linalg.norm(np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), axis=1)
    return (a[:, None] * p.mean(axis=1)).sum(0) / a.sum()


def test_icosphere_pattern():
    xyz, tris = inputs.icosphere(2)
    row_ptr, col = orc.pattern(xyz.shape[0], tris)
    deg = np.diff(row_ptr)
    # 12 vertices of valence 5, the rest valence 6; plus the diagonal
    assert sorted(set(deg.tolist())) == [6, 7] and (deg == 6).sum() == 12
    assert col.shape[0] == xyz.shape[0] + 2 * 480


def test_sphere_laplace_beltrami_spectrum():
    R = 2.0
    u, tris = inputs.icosphere(3)
    mats = orc.assemble(R * u, tris, None, 1.0, 1.0)
    K, M = mats.dense("K"), mats.dense("M")
    assert M.sum() == pytest.approx(4 * np.pi * R ** 2, rel=2e-2)
    lam = scipy.linalg.eigh(K, M, eigvals_only=True)
    assert abs(lam[0]) < 1e-10
    np.testing.assert_allclose(lam[1:4], 2.0 / R ** 2, rtol=1e-2)      # l = 1
    np.testing.assert_allclose(lam[4:9], 6.0 / R ** 2, rtol=2e-2)      # l = 2
    assert lam[9] > 8.0 / R ** 2                                        # l = 3 next (12 / R^2)


def test_degenerate_triangle_rejected():
    xyz = np.array([[0.0, 0, 0], [1, 0, 0], [2, 0, 0], [0, 1, 0]])
    with pytest.raises(ValueError):
        orc.assemble(xyz, np.array([[0, 1, 2], [0, 1, 3]], np.int32), None, 1.0, 1.0)


def test_lumped_surface_mass_is_a_third_of_the_incident_areas():
    # row-sum lumping of the P1 surface mass: node i gets area/3 of every
    # triangle it belongs to (the consistent row sums are area/12 * (2+1+1))
    xyz, tris = inputs.icosphere(2)
    xyz = xyz * np.array([3.0, 2.0, 1.5])
    mats = orc.lumped(orc.assemble(xyz, tris, None, 1.0, 1.0))
    p = xyz[tris]
    area = 0.5 * np.linalg.norm(np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), axis=1)
    expect = np.zeros(xyz.shape[0])
    for k in range(3):
        np.add.at(expect, tris[:, k], area / 3.0)
    D = mats.dense("M")
    np.testing.assert_allclose(np.diag(D), expect, rtol=1e-13)
    assert not (D - np.diag(np.diag(D))).any()


def test_pattern_of_a_node_shared_by_2000_triangles():
    # a closed fan: the centre node shares all 2000 triangles, so its row
    # holds every node; rim nodes see the centre and their two neighbours
    k = 2000
    ang = 2 * np.pi * np.arange(k) / k
    xyz = np.concatenate([[[0.0, 0.0, 0.0]], np.stack([np.cos(ang), np.sin(ang), 0 * ang], 1)])
    tris = np.stack([np.zeros(k, np.int32), 1 + np.arange(k), 1 + (np.arange(k) + 1) % k],
                    axis=1).astype(np.int32)
    row_ptr, col = orc.pattern(k + 1, tris)
    assert row_ptr[1] - row_ptr[0] == k + 1
    assert np.array_equal(col[:k + 1], np.arange(k + 1))
    assert np.all(np.diff(row_ptr)[1:] == 4)
    mats = orc.assemble(xyz, tris, None, 1.0, 1.0)
    # the metric's determinant |e1|^2 |e2|^2 - (e1.e2)^2 cancels for these
    # 0.18-degree slivers: relative rounding up to about eps / sin^2(angle),
    # 2e-11 here
    assert mats.M.sum() == pytest.approx(0.5 * k * np.sin(2 * np.pi / k), rel=1e-10)


def test_surface_inputs_are_seeded_and_carry_the_atrial_parameters():
    a = inputs.batch_surfaces(n_inst=3, seed=5, n_steps=10)
    b = inputs.batch_surfaces(n_inst=3, seed=5, n_steps=10)
    for ia, ib in zip(a.instances, b.instances):
        assert np.array_equal(ia.mesh.xyz, ib.mesh.xyz) and ia.sigma_l == ib.sigma_l
        assert np.array_equal(ia.stimuli[0].nodes, ib.stimuli[0].nodes)
        assert ia.mesh.tets.shape[1] == 3 and ia.stimuli[0].nodes.size > 0
    assert a.instance_spec(1).ionic_params == inputs.ATRIUM_MS_PARAMS
    sp = inputs.atrium_surface(level=3, n_steps=10)
    assert sp.ionic_params == inputs.ATRIUM_MS_PARAMS and sp.mesh.n_nodes == 642
    assert (sp.rtol, sp.atol, sp.rel_mode, sp.max_iter, sp.dt) == (1e-5, 1e-5, 1, 100, 0.01)
