"""The N-version workload's inputs and the diagonal sampling of nodal fields
(host only)."""
import numpy as np

from paper_2510_12011_amd import inputs, nversion as nv


def test_nversion_inputs():
    """Grid and tet counts, the stimulated corner cube, chi * I_stim = the
    volumetric 50 uA/mm^3, Table 2's conductivities and time step."""
    sp = inputs.nversion(0.5, 10)
    assert sp.mesh.n_nodes == 41 * 15 * 7
    assert sp.mesh.n_tets == 6 * 40 * 14 * 6
    st = sp.stimuli[0]
    assert len(st.nodes) == 4 ** 3 and st.start == 0.0 and st.duration == 2.0
    assert abs(sp.chi * st.intensity - 50.0) < 1e-12
    assert (sp.sigma_l, sp.sigma_t, sp.dt, sp.cm, sp.chi) == (0.1334177, 0.0173515, 0.005, 0.01, 140.0)
    assert len(inputs.nversion(0.2, 10).stimuli[0].nodes) == 8 ** 3
    assert np.array_equal(sp.mesh.xyz, sp.mesh.grid)   # no jitter


def _brute_force(mesh, field, p):
    """Value at p of the P1 interpolant, from the tet of the mesh that
    contains p (barycentric coordinates by a linear solve)."""
    for t in mesh.tets:
        x = mesh.xyz[t]
        lam = np.linalg.solve(np.vstack([x.T, np.ones(4)]), np.append(p, 1.0))
        if lam.min() >= -1e-12:
            return lam @ field[t]
    raise AssertionError("point outside the mesh")


def test_kuhn_interpolation_matches_the_containing_tet():
    """Random nodal field, random points: the sorted-coordinate rule equals
    the barycentric interpolant of the containing tet; nodes are exact."""
    sp = inputs.nversion(0.5, 10)
    m = sp.mesh
    rng = np.random.default_rng(3)
    field = rng.normal(size=m.n_nodes)
    # points in a few hexes only, so the brute-force search stays small
    cells = [(0, 0, 0), (7, 3, 2), (39, 13, 5), (20, 10, 1)]
    pts = np.concatenate([(np.array(c) + rng.uniform(0, 1, size=(6, 3))) * 0.5 for c in cells])
    got = nv.kuhn_interpolate(field, (40, 14, 6), nv.DIAGONAL, pts)
    sub = [i for i in range(m.n_tets)
           if any(np.all(np.floor(m.xyz[m.tets[i]].min(axis=0) / 0.5 + 1e-9) == c) for c in cells)]

    class Sub:
        pass
    s = Sub()
    s.xyz, s.tets = m.xyz, m.tets[sub]
    ref = np.array([_brute_force(s, field, p) for p in pts])
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)
    nodes = nv.diagonal_points(3)            # P1, the centre, P8 are grid nodes at h = 0.5
    ids = [0, (20 * 15 + 7) * 7 + 3, m.n_nodes - 1]
    np.testing.assert_allclose(nv.kuhn_interpolate(field, (40, 14, 6), nv.DIAGONAL, nodes),
                               field[ids], rtol=0, atol=1e-14)
