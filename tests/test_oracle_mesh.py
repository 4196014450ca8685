"""Pins of the mesh-refinement oracle (oracle/mesh.py), independent of the
HIP library: closed-form angles, exact predicates on degenerate inputs,
Delaunay triangulations from an independent library (scipy's Qhull) accepted,
and every planted mistake (flipped edge, reversed triangle, broken
neighbour, missing triangle, moved or orphaned point, skinny triangle,
encroached boundary edge) rejected."""
import math

import numpy as np
import pytest

from oracle import mesh as om
from oracle.validate import ValidationError
from paper_1607_05707_amd import meshgen


def _tri_mesh(points, tris):
    """Mesh arrays from explicit counter-clockwise triangles (neighbours by
    matching reversed edges)."""
    P = np.asarray(points, dtype=np.float64)
    T = np.zeros((len(tris), 4), dtype=np.int32)
    N = np.full((len(tris), 4), -1, dtype=np.int32)
    for i, t in enumerate(tris):
        T[i, :3] = t
        T[i, 3] = 1
    edges = {}
    for i, t in enumerate(tris):
        for k in range(3):
            edges[(t[k], t[(k + 1) % 3])] = (i, k)
    for (a, b), (i, k) in edges.items():
        if (b, a) in edges:
            N[i, k] = edges[(b, a)][0]
    return P, T, N


def test_min_angle_closed_forms():
    s3 = math.sqrt(3.0)
    cases = [([(0, 0), (1, 0), (0.5, s3 / 2)], 60.0),   # equilateral
             ([(0, 0), (1, 0), (0, 1)], 45.0),           # right isoceles
             ([(0, 0), (s3, 0), (0, 1)], 30.0),          # 30-60-90
             ([(0, 0), (s3, 0), (s3 / 2, 0.5)], 30.0),   # 30-30-120
             ([(0, 0), (1, 0), (0.5, 0.5 * math.tan(math.radians(10)))], 10.0)]
    for pts, want in cases:
        got = om.min_angles(np.array(pts), np.array([[0, 1, 2]]))[0]
        assert abs(got - want) < 1e-9, (pts, got, want)


def test_exact_predicates_on_degenerate_configurations():
    # four corners of a square are cocircular: the incircle sign is exactly 0
    a, b, c, d = (0.0, 0.0), (1.0, 0.0), (1.0, 1.0), (0.0, 1.0)
    assert om.incircle_sign([a], [b], [c], [d])[0] == 0
    # a point nudged by one unit in the last place inside / outside
    inside = (np.nextafter(0.0, 1.0), np.nextafter(1.0, 0.0))
    outside = (-np.nextafter(0.0, 1.0), 1.0)
    assert om.incircle_sign([a], [b], [c], [inside])[0] == 1
    assert om.incircle_sign([a], [b], [c], [outside])[0] == -1
    # collinear points and a point one ulp off the line
    assert om.orient_sign([(0.1, 0.1)], [(0.2, 0.2)], [(0.3, 0.3)])[0] == 0
    assert om.orient_sign([(0.0, 0.0)], [(1.0, 1.0)], [(0.5, np.nextafter(0.5, 1.0))])[0] == 1
    assert om.orient_sign([(0.0, 0.0)], [(1.0, 1.0)], [(0.5, np.nextafter(0.5, 0.0))])[0] == -1
    # cross-check the filtered signs against exact rational signs on random
    # near-degenerate inputs (points on a circle, rounded to doubles)
    rng = np.random.default_rng(3)
    ang = rng.uniform(0, 2 * math.pi, (400, 4))
    pts = np.stack([0.5 + 0.25 * np.cos(ang), 0.5 + 0.25 * np.sin(ang)], -1)
    s = om.incircle_sign(pts[:, 0], pts[:, 1], pts[:, 2], pts[:, 3])
    o = om.orient_sign(pts[:, 0], pts[:, 1], pts[:, 2])
    for i in range(400):
        exact_o = om._orient_exact(pts[i, 0], pts[i, 1], pts[i, 2])
        assert o[i] == exact_o
        exact = om._incircle_exact(pts[i, 0], pts[i, 1], pts[i, 2], pts[i, 3])
        assert s[i] == exact


def test_square_of_two_triangles():
    # both diagonals of the unit square are Delaunay (four cocircular points)
    pts = [(0, 0), (1, 0), (1, 1), (0, 1)]
    for tris in ([(0, 1, 2), (0, 2, 3)], [(0, 1, 3), (1, 2, 3)]):
        P, T, N = _tri_mesh(pts, tris)
        st = om.check_mesh(P, T, N, min_angle=45.0)
        assert st["triangles"] == 2 and abs(st["min_angle"] - 45.0) < 1e-9
    with pytest.raises(ValidationError):
        om.check_mesh(P, T, N, min_angle=46.0)


def test_accepts_a_quality_mesh_of_known_angles():
    # an m x m grid of cells, each split into four right isoceles triangles
    # at its centre: Delaunay (the corners of a cell and its centre are
    # cocircular: m a power of two keeps every coordinate exact), every
    # angle 45 or 90 degrees, boundary edges seen at 90
    m = 8
    pts = [(i / m, j / m) for j in range(m + 1) for i in range(m + 1)]
    tris = []
    for j in range(m):
        for i in range(m):
            c = len(pts)
            pts.append(((i + 0.5) / m, (j + 0.5) / m))
            v00, v10 = j * (m + 1) + i, j * (m + 1) + i + 1
            v01, v11 = v00 + m + 1, v10 + m + 1
            tris += [(v00, v10, c), (v10, v11, c), (v11, v01, c), (v01, v00, c)]
    P, T, N = _tri_mesh(pts, tris)
    st = om.check_mesh(P, T, N, min_angle=45.0)
    assert st["triangles"] == 4 * m * m and abs(st["min_angle"] - 45.0) < 1e-9
    with pytest.raises(ValidationError, match="angle"):
        om.check_mesh(P, T, N, min_angle=45.5)


def _scipy_mesh(n, seed):
    m = meshgen.random_square(n, seed, tri_factor=1.0, pt_factor=1.0)
    return m.pts[:m.npts], m.tri[:m.ntri].copy(), m.nbr[:m.ntri].copy(), m


def test_accepts_independent_delaunay_triangulations():
    for n, seed in ((50, 1), (400, 2), (3000, 3)):
        P, T, N, m = _scipy_mesh(n, seed)
        st = om.check_mesh(P, T, N, check_quality=False, check_encroachment=False, input_pts=m.input_pts)
        # Euler: a triangulation of a disk with V vertices, B of them on the
        # boundary, has 2V - B - 2 triangles
        k = len(P) - n
        assert st["triangles"] == 2 * len(P) - k - 2
        assert abs(st["area"] - 1.0) < 1e-12


def _interior_edge(T, N):
    for t in range(T.shape[0]):
        for k in range(3):
            if N[t, k] >= 0:
                return t, k
    raise AssertionError


def _flip(T, N, t, k):
    """Flip edge k of triangle t (and its twin) in place: a valid but (for a
    Delaunay input) non-Delaunay triangulation when the quad is convex."""
    q = N[t, k]
    a, b, c = T[t, k], T[t, (k + 1) % 3], T[t, (k + 2) % 3]
    j = [x for x in range(3) if T[q, x] == b][0]
    d = T[q, (j + 2) % 3]
    # neighbours outside the quad
    n_bc, n_ca = N[t, (k + 1) % 3], N[t, (k + 2) % 3]
    n_ad, n_db = N[q, (j + 1) % 3], N[q, (j + 2) % 3]
    T[t, :3] = (c, a, d)
    T[q, :3] = (d, b, c)
    N[t, :3] = (n_ca, n_ad, q)
    N[q, :3] = (n_db, n_bc, t)
    for nb, old, new in ((n_ad, q, t), (n_bc, t, q)):
        if nb >= 0:
            for x in range(3):
                if N[nb, x] == old:
                    N[nb, x] = new


def test_rejects_planted_mistakes():
    P, T0, N0, m = _scipy_mesh(400, 5)
    om.check_mesh(P, T0, N0, check_quality=False, check_encroachment=False)
    # a flipped edge: still a triangulation, no longer Delaunay
    flipped = 0
    for t in range(T0.shape[0]):
        for k in range(3):
            q = N0[t, k]
            if q < 0:
                continue
            T, N = T0.copy(), N0.copy()
            a, b, c = T[t, k], T[t, (k + 1) % 3], T[t, (k + 2) % 3]
            j = [x for x in range(3) if T[q, x] == b][0]
            d = T[q, (j + 2) % 3]
            pa, pb, pc, pd = P[a], P[b], P[c], P[d]
            convex = (om.orient_sign([pc], [pa], [pd])[0] > 0 and om.orient_sign([pd], [pb], [pc])[0] > 0)
            if not convex:
                continue
            if om.incircle_sign([pc], [pa], [pd], [pb])[0] <= 0:
                continue  # b on the circle through c, a, d: the flip stays Delaunay
            _flip(T, N, t, k)
            with pytest.raises(ValidationError, match="locally Delaunay"):
                om.check_mesh(P, T, N, check_quality=False, check_encroachment=False)
            flipped += 1
            if flipped >= 5:
                break
        if flipped >= 5:
            break
    assert flipped == 5
    t, k = _interior_edge(T0, N0)
    # a reversed triangle
    T, N = T0.copy(), N0.copy()
    T[t, :3] = T[t, [0, 2, 1]]
    with pytest.raises(ValidationError):
        om.check_mesh(P, T, N, check_quality=False, check_encroachment=False)
    # a neighbour entry pointing elsewhere
    T, N = T0.copy(), N0.copy()
    N[t, k] = (N[t, k] + 1) % T.shape[0]
    with pytest.raises(ValidationError):
        om.check_mesh(P, T, N, check_quality=False, check_encroachment=False)
    # a missing (dead) triangle
    T, N = T0.copy(), N0.copy()
    T[t, 3] = 0
    with pytest.raises(ValidationError):
        om.check_mesh(P, T, N, check_quality=False, check_encroachment=False)
    # an interior point moved (breaks orientation or Delaunay somewhere) and a
    # boundary point moved off the boundary
    n_b = P.shape[0] - 400
    for idx, delta in ((n_b + 7, (0.3, 0.2)), (1, (0.0, 1e-3))):
        Q = P.copy()
        Q[idx] = np.clip(Q[idx] + np.array(delta), 0.0, 1.0) if idx >= n_b else Q[idx] + np.array(delta)
        with pytest.raises(ValidationError):
            om.check_mesh(Q, T0, N0, check_quality=False, check_encroachment=False)
    # an orphan point, and input points not kept under their indices
    Q = np.concatenate([P, [[0.5, 0.5]]])
    with pytest.raises(ValidationError, match="not a vertex"):
        om.check_mesh(Q, T0, N0, check_quality=False, check_encroachment=False)
    wrong = m.input_pts.copy()
    wrong[[10, 11]] = wrong[[11, 10]]
    with pytest.raises(ValidationError, match="input points"):
        om.check_mesh(P, T0, N0, check_quality=False, check_encroachment=False, input_pts=wrong)


def test_quality_and_encroachment_checks():
    # a random Delaunay mesh has triangles far below 30 degrees
    P, T, N, _ = _scipy_mesh(400, 6)
    with pytest.raises(ValidationError, match="angle"):
        om.check_mesh(P, T, N, check_encroachment=False)
    # a right triangle whose right angle faces a boundary edge (90 degrees:
    # allowed) and one whose apex sees it at about 127 degrees (encroached)
    for apex, ok in (((0.5, 0.5), True), ((0.5, 0.25), False)):
        pts = [(0, 0), (1, 0), (1, 1), (0, 1), apex]
        tris = [(0, 1, 4), (1, 2, 4), (2, 3, 4), (3, 0, 4)]
        P2, T2, N2 = _tri_mesh(pts, tris)
        if ok:
            om.check_mesh(P2, T2, N2, min_angle=0.0)
        else:
            with pytest.raises(ValidationError, match="encroached"):
                om.check_mesh(P2, T2, N2, min_angle=0.0)


def test_generator_layout():
    m = meshgen.random_square(1000, 9)
    assert m.pts.shape[0] >= 6 * m.npts and m.tri.shape[0] >= 8 * m.ntri
    assert (m.tri[m.ntri:, 3] == 0).all() and (m.tri[:m.ntri, 3] == 1).all()
    # boundary points: k per side, evenly spaced, corners included
    k = (m.npts - 1000) // 4
    side = m.pts[:k, :]
    assert np.array_equal(side[:, 1], np.zeros(k)) and np.allclose(np.diff(side[:, 0]), 1.0 / k)
    # interior points strictly inside; deterministic by seed
    inner = m.pts[4 * k:m.npts]
    assert ((inner > 0) & (inner < 1)).all()
    assert np.array_equal(meshgen.random_square(1000, 9).pts, m.pts)
    assert not np.array_equal(meshgen.random_square(1000, 10).pts, m.pts)
