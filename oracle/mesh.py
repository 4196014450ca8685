"""CPU oracle for Delaunay mesh refinement (the workload of the Exclusive
construct, Section 3: the refine kernel and the Pipe that drives it).

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
bench's CPU-baseline leg may import this module.  It shares no code with the
HIP library and never calls it.

A refined mesh is not unique (it depends on the order in which bad
triangles are fixed), so the oracle is a complete checker of what every
correct result must satisfy, from the definitions:

* conformity: every live triangle is positively oriented; every edge is
  shared by exactly two live triangles with opposite orientation (their
  neighbour entries point at each other), or is a boundary edge lying on the
  boundary of the unit-square domain, and the boundary edges cover the
  square's perimeter once; the areas sum to the domain's.  Together these
  make the live triangles a triangulation of the square;
* Delaunay: every interior edge is locally Delaunay (the vertex across it
  is not strictly inside the triangle's circumcircle); by Delaunay's lemma
  the whole triangulation is then Delaunay;
* quality: every live triangle's smallest angle is at least the bound;
* no encroached boundary edge: the vertex opposite a boundary edge sees it
  at an angle of at most 90 degrees (the half of the edge's diametral disk
  inside the domain is empty);
* refinement: the input points keep their indices and coordinates, every
  point is a vertex of some live triangle.

Predicates.  orient(a, b, c) and incircle(a, b, c, d) are evaluated in
double precision with a forward error bound; when the value is within the
bound of zero the sign is recomputed exactly with rational arithmetic over
the (exactly representable) double coordinates.  Angles are compared in
double precision with a tolerance (``angle_tol`` degrees), since rounding
can decide a triangle at the bound either way.

Layout (the library's): points float64[P, 2]; triangles int32[T, 4] as
(v0, v1, v2, live flag); neighbours int32[T, 4] where entry i is the
triangle across edge (v_i, v_(i+1) mod 3), -1 on the domain boundary.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from .validate import ValidationError

EPS = np.finfo(np.float64).eps
# forward error bounds of the double-precision determinants, relative to the
# permanent (sum of absolute products); generous multiples of the classical
# constants (3 eps for orient, 10 eps for incircle)
_ORIENT_BOUND = 8.0 * EPS
_INCIRCLE_BOUND = 32.0 * EPS


def _orient_exact(a, b, c) -> int:
    ax, ay, bx, by, cx, cy = (Fraction(float(v)) for v in (a[0], a[1], b[0], b[1], c[0], c[1]))
    d = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)
    return (d > 0) - (d < 0)


def _incircle_exact(a, b, c, d) -> int:
    dx, dy = Fraction(float(d[0])), Fraction(float(d[1]))
    rows = []
    for p in (a, b, c):
        x = Fraction(float(p[0])) - dx
        y = Fraction(float(p[1])) - dy
        rows.append((x, y, x * x + y * y))
    (ax, ay, al), (bx, by, bl), (cx, cy, cl) = rows
    det = ax * (by * cl - bl * cy) - ay * (bx * cl - bl * cx) + al * (bx * cy - by * cx)
    return (det > 0) - (det < 0)


def orient_sign(a, b, c) -> np.ndarray:
    """Sign of the orientation determinant of (a, b, c) rows: +1 counter-
    clockwise, -1 clockwise, 0 collinear (exact)."""
    a, b, c = (np.atleast_2d(np.asarray(x, dtype=np.float64)) for x in (a, b, c))
    t1 = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1])
    t2 = (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    det = t1 - t2
    bound = _ORIENT_BOUND * (np.abs(t1) + np.abs(t2))
    sign = np.sign(det).astype(np.int64)
    unsure = np.flatnonzero(np.abs(det) <= bound)
    for i in unsure:
        sign[i] = _orient_exact(a[i], b[i], c[i])
    return sign


def incircle_sign(a, b, c, d) -> np.ndarray:
    """Sign of the incircle determinant: +1 when d is strictly inside the
    circle through the counter-clockwise triangle (a, b, c), 0 on it, -1
    outside (exact)."""
    a, b, c, d = (np.atleast_2d(np.asarray(x, dtype=np.float64)) for x in (a, b, c, d))
    ax, ay = a[:, 0] - d[:, 0], a[:, 1] - d[:, 1]
    bx, by = b[:, 0] - d[:, 0], b[:, 1] - d[:, 1]
    cx, cy = c[:, 0] - d[:, 0], c[:, 1] - d[:, 1]
    al, bl, cl = ax * ax + ay * ay, bx * bx + by * by, cx * cx + cy * cy
    t1 = ax * (by * cl - bl * cy)
    t2 = ay * (bx * cl - bl * cx)
    t3 = al * (bx * cy - by * cx)
    det = t1 - t2 + t3
    perm = (np.abs(ax) * (np.abs(by * cl) + np.abs(bl * cy)) + np.abs(ay) * (np.abs(bx * cl) + np.abs(bl * cx)) +
            al * (np.abs(bx * cy) + np.abs(by * cx)))
    sign = np.sign(det).astype(np.int64)
    unsure = np.flatnonzero(np.abs(det) <= _INCIRCLE_BOUND * perm)
    for i in unsure:
        sign[i] = _incircle_exact(a[i], b[i], c[i], d[i])
    return sign


def min_angles(pts, tri) -> np.ndarray:
    """Smallest interior angle (degrees) of every triangle, from the dot
    products of its edge vectors at each corner."""
    p = np.asarray(pts, dtype=np.float64)
    t = np.asarray(tri)[:, :3]
    out = np.full(t.shape[0], 180.0)
    for k in range(3):
        o = p[t[:, k]]
        u = p[t[:, (k + 1) % 3]] - o
        v = p[t[:, (k + 2) % 3]] - o
        cosang = (u * v).sum(1) / (np.linalg.norm(u, axis=1) * np.linalg.norm(v, axis=1))
        out = np.minimum(out, np.degrees(np.arccos(np.clip(cosang, -1.0, 1.0))))
    return out


def _on_side(p, which) -> np.ndarray:
    # unit-square sides: x = 0, x = 1, y = 0, y = 1
    axis, value = which
    return p[:, axis] == value


def check_mesh(pts, tri, nbr, *, npts=None, input_pts=None, min_angle=30.0, angle_tol=1e-6,
               check_encroachment=True, check_quality=True) -> dict:
    """Raise ValidationError unless the live triangles form a conforming
    Delaunay triangulation of the unit square with every angle at least
    `min_angle` (and, with `input_pts`, containing the input points under
    their indices).  Returns the mesh's statistics."""
    P = np.asarray(pts, dtype=np.float64)
    if npts is not None:
        P = P[:npts]
    T4 = np.asarray(tri, dtype=np.int64)
    N4 = np.asarray(nbr, dtype=np.int64)
    if T4.ndim != 2 or T4.shape[1] != 4 or N4.shape != T4.shape:
        raise ValidationError("triangles and neighbours must be [T, 4] arrays")
    live = np.flatnonzero(T4[:, 3] != 0)
    if live.size == 0:
        raise ValidationError("no live triangle")
    t = T4[live, :3]
    if (t < 0).any() or (t >= P.shape[0]).any():
        raise ValidationError("a live triangle names a point out of range")
    if ((t[:, 0] == t[:, 1]) | (t[:, 1] == t[:, 2]) | (t[:, 0] == t[:, 2])).any():
        raise ValidationError("a live triangle repeats a vertex")
    # orientation
    osg = orient_sign(P[t[:, 0]], P[t[:, 1]], P[t[:, 2]])
    if (osg <= 0).any():
        bad = live[np.flatnonzero(osg <= 0)[0]]
        raise ValidationError(f"triangle {bad} is not positively oriented")
    # neighbour symmetry, edge by edge
    is_live = np.zeros(T4.shape[0], dtype=bool)
    is_live[live] = True
    nb = N4[live, :3]
    a_all = t
    b_all = t[:, [1, 2, 0]]
    boundary_len = 0.0
    interior = []
    for k in range(3):
        a, b, q = a_all[:, k], b_all[:, k], nb[:, k]
        inner = q >= 0
        if (q[inner] >= T4.shape[0]).any():
            raise ValidationError("a neighbour index is out of range")
        qi = q[inner]
        if not is_live[qi].all():
            raise ValidationError("a live triangle's neighbour is not live")
        # the neighbour must hold the reversed edge and point back
        back_ok = np.zeros(qi.size, dtype=bool)
        src = live[inner]
        for j in range(3):
            ta = T4[qi, j]
            tb = T4[qi, (j + 1) % 3]
            back_ok |= (ta == b[inner]) & (tb == a[inner]) & (N4[qi, j] == src)
        if not back_ok.all():
            i = np.flatnonzero(~back_ok)[0]
            raise ValidationError(f"edge {int(a[inner][i])}-{int(b[inner][i])} of triangle {int(src[i])}: "
                                  "neighbour does not hold the reversed edge pointing back")
        interior.append((live[inner], k, qi))
        # boundary edges: both ends on the same side of the square, the
        # domain to their left (counter-clockwise perimeter)
        pa, pb = P[a[~inner]], P[b[~inner]]
        on_some = np.zeros(pa.shape[0], dtype=bool)
        for which in ((0, 0.0), (0, 1.0), (1, 0.0), (1, 1.0)):
            on_some |= _on_side(pa, which) & _on_side(pb, which)
        if not on_some.all():
            i = np.flatnonzero(~on_some)[0]
            raise ValidationError(f"boundary edge {int(a[~inner][i])}-{int(b[~inner][i])} is not on the domain boundary")
        boundary_len += float(np.linalg.norm(pb - pa, axis=1).sum())
    if abs(boundary_len - 4.0) > 1e-9:
        raise ValidationError(f"boundary edges cover {boundary_len} of the perimeter 4")
    area = 0.5 * ((P[t[:, 1], 0] - P[t[:, 0], 0]) * (P[t[:, 2], 1] - P[t[:, 0], 1]) -
                  (P[t[:, 1], 1] - P[t[:, 0], 1]) * (P[t[:, 2], 0] - P[t[:, 0], 0]))
    if abs(float(area.sum()) - 1.0) > 1e-9:
        raise ValidationError(f"live triangles cover area {float(area.sum())}, not 1")
    # locally Delaunay: the apex across each interior edge is not strictly
    # inside the circumcircle
    for rows, k, q in interior:
        tt = T4[rows, :3]
        ea = tt[:, k]
        eb = tt[:, (k + 1) % 3]
        qq = T4[q, :3]
        apex = np.where((qq != ea[:, None]) & (qq != eb[:, None]), qq, -1).max(1)
        s = incircle_sign(P[tt[:, 0]], P[tt[:, 1]], P[tt[:, 2]], P[apex])
        if (s > 0).any():
            i = np.flatnonzero(s > 0)[0]
            raise ValidationError(f"edge {int(ea[i])}-{int(eb[i])} of triangle {int(rows[i])} is not locally Delaunay")
    ang = min_angles(P, t)
    if check_quality and (ang < min_angle - angle_tol).any():
        i = np.flatnonzero(ang < min_angle - angle_tol)[0]
        raise ValidationError(f"triangle {int(live[i])} has an angle of {ang[i]:.6f} degrees, below {min_angle}")
    if check_encroachment:
        for k in range(3):
            bd = nb[:, k] < 0
            o = P[t[bd, (k + 2) % 3]]
            u = P[t[bd, k]] - o
            v = P[t[bd, (k + 1) % 3]] - o
            cosang = (u * v).sum(1) / (np.linalg.norm(u, axis=1) * np.linalg.norm(v, axis=1))
            if (cosang < np.cos(np.radians(90.0 + angle_tol))).any():
                raise ValidationError("a boundary edge is encroached (seen at more than 90 degrees)")
    used = np.zeros(P.shape[0], dtype=bool)
    used[t.ravel()] = True
    if not used.all():
        raise ValidationError(f"point {int(np.flatnonzero(~used)[0])} is not a vertex of any live triangle")
    if input_pts is not None:
        ip = np.asarray(input_pts, dtype=np.float64)
        if ip.shape[0] > P.shape[0] or not np.array_equal(P[:ip.shape[0]], ip):
            raise ValidationError("the input points are not kept under their indices")
    return {"triangles": int(live.size), "points": int(P.shape[0]), "min_angle": float(ang.min()),
            "area": float(area.sum())}
