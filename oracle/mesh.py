"""Geometry and face adjacency of a conforming tetrahedral mesh (oracle).

Test infrastructure only; see ``oracle/__init__``.

Each element is mapped from the reference tetrahedron by x = x0 + J xi with
J = [x1-x0, x2-x0, x3-x0] (Sec. 4.1: every element is mapped to the reference
element). Either orientation is accepted; volumes use |det J|. Face i is the
face opposite local vertex i and is parametrised by its vertices in ascending
local order: x = X_f0 + s (X_f1 - X_f0) + t (X_f2 - X_f0).

Interior faces (and the two sides of a dynamic-rupture fault face, kind 7)
are matched by their sorted global vertex triples; periodic faces by their
centroids modulo the box period.
"""
from __future__ import annotations

import numpy as np

REF_VERTS = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
FACE_VERTS = [tuple(v for v in range(4) if v != i) for i in range(4)]


class Geometry:
    def __init__(self, xyz, tet):
        self.xyz = np.asarray(xyz, dtype=np.float64)
        self.tet = np.asarray(tet, dtype=np.int64)
        X = self.xyz[self.tet]                      # [E, 4, 3]
        self.X = X
        self.x0 = X[:, 0, :]
        self.J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
        self.detJ = np.linalg.det(self.J)
        if np.any(np.abs(self.detJ) <= 1e-300):
            raise ValueError("degenerate element")
        self.absdet = np.abs(self.detJ)
        self.Jinv = np.linalg.inv(self.J)            # xi_d = Jinv[d, e] (x_e - x0_e)
        E = X.shape[0]
        self.normal = np.empty((E, 4, 3))
        self.area = np.empty((E, 4))
        for i, (a, b, c) in enumerate(FACE_VERTS):
            cr = np.cross(X[:, b] - X[:, a], X[:, c] - X[:, a])
            nrm = np.linalg.norm(cr, axis=1)
            nn = cr / nrm[:, None]
            # outward: pointing away from the opposite vertex i
            s = np.einsum("ei,ei->e", nn, X[:, i] - X[:, a])
            nn = np.where((s > 0)[:, None], -nn, nn)
            self.normal[:, i] = nn
            self.area[:, i] = 0.5 * nrm
        self.volume = self.absdet / 6.0
        # insphere diameter h = 6 V / sum of face areas (CFL length, Sec. 4.4)
        self.h = 6.0 * self.volume / self.area.sum(axis=1)

    def to_ref(self, elems, x):
        """Reference coordinates of physical points x[..., 3] in elements elems[...]."""
        return np.einsum("...de,...e->...d", self.Jinv[elems], x - self.x0[elems])

    def face_points(self, elems, faces, st):
        """Physical points of face-parameter points st[q, 2] on (elems, faces) -> [n, q, 3]."""
        fv = np.array(FACE_VERTS)[faces]            # [n, 3]
        X = self.X[elems]                           # [n, 4, 3]
        P0 = np.take_along_axis(X, fv[:, 0][:, None, None].repeat(3, 2), 1)[:, 0]
        P1 = np.take_along_axis(X, fv[:, 1][:, None, None].repeat(3, 2), 1)[:, 0]
        P2 = np.take_along_axis(X, fv[:, 2][:, None, None].repeat(3, 2), 1)[:, 0]
        return (P0[:, None, :] + st[None, :, 0:1] * (P1 - P0)[:, None, :]
                + st[None, :, 1:2] * (P2 - P0)[:, None, :])


def ref_face_points(face: int, st):
    """Reference-tetrahedron points of face-parameter points st[q, 2] on face ``face``."""
    a, b, c = FACE_VERTS[face]
    V = REF_VERTS
    return V[a] + st[:, 0:1] * (V[b] - V[a]) + st[:, 1:2] * (V[c] - V[a])


def adjacency(tet, face_kind, xyz, period):
    """Neighbour element, neighbour face and periodic shift of every face.

    Returns nb [E, 4] (-1 on physical boundaries), nbf [E, 4], shift [E, 4, 3]
    such that a point x on the face corresponds to x + shift in the neighbour.
    """
    tet = np.asarray(tet, dtype=np.int64)
    face_kind = np.asarray(face_kind)
    E = tet.shape[0]
    nb = -np.ones((E, 4), dtype=np.int64)
    nbf = -np.ones((E, 4), dtype=np.int64)
    shift = np.zeros((E, 4, 3))
    # interior and fault faces: sort the sorted vertex triples; a matched face is a run of two
    ee, ff = np.nonzero((face_kind == 0) | (face_kind == 7))
    if ee.size:
        keys = np.sort(tet[ee[:, None], np.array(FACE_VERTS)[ff]], axis=1)
        order = np.lexsort((keys[:, 2], keys[:, 1], keys[:, 0]))
        k = keys[order]
        pair = np.nonzero(np.all(k[1:] == k[:-1], axis=1))[0]
        if 2 * pair.size != ee.size or np.any(np.diff(pair) < 2):
            raise ValueError("interior faces without exactly one neighbour")
        a, b = order[pair], order[pair + 1]
        if np.any(face_kind[ee[a], ff[a]] != face_kind[ee[b], ff[b]]):
            raise ValueError("a fault face must meet a fault face")
        nb[ee[a], ff[a]], nbf[ee[a], ff[a]] = ee[b], ff[b]
        nb[ee[b], ff[b]], nbf[ee[b], ff[b]] = ee[a], ff[a]
    # periodic faces: match centroids modulo the period
    period = np.asarray(period, dtype=np.float64)
    per = [(int(e), int(i)) for e, i in np.argwhere(face_kind == 1)]
    if per:
        L = max(float(np.max(np.abs(xyz))), 1.0)
        cen = {}
        for (e, i) in per:
            c = xyz[[tet[e, v] for v in FACE_VERTS[i]]].mean(axis=0)
            red = c.copy()
            for ax in range(3):
                if period[ax] > 0:
                    red[ax] = np.mod(red[ax], period[ax])
                    if abs(red[ax] - period[ax]) < 1e-9 * L:
                        red[ax] = 0.0
            key = tuple(np.round(red / (1e-7 * L)).astype(np.int64))
            cen.setdefault(key, []).append((e, i, c))
        for key, lst in cen.items():
            if len(lst) != 2:
                raise ValueError("unmatched periodic face")
            (e1, i1, c1), (e2, i2, c2) = lst
            nb[e1, i1], nbf[e1, i1], shift[e1, i1] = e2, i2, c2 - c1
            nb[e2, i2], nbf[e2, i2], shift[e2, i2] = e1, i1, c1 - c2
    return nb, nbf, shift
