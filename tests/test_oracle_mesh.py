"""Pins of the oracle's face matching and LTS cluster assignment (CPU).

Face matching is checked against a brute-force search over all face pairs;
the cluster normalisation of Sec. 4.4 (neighbours differ by at most one
cluster) against its closed form: the largest labelling with c_K <= raw c_K
and c_K <= c_J + 1 for face neighbours is c_K = min_J (raw c_J + d(K, J)),
with d the face-graph distance.
"""
import numpy as np

from oracle.mesh import FACE_VERTS, adjacency
from oracle.solver import assign_clusters
from paper_2107_06640_amd import inputs


def brute_neighbours(tet, face_kind):
    E = tet.shape[0]
    nb = -np.ones((E, 4), dtype=np.int64)
    faces = {(e, i): frozenset(int(tet[e, v]) for v in FACE_VERTS[i]) for e in range(E) for i in range(4)}
    for (e, i), s in faces.items():
        if face_kind[e, i] != 0:
            continue
        hits = [(e2, i2) for (e2, i2), s2 in faces.items() if s2 == s and (e2, i2) != (e, i)]
        assert len(hits) == 1
        nb[e, i] = hits[0][0]
    return nb


def test_interior_matching_matches_brute_force():
    mesh = inputs.box_mesh(2, 3, 2, jitter=0.2, seed=1,
                           sides={"x-": "absorbing", "x+": "absorbing", "y-": "wall", "y+": "free",
                                  "z-": "absorbing", "z+": "absorbing"})
    nb, nbf, _ = adjacency(mesh.tet, mesh.face_kind, mesh.xyz, mesh.period)
    assert np.array_equal(nb, brute_neighbours(mesh.tet, mesh.face_kind))
    e, i = np.nonzero(nb >= 0)
    # the neighbour's neighbour across the matched face is the element itself
    assert np.array_equal(nb[nb[e, i], nbf[e, i]], e)


def test_unmatched_interior_face_is_rejected():
    mesh = inputs.box_mesh(1, 1, 1, sides={k: "absorbing" for k in ("x-", "x+", "y-", "y+", "z-", "z+")})
    fk = mesh.face_kind.copy()
    e, i = np.argwhere(fk == inputs.FACE_ABSORBING)[0]
    fk[e, i] = inputs.FACE_INTERIOR
    try:
        adjacency(mesh.tet, fk, mesh.xyz, mesh.period)
    except ValueError:
        return
    raise AssertionError("an interior face without a neighbour was accepted")


def graph_distance(nb):
    E = nb.shape[0]
    d = np.full((E, E), 10 ** 6, dtype=np.int64)
    np.fill_diagonal(d, 0)
    for e in range(E):
        for j in nb[e]:
            if j >= 0:
                d[e, j] = min(d[e, j], 1)
    for k in range(E):  # Floyd-Warshall
        d = np.minimum(d, d[:, k:k + 1] + d[k:k + 1, :])
    return d


def test_cluster_normalisation_closed_form():
    rng = np.random.default_rng(5)
    mesh = inputs.box_mesh(3, 3, 3, jitter=0.1, seed=2)
    nb, _, _ = adjacency(mesh.tet, mesh.face_kind, mesh.xyz, mesh.period)
    E = mesh.n_elements
    dt = 2.0 ** rng.uniform(0.0, 5.0, E)  # raw clusters 0..4, scattered
    for C in (1, 2, 3, 5):
        c, dt_min = assign_clusters(dt, nb, C)
        raw = np.clip(np.floor(np.log2(dt / dt.min())).astype(np.int64), 0, C - 1)
        want = (raw[None, :] + graph_distance(nb)).min(axis=1)
        assert dt_min == dt.min()
        assert np.array_equal(c, want)
        e, i = np.nonzero(nb >= 0)
        assert np.all(np.abs(c[e] - c[nb[e, i]]) <= 1)
