"""Seeded synthetic inputs shared by the library tests, the benchmark and the oracle.

This module holds no arithmetic of the numerical method: it only builds meshes
(vertex coordinates, tetrahedra, boundary tags), per-element material
parameters and random modal coefficients. Both the CPU oracle and the GPU path
take these as *inputs*.

Workload shapes follow the paper's setting (Sec. 3 and Sec. 6): a layered
elastic solid below an acoustic water layer whose top is the sea surface z = 0
(gravity free-surface boundary, Sec. 4.3), meshed by conforming tetrahedra
(Sec. 4.1). The paper's own meshes (Palu, ASCETE Scenario A) are not available,
so these boxes stand in for them.

Face-kind codes (face i of a tetrahedron is the face opposite its local vertex i):
    0 interior, 1 periodic, 2 gravity free surface, 3 absorbing (zero ghost),
    4 rigid wall, 5 traction-free surface (g = 0), 6 prescribed velocity
    (the uplift history of the seafloor forcing).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

FACE_INTERIOR = 0
FACE_PERIODIC = 1
FACE_GRAVITY = 2
FACE_ABSORBING = 3
FACE_WALL = 4
FACE_FREE = 5
FACE_VELOCITY = 6
FACE_FAULT = 7

_KIND = {
    "periodic": FACE_PERIODIC,
    "gravity": FACE_GRAVITY,
    "absorbing": FACE_ABSORBING,
    "wall": FACE_WALL,
    "free": FACE_FREE,
    "velocity": FACE_VELOCITY,
}

# Rock and water parameters of the paper's coupled setting (Sec. 3); the rock
# values are those used for the synthetic workloads.
ROCK = dict(rho=2700.0, cp=6000.0, cs=3464.0)
WATER = dict(rho=1000.0, cp=1500.0, cs=0.0)


def lame(rho: float, cp: float, cs: float) -> tuple[float, float, float]:
    """(rho, lambda, mu) from density and wave speeds."""
    mu = rho * cs * cs
    lam = rho * cp * cp - 2.0 * mu
    return rho, lam, mu


@dataclass
class Mesh:
    xyz: np.ndarray          # [n_vertices, 3] float64
    tet: np.ndarray          # [n_elements, 4] int64
    face_kind: np.ndarray    # [n_elements, 4] int8
    period: np.ndarray       # [3] float64, 0 = not periodic
    info: dict = field(default_factory=dict)

    @property
    def n_elements(self) -> int:
        return int(self.tet.shape[0])


def kuhn_tets() -> list[tuple[int, int, int, int]]:
    """The 6 tetrahedra of a unit cube sharing its main diagonal.

    Cube corners are numbered by bits (i + 2 j + 4 k). Each tetrahedron is the
    monotone path 0 -> e_a -> e_a + e_b -> 7 for a permutation (a, b, c) of
    the axes. Half of them are negatively oriented on purpose: the library and
    the oracle must accept either orientation.
    """
    out = []
    for perm in itertools.permutations(range(3)):
        c0 = 0
        c1 = c0 | (1 << perm[0])
        c2 = c1 | (1 << perm[1])
        c3 = 7
        out.append((c0, c1, c2, c3))
    return out


def box_mesh(nx: int, ny: int, nz: int, *, x_nodes=None, y_nodes=None, z_nodes=None,
             lengths=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0),
             sides=None, jitter: float = 0.0, seed: int = 0) -> Mesh:
    """Structured box of nx*ny*nz cubes, each split into 6 Kuhn tetrahedra.

    ``sides`` maps "x-", "x+", "y-", "y+", "z-", "z+" to one of "periodic",
    "gravity", "absorbing", "wall", "free" (default: all periodic). Opposite
    sides must both be periodic or both not. ``*_nodes`` override uniform
    node coordinates along an axis. ``jitter`` moves strictly interior
    vertices by a seeded uniform offset of +-jitter times the local spacing.
    """
    sides = dict(sides or {})
    for s in ("x-", "x+", "y-", "y+", "z-", "z+"):
        sides.setdefault(s, "periodic")
    for ax in "xyz":
        if (sides[ax + "-"] == "periodic") != (sides[ax + "+"] == "periodic"):
            raise ValueError(f"axis {ax}: periodic must be set on both sides")

    def nodes(n, given, length, o):
        if given is not None:
            g = np.asarray(given, dtype=np.float64)
            if g.shape != (n + 1,):
                raise ValueError("node array has the wrong length")
            return g
        return o + length * np.arange(n + 1) / n

    xs = nodes(nx, x_nodes, lengths[0], origin[0])
    ys = nodes(ny, y_nodes, lengths[1], origin[1])
    zs = nodes(nz, z_nodes, lengths[2], origin[2])

    X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).copy()

    def vid(i, j, k):
        return (i * (ny + 1) + j) * (nz + 1) + k

    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        hx = np.diff(xs).min()
        hy = np.diff(ys).min()
        hz_all = np.diff(zs)
        I, J, K = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
        inner = ((I > 0) & (I < nx) & (J > 0) & (J < ny) & (K > 0) & (K < nz)).ravel()
        kk = K.ravel()
        hz_loc = np.minimum(hz_all[np.clip(kk - 1, 0, nz - 1)], hz_all[np.clip(kk, 0, nz - 1)])
        off = rng.uniform(-jitter, jitter, size=(xyz.shape[0], 3))
        off[:, 0] *= hx
        off[:, 1] *= hy
        off[:, 2] *= hz_loc
        off[~inner] = 0.0
        xyz = xyz + off

    corners = np.array([[c & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)])
    tets_local = kuhn_tets()
    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    n_cells = ci.size
    tet = np.empty((n_cells, 6, 4), dtype=np.int64)
    corner_xyz_idx = np.empty((n_cells, 8), dtype=np.int64)
    for c in range(8):
        corner_xyz_idx[:, c] = vid(ci + corners[c, 0], cj + corners[c, 1], ck + corners[c, 2])
    for t, loc in enumerate(tets_local):
        for v in range(4):
            tet[:, t, v] = corner_xyz_idx[:, loc[v]]
    tet = tet.reshape(-1, 4)

    # Boundary tags: a face lies on a box side when all its vertices do.
    face_kind = np.zeros((tet.shape[0], 4), dtype=np.int8)
    cell_of = np.repeat(np.arange(n_cells), 6)
    loc_of = np.tile(np.arange(6), n_cells)
    for f in range(4):
        others = [v for v in range(4) if v != f]
        cc = np.array([[tets_local[t][v] for v in others] for t in range(6)])  # [6, 3] corner ids
        cb = corners[cc[loc_of]]  # [E, 3, 3] corner bits
        cell_idx = np.stack([ci[cell_of], cj[cell_of], ck[cell_of]], axis=1)
        ncell = (nx, ny, nz)
        for ax, name in enumerate("xyz"):
            on_lo = np.all(cb[:, :, ax] == 0, axis=1) & (cell_idx[:, ax] == 0)
            on_hi = np.all(cb[:, :, ax] == 1, axis=1) & (cell_idx[:, ax] == ncell[ax] - 1)
            face_kind[on_lo, f] = _KIND[sides[name + "-"]]
            face_kind[on_hi, f] = _KIND[sides[name + "+"]]

    period = np.zeros(3)
    for ax, (name, arr) in enumerate(zip("xyz", (xs, ys, zs))):
        if sides[name + "-"] == "periodic":
            period[ax] = arr[-1] - arr[0]
    return Mesh(xyz=xyz, tet=tet, face_kind=face_kind, period=period,
                info=dict(nx=nx, ny=ny, nz=nz, sides=sides, jitter=jitter, seed=seed))


def centroids(mesh: Mesh) -> np.ndarray:
    return mesh.xyz[mesh.tet].mean(axis=1)


def layered_materials(mesh: Mesh, z_seafloor: float, rock=ROCK, water=WATER):
    """Per-element (rho, lambda, mu): water above ``z_seafloor``, rock below."""
    zc = centroids(mesh)[:, 2]
    wet = zc > z_seafloor
    rr, lr, mr = lame(**rock)
    rw, lw, mw = lame(**water)
    rho = np.where(wet, rw, rr)
    lam = np.where(wet, lw, lr)
    mu = np.where(wet, mw, mr)
    return rho.astype(np.float64), lam.astype(np.float64), mu.astype(np.float64)


# A soft sedimentary layer between the water and the rock: the elastic-elastic
# faces between it and the rock have different S impedances on both sides.
SEDIMENT = dict(rho=2000.0, cp=2500.0, cs=1100.0)


def three_layer_materials(mesh: Mesh, z_seafloor: float, z_sediment: float, rock=ROCK, sediment=SEDIMENT,
                          water=WATER):
    """Per-element (rho, lambda, mu): water above ``z_seafloor``, sediment down to ``z_sediment``, rock below."""
    zc = centroids(mesh)[:, 2]
    layer = np.where(zc > z_seafloor, 0, np.where(zc > z_sediment, 1, 2))
    tab = np.array([lame(**water), lame(**sediment), lame(**rock)])
    return tuple(np.ascontiguousarray(tab[layer, i]) for i in range(3))


def uniform_materials(mesh: Mesh, rho: float, cp: float, cs: float):
    r, l, m = lame(rho, cp, cs)
    E = mesh.n_elements
    return np.full(E, r), np.full(E, l), np.full(E, m)


def random_dofs(n_elements: int, n_basis: int, seed: int = 0, *, stress_scale=1.0e6,
                velocity_scale=1.0, decay=0.5, acoustic=None) -> np.ndarray:
    """Random modal coefficients [E][B][9] with magnitudes decaying by degree.

    ``acoustic`` (bool array, optional) marks elements whose stress must be
    isotropic (sigma = -p I, zero shear) as in the paper's acoustic embedding.
    The degree of basis function l is recovered from the dimension counts
    C(d+3, 3) only (no basis arithmetic).
    """
    rng = np.random.default_rng(seed)
    q = rng.standard_normal((n_elements, n_basis, 9))
    deg = np.zeros(n_basis)
    d, cnt = 0, 0
    for l in range(n_basis):
        while l >= (d + 1) * (d + 2) * (d + 3) // 6:
            d += 1
        deg[l] = d
    q *= (decay ** deg)[None, :, None]
    q[:, :, :6] *= stress_scale
    q[:, :, 6:] *= velocity_scale
    if acoustic is not None:
        a = np.asarray(acoustic, dtype=bool)
        p = q[a, :, 0].copy()
        q[a, :, 0] = p
        q[a, :, 1] = p
        q[a, :, 2] = p
        q[a, :, 3:6] = 0.0
    return q


def pulse_dofs(mesh: Mesh, n_basis: int, z_center: float, cell: float, seed: int = 0,
               n_pulses: int = 3) -> np.ndarray:
    """Seeded sum of Gaussian v_z pulses centred at depth ``z_center``, one value per element.

    Widths 2-5 cells, amplitudes U[0.5, 1.5] m/s, centres at least two widths
    from the lateral edges. The pulse is sampled at each element's centroid
    and carried by the constant basis function only (its value on the unit-
    norm reference basis is sqrt(6), the reference volume being 1/6), so the
    initial state is piecewise constant.
    """
    rng = np.random.default_rng(seed)
    c = centroids(mesh)
    lo, hi = mesh.xyz.min(axis=0), mesh.xyz.max(axis=0)
    v = np.zeros(mesh.n_elements)
    for _ in range(n_pulses):
        w = rng.uniform(2.0, 5.0) * cell
        a = rng.uniform(0.5, 1.5)
        m = np.minimum(2 * w, 0.45 * (hi[:2] - lo[:2]))
        cx = rng.uniform(lo[0] + m[0], hi[0] - m[0])
        cy = rng.uniform(lo[1] + m[1], hi[1] - m[1])
        r2 = (c[:, 0] - cx) ** 2 + (c[:, 1] - cy) ** 2 + (c[:, 2] - z_center) ** 2
        v += a * np.exp(-r2 / (2 * w * w))
    q = np.zeros((mesh.n_elements, n_basis, 9))
    q[:, 0, 8] = v / np.sqrt(6.0)
    return q


def uplift_sources(seed: int, lx: float, ly: float, n_min: int = 1, n_max: int = 4):
    """Seeded seafloor uplift: 1-4 Gaussians (amplitude 0.5-3 m, width 2-6 km, rise time 5-30 s).

    Returns a list of (amplitude, x, y, width, rise time); centres keep one
    width from the lateral edges when the box allows it.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(int(rng.integers(n_min, n_max + 1))):
        a = rng.uniform(0.5, 3.0)
        w = rng.uniform(2000.0, 6000.0)
        mx, my = min(w, 0.45 * lx), min(w, 0.45 * ly)
        out.append((a, rng.uniform(mx, lx - mx), rng.uniform(my, ly - my), w, rng.uniform(5.0, 30.0)))
    return out


def uplift_rate(x, y, sources):
    """Mean uplift rate sum_j A_j/T_j exp(-r_j^2 / (2 w_j^2)) at points (x, y), m/s."""
    v = np.zeros(np.broadcast(x, y).shape)
    for a, cx, cy, w, tr in sources:
        v = v + (a / tr) * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * w * w))
    return v


def uplift_dofs(mesh: Mesh, n_basis: int, z_floor: float, sources, thickness: float, elastic) -> np.ndarray:
    """Initial v_z of the rock under the seafloor: the uplift rate times exp(-(z - z_floor)^2 / (2 h^2)).

    Piecewise constant (constant basis function only, value sqrt(6) on the
    unit-norm reference basis); zero in the water.
    """
    c = centroids(mesh)
    v = uplift_rate(c[:, 0], c[:, 1], sources) * np.exp(-((c[:, 2] - z_floor) ** 2) / (2 * thickness ** 2))
    q = np.zeros((mesh.n_elements, n_basis, 9))
    q[:, 0, 8] = np.where(np.asarray(elastic, bool), v, 0.0) / np.sqrt(6.0)
    return q


# ---------------------------------------------------------------------------
# Workload builders. Sizes are those of the benchmark configurations; the
# functions take a ``scale`` to build smaller meshes of the same shape.

def cfg1_mesh(n: int = 6, seed: int = 0) -> Mesh:
    """Unit cube, n^3 cubes x 6 tets, periodic on all sides."""
    m = box_mesh(n, n, n, lengths=(1.0, 1.0, 1.0))
    m.info.update(name="cfg1-plane-wave", seed=seed)
    return m


def coupled_box(nx: int, ny: int, nz: int, *, cell: float, water_layers: int,
                z_nodes=None, jitter: float = 0.0, seed: int = 0, bottom="absorbing"):
    """Ocean-over-solid box: lateral periodic, bottom ``bottom``, top gravity (z = 0)."""
    if z_nodes is None:
        z_nodes = -cell * (nz - np.arange(nz + 1, dtype=np.float64))
    z_nodes = np.asarray(z_nodes, dtype=np.float64)
    m = box_mesh(nx, ny, nz, lengths=(nx * cell, ny * cell, 0.0), z_nodes=z_nodes,
                 sides={"z-": bottom, "z+": "gravity"}, jitter=jitter, seed=seed)
    z_floor = z_nodes[nz - water_layers]
    rho, lam, mu = layered_materials(m, z_floor)
    m.info.update(z_seafloor=float(z_floor), cell=cell, water_layers=water_layers)
    return m, (rho, lam, mu)


def fault_box(nx: int, ny: int, nz: int, *, cell: float, k_fault: int, jitter: float = 0.0, seed: int = 0,
              rock=ROCK, z_nodes=None):
    """All-rock box with a horizontal dynamic-rupture fault.

    Lateral sides periodic, top and bottom absorbing; the interior faces whose
    three vertices lie on vertex layer ``k_fault`` (0 < k_fault < nz) are
    fault faces (kind 7), seen from both sides. ``z_nodes`` (default: layers
    of thickness ``cell`` with the fault at z = 0) sets the vertex layers.
    The fault is the plane z = z_nodes[k_fault] unless ``jitter`` moves its
    vertices.
    """
    if not 0 < k_fault < nz:
        raise ValueError("the fault must be an interior vertex layer")
    if z_nodes is None:
        z_nodes = cell * (np.arange(nz + 1, dtype=np.float64) - k_fault)
    z_nodes = np.asarray(z_nodes, dtype=np.float64)
    m = box_mesh(nx, ny, nz, lengths=(nx * cell, ny * cell, 0.0), z_nodes=z_nodes,
                 sides={"z-": "absorbing", "z+": "absorbing"}, jitter=jitter, seed=seed)
    k_of = m.tet % (nz + 1)                         # vertex layer of each element vertex
    for f in range(4):
        others = [v for v in range(4) if v != f]
        on = np.all(k_of[:, others] == k_fault, axis=1) & (m.face_kind[:, f] == FACE_INTERIOR)
        m.face_kind[on, f] = FACE_FAULT
    rho, lam, mu = uniform_materials(m, rock["rho"], rock["cp"], rock["cs"])
    m.info.update(cell=cell, k_fault=k_fault, z_fault=float(z_nodes[k_fault]))
    return m, (rho, lam, mu)


def cfg2(scale: int = 1, seed: int = 0):
    """40x40x20 cubes x 6 tets (192 000 elements), 500 m cells, top 5 layers water."""
    nx, ny, nz = 40 // scale, 40 // scale, 20 // scale
    m, mat = coupled_box(nx, ny, nz, cell=500.0, water_layers=max(1, nz // 4), seed=seed)
    m.info.update(name="cfg2-coupled-gravity")
    return m, mat


def cfg5(scale: int = 1, seed: int = 0, bottom: str = "absorbing"):
    """24x24x12 cubes of 1 km x 6 tets (41 472 elements), top 3 layers water (surrogate data).

    bottom="velocity" makes the bottom of the solid the prescribed-velocity
    boundary that the uplift history drives.
    """
    nx, ny, nz = 24 // scale, 24 // scale, 12 // scale
    m, mat = coupled_box(nx, ny, nz, cell=1000.0, water_layers=max(1, nz // 4), seed=seed, bottom=bottom)
    m.info.update(name="cfg5-surrogate")
    return m, mat


def graded_z_nodes(nz: int, h_bottom: float, h_top: float) -> np.ndarray:
    """Layer interfaces from the bottom to z = 0, thickness graded geometrically."""
    r = (h_top / h_bottom) ** (1.0 / max(nz - 1, 1))
    th = h_bottom * r ** np.arange(nz)
    z = np.concatenate([[0.0], np.cumsum(th[::-1])])  # from the top down
    return -z[::-1]


def cfg3(scale: int = 1, seed: int = 0, jitter: float = 0.2):
    """Graded, jittered ocean-over-solid box: 72x72x64 cubes x 6 (about 2.0 M tets).

    Horizontal 500 m cells; vertical layers graded geometrically from 500 m at
    the bottom to 125 m at the sea surface; top quarter of the depth is water.
    """
    nx, ny, nz = 72 // scale, 72 // scale, 64 // scale
    zn = graded_z_nodes(nz, 500.0, 125.0)
    depth = -zn[0]
    k_floor = int(np.searchsorted(zn, -0.25 * depth))
    water_layers = nz - k_floor
    m, mat = coupled_box(nx, ny, nz, cell=500.0, water_layers=water_layers, z_nodes=zn,
                         jitter=jitter, seed=seed)
    m.info.update(name="cfg3-graded-lts")
    return m, mat
