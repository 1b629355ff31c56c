"""Helpers shared by the GPU parity tests: oracle set-up, error norms, sub-meshes."""
from __future__ import annotations

import numpy as np

from oracle.solver import Oracle
from paper_2107_06640_amd import inputs


def oracle_for(mesh, mats, order, **kw):
    rho, lam, mu = mats
    return Oracle(mesh.xyz, mesh.tet, mesh.face_kind, mesh.period, rho, lam, mu, order - 1, **kw)


def field_errors(got, ref, weight=None):
    """Relative L2 error per quantity of DOF arrays [E, B, 9].

    The basis is orthonormal, so the physical L2 norm is the coefficient norm
    weighted by |det J|. Fields whose reference norm is zero are measured
    against the largest field norm.
    """
    w = np.ones(got.shape[0]) if weight is None else weight
    err = np.sqrt(np.einsum("e,ebp->p", w, (got - ref) ** 2))
    nrm = np.sqrt(np.einsum("e,ebp->p", w, ref ** 2))
    den = np.where(nrm > 0, nrm, nrm.max())
    return err / den


def submesh(mesh, mats, ids):
    """Elements ``ids`` plus their face neighbours as a stand-alone mesh.

    Faces of the neighbour ring that lead outside the sub-mesh become
    absorbing; only the results of ``ids`` are meaningful after one global
    time step. Returns (sub mesh, sub materials, element map, index of ids).
    """
    from oracle.mesh import adjacency
    nb, _, _ = adjacency(mesh.tet, mesh.face_kind, mesh.xyz, mesh.period)
    ids = np.asarray(ids)
    ring = np.unique(np.concatenate([ids, nb[ids][nb[ids] >= 0]]))
    inside = np.zeros(mesh.n_elements, bool)
    inside[ring] = True
    fk = mesh.face_kind[ring].copy()
    nbr = nb[ring]
    for k in range(ring.size):
        for f in range(4):
            if fk[k, f] in (inputs.FACE_INTERIOR, inputs.FACE_PERIODIC) and not inside[nbr[k, f]]:
                fk[k, f] = inputs.FACE_ABSORBING
    verts, tet = np.unique(mesh.tet[ring], return_inverse=True)
    sub = inputs.Mesh(xyz=mesh.xyz[verts], tet=tet.reshape(-1, 4), face_kind=fk, period=mesh.period.copy())
    rho, lam, mu = mats
    pos = np.searchsorted(ring, ids)
    return sub, (rho[ring], lam[ring], mu[ring]), ring, pos


def element_errors(got, ref):
    """Per-element relative L2 error [E], the worse of the stress and the velocity block.

    Each block of an element is measured against its own norm (orthonormal
    basis: the coefficient norm is the L2 norm on the reference element), so
    an error confined to one element is not diluted by the others as in the
    per-field norm. Blocks whose own norm is below 1e-6 of the largest
    element norm of that block (zero shear stress in the water, for example)
    are measured against that floor instead.
    """
    out = np.zeros(got.shape[0])
    for sl in (slice(0, 6), slice(6, 9)):
        err = np.sqrt(((got[:, :, sl] - ref[:, :, sl]) ** 2).sum(axis=(1, 2)))
        nrm = np.sqrt((ref[:, :, sl] ** 2).sum(axis=(1, 2)))
        den = np.maximum(nrm, 1e-6 * nrm.max())
        out = np.maximum(out, err / den)
    return out
