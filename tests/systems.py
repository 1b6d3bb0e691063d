"""Tiny hand-built systems for closed-form checks (no force-field arithmetic here)."""
import math

import numpy as np

from synth import COULOMB_KCAL


def make_system(x, q=None, sigma=None, eps=None, bonds=(), bond_k=(), bond_r0=(),
                angles=(), angle_k=(), angle_t0=(), dihedrals=(), dihedral_v=(),
                coulomb_c=COULOMB_KCAL):
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    n = x.shape[0]
    z = np.zeros(n)
    return {
        "n_atoms": n, "x": x,
        "q": z.copy() if q is None else np.asarray(q, float),
        "sigma": np.full(n, 3.0) if sigma is None else np.asarray(sigma, float),
        "eps": z.copy() if eps is None else np.asarray(eps, float),
        "bonds": np.asarray(bonds, np.int32).reshape(-1, 2),
        "bond_k": np.asarray(bond_k, float), "bond_r0": np.asarray(bond_r0, float),
        "angles": np.asarray(angles, np.int32).reshape(-1, 3),
        "angle_k": np.asarray(angle_k, float), "angle_t0": np.asarray(angle_t0, float),
        "dihedrals": np.asarray(dihedrals, np.int32).reshape(-1, 4),
        "dihedral_v": np.asarray(dihedral_v, float).reshape(-1, 4),
        "coulomb_c": float(coulomb_c),
    }


def dihedral_points(phi, bond=1.5):
    """Four atoms whose a-b-c-d dihedral is phi in the IUPAC sense (cis = 0):
    b at the origin, c on +z, a in the xz half-plane x > 0, d rotated by phi
    about the b->c axis."""
    return np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, bond],
                     [math.cos(phi), math.sin(phi), bond]])


def random_rotation(rng):
    a = rng.normal(size=(3, 3))
    qm, rm = np.linalg.qr(a)
    qm = qm @ np.diag(np.sign(np.diag(rm)))
    if np.linalg.det(qm) < 0:
        qm[:, 0] = -qm[:, 0]
    return qm


def torsion_chain(n, seed):
    """A clash-free chain (dihedrals within 1 rad of trans, no noise) with the
    generator's charges and LJ parameters plus random torsion terms, for
    gradient checks of every term."""
    from synth import chain_system
    from synth.chain import _backbone
    s = chain_system(n, seed)
    rng = np.random.default_rng(seed)
    dih = math.pi + rng.uniform(-1.0, 1.0, size=max(n - 3, 0))
    s["x"] = _backbone(n, dih)
    nd = max(n - 3, 0)
    s["dihedrals"] = np.stack([np.arange(nd) + k for k in range(4)], axis=1).astype(np.int32)
    s["dihedral_v"] = rng.uniform(-2.0, 2.0, size=(nd, 4))
    return s


def crosslinked_chain(n, seed):
    """torsion_chain(n, seed) plus cross-link bonds, and the angles around
    them, between atoms far apart in index: their 1-2 and 1-3 exclusions
    reach well beyond 64 atoms (in diagonal and in off-diagonal pair tiles
    for every block size)."""
    s = torsion_chain(n, seed)
    links = [(10, 100), (5, min(700, n - 100)), (n // 2, n - 50), (n - 200, n - 40)]
    bonds = [tuple(b) for b in s["bonds"]] + links
    angles = [tuple(a) for a in s["angles"]]
    for i, j in links:
        angles += [(i - 1, i, j), (i, j, j + 1)]
    s["bonds"] = np.asarray(bonds, np.int32)
    s["bond_k"] = np.concatenate([s["bond_k"], np.full(len(links), 300.0)])
    s["bond_r0"] = np.concatenate([s["bond_r0"], np.full(len(links), 1.5)])
    s["angles"] = np.asarray(angles, np.int32)
    s["angle_k"] = np.concatenate([s["angle_k"], np.full(2 * len(links), 50.0)])
    s["angle_t0"] = np.concatenate([s["angle_t0"], np.full(2 * len(links), math.radians(109.5))])
    return s
