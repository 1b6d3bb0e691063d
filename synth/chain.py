"""Seeded synthetic macromolecule-like chains.

The paper minimizes the force field of protein complexes with n ~ 10^4
variables (section 2) starting from poses with clashing atoms (section 3, the
huge start energies).  Those structures and their parameter tables are not
available, so every workload here is a synthetic chain with the same kind of
structure: a freely rotating backbone with fixed bond length and bond angle,
Gaussian positional noise (which creates the clashes), random partial charges
with zero net charge and random Lennard-Jones radii and well depths.

Recipe (all of it a reading; the paper has no synthetic workload):

1. PRNG: SplitMix64 (Steele, Lea, Flood 2014) seeded with ``seed``.  A uniform
   is ``(u >> 11) * 2**-53``; a normal is Box-Muller on ``(1 - u1, u2)`` using
   both outputs in order.
2. Draw order: ``N-3`` dihedrals U(-pi, pi); ``3N`` noise normals (atom-major
   x, y, z); ``N`` charges; ``N`` sigmas; ``N`` epsilons.
3. Backbone: atom 0 at the origin, atom 1 at (1.5, 0, 0), atom 2 in the xy
   plane at a 109.5 degree bond angle; atom k >= 3 placed by the natural
   extension reference frame construction (Parsons et al. 2005) from atoms
   k-3..k-1 with bond 1.5 A, angle 109.5 degrees and the k-th dihedral.
4. Optional compaction (before the noise): 200 gradient steps of a harmonic
   radius-of-gyration restraint ``k_rg * N / 2 * (Rg - Rt)^2`` towards the
   radius of a uniform globule of density 0.03 atoms/A^3, with the chain's
   local shape held by an elastic network of 1-2 and 1-3 distance springs.
5. Noise N(0, 0.3^2) A per coordinate, then the centroid is moved to 0.
6. Parameters: q ~ U(-0.5, 0.5) shifted to zero mean (e); sigma ~ U(3, 4) A;
   epsilon ~ U(0.05, 0.2) kcal/mol.
7. Topology: bonds (k, k+1) with K = 300 kcal/mol/A^2 and r0 = 1.5 A; angles
   (k, k+1, k+2) with the vertex in the middle, K = 50 kcal/mol/rad^2 and
   theta0 = 109.5 degrees; no dihedrals.

Units: A, radians, elementary charges, kcal/mol.  The Coulomb constant handed
out with every system is the paper's 1389.38757 (kJ mol^-1 A e^-2) divided by
4.184 kJ/kcal.
"""
from __future__ import annotations

import math

import numpy as np

GENERATOR_VERSION = 1

# Coulomb constant in kcal*A/(mol*e^2): the paper's value is in kJ/mol.
COULOMB_KCAL = 1389.38757 / 4.184

BOND_LENGTH = 1.5                          # A
BOND_ANGLE = math.radians(109.5)           # rad
BOND_K = 300.0                             # kcal/mol/A^2
ANGLE_K = 50.0                             # kcal/mol/rad^2
NOISE_SD = 0.3                             # A
GLOBULE_DENSITY = 0.03                     # atoms / A^3

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15
_MIX1 = 0xBF58476D1CE4E5B9
_MIX2 = 0x94D049BB133111EB


class SplitMix64:
    """Counter-based SplitMix64 stream, vectorised with numpy uint64."""

    def __init__(self, seed: int):
        self.state = int(seed) & _MASK

    def next_u64(self, n: int) -> np.ndarray:
        k = np.arange(1, n + 1, dtype=np.uint64)
        with np.errstate(over="ignore"):
            z = np.uint64(self.state) + k * np.uint64(_GAMMA)
            z = (z ^ (z >> np.uint64(30))) * np.uint64(_MIX1)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(_MIX2)
            z = z ^ (z >> np.uint64(31))
        self.state = (self.state + n * _GAMMA) & _MASK
        return z

    def uniform(self, n: int) -> np.ndarray:
        return (self.next_u64(n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)

    def normal(self, n: int) -> np.ndarray:
        m = (n + 1) // 2
        u = self.uniform(2 * m)
        u1, u2 = u[0::2], u[1::2]
        rad = np.sqrt(-2.0 * np.log1p(-u1))
        z = np.empty(2 * m)
        z[0::2] = rad * np.cos(2.0 * math.pi * u2)
        z[1::2] = rad * np.sin(2.0 * math.pi * u2)
        return z[:n]


def _place(a, b, c, bond, angle, torsion):
    """Natural extension reference frame: the atom bonded to ``c`` with bond
    length ``bond``, bond angle b-c-new ``angle`` and dihedral a-b-c-new
    ``torsion``."""
    bcx, bcy, bcz = c[0] - b[0], c[1] - b[1], c[2] - b[2]
    inv = 1.0 / math.sqrt(bcx * bcx + bcy * bcy + bcz * bcz)
    bcx, bcy, bcz = bcx * inv, bcy * inv, bcz * inv
    abx, aby, abz = b[0] - a[0], b[1] - a[1], b[2] - a[2]
    nx = aby * bcz - abz * bcy
    ny = abz * bcx - abx * bcz
    nz = abx * bcy - aby * bcx
    inv = 1.0 / math.sqrt(nx * nx + ny * ny + nz * nz)
    nx, ny, nz = nx * inv, ny * inv, nz * inv
    mx = ny * bcz - nz * bcy
    my = nz * bcx - nx * bcz
    mz = nx * bcy - ny * bcx
    d0 = -bond * math.cos(angle)
    d1 = bond * math.sin(angle) * math.cos(torsion)
    d2 = bond * math.sin(angle) * math.sin(torsion)
    return (c[0] + d0 * bcx + d1 * mx + d2 * nx,
            c[1] + d0 * bcy + d1 * my + d2 * ny,
            c[2] + d0 * bcz + d1 * mz + d2 * nz)


def _backbone(n: int, dihedrals: np.ndarray) -> np.ndarray:
    pts = [(0.0, 0.0, 0.0)]
    if n > 1:
        pts.append((BOND_LENGTH, 0.0, 0.0))
    if n > 2:
        pts.append((BOND_LENGTH - BOND_LENGTH * math.cos(BOND_ANGLE),
                    BOND_LENGTH * math.sin(BOND_ANGLE), 0.0))
    for k in range(3, n):
        pts.append(_place(pts[k - 3], pts[k - 2], pts[k - 1],
                          BOND_LENGTH, BOND_ANGLE, float(dihedrals[k - 3])))
    return np.asarray(pts, dtype=np.float64).reshape(n, 3)


def _compact(x: np.ndarray, steps: int = 200, k_rg: float = 50.0,
             k_net: float = 100.0, eta: float = 1e-3, substeps: int = 4) -> np.ndarray:
    """Pull the chain towards a globule: ``steps`` gradient steps on a harmonic
    radius-of-gyration restraint, each followed by ``substeps`` relaxation
    steps of an elastic network of 1-2 and 1-3 distance springs that keeps
    the local chain shape (bond length and the 1-3 span of the bond angle)."""
    n = x.shape[0]
    x = x.copy()
    r_target = math.sqrt(3.0 / 5.0) * (3.0 * n / (4.0 * math.pi * GLOBULE_DENSITY)) ** (1.0 / 3.0)
    span13 = 2.0 * BOND_LENGTH * math.sin(BOND_ANGLE / 2.0)
    for _ in range(steps):
        c = x.mean(axis=0)
        d = x - c
        rg = math.sqrt(float((d * d).sum()) / n)
        if rg > r_target:
            x -= eta * k_rg * (rg - r_target) / rg * d
        for _ in range(substeps):
            grad = np.zeros_like(x)
            for off, rest in ((1, BOND_LENGTH), (2, span13)):
                v = x[off:] - x[:-off]
                r = np.sqrt((v * v).sum(axis=1, keepdims=True))
                f = k_net * (r - rest) / r * v
                grad[off:] += f
                grad[:-off] -= f
            x -= eta * grad
    return x


def chain_system(n_atoms: int, seed: int, compact: bool = False) -> dict:
    """One synthetic chain system; arrays are numpy (float64 / int32)."""
    n = int(n_atoms)
    if n < 1:
        raise ValueError("n_atoms must be >= 1")
    rng = SplitMix64(seed)
    dihedrals = rng.uniform(max(n - 3, 0)) * (2.0 * math.pi) - math.pi
    noise = rng.normal(3 * n).reshape(n, 3) * NOISE_SD
    q = rng.uniform(n) - 0.5
    q -= q.mean()
    sigma = 3.0 + rng.uniform(n)
    eps = 0.05 + 0.15 * rng.uniform(n)

    x = _backbone(n, dihedrals)
    if compact and n > 2:
        x = _compact(x)
    x = x + noise
    x -= x.mean(axis=0)

    nb = max(n - 1, 0)
    na = max(n - 2, 0)
    bonds = np.stack([np.arange(nb), np.arange(1, nb + 1)], axis=1).astype(np.int32)
    angles = np.stack([np.arange(na), np.arange(1, na + 1), np.arange(2, na + 2)],
                      axis=1).astype(np.int32)
    return {
        "n_atoms": n,
        "x": np.ascontiguousarray(x),
        "q": q, "sigma": sigma, "eps": eps,
        "bonds": bonds.reshape(nb, 2),
        "bond_k": np.full(nb, BOND_K), "bond_r0": np.full(nb, BOND_LENGTH),
        "angles": angles.reshape(na, 3),
        "angle_k": np.full(na, ANGLE_K), "angle_t0": np.full(na, BOND_ANGLE),
        "dihedrals": np.zeros((0, 4), dtype=np.int32),
        "dihedral_v": np.zeros((0, 4)),
        "coulomb_c": COULOMB_KCAL,
        "seed": int(seed),
        "generator_version": GENERATOR_VERSION,
    }


# The named workloads: (atoms, seed, compacted).
CONFIGS = {
    "chain512": (512, 0, False),
    "chain10k": (10_000, 1, False),
    "chain50k": (50_000, 2, True),
}


def config_system(name: str) -> dict:
    n, seed, compact = CONFIGS[name]
    return chain_system(n, seed, compact)


def batch_sizes(count: int = 256, lo: int = 200, hi: int = 4000, seed: int = 99) -> list:
    """Chain sizes log-uniform in [lo, hi] for a batch of independent chains
    (chain b uses seed 100 + b)."""
    u = SplitMix64(seed).uniform(count)
    return [int(round(math.exp(math.log(lo) + t * (math.log(hi) - math.log(lo))))) for t in u]
