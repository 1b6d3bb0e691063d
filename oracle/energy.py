"""ctypes binding of the oracle's C energy/gradient (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ff_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

TERM_NAMES = ("stretch", "bend", "torsion", "coulomb", "vdw")


def build() -> str:
    """Compile the oracle's C source into ``liboracle.so`` (always rebuilds)."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-Wall", "-Wextra", "-Werror", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class _CSystem(C.Structure):
    _fields_ = [
        ("n_atoms", C.c_int32),
        ("q", C.POINTER(C.c_double)), ("sigma", C.POINTER(C.c_double)), ("eps", C.POINTER(C.c_double)),
        ("n_bonds", C.c_int32), ("bond", C.POINTER(C.c_int32)),
        ("bond_k", C.POINTER(C.c_double)), ("bond_r0", C.POINTER(C.c_double)),
        ("n_angles", C.c_int32), ("angle", C.POINTER(C.c_int32)),
        ("angle_k", C.POINTER(C.c_double)), ("angle_t0", C.POINTER(C.c_double)),
        ("n_dihedrals", C.c_int32), ("dihedral", C.POINTER(C.c_int32)),
        ("dihedral_v", C.POINTER(C.c_double)),
        ("coulomb_c", C.c_double),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        lib.oracle_energy_grad.argtypes = [C.POINTER(_CSystem), C.POINTER(C.c_double),
                                           C.POINTER(C.c_double), C.POINTER(C.c_double)]
        lib.oracle_energy_grad.restype = C.c_int
        lib.oracle_atom_gradients.argtypes = [C.POINTER(_CSystem), C.POINTER(C.c_double),
                                              C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_double)]
        lib.oracle_atom_gradients.restype = C.c_int
        lib.oracle_num_threads.restype = C.c_int
        lib.oracle_set_num_threads.argtypes = [C.c_int]
        lib.oracle_set_num_threads.restype = None
        lib.oracle_abs_pair_force.argtypes = [C.POINTER(_CSystem), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        lib.oracle_abs_pair_force.restype = C.c_int
        _lib = lib
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


class System:
    """Host copy of a system (dict as produced by ``synth``) for the oracle."""

    def __init__(self, d: dict):
        f64 = lambda k: np.ascontiguousarray(d[k], dtype=np.float64).ravel()  # noqa: E731
        i32 = lambda k: np.ascontiguousarray(d[k], dtype=np.int32).ravel()  # noqa: E731
        self.n = int(d["n_atoms"])
        self._keep = dict(q=f64("q"), sigma=f64("sigma"), eps=f64("eps"),
                          bond=i32("bonds"), bond_k=f64("bond_k"), bond_r0=f64("bond_r0"),
                          angle=i32("angles"), angle_k=f64("angle_k"), angle_t0=f64("angle_t0"),
                          dihedral=i32("dihedrals"), dihedral_v=f64("dihedral_v"))
        k = self._keep
        self.c = _CSystem(
            self.n, _dptr(k["q"]), _dptr(k["sigma"]), _dptr(k["eps"]),
            len(k["bond_k"]), _iptr(k["bond"]), _dptr(k["bond_k"]), _dptr(k["bond_r0"]),
            len(k["angle_k"]), _iptr(k["angle"]), _dptr(k["angle_k"]), _dptr(k["angle_t0"]),
            len(k["dihedral"]) // 4, _iptr(k["dihedral"]), _dptr(k["dihedral_v"]),
            float(d["coulomb_c"]))


def _as_system(s):
    return s if isinstance(s, System) else System(s)


def energy_terms(sys, x, want_grad: bool = True):
    """(terms dict, gradient [N][3] or None) at coordinates x [N][3]."""
    s = _as_system(sys)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(s.n, 3)
    terms = np.zeros(5)
    grad = np.zeros((s.n, 3)) if want_grad else None
    rc = _load().oracle_energy_grad(C.byref(s.c), _dptr(x), _dptr(terms),
                                    _dptr(grad) if want_grad else None)
    if rc != 0:
        raise ValueError(f"oracle_energy_grad failed ({rc})")
    return dict(zip(TERM_NAMES, terms.tolist())), grad


def energy_grad(sys, x, want_grad: bool = True):
    """Total energy (the terms summed in a fixed order) and gradient."""
    terms, grad = energy_terms(sys, x, want_grad)
    e = 0.0
    for k in TERM_NAMES:
        e += terms[k]
    return e, grad


def atom_gradients(sys, x, atoms):
    s = _as_system(sys)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(s.n, 3)
    atoms = np.ascontiguousarray(atoms, dtype=np.int32)
    out = np.zeros((len(atoms), 3))
    rc = _load().oracle_atom_gradients(C.byref(s.c), _dptr(x), _iptr(atoms), len(atoms), _dptr(out))
    if rc != 0:
        raise ValueError(f"oracle_atom_gradients failed ({rc})")
    return out


def abs_pair_force(sys, x):
    """Per atom, the sum over its non-excluded partners of |dE_ij/dr|: the
    scale against which rounding errors of a gradient component are stated
    (test tolerances only)."""
    s = _as_system(sys)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(s.n, 3)
    out = np.zeros(s.n)
    rc = _load().oracle_abs_pair_force(C.byref(s.c), _dptr(x), _dptr(out))
    if rc != 0:
        raise ValueError(f"oracle_abs_pair_force failed ({rc})")
    return out


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads used by later oracle calls from this thread."""
    _load().oracle_set_num_threads(int(n))


def energy_profile(system, x, t):
    """E(x + t u) for every t, u = -grad E(x)/|grad E(x)| the unit antigradient
    at x (u = 0 if the gradient vanishes): the one-dimensional slice the paper
    uses to show how non-convex the energy is near a start point (section 3)."""
    sysc = system if isinstance(system, System) else System(system)
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    _, g = energy_grad(sysc, x)
    nrm = float(np.linalg.norm(g))
    u = -g / nrm if nrm > 0.0 else np.zeros_like(g)
    return np.array([energy_grad(sysc, x + tk * u)[0] for tk in np.asarray(t, dtype=np.float64).ravel()])
