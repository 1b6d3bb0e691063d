"""Iterate-parity cases of the FP64 minimizer and their gates, shared by the
GPU parity tests (tests/test_gpu_minimize.py) and the oracle's own
sensitivity test (tests/test_oracle_sensitivity.py), so that every gate the
GPU is held to is backed by a measurement anyone can rerun on the CPU.

A case names a system, a method with its parameters and a number of
iterations.  Its gates are windows of iterations: the energies after
iterations [previous end, end) must agree with the oracle's to the window's
relative tolerance; the accepted steps agree to 1e-6 over the first window;
evaluation counts (the line-search decisions) agree over all compared
iterations; `x_tol` bounds the final coordinates (A) where given.

Why these numbers: two correct FP64 implementations differ by the rounding
of their sums (a few units in the last place), and the minimization
amplifies such a difference at a rate that depends on the method and the
system.  The sensitivity test perturbs the oracle's E and grad E by that
much (PERTURB_E relative, PERTURB_G of |grad E|_inf per component, random
signs) and checks that its own trajectory stays inside every gate with a
margin of 10, and that a window looser than 1e-9 is needed (the perturbed
oracle leaves 1e-9 there)."""
from __future__ import annotations

import numpy as np

PERTURB_E = 2.0 ** -48        # relative, on E
PERTURB_G = 2.0 ** -50        # times |grad E|_inf, on each gradient component
SEEDS = (1, 2, 3)
MARGIN = 10.0


def _system(name):
    from synth import chain_system, config_system
    from tests.systems import torsion_chain
    if name == "chain512":
        return config_system("chain512")
    if name == "torsion200":
        s = torsion_chain(200, 5)
        s["x"] = s["x"] + np.random.default_rng(2).normal(scale=0.2, size=s["x"].shape)
        return s
    if name == "torsion300":
        return torsion_chain(300, 7)
    if name == "crosslinked600":
        from tests.systems import crosslinked_chain
        return crosslinked_chain(600, 8)
    kind, seed = name.split("_")
    return chain_system(int(kind[5:]), int(seed))


# name: (system, method, keyword arguments shared by oracle.MinParams and
#        Context.minimize, iterations, windows [(end, rtol)], x_tol or None)
CASES = {
    "chain512-lbfgs": ("chain512", "lbfgs", {}, 50, [(50, 1e-9)], 1e-8),
    "chain512-gd": ("chain512", "gd", {}, 50, [(30, 1e-9), (50, 1e-7)], 1e-6),
    "chain512-cg": ("chain512", "cg", {}, 50, [(30, 1e-9), (50, 1e-6)], 1e-5),
    "chain512-fgm": ("chain512", "fgm", {}, 30, [(10, 1e-9), (20, 1e-8), (30, 1e-6)], None),
    "chain512-fgm-restart": ("chain512", "fgm", {"fgm_restart": True}, 30, [(10, 1e-9), (20, 1e-8), (30, 1e-6)],
                             None),
    "torsion200-lbfgs-m5": ("torsion200", "lbfgs", {"m": 5}, 40, [(40, 1e-9)], None),
    "torsion200-cg": ("torsion200", "cg", {}, 40, [(40, 1e-9)], None),
    "chain400_21-lbfgs-K3": ("chain400_21", "lbfgs", {"ls_K": 3}, 25, [(20, 1e-9), (25, 1e-8)], None),
    "chain400_21-lbfgs-K4": ("chain400_21", "lbfgs", {"ls_K": 4}, 25, [(25, 1e-9)], None),
    "chain350_22-lbfgs-lsh": ("chain350_22", "lbfgs", {"linesearch": 1}, 30, [(10, 1e-9), (20, 1e-7), (30, 1e-6)],
                              None),
    "chain350_22-fgm-lspar": ("chain350_22", "fgm", {"linesearch": 0}, 30, [(20, 1e-9), (30, 1e-8)], None),
    "chain260_24-lbfgs-g0off-K2": ("chain260_24", "lbfgs", {"ls_K": 2, "ls_par_g0": False}, 25, [(25, 1e-9)], None),
    "chain260_24-lbfgs-g0off-K3": ("chain260_24", "lbfgs", {"ls_K": 3, "ls_par_g0": False}, 25, [(25, 1e-9)], None),
    "torsion300-hb": ("torsion300", "hb", {"hb_alpha": 1e-3, "hb_beta": 0.8}, 100, [(100, 1e-9)], None),
    "chain512-ogm": ("chain512", "ogm", {}, 50, [(10, 1e-9), (50, 1e-8)], None),
    "torsion300-ogm": ("torsion300", "ogm", {}, 50, [(10, 1e-8), (20, 1e-6), (50, 1e-5)], None),
    "chain300_23-cg-fr": ("chain300_23", "cg", {"cg_beta": "fr"}, 30, [(30, 1e-9)], None),
    "chain300_23-cg-hs": ("chain300_23", "cg", {"cg_beta": "hs"}, 30, [(30, 1e-9)], None),
    "chain300_23-cg-prp+": ("chain300_23", "cg", {"cg_beta": "prp+"}, 30, [(20, 1e-9), (30, 1e-8)], None),
    "chain300_23-cg-cd": ("chain300_23", "cg", {"cg_beta": "cd"}, 30, [(30, 1e-9)], None),
    "chain300_23-cg-ls": ("chain300_23", "cg", {"cg_beta": "ls"}, 30, [(30, 1e-9)], None),
    "chain300_23-cg-dy": ("chain300_23", "cg", {"cg_beta": "dy"}, 30, [(30, 1e-9)], None),
    # exclusions more than 64 atoms apart (cross-links and the angles around them)
    "crosslinked600-lbfgs": ("crosslinked600", "lbfgs", {}, 20, [(5, 1e-9), (12, 1e-8), (15, 1e-7), (20, 1e-5)],
                             None),
}


def system(case: str) -> dict:
    return _system(CASES[case][0])


def oracle_params(case: str):
    import oracle
    _, method, kw, n_iter, _, _ = CASES[case]
    kw = dict(kw)
    if "cg_beta" in kw:
        kw["cg_beta"] = {"prp": oracle.CG_PRP, "fr": oracle.CG_FR, "hs": oracle.CG_HS, "prp+": oracle.CG_PRP_PLUS,
                         "cd": oracle.CG_CD, "ls": oracle.CG_LS, "dy": oracle.CG_DY}[kw["cg_beta"]]
    m = {"gd": oracle.GD, "fgm": oracle.FGM, "cg": oracle.CG, "lbfgs": oracle.LBFGS, "hb": oracle.HB,
         "ogm": oracle.OGM}[method]
    return oracle.MinParams(method=m, max_iter=n_iter, **kw)


def gpu_kwargs(case: str) -> dict:
    _, method, kw, n_iter, _, _ = CASES[case]
    return dict(kw, method=method, max_iter=n_iter, m=max(kw.get("m", 10), 1))


def window_errors(f_ref, f, windows):
    """Largest relative energy difference in each window."""
    out, start = [], 0
    for end, _ in windows:
        a, b = np.asarray(f_ref[start:end]), np.asarray(f[start:end])
        out.append(float(np.max(np.abs(b - a) / np.abs(a))) if len(a) else 0.0)
        start = end
    return out
