"""How far two correct FP64 implementations of the minimizers can drift
apart, measured on the oracle itself, for every iterate-parity case the GPU
is held to (tests/parity_cases.py).

The oracle's E and grad E are perturbed by a few units in the last place
(PERTURB_E relative on E, PERTURB_G of |grad E|_inf on each gradient
component, random signs, three seeds): the size of the rounding difference
between two summation orders of these sums.  The perturbed run must take
the same line-search decisions, and its energies must stay within every
gate window with a margin of MARGIN; a window looser than 1e-9 must be
needed, i.e. the perturbed run must leave 1e-9/MARGIN there, or the window
could be tightened."""
import numpy as np
import pytest

import oracle
from tests import parity_cases as P


def _perturbed(fg, seed):
    rng = np.random.default_rng(seed)

    def f(v):
        e, g = fg(v)
        g = np.asarray(g, dtype=np.float64).ravel()
        e = e + P.PERTURB_E * abs(e) * rng.choice([-1.0, 1.0])
        return e, g + rng.choice([-1.0, 1.0], size=g.size) * (P.PERTURB_G * np.abs(g).max())

    return f


@pytest.mark.parametrize("case", sorted(P.CASES))
def test_gates_hold_the_oracle_against_its_own_rounding(case):
    s = P.system(case)
    sysc = oracle.System(s)

    def fg(v):
        return oracle.energy_grad(sysc, v.reshape(-1, 3))

    p = P.oracle_params(case)
    ref = oracle.minimize(fg, s["x"].ravel(), p)
    _, _, _, n_iter, windows, x_tol = P.CASES[case]
    assert ref.iters == n_iter
    f_ref = [t[0] for t in ref.trace]
    worst = [0.0] * len(windows)
    for seed in P.SEEDS:
        r = oracle.minimize(_perturbed(fg, seed), s["x"].ravel(), p)
        assert r.iters == ref.iters and r.term == ref.term
        assert [t[2] for t in r.trace] == [t[2] for t in ref.trace], f"seed {seed}: decisions differ"
        err = P.window_errors(f_ref, [t[0] for t in r.trace], windows)
        worst = [max(a, b) for a, b in zip(worst, err)]
        if x_tol is not None:
            assert np.abs(r.x - ref.x).max() * P.MARGIN <= x_tol, f"seed {seed}: final x"
    for (end, rtol), w in zip(windows, worst):
        assert w * P.MARGIN <= rtol, f"window to {end}: drift {w:.2e} against gate {rtol:.0e}"
        if rtol > 1e-9:
            assert w * P.MARGIN > 1e-9, f"window to {end}: drift {w:.2e} would fit a 1e-9 gate"
