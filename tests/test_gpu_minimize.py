"""GPU minimizer parity against the FP64 CPU oracle, through the C ABI.

FP64 mode follows the oracle iterate by iterate on every case of
tests/parity_cases.py: the same line-search decisions (equal evaluation
counts after every iteration), energies within each case's gate windows and
steps within 1e-6 over the first window.  The gates are backed by the
oracle's own sensitivity to rounding-level perturbations
(tests/test_oracle_sensitivity.py): each window is the tightest of 1e-9,
1e-8, ... that the perturbed oracle stays inside with a margin of 10.
FP32 mode is checked on its final state: the certified energy and gradient
norm reported for the returned point must be what the oracle computes there.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1810_03358_amd as ff
from synth import chain_system, config_system
from tests import parity_cases as P
from tests.systems import make_system, torsion_chain

pytestmark = pytest.mark.gpu

OMETHOD = {"gd": oracle.GD, "fgm": oracle.FGM, "cg": oracle.CG, "lbfgs": oracle.LBFGS, "hb": oracle.HB,
           "ogm": oracle.OGM}


def oracle_run(s, method, **kw):
    sysc = oracle.System(s)
    p = oracle.MinParams(method=OMETHOD[method], **kw)
    return oracle.minimize(lambda v: oracle.energy_grad(sysc, v.reshape(-1, 3)), s["x"].ravel(), p)


def gpu_run(s, method, ctx=None, x=None, **kw):
    ctx = ctx or ff.Context(s, m_max=max(10, kw.get("m", 10)))
    xt = torch.tensor(s["x"] if x is None else x, dtype=torch.float64, device="cuda").reshape(-1, 3).contiguous()
    r = ctx.minimize(xt, method, **kw)
    return r, xt.cpu().numpy(), ctx.trace(), ctx


@pytest.mark.parametrize("case", sorted(P.CASES))
def test_fp64_iterates_match_the_oracle(case):
    print(f"parity case {case}", flush=True)
    s = P.system(case)
    sysc = oracle.System(s)
    ref = oracle.minimize(lambda v: oracle.energy_grad(sysc, v.reshape(-1, 3)), s["x"].ravel(),
                          P.oracle_params(case))
    kw = P.gpu_kwargs(case)
    r, x, tr, _ = gpu_run(s, precision="fp64", **kw)
    assert r["term"] == ref.term and r["iters"] == ref.iters and r["evals"] == ref.evals
    _, method, _, n_iter, windows, x_tol = P.CASES[case]
    n = len(ref.trace)
    assert n == n_iter and len(tr) >= n
    np.testing.assert_array_equal(tr[:n, 2], [t[2] for t in ref.trace])      # same LS decisions
    errs = P.window_errors([t[0] for t in ref.trace], tr[:n, 0], windows)
    for (end, rtol), e in zip(windows, errs):
        assert e <= rtol, f"energies before iteration {end}: {e:.2e} > {rtol:.0e}"
    k = windows[0][0]
    np.testing.assert_allclose(tr[:k, 1], [t[1] for t in ref.trace[:k]], rtol=1e-6, atol=0)
    assert r["energy"] == pytest.approx(ref.f, rel=windows[-1][1])
    if x_tol is not None:
        assert np.abs(x.ravel() - ref.x).max() <= x_tol
    if method == "hb":
        assert np.all(tr[:n, 1] == kw["hb_alpha"]) and r["evals"] == n + 1


def test_two_atom_lj_converges_to_the_closed_form_minimum():
    sig, eps = 3.3, 0.2
    s = make_system([[0, 0, 0], [1.5 * sig, 0.0, 0.0]], sigma=[sig, sig], eps=[eps, eps])
    r, x, _, _ = gpu_run(s, "lbfgs", tol=1e-8, max_iter=200)
    assert r["term"] == ff.FF_CONVERGED
    assert np.linalg.norm(x[1] - x[0]) == pytest.approx(2 ** (1 / 6) * sig, rel=1e-6)
    assert r["energy"] == pytest.approx(-eps, rel=1e-10)


def test_termination_paths():
    # coincident atoms: the start energy is not finite
    s = make_system([[0, 0, 0], [0, 0, 0], [3, 0, 0]], q=[0.1, 0.1, 0.1], eps=[0.1] * 3)
    r, _, _, _ = gpu_run(s, "lbfgs")
    assert r["term"] == ff.FF_NONFINITE_START and r["evals"] == 1
    # no iteration allowed
    s = chain_system(100, 3)
    r, x, _, _ = gpu_run(s, "cg", max_iter=0)
    assert r["term"] == ff.FF_MAX_ITER and r["iters"] == 0 and r["evals"] == 1
    np.testing.assert_array_equal(x, s["x"])
    # one iteration
    r, _, _, _ = gpu_run(s, "gd", max_iter=1)
    assert r["term"] == ff.FF_MAX_ITER and r["iters"] == 1 and r["evals"] == 3


def test_resume_continues_exactly():
    s = chain_system(600, 8)
    r20, x20, tr20, _ = gpu_run(s, "lbfgs", max_iter=20)
    ctx = ff.Context(s, m_max=10)
    xt = torch.tensor(s["x"], dtype=torch.float64, device="cuda")
    ctx.minimize(xt, "lbfgs", max_iter=10)
    r = ctx.minimize(xt, "lbfgs", max_iter=10, resume=True)
    assert r["iters"] == 10
    np.testing.assert_array_equal(xt.cpu().numpy(), x20)


def test_fp32_mode_certifies_the_returned_point():
    s = config_system("chain512")
    r, x, _, _ = gpu_run(s, "lbfgs", max_iter=300, precision="fp32")
    assert r["term"] in (ff.FF_MAX_ITER, ff.FF_CONVERGED, ff.FF_LS_FAILED)
    e_ref, g_ref = oracle.energy_grad(s, x)
    assert r["energy"] == pytest.approx(e_ref, rel=1e-9)
    assert r["grad_inf"] == pytest.approx(np.abs(g_ref).max(), rel=1e-6)
    ref = oracle_run(s, "lbfgs", max_iter=300)
    # both runs descend from 1e13 to the same energy scale
    assert r["energy"] < 0 and abs(r["energy"] - ref.f) < 0.05 * abs(ref.f)


def test_fp32_converges_with_fp64_end_game():
    s = chain_system(120, 31)
    r, x, _, _ = gpu_run(s, "lbfgs", max_iter=5000, precision="fp32")
    assert r["term"] == ff.FF_CONVERGED
    assert r["evals_fp64"] >= 1
    e_ref, g_ref = oracle.energy_grad(s, x)
    assert np.abs(g_ref).max() < 1e-3


def test_heavy_ball_divergence_stops_at_the_last_finite_point():
    s = torsion_chain(120, 9)
    kw = dict(max_iter=10, hb_alpha=1e300, hb_beta=0.0)
    ref = oracle_run(s, "hb", **kw)
    r, x, _, _ = gpu_run(s, "hb", **kw)
    assert ref.term == oracle.DIVERGED and r["term"] == ff.FF_DIVERGED
    assert r["iters"] == ref.iters == 0 and r["evals"] == ref.evals == 2
    np.testing.assert_array_equal(x, s["x"])
    assert r["energy"] == pytest.approx(ref.f, rel=1e-12)


def test_fp32_stagnation_switches_to_fp64_and_converges():
    """A compacted 595-atom chain on which FP32 line searches end up
    accepting steps of 1e-9 A on FP32 noise: the run must switch to FP64,
    restart its step length and converge (it used to stop with LS_FAILED at
    |g|_inf = 0.13)."""
    rng = np.random.default_rng(11)
    sizes = rng.integers(300, 600, size=56)
    s = chain_system(int(sizes[48]), 500_048, compact=True)
    r, x, _, _ = gpu_run(s, "lbfgs", max_iter=30000, precision="fp32")
    assert r["term"] == ff.FF_CONVERGED and r["evals_fp64"] >= 1
    e_ref, g_ref = oracle.energy_grad(s, x)
    assert np.abs(g_ref).max() < 1e-3
    assert r["energy"] == pytest.approx(e_ref, rel=1e-9)
