"""GPU minimizer parity against the FP64 CPU oracle, through the C ABI.

FP64 mode follows the oracle iterate by iterate: the same line-search
decisions (equal evaluation counts after every iteration), energies within
1e-9 relative over the first 20 iterations and steps within 1e-6.  Further
out the trajectories separate at the rate the problem itself amplifies
rounding: perturbing the oracle's E and grad E by one ulp (relative 2^-52)
moves its own energies by 1e-11 (GD), 1e-9 (CG), 4e-12 (L-BFGS) and 2e-3
(FGM, whose momentum is unstable on this workload) by iteration 50, and by
5e-6 at iteration 40 for FGM with restarts, with identical decisions.  So
iterations 20..50 are gated at 1e-6 relative for GD, CG and L-BFGS, and the
FGM variants' energies are compared up to iteration 30.
Heavy ball (no decisions) amplifies a one-ulp perturbation to 1e-14 over 100
iterations and the optimized gradient method to 1.4e-13 over 50 on chain512
(every iteration gated at 1e-9), to 9e-10 on a 300-atom torsion chain (1e-9
for 10 iterations, then 1e-6).
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


def compare_traces(tr, ref, n, tight=20, loose=1e-6, loose_until=None):
    fr = np.array([t[0] for t in ref.trace[:n]])
    hr = np.array([t[1] for t in ref.trace[:n]])
    er = np.array([t[2] for t in ref.trace[:n]])
    assert len(tr) >= len(fr)
    np.testing.assert_array_equal(tr[: len(fr), 2], er)             # same LS decisions
    k = min(tight, len(fr))
    np.testing.assert_allclose(tr[:k, 0], fr[:k], rtol=1e-9, atol=0)
    np.testing.assert_allclose(tr[:k, 1], hr[:k], rtol=1e-6, atol=0)
    m = len(fr) if loose_until is None else min(loose_until, len(fr))
    np.testing.assert_allclose(tr[:m, 0], fr[:m], rtol=loose, atol=0)


@pytest.mark.parametrize("method", ["lbfgs", "cg", "gd", "fgm"])
def test_fp64_iterates_match_oracle_chain512(method):
    s = config_system("chain512")
    ref = oracle_run(s, method, max_iter=50)
    r, x, tr, _ = gpu_run(s, method, max_iter=50, precision="fp64")
    assert r["term"] == ref.term and r["iters"] == ref.iters and r["evals"] == ref.evals
    if method == "fgm":
        compare_traces(tr, ref, 50, loose_until=30)
    else:
        compare_traces(tr, ref, 50)
        assert r["energy"] == pytest.approx(ref.f, rel=1e-6)
        assert np.abs(x.ravel() - ref.x).max() < 1e-4


@pytest.mark.parametrize("method", ["lbfgs", "cg"])
def test_fp64_iterates_torsion_chain(method):
    s = torsion_chain(200, 5)
    s["x"] = s["x"] + np.random.default_rng(2).normal(scale=0.2, size=s["x"].shape)
    ref = oracle_run(s, method, max_iter=40, m=5)
    r, x, tr, _ = gpu_run(s, method, max_iter=40, m=5, precision="fp64")
    assert r["term"] == ref.term and r["iters"] == ref.iters
    compare_traces(tr, ref, 40)


@pytest.mark.parametrize("K", [3, 4])
def test_fp64_ls_par_more_trials(K):
    s = chain_system(400, 21)
    ref = oracle_run(s, "lbfgs", max_iter=25, ls_K=K)
    r, x, tr, _ = gpu_run(s, "lbfgs", max_iter=25, ls_K=K)
    assert r["evals"] == ref.evals
    compare_traces(tr, ref, 25)


def test_fp64_ls_h_for_lbfgs_and_ls_par_for_fgm():
    s = chain_system(350, 22)
    for method, ls in (("lbfgs", oracle.LS_H), ("fgm", oracle.LS_PAR)):
        ref = oracle_run(s, method, max_iter=30, linesearch=ls)
        r, x, tr, _ = gpu_run(s, method, max_iter=30, linesearch=ls)
        assert r["evals"] == ref.evals, method
        compare_traces(tr, ref, 30)


@pytest.mark.parametrize("beta", ["fr", "hs", "prp+", "cd", "ls", "dy"])
def test_fp64_cg_variants(beta):
    s = chain_system(300, 23)
    code = {"fr": oracle.CG_FR, "hs": oracle.CG_HS, "prp+": oracle.CG_PRP_PLUS, "cd": oracle.CG_CD,
            "ls": oracle.CG_LS, "dy": oracle.CG_DY}[beta]
    ref = oracle_run(s, "cg", max_iter=30, cg_beta=code)
    r, x, tr, _ = gpu_run(s, "cg", max_iter=30, cg_beta=beta)
    assert r["term"] == ref.term and r["evals"] == ref.evals
    compare_traces(tr, ref, 30)


def test_fp64_fgm_with_restart():
    s = config_system("chain512")
    ref = oracle_run(s, "fgm", max_iter=40, fgm_restart=True)
    r, x, tr, _ = gpu_run(s, "fgm", max_iter=40, fgm_restart=True)
    assert r["term"] == ref.term and r["evals"] == ref.evals
    compare_traces(tr, ref, 40, loose_until=30)


@pytest.mark.parametrize("K", [2, 3])
def test_fp64_ls_par_without_g0(K):
    s = chain_system(260, 24)
    ref = oracle_run(s, "lbfgs", max_iter=25, ls_K=K, ls_par_g0=False)
    r, x, tr, _ = gpu_run(s, "lbfgs", max_iter=25, ls_K=K, ls_par_g0=False)
    assert r["term"] == ref.term and r["evals"] == ref.evals
    compare_traces(tr, ref, 25)


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


def test_fp64_heavy_ball_matches_the_oracle():
    s = torsion_chain(300, 7)
    kw = dict(max_iter=100, hb_alpha=1e-3, hb_beta=0.8)
    ref = oracle_run(s, "hb", **kw)
    r, _, tr, _ = gpu_run(s, "hb", **kw)
    assert r["term"] == ref.term and r["iters"] == ref.iters == 100 and r["evals"] == ref.evals == 101
    compare_traces(tr, ref, 100, tight=100)
    assert np.all(tr[:100, 1] == 1e-3)


def test_heavy_ball_divergence_stops_at_the_last_finite_point():
    s = torsion_chain(120, 9)
    kw = dict(max_iter=10, hb_alpha=1e300, hb_beta=0.0)
    ref = oracle_run(s, "hb", **kw)
    r, x, _, _ = gpu_run(s, "hb", **kw)
    assert ref.term == oracle.DIVERGED and r["term"] == ff.FF_DIVERGED
    assert r["iters"] == ref.iters == 0 and r["evals"] == ref.evals == 2
    np.testing.assert_array_equal(x, s["x"])
    assert r["energy"] == pytest.approx(ref.f, rel=1e-12)


@pytest.mark.parametrize("system", ["chain512", "torsion300"])
def test_fp64_ogm_iterates_match_the_oracle(system):
    s = config_system("chain512") if system == "chain512" else torsion_chain(300, 7)
    ref = oracle_run(s, "ogm", max_iter=50)
    r, _, tr, _ = gpu_run(s, "ogm", max_iter=50)
    assert r["term"] == ref.term and r["iters"] == ref.iters and r["evals"] == ref.evals
    # a one-ulp perturbation grows to 1.4e-13 (chain512) and 9e-10 (torsion300)
    # by iteration 50 in the oracle itself
    compare_traces(tr, ref, 50, tight=50 if system == "chain512" else 10)


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
