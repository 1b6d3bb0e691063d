"""Batched evaluation and minimization: several independent systems of
uneven size in one context, each checked against the FP64 CPU oracle."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1810_03358_amd as ff
from synth import batch_sizes, chain_system
from tests.systems import make_system, torsion_chain

pytestmark = pytest.mark.gpu


def batch_systems():
    return [chain_system(1, 40), chain_system(65, 41), torsion_chain(150, 42), chain_system(300, 43),
            chain_system(513, 44), chain_system(1200, 45)]


def concat(systems):
    return torch.tensor(np.concatenate([s["x"] for s in systems]), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_energy_grad_matches_oracle_per_system(prec):
    systems = batch_systems()
    ctx = ff.Context(systems, m_max=0)
    x = concat(systems)
    e, g = ctx.energy_grad(x, prec)
    torch.cuda.synchronize()
    e = e.cpu().numpy()
    g = g.cpu().numpy()
    off = 0
    for k, s in enumerate(systems):
        e_ref, g_ref = oracle.energy_grad(s, s["x"])
        gk = g[off: off + s["n_atoms"]]
        off += s["n_atoms"]
        assert abs(e[k] - e_ref) <= 1e-6 * max(abs(e_ref), 1e-12), (k, e[k], e_ref)
        scale = max(np.abs(g_ref).max(), 1e-12)
        tol = 1e-11 if prec == "fp64" else 2e-5
        assert np.abs(gk - g_ref).max() <= tol * scale, (k, prec)


def test_batch_minimize_fp64_each_system_follows_the_oracle():
    systems = [chain_system(200, 50), chain_system(333, 51), torsion_chain(120, 52), chain_system(480, 53)]
    systems[2]["x"] = systems[2]["x"] + np.random.default_rng(3).normal(scale=0.2, size=systems[2]["x"].shape)
    ctx = ff.Context(systems, m_max=10)
    x = concat(systems)
    res = ctx.minimize(x, "lbfgs", max_iter=20, precision="fp64")
    xs = x.cpu().numpy()
    off = 0
    for k, s in enumerate(systems):
        sysc = oracle.System(s)
        ref = oracle.minimize(lambda v: oracle.energy_grad(sysc, v.reshape(-1, 3)), s["x"].ravel(),
                              oracle.MinParams(method=oracle.LBFGS, max_iter=20))
        r = res[k]
        assert r["term"] == ref.term and r["iters"] == ref.iters and r["evals"] == ref.evals, k
        assert r["energy"] == pytest.approx(ref.f, rel=1e-9), k
        xk = xs[off: off + s["n_atoms"]]
        off += s["n_atoms"]
        assert np.abs(xk.ravel() - ref.x).max() < 1e-7, k
    tr = ctx.trace()
    assert len(tr) == 20


def test_batch_systems_stop_independently():
    sig, eps = 3.3, 0.2
    lj = make_system([[0, 0, 0], [1.5 * sig, 0.0, 0.0]], sigma=[sig, sig], eps=[eps, eps])
    clash = make_system([[0, 0, 0], [0, 0, 0], [3, 0, 0]], q=[0.1, 0.1, 0.1], eps=[0.1] * 3)
    chain = chain_system(250, 60)
    systems = [chain, lj, clash]
    ctx = ff.Context(systems, m_max=10)
    x = concat(systems)
    res = ctx.minimize(x, "lbfgs", tol=1e-8, max_iter=60)
    assert res[0]["term"] == ff.FF_MAX_ITER and res[0]["iters"] == 60
    assert res[1]["term"] == ff.FF_CONVERGED and res[1]["energy"] == pytest.approx(-eps, rel=1e-10)
    assert res[2]["term"] == ff.FF_NONFINITE_START and res[2]["evals"] == 1
    xs = x.cpu().numpy()
    d = np.linalg.norm(xs[250 + 1] - xs[250])
    assert d == pytest.approx(2 ** (1 / 6) * sig, rel=1e-6)


def test_batch_fp32_certified_results():
    sizes = batch_sizes(12, 200, 1000, seed=7)
    systems = [chain_system(n, 100 + k) for k, n in enumerate(sizes)]
    ctx = ff.Context(systems, m_max=10)
    x = concat(systems)
    res = ctx.minimize(x, "lbfgs", max_iter=150, precision="fp32")
    xs = x.cpu().numpy()
    off = 0
    for k, s in enumerate(systems):
        xk = xs[off: off + s["n_atoms"]]
        off += s["n_atoms"]
        e_ref, g_ref = oracle.energy_grad(s, xk)
        assert res[k]["energy"] == pytest.approx(e_ref, rel=1e-9), k
        assert res[k]["grad_inf"] == pytest.approx(np.abs(g_ref).max(), rel=1e-6), k
        assert res[k]["energy"] < 0


def test_batch_mixed_precision_cycles():
    """In FP32 mode a small system reaches its FP64 end game while a chain of
    the same batch is still evaluated in FP32: cycles then run both pair
    kernels, each on its own systems."""
    sig, eps = 3.3, 0.2
    lj = make_system([[0, 0, 0], [1.5 * sig, 0.0, 0.0]], sigma=[sig, sig], eps=[eps, eps])
    chain = chain_system(400, 61)
    systems = [chain, lj]
    ctx = ff.Context(systems, m_max=10)
    x = concat(systems)
    res = ctx.minimize(x, "lbfgs", tol=1e-8, max_iter=100, precision="fp32")
    assert res[1]["term"] == ff.FF_CONVERGED and res[1]["evals_fp64"] >= 1
    assert res[1]["energy"] == pytest.approx(-eps, rel=1e-10)
    assert res[0]["term"] == ff.FF_MAX_ITER
    xs = x.cpu().numpy()
    e_ref, g_ref = oracle.energy_grad(chain, xs[:400])
    assert res[0]["energy"] == pytest.approx(e_ref, rel=1e-9)
    assert res[0]["grad_inf"] == pytest.approx(np.abs(g_ref).max(), rel=1e-6)


def test_batch_fp32_resume_across_the_fp64_switch():
    """FP32 mode on two chains that both switch to FP64 evaluations before
    they converge: one call, and the same run cut short after both have
    switched and then resumed, end bit-identical.  Once every system of a
    batch has switched (or stopped), cycles run without the FP32 pair
    kernel; on resume that state is rebuilt from the stored control blocks."""
    systems = [chain_system(120, 31), chain_system(150, 32)]
    ctx = ff.Context(systems, m_max=10)
    xa = concat(systems)
    ra = ctx.minimize(xa, "lbfgs", max_iter=5000, precision="fp32")
    assert all(r["term"] == ff.FF_CONVERGED and r["evals_fp64"] >= 1 for r in ra)
    cut = min(r["iters"] for r in ra) - 3
    ctxb = ff.Context(systems, m_max=10)
    xb = concat(systems)
    rb1 = ctxb.minimize(xb, "lbfgs", max_iter=cut, precision="fp32")
    assert all(r["evals_fp64"] >= 1 for r in rb1), [r["evals_fp64"] for r in rb1]
    rb2 = ctxb.minimize(xb, "lbfgs", max_iter=5000, precision="fp32", resume=True)
    np.testing.assert_array_equal(xb.cpu().numpy(), xa.cpu().numpy())
    for a, b1, b2 in zip(ra, rb1, rb2):
        assert b2["term"] == a["term"] and b1["iters"] + b2["iters"] == a["iters"]
        assert b2["energy"] == a["energy"]
