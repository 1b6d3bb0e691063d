"""Every pair-kernel tiling (configuration x chunk length) against the FP64
oracle, and the autotuner's choice, through the C ABI.

The tiling changes only the order in which pair partials are summed, so each
configuration must meet the same gates as the default one: FP64 energy and
gradient element-wise to 1e-11 relative (of the largest component); FP32 mode
energy to 1e-6 relative and every gradient component within the FP32 rounding
model of the energy tests (2^-16 of the summed absolute pair forces on its
atom), on a clash-free chain whose size leaves a ragged last I-block and j-tile
for every block size.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1810_03358_amd as ff
from synth import chain_system
from tests.systems import crosslinked_chain, torsion_chain
from tests.test_gpu_energy import FP32_ELEM, abs_pair_force_sum, fp32_elem_ratio

pytestmark = pytest.mark.gpu

CONFIGS = list(range(len(ff.tile_configs())))


def _run(s, x, prec, tiling):
    ctx = ff.Context(s, m_max=0, tiling=tiling)
    expected = tuple(tiling) if len(tiling) == 3 else tuple(tiling) + (tiling[1],)
    assert ctx.tiling == expected
    xt = torch.tensor(np.asarray(x).reshape(-1, 3), dtype=torch.float64, device="cuda")
    e, g = ctx.energy_grad(xt, prec)
    torch.cuda.synchronize()
    out = float(e.cpu()[0]), g.cpu().numpy()
    ctx.close()
    return out


@pytest.fixture(scope="module")
def system():
    s = torsion_chain(1100, 5)           # clash-free, all term kinds; 1100 = 2*512 + 76
    e, g = oracle.energy_grad(s, s["x"])
    return s, e, g, abs_pair_force_sum(s, s["x"])


@pytest.mark.parametrize("cfg", CONFIGS)
@pytest.mark.parametrize("chunks", [(1, 1), (3, 3), (2, 5)])
def test_every_tiling_matches_the_oracle(system, cfg, chunks):
    """chunks = (FP32 kernel's, FP64 kernel's chunk length); lengths above one
    also put each I-block's last j-tiles into one-tile chunks."""
    s, e_ref, g_ref, pair_force_sum = system
    print(f"tiling cfg={cfg} chunks={chunks} n={s['n_atoms']}", flush=True)
    e, g = _run(s, s["x"], "fp64", (cfg,) + chunks)
    assert abs(e - e_ref) <= 1e-11 * abs(e_ref)
    np.testing.assert_allclose(g, g_ref, rtol=0, atol=1e-11 * np.abs(g_ref).max())
    e32, g32 = _run(s, s["x"], "fp32", (cfg,) + chunks)
    assert abs(e32 - e_ref) <= 1e-6 * abs(e_ref)
    bound = FP32_ELEM * pair_force_sum[:, None] + 1e-9 * np.abs(g_ref).max()
    print(f"fp32 element ratio {fp32_elem_ratio(g32, g_ref, pair_force_sum[:, None]):.3e}")
    assert np.all(np.abs(g32 - g_ref) <= bound), np.abs(g32 - g_ref).max()


def test_autotune_returns_a_working_tiling():
    sizes = [300, 77, 1030]
    systems = [chain_system(n, 40 + k) for k, n in enumerate(sizes)]
    x = torch.tensor(np.concatenate([s["x"] for s in systems]), dtype=torch.float64, device="cuda").contiguous()
    print("autotune batch", sizes, flush=True)
    tiling, ms = ff.autotune(systems, x, "fp32", reps=2)
    assert 0 <= tiling[0] < len(ff.tile_configs()) and tiling[1] in (1, 2, 4, 8, 16)
    assert 0.0 < ms < 1000.0
    ctx = ff.Context(systems, m_max=0, tiling=tiling)
    e, _ = ctx.energy_grad(x, "fp64")
    torch.cuda.synchronize()
    for k, s in enumerate(systems):
        e_ref, _ = oracle.energy_grad(s, s["x"])
        assert abs(float(e.cpu()[k]) - e_ref) <= 1e-9 * abs(e_ref)


@pytest.fixture(scope="module")
def linked():
    s = crosslinked_chain(1100, 5)
    e, g = oracle.energy_grad(s, s["x"])
    return s, e, g, abs_pair_force_sum(s, s["x"])


@pytest.mark.parametrize("cfg", CONFIGS)
def test_far_exclusions_match_the_oracle_for_every_tiling(linked, cfg):
    s, e_ref, g_ref, pair_force_sum = linked
    print(f"far exclusions cfg={cfg}", flush=True)
    e, g = _run(s, s["x"], "fp64", (cfg, 2, 4))
    assert abs(e - e_ref) <= 1e-11 * abs(e_ref)
    np.testing.assert_allclose(g, g_ref, rtol=0, atol=1e-11 * np.abs(g_ref).max())
    e32, g32 = _run(s, s["x"], "fp32", (cfg, 2, 4))
    assert abs(e32 - e_ref) <= 1e-6 * abs(e_ref)
    bound = FP32_ELEM * pair_force_sum[:, None] + 1e-9 * np.abs(g_ref).max()
    print(f"fp32 element ratio {fp32_elem_ratio(g32, g_ref, pair_force_sum[:, None]):.3e}")
    assert np.all(np.abs(g32 - g_ref) <= bound), np.abs(g32 - g_ref).max()


def test_fp32_mode_minimization_with_separate_chunk_tables():
    """FP32 mode runs both pair kernels in one minimization (FP32 evaluations,
    then the FP64 end game); with different chunk lengths each kernel walks
    its own chunk table and the finalize reads the matching partial rows."""
    s = chain_system(1100, 31)
    print("fp32-mode minimize, tiling (4, 1, 3)", flush=True)
    ctx = ff.Context(s, m_max=10, tiling=(4, 1, 3))
    x = torch.tensor(s["x"], dtype=torch.float64, device="cuda")
    r = ctx.minimize(x, "lbfgs", max_iter=400, precision="fp32", tol=1.0)
    assert r["evals_fp64"] >= 1 and r["evals"] > r["evals_fp64"]
    xs = x.cpu().numpy()
    e_ref, g_ref = oracle.energy_grad(s, xs)
    assert r["energy"] == pytest.approx(e_ref, rel=1e-9)
    assert r["grad_inf"] == pytest.approx(np.abs(g_ref).max(), rel=1e-6)
    e0, _ = oracle.energy_grad(s, s["x"])         # 1.9e13: clashes at the start
    assert r["energy"] < 1e-6 * e0
