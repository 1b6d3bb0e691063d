"""ff_energy_grad_noalloc (the entry point for callers that cannot allocate
device memory) against ff_energy_grad on a context, through the C ABI.

Both pack the system the same way, pick the same tiling and run the same
kernels, so energies and gradients must be identical bit for bit; both are
also checked against the FP64 oracle (energy 1e-6 and gradient norms 1e-5
relative in both precisions, FP64 element-wise to 1e-11 of the largest
component).  Two calls in a row share the library's static scratch: the
second, with a smaller system, must not see anything of the first.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1810_03358_amd as ff
from tests.systems import crosslinked_chain, torsion_chain

pytestmark = pytest.mark.gpu


def _noalloc(s, prec):
    x = torch.tensor(s["x"], dtype=torch.float64, device="cuda").contiguous()
    e = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    g = torch.full_like(x, float("nan"))
    ff.energy_grad_noalloc(s, x, e, g, prec)
    torch.cuda.synchronize()
    return float(e.cpu()[0]), g.cpu().numpy()


def _context(s, prec):
    ctx = ff.Context(s, m_max=0)
    x = torch.tensor(s["x"], dtype=torch.float64, device="cuda").contiguous()
    e, g = ctx.energy_grad(x, prec)
    torch.cuda.synchronize()
    out = float(e.cpu()[0]), g.cpu().numpy()
    ctx.close()
    return out


def _check_oracle(s, e, g, prec):
    e_ref, g_ref = oracle.energy_grad(s, s["x"])
    assert abs(e - e_ref) <= 1e-6 * abs(e_ref)
    n2, ni = np.linalg.norm(g_ref), np.abs(g_ref).max()
    assert abs(np.linalg.norm(g) - n2) <= 1e-5 * n2 and abs(np.abs(g).max() - ni) <= 1e-5 * ni
    if prec == "fp64":
        assert abs(e - e_ref) <= 1e-11 * abs(e_ref)
        np.testing.assert_allclose(g, g_ref, rtol=0, atol=1e-11 * ni)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_the_context_entry_point_on_two_calls(prec):
    # 3100 atoms: 256-atom I-blocks with a ragged last block, torsions and
    # exclusions more than 64 atoms apart; then 700 atoms: 64-atom blocks
    first = crosslinked_chain(3100, 11)
    second = torsion_chain(700, 12)
    results = []
    for s in (first, second):
        print(f"noalloc {prec} n={s['n_atoms']}", flush=True)
        e, g = _noalloc(s, prec)
        e_c, g_c = _context(s, prec)
        assert e == e_c
        np.testing.assert_array_equal(g, g_c)
        _check_oracle(s, e, g, prec)
        results.append((e, g))
    # the first system again after the second: the same bits
    e, g = _noalloc(first, prec)
    assert e == results[0][0]
    np.testing.assert_array_equal(g, results[0][1])


def test_noalloc_near_the_scratch_limit():
    """A 22,000-atom chain: its energy-only layout takes most of the static
    scratch (about 23,000 atoms fit), so the far end of the array is used;
    the results are those of the context path, bit for bit, in both
    precisions, then a small system follows."""
    from synth import chain_system
    big = chain_system(22_000, 13)
    for prec in ("fp64", "fp32"):
        print(f"noalloc {prec} n={big['n_atoms']}", flush=True)
        e, g = _noalloc(big, prec)
        e_c, g_c = _context(big, prec)
        assert e == e_c
        np.testing.assert_array_equal(g, g_c)
    e_ref, g_ref = oracle.energy_grad(big, big["x"])
    assert abs(e - e_ref) <= 1e-6 * abs(e_ref)
    small = torsion_chain(300, 14)
    e, g = _noalloc(small, "fp64")
    e_c, g_c = _context(small, "fp64")
    assert e == e_c
    np.testing.assert_array_equal(g, g_c)
