"""Error of each precision mode against the FP64 oracle, stated per workload.

For the three named chains (512, 10,000 and 50,000 atoms) at the start point
and at a relaxed point (GPU FP64 L-BFGS iterations from the start), both
modes are compared with the oracle's full evaluation: relative energy error,
relative error of |grad E|_2 and of |grad E|_inf, and the largest component
error relative to |grad E|_inf.  Gates: energy 1e-6 and gradient norms 1e-5
relative in both modes (FP32 mode: where |grad E|_inf >= 1, as elsewhere);
largest component error relative to |grad E|_inf: 1e-12 in FP64 mode and
RC_FP32 in FP32 mode, a constant calibrated once on chain512 (start and
relaxed point: at most 1.4e-6 measured; 2.1e-6 with a later default
tiling, whose summation order reaches another 300-iteration point) and frozen at about three times
that.  The printed table is the measured error (run with -s to see it).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1810_03358_amd as ff
from synth import config_system

pytestmark = pytest.mark.gpu

RELAX = {"chain512": 300, "chain10k": 200, "chain50k": 100}
RC_FP64 = 1e-12
RC_FP32 = 2.0 ** -18          # calibrated on chain512, then frozen


@pytest.mark.parametrize("name", ["chain512", "chain10k", "chain50k"])
def test_error_against_the_oracle_per_workload(name):
    s = config_system(name)
    ctx = ff.Context(s, m_max=10)
    x = torch.tensor(s["x"], dtype=torch.float64, device="cuda").contiguous()
    points = {"start": x.clone()}
    ctx.minimize(x, "lbfgs", max_iter=RELAX[name], precision="fp64")
    points[f"after {RELAX[name]} L-BFGS iterations"] = x
    for where, xp in points.items():
        xh = xp.cpu().numpy()
        e_ref, g_ref = oracle.energy_grad(s, xh)
        n2r, nir = np.linalg.norm(g_ref), np.abs(g_ref).max()
        for prec in ("fp64", "fp32"):
            e, g = ctx.energy_grad(xp, prec)
            torch.cuda.synchronize()
            e, g = float(e.cpu()[0]), g.cpu().numpy()
            re = abs(e - e_ref) / abs(e_ref)
            r2 = abs(np.linalg.norm(g) - n2r) / n2r
            ri = abs(np.abs(g).max() - nir) / nir
            rc = np.abs(g - g_ref).max() / nir
            print(f"\n{name} {where} {prec}: E {e_ref:.6e} rel err {re:.2e}; |g|_2 {n2r:.4e} rel err {r2:.2e}; "
                  f"|g|_inf {nir:.4e} rel err {ri:.2e}; max component err / |g|_inf {rc:.2e}")
            assert re <= 1e-6
            if prec == "fp64" or nir >= 1.0:
                assert r2 <= 1e-5 and ri <= 1e-5
            assert rc <= (RC_FP64 if prec == "fp64" else RC_FP32)
