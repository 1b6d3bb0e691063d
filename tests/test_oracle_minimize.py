"""Pins of the oracle's line searches and methods (section 5 of the paper)
against what the mathematics fixes on quadratics, plus the chain workload."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import MinParams, minimize

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


def quad(A, b):
    """f = x'Ax/2 - b'x with its gradient; A is a dense matrix or a diagonal."""
    if A.ndim == 1:
        def fg(x):
            return 0.5 * float(x @ (A * x)) - float(b @ x), A * x - b
    else:
        def fg(x):
            Ax = A @ x
            return 0.5 * float(x @ Ax) - float(b @ x), Ax - b
    return fg


# --------------------------------------------------------------------- P11

@pytest.mark.parametrize("a,b,h0", [(2.0, -3.0, 0.5), (0.7, -0.05, 0.02), (5.0, -1.0, 1.0)])
def test_ls_par_vertex_is_exact_on_a_parabola(a, b, h0):
    c = 1.25
    probes = []

    def fg(x):
        probes.append(float(x[0]))
        return a * x[0] ** 2 + b * x[0] + c, np.array([2 * a * x[0] + b])

    ok, h, f, g, hmin = oracle.ls_par(fg, np.zeros(1), np.ones(1), h0, c, b, K=2)
    vertex = -b / (2 * a)
    assert ok and len(probes) == 2 and probes[0] == h0
    assert probes[1] == pytest.approx(vertex, rel=1e-12)
    assert h == pytest.approx(vertex, rel=1e-12)
    assert f == pytest.approx(c - b * b / (4 * a), rel=1e-12)
    assert hmin == min(probes)


def test_ls_par_extra_trials_stay_exact_on_a_parabola():
    a, b, c = 3.0, -2.0, 0.0
    probes = []

    def fg(x):
        probes.append(float(x[0]))
        return a * x[0] ** 2 + b * x[0] + c, np.array([2 * a * x[0] + b])

    ok, h, f, _, _ = oracle.ls_par(fg, np.zeros(1), np.ones(1), 0.1, c, b, K=4)
    assert ok and len(probes) == 4
    assert h == pytest.approx(-b / (2 * a), rel=1e-12)


# --------------------------------------------------------------------- P12

def test_ls_h_halving_sequence_on_an_increasing_slice():
    probes = []

    def fg(x):
        probes.append(float(x[0]))
        return float(x[0]), np.ones(1)          # f(h) = h > f* = 0 for every h > 0

    h0, km, eps_h = 0.1, 0.5, 1e-10
    ok, h, f, g = oracle.ls_h(fg, np.zeros(1), np.ones(1), h0, 0.0, 2.0, km, eps_h)
    assert not ok and h == 0.0 and f == 0.0
    expect = [h0]
    while expect[-1] * km > eps_h:
        expect.append(expect[-1] * km)
    assert probes == expect


def test_ls_h_doubles_on_success():
    probes = []

    def fg(x):
        probes.append(float(x[0]))
        return (x[0] - 1.0) ** 2, np.array([2 * (x[0] - 1.0)])

    ok, h, f, _ = oracle.ls_h(fg, np.zeros(1), np.ones(1), 0.3, 1.0)
    assert ok and probes == [0.3, 0.6] and h == 0.6
    probes.clear()
    ok, h, f, _ = oracle.ls_h(fg, np.zeros(1), np.ones(1), 0.7, 1.0)
    assert ok and probes == [0.7, 1.4] and h == 0.7      # doubling overshoots: keep h0


# --------------------------------------------------------------------- P13

def test_gd_exact_line_search_rate():
    with open(GOLDEN) as fh:
        gq = json.load(fh)["gd_quadratic"]
    kappa = gq["kappa"]
    fg = quad(np.array([1.0, kappa]), np.zeros(2))
    res = minimize(fg, [kappa, 1.0], MinParams(method=oracle.GD, tol=1e-9, max_iter=40, h_init=1.0))
    fs = [fg(np.array([kappa, 1.0]))[0]] + [t[0] for t in res.trace]
    ratios = [fs[k + 1] / fs[k] for k in range(len(fs) - 1) if fs[k] > 1e-20]
    assert len(ratios) >= 20
    for r in ratios:
        assert r == pytest.approx(gq["ratio"], rel=1e-9)


# --------------------------------------------------------------------- P14

def _spd(n, seed, lo=1.0, hi=50.0):
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    lam = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n))
    return (q * lam) @ q.T, rng.normal(size=n)


def test_lbfgs_full_memory_matches_cg_and_terminates():
    n = 30
    A, b = _spd(n, 0)
    fg = quad(A, b)
    x0 = np.zeros(n)
    cg = minimize(fg, x0, MinParams(method=oracle.CG, tol=1e-14, max_iter=10, cg_restart=1000, h_init=1.0))
    lb = minimize(fg, x0, MinParams(method=oracle.LBFGS, m=n, tol=1e-14, max_iter=10, h_init=1.0))
    for (fc, hc, _), (fl, hl, _) in zip(cg.trace, lb.trace):
        assert fl == pytest.approx(fc, rel=1e-12)
        assert hl == pytest.approx(hc, rel=1e-9)
    assert np.abs(lb.x - cg.x).max() < 1e-9 * np.abs(cg.x).max()
    full = minimize(fg, x0, MinParams(method=oracle.LBFGS, m=n, tol=0.0, max_iter=n, h_init=1.0))
    assert full.iters == n or full.term != oracle.MAX_ITER
    # exact arithmetic terminates at step n; the parabola fit of LS_PAR is exact
    # only up to rounding, so ask for 7 orders of magnitude (GD would reduce the
    # gradient by less than one order in n steps at this conditioning)
    assert np.linalg.norm(fg(full.x)[1]) < 1e-7 * np.linalg.norm(b)


def test_cg_finds_the_quadratic_minimum():
    n = 30
    A, b = _spd(n, 1)
    # tol is chosen so that the f-decrease of the last steps (~|g|^2/L) stays
    # well above the rounding of f: the line searches compare f values
    res = minimize(quad(A, b), np.zeros(n), MinParams(method=oracle.CG, tol=1e-6, max_iter=500, h_init=1.0))
    assert res.term == oracle.CONVERGED
    assert np.abs(res.x - np.linalg.solve(A, b)).max() < 1e-5


# --------------------------------------------------------------------- P15

def test_lbfgs_large_quadratic():
    n = 3000
    rng = np.random.default_rng(7)
    lam = np.exp(rng.uniform(0.0, math.log(1e3), size=n))
    b = rng.normal(size=n)
    # f ~ -200 here: below |g|_inf ~ 1e-6 the decrease per step reaches the
    # rounding of f, which the line searches compare, so stop at 1e-5
    res = minimize(quad(lam, b), np.zeros(n), MinParams(method=oracle.LBFGS, m=10, tol=1e-5,
                                                        max_iter=3000, h_init=1.0))
    assert res.term == oracle.CONVERGED
    assert np.abs(res.x - b / lam).max() < 1e-5


# --------------------------------------------------------------------- P16

def test_fgm_coefficients():
    with open(GOLDEN) as fh:
        gf = json.load(fh)["fgm"]
    th = 1.0
    for k in range(3):
        t, b = oracle.fgm_coefficients(th)
        assert t == pytest.approx(gf["theta"][k], abs=1e-15)
        assert b == pytest.approx(gf["beta"][k], abs=1e-15)
        th = t
    assert oracle.fgm_coefficients(1.0)[0] == pytest.approx(gf["theta0_closed_form"], abs=1e-16)
    th = 1.0
    for _ in range(200):
        t, b = oracle.fgm_coefficients(th)
        assert t * t == pytest.approx((1 - t) * th * th, rel=1e-13)   # theta_k^2 = (1-theta_k) theta_{k-1}^2
        assert 0.0 <= b < 1.0
        th = t


def test_fgm_best_point_is_monotone():
    """Algorithm 1 keeps the best point because the method is not monotone.
    With a line-search step in place of 1/L and no restart it need not converge
    on an ill-conditioned quadratic, so only what the algorithm guarantees is
    pinned here: the returned point is the best iterate, and it improves."""
    n = 40
    A, b = _spd(n, 3, 1.0, 100.0)
    fg = quad(A, b)
    fmin = fg(np.linalg.solve(A, b))[0]
    res = minimize(fg, np.zeros(n), MinParams(method=oracle.FGM, tol=1e-7, max_iter=300, h_init=1.0))
    best = min(t[0] for t in res.trace)
    assert res.f == best and fg(res.x)[0] == best
    assert res.f - fmin < 0.1 * (0.0 - fmin)


def test_fgm_with_restart_converges_on_a_quadratic():
    """With the function-value restart the accelerated method converges
    linearly on a strictly convex quadratic (O'Donoghue and Candes 2015)."""
    n = 40
    A, b = _spd(n, 3, 1.0, 100.0)
    fg = quad(A, b)
    res = minimize(fg, np.zeros(n), MinParams(method=oracle.FGM, tol=1e-6, max_iter=3000, h_init=1.0,
                                              fgm_restart=True))
    assert res.term == oracle.CONVERGED and res.iters < 1000
    assert np.abs(res.x - np.linalg.solve(A, b)).max() < 1e-5


def test_fgm_isotropic_quadratic_one_step():
    lam = np.full(5, 2.0)
    b = np.arange(1.0, 6.0)
    fg = quad(lam, b)
    # along -grad the minimum is at distance |g|/2 = |b|/2; h_init is chosen so
    # that LS_H's doubling lands on it exactly
    h = float(np.linalg.norm(b)) / 4
    res = minimize(fg, np.zeros(5), MinParams(method=oracle.FGM, tol=1e-12, max_iter=5, h_init=h))
    assert res.term == oracle.CONVERGED and res.iters == 1
    assert np.abs(res.x - b / 2).max() < 1e-15 * 10


# ------------------------------------------------------------ termination paths

def test_nonfinite_start():
    def fg(x):
        return math.inf, np.zeros_like(x)
    res = minimize(fg, np.zeros(3), MinParams())
    assert res.term == oracle.NONFINITE_START and res.evals == 1


def test_max_iter_one_and_counts():
    fg = quad(np.array([1.0, 10.0]), np.zeros(2))
    res = minimize(fg, [3.0, 1.0], MinParams(method=oracle.LBFGS, max_iter=1, tol=1e-12))
    assert res.term == oracle.MAX_ITER and res.iters == 1 and res.evals == 3   # start + 2 trials


def test_ls_failure_on_an_ascent_only_objective():
    # f decreases nowhere along any direction from 0 at the chosen scale: |x|^0.5
    def fg(x):
        r = float(np.linalg.norm(x))
        return (r if r > 0 else 0.0) ** 0.5 - 1e9 * (r == 0), x
    res = minimize(lambda x: (float(np.sum(np.abs(x))) * 0 + 1.0, np.ones_like(x)), np.zeros(3),
                   MinParams(method=oracle.CG, tol=1e-3))
    assert res.term == oracle.LS_FAILED


# --------------------------------------------------------------- P17 chain 512

def test_chain512_lbfgs_descends():
    """Full-chain run (parity unpinned beyond the invariants: no printed value
    exists).  Every accepted L-BFGS step lowers E strictly, and 200 iterations
    take the clash-dominated start energy down by many orders of magnitude."""
    from synth import config_system
    s = config_system("chain512")
    sysc = oracle.System(s)
    e0, g0 = oracle.energy_grad(sysc, s["x"])
    res = minimize(lambda x: oracle.energy_grad(sysc, x.reshape(-1, 3)), s["x"].ravel(),
                   MinParams(method=oracle.LBFGS, m=10, tol=1e-3, max_iter=200))
    assert res.term == oracle.MAX_ITER and res.iters == 200
    fs = [e0] + [t[0] for t in res.trace]
    assert all(b < a for a, b in zip(fs, fs[1:]))
    assert e0 > 1e10 and res.f < 0
    assert np.abs(res.g).max() < 1e-6 * np.abs(g0).max()
    assert res.evals == 1 + 2 * 200          # LS_PAR: two oracle calls per iteration


# ------------------------------------------------------- CG variants, G0=false

@pytest.mark.parametrize("variant", [oracle.CG_FR, oracle.CG_HS, oracle.CG_PRP_PLUS, oracle.CG_CD,
                                     oracle.CG_LS, oracle.CG_DY])
def test_cg_variants_coincide_on_a_quadratic(variant):
    """With exact line searches on a strictly convex quadratic the gradients
    are mutually orthogonal and orthogonal to the previous direction, so every
    beta formula of section 5.1 reduces to the same value: the iterates of all
    variants coincide with PRP's."""
    n = 30
    A, b = _spd(n, 4)
    fg = quad(A, b)
    ref = minimize(fg, np.zeros(n), MinParams(method=oracle.CG, tol=1e-14, max_iter=8, cg_restart=1000, h_init=1.0))
    res = minimize(fg, np.zeros(n), MinParams(method=oracle.CG, tol=1e-14, max_iter=8, cg_restart=1000, h_init=1.0,
                                              cg_beta=variant))
    for (f1, h1, _), (f2, h2, _) in zip(ref.trace, res.trace):
        assert f2 == pytest.approx(f1, rel=1e-11)
        assert h2 == pytest.approx(h1, rel=1e-7)


def test_cg_beta_values_on_orthogonal_gradients():
    g = np.array([1.0, 0.0, 0.0])
    gn = np.array([0.0, 2.0, 0.0])
    r = -g
    # <gn, g> = 0 and <r, gn> = 0: all variants give |gn|^2 / |g|^2 = 4
    for v in (oracle.CG_PRP, oracle.CG_FR, oracle.CG_HS, oracle.CG_PRP_PLUS, oracle.CG_CD, oracle.CG_LS,
              oracle.CG_DY):
        assert oracle.cg_beta(v, g, gn, r) == pytest.approx(4.0, rel=1e-15)
    # a zero denominator restarts
    assert oracle.cg_beta(oracle.CG_HS, g, g, r) == 0.0


def test_ls_par_without_g0_is_exact_on_a_parabola():
    a, b, c = 2.0, -3.0, 0.5
    probes = []

    def fg(x):
        probes.append(float(x[0]))
        return a * x[0] ** 2 + b * x[0] + c, np.array([2 * a * x[0] + b])

    ok, h, f, _, hmin = oracle.ls_par(fg, np.zeros(1), np.ones(1), 1.0, c, 0.0, K=3, g0=False)
    assert probes[:2] == [-0.5, 0.5] and len(probes) == 3
    assert ok and h == pytest.approx(-b / (2 * a), rel=1e-12) and hmin == 0.5


# ------------------------------------------------------------- heavy ball (eq. HB)

def _hb_closed_form(lam, alpha, beta, e0, k):
    """Component of the heavy-ball error after k steps on f = lam e^2 / 2:
    e_{k+1} = (1 + beta - alpha lam) e_k - beta e_{k-1}, e_{-1} = e_0, solved
    through the roots of z^2 - (1 + beta - alpha lam) z + beta = 0."""
    a = 1.0 + beta - alpha * lam
    disc = complex(a * a - 4.0 * beta)
    r1, r2 = (a + disc ** 0.5) / 2.0, (a - disc ** 0.5) / 2.0
    e1 = (1.0 - alpha * lam) * e0
    if abs(r1 - r2) < 1e-12:                 # double root: e_k = (c1 + c2 k) r^k
        c1 = e0
        c2 = e1 / r1 - e0
        return ((c1 + c2 * k) * r1 ** k).real
    c2 = (e1 - r1 * e0) / (r2 - r1)
    c1 = e0 - c2
    return (c1 * r1 ** k + c2 * r2 ** k).real


@pytest.mark.parametrize("alpha,beta", [(0.08, 0.5), (0.15, 0.3), (0.05, 0.9)])
def test_heavy_ball_follows_its_eigen_closed_form(alpha, beta):
    lam = np.array([1.0, 4.0, 10.0])
    x0 = np.array([1.0, -2.0, 0.5])
    r = minimize(quad(lam, np.zeros(3)), x0,
                 MinParams(method=oracle.HB, hb_alpha=alpha, hb_beta=beta, tol=1e-300, max_iter=40))
    assert r.term == oracle.MAX_ITER and r.iters == 40 and r.evals == 41
    for k, (f, h, ev) in enumerate(r.trace, start=1):
        e = np.array([_hb_closed_form(l, alpha, beta, x, k) for l, x in zip(lam, x0)])
        assert f == pytest.approx(0.5 * float(lam @ (e * e)), rel=1e-10, abs=1e-300)
        assert h == alpha and ev == k + 1
    e40 = np.array([_hb_closed_form(l, alpha, beta, x, 40) for l, x in zip(lam, x0)])
    np.testing.assert_allclose(r.x, e40, rtol=1e-9, atol=1e-14)


def test_heavy_ball_without_momentum_is_the_fixed_step_gradient_method():
    lam = np.array([0.5, 2.0, 3.0])
    x0 = np.array([3.0, 1.0, -1.0])
    alpha = 0.3
    r = minimize(quad(lam, np.zeros(3)), x0, MinParams(method=oracle.HB, hb_alpha=alpha, hb_beta=0.0,
                                                        tol=1e-300, max_iter=25))
    np.testing.assert_allclose(r.x, (1.0 - alpha * lam) ** 25 * x0, rtol=1e-12)


def test_heavy_ball_reports_divergence():
    def fg(x):
        return float(np.sum(x ** 4)), 4.0 * x ** 3
    with np.errstate(over="ignore", invalid="ignore"):
        r = minimize(fg, np.array([2.0]), MinParams(method=oracle.HB, hb_alpha=1.0, hb_beta=0.0, max_iter=100))
    assert r.term == oracle.DIVERGED and np.isfinite(r.f) and r.iters < 10


def test_heavy_ball_needs_its_parameters():
    with pytest.raises(ValueError):
        minimize(quad(np.ones(2), np.zeros(2)), np.ones(2), MinParams(method=oracle.HB))


# ------------------------------------------------ optimized gradient method (eq. optim)

def test_ogm_t_sequence():
    t = 1.0
    t1 = oracle.ogm_t_next(t)
    assert t1 == pytest.approx((1.0 + math.sqrt(5.0)) / 2.0, rel=1e-15)
    for k in range(200):
        tn = oracle.ogm_t_next(t)
        assert tn * tn - tn == pytest.approx(t * t, rel=1e-13)
        assert tn >= (k + 2) / 2.0
        t = tn


def _exact_step(A, x, d):
    """x - h d with h minimizing x'Ax/2 along -d (closed form)."""
    g = A @ x
    return x - (float(g @ d) / float(d @ (A @ d))) * d


def test_ogm_first_two_steps_by_hand_on_a_quadratic():
    A = np.array([[3.0, 1.0, 0.0], [1.0, 2.0, 0.5], [0.0, 0.5, 1.0]])
    x0 = np.array([1.0, -1.0, 2.0])
    fg = quad(A, np.zeros(3))
    # h_init = 0.5: the exact steps (1.10, then 0.06) lie inside LS_PAR's
    # window [h1/100, 10 h1], so both line searches are exact on a quadratic
    r = minimize(fg, x0, MinParams(method=oracle.OGM, tol=1e-300, max_iter=2, h_init=0.5))
    assert r.iters == 2
    # iteration 0: y = x0, d = (1 - 1/t1) g0 + (2/t1) g0, an exact step along -g0
    t1 = (1.0 + math.sqrt(5.0)) / 2.0
    g0 = A @ x0
    x1 = _exact_step(A, x0, g0)
    # iteration 1: anchor x0, gradient sum t0 g0 + t1 g1
    t2 = 0.5 * (1.0 + math.sqrt(4.0 * t1 * t1 + 1.0))
    g1 = A @ x1
    y = (1.0 - 1.0 / t2) * x1 + x0 / t2
    d = (1.0 - 1.0 / t2) * g1 + (2.0 / t2) * (g0 + t1 * g1)
    x2 = _exact_step(A, y, d)
    f = lambda x: 0.5 * float(x @ (A @ x))
    assert r.trace[0][0] == pytest.approx(f(x1), rel=1e-11)
    assert r.trace[1][0] == pytest.approx(f(x2), rel=1e-9)
    np.testing.assert_allclose(r.x, x2, rtol=1e-8, atol=1e-12)
    # two evaluations of the first iteration (LS_PAR), three of the second (y, two trials)
    assert [e for _, _, e in r.trace] == [3, 6]


def test_ogm_isotropic_quadratic_one_step():
    x0 = np.array([3.0, -4.0, 1.0])
    # the exact step |x0| = 5.1 lies in LS_PAR's window [h1/100, 10 h1] for h1 = 1
    r = minimize(quad(np.full(3, 2.0), np.zeros(3)), x0, MinParams(method=oracle.OGM, tol=1e-9, h_init=1.0))
    assert r.term == oracle.CONVERGED and r.iters == 1


def test_ogm_converges_on_an_ill_conditioned_quadratic():
    rng = np.random.default_rng(3)
    lam = np.geomspace(1.0, 100.0, 60)
    b = rng.normal(size=60)
    r = minimize(quad(lam, b), np.zeros(60), MinParams(method=oracle.OGM, tol=1e-7, max_iter=2000))
    assert r.term == oracle.CONVERGED
    np.testing.assert_allclose(r.x, b / lam, rtol=0, atol=1e-6)


# ------------------------------------------- CG beta at non-orthogonal gradients

def test_cg_beta_values_by_hand_at_non_orthogonal_gradients():
    """Every beta of section 5.1 at one (g_k, g_{k+1}, d_k) where the seven
    formulas give six different values, each worked out by hand:
    g = (1, 0), g+ = (1, 2), d = (-3, 1), so y = g+ - g = (0, 2),
    <g+, y> = 4, |g+|^2 = 5, |g|^2 = 1, <d, y> = 2, -<d, g> = 3.
    A swapped numerator or denominator between any two variants changes
    the value."""
    g, gn, d = np.array([1.0, 0.0]), np.array([1.0, 2.0]), np.array([-3.0, 1.0])
    expect = {oracle.CG_PRP: 4.0,         # <g+, y> / |g|^2
              oracle.CG_FR: 5.0,          # |g+|^2 / |g|^2
              oracle.CG_HS: 2.0,          # <g+, y> / <d, y>
              oracle.CG_PRP_PLUS: 4.0,    # max(0, PRP)
              oracle.CG_CD: 5.0 / 3.0,    # |g+|^2 / (-<d, g>)
              oracle.CG_LS: 4.0 / 3.0,    # <g+, y> / (-<d, g>)
              oracle.CG_DY: 2.5}          # |g+|^2 / <d, y>
    for v, b in expect.items():
        assert oracle.cg_beta(v, g, gn, d) == b, v


def test_cg_beta_prp_plus_clamps_a_negative_prp():
    """g = (2, 0), g+ = (1, 0.5): y = (-1, 0.5), <g+, y> = -0.75, |g|^2 = 4,
    so PRP = -0.1875 while PRP+ = 0."""
    g, gn, d = np.array([2.0, 0.0]), np.array([1.0, 0.5]), np.array([-2.0, 0.0])
    assert oracle.cg_beta(oracle.CG_PRP, g, gn, d) == -0.1875
    assert oracle.cg_beta(oracle.CG_PRP_PLUS, g, gn, d) == 0.0
    # the same point through the other denominators: <d, y> = 2, -<d, g> = 4
    assert oracle.cg_beta(oracle.CG_HS, g, gn, d) == -0.375
    assert oracle.cg_beta(oracle.CG_LS, g, gn, d) == -0.1875
    assert oracle.cg_beta(oracle.CG_DY, g, gn, d) == 0.625
    assert oracle.cg_beta(oracle.CG_CD, g, gn, d) == 0.3125
    assert oracle.cg_beta(oracle.CG_FR, g, gn, d) == 0.3125


def test_cg_beta_zero_denominators_restart():
    g, gn = np.array([1.0, 0.0]), np.array([1.0, 2.0])
    d_perp_y = np.array([1.0, 0.0])            # <d, y> = 0: HS and DY restart
    assert oracle.cg_beta(oracle.CG_HS, g, gn, d_perp_y) == 0.0
    assert oracle.cg_beta(oracle.CG_DY, g, gn, d_perp_y) == 0.0
    d_perp_g = np.array([0.0, 1.0])            # <d, g> = 0: CD and LS restart
    assert oracle.cg_beta(oracle.CG_CD, g, gn, d_perp_g) == 0.0
    assert oracle.cg_beta(oracle.CG_LS, g, gn, d_perp_g) == 0.0
    z = np.zeros(2)                            # |g| = 0: PRP, FR, PRP+ restart
    for v in (oracle.CG_PRP, oracle.CG_FR, oracle.CG_PRP_PLUS):
        assert oracle.cg_beta(v, z, gn, d_perp_y) == 0.0


# ------------------------------------------------------- LS_PAR branch by branch

def _slice(f):
    """A 1-D objective f(h) along r = e_1 from x = 0, recording its probes."""
    probes = []

    def fg(x):
        h = float(x[0])
        probes.append(h)
        v = f(h)
        return v, np.array([0.0])

    return fg, probes


def test_ls_par_vertex_clamped_at_ten_h1():
    """f(h) = -h + h^2/1024 (f* = 0, slope -1): the first parabola is f
    itself, with vertex 512 h1, so the second trial is clamped to 10 h1."""
    fg, probes = _slice(lambda h: -h + h * h / 1024.0)
    ok, h, f, _, hmin = oracle.ls_par(fg, np.zeros(1), np.ones(1), 1.0, 0.0, -1.0, K=2)
    assert probes == [1.0, 10.0]
    assert ok and h == 10.0 and f == -10.0 + 100.0 / 1024.0 and hmin == 1.0


def test_ls_par_vertex_clamped_at_h1_over_100():
    """f(h) = -h + 128 h^2: vertex at h1/256, clamped up to h1/100."""
    fg, probes = _slice(lambda h: -h + 128.0 * h * h)
    ok, h, f, _, hmin = oracle.ls_par(fg, np.zeros(1), np.ones(1), 1.0, 0.0, -1.0, K=2)
    assert probes == [1.0, 0.01]
    # f(0.01) = -0.01 + 0.0128 > 0 = f*: no decrease, the search fails
    assert not ok and h == 0.0 and f == 0.0 and hmin == 0.01


@pytest.mark.parametrize("curv", [0.0, -1.0])
def test_ls_par_non_convex_first_parabola_grows_the_step(curv):
    """f(h) = -h + curv h^2 with curv <= 0 (a = curv <= 0): the second trial
    is k+ h1."""
    fg, probes = _slice(lambda h: -h + curv * h * h)
    ok, h, f, _, _ = oracle.ls_par(fg, np.zeros(1), np.ones(1), 0.25, 0.0, -1.0, K=2, k_plus=3.0)
    assert probes == [0.25, 0.75]
    assert ok and h == 0.75


def test_ls_par_non_finite_first_trial_shrinks():
    """f = inf beyond h = 0.5 (a clash): the second trial is k- h1."""
    fg, probes = _slice(lambda h: math.inf if h > 0.5 else -h)
    ok, h, f, _, hmin = oracle.ls_par(fg, np.zeros(1), np.ones(1), 1.0, 0.0, -1.0, K=2, k_minus=0.25)
    assert probes == [1.0, 0.25]
    assert ok and h == 0.25 and f == -0.25 and hmin == 0.25


def test_ls_par_third_trial_on_a_concave_slice_takes_the_midpoint():
    """K = 3 on f(h) = -h - h^2: trials 1 and then 2 (a < 0: k+ h1); the
    parabola through the three best points (2, -6), (1, -2), (0, 0) is f
    itself, concave, so the third trial is the midpoint of the best two,
    1.5.  The best trial (h = 2) is returned."""
    fg, probes = _slice(lambda h: -h - h * h)
    ok, h, f, _, hmin = oracle.ls_par(fg, np.zeros(1), np.ones(1), 1.0, 0.0, -1.0, K=3)
    assert probes == [1.0, 2.0, 1.5]
    assert ok and h == 2.0 and f == -6.0 and hmin == 1.0


def test_ls_par_third_trial_vertex_behind_the_base_takes_the_midpoint():
    """K = 3 with G0 on f(h) = h^2 + h, an ascent slice handed a descent
    slope: the parabola through the three best points has its vertex at
    h = -0.5, behind the base point; the search stays on h > 0 and takes the
    midpoint of the best two instead, then fails (no trial is below f*)."""
    fg, probes = _slice(lambda h: h * h + h)
    # slope -1 passed in (as if the gradient said descent): the first
    # parabola through (0, 0), slope -1 and (1, 2) has a = 3 and vertex 1/6
    ok, h, f, _, _ = oracle.ls_par(fg, np.zeros(1), np.ones(1), 1.0, 0.0, -1.0, K=3)
    h2 = min(max(1.0 / 6.0, 0.01), 10.0)
    assert probes[:2] == [1.0, h2]
    # best three: (0, 0), (1/6, 0.1944), (1, 2): their parabola is f itself,
    # vertex -0.5 < 0, so the third trial is the midpoint of 0 and 1/6
    assert probes[2] == 0.5 * (0.0 + h2)
    assert not ok and h == 0.0


def test_ls_par_ties_rank_the_smaller_step_first():
    """Two trials with equal energy: the smaller step wins."""
    vals = {1.0: -1.0, 2.0: -1.0}
    fg, probes = _slice(lambda h: vals[h])
    # f1 = -1 at h1 = 1 with slope -1: a = 0, so the second trial is 2 h1
    ok, h, f, _, _ = oracle.ls_par(fg, np.zeros(1), np.ones(1), 1.0, 0.0, -1.0, K=2)
    assert probes == [1.0, 2.0] and ok and h == 1.0 and f == -1.0


def test_ls_h_equal_energy_keeps_shrinking():
    """LS_H accepts only a strict decrease: on a flat slice f = f* it shrinks
    down to eps_h and fails."""
    fg, probes = _slice(lambda h: 0.0)
    ok, h, f, _ = oracle.ls_h(fg, np.zeros(1), np.ones(1), 1.0, 0.0, 2.0, 0.5, 1e-3)
    assert not ok and h == 0.0
    assert probes == [1.0, 0.5, 0.25, 0.125, 0.0625, 0.03125, 0.015625, 0.0078125, 0.00390625, 0.001953125]


def test_failed_ls_par_falls_back_to_ls_h_from_the_smallest_trial():
    """f(h) = -h + 128 h^2 from h0 = 1: LS_PAR tries 1 and 0.01 and finds no
    decrease (f(0.01) = 0.0028 > 0); the fallback LS_H starts at the smallest
    trial step 0.01, fails there again and halves to 0.005, where
    f = -0.0018 < 0."""
    from oracle.minimize import _search
    fg, probes = _slice(lambda h: -h + 128.0 * h * h)
    ok, h, f, _ = _search(fg, np.zeros(1), np.ones(1), 1.0, 0.0, -1.0, MinParams(method=oracle.LBFGS))
    assert probes == [1.0, 0.01, 0.01, 0.005]
    assert ok and h == 0.005 and f == -0.005 + 128.0 * 0.005 * 0.005
