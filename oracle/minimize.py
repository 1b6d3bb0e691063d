"""Oracle minimizers: line searches and first-order methods of section 5.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy, FP64,
every step in the paper's order.  ``fg(x) -> (f, g)`` is any objective with
its gradient over a flat float64 vector.

Readings where the paper is silent, ambiguous or inconsistent (each one is
the rule the GPU library implements as well):

* every method normalizes its descent direction every iteration (section 5.1
  says so for all algorithms, while Algorithm 3 only shows it at k = 0);
* L-BFGS scales the first-loop result by <s, y>/<y, y> of the newest stored
  pair (Algorithm 3 names a pair that does not exist yet) and its loops run
  over the min(k, m) stored pairs; a pair is stored only if
  <s, y> > eps_mach <y, y>;
* the LS_PAR loop body runs K-2 times, so K trial points in total (K = 2 by
  default: two oracle calls, section 5.2);
* LS_PAR's first parabola: a = (f1 - f* - s0 h1)/h1^2; if f1 is finite and
  a > 0 the second trial is the vertex -s0/(2a) clamped to [h1/100, 10 h1];
  if a <= 0 it is k+ h1; if f1 is not finite it is k- h1;
* LS_PAR's later parabolas go through the three best points; if that parabola
  is degenerate or not convex the midpoint of the two best points is used;
* trials are ranked by (f, h): a non-finite f ranks last, ties go to the
  smaller step; a line search succeeds only on a strict decrease f < f*;
* LS_H keeps halving while f is not strictly below f* (Algorithm 5 tests
  "greater than" in its loop and "less than" on entry);
* GD, CG and L-BFGS fall back to LS_H started from the smallest LS_PAR trial
  step when LS_PAR fails; if that fails too, CG and L-BFGS restart once from
  -g (CG: r = -g; L-BFGS: history cleared), FGM restarts its momentum once
  (x^{k-1} = x^k, theta = 1), and otherwise the run stops with LS_FAILED;
* the first step is h_init = 0.1 A; later line searches start from the last
  accepted step length |h| (section 5.2), and from h_init after a restart;
* LS_PAR with G0 = false starts from the symmetric trials -h0/2, +h0/2 and
  may return a negative step; the LS_H fallback then starts from the
  smallest positive trial step;
* CG uses the usual positive PRP beta = <g+, g+ - g>/|g|^2 by default
  (section 4 prints the beta formulas with a leading minus sign; the other
  variants named in section 5.1 are in ``cg_beta``) and restarts from -g every
  ``cg_restart`` iterations (default: the dimension 3N) and whenever its
  direction is not a descent direction;
* optional FGM variant (off by default): the adaptive restart of O'Donoghue
  and Candes 2015 sets theta back to 1 whenever an iterate has a higher
  energy than the one before it;
* heavy ball (eq. HB) runs as printed: constant alpha and beta, x^{-1} = x^0,
  no line search and no normalization; a non-finite E or gradient at a new
  iterate stops the run with DIVERGED (the last finite iterate is returned);
* the optimized gradient method (eq. optim) replaces 1/L by a line search
  from y^{k+1} along -d^{k+1}/|d^{k+1}|, as the text following the method
  suggests, with the methods' default line search (LS_PAR, then LS_H);
  t_0 = 1 and the anchor x^0 is the start point; E and its gradient are
  evaluated at y^{k+1} unless y^{k+1} is the current point (the anchor is
  the current point right after a (re)start, where the direction is -g);
  when the direction is not a descent direction at y^{k+1} or the line search
  fails, the method restarts at the current point (x^0 := x^k, t := 1, the
  gradient sum := the current gradient); a failure right after a restart
  stops the run with LS_FAILED; the last iterate is returned;
* stop when |grad|_inf < tol at the current point (FGM: at its best point),
  or after max_iter iterations.
"""
from __future__ import annotations

import math
from collections import deque
from dataclasses import dataclass, field

import numpy as np

GD, FGM, CG, LBFGS, HB, OGM = 0, 1, 2, 3, 4, 5
LS_PAR, LS_H = 0, 1
# CG beta variants named in section 5.1 (formulas as collected by Andrei 2008)
CG_PRP, CG_FR, CG_HS, CG_PRP_PLUS, CG_CD, CG_LS, CG_DY = 0, 1, 2, 3, 4, 5, 6
CONVERGED, MAX_ITER, LS_FAILED, NONFINITE_START, DIVERGED = 0, 1, 2, 3, 4
EPS_MACH = float(np.finfo(np.float64).eps)


@dataclass
class MinParams:
    method: int = LBFGS
    m: int = 10
    tol: float = 1e-3
    max_iter: int = 2000
    linesearch: int = -1        # -1: LS_H for FGM, LS_PAR otherwise (section 5.3)
    ls_K: int = 2
    h_init: float = 0.1
    k_plus: float = 2.0
    k_minus: float = 0.5
    eps_h: float = 1e-10
    cg_restart: int = 0         # 0: the dimension of x
    cg_beta: int = CG_PRP
    ls_par_g0: bool = True      # Algorithm 6's G0: use f and the slope at the base point
    fgm_restart: bool = False   # restart FGM's momentum when f(x^{k+1}) > f(x^k)
    hb_alpha: float = 0.0       # heavy ball: step on the gradient (> 0)
    hb_beta: float = 0.0        # heavy ball: momentum in [0, 1)

    def primary_ls(self) -> int:
        if self.linesearch in (LS_PAR, LS_H):
            return self.linesearch
        return LS_H if self.method == FGM else LS_PAR


@dataclass
class MinResult:
    x: np.ndarray
    f: float
    g: np.ndarray
    term: int
    iters: int
    evals: int
    trace: list = field(default_factory=list)   # per accepted iteration: (f, h, evals)


def _rank(f: float, h: float):
    return (f if math.isfinite(f) else math.inf, h)


def _finite_point(f, g) -> bool:
    return math.isfinite(f) and bool(np.all(np.isfinite(g)))


# ---------------------------------------------------------------- line searches

def _parabola3_vertex(p0, p1, p2):
    """Vertex of the parabola through three (h, f) points, or None if the
    parabola is degenerate or not convex."""
    (ha, fa), (hb, fb), (hc, fc) = p0, p1, p2
    if not (math.isfinite(fa) and math.isfinite(fb) and math.isfinite(fc)):
        return None
    if ha == hb or hb == hc or ha == hc:
        return None
    d1 = (fb - fa) / (hb - ha)
    d2 = ((fc - fb) / (hc - hb) - d1) / (hc - ha)
    if not (d2 > 0.0) or not math.isfinite(d2):
        return None
    h = 0.5 * (ha + hb) - d1 / (2.0 * d2)
    return h if math.isfinite(h) else None


def ls_par(fg, x, r, h0, f_star, s0, K=2, k_plus=2.0, k_minus=0.5, g0=True):
    """LS_PAR, Algorithm 6.  With g0 (G0 = true) the first parabola uses f* and
    the slope s0 = <grad f(x), r>; without it the first two trials are the
    symmetric steps -h0/2 and +h0/2.  Returns (ok, h, f, g, smallest positive
    trial step or None)."""
    trials = []

    def probe(h):
        f, g = fg(x + h * r)
        trials.append((h, f, g))
        return f

    if g0:
        h1 = h0
        f1 = probe(h1)
        # parabola through (0, f*) with slope s0 and through (h1, f1)
        if math.isfinite(f1):
            a = (f1 - f_star - s0 * h1) / (h1 * h1)
            if a > 0.0:
                h2 = min(max(-s0 / (2.0 * a), 0.01 * h1), 10.0 * h1)
            else:
                h2 = k_plus * h1
        else:
            h2 = k_minus * h1
        probe(h2)
    else:
        probe(-0.5 * h0)
        probe(0.5 * h0)
    for _ in range(K - 2):
        pts = sorted([(0.0, f_star)] + [(h, f) for h, f, _ in trials], key=lambda p: _rank(p[1], p[0]))
        h3 = _parabola3_vertex(pts[0], pts[1], pts[2])
        # with G0 the search runs along the descent direction only (h > 0);
        # the symmetric start of G0 = false may also step backwards
        if h3 is None or h3 == 0.0 or (g0 and h3 < 0.0):
            h3 = 0.5 * (pts[0][0] + pts[1][0])
        probe(h3)
    pos = [h for h, _, _ in trials if h > 0.0]
    h_min = min(pos) if pos else None
    h, f, g = min(trials, key=lambda t: _rank(t[1], t[0]))
    if f < f_star:
        return True, h, f, g, h_min
    return False, 0.0, f_star, None, h_min


def ls_h(fg, x, r, h0, f_star, k_plus=2.0, k_minus=0.5, eps_h=1e-10):
    """LS_H, Algorithm 5.  Returns (ok, h, f, g)."""
    f0, g0 = fg(x + h0 * r)
    if f0 < f_star:
        h1 = k_plus * h0
        f1, g1 = fg(x + h1 * r)
        if f1 < f0:
            return True, h1, f1, g1
        return True, h0, f0, g0
    h2 = k_minus * h0
    f2, g2 = fg(x + h2 * r)
    while not (f2 < f_star):
        h2 = k_minus * h2
        if h2 <= eps_h:
            return False, 0.0, f_star, None
        f2, g2 = fg(x + h2 * r)
    return True, h2, f2, g2


def _search(fg, x, r, h0, f_star, s0, p: MinParams):
    """The method's line search: the primary one, and LS_H from the smallest
    trial step if the primary LS_PAR fails."""
    if p.primary_ls() == LS_H:
        return ls_h(fg, x, r, h0, f_star, p.k_plus, p.k_minus, p.eps_h)
    ok, h, f, g, h_min = ls_par(fg, x, r, h0, f_star, s0, p.ls_K, p.k_plus, p.k_minus, p.ls_par_g0)
    if ok or h_min is None:
        return ok, h, f, g
    return ls_h(fg, x, r, h_min, f_star, p.k_plus, p.k_minus, p.eps_h)


# ------------------------------------------------------------------ directions

def lbfgs_direction(g, hist):
    """Algorithm 3 (unnormalized; the caller normalizes)."""
    r = -g
    if not hist:
        return r
    alphas = []
    for s, y, rho in reversed(hist):              # newest -> oldest
        a = rho * float(np.dot(s, r))
        r = r - a * y
        alphas.append(a)
    s_new, y_new, _ = hist[-1]
    r = (float(np.dot(s_new, y_new)) / float(np.dot(y_new, y_new))) * r
    for (s, y, rho), a in zip(hist, reversed(alphas)):   # oldest -> newest
        b = rho * float(np.dot(y, r))
        r = r + (a - b) * s
    return r


def cg_beta(variant, g, g_new, r):
    """beta_k of the CG variants of section 5.1 (g = g_k, g_new = g_{k+1},
    r = d_k the previous unnormalized direction, y = g_new - g).  A zero or
    non-finite denominator gives beta = 0 (a restart)."""
    y = g_new - g
    gg = float(np.dot(g, g))
    if variant == CG_PRP:
        num, den = float(np.dot(g_new, y)), gg
    elif variant == CG_FR:
        num, den = float(np.dot(g_new, g_new)), gg
    elif variant == CG_HS:
        num, den = float(np.dot(g_new, y)), float(np.dot(r, y))
    elif variant == CG_PRP_PLUS:
        num, den = max(0.0, float(np.dot(g_new, y))), gg
    elif variant == CG_CD:
        num, den = float(np.dot(g_new, g_new)), -float(np.dot(r, g))
    elif variant == CG_LS:
        num, den = float(np.dot(g_new, y)), -float(np.dot(r, g))
    elif variant == CG_DY:
        num, den = float(np.dot(g_new, g_new)), float(np.dot(r, y))
    else:
        raise ValueError(f"unknown CG variant {variant}")
    if den == 0.0:
        return 0.0
    beta = num / den
    return beta if math.isfinite(beta) else 0.0


def _ginf(g) -> float:
    return float(np.max(np.abs(g))) if g.size else 0.0


# --------------------------------------------------------------------- methods

def _gd_cg_lbfgs(fg, x, f, g, p: MinParams, res: MinResult):
    n = x.size
    restart_every = p.cg_restart if p.cg_restart > 0 else n
    h_prev = p.h_init
    hist = deque()
    r = -g                       # CG's running direction (Algorithm 2)
    steepest = True
    k = 0
    while True:
        if _ginf(g) < p.tol:
            res.term = CONVERGED
            break
        if k == p.max_iter:
            res.term = MAX_ITER
            break
        if p.method == GD:
            r = -g
            steepest = True
        elif p.method == LBFGS:
            r = lbfgs_direction(g, hist)
            steepest = not hist
        if float(np.dot(g, r)) >= 0.0:           # not a descent direction
            r = -g
            steepest = True
            hist.clear()
        rn = r / float(np.linalg.norm(r))
        ok, h, f_new, g_new = _search(fg, x, rn, h_prev, f, float(np.dot(g, rn)), p)
        if not ok:
            if not steepest and p.method in (CG, LBFGS):
                r = -g
                steepest = True
                hist.clear()
                h_prev = p.h_init
                continue
            res.term = LS_FAILED
            break
        x_new = x + h * rn
        if p.method == LBFGS:
            s = x_new - x
            y = g_new - g
            sy = float(np.dot(s, y))
            if sy > EPS_MACH * float(np.dot(y, y)):
                hist.append((s, y, 1.0 / sy))
                if len(hist) > p.m:
                    hist.popleft()
        elif p.method == CG:
            beta = cg_beta(p.cg_beta, g, g_new, r)
            if (k + 1) % restart_every == 0:
                r = -g_new
                steepest = True
            else:
                r = -g_new + beta * r
                steepest = False
        x, f, g = x_new, f_new, g_new
        h_prev = abs(h)
        k += 1
        res.trace.append((f, h, res.evals))
    res.x, res.f, res.g, res.iters = x, f, g, k


def fgm_coefficients(theta_prev: float):
    """theta_k and beta_k of Algorithm 1 from theta_{k-1}."""
    theta = 0.5 * theta_prev * (math.sqrt(theta_prev * theta_prev + 4.0) - theta_prev)
    beta = theta_prev * (1.0 - theta_prev) / (theta_prev * theta_prev + theta)
    return theta, beta


def _fgm(fg, x, f, g, p: MinParams, res: MinResult):
    """Algorithm 1; returns the best point seen."""
    x_prev = x
    theta_prev = 1.0
    best = (x, f, g)
    h_prev = p.h_init
    k = 0
    while True:
        if _ginf(best[2]) < p.tol:
            res.term = CONVERGED
            break
        if k == p.max_iter:
            res.term = MAX_ITER
            break
        theta, beta = fgm_coefficients(theta_prev)
        if beta > 0.0:
            w = x + beta * (x - x_prev)
            fw, gw = fg(w)
        else:
            w, fw, gw = x, f, g
        ok = _finite_point(fw, gw) and float(np.linalg.norm(gw)) > 0.0
        if ok:
            r = -gw / float(np.linalg.norm(gw))
            ok, h, f_new, g_new = _search(fg, w, r, h_prev, fw, float(np.dot(gw, r)), p)
        if not ok:
            if beta > 0.0:                     # restart the momentum once
                x_prev = x
                theta_prev = 1.0
                h_prev = p.h_init
                continue
            res.term = LS_FAILED
            break
        x_new = w + h * r
        f_old = f
        x_prev, x, f, g = x, x_new, f_new, g_new
        theta_prev = theta
        if p.fgm_restart and f_new > f_old:
            theta_prev = 1.0                   # function-value restart: no momentum next

        h_prev = abs(h)
        if f_new < best[1]:
            best = (x_new, f_new, g_new)
        k += 1
        res.trace.append((f_new, h, res.evals))
    res.x, res.f, res.g, res.iters = best[0], best[1], best[2], k


def _heavy_ball(fg, x, f, g, p: MinParams, res: MinResult):
    """Eq. HB: x^{k+1} = x^k - alpha grad f(x^k) + beta (x^k - x^{k-1})."""
    x_prev = x
    k = 0
    while True:
        if _ginf(g) < p.tol:
            res.term = CONVERGED
            break
        if k == p.max_iter:
            res.term = MAX_ITER
            break
        x_new = x - p.hb_alpha * g + p.hb_beta * (x - x_prev)
        f_new, g_new = fg(x_new)
        if not _finite_point(f_new, g_new):
            res.term = DIVERGED
            break
        x_prev, x, f, g = x, x_new, f_new, g_new
        k += 1
        res.trace.append((f, p.hb_alpha, res.evals))
    res.x, res.f, res.g, res.iters = x, f, g, k


def ogm_t_next(t: float) -> float:
    """t_{k+1} of eq. optim from t_k."""
    return 0.5 * (1.0 + math.sqrt(4.0 * t * t + 1.0))


def _ogm(fg, x, f, g, p: MinParams, res: MinResult):
    """Eq. optim with the line search in place of 1/L:
    y^{k+1} = (1 - 1/t_{k+1}) x^k + x^0 / t_{k+1},
    d^{k+1} = (1 - 1/t_{k+1}) g(x^k) + (2/t_{k+1}) sum_{j<=k} t_j g(x^j),
    x^{k+1} = y^{k+1} + h r with r = -d^{k+1}/|d^{k+1}|."""
    x0 = x                      # anchor
    t = 1.0                     # t_0
    S = g.copy()                # sum_j t_j g(x^j) = t_0 g(x^0)
    h_prev = p.h_init
    k = 0
    while True:
        if _ginf(g) < p.tol:
            res.term = CONVERGED
            break
        if k == p.max_iter:
            res.term = MAX_ITER
            break
        t_next = ogm_t_next(t)
        th = 1.0 / t_next
        d = (1.0 - th) * g + (2.0 * th) * S
        at_anchor = x0 is x
        if at_anchor:
            y, fy, gy = x, f, g
        else:
            y = (1.0 - th) * x + th * x0
            fy, gy = fg(y)
        dn = float(np.linalg.norm(d))
        ok = _finite_point(fy, gy) and dn > 0.0 and math.isfinite(dn)
        if ok:
            r = -d / dn
            s0 = float(np.dot(gy, r))
            ok = s0 < 0.0
        if ok:
            ok, h, f_new, g_new = _search(fg, y, r, h_prev, fy, s0, p)
        if not ok:
            if not at_anchor:           # restart at the current point
                x0, t, S = x, 1.0, g.copy()
                h_prev = p.h_init
                continue
            res.term = LS_FAILED
            break
        x = y + h * r
        f, g = f_new, g_new
        t = t_next
        S = S + t * g
        h_prev = abs(h)
        k += 1
        res.trace.append((f, h, res.evals))
    res.x, res.f, res.g, res.iters = x, f, g, k


def minimize(fg, x0, p: MinParams | None = None) -> MinResult:
    """Local minimization from x0 (section 2: the local minimum reachable from
    a good start)."""
    p = p or MinParams()
    res = MinResult(x=None, f=math.nan, g=None, term=MAX_ITER, iters=0, evals=0)

    def counted(x):
        res.evals += 1
        f, g = fg(x)
        return float(f), np.asarray(g, dtype=np.float64).ravel()

    x = np.array(x0, dtype=np.float64).ravel()
    f, g = counted(x)
    if not _finite_point(f, g):
        res.x, res.f, res.g, res.term = x, f, g, NONFINITE_START
        return res
    if p.method == FGM:
        _fgm(counted, x, f, g, p, res)
    elif p.method in (GD, CG, LBFGS):
        _gd_cg_lbfgs(counted, x, f, g, p, res)
    elif p.method == HB:
        if not (p.hb_alpha > 0.0 and 0.0 <= p.hb_beta < 1.0):
            raise ValueError("heavy ball needs hb_alpha > 0 and 0 <= hb_beta < 1")
        _heavy_ball(counted, x, f, g, p, res)
    elif p.method == OGM:
        _ogm(counted, x, f, g, p, res)
    else:
        raise ValueError(f"unknown method {p.method}")
    return res
