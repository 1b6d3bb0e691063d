// On-device decision logic of the minimizer: line searches LS_PAR and LS_H
// (section 5.2, Algorithms 6 and 5) and the methods GD (section 4, eq. 4),
// FGM (Algorithm 1), CG with the Polak-Ribiere-Polyak beta (Algorithm 2) and
// L-BFGS (Algorithms 3 and 4), written as a state machine that advances once
// per energy+gradient evaluation and once per accepted step.  It runs in one
// thread of the last workgroup of the finalize or accept kernel (the L-BFGS
// coefficient algebra runs on that whole workgroup just before it); all its
// state lives in the control block, so iterates never go back to the host.
//
// Readings where the paper is silent (identical to the rules of the CPU
// reference implementation used to check this library):
//  - every method normalizes its direction every iteration;
//  - L-BFGS scales by <s,y>/<y,y> of the newest stored pair, stores a pair
//    only if <s,y> > eps_mach <y,y>, and runs its two loops over the
//    min(k, m) stored pairs; here the two loops run on the coefficients of
//    the direction in the basis {s_i, y_i, g} with the Gram matrix of that
//    basis (the vector-free form of the two-loop recursion, Chen et al. 2014),
//    which gives the same direction in exact arithmetic;
//  - LS_PAR takes K trial points (its loop body runs K-2 times); first
//    parabola a = (f1 - f* - s0 h1)/h1^2, vertex -s0/(2a) clamped to
//    [h1/100, 10 h1] if a > 0, k+ h1 if a <= 0, k- h1 if f1 is not finite;
//    later parabolas through the three best points, midpoint of the two best
//    if that parabola is degenerate or not convex;
//  - trials rank by (f, h) with non-finite f last; success needs f < f*;
//  - LS_H shrinks while f is not strictly below f*;
//  - GD, CG and L-BFGS fall back to LS_H from the smallest LS_PAR trial step;
//    then CG and L-BFGS restart once from -g, FGM restarts its momentum once;
//  - h starts at h_init and then at the last accepted step, h_init again
//    after a restart;
//  - CG: beta = <g+, g+ - g>/|g|^2 by default (or another variant named in
//    section 5.1), restart every cg_restart iterations and whenever the
//    direction is not a descent direction;
//  - LS_PAR without G0 starts from -h0/2, +h0/2 and may step backwards; the
//    next search starts from |h|;
//  - stop when |g|_inf < tol at the current point (FGM: the best point) or
//    after max_iter iterations.
// In FF_FP32_ACC64 mode the run switches to FP64 evaluations once both line
// searches fail in FP32, an accepted FP32 step lowers E by less than
// 2^-23 |E|, or |g|_inf < 10 tol; it decides convergence only on FP64
// gradients and re-evaluates the returned point in FP64.
#pragma once
#include "ff_internal.h"

namespace ff {

enum { M_GD = 0, M_FGM = 1, M_CG = 2, M_LBFGS = 3, M_HB = 4, M_OGM = 5 };
enum { T_CONVERGED = 0, T_MAX_ITER = 1, T_LS_FAILED = 2, T_NONFINITE = 3, T_DIVERGED = 4 };
enum { P_FP64 = 0, P_FP32 = 1 };

constexpr double kEpsMach = 2.220446049250313e-16;

__device__ inline bool finite_d(double v) { return isfinite(v); }

__device__ inline double rank_key(double f) { return isfinite(f) ? f : __builtin_inf(); }

__device__ inline bool rank_less(double f1, double h1, double f2, double h2) {
    const double k1 = rank_key(f1), k2 = rank_key(f2);
    return k1 < k2 || (k1 == k2 && h1 < h2);
}

__device__ inline int alloc_slot(const Ctl* c) {
    for (int s = 0; s < kNumSlots; ++s) {
        if (s == c->cur || s == c->prev_x || s == c->best || s == c->w || s == c->ls_base || s == c->ls_best)
            continue;
        return s;
    }
    return -1;   // cannot happen: at most six roles are live
}

// ------------------------------------------------------------ requests
__device__ inline void request_eval(Ctl* c, int mode, int target, int want_slope) {
    c->action = ACT_EVAL;
    c->point_mode = mode;
    c->target = target;
    c->prec = c->prec_now;
    c->want_slope = want_slope;
    c->slope_slot = mode == PM_OGM_Y ? target : c->base;
    c->accept = 0;
}

// The system needs no FP32 evaluation any more (it switched to FP64 or it
// stops): counted once per ff_minimize call, so that the host can leave the
// FP32 pair kernel out of the iteration graph once every system is there.
__device__ inline void release_fp32(Ctl* c) {
    if (c->fp32_released) return;
    c->fp32_released = 1;
    if (c->batch) atomicAdd(&c->batch->n_fp64, 1u);
}

__device__ inline void finish_done(Ctl* c, int slot) {
    release_fp32(c);
    c->result_slot = slot;
    c->phase = PH_DONE;
    c->done = 1;
    c->action = ACT_NONE;
    c->accept = 0;
    if (c->batch) atomicAdd(&c->batch->n_done, 1u);
}

__device__ inline void finish(Ctl* c, int term) {
    release_fp32(c);
    c->term = term;
    const int slot = (c->p.method == M_FGM && c->best >= 0) ? c->best : c->cur;
    if (c->p.precision == P_FP32 && c->p.certify && term != T_NONFINITE && c->slot_prec[slot] != P_FP64) {
        c->prec_now = P_FP64;
        c->phase = PH_CERTIFY;
        c->result_slot = slot;
        request_eval(c, PM_USE, slot, 0);
        return;
    }
    finish_done(c, slot);
}

__device__ inline void lbfgs_clear(Ctl* c);

// OGM restart at the current point: anchor x^0 := x^k, t := 1, and the
// weighted gradient sum := the current gradient.
__device__ inline void ogm_restart(Ctl* c) {
    c->prev_x = c->cur;
    c->ogm_t = 1.0;
    c->ogm_s_anchor = 1;
    c->h_prev = c->p.h_init;
}

// Re-evaluate `slot` in FP64 (precision escalation of the mixed mode).  The
// stored L-BFGS pairs and the CG direction were built from FP32 gradients
// and their products with g would no longer match the FP64 gradient, so the
// next direction starts again from -g.
__device__ inline void escalate(Ctl* c, int slot) {
    release_fp32(c);
    c->escalated = 1;
    c->prec_now = P_FP64;
    c->phase = PH_REEVAL64;
    c->steepest = 1;
    // a restart: the next search starts from h_init, not from the last
    // FP32 step (which may have shrunk to the FP32 noise level)
    c->h_prev = c->p.h_init;
    lbfgs_clear(c);
    if (c->p.method == M_OGM) ogm_restart(c);
    request_eval(c, PM_USE, slot, 0);
}

// ----------------------------------------------------------- line search
__device__ inline void ls_trial(Ctl* c, double h, bool first) {
    c->ls_hcur = h;
    c->h = h;
    c->base = c->ls_base;
    const int t = alloc_slot(c);
    request_eval(c, first ? PM_DIR_TRIAL : PM_TRIAL, t, first ? 1 : 0);
}

__device__ inline void ls_start(Ctl* c, int base, double h0, int kind, bool first) {
    c->phase = PH_LS;
    c->ls_kind = kind;
    c->ls_base = base;
    c->ls_fstar = c->e[base];
    c->ls_h0 = h0;
    c->ls_best = -1;
    c->ls_ntrials = 0;
    c->ls_hmin = __builtin_inf();
    c->ls_hstage = LSH_F0;
    // LS_PAR without G0 starts from the symmetric trials -h0/2, +h0/2
    ls_trial(c, (kind == LSK_PAR && !c->p.ls_g0) ? -0.5 * h0 : h0, first);
}

__device__ void ls_success(Ctl* c, int slot, double h);
__device__ void ls_failed(Ctl* c);

__device__ inline double parabola3_vertex(double ha, double fa, double hb, double fb, double hc, double fc,
                                          bool& ok) {
    ok = false;
    if (!(isfinite(fa) && isfinite(fb) && isfinite(fc))) return 0.0;
    if (ha == hb || hb == hc || ha == hc) return 0.0;
    const double d1 = (fb - fa) / (hb - ha);
    const double d2 = ((fc - fb) / (hc - hb) - d1) / (hc - ha);
    if (!(d2 > 0.0) || !isfinite(d2)) return 0.0;
    const double h = 0.5 * (ha + hb) - d1 / (2.0 * d2);
    ok = isfinite(h);
    return h;
}

__device__ inline void ls_after_trial(Ctl* c) {
    const int t = c->target;
    const double f = c->e[t];
    const double h = c->ls_hcur;
    if (c->ls_kind == LSK_PAR) {
        const int n = c->ls_ntrials;
        c->ls_th[n] = h;
        c->ls_tf[n] = f;
        c->ls_ntrials = n + 1;
        if (h > 0.0) c->ls_hmin = fmin(c->ls_hmin, h);
        if (c->ls_best < 0 || rank_less(f, h, c->e[c->ls_best], c->ls_th[kMaxLsTrials])) {
            c->ls_best = t;
            c->ls_th[kMaxLsTrials] = h;       // step of the best trial
        }
        if (c->ls_ntrials == 1 && !c->p.ls_g0) {
            ls_trial(c, 0.5 * c->ls_h0, false);
            return;
        }
        if (c->ls_ntrials == 1) {
            const double s0 = c->slope, fs = c->ls_fstar;
            double h2;
            if (isfinite(f)) {
                const double a = (f - fs - s0 * h) / (h * h);
                if (a > 0.0)
                    h2 = fmin(fmax(-s0 / (2.0 * a), 0.01 * h), 10.0 * h);
                else
                    h2 = c->p.k_plus * h;
            } else {
                h2 = c->p.k_minus * h;
            }
            ls_trial(c, h2, false);
            return;
        }
        if (c->ls_ntrials < c->p.ls_K) {
            // three best of {(0, f*)} and the trials, ranked by (f, h)
            double bh[3], bf[3];
            int nb = 0;
            bool used[kMaxLsTrials + 1] = {};
            const int total = c->ls_ntrials + 1;
            for (int r = 0; r < 3; ++r) {
                int pick = -1;
                double ph = 0.0, pf = 0.0;
                for (int q = 0; q < total; ++q) {
                    if (used[q]) continue;
                    const double qh = q == 0 ? 0.0 : c->ls_th[q - 1];
                    const double qf = q == 0 ? c->ls_fstar : c->ls_tf[q - 1];
                    if (pick < 0 || rank_less(qf, qh, pf, ph)) { pick = q; ph = qh; pf = qf; }
                }
                used[pick] = true;
                bh[nb] = ph; bf[nb] = pf; ++nb;
            }
            bool ok;
            double h3 = parabola3_vertex(bh[0], bf[0], bh[1], bf[1], bh[2], bf[2], ok);
            // with G0 the search runs along the descent direction only (h > 0)
            if (!ok || h3 == 0.0 || (c->p.ls_g0 && h3 < 0.0)) h3 = 0.5 * (bh[0] + bh[1]);
            ls_trial(c, h3, false);
            return;
        }
        const int b = c->ls_best;
        if (c->e[b] < c->ls_fstar) {
            ls_success(c, b, c->ls_th[kMaxLsTrials]);
        } else if (!c->ls_fallback_done && isfinite(c->ls_hmin)) {
            // LS_H from the smallest trial step, same base and direction
            c->ls_fallback_done = 1;
            const double h0 = c->ls_hmin;
            c->ls_best = -1;
            c->ls_kind = LSK_H;
            c->ls_hstage = LSH_F0;
            c->ls_h0 = h0;
            ls_trial(c, h0, false);
        } else {
            ls_failed(c);
        }
        return;
    }
    // LS_H
    const double fs = c->ls_fstar;
    if (c->ls_hstage == LSH_F0) {
        if (f < fs) {
            c->ls_best = t;
            c->ls_hstage = LSH_F1;
            ls_trial(c, c->p.k_plus * h, false);
        } else {
            c->ls_hstage = LSH_SHRINK;
            ls_trial(c, c->p.k_minus * h, false);
        }
    } else if (c->ls_hstage == LSH_F1) {
        if (f < c->e[c->ls_best]) ls_success(c, t, h);
        else ls_success(c, c->ls_best, c->ls_h0);
    } else {
        if (f < fs) {
            ls_success(c, t, h);
        } else {
            const double h2 = c->p.k_minus * h;
            if (h2 <= c->p.eps_h) ls_failed(c);
            else ls_trial(c, h2, false);
        }
    }
}

// ------------------------------------------------------------- directions
__device__ inline int ring_slot(const Ctl* c, int i) {
    const int q = c->hist_head + i;
    return q >= c->hist_m ? q - c->hist_m : q;
}
__device__ inline int gpos_s(int slot) { return slot; }
__device__ inline int gpos_y(int slot) { return kMaxM + slot; }
constexpr int kGposG = 2 * kMaxM;
__device__ inline double& gram_at(Ctl* c, int a, int b) { return c->gram[a * kGramDim + b]; }

__device__ inline void lbfgs_clear(Ctl* c) {
    c->hist_n = 0;
    c->hist_head = 0;
    c->hist_m = c->p.m;
    c->lb_ready = 0;
    c->spare_s = V_S0;
    c->spare_y = V_Y0;
    c->spare_s_next = V_S0 + 1;
    c->spare_y_next = V_Y0 + 1;
}

__device__ inline void set_steepest(Ctl* c) {
    c->n_terms = 1;
    c->term_vec[0] = V_G0 + c->cur;
    c->term_coef[0] = -1.0;
    c->dir_scale = sqrt(c->g2[c->cur]);
    c->steepest = 1;
}

// Starts the next iteration at the current point.  For L-BFGS with stored
// pairs the direction's terms were filled by the workgroup step that ran
// just before (lb_ready); they are used here or dropped.
__device__ inline void begin_iteration(Ctl* c) {
    const MinParamsDev& p = c->p;
    const int lb_ready = c->lb_ready;
    c->lb_ready = 0;
    c->accept = 0;
    c->w = -1;
    c->ls_base = -1;
    c->ls_best = -1;
    const int pt = (p.method == M_FGM) ? c->best : c->cur;
    if (c->ginf[pt] < p.tol) {
        if (p.precision == P_FP32 && c->slot_prec[pt] != P_FP64) { escalate(c, pt); return; }
        finish(c, T_CONVERGED);
        return;
    }
    if (c->iters >= c->iters_limit) { finish(c, T_MAX_ITER); return; }
    if (p.precision == P_FP32 && !c->escalated && (c->ginf[c->cur] < 10.0 * p.tol || c->stall32)) {
        escalate(c, c->cur);
        return;
    }
    c->write_r = 0;
    switch (p.method) {
    case M_GD:
        set_steepest(c);
        break;
    case M_CG:
        if (!c->steepest) {
            const double beta = c->cg_beta;
            const double gr = -c->g2[c->cur] + beta * c->r_dot_g_old;   // <g, -g + beta r_old>
            if (gr < 0.0) {
                c->n_terms = 2;
                c->term_vec[0] = V_G0 + c->cur; c->term_coef[0] = -1.0;
                c->term_vec[1] = V_R;            c->term_coef[1] = beta;
                const double n2 = c->g2[c->cur] - 2.0 * beta * c->r_dot_g_old + beta * beta * c->r_norm2;
                c->dir_scale = sqrt(n2);
                c->r_norm2 = n2;
            } else {
                set_steepest(c);
                c->r_norm2 = c->g2[c->cur];
            }
        } else {
            set_steepest(c);
            c->r_norm2 = c->g2[c->cur];
        }
        c->write_r = 1;
        break;
    case M_LBFGS:
        if (c->hist_n > 0 && lb_ready == 1) {
            c->steepest = 0;
        } else {
            lbfgs_clear(c);
            set_steepest(c);
        }
        break;
    case M_HB: {
        // eq. HB: x^{k+1} = x^k - alpha g^k + beta (x^k - x^{k-1}), no line search
        const int t = alloc_slot(c);
        c->base = c->cur;
        c->prev = c->prev_x;
        c->h = p.hb_alpha;
        c->beta = p.hb_beta;
        c->phase = PH_HB;
        request_eval(c, PM_HB, t, 0);
        return;
    }
    case M_OGM: {
        // eq. optim: d = (1 - 1/t+) g^k + (2/t+) S, S = sum_j t_j g^j; the search
        // runs from y = (1 - 1/t+) x^k + x^0 / t+ along r = -d/|d|
        const double t_next = 0.5 * (1.0 + sqrt(4.0 * c->ogm_t * c->ogm_t + 1.0));
        const double th = 1.0 / t_next;
        const double a = 1.0 - th, b = 2.0 * th;
        const double gg = c->g2[c->cur];
        const double gS = c->ogm_s_anchor ? gg : c->ogm_gS;
        const double SS = c->ogm_s_anchor ? gg : c->ogm_SS;
        c->ogm_t_next = t_next;
        c->n_terms = 2;
        c->term_vec[0] = V_G0 + c->cur;
        c->term_coef[0] = -a;
        c->term_vec[1] = c->ogm_s_anchor ? V_G0 + c->prev_x : V_R;
        c->term_coef[1] = -b;
        c->dir_scale = sqrt(a * a * gg + 2.0 * a * b * gS + b * b * SS);
        c->steepest = c->prev_x == c->cur;
        if (c->prev_x != c->cur) {
            c->w = alloc_slot(c);
            c->base = c->cur;
            c->prev = c->prev_x;
            c->beta = th;
            c->phase = PH_OGM_Y;
            request_eval(c, PM_OGM_Y, c->w, 1);     // E, grad E and <grad E(y), r> at y
            return;
        }
        break;    // the anchor is the current point: y = x^k, r = -g/|g|
    }
    case M_FGM: {
        const double tp = c->theta_prev;
        const double theta = 0.5 * tp * (sqrt(tp * tp + 4.0) - tp);
        const double beta = tp * (1.0 - tp) / (tp * tp + theta);
        c->fgm_theta = theta;
        c->fgm_beta = beta;
        if (beta > 0.0) {
            c->w = alloc_slot(c);
            c->beta = beta;
            c->base = c->cur;
            c->prev = c->prev_x;
            c->phase = PH_MOMENTUM;
            request_eval(c, PM_MOMENTUM, c->w, 0);
            return;
        }
        c->w = c->cur;
        set_steepest(c);   // direction -g(w) with w = x^k
        break;
    }
    }
    const int primary = p.linesearch == 1 || (p.linesearch < 0 && p.method == M_FGM) ? LSK_H : LSK_PAR;
    c->ls_fallback_done = primary == LSK_H;
    ls_start(c, p.method == M_FGM ? c->w : c->cur, c->h_prev, primary, true);
}

__device__ inline void fgm_after_momentum(Ctl* c) {
    const int w = c->target;
    const bool ok = isfinite(c->e[w]) && isfinite(c->g2[w]) && c->g2[w] > 0.0;
    if (!ok) { ls_failed(c); return; }
    c->n_terms = 1;
    c->term_vec[0] = V_G0 + w;
    c->term_coef[0] = -1.0;
    c->dir_scale = sqrt(c->g2[w]);
    c->write_r = 0;
    const int primary = c->p.linesearch == 0 ? LSK_PAR : LSK_H;
    c->ls_fallback_done = primary == LSK_H;
    ls_start(c, w, c->h_prev, primary, true);
}

__device__ void ls_success(Ctl* c, int slot, double h) {
    // FP32 mode: a decrease below 2^-23 |E| (twice the FP32 unit roundoff;
    // the measured FP32 error of E is about 1e-7 |E|) cannot be told from
    // rounding, so the next iteration switches to FP64
    if (c->p.precision == P_FP32 && !c->escalated && c->ls_base >= 0 && c->slot_prec[slot] == P_FP32) {
        const double f0 = c->e[c->ls_base];
        if (f0 - c->e[slot] < fabs(f0) * 0x1p-23) c->stall32 = 1;
    }
    c->h_prev = fabs(h);
    c->accept_h = h;
    c->accept = 1;
    c->acc_new = slot;
    c->acc_old = c->ls_base;
    // L-BFGS: the new pair's own products, then one row per stored pair;
    // CG: its beta products; OGM: the update of its gradient sum
    c->acc_rows = c->p.method == M_LBFGS ? c->hist_n + 1
                : (c->p.method == M_CG || c->p.method == M_OGM ? 1 : 0);
    c->action = ACT_NONE;
}

__device__ void ls_failed(Ctl* c) {
    const MinParamsDev& p = c->p;
    if (p.precision == P_FP32 && !c->escalated) {
        c->ls_base = -1; c->ls_best = -1;
        escalate(c, c->cur);
        return;
    }
    if ((p.method == M_CG || p.method == M_LBFGS) && !c->steepest) {
        c->steepest = 1;
        lbfgs_clear(c);
        c->h_prev = p.h_init;
        begin_iteration(c);
        return;
    }
    if (p.method == M_OGM && c->prev_x != c->cur) {
        ogm_restart(c);
        begin_iteration(c);
        return;
    }
    if (p.method == M_FGM && c->fgm_beta > 0.0) {
        c->prev_x = c->cur;
        c->theta_prev = 1.0;
        c->h_prev = p.h_init;
        begin_iteration(c);
        return;
    }
    finish(c, T_LS_FAILED);
}

// beta of the CG variants (section 5.1) from |g|^2, |g+|^2, <g+,g>, <g+,d>,
// <d,g>; y = g+ - g.  A zero or non-finite denominator gives 0 (a restart).
__device__ inline double cg_beta(int variant, double gg, double gngn, double gng, double gnd, double dg) {
    const double gny = gngn - gng;        // <g+, y>
    const double dy = gnd - dg;           // <d, y>
    double num, den;
    switch (variant) {
    case 1: num = gngn; den = gg; break;                    // FR
    case 2: num = gny; den = dy; break;                     // HS
    case 3: num = fmax(0.0, gny); den = gg; break;          // PRP+
    case 4: num = gngn; den = -dg; break;                   // CD
    case 5: num = gny; den = -dg; break;                    // LS
    case 6: num = gngn; den = dy; break;                    // DY
    default: num = gny; den = gg; break;                    // PRP
    }
    if (den == 0.0) return 0.0;
    const double b = num / den;
    return isfinite(b) ? b : 0.0;
}

// After the accept pass, first part: method state from the dot products.
// Returns true when L-BFGS direction coefficients have to be computed (by the
// whole workgroup) before accept_finish starts the next iteration.
__device__ inline bool accept_update(Ctl* c, const double* dots) {
    const MinParamsDev& p = c->p;
    const int nw = c->acc_new, old = c->acc_old;
    switch (p.method) {
    case M_GD:
        c->cur = nw;
        break;
    case M_CG: {
        // dots: [0] <g_new, g_old>, [1] <g_new, r_old>, [2] <r_old, g_old>
        const double beta = cg_beta(p.cg_beta, c->g2[old], c->g2[nw], dots[0], dots[1], dots[2]);
        const int restart_every = p.cg_restart > 0 ? p.cg_restart : 3 * c->n_atoms;
        if ((c->iters + 1) % restart_every == 0) {
            c->steepest = 1;
        } else {
            c->steepest = 0;
            c->cg_beta = beta;
            c->r_dot_g_old = dots[1];
        }
        c->cur = nw;
        break;
    }
    case M_LBFGS: {
        // dots: [0] <s,y> [1] <y,y> [2] <s,s> [3] <g,s> [4] <g,y> [5] <g,g>,
        // then for the pair in slot q: dots[6 + 6q ..] = <s,S_q> <s,Y_q>
        // <y,S_q> <y,Y_q> <g,S_q> <g,Y_q>
        const double sy = dots[0], yy = dots[1];
        const int n_old = c->hist_n;
        const bool full = n_old == c->hist_m;
        if (sy > kEpsMach * yy) {
            // the new pair takes the slot of the oldest one when the memory is full
            const int q = full ? c->hist_head : ring_slot(c, n_old);
            const int drop_s = c->hist_s[q], drop_y = c->hist_y[q];
            for (int i = full ? 1 : 0; i < n_old; ++i) {
                const int r = ring_slot(c, i);
                const double* d6 = dots + 6 + 6 * r;
                gram_at(c, gpos_s(q), gpos_s(r)) = gram_at(c, gpos_s(r), gpos_s(q)) = d6[0];
                gram_at(c, gpos_s(q), gpos_y(r)) = gram_at(c, gpos_y(r), gpos_s(q)) = d6[1];
                gram_at(c, gpos_y(q), gpos_s(r)) = gram_at(c, gpos_s(r), gpos_y(q)) = d6[2];
                gram_at(c, gpos_y(q), gpos_y(r)) = gram_at(c, gpos_y(r), gpos_y(q)) = d6[3];
                gram_at(c, kGposG, gpos_s(r)) = gram_at(c, gpos_s(r), kGposG) = d6[4];
                gram_at(c, kGposG, gpos_y(r)) = gram_at(c, gpos_y(r), kGposG) = d6[5];
            }
            gram_at(c, gpos_s(q), gpos_s(q)) = dots[2];
            gram_at(c, gpos_s(q), gpos_y(q)) = gram_at(c, gpos_y(q), gpos_s(q)) = sy;
            gram_at(c, gpos_y(q), gpos_y(q)) = yy;
            gram_at(c, kGposG, gpos_s(q)) = gram_at(c, gpos_s(q), kGposG) = dots[3];
            gram_at(c, kGposG, gpos_y(q)) = gram_at(c, gpos_y(q), kGposG) = dots[4];
            c->hist_s[q] = c->spare_s;
            c->hist_y[q] = c->spare_y;
            c->rho[q] = 1.0 / sy;
            if (full) {
                c->hist_head = c->hist_head + 1 == c->hist_m ? 0 : c->hist_head + 1;
                c->spare_s = drop_s;
                c->spare_y = drop_y;
            } else {
                c->hist_n = n_old + 1;
                c->spare_s = c->spare_s_next++;
                c->spare_y = c->spare_y_next++;
            }
        } else {
            for (int i = 0; i < n_old; ++i) {
                const int r = ring_slot(c, i);
                const double* d6 = dots + 6 + 6 * r;
                gram_at(c, kGposG, gpos_s(r)) = gram_at(c, gpos_s(r), kGposG) = d6[4];
                gram_at(c, kGposG, gpos_y(r)) = gram_at(c, gpos_y(r), kGposG) = d6[5];
            }
        }
        gram_at(c, kGposG, kGposG) = dots[5];
        c->cur = nw;
        return c->hist_n > 0;
    }
    case M_HB:
        c->prev_x = c->cur;          // x^{k-1}
        c->cur = nw;
        break;
    case M_OGM:
        // dots: [0] <g_new, S_new>, [1] <S_new, S_new> with S_new = S + t+ g_new
        c->cur = nw;
        c->ogm_t = c->ogm_t_next;
        c->ogm_gS = dots[0];
        c->ogm_SS = dots[1];
        c->ogm_s_anchor = 0;
        break;
    case M_FGM: {
        const double f_old = c->e[c->cur];
        c->prev_x = c->cur;
        c->cur = nw;
        c->theta_prev = c->fgm_theta;
        // optional function-value restart: no momentum after an uphill step
        if (p.fgm_restart && c->e[nw] > f_old) c->theta_prev = 1.0;
        if (c->e[nw] < c->e[c->best]) c->best = nw;
        break;
    }
    }
    return false;
}

// After the accept pass, second part: trace entry, iteration count, next
// iteration.
__device__ inline void accept_finish(Ctl* c) {
    const int nw = c->acc_new;
    const int ti = c->iters - c->iters_base;
    if (c->trace_ptr && ti < c->trace_cap) {
        double* tr = c->trace_ptr + 3 * (size_t)ti;
        tr[0] = c->e[nw];
        tr[1] = c->accept_h;
        tr[2] = (double)c->evals;
        c->n_trace = ti + 1;
    }
    c->iters += 1;
    begin_iteration(c);
}

// After an evaluation (finalize's last workgroup).
__device__ inline void after_eval(Ctl* c) {
    c->evals += 1;
    if (c->batch) atomicAdd(&c->batch->evals, 1u);
    if (c->prec == P_FP64) c->evals64 += 1;
    const int t = c->target;
    c->slot_prec[t] = c->prec;
    switch (c->phase) {
    case PH_START:
        if (!isfinite(c->e[t]) || !isfinite(c->g2[t])) { c->term = T_NONFINITE; finish_done(c, t); return; }
        if (c->p.method == M_FGM) c->best = t;
        begin_iteration(c);
        return;
    case PH_MOMENTUM:
        fgm_after_momentum(c);
        return;
    case PH_LS:
        ls_after_trial(c);
        return;
    case PH_REEVAL64:
        begin_iteration(c);
        return;
    case PH_CERTIFY:
        finish_done(c, t);
        return;
    case PH_HB:
        if (!isfinite(c->e[t]) || !isfinite(c->g2[t])) { finish(c, T_DIVERGED); return; }
        c->accept_h = c->p.hb_alpha;
        c->accept = 1;
        c->acc_new = t;
        c->acc_old = c->cur;
        c->acc_rows = 0;
        c->action = ACT_NONE;
        return;
    case PH_OGM_Y: {
        const bool ok = isfinite(c->e[t]) && isfinite(c->g2[t]) && isfinite(c->slope) && c->slope < 0.0 &&
                        isfinite(c->dir_scale) && c->dir_scale > 0.0;
        if (!ok) {                                  // not a descent direction at y: restart
            ogm_restart(c);
            begin_iteration(c);
            return;
        }
        const int primary = c->p.linesearch == 1 ? LSK_H : LSK_PAR;
        c->ls_fallback_done = primary == LSK_H;
        ls_start(c, t, c->h_prev, primary, false);  // direction and slope from the y evaluation
        return;
    }
    default:
        c->action = ACT_NONE;
        return;
    }
}

}  // namespace ff
