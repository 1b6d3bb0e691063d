// Per-evaluation finalize (gradient gather, norms, energy total) and the
// optimizer's vector passes: trial point / direction construction and the
// accept pass (history vectors and their dot products).  Each kernel closes
// with a deterministic fixed-order reduction in its last workgroup
// (last-block-done ticket), which then runs the decision step.
#include "ff_decide.h"

namespace ff {


// Wavefront sum of a double (xor butterfly).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Sum (or max for index 0 if first_is_max) of NV per-thread values over a
// 256-thread block; thread 0 receives the totals in out[].
template <int NV>
__device__ __forceinline__ void block_reduce(double (&v)[NV], bool first_is_max, double* out) {
    __shared__ double s[kFinBlock / 64][NV > 0 ? NV : 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double r = (k == 0 && first_is_max) ? wave_max(v[k]) : wave_sum(v[k]);
        if (lane == 0) s[wave][k] = r;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double r = s[0][k];
            for (int w = 1; w < kFinBlock / 64; ++w) r = (k == 0 && first_is_max) ? fmax(r, s[w][k]) : r + s[w][k];
            out[k] = r;
        }
    }
    __syncthreads();
}

// Last-block-done over `count` workgroups: returns true in every thread of
// the workgroup that finished last, which also resets the ticket counter.
__device__ __forceinline__ bool last_block(uint32_t* ticket, uint32_t count) {
    __shared__ int is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t = atomicAdd(ticket, 1u);
        is_last = (t == count - 1);
    }
    __syncthreads();
    if (is_last) {
        __threadfence();
        if (threadIdx.x == 0) atomicExch(ticket, 0u);
    }
    return is_last != 0;
}

// Fixed-order sum of n doubles by one 256-thread block (result in thread 0).
__device__ __forceinline__ double block_sum_array(const double* p, int n, bool is_max = false) {
    double v = is_max ? 0.0 : 0.0;
    for (int i = threadIdx.x; i < n; i += kFinBlock) v = is_max ? fmax(v, p[i]) : v + p[i];
    double arr[1] = {v};
    __shared__ double res;
    double out[1];
    block_reduce<1>(arr, is_max, out);
    if (threadIdx.x == 0) res = out[0];
    __syncthreads();
    const double r = res;
    __syncthreads();
    return r;
}

// ------------------------------------------------------------------ finalize
// Pair part of the gradient of `atom`: the i-side partials of every chunk of
// its I-block, then the j-side partials of every unit that holds its j-tile,
// in a fixed order.  T is the storage type of the partials (FP32 mode: float).
template <typename T>
__device__ __forceinline__ void gather_pair(const Args& a, int row0, int atom, double& gx, double& gy, double& gz) {
    const Layout& L = a.L;
    const int row = atom / L.block, il = atom - row * L.block;
    const int t = atom / kTile, jl = atom - t * kTile;
    const RowInfo* R = at<RowInfo>(a.ws, L.off_rows);
    const T* Pi = at<T>(a.ws, L.off_pi);
    const T* Pj = at<T>(a.ws, L.off_pj);
    const RowInfo ri = R[row];
    for (int ch = ri.chunk_start; ch < ri.chunk_start + ri.n_chunks; ++ch) {
        const T* p = Pi + ((size_t)ch * L.block + il) * 3;
        gx += (double)p[0]; gy += (double)p[1]; gz += (double)p[2];
    }
    for (int r = row0; r <= row; ++r) {
        const RowInfo rr = R[r];
        const T* p = Pj + ((size_t)(rr.unit_start + t - rr.t0) * kTile + jl) * 3;
        gx += (double)p[0]; gy += (double)p[1]; gz += (double)p[2];
    }
}

// One thread per atom: gradient = sum of the pair partials of its I-block
// (all chunks of its row), of the j partials of every unit holding it, and
// of its bonded-term slots.  Then |g|_inf, |g|^2, optionally <g_base, d>, and
// E = sum of the pair-workgroup and bonded-block energies.
// Grid: (largest per-system block count, 1, systems); atoms are local to the
// system, reductions and the decision step are per system.
__global__ void __launch_bounds__(kFinBlock) k_finalize(Args a) {
    const Layout& L = a.L;
    const int sys = blockIdx.z;
    const SysInfo si = sys_info(a)[sys];
    if ((int)blockIdx.x >= si.fin_blocks) return;
    Ctl* c = ctl_at(a, sys);
    if (!a.direct && (c->action != ACT_EVAL || c->target < 0 || c->target >= kNumSlots)) return;
    double* G = a.direct ? (a.g_out ? a.g_out + 3 * (size_t)si.uoff : nullptr) : vec(a, V_G0 + c->target, si);
    const bool want_slope = !a.direct && c->want_slope;
    const int atom = blockIdx.x * kFinBlock + threadIdx.x;
    double gx = 0.0, gy = 0.0, gz = 0.0;
    if (atom < si.n) {
        const int ga = si.aoff + atom;      // global padded atom
        const bool p32 = a.direct ? a.direct_prec == 1 : c->prec == 1;
        if (p32) gather_pair<float>(a, si.row0, ga, gx, gy, gz);
        else gather_pair<double>(a, si.row0, ga, gx, gy, gz);
        const int* inc0 = at<int>(a.ws, L.off_inc_start);
        const int* inc = at<int>(a.ws, L.off_inc);
        const double* FB = at<double>(a.ws, L.off_fb);
        for (int k = inc0[ga]; k < inc0[ga + 1]; ++k) {
            const double* p = FB + 3 * (size_t)inc[k];
            gx += p[0]; gy += p[1]; gz += p[2];
        }
        if (G) { G[3 * (size_t)atom] = gx; G[3 * (size_t)atom + 1] = gy; G[3 * (size_t)atom + 2] = gz; }
    }
    double v[3];
    v[0] = fmax(fabs(gx), fmax(fabs(gy), fabs(gz)));
    if (isnan(gx) || isnan(gy) || isnan(gz)) v[0] = __builtin_inf();
    v[1] = gx * gx + gy * gy + gz * gz;
    v[2] = 0.0;
    if (want_slope && atom < si.n) {
        const double* gb = vec(a, V_G0 + c->base, si);
        const double* d = vec(a, V_D, si);
        const size_t o = 3 * (size_t)atom;
        v[2] = gb[o] * d[o] + gb[o + 1] * d[o + 1] + gb[o + 2] * d[o + 2];
    }
    double* red = at<double>(a.ws, L.off_red) + si.red0;
    double tot[3];
    block_reduce<3>(v, true, tot);
    if (threadIdx.x == 0) { red[3 * blockIdx.x] = tot[0]; red[3 * blockIdx.x + 1] = tot[1]; red[3 * blockIdx.x + 2] = tot[2]; }
    if (!last_block(&c->ticket_fin, si.fin_blocks)) return;
    // ---- last workgroup of this system: totals in a fixed order
    double w[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < si.fin_blocks; b += kFinBlock) {
        w[0] = fmax(w[0], red[3 * b]);
        w[1] += red[3 * b + 1];
        w[2] += red[3 * b + 2];
    }
    double gt[3];
    block_reduce<3>(w, true, gt);
    const double e_pair = block_sum_array(at<double>(a.ws, L.off_ep) + si.chunk0, si.n_chunks);
    const double e_bond = block_sum_array(at<double>(a.ws, L.off_eb) + si.eb0, si.bonded_blocks);
    if (threadIdx.x != 0) return;
    const double E = e_pair + e_bond;
    if (a.direct) {
        if (a.e_out) a.e_out[sys] = E;
        return;
    }
    const int t = c->target;
    c->e[t] = E;
    c->ginf[t] = gt[0];
    c->g2[t] = gt[1];
    if (want_slope) c->slope = gt[2];
    after_eval(c);
}

// ------------------------------------------------------------------- prepare
// Builds the point to evaluate: a trial x + h d, the direction itself
// (d = r / |r| with r a linear combination of stored vectors) followed by the
// trial, or the FGM momentum point.  Rounding is kept explicit (no
// contraction) so that trial points are reproducible.
__global__ void __launch_bounds__(kFinBlock) k_prepare(Args a) {
    const int sys = blockIdx.z;
    const SysInfo si = sys_info(a)[sys];
    const Ctl* c = ctl_at(a, sys);
    if (c->action != ACT_EVAL || c->point_mode == PM_USE) return;
    if (c->target < 0 || c->target >= kNumSlots || c->base < 0 || c->base >= kNumSlots) return;
    if (c->point_mode == PM_MOMENTUM && (c->prev < 0 || c->prev >= kNumSlots)) return;
    const int n3 = 3 * si.n;
    const int i = blockIdx.x * kFinBlock + threadIdx.x;
    if (i >= n3) return;
    double* xt = vec(a, V_X0 + c->target, si);
    const double* xb = vec(a, V_X0 + c->base, si);
    if (c->point_mode == PM_MOMENTUM) {
        const double* xp = vec(a, V_X0 + c->prev, si);
        xt[i] = __dadd_rn(xb[i], __dmul_rn(c->beta, __dsub_rn(xb[i], xp[i])));
        return;
    }
    double* d = vec(a, V_D, si);
    double di;
    if (c->point_mode == PM_DIR_TRIAL) {
        double r = __dmul_rn(c->term_coef[0], vec(a, c->term_vec[0], si)[i]);
        for (int k = 1; k < c->n_terms; ++k) r = __dadd_rn(r, __dmul_rn(c->term_coef[k], vec(a, c->term_vec[k], si)[i]));
        if (c->write_r) vec(a, V_R, si)[i] = r;
        di = __ddiv_rn(r, c->dir_scale);
        d[i] = di;
    } else {
        di = d[i];
    }
    xt[i] = __dadd_rn(xb[i], __dmul_rn(c->h, di));
}

// -------------------------------------------------------------------- accept
// After a successful line search: method-specific vectors and dot products.
//  CG:     <g_new, g_old>, <g_new, r_old>, <r_old, g_old>
//  L-BFGS: s = x_new - x_old and y = g_new - g_old (written to the spare
//          history vectors), <s,y> <y,y> <s,s> <g,s> <g,y> <g,g> and, for
//          every stored pair i, <s,S_i> <s,Y_i> <y,S_i> <y,Y_i> <g,S_i> <g,Y_i>.
// Grid: (accept_bx, kMaxM + 1).  Row 0 computes the first group of six, row
// r >= 1 the six products with stored pair r-1 (s and y are recomputed from
// the point vectors in every row, with the same arithmetic); each block
// strides over its share of the 3N elements and reduces once.  The last
// block sums the per-block partials of every dot in block order.
__global__ void __launch_bounds__(kFinBlock) k_accept(Args a) {
    const int sys = blockIdx.z;
    const SysInfo si = sys_info(a)[sys];
    Ctl* c = ctl_at(a, sys);
    if (!c->accept) return;
    const int n3 = 3 * si.n;
    const int method = c->p.method;
    const int row = blockIdx.y;
    const int nh = method == M_LBFGS ? c->hist_n : 0;
    const bool active = (method == M_LBFGS && row <= nh) || (method == M_CG && row == 0);
    double* red = at<double>(a.ws, a.L.off_red) + si.red0;
    const int nbx = gridDim.x;
    if (active) {
        double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        const double* xn = vec(a, V_X0 + c->acc_new, si);
        const double* xo = vec(a, V_X0 + c->acc_old, si);
        const double* gn = vec(a, V_G0 + c->acc_new, si);
        const double* go = vec(a, V_G0 + c->acc_old, si);
        const int stride = nbx * kFinBlock;
        if (method == M_CG) {
            const double* r = vec(a, V_R, si);
            for (int i = blockIdx.x * kFinBlock + threadIdx.x; i < n3; i += stride) {
                v[0] += gn[i] * go[i];
                v[1] += gn[i] * r[i];
                v[2] += r[i] * go[i];
            }
        } else if (row == 0) {
            double* ss = vec(a, c->spare_s, si);
            double* yy = vec(a, c->spare_y, si);
            for (int i = blockIdx.x * kFinBlock + threadIdx.x; i < n3; i += stride) {
                const double s = __dsub_rn(xn[i], xo[i]);
                const double g = gn[i];
                const double y = __dsub_rn(g, go[i]);
                ss[i] = s;
                yy[i] = y;
                v[0] += s * y; v[1] += y * y; v[2] += s * s;
                v[3] += g * s; v[4] += g * y; v[5] += g * g;
            }
        } else {
            const double* S = vec(a, c->hist_s[row - 1], si);
            const double* Y = vec(a, c->hist_y[row - 1], si);
            for (int i = blockIdx.x * kFinBlock + threadIdx.x; i < n3; i += stride) {
                const double s = __dsub_rn(xn[i], xo[i]);
                const double g = gn[i];
                const double y = __dsub_rn(g, go[i]);
                const double Si = S[i], Yi = Y[i];
                v[0] += s * Si; v[1] += s * Yi; v[2] += y * Si;
                v[3] += y * Yi; v[4] += g * Si; v[5] += g * Yi;
            }
        }
        double tot[6];
        block_reduce<6>(v, false, tot);
        if (threadIdx.x == 0)
            for (int k = 0; k < 6; ++k) red[((size_t)row * nbx + blockIdx.x) * 6 + k] = tot[k];
    }
    // every block takes a ticket; the last one finishes the reduction
    __shared__ int is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t = atomicAdd(&c->ticket_acc, 1u);
        is_last = (t == gridDim.x * gridDim.y - 1);
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    __shared__ double dots[kMaxDots];
    const int nd = method == M_LBFGS ? 6 * (nh + 1) : (method == M_CG ? 3 : 0);
    for (int k = threadIdx.x; k < nd; k += kFinBlock) {
        const int r = k / 6, q = k - 6 * r;
        double acc = 0.0;
        for (int b = 0; b < nbx; ++b) acc += red[((size_t)r * nbx + b) * 6 + q];
        dots[k] = acc;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    c->ticket_acc = 0u;
    after_accept(c, dots);
}

// ---------------------------------------------------------------------- kick
// Starts (or resumes) a minimization: one thread sets up the control block.
// One workgroup per system (system 0 keeps the per-iteration trace).
__global__ void k_kick(Args a, MinParamsDev p, int resume, double* trace, int trace_cap) {
    if (threadIdx.x != 0) return;
    const int sys = blockIdx.x;
    Ctl* c = ctl_at(a, sys);
    if (sys != 0) trace = nullptr;
    c->batch = at<BatchState>(a.ws, a.L.off_batch);
    c->n_atoms = sys_info(a)[sys].n;
    if (resume) {
        c->p = p;
        c->done = 0;
        c->iters_limit = c->iters + p.max_iter;
        c->trace_ptr = trace;
        c->trace_cap = trace_cap;
        c->n_trace = 0;
        c->iters_base = c->iters;
        begin_iteration(c);
        return;
    }
    c->p = p;
    c->phase = PH_START;
    c->done = 0;
    c->term = -1;
    c->iters = 0;
    c->iters_base = 0;
    c->evals = 0;
    c->evals64 = 0;
    c->iters_limit = p.max_iter;
    c->cur = 0;
    c->prev_x = p.method == M_FGM ? 0 : -1;
    c->best = -1;
    c->w = -1;
    c->ls_base = -1;
    c->ls_best = -1;
    c->prec_now = p.precision;
    c->escalated = 0;
    c->h_prev = p.h_init;
    c->steepest = 1;
    c->theta_prev = 1.0;
    c->fgm_beta = 0.0;
    c->cg_beta = 0.0;
    c->accept = 0;
    c->result_slot = 0;
    lbfgs_clear(c);
    for (int s = 0; s < kNumSlots; ++s) c->slot_prec[s] = -1;
    c->trace_ptr = trace;
    c->trace_cap = trace_cap;
    c->n_trace = 0;
    c->ticket_fin = c->ticket_acc = c->ticket_prep = 0u;
    request_eval(c, PM_USE, 0, 0);
}

// Zeroes the batch counters (before a minimization starts).
__global__ void k_reset_batch(Args a) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    BatchState* b = at<BatchState>(a.ws, a.L.off_batch);
    b->n_done = 0u;
    b->evals = 0u;
}

// Clears the tickets and marks every system idle (after ff_create).
__global__ void k_reset_ctl(Args a) {
    if (threadIdx.x != 0) return;
    Ctl* c = ctl_at(a, blockIdx.x);
    c->batch = nullptr;
    c->ticket_fin = c->ticket_acc = c->ticket_prep = 0u;
    c->action = ACT_NONE;
    c->accept = 0;
    c->done = 1;
    c->phase = PH_IDLE;
    c->iters = 0;
}

hipError_t launch_finalize(const Args& a, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(a.L.max_fin_blocks, 1, a.L.n_sys), dim3(kFinBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cycle_vec(const Args& a, int which, hipStream_t s) {
    if (which == 0)
        hipLaunchKernelGGL(k_prepare, dim3(a.L.max_vec_blocks, 1, a.L.n_sys), dim3(kFinBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_accept, dim3(a.L.accept_bx, kMaxM + 1, a.L.n_sys), dim3(kFinBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_kick(const Args& a, const MinParamsDev& p, int resume, double* trace, int trace_cap,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_reset_batch, dim3(1), dim3(64), 0, s, a);
    hipLaunchKernelGGL(k_kick, dim3(a.L.n_sys), dim3(64), 0, s, a, p, resume, trace, trace_cap);
    return hipGetLastError();
}

hipError_t launch_reset(const Args& a, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_ctl, dim3(a.L.n_sys), dim3(64), 0, s, a);
    hipLaunchKernelGGL(k_reset_batch, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace ff
