// Per-evaluation finalize (gradient gather, norms, energy total) and the
// optimizer's vector passes: trial point / direction construction and the
// accept pass (history vectors and their dot products).  A pass that ends in
// a reduction writes per-workgroup partials; a second kernel with one
// workgroup per system sums them in a fixed order and runs the decision step.
// (No workgroup waits for others inside a kernel: on this GPU each XCD has its
// own L2, and the device-scope fence such a handshake needs writes the L2
// back every time; the kernel boundary does that once.)
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

// -------------------------------------------------------- L-BFGS direction
// Coefficients of the L-BFGS direction r = -H g (Algorithm 3) in the basis
// {s_0..s_{n-1}, y_0..y_{n-1}, g} of the stored pairs (oldest first) and the
// current gradient, from the Gram matrix of that basis: the two loops of the
// recursion act on coefficient vectors, every inner product becomes a row of
// the Gram matrix times the coefficients.  The workgroup copies the active
// (2n+1)^2 block into LDS; the first wavefront runs the loops, one wavefront
// sum per inner product (lane k holds coefficients k and k + 64).  On a
// descent direction (<g, r> < 0) the terms of r and |r| are written to the
// control block and lb_ready = 1, otherwise lb_ready = -1.  Every thread of
// the workgroup calls this; hist_n >= 1.
__device__ void lbfgs_direction_block(Ctl* c) {
    __shared__ double gs[kGramDim * kGramDim];
    __shared__ double cs[kGramDim];
    __shared__ int pos[kGramDim];
    const int n = c->hist_n;
    const int nb = 2 * n + 1;
    for (int k = threadIdx.x; k < nb; k += blockDim.x)
        pos[k] = k < n ? gpos_s(ring_slot(c, k)) : (k < 2 * n ? gpos_y(ring_slot(c, k - n)) : kGposG);
    __syncthreads();
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
        const int r = e / nb, q = e - r * nb;
        gs[e] = c->gram[pos[r] * kGramDim + pos[q]];
    }
    __syncthreads();
    if (threadIdx.x >= 64) return;
    const int l = threadIdx.x, l2 = l + 64;
    double c0 = l == 2 * n ? -1.0 : 0.0;     // coefficient of basis element l
    double c1 = l2 == 2 * n ? -1.0 : 0.0;    // ... and of l + 64
    const double rho_l = l < n ? c->rho[ring_slot(c, l)] : 0.0;
    auto row_times_coef = [&](int r) {
        double v = 0.0;
        if (l < nb) v = gs[r * nb + l] * c0;
        if (l2 < nb) v += gs[r * nb + l2] * c1;
        return wave_sum(v);
    };
    double alpha_l = 0.0;
    for (int i = n - 1; i >= 0; --i) {             // newest to oldest
        const double a = __shfl(rho_l, i, 64) * row_times_coef(i);
        if (l == i) alpha_l = a;
        if (l == n + i) c0 -= a;
        if (l2 == n + i) c1 -= a;
    }
    const double gamma = gs[(n - 1) * nb + (2 * n - 1)] / gs[(2 * n - 1) * nb + (2 * n - 1)];
    c0 *= gamma;
    c1 *= gamma;
    for (int i = 0; i < n; ++i) {                  // oldest to newest
        const double b = __shfl(rho_l, i, 64) * row_times_coef(n + i);
        const double ai = __shfl(alpha_l, i, 64);
        if (l == i) c0 += ai - b;
    }
    const double gr = row_times_coef(2 * n);       // <g, r>
    if (l < nb) cs[l] = c0;
    if (l2 < nb) cs[l2] = c1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // |r|^2 = c^T G c
    double part = 0.0;
    if (l < nb && c0 != 0.0) {
        double t = 0.0;
        for (int q = 0; q < nb; ++q) t += gs[l * nb + q] * cs[q];
        part = c0 * t;
    }
    if (l2 < nb && c1 != 0.0) {
        double t = 0.0;
        for (int q = 0; q < nb; ++q) t += gs[l2 * nb + q] * cs[q];
        part += c1 * t;
    }
    const double nrm2 = wave_sum(part);
    const bool ok = gr < 0.0 && nrm2 > 0.0 && isfinite(nrm2);
    if (ok) {
        auto term = [&](int k, double coef) {
            c->term_vec[k] = k < n ? c->hist_s[ring_slot(c, k)]
                           : (k < 2 * n ? c->hist_y[ring_slot(c, k - n)] : V_G0 + c->cur);
            c->term_coef[k] = coef;
        };
        if (l < nb) term(l, c0);
        if (l2 < nb) term(l2, c1);
    }
    if (l == 0) {
        if (ok) {
            c->n_terms = nb;
            c->dir_scale = sqrt(nrm2);
        }
        c->lb_ready = ok ? 1 : -1;
    }
}

// ------------------------------------------------------------------ finalize
// Pair partials of one 64-atom tile t of I-block `row`, summed over its
// partial rows in a fixed order.  The tile's rows are the i-side partials
// of every chunk of its I-block, then the j-side partials of every unit that
// holds tile t (I-blocks row0..row).  Each row is 192 contiguous values
// (64 atoms x xyz); wavefront w of the workgroup sums rows w, w+4, ... (lane
// l holds values l, l+64, l+128), the four wavefront sums are then added in
// order.  T is the storage type of the partials (FP32 mode: float).
template <typename T>
__device__ __forceinline__ void gather_tile(const Args& a, const SysInfo& si, int row, int t,
                                            double* tot /* LDS [192] */) {
    __shared__ double part[kFinBlock / 64][3 * kTile];
    const Layout& L = a.L;
    const RowInfo* R = at<RowInfo>(a.ws, L.off_rows);
    const T* Pi = at<T>(a.ws, L.off_pi);
    const T* Pj = at<T>(a.ws, L.off_pj);
    const int row0 = si.row0;
    const RowInfo ri = R[row];
    const int il0 = t * kTile - row * L.block;
    constexpr int tab = sizeof(T) == 4 ? 0 : 1;          // chunk table of the kernel that wrote Pi
    const int n_i = ri.n_chunks[tab], nseg = n_i + row - row0 + 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int kWaves = kFinBlock / 64;
    // Units of a system are numbered row by row, local row r holding tiles
    // r*B/64 .. nt-1, so the unit of (row r, tile tl) has a closed form and
    // the addresses need no table loads.
    const long long u0 = R[row0].unit_start;
    const long long nt = si.np / kTile, b64 = L.block / kTile;
    const long long tl = t - si.aoff / kTile;
    auto seg = [&](int sg) -> const T* {
        if (sg < n_i) return Pi + ((size_t)(ri.chunk_start[tab] + sg) * L.block + il0) * 3;
        const long long r = sg - n_i;
        const long long unit = u0 + r * nt - b64 * r * (r - 1) / 2 + (tl - r * b64);
        return Pj + (size_t)unit * (3 * kTile);
    };
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    int sg = wave;
    // four rows in flight per wavefront, added in row order
    for (; sg + 3 * kWaves < nseg; sg += 4 * kWaves) {
        const T* p0 = seg(sg);
        const T* p1 = seg(sg + kWaves);
        const T* p2 = seg(sg + 2 * kWaves);
        const T* p3 = seg(sg + 3 * kWaves);
        const T v00 = p0[lane], v01 = p0[lane + 64], v02 = p0[lane + 128];
        const T v10 = p1[lane], v11 = p1[lane + 64], v12 = p1[lane + 128];
        const T v20 = p2[lane], v21 = p2[lane + 64], v22 = p2[lane + 128];
        const T v30 = p3[lane], v31 = p3[lane + 64], v32 = p3[lane + 128];
        a0 += (double)v00; a1 += (double)v01; a2 += (double)v02;
        a0 += (double)v10; a1 += (double)v11; a2 += (double)v12;
        a0 += (double)v20; a1 += (double)v21; a2 += (double)v22;
        a0 += (double)v30; a1 += (double)v31; a2 += (double)v32;
    }
    for (; sg < nseg; sg += kWaves) {
        const T* p0 = seg(sg);
        a0 += (double)p0[lane]; a1 += (double)p0[lane + 64]; a2 += (double)p0[lane + 128];
    }
    part[wave][lane] = a0;
    part[wave][lane + 64] = a1;
    part[wave][lane + 128] = a2;
    __syncthreads();
    if (threadIdx.x < 3 * kTile) {
        double v = part[0][threadIdx.x];
        for (int w = 1; w < kWaves; ++w) v += part[w][threadIdx.x];
        tot[threadIdx.x] = v;
    }
    __syncthreads();
}

// One workgroup per 64-atom tile of a system: gradient = pair partials of
// the tile (gather_tile) + the bonded-term slots of each atom (staged through
// LDS, added in slot order).  Per-workgroup partials: max |g|, |g|^2,
// optionally <g_base, d>, and a share of the pair-workgroup and bonded-block
// energies (k_fin_reduce adds them up).  Grid: every tile of every system
// (flat, map_fin).
__global__ void __launch_bounds__(kFinBlock) k_finalize(Args a) {
    const Layout& L = a.L;
    const int2 mb = at<int2>(a.ws, L.off_map_fin)[blockIdx.x];
    const int sys = mb.x, blk = mb.y;                    // system and its tile
    const SysInfo si = sys_info(a)[sys];
    Ctl* c = ctl_at(a, sys);
    if (!a.direct && (c->action != ACT_EVAL || c->target < 0 || c->target >= kNumSlots)) return;
    double* G = a.direct ? (a.g_out ? a.g_out + 3 * (size_t)si.uoff : nullptr) : vec(a, V_G0 + c->target, si);
    const bool want_slope = !a.direct && c->want_slope;
    const int t = si.aoff / kTile + blk;                 // global tile
    const int row = t * kTile / L.block;                 // its I-block
    __shared__ double tot[3 * kTile];
    __shared__ double fbv[kFinBlock][3];
    const bool p32 = a.direct ? a.direct_prec == 1 : c->prec == 1;
    if (p32) gather_tile<float>(a, si, row, t, tot);
    else gather_tile<double>(a, si, row, t, tot);
    // bonded-term slots of the tile's atoms: contiguous in the incidence list
    const int* inc0 = at<int>(a.ws, L.off_inc_start);
    const int* inc = at<int>(a.ws, L.off_inc);
    const double* FB = at<double>(a.ws, L.off_fb);
    const int ga = t * kTile + (int)threadIdx.x;         // global padded atom (threads < 64)
    const int k_lo = inc0[t * kTile], k_hi = inc0[t * kTile + kTile];
    int my_lo = 0, my_hi = 0;
    double gx = 0.0, gy = 0.0, gz = 0.0;
    if (threadIdx.x < kTile) {
        my_lo = inc0[ga];
        my_hi = inc0[ga + 1];
        gx = tot[3 * threadIdx.x];
        gy = tot[3 * threadIdx.x + 1];
        gz = tot[3 * threadIdx.x + 2];
    }
    for (int base = k_lo; base < k_hi; base += kFinBlock) {
        const int k = base + (int)threadIdx.x;
        if (k < k_hi) {
            const double* p = FB + 3 * (size_t)inc[k];
            fbv[threadIdx.x][0] = p[0];
            fbv[threadIdx.x][1] = p[1];
            fbv[threadIdx.x][2] = p[2];
        }
        __syncthreads();
        if (threadIdx.x < kTile) {
            const int e = min(my_hi, base + kFinBlock);
            for (int q = max(my_lo, base); q < e; ++q) {
                gx += fbv[q - base][0]; gy += fbv[q - base][1]; gz += fbv[q - base][2];
            }
        }
        __syncthreads();
    }
    const int atom = blk * kTile + (int)threadIdx.x;          // local atom
    const bool real = threadIdx.x < kTile && atom < si.n;
    if (!real) gx = gy = gz = 0.0;
    if (real && G) { G[3 * (size_t)atom] = gx; G[3 * (size_t)atom + 1] = gy; G[3 * (size_t)atom + 2] = gz; }
    double v[4];
    v[0] = fmax(fabs(gx), fmax(fabs(gy), fabs(gz)));
    if (isnan(gx) || isnan(gy) || isnan(gz)) v[0] = __builtin_inf();
    v[1] = gx * gx + gy * gy + gz * gz;
    v[2] = 0.0;
    if (want_slope && real) {
        const double* gb = vec(a, V_G0 + c->slope_slot, si);
        const double* d = vec(a, V_D, si);
        const size_t o = 3 * (size_t)atom;
        v[2] = gb[o] * d[o] + gb[o + 1] * d[o + 1] + gb[o + 2] * d[o + 2];
    }
    // this workgroup's share of the pair-workgroup and bonded-block energies
    {
        const int nb = si.fin_blocks, b = blk;
        const int tab = p32 ? 0 : 1;                     // chunk table of the pair kernel that ran
        const double* ep = at<double>(a.ws, L.off_ep) + si.chunk0[tab];
        const double* eb = at<double>(a.ws, L.off_eb) + si.eb0;
        const int nc = si.n_chunks[tab];
        const int p0 = (int)((long long)nc * b / nb), p1 = (int)((long long)nc * (b + 1) / nb);
        const int q0 = (int)((long long)si.bonded_blocks * b / nb), q1 = (int)((long long)si.bonded_blocks * (b + 1) / nb);
        double e = 0.0;
        for (int k = p0 + (int)threadIdx.x; k < p1; k += kFinBlock) e += ep[k];
        for (int k = q0 + (int)threadIdx.x; k < q1; k += kFinBlock) e += eb[k];
        v[3] = e;
    }
    double* red = at<double>(a.ws, L.off_red) + si.red0;
    double tr[4];
    block_reduce<4>(v, true, tr);
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) red[4 * blk + k] = tr[k];
}

// Totals of one system's finalize partials in a fixed order, then E, the
// norms and the decision step (ff_energy_grad: the energy only).
// Grid: (systems).
__global__ void __launch_bounds__(kFinBlock) k_fin_reduce(Args a) {
    const int sys = blockIdx.x;
    const SysInfo si = sys_info(a)[sys];
    Ctl* c = ctl_at(a, sys);
    if (!a.direct && (c->action != ACT_EVAL || c->target < 0 || c->target >= kNumSlots)) return;
    const bool want_slope = !a.direct && c->want_slope;
    const double* red = at<double>(a.ws, a.L.off_red) + si.red0;
    double w[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int b = threadIdx.x; b < si.fin_blocks; b += kFinBlock) {
        w[0] = fmax(w[0], red[4 * b]);
        w[1] += red[4 * b + 1];
        w[2] += red[4 * b + 2];
        w[3] += red[4 * b + 3];
    }
    double gt[4];
    block_reduce<4>(w, true, gt);
    if (threadIdx.x != 0) return;
    const double E = gt[3];
    if (a.direct) {
        if (a.e_out) a.e_out[sys] = E;
        if (a.g2_out) a.g2_out[sys] = gt[1];
        return;
    }
    const int tg = c->target;
    c->e[tg] = E;
    c->ginf[tg] = gt[0];
    c->g2[tg] = gt[1];
    if (want_slope) c->slope = gt[2];
    after_eval(c);
}

// ------------------------------------------------------------------- prepare
// Builds the point to evaluate: a trial x + h d, the direction itself
// (d = r / |r| with r a linear combination of stored vectors) followed by the
// trial, or the FGM momentum point.  Rounding is kept explicit (no
// contraction) so that trial points are reproducible.
__global__ void __launch_bounds__(kFinBlock) k_prepare(Args a) {
    const int2 mb = at<int2>(a.ws, a.L.off_map_vec)[blockIdx.x];
    const int sys = mb.x;
    const SysInfo si = sys_info(a)[sys];
    const Ctl* c = ctl_at(a, sys);
    if (c->action != ACT_EVAL || c->point_mode == PM_USE) return;
    if (c->target < 0 || c->target >= kNumSlots || c->base < 0 || c->base >= kNumSlots) return;
    const int pm = c->point_mode;
    if ((pm == PM_MOMENTUM || pm == PM_HB || pm == PM_OGM_Y) && (c->prev < 0 || c->prev >= kNumSlots)) return;
    const int n3 = 3 * si.n;
    const int i = mb.y * kFinBlock + threadIdx.x;
    if (i >= n3) return;
    double* xt = vec(a, V_X0 + c->target, si);
    const double* xb = vec(a, V_X0 + c->base, si);
    if (pm == PM_MOMENTUM) {
        const double* xp = vec(a, V_X0 + c->prev, si);
        xt[i] = __dadd_rn(xb[i], __dmul_rn(c->beta, __dsub_rn(xb[i], xp[i])));
        return;
    }
    if (pm == PM_HB) {
        const double* xp = vec(a, V_X0 + c->prev, si);
        const double* gb = vec(a, V_G0 + c->base, si);
        xt[i] = __dadd_rn(__dsub_rn(xb[i], __dmul_rn(c->h, gb[i])), __dmul_rn(c->beta, __dsub_rn(xb[i], xp[i])));
        return;
    }
    double* d = vec(a, V_D, si);
    double di;
    if (pm == PM_DIR_TRIAL || pm == PM_OGM_Y) {
        double r = __dmul_rn(c->term_coef[0], vec(a, c->term_vec[0], si)[i]);
        for (int k = 1; k < c->n_terms; ++k) r = __dadd_rn(r, __dmul_rn(c->term_coef[k], vec(a, c->term_vec[k], si)[i]));
        if (c->write_r) vec(a, V_R, si)[i] = r;
        di = __ddiv_rn(r, c->dir_scale);
        d[i] = di;
    } else {
        di = d[i];
    }
    if (pm == PM_OGM_Y) {
        const double* xa = vec(a, V_X0 + c->prev, si);
        xt[i] = __dadd_rn(__dmul_rn(1.0 - c->beta, xb[i]), __dmul_rn(c->beta, xa[i]));
        return;
    }
    xt[i] = __dadd_rn(xb[i], __dmul_rn(c->h, di));
}

// -------------------------------------------------------------------- accept
// After a successful line search: method-specific vectors and dot products.
//  CG:     <g_new, g_old>, <g_new, r_old>, <r_old, g_old>
//  L-BFGS: s = x_new - x_old and y = g_new - g_old (written to the spare
//          history vectors), <s,y> <y,y> <s,s> <g,s> <g,y> <g,g> and, for
//          the pair in every occupied history slot q, <s,S_q> <s,Y_q>
//          <y,S_q> <y,Y_q> <g,S_q> <g,Y_q>.
// Grid: (accept workgroups of every system (flat, map_acc), 1 + largest
// L-BFGS memory).  Row 0 computes the first group of six, row r >= 1 the six
// products with the pair in slot r-1 (s and y are recomputed from the point
// vectors in every row, with the same arithmetic); each workgroup strides over
// its share of the 3N elements and writes one partial per product
// (k_accept_reduce adds them up in workgroup order).
__global__ void __launch_bounds__(kFinBlock) k_accept(Args a) {
    const int2 mb = at<int2>(a.ws, a.L.off_map_acc)[blockIdx.x];
    const int sys = mb.x, bx = mb.y;
    const SysInfo si = sys_info(a)[sys];
    Ctl* c = ctl_at(a, sys);
    if (!c->accept) return;
    const int n3 = 3 * si.n;
    const int method = c->p.method;
    const int row = blockIdx.y;
    // acc_rows is fixed while this pass runs (the reduce kernel changes
    // hist_n afterwards)
    const int rows = c->acc_rows;
    const bool active = row < rows;
    double* red = at<double>(a.ws, a.L.off_red) + si.red0;
    const int nbx = si.acc_bx;
    if (active) {
        double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        const double* xn = vec(a, V_X0 + c->acc_new, si);
        const double* xo = vec(a, V_X0 + c->acc_old, si);
        const double* gn = vec(a, V_G0 + c->acc_new, si);
        const double* go = vec(a, V_G0 + c->acc_old, si);
        const int stride = nbx * kFinBlock;
        if (method == M_OGM) {
            // S += t_{k+1} g_new (S is the anchor's gradient after a restart)
            const double* src = c->ogm_s_anchor ? vec(a, V_G0 + c->prev_x, si) : vec(a, V_R, si);
            double* S = vec(a, V_R, si);
            const double t = c->ogm_t_next;
            for (int i = bx * kFinBlock + threadIdx.x; i < n3; i += stride) {
                const double sn = __dadd_rn(src[i], __dmul_rn(t, gn[i]));
                S[i] = sn;
                v[0] += gn[i] * sn;
                v[1] += sn * sn;
            }
        } else if (method == M_CG) {
            const double* r = vec(a, V_R, si);
            for (int i = bx * kFinBlock + threadIdx.x; i < n3; i += stride) {
                v[0] += gn[i] * go[i];
                v[1] += gn[i] * r[i];
                v[2] += r[i] * go[i];
            }
        } else if (row == 0) {
            double* ss = vec(a, c->spare_s, si);
            double* yy = vec(a, c->spare_y, si);
            for (int i = bx * kFinBlock + threadIdx.x; i < n3; i += stride) {
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
            for (int i = bx * kFinBlock + threadIdx.x; i < n3; i += stride) {
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
            for (int k = 0; k < 6; ++k) red[((size_t)row * nbx + bx) * 6 + k] = tot[k];
    }
}

// Sums the accept pass's per-workgroup products in a fixed order, then the
// method update and the next iteration (L-BFGS: coefficients of the next
// direction computed by the workgroup first).  Grid: (systems).
__global__ void __launch_bounds__(kFinBlock) k_accept_reduce(Args a) {
    const int sys = blockIdx.x;
    const SysInfo si = sys_info(a)[sys];
    Ctl* c = ctl_at(a, sys);
    if (!c->accept) return;
    const int method = c->p.method;
    const int rows = c->acc_rows;
    const int nbx = si.acc_bx;
    const double* red = at<double>(a.ws, a.L.off_red) + si.red0;
    __shared__ double dots[kMaxDots];
    const int nd = method == M_LBFGS || method == M_OGM ? 6 * rows : (method == M_CG ? 3 : 0);
    for (int k = threadIdx.x; k < nd; k += kFinBlock) {
        const int r = k / 6, q = k - 6 * r;
        double acc = 0.0;
#pragma unroll 16
        for (int b = 0; b < nbx; ++b) acc += red[((size_t)r * nbx + b) * 6 + q];
        dots[k] = acc;
    }
    __shared__ int need_dir;
    __syncthreads();
    if (threadIdx.x == 0) need_dir = accept_update(c, dots) ? 1 : 0;
    __syncthreads();
    if (need_dir) lbfgs_direction_block(c);
    __syncthreads();
    if (threadIdx.x == 0) accept_finish(c);
}

// ---------------------------------------------------------------------- kick
// Starts (or resumes) a minimization: one thread sets up the control block.
// One workgroup per system (system 0 keeps the per-iteration trace).
__global__ void k_kick(Args a, MinParamsDev p, int resume, double* trace, int trace_cap) {
    const int sys = blockIdx.x;
    Ctl* c = ctl_at(a, sys);
    if (resume) {
        // continue where the previous call stopped; the L-BFGS direction is
        // recomputed from the stored pairs exactly as after an accept
        __shared__ int need_dir;
        if (threadIdx.x == 0) {
            c->batch = at<BatchState>(a.ws, a.L.off_batch);
            c->n_atoms = sys_info(a)[sys].n;
            const bool same_memory = c->p.method == M_LBFGS && p.method == M_LBFGS && c->hist_m == p.m;
            c->p = p;
            if (!same_memory) lbfgs_clear(c);
            c->done = 0;
            c->iters_limit = c->iters + p.max_iter;
            c->trace_ptr = sys == 0 ? trace : nullptr;
            c->trace_cap = trace_cap;
            c->n_trace = 0;
            c->iters_base = c->iters;
            c->fp32_released = 0;
            if (c->escalated) release_fp32(c);
            need_dir = p.method == M_LBFGS && c->hist_n > 0;
        }
        __syncthreads();
        if (need_dir) lbfgs_direction_block(c);
        __syncthreads();
        if (threadIdx.x == 0) begin_iteration(c);
        return;
    }
    if (threadIdx.x != 0) return;
    if (sys != 0) trace = nullptr;
    c->batch = at<BatchState>(a.ws, a.L.off_batch);
    c->n_atoms = sys_info(a)[sys].n;
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
    c->prev_x = (p.method == M_FGM || p.method == M_HB || p.method == M_OGM) ? 0 : -1;
    c->ogm_t = 1.0;
    c->ogm_s_anchor = 1;
    c->best = -1;
    c->w = -1;
    c->ls_base = -1;
    c->ls_best = -1;
    c->prec_now = p.precision;
    c->escalated = 0;
    c->stall32 = 0;
    c->fp32_released = 0;
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
    request_eval(c, PM_USE, 0, 0);
}

// Zeroes the batch counters (before a minimization starts).
__global__ void k_reset_batch(Args a) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    BatchState* b = at<BatchState>(a.ws, a.L.off_batch);
    b->n_done = 0u;
    b->evals = 0u;
    b->n_fp64 = 0u;
}

// Marks every system idle (after ff_create).
__global__ void k_reset_ctl(Args a) {
    if (threadIdx.x != 0) return;
    Ctl* c = ctl_at(a, blockIdx.x);
    c->batch = nullptr;
    c->action = ACT_NONE;
    c->accept = 0;
    c->done = 1;
    c->phase = PH_IDLE;
    c->iters = 0;
}

// Point of the energy profile: x + t u with u = -g / |g| per system (u = 0
// where g = 0), all in the caller's concatenated layout.  Grid: flat over
// every system's 3n elements (map_vec).
__global__ void __launch_bounds__(kFinBlock) k_profile_point(Args a, const double* x, const double* g,
                                                             const double* g2, double t, double* xt) {
    const int2 mb = at<int2>(a.ws, a.L.off_map_vec)[blockIdx.x];
    const SysInfo si = sys_info(a)[mb.x];
    const int i = mb.y * kFinBlock + threadIdx.x;
    if (i >= 3 * si.n) return;
    const size_t o = 3 * (size_t)si.uoff + i;
    const double nrm = sqrt(g2[mb.x]);
    const double u = nrm > 0.0 ? __ddiv_rn(-g[o], nrm) : 0.0;
    xt[o] = __dadd_rn(x[o], __dmul_rn(t, u));
}

hipError_t launch_profile_point(const Args& a, const double* x, const double* g, const double* g2, double t,
                                double* xt, hipStream_t s) {
    hipLaunchKernelGGL(k_profile_point, dim3(a.L.n_vec_blocks), dim3(kFinBlock), 0, s, a, x, g, g2, t, xt);
    return hipGetLastError();
}

hipError_t launch_finalize(const Args& a, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(a.L.n_fin_blocks), dim3(kFinBlock), 0, s, a);
    hipLaunchKernelGGL(k_fin_reduce, dim3(a.L.n_sys), dim3(kFinBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cycle_vec(const Args& a, int which, hipStream_t s) {
    if (which == 0)
        hipLaunchKernelGGL(k_prepare, dim3(a.L.n_vec_blocks), dim3(kFinBlock), 0, s, a);
    else {
        hipLaunchKernelGGL(k_accept, dim3(a.L.n_acc_blocks, a.L.acc_rows), dim3(kFinBlock), 0, s, a);
        hipLaunchKernelGGL(k_accept_reduce, dim3(a.L.n_sys), dim3(kFinBlock), 0, s, a);
    }
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
