// Nonbonded all-pairs energy and gradient (Coulomb + 12-6 Lennard-Jones with
// geometric mixing, section 2 of the paper) and the bonded terms (stretch,
// bend, OPLS torsion, section 2), for one evaluation point.
//
// Work decomposition.  Atoms are padded to np (multiple of 512) with
// zero-parameter atoms placed far away.  The upper triangle of the pair
// matrix is cut into units (I-block of B atoms) x (j-tile of 64 atoms), j-tile
// index t >= B*row/64; a workgroup ("chunk") walks a run of j-tiles of one
// I-block.  Each lane keeps IPL i-atoms in registers; the j-tile sits in LDS
// twice in a row so that at step s lane l reads entry l+s (atom (l+s) mod 64)
// with an immediate offset.  The gradient on j is accumulated in a register
// that moves one lane down after every step (DPP wave rotation), so after 64
// steps every lane again holds the sum for "its" j.  Per-tile FP32 sums are
// folded into FP64; per-unit j sums and per-chunk i sums are written to
// partial buffers that the finalize kernel adds up in a fixed order, so the
// result is deterministic.  Newton's third law is used: every pair is
// computed once.
//
// Per pair, with per-atom factors prepared once per system
//   c12 = 2 sqrt(eps) sigma^6,  c6 = 2 sqrt(eps) sigma^3,  q^ = sqrt(C) q
// (so c12_i c12_j = 4 eps_ij sigma_ij^12, c6_i c6_j = 4 eps_ij sigma_ij^6,
//  q^_i q^_j = C q_i q_j), the terms of section 2 are
//   e12 = c12_i c12_j / r^12, e6 = c6_i c6_j / r^6, ec = q^_i q^_j / r
//   E  += e12 - e6 + ec
//   f   = (12 e12 - 6 e6 + ec) / r^2,  d = x_j - x_i
//   grad_i += f d,  grad_j -= f d.
// They are evaluated as follows, with the i-atom's factors held as 12 c12_i
// and 6 c6_i (s = 1/r^6, A = 12 c12_i c12_j, B = 6 c6_i c6_j):
//   u = A s - B                  (12 e12 - 6 e6 = u s)
//   f = (u s + ec) / r^2
//   L += (u - B) s               (12 e12 - 12 e6 = (u - B) s),  Ec += ec
// and E = L / 12 + Ec: 13 operations after 1/r instead of 16 for the direct
// form.  The Lennard-Jones and Coulomb sums are kept apart: one FP32 sum of
// both (or of 12 E) loses about 1e-6 of |E| at relaxed 10^4-atom chains.
#include "ff_internal.h"

namespace ff {

// Unroll of the 64-step j loop of the FP32 kernel: with one i-atom per lane
// four steps keep enough independent work in flight; with two the register
// budget of an unroll by four would cost a wavefront per SIMD (measured on
// the 50k chain: 1.05 ms with unroll 2 against 1.19 ms with 4 for 2 atoms per
// lane; 1.05 against 1.07 ms the other way round for 1 atom per lane).
template <int IPL>
constexpr int kUnroll32 = IPL == 1 ? 4 : 2;

#ifndef FF_DPP_ROTATE
#define FF_DPP_ROTATE 0x134   // wave_rol:1 -- lane l receives lane (l+1) mod 64
#endif

__device__ __forceinline__ float rotate_down(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), FF_DPP_ROTATE, 0xF, 0xF, false));
}
__device__ __forceinline__ double rotate_down(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), FF_DPP_ROTATE, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), FF_DPP_ROTATE, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Does system `sys` evaluate in precision `prec` this cycle?
__device__ __forceinline__ bool eval_active(const Args& a, int sys, int prec) {
    if (a.direct) return a.direct_prec == prec;
    const Ctl* c = ctl_at(a, sys);
    return c->action == ACT_EVAL && c->prec == prec && c->target >= 0 && c->target < kNumSlots;
}

// Coordinates of system `si` for this evaluation ([n][3], local atom index).
__device__ __forceinline__ const double* eval_coords(const Args& a, int sys, const SysInfo& si) {
    if (a.direct) return a.xyz_in + 3 * (size_t)si.uoff;
    return vec(a, V_X0 + ctl_at(a, sys)->target, si);
}

__device__ __forceinline__ void load_pos(const double* X, int32_t atom, int32_t n, double* p) {
    if (atom < n) {
        p[0] = X[3 * (size_t)atom];
        p[1] = X[3 * (size_t)atom + 1];
        p[2] = X[3 * (size_t)atom + 2];
    } else {
        pad_position(atom, n, p);
    }
}

// ------------------------------------------------------------------ bonded
// One thread per bond, angle or dihedral; FP64.  The gradient of each term
// on each of its atoms goes to its own slot (no scatter), the energy to a
// per-block partial.
// Energy of bonded term t (bonds, then angles, then dihedrals) and its
// gradient on each of its atoms, written to the term's own slots.
__device__ double bonded_term(const Args& a, const double* X, const SysInfo& si, int t) {
    const Layout& L = a.L;
    double e = 0.0;
    double* FB = at<double>(a.ws, L.off_fb);
    if (t < si.n_bonds) {
        t += si.bond0;
        const int2 b = at<int2>(a.ws, L.off_bond)[t];
        const double2 kp = at<double2>(a.ws, L.off_bondp)[t];   // (K, r0)
        double d[3], r2 = 0.0;
        for (int c = 0; c < 3; ++c) { d[c] = X[3 * b.x + c] - X[3 * b.y + c]; r2 += d[c] * d[c]; }
        const double r = sqrt(r2);
        const double dr = r - kp.y;
        e = kp.x * dr * dr;
        const double s = 2.0 * kp.x * dr / r;
        double* o = FB + 6 * (size_t)t;
        for (int c = 0; c < 3; ++c) { o[c] = s * d[c]; o[3 + c] = -s * d[c]; }
    } else if (t < si.n_bonds + si.n_angles) {
        const int k = t - si.n_bonds + si.angle0;
        const int* ia = at<int>(a.ws, L.off_angle) + 3 * k;
        const double2 kp = at<double2>(a.ws, L.off_anglep)[k];  // (K, theta0)
        double u[3], v[3];
        for (int c = 0; c < 3; ++c) {
            u[c] = X[3 * ia[0] + c] - X[3 * ia[1] + c];
            v[c] = X[3 * ia[2] + c] - X[3 * ia[1] + c];
        }
        // w = u x v; theta = atan2(|w|, u.v);
        // d theta/d x_i = (u x w)/(|u|^2 |w|), d theta/d x_k = -(v x w)/(|v|^2 |w|)
        const double w[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
        const double nw = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        const double uv = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
        const double th = atan2(nw, uv);
        const double dth = th - kp.y;
        e = kp.x * dth * dth;
        const double de = 2.0 * kp.x * dth;
        const double uxw[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
        const double vxw[3] = {v[1] * w[2] - v[2] * w[1], v[2] * w[0] - v[0] * w[2], v[0] * w[1] - v[1] * w[0]};
        const double si = de / (uu * nw), sk = -de / (vv * nw);
        double* o = FB + 6 * (size_t)L.n_bonds + 9 * (size_t)k;
        for (int c = 0; c < 3; ++c) {
            const double gi = si * uxw[c], gk = sk * vxw[c];
            o[c] = gi;
            o[3 + c] = -(gi + gk);
            o[6 + c] = gk;
        }
    } else if (t < si.n_bonds + si.n_angles + si.n_dihedrals) {
        const int k = t - si.n_bonds - si.n_angles + si.dih0;
        const int* id = at<int>(a.ws, L.off_dih) + 4 * k;
        const double* V = at<double>(a.ws, L.off_dihp) + 4 * k;
        // F = x_a - x_b, G = x_b - x_c, H = x_d - x_c (Blondel and Karplus 1996)
        double F[3], G[3], H[3];
        for (int c = 0; c < 3; ++c) {
            F[c] = X[3 * id[0] + c] - X[3 * id[1] + c];
            G[c] = X[3 * id[1] + c] - X[3 * id[2] + c];
            H[c] = X[3 * id[3] + c] - X[3 * id[2] + c];
        }
        const double A[3] = {F[1] * G[2] - F[2] * G[1], F[2] * G[0] - F[0] * G[2], F[0] * G[1] - F[1] * G[0]};
        const double Bv[3] = {H[1] * G[2] - H[2] * G[1], H[2] * G[0] - H[0] * G[2], H[0] * G[1] - H[1] * G[0]};
        const double AA = A[0] * A[0] + A[1] * A[1] + A[2] * A[2];
        const double BB = Bv[0] * Bv[0] + Bv[1] * Bv[1] + Bv[2] * Bv[2];
        const double GG = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
        const double nG = sqrt(GG);
        // cos phi = A.B/(|A||B|); sin phi from (B x A).G/|G| (cis = 0)
        const double AxB_G = (Bv[1] * A[2] - Bv[2] * A[1]) * G[0] + (Bv[2] * A[0] - Bv[0] * A[2]) * G[1] +
                             (Bv[0] * A[1] - Bv[1] * A[0]) * G[2];
        const double phi = atan2(AxB_G / nG, A[0] * Bv[0] + A[1] * Bv[1] + A[2] * Bv[2]);
        double s1, c1, s2, c2, s3, c3, s4, c4;
        sincos(phi, &s1, &c1);
        sincos(2.0 * phi, &s2, &c2);
        sincos(3.0 * phi, &s3, &c3);
        sincos(4.0 * phi, &s4, &c4);
        e = 0.5 * (V[0] * (1.0 + c1) + V[1] * (1.0 - c2) + V[2] * (1.0 + c3) + V[3] * (1.0 - c4));
        const double de = 0.5 * (-V[0] * s1 + 2.0 * V[1] * s2 - 3.0 * V[2] * s3 + 4.0 * V[3] * s4);
        const double FG = F[0] * G[0] + F[1] * G[1] + F[2] * G[2];
        const double HG = H[0] * G[0] + H[1] * G[1] + H[2] * G[2];
        double* o = FB + 6 * (size_t)L.n_bonds + 9 * (size_t)L.n_angles + 12 * (size_t)k;
        for (int c = 0; c < 3; ++c) {
            const double ga = -nG / AA * A[c];
            const double gd = nG / BB * Bv[c];
            const double gb = nG / AA * A[c] + FG / (AA * nG) * A[c] - HG / (BB * nG) * Bv[c];
            const double gc = HG / (BB * nG) * Bv[c] - FG / (AA * nG) * A[c] - nG / BB * Bv[c];
            o[c] = de * ga;
            o[3 + c] = de * gb;
            o[6 + c] = de * gc;
            o[9 + c] = de * gd;
        }
    }
    return e;
}

__device__ void bonded_block(const Args& a, const double* X, const SysInfo& si, int blk, int nthreads) {
    double e = 0.0;
    const int first = blk * kBondedPerBlock;
    for (int t = first + (int)threadIdx.x; t < first + kBondedPerBlock; t += nthreads) e += bonded_term(a, X, si, t);
    // deterministic block sum of the term energies
    __shared__ double red[kBondedPerBlock];
    red[threadIdx.x] = e;
    __syncthreads();
    for (int s = nthreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) at<double>(a.ws, a.L.off_eb)[si.eb0 + blk] = red[0];
}

// Bonded terms of one evaluation (any precision mode: always FP64).
// Grid: every bonded block of every system (flat, map_bonded).
__global__ void __launch_bounds__(kBondedPerBlock) k_bonded(Args a) {
    const int2 m = at<int2>(a.ws, a.L.off_map_bonded)[blockIdx.x];
    const int sys = m.x;
    const SysInfo si = sys_info(a)[sys];
    if (!(eval_active(a, sys, 0) || eval_active(a, sys, 1))) return;
    bonded_block(a, eval_coords(a, sys, si), si, m.y, kBondedPerBlock);
}

// ---------------------------------------------------------------- FP32 pairs

// i-atoms of one lane: high halves of the coordinates and the per-atom
// factors stay in registers; the low halves live in LDS (s_ilo) because only
// the rare close-pair path reads them.
template <int IPL>
struct IAtoms32 {
    float xh[IPL], yh[IPL], zh[IPL];
    float a12[IPL], b6[IPL], q[IPL];     // 12 c12, 6 c6, q^
};

// A pair closer than sqrt(kCorrR2) by the high halves: redo the displacement
// with both halves in FP64.  Below sqrt(kClashR2) the whole pair is evaluated
// in FP64 (clash energies reach 1e15 kcal/mol at the start of a minimization)
// and the FP32 path is switched off for it by r2 = inf.
template <int IPL>
__device__ __forceinline__ void close_pair32(const IAtoms32<IPL>& I, int k, float4 pj, float4 lo, float4 ilo,
                                          float2 cj, float& dx, float& dy, float& dz, float& r2,
                                          double& gx, double& gy, double& gz, double& e64,
                                          float& fjx, float& fjy, float& fjz) {
    const double ddx = ((double)pj.x - (double)I.xh[k]) + ((double)lo.x - (double)ilo.x);
    const double ddy = ((double)pj.y - (double)I.yh[k]) + ((double)lo.y - (double)ilo.y);
    const double ddz = ((double)pj.z - (double)I.zh[k]) + ((double)lo.z - (double)ilo.z);
    const double rr = ddx * ddx + ddy * ddy + ddz * ddz;
    if (rr < kClashR2) {
        const double rinv = 1.0 / sqrt(rr);
        const double rinv2 = rinv * rinv;
        const double rinv6 = rinv2 * rinv2 * rinv2;
        const double A = (double)I.a12[k] * (double)cj.x, B = (double)I.b6[k] * (double)cj.y;
        const double u = A * rinv6 - B;
        const double ec = (double)I.q[k] * (double)pj.w * rinv;
        e64 += (u - B) * rinv6 * (1.0 / 12.0) + ec;
        const double f = (u * rinv6 + ec) * rinv2;
        gx += f * ddx; gy += f * ddy; gz += f * ddz;
        fjx -= (float)(f * ddx); fjy -= (float)(f * ddy); fjz -= (float)(f * ddz);
        r2 = __builtin_inff();
    } else {
        dx = (float)ddx; dy = (float)ddy; dz = (float)ddz;
        r2 = __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, dx * dx));
    }
}

template <int IPL, bool MASKED, bool CHECK, bool FAR = false>
__device__ __forceinline__ void tile32(const float4* __restrict__ s_xq, const float2* __restrict__ s_c,
                                       const float4* __restrict__ s_lo, const float4* __restrict__ s_ilo,
                                       int lane, int il0, int i0, int J0, const uint64_t* __restrict__ EX,
                                       const uint64_t* __restrict__ s_far,
                                       const IAtoms32<IPL>& I, float (&fx)[IPL], float (&fy)[IPL],
                                       float (&fz)[IPL], double (&gx)[IPL], double (&gy)[IPL],
                                       double (&gz)[IPL], float& fjx, float& fjy, float& fjz,
                                       float& elj, float& ec32, double& e64) {
    uint64_t excl[IPL];
    if (MASKED) {
#pragma unroll
        for (int k = 0; k < IPL; ++k) excl[k] = EX[i0 + k * 64];
    }
#pragma unroll kUnroll32<IPL>
    for (int s = 0; s < kTile; ++s) {
        const int js = lane + s;
        const float4 pj = s_xq[js];
        const float2 cj = s_c[js];
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
            float dx = pj.x - I.xh[k];
            float dy = pj.y - I.yh[k];
            float dz = pj.z - I.zh[k];
            float r2 = __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, dx * dx));
            if (MASKED) {
                const int delta = J0 + (js & (kTile - 1)) - (i0 + k * 64);
                const unsigned dm1 = (unsigned)(delta - 1);
                bool ex = dm1 < (unsigned)kExclWindow && ((excl[k] >> (dm1 & 63u)) & 1ull);
                // far exclusions: this unit's mask of the i-atom, read from LDS
                // every step (a register copy would raise the kernel's VGPRs)
                if (FAR) ex = ex || ((s_far[il0 + k * 64] >> (js & (kTile - 1))) & 1ull);
                r2 = (delta > 0 && !ex) ? r2 : __builtin_inff();
            }
            if (CHECK && r2 < kCorrR2)
                close_pair32<IPL>(I, k, pj, s_lo[js], s_ilo[il0 + k * 64], cj, dx, dy, dz, r2, gx[k], gy[k],
                                  gz[k], e64, fjx, fjy, fjz);
            const float rinv = __builtin_amdgcn_rsqf(r2);
            const float rinv2 = rinv * rinv;
            const float rinv6 = rinv2 * rinv2 * rinv2;
            const float A = I.a12[k] * cj.x;
            const float B = I.b6[k] * cj.y;
            const float ec = I.q[k] * pj.w * rinv;
            const float u = __fmaf_rn(A, rinv6, -B);
            const float f = __fmaf_rn(u, rinv6, ec) * rinv2;
            elj = __fmaf_rn(u - B, rinv6, elj);
            ec32 += ec;
            fx[k] = __fmaf_rn(f, dx, fx[k]);
            fy[k] = __fmaf_rn(f, dy, fy[k]);
            fz[k] = __fmaf_rn(f, dz, fz[k]);
            fjx = __fmaf_rn(-f, dx, fjx);
            fjy = __fmaf_rn(-f, dy, fjy);
            fjz = __fmaf_rn(-f, dz, fjz);
        }
        fjx = rotate_down(fjx);
        fjy = rotate_down(fjy);
        fjz = rotate_down(fjz);
    }
}

__device__ __forceinline__ float wave_minf(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_maxf(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ void split(double v, float& hi, float& lo) {
    hi = (float)v;
    lo = (float)(v - (double)hi);
}

template <int WAVES>
__device__ __forceinline__ void block_energy_store(double e, double* out) {
    __shared__ double red[64 * WAVES];
    red[threadIdx.x] = e;
    __syncthreads();
    for (int s = 32 * WAVES; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// HAS_FAR: the context has excluded pairs more than kExclWindow apart (the
// kernel then checks every tile for a far-exclusion mask; the check costs a
// few registers, so contexts without such pairs run the kernel without it).
// Occupancy floor: with two atoms per lane the kernel fits 168 VGPRs, three
// wavefronts per SIMD, but the compiler's own choice exceeds that by a few
// registers and loses a wavefront.  (The far-exclusion variant would spill
// at 168 and keeps the compiler's choice.)
template <int IPL, bool HAS_FAR>
constexpr int kPair32MinWaves = IPL == 2 && !HAS_FAR ? 3 : 1;

template <int WAVES, int IPL, bool HAS_FAR>
__global__ void __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(kPair32MinWaves<IPL, HAS_FAR>)))
k_pair32(Args a) {
    const Layout& L = a.L;
    const int wg = blockIdx.x;
    const ChunkInfo ch = at<ChunkInfo>(a.ws, L.off_chunks[0])[wg];
    if (!eval_active(a, ch.sys, 1)) return;
    const SysInfo si = sys_info(a)[ch.sys];
    const double* X = eval_coords(a, ch.sys, si);
    constexpr int B = 64 * WAVES * IPL;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = si.n, aoff = si.aoff;
    const float* C12 = at<float>(a.ws, L.off_c12);
    const float* C6 = at<float>(a.ws, L.off_c6);
    const float* Q = at<float>(a.ws, L.off_q);
    const uint64_t* EX = at<uint64_t>(a.ws, L.off_excl);
    const int32_t* FU = at<int32_t>(a.ws, L.off_far_unit);
    const uint64_t* FM = at<uint64_t>(a.ws, L.off_far_mask);
    const int I0 = ch.row * B;

    IAtoms32<IPL> I;
    double gx[IPL], gy[IPL], gz[IPL];
    __shared__ float4 s_ilo[B];
    const int il0 = wave * 64 * IPL + lane;     // local index of this lane's first i-atom
    const int i0 = I0 + il0;
    // Coordinates relative to the I-block's first atom: the FP32 displacement
    // of a pair beyond the double-single range then carries the rounding of
    // the pair's own distance, not of the atoms' distance from the origin
    // (for a 1e-3 A step of a relaxed 10,000-atom chain this cuts the rounding
    // noise of the energy difference about 60-fold).
    // (kept in LDS for the j-tile staging: registers are at their limit)
    __shared__ double s_org[3];
    double org[3];
    load_pos(X, I0 - aoff, n, org);
    if (threadIdx.x == 0) { s_org[0] = org[0]; s_org[1] = org[1]; s_org[2] = org[2]; }
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int i = i0 + k * 64;
        double p[3];
        load_pos(X, i - aoff, n, p);
        float4 lo;
        split(p[0] - org[0], I.xh[k], lo.x);
        split(p[1] - org[1], I.yh[k], lo.y);
        split(p[2] - org[2], I.zh[k], lo.z);
        lo.w = 0.0f;
        s_ilo[il0 + k * 64] = lo;
        I.a12[k] = 12.0f * C12[i]; I.b6[k] = 6.0f * C6[i]; I.q[k] = Q[i];
        gx[k] = gy[k] = gz[k] = 0.0;
    }
    // bounding box of this wave's i-atoms: a j-tile whose box is farther than
    // sqrt(kCorrR2) cannot hold a close pair, so it runs the unchecked body
    float ib[6];
    ib[0] = ib[3] = I.xh[0];
    ib[1] = ib[4] = I.yh[0];
    ib[2] = ib[5] = I.zh[0];
#pragma unroll
    for (int k = 1; k < IPL; ++k) {
        ib[0] = fminf(ib[0], I.xh[k]); ib[3] = fmaxf(ib[3], I.xh[k]);
        ib[1] = fminf(ib[1], I.yh[k]); ib[4] = fmaxf(ib[4], I.yh[k]);
        ib[2] = fminf(ib[2], I.zh[k]); ib[5] = fmaxf(ib[5], I.zh[k]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) { ib[c] = wave_minf(ib[c]); ib[3 + c] = wave_maxf(ib[3 + c]); }
    __shared__ float s_jbox[6];
    __shared__ float4 s_xq[2 * kTile];
    __shared__ float2 s_c[2 * kTile];
    __shared__ float4 s_lo[2 * kTile];
    __shared__ float s_fj[WAVES][3][kTile];
    __shared__ uint64_t s_far[HAS_FAR ? B : 1];      // far-exclusion masks of a far unit
    double e64 = 0.0;
    const int t_masked_end = (I0 + B) / kTile + 1;   // tiles that can hold j <= i or exclusions
    for (int t = ch.t_begin; t < ch.t_end; ++t) {
        const int J0 = t * kTile;
        __syncthreads();
        if (threadIdx.x < kTile) {
            const int j = J0 + threadIdx.x;
            double p[3];
            load_pos(X, j - aoff, n, p);
            float4 h, l;
            split(p[0] - s_org[0], h.x, l.x);
            split(p[1] - s_org[1], h.y, l.y);
            split(p[2] - s_org[2], h.z, l.z);
            h.w = Q[j];
            l.w = 0.0f;
            const float2 c = make_float2(C12[j], C6[j]);
            s_xq[threadIdx.x] = h; s_xq[threadIdx.x + kTile] = h;
            s_lo[threadIdx.x] = l; s_lo[threadIdx.x + kTile] = l;
            s_c[threadIdx.x] = c;  s_c[threadIdx.x + kTile] = c;
            const float b0 = wave_minf(h.x), b1 = wave_minf(h.y), b2 = wave_minf(h.z);
            const float b3 = wave_maxf(h.x), b4 = wave_maxf(h.y), b5 = wave_maxf(h.z);
            if (threadIdx.x == 0) {
                s_jbox[0] = b0; s_jbox[1] = b1; s_jbox[2] = b2;
                s_jbox[3] = b3; s_jbox[4] = b4; s_jbox[5] = b5;
            }
        }
        __syncthreads();
        float fx[IPL], fy[IPL], fz[IPL];
#pragma unroll
        for (int k = 0; k < IPL; ++k) fx[k] = fy[k] = fz[k] = 0.0f;
        float fjx = 0.0f, fjy = 0.0f, fjz = 0.0f, elj = 0.0f, ec32 = 0.0f;
        const float gxb = fmaxf(0.0f, fmaxf(s_jbox[0] - ib[3], ib[0] - s_jbox[3]));
        const float gyb = fmaxf(0.0f, fmaxf(s_jbox[1] - ib[4], ib[1] - s_jbox[4]));
        const float gzb = fmaxf(0.0f, fmaxf(s_jbox[2] - ib[5], ib[2] - s_jbox[5]));
        const bool far = gxb * gxb + gyb * gyb + gzb * gzb >= kCorrR2;
        const int fu = HAS_FAR ? FU[ch.unit_base + t - ch.t_begin] : -1;
        if (HAS_FAR && fu >= 0) {
            // the unit holds excluded pairs more than kExclWindow apart: each
            // lane copies the masks of its i-atoms (and only reads its own)
#pragma unroll
            for (int k = 0; k < IPL; ++k) s_far[il0 + k * 64] = FM[(size_t)fu * B + il0 + k * 64];
            tile32<IPL, true, true, true>(s_xq, s_c, s_lo, s_ilo, lane, il0, i0, J0, EX, s_far, I, fx, fy, fz, gx,
                                          gy, gz, fjx, fjy, fjz, elj, ec32, e64);
        } else if (t < t_masked_end)
            tile32<IPL, true, true>(s_xq, s_c, s_lo, s_ilo, lane, il0, i0, J0, EX, s_far, I, fx, fy, fz, gx, gy, gz,
                                    fjx, fjy, fjz, elj, ec32, e64);
        else if (!far)
            tile32<IPL, false, true>(s_xq, s_c, s_lo, s_ilo, lane, il0, i0, J0, EX, s_far, I, fx, fy, fz, gx, gy, gz,
                                     fjx, fjy, fjz, elj, ec32, e64);
        else
            tile32<IPL, false, false>(s_xq, s_c, s_lo, s_ilo, lane, il0, i0, J0, EX, s_far, I, fx, fy, fz, gx, gy, gz,
                                      fjx, fjy, fjz, elj, ec32, e64);
#pragma unroll
        for (int k = 0; k < IPL; ++k) { gx[k] += fx[k]; gy[k] += fy[k]; gz[k] += fz[k]; }
        e64 += (double)elj * (1.0 / 12.0) + (double)ec32;
        s_fj[wave][0][lane] = fjx;
        s_fj[wave][1][lane] = fjy;
        s_fj[wave][2][lane] = fjz;
        __syncthreads();
        if (wave == 0) {
            double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) {
                sx += (double)s_fj[w][0][lane];
                sy += (double)s_fj[w][1][lane];
                sz += (double)s_fj[w][2][lane];
            }
            float* pj = at<float>(a.ws, L.off_pj) + ((size_t)(ch.unit_base + t - ch.t_begin) * kTile + lane) * 3;
            pj[0] = (float)sx; pj[1] = (float)sy; pj[2] = (float)sz;
        }
    }
    // FP32 mode stores its partial sums in single precision (they are FP32
    // tile sums already); the finalize adds them up in FP64
    float* pi = at<float>(a.ws, L.off_pi) + (size_t)ch.slot * B * 3;
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int il = wave * 64 * IPL + k * 64 + lane;
        pi[3 * il] = (float)gx[k]; pi[3 * il + 1] = (float)gy[k]; pi[3 * il + 2] = (float)gz[k];
    }
    block_energy_store<WAVES>(e64, at<double>(a.ws, L.off_ep) + ch.slot);
}

// ---------------------------------------------------------------- FP64 pairs

// 1/sqrt(x) for finite x > 0: v_rsq_f64, then y (1 + e/2 + 3e^2/8) with
// e = 1 - x y^2 (the error of the estimate enters cubed), the same
// arithmetic rsqrt uses for such x.
__device__ __forceinline__ double rsqrt_finite(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

template <int IPL, bool MASKED, bool FAR = false>
__device__ __forceinline__ void tile64(const double4* __restrict__ s_xq, const double2* __restrict__ s_c,
                                       int lane, int J0, const double (&xi)[IPL], const double (&yi)[IPL],
                                       const double (&zi)[IPL], const double (&a12i)[IPL],
                                       const double (&b6i)[IPL], const double (&qi)[IPL],
                                       const uint64_t (&excl)[IPL], const uint64_t (&fmask)[IPL], const int (&idx)[IPL],
                                       double (&gx)[IPL], double (&gy)[IPL], double (&gz)[IPL],
                                       double& fjx, double& fjy, double& fjz, double& elj, double& ecs) {
#pragma unroll 2
    for (int s = 0; s < kTile; ++s) {
        const int js = lane + s;
        const double4 pj = s_xq[js];
        const double2 cj = s_c[js];
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
            const double dx = pj.x - xi[k], dy = pj.y - yi[k], dz = pj.z - zi[k];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (MASKED) {
                const int delta = J0 + (js & (kTile - 1)) - idx[k];
                const unsigned dm1 = (unsigned)(delta - 1);
                bool ex = dm1 < (unsigned)kExclWindow && ((excl[k] >> (dm1 & 63u)) & 1ull);
                if (FAR) ex = ex || ((fmask[k] >> (js & (kTile - 1))) & 1ull);
                r2 = (delta > 0 && !ex) ? r2 : __builtin_inf();
            }
            // unmasked tiles hold no excluded pair, so r2 is finite and
            // positive (or 0 for coincident atoms, which gives a non-finite
            // energy either way): the hardware estimate and one correction
            // step, without the special-value handling rsqrt adds
            const double rinv = MASKED ? rsqrt(r2) : rsqrt_finite(r2);
            const double rinv2 = rinv * rinv;
            const double rinv6 = rinv2 * rinv2 * rinv2;
            const double A = a12i[k] * cj.x;
            const double B = b6i[k] * cj.y;
            const double ec = qi[k] * pj.w * rinv;
            const double u = fma(A, rinv6, -B);
            const double f = fma(u, rinv6, ec) * rinv2;
            elj = fma(u - B, rinv6, elj);
            ecs += ec;
            gx[k] += f * dx; gy[k] += f * dy; gz[k] += f * dz;
            fjx -= f * dx; fjy -= f * dy; fjz -= f * dz;
        }
        fjx = rotate_down(fjx);
        fjy = rotate_down(fjy);
        fjz = rotate_down(fjz);
    }
}

template <int WAVES, int IPL>
__device__ __forceinline__ void pair64_chunk(const Args& a, int wg) {
    const Layout& L = a.L;
    const ChunkInfo ch = at<ChunkInfo>(a.ws, L.off_chunks[1])[wg];
    if (!eval_active(a, ch.sys, 0)) return;
    const SysInfo si = sys_info(a)[ch.sys];
    const double* X = eval_coords(a, ch.sys, si);
    constexpr int B = 64 * WAVES * IPL;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = si.n, aoff = si.aoff;
    const double* C12 = at<double>(a.ws, L.off_c12d);
    const double* C6 = at<double>(a.ws, L.off_c6d);
    const double* Q = at<double>(a.ws, L.off_qd);
    const uint64_t* EX = at<uint64_t>(a.ws, L.off_excl);
    const int32_t* FU = at<int32_t>(a.ws, L.off_far_unit);
    const uint64_t* FM = at<uint64_t>(a.ws, L.off_far_mask);
    const uint64_t fnone[IPL] = {};
    const int I0 = ch.row * B;

    double xi[IPL], yi[IPL], zi[IPL], a12i[IPL], b6i[IPL], qi[IPL], gx[IPL], gy[IPL], gz[IPL];
    uint64_t excl[IPL];
    int idx[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int i = I0 + wave * 64 * IPL + k * 64 + lane;
        double p[3];
        load_pos(X, i - aoff, n, p);
        xi[k] = p[0]; yi[k] = p[1]; zi[k] = p[2];
        a12i[k] = 12.0 * C12[i]; b6i[k] = 6.0 * C6[i]; qi[k] = Q[i];
        excl[k] = EX[i];
        idx[k] = i;
        gx[k] = gy[k] = gz[k] = 0.0;
    }
    __shared__ double4 s_xq[2 * kTile];
    __shared__ double2 s_c[2 * kTile];
    __shared__ double s_fj[WAVES][3][kTile];
    double elj = 0.0, ecs = 0.0;     // 12 x Lennard-Jones energy, Coulomb energy
    const int t_masked_end = (I0 + B) / kTile + 1;
    for (int t = ch.t_begin; t < ch.t_end; ++t) {
        const int J0 = t * kTile;
        __syncthreads();
        if (threadIdx.x < kTile) {
            const int j = J0 + threadIdx.x;
            double p[3];
            load_pos(X, j - aoff, n, p);
            const double4 h = make_double4(p[0], p[1], p[2], Q[j]);
            const double2 c = make_double2(C12[j], C6[j]);
            s_xq[threadIdx.x] = h; s_xq[threadIdx.x + kTile] = h;
            s_c[threadIdx.x] = c;  s_c[threadIdx.x + kTile] = c;
        }
        __syncthreads();
        double fjx = 0.0, fjy = 0.0, fjz = 0.0;
        const int fu = FU[ch.unit_base + t - ch.t_begin];
        if (fu >= 0) {
            uint64_t fmask[IPL];
#pragma unroll
            for (int k = 0; k < IPL; ++k) fmask[k] = FM[(size_t)fu * B + wave * 64 * IPL + k * 64 + lane];
            tile64<IPL, true, true>(s_xq, s_c, lane, J0, xi, yi, zi, a12i, b6i, qi, excl, fmask, idx, gx, gy, gz,
                                    fjx, fjy, fjz, elj, ecs);
        } else if (t < t_masked_end) {
            tile64<IPL, true>(s_xq, s_c, lane, J0, xi, yi, zi, a12i, b6i, qi, excl, fnone, idx, gx, gy, gz, fjx, fjy,
                              fjz, elj, ecs);
        } else {
            tile64<IPL, false>(s_xq, s_c, lane, J0, xi, yi, zi, a12i, b6i, qi, excl, fnone, idx, gx, gy, gz, fjx,
                               fjy, fjz, elj, ecs);
        }
        s_fj[wave][0][lane] = fjx;
        s_fj[wave][1][lane] = fjy;
        s_fj[wave][2][lane] = fjz;
        __syncthreads();
        if (wave == 0) {
            double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) { sx += s_fj[w][0][lane]; sy += s_fj[w][1][lane]; sz += s_fj[w][2][lane]; }
            double* pj = at<double>(a.ws, L.off_pj) + ((size_t)(ch.unit_base + t - ch.t_begin) * kTile + lane) * 3;
            pj[0] = sx; pj[1] = sy; pj[2] = sz;
        }
    }
    double* pi = at<double>(a.ws, L.off_pi) + (size_t)ch.slot * B * 3;
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int il = wave * 64 * IPL + k * 64 + lane;
        pi[3 * il] = gx[k]; pi[3 * il + 1] = gy[k]; pi[3 * il + 2] = gz[k];
    }
    block_energy_store<WAVES>(elj * (1.0 / 12.0) + ecs, at<double>(a.ws, L.off_ep) + ch.slot);
}

// The FP64 kernel walks the chunks with a grid stride: in FP32 mode (and in
// cycles without an evaluation) its workgroups only check and exit, and a
// capped grid keeps that cheap.  The cap allows 16384 wavefronts (four per
// SIMD) and at least 4096 workgroups: one-wavefront workgroups (the batch
// tiling) would otherwise leave three quarters of the chip idle.
constexpr int kPair64Waves = 16384;
__host__ __device__ constexpr int pair64_grid_cap(int waves) {
    return kPair64Waves / waves > 4096 ? kPair64Waves / waves : 4096;
}

template <int WAVES, int IPL>
__global__ void __launch_bounds__(64 * WAVES) k_pair64(Args a) {
    // one activity check for the whole launch: a single system's, or, for a
    // batch, whether any system evaluates in FP64 this cycle (the threads
    // read the control blocks side by side); then each chunk checks its own
    // system
    if (a.L.n_sys == 1) {
        if (!eval_active(a, 0, 0)) return;
    } else if (!a.direct) {
        int any = 0;
        for (int s = threadIdx.x; s < a.L.n_sys && !any; s += blockDim.x) any = eval_active(a, s, 0) ? 1 : 0;
        if (!__syncthreads_or(any)) return;
    }
    for (int wg = blockIdx.x; wg < a.L.n_chunks[1]; wg += gridDim.x) pair64_chunk<WAVES, IPL>(a, wg);
}

// ------------------------------------------------------------- host launch
// Tile configurations (index = Layout::cfg): I-block of B = 64 * waves * ipl
// atoms.  Both precisions use the same B (the same rows and units); each
// walks its own chunk table.
#define FF_PAIR_CASE(ID)                                                                           \
    case ID: {                                                                                     \
        constexpr TileConfig T = kTileConfigs[ID];                                                 \
        if (prec && a.L.n_far_units > 0)                                                              \
            hipLaunchKernelGGL((k_pair32<T.waves32, T.ipl32, true>), dim3(grid), dim3(64 * T.waves32), 0, s, a); \
        else if (prec)                                                                                \
            hipLaunchKernelGGL((k_pair32<T.waves32, T.ipl32, false>), dim3(grid), dim3(64 * T.waves32), 0, s, a); \
        else hipLaunchKernelGGL((k_pair64<T.waves64, T.ipl64>),                                        \
                                dim3(grid < pair64_grid_cap(T.waves64) ? grid : pair64_grid_cap(T.waves64)), \
                                dim3(64 * T.waves64), 0, s, a);                                                 \
        break;                                                                                     \
    }

hipError_t launch_pair(const Args& a, int prec, hipStream_t s) {
    const int grid = a.L.n_chunks[prec ? 0 : 1];
    switch (a.L.cfg) {
        FF_PAIR_CASE(0)
        FF_PAIR_CASE(1)
        FF_PAIR_CASE(2)
        FF_PAIR_CASE(3)
        FF_PAIR_CASE(4)
        FF_PAIR_CASE(5)
        FF_PAIR_CASE(6)
        FF_PAIR_CASE(7)
        FF_PAIR_CASE(8)
        FF_PAIR_CASE(9)
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_bonded(const Args& a, hipStream_t s) {
    hipLaunchKernelGGL(k_bonded, dim3(a.L.n_bonded_blocks), dim3(kBondedPerBlock), 0, s, a);
    return hipGetLastError();
}


}  // namespace ff
