// Learned warm start (beyond the paper): per-atom features from the 16
// nearest atoms of the same system, a 3-layer perceptron (BF16 weights and
// activations, FP32 accumulation on the matrix cores) that predicts a
// displacement of every atom, its training kernels, and the application of
// the displacement before a minimization.  The minimizer keeps the last word: a
// displaced start is kept per system only where the energy prefers it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "ff.h"
#include "ff_learn.h"

namespace ff {

// ------------------------------------------------------------------ BF16
// Round to nearest even from FP32 (values here are finite).
__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// ------------------------------------------------------------- features
// One thread per atom: the 16 nearest other atoms of its system by FP64
// squared distance (ties to the lower index), then
//   f[0..2]          = q, sigma - 3.5, 10 eps of the atom,
//   f[3+7k .. 9+7k]  = (x_j - x_i)/4 (3 values), r/4, q_j, sigma_j - 3.5, 10 eps_j
// for the k-th neighbour (zeros for missing neighbours), then the place of the
// atom in its system: (x_i - c)/16 (3 values) and |x_i - c|/16 with c the
// centroid (a sum in atom order divided by n), and n/4096; zeros up to
// FF_LEARN_FEATURES.  Each value is rounded FP64 -> FP32 -> BF16.
__global__ void k_features(const double* __restrict__ xyz, const double* __restrict__ q,
                           const double* __restrict__ sig, const double* __restrict__ eps,
                           const int32_t* __restrict__ sys_first, const int32_t* __restrict__ atom_sys, int n_total,
                           uint16_t* __restrict__ feat, int32_t* __restrict__ nbr) {
#pragma clang fp contract(off)
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_total) return;
    const int s = atom_sys[i];
    const int j0 = sys_first[s], j1 = sys_first[s + 1];
    const double xi = xyz[3 * (size_t)i], yi = xyz[3 * (size_t)i + 1], zi = xyz[3 * (size_t)i + 2];
    double bd[FF_LEARN_NEIGHBORS];
    int bj[FF_LEARN_NEIGHBORS];
#pragma unroll
    for (int k = 0; k < FF_LEARN_NEIGHBORS; ++k) { bd[k] = __builtin_inf(); bj[k] = -1; }
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int j = j0; j < j1; ++j) {
        const double xj = xyz[3 * (size_t)j], yj = xyz[3 * (size_t)j + 1], zj = xyz[3 * (size_t)j + 2];
        sx += xj; sy += yj; sz += zj;
        if (j == i) continue;
        const double dx = xj - xi, dy = yj - yi, dz = zj - zi;
        const double d2 = dx * dx + dy * dy + dz * dz;
        // candidates arrive in increasing j, so a tie never displaces an entry
        if (!(d2 < bd[FF_LEARN_NEIGHBORS - 1])) continue;
        double cd = d2;
        int cj = j;
#pragma unroll
        for (int k = 0; k < FF_LEARN_NEIGHBORS; ++k) {
            if (cd < bd[k]) {
                const double td = bd[k];
                const int tj = bj[k];
                bd[k] = cd; bj[k] = cj;
                cd = td; cj = tj;
            }
        }
    }
    uint16_t* f = feat + (size_t)i * FF_LEARN_FEATURES;
    f[0] = to_bf16((float)q[i]);
    f[1] = to_bf16((float)(sig[i] - 3.5));
    f[2] = to_bf16((float)(10.0 * eps[i]));
#pragma unroll
    for (int k = 0; k < FF_LEARN_NEIGHBORS; ++k) {
        const int j = bj[k];
        uint16_t* g = f + 3 + 7 * k;
        if (nbr) nbr[(size_t)i * FF_LEARN_NEIGHBORS + k] = j;
        if (j < 0) {
            for (int c = 0; c < 7; ++c) g[c] = 0;
            continue;
        }
        const double dx = xyz[3 * (size_t)j] - xi, dy = xyz[3 * (size_t)j + 1] - yi, dz = xyz[3 * (size_t)j + 2] - zi;
        g[0] = to_bf16((float)(dx / 4.0));
        g[1] = to_bf16((float)(dy / 4.0));
        g[2] = to_bf16((float)(dz / 4.0));
        g[3] = to_bf16((float)(sqrt(bd[k]) / 4.0));
        g[4] = to_bf16((float)q[j]);
        g[5] = to_bf16((float)(sig[j] - 3.5));
        g[6] = to_bf16((float)(10.0 * eps[j]));
    }
    const double n = (double)(j1 - j0);
    const double cx = xi - sx / n, cy = yi - sy / n, cz = zi - sz / n;
    uint16_t* h = f + 3 + 7 * FF_LEARN_NEIGHBORS;
    h[0] = to_bf16((float)(cx / 16.0));
    h[1] = to_bf16((float)(cy / 16.0));
    h[2] = to_bf16((float)(cz / 16.0));
    h[3] = to_bf16((float)(sqrt(cx * cx + cy * cy + cz * cz) / 16.0));
    h[4] = to_bf16((float)(n / 4096.0));
    for (int c = 8 + 7 * FF_LEARN_NEIGHBORS; c < FF_LEARN_FEATURES; ++c) f[c] = 0;
}

// ------------------------------------------------------------------ GEMM
// C[m][n] = sum_k A(m, k) B(k, n) with A(m, k) = A[m*sa0 + k*sa1] and
// B(k, n) = B[k*sb0 + n*sb1] (BF16), FP32 accumulation on the matrix cores
// (v_mfma_f32_16x16x16_bf16: lane l holds row l%16 / column l%16 and k =
// 4*(l/16)+q of its A / B fragment, rows 4*(l/16)+q of column l%16 of D).
// Epilogue: + bias[n] (FP32, optional), ReLU (optional), FP32 result to C
// (optional) and its BF16 rounding to Cb (optional).  One wavefront per
// 16x16 tile of C and per slice [y*kc, (y+1)*kc) of k (blockIdx.y = y);
// out-of-range rows, columns and k read as zero.  With several slices
// (P != null) each wave stores its raw FP32 sums to P[y][m][n] and
// k_splitk_reduce adds the slices in order and applies the epilogue, so the
// result does not depend on timing.
typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_gemm(int m, int n, int kdim, int kc, const uint16_t* __restrict__ A,
                                              long sa0, long sa1, const uint16_t* __restrict__ B, long sb0,
                                              long sb1, const float* __restrict__ bias, int relu,
                                              float* __restrict__ C, long ldc, uint16_t* __restrict__ Cb,
                                              long ldcb, float* __restrict__ P) {
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int tiles_n = (n + 15) / 16;
    const long tile = (long)blockIdx.x * 4 + wave;
    const int tm = (int)(tile / tiles_n), tn = (int)(tile % tiles_n);
    if ((long)tm * 16 >= m) return;
    const int row = tm * 16 + (l & 15), col = tn * 16 + (l & 15), kq = 4 * (l >> 4);
    const int k_lo = blockIdx.y * kc, k_hi = min(kdim, k_lo + kc);
    f32x4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = k_lo; k0 < k_hi; k0 += 16) {
        bf16x4_t av, bv;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = k0 + kq + q;
            av[q] = (row < m && k < k_hi) ? (short)A[row * sa0 + k * sa1] : (short)0;
            bv[q] = (col < n && k < k_hi) ? (short)B[k * sb0 + col * sb1] : (short)0;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = tm * 16 + kq + q;
        if (r >= m || col >= n) continue;
        float v = acc[q];
        if (P) {
            P[((long)blockIdx.y * m + r) * n + col] = v;
            continue;
        }
        if (bias) v += bias[col];
        if (relu) v = fmaxf(v, 0.0f);
        if (C) C[r * ldc + col] = v;
        if (Cb) Cb[r * ldcb + col] = to_bf16(v);
    }
}

__global__ void k_splitk_reduce(int m, int n, int slices, const float* __restrict__ P,
                                const float* __restrict__ bias, int relu, float* __restrict__ C, long ldc,
                                uint16_t* __restrict__ Cb, long ldcb) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)m * n) return;
    const int r = (int)(e / n), col = (int)(e - (long)r * n);
    float v = 0.0f;
    for (int y = 0; y < slices; ++y) v += P[(long)y * m * n + e];
    if (bias) v += bias[col];
    if (relu) v = fmaxf(v, 0.0f);
    if (C) C[r * ldc + col] = v;
    if (Cb) Cb[r * ldcb + col] = to_bf16(v);
}

// Scratch for the k slices of a product with few output tiles and a long k
// (the weight gradients): at most kMaxSlices slices of a 128 x 128 result.
constexpr int kMaxSlices = 64;
constexpr long kSplitFloats = (long)kMaxSlices * FF_LEARN_HIDDEN * FF_LEARN_HIDDEN;

// LDS-tiled product for operands whose elements run contiguously along k
// or along the other index (every product of the network): a workgroup
// computes a 64 x 64 block of C from 64 x 32 tiles of A and 32 x 64 tiles of
// B staged in LDS with 16-byte loads, each of its four wavefronts a 32 x 32
// quarter (2 x 2 matrix-core tiles) reading 8-byte fragments.  Both tiles are
// kept k-contiguous in LDS: element (r, k) at r * kLdk + k, rows padded to 40
// values so that the 16 rows a fragment read touches fall on different banks.
// A_K: A(i, k) = A[i * sa + k], else A[k * sa + i]; B_K: B(k, j) = B[j * sb + k],
// else B[k * sb + j].  Out-of-range elements load as zero.  k slices, the
// epilogue and the partial sums P as in k_gemm; kc is a multiple of 32.
constexpr int kGbm = 64, kGbn = 64, kGbk = 32, kLdk = kGbk + 8;

template <bool KCONT>
__device__ __forceinline__ void stage_tile(const uint16_t* __restrict__ g, long st, int r0, int r_end, int k0,
                                           int k_end, bool vec_ok, uint16_t* __restrict__ lds) {
    const int t = threadIdx.x;
    uint16_t v[8];
    if (KCONT) {
        // 64 rows x 32 k: thread t loads k [seg, seg + 8) of row t / 4
        const int r = t >> 2, seg = (t & 3) * 8;
        const int row = r0 + r, k = k0 + seg;
        if (vec_ok && row < r_end && k + 8 <= k_end) {
            *(uint4*)v = *(const uint4*)(g + row * st + k);
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = (row < r_end && k + q < k_end) ? g[row * st + k + q] : (uint16_t)0;
        }
        *(uint4*)(lds + r * kLdk + seg) = *(const uint4*)v;
    } else {
        // 32 k x 64 rows: thread t loads rows [seg, seg + 8) of k = t / 8
        const int kk = t >> 3, seg = (t & 7) * 8;
        const int k = k0 + kk, row = r0 + seg;
        if (vec_ok && k < k_end && row + 8 <= r_end) {
            *(uint4*)v = *(const uint4*)(g + k * st + row);
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = (k < k_end && row + q < r_end) ? g[k * st + row + q] : (uint16_t)0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) lds[(seg + q) * kLdk + kk] = v[q];
    }
}

template <bool A_K, bool B_K>
__global__ void __launch_bounds__(256) k_gemm_lds(int m, int n, int kdim, int kc, const uint16_t* __restrict__ A,
                                                  long sa, const uint16_t* __restrict__ B, long sb, int vec_ok,
                                                  const float* __restrict__ bias, int relu, float* __restrict__ C,
                                                  long ldc, uint16_t* __restrict__ Cb, long ldcb,
                                                  float* __restrict__ P) {
    __shared__ __attribute__((aligned(16))) uint16_t As[kGbm * kLdk];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kGbn * kLdk];
    const int tiles_n = (n + kGbn - 1) / kGbn;
    const int m0 = (int)(blockIdx.x / tiles_n) * kGbm, n0 = (int)(blockIdx.x % tiles_n) * kGbn;
    const int k_lo = blockIdx.y * kc, k_hi = min(kdim, k_lo + kc);
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int fr = l & 15, fk = 4 * (l >> 4);
    f32x4_t acc[2][2] = {};
    for (int k0 = k_lo; k0 < k_hi; k0 += kGbk) {
        stage_tile<A_K>(A, sa, m0, m, k0, k_hi, vec_ok, As);
        stage_tile<B_K>(B, sb, n0, n, k0, k_hi, vec_ok, Bs);
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kGbk; ks += 16) {
            bf16x4_t af[2], bf[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                af[u] = *(const bf16x4_t*)(As + (wm + 16 * u + fr) * kLdk + ks + fk);
                bf[u] = *(const bf16x4_t*)(Bs + (wn + 16 * u + fr) * kLdk + ks + fk);
            }
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int w = 0; w < 2; ++w)
                    acc[u][w] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[u], bf[w], acc[u][w], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int w = 0; w < 2; ++w)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = m0 + wm + 16 * u + fk + q, col = n0 + wn + 16 * w + fr;
                if (r >= m || col >= n) continue;
                float v = acc[u][w][q];
                if (P) {
                    P[((long)blockIdx.y * m + r) * n + col] = v;
                    continue;
                }
                if (bias) v += bias[col];
                if (relu) v = fmaxf(v, 0.0f);
                if (C) C[r * ldc + col] = v;
                if (Cb) Cb[r * ldcb + col] = to_bf16(v);
            }
}

hipError_t launch_gemm(int m, int n, int k, const uint16_t* A, long sa0, long sa1, const uint16_t* B, long sb0,
                       long sb1, const float* bias, int relu, float* C, long ldc, uint16_t* Cb, long ldcb,
                       hipStream_t s, float* split = nullptr, long split_floats = 0) {
    // the tiled kernel takes operands contiguous along one index, blocks of
    // at least 64 x 64 x 32; 16-byte loads where strides and bases allow
    const bool a_k = sa1 == 1, a_m = sa0 == 1 && !a_k, b_k = sb0 == 1, b_n = sb1 == 1 && !b_k;
    const bool tiled = (a_k || a_m) && (b_k || b_n) && m >= kGbm && n >= kGbn && k >= kGbk;
    const long blocks = tiled ? (long)((m + kGbm - 1) / kGbm) * ((n + kGbn - 1) / kGbn)
                              : ((long)((m + 15) / 16) * ((n + 15) / 16) + 3) / 4;
    int slices = 1;
    // split k when the output blocks alone cannot fill the chip: slices of >= 256
    if (split && blocks < 256 && k >= 512) {
        const long by_k = k / 256, by_ws = split_floats / ((long)m * n);
        slices = (int)std::max(1L, std::min({by_k, by_ws, (long)kMaxSlices}));
    }
    const int step = tiled ? kGbk : 16;
    const int kc = slices == 1 ? k : ((k + slices - 1) / slices + step - 1) / step * step;
    slices = (k + kc - 1) / kc;
    float* P = slices > 1 ? split : nullptr;
    if (tiled) {
        const long sa = a_k ? sa0 : sa1, sb = b_k ? sb1 : sb0;
        const int vec = ((uintptr_t)A % 16 == 0) && ((uintptr_t)B % 16 == 0) && sa % 8 == 0 && sb % 8 == 0;
        const dim3 grid((unsigned)blocks, (unsigned)slices);
        if (a_k && b_k)
            hipLaunchKernelGGL((k_gemm_lds<true, true>), grid, dim3(256), 0, s, m, n, k, kc, A, sa, B, sb, vec, bias,
                               relu, C, ldc, Cb, ldcb, P);
        else if (a_k)
            hipLaunchKernelGGL((k_gemm_lds<true, false>), grid, dim3(256), 0, s, m, n, k, kc, A, sa, B, sb, vec, bias,
                               relu, C, ldc, Cb, ldcb, P);
        else if (b_k)
            hipLaunchKernelGGL((k_gemm_lds<false, true>), grid, dim3(256), 0, s, m, n, k, kc, A, sa, B, sb, vec, bias,
                               relu, C, ldc, Cb, ldcb, P);
        else
            hipLaunchKernelGGL((k_gemm_lds<false, false>), grid, dim3(256), 0, s, m, n, k, kc, A, sa, B, sb, vec,
                               bias, relu, C, ldc, Cb, ldcb, P);
    } else {
        hipLaunchKernelGGL(k_gemm, dim3((unsigned)blocks, (unsigned)slices), dim3(256), 0, s, m, n, k, kc, A, sa0, sa1,
                           B, sb0, sb1, bias, relu, C, ldc, Cb, ldcb, P);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !P) return e;
    const long mn = (long)m * n;
    hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s, m, n, slices, P, bias,
                       relu, C, ldc, Cb, ldcb);
    return hipGetLastError();
}

// ------------------------------------------------------ loss and backward
// dY = 2 (Y - T) / (3 n) over the 3 used outputs (zero in the padding), as
// FP32 and BF16; per-row squared errors for the loss.
__global__ void k_mse(int n, const float* __restrict__ Y, const float* __restrict__ T, float* __restrict__ dY,
                      uint16_t* __restrict__ dYb, float* __restrict__ row_loss) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float l = 0.0f;
    for (int c = 0; c < FF_LEARN_OUT_PAD; ++c) {
        float d = 0.0f;
        if (c < 3) {
            const float e = Y[(size_t)i * FF_LEARN_OUT_PAD + c] - T[3 * (size_t)i + c];
            l += e * e;
            d = 2.0f * e / (3.0f * (float)n);
        }
        dY[(size_t)i * FF_LEARN_OUT_PAD + c] = d;
        dYb[(size_t)i * FF_LEARN_OUT_PAD + c] = to_bf16(d);
    }
    row_loss[i] = l;
}

// dH = dH * (H > 0), then its BF16 copy.
__global__ void k_relu_back(long count, const float* __restrict__ H, float* __restrict__ dH,
                            uint16_t* __restrict__ dHb) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float v = H[i] > 0.0f ? dH[i] : 0.0f;
    dH[i] = v;
    dHb[i] = to_bf16(v);
}

// out[c] = scale * sum_i X[i][c] for an FP32 [n][cols] matrix (bias
// gradients, and the loss from per-row errors).  One block per column; each
// thread sums a fixed stride of rows in FP64, then a fixed-order tree, so the
// result does not depend on timing.
__global__ void __launch_bounds__(256) k_colsum(int n, int cols, const float* __restrict__ X, double scale,
                                                float* __restrict__ out) {
    __shared__ double red[256];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += X[(size_t)i * cols + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = (float)(scale * red[0]);
}

// ------------------------------------------------------------------ Adam
__global__ void k_adam(int count, float* __restrict__ w, uint16_t* __restrict__ wb, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = to_bf16(wi);
}

// ------------------------------------------------------------- apply
// x_out = x_in + scale * disp (FP32 displacement [n][3], padded rows of
// FF_LEARN_OUT_PAD), FP64 points.
__global__ void k_displace(long n3, const double* __restrict__ x, const float* __restrict__ disp, double scale,
                           double* __restrict__ out) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3) return;
    const long a = i / 3, c = i - 3 * a;
    out[i] = x[i] + scale * (double)disp[a * FF_LEARN_OUT_PAD + c];
}

__global__ void k_to_bf16(long n, const float* __restrict__ x, uint16_t* __restrict__ out) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = to_bf16(x[i]);
}

__global__ void k_delta(long n3, const double* __restrict__ a, const double* __restrict__ b, float* __restrict__ out) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n3) out[i] = (float)(b[i] - a[i]);
}

__device__ __forceinline__ bool take_new(double e_old, double e_new) {
    return e_new < e_old && e_new - e_new == 0.0;   // finite and lower
}

// out may alias x_old (each element is read and written by one thread)
__global__ void k_select(long n3, const double* x_old, const double* __restrict__ x_new,
                         const double* __restrict__ e_old, const double* __restrict__ e_new,
                         const int32_t* __restrict__ atom_sys, double* out) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3) return;
    const int s = atom_sys[i / 3];
    out[i] = take_new(e_old[s], e_new[s]) ? x_new[i] : x_old[i];
}

// runs after k_select (same stream), so e_out may alias e_old
__global__ void k_chosen(int n_sys, const double* e_old, const double* __restrict__ e_new, int32_t* chosen,
                         double* e_out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_sys) return;
    const bool t = take_new(e_old[s], e_new[s]);
    if (chosen) chosen[s] = t ? 1 : 0;
    if (e_out) e_out[s] = t ? e_new[s] : e_old[s];
}

__global__ void k_gather(const uint32_t* __restrict__ src, const int32_t* __restrict__ idx, long n_rows,
                         int words, uint32_t* __restrict__ dst) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_rows * words) return;
    const long r = t / words, w = t - r * words;
    dst[t] = src[(long)idx[r] * words + w];
}

}  // namespace ff

// =================================================================== C ABI
using namespace ff;

namespace {
thread_local std::string g_learn_err;
ff_status lfail(ff_status st, const char* fmt, ...) {
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_learn_err = buf;
    return st;
}
#define L_TRY(expr)                                                                             \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return lfail(FF_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// parameter offsets (floats) in the packed vector
constexpr long kW1 = 0, kB1 = kW1 + (long)FF_LEARN_FEATURES * FF_LEARN_HIDDEN;
constexpr long kW2 = kB1 + FF_LEARN_HIDDEN, kB2 = kW2 + (long)FF_LEARN_HIDDEN * FF_LEARN_HIDDEN;
constexpr long kW3 = kB2 + FF_LEARN_HIDDEN, kB3 = kW3 + (long)FF_LEARN_HIDDEN * FF_LEARN_OUT_PAD;
constexpr long kParams = kB3 + FF_LEARN_OUT_PAD;

// activation workspace (bytes) for n rows
size_t act_bytes(long n) {
    const long h = FF_LEARN_HIDDEN, o = FF_LEARN_OUT_PAD;
    return (size_t)n * (2 * h * 4 + 2 * h * 2 + o * 4) + 256 * 8;
}
struct Act {
    float *h1, *h2, *y;
    uint16_t *h1b, *h2b;
};
Act carve(void* ws, long n) {
    char* p = (char*)ws;
    auto take = [&](size_t b) { char* r = p; p += (b + 255) & ~(size_t)255; return r; };
    const long h = FF_LEARN_HIDDEN;
    Act a;
    a.h1 = (float*)take((size_t)n * h * 4);
    a.h2 = (float*)take((size_t)n * h * 4);
    a.h1b = (uint16_t*)take((size_t)n * h * 2);
    a.h2b = (uint16_t*)take((size_t)n * h * 2);
    a.y = (float*)take((size_t)n * FF_LEARN_OUT_PAD * 4);
    return a;
}
}  // namespace

extern "C" {

int32_t ff_learn_param_count(void) { return (int32_t)kParams; }

// forward: the activations; backward: activations, their gradients and the
// k-slice scratch of the weight gradients
size_t backward_bytes(long n) { return 2 * act_bytes(n) + (size_t)kSplitFloats * 4; }

size_t ff_learn_workspace_bytes(int32_t n_rows) { return n_rows < 1 ? 0 : backward_bytes(n_rows) + 2 * 256; }

const char* ff_learn_last_error(void) { return g_learn_err.c_str(); }

ff_status ff_learn_features(int32_t n_sys, int32_t n_total, const double* xyz, const double* q,
                            const double* sigma, const double* eps, const int32_t* sys_first,
                            const int32_t* atom_sys, uint16_t* features, int32_t* neighbors, void* stream) {
    g_learn_err.clear();
    if (n_sys < 1 || n_total < 1) return lfail(FF_ERR_ARG, "need at least one system and one atom");
    if (!xyz || !q || !sigma || !eps || !sys_first || !atom_sys || !features) return lfail(FF_ERR_ARG, "null pointer");
    hipLaunchKernelGGL(k_features, dim3((n_total + 127) / 128), dim3(128), 0, (hipStream_t)stream, xyz, q, sigma,
                       eps, sys_first, atom_sys, n_total, features, neighbors);
    L_TRY(hipGetLastError());
    return FF_OK;
}

ff_status ff_learn_gemm(int32_t m, int32_t n, int32_t k, const uint16_t* a, int64_t sa0, int64_t sa1,
                        const uint16_t* b, int64_t sb0, int64_t sb1, const float* bias, int32_t relu, float* c,
                        int64_t ldc, uint16_t* cb, int64_t ldcb, void* stream) {
    g_learn_err.clear();
    if (m < 1 || n < 1 || k < 1 || !a || !b || (!c && !cb)) return lfail(FF_ERR_ARG, "bad GEMM arguments");
    L_TRY(launch_gemm(m, n, k, a, sa0, sa1, b, sb0, sb1, bias, relu, c, ldc, cb, ldcb, (hipStream_t)stream));
    return FF_OK;
}

ff_status ff_learn_forward(const float* params, const uint16_t* params_bf16, const uint16_t* features,
                           int32_t n_rows, void* workspace, size_t workspace_bytes, float* out, void* stream) {
    g_learn_err.clear();
    if (!params || !params_bf16 || !features || n_rows < 1 || !workspace || !out)
        return lfail(FF_ERR_ARG, "null argument or no rows");
    if (workspace_bytes < act_bytes(n_rows) || ((uintptr_t)workspace & 255))
        return lfail(FF_ERR_WORKSPACE, "workspace too small or misaligned");
    hipStream_t st = (hipStream_t)stream;
    const Act t = carve(workspace, n_rows);
    const long F = FF_LEARN_FEATURES, H = FF_LEARN_HIDDEN, O = FF_LEARN_OUT_PAD;
    // H1 = relu(X W1 + b1), H2 = relu(H1 W2 + b2), Y = H2 W3 + b3
    L_TRY(launch_gemm(n_rows, H, F, features, F, 1, params_bf16 + kW1, H, 1, params + kB1, 1, t.h1, H, t.h1b, H, st));
    L_TRY(launch_gemm(n_rows, H, H, t.h1b, H, 1, params_bf16 + kW2, H, 1, params + kB2, 1, t.h2, H, t.h2b, H, st));
    L_TRY(launch_gemm(n_rows, O, H, t.h2b, H, 1, params_bf16 + kW3, O, 1, params + kB3, 0, out, O, nullptr, 0, st));
    return FF_OK;
}

ff_status ff_learn_backward(const float* params, const uint16_t* params_bf16, const uint16_t* features,
                            int32_t n_rows, void* workspace, size_t workspace_bytes, const float* target,
                            float* grad, float* loss, void* stream) {
    g_learn_err.clear();
    if (!params || !params_bf16 || !features || n_rows < 1 || !workspace || !target || !grad || !loss)
        return lfail(FF_ERR_ARG, "null argument or no rows");
    const size_t need = backward_bytes(n_rows);
    if (workspace_bytes < need || ((uintptr_t)workspace & 255))
        return lfail(FF_ERR_WORKSPACE, "workspace too small or misaligned (%zu needed)", need);
    hipStream_t st = (hipStream_t)stream;
    const long F = FF_LEARN_FEATURES, H = FF_LEARN_HIDDEN, O = FF_LEARN_OUT_PAD;
    const long n = n_rows;
    // forward into the first half of the workspace, gradients of the
    // activations into the second half
    const Act t = carve(workspace, n);
    const Act d = carve((char*)workspace + act_bytes(n), n);
    float* split = (float*)((char*)workspace + 2 * act_bytes(n));
    L_TRY(launch_gemm(n_rows, H, F, features, F, 1, params_bf16 + kW1, H, 1, params + kB1, 1, t.h1, H, t.h1b, H, st));
    L_TRY(launch_gemm(n_rows, H, H, t.h1b, H, 1, params_bf16 + kW2, H, 1, params + kB2, 1, t.h2, H, t.h2b, H, st));
    L_TRY(launch_gemm(n_rows, O, H, t.h2b, H, 1, params_bf16 + kW3, O, 1, params + kB3, 0, t.y, O, nullptr, 0, st));
    // dY (FP32 in d.y, BF16 in d.h2b's first n*O entries), per-row errors in d.h1
    uint16_t* dyb = d.h2b;
    float* row_loss = d.h1;
    hipLaunchKernelGGL(k_mse, dim3((n_rows + 255) / 256), dim3(256), 0, st, n_rows, t.y, target, d.y, dyb, row_loss);
    L_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(256), 0, st, n_rows, 1, row_loss, 1.0 / (3.0 * n), loss);
    L_TRY(hipGetLastError());
    // layer 3: dW3 = H2^T dY, db3 = colsum dY, dH2 = dY W3^T (masked by H2 > 0)
    L_TRY(launch_gemm(H, O, n_rows, t.h2b, 1, H, dyb, O, 1, nullptr, 0, grad + kW3, O, nullptr, 0, st, split,
                      kSplitFloats));
    hipLaunchKernelGGL(k_colsum, dim3(O), dim3(256), 0, st, n_rows, (int)O, d.y, 1.0, grad + kB3);
    L_TRY(hipGetLastError());
    L_TRY(launch_gemm(n_rows, H, O, dyb, O, 1, params_bf16 + kW3, 1, O, nullptr, 0, d.h2, H, nullptr, 0, st));
    hipLaunchKernelGGL(k_relu_back, dim3((unsigned)((n * H + 255) / 256)), dim3(256), 0, st, n * H, t.h2, d.h2, d.h2b);
    L_TRY(hipGetLastError());
    // layer 2: dW2 = H1^T dH2, db2, dH1 = dH2 W2^T (masked by H1 > 0)
    L_TRY(launch_gemm(H, H, n_rows, t.h1b, 1, H, d.h2b, H, 1, nullptr, 0, grad + kW2, H, nullptr, 0, st, split,
                      kSplitFloats));
    hipLaunchKernelGGL(k_colsum, dim3(H), dim3(256), 0, st, n_rows, (int)H, d.h2, 1.0, grad + kB2);
    L_TRY(hipGetLastError());
    L_TRY(launch_gemm(n_rows, H, H, d.h2b, H, 1, params_bf16 + kW2, 1, H, nullptr, 0, d.h1, H, nullptr, 0, st));
    hipLaunchKernelGGL(k_relu_back, dim3((unsigned)((n * H + 255) / 256)), dim3(256), 0, st, n * H, t.h1, d.h1, d.h1b);
    L_TRY(hipGetLastError());
    // layer 1: dW1 = X^T dH1, db1
    L_TRY(launch_gemm(F, H, n_rows, features, 1, F, d.h1b, H, 1, nullptr, 0, grad + kW1, H, nullptr, 0, st, split,
                      kSplitFloats));
    hipLaunchKernelGGL(k_colsum, dim3(H), dim3(256), 0, st, n_rows, (int)H, d.h1, 1.0, grad + kB1);
    L_TRY(hipGetLastError());
    return FF_OK;
}

ff_status ff_learn_adam(float* params, uint16_t* params_bf16, const float* grad, float* m, float* v, int32_t step,
                        float lr, float beta1, float beta2, float eps, void* stream) {
    g_learn_err.clear();
    if (!params || !grad || !m || !v || step < 1 || !(lr > 0.0f)) return lfail(FF_ERR_ARG, "bad Adam arguments");
    const float c1 = 1.0f - std::pow(beta1, (float)step), c2 = 1.0f - std::pow(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((kParams + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       (int)kParams, params, params_bf16, grad, m, v, lr, beta1, beta2, eps, c1, c2);
    L_TRY(hipGetLastError());
    return FF_OK;
}

ff_status ff_learn_displace(const double* xyz, const float* disp, int32_t n_atoms, double scale, double* out,
                            void* stream) {
    g_learn_err.clear();
    if (!xyz || !disp || !out || n_atoms < 1 || !std::isfinite(scale)) return lfail(FF_ERR_ARG, "bad arguments");
    const long n3 = 3L * n_atoms;
    hipLaunchKernelGGL(k_displace, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, (hipStream_t)stream, n3, xyz,
                       disp, scale, out);
    L_TRY(hipGetLastError());
    return FF_OK;
}

ff_status ff_learn_to_bf16(const float* x, int64_t n, uint16_t* out, void* stream) {
    g_learn_err.clear();
    if (!x || !out || n < 1) return lfail(FF_ERR_ARG, "bad conversion arguments");
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, (long)n, x,
                       out);
    L_TRY(hipGetLastError());
    return FF_OK;
}

ff_status ff_learn_delta(const double* x_start, const double* x_min, int32_t n_atoms, float* out, void* stream) {
    g_learn_err.clear();
    if (!x_start || !x_min || !out || n_atoms < 1) return lfail(FF_ERR_ARG, "bad delta arguments");
    const long n3 = 3L * n_atoms;
    hipLaunchKernelGGL(k_delta, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, (hipStream_t)stream, n3, x_start,
                       x_min, out);
    L_TRY(hipGetLastError());
    return FF_OK;
}

ff_status ff_learn_gather_rows(const void* src, const int32_t* idx, int32_t n_rows, int32_t row_bytes, void* dst,
                               void* stream) {
    g_learn_err.clear();
    if (!src || !idx || !dst || n_rows < 1 || row_bytes < 4 || (row_bytes & 3))
        return lfail(FF_ERR_ARG, "bad gather arguments");
    const int words = row_bytes / 4;
    const long tot = (long)n_rows * words;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       (const uint32_t*)src, idx, (long)n_rows, words, (uint32_t*)dst);
    L_TRY(hipGetLastError());
    return FF_OK;
}

ff_status ff_learn_select(int32_t n_sys, int32_t n_total, const double* x_old, const double* x_new,
                          const double* e_old, const double* e_new, const int32_t* atom_sys, double* out,
                          int32_t* chosen, double* e_out, void* stream) {
    g_learn_err.clear();
    if (n_sys < 1 || n_total < 1 || !x_old || !x_new || !e_old || !e_new || !atom_sys || !out)
        return lfail(FF_ERR_ARG, "bad select arguments");
    hipStream_t st = (hipStream_t)stream;
    const long n3 = 3L * n_total;
    hipLaunchKernelGGL(k_select, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, st, n3, x_old, x_new, e_old,
                       e_new, atom_sys, out);
    L_TRY(hipGetLastError());
    if (chosen || e_out) {
        hipLaunchKernelGGL(k_chosen, dim3((n_sys + 255) / 256), dim3(256), 0, st, n_sys, e_old, e_new, chosen,
                           e_out);
        L_TRY(hipGetLastError());
    }
    return FF_OK;
}

}  // extern "C"
