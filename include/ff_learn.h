/*
 * ff_learn.h -- learned warm start for the force-field minimizer
 * (libff_mi355x.so, beside ff.h).
 *
 * Not part of the paper.  The paper minimizes the same force field from many
 * clashing poses (sections 3 and 5.3); this part learns, from (start,
 * minimum) pairs that ff_minimize itself produces, a per-atom displacement
 * that is applied to a start before L-BFGS.  The minimizer keeps the last word:
 * a displaced start is kept per system only where the energy prefers it
 * (ff_learn_select compares two points of every system).
 *
 * The network is a 3-layer perceptron on per-atom features:
 *   H1 = relu(X W1 + b1), H2 = relu(H1 W2 + b2), Y = H2 W3 + b3,
 * X [n][FF_LEARN_FEATURES], W1 [FEATURES][HIDDEN], W2 [HIDDEN][HIDDEN],
 * W3 [HIDDEN][OUT_PAD]; columns 0..2 of Y are the predicted displacement
 * (Angstrom) of the atom; columns 3..OUT_PAD-1 pad the last product to the
 * matrix-core tile (the loss ignores them, so their weights never change).
 * Features, weights and activations that feed a product are BF16; products
 * accumulate in FP32 on the matrix cores; biases, the output and every
 * gradient are FP32.
 *
 * Conventions: as in ff.h (device pointers, caller-owned memory, `stream` a
 * hipStream_t as void*, negative ff_status = nothing computed, described by
 * ff_learn_last_error()).  BF16 values are uint16_t bit patterns (the upper
 * half of the FP32 pattern, rounded to nearest even).  Row-major matrices.
 */
#ifndef FF_MI355X_LEARN_H
#define FF_MI355X_LEARN_H

#include "ff.h"

#ifdef __cplusplus
extern "C" {
#endif

#define FF_LEARN_NEIGHBORS 16
#define FF_LEARN_FEATURES 128
#define FF_LEARN_HIDDEN 128
#define FF_LEARN_OUT_PAD 16

/* Packed parameter vector (FP32, and its BF16 copy, same offsets):
 * W1, b1, W2, b2, W3, b3 in this order, each row-major.  Returns its length
 * (128*128 + 128 + 128*128 + 128 + 128*16 + 16 = 35 088). */
int32_t ff_learn_param_count(void);

/* Device workspace for ff_learn_forward and ff_learn_backward with up to
 * n_rows rows (the forward pass uses its first part: the activations; the
 * backward pass also holds their gradients and 4 MiB of per-slice partial
 * sums for the weight gradients).  0 for n_rows < 1. */
size_t ff_learn_workspace_bytes(int32_t n_rows);

/* Description of the last error of an ff_learn_* call on this thread. */
const char *ff_learn_last_error(void);

/* Per-atom features of n_sys systems whose atoms are concatenated
 * (n_total atoms).  sys_first [n_sys + 1] holds the first atom of each system
 * and n_total last; atom_sys [n_total] the system of each atom (both device,
 * consistent with each other: the kernel trusts them).  xyz [n_total][3], q,
 * sigma, eps [n_total] are FP64 device arrays.  For atom i, with its
 * FF_LEARN_NEIGHBORS nearest other atoms j_0, j_1, ... of the same system
 * (FP64 squared distance, ties to the lower index):
 *   row i = q_i, sigma_i - 3.5, 10 eps_i, then for each neighbour k
 *           (x_j - x_i)/4, (y_j - y_i)/4, (z_j - z_i)/4, r_ij/4, q_j,
 *           sigma_j - 3.5, 10 eps_j (zeros for missing neighbours),
 *           then (x_i - c)/16 (3 values), |x_i - c|/16 and n_s/4096, with
 *           c the centroid of the n_s atoms of the system (coordinates
 *           summed in atom order, divided by n_s),
 * zeros up to FF_LEARN_FEATURES; every value is
 * rounded FP64 -> FP32 -> BF16.  features [n_total][FF_LEARN_FEATURES] BF16
 * (device, written); neighbors [n_total][FF_LEARN_NEIGHBORS] (device, may be
 * NULL) receives j_k, -1 where missing.  Cost O(sum of n_s^2). */
ff_status ff_learn_features(int32_t n_sys, int32_t n_total, const double *xyz, const double *q,
                            const double *sigma, const double *eps, const int32_t *sys_first,
                            const int32_t *atom_sys, uint16_t *features, int32_t *neighbors,
                            void *stream);

/* C = epilogue(A B), A(i, k) = a[i*sa0 + k*sa1] for i < m, k < k_dim,
 * B(k, j) = b[k*sb0 + j*sb1] for j < n (BF16, device; the strides express
 * transposes).  FP32 accumulation on the matrix cores.  Epilogue: + bias[j]
 * (FP32, NULL for none), then max(., 0) if relu != 0; the FP32 result goes
 * to c[i*ldc + j] and its BF16 rounding to cb[i*ldcb + j] (either may be
 * NULL, not both). */
ff_status ff_learn_gemm(int32_t m, int32_t n, int32_t k_dim, const uint16_t *a, int64_t sa0, int64_t sa1,
                        const uint16_t *b, int64_t sb0, int64_t sb1, const float *bias, int32_t relu,
                        float *c, int64_t ldc, uint16_t *cb, int64_t ldcb, void *stream);

/* Y [n_rows][FF_LEARN_OUT_PAD] (FP32, device) of the network at features
 * [n_rows][FF_LEARN_FEATURES] (BF16).  params / params_bf16: the packed
 * vector (device).  workspace: device, 256-byte aligned, at least
 * ff_learn_workspace_bytes(n_rows). */
ff_status ff_learn_forward(const float *params, const uint16_t *params_bf16, const uint16_t *features,
                           int32_t n_rows, void *workspace, size_t workspace_bytes, float *out,
                           void *stream);

/* Loss and gradient for one minibatch: loss = mean over rows i and columns
 * c < 3 of (Y_ic - target_ic)^2, target [n_rows][3] FP32 (device).  grad
 * (FP32, packed like params, device) is overwritten with d loss / d params,
 * computed from BF16 copies of the forward activations and of the output
 * and hidden-layer gradients, FP32 accumulation; bias gradients are FP32
 * column sums; the weight gradients sum their k slices in a fixed order.
 * loss: one FP32 on the device.  workspace: device, 256-byte aligned, at
 * least ff_learn_workspace_bytes(n_rows). */
ff_status ff_learn_backward(const float *params, const uint16_t *params_bf16, const uint16_t *features,
                            int32_t n_rows, void *workspace, size_t workspace_bytes, const float *target,
                            float *grad, float *loss, void *stream);

/* One Adam step (Kingma and Ba 2015, bias-corrected; step = 1, 2, ...) on the
 * packed FP32 parameters with first / second moment buffers m, v (device,
 * zero before step 1); params_bf16 (may be NULL) receives the BF16 rounding
 * of the new parameters. */
ff_status ff_learn_adam(float *params, uint16_t *params_bf16, const float *grad, float *m, float *v,
                        int32_t step, float lr, float beta1, float beta2, float eps, void *stream);

/* dst row r = src row idx[r] for r < n_rows (row_bytes a multiple of 4;
 * device; idx entries must lie in the source). */
ff_status ff_learn_gather_rows(const void *src, const int32_t *idx, int32_t n_rows, int32_t row_bytes,
                               void *dst, void *stream);

/* out[i] = BF16 rounding of x[i], i < n (device). */
ff_status ff_learn_to_bf16(const float *x, int64_t n, uint16_t *out, void *stream);

/* Training targets: out [n_atoms][3] FP32 = x_min - x_start (FP64 [n_atoms][3]
 * each; device). */
ff_status ff_learn_delta(const double *x_start, const double *x_min, int32_t n_atoms, float *out,
                         void *stream);

/* out = xyz + scale * disp (FP64 [n_atoms][3]; disp is the network output,
 * FP32 rows of FF_LEARN_OUT_PAD, columns 0..2 used).  Device pointers. */
ff_status ff_learn_displace(const double *xyz, const float *disp, int32_t n_atoms, double scale,
                            double *out, void *stream);

/* Per system s: atoms of s in out take x_new if e_new[s] is finite and below
 * e_old[s], else x_old (FP64 [n_total][3], energies [n_sys], atom_sys
 * [n_total], all device).  chosen [n_sys] (device, may be NULL) receives 1
 * where x_new was taken; e_out [n_sys] (device, may be NULL, may alias e_old)
 * the energy of the point taken.  out may alias x_old. */
ff_status ff_learn_select(int32_t n_sys, int32_t n_total, const double *x_old, const double *x_new,
                          const double *e_old, const double *e_new, const int32_t *atom_sys, double *out,
                          int32_t *chosen, double *e_out, void *stream);

#ifdef __cplusplus
}
#endif

#endif
