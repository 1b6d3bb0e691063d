/*
 * ff.h -- C ABI of the MI355X force-field minimization library (libff_mi355x.so).
 *
 * The library evaluates the macromolecular force field of section 2 of
 * "Algorithms for local minimization of the force field for 3D
 * macromolecules" (arXiv 1810.03358) -- harmonic bond stretch and angle bend,
 * OPLS torsion, Coulomb and 12-6 Lennard-Jones with geometric mixing over all
 * non-excluded atom pairs -- together with its gradient, and minimizes it
 * locally from a given start (the problem statement at the end of section 2)
 * with the first-order methods of section 5.1 and the line searches of
 * section 5.2.  Everything after the start point is on the GPU: the host only
 * launches work and polls a completion flag.
 *
 * Conventions shared by every entry point
 *  - Units: Angstrom, radians, elementary charges, kcal/mol.  The Coulomb
 *    constant is a field of ff_system (332.0715989 kcal A/(mol e^2) is the
 *    paper's 1389.38757 kJ value expressed in kcal).
 *  - Coordinates and gradients are FP64 arrays [n_atoms][3] (x, y, z of atom
 *    0, then atom 1, ...), in DEVICE memory.
 *  - The caller owns all memory.  The library never allocates device memory:
 *    every device buffer it uses lives in the caller's workspace (size from
 *    ff_workspace_bytes, device memory, 256-byte aligned).  The only host
 *    allocation is the small ff_ctx object.
 *  - `stream` is a hipStream_t passed as void* (NULL: the default stream).
 *    One context serves one stream at a time; calls on one context must not
 *    overlap.
 *  - Errors: a negative ff_status means nothing was computed; ff_last_error()
 *    returns a thread-local description.  Termination reasons of a
 *    minimization are not errors (ff_min_result.term).
 */
#ifndef FF_MI355X_H
#define FF_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FF_OK = 0,
    FF_ERR_ARG = -1,          /* bad pointer, size, index, parameter */
    FF_ERR_HIP = -2,          /* a HIP runtime call failed */
    FF_ERR_WORKSPACE = -3,    /* workspace too small or misaligned */
    FF_ERR_UNSUPPORTED = -4   /* valid input outside what this build handles */
} ff_status;

/* Methods of section 5.1: steepest descent with a line search (section 4,
 * eq. 4), FGM (Algorithm 1), CG with the Polak-Ribiere-Polyak beta
 * (Algorithm 2), L-BFGS (Algorithms 3 and 4); and of section 4: the heavy-ball
 * method (eq. HB, constant steps hb_alpha, hb_beta, no line search) and the
 * optimized gradient method (eq. optim, with the line search the text puts
 * in place of 1/L, restarting at the current point when its direction is not
 * a descent direction or the line search fails). */
typedef enum { FF_GD = 0, FF_FGM = 1, FF_CG = 2, FF_LBFGS = 3, FF_HB = 4, FF_OGM = 5 } ff_method;

/* Arithmetic of the pair sum.  FF_FP64: FP64 throughout.  FF_FP32_ACC64:
 * pair terms in FP32 on double-single coordinate differences, accumulated
 * in FP64 per tile; bonded terms, reductions and every optimizer decision in
 * FP64 (section 5.3 runs the paper's library in single precision). */
typedef enum { FF_FP64 = 0, FF_FP32_ACC64 = 1 } ff_precision;

/* Why a minimization stopped. */
typedef enum {
    FF_CONVERGED = 0,         /* |grad E|_inf < tol at the returned point */
    FF_MAX_ITER = 1,          /* max_iter iterations done */
    FF_LS_FAILED = 2,         /* no relaxing step even after the restart
                                 (the "dead end" of section 5.1) */
    FF_NONFINITE_START = 3,   /* E or grad E not finite at the start point */
    FF_DIVERGED = 4           /* heavy ball: a step reached a non-finite E or
                                 grad E (the last finite iterate is returned) */
} ff_term;

/* beta of the CG variants named in section 5.1 (y = g_{k+1} - g_k, d = the
 * previous unnormalized direction): PRP <g+,y>/|g|^2, FR |g+|^2/|g|^2,
 * HS <g+,y>/<d,y>, PRP+ max(0, PRP), CD |g+|^2/(-<d,g>), LS <g+,y>/(-<d,g>),
 * DY |g+|^2/<d,y>.  A zero or non-finite denominator restarts (beta = 0). */
typedef enum { FF_CG_PRP = 0, FF_CG_FR = 1, FF_CG_HS = 2, FF_CG_PRP_PLUS = 3,
               FF_CG_CD = 4, FF_CG_LS = 5, FF_CG_DY = 6 } ff_cg_beta;

/* Line searches of section 5.2: LS_PAR (Algorithm 6), LS_H (Algorithm 5). */
typedef enum { FF_LS_DEFAULT = -1, FF_LS_PAR = 0, FF_LS_H = 1 } ff_linesearch;

/* ff_min_params.flags */
#define FF_MIN_RESUME      1  /* continue from the state a previous ff_minimize
                                 left in this context (same method, m and
                                 precision; x must be that call's output) */
#define FF_MIN_NO_CERTIFY  2  /* skip the closing FP64 evaluation (FP32 mode) */

/* System description: HOST pointers, read only during ff_create.
 * Angles are (i, vertex, k).  Excluded pairs are the bonded pairs and the
 * outer atoms of every angle; 1-4 pairs interact at full strength; there is
 * no cutoff.  Any topology is accepted: excluded pairs up to 64 atoms apart in
 * index use a per-atom bitmask, farther ones (cross-links, ring closures)
 * per-tile masks (a slightly slower pair kernel is used for such systems). */
typedef struct {
    int32_t n_atoms;
    const double *q, *sigma, *eps;                      /* [n_atoms] e, A, kcal/mol */
    int32_t n_bonds;
    const int32_t *bond;                                /* [n_bonds][2] */
    const double *bond_k, *bond_r0;                     /* [n_bonds] E = K (r - r0)^2 */
    int32_t n_angles;
    const int32_t *angle;                               /* [n_angles][3] */
    const double *angle_k, *angle_t0;                   /* [n_angles] E = K (theta - theta0)^2 */
    int32_t n_dihedrals;
    const int32_t *dihedral;                            /* [n_dihedrals][4] */
    const double *dihedral_v;                           /* [n_dihedrals][4] V1..V4 */
    double coulomb_c;                                   /* kcal A / (mol e^2) */
} ff_system;

/* Minimizer parameters (host struct).  ff_default_params fills the defaults
 * given in brackets. */
typedef struct {
    int32_t method;       /* ff_method [FF_LBFGS] */
    int32_t m;            /* L-BFGS memory, 1..32 [10] */
    double tol;           /* stop when |grad E|_inf < tol, kcal/mol/A, > 0 [1e-3] */
    int32_t max_iter;     /* >= 0 [2000] */
    int32_t precision;    /* ff_precision [FF_FP64] */
    int32_t linesearch;   /* ff_linesearch [FF_LS_DEFAULT: LS_H for FGM, else LS_PAR] */
    int32_t ls_K;         /* LS_PAR trial count, 2..8 [2] */
    double h_init;        /* first step along the unit direction, A [0.1] */
    double k_plus;        /* LS growth factor > 1 [2] */
    double k_minus;       /* LS shrink factor in (0,1) [0.5] */
    double eps_h;         /* LS_H gives up below this step, A [1e-10] */
    int32_t cg_restart;   /* CG restarts from -g every cg_restart iterations; 0: 3N [0] */
    int32_t flags;        /* FF_MIN_* [0] */
    int32_t cg_beta;      /* ff_cg_beta [FF_CG_PRP] */
    int32_t ls_par_g0;    /* Algorithm 6's G0: 1 = first parabola from f and the
                             slope at the base point, 0 = symmetric trials
                             -h0/2, +h0/2 (steps may then be negative) [1] */
    int32_t fgm_restart;  /* 1: FGM restarts its momentum (theta = 1) whenever an
                             iterate's energy exceeds the previous one
                             (function-value adaptive restart); 0: Algorithm 1
                             as printed [0] */
    double hb_alpha;      /* heavy ball: gradient step, > 0 (required) [0] */
    double hb_beta;       /* heavy ball: momentum, in [0, 1) [0] */
} ff_min_params;

/* Outcome of ff_minimize (host struct). */
typedef struct {
    int32_t term;         /* ff_term */
    int32_t iters;        /* accepted iterations */
    int32_t evals;        /* energy+gradient evaluations (all precisions) */
    int32_t evals_fp64;   /* of which in FP64 */
    double energy;        /* E at the returned point (FP64 unless NO_CERTIFY) */
    double grad_inf;      /* |grad E|_inf there */
    double grad_2;        /* |grad E|_2 there */
} ff_min_result;

typedef struct ff_ctx ff_ctx;   /* opaque host object bound to one workspace */

/* A context holds a batch of n_sys >= 1 independent systems.  Their
 * coordinates and gradients are passed concatenated: [sum of n_atoms][3] FP64,
 * system 0 first.  Energies and results are per system.  Every system of a
 * batch is minimized at the same time (the paper minimizes many docking poses
 * independently, section 5.3); each one stops on its own criterion. */

/* Bytes of device workspace a system needs; m_max is the largest L-BFGS
 * memory ff_minimize will be asked for (0 if only ff_energy_grad is used).
 * Returns 0 on invalid input. */
size_t ff_workspace_bytes(const ff_system *sys, int32_t m_max);
size_t ff_workspace_bytes_batch(const ff_system *systems, int32_t n_sys, int32_t m_max);

/* Validate the system(s) (indices in range, sizes, exclusion window), pack
 * parameters and topology into the workspace and return a context.  Blocks
 * until the upload on `stream` is done.  ff_create is a batch of one. */
ff_status ff_create(const ff_system *sys, void *workspace, size_t workspace_bytes,
                    int32_t m_max, void *stream, ff_ctx **out);
ff_status ff_create_batch(const ff_system *systems, int32_t n_sys, void *workspace,
                          size_t workspace_bytes, int32_t m_max, void *stream, ff_ctx **out);

/* Number of systems in the context. */
int32_t ff_batch_size(const ff_ctx *ctx);

/* Tiling of the pair kernel.  The pair matrix of each system is cut into
 * I-blocks of `block` atoms against j-tiles of 64 atoms, and one workgroup
 * walks a chunk of consecutive j-tiles of one I-block: `chunk` tiles in the
 * FP32 kernel, `chunk64` in the FP64 kernel (each has its own chunk table).
 * With chunks longer than one tile, the last sixteenth of each I-block's
 * j-tiles (at least one) goes to one-tile chunks that end the launch, so that
 * it drains on short workgroups.  A tile configuration fixes the block size
 * and the wavefronts and i-atoms per lane of the FP32 and FP64 kernels.
 * ff_create / ff_create_batch choose one from the system sizes; the
 * functions below name one explicitly.  The tiling changes only speed and the
 * summation order of the pair partials (results agree to rounding). */
int32_t ff_num_tile_configs(void);
/* Shape of configuration `cfg` (0 .. ff_num_tile_configs()-1); any output may
 * be NULL.  FF_ERR_ARG if cfg is out of range. */
ff_status ff_tile_config_info(int32_t cfg, int32_t *block, int32_t *waves32, int32_t *ipl32,
                              int32_t *waves64, int32_t *ipl64);
/* Workspace bytes and context creation with an explicit configuration and
 * chunk lengths (1..4096; chunk64 = 0 takes `chunk` for both kernels);
 * 0 / FF_ERR_ARG on invalid input. */
size_t ff_workspace_bytes_tiled(const ff_system *systems, int32_t n_sys, int32_t m_max,
                                int32_t tile_config, int32_t chunk, int32_t chunk64);
ff_status ff_create_tiled(const ff_system *systems, int32_t n_sys, void *workspace,
                          size_t workspace_bytes, int32_t m_max, int32_t tile_config, int32_t chunk,
                          int32_t chunk64, void *stream, ff_ctx **out);
/* Tiling of an existing context; any output may be NULL. */
ff_status ff_get_tiling(const ff_ctx *ctx, int32_t *tile_config, int32_t *chunk, int32_t *chunk64);

/* Autotuner: for every tile configuration and chunk length in {1, 2, 4, 8,
 * 16} (the same for both kernels) whose layout fits, builds a temporary context for the systems in
 * `workspace` (device, 256-byte aligned, overwritten), times `reps`
 * back-to-back energy+gradient evaluations at xyz (device, concatenated
 * [n][3]) in `precision` with HIP events on `stream`, and returns the fastest
 * configuration and its mean time per evaluation in ms.  Configurations that
 * do not fit the workspace are skipped (FF_ERR_WORKSPACE if none fits);
 * ff_autotune_workspace_bytes gives the size that fits all of them.  Blocks
 * until done.  The result is then passed to ff_create_tiled (as chunk and
 * chunk64, or as the chunk of the tuned precision only). */
size_t ff_autotune_workspace_bytes(const ff_system *systems, int32_t n_sys);
ff_status ff_autotune(const ff_system *systems, int32_t n_sys, const double *xyz, void *workspace,
                      size_t workspace_bytes, int32_t precision, int32_t reps, void *stream,
                      int32_t *tile_config, int32_t *chunk, double *ms_per_eval);

/* Release the host context (the workspace stays the caller's). */
ff_status ff_destroy(ff_ctx *ctx);

/* E(x) and grad E(x) of section 2 at xyz (device, concatenated [n][3]).
 * energy: device pointer to n_sys doubles; grad: device [n][3] or NULL.
 * Enqueued on `stream`, returns without waiting.  A clash gives IEEE inf/NaN
 * values, not an error. */
ff_status ff_energy_grad(ff_ctx *ctx, const double *xyz, double *energy, double *grad,
                         int32_t precision, void *stream);

/* For callers that cannot allocate device memory (serving loops and
 * harnesses that forbid hipMalloc): ff_energy_grad of ONE system with neither
 * a context nor a caller workspace.  The library keeps a static device array
 * of FF_NOALLOC_SCRATCH_BYTES on every GPU it runs on (held until the process
 * ends) and packs the system into it on every call: the same packing, tiling
 * and kernels as ff_create followed by ff_energy_grad, hence the same results.
 *  - sys: host struct as for ff_create; xyz [n_atoms][3], energy [1] and grad
 *    [n_atoms][3] (or NULL): device pointers; precision: ff_precision.
 *  - Blocks until the packed system has been copied to the device (the copy
 *    is ordered after earlier work on `stream`), then enqueues the evaluation
 *    on `stream` and returns.  Not for HIP graph capture (it copies from host
 *    memory and waits for that copy).
 *  - Allocates nothing: no hipMalloc / hipHostMalloc, no stream, event or
 *    graph creation, no heap memory.
 *  - All calls on one GPU share that GPU's array, which keeps the last call's
 *    contents: calls on one stream are ordered, but a call whose evaluation
 *    can overlap another call's on the same GPU (other streams, other
 *    threads) races with it.
 *  - A system whose workspace exceeds FF_NOALLOC_SCRATCH_BYTES (chains of up
 *    to about 23,000 atoms fit) gives FF_ERR_UNSUPPORTED before any device
 *    work; other errors as for ff_create and ff_energy_grad. */
#define FF_NOALLOC_SCRATCH_BYTES (128u << 20)
ff_status ff_energy_grad_noalloc(const ff_system *sys, const double *xyz, double *energy, double *grad,
                                 int32_t precision, void *stream);

/* Local minimization from xyz_inout (device, concatenated [n][3]); on return
 * it holds the result points: the last iterate for GD, CG, L-BFGS, heavy ball
 * and OGM, the best iterate for FGM (Algorithm 1).  result: host array of n_sys entries.
 * Blocks until every system has stopped. */
ff_status ff_minimize(ff_ctx *ctx, double *xyz_inout, const ff_min_params *params,
                      ff_min_result *result, void *stream);

/* Per-iteration trace of system 0 in the last ff_minimize on this context, for
 * diagnostics and tests: host_out[3k .. 3k+2] = (E after iteration k, the
 * accepted step h, evaluations done so far), up to max_entries (the library
 * keeps the first 4096 iterations of a call).  Returns the number of entries
 * written or a negative ff_status.  Blocks on `stream`. */
int32_t ff_get_trace(ff_ctx *ctx, double *host_out, int32_t max_entries, void *stream);

/* Diagnostic of section 3 (the non-convexity of the problem near the start):
 * the energy along the unit antigradient at xyz (device, concatenated [n][3]),
 *   e_out[k * n_sys + s] = E_s(x_s + t[k] u_s),  u_s = -grad E_s(x_s) / |grad E_s(x_s)|
 * (u_s = 0 if the gradient is zero), for k < n_t <= 4096; t and e_out are HOST
 * arrays, t finite (negative values step uphill).  Uses the context's vector
 * workspace, so a following ff_minimize cannot resume.  Blocks until done. */
ff_status ff_energy_profile(ff_ctx *ctx, const double *xyz, const double *t, int32_t n_t,
                            double *e_out, int32_t precision, void *stream);

/* Measurement helper: average duration in milliseconds of `reps`
 * back-to-back launches of the nonbonded pair kernel alone at xyz (device),
 * timed with HIP events recorded on `stream`.  Overwrites the workspace's
 * partial-sum buffers; blocks until done. */
ff_status ff_time_pair(ff_ctx *ctx, const double *xyz, int32_t precision, int32_t reps,
                       void *stream, double *avg_ms);

/* Fill the defaults listed in ff_min_params. */
void ff_default_params(ff_min_params *params);

/* Thread-local text of the last error ("" if none). */
const char *ff_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FF_MI355X_H */
