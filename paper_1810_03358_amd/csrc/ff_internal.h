// Internal layout shared by the kernels and the host side of libff_mi355x.
//
// A context holds a batch of one or more independent systems.  Workspace
// (caller-allocated device memory) =
//   [per-system info | packed parameters | tile tables | topology |
//    grid maps | far-exclusion masks]   (packed once, read only)
//   [batch counters | per-system control blocks | pair partials |
//    bonded partials | reduction partials | FP64 vectors]   (kernel state)
// Every region starts on a 256-byte boundary.  Systems are concatenated: each
// is padded to a multiple of the I-block size and occupies a contiguous range
// of padded atoms (and 3x that range in every FP64 vector).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ff {

constexpr int kTile = 64;            // j-tile: one atom per lane of a wavefront
constexpr int kExclWindow = 64;      // exclusions of this reach live in a per-atom bitmask;
                                     // farther ones in per-unit masks (far units)
constexpr int kMaxM = 32;            // largest L-BFGS memory
constexpr int kNumSlots = 8;         // point slots (x and grad) of the optimizer
constexpr int kMaxTerms = 2 * kMaxM + 2;   // linear-combination terms of a direction
constexpr int kGramDim = 2 * kMaxM + 1;    // Gram matrix over {s_i, y_i, g}
constexpr int kFinBlock = 256;       // threads of the finalize / vector kernels
constexpr int kMaxDots = 6 * kMaxM + 8;    // dot products per vector pass
constexpr int kMaxLsTrials = 8;
constexpr int kBondedPerBlock = 256;  // bonded terms per workgroup
constexpr int kTraceCap = 4096;       // per-iteration trace entries kept
constexpr int kMaxChunk = 4096;       // j-tiles per pair workgroup, upper bound
constexpr int kMaxProfile = 4096;     // points of one energy profile

// Distances (A^2) below which the FP32 pair path first corrects the
// displacement with the low halves of the double-single coordinates and,
// below the second one, evaluates the pair entirely in FP64 (clashes).
constexpr float kCorrR2 = 25.0f;
constexpr double kClashR2 = 4.0;

// ---------------------------------------------------------------- vector ids
// All FP64 optimizer vectors have 3*np doubles and are laid out back to back
// with stride vstride; a vector is named by its index.
enum VecId : int32_t {
    V_X0 = 0,                          // point slots x[0..kNumSlots)
    V_G0 = V_X0 + kNumSlots,           // gradient slots g[0..kNumSlots)
    V_D = V_G0 + kNumSlots,            // current unit direction
    V_R,                               // CG running (unnormalized) direction
    V_S0,                              // L-BFGS s vectors (kMaxM + 1 incl. spare)
    V_Y0 = V_S0 + kMaxM + 1,           // L-BFGS y vectors
    V_COUNT = V_Y0 + kMaxM + 1
};

// ------------------------------------------------------------ control block
enum Action : int32_t { ACT_NONE = 0, ACT_EVAL = 1 };
enum PointMode : int32_t {
    PM_USE = 0,        // evaluate x[target] as it is
    PM_TRIAL = 1,      // x[target] = x[base] + h * d
    PM_DIR_TRIAL = 2,  // d = sum_k coef_k v_k (optionally also r), then as PM_TRIAL
    PM_MOMENTUM = 3,   // x[target] = x[base] + beta * (x[base] - x[prev])
    PM_HB = 4,         // x[target] = x[base] - h g[base] + beta (x[base] - x[prev])
    PM_OGM_Y = 5       // d as in PM_DIR_TRIAL, x[target] = (1 - beta) x[base] + beta x[prev]
};
enum Phase : int32_t {
    PH_IDLE = 0, PH_START, PH_LS, PH_MOMENTUM, PH_REEVAL64, PH_CERTIFY, PH_DONE, PH_HB, PH_OGM_Y
};
enum LsKind : int32_t { LSK_PAR = 0, LSK_H = 1 };
enum LsHStage : int32_t { LSH_F0 = 0, LSH_F1 = 1, LSH_SHRINK = 2 };

// Batch-wide counters polled by the host.
struct BatchState {
    uint32_t n_done;      // systems finished in the current ff_minimize
    uint32_t evals;       // evaluations of all systems (progress watchdog)
    uint32_t n_fp64;      // systems whose mixed-precision run has switched to FP64
    uint32_t pad_;
};

struct MinParamsDev {
    int32_t method, m, max_iter, precision, linesearch, ls_K, cg_restart, certify, cg_beta, ls_g0, fgm_restart;
    double tol, h_init, k_plus, k_minus, eps_h, hb_alpha, hb_beta;
};

struct Ctl {
    // ---- request for the next evaluation cycle (written by the decision step)
    int32_t action;
    int32_t point_mode;
    int32_t prec;            // ff_precision of this evaluation
    int32_t target;          // slot evaluated
    int32_t base;            // trial base slot
    int32_t prev;            // momentum: previous point slot
    int32_t want_slope;      // finalize also computes <g[slope_slot], d>
    int32_t slope_slot;      // base point of that product (the evaluated point for PM_OGM_Y)
    int32_t write_r;         // PM_DIR_TRIAL: also store the unnormalized r
    double h;                // trial step
    double beta;             // momentum coefficient
    int32_t n_terms;
    int32_t term_vec[kMaxTerms];
    double term_coef[kMaxTerms];   // coefficients of r (unnormalized)
    double dir_scale;              // |r|: d = r / dir_scale

    // ---- accept request for the vector pass after a successful line search
    int32_t accept;          // 1: k_accept has work this cycle
    int32_t acc_new, acc_old;
    int32_t acc_rows;        // rows of products of that pass (fixed while it runs)

    // ---- per-slot results
    double e[kNumSlots], ginf[kNumSlots], g2[kNumSlots];
    int32_t slot_prec[kNumSlots];
    double slope;            // <g[base], d> of the current line search

    // ---- optimizer state
    MinParamsDev p;
    int32_t phase, done, term, iters, evals, evals64, iters_limit, iters_base;
    int32_t cur, prev_x, best, w;          // slots
    int32_t prec_now;                      // precision of the running phase
    int32_t escalated;
    int32_t stall32;                       // an FP32 step gained less than FP32 can resolve
    int32_t fp32_released;                 // counted in BatchState::n_fp64 (needs no FP32 evaluation any more)
    double h_prev;
    // line search
    int32_t ls_kind, ls_hstage, ls_base, ls_best, ls_ntrials, ls_primary, ls_fallback_done;
    double ls_fstar, ls_s0, ls_hcur, ls_hmin, ls_h0;
    double ls_th[kMaxLsTrials + 1], ls_tf[kMaxLsTrials + 1];
    // method state
    int32_t steepest;        // the current direction is -g
    double theta_prev, fgm_theta, fgm_beta;  // FGM
    double accept_h;                         // step of the last accepted trial
    double cg_beta, r_norm2, r_dot_g_old, g_dot_g_old;   // CG
    // OGM: t_k, t_{k+1}, and <g, S>, <S, S> of the weighted gradient sum S
    // (vector V_R; before the first accept after a (re)start S is the anchor's
    // gradient itself: ogm_s_anchor = 1).  The anchor x^0 is slot prev_x.
    double ogm_t, ogm_t_next, ogm_gS, ogm_SS;
    int32_t ogm_s_anchor;
    // L-BFGS history: a ring of hist_m slots; stored pair i (0 = oldest,
    // i < hist_n) sits in slot (hist_head + i) mod hist_m.  Everything below
    // is indexed by slot, so storing a pair never moves the others.
    int32_t hist_n, hist_head, hist_m;
    int32_t hist_s[kMaxM + 1], hist_y[kMaxM + 1];   // vector ids by slot
    int32_t spare_s, spare_y;                        // vector ids for the next pair
    int32_t spare_s_next, spare_y_next;              // first never-used ids
    double rho[kMaxM];                               // 1 / <s, y> by slot
    // Gram matrix of {s of slot q at q, y of slot q at kMaxM + q, g at 2 kMaxM}
    double gram[kGramDim * kGramDim];
    int32_t lb_ready;        // direction coefficients for the next iteration:
                             // 1 computed (terms filled), -1 not a descent direction, 0 none
    int32_t result_slot;
    // per-iteration trace (E, accepted h, evaluations so far); system 0 only
    double* trace_ptr;
    int32_t trace_cap, n_trace;
    BatchState* batch;       // batch-wide counters
    int32_t n_atoms;         // atoms of this system

};

// ------------------------------------------------------- pair tile configs
// I-block of `block` atoms; the FP32 and FP64 kernels split it into
// waves x 64 lanes x ipl atoms per lane.  Both precisions of one
// configuration share the block size, hence the rows and units of the pair
// matrix; each precision has its own chunk length and chunk table (index 0:
// FP32 kernel, 1: FP64 kernel).
struct TileConfig { int block, waves32, ipl32, waves64, ipl64; };
constexpr TileConfig kTileConfigs[] = {
    {64, 1, 1, 1, 1},     // 0
    {256, 4, 1, 4, 1},    // 1
    {512, 4, 2, 8, 1},    // 2
    {512, 8, 1, 8, 1},    // 3
    {256, 2, 2, 4, 1},    // 4
    {128, 2, 1, 2, 1},    // 5
    {128, 1, 2, 2, 1},    // 6
    {256, 2, 2, 2, 2},    // 7: as 4, with two atoms per lane in FP64 too
    {256, 2, 2, 1, 4},    // 8: as 4, with four atoms per lane in FP64
    {128, 1, 2, 1, 2},    // 9: as 6, with two atoms per lane in FP64 too
};
constexpr int kNumTileConfigs = sizeof(kTileConfigs) / sizeof(kTileConfigs[0]);

// ------------------------------------------------------------- tile tables
// The chunk table is in launch order: every chunk of the full length first,
// then the shorter ones, so that the last workgroups of a launch are the
// shortest.  With chunks longer than one j-tile, the last 1/kTailDiv of each
// I-block's j-tiles (at least one) go to one-tile chunks, which end the
// launch.  A chunk's `slot` numbers it within its I-block in j order (the
// I-block's chunks hold consecutive slots): the slot indexes its i-side
// partial row and its energy share.
constexpr int kTailDiv = 16;
struct ChunkInfo {        // one workgroup of the pair kernel
    int32_t row;          // I-block index (global)
    int32_t t_begin, t_end;   // j-tiles [t_begin, t_end) (global)
    int32_t unit_base;    // index of unit (row, t_begin) in the Fj partial array
    int32_t sys;          // system the chunk belongs to
    int32_t slot;         // i-side partial row and energy share of the chunk
    int32_t pad_[2];
};
struct RowInfo {          // one I-block
    int32_t unit_start;   // unit index of (row, t0)
    int32_t t0;           // first j-tile (diagonal)
    int32_t chunk_start[2];   // slot of its first chunk, per chunk table
    int32_t n_chunks[2];
};

// One system of a batch.  Atom indices in its topology are local (0..n-1);
// "global" indices count padded atoms over the whole batch.
struct SysInfo {
    int32_t n;            // atoms
    int32_t np;           // padded atoms (multiple of the I-block size)
    int32_t aoff;         // first padded atom (global); vectors start at 3*aoff
    int32_t uoff;         // first atom in the caller's concatenated [sum n][3] arrays
    int32_t row0, nb;     // first I-block (global) and count
    int32_t chunk0[2], n_chunks[2];   // first slot and chunks, per chunk table
    int32_t n_bonds, n_angles, n_dihedrals;
    int32_t bond0, angle0, dih0;   // first bond / angle / torsion in the batch-wide arrays
    int32_t bonded_blocks, eb0;
    int32_t fin_blocks, vec_blocks;
    int32_t acc_bx;       // accept-pass workgroups per product row
    int32_t red0;         // first double of this system's reduction partials
};

struct Layout {
    int32_t n_sys;
    int32_t n, np, nb, nt, block, n_units;   // n, np: totals over the batch
    int32_t chunk[2], n_chunks[2];        // chunk length and chunks: [0] FP32 kernel, [1] FP64 kernel
    int32_t n_bonds, n_angles, n_dihedrals, n_terms_slots, n_bonded_blocks;
    int32_t n_far_units;      // units holding an excluded pair more than kExclWindow apart
    int32_t n_fin_blocks;
    // flat grids: workgroup b of a pass handles (system, local block) = map[b]
    int32_t n_vec_blocks, n_acc_blocks;
    int32_t acc_rows;         // y-extent of the accept grid: 1 + largest L-BFGS memory
    int32_t m_max;
    int32_t cfg;              // tile configuration index
    size_t vstride;           // doubles between vectors
    size_t ctl_stride;        // bytes between control blocks
    // byte offsets
    size_t off_batch, off_sys;
    size_t off_ctl, off_c12, off_c6, off_q, off_c12d, off_c6d, off_qd, off_excl;
    size_t off_chunks[2], off_rows, off_pi, off_pj, off_ep;   // i-side partials and energies: max over the tables
    size_t off_bond, off_bondp, off_angle, off_anglep, off_dih, off_dihp;
    size_t off_fb, off_eb, off_inc_start, off_inc;
    size_t off_red, off_vec;
    size_t off_map_fin, off_map_vec, off_map_bonded, off_map_acc;   // int2 maps of the flat grids
    size_t off_far_unit;      // int32 per unit: its far-mask block, or -1
    size_t off_far_mask;      // uint64 [n_far_units][block]: bit jl = pair (i, tile atom jl) excluded
    size_t static_end;        // [0, static_end): the packed regions, written once per context
    size_t total;
};

// Kernel arguments: everything is derived from the workspace base and the
// layout, plus the direct-mode pointers of ff_energy_grad.
struct Args {
    Layout L;
    char* ws;
    const double* xyz_in;    // direct mode: coordinates, [sum n][3] over the batch
    double* e_out;           // direct mode: energies [n_sys]
    double* g_out;           // direct mode: gradient [sum n][3] or null
    double* g2_out;          // direct mode: |grad E|^2 per system, or null
    int32_t direct;          // 1: ff_energy_grad, 0: optimizer cycle
    int32_t direct_prec;
};

template <typename T>
__host__ __device__ inline T* at(char* ws, size_t off) { return reinterpret_cast<T*>(ws + off); }

// Vector `id`, at the start of system `si`.
__host__ __device__ inline double* vec(const Args& a, int32_t id, const SysInfo& si) {
    return at<double>(a.ws, a.L.off_vec) + (size_t)id * a.L.vstride + 3 * (size_t)si.aoff;
}

__host__ __device__ inline SysInfo* sys_info(const Args& a) { return at<SysInfo>(a.ws, a.L.off_sys); }

__host__ __device__ inline Ctl* ctl_at(const Args& a, int sys) {
    return reinterpret_cast<Ctl*>(a.ws + a.L.off_ctl + (size_t)sys * a.L.ctl_stride);
}

// Coordinates of padding atoms (index >= n): far away, mutually separated,
// with zero parameters, so every pair they are in contributes exactly zero.
__host__ __device__ inline void pad_position(int32_t a, int32_t n, double* p) {
    p[0] = 1.0e6 + 16.0 * (double)(a - n);
    p[1] = -1.0e6;
    p[2] = 1.0e6;
}

}  // namespace ff
