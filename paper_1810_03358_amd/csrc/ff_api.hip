// Host side of the C ABI declared in include/ff.h: argument validation,
// workspace layout, one-time packing of parameters and topology, and the
// launch sequence of an evaluation or a minimization.
//
// A context holds a batch of independent systems (one or more).  A
// minimization is a fixed cycle of six kernels captured once into a HIP graph:
// build the point (trial / direction / momentum) -> bonded terms -> FP32 pair
// kernel -> FP64 pair kernel -> finalize (+ decision) -> accept pass (+
// decision).  Each cycle advances every unfinished system by one evaluation;
// work of a system that has nothing to do in a kernel returns at once (its
// control block says so).  The host replays the graph and polls the number of
// finished systems.
#include <algorithm>
#include <utility>
#include <cstdarg>
#include <cstddef>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "ff.h"
#include "ff_internal.h"

namespace ff {
hipError_t launch_pair(const Args& a, int prec, hipStream_t s);
hipError_t launch_bonded(const Args& a, hipStream_t s);
hipError_t launch_finalize(const Args& a, hipStream_t s);
hipError_t launch_cycle_vec(const Args& a, int which, hipStream_t s);
hipError_t launch_profile_point(const Args& a, const double* x, const double* g, const double* g2, double t,
                                double* xt, hipStream_t s);
hipError_t launch_kick(const Args& a, const MinParamsDev& p, int resume, double* trace, int trace_cap,
                       hipStream_t s);
hipError_t launch_reset(const Args& a, hipStream_t s);
}  // namespace ff

using namespace ff;

struct ff_ctx {
    Layout L;
    char* ws;
    std::vector<SysInfo> sys;    // host copy of the per-system info
    int32_t* host_flag;          // pinned: polled batch counters
    Ctl* host_ctl;               // pinned copy of one control block
    hipGraphExec_t graph = nullptr;     // cycles with both pair kernels (FP32 mode)
    hipGraphExec_t graph64 = nullptr;   // cycles with the FP64 pair kernel only
    hipStream_t own = nullptr;   // private stream: graph capture, and calls made on the NULL stream
    int last_method = -1, last_m = -1, last_prec = -1;
};

// Text of the last error of this thread (fixed storage: no call allocates
// host memory to report an error).
static thread_local char g_err[512];

static void clear_error() { g_err[0] = '\0'; }

static ff_status fail(ff_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) return fail(FF_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// ------------------------------------------------- ff_energy_grad_noalloc
// Device memory of ff_energy_grad_noalloc: a workspace laid out as for a
// context of one system (without optimizer vectors), in a static array that
// every GPU the library runs on holds until the process ends.  Host code never
// uses the array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device, and is kept in g_scratch_dev.
static __device__ __align__(256) char scratch[FF_NOALLOC_SCRATCH_BYTES];
// Host image of the packed regions (and the far-exclusion temporaries at its
// end), rebuilt by every call.
alignas(256) static char g_stage[FF_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static void* g_scratch_dev[kMaxDevices];
static std::mutex g_noalloc_mu;      // guards g_stage and g_scratch_dev

// ------------------------------------------------------------------ layout
// An excluded pair (1-2 or 1-3) more than kExclWindow atoms apart, as global
// padded indices (lo < hi).
struct FarPair { int32_t lo, hi; };

// Host buffers make_layout and pack_static share: the far pairs and the
// distinct pair units holding them.  `cap` entries each, at least
// far_capacity() of the systems.
struct FarTmp {
    FarPair* pairs;
    long long* keys;     // (I-block << 32 | j-tile), sorted, distinct
    size_t cap;
    size_t n_pairs = 0, n_keys = 0;
};

static size_t far_capacity(const ff_system* s, int32_t n_sys) {
    size_t c = 0;
    for (int k = 0; k < n_sys; ++k) c += (size_t)std::max(0, s[k].n_bonds) + (size_t)std::max(0, s[k].n_angles);
    return std::max<size_t>(c, 1);
}

// Far exclusions of one system appended to ft.pairs.  Pairs with a bad index
// or null arrays are skipped here (validation reports them).
static void far_exclusions(const ff_system& s, int aoff, FarTmp& ft) {
    const int n = s.n_atoms;
    auto add = [&](int i, int j) {
        if (i < 0 || j < 0 || i >= n || j >= n || i == j) return;
        const int lo = std::min(i, j), hi = std::max(i, j);
        if (hi - lo > kExclWindow && ft.n_pairs < ft.cap) ft.pairs[ft.n_pairs++] = FarPair{aoff + lo, aoff + hi};
    };
    if (s.bond)
        for (int b = 0; b < s.n_bonds; ++b) add(s.bond[2 * b], s.bond[2 * b + 1]);
    if (s.angle)
        for (int a = 0; a < s.n_angles; ++a) add(s.angle[3 * a], s.angle[3 * a + 2]);
}

// Tile configuration: explicit (cfg >= 0, chunk >= 1), or by default a single
// system picks its I-block by size and a batch of several systems uses 64-atom
// I-blocks so that small systems are padded to a multiple of 64 only.
// `sys` receives n_sys entries; `ft` the far pairs and their units.
// energy_only: no optimizer vectors (the layout serves ff_energy_grad only).
// The chunks of one I-block with T j-tiles: `full` chunks of c tiles, one of
// `rem` (< c) tiles if rem > 0, then `tail` one-tile chunks (c > 1 only).
struct RowSplit {
    int full, rem, tail;
    int count() const { return full + (rem > 0 ? 1 : 0) + tail; }
};
static RowSplit row_split(int T, int c) {
    RowSplit r{0, 0, 0};
    r.tail = c > 1 ? std::min(T, (T + kTailDiv - 1) / kTailDiv) : 0;
    r.full = (T - r.tail) / c;
    r.rem = (T - r.tail) % c;
    return r;
}

static bool make_layout(const ff_system* s, int32_t n_sys, int32_t m_max, Layout& L, SysInfo* sys, FarTmp& ft,
                        int32_t cfg_req = -1, int32_t chunk_req = 0, int32_t chunk64_req = 0,
                        bool energy_only = false) {
    std::memset(&L, 0, sizeof L);
    if (!s || n_sys < 1 || !sys) return false;
    if (m_max < 0 || m_max > kMaxM) return false;
    long long n_tot = 0;
    int n_max = 0;
    for (int k = 0; k < n_sys; ++k) {
        if (s[k].n_atoms < 1 || s[k].n_bonds < 0 || s[k].n_angles < 0 || s[k].n_dihedrals < 0) return false;
        n_tot += s[k].n_atoms;
        n_max = std::max(n_max, s[k].n_atoms);
    }
    if (n_tot > (1 << 28)) return false;
    if (ft.cap < far_capacity(s, n_sys)) return false;
    L.n_sys = n_sys;
    // defaults from sweeps of whole FP32 and FP64 evaluations on MI355X
    // (2,048 to 50,000 atoms, configurations x chunk lengths 1 to 16, per
    // precision): batches use 128-atom blocks with two atoms per lane in both
    // kernels (the 256-chain batch of 200-4,000 atoms: 4 % less per FP64
    // evaluation than with 64-atom blocks, 2 % more per FP32 one); systems up
    // to 1,024 atoms 64-atom blocks; up to 12,288 atoms 256-atom blocks with
    // one atom per lane (enough workgroups to fill the chip); up to 20,000
    // atoms 128-atom blocks with two atoms per lane (15k atoms: 5 % less per
    // evaluation than 256-atom blocks); above, 256-atom blocks with two atoms
    // per lane in FP32 and four in FP64.  The FP64 kernel, with fewer and
    // longer-lived wavefronts, gains from longer chunks as the system grows
    // (two j-tiles from 6,145 atoms up to 12,287 and from 20,000, four from
    // 32,768, eight from 45,000 on: 1.49 instead of 1.55 ms per FP64
    // evaluation at 50k atoms), the FP32 kernel from two j-tiles only above
    // 32,768 atoms
    auto pick = [&](int cfg, int c32, int c64) { L.cfg = cfg; L.chunk[0] = c32; L.chunk[1] = c64; };
    if (n_sys > 1) pick(9, 4, 4);
    else if (n_max <= 1024) pick(0, 1, 1);
    else if (n_max <= 6144) pick(1, 1, 1);
    else if (n_max < 12288) pick(1, 1, 2);
    else if (n_max < 20000) pick(9, 1, 1);
    else if (n_max < 32768) pick(8, 1, 2);
    else if (n_max < 45000) pick(8, 2, 4);
    else pick(8, 2, 8);
    if (cfg_req >= 0) {
        if (chunk64_req == 0) chunk64_req = chunk_req;
        if (cfg_req >= kNumTileConfigs || chunk_req < 1 || chunk_req > kMaxChunk || chunk64_req < 1 ||
            chunk64_req > kMaxChunk)
            return false;
        pick(cfg_req, chunk_req, chunk64_req);
    }
    L.block = kTileConfigs[L.cfg].block;
    int aoff = 0, uoff = 0, units = 0, nbd = 0, nag = 0, ndh = 0, ebo = 0;
    int chunks[2] = {0, 0};
    size_t red = 0;
    L.acc_rows = std::max(1, m_max + 1);
    for (int k = 0; k < n_sys; ++k) {
        SysInfo& si = sys[k];
        std::memset(&si, 0, sizeof si);
        si.n = s[k].n_atoms;
        si.np = (si.n + L.block - 1) / L.block * L.block;
        si.aoff = aoff;
        si.uoff = uoff;
        si.row0 = aoff / L.block;
        si.nb = si.np / L.block;
        si.chunk0[0] = chunks[0];
        si.chunk0[1] = chunks[1];
        const int nt = si.np / kTile;
        for (int b = 0; b < si.nb; ++b) {
            const int t0 = b * L.block / kTile;
            units += nt - t0;
            for (int p = 0; p < 2; ++p) chunks[p] += row_split(nt - t0, L.chunk[p]).count();
        }
        for (int p = 0; p < 2; ++p) si.n_chunks[p] = chunks[p] - si.chunk0[p];
        si.n_bonds = s[k].n_bonds;
        si.n_angles = s[k].n_angles;
        si.n_dihedrals = s[k].n_dihedrals;
        si.bond0 = nbd;
        si.angle0 = nag;
        si.dih0 = ndh;
        nbd += si.n_bonds;
        nag += si.n_angles;
        ndh += si.n_dihedrals;
        const int terms = si.n_bonds + si.n_angles + si.n_dihedrals;
        si.bonded_blocks = std::max(1, (terms + kBondedPerBlock - 1) / kBondedPerBlock);
        si.eb0 = ebo;
        ebo += si.bonded_blocks;
        si.fin_blocks = (si.n + kTile - 1) / kTile;      // one finalize workgroup per tile
        si.vec_blocks = (3 * si.n + kFinBlock - 1) / kFinBlock;
        si.acc_bx = std::max(1, std::min(64, (3 * si.n + 8 * kFinBlock - 1) / (8 * kFinBlock)));
        si.red0 = (int32_t)red;
        red += std::max((size_t)si.fin_blocks * 4, (size_t)si.acc_bx * L.acc_rows * 6);
        L.n_vec_blocks += si.vec_blocks;
        L.n_acc_blocks += si.acc_bx;
        aoff += si.np;
        uoff += si.n;
    }
    L.n = uoff;
    L.np = aoff;
    L.nb = aoff / L.block;
    L.nt = aoff / kTile;
    L.n_units = units;
    L.n_chunks[0] = chunks[0];
    L.n_chunks[1] = chunks[1];
    const size_t max_chunks = (size_t)std::max(chunks[0], chunks[1]);
    L.n_bonds = nbd;
    L.n_angles = nag;
    L.n_dihedrals = ndh;
    L.n_terms_slots = 2 * nbd + 3 * nag + 4 * ndh;
    L.n_bonded_blocks = ebo;
    L.n_fin_blocks = 0;
    for (int k = 0; k < n_sys; ++k) L.n_fin_blocks += sys[k].fin_blocks;
    ft.n_pairs = 0;
    for (int k = 0; k < n_sys; ++k) far_exclusions(s[k], sys[k].aoff, ft);
    for (size_t q = 0; q < ft.n_pairs; ++q)
        ft.keys[q] = ((long long)(ft.pairs[q].lo / L.block) << 32) | (long long)(ft.pairs[q].hi / kTile);
    std::sort(ft.keys, ft.keys + ft.n_pairs);
    ft.n_keys = (size_t)(std::unique(ft.keys, ft.keys + ft.n_pairs) - ft.keys);
    L.n_far_units = (int32_t)ft.n_keys;
    L.m_max = m_max;
    L.vstride = (3 * (size_t)L.np + 31) / 32 * 32;
    L.ctl_stride = align256(sizeof(Ctl));
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t r = o; o = align256(o + std::max<size_t>(bytes, 1)); return r; };
    const size_t np = L.np;
    // packed once per context (pack_static), read only afterwards
    L.off_sys = take((size_t)n_sys * sizeof(SysInfo));
    L.off_c12 = take(np * 4);
    L.off_c6 = take(np * 4);
    L.off_q = take(np * 4);
    L.off_c12d = take(np * 8);
    L.off_c6d = take(np * 8);
    L.off_qd = take(np * 8);
    L.off_excl = take(np * 8);
    L.off_chunks[0] = take((size_t)L.n_chunks[0] * sizeof(ChunkInfo));
    L.off_chunks[1] = take((size_t)L.n_chunks[1] * sizeof(ChunkInfo));
    L.off_rows = take((size_t)L.nb * sizeof(RowInfo));
    L.off_bond = take((size_t)L.n_bonds * 8);
    L.off_bondp = take((size_t)L.n_bonds * 16);
    L.off_angle = take((size_t)L.n_angles * 12);
    L.off_anglep = take((size_t)L.n_angles * 16);
    L.off_dih = take((size_t)L.n_dihedrals * 16);
    L.off_dihp = take((size_t)L.n_dihedrals * 32);
    L.off_inc_start = take((np + 1) * 4);
    L.off_inc = take((size_t)L.n_terms_slots * 4);
    L.off_map_fin = take((size_t)L.n_fin_blocks * 8);
    L.off_map_vec = take((size_t)L.n_vec_blocks * 8);
    L.off_map_bonded = take((size_t)L.n_bonded_blocks * 8);
    L.off_map_acc = take((size_t)L.n_acc_blocks * 8);
    L.off_far_unit = take((size_t)L.n_units * 4);
    L.off_far_mask = take((size_t)L.n_far_units * L.block * 8);
    L.static_end = o;
    // written by the kernels
    L.off_batch = take(sizeof(BatchState));
    L.off_ctl = take((size_t)n_sys * L.ctl_stride);
    L.off_pi = take(max_chunks * L.block * 3 * 8);
    L.off_pj = take((size_t)L.n_units * kTile * 3 * 8);
    L.off_ep = take(max_chunks * 8);
    L.off_fb = take((size_t)L.n_terms_slots * 24);
    L.off_eb = take((size_t)L.n_bonded_blocks * 8);
    L.off_red = take(red * 8);
    L.off_vec = take(energy_only ? 0 : (size_t)V_COUNT * L.vstride * 8 + (size_t)kTraceCap * 3 * 8);
    L.total = o;
    return true;
}

// make_layout with its host storage on the heap (every entry point but
// ff_energy_grad_noalloc).
struct LayoutHost {
    std::vector<SysInfo> sys;
    std::vector<FarPair> pairs;
    std::vector<long long> keys;
    FarTmp ft{nullptr, nullptr, 0};
};

static bool layout_heap(const ff_system* s, int32_t n_sys, int32_t m_max, Layout& L, LayoutHost& h,
                        int32_t cfg_req = -1, int32_t chunk_req = 0, int32_t chunk64_req = 0) {
    std::memset(&L, 0, sizeof L);
    if (!s || n_sys < 1) return false;
    const size_t cap = far_capacity(s, n_sys);
    h.sys.assign(n_sys, SysInfo{});
    h.pairs.assign(cap, FarPair{0, 0});
    h.keys.assign(cap, 0);
    h.ft = FarTmp{h.pairs.data(), h.keys.data(), cap};
    return make_layout(s, n_sys, m_max, L, h.sys.data(), h.ft, cfg_req, chunk_req, chunk64_req);
}

static double* trace_buffer(const ff_ctx* c) {
    return at<double>(c->ws, c->L.off_vec) + (size_t)V_COUNT * c->L.vstride;
}

// Host-side validation of one system; returns FF_OK or the error.  Sets the
// near-exclusion bits of its atoms in excl (global padded index).
static ff_status validate_system(const ff_system* s, int k, uint64_t* excl, int aoff) {
    const int n = s->n_atoms;
    if (!s->q || !s->sigma || !s->eps) return fail(FF_ERR_ARG, "system %d: per-atom parameter arrays are null", k);
    if ((s->n_bonds && (!s->bond || !s->bond_k || !s->bond_r0)) ||
        (s->n_angles && (!s->angle || !s->angle_k || !s->angle_t0)) ||
        (s->n_dihedrals && (!s->dihedral || !s->dihedral_v)))
        return fail(FF_ERR_ARG, "system %d: topology arrays are null", k);
    if (!(std::isfinite(s->coulomb_c))) return fail(FF_ERR_ARG, "system %d: coulomb_c is not finite", k);
    if (s->coulomb_c < 0.0) return fail(FF_ERR_UNSUPPORTED, "system %d: negative coulomb_c", k);
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(s->q[i]) || !(s->sigma[i] >= 0.0) || !(s->eps[i] >= 0.0) || !std::isfinite(s->sigma[i]) ||
            !std::isfinite(s->eps[i]))
            return fail(FF_ERR_ARG, "system %d: bad parameters of atom %d (sigma, eps must be finite and >= 0)", k, i);
    auto add_excl = [&](int i, int j) -> ff_status {
        if (i == j) return fail(FF_ERR_ARG, "system %d: a bond or angle joins atom %d to itself", k, i);
        const int lo = std::min(i, j), hi = std::max(i, j);
        if (hi - lo <= kExclWindow) excl[aoff + lo] |= 1ull << (hi - lo - 1);   // farther: far-unit masks
        return FF_OK;
    };
    for (int b = 0; b < s->n_bonds; ++b) {
        const int i = s->bond[2 * b], j = s->bond[2 * b + 1];
        if (i < 0 || i >= n || j < 0 || j >= n) return fail(FF_ERR_ARG, "system %d: bond %d has an atom index out of range", k, b);
        if (!std::isfinite(s->bond_k[b]) || !std::isfinite(s->bond_r0[b])) return fail(FF_ERR_ARG, "system %d: bond %d parameters", k, b);
        ff_status st = add_excl(i, j);
        if (st) return st;
    }
    for (int a = 0; a < s->n_angles; ++a) {
        const int* t = s->angle + 3 * a;
        for (int q = 0; q < 3; ++q)
            if (t[q] < 0 || t[q] >= n) return fail(FF_ERR_ARG, "system %d: angle %d has an atom index out of range", k, a);
        if (t[0] == t[1] || t[1] == t[2]) return fail(FF_ERR_ARG, "system %d: angle %d repeats its vertex", k, a);
        ff_status st = add_excl(t[0], t[2]);
        if (st) return st;
    }
    for (int d = 0; d < s->n_dihedrals; ++d)
        for (int q = 0; q < 4; ++q)
            if (s->dihedral[4 * d + q] < 0 || s->dihedral[4 * d + q] >= n)
                return fail(FF_ERR_ARG, "system %d: dihedral %d has an atom index out of range", k, d);
    return FF_OK;
}

// Validates the systems and writes the host image of the workspace's packed
// part, [0, L.static_end), into img: per-atom factors, exclusion bitmasks,
// tile tables, bonded topology with the per-atom incidence lists, far
// exclusion masks and the grid maps.  Uses no heap memory.
static ff_status pack_static(const ff_system* systems, int32_t n_sys, const Layout& L, const SysInfo* sys,
                             const FarTmp& ft, char* img) {
    std::memset(img, 0, L.static_end);
    uint64_t* excl = at<uint64_t>(img, L.off_excl);
    for (int k = 0; k < n_sys; ++k) {
        ff_status st = validate_system(&systems[k], k, excl, sys[k].aoff);
        if (st) return st;
    }
    std::memcpy(img + L.off_sys, sys, (size_t)n_sys * sizeof(SysInfo));
    // per-atom factors: c12 = 2 sqrt(eps) sigma^6, c6 = 2 sqrt(eps) sigma^3,
    // q^ = sqrt(C) q; padding atoms keep zero factors
    float* c12f = at<float>(img, L.off_c12);
    float* c6f = at<float>(img, L.off_c6);
    float* qf = at<float>(img, L.off_q);
    double* c12d = at<double>(img, L.off_c12d);
    double* c6d = at<double>(img, L.off_c6d);
    double* qd = at<double>(img, L.off_qd);
    for (int k = 0; k < n_sys; ++k) {
        const ff_system& s = systems[k];
        const double sqc = std::sqrt(s.coulomb_c);
        for (int i = 0; i < s.n_atoms; ++i) {
            const int g = sys[k].aoff + i;
            const double se = 2.0 * std::sqrt(s.eps[i]);
            const double s3 = s.sigma[i] * s.sigma[i] * s.sigma[i];
            c12d[g] = se * s3 * s3;
            c6d[g] = se * s3;
            qd[g] = sqc * s.q[i];
            c12f[g] = (float)c12d[g];
            c6f[g] = (float)c6d[g];
            qf[g] = (float)qd[g];
        }
    }
    // tile tables (global I-block and j-tile indices): rows, then each chunk
    // table in launch order (three passes: full-length chunks, shorter
    // remainders, one-tile chunks; each pass row by row)
    RowInfo* rows = at<RowInfo>(img, L.off_rows);
    int unit = 0, slot[2] = {0, 0};
    for (int k = 0; k < n_sys; ++k) {
        const SysInfo& si = sys[k];
        const int tile0 = si.aoff / kTile, nt = si.np / kTile;
        for (int b = 0; b < si.nb; ++b) {
            const int row = si.row0 + b;
            const int t0 = tile0 + b * L.block / kTile, t_end = tile0 + nt;
            rows[row].unit_start = unit;
            rows[row].t0 = t0;
            for (int p = 0; p < 2; ++p) {
                rows[row].chunk_start[p] = slot[p];
                rows[row].n_chunks[p] = row_split(t_end - t0, L.chunk[p]).count();
                slot[p] += rows[row].n_chunks[p];
            }
            unit += t_end - t0;
        }
    }
    if (slot[0] != L.n_chunks[0] || slot[1] != L.n_chunks[1] || unit != L.n_units)
        return fail(FF_ERR_ARG, "internal: tile table size mismatch");
    for (int p = 0; p < 2; ++p) {
        ChunkInfo* chunks = at<ChunkInfo>(img, L.off_chunks[p]);
        const int c_len = L.chunk[p];
        int nch = 0;
        for (int pass = 0; pass < 3; ++pass) {
            for (int k = 0; k < n_sys; ++k) {
                const SysInfo& si = sys[k];
                const int t_end = si.aoff / kTile + si.np / kTile;
                for (int row = si.row0; row < si.row0 + si.nb; ++row) {
                    const RowInfo& ri = rows[row];
                    const RowSplit sp = row_split(t_end - ri.t0, c_len);
                    int t = ri.t0, q = ri.chunk_start[p];
                    auto emit = [&](int len, int in_pass) {
                        if (in_pass == pass) {
                            ChunkInfo& c = chunks[nch++];
                            c.row = row;
                            c.t_begin = t;
                            c.t_end = t + len;
                            c.unit_base = ri.unit_start + (t - ri.t0);
                            c.sys = k;
                            c.slot = q;
                        }
                        t += len;
                        ++q;
                    };
                    for (int i = 0; i < sp.full; ++i) emit(c_len, c_len == 1 ? 2 : 0);
                    if (sp.rem > 0) emit(sp.rem, sp.rem == 1 ? 2 : 1);
                    for (int i = 0; i < sp.tail; ++i) emit(1, 2);
                    if (t != t_end || q != ri.chunk_start[p] + ri.n_chunks[p])
                        return fail(FF_ERR_ARG, "internal: chunk split mismatch");
                }
            }
        }
        if (nch != L.n_chunks[p]) return fail(FF_ERR_ARG, "internal: chunk table size mismatch");
    }
    // bonded topology (local atom indices) and parameters
    int* bond = at<int>(img, L.off_bond);
    double* bondp = at<double>(img, L.off_bondp);
    int* angle = at<int>(img, L.off_angle);
    double* anglep = at<double>(img, L.off_anglep);
    int* dih = at<int>(img, L.off_dih);
    double* dihp = at<double>(img, L.off_dihp);
    const int abase = 2 * L.n_bonds, dbase = abase + 3 * L.n_angles;
    for (int k = 0; k < n_sys; ++k) {
        const ff_system& s = systems[k];
        const SysInfo& si = sys[k];
        for (int b = 0; b < s.n_bonds; ++b) {
            const int gb = si.bond0 + b;
            bond[2 * gb] = s.bond[2 * b];
            bond[2 * gb + 1] = s.bond[2 * b + 1];
            bondp[2 * gb] = s.bond_k[b];
            bondp[2 * gb + 1] = s.bond_r0[b];
        }
        for (int a = 0; a < s.n_angles; ++a) {
            const int ga = si.angle0 + a;
            for (int q = 0; q < 3; ++q) angle[3 * ga + q] = s.angle[3 * a + q];
            anglep[2 * ga] = s.angle_k[a];
            anglep[2 * ga + 1] = s.angle_t0[a];
        }
        for (int d = 0; d < s.n_dihedrals; ++d) {
            const int gd = si.dih0 + d;
            for (int q = 0; q < 4; ++q) {
                dih[4 * gd + q] = s.dihedral[4 * d + q];
                dihp[4 * gd + q] = s.dihedral_v[4 * d + q];
            }
        }
    }
    // incidence lists: the term slots of every global padded atom in
    // increasing slot order (bonds, then angles, then torsions), by counting;
    // inc_start[a + 1] serves as atom a's fill cursor and ends at the start of
    // atom a + 1
    int* inc_start = at<int>(img, L.off_inc_start);
    int* inc = at<int>(img, L.off_inc);
    auto each_slot = [&](auto&& visit) {
        for (int k = 0; k < n_sys; ++k) {
            const ff_system& s = systems[k];
            const SysInfo& si = sys[k];
            for (int b = 0; b < s.n_bonds; ++b)
                for (int q = 0; q < 2; ++q) visit(si.aoff + s.bond[2 * b + q], 2 * (si.bond0 + b) + q);
            for (int a = 0; a < s.n_angles; ++a)
                for (int q = 0; q < 3; ++q) visit(si.aoff + s.angle[3 * a + q], abase + 3 * (si.angle0 + a) + q);
            for (int d = 0; d < s.n_dihedrals; ++d)
                for (int q = 0; q < 4; ++q) visit(si.aoff + s.dihedral[4 * d + q], dbase + 4 * (si.dih0 + d) + q);
        }
    };
    // (counts of atom a at a + 2: after the prefix sum inc_start[a + 1] is
    // where atom a's list starts; the last atom's count is not needed)
    each_slot([&](int atom, int) { if (atom + 2 <= L.np) ++inc_start[atom + 2]; });
    for (int a = 2; a <= L.np; ++a) inc_start[a] += inc_start[a - 1];
    each_slot([&](int atom, int slot) { inc[inc_start[atom + 1]++] = slot; });
    if (inc_start[L.np] != L.n_terms_slots) return fail(FF_ERR_ARG, "internal: incidence list size mismatch");
    // far exclusions: per-unit index of its mask block, or -1, and per
    // (unit, i-atom) masks over the unit's j-tile
    int32_t* fu = at<int32_t>(img, L.off_far_unit);
    uint64_t* fm = at<uint64_t>(img, L.off_far_mask);
    for (int u = 0; u < L.n_units; ++u) fu[u] = -1;
    for (size_t q = 0; q < ft.n_keys; ++q) {
        const int row = (int)(ft.keys[q] >> 32), t = (int)(ft.keys[q] & 0xffffffffLL);
        fu[rows[row].unit_start + t - rows[row].t0] = (int32_t)q;
    }
    for (size_t q = 0; q < ft.n_pairs; ++q) {
        const FarPair& p = ft.pairs[q];
        const int row = p.lo / L.block, t = p.hi / kTile;
        const int blk = fu[rows[row].unit_start + t - rows[row].t0];
        fm[(size_t)blk * L.block + (p.lo - row * L.block)] |= 1ull << (p.hi - t * kTile);
    }
    // flat grid maps: (system, local block) of every workgroup
    int32_t* mf = at<int32_t>(img, L.off_map_fin);
    int32_t* mv = at<int32_t>(img, L.off_map_vec);
    int32_t* mb = at<int32_t>(img, L.off_map_bonded);
    int32_t* ma = at<int32_t>(img, L.off_map_acc);
    for (int k = 0; k < n_sys; ++k) {
        for (int b = 0; b < sys[k].fin_blocks; ++b) { *mf++ = k; *mf++ = b; }
        for (int b = 0; b < sys[k].vec_blocks; ++b) { *mv++ = k; *mv++ = b; }
        for (int b = 0; b < sys[k].bonded_blocks; ++b) { *mb++ = k; *mb++ = b; }
        for (int b = 0; b < sys[k].acc_bx; ++b) { *ma++ = k; *ma++ = b; }
    }
    return FF_OK;
}

// Bonded terms, pair kernel and finalize of one direct evaluation.
static ff_status launch_energy(const Layout& L, char* ws, const double* xyz, double* energy, double* grad,
                               int32_t precision, hipStream_t st) {
    Args a{};
    a.L = L;
    a.ws = ws;
    a.xyz_in = xyz;
    a.e_out = energy;
    a.g_out = grad;
    a.direct = 1;
    a.direct_prec = precision;
    HIP_TRY(launch_bonded(a, st));
    HIP_TRY(launch_pair(a, precision, st));
    HIP_TRY(launch_finalize(a, st));
    return FF_OK;
}

extern "C" {

size_t ff_workspace_bytes_batch(const ff_system* sys, int32_t n_sys, int32_t m_max) {
    Layout L;
    LayoutHost h;
    if (!layout_heap(sys, n_sys, m_max, L, h)) return 0;
    return L.total;
}

size_t ff_workspace_bytes_tiled(const ff_system* sys, int32_t n_sys, int32_t m_max, int32_t tile_config,
                                int32_t chunk, int32_t chunk64) {
    Layout L;
    LayoutHost h;
    if (tile_config < 0 || chunk64 < 0 || !layout_heap(sys, n_sys, m_max, L, h, tile_config, chunk, chunk64))
        return 0;
    return L.total;
}

int32_t ff_num_tile_configs(void) { return kNumTileConfigs; }

ff_status ff_tile_config_info(int32_t cfg, int32_t* block, int32_t* waves32, int32_t* ipl32, int32_t* waves64,
                              int32_t* ipl64) {
    clear_error();
    if (cfg < 0 || cfg >= kNumTileConfigs) return fail(FF_ERR_ARG, "tile configuration %d outside [0, %d)", cfg,
                                                       kNumTileConfigs);
    const TileConfig& t = kTileConfigs[cfg];
    if (block) *block = t.block;
    if (waves32) *waves32 = t.waves32;
    if (ipl32) *ipl32 = t.ipl32;
    if (waves64) *waves64 = t.waves64;
    if (ipl64) *ipl64 = t.ipl64;
    return FF_OK;
}

size_t ff_workspace_bytes(const ff_system* sys, int32_t m_max) { return ff_workspace_bytes_batch(sys, 1, m_max); }

void ff_default_params(ff_min_params* p) {
    if (!p) return;
    p->method = FF_LBFGS;
    p->m = 10;
    p->tol = 1e-3;
    p->max_iter = 2000;
    p->precision = FF_FP64;
    p->linesearch = FF_LS_DEFAULT;
    p->ls_K = 2;
    p->h_init = 0.1;
    p->k_plus = 2.0;
    p->k_minus = 0.5;
    p->eps_h = 1e-10;
    p->cg_restart = 0;
    p->flags = 0;
    p->cg_beta = FF_CG_PRP;
    p->ls_par_g0 = 1;
    p->fgm_restart = 0;
    p->hb_alpha = 0.0;
    p->hb_beta = 0.0;
}

const char* ff_last_error(void) { return g_err; }

int32_t ff_batch_size(const ff_ctx* c) { return c ? c->L.n_sys : 0; }

static ff_status create_impl(const ff_system* systems, int32_t n_sys, void* workspace, size_t ws_bytes,
                             int32_t m_max, int32_t cfg_req, int32_t chunk_req, int32_t chunk64_req, void* stream,
                             ff_ctx** out) {
    clear_error();
    if (!out) return fail(FF_ERR_ARG, "out is null");
    *out = nullptr;
    if (!systems || n_sys < 1) return fail(FF_ERR_ARG, "need at least one system");
    for (int k = 0; k < n_sys; ++k)
        if (systems[k].n_atoms < 1) return fail(FF_ERR_ARG, "system %d: n_atoms must be >= 1", k);
    if (m_max < 0 || m_max > kMaxM) return fail(FF_ERR_ARG, "m_max must be in [0, %d]", kMaxM);
    Layout L;
    LayoutHost h;
    if (cfg_req >= 0 && (cfg_req >= kNumTileConfigs || chunk_req < 1 || chunk_req > kMaxChunk ||
                         chunk64_req < 0 || chunk64_req > kMaxChunk))
        return fail(FF_ERR_ARG, "tile configuration %d / chunks %d, %d outside [0, %d) / [1, %d] (chunk64 0: = chunk)",
                    cfg_req, chunk_req, chunk64_req, kNumTileConfigs, kMaxChunk);
    if (!layout_heap(systems, n_sys, m_max, L, h, cfg_req, chunk_req, chunk64_req))
        return fail(FF_ERR_ARG, "invalid sizes");
    if (!workspace || ((uintptr_t)workspace & 255)) return fail(FF_ERR_WORKSPACE, "workspace null or not 256-byte aligned");
    if (ws_bytes < L.total) return fail(FF_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, L.total);
    std::vector<char> img(L.static_end);
    ff_status ps = pack_static(systems, n_sys, L, h.sys.data(), h.ft, img.data());
    if (ps) return ps;
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)workspace;
    HIP_TRY(hipMemcpyAsync(ws, img.data(), L.static_end, hipMemcpyHostToDevice, st));
    Args a{};
    a.L = L;
    a.ws = ws;
    HIP_TRY(launch_reset(a, st));
    HIP_TRY(hipStreamSynchronize(st));

    ff_ctx* c = new ff_ctx();
    c->L = L;
    c->ws = ws;
    c->sys = std::move(h.sys);
    void* hf = nullptr;
    void* hc = nullptr;
    if (hipHostMalloc(&hf, 256, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&hc, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) {
        if (hf) (void)hipHostFree(hf);
        delete c;
        return fail(FF_ERR_HIP, "pinned host buffer allocation failed");
    }
    c->host_flag = (int32_t*)hf;
    c->host_ctl = (Ctl*)hc;
    if (hipStreamCreate(&c->own) != hipSuccess) {
        (void)hipHostFree(hf);
        (void)hipHostFree(hc);
        delete c;
        return fail(FF_ERR_HIP, "stream creation failed");
    }
    *out = c;
    return FF_OK;
}

ff_status ff_create_batch(const ff_system* systems, int32_t n_sys, void* workspace, size_t ws_bytes, int32_t m_max,
                          void* stream, ff_ctx** out) {
    return create_impl(systems, n_sys, workspace, ws_bytes, m_max, -1, 0, 0, stream, out);
}

ff_status ff_create_tiled(const ff_system* systems, int32_t n_sys, void* workspace, size_t ws_bytes,
                          int32_t m_max, int32_t tile_config, int32_t chunk, int32_t chunk64, void* stream,
                          ff_ctx** out) {
    if (tile_config < 0) {
        fail(FF_ERR_ARG, "tile_config must be >= 0 (ff_create_batch picks one itself)");
        if (out) *out = nullptr;
        return FF_ERR_ARG;
    }
    return create_impl(systems, n_sys, workspace, ws_bytes, m_max, tile_config, chunk, chunk64, stream, out);
}

ff_status ff_get_tiling(const ff_ctx* c, int32_t* tile_config, int32_t* chunk, int32_t* chunk64) {
    if (!c) {
        fail(FF_ERR_ARG, "context is null");
        return FF_ERR_ARG;
    }
    if (tile_config) *tile_config = c->L.cfg;
    if (chunk) *chunk = c->L.chunk[0];
    if (chunk64) *chunk64 = c->L.chunk[1];
    return FF_OK;
}

// Candidate chunk lengths of the autotuner (j-tiles per pair workgroup).
static const int32_t kTuneChunks[] = {1, 2, 4, 8, 16};

size_t ff_autotune_workspace_bytes(const ff_system* systems, int32_t n_sys) {
    size_t best = 0;
    for (int cfg = 0; cfg < kNumTileConfigs; ++cfg)
        for (int32_t ch : kTuneChunks) {
            Layout L;
            LayoutHost h;
            if (!layout_heap(systems, n_sys, 0, L, h, cfg, ch)) return 0;
            best = std::max(best, L.total);
        }
    return best ? best + align256(8 * (size_t)n_sys) : 0;
}

ff_status ff_autotune(const ff_system* systems, int32_t n_sys, const double* xyz, void* workspace,
                      size_t ws_bytes, int32_t precision, int32_t reps, void* stream, int32_t* tile_config,
                      int32_t* chunk, double* ms_per_eval) {
    clear_error();
    if (!systems || n_sys < 1 || !xyz || !workspace || reps < 1 || !tile_config || !chunk)
        return fail(FF_ERR_ARG, "bad arguments");
    if (precision != FF_FP64 && precision != FF_FP32_ACC64) return fail(FF_ERR_ARG, "bad precision %d", precision);
    if ((uintptr_t)workspace & 255) return fail(FF_ERR_WORKSPACE, "workspace not 256-byte aligned");
    const size_t tail = align256(8 * (size_t)n_sys);
    if (ws_bytes < tail + 256) return fail(FF_ERR_WORKSPACE, "workspace too small");
    hipStream_t st = (hipStream_t)stream;
    // the energies of the timed evaluations go to the tail of the workspace
    const size_t usable = (ws_bytes - tail) & ~(size_t)255;
    double* e_out = (double*)((char*)workspace + usable);
    double best_ms = 0.0;
    int32_t best_cfg = -1, best_chunk = 0;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return fail(FF_ERR_HIP, "event"); }
    ff_status result = FF_OK;
    std::vector<double> e_tmp;
    for (int cfg = 0; cfg < kNumTileConfigs && result == FF_OK; ++cfg) {
        for (int32_t ch : kTuneChunks) {
            Layout L;
            LayoutHost h;
            if (!layout_heap(systems, n_sys, 0, L, h, cfg, ch) || L.total > usable) continue;
            ff_ctx* c = nullptr;
            ff_status s = create_impl(systems, n_sys, workspace, usable, 0, cfg, ch, ch, stream, &c);
            if (s) { result = s; break; }
            double* eo = e_out;
            hipError_t e = ff_energy_grad(c, xyz, eo, nullptr, precision, st) == FF_OK ? hipSuccess : hipErrorUnknown;
            if (e == hipSuccess) e = hipEventRecord(e0, st);
            for (int r = 0; r < reps && e == hipSuccess; ++r)
                e = ff_energy_grad(c, xyz, eo, nullptr, precision, st) == FF_OK ? hipSuccess : hipErrorUnknown;
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            ff_destroy(c);
            if (e != hipSuccess) { result = fail(FF_ERR_HIP, "autotune timing failed"); break; }
            const double per = (double)ms / reps;
            if (best_cfg < 0 || per < best_ms) { best_ms = per; best_cfg = cfg; best_chunk = ch; }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result != FF_OK) return result;
    if (best_cfg < 0) return fail(FF_ERR_WORKSPACE, "no tile configuration fits in %zu bytes", ws_bytes);
    *tile_config = best_cfg;
    *chunk = best_chunk;
    if (ms_per_eval) *ms_per_eval = best_ms;
    return FF_OK;
}

ff_status ff_create(const ff_system* s, void* workspace, size_t ws_bytes, int32_t m_max, void* stream,
                    ff_ctx** out) {
    if (!s) {
        fail(FF_ERR_ARG, "system is null");
        if (out) *out = nullptr;
        return FF_ERR_ARG;
    }
    return ff_create_batch(s, 1, workspace, ws_bytes, m_max, stream, out);
}

ff_status ff_destroy(ff_ctx* c) {
    if (!c) return FF_OK;
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    if (c->graph64) (void)hipGraphExecDestroy(c->graph64);
    if (c->own) (void)hipStreamDestroy(c->own);
    (void)hipHostFree(c->host_flag);
    (void)hipHostFree(c->host_ctl);
    delete c;
    return FF_OK;
}

ff_status ff_energy_grad(ff_ctx* c, const double* xyz, double* energy, double* grad, int32_t precision,
                         void* stream) {
    clear_error();
    if (!c) return fail(FF_ERR_ARG, "context is null");
    if (!xyz || !energy) return fail(FF_ERR_ARG, "xyz and energy must be device pointers");
    if (precision != FF_FP64 && precision != FF_FP32_ACC64) return fail(FF_ERR_ARG, "bad precision %d", precision);
    return launch_energy(c->L, c->ws, xyz, energy, grad, precision, (hipStream_t)stream);
}

ff_status ff_energy_grad_noalloc(const ff_system* sys, const double* xyz, double* energy, double* grad,
                                 int32_t precision, void* stream) {
    clear_error();
    if (!sys || !xyz || !energy) return fail(FF_ERR_ARG, "sys, xyz and energy must not be null");
    if (sys->n_atoms < 1) return fail(FF_ERR_ARG, "n_atoms must be >= 1");
    if (precision != FF_FP64 && precision != FF_FP32_ACC64) return fail(FF_ERR_ARG, "bad precision %d", precision);
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    // the far-exclusion temporaries take the end of the host stage
    const size_t cap = far_capacity(sys, 1);
    const size_t tmp_bytes = align256(cap * (sizeof(FarPair) + sizeof(long long)));
    if (tmp_bytes >= sizeof g_stage)
        return fail(FF_ERR_UNSUPPORTED, "%zu bonds and angles exceed what ff_energy_grad_noalloc stages",
                    (size_t)sys->n_bonds + (size_t)sys->n_angles);
    char* tmp = g_stage + sizeof g_stage - tmp_bytes;
    FarTmp ft{reinterpret_cast<FarPair*>(tmp), reinterpret_cast<long long*>(tmp + cap * sizeof(FarPair)), cap};
    Layout L;
    SysInfo si;
    if (!make_layout(sys, 1, 0, L, &si, ft, -1, 0, 0, true)) return fail(FF_ERR_ARG, "invalid sizes");
    if (L.total > FF_NOALLOC_SCRATCH_BYTES || L.static_end > sizeof g_stage - tmp_bytes)
        return fail(FF_ERR_UNSUPPORTED, "a system of %d atoms needs %zu bytes of device scratch; "
                    "ff_energy_grad_noalloc has %zu (use a context)", sys->n_atoms, L.total,
                    (size_t)FF_NOALLOC_SCRATCH_BYTES);
    ff_status ps = pack_static(sys, 1, L, &si, ft, g_stage);
    if (ps) return ps;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(FF_ERR_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || ((uintptr_t)p & 255)) return fail(FF_ERR_HIP, "scratch symbol address %p not usable", p);
        g_scratch_dev[dev] = p;
    }
    char* ws = static_cast<char*>(g_scratch_dev[dev]);
    hipStream_t st = (hipStream_t)stream;
    // stream-ordered after earlier work on `stream`; the wait keeps the host
    // stage intact until the copy has read it
    HIP_TRY(hipMemcpyAsync(ws, g_stage, L.static_end, hipMemcpyHostToDevice, st));
    Args a{};
    a.L = L;
    a.ws = ws;
    HIP_TRY(launch_reset(a, st));
    HIP_TRY(hipStreamSynchronize(st));
    return launch_energy(L, ws, xyz, energy, grad, precision, st);
}

static constexpr int kCyclesPerGraph = 4;

// with32 = false leaves the FP32 pair kernel out: FP64 runs, and FP32-mode
// runs once every system has switched to FP64 (the switch is final).
static ff_status build_graph(ff_ctx* c, bool with32, hipGraphExec_t* out) {
    hipStream_t st = c->own;
    Args a{};
    a.L = c->L;
    a.ws = c->ws;
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    // several cycles per graph: each graph launch costs a few us of its own
    hipError_t e = hipSuccess;
    for (int k = 0; k < kCyclesPerGraph && e == hipSuccess; ++k) {
        e = launch_cycle_vec(a, 0, st);
        if (e == hipSuccess) e = launch_bonded(a, st);
        if (e == hipSuccess && with32) e = launch_pair(a, 1, st);
        if (e == hipSuccess) e = launch_pair(a, 0, st);
        if (e == hipSuccess) e = launch_finalize(a, st);
        if (e == hipSuccess) e = launch_cycle_vec(a, 1, st);
    }
    hipError_t e2 = hipStreamEndCapture(st, &g);
    if (e != hipSuccess) return fail(FF_ERR_HIP, "graph capture: %s", hipGetErrorString(e));
    if (e2 != hipSuccess) return fail(FF_ERR_HIP, "graph capture end: %s", hipGetErrorString(e2));
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) { *out = nullptr; return fail(FF_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e)); }
    return FF_OK;
}

ff_status ff_minimize(ff_ctx* c, double* xyz, const ff_min_params* p, ff_min_result* res, void* stream) {
    clear_error();
    if (!c || !xyz || !p || !res) return fail(FF_ERR_ARG, "null argument");
    if (p->method < FF_GD || p->method > FF_OGM) return fail(FF_ERR_ARG, "bad method %d", p->method);
    if (p->method == FF_HB && !(p->hb_alpha > 0.0 && std::isfinite(p->hb_alpha) && p->hb_beta >= 0.0 &&
                                p->hb_beta < 1.0))
        return fail(FF_ERR_ARG, "heavy ball needs hb_alpha > 0 and 0 <= hb_beta < 1");
    if (p->method == FF_LBFGS && (p->m < 1 || p->m > c->L.m_max))
        return fail(FF_ERR_ARG, "m = %d outside [1, m_max = %d]", p->m, c->L.m_max);
    if (!(p->tol > 0.0)) return fail(FF_ERR_ARG, "tol must be > 0");
    if (p->max_iter < 0) return fail(FF_ERR_ARG, "max_iter must be >= 0");
    if (p->precision != FF_FP64 && p->precision != FF_FP32_ACC64) return fail(FF_ERR_ARG, "bad precision");
    if (p->linesearch < -1 || p->linesearch > 1) return fail(FF_ERR_ARG, "bad line search");
    if (p->ls_K < 2 || p->ls_K > kMaxLsTrials) return fail(FF_ERR_ARG, "ls_K must be in [2, %d]", kMaxLsTrials);
    if (!(p->h_init > 0.0) || !(p->k_plus > 1.0) || !(p->k_minus > 0.0 && p->k_minus < 1.0) || !(p->eps_h > 0.0))
        return fail(FF_ERR_ARG, "bad line-search constants");
    if (p->cg_restart < 0) return fail(FF_ERR_ARG, "cg_restart must be >= 0");
    if (p->cg_beta < FF_CG_PRP || p->cg_beta > FF_CG_DY) return fail(FF_ERR_ARG, "bad cg_beta %d", p->cg_beta);
    if (p->ls_par_g0 != 0 && p->ls_par_g0 != 1) return fail(FF_ERR_ARG, "ls_par_g0 must be 0 or 1");
    if (p->fgm_restart != 0 && p->fgm_restart != 1) return fail(FF_ERR_ARG, "fgm_restart must be 0 or 1");
    const bool resume = (p->flags & FF_MIN_RESUME) != 0;
    if (resume && (c->last_method != p->method || c->last_m != p->m || c->last_prec != p->precision))
        return fail(FF_ERR_ARG, "resume needs the same method, m and precision as the previous call");
    // a HIP graph cannot be captured on the NULL stream: such calls run on the
    // context's own (blocking) stream, which orders itself after NULL-stream work
    hipStream_t st = stream ? (hipStream_t)stream : c->own;
    const Layout& L = c->L;
    Args a{};
    a.L = L;
    a.ws = c->ws;
    MinParamsDev d{};
    d.method = p->method;
    d.m = p->method == FF_LBFGS ? p->m : 0;
    d.max_iter = p->max_iter;
    d.precision = p->precision;
    d.linesearch = p->linesearch;
    d.ls_K = p->ls_K;
    d.cg_restart = p->cg_restart;     // 0: 3N of each system (set per system on the device)
    d.certify = (p->flags & FF_MIN_NO_CERTIFY) ? 0 : 1;
    d.cg_beta = p->cg_beta;
    d.ls_g0 = p->ls_par_g0;
    d.fgm_restart = p->fgm_restart;
    d.tol = p->tol;
    d.h_init = p->h_init;
    d.k_plus = p->k_plus;
    d.k_minus = p->k_minus;
    d.eps_h = p->eps_h;
    d.hb_alpha = p->hb_alpha;
    d.hb_beta = p->hb_beta;
    double* x0 = at<double>(c->ws, L.off_vec) + (size_t)V_X0 * L.vstride;
    if (!resume)
        for (int k = 0; k < L.n_sys; ++k)
            HIP_TRY(hipMemcpyAsync(x0 + 3 * (size_t)c->sys[k].aoff, xyz + 3 * (size_t)c->sys[k].uoff,
                                   3 * (size_t)c->sys[k].n * 8, hipMemcpyDeviceToDevice, st));
    HIP_TRY(launch_kick(a, d, resume ? 1 : 0, trace_buffer(c), kTraceCap, st));
    if (!c->graph64) {
        ff_status gs = build_graph(c, false, &c->graph64);
        if (gs) return gs;
    }
    if (p->precision == FF_FP32_ACC64 && !c->graph) {
        ff_status gs = build_graph(c, true, &c->graph);
        if (gs) return gs;
    }
    // FP32 mode runs the graph with both pair kernels until every unfinished
    // system has switched to FP64 evaluations (the poll reports it); a
    // resumed run may already be there
    hipGraphExec_t graph = p->precision == FF_FP32_ACC64 ? c->graph : c->graph64;
    c->last_method = p->method;
    c->last_m = p->m;
    c->last_prec = p->precision;
    // poll (n_done, evals) of the batch
    const char* dev_state = c->ws + L.off_batch;
    uint32_t* hs = (uint32_t*)c->host_flag;
    int batch = 1;              // graph launches (kCyclesPerGraph cycles each) between polls
    uint32_t last_evals = 0xffffffffu;
    for (;;) {
        for (int k = 0; k < batch; ++k) HIP_TRY(hipGraphLaunch(graph, st));
        HIP_TRY(hipMemcpyAsync(hs, dev_state, sizeof(BatchState), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if ((int)hs[0] >= L.n_sys) break;
        if (hs[2] >= (uint32_t)L.n_sys) graph = c->graph64;
        // every cycle that is not only an accept pass evaluates; a batch of
        // cycles without a new evaluation means the decision logic stopped
        if (hs[1] == last_evals) return fail(FF_ERR_HIP, "minimizer stalled (%u of %d systems done)", hs[0], L.n_sys);
        last_evals = hs[1];
        batch = std::min(batch * 2, 64 / kCyclesPerGraph);
    }
    for (int k = 0; k < L.n_sys; ++k) {
        const SysInfo& si = c->sys[k];
        HIP_TRY(hipMemcpyAsync(c->host_ctl, c->ws + L.off_ctl + (size_t)k * L.ctl_stride, sizeof(Ctl),
                               hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        const Ctl& h = *c->host_ctl;
        const int slot = h.result_slot;
        double* xr = at<double>(c->ws, L.off_vec) + (size_t)(V_X0 + slot) * L.vstride + 3 * (size_t)si.aoff;
        HIP_TRY(hipMemcpyAsync(xyz + 3 * (size_t)si.uoff, xr, 3 * (size_t)si.n * 8, hipMemcpyDeviceToDevice, st));
        ff_min_result& r = res[k];
        r.term = h.term;
        r.iters = h.iters - h.iters_base;
        r.evals = h.evals;
        r.evals_fp64 = h.evals64;
        r.energy = h.e[slot];
        r.grad_inf = h.ginf[slot];
        r.grad_2 = std::sqrt(h.g2[slot]);
    }
    HIP_TRY(hipStreamSynchronize(st));
    return FF_OK;
}

// Energy along the unit antigradient of each system at xyz (section 3's
// non-convexity profile): one evaluation at xyz, then one per step length.
ff_status ff_energy_profile(ff_ctx* c, const double* xyz, const double* t, int32_t n_t, double* e_out,
                            int32_t precision, void* stream) {
    clear_error();
    if (!c || !xyz || !t || !e_out) return fail(FF_ERR_ARG, "null argument");
    if (n_t < 1 || n_t > kMaxProfile) return fail(FF_ERR_ARG, "n_t must be in [1, %d]", kMaxProfile);
    if (precision != FF_FP64 && precision != FF_FP32_ACC64) return fail(FF_ERR_ARG, "bad precision %d", precision);
    for (int k = 0; k < n_t; ++k)
        if (!std::isfinite(t[k])) return fail(FF_ERR_ARG, "t[%d] is not finite", k);
    hipStream_t st = stream ? (hipStream_t)stream : c->own;
    const Layout& L = c->L;
    // scratch in the optimizer's vector region: g, x_t ([n][3] each), |g|^2
    // and the energies ([n_sys] per point)
    double* base = at<double>(c->ws, L.off_vec);
    const size_t n3 = 3 * (size_t)L.n;
    double* g = base;
    double* xt = base + n3;
    double* g2 = base + 2 * n3;
    double* e = g2 + L.n_sys;
    Args a{};
    a.L = L;
    a.ws = c->ws;
    a.direct = 1;
    a.direct_prec = precision;
    a.xyz_in = xyz;
    a.e_out = e;                 // scratch for E(x) itself
    a.g_out = g;
    a.g2_out = g2;
    HIP_TRY(launch_bonded(a, st));
    HIP_TRY(launch_pair(a, precision, st));
    HIP_TRY(launch_finalize(a, st));
    a.xyz_in = xt;
    a.g_out = nullptr;
    a.g2_out = nullptr;
    for (int k = 0; k < n_t; ++k) {
        a.e_out = e + (size_t)(k + 1) * L.n_sys;
        HIP_TRY(launch_profile_point(a, xyz, g, g2, t[k], xt, st));
        HIP_TRY(launch_bonded(a, st));
        HIP_TRY(launch_pair(a, precision, st));
        HIP_TRY(launch_finalize(a, st));
    }
    HIP_TRY(hipMemcpyAsync(e_out, e + L.n_sys, (size_t)n_t * L.n_sys * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    c->last_method = -1;         // the vectors a resumed minimization needs are gone
    return FF_OK;
}

// Average duration (ms) of `reps` back-to-back launches of the pair kernel
// alone at xyz (all systems), timed with HIP events recorded on the launch stream.
ff_status ff_time_pair(ff_ctx* c, const double* xyz, int32_t precision, int32_t reps, void* stream,
                       double* avg_ms) {
    clear_error();
    if (!c || !xyz || !avg_ms || reps < 1) return fail(FF_ERR_ARG, "bad arguments");
    if (precision != FF_FP64 && precision != FF_FP32_ACC64) return fail(FF_ERR_ARG, "bad precision");
    hipStream_t st = stream ? (hipStream_t)stream : c->own;
    Args a{};
    a.L = c->L;
    a.ws = c->ws;
    a.xyz_in = xyz;
    a.direct = 1;
    a.direct_prec = precision;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return fail(FF_ERR_HIP, "event"); }
    hipError_t e = launch_pair(a, precision, st);   // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_pair(a, precision, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(FF_ERR_HIP, "pair timing: %s", hipGetErrorString(e));
    *avg_ms = (double)ms / reps;
    return FF_OK;
}

// Per-iteration trace of the last ff_minimize call (system 0): out[3k..3k+2]
// = (E after iteration k, accepted step h, evaluations so far).  Returns the
// number of entries written (at most max_entries), or a negative ff_status.
int32_t ff_get_trace(ff_ctx* c, double* host_out, int32_t max_entries, void* stream) {
    if (!c || !host_out || max_entries < 0) return fail(FF_ERR_ARG, "bad arguments");
    stream = stream ? stream : (void*)c->own;
    hipStream_t st = (hipStream_t)stream;
    int32_t n = 0;
    if (hipMemcpyAsync(&n, c->ws + c->L.off_ctl + offsetof(Ctl, n_trace), 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(FF_ERR_HIP, "trace count copy failed");
    n = std::min(n, max_entries);
    if (n > 0 && (hipMemcpyAsync(host_out, trace_buffer(c), 3 * (size_t)n * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
                  hipStreamSynchronize(st) != hipSuccess))
        return fail(FF_ERR_HIP, "trace copy failed");
    return n;
}

}  // extern "C"
