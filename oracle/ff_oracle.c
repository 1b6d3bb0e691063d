/*
 * Oracle: plain FP64 CPU evaluation of the force-field energy and gradient.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links or calls
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no code with the HIP library.
 *
 * What it computes is the energy of section 2 of the paper, written out term
 * by term, in double precision, with no tiling, no reordering and no
 * precision tricks:
 *
 *   E = sum_bonds     K (r - r0)^2                          (stretch, section 2)
 *     + sum_angles    K_theta (theta - theta0)^2            (bend, section 2)
 *     + sum_dihedrals 1/2 [V1 (1 + cos phi) + V2 (1 - cos 2phi)
 *                          + V3 (1 + cos 3phi) + V4 (1 - cos 4phi)]   (torsion)
 *     + sum_{i<j, not excluded} C q_i q_j / r_ij            (Coulomb)
 *     + sum_{i<j, not excluded} 4 sqrt(eps_i eps_j)
 *           [ (sqrt(sig_i sig_j)/r_ij)^12 - (sqrt(sig_i sig_j)/r_ij)^6 ]  (Lennard-Jones,
 *                                                 geometric mixing as in section 2)
 *
 * Readings where the paper is silent:
 *  - excluded pairs are exactly the 1-2 pairs (bonds) and 1-3 pairs (the two
 *    outer atoms of each angle); 1-4 pairs interact at full strength;
 *  - no cutoff: every non-excluded pair interacts;
 *  - the angle is theta = atan2(|u x v|, u . v) with u, v the bond vectors out
 *    of the vertex (the middle atom of the triple);
 *  - the dihedral uses the IUPAC convention (cis = 0, trans = pi).
 *
 * The gradient is the analytic derivative of each term (section 2 prefers
 * explicit formulas to automatic differentiation).  Nonbonded: every row i
 * loops over all j (each pair is visited twice, no force scatter), so the
 * OpenMP loop over rows writes disjoint output and is deterministic for any
 * thread count; the energy counts only j > i and the row energies are summed
 * in index order afterwards.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t n_atoms;
    const double *q, *sigma, *eps;
    int32_t n_bonds;
    const int32_t *bond;        /* [n_bonds][2] */
    const double *bond_k, *bond_r0;
    int32_t n_angles;
    const int32_t *angle;       /* [n_angles][3], vertex in the middle */
    const double *angle_k, *angle_t0;
    int32_t n_dihedrals;
    const int32_t *dihedral;    /* [n_dihedrals][4] */
    const double *dihedral_v;   /* [n_dihedrals][4] = V1..V4 */
    double coulomb_c;
} oracle_system;

enum { T_STRETCH = 0, T_BEND = 1, T_TORSION = 2, T_COULOMB = 3, T_VDW = 4 };

/* Exclusion lists: for every atom the (unsorted) list of atoms it must not
 * interact with, in compressed-row form. */
typedef struct {
    int32_t *start; /* [n+1] */
    int32_t *list;
} excl_t;

static int in_range(int32_t a, int32_t n) { return a >= 0 && a < n; }

static int build_exclusions(const oracle_system *s, excl_t *ex)
{
    int32_t n = s->n_atoms;
    int32_t *count = calloc((size_t)n + 1, sizeof(int32_t));
    if (!count) return -2;
    for (int32_t b = 0; b < s->n_bonds; ++b) {
        int32_t i = s->bond[2 * b], j = s->bond[2 * b + 1];
        count[i]++; count[j]++;
    }
    for (int32_t a = 0; a < s->n_angles; ++a) {
        int32_t i = s->angle[3 * a], k = s->angle[3 * a + 2];
        count[i]++; count[k]++;
    }
    ex->start = malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t total = 0;
    for (int32_t i = 0; i < n; ++i) { ex->start[i] = total; total += count[i]; }
    ex->start[n] = total;
    ex->list = malloc((size_t)(total > 0 ? total : 1) * sizeof(int32_t));
    memset(count, 0, ((size_t)n + 1) * sizeof(int32_t));
    for (int32_t b = 0; b < s->n_bonds; ++b) {
        int32_t i = s->bond[2 * b], j = s->bond[2 * b + 1];
        ex->list[ex->start[i] + count[i]++] = j;
        ex->list[ex->start[j] + count[j]++] = i;
    }
    for (int32_t a = 0; a < s->n_angles; ++a) {
        int32_t i = s->angle[3 * a], k = s->angle[3 * a + 2];
        ex->list[ex->start[i] + count[i]++] = k;
        ex->list[ex->start[k] + count[k]++] = i;
    }
    free(count);
    return 0;
}

static void free_exclusions(excl_t *ex) { free(ex->start); free(ex->list); }

static int excluded(const excl_t *ex, int32_t i, int32_t j)
{
    for (int32_t p = ex->start[i]; p < ex->start[i + 1]; ++p)
        if (ex->list[p] == j) return 1;
    return 0;
}

static int validate(const oracle_system *s)
{
    int32_t n = s->n_atoms;
    if (n < 1) return -1;
    for (int32_t b = 0; b < s->n_bonds; ++b)
        if (!in_range(s->bond[2 * b], n) || !in_range(s->bond[2 * b + 1], n) ||
            s->bond[2 * b] == s->bond[2 * b + 1]) return -1;
    for (int32_t a = 0; a < s->n_angles; ++a)
        for (int c = 0; c < 3; ++c) if (!in_range(s->angle[3 * a + c], n)) return -1;
    for (int32_t d = 0; d < s->n_dihedrals; ++d)
        for (int c = 0; c < 4; ++c) if (!in_range(s->dihedral[4 * d + c], n)) return -1;
    return 0;
}

/* ---- nonbonded pair: energy parts and dE/dr ---------------------------- */
static void pair_terms(const oracle_system *s, int32_t i, int32_t j, double r,
                       double *e_coul, double *e_vdw, double *de_dr)
{
    double c = s->coulomb_c * s->q[i] * s->q[j];
    double sig = sqrt(s->sigma[i] * s->sigma[j]);
    double eps = sqrt(s->eps[i] * s->eps[j]);
    double sr = sig / r;
    double sr6 = sr * sr * sr * sr * sr * sr;
    double sr12 = sr6 * sr6;
    *e_coul = c / r;
    *e_vdw = 4.0 * eps * (sr12 - sr6);
    /* d/dr of C q q / r and of 4 eps (s^12 r^-12 - s^6 r^-6) */
    *de_dr = -c / (r * r) + 4.0 * eps * (-12.0 * sr12 + 6.0 * sr6) / r;
}

/* Nonbonded row of atom i: gradient of atom i (all j) and, if want_energy,
 * the energy of pairs (i, j > i). */
static void nonbonded_row(const oracle_system *s, const excl_t *ex, const double *x,
                          int32_t i, double *gi, double *e_coul, double *e_vdw)
{
    double gx = 0, gy = 0, gz = 0, ec = 0, ev = 0;
    for (int32_t j = 0; j < s->n_atoms; ++j) {
        if (j == i || excluded(ex, i, j)) continue;
        double dx = x[3 * i] - x[3 * j];
        double dy = x[3 * i + 1] - x[3 * j + 1];
        double dz = x[3 * i + 2] - x[3 * j + 2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        double c, v, d;
        pair_terms(s, i, j, r, &c, &v, &d);
        gx += d * dx / r; gy += d * dy / r; gz += d * dz / r;
        if (j > i) { ec += c; ev += v; }
    }
    if (gi) { gi[0] = gx; gi[1] = gy; gi[2] = gz; }
    *e_coul = ec; *e_vdw = ev;
}

static void nonbonded_row_energy(const oracle_system *s, const excl_t *ex, const double *x,
                                 int32_t i, double *e_coul, double *e_vdw)
{
    double ec = 0, ev = 0;
    for (int32_t j = i + 1; j < s->n_atoms; ++j) {
        if (excluded(ex, i, j)) continue;
        double dx = x[3 * i] - x[3 * j];
        double dy = x[3 * i + 1] - x[3 * j + 1];
        double dz = x[3 * i + 2] - x[3 * j + 2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        double c, v, d;
        pair_terms(s, i, j, r, &c, &v, &d);
        ec += c; ev += v;
    }
    *e_coul = ec; *e_vdw = ev;
}

/* ---- bonded terms: energy of term t and its gradient on its atoms ------ */
static double bond_term(const oracle_system *s, const double *x, int32_t b, double g[2][3])
{
    int32_t i = s->bond[2 * b], j = s->bond[2 * b + 1];
    double d[3], r = 0;
    for (int c = 0; c < 3; ++c) { d[c] = x[3 * i + c] - x[3 * j + c]; r += d[c] * d[c]; }
    r = sqrt(r);
    double dr = r - s->bond_r0[b];
    double de_dr = 2.0 * s->bond_k[b] * dr;
    for (int c = 0; c < 3; ++c) { g[0][c] = de_dr * d[c] / r; g[1][c] = -g[0][c]; }
    return s->bond_k[b] * dr * dr;
}

static double angle_term(const oracle_system *s, const double *x, int32_t a, double g[3][3])
{
    int32_t i = s->angle[3 * a], j = s->angle[3 * a + 1], k = s->angle[3 * a + 2];
    double u[3], v[3], nu = 0, nv = 0, uv = 0;
    for (int c = 0; c < 3; ++c) {
        u[c] = x[3 * i + c] - x[3 * j + c];
        v[c] = x[3 * k + c] - x[3 * j + c];
        nu += u[c] * u[c]; nv += v[c] * v[c]; uv += u[c] * v[c];
    }
    nu = sqrt(nu); nv = sqrt(nv);
    double cr[3] = { u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0] };
    double ncr = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    double theta = atan2(ncr, uv);
    double dth = theta - s->angle_t0[a];
    double de_dth = 2.0 * s->angle_k[a] * dth;
    double cost = cos(theta), sint = sin(theta);
    for (int c = 0; c < 3; ++c) {
        double uh = u[c] / nu, vh = v[c] / nv;
        /* d theta / d x_i = -(v^ - cos(theta) u^) / (|u| sin(theta)), same for k with u <-> v */
        double dti = -(vh - cost * uh) / (nu * sint);
        double dtk = -(uh - cost * vh) / (nv * sint);
        g[0][c] = de_dth * dti;
        g[2][c] = de_dth * dtk;
        g[1][c] = -(g[0][c] + g[2][c]);
    }
    return s->angle_k[a] * dth * dth;
}

static void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static double dihedral_angle(const double *x, const int32_t *at, double b1[3], double b2[3],
                             double b3[3], double n1[3], double n2[3])
{
    for (int c = 0; c < 3; ++c) {
        b1[c] = x[3 * at[1] + c] - x[3 * at[0] + c];
        b2[c] = x[3 * at[2] + c] - x[3 * at[1] + c];
        b3[c] = x[3 * at[3] + c] - x[3 * at[2] + c];
    }
    cross3(b1, b2, n1);
    cross3(b2, b3, n2);
    double nb2 = sqrt(dot3(b2, b2));
    return atan2(nb2 * dot3(b1, n2), dot3(n1, n2));
}

static double torsion_term(const oracle_system *s, const double *x, int32_t d, double g[4][3])
{
    const int32_t *at = &s->dihedral[4 * d];
    const double *V = &s->dihedral_v[4 * d];
    double b1[3], b2[3], b3[3], n1[3], n2[3];
    double phi = dihedral_angle(x, at, b1, b2, b3, n1, n2);
    double e = 0.5 * (V[0] * (1 + cos(phi)) + V[1] * (1 - cos(2 * phi)) +
                      V[2] * (1 + cos(3 * phi)) + V[3] * (1 - cos(4 * phi)));
    double de_dphi = 0.5 * (-V[0] * sin(phi) + 2 * V[1] * sin(2 * phi) -
                            3 * V[2] * sin(3 * phi) + 4 * V[3] * sin(4 * phi));
    /* Singularity-free dihedral derivatives (Blondel and Karplus 1996). */
    double nb2sq = dot3(b2, b2), nb2 = sqrt(nb2sq);
    double n1sq = dot3(n1, n1), n2sq = dot3(n2, n2);
    double f1 = dot3(b1, b2) / nb2sq, f3 = dot3(b3, b2) / nb2sq;
    for (int c = 0; c < 3; ++c) {
        double da = -nb2 / n1sq * n1[c];
        double dd = nb2 / n2sq * n2[c];
        double db = -(1.0 + f1) * da + f3 * dd;
        double dc = f1 * da - (1.0 + f3) * dd;
        g[0][c] = de_dphi * da;
        g[1][c] = de_dphi * db;
        g[2][c] = de_dphi * dc;
        g[3][c] = de_dphi * dd;
    }
    return e;
}

/* ---- public entry points ------------------------------------------------ */

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following calls from this thread (timing on fewer cores). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Energy terms [stretch, bend, torsion, coulomb, vdw] at x ([N][3]), and the
 * gradient ([N][3]) if grad != NULL.  Returns 0, -1 on a bad index or size,
 * -2 on allocation failure. */
int oracle_energy_grad(const oracle_system *s, const double *x, double *terms, double *grad)
{
    if (validate(s)) return -1;
    excl_t ex;
    if (build_exclusions(s, &ex)) return -2;
    int32_t n = s->n_atoms;
    double *row_c = calloc((size_t)n, sizeof(double));
    double *row_v = calloc((size_t)n, sizeof(double));

    #pragma omp parallel for schedule(dynamic, 16)
    for (int32_t i = 0; i < n; ++i) {
        if (grad) nonbonded_row(s, &ex, x, i, &grad[3 * i], &row_c[i], &row_v[i]);
        else nonbonded_row_energy(s, &ex, x, i, &row_c[i], &row_v[i]);
    }
    double ec = 0, ev = 0;
    for (int32_t i = 0; i < n; ++i) { ec += row_c[i]; ev += row_v[i]; }
    free(row_c); free(row_v);

    double es = 0, eb = 0, et = 0;
    for (int32_t b = 0; b < s->n_bonds; ++b) {
        double g[2][3];
        es += bond_term(s, x, b, g);
        if (grad) for (int p = 0; p < 2; ++p) for (int c = 0; c < 3; ++c)
            grad[3 * s->bond[2 * b + p] + c] += g[p][c];
    }
    for (int32_t a = 0; a < s->n_angles; ++a) {
        double g[3][3];
        eb += angle_term(s, x, a, g);
        if (grad) for (int p = 0; p < 3; ++p) for (int c = 0; c < 3; ++c)
            grad[3 * s->angle[3 * a + p] + c] += g[p][c];
    }
    for (int32_t d = 0; d < s->n_dihedrals; ++d) {
        double g[4][3];
        et += torsion_term(s, x, d, g);
        if (grad) for (int p = 0; p < 4; ++p) for (int c = 0; c < 3; ++c)
            grad[3 * s->dihedral[4 * d + p] + c] += g[p][c];
    }
    terms[T_STRETCH] = es; terms[T_BEND] = eb; terms[T_TORSION] = et;
    terms[T_COULOMB] = ec; terms[T_VDW] = ev;
    free_exclusions(&ex);
    return 0;
}

/* Scale of the rounding error of atom i's nonbonded gradient: out[i] =
 * sum over non-excluded j of |dE_ij/dr| (the magnitudes of the pair forces
 * that are summed into atom i's gradient; Coulomb and Lennard-Jones parts
 * added as magnitudes).  Test-side only: tolerances of reduced-precision
 * sums are stated as multiples of it. */
int oracle_abs_pair_force(const oracle_system *s, const double *x, double *out)
{
    if (validate(s)) return -1;
    excl_t ex;
    if (build_exclusions(s, &ex)) return -2;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int32_t i = 0; i < s->n_atoms; ++i) {
        double acc = 0.0;
        for (int32_t j = 0; j < s->n_atoms; ++j) {
            if (j == i || excluded(&ex, i, j)) continue;
            double dx = x[3 * i] - x[3 * j];
            double dy = x[3 * i + 1] - x[3 * j + 1];
            double dz = x[3 * i + 2] - x[3 * j + 2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double c = s->coulomb_c * s->q[i] * s->q[j];
            double sig = sqrt(s->sigma[i] * s->sigma[j]);
            double eps = sqrt(s->eps[i] * s->eps[j]);
            double sr = sig / r;
            double sr6 = sr * sr * sr * sr * sr * sr;
            acc += fabs(c) / (r * r) + 4.0 * eps * (12.0 * sr6 * sr6 + 6.0 * sr6) / r;
        }
        out[i] = acc;
    }
    free_exclusions(&ex);
    return 0;
}

/* Gradient of the listed atoms only (out: [count][3]); O(N) per atom, for
 * spot checks of large systems. */
int oracle_atom_gradients(const oracle_system *s, const double *x, const int32_t *atoms,
                          int32_t count, double *out)
{
    if (validate(s)) return -1;
    for (int32_t t = 0; t < count; ++t) if (!in_range(atoms[t], s->n_atoms)) return -1;
    excl_t ex;
    if (build_exclusions(s, &ex)) return -2;
    #pragma omp parallel for schedule(static)
    for (int32_t t = 0; t < count; ++t) {
        int32_t i = atoms[t];
        double ec, ev, *gi = &out[3 * t];
        nonbonded_row(s, &ex, x, i, gi, &ec, &ev);
        for (int32_t b = 0; b < s->n_bonds; ++b) {
            for (int p = 0; p < 2; ++p) if (s->bond[2 * b + p] == i) {
                double g[2][3];
                bond_term(s, x, b, g);
                for (int c = 0; c < 3; ++c) gi[c] += g[p][c];
            }
        }
        for (int32_t a = 0; a < s->n_angles; ++a) {
            for (int p = 0; p < 3; ++p) if (s->angle[3 * a + p] == i) {
                double g[3][3];
                angle_term(s, x, a, g);
                for (int c = 0; c < 3; ++c) gi[c] += g[p][c];
            }
        }
        for (int32_t d = 0; d < s->n_dihedrals; ++d) {
            for (int p = 0; p < 4; ++p) if (s->dihedral[4 * d + p] == i) {
                double g[4][3];
                torsion_term(s, x, d, g);
                for (int c = 0; c < 3; ++c) gi[c] += g[p][c];
            }
        }
    }
    free_exclusions(&ex);
    return 0;
}
