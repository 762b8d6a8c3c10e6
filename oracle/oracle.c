/*
 * Plain FP64 CPU oracle of the biased neutron history loop.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  It shares no code
 * with the GPU library.  Every function below follows the passage of the paper
 * named in its comment; where the paper is silent the reading taken is stated.
 *
 * Deliberately slow and simple: every random draw recomputes its Philox block,
 * every step recomputes the cross sections, geometry is intersected solid by
 * solid with the textbook formulas.
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Random numbers                                                            */
/* ------------------------------------------------------------------------ */

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11): each round
 * multiplies counter words 0 and 2 by two odd constants, forms the new counter
 * from the high/low product halves xored with the other words and the key,
 * and the key is bumped by two Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Draw k of history h: block k/2 with counter (block, history) and key = seed;
 * even draws take words 0,1, odd draws words 2,3; the two words make a 53-bit
 * uniform in [0,1). */
double orc_uniform(uint64_t seed, uint64_t history, uint32_t draw)
{
    uint64_t block = draw >> 1;
    uint32_t ctr[4] = {(uint32_t)block, (uint32_t)(block >> 32), (uint32_t)history, (uint32_t)(history >> 32)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    uint32_t a = (draw & 1) ? w[2] : w[0];
    uint32_t b = (draw & 1) ? w[3] : w[1];
    double hi = (double)(a >> 5);   /* 27 bits */
    double lo = (double)(b >> 6);   /* 26 bits */
    return (hi * 67108864.0 + lo) * (1.0 / 9007199254740992.0);
}

typedef struct {
    uint64_t seed, history;
    uint32_t k;
} rng_t;

static double next_u(rng_t* r) { return orc_uniform(r->seed, r->history, r->k++); }

/* ------------------------------------------------------------------------ */
/* Units                                                                     */
/* ------------------------------------------------------------------------ */

/* E = h^2 / (2 m_n lambda^2), with CODATA 2018 constants. */
double orc_ev_from_angstrom(double lambda)
{
    const double h = 6.62607015e-34;          /* J s */
    const double mn = 1.67492749804e-27;      /* kg */
    const double ev = 1.602176634e-19;        /* J */
    double c = h * h / (2.0 * mn) / ev * 1e20; /* eV A^2 */
    return c / (lambda * lambda);
}

static double angstrom_from_ev(double e)
{
    double c = orc_ev_from_angstrom(1.0);
    return sqrt(c / e);
}

/* ------------------------------------------------------------------------ */
/* Cross sections (neutron scattering cross section section)                 */
/* ------------------------------------------------------------------------ */

/* Macroscopic cross sections in 1/mm at wavelength lambda:
 *   out[0] absorption  n sigma_abs_ref lambda / 1.798       (1/v law)
 *   out[1] incoherent  n sigma_inc                          (bound, isotropic)
 *   out[2] coherent    n lambda^2/(2 v0 N) sum_{2d>lambda} m d |F|^2
 *          (powder average of the coherent elastic scattering function: the
 *           delta on Q = tau contributes when tau < 2k, i.e. 2d > lambda)
 *   out[3] number of active Bragg families.
 * n in 1/A^3 times sigma in barn (1e-8 A^2) gives 1/A; times 1e7 gives 1/mm. */
/* linear interpolation in a table of rows (x_i, y_i), x increasing, constant
 * beyond the first and last rows */
static double table_interp(int n, const double* x, const double* y, double v)
{
    if (v <= x[0]) return y[0];
    if (v >= x[n - 1]) return y[n - 1];
    int i = 0;
    while (x[i + 1] < v) ++i;
    return y[i] + (y[i + 1] - y[i]) * (v - x[i]) / (x[i + 1] - x[i]);
}

void orc_macro_xs(const orc_material* m, double lambda, double out[4])
{
    const double barn_per_A3_to_per_mm = 1e-8 * 1e7;
    double sa = m->sigma_abs_ref * lambda / 1.798;
    double si = m->sigma_inc;
    if (m->n_table >= 2) {
        /* tabulated cross sections replace the 1/v law and the constant sigma_inc */
        sa = table_interp(m->n_table, m->table_lambda, m->table_sigma_abs, lambda);
        si = table_interp(m->n_table, m->table_lambda, m->table_sigma_inc, lambda);
    }
    double sum = 0.0;
    int active = 0;
    for (int j = 0; j < m->n_families; ++j) {
        if (2.0 * m->d[j] > lambda) {
            sum += m->mult[j] * m->d[j] * m->f2[j];
            active++;
        }
    }
    double sc = 0.0;
    if (m->cell_volume > 0.0 && m->atoms_per_cell > 0)
        sc = lambda * lambda / (2.0 * m->cell_volume * m->atoms_per_cell) * sum;
    out[0] = m->number_density * sa * barn_per_A3_to_per_mm;
    out[1] = m->number_density * si * barn_per_A3_to_per_mm;
    out[2] = m->number_density * sc * barn_per_A3_to_per_mm;
    out[3] = (double)active;
}

/* ------------------------------------------------------------------------ */
/* Geometry                                                                  */
/* ------------------------------------------------------------------------ */

/* Face ids. box: 0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z.
 * cylinder / shell: 0 outer lateral, 1 low cap, 2 high cap, 3 inner lateral.
 * sphere / shell: 0 outer, 3 inner. */

typedef struct {
    double a, b;
    int fa, fb;
    int empty;
} ival;

static ival ival_all(void) { ival r = {-INFINITY, INFINITY, -1, -1, 0}; return r; }
static ival ival_none(void) { ival r = {0, 0, -1, -1, 1}; return r; }

static ival ival_and(ival x, ival y)
{
    if (x.empty || y.empty) return ival_none();
    ival r;
    if (x.a >= y.a) { r.a = x.a; r.fa = x.fa; } else { r.a = y.a; r.fa = y.fa; }
    if (x.b <= y.b) { r.b = x.b; r.fb = x.fb; } else { r.b = y.b; r.fb = y.fb; }
    r.empty = !(r.a <= r.b);
    return r;
}

/* the set of t with lo <= p + t u <= hi along one coordinate */
static ival slab(double p, double u, double lo, double hi, int face_lo, int face_hi)
{
    if (u == 0.0) return (p >= lo && p <= hi) ? ival_all() : ival_none();
    double t1 = (lo - p) / u, t2 = (hi - p) / u;
    ival r;
    if (u > 0) { r.a = t1; r.fa = face_lo; r.b = t2; r.fb = face_hi; }
    else { r.a = t2; r.fa = face_hi; r.b = t1; r.fb = face_lo; }
    r.empty = 0;
    return r;
}

/* the set of t with |q_perp + t u_perp| <= r (infinite cylinder) */
static ival radial(double qb, double qc, double ub, double uc, double r, int face)
{
    double A = ub * ub + uc * uc;
    double B = qb * ub + qc * uc;
    double C = qb * qb + qc * qc - r * r;
    if (A == 0.0) return (C <= 0.0) ? ival_all() : ival_none();
    double disc = B * B - A * C;
    if (disc < 0.0) return ival_none();
    double s = sqrt(disc);
    ival res = {(-B - s) / A, (-B + s) / A, face, face, 0};
    return res;
}

static ival ball(const double q[3], const double u[3], double r, int face)
{
    double A = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double B = q[0] * u[0] + q[1] * u[1] + q[2] * u[2];
    double C = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] - r * r;
    double disc = B * B - A * C;
    if (disc < 0.0) return ival_none();
    double s = sqrt(disc);
    ival res = {(-B - s) / A, (-B + s) / A, face, face, 0};
    return res;
}

static ival cylinder_ival(const double q[3], const double u[3], int axis, double r, double h, int lateral_face)
{
    int b = (axis + 1) % 3, c = (axis + 2) % 3;
    ival rad = radial(q[b], q[c], u[b], u[c], r, lateral_face);
    ival ax = slab(q[axis], u[axis], -0.5 * h, 0.5 * h, 1, 2);
    return ival_and(rad, ax);
}

/* outer minus inner: up to two pieces, zero-length pieces dropped */
static int subtract(ival o, ival in, ival out[2])
{
    if (o.empty) return 0;
    if (in.empty || in.b <= o.a || in.a >= o.b) { out[0] = o; return 1; }
    int n = 0;
    if (in.a > o.a) { ival r = {o.a, in.a, o.fa, in.fa, 0}; out[n++] = r; }
    if (in.b < o.b) { ival r = {in.b, o.b, in.fb, o.fb, 0}; out[n++] = r; }
    return n;
}

static int solid_ivals(const orc_volume* v, const double p[3], const double u[3], ival out[2])
{
    double q[3] = {p[0] - v->center[0], p[1] - v->center[1], p[2] - v->center[2]};
    switch (v->kind) {
    case ORC_BOX: {
        ival r = ival_all();
        for (int k = 0; k < 3; ++k)
            r = ival_and(r, slab(q[k], u[k], -0.5 * v->size[k], 0.5 * v->size[k], 2 * k, 2 * k + 1));
        if (r.empty) return 0;
        out[0] = r;
        return 1;
    }
    case ORC_CYLINDER: {
        ival r = cylinder_ival(q, u, v->axis, v->size[0], v->size[1], 0);
        if (r.empty) return 0;
        out[0] = r;
        return 1;
    }
    case ORC_CYL_SHELL: {
        ival o = cylinder_ival(q, u, v->axis, v->size[1], v->size[2], 0);
        ival in = cylinder_ival(q, u, v->axis, v->size[0], v->size[2], 3);
        return subtract(o, in, out);
    }
    case ORC_SPHERE: {
        ival r = ball(q, u, v->size[0], 0);
        if (r.empty) return 0;
        out[0] = r;
        return 1;
    }
    case ORC_SPH_SHELL: {
        ival o = ball(q, u, v->size[1], 0);
        ival in = ball(q, u, v->size[0], 3);
        return subtract(o, in, out);
    }
    }
    return 0;
}

int orc_intervals(const orc_volume* v, const double p[3], const double u[3],
                  double t_in[2], double t_out[2], int32_t face_in[2], int32_t face_out[2])
{
    ival iv[2];
    int n = solid_ivals(v, p, u, iv);
    for (int i = 0; i < n; ++i) {
        t_in[i] = iv[i].a; t_out[i] = iv[i].b;
        face_in[i] = iv[i].fa; face_out[i] = iv[i].fb;
    }
    return n;
}

int orc_contains(const orc_volume* v, const double p[3])
{
    double q[3] = {p[0] - v->center[0], p[1] - v->center[1], p[2] - v->center[2]};
    switch (v->kind) {
    case ORC_BOX:
        return fabs(q[0]) <= 0.5 * v->size[0] && fabs(q[1]) <= 0.5 * v->size[1] && fabs(q[2]) <= 0.5 * v->size[2];
    case ORC_CYLINDER: {
        int a = v->axis, b = (a + 1) % 3, c = (a + 2) % 3;
        return q[b] * q[b] + q[c] * q[c] <= v->size[0] * v->size[0] && fabs(q[a]) <= 0.5 * v->size[1];
    }
    case ORC_CYL_SHELL: {
        int a = v->axis, b = (a + 1) % 3, c = (a + 2) % 3;
        double rho2 = q[b] * q[b] + q[c] * q[c];
        return rho2 >= v->size[0] * v->size[0] && rho2 <= v->size[1] * v->size[1] && fabs(q[a]) <= 0.5 * v->size[2];
    }
    case ORC_SPHERE:
        return q[0] * q[0] + q[1] * q[1] + q[2] * q[2] <= v->size[0] * v->size[0];
    case ORC_SPH_SHELL: {
        double r2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
        return r2 >= v->size[0] * v->size[0] && r2 <= v->size[1] * v->size[1];
    }
    }
    return 0;
}

/* Innermost volume containing p: the world first, then descend into the child
 * that contains the point (children never overlap).  -1 if outside the world
 * (the tracing phase then terminates the particle). */
static int locate(const orc_problem* P, const double p[3])
{
    if (!orc_contains(&P->volumes[0], p)) return -1;
    int cur = 0;
    for (;;) {
        int next = -1;
        for (int i = 0; i < P->n_volumes; ++i)
            if (P->volumes[i].parent == cur && orc_contains(&P->volumes[i], p)) { next = i; break; }
        if (next < 0) return cur;
        cur = next;
    }
}

/* Outward unit normal of face f of volume v at point p (used by mirrors). */
static void face_normal(const orc_volume* v, int f, const double p[3], double n[3])
{
    n[0] = n[1] = n[2] = 0.0;
    double q[3] = {p[0] - v->center[0], p[1] - v->center[1], p[2] - v->center[2]};
    if (v->kind == ORC_BOX) {
        n[f / 2] = (f & 1) ? 1.0 : -1.0;
        return;
    }
    if (v->kind == ORC_CYLINDER || v->kind == ORC_CYL_SHELL) {
        int a = v->axis, b = (a + 1) % 3, c = (a + 2) % 3;
        if (f == 1) { n[a] = -1.0; return; }
        if (f == 2) { n[a] = 1.0; return; }
        double r = sqrt(q[b] * q[b] + q[c] * q[c]);
        double s = (f == 3) ? -1.0 : 1.0;
        n[b] = s * q[b] / r; n[c] = s * q[c] / r;
        return;
    }
    double r = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    double s = (f == 3) ? -1.0 : 1.0;
    for (int k = 0; k < 3; ++k) n[k] = s * q[k] / r;
}

/* ------------------------------------------------------------------------ */
/* Mirror (mirror and disk chopper section, reflectivity equation)           */
/* ------------------------------------------------------------------------ */

/* "tanh": the McStas empirical form of the paper,
 *     R0                                                   Q <= Qc
 *     R0/2 (1 - alpha (Q - Qc)) (1 - tanh((Q - m Qc)/W))    Q >  Qc
 * "linear": the piecewise-linear supermirror used by the guide workload,
 *     R0 for Q <= Qc, R0 - alpha (Q - Qc) for Qc < Q <= m Qc, 0 beyond.
 * Negative values are clipped to 0. */
double orc_mirror_reflectivity(const orc_volume* v, double Q)
{
    double R;
    if (Q <= v->Qc) return v->R0;
    if (v->mirror_model == ORC_MIRROR_TANH) {
        R = 0.5 * v->R0 * (1.0 - v->alpha * (Q - v->Qc)) * (1.0 - tanh((Q - v->m * v->Qc) / v->W));
    } else {
        if (Q > v->m * v->Qc) return 0.0;
        R = v->R0 - v->alpha * (Q - v->Qc);
    }
    return R > 0.0 ? R : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Event hash: FNV-1a (64 bit) over each event word's four bytes              */
/* ------------------------------------------------------------------------ */

static void hash_event(uint64_t* h, int code, int arg)
{
    uint32_t word = ((uint32_t)code << 24) | ((uint32_t)arg & 0xFFFFFFu);
    for (int i = 0; i < 4; ++i) {
        *h ^= (word >> (8 * i)) & 0xFFu;
        *h *= 1099511628211ull;
    }
}

/* ------------------------------------------------------------------------ */
/* Source (particle gun section)                                             */
/* ------------------------------------------------------------------------ */

static void sample_source(const orc_source* s, rng_t* r, double p[3], double u[3], double* lam)
{
    p[0] = s->origin[0]; p[1] = s->origin[1]; p[2] = s->origin[2];
    u[0] = s->dir[0]; u[1] = s->dir[1]; u[2] = s->dir[2];
    if (s->kind == ORC_RECT || s->kind == ORC_RECT_DIVERGENT || s->kind == ORC_MODERATOR) {
        double a = next_u(r);
        double b = next_u(r);
        p[0] += (a - 0.5) * s->size[0];
        p[1] += (b - 0.5) * s->size[1];
    }
    if (s->kind == ORC_MODERATOR) {
        /* moderator-surface gun: aim from the source point at a uniform point of the slit */
        double sx = s->slit_center[0] + (next_u(r) - 0.5) * s->slit_size[0];
        double sy = s->slit_center[1] + (next_u(r) - 0.5) * s->slit_size[1];
        double v[3] = {sx - p[0], sy - p[1], s->slit_center[2] - p[2]};
        double nrm = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        u[0] = v[0] / nrm; u[1] = v[1] / nrm; u[2] = v[2] / nrm;
    } else if (s->kind == ORC_RECT_DIVERGENT) {
        double ax = (2.0 * next_u(r) - 1.0) * s->div_deg[0] * PI / 180.0;
        double ay = (2.0 * next_u(r) - 1.0) * s->div_deg[1] * PI / 180.0;
        double v[3] = {tan(ax), tan(ay), 1.0};
        double nrm = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        u[0] = v[0] / nrm; u[1] = v[1] / nrm; u[2] = v[2] / nrm;
    } else {
        double nrm = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        u[0] /= nrm; u[1] /= nrm; u[2] /= nrm;
    }
    if (s->spectrum == ORC_MONO) {
        *lam = s->lam0;
    } else if (s->spectrum == ORC_UNIFORM) {
        *lam = s->lam_lo + next_u(r) * (s->lam_hi - s->lam_lo);
    } else {
        /* Maxwell-Boltzmann energy density sqrt(E) exp(-E/kT), i.e. Gamma(3/2)
         * in units of kT: an exponential plus half a squared normal, the
         * latter from the Box-Muller cosine; rejection to [lam_lo, lam_hi]. */
        double l = s->lam0;
        for (int attempt = 0; attempt < 64; ++attempt) {
            double x1 = 1.0 - next_u(r);
            double x2 = 1.0 - next_u(r);
            double u3 = next_u(r);
            double c = cos(0.5 * PI * u3);
            double e = s->kT * (-log(x1) - log(x2) * c * c);
            l = angstrom_from_ev(e);
            if (l >= s->lam_lo && l <= s->lam_hi) break;
            if (attempt == 63) l = l < s->lam_lo ? s->lam_lo : s->lam_hi;
        }
        *lam = l;
    }
}

/* ------------------------------------------------------------------------ */
/* Tallies                                                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    double** sw;
    double** sw2;
} acc_t;

static int tally_bin(const orc_tally* t, double value, int axis)
{
    double lo = t->lo[axis], hi = t->hi[axis];
    int n = t->nbins[axis];
    if (!(value >= lo && value <= hi)) return -1;
    if (value == hi) return n - 1;
    int i = (int)floor((value - lo) / (hi - lo) * n);
    if (i >= n) i = n - 1;
    return i;
}

/* first_coll = 1: the history's first collision just happened (only the
 * first-collision tallies fire); first_coll = 0: the history ended with `term` */
static void score(const orc_problem* P, acc_t* acc, int first_coll, int term, int det_vol, const double p[3],
                  const double u[3], double lam, double w, int nscat, double tof)
{
    for (int ti = 0; ti < P->n_tallies; ++ti) {
        const orc_tally* t = &P->tallies[ti];
        if ((t->trigger == ORC_TRIG_FIRST_COLLISION) != (first_coll != 0)) continue;
        if (t->trigger == ORC_TRIG_ESCAPE && term != ORC_END_ESCAPE) continue;
        if (t->trigger == ORC_TRIG_ABSORB && term != ORC_END_ABSORB) continue;
        if (t->trigger == ORC_TRIG_DETECT) {
            if (term != ORC_END_DETECT) continue;
            if (t->trigger_volume >= 0 && t->trigger_volume != det_vol) continue;
        }
        if (t->filter == ORC_FILT_UNSCATTERED && nscat != 0) continue;
        if (t->filter == ORC_FILT_SCATTERED && nscat < 1) continue;
        if (t->filter == ORC_FILT_NSCAT_EQ && nscat != t->filter_arg) continue;
        long flat = 0;
        int ok = 1;
        for (int a = 0; a < t->naxes; ++a) {
            double x = 0.0;
            switch (t->quantity[a]) {
            case ORC_Q_THETA2: {
                double bn = sqrt(t->beam[0] * t->beam[0] + t->beam[1] * t->beam[1] + t->beam[2] * t->beam[2]);
                double c = (u[0] * t->beam[0] + u[1] * t->beam[1] + u[2] * t->beam[2]) / bn;
                if (c > 1.0) c = 1.0;
                if (c < -1.0) c = -1.0;
                x = acos(c) * 180.0 / PI;
                break;
            }
            case ORC_Q_LAMBDA: x = lam; break;
            case ORC_Q_X: x = p[0]; break;
            case ORC_Q_Y: x = p[1]; break;
            case ORC_Q_Z: x = p[2]; break;
            case ORC_Q_DIVX: x = atan2(u[0], u[2]) * 180.0 / PI; break;
            case ORC_Q_DIVY: x = atan2(u[1], u[2]) * 180.0 / PI; break;
            case ORC_Q_NSCAT: x = (double)nscat; break;
            case ORC_Q_TOF: x = tof; break;
            case ORC_Q_Q: {
                /* momentum transfer of elastic scattering from the beam direction to u:
                   |k_out - k_in| = 2 k sin(alpha / 2), k = 2 pi / lambda, with
                   sin(alpha / 2) = sqrt((1 - cos alpha) / 2) (DeltaMomentum scorer) */
                double bn = sqrt(t->beam[0] * t->beam[0] + t->beam[1] * t->beam[1] + t->beam[2] * t->beam[2]);
                double c = (u[0] * t->beam[0] + u[1] * t->beam[1] + u[2] * t->beam[2]) / bn;
                if (c > 1.0) c = 1.0;
                if (c < -1.0) c = -1.0;
                x = 4.0 * PI / lam * sqrt((1.0 - c) / 2.0);
                break;
            }
            }
            int b = tally_bin(t, x, a);
            if (b < 0) { ok = 0; break; }
            flat = flat * t->nbins[a] + b;
        }
        if (!ok) continue;
        acc->sw[ti][flat] += w;
        acc->sw2[ti][flat] += w * w;
    }
}

/* ------------------------------------------------------------------------ */
/* One history (simulation flow section)                                     */
/* ------------------------------------------------------------------------ */

/* h / m_n in mm A / s (CODATA 2018): a neutron of wavelength lambda [A] moves
 * at h / (m_n lambda) */
#define H_OVER_MN (6.62607015e-34 / 1.67492749804e-27 * 1e13)

/* Disk chopper (mirror and disk chopper section, Table tableDiskChopper): the
 * polar angle phi of the crossing point about the disk axis (from the next axis
 * towards the one after), the disk turned by phase + 2 pi f t; the point is open
 * when it lies outside the black inner radius and within theta0 after the start
 * of one of the n evenly spread windows. */
static int chopper_open(const orc_volume* V, const double p[3], double t)
{
    int a = V->axis, b = (a + 1) % 3, c = (a + 2) % 3;
    double qb = p[b] - V->center[b], qc = p[c] - V->center[c];
    double rho = sqrt(qb * qb + qc * qc);
    if (rho < V->chop_r) return 0;
    double phi = atan2(qc, qb);
    double ang = phi - V->chop_phase * PI / 180.0 - 2.0 * PI * V->chop_freq * t;
    double per = 2.0 * PI / V->chop_n;
    double m = fmod(ang, per);
    if (m < 0.0) m += per;
    return m < V->chop_theta0 * PI / 180.0;
}

static void run_history(const orc_problem* P, uint64_t seed, uint64_t hid, acc_t* acc, orc_record* rec,
                        orc_stats* st)
{
    rng_t rng = {seed, hid, 0};
    double p[3], u[3], lam;
    sample_source(P->source, &rng, p, u, &lam);
    double w = 1.0;
    double t = 0.0;   /* time since emission, s */
    int nscat = 0, steps = 0, term = 0, det_vol = -1;
    uint64_t hash = 14695981039346656037ull;
    int region = locate(P, p);
    hash_event(&hash, ORC_EV_SOURCE, region);

    if (region < 0) {
        term = ORC_END_OUTSIDE;
    }
    while (term == 0) {
        if (steps >= ORC_MAX_STEPS) {
            term = ORC_END_CAPPED;
            hash_event(&hash, ORC_EV_CAPPED, 0);
            break;
        }
        steps++;
        const orc_volume* V = &P->volumes[region];

        /* distance to leave the current volume: end of the piece ahead */
        ival iv[2];
        int ni = solid_ivals(V, p, u, iv);
        double d_exit = INFINITY;
        int exit_face = -1;
        for (int i = 0; i < ni; ++i)
            if (iv[i].b > 0.0 && iv[i].b < d_exit) { d_exit = iv[i].b; exit_face = iv[i].fb; }
        if (d_exit == INFINITY) { d_exit = 0.0; exit_face = -1; }

        /* distance to enter a daughter volume */
        double d_child = INFINITY;
        int child = -1;
        for (int c = 0; c < P->n_volumes; ++c) {
            if (P->volumes[c].parent != region) continue;
            ival cv[2];
            int nc = solid_ivals(&P->volumes[c], p, u, cv);
            for (int i = 0; i < nc; ++i)
                if (cv[i].a > 0.0 && cv[i].a < d_child) { d_child = cv[i].a; child = c; }
        }
        int to_child = d_child < d_exit;
        double d_b = to_child ? d_child : d_exit;

        /* total and biased cross sections of the current material; a process
         * whose bias factor is 0 is removed from both */
        double sig = 0.0, sig_g = 0.0, sa = 0.0, si = 0.0, sc = 0.0, ga = 0.0, gs = 0.0;
        int nact = 0;
        const orc_material* M = NULL;
        if (V->material >= 0) {
            M = &P->materials[V->material];
            double xs[4];
            orc_macro_xs(M, lam, xs);
            ga = M->abs_bias; gs = M->scatter_bias;
            sa = ga > 0.0 ? xs[0] : 0.0;
            si = gs > 0.0 ? xs[1] : 0.0;
            sc = gs > 0.0 ? xs[2] : 0.0;
            nact = (int)xs[3];
            sig = sa + si + sc;
            sig_g = ga * sa + gs * (si + sc);
        }

        int collide = 0;
        double x = d_b;
        if (sig_g > 0.0) {
            /* biased step length l_g = -ln(xi) / (g rho sigma), xi in (0,1] */
            double xi = 1.0 - next_u(&rng);
            double l = -log(xi) / sig_g;
            if (l < d_b) { collide = 1; x = l; }
        }
        for (int k = 0; k < 3; ++k) p[k] += x * u[k];
        /* time of flight: speed h / (m_n lambda) */
        t += x * lam / H_OVER_MN;
        /* weight correction for the move: exp(sum_i (g_i - 1) rho sigma_i x) */
        if (sig_g > 0.0) w *= exp((sig_g - sig) * x);

        if (collide) {
            /* process chosen with probability g_p sigma_p / sigma_g, in the fixed
             * order absorption, incoherent, coherent; a process of zero width is
             * never chosen, even when rounding puts r on its edge */
            double r = next_u(&rng) * sig_g;
            double wa = ga * sa, wi = gs * si, wc = gs * sc;
            if (r < wa || wi + wc == 0.0) {
                w *= 1.0 / ga;
                term = ORC_END_ABSORB;
                hash_event(&hash, ORC_EV_ABS, 0);
                if (nscat == 0) score(P, acc, 1, term, -1, p, u, lam, w, nscat, t);
                break;
            }
            w *= 1.0 / gs;
            if (r < wa + wi || wc == 0.0 || nact == 0) {
                /* bound incoherent elastic: isotropic in the lab frame */
                double mu = 2.0 * next_u(&rng) - 1.0;
                double phi = 2.0 * PI * next_u(&rng);
                double st_ = sqrt(1.0 - mu * mu);
                u[0] = st_ * cos(phi); u[1] = st_ * sin(phi); u[2] = mu;
                hash_event(&hash, ORC_EV_INC, 0);
            } else {
                /* powder Bragg: family j with probability m_j d_j F_j^2 / sum,
                 * scattering angle from 2 d sin(theta) = lambda, azimuth uniform */
                double total = 0.0;
                for (int j = 0; j < nact; ++j) total += M->mult[j] * M->d[j] * M->f2[j];
                double c = next_u(&rng) * total;
                int fam = nact - 1;
                double cum = 0.0;
                for (int j = 0; j < nact; ++j) {
                    cum += M->mult[j] * M->d[j] * M->f2[j];
                    if (cum > c) { fam = j; break; }
                }
                double cos2t = 1.0 - lam * lam / (2.0 * M->d[fam] * M->d[fam]);
                double sin2t = sqrt(1.0 - cos2t * cos2t);
                double phi = 2.0 * PI * next_u(&rng);
                double ax[3] = {0.0, 0.0, 0.0};
                if (fabs(u[0]) < 0.9) ax[0] = 1.0; else ax[1] = 1.0;
                double e1[3] = {u[1] * ax[2] - u[2] * ax[1], u[2] * ax[0] - u[0] * ax[2], u[0] * ax[1] - u[1] * ax[0]};
                double n1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
                e1[0] /= n1; e1[1] /= n1; e1[2] /= n1;
                double e2[3] = {u[1] * e1[2] - u[2] * e1[1], u[2] * e1[0] - u[0] * e1[2], u[0] * e1[1] - u[1] * e1[0]};
                double cp = cos(phi), sp = sin(phi);
                double nu[3];
                for (int k = 0; k < 3; ++k) nu[k] = cos2t * u[k] + sin2t * (cp * e1[k] + sp * e2[k]);
                u[0] = nu[0]; u[1] = nu[1]; u[2] = nu[2];
                hash_event(&hash, ORC_EV_COH, fam);
            }
            nscat++;
            if (nscat == 1) score(P, acc, 1, 0, -1, p, u, lam, w, nscat, t);
            continue;
        }

        /* relocation: the particle is on a boundary */
        if (to_child) {
            region = child;
            hash_event(&hash, ORC_EV_ENTER, region);
            if (P->volumes[region].is_detector) {
                term = ORC_END_DETECT;
                det_vol = region;
                hash_event(&hash, ORC_EV_DETECT, region);
            } else if (P->volumes[region].chop_n > 0 && !chopper_open(&P->volumes[region], p, t)) {
                /* ray-tracing mask of the disk chopper: 0 outside an open window */
                w = 0.0;
                term = ORC_END_KILL;
                hash_event(&hash, ORC_EV_KILL, 0);
            }
            continue;
        }
        if (exit_face >= 0 && (V->mirror_mask >> exit_face) & 1) {
            /* specular reflection, weight times R(Q), Q = 4 pi sin(theta) / lambda */
            double n[3];
            face_normal(V, exit_face, p, n);
            double un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
            double Q = 4.0 * PI * fabs(un) / lam;
            double R = orc_mirror_reflectivity(V, Q);
            w *= R;
            for (int k = 0; k < 3; ++k) u[k] = u[k] - 2.0 * n[k] * un;
            hash_event(&hash, ORC_EV_MIRROR, exit_face);
            if (!(w > 0.0)) {
                term = ORC_END_KILL;
                hash_event(&hash, ORC_EV_KILL, 0);
            }
            continue;
        }
        if (region == 0) {
            term = ORC_END_ESCAPE;
            hash_event(&hash, ORC_EV_ESCAPE, 0);
            break;
        }
        region = V->parent;
        hash_event(&hash, ORC_EV_EXIT, region);
    }

    if (term == ORC_END_ESCAPE || term == ORC_END_ABSORB || term == ORC_END_DETECT)
        score(P, acc, 0, term, det_vol, p, u, lam, w, nscat, t);

    st->histories++;
    st->steps += (uint64_t)steps;
    st->draws += rng.k;
    switch (term) {
    case ORC_END_ESCAPE: st->escaped++; break;
    case ORC_END_ABSORB: st->absorbed++; break;
    case ORC_END_KILL: st->killed++; break;
    case ORC_END_DETECT: st->detected++; break;
    case ORC_END_CAPPED: st->capped++; break;
    case ORC_END_OUTSIDE: st->outside++; break;
    }
    if (rec) {
        rec->hash = hash;
        rec->w = w;
        for (int k = 0; k < 3; ++k) { rec->pos[k] = p[k]; rec->dir[k] = u[k]; }
        rec->lambda = lam;
        rec->term = term;
        rec->n_scat = nscat;
        rec->n_steps = steps;
        rec->n_draws = (int32_t)rng.k;
        rec->region = region;
        rec->tof = (float)t;
    }
}

/* ------------------------------------------------------------------------ */
/* Driver                                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    const orc_problem* P;
    uint64_t seed, first, n;
    acc_t acc;
    orc_record* rec;
    orc_stats st;
} job_t;

static long tally_size(const orc_tally* t)
{
    long n = 1;
    for (int a = 0; a < t->naxes; ++a) n *= t->nbins[a];
    return n;
}

static void* job_main(void* arg)
{
    job_t* j = (job_t*)arg;
    for (uint64_t i = 0; i < j->n; ++i)
        run_history(j->P, j->seed, j->first + i, &j->acc, j->rec ? &j->rec[i] : NULL, &j->st);
    return NULL;
}

int orc_run(const orc_problem* P, uint64_t seed, uint64_t first, uint64_t n, int nthreads,
            double* const* sumw, double* const* sumw2, orc_record* records, orc_stats* stats)
{
    if (!P || P->n_volumes < 1 || !P->source) return -1;
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > n) nthreads = n > 0 ? (int)n : 1;
    job_t* jobs = (job_t*)calloc((size_t)nthreads, sizeof(job_t));
    pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) return -2;
    uint64_t base = n / nthreads, rem = n % nthreads, start = first;
    for (int t = 0; t < nthreads; ++t) {
        job_t* j = &jobs[t];
        j->P = P; j->seed = seed; j->first = start; j->n = base + ((uint64_t)t < rem ? 1 : 0);
        j->rec = records ? records + (start - first) : NULL;
        start += j->n;
        j->acc.sw = (double**)calloc((size_t)(P->n_tallies + 1), sizeof(double*));
        j->acc.sw2 = (double**)calloc((size_t)(P->n_tallies + 1), sizeof(double*));
        for (int ti = 0; ti < P->n_tallies; ++ti) {
            long nb = tally_size(&P->tallies[ti]);
            if (nthreads == 1) {
                j->acc.sw[ti] = sumw[ti];
                j->acc.sw2[ti] = sumw2[ti];
            } else {
                j->acc.sw[ti] = (double*)calloc((size_t)nb, sizeof(double));
                j->acc.sw2[ti] = (double*)calloc((size_t)nb, sizeof(double));
                if (!j->acc.sw[ti] || !j->acc.sw2[ti]) return -2;
            }
        }
    }
    if (nthreads == 1) {
        job_main(&jobs[0]);
    } else {
        for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, job_main, &jobs[t]);
        for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    }
    orc_stats total;
    memset(&total, 0, sizeof(total));
    for (int t = 0; t < nthreads; ++t) {
        job_t* j = &jobs[t];
        for (int ti = 0; ti < P->n_tallies && nthreads > 1; ++ti) {
            long nb = tally_size(&P->tallies[ti]);
            for (long b = 0; b < nb; ++b) {
                sumw[ti][b] += j->acc.sw[ti][b];
                sumw2[ti][b] += j->acc.sw2[ti][b];
            }
            free(j->acc.sw[ti]);
            free(j->acc.sw2[ti]);
        }
        free(j->acc.sw);
        free(j->acc.sw2);
        total.histories += j->st.histories; total.escaped += j->st.escaped; total.absorbed += j->st.absorbed;
        total.killed += j->st.killed; total.detected += j->st.detected; total.capped += j->st.capped;
        total.outside += j->st.outside; total.steps += j->st.steps; total.draws += j->st.draws;
    }
    if (stats) *stats = total;
    free(jobs);
    free(th);
    return 0;
}
