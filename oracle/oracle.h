/*
 * Plain FP64 CPU oracle of the biased neutron history loop.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against an independent, slow, obviously correct implementation.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or constant generator with the GPU library.
 *
 * What it computes (one neutron history, all in double precision):
 *   - Philox4x32-10 counter-based random numbers keyed on (seed, history, draw)
 *   - source sampling (pencil, rectangle, divergent rectangle; mono, uniform
 *     and Maxwellian spectra)
 *   - macroscopic cross sections: 1/v absorption, constant bound incoherent
 *     elastic and powder Bragg coherent elastic (the powder average of the
 *     coherent elastic scattering function)
 *   - free flight under cross-section biasing (sigma_g = g sigma) with the
 *     probability-conserving weight correction (biasing mechanism section,
 *     step-length and weight equations)
 *   - relocation across volume boundaries, mirror reflection with the
 *     empirical reflectivity R(Q) and specular direction (mirror section)
 *   - process choice, absorption, isotropic incoherent and Debye-Scherrer
 *     coherent scattering
 *   - weighted tallies (sum of w and w^2 per bin)
 *
 * Units: mm, Angstrom, barn, eV, degrees.
 */
#ifndef PROMPT_ORACLE_H
#define PROMPT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_BOX = 0, ORC_CYLINDER = 1, ORC_CYL_SHELL = 2, ORC_SPHERE = 3, ORC_SPH_SHELL = 4 };
enum { ORC_PENCIL = 0, ORC_RECT = 1, ORC_RECT_DIVERGENT = 2, ORC_MODERATOR = 3 };
enum { ORC_MONO = 0, ORC_UNIFORM = 1, ORC_MAXWELL = 2 };
/* FIRST_COLLISION fires at a history's first absorption or scattering, with the
 * state just after it (collision point, outgoing direction, weight including the
 * 1/g factor of the chosen process, scattering count 1, or 0 for an absorption);
 * the other triggers fire once, when the history ends */
enum { ORC_TRIG_ESCAPE = 0, ORC_TRIG_ABSORB = 1, ORC_TRIG_DETECT = 2, ORC_TRIG_FIRST_COLLISION = 3 };
enum { ORC_FILT_ALL = 0, ORC_FILT_UNSCATTERED = 1, ORC_FILT_SCATTERED = 2, ORC_FILT_NSCAT_EQ = 3 };
enum { ORC_Q_THETA2 = 0, ORC_Q_LAMBDA = 1, ORC_Q_X = 2, ORC_Q_Y = 3, ORC_Q_Z = 4,
       ORC_Q_DIVX = 5, ORC_Q_DIVY = 6, ORC_Q_NSCAT = 7, ORC_Q_Q = 8, ORC_Q_TOF = 9 };
enum { ORC_MIRROR_LINEAR = 0, ORC_MIRROR_TANH = 1 };
/* termination codes */
enum { ORC_END_ESCAPE = 1, ORC_END_ABSORB = 2, ORC_END_KILL = 3, ORC_END_DETECT = 4,
       ORC_END_CAPPED = 5, ORC_END_OUTSIDE = 6 };
/* event codes folded into the per-history event hash */
enum { ORC_EV_SOURCE = 1, ORC_EV_ENTER = 2, ORC_EV_EXIT = 3, ORC_EV_MIRROR = 4, ORC_EV_ABS = 5,
       ORC_EV_INC = 6, ORC_EV_COH = 7, ORC_EV_ESCAPE = 8, ORC_EV_KILL = 9, ORC_EV_DETECT = 10,
       ORC_EV_CAPPED = 11 };

#define ORC_MAX_STEPS 10000

typedef struct {
    double number_density;   /* atoms per A^3 */
    double sigma_inc;        /* b */
    double sigma_abs_ref;    /* b at 1.798 A */
    double scatter_bias;     /* g_s >= 0, 0 removes scattering */
    double abs_bias;         /* g_a >= 0, 0 removes absorption */
    double cell_volume;      /* A^3 */
    int32_t atoms_per_cell;
    int32_t n_families;
    const double* d;         /* A, canonical order (descending) */
    const int32_t* mult;
    const double* f2;        /* b per cell */
    int32_t n_table;         /* 0, or rows of tabulated sigma_abs, sigma_inc */
    int32_t table_pad;
    const double* table_lambda;
    const double* table_sigma_abs;
    const double* table_sigma_inc;
} orc_material;

typedef struct {
    int32_t kind, axis, parent, material, is_detector, mirror_mask;
    double center[3];
    double size[3];
    int32_t mirror_model;
    int32_t pad;
    double R0, Qc, alpha, m, W;
    int32_t chop_n;          /* disk chopper windows (0 = none), cylinder volumes */
    int32_t chop_pad;
    double chop_r, chop_freq, chop_theta0, chop_phase;   /* mm, Hz, degrees, degrees */
} orc_volume;

typedef struct {
    int32_t kind, spectrum;
    double origin[3], dir[3], size[2], div_deg[2];
    double lam0, lam_lo, lam_hi, kT;
    double slit_center[3], slit_size[2];
} orc_source;

typedef struct {
    int32_t trigger, trigger_volume, filter, filter_arg, naxes;
    int32_t quantity[4];
    int32_t nbins[4];
    int32_t pad;
    double lo[4], hi[4];
    double beam[3];
} orc_tally;

typedef struct {
    int32_t n_materials, n_volumes, n_tallies, pad;
    const orc_material* materials;
    const orc_volume* volumes;
    const orc_source* source;
    const orc_tally* tallies;
} orc_problem;

/* per-history outcome (96 bytes); tof: time since emission in s, rounded to FP32 */
typedef struct {
    uint64_t hash;
    double w;
    double pos[3];
    double dir[3];
    double lambda;
    int32_t term, n_scat, n_steps, n_draws, region;
    float tof;
} orc_record;

typedef struct {
    uint64_t histories, escaped, absorbed, killed, detected, capped, outside, steps, draws;
} orc_stats;

/* Run histories [first, first+n).  sumw[t], sumw2[t] are caller arrays of the
 * tally's bin count, accumulated into (not cleared).  records may be NULL, else
 * n entries.  nthreads >= 1 splits the history range across POSIX threads. */
int orc_run(const orc_problem* prob, uint64_t seed, uint64_t first, uint64_t n, int nthreads,
            double* const* sumw, double* const* sumw2, orc_record* records, orc_stats* stats);

/* pieces exposed for the pin tests */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_uniform(uint64_t seed, uint64_t history, uint32_t draw);
int orc_intervals(const orc_volume* v, const double p[3], const double u[3],
                  double t_in[2], double t_out[2], int32_t face_in[2], int32_t face_out[2]);
int orc_contains(const orc_volume* v, const double p[3]);
void orc_macro_xs(const orc_material* m, double lambda, double out[4]);
double orc_mirror_reflectivity(const orc_volume* v, double Q);
double orc_ev_from_angstrom(double lambda);

#ifdef __cplusplus
}
#endif
#endif
