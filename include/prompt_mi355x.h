/*
 * prompt_mi355x: MI355X-native biased neutron history loop behind a C-ABI.
 *
 * The library runs the per-neutron history loop of "Prompt: probability-
 * conserved cross section biasing Monte Carlo particle transport system"
 * (Pan et al., arXiv 2304.06226) on one AMD Instinct MI355X (gfx950):
 *   source neutron (particle gun section) ->
 *   free flight through boxes, cylinders, spheres and shells under biased
 *   cross sections sigma_g = g sigma, with the probability-conserving weight
 *   correction (cross section biasing mechanism section, step-length and
 *   weight equations) ->
 *   absorption, bound incoherent or powder-Bragg coherent elastic scattering
 *   (neutron scattering cross section section) or mirror reflection (mirror
 *   section, reflectivity and reflection equations) ->
 *   weighted tallies (scorer section).
 *
 * Conventions
 *   - Units: mm, Angstrom, barn, eV, degrees.  Number densities in 1/A^3.
 *   - Every call returns PR_OK (0) or a negative PR_E* code; the message of
 *     the last failure is kept per context (pr_last_error).  No exception or
 *     abort crosses the ABI.
 *   - create_* calls deep-copy caller arrays; the caller keeps its inputs.
 *     The context owns every object it creates (freed by pr_destroy),
 *     including the device storage of tallies, except storage the caller
 *     passes to pr_create_tally_in and workspaces passed to pr_run_histories,
 *     which stay the caller's.
 *   - "stream" arguments are hipStream_t values passed as void* (NULL = the
 *     default stream).  Runs and resets are asynchronous on that stream;
 *     pr_read_* calls wait for the whole device, so results are complete
 *     whichever streams the runs were issued on.  Runs of one context may
 *     overlap on different streams: each run has its own history-claim
 *     counter (a caller workspace, or a slot of the context's ring whose reuse
 *     waits for the run that last held it), tallies and statistics are summed
 *     with atomics.  A reset that should not race a run must be ordered after
 *     it by the caller (same stream, or an event).
 *   - One context per host thread.  A context is bound to one HIP device.
 *   - Random numbers: draw k of history h is taken from Philox4x32-10 with
 *     key = seed and counter = (k/2, h); even draws use words 0-1, odd draws
 *     words 2-3.  History ids are global, so running [0,k) and [k,n) gives the
 *     same histories as [0,n) (split and resume).
 */
#ifndef PROMPT_MI355X_H
#define PROMPT_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define PR_OK 0
#define PR_EINVAL (-1)      /* a field is invalid; the message names it */
#define PR_ENOTFOUND (-2)   /* an id does not name an object of this context */
#define PR_EOVERLAP (-3)    /* volumes overlap or a daughter leaves its mother */
#define PR_EWORKSPACE (-4)  /* a caller buffer is too small */
#define PR_EDEVICE (-5)     /* a HIP call failed; the message holds its error string */
#define PR_ENOMEM (-6)      /* host or device allocation failed */
#define PR_ECAPPED (-7)     /* pr_read_stats: the statistics are complete and filled in, but some history
                               since the last pr_reset_stats reached PR_MAX_STEPS (terminated there,
                               counted in pr_run_stats.capped, scored by no tally) */

/* ---- enumerations ---- */
enum { PR_BOX = 0, PR_CYLINDER = 1, PR_CYL_SHELL = 2, PR_SPHERE = 3, PR_SPH_SHELL = 4 };
enum { PR_PENCIL = 0, PR_RECT = 1, PR_RECT_DIVERGENT = 2, PR_MODERATOR = 3 };
enum { PR_MONO = 0, PR_UNIFORM = 1, PR_MAXWELL = 2 };
/* PR_TRIG_FIRST_COLLISION (a debugging trigger, FP64 policies of pr_run_histories
 * only): fires at a history's first absorption or scattering, scoring the state
 * just after it: the collision point, the outgoing direction (unchanged for an
 * absorption), the weight including the 1/g factor of the chosen process, and
 * the scattering count (1 after a scattering, 0 after an absorption).  Its
 * expectation per source neutron is the first-collision probability of the free
 * flight law (cross section section) whatever the bias factors. */
enum { PR_TRIG_ESCAPE = 0, PR_TRIG_ABSORB = 1, PR_TRIG_DETECT = 2, PR_TRIG_FIRST_COLLISION = 3 };
enum { PR_FILT_ALL = 0, PR_FILT_UNSCATTERED = 1, PR_FILT_SCATTERED = 2, PR_FILT_NSCAT_EQ = 3 };
enum { PR_Q_THETA2 = 0, PR_Q_LAMBDA = 1, PR_Q_X = 2, PR_Q_Y = 3, PR_Q_Z = 4, PR_Q_DIVX = 5, PR_Q_DIVY = 6,
       PR_Q_NSCAT = 7, PR_Q_Q = 8, PR_Q_TOF = 9 };
enum { PR_MIRROR_LINEAR = 0, PR_MIRROR_TANH = 1 };
/* Tally accumulators: FP64 sums (gfx950 adds FP64 atomically in LDS and in global
 * memory).  PR_ACC_KAHAN_FP32 is reserved and rejected with PR_EINVAL. */
enum { PR_ACC_FP64 = 0, PR_ACC_KAHAN_FP32 = 1 };
/* precision policies of pr_run_histories */
enum {
    PR_FP64_PLAIN = 0,   /* one thread per history, everything in FP64, global tables and atomics */
    PR_FP32_MIXED = 1,   /* persistent lanes refilled from a wave-shared history counter; FP32
                            positions, directions, cross sections and sampling; FP64 weight
                            product and tallies; LDS-staged tables, LDS-privatised small tallies
                            (or, under a monochromatic source, the slice of a tally at the source
                            wavelength's bin).  Every volume is entered whatever its thickness;
                            a history that leaves a daughter by a move shorter than 2^-20
                            (|x|+|y|+|z|) (an FP32 position may not change over it) does not
                            re-enter that daughter in its next step through a piece that short,
                            so rays grazing an edge make progress.  First-collision tallies are
                            not accepted (PR_EINVAL) */
    PR_FP64_PERSISTENT = 2  /* the persistent lanes, LDS-privatised tallies and bin cache of
                            PR_FP32_MIXED around the FP64 step of PR_FP64_PLAIN: every
                            history's events, final weight and exit state equal
                            PR_FP64_PLAIN's bit for bit, and tallies agree to the rounding
                            of the order of summation.  Scene tables are read from global
                            memory; the launch tuning (block, blocks per CU, refill
                            threshold, chunk, bin cache) is the one PR_FP32_MIXED uses,
                            waves_per_simd excepted */
};
/* termination codes written to history records */
enum { PR_END_ESCAPE = 1, PR_END_ABSORB = 2, PR_END_KILL = 3, PR_END_DETECT = 4, PR_END_CAPPED = 5,
       PR_END_OUTSIDE = 6 };

#define PR_MAX_STEPS 10000   /* steps per history before it is killed and counted as capped */
#define PR_MAX_TALLIES 8     /* tallies per run */

typedef struct pr_ctx pr_ctx;

/* Material (simulation physics section; material listing with bias factors).
 *   Sigma_abs(lambda) = 0.1 n sigma_abs_ref lambda / 1.798          [1/mm]  (1/v law)
 *   Sigma_inc         = 0.1 n sigma_inc                              [1/mm]
 *   Sigma_coh(lambda) = 0.1 n lambda^2 / (2 v0 N) sum_{2 d_j > lambda} m_j d_j F2_j
 * (the powder average of the coherent elastic scattering function).  Bias
 * factors scale the cross sections used for sampling (sigma_g = g sigma); a
 * factor of 0 removes that process.  d must be in canonical order (non-
 * increasing); families with equal d stay separate.  Arrays are copied. */
typedef struct {
    double number_density;    /* atoms / A^3, > 0 */
    double sigma_inc;         /* b, >= 0 */
    double sigma_abs_ref;     /* b at 1.798 A, >= 0 */
    double scatter_bias;      /* >= 0 (default 1) */
    double abs_bias;          /* >= 0 (default 1) */
    double cell_volume;       /* A^3; 0 together with n_families = 0 means no Bragg scattering */
    int32_t atoms_per_cell;   /* N */
    int32_t n_families;       /* 0..1024 */
    const double* d;          /* [n_families] A, > 0, non-increasing */
    const int32_t* mult;      /* [n_families] > 0 */
    const double* f2;         /* [n_families] b per cell, >= 0 */
    /* Optional tabulated cross sections (stand-ins for externally computed
     * materials): with n_table >= 2 rows, sigma_abs(lambda) and sigma_inc(lambda)
     * are interpolated linearly in lambda between rows (constant beyond the first
     * and last rows) and replace the 1/v law and the constant sigma_inc; the
     * interpolation error on [l_i, l_i+1] is at most (l_i+1 - l_i)^2 / 8 times the
     * largest |sigma''| there.  Coherent scattering stays the Bragg sum. */
    int32_t n_table;          /* 0, or 2..4096 */
    int32_t table_pad;
    const double* table_lambda;     /* [n_table] A, > 0, strictly increasing */
    const double* table_sigma_abs;  /* [n_table] b, >= 0 */
    const double* table_sigma_inc;  /* [n_table] b, >= 0 */
} pr_material_desc;

/* Mirror on faces of a volume (mirror section).  "tanh": the empirical form
 *   R = R0 (Q <= Qc), R0/2 (1 - alpha (Q - Qc)) (1 - tanh((Q - m Qc)/W)) (Q > Qc);
 * "linear": R0 up to Qc, R0 - alpha (Q - Qc) up to m Qc, 0 beyond.
 * Q = 4 pi |u.n| / lambda.  The weight is multiplied by R (clipped at 0) and
 * the direction reflected, u' = u - 2 n (u.n); R = 0 ends the history. */
typedef struct {
    int32_t model;            /* PR_MIRROR_* */
    int32_t pad;
    double R0, Qc, alpha, m, W;
} pr_mirror_desc;

/* Disk chopper (mirror and disk chopper section; Table tableDiskChopper),
 * carried by a PR_CYLINDER volume (the disk, normally very thin) whose axis
 * is the rotation axis and whose radius is the outer radius R.  When a neutron
 * enters the disk at position p and time t its weight is multiplied by the
 * ray-tracing mask epsilon (0 or 1): with rho, phi the polar coordinates of p
 * about the axis (phi from the next axis towards the one after, right-handed:
 * x -> y about z, y -> z about x, z -> x about y), epsilon = 1 iff rho >= r and
 * (phi - phase - 2 pi rot_freq t) mod (2 pi / n) < theta0; epsilon = 0 ends the
 * history (killed).  n = 0: no chopper. */
typedef struct {
    int32_t n;                /* number of windows, evenly spread over 2 pi (0 = none) */
    int32_t pad;
    double r;                 /* mm, inner (black) radius */
    double rot_freq;          /* Hz, positive = right-handed about the axis */
    double theta0;            /* degrees, opening angle of a window */
    double phase;             /* degrees, window start at t = 0 */
} pr_chopper_desc;

/* Volume (geometry section).  size by kind:
 *   PR_BOX        {side_x, side_y, side_z} (full sides, axis aligned)
 *   PR_CYLINDER   {r, h}               axis = 0,1,2
 *   PR_CYL_SHELL  {r_in, r_out, h}     open-ended tube wall (the bore belongs to the mother)
 *   PR_SPHERE     {r}
 *   PR_SPH_SHELL  {r_in, r_out}
 * Volume 0 is the world (parent -1); leaving it is an escape.  Every other
 * volume names its mother (a lower index) and must lie strictly inside it and
 * strictly apart from its sisters (checked: PR_EOVERLAP).  Face ids used by
 * mirror_mask bits: box 0..5 = -x,+x,-y,+y,-z,+z; cylinder and shell 0 outer
 * wall, 1 low cap, 2 high cap, 3 inner wall; sphere 0 outer, 3 inner.  A
 * mirror acts when the particle leaves the volume through a masked face. */
typedef struct {
    int32_t kind;             /* PR_BOX .. PR_SPH_SHELL */
    int32_t axis;             /* cylinders: 0 x, 1 y, 2 z */
    int32_t parent;           /* -1 for volume 0, else a lower index */
    int32_t material;         /* material id or -1 (vacuum) */
    int32_t is_detector;      /* 1: entering it ends the history and fires PR_TRIG_DETECT tallies */
    int32_t mirror_mask;      /* faces carrying the mirror */
    double center[3];         /* mm */
    double size[3];           /* mm, see above */
    pr_mirror_desc mirror;
    pr_chopper_desc chopper;
} pr_volume_desc;

/* Source (particle gun section).  PR_PENCIL: origin and direction.
 * PR_RECT: origin + ((u0 - 1/2) size_x, (u1 - 1/2) size_y, 0), direction dir.
 * PR_RECT_DIVERGENT: as PR_RECT, then alpha_x, alpha_y uniform in
 * [-div, div] degrees and direction ~ (tan alpha_x, tan alpha_y, 1).
 * PR_MODERATOR (the moderator-surface guns): the position as PR_RECT on the
 * source rectangle, then a point slit_center + ((u2 - 1/2) slit_x,
 * (u3 - 1/2) slit_y, 0) on the slit rectangle; the direction joins the two
 * (dir is not used; slit_center z must differ from origin z).  A uniform
 * spectrum mean +- range is lam_lo = mean - range, lam_hi = mean + range.
 * Spectrum: PR_MONO lam0; PR_UNIFORM lambda uniform in [lam_lo, lam_hi];
 * PR_MAXWELL energy density ~ sqrt(E) exp(-E/kT), rejected to [lam_lo, lam_hi]
 * (at most 64 tries of three draws).  Draw order: position, divergence, lambda. */
typedef struct {
    int32_t kind;             /* PR_PENCIL, PR_RECT, PR_RECT_DIVERGENT, PR_MODERATOR */
    int32_t spectrum;         /* PR_MONO, PR_UNIFORM, PR_MAXWELL */
    double origin[3];         /* mm */
    double dir[3];            /* non-zero; PR_RECT_DIVERGENT requires +z */
    double size[2];           /* mm */
    double div_deg[2];        /* degrees */
    double lam0, lam_lo, lam_hi;   /* A */
    double kT;                /* eV */
    double slit_center[3];    /* mm, PR_MODERATOR */
    double slit_size[2];      /* mm, PR_MODERATOR */
} pr_source_desc;

typedef struct {
    int32_t quantity;         /* PR_Q_*: 2theta = acos(u.beam) deg; lambda A; x,y,z mm;
                                 div_x = atan2(u_x, u_z) deg; div_y = atan2(u_y, u_z) deg; n_scat;
                                 Q = |k_out - k_beam| = (4 pi / lambda) sqrt((1 - u.beam) / 2) 1/A,
                                 the momentum transfer of elastic scattering out of the beam direction
                                 (the DeltaMomentum scorer, Table tableScorer); tof = time since
                                 emission in s (TOF scorer; sources emit at t = 0, a neutron moves at
                                 v = h / (m_n lambda)) */
    int32_t nbins;            /* >= 1 */
    double lo, hi;            /* hi > lo; bin = floor((x - lo) / (hi - lo) nbins); x = hi goes to the
                                 last bin; values outside [lo, hi] are not scored */
} pr_tally_axis;

/* Tally (scorer section): fires once per history at its end when the
 * trigger and filter match, adding w to sum_w and w^2 to sum_w2 of one bin
 * (row-major over the axes, axis 0 slowest; 0 axes = one counter bin). */
typedef struct {
    int32_t trigger;          /* PR_TRIG_* */
    int32_t trigger_volume;   /* PR_TRIG_DETECT: detector volume index, -1 = any */
    int32_t filter;           /* PR_FILT_* on the history's scattering count */
    int32_t filter_arg;       /* k of PR_FILT_NSCAT_EQ */
    int32_t naxes;            /* 0..4 */
    int32_t accumulator;      /* PR_ACC_FP64 */
    pr_tally_axis axes[4];
    double beam[3];           /* 2theta reference direction (need not be normalised) */
} pr_tally_desc;

/* Per-history outcome (96 bytes, little endian), written when a record
 * buffer is given: FNV-1a hash of the event sequence, final weight, final
 * position and direction, wavelength, termination code, scatterings, steps,
 * random draws consumed, the final volume and the time since emission in s
 * (rounded to FP32; 0 unless the run tracks time, i.e. its scene holds a disk
 * chopper or a tally bins the time of flight). */
typedef struct {
    uint64_t hash;
    double w;
    double pos[3];
    double dir[3];
    double lambda;
    int32_t term, n_scat, n_steps, n_draws, region;
    float tof;
} pr_history_record;

typedef struct {
    uint64_t histories, escaped, absorbed, killed, detected, capped, outside, steps, draws, scatters;
} pr_run_stats;

/* ---- context ---- */
/* Create a context on HIP device hip_device with run seed `seed` (the
 * launcher's default is 4096).  *out receives the context or NULL. */
int pr_init(pr_ctx** out, int hip_device, uint64_t seed);
void pr_destroy(pr_ctx* ctx);
const char* pr_last_error(const pr_ctx* ctx);
int pr_set_seed(pr_ctx* ctx, uint64_t seed);

/* ---- problem objects ---- */
int pr_create_material(pr_ctx* ctx, const pr_material_desc* desc, int32_t* id);
/* n volumes, volume 0 the world; validates kinds, sizes, tree and overlaps. */
int pr_create_geometry(pr_ctx* ctx, const pr_volume_desc* volumes, int32_t n, int32_t* id);
int pr_create_source(pr_ctx* ctx, const pr_source_desc* desc, int32_t* id);
/* allocates and zeroes the tally's device storage: 2 x nbins doubles, (sum w,
 * sum w^2) interleaved per bin so that the two atomics of a score update one
 * 16-byte pair; pr_read_tally returns them as separate arrays.  Synchronises
 * the device. */
int pr_create_tally(pr_ctx* ctx, const pr_tally_desc* desc, int32_t* id);
/* Bytes of device storage a tally of this description needs (2 x nbins doubles);
 * validates the description as pr_create_tally does. */
int pr_tally_storage_size(pr_ctx* ctx, const pr_tally_desc* desc, size_t* bytes);
/* As pr_create_tally, with the tally's storage in the caller's device buffer
 * dev_storage of storage_bytes bytes (16-byte aligned, at least
 * pr_tally_storage_size bytes; PR_EWORKSPACE if smaller): the library zeroes it
 * (synchronising the device), accumulates into it with the layout above and
 * never frees it.  The buffer must stay valid until pr_destroy or until no run
 * uses the tally any more. */
int pr_create_tally_in(pr_ctx* ctx, const pr_tally_desc* desc, void* dev_storage, size_t storage_bytes,
                       int32_t* id);
int pr_tally_nbins(pr_ctx* ctx, int32_t tally, uint64_t* nbins);

/* ---- running ---- */
/* Bytes of device workspace a run of this precision uses when the caller
 * provides it (its history-claim counter; 256). */
int pr_workspace_size(pr_ctx* ctx, int32_t precision, size_t* bytes);
/* Run histories [first_history, first_history + n) of source `src` through
 * geometry `geom`, scoring into the n_tallies tallies listed (the simulation
 * flow section: source, transport, scoring).  precision is PR_FP64_PLAIN,
 * PR_FP32_MIXED or PR_FP64_PERSISTENT.  records_dev is NULL or a device buffer
 * of n pr_history_record entries (record i is history first_history + i).
 * dev_workspace is NULL or a caller device buffer of ws_bytes >=
 * pr_workspace_size bytes (8-byte aligned; PR_EWORKSPACE if smaller), owned by
 * the caller, that the run uses as scratch until it completes on `stream`; with
 * NULL the run takes a slot of the context's counter ring.  Asynchronous on
 * `stream`; tallies and run statistics accumulate across runs until reset.
 * n is at most 2^48 and first_history at most 2^62 (PR_EINVAL). */
int pr_run_histories(pr_ctx* ctx, int32_t geom, int32_t src, const int32_t* tallies, int32_t n_tallies,
                     uint64_t first_history, uint64_t n, int32_t precision, void* records_dev, void* dev_workspace,
                     size_t ws_bytes, void* stream);

/* ---- batched runs ---- */
/* One simulation of a batch: geometry, source, up to PR_MAX_TALLIES tallies and
 * its history range [first_history, first_history + n).  Give the simulations
 * of a batch disjoint history ranges (e.g. consecutive ones) so that their
 * random-number streams are disjoint. */
typedef struct {
    int32_t geom;
    int32_t src;
    int32_t n_tallies;
    int32_t tallies[PR_MAX_TALLIES];
    int32_t pad;
    uint64_t first_history;
    uint64_t n;
} pr_sim;

/* Run nsims independent simulations of uneven size and geometry in one
 * persistent launch per class of simulations (scene staged in LDS or not,
 * daughter grid or not) of the PR_FP32_MIXED policy (the only policy
 * accepted; first-collision tallies are not).  Each block starts on the simulation under its share of the
 * concatenated history ranges, stages that simulation's scene and tallies in
 * LDS, and its waves claim chunks of that simulation's histories from the
 * simulation's own counter until none are left; the block then merges its
 * tallies and moves to the next simulation that still has histories.
 * Asynchronous on `stream`; each simulation's histories are exactly those of
 * pr_run_histories over the same range.  The descriptors are copied: sims may
 * be reused as soon as the call returns. */
int pr_run_batch(pr_ctx* ctx, const pr_sim* sims, int32_t nsims, int32_t precision, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): pr_run_batch without
 * any device or pinned-host allocation.  The batch's descriptors and
 * per-simulation claim counters go to a fixed 2 MiB device array compiled into
 * the library (one per GPU, held until the process ends) instead of the
 * context's descriptor ring; they are copied there from a context-owned host
 * image with hipMemcpyAsync on `stream`, and the counters are cleared by a kernel
 * on `stream`.  Results are those of pr_run_batch over the same simulations.
 * Batches whose descriptors exceed the array (about 3000 simulations with one
 * tally each) return PR_EWORKSPACE.  Every call on a GPU uses the same array:
 * calls ordered on one stream are safe, calls that overlap in time on one GPU
 * (other streams, other contexts) race and must not be issued. */
int pr_run_batch_static(pr_ctx* ctx, const pr_sim* sims, int32_t nsims, int32_t precision, void* stream);

/* ---- prepared batches (repeated steps, HIP graph capture) ----
 * pr_prepare_batch validates sims as pr_run_batch does, uploads their
 * descriptors once into device memory owned by the context and freezes the
 * launch tuning; *batch receives its id.  Each pr_run_prepared then runs every
 * simulation over histories [first_history + offset, first_history + offset +
 * n) with the batch's device-resident offset (0 at preparation) and afterwards
 * adds `stride` to that offset (ids wrap modulo 2^64), so successive runs or
 * graph replays continue with fresh histories when stride covers the batch's id
 * span.  A run consists of kernel launches on `stream` only (no host copies,
 * allocations, memsets or synchronisation), so it may be captured into a HIP
 * graph and replayed; the histories of its tallies are counted on the device
 * and included in pr_read_tally's n_hist.  Runs of one prepared batch must
 * not overlap in time (they share its work counters).  Errors as pr_run_batch;
 * PR_ENOTFOUND for an unknown or released batch.  pr_release_batch synchronises
 * the device and frees the batch's device memory. */
int pr_prepare_batch(pr_ctx* ctx, const pr_sim* sims, int32_t nsims, int32_t precision, uint64_t stride,
                     int32_t* batch);
int pr_run_prepared(pr_ctx* ctx, int32_t batch, void* stream);
int pr_release_batch(pr_ctx* ctx, int32_t batch);

/* ---- launch tuning of the persistent policies (PR_FP32_MIXED, PR_FP64_PERSISTENT) ---- */
/* block: threads per block, a multiple of 64 up to 1024 (launches clamp it to
 * their kernel's limit: 1024 for the FP32 kernels without a daughter grid, 512
 * with one, 256 for PR_FP64_PERSISTENT and for batches without a grid);
 * blocks_per_cu: resident
 * blocks per compute unit of the persistent grid (0 = occupancy limit);
 * refill_threshold: idle lanes of a wave that trigger a refill (1..64);
 * lds_tally_bytes: LDS per block for privatised tallies (tallies are
 * privatised in order while they fit); bin_cache_slots: LDS bin-cache slots
 * given to each tally that is not privatised (0 or a power of two <= 4096);
 * chunk: history indices a wave claims from the shared counter (batched
 * runs: from the simulation's own counter) per atomic;
 * grid_chunk: the claim size for scenes that navigate a daughter grid (their
 * histories vary more in length, so smaller claims balance the waves), 0 =
 * chunk; in a batch it applies to the class of grid scenes;
 * grid_walk_cells: 0, or 2..1024: in the FP32 policy (single runs and batches)
 * a daughter-grid walk that has visited this many cells without finding the
 * nearest daughter entry pauses at the far wall of the last cell: the history
 * moves there without an event (a virtual boundary; the free flight is
 * memoryless, so no expectation changes) and walks on in its next step, so a
 * wave does not wait for its longest walk.  0: walks run to the end.  The FP64
 * policies always walk to the end (their histories match the oracle's event by
 * event);
 * waves_per_simd: 4 or 5 (0 means 4): resident waves per SIMD the FP32
 * kernels without a daughter grid are compiled for (5 holds them to 96 VGPRs,
 * spilling some state to scratch; which is faster depends on the workload);
 * kernels with a daughter grid always run 4, and PR_FP64_PERSISTENT runs 2
 * (3 with a daughter grid), as PR_FP64_PLAIN does.
 * Scenes with a daughter grid whose grid, box bounds and tables are staged in
 * LDS run blocks of 256 or 512 threads, whichever keeps the most waves
 * resident per CU, unless blocks_per_cu is set (then `block` is used).
 * vacuum_steps: 1 (default) or 0.  At 1, steps that draw nothing are taken
 * early where the scene allows it (scenes without a daughter grid): a history
 * leaving the only, convex daughter of a vacuum, mirrorless box, cylinder or
 * sphere world crosses the world in the same step; a history born in vacuum
 * takes its first step as soon as it is drawn (a pencil beam of one
 * wavelength: later histories copy the state the first one reached there);
 * and, in scenes without mirrors whose material volumes sit in vacuum
 * (PR_FP32_MIXED and PR_FP64_PERSISTENT), a history that leaves material for
 * vacuum takes its vacuum step before the wave's other histories step again.
 * Histories and records are the same either way, except that for a ray that
 * grazes the lone sample's surface as it leaves, rounding could let a separate
 * world step find a re-entry that the folded crossing does not look for
 * (impossible in exact arithmetic: the solid is convex; not seen in tests).
 * Results do not depend on these settings beyond floating-point summation
 * order. */
typedef struct {
    int32_t block;
    int32_t blocks_per_cu;
    int32_t refill_threshold;
    int32_t lds_tally_bytes;
    int32_t bin_cache_slots;
    int32_t chunk;
    int32_t waves_per_simd;
    int32_t grid_chunk;
    int32_t grid_walk_cells;
    int32_t vacuum_steps;
} pr_tuning;

int pr_set_tuning(pr_ctx* ctx, const pr_tuning* tuning);
int pr_get_tuning(pr_ctx* ctx, pr_tuning* tuning);

/* Pick the launch tuning for a workload by measurement: coordinate descent
 * (two passes) over refill threshold, chunk, resident blocks per CU,
 * bin-cache slots, waves per SIMD, block size and (when a scene has a daughter
 * grid) the grid claim size and the grid walk length, each candidate timed with
 * HIP events on `stream` over a sample of the workload (every simulation's
 * history count times sample_fraction, at least 1; the best claim size depends
 * on the launch's size, so 1 tunes for the full workload).  nsims = 1 tunes pr_run_histories'
 * PR_FP32_MIXED policy, nsims > 1 tunes pr_run_batch.  Trial runs score into
 * a context-owned scratch buffer and scratch statistics: the caller's tallies
 * and run statistics are untouched.  The best tuning is set on the context and
 * written to *best.  Synchronises `stream`. */
int pr_autotune(pr_ctx* ctx, const pr_sim* sims, int32_t nsims, double sample_fraction, pr_tuning* best,
                void* stream);

/* ---- results ---- */
/* Wait for the device (every stream) and copy the tally into host arrays of
 * nbins doubles each (either may be NULL); *n_hist receives the histories run
 * since the last reset.  The mean per source neutron is sum_w / n_hist. */
int pr_read_tally(pr_ctx* ctx, int32_t tally, double* sum_w, double* sum_w2, uint64_t* n_hist, size_t nbins,
                  void* stream);
/* As pr_read_tally for bins [offset, offset + count). */
int pr_read_tally_range(pr_ctx* ctx, int32_t tally, uint64_t offset, uint64_t count, double* sum_w,
                        double* sum_w2, void* stream);
int pr_reset_tally(pr_ctx* ctx, int32_t tally, void* stream);
/* Run statistics accumulated since the last pr_reset_stats (waits for the device).
 * Returns PR_ECAPPED, with *out filled in, when out->capped > 0. */
int pr_read_stats(pr_ctx* ctx, pr_run_stats* out, void* stream);
int pr_reset_stats(pr_ctx* ctx, void* stream);

#ifdef __cplusplus
}
#endif
#endif
