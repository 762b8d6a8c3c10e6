// Internal device-side layout and history-step machinery of prompt_mi355x.
//
// One history = source sample, then steps until absorption, escape, a mirror
// kill or detection.  A step locates the nearest boundary (own exit or daughter
// entry), samples a biased free flight, moves, corrects the weight and either
// collides or relocates.  The step is written once, templated on the real
// type R (double for the plain policy, float for the mixed policy) and on a
// scene view whose arrays live in global memory (plain) or LDS (mixed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/prompt_mi355x.h"

namespace prk {

constexpr int kMaxSteps = PR_MAX_STEPS;
// h / m_n in mm A / s (CODATA 2018): a neutron of wavelength lambda [A] moves at h / (m_n lambda)
constexpr double kHOverMn = 6.62607015e-34 / 1.67492749804e-27 * 1e13;
// bit of SceneT::kinds set when some volume carries a disk chopper
constexpr int kChopperBit = 8;
// bit of SceneT::kinds set when the run needs the time of flight (a chopper or a TOF tally)
constexpr int kTimeBit = 9;
constexpr int kMaxTallies = PR_MAX_TALLIES;
constexpr int kWave = 64;

// -------------------------------------------------------------------------
// Scene layout (host builds it once per geometry; arrays in device memory)
// -------------------------------------------------------------------------

// Volume with kind-specific sizes pre-digested:
//   box: s = half sides; cylinder: s = {r, h/2, -}; cyl shell: {r_in, r_out, h/2};
//   sphere: {r}; sph shell: {r_in, r_out}.
template <class R>
struct VolT {
    R c[3];
    R s[3];
    int32_t kind, axis, parent, mat;
    int32_t detector, mirror_mask, child_begin, child_count;
    int32_t mirror_model, grid;   // grid: index of the daughter grid, -1 = scan the daughter list
    // Boundary candidates of a step in this volume: item 0 is the volume itself,
    // item i (1..7) its daughter i-1 (daughters behind a grid are not items).
    // Byte k of kind_items (k = PR_BOX .. PR_SPHERE) and byte 0 of kind_items4
    // (PR_SPH_SHELL) hold the bit set of the items of that solid kind;
    // det_items the items that are detector volumes.
    // Byte 3 of kind_items4 (exit_escapes): 1 + the world's solid kind when this
    // volume is the only daughter of a vacuum, mirrorless world and is itself
    // convex (box, cylinder, sphere): a history leaving it can only fly on to the
    // world's boundary (no draws, nothing to meet), a step the leaving step takes
    // at once; 0 otherwise.
    uint32_t kind_items, kind_items4, det_items;
    R R0, Qc, alpha, mQc, W;
    // disk chopper carried by a cylinder (chop_n = 0: none); angles in radians,
    // chop_omega = 2 pi rot_freq, chop_period = 2 pi / chop_n
    int32_t chop_n;
    R chop_r, chop_omega, chop_theta0, chop_phase, chop_period;
};

// Uniform grid over the daughters of a volume with many daughters: cell c holds
// the daughters whose (padded) bounding boxes overlap it, cell_items[cell_start[
// cells_off + c] .. cell_start[cells_off + c + 1]).
template <class R>
struct GridT {
    R lo[3], hi[3], cell[3], inv_cell[3];
    int32_t n[3];
    int32_t cells_off;
};

// Material in macroscopic units (1/mm):
//   Sigma_a = sa_per_lambda * lambda, Sigma_i = si, Sigma_c = sc_k * lambda^2 * C(lambda)
// with C(lambda) = cum[J-1], J = number of Bragg edges 2d above lambda.
template <class R>
struct MatT {
    R sa_per_lambda, si, sc_k, ga, gs;
    int32_t fam_begin, nfam;
    double inv_ga, inv_gs;   // 1 / ga, 1 / gs in FP64 (weight factors of an interaction)
    // tabulated sigma_abs(lambda), sigma_inc(lambda): tab_n rows (TabT) stored in the
    // family row array at tab_begin (tab_n = 0: the 1/v law and constant sigma_inc);
    // tab_k converts barn to 1/mm for this material's number density
    int32_t tab_begin, tab_n;
    R tab_k;
};

// Bragg family tables, all materials concatenated (canonical order per material)
template <class R>
struct FamT {
    R edge;     // 2 d
    R cum;      // prefix sum of m d F^2 within the material
    R inv2d2;   // 1 / (2 d^2): cos(2 theta) = 1 - lambda^2 inv2d2
    R pad;
};

// Axis-aligned box bounds of a volume (centre, half sides), kept apart from the
// volume table so that grid navigation over many boxes reads 24 bytes per box.
template <class R>
struct BoxT {
    R c[3];
    R s[3];
};

// A grid cell item is a daughter's volume index (bits 0-27), its solid kind
// (bits 28-30) and whether it is a detector volume (bit 31).
constexpr uint32_t kItemVol = 0x0FFFFFFFu;
constexpr int kItemKindShift = 28;
constexpr uint32_t kItemDet = 0x80000000u;
__host__ __device__ inline int item_kind(uint32_t it) { return (int)((it >> kItemKindShift) & 7u); }

// A row of tabulated microscopic cross sections (b) at wavelength lam (A); rows
// share the family row array (same size and alignment as FamT).
template <class R>
struct TabT {
    R lam, sa, si, pad;
};

template <class R>
struct SceneT {
    const VolT<R>* vols;
    const MatT<R>* mats;
    const FamT<R>* fams;
    const int32_t* children;
    const GridT<R>* grids;
    const int32_t* cell_start;
    const int32_t* cell_items;
    const BoxT<R>* boxes;   // box bounds by volume index (grid scenes)
    uint32_t kinds;         // bit k set: some volume of the scene has solid kind k
};

struct SourceDev {
    int32_t kind, spectrum;
    double o[3], u[3];
    double size[2];
    double div_rad[2];
    double lam0, lam_lo, lam_hi, kT;
    double e_const;   // h^2 / (2 m_n) in eV A^2
    double slit[3], slit_size[2];   // moderator source: slit centre and sides
};

// One axis of a tally.  The FP32 copies of its range and scale are the FP64
// values rounded to nearest, as a conversion on the device would round them,
// so the FP32 policy bins with them directly.
struct TallyAxis {
    int32_t quantity, nbins;
    float lo_f, hi_f, scale_f;
    int32_t pad;
    double lo, hi, scale;   // scale = nbins / (hi - lo)
};

template <class R>
__device__ __forceinline__ void axis_range(const TallyAxis& A, R& lo, R& hi, R& scale);
template <>
__device__ __forceinline__ void axis_range<double>(const TallyAxis& A, double& lo, double& hi, double& scale) {
    lo = A.lo; hi = A.hi; scale = A.scale;
}
template <>
__device__ __forceinline__ void axis_range<float>(const TallyAxis& A, float& lo, float& hi, float& scale) {
    lo = A.lo_f; hi = A.hi_f; scale = A.scale_f;
}

// Which finished histories a tally takes, in a form one scalar load brings in:
// its trigger as a set of termination codes (plus the detector volume for a
// detection trigger) and its scattering-count filter as an inclusive range.
// Termination code under which first-collision tallies fire (the history is
// still alive then; codes 1..6 are the PR_END_* values).
constexpr int kTermFirstCollision = 7;

struct TallyHead {
    uint32_t term_mask;           // bit per termination code that triggers the tally (kTermFirstCollision included)
    int32_t volume;               // detection trigger: required final region (-1: any)
    int32_t nscat_lo, nscat_hi;   // scattering-count filter
    int32_t naxes;
    uint32_t qmask;               // quantities its axes bin (bit per PR_Q_* value)
    // The privatised copy may hold only the slice of bins whose axis fix_axis has
    // bin fix_bin (a wavelength axis under a monochromatic source: every score
    // lands there); scores outside the slice go to global memory.  -1: whole tally.
    int32_t fix_axis, fix_bin;
};

struct TallyDev {
    TallyHead head;
    int32_t lds_offset;   // privatised copy in LDS (offset in doubles), -1 = none
    int32_t cache_base;   // first slot of this tally's LDS bin cache, -1 = none
    int32_t cache_bits;   // log2 of its slot count
    int32_t lds_bins;     // bins of the privatised copy (the whole tally, or the slice)
    float beam_f[4];      // the beam direction rounded to FP32 (the FP32 policy's copy)
    TallyAxis ax[4];
    double beam[3];                  // unit vector
    double* sw;      // device storage: (sum w, sum w^2) interleaved per bin
    double* sw2;     // = sw + 1
    int64_t total;
};

enum : int { ST_HIST = 0, ST_ESC, ST_ABS, ST_KILL, ST_DET, ST_CAP, ST_OUT, ST_STEPS, ST_DRAWS, ST_SCAT, ST_N };

struct Params {
    // scene (both precisions; the mixed policy stages the float copy into LDS)
    const VolT<double>* vols_d;
    const MatT<double>* mats_d;
    const FamT<double>* fams_d;
    const VolT<float>* vols_f;
    const MatT<float>* mats_f;
    const FamT<float>* fams_f;
    const BoxT<double>* boxes_d;
    const BoxT<float>* boxes_f;
    const int32_t* children;
    const GridT<double>* grids_d;
    const GridT<float>* grids_f;
    const int32_t* cell_start;
    const int32_t* cell_items;
    int32_t n_vols, n_mats, n_fams, n_children;
    int32_t n_grids, n_cell_start, n_cell_items;
    int32_t scene_in_lds;          // mixed policy: stage the FP32 scene into LDS (else read it from global memory);
                                   // grid scenes stage all but the volume table, plus the box bounds
    int32_t has_grid;              // some volume navigates its daughters through a grid
    uint32_t kinds;                // solid kinds present in the scene (bit per kind)
    int32_t fp64;                  // persistent policy with FP64 transport (FP64 scene, read from global memory)
    SourceDev src;
    int32_t n_tallies, lds_tally_doubles;
    int32_t cache_slots;           // LDS bin-cache slots over all cached tallies (mixed policy)
    uint32_t qmask;                // quantities the tallies bin (bit per PR_Q_* value)
    TallyDev tallies[kMaxTallies];
    uint64_t seed, first, n;
    pr_history_record* records;
    unsigned long long* stats;
    unsigned long long* counter;   // history counter of the persistent policy
    int32_t refill_threshold;      // persistent policy: refill once this many lanes of a wave are idle
    int32_t chunk;                 // persistent policy: history indices a wave claims per atomic
    int32_t waves;                 // FP32 persistent policy: waves per SIMD the launched variant is built for (4 or 5)
    int32_t has_fc;                // some tally of the run fires at the first collision
    int32_t walk_cells;            // FP32 grid walks pause after this many cells (0: never)
    int32_t paired;                // FP32 without a grid: a tally scores straight into global memory, so the
                                   // wave's scores leave as paired-lane atomics (the FP64 kernels always do)
    int32_t esc;                   // 1: some volume is marked exit_escapes (the world-crossing kernels apply);
                                   // 2: FP32 fold passes (a step from material into vacuum is followed by the
                                   // vacuum step before the wave's other lanes step again); 0: neither
};

// Batched runs: many simulations (each its own geometry, source and tallies)
// in one launch.  A block works on one simulation at a time: it stages the
// simulation's FP32 scene and tallies into LDS (when they fit), its waves claim
// chunks of that simulation's histories from the simulation's own counter until
// none are left, and only then does the block flush and move on.
struct SimDev {
    // the simulation's own FP32 scene (local indices; world = volume 0)
    const VolT<float>* vols;
    const MatT<float>* mats;
    const FamT<float>* fams;
    const int32_t* children;
    const GridT<float>* grids;
    const int32_t* cell_start;
    const int32_t* cell_items;
    const BoxT<float>* boxes;
    int32_t n_vols, n_mats, n_fams, n_children, n_grids, n_cell_start, n_cell_items;
    int32_t scene_in_lds;          // stage the scene into LDS (else read it from global memory)
    int32_t tally_begin, tally_count;
    int32_t privatised;            // 1: tallies privatised in LDS at TallyDev::lds_offset; 0: LDS bin cache
    uint32_t kinds;                // solid kinds present in the scene (bit per kind)
    uint64_t first;                // history id of the simulation's first history
    uint64_t n;                    // histories
    uint64_t hist_begin;           // position of this simulation's first history in its class
    SourceDev src;
};

struct BatchParams {
    const SimDev* sims;
    const TallyDev* tallies;          // per-simulation tally entries
    const uint64_t* tally_key_base;   // per entry: bin-cache key base within its simulation
    int32_t nsims, ntallies;
    int32_t lds_tally_doubles;        // LDS tally region (privatised tallies, or bin-cache values)
    int32_t cache_bits;               // bin cache of 2^cache_bits slots (values in the tally region)
    int32_t lds_scene_bytes;          // LDS scene region
    int32_t refill_threshold;
    int32_t waves;                    // waves per SIMD the launched variant is built for (4 or 5)
    int32_t walk_cells;               // grid walks pause after this many cells (0: never)
    uint64_t total_histories, chunk, seed;
    unsigned long long* stats;
    unsigned long long* sim_next;     // per simulation: next history index to claim (zeroed per launch)
    const unsigned long long* shift;  // prepared batches: history-id offset added to every simulation (or null)
};

// -------------------------------------------------------------------------
// Precision policies
// -------------------------------------------------------------------------

template <class R>
struct M;

template <>
struct M<double> {
    static __device__ __forceinline__ double log_(double x) { return ::log(x); }
    static __device__ __forceinline__ double exp_(double x) { return ::exp(x); }
    static __device__ __forceinline__ double sqrt_(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double div_(double a, double b) { return a / b; }
    static __device__ __forceinline__ double tan_(double x) { return ::tan(x); }
    static __device__ __forceinline__ double cos_(double x) { return ::cos(x); }
    // phi = 2 pi u; (cos phi, sin phi)
    static __device__ __forceinline__ void cs2pi(double u, double* c, double* s) {
        double phi = 2.0 * 3.14159265358979323846 * u;
        *c = ::cos(phi);
        *s = ::sin(phi);
    }
    static __device__ __forceinline__ double acos_deg(double c) { return ::acos(c) * (180.0 / 3.14159265358979323846); }
    static __device__ __forceinline__ double atan2_deg(double y, double x) {
        return ::atan2(y, x) * (180.0 / 3.14159265358979323846);
    }
    static __device__ __forceinline__ double tanh_(double x) { return ::tanh(x); }
    static __device__ __forceinline__ double atan2_(double y, double x) { return ::atan2(y, x); }
    static __device__ __forceinline__ double fmod_(double x, double y) { return ::fmod(x, y); }
    // 53-bit uniform in [0,1) from two Philox words
    static __device__ __forceinline__ double uni(uint32_t a, uint32_t b) {
        return (double)(a >> 5) * (1.0 / 134217728.0) + (double)(b >> 6) * (1.0 / 9007199254740992.0);
    }
};

template <>
struct M<float> {
    // natural log from the hardware log2: arguments here are uniforms in
    // [2^-24, 1] or positive energies, never denormal
    static __device__ __forceinline__ float log_(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945f; }
    static __device__ __forceinline__ float exp_(float x) { return __expf(x); }
    // hardware square root (about 1 ulp), without the correctly rounded fix-up sequence
    static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float div_(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    static __device__ __forceinline__ float tan_(float x) { return ::tanf(x); }
    static __device__ __forceinline__ float cos_(float x) { return __cosf(x); }
    // the hardware sine/cosine take their argument in revolutions: sin(2 pi u)
    static __device__ __forceinline__ void cs2pi(float u, float* c, float* s) {
        *c = __builtin_amdgcn_cosf(u);
        *s = __builtin_amdgcn_sinf(u);
    }
    static __device__ __forceinline__ float acos_deg(float c) { return ::acosf(c) * (180.0f / 3.14159265f); }
    static __device__ __forceinline__ float atan2_deg(float y, float x) { return ::atan2f(y, x) * (180.0f / 3.14159265f); }
    static __device__ __forceinline__ float tanh_(float x) { return ::tanhf(x); }
    static __device__ __forceinline__ float atan2_(float y, float x) { return ::atan2f(y, x); }
    static __device__ __forceinline__ float fmod_(float x, float y) { return ::fmodf(x, y); }
    // 24-bit uniform in [0,1) from the first word of the pair
    static __device__ __forceinline__ float uni(uint32_t a, uint32_t) { return (float)(a >> 8) * (1.0f / 16777216.0f); }
};

// floor to an integer in the value's own precision (the floor of a float is a
// float, so FP32 needs no FP64 round trip)
template <class R>
__device__ __forceinline__ int floor_i(R x) {
    if constexpr (sizeof(R) == 4) return (int)__builtin_floorf(x);
    else return (int)__builtin_floor(x);
}

// -------------------------------------------------------------------------
// Philox4x32-10, counter = (block, history), key = seed
// -------------------------------------------------------------------------

struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 multiply-add per product gives both halves
        // (v_mad_u64_u32 instead of a mul_lo/mul_hi pair)
        const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57u;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// -------------------------------------------------------------------------
// Particle state (registers)
// -------------------------------------------------------------------------

template <class R>
struct PState {
    R p[3], u[3];
    R lam;
    double w;
    uint64_t h;
    uint64_t hash;
    uint32_t k;          // draws consumed so far (the draw index of the next draw)
    uint32_t c2, c3;     // FP64 draws: words 2,3 of the current block (odd draws)
    R ub0, ub1, ub2, ub3, ub4;   // FP32 draws: buffered uniforms for draws k .. k+nbuf-1
    int32_t nbuf;
    int32_t region, nscat, steps, term;
    // cross sections cached for material xs_mat at wavelength lam (-2: none); a
    // state must start with xs_mat = -2 before its first source()
    int32_t xs_mat, nact;
    R sa, si, sc, sig, sig_g, ga, gs, cl;
    R t;   // time since emission, s
};

// FP64 draws: the block of draw k is computed when k is even, its second word
// pair kept for the odd draw that follows.
__device__ __forceinline__ double draw(PState<double>& s, uint64_t seed) {
    uint32_t a, b;
    if ((s.k & 1u) == 0u) {
        uint32_t blk = s.k >> 1;
        U4 o = philox10(blk, 0u, (uint32_t)s.h, (uint32_t)(s.h >> 32), (uint32_t)seed, (uint32_t)(seed >> 32));
        a = o.x;
        b = o.y;
        s.c2 = o.z;
        s.c3 = o.w;
    } else {
        a = s.c2;
        b = s.c3;
    }
    s.k++;
    return M<double>::uni(a, b);
}

// FP32 draws are buffered: one generation site per step fills the buffer with
// the uniforms of the next draw indices (word 0 of a block for its even draw,
// word 2 for its odd draw), so a wave runs the Philox rounds once per step
// instead of once per draw site.  Values depend only on the draw index.
__device__ __forceinline__ void push_u(PState<float>& s, float v) {
    s.ub0 = s.nbuf == 0 ? v : s.ub0;
    s.ub1 = s.nbuf == 1 ? v : s.ub1;
    s.ub2 = s.nbuf == 2 ? v : s.ub2;
    s.ub3 = s.nbuf == 3 ? v : s.ub3;
    s.ub4 = s.nbuf == 4 ? v : s.ub4;
    s.nbuf++;
}

__device__ __forceinline__ void gen_block(PState<float>& s, uint64_t seed) {
    const uint32_t idx = s.k + (uint32_t)s.nbuf;
    U4 o = philox10(idx >> 1, 0u, (uint32_t)s.h, (uint32_t)(s.h >> 32), (uint32_t)seed, (uint32_t)(seed >> 32));
    if ((idx & 1u) == 0u) push_u(s, M<float>::uni(o.x, 0u));
    push_u(s, M<float>::uni(o.z, 0u));
}

__device__ __forceinline__ float draw(PState<float>& s, uint64_t seed) {
    if (s.nbuf == 0) gen_block(s, seed);
    const float v = s.ub0;
    s.ub0 = s.ub1;
    s.ub1 = s.ub2;
    s.ub2 = s.ub3;
    s.ub3 = s.ub4;
    s.nbuf--;
    s.k++;
    return v;
}

// next draw after prefetch() guaranteed it is buffered (FP32: no generation
// code at the call site); FP64 draws are generated at use
__device__ __forceinline__ double draw_ready(PState<double>& s, uint64_t seed) { return draw(s, seed); }
__device__ __forceinline__ float draw_ready(PState<float>& s, uint64_t) {
    const float v = s.ub0;
    s.ub0 = s.ub1;
    s.ub1 = s.ub2;
    s.ub2 = s.ub3;
    s.ub3 = s.ub4;
    s.nbuf--;
    s.k++;
    return v;
}

// make at least `need` draws available without further generation (FP32);
// FP64 draws are generated at use
__device__ __forceinline__ void prefetch(PState<double>&, uint64_t, int) {}
__device__ __forceinline__ void prefetch(PState<float>& s, uint64_t seed, int need) {
    while (s.nbuf < need) gen_block(s, seed);
}

template <bool REC>
__device__ __forceinline__ void hash_ev(uint64_t& h, int code, int arg) {
    if (!REC) return;
    uint32_t word = ((uint32_t)code << 24) | ((uint32_t)arg & 0xFFFFFFu);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        h ^= (word >> (8 * i)) & 0xFFu;
        h *= 1099511628211ull;
    }
}

enum : int { EV_SOURCE = 1, EV_ENTER = 2, EV_EXIT = 3, EV_MIRROR = 4, EV_ABS = 5, EV_INC = 6, EV_COH = 7,
             EV_ESCAPE = 8, EV_KILL = 9, EV_DETECT = 10, EV_CAPPED = 11 };

// -------------------------------------------------------------------------
// Geometry: pieces of the ray inside a solid (at most two, for shells)
// -------------------------------------------------------------------------

template <class R>
struct Pieces {
    // at most two pieces [a0,b0], [a1,b1] (shells); fa/fb are the face ids at the ends
    R a0, b0, a1, b1;
    int fa0, fb0, fa1, fb1;
    int n;
};


// component i of a 3-vector by selects (no dynamically indexed private array)
template <class R>
__device__ __forceinline__ R pick(const R v[3], int i) {
    return i == 0 ? v[0] : (i == 1 ? v[1] : v[2]);
}

template <class R>
__device__ __forceinline__ R rinf() {
    return (R)__builtin_huge_val();
}

// t-range where lo <= q + t u <= hi on one coordinate; returns false if empty
template <class R>
__device__ __forceinline__ bool slab1(R q, R u, R lo, R hi, int flo, int fhi, R& ta, R& tb, int& fa, int& fb) {
    if (u == (R)0) {
        if (q >= lo && q <= hi) {
            ta = -rinf<R>();
            tb = rinf<R>();
            fa = fb = -1;
            return true;
        }
        return false;
    }
    R t1 = M<R>::div_(lo - q, u), t2 = M<R>::div_(hi - q, u);
    if (u > (R)0) {
        ta = t1; tb = t2; fa = flo; fb = fhi;
    } else {
        ta = t2; tb = t1; fa = fhi; fb = flo;
    }
    return true;
}

// intersect [ta,tb] with [xa,xb] keeping faces; false if empty
template <class R>
__device__ __forceinline__ bool clip(R& ta, R& tb, int& fa, int& fb, R xa, R xb, int xfa, int xfb) {
    if (xa > ta) { ta = xa; fa = xfa; }
    if (xb < tb) { tb = xb; fb = xfb; }
    return ta <= tb;
}

// |q_perp + t u_perp| <= r
template <class R>
__device__ __forceinline__ bool disc_range(R qb, R qc, R ub, R uc, R r, R& ta, R& tb) {
    R A = ub * ub + uc * uc;
    R B = qb * ub + qc * uc;
    R C = qb * qb + qc * qc - r * r;
    if (A == (R)0) {
        if (C <= (R)0) { ta = -rinf<R>(); tb = rinf<R>(); return true; }
        return false;
    }
    R D = B * B - A * C;
    if (D < (R)0) return false;
    R sq = M<R>::sqrt_(D);
    ta = M<R>::div_(-B - sq, A);
    tb = M<R>::div_(-B + sq, A);
    return true;
}

template <class R>
__device__ __forceinline__ bool ball_range(const R q[3], const R u[3], R r, R& ta, R& tb) {
    R A = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    R B = q[0] * u[0] + q[1] * u[1] + q[2] * u[2];
    R C = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] - r * r;
    R D = B * B - A * C;
    if (D < (R)0) return false;
    R sq = M<R>::sqrt_(D);
    ta = M<R>::div_(-B - sq, A);
    tb = M<R>::div_(-B + sq, A);
    return true;
}

template <class R>
__device__ __forceinline__ bool cyl_range(const R q[3], const R u[3], int ax, R r, R hh, int lat, R& ta, R& tb, int& fa,
                                          int& fb) {
    const int b = ax == 0 ? 1 : (ax == 1 ? 2 : 0);
    const int c = ax == 0 ? 2 : (ax == 1 ? 0 : 1);
    R ra, rb;
    if (!disc_range<R>(pick(q, b), pick(q, c), pick(u, b), pick(u, c), r, ra, rb)) return false;
    int za, zb;
    R sa, sb;
    if (!slab1<R>(pick(q, ax), pick(u, ax), -hh, hh, 1, 2, sa, sb, za, zb)) return false;
    ta = ra; tb = rb; fa = lat; fb = lat;
    if (ra == -rinf<R>()) { fa = -1; fb = -1; }
    return clip<R>(ta, tb, fa, fb, sa, sb, za, zb);
}

// outer piece minus inner piece
template <class R>
__device__ __forceinline__ void subtract(Pieces<R>& P, R oa, R ob, int ofa, int ofb, bool has_in, R ia, R ib, int ifa,
                                         int ifb) {
    if (!has_in || ib <= oa || ia >= ob) {
        P.a0 = oa; P.b0 = ob; P.fa0 = ofa; P.fb0 = ofb; P.n = 1;
        return;
    }
    const bool lo = ia > oa, hi = ib < ob;
    // first piece: the part before the inner solid if any, else the part after it
    P.a0 = lo ? oa : ib; P.b0 = lo ? ia : ob; P.fa0 = lo ? ofa : ifb; P.fb0 = lo ? ifa : ofb;
    P.a1 = ib; P.b1 = ob; P.fa1 = ifb; P.fb1 = ofb;
    P.n = (lo ? 1 : 0) + (hi ? 1 : 0);
}

// Sliver length of the FP32 policy: about eight ulps of the largest coordinate.
// A move shorter than this may leave an FP32 position unchanged.  A ray grazing
// an edge or touching a curved surface can cut a daughter piece that short: the
// history enters the daughter, finds its exit at distance ~0, returns to the
// mother without having moved, and would find the same piece ahead again, for
// ever.  So in FP32 a move that enters a daughter and is shorter than the sliver
// length carries the position the sliver length along the direction (the weight
// and the time of flight take the true distance): a sliver piece then lies behind
// the history, which leaves the daughter at once and does not find it again.
// Every piece is entered as in FP64, however thin (a 1 um chopper disk far from
// the origin included: its mask applies); what the rule gives up is the
// attenuation of at most one sliver length of path per such entry.  FP64 needs no
// such rule.
template <class R>
__device__ __forceinline__ R sliver_tol(const R p[3]) {
    if constexpr (sizeof(R) == 4)   // 3 * 2^-20 * max |coordinate| (one max3 and one multiply)
        return __builtin_fmaxf(__builtin_fmaxf(__builtin_fabsf(p[0]), __builtin_fabsf(p[1])), __builtin_fabsf(p[2])) *
               2.86102294921875e-06f;
    else
        return (R)0;
}

// FP32: after a move of length x that ended at a paused grid walk's virtual
// boundary, advance the position to at least the sliver length along the
// direction (no surface lies there).  Only lanes taking that branch pay.
__device__ __forceinline__ void sliver_advance(PState<float>& s, float x) {
    const float tol = sliver_tol<float>(s.p);
    if (x < tol) {
        const float e = tol - x;
        s.p[0] += e * s.u[0];
        s.p[1] += e * s.u[1];
        s.p[2] += e * s.u[2];
    }
}
__device__ __forceinline__ void sliver_advance(PState<double>&, double) {}

// distance to where the ray enters a daughter's first piece ahead (rinf: none)
template <class R>
__device__ __forceinline__ R entry_distance(const Pieces<R>& P) {
    if (P.n > 0 && P.a0 > (R)0) return P.a0;
    if (P.n > 1 && P.a1 > (R)0) return P.a1;
    return rinf<R>();
}

template <class R>
__device__ __forceinline__ void box_pieces(const R q[3], const R u[3], const R h[3], Pieces<R>& P) {
    P.n = 0;
    R ta = -rinf<R>(), tb = rinf<R>();
    int fa = -1, fb = -1;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        R xa, xb;
        int xfa, xfb;
        if (!slab1<R>(q[k], u[k], -h[k], h[k], 2 * k, 2 * k + 1, xa, xb, xfa, xfb)) return;
        if (!clip<R>(ta, tb, fa, fb, xa, xb, xfa, xfb)) return;
    }
    P.a0 = ta; P.b0 = tb; P.fa0 = fa; P.fb0 = fb; P.n = 1;
}

template <class R>
__device__ __forceinline__ void pieces(const VolT<R>& V, const R p[3], const R u[3], Pieces<R>& P);

// pieces of a grid daughter: boxes from the compact box table, other kinds
// from the volume table
template <class R>
__device__ __forceinline__ void item_pieces(const SceneT<R>& S, uint32_t it, const R p[3], const R u[3], Pieces<R>& P) {
    const int c = (int)(it & kItemVol);
    if (item_kind(it) == PR_BOX) {
        const BoxT<R>& B = S.boxes[c];
        R q[3] = {p[0] - B.c[0], p[1] - B.c[1], p[2] - B.c[2]};
        box_pieces<R>(q, u, B.s, P);
    } else {
        pieces<R>(S.vols[c], p, u, P);
    }
}

// pieces of the ray p + t u inside a solid of compile-time kind K
template <class R, int K>
__device__ __forceinline__ void pieces_kind(const VolT<R>& V, const R p[3], const R u[3], Pieces<R>& P) {
    R q[3] = {p[0] - V.c[0], p[1] - V.c[1], p[2] - V.c[2]};
    P.n = 0;
    if (K == PR_BOX) {
        box_pieces<R>(q, u, V.s, P);
    } else if (K == PR_CYLINDER) {
        R ta, tb;
        int fa, fb;
        if (!cyl_range<R>(q, u, V.axis, V.s[0], V.s[1], 0, ta, tb, fa, fb)) return;
        P.a0 = ta; P.b0 = tb; P.fa0 = fa; P.fb0 = fb; P.n = 1;
    } else if (K == PR_CYL_SHELL) {
        R oa, ob, ia, ib;
        int ofa, ofb, ifa, ifb;
        if (!cyl_range<R>(q, u, V.axis, V.s[1], V.s[2], 0, oa, ob, ofa, ofb)) return;
        bool hin = cyl_range<R>(q, u, V.axis, V.s[0], V.s[2], 3, ia, ib, ifa, ifb);
        subtract<R>(P, oa, ob, ofa, ofb, hin, ia, ib, ifa, ifb);
    } else if (K == PR_SPHERE) {
        R ta, tb;
        if (!ball_range<R>(q, u, V.s[0], ta, tb)) return;
        P.a0 = ta; P.b0 = tb; P.fa0 = 0; P.fb0 = 0; P.n = 1;
    } else {  // spherical shell
        R oa, ob, ia, ib;
        if (!ball_range<R>(q, u, V.s[1], oa, ob)) return;
        bool hin = ball_range<R>(q, u, V.s[0], ia, ib);
        subtract<R>(P, oa, ob, 0, 0, hin, ia, ib, 3, 3);
    }
}

template <class R>
__device__ __forceinline__ void pieces(const VolT<R>& V, const R p[3], const R u[3], Pieces<R>& P) {
    P.n = 0;
    switch (V.kind) {
    case PR_BOX: pieces_kind<R, PR_BOX>(V, p, u, P); return;
    case PR_CYLINDER: pieces_kind<R, PR_CYLINDER>(V, p, u, P); return;
    case PR_CYL_SHELL: pieces_kind<R, PR_CYL_SHELL>(V, p, u, P); return;
    case PR_SPHERE: pieces_kind<R, PR_SPHERE>(V, p, u, P); return;
    default: pieces_kind<R, PR_SPH_SHELL>(V, p, u, P); return;
    }
}

template <class R>
__device__ __forceinline__ bool contains(const VolT<R>& V, const R p[3]) {
    R q[3] = {p[0] - V.c[0], p[1] - V.c[1], p[2] - V.c[2]};
    switch (V.kind) {
    case PR_BOX:
        return __builtin_fabs((double)q[0]) <= (double)V.s[0] && __builtin_fabs((double)q[1]) <= (double)V.s[1] &&
               __builtin_fabs((double)q[2]) <= (double)V.s[2];
    case PR_CYLINDER:
    case PR_CYL_SHELL: {
        const int a = V.axis, b = a == 0 ? 1 : (a == 1 ? 2 : 0), c = a == 0 ? 2 : (a == 1 ? 0 : 1);
        const R qa = pick(q, a), qb = pick(q, b), qc = pick(q, c);
        R rho2 = qb * qb + qc * qc;
        R hh = V.kind == PR_CYLINDER ? V.s[1] : V.s[2];
        R ro = V.kind == PR_CYLINDER ? V.s[0] : V.s[1];
        bool in = rho2 <= ro * ro && (qa <= hh && qa >= -hh);
        if (V.kind == PR_CYL_SHELL) in = in && rho2 >= V.s[0] * V.s[0];
        return in;
    }
    case PR_SPHERE:
        return q[0] * q[0] + q[1] * q[1] + q[2] * q[2] <= V.s[0] * V.s[0];
    default: {
        R r2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
        return r2 >= V.s[0] * V.s[0] && r2 <= V.s[1] * V.s[1];
    }
    }
}

template <class R>
__device__ __forceinline__ bool item_contains(const SceneT<R>& S, uint32_t it, const R p[3]) {
    const int c = (int)(it & kItemVol);
    if (item_kind(it) == PR_BOX) {
        const BoxT<R>& B = S.boxes[c];
        const R q[3] = {p[0] - B.c[0], p[1] - B.c[1], p[2] - B.c[2]};
        return __builtin_fabs((double)q[0]) <= (double)B.s[0] && __builtin_fabs((double)q[1]) <= (double)B.s[1] &&
               __builtin_fabs((double)q[2]) <= (double)B.s[2];
    }
    return contains<R>(S.vols[c], p);
}

// outward normal of face f at point p
template <class R>
__device__ __forceinline__ void normal(const VolT<R>& V, int f, const R p[3], R n[3]) {
    if (V.kind == PR_BOX) {
        const int k = f >> 1;
        const R sg = (f & 1) ? (R)1 : (R)-1;
        n[0] = k == 0 ? sg : (R)0;
        n[1] = k == 1 ? sg : (R)0;
        n[2] = k == 2 ? sg : (R)0;
        return;
    }
    R q[3] = {p[0] - V.c[0], p[1] - V.c[1], p[2] - V.c[2]};
    if (V.kind == PR_CYLINDER || V.kind == PR_CYL_SHELL) {
        const int a = V.axis, b = a == 0 ? 1 : (a == 1 ? 2 : 0), c = a == 0 ? 2 : (a == 1 ? 0 : 1);
        R na = (R)0, nb = (R)0, nc = (R)0;
        if (f == 1 || f == 2) {
            na = f == 2 ? (R)1 : (R)-1;
        } else {
            const R qb = pick(q, b), qc = pick(q, c);
            R r = M<R>::sqrt_(qb * qb + qc * qc);
            R sg = f == 3 ? (R)-1 : (R)1;
            nb = sg * M<R>::div_(qb, r);
            nc = sg * M<R>::div_(qc, r);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) n[k] = k == a ? na : (k == b ? nb : nc);
        return;
    }
    R r = M<R>::sqrt_(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    R sg = f == 3 ? (R)-1 : (R)1;
#pragma unroll
    for (int k = 0; k < 3; ++k) n[k] = sg * M<R>::div_(q[k], r);
}

// Disk chopper mask at crossing point p and time t: polar angle about the disk
// axis (from the next axis towards the one after), disk turned by phase + omega t;
// open outside the black inner radius and within theta0 after a window start.
template <class R>
__device__ __forceinline__ bool chopper_open(const VolT<R>& V, const R p[3], R t) {
    const int a = V.axis, b = a == 0 ? 1 : (a == 1 ? 2 : 0), c = a == 0 ? 2 : (a == 1 ? 0 : 1);
    const R qb = pick(p, b) - pick(V.c, b), qc = pick(p, c) - pick(V.c, c);
    const R rho = M<R>::sqrt_(qb * qb + qc * qc);
    if (rho < V.chop_r) return false;
    const R ang = M<R>::atan2_(qc, qb) - V.chop_phase - V.chop_omega * t;
    R m = M<R>::fmod_(ang, V.chop_period);
    if (m < (R)0) m += V.chop_period;
    return m < V.chop_theta0;
}

template <class R>
__device__ __forceinline__ R reflectivity(const VolT<R>& V, R Q) {
    if (Q <= V.Qc) return V.R0;
    R r;
    if (V.mirror_model == PR_MIRROR_TANH) {
        r = (R)0.5 * V.R0 * ((R)1 - V.alpha * (Q - V.Qc)) * ((R)1 - M<R>::tanh_(M<R>::div_(Q - V.mQc, V.W)));
    } else {
        if (Q > V.mQc) return (R)0;
        r = V.R0 - V.alpha * (Q - V.Qc);
    }
    return r > (R)0 ? r : (R)0;
}

// innermost volume containing p below the world volume `root`, -1 outside it
template <class R, bool GRID>
__device__ __forceinline__ int locate(const SceneT<R>& S, const R p[3], int root) {
    if (!contains<R>(S.vols[root], p)) return -1;
    int cur = root;
    for (int depth = 0; depth < 64; ++depth) {
        const VolT<R>& V = S.vols[cur];
        int next = -1;
        if (GRID && V.grid >= 0) {
            // only the daughters listed in the grid cell holding p can contain it
            const GridT<R>& G = S.grids[V.grid];
            bool in = true;
            int cell = 0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                in = in && p[k] >= G.lo[k] && p[k] <= G.hi[k];
                int i = floor_i<R>((p[k] - G.lo[k]) * G.inv_cell[k]);
                i = i < 0 ? 0 : (i >= G.n[k] ? G.n[k] - 1 : i);
                cell = cell * G.n[k] + i;
            }
            if (in) {
                const int je = S.cell_start[G.cells_off + cell + 1];
                for (int j = S.cell_start[G.cells_off + cell]; j < je; ++j) {
                    const uint32_t it = (uint32_t)S.cell_items[j];
                    if (item_contains<R>(S, it, p)) { next = (int)(it & kItemVol); break; }
                }
            }
        } else {
            for (int i = 0; i < V.child_count; ++i) {
                int c = S.children[V.child_begin + i];
                if (contains<R>(S.vols[c], p)) { next = c; break; }
            }
        }
        if (next < 0) break;
        cur = next;
    }
    return cur;
}

// -------------------------------------------------------------------------
// Source
// -------------------------------------------------------------------------

template <class R, bool REC, bool GRID>
__device__ __forceinline__ void source(PState<R>& s, const SourceDev& src, const SceneT<R>& S, uint64_t seed, uint64_t h,
                                       int root, int start_region = -2) {
    s.h = h;
    s.k = 0;
    s.nbuf = 0;
    s.w = 1.0;
    s.t = (R)0;
    s.nscat = 0;
    s.steps = 0;
    s.term = 0;
    s.hash = 14695981039346656037ull;
    R p[3] = {(R)src.o[0], (R)src.o[1], (R)src.o[2]};
    R u[3] = {(R)src.u[0], (R)src.u[1], (R)src.u[2]};
    if (src.kind != PR_PENCIL) {
        R a = draw(s, seed);
        R b = draw(s, seed);
        p[0] += (a - (R)0.5) * (R)src.size[0];
        p[1] += (b - (R)0.5) * (R)src.size[1];
    }
    if (src.kind == PR_MODERATOR) {
        // the direction joins the source point to a uniform point of the slit
        R a = draw(s, seed);
        R b = draw(s, seed);
        R v[3] = {(R)src.slit[0] + (a - (R)0.5) * (R)src.slit_size[0] - p[0],
                  (R)src.slit[1] + (b - (R)0.5) * (R)src.slit_size[1] - p[1], (R)src.slit[2] - p[2]};
        R nrm = M<R>::sqrt_(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        u[0] = M<R>::div_(v[0], nrm);
        u[1] = M<R>::div_(v[1], nrm);
        u[2] = M<R>::div_(v[2], nrm);
    }
    if (src.kind == PR_RECT_DIVERGENT) {
        R ax = ((R)2 * draw(s, seed) - (R)1) * (R)src.div_rad[0];
        R ay = ((R)2 * draw(s, seed) - (R)1) * (R)src.div_rad[1];
        R tx = M<R>::tan_(ax), ty = M<R>::tan_(ay);
        R nrm = M<R>::sqrt_(tx * tx + ty * ty + (R)1);
        u[0] = M<R>::div_(tx, nrm);
        u[1] = M<R>::div_(ty, nrm);
        u[2] = M<R>::div_((R)1, nrm);
    }
    R lam = (R)src.lam0;
    if (src.spectrum == PR_UNIFORM) {
        lam = (R)src.lam_lo + draw(s, seed) * (R)(src.lam_hi - src.lam_lo);
    } else if (src.spectrum == PR_MAXWELL) {
        // Gamma(3/2) energy in units of kT: exponential + half a squared normal
        for (int t = 0; t < 64; ++t) {
            R x1 = (R)1 - draw(s, seed);
            R x2 = (R)1 - draw(s, seed);
            R u3 = draw(s, seed);
            R c = M<R>::cos_((R)(0.5 * 3.14159265358979323846) * u3);
            R e = (R)src.kT * (-M<R>::log_(x1) - M<R>::log_(x2) * c * c);
            lam = M<R>::sqrt_(M<R>::div_((R)src.e_const, e));
            if (lam >= (R)src.lam_lo && lam <= (R)src.lam_hi) break;
            if (t == 63) lam = lam < (R)src.lam_lo ? (R)src.lam_lo : (R)src.lam_hi;
        }
    }
    for (int i = 0; i < 3; ++i) {
        s.p[i] = p[i];
        s.u[i] = u[i];
    }
    // the cached cross sections depend on (material, lambda) only: a lane keeps
    // them from its previous history when the wavelength is the same
    if (!(lam == s.lam)) s.xs_mat = -2;
    s.lam = lam;
    // start_region >= -1: the caller located this (fixed) source point already
    s.region = start_region >= -1 ? start_region : locate<R, GRID>(S, s.p, root);
    hash_ev<REC>(s.hash, EV_SOURCE, s.region);
    if (s.region < 0) s.term = PR_END_OUTSIDE;
}

// -------------------------------------------------------------------------
// Cross sections at the history's wavelength (cached per material)
// -------------------------------------------------------------------------

template <class R>
__device__ __forceinline__ void load_xs(PState<R>& s, const SceneT<R>& S, int mat) {
    const MatT<R>& Mt = S.mats[mat];
    // J = number of edges 2d > lambda (edges non-increasing): binary search
    int lo = 0, hi = Mt.nfam;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (S.fams[Mt.fam_begin + mid].edge > s.lam) lo = mid + 1; else hi = mid;
    }
    s.nact = lo;
    R cl = lo > 0 ? S.fams[Mt.fam_begin + lo - 1].cum : (R)0;
    s.cl = cl;
    s.ga = Mt.ga;
    s.gs = Mt.gs;
    R sa = Mt.sa_per_lambda * s.lam, si = Mt.si;
    if (Mt.tab_n > 0) {
        // linear interpolation between the rows around lambda, constant beyond the ends
        const TabT<R>* T = (const TabT<R>*)(S.fams + Mt.tab_begin);
        const int n = Mt.tab_n;
        const R v = s.lam;
        R a, b;
        if (v <= T[0].lam) {
            a = T[0].sa;
            b = T[0].si;
        } else if (v >= T[n - 1].lam) {
            a = T[n - 1].sa;
            b = T[n - 1].si;
        } else {
            int l = 0, h = n - 1;   // first row with lam >= v
            while (l < h) {
                const int mid = (l + h) >> 1;
                if (T[mid].lam < v) l = mid + 1; else h = mid;
            }
            const TabT<R>& r0 = T[l - 1];
            const TabT<R>& r1 = T[l];
            a = r0.sa + M<R>::div_((r1.sa - r0.sa) * (v - r0.lam), r1.lam - r0.lam);
            b = r0.si + M<R>::div_((r1.si - r0.si) * (v - r0.lam), r1.lam - r0.lam);
        }
        sa = Mt.tab_k * a;
        si = Mt.tab_k * b;
    }
    s.sa = Mt.ga > (R)0 ? sa : (R)0;
    s.si = Mt.gs > (R)0 ? si : (R)0;
    s.sc = Mt.gs > (R)0 ? Mt.sc_k * s.lam * s.lam * cl : (R)0;
    s.sig = s.sa + s.si + s.sc;
    s.sig_g = s.ga * s.sa + s.gs * (s.si + s.sc);
    s.xs_mat = mat;
}

// -------------------------------------------------------------------------
// Nearest daughter entry through a uniform grid (3-D DDA over the cells the
// ray crosses inside the grid box, up to tmax; stops once the best entry found
// lies within the cells already visited)
// -------------------------------------------------------------------------

// walk_cells > 0 (FP32): after that many cells without a definitive answer the
// walk pauses and d_pause receives the far wall of the last cell visited; the
// step then moves there without an event (a virtual boundary) and the next step
// walks on from there, so a wave no longer waits for its longest walk.  The
// free flight is memoryless, so pausing changes no expectation.
template <class R>
__device__ __forceinline__ void grid_nearest(const SceneT<R>& S, const GridT<R>& G, const R p[3], const R u[3], R tmax,
                                             int walk_cells, R& d_child, int& child, int& child_det, R& d_pause) {
    R t0 = (R)0, t1 = tmax;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (u[k] == (R)0) {
            if (p[k] < G.lo[k] || p[k] > G.hi[k]) return;
        } else {
            R ta = M<R>::div_(G.lo[k] - p[k], u[k]), tb = M<R>::div_(G.hi[k] - p[k], u[k]);
            if (ta > tb) { R t = ta; ta = tb; tb = t; }
            t0 = ta > t0 ? ta : t0;
            t1 = tb < t1 ? tb : t1;
        }
    }
    if (t0 > t1) return;
    int ix[3], st[3];
    R tn[3], td[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const R x = p[k] + t0 * u[k];
        int i = floor_i<R>((x - G.lo[k]) * G.inv_cell[k]);
        i = i < 0 ? 0 : (i >= G.n[k] ? G.n[k] - 1 : i);
        ix[k] = i;
        if (u[k] > (R)0) {
            st[k] = 1;
            tn[k] = M<R>::div_(G.lo[k] + (R)(i + 1) * G.cell[k] - p[k], u[k]);
            td[k] = M<R>::div_(G.cell[k], u[k]);
        } else if (u[k] < (R)0) {
            st[k] = -1;
            tn[k] = M<R>::div_(G.lo[k] + (R)i * G.cell[k] - p[k], u[k]);
            td[k] = M<R>::div_(-G.cell[k], u[k]);
        } else {
            st[k] = 0;
            tn[k] = rinf<R>();
            td[k] = rinf<R>();
        }
    }
    const int max_cells = G.n[0] + G.n[1] + G.n[2] + 3;
    for (int it = 0; it < max_cells; ++it) {
        const int cell = (ix[0] * G.n[1] + ix[1]) * G.n[2] + ix[2];
        const int jb = S.cell_start[G.cells_off + cell], je = S.cell_start[G.cells_off + cell + 1];
        for (int j = jb; j < je; ++j) {
            const uint32_t item = (uint32_t)S.cell_items[j];
            Pieces<R> Q;
            item_pieces<R>(S, item, p, u, Q);
            const R a = entry_distance<R>(Q);
            if (a < d_child) {
                d_child = a;
                child = (int)(item & kItemVol);
                child_det = (item & kItemDet) ? 1 : 0;
            }
        }
        // leave through the nearest cell wall (selects, no indexed private arrays)
        const bool ax0 = tn[0] <= tn[1] && tn[0] <= tn[2];
        const bool ax1 = !ax0 && tn[1] <= tn[2];
        const R tc = ax0 ? tn[0] : (ax1 ? tn[1] : tn[2]);
        if (d_child <= tc || tc > t1) break;
        if (it + 1 == walk_cells) {
            d_pause = tc;
            break;
        }
        if (ax0) { ix[0] += st[0]; tn[0] += td[0]; }
        else if (ax1) { ix[1] += st[1]; tn[1] += td[1]; }
        else { ix[2] += st[2]; tn[2] += td[2]; }
        if (ix[0] < 0 || ix[0] >= G.n[0] || ix[1] < 0 || ix[1] >= G.n[1] || ix[2] < 0 || ix[2] >= G.n[2]) break;
    }
}

// -------------------------------------------------------------------------
// One step of the history loop
// -------------------------------------------------------------------------

// Boundary candidates of kind K for this lane (bit set `items`, see VolT): the
// exit of the lane's own volume (item 0) and the entry into its daughters.  The
// loop runs while any lane of the wave has an item of kind K left, so the kind's
// intersection code is executed once per round for all those lanes together.
// A daughter is entered at the start of its first piece ahead (a > 0); among
// equal entry distances the lower daughter index wins, as in a scan in order.
template <class R, int K, class ST>
__device__ __forceinline__ void scan_kind(const SceneT<R>& S, const VolT<R>& V, const ST& s, uint32_t items, R& d_exit,
                                          int& face, R& d_child, int& child, int& child_item, int& child_det) {
    if (((S.kinds >> K) & 1u) == 0u) return;
    while (__ballot(items != 0u) != 0ull) {
        if (items != 0u) {
            const int i = __builtin_ctz(items);
            items &= items - 1u;
            const int vid = i == 0 ? s.region : S.children[V.child_begin + i - 1];
            Pieces<R> P;
            pieces_kind<R, K>(S.vols[vid], s.p, s.u, P);
            if (i == 0) {
                if (P.n > 0 && P.b0 > (R)0) { d_exit = P.b0; face = P.fb0; }
                if (P.n > 1 && P.b1 > (R)0 && P.b1 < d_exit) { d_exit = P.b1; face = P.fb1; }
            } else {
                const R a = entry_distance<R>(P);
                if (a < d_child || (a == d_child && a != rinf<R>() && i < child_item)) {
                    d_child = a;
                    child = vid;
                    child_item = i;
                    child_det = (int)((V.det_items >> i) & 1u);
                }
            }
        }
    }
}


// Distance to where the ray leaves volume W from inside it (the end of its first
// piece ahead; 0 when none), exactly as a step's boundary scan finds it for the
// volume itself.  kind: W's solid kind (box, cylinder or sphere).
template <class R>
__device__ __forceinline__ R own_exit(const VolT<R>& W, int kind, const R p[3], const R u[3]) {
    Pieces<R> P;
    P.n = 0;
    if (kind == PR_BOX) pieces_kind<R, PR_BOX>(W, p, u, P);
    else if (kind == PR_CYLINDER) pieces_kind<R, PR_CYLINDER>(W, p, u, P);
    else pieces_kind<R, PR_SPHERE>(W, p, u, P);
    R d = rinf<R>();
    if (P.n > 0 && P.b0 > (R)0) d = P.b0;
    if (P.n > 1 && P.b1 > (R)0 && P.b1 < d) d = P.b1;
    return d == rinf<R>() ? (R)0 : d;
}

// One step; returns true when the step was the history's first collision
// (absorption or scattering), the event of first-collision tallies.  ESC == 1:
// a history leaving a volume marked exit_escapes takes the world crossing that
// follows in the same step (kernels built without it leave that to the next
// step; the history is the same either way, short of rounding on a ray that
// grazes the daughter as it leaves, where the next step could find a re-entry).
template <class R, bool REC, bool GRID, int ESC = 0>
__device__ __forceinline__ bool step(PState<R>& s, const SceneT<R>& S, uint64_t seed, int walk_cells = 0) {
    if (s.steps >= kMaxSteps) {
        s.term = PR_END_CAPPED;
        hash_ev<REC>(s.hash, EV_CAPPED, 0);
        return false;
    }
    s.steps++;
    const VolT<R>& V = S.vols[s.region];

    // nearest boundary: leave this volume, or enter a daughter.  The candidate
    // solids are taken one solid kind at a time over the whole wave, so lanes in
    // different volumes that need the same kind of intersection run it together.
    R d_exit = rinf<R>();
    int face = -1;
    R d_child = rinf<R>();
    int child = -1, child_item = 0, child_det = 0;
    scan_kind<R, PR_BOX>(S, V, s, V.kind_items & 0xFFu, d_exit, face, d_child, child, child_item, child_det);
    scan_kind<R, PR_CYLINDER>(S, V, s, (V.kind_items >> 8) & 0xFFu, d_exit, face, d_child, child, child_item, child_det);
    scan_kind<R, PR_CYL_SHELL>(S, V, s, (V.kind_items >> 16) & 0xFFu, d_exit, face, d_child, child, child_item, child_det);
    scan_kind<R, PR_SPHERE>(S, V, s, V.kind_items >> 24, d_exit, face, d_child, child, child_item, child_det);
    scan_kind<R, PR_SPH_SHELL>(S, V, s, V.kind_items4 & 0xFFu, d_exit, face, d_child, child, child_item, child_det);
    if (d_exit == rinf<R>()) { d_exit = (R)0; face = -1; }
    R d_pause = rinf<R>();
    if (GRID && V.grid >= 0)
        grid_nearest<R>(S, S.grids[V.grid], s.p, s.u, d_exit, sizeof(R) == 4 ? walk_cells : 0, d_child, child,
                        child_det, d_pause);
    bool to_child = d_child < d_exit;
    R d_b = to_child ? d_child : d_exit;
    // a paused grid walk (FP32): the far wall of its last cell is a virtual boundary
    const bool pause = GRID && d_pause < d_b;
    if (pause) {
        d_b = d_pause;
        to_child = false;
    }

    R sig = (R)0, sig_g = (R)0;
    if (V.mat >= 0) {
        if (s.xs_mat != V.mat) load_xs<R>(s, S, V.mat);
        sig = s.sig;
        sig_g = s.sig_g;
    }

    bool collide = false;
    R x = d_b;
    if (sig_g > (R)0) {
        prefetch(s, seed, 4);   // flight, process and two scattering draws
        R xi = (R)1 - draw_ready(s, seed);
        R l = M<R>::div_(-M<R>::log_(xi), sig_g);
        if (l < d_b) { collide = true; x = l; }
    }
    // FP32: an entry move shorter than the sliver length carries the position the
    // sliver length (see sliver_tol); weight and time take x
    R xm = x;
    if constexpr (sizeof(R) == 4) {
        if (!collide && to_child) xm = __builtin_fmaxf(x, sliver_tol<R>(s.p));
    }
    s.p[0] += xm * s.u[0];
    s.p[1] += xm * s.u[1];
    s.p[2] += xm * s.u[2];
    if ((S.kinds >> kTimeBit) & 1u) s.t += M<R>::div_(x * s.lam, (R)kHOverMn);
    if (sig_g > (R)0) s.w *= (double)M<R>::exp_((sig_g - sig) * x);

    if (collide) {
        R r = draw_ready(s, seed) * sig_g;
        R wa = s.ga * s.sa, wi = s.gs * s.si, wc = s.gs * s.sc;
        if (r < wa || wi + wc == (R)0) {
            s.w *= S.mats[s.xs_mat].inv_ga;
            s.term = PR_END_ABSORB;
            hash_ev<REC>(s.hash, EV_ABS, 0);
            return s.nscat == 0;
        }
        s.w *= S.mats[s.xs_mat].inv_gs;
        bool inc = r < wa + wi || wc == (R)0 || s.nact == 0;
        R u1 = draw_ready(s, seed);
        R u2 = draw_ready(s, seed);
        R c2t;
        int fam = 0;
        if (inc) {
            c2t = (R)2 * u1 - (R)1;
        } else {
            // family j: first with cumulative m d F^2 above u1 * C(lambda)
            const MatT<R>& Mt = S.mats[s.xs_mat];
            R cut = u1 * s.cl;
            int lo = 0, hi = s.nact - 1;
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if (S.fams[Mt.fam_begin + mid].cum > cut) hi = mid; else lo = mid + 1;
            }
            fam = lo;
            c2t = (R)1 - s.lam * s.lam * S.fams[Mt.fam_begin + fam].inv2d2;
        }
        R s2t = M<R>::sqrt_((R)1 - c2t * c2t);
        R cp, sp;
        M<R>::cs2pi(u2, &cp, &sp);
        R nu[3];
        if (inc) {
            // isotropic: polar axis z of the laboratory frame
            nu[0] = s2t * cp;
            nu[1] = s2t * sp;
            nu[2] = c2t;
            hash_ev<REC>(s.hash, EV_INC, 0);
        } else {
            // Debye-Scherrer cone about the incoming direction
            R ax0 = __builtin_fabs((double)s.u[0]) < 0.9 ? (R)1 : (R)0;
            R ax1 = (R)1 - ax0;
            // e1 = u x a (a = x or y), normalised; e2 = u x e1
            R e1[3] = {-s.u[2] * ax1, s.u[2] * ax0, s.u[0] * ax1 - s.u[1] * ax0};
            R inv = M<R>::div_((R)1, M<R>::sqrt_(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]));
            e1[0] *= inv; e1[1] *= inv; e1[2] *= inv;
            R e2[3] = {s.u[1] * e1[2] - s.u[2] * e1[1], s.u[2] * e1[0] - s.u[0] * e1[2], s.u[0] * e1[1] - s.u[1] * e1[0]};
#pragma unroll
            for (int k = 0; k < 3; ++k) nu[k] = c2t * s.u[k] + s2t * (cp * e1[k] + sp * e2[k]);
            hash_ev<REC>(s.hash, EV_COH, fam);
        }
        s.u[0] = nu[0];
        s.u[1] = nu[1];
        s.u[2] = nu[2];
        s.nscat++;
        return s.nscat == 1;
    }

    if (pause) {   // no event: the next step walks on from here
        sliver_advance(s, x);
        return false;
    }
    if (to_child) {
        s.region = child;
        hash_ev<REC>(s.hash, EV_ENTER, child);
        if (child_det) {
            s.term = PR_END_DETECT;
            hash_ev<REC>(s.hash, EV_DETECT, child);
        } else if ((S.kinds >> kChopperBit) & 1u) {
            const VolT<R>& C = S.vols[child];
            if (C.chop_n > 0 && !chopper_open<R>(C, s.p, s.t)) {
                // ray-tracing mask of the disk chopper: 0 outside an open window
                s.w = 0.0;
                s.term = PR_END_KILL;
                hash_ev<REC>(s.hash, EV_KILL, 0);
            }
        }
        return false;
    }
    if (face >= 0 && ((V.mirror_mask >> face) & 1)) {
        R n[3];
        normal<R>(V, face, s.p, n);
        R un = s.u[0] * n[0] + s.u[1] * n[1] + s.u[2] * n[2];
        R Q = M<R>::div_((R)(4.0 * 3.14159265358979323846) * (R)__builtin_fabs((double)un), s.lam);
        R refl = reflectivity<R>(V, Q);
        s.w *= (double)refl;
#pragma unroll
        for (int k = 0; k < 3; ++k) s.u[k] = s.u[k] - (R)2 * n[k] * un;
        hash_ev<REC>(s.hash, EV_MIRROR, face);
        if (!(s.w > 0.0)) {
            s.term = PR_END_KILL;
            hash_ev<REC>(s.hash, EV_KILL, 0);
        }
        return false;
    }
    if (V.parent < 0) {   // leaving a world volume
        s.term = PR_END_ESCAPE;
        hash_ev<REC>(s.hash, EV_ESCAPE, 0);
        return false;
    }
    s.region = V.parent;
    hash_ev<REC>(s.hash, EV_EXIT, s.region);
    const int exit_escapes = (int)(V.kind_items4 >> 24);
    if (ESC == 1 && exit_escapes && s.steps < kMaxSteps) {
        // the next step can only cross the vacuum world to its boundary: take it
        // now, as that step would (same distance, move and time; the step cap is
        // left to the next step)
        s.steps++;
        const R xw = own_exit<R>(S.vols[s.region], exit_escapes - 1, s.p, s.u);
        s.p[0] += xw * s.u[0];
        s.p[1] += xw * s.u[1];
        s.p[2] += xw * s.u[2];
        if ((S.kinds >> kTimeBit) & 1u) s.t += M<R>::div_(xw * s.lam, (R)kHOverMn);
        s.term = PR_END_ESCAPE;
        hash_ev<REC>(s.hash, EV_ESCAPE, 0);
    }
    return false;
}

// -------------------------------------------------------------------------
// Tally bin of a finished history (-1: not scored)
// -------------------------------------------------------------------------

// Divergence angles of a finished history (they do not depend on the tally),
// computed once per scoring pass and only when some tally of the launch bins
// them: qmask is uniform, so the guards are scalar branches.
template <class R>
struct HistAngles {
    R divx, divy;
};

template <class R>
__device__ __forceinline__ HistAngles<R> hist_angles(const PState<R>& s, uint32_t qmask) {
    HistAngles<R> q{(R)0, (R)0};
    if (qmask & (1u << PR_Q_DIVX)) q.divx = M<R>::atan2_deg(s.u[0], s.u[2]);
    if (qmask & (1u << PR_Q_DIVY)) q.divy = M<R>::atan2_deg(s.u[1], s.u[2]);
    return q;
}

template <class R>
__device__ __forceinline__ R beam_component(const TallyDev& T, int k);
template <>
__device__ __forceinline__ double beam_component<double>(const TallyDev& T, int k) { return T.beam[k]; }
template <>
__device__ __forceinline__ float beam_component<float>(const TallyDev& T, int k) { return T.beam_f[k]; }

// A score's bin: -1 when not scored; otherwise the flat index over all axes,
// except for a tally privatised as a slice (fix_axis >= 0), where it is the
// index within the slice, or the flat index with kOffSlice set for a bin outside
// the slice.
constexpr int64_t kOffSlice = 1ll << 62;

// term: the history's termination code, or kTermFirstCollision at its first
// collision.  q: the history's divergence angles, computed once for all tallies
// (PRE), or left to each divergence axis to compute (fewer values live across
// the loop).  SLICED: the tally is privatised as a slice (a separate instance,
// so that the bins of other tallies carry none of the slice arithmetic).
// UNROLL: the axis loop unrolled (the batch kernels, short of registers, keep it
// rolled).
template <class R, bool PRE, bool SLICED, bool UNROLL = true>
__device__ __forceinline__ int64_t tally_bin_t(const TallyDev& T, const PState<R>& s, int term, const HistAngles<R>& q) {
    const TallyHead h = T.head;
    if (!(((h.term_mask >> term) & 1u) && s.nscat >= h.nscat_lo && s.nscat <= h.nscat_hi &&
          (h.volume < 0 || h.volume == s.region)))
        return -1;
    // cosine of the angle to the beam, for the 2-theta and momentum-transfer axes
    R c = (R)0;
    if (h.qmask & ((1u << PR_Q_THETA2) | (1u << PR_Q_Q))) {
        c = s.u[0] * beam_component<R>(T, 0) + s.u[1] * beam_component<R>(T, 1) + s.u[2] * beam_component<R>(T, 2);
        c = c > (R)1 ? (R)1 : (c < (R)-1 ? (R)-1 : c);
    }
    int64_t flat = 0, slice = 0;
    bool in_slice = true;
    (void)slice;
    (void)in_slice;
    // unrolled over the at most four axes (UNROLL), so the scalar loads of every
    // axis's descriptor issue together instead of one loop trip after another
#pragma unroll
    for (int a = 0; a < (UNROLL ? 4 : h.naxes); ++a) {
        if (a >= h.naxes) break;
        const TallyAxis& A = T.ax[a];
        const int32_t quantity = A.quantity, n = A.nbins;
        R lo, hi, scale;
        axis_range<R>(A, lo, hi, scale);
        R x;
        switch (quantity) {
        case PR_Q_THETA2: x = M<R>::acos_deg(c); break;
        case PR_Q_LAMBDA: x = s.lam; break;
        case PR_Q_X: x = s.p[0]; break;
        case PR_Q_Y: x = s.p[1]; break;
        case PR_Q_Z: x = s.p[2]; break;
        case PR_Q_DIVX: x = PRE ? q.divx : M<R>::atan2_deg(s.u[0], s.u[2]); break;
        case PR_Q_DIVY: x = PRE ? q.divy : M<R>::atan2_deg(s.u[1], s.u[2]); break;
        case PR_Q_TOF: x = s.t; break;
        case PR_Q_Q:
            // momentum transfer from the beam direction: (4 pi / lambda) sin(alpha / 2)
            x = M<R>::div_((R)(4.0 * 3.14159265358979323846), s.lam) * M<R>::sqrt_(((R)1 - c) / (R)2);
            break;
        default: x = (R)s.nscat; break;
        }
        if (!(x >= lo && x <= hi)) return -1;
        // FP32: floorf of the FP32 product (the same integer as the floor of its
        // exact double conversion, without the FP64 round trip)
        int b;
        if constexpr (sizeof(R) == 4) b = (int)__builtin_floorf((x - lo) * scale);
        else b = (int)__builtin_floor((x - lo) * scale);
        if (x == hi || b >= n) b = n - 1;
        if (b < 0) b = 0;
        flat = flat * n + b;
        if constexpr (SLICED) {
            if (a == h.fix_axis) in_slice = b == h.fix_bin;
            else slice = slice * n + b;
        }
    }
    if constexpr (!SLICED) return flat;
    return in_slice ? slice : (flat | kOffSlice);
}

template <class R, bool PRE = true>
__device__ __forceinline__ int64_t tally_bin(const TallyDev& T, const PState<R>& s, int term, const HistAngles<R>& q) {
    return T.head.fix_axis >= 0 ? tally_bin_t<R, PRE, true>(T, s, term, q) : tally_bin_t<R, PRE, false>(T, s, term, q);
}

// flat index of bin i of a tally's slice (inverse of the slice index)
__device__ __forceinline__ int64_t slice_to_flat(const TallyDev& T, int64_t i) {
    const int k = T.head.fix_axis;
    if (k < 0) return i;
    int64_t stride = 1;   // bins of the axes after k
    for (int a = k + 1; a < T.head.naxes; ++a) stride *= T.ax[a].nbins;
    const int64_t hi = i / stride, lo = i - hi * stride;
    return (hi * T.ax[k].nbins + T.head.fix_bin) * stride + lo;
}

template <class R>
__device__ __forceinline__ void write_record(pr_history_record* rec, const PState<R>& s) {
    rec->hash = s.hash;
    rec->w = s.w;
    for (int k = 0; k < 3; ++k) {
        rec->pos[k] = (double)s.p[k];
        rec->dir[k] = (double)s.u[k];
    }
    rec->lambda = (double)s.lam;
    rec->term = s.term;
    rec->n_scat = s.nscat;
    rec->n_steps = s.steps;
    rec->n_draws = (int32_t)s.k;
    rec->region = s.region;
    rec->tof = (float)s.t;
}

}  // namespace prk
