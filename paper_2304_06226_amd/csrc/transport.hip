// HIP kernels of the history loop and their launchers.
//
// PR_FP64_PLAIN: one thread per history, FP64 throughout, scene read from
//   global memory, tallies scored with global FP64 atomics.
// PR_FP32_MIXED: persistent waves.  Each lane holds one live history; when
//   enough lanes of a wave are idle the wave claims that many new history ids
//   with one atomic and hands them out by lane rank (ballot / popcount /
//   mbcnt), so lanes stay busy until the work runs out.  The scene (volumes,
//   materials, Bragg tables) is staged into LDS as FP32; small tallies are
//   privatised in LDS and merged into global memory once per block; the
//   weight product and every tally accumulation stay FP64.
// PR_FP64_PERSISTENT: the same persistent waves and LDS tallies around the
//   FP64 step of the plain kernel, so each history's events, weight and exit
//   state equal the plain kernel's bit for bit.
// Batched (k_batch): the mixed policy over many simulations at once; a block
//   stages one simulation's scene and tallies in LDS and its waves claim chunks
//   of that simulation's histories from its own counter until none are left,
//   then the block flushes and moves to the next simulation with work.
#include "device.h"
#include "launch.h"

namespace prk {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// sum of a 64-bit value over the wave, result valid in every lane
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// per-lane end-of-history counters; 32 bits per lane (a lane runs far fewer than
// 2^32 / 10^4 histories per launch), summed over the wave in 64 bits at the end
struct Counters {
    uint32_t c[ST_N];
};

template <class R>
__device__ __forceinline__ void count_end(Counters& k, const PState<R>& s) {
    k.c[ST_HIST] += 1u;
    k.c[ST_STEPS] += (uint32_t)s.steps;
    k.c[ST_DRAWS] += s.k;
    k.c[ST_SCAT] += (uint32_t)s.nscat;
    // one add per class with constant indices (a switch here becomes an indexed private array)
    k.c[ST_ESC] += s.term == PR_END_ESCAPE ? 1u : 0u;
    k.c[ST_ABS] += s.term == PR_END_ABSORB ? 1u : 0u;
    k.c[ST_KILL] += s.term == PR_END_KILL ? 1u : 0u;
    k.c[ST_DET] += s.term == PR_END_DETECT ? 1u : 0u;
    k.c[ST_CAP] += s.term == PR_END_CAPPED ? 1u : 0u;
    k.c[ST_OUT] += s.term == PR_END_OUTSIDE ? 1u : 0u;
}

__device__ __forceinline__ void flush_counters(const Counters& k, unsigned long long* g) {
#pragma unroll
    for (int i = 0; i < ST_N; ++i) {
        unsigned long long t = wave_sum((unsigned long long)k.c[i]);
        if (lane_id() == 0 && t) atomicAdd(g + i, t);
    }
}

// Global tallies store (sum w, sum w^2) interleaved per bin, so the two atomics
// of a score update the same 16-byte pair (one memory-side line, not two).
__device__ __forceinline__ void add_global(const TallyDev& T, int64_t b, double w, double w2) {
    atomicAdd(T.sw + 2 * b, w);
    atomicAdd(T.sw + 2 * b + 1, w2);
}

// Add the pair (v0, v1) to bin b of global pair storage sw for every lane with
// `need` (SQUARE: v1 = v0^2, a score); called by a converged wave.  Lanes 2j and
// 2j+1 of one atomic instruction carry the two words of lane j's pair (then of
// lane 32 + j), so the two FP64 atomics of a pair leave the wave as one request
// on one 16-byte pair instead of two requests from two instructions.  Halves of
// the wave without a pair are skipped.
template <bool SQUARE>
__device__ __forceinline__ void add_pairs_wave(double* sw, int64_t b, double v0, double v1, bool need) {
    const unsigned long long m = __ballot(need);
    if (m == 0ull) return;
    const int lane = lane_id();
    const int odd = lane & 1;
#pragma unroll 1
    for (int r = 0; r < 2; ++r) {
        if (((m >> (32 * r)) & 0xFFFFFFFFull) == 0ull) continue;
        const int src = 32 * r + (lane >> 1);
        const long long bs = __shfl((long long)b, src, kWave);
        const double a = __shfl(v0, src, kWave);
        const double c = SQUARE ? a * a : __shfl(v1, src, kWave);
        if ((m >> src) & 1ull) atomicAdd(sw + 2 * bs + odd, odd ? c : a);
    }
}

// a score w (adds w and w^2) from every lane with `need`, converged wave
__device__ __forceinline__ void add_global_wave(double* sw, int64_t b, double w, bool need) {
    add_pairs_wave<true>(sw, b, w, 0.0, need);
}

// ------------------------------------------------------------------------
// FP64 plain
// ------------------------------------------------------------------------

// The grid variant is held to three waves per SIMD (168 VGPRs): its grid walk
// is latency-bound, and the third wave hides more of it (1000-box imaging
// 48.9 -> 38.3 ms); the other variants run two, as they would anyway.
// One thread per history (a loop over several histories per thread costs the grid
// variant registers: imaging 38 -> 43 ms; the host splits very large runs into
// several launches instead).  FC: the run has
// first-collision tallies (a separate instance: their scoring inside the step
// loop costs the other runs registers, imaging 43 -> 53 ms).
// ESC: the world crossing after leaving an exit_escapes volume is taken in the
// leaving step (scenes without a grid; not with first-collision tallies).
template <bool REC, bool GRID, bool FC, bool ESC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(GRID ? 3 : 2, 8))) void k_plain(Params P) {
    const SceneT<double> S{P.vols_d, P.mats_d, P.fams_d, P.children, P.grids_d, P.cell_start, P.cell_items, P.boxes_d,
                           P.kinds};
    Counters cnt = {};
    {
        const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
        const bool live = i < P.n;
        PState<double> s;
        s.xs_mat = -2;
        s.lam = -1.0;
        s.term = PR_END_OUTSIDE;
        s.nscat = 0;
        if (live) {
            source<double, REC, GRID>(s, P.src, S, P.seed, P.first + i, 0);
            while (s.term == 0) {
                const bool first = step<double, REC, GRID, ESC>(s, S, P.seed);
                if (FC && first) {
                    // first-collision tallies score the state just after the collision
                    const HistAngles<double> q = hist_angles<double>(s, P.qmask);
                    for (int t = 0; t < P.n_tallies; ++t) {
                        const int64_t b = tally_bin<double>(P.tallies[t], s, kTermFirstCollision, q);
                        if (b >= 0) add_global(P.tallies[t], b, s.w, s.w * s.w);
                    }
                }
            }
        }
        // scoring with the whole wave converged (paired-lane global atomics); the
        // grid variant scores per lane (the wave-level form costs it registers it
        // does not have: imaging 38 -> 49 ms)
        const bool scoring = live && (s.term == PR_END_ESCAPE || s.term == PR_END_ABSORB || s.term == PR_END_DETECT);
        if constexpr (GRID) {
            if (scoring) {
                const HistAngles<double> q = hist_angles<double>(s, P.qmask);
                for (int t = 0; t < P.n_tallies; ++t) {
                    const int64_t b = tally_bin<double>(P.tallies[t], s, s.term, q);
                    if (b >= 0) add_global(P.tallies[t], b, s.w, s.w * s.w);
                }
            }
        } else if (__ballot(scoring) != 0ull) {
            const HistAngles<double> q = hist_angles<double>(s, P.qmask);
            for (int t = 0; t < P.n_tallies; ++t) {
                const TallyDev& T = P.tallies[t];
                const int64_t b = scoring ? tally_bin<double>(T, s, s.term, q) : -1;
                add_global_wave(T.sw, b, s.w, b >= 0);
            }
        }
        if (live) {
            if (REC) write_record<double>(P.records + i, s);
            count_end<double>(cnt, s);
        }
    }
    flush_counters(cnt, P.stats);
}

// ------------------------------------------------------------------------
// Persistent policies (FP32 mixed, FP64)
// ------------------------------------------------------------------------

// LDS of a mixed-policy block: [privatised tallies (doubles)] [bin-cache values
// (2 doubles per slot)] [bin-cache keys (u32 per slot)] [scene, when staged:
// volumes, materials, Bragg tables, daughter lists, grids, grid cells]
struct LdsLayout {
    int cache_vals, cache_keys, vols, mats, fams, children, grids, cell_start, cell_items, boxes, bytes;   // byte offsets
};

__host__ __device__ inline int align16(int x) { return (x + 15) & ~15; }

__host__ __device__ inline LdsLayout lds_layout(const Params& P) {
    LdsLayout L;
    const int st = P.scene_in_lds ? 1 : 0;
    // grid scenes keep the volume table in global memory and stage the box bounds
    const int sv = P.scene_in_lds && !P.has_grid ? 1 : 0;
    const int sb = P.scene_in_lds && P.has_grid ? 1 : 0;
    int off = P.lds_tally_doubles * 8;
    L.cache_vals = off;
    off += P.cache_slots * 16;
    L.cache_keys = off;
    off = align16(off + P.cache_slots * 4);
    L.vols = off;
    off = align16(off + sv * P.n_vols * (int)sizeof(VolT<float>));
    L.mats = off;
    off = align16(off + st * P.n_mats * (int)sizeof(MatT<float>));
    L.fams = off;
    off = align16(off + st * P.n_fams * (int)sizeof(FamT<float>));
    L.children = off;
    off = align16(off + st * P.n_children * 4);
    L.grids = off;
    off = align16(off + st * P.n_grids * (int)sizeof(GridT<float>));
    L.cell_start = off;
    off = align16(off + st * P.n_cell_start * 4);
    L.cell_items = off;
    off = align16(off + st * P.n_cell_items * 4);
    L.boxes = off;
    off = align16(off + sb * P.n_vols * (int)sizeof(BoxT<float>));
    L.bytes = off;
    return L;
}

constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;

// Score w into tally T (b: the bin from tally_bin, -1 = none): the block's
// privatised copy when the bin lies in it (the whole tally, or its slice), else
// the block's LDS bin cache (a slot is claimed by the first bin that hashes to
// it; two probes), else global memory.  Returns the global bin, or -1 when the
// score was taken in LDS or there is none.
__device__ __forceinline__ int64_t score_lds(const TallyDev& T, int64_t b, double w, double* lds, double* cvals,
                                             uint32_t* ckeys) {
    if (b < 0) return -1;
    if (T.lds_offset >= 0) {
        if (T.head.fix_axis < 0 || (b & kOffSlice) == 0) {
            atomicAdd(lds + T.lds_offset + b, w);
            atomicAdd(lds + T.lds_offset + T.lds_bins + b, w * w);
            return -1;
        }
        return b & ~kOffSlice;   // outside the privatised slice
    }
    if (T.cache_base >= 0 && b < (int64_t)kEmptyKey) {
        const uint32_t key = (uint32_t)b;
        const uint32_t h = (key * 2654435761u) >> (32 - T.cache_bits);
        const uint32_t mask = (1u << T.cache_bits) - 1u;
#pragma unroll
        for (int probe = 0; probe < 2; ++probe) {
            const uint32_t slot = (uint32_t)T.cache_base + ((h ^ (uint32_t)probe) & mask);
            uint32_t k = __hip_atomic_load(ckeys + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (k == kEmptyKey) {
                k = atomicCAS(ckeys + slot, kEmptyKey, key);
                if (k == kEmptyKey) k = key;
            }
            if (k == key) {
                atomicAdd(cvals + 2 * slot, w);
                atomicAdd(cvals + 2 * slot + 1, w * w);
                return -1;
            }
        }
    }
    return b;
}

// Scoring by a converged wave (every lane calls; b < 0: no score): global scores
// leave as paired-lane atomics.
__device__ __forceinline__ void score_wave(const TallyDev& T, int64_t b, double w, double* lds, double* cvals,
                                           uint32_t* ckeys) {
    const int64_t g = score_lds(T, b, w, lds, cvals, ckeys);
    add_global_wave(T.sw, g, w, g >= 0);
}

// Scoring from one lane in divergent code: per-lane global atomics (two requests
// per score).  The FP32 kernels score this way: shuffling scores between lanes
// at the refill point cost them more instructions and registers than the atomics
// it saves (headline +1.7 %, imaging +10 %).
__device__ __forceinline__ void score_lane(const TallyDev& T, int64_t b, double w, double* lds, double* cvals,
                                           uint32_t* ckeys) {
    const int64_t g = score_lds(T, b, w, lds, cvals, ckeys);
    if (g >= 0) add_global(T, g, w, w * w);
}

// Merge n_pairs (value, square) LDS sums a[i], a[n + i] into global pairs at
// flat(i): the block walks the interleaved words, so consecutive lanes write
// consecutive words of the destination pairs; zero words are skipped.
template <class Flat>
__device__ __forceinline__ void merge_pairs(double* sw, const double* a, int64_t n, Flat flat) {
    for (int64_t j = threadIdx.x; j < 2 * n; j += blockDim.x) {
        const int64_t i = j >> 1;
        const int odd = (int)(j & 1);
        const double v = a[odd * n + i];
        if (v != 0.0) atomicAdd(sw + 2 * flat(i) + odd, v);
    }
}

__device__ __forceinline__ void copy_words(void* dst, const void* src, int bytes) {
    const uint32_t* s = (const uint32_t*)src;
    uint32_t* d = (uint32_t*)dst;
    for (int i = threadIdx.x; i < bytes / 4; i += blockDim.x) d[i] = s[i];
}

// Scene of a persistent launch: the FP32 tables, staged in LDS (SLDS) or read
// from global memory, or the FP64 tables in global memory.
template <class R, bool SLDS, bool GRID>
struct PersistentScene;

template <bool SLDS, bool GRID>
struct PersistentScene<float, SLDS, GRID> {
    static __device__ __forceinline__ SceneT<float> get(const Params& P, char* base, const LdsLayout& L) {
        return SLDS ? SceneT<float>{GRID ? P.vols_f : (const VolT<float>*)(base + L.vols),
                                    (const MatT<float>*)(base + L.mats), (const FamT<float>*)(base + L.fams),
                                    (const int32_t*)(base + L.children), (const GridT<float>*)(base + L.grids),
                                    (const int32_t*)(base + L.cell_start), (const int32_t*)(base + L.cell_items),
                                    GRID ? (const BoxT<float>*)(base + L.boxes) : P.boxes_f, P.kinds}
                    : SceneT<float>{P.vols_f, P.mats_f, P.fams_f, P.children, P.grids_f, P.cell_start, P.cell_items,
                                    P.boxes_f, P.kinds};
    }
};

template <bool GRID>
struct PersistentScene<double, false, GRID> {
    static __device__ __forceinline__ SceneT<double> get(const Params& P, char*, const LdsLayout&) {
        return SceneT<double>{P.vols_d, P.mats_d, P.fams_d, P.children, P.grids_d, P.cell_start, P.cell_items,
                              P.boxes_d, P.kinds};
    }
};

// lane l's value of x, as a wave-uniform value
template <class R>
__device__ __forceinline__ R readlane_r(R x, int l) {
    if constexpr (sizeof(R) == 4) {
        return __builtin_bit_cast(R, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
    } else {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
        const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
        const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
        return __builtin_bit_cast(R, ((unsigned long long)hi << 32) | lo);
    }
}

// R = float: the FP32 mixed policy; R = double: the persistent FP64 policy, whose
// histories take exactly the arithmetic of the plain kernel.
// WPE resident waves per SIMD (FP32: 4 or 5, grid variants 4; FP64: 2, grid 3,
// as the plain kernel).  The FP32 grid variants would take 151 VGPRs (three
// waves); held to 128 they spill a few values to scratch, and the extra wave
// per SIMD hides the latency of the grid walk (1000-box imaging 10.3 -> 8.6 ms).
// Five waves (96 VGPRs) help some scenes and hurt others, so it is a launch
// choice.
// Block sizes: up to 1024 threads for the FP32 kernels without a grid (fewer
// blocks merge their LDS tallies at the end), 512 with a grid, 256 in FP64.
// PAIR (FP32 without a grid): paired-lane global scores, for runs with a tally
// that scores straight into global memory.  FC (FP64): the run has
// first-collision tallies.  ESC, steps that draw nothing taken early (no history
// changes, short of rounding on a grazing exit in 1): 1 (no grid; FP32 with four waves and per-lane scoring, and
// FP64): the world crossing after leaving an exit_escapes volume is taken in the
// leaving step; 2 (FP32 with the scene in LDS, no grid): a lane whose step took
// it from material into vacuum takes its vacuum step in a fold pass, before the
// wave's other lanes step again; with 1 and 2 a history born in a vacuum volume
// takes its first step in the refill pass, with the wave's other new histories.
// Built only where it pays: the extra code slows the other instances down.  The
// batch kernels without a grid take the world crossing of 1 (their newborns
// start from a copied first step instead of a refill-pass step).
template <class R, bool REC, bool SLDS, bool GRID, int WPE, bool PAIR, bool FC, int ESC>
__global__ __launch_bounds__(GRID ? 512 : (sizeof(R) == 4 ? 1024 : 256)) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
void k_mixed(Params P) {
    // FP64 without a grid, and FP32 runs whose tallies score straight into global
    // memory: the wave scores together and the global scores leave as paired-lane
    // atomics (one 16-byte request per score instead of two 8-byte ones: half the
    // memory transactions); the rest score per lane, which holds fewer registers
    constexpr bool kPaired = (sizeof(R) == 8 && !GRID) || PAIR;
    extern __shared__ double lds[];
    const LdsLayout L = lds_layout(P);
    char* base = (char*)lds;
    double* cvals = (double*)(base + L.cache_vals);
    uint32_t* ckeys = (uint32_t*)(base + L.cache_keys);
    if (SLDS) {
        if (!GRID) copy_words(base + L.vols, P.vols_f, P.n_vols * (int)sizeof(VolT<float>));
        if (GRID) copy_words(base + L.boxes, P.boxes_f, P.n_vols * (int)sizeof(BoxT<float>));
        copy_words(base + L.mats, P.mats_f, P.n_mats * (int)sizeof(MatT<float>));
        copy_words(base + L.fams, P.fams_f, P.n_fams * (int)sizeof(FamT<float>));
        copy_words(base + L.children, P.children, P.n_children * 4);
        copy_words(base + L.grids, P.grids_f, P.n_grids * (int)sizeof(GridT<float>));
        copy_words(base + L.cell_start, P.cell_start, P.n_cell_start * 4);
        copy_words(base + L.cell_items, P.cell_items, P.n_cell_items * 4);
    }
    for (int i = threadIdx.x; i < P.lds_tally_doubles + 2 * P.cache_slots; i += blockDim.x) lds[i] = 0.0;
    for (int i = threadIdx.x; i < P.cache_slots; i += blockDim.x) ckeys[i] = kEmptyKey;
    __syncthreads();
    const SceneT<R> S = PersistentScene<R, SLDS, GRID>::get(P, base, L);

    Counters cnt = {};
    PState<R> s;
    s.term = 1;            // idle, no history
    s.xs_mat = -2;         // no cached cross sections
    s.lam = (R)-1;
    bool pending = false;  // finished history not yet scored
    bool exhausted = false;
    // the wave's current chunk of history indices [cnext, cend), claimed with one
    // atomic per chunk; values are wave-uniform
    unsigned long long cnext = 0, cend = 0;
    const unsigned long long chunk = (unsigned long long)P.chunk;
    const int lane = lane_id();
    // a pencil starts every history at the same point: locate it once
    int start_region = -2;
    if (P.src.kind == PR_PENCIL) {
        const R o[3] = {(R)P.src.o[0], (R)P.src.o[1], (R)P.src.o[2]};
        start_region = locate<R, GRID>(S, o, 0);
    }
    bool again = false;   // ESC == 2: the lane's last step took it from material into vacuum
    // A pencil beam of one wavelength starting in vacuum: every history draws
    // nothing until it has taken its first step, so that step ends in the same
    // state for all of them.  After the wave's first newborn has taken it, the
    // state is kept in wave-uniform registers and later newborns start from it
    // (builds without records only: records also carry the event hash).
    constexpr bool kTmpl = ESC == 1 && !REC;
    const bool tmpl_ok = kTmpl && P.src.kind == PR_PENCIL && P.src.spectrum == PR_MONO && start_region >= 0 &&
                         S.vols[start_region].mat < 0;
    bool have_tmpl = false;
    R tp0 = (R)0, tp1 = (R)0, tp2 = (R)0, tt = (R)0;
    int treg = 0, tsteps = 0, tterm = 0;
    for (;;) {
        // ESC == 2, a fold pass: only the lanes that just left material for vacuum
        // step (the vacuum step, which draws nothing), with no refill before it
        const bool fold_pass = ESC == 2 && __ballot(again) != 0ull;
        const bool idle = s.term != 0;
        const unsigned long long idle_mask = __ballot(idle);
        const int n_idle = __popcll(idle_mask);
        if (!fold_pass && (n_idle >= P.refill_threshold || n_idle == kWave)) {
            // score the histories that ended since the last refill, all together
            if (kPaired && __ballot(pending) != 0ull) {
                const bool scoring =
                    pending && (s.term == PR_END_ESCAPE || s.term == PR_END_ABSORB || s.term == PR_END_DETECT);
                const HistAngles<R> q = hist_angles<R>(s, P.qmask);
                for (int t = 0; t < P.n_tallies; ++t) {
                    const TallyDev& T = P.tallies[t];
                    const int64_t b = scoring ? tally_bin<R>(T, s, s.term, q) : -1;
                    score_wave(T, b, s.w, lds, cvals, ckeys);
                }
            }
            if (pending) {
                if (!kPaired && (s.term == PR_END_ESCAPE || s.term == PR_END_ABSORB || s.term == PR_END_DETECT)) {
                    const HistAngles<R> q = hist_angles<R>(s, P.qmask);
                    if constexpr (GRID) {
                        // two tallies per trip: their descriptors' scalar loads issue
                        // together (the imaging scene's two image tallies: -5 %)
#pragma unroll 2
                        for (int t = 0; t < P.n_tallies; ++t) {
                            const TallyDev& T = P.tallies[t];
                            score_lane(T, tally_bin<R>(T, s, s.term, q), s.w, lds, cvals, ckeys);
                        }
                    } else {
                        for (int t = 0; t < P.n_tallies; ++t) {
                            const TallyDev& T = P.tallies[t];
                            score_lane(T, tally_bin<R>(T, s, s.term, q), s.w, lds, cvals, ckeys);
                        }
                    }
                }
                if (REC) write_record<R>(P.records + (s.h - P.first), s);
                count_end<R>(cnt, s);
                pending = false;
            }
            if (!exhausted && cnext >= cend) {
                const int leader = __ffsll((long long)idle_mask) - 1;
                unsigned long long got = 0;
                if (lane == leader) got = atomicAdd(P.counter, chunk);
                got = __shfl(got, leader, kWave);
                cnext = got;
                cend = got + chunk < P.n ? got + chunk : P.n;
                if (got >= P.n) exhausted = true;
            }
            if (!exhausted) {
                const unsigned long long avail = cend - cnext;
                const unsigned long long take = (unsigned long long)n_idle < avail ? (unsigned long long)n_idle : avail;
                bool born = false;
                if (idle) {
                    const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(idle_mask >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)idle_mask, 0u));
                    if ((unsigned long long)rank < take) {
                        born = true;
                        if (kTmpl && have_tmpl) {
                            // the state source() and the first step would give (no draws)
                            s.h = P.first + cnext + (unsigned long long)rank;
                            s.k = 0;
                            s.nbuf = 0;
                            s.w = 1.0;
                            s.nscat = 0;
                            s.p[0] = tp0;
                            s.p[1] = tp1;
                            s.p[2] = tp2;
                            s.u[0] = (R)P.src.u[0];
                            s.u[1] = (R)P.src.u[1];
                            s.u[2] = (R)P.src.u[2];
                            const R lam = (R)P.src.lam0;
                            if (!(lam == s.lam)) s.xs_mat = -2;
                            s.lam = lam;
                            s.t = tt;
                            s.region = treg;
                            s.steps = tsteps;
                            s.term = tterm;
                        } else {
                            source<R, REC, GRID>(s, P.src, S, P.seed, P.first + cnext + (unsigned long long)rank, 0,
                                                 start_region);
                            // born in a vacuum volume: the first step draws nothing and is
                            // taken here, with the wave's other new histories
                            if (ESC && s.term == 0 && S.vols[s.region].mat < 0)
                                step<R, REC, GRID, ESC>(s, S, P.seed, P.walk_cells);
                        }
                        pending = s.term != 0;   // born outside the world, or ended: counted at the next refill
                    }
                }
                if (tmpl_ok && !have_tmpl) {
                    const unsigned long long bm = __ballot(born);
                    if (bm != 0ull) {
                        const int l = __ffsll((long long)bm) - 1;
                        tp0 = readlane_r<R>(s.p[0], l);
                        tp1 = readlane_r<R>(s.p[1], l);
                        tp2 = readlane_r<R>(s.p[2], l);
                        tt = readlane_r<R>(s.t, l);
                        treg = __builtin_amdgcn_readlane(s.region, l);
                        tsteps = __builtin_amdgcn_readlane(s.steps, l);
                        tterm = __builtin_amdgcn_readlane(s.term, l);
                        have_tmpl = true;
                    }
                }
                cnext += take;
                if (cnext >= cend && cend >= P.n) exhausted = true;
            }
        }
        if (__ballot(s.term == 0) == 0ull) {
            if (exhausted && __ballot(pending) == 0ull) break;
            continue;
        }
        bool first = false;
        if (s.term == 0 && (!fold_pass || again)) {
            const int m0 = ESC == 2 ? S.vols[s.region].mat : 0;
            first = step<R, REC, GRID, ESC>(s, S, P.seed, P.walk_cells);
            pending = s.term != 0;
            if (ESC == 2) again = !fold_pass && s.term == 0 && m0 >= 0 && S.vols[s.region].mat < 0;
        } else if (ESC == 2) {
            again = false;
        }
        // first-collision tallies (a debugging trigger of the FP64 policies) score
        // the state just after the collision
        if (FC && __ballot(first) != 0ull) {
            const HistAngles<R> q = hist_angles<R>(s, P.qmask);
            for (int t = 0; t < P.n_tallies; ++t) {
                const TallyDev& T = P.tallies[t];
                const int64_t b = first ? tally_bin<R>(T, s, kTermFirstCollision, q) : -1;
                if constexpr (kPaired) score_wave(T, b, s.w, lds, cvals, ckeys);
                else score_lane(T, b, s.w, lds, cvals, ckeys);
            }
        }
    }
    flush_counters(cnt, P.stats);
    __syncthreads();
    // merge the block's privatised tallies and cached bins (non-zero bins only)
    for (int t = 0; t < P.n_tallies; ++t) {
        const TallyDev& T = P.tallies[t];
        if (T.cache_base >= 0) {
            const int ns = 1 << T.cache_bits;
            for (int base = 0; base < ns; base += blockDim.x) {
                const int i = base + (int)threadIdx.x;
                const int slot = T.cache_base + i;
                const uint32_t key = i < ns ? ckeys[slot] : kEmptyKey;
                const bool used = key != kEmptyKey;
                add_pairs_wave<false>(T.sw, used ? (int64_t)key : 0, used ? cvals[2 * slot] : 0.0,
                                      used ? cvals[2 * slot + 1] : 0.0, used);
            }
        }
        if (T.lds_offset < 0) continue;
        merge_pairs(T.sw, lds + T.lds_offset, T.lds_bins, [&](int64_t i) { return slice_to_flat(T, i); });
    }
}

// ------------------------------------------------------------------------
// Batched FP32 mixed: many simulations in one persistent launch
// ------------------------------------------------------------------------

// LDS of a batch block: [tally region (doubles): privatised tallies of the
// staged simulation, or bin-cache values] [bin-cache keys] [staged scene]
struct SceneLds {
    int vols, mats, fams, children, grids, cell_start, cell_items, boxes, bytes;
};

// grid scenes (grid != 0) keep the volume table in global memory and stage the box bounds
__host__ __device__ inline SceneLds scene_lds_layout(int nv, int nm, int nf, int nc, int ng, int ncs, int nci, int grid) {
    SceneLds L;
    int off = 0;
    L.vols = off;
    off = align16(off + (grid ? 0 : nv) * (int)sizeof(VolT<float>));
    L.mats = off;
    off = align16(off + nm * (int)sizeof(MatT<float>));
    L.fams = off;
    off = align16(off + nf * (int)sizeof(FamT<float>));
    L.children = off;
    off = align16(off + nc * 4);
    L.grids = off;
    off = align16(off + ng * (int)sizeof(GridT<float>));
    L.cell_start = off;
    off = align16(off + ncs * 4);
    L.cell_items = off;
    off = align16(off + nci * 4);
    L.boxes = off;
    off = align16(off + (grid ? nv : 0) * (int)sizeof(BoxT<float>));
    L.bytes = off;
    return L;
}

int batch_scene_lds_bytes(int nv, int nm, int nf, int nc, int ng, int ncs, int nci, int grid) {
    return scene_lds_layout(nv, nm, nf, nc, ng, ncs, nci, grid).bytes;
}

struct BlockCtl {
    int sim;   // simulation the block works on next (-1: no work left)
};

// simulation holding position pos of the class's concatenated history ranges
__device__ __forceinline__ int sim_of_position(const BatchParams& B, unsigned long long pos) {
    int lo = 0, hi = B.nsims - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (B.sims[mid].hist_begin <= pos) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Score w into entry t of the staged simulation from one lane: the privatised
// LDS copy, else the LDS bin cache, else global memory.
__device__ __forceinline__ void score_block(const BatchParams& B, const SimDev& sd, int t, int64_t b, double w,
                                            double* ltal, uint32_t* ckeys) {
    const TallyDev& T = B.tallies[t];
    bool global = true;
    if (sd.privatised) {
        atomicAdd(ltal + T.lds_offset + b, w);
        atomicAdd(ltal + T.lds_offset + T.total + b, w * w);
        return;
    }
    const uint64_t key64 = B.tally_key_base[t] + (uint64_t)b;
    if (B.cache_bits > 0 && key64 < (uint64_t)kEmptyKey) {
        const uint32_t key = (uint32_t)key64;
        const uint32_t h = (key * 2654435761u) >> (32 - B.cache_bits);
        const uint32_t mask = (1u << B.cache_bits) - 1u;
#pragma unroll
        for (int probe = 0; probe < 2; ++probe) {
            const uint32_t slot = (h ^ (uint32_t)probe) & mask;
            uint32_t k = __hip_atomic_load(ckeys + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (k == kEmptyKey) {
                k = atomicCAS(ckeys + slot, kEmptyKey, key);
                if (k == kEmptyKey) k = key;
            }
            if (k == key) {
                atomicAdd(ltal + 2 * slot, w);
                atomicAdd(ltal + 2 * slot + 1, w * w);
                global = false;
                break;
            }
        }
    }
    if (global) add_global(T, b, w, w * w);
}

// merge the staged simulation's LDS tallies into global memory (whole block)
__device__ __forceinline__ void flush_block(const BatchParams& B, const SimDev& sd, const double* ltal,
                                            const uint32_t* ckeys) {
    if (sd.privatised) {
        for (int t = sd.tally_begin; t < sd.tally_begin + sd.tally_count; ++t) {
            const TallyDev& T = B.tallies[t];
            merge_pairs(T.sw, ltal + T.lds_offset, T.total, [](int64_t i) { return i; });
        }
    } else if (B.cache_bits > 0) {
        const int nslots = 1 << B.cache_bits;
        for (int base = 0; base < nslots; base += blockDim.x) {
            const int i = base + (int)threadIdx.x;
            const uint32_t key = i < nslots ? ckeys[i] : kEmptyKey;
            const bool used = key != kEmptyKey;
            int t = sd.tally_begin;
            while (used && t + 1 < sd.tally_begin + sd.tally_count && B.tally_key_base[t + 1] <= key) ++t;
            // the entries of one simulation may differ from lane to lane: one pass per entry
            for (int e = sd.tally_begin; e < sd.tally_begin + sd.tally_count; ++e) {
                const bool mine = used && t == e;
                const uint64_t b = mine ? key - B.tally_key_base[e] : 0;
                add_pairs_wave<false>(B.tallies[e].sw, (int64_t)b, mine ? ltal[2 * i] : 0.0, mine ? ltal[2 * i + 1] : 0.0,
                                      mine);
            }
        }
    }
}

// the block's waves run histories of simulation `sim`, claiming chunks from its
// counter, until the simulation has none left
template <bool SLDS, bool GRID, int WPE>
__device__ __forceinline__ void run_sim(const BatchParams& B, const SimDev& sd, int sim, char* scene, double* ltal,
                                        uint32_t* ckeys, Counters& cnt, unsigned long long shift) {
    SceneT<float> S;
    if (SLDS) {
        const SceneLds L = scene_lds_layout(sd.n_vols, sd.n_mats, sd.n_fams, sd.n_children, sd.n_grids,
                                            sd.n_cell_start, sd.n_cell_items, GRID ? 1 : 0);
        S = SceneT<float>{GRID ? sd.vols : (const VolT<float>*)(scene + L.vols), (const MatT<float>*)(scene + L.mats),
                          (const FamT<float>*)(scene + L.fams), (const int32_t*)(scene + L.children),
                          (const GridT<float>*)(scene + L.grids), (const int32_t*)(scene + L.cell_start),
                          (const int32_t*)(scene + L.cell_items),
                          GRID ? (const BoxT<float>*)(scene + L.boxes) : sd.boxes, sd.kinds};
    } else {
        S = SceneT<float>{sd.vols, sd.mats, sd.fams, sd.children, sd.grids, sd.cell_start, sd.cell_items, sd.boxes,
                          sd.kinds};
    }
    PState<float> s;
    s.term = 1;
    s.xs_mat = -2;   // material indices are the simulation's own
    s.lam = -1.f;
    bool pending = false;
    bool exhausted = false;
    unsigned long long cnext = 0, cend = 0;
    // a pencil starts every history of the simulation at the same point: locate it once
    int start_region = -2;
    if (sd.src.kind == PR_PENCIL) {
        const float o[3] = {(float)sd.src.o[0], (float)sd.src.o[1], (float)sd.src.o[2]};
        start_region = locate<float, GRID>(S, o, 0);
    }
    // A pencil beam of one wavelength starting in vacuum: every history reaches the
    // same state after its first step (it draws nothing until then).  Once a lane
    // of the wave has taken a first step, that state is kept in wave-uniform
    // registers and later newborns start from it.
    // (scenes without a daughter grid: the code costs the grid instances registers)
    const bool tmpl_ok = !GRID && sd.src.kind == PR_PENCIL && sd.src.spectrum == PR_MONO && start_region >= 0 &&
                         S.vols[start_region].mat < 0;
    bool have_tmpl = false;
    float tp0 = 0.f, tp1 = 0.f, tp2 = 0.f, tt = 0.f;
    int treg = 0, tsteps = 0, tterm = 0;
    const unsigned long long end = sd.n;
    unsigned long long* counter = B.sim_next + sim;
    const int lane = lane_id();
    for (;;) {
        const bool idle = s.term != 0;
        const unsigned long long idle_mask = __ballot(idle);
        const int n_idle = __popcll(idle_mask);
        if (n_idle >= B.refill_threshold || n_idle == kWave) {
            if (pending) {
                if (s.term == PR_END_ESCAPE || s.term == PR_END_ABSORB || s.term == PR_END_DETECT) {
                    const HistAngles<float> q{0.f, 0.f};
                    for (int t = sd.tally_begin; t < sd.tally_begin + sd.tally_count; ++t) {
                        const int64_t b = tally_bin_t<float, false, false, false>(B.tallies[t], s, s.term, q);   // whole tallies only
                        if (b >= 0) score_block(B, sd, t, b, s.w, ltal, ckeys);
                    }
                }
                count_end<float>(cnt, s);
                pending = false;
            }
            if (!exhausted && cnext >= cend) {
                const int leader = __ffsll((long long)idle_mask) - 1;
                unsigned long long got = 0;
                if (lane == leader) got = atomicAdd(counter, B.chunk);
                got = __shfl(got, leader, kWave);
                if (got >= end) {
                    exhausted = true;
                } else {
                    cnext = got;
                    cend = got + B.chunk < end ? got + B.chunk : end;
                }
            }
            if (!exhausted && cnext < cend) {
                const unsigned long long avail = cend - cnext;
                const unsigned long long take = (unsigned long long)n_idle < avail ? (unsigned long long)n_idle : avail;
                if (idle) {
                    const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(idle_mask >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)idle_mask, 0u));
                    if ((unsigned long long)rank < take) {
                        const unsigned long long h = sd.first + shift + cnext + (unsigned long long)rank;
                        if (!GRID && have_tmpl) {
                            // the state source() and the first step would give (no draws)
                            s.h = h;
                            s.k = 0;
                            s.nbuf = 0;
                            s.w = 1.0;
                            s.nscat = 0;
                            s.p[0] = tp0;
                            s.p[1] = tp1;
                            s.p[2] = tp2;
                            s.u[0] = (float)sd.src.u[0];
                            s.u[1] = (float)sd.src.u[1];
                            s.u[2] = (float)sd.src.u[2];
                            const float lam = (float)sd.src.lam0;
                            if (!(lam == s.lam)) s.xs_mat = -2;
                            s.lam = lam;
                            s.t = tt;
                            s.region = treg;
                            s.steps = tsteps;
                            s.term = tterm;
                        } else {
                            source<float, false, GRID>(s, sd.src, S, B.seed, h, 0, start_region);
                        }
                        pending = s.term != 0;
                    }
                }
                cnext += take;
            }
        }
        if (__ballot(s.term == 0) == 0ull) {
            if (exhausted && __ballot(pending) == 0ull) break;
            continue;
        }
        if (s.term == 0) {
            step<float, false, GRID, GRID ? 0 : 1>(s, S, B.seed, B.walk_cells);
            pending = s.term != 0;
        }
        if (tmpl_ok && !have_tmpl) {
            // a lane that has just taken its first step (its history's only one so far)
            const unsigned long long fm = __ballot(s.steps == 1 && (s.term == 0 || pending));
            if (fm != 0ull) {
                const int l = __ffsll((long long)fm) - 1;
                tp0 = readlane_r<float>(s.p[0], l);
                tp1 = readlane_r<float>(s.p[1], l);
                tp2 = readlane_r<float>(s.p[2], l);
                tt = readlane_r<float>(s.t, l);
                treg = __builtin_amdgcn_readlane(s.region, l);
                tsteps = __builtin_amdgcn_readlane(s.steps, l);
                tterm = __builtin_amdgcn_readlane(s.term, l);
                have_tmpl = true;
            }
        }
    }
}

template <bool SLDS, bool GRID, int WPE>
__global__ __launch_bounds__(GRID ? 512 : 256) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void k_batch(
    BatchParams B) {
    extern __shared__ double lds[];
    __shared__ BlockCtl ctl;
    double* ltal = lds;
    const int nslots = B.cache_bits > 0 ? (1 << B.cache_bits) : 0;
    uint32_t* ckeys = (uint32_t*)(lds + B.lds_tally_doubles);
    char* scene = (char*)ckeys + align16(nslots * 4);
    Counters cnt = {};
    int staged = -1;
    const unsigned long long shift = B.shift ? *B.shift : 0ull;
    // Each block starts on the simulation under its share of the concatenated
    // history ranges and stays with a simulation until its counter runs out, so
    // LDS staging, tally flushes and block-wide waits happen once per visit.
    if (threadIdx.x == 0) {
        const unsigned long long pos =
            (unsigned long long)((double)B.total_histories * (double)blockIdx.x / (double)gridDim.x);
        ctl.sim = sim_of_position(B, pos < B.total_histories ? pos : B.total_histories - 1);
    }
    for (;;) {
        if (threadIdx.x == 0) {
            // the first simulation from ctl.sim on (cyclically) that still has histories
            int sm = ctl.sim, tries = 0;
            while (tries < B.nsims &&
                   __hip_atomic_load(B.sim_next + sm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= B.sims[sm].n) {
                sm = sm + 1 < B.nsims ? sm + 1 : 0;
                ++tries;
            }
            ctl.sim = tries < B.nsims ? sm : -1;
        }
        __syncthreads();
        // block-uniform: read once into scalar registers so the simulation's
        // descriptor is fetched with scalar loads
        const int sim = __builtin_amdgcn_readfirstlane(ctl.sim);
        if (sim < 0) break;
        const SimDev& sd = B.sims[sim];
        if (sim != staged) {
            if (staged >= 0) {
                flush_block(B, B.sims[staged], ltal, ckeys);
                __syncthreads();
            }
            for (int i = threadIdx.x; i < B.lds_tally_doubles; i += blockDim.x) ltal[i] = 0.0;
            for (int i = threadIdx.x; i < nslots; i += blockDim.x) ckeys[i] = kEmptyKey;
            if (SLDS) {
                const SceneLds L = scene_lds_layout(sd.n_vols, sd.n_mats, sd.n_fams, sd.n_children, sd.n_grids,
                                                    sd.n_cell_start, sd.n_cell_items, GRID ? 1 : 0);
                if (!GRID) copy_words(scene + L.vols, sd.vols, sd.n_vols * (int)sizeof(VolT<float>));
                if (GRID) copy_words(scene + L.boxes, sd.boxes, sd.n_vols * (int)sizeof(BoxT<float>));
                copy_words(scene + L.mats, sd.mats, sd.n_mats * (int)sizeof(MatT<float>));
                copy_words(scene + L.fams, sd.fams, sd.n_fams * (int)sizeof(FamT<float>));
                copy_words(scene + L.children, sd.children, sd.n_children * 4);
                copy_words(scene + L.grids, sd.grids, sd.n_grids * (int)sizeof(GridT<float>));
                copy_words(scene + L.cell_start, sd.cell_start, sd.n_cell_start * 4);
                copy_words(scene + L.cell_items, sd.cell_items, sd.n_cell_items * 4);
            }
            __syncthreads();
            staged = sim;
        }
        run_sim<SLDS, GRID, WPE>(B, sd, sim, scene, ltal, ckeys, cnt, shift);
        __syncthreads();
        if (threadIdx.x == 0) ctl.sim = sim + 1 < B.nsims ? sim + 1 : 0;
    }
    if (staged >= 0) flush_block(B, B.sims[staged], ltal, ckeys);
    flush_counters(cnt, B.stats);
}

// End of a prepared batch run: add each tally's histories to its device
// history count, then advance the history-id offset by the stride.
__global__ void k_prepared_tail(unsigned long long* const* hist, const unsigned long long* add, int n,
                                unsigned long long* shift, unsigned long long stride) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) *hist[i] += add[i];
    if (i == 0) *shift += stride;
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void k_zero_f64(double* p, uint64_t n) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0.0;
}

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------

int mixed_lds_bytes(const Params& P) { return lds_layout(P).bytes; }

int mixed_max_block(const Params& P) { return P.has_grid ? 512 : (P.fp64 ? 256 : 1024); }
int batch_max_block(bool grid_nav) { return grid_nav ? 512 : 256; }

hipError_t launch_plain(const Params& P, bool rec, hipStream_t st) {
    const int block = 256;
    static const void* const kernels[10] = {
        (const void*)k_plain<false, false, false, false>, (const void*)k_plain<true, false, false, false>,
        (const void*)k_plain<false, true, false, false>,  (const void*)k_plain<true, true, false, false>,
        (const void*)k_plain<false, false, true, false>,  (const void*)k_plain<true, false, true, false>,
        (const void*)k_plain<false, true, true, false>,   (const void*)k_plain<true, true, true, false>,
        (const void*)k_plain<false, false, false, true>,  (const void*)k_plain<true, false, false, true>};
    const bool esc = P.esc == 1 && !P.has_grid && !P.has_fc;
    const int v = esc ? 8 + (rec ? 1 : 0) : (rec ? 1 : 0) + (P.has_grid ? 2 : 0) + (P.has_fc ? 4 : 0);
    // one thread per history, at most 2^30 histories (2^22 blocks) per launch
    const uint64_t per_launch = 1ull << 30;
    for (uint64_t off = 0; off < P.n; off += per_launch) {
        Params Q = P;
        Q.first = P.first + off;
        Q.n = P.n - off < per_launch ? P.n - off : per_launch;
        Q.records = P.records ? P.records + off : nullptr;
        void* args[] = {(void*)&Q};
        const hipError_t e =
            hipLaunchKernel(kernels[v], dim3((unsigned)((Q.n + block - 1) / block)), dim3(block), args, 0, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// variant index: FP32: bit 0 scene in LDS, bit 1 daughter grid, bit 2 five
// waves per SIMD (no grid only), bit 3 paired global scores (no grid only);
// FP64 (scene in global memory): 6, grid 7, with first-collision tallies 16, 17;
// + 20 with the world-crossing code (FP32 four-wave per-lane scoring without a
// grid: 20, 21; FP64 without a grid or first-collision tallies: 26)
static int mixed_variant(const Params& P) {
    if (P.fp64) return P.has_fc ? (P.has_grid ? 17 : 16) : (P.has_grid ? 7 : (P.esc == 1 ? 26 : P.esc == 2 ? 27 : 6));
    const int v = (P.scene_in_lds ? 1 : 0) + (P.has_grid ? 2 : 0) + (P.waves == 5 && !P.has_grid ? 4 : 0) +
                  (P.paired && !P.has_grid ? 8 : 0);
    if (P.esc == 1) return v <= 1 ? v + 20 : v;
    // fold passes: built for the LDS-scene instances (the others run without them)
    if (P.esc == 2) return v == 1 ? 28 : v == 9 ? 29 : v == 13 ? 30 : v;
    return v;
}

// the kernel of a variant index
template <bool REC>
static const void* mixed_kernel(int v) {
    switch (v) {
    case 0: return (const void*)k_mixed<float, REC, false, false, 4, false, false, 0>;
    case 1: return (const void*)k_mixed<float, REC, true, false, 4, false, false, 0>;
    case 2: return (const void*)k_mixed<float, REC, false, true, 4, false, false, 0>;
    case 3: return (const void*)k_mixed<float, REC, true, true, 4, false, false, 0>;
    case 4: return (const void*)k_mixed<float, REC, false, false, 5, false, false, 0>;
    case 5: return (const void*)k_mixed<float, REC, true, false, 5, false, false, 0>;
    case 6: return (const void*)k_mixed<double, REC, false, false, 2, false, false, 0>;
    case 7: return (const void*)k_mixed<double, REC, false, true, 3, false, false, 0>;
    case 8: return (const void*)k_mixed<float, REC, false, false, 4, true, false, 0>;
    case 9: return (const void*)k_mixed<float, REC, true, false, 4, true, false, 0>;
    case 12: return (const void*)k_mixed<float, REC, false, false, 5, true, false, 0>;
    case 13: return (const void*)k_mixed<float, REC, true, false, 5, true, false, 0>;
    case 16: return (const void*)k_mixed<double, REC, false, false, 2, false, true, 0>;
    case 17: return (const void*)k_mixed<double, REC, false, true, 3, false, true, 0>;
    case 20: return (const void*)k_mixed<float, REC, false, false, 4, false, false, 1>;
    case 21: return (const void*)k_mixed<float, REC, true, false, 4, false, false, 1>;
    case 26: return (const void*)k_mixed<double, REC, false, false, 2, false, false, 1>;
    case 27: return (const void*)k_mixed<double, REC, false, false, 2, false, false, 2>;
    case 28: return (const void*)k_mixed<float, REC, true, false, 4, false, false, 2>;
    case 29: return (const void*)k_mixed<float, REC, true, false, 4, true, false, 2>;
    case 30: return (const void*)k_mixed<float, REC, true, false, 5, true, false, 2>;
    default: return nullptr;   // no such variant: the launch reports an error
    }
}

hipError_t launch_mixed(const Params& P, bool rec, int grid, int block, hipStream_t st) {
    if (P.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, P.counter, 1);
    const int lds = mixed_lds_bytes(P);
    const int v = mixed_variant(P);
    const void* k = rec ? mixed_kernel<true>(v) : mixed_kernel<false>(v);
    if (!k) return hipErrorInvalidDeviceFunction;
    void* args[] = {(void*)&P};
    return hipLaunchKernel(k, dim3(grid), dim3(block), args, (size_t)lds, st);
}

int mixed_occupancy(const Params& P, int block) {
    int nb = 0;
    const int lds = mixed_lds_bytes(P);
    const void* k = mixed_kernel<false>(mixed_variant(P));
    if (!k) return 1;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, block, lds);
    if (e != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

int batch_lds_bytes(const BatchParams& B) {
    const int nslots = B.cache_bits > 0 ? (1 << B.cache_bits) : 0;
    return B.lds_tally_doubles * 8 + align16(nslots * 4) + B.lds_scene_bytes;
}

// variant index: bit 0 scene in LDS, bit 1 daughter grid, bit 2 five waves per SIMD (no grid only)
static int batch_variant(const BatchParams& B, bool slds, bool grid_nav) {
    return (slds ? 1 : 0) + (grid_nav ? 2 : 0) + (B.waves == 5 && !grid_nav ? 4 : 0);
}

// one persistent launch per (scene placement, grid) class of simulations
hipError_t launch_batch(const BatchParams& B, bool slds, bool grid_nav, int grid, int block, hipStream_t st) {
    if (B.total_histories == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u64, dim3((B.nsims + 63) / 64), dim3(64), 0, st, B.sim_next, B.nsims);
    const int lds = batch_lds_bytes(B);
    switch (batch_variant(B, slds, grid_nav)) {
    case 0: hipLaunchKernelGGL((k_batch<false, false, 4>), dim3(grid), dim3(block), lds, st, B); break;
    case 1: hipLaunchKernelGGL((k_batch<true, false, 4>), dim3(grid), dim3(block), lds, st, B); break;
    case 2: hipLaunchKernelGGL((k_batch<false, true, 4>), dim3(grid), dim3(block), lds, st, B); break;
    case 3: hipLaunchKernelGGL((k_batch<true, true, 4>), dim3(grid), dim3(block), lds, st, B); break;
    case 4: hipLaunchKernelGGL((k_batch<false, false, 5>), dim3(grid), dim3(block), lds, st, B); break;
    default: hipLaunchKernelGGL((k_batch<true, false, 5>), dim3(grid), dim3(block), lds, st, B); break;
    }
    return hipGetLastError();
}

int batch_occupancy(const BatchParams& B, bool slds, bool grid_nav, int block) {
    int nb = 0;
    const int lds = batch_lds_bytes(B);
    hipError_t e;
    switch (batch_variant(B, slds, grid_nav)) {
    case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<false, false, 4>, block, lds); break;
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<true, false, 4>, block, lds); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<false, true, 4>, block, lds); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<true, true, 4>, block, lds); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<false, false, 5>, block, lds); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<true, false, 5>, block, lds); break;
    }
    if (e != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

hipError_t prepared_tail(unsigned long long* const* hist, const unsigned long long* add, int n,
                         unsigned long long* shift, unsigned long long stride, hipStream_t st) {
    hipLaunchKernelGGL(k_prepared_tail, dim3((n + 255) / 256 > 0 ? (n + 255) / 256 : 1), dim3(256), 0, st, hist, add, n,
                       shift, stride);
    return hipGetLastError();
}

hipError_t zero_u64(unsigned long long* p, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_u64, dim3((n + 63) / 64), dim3(64), 0, st, p, n);
    return hipGetLastError();
}

hipError_t zero_f64(double* p, uint64_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

}  // namespace prk
