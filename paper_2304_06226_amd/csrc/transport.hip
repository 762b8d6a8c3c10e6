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
// Batched (k_batch): the mixed policy over many simulations at once; each
//   lane carries its history's simulation, waves claim chunks of one
//   simulation at a time from a shared chunk space, scenes are read from
//   global memory and one LDS bin cache serves every simulation's tallies.
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

// ------------------------------------------------------------------------
// FP64 plain
// ------------------------------------------------------------------------

template <bool REC>
__global__ __launch_bounds__(256) void k_plain(Params P) {
    const SceneT<double> S{P.vols_d, P.mats_d, P.fams_d, P.children, P.grids_d, P.cell_start, P.cell_items};
    Counters cnt = {};
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P.n) {
        PState<double> s;
        source<double, REC>(s, P.src, S, P.seed, P.first + i, 0);
        while (s.term == 0) step<double, REC>(s, S, P.seed);
        if (s.term == PR_END_ESCAPE || s.term == PR_END_ABSORB || s.term == PR_END_DETECT) {
            for (int t = 0; t < P.n_tallies; ++t) {
                const TallyDev& T = P.tallies[t];
                int64_t b = tally_bin<double>(T, s);
                if (b >= 0) {
                    atomicAdd(T.sw + b, s.w);
                    atomicAdd(T.sw2 + b, s.w * s.w);
                }
            }
        }
        if (REC) write_record<double>(P.records + i, s);
        count_end<double>(cnt, s);
    }
    flush_counters(cnt, P.stats);
}

// ------------------------------------------------------------------------
// FP32 mixed, persistent
// ------------------------------------------------------------------------

// LDS of a mixed-policy block: [privatised tallies (doubles)] [bin-cache values
// (2 doubles per slot)] [bin-cache keys (u32 per slot)] [scene, when staged:
// volumes, materials, Bragg tables, daughter lists, grids, grid cells]
struct LdsLayout {
    int cache_vals, cache_keys, vols, mats, fams, children, grids, cell_start, cell_items, bytes;   // byte offsets
};

__host__ __device__ inline int align16(int x) { return (x + 15) & ~15; }

__host__ __device__ inline LdsLayout lds_layout(const Params& P) {
    LdsLayout L;
    const int st = P.scene_in_lds ? 1 : 0;
    int off = P.lds_tally_doubles * 8;
    L.cache_vals = off;
    off += P.cache_slots * 16;
    L.cache_keys = off;
    off = align16(off + P.cache_slots * 4);
    L.vols = off;
    off = align16(off + st * P.n_vols * (int)sizeof(VolT<float>));
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
    L.bytes = off;
    return L;
}

constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;

// Score w into bin b of tally T from a mixed-policy lane: the block's
// privatised copy if there is one, else the block's LDS bin cache (a slot is
// claimed by the first bin that hashes to it; two probes), else global atomics.
__device__ __forceinline__ void score_mixed(const TallyDev& T, int64_t b, double w, double* lds, double* cvals,
                                            uint32_t* ckeys) {
    if (T.lds_offset >= 0) {
        atomicAdd(lds + T.lds_offset + b, w);
        atomicAdd(lds + T.lds_offset + T.total + b, w * w);
        return;
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
                return;
            }
        }
    }
    atomicAdd(T.sw + b, w);
    atomicAdd(T.sw2 + b, w * w);
}

__device__ __forceinline__ void copy_words(void* dst, const void* src, int bytes) {
    const uint32_t* s = (const uint32_t*)src;
    uint32_t* d = (uint32_t*)dst;
    for (int i = threadIdx.x; i < bytes / 4; i += blockDim.x) d[i] = s[i];
}

template <bool REC, bool SLDS>
__global__ __launch_bounds__(256) void k_mixed(Params P) {
    extern __shared__ double lds[];
    const LdsLayout L = lds_layout(P);
    char* base = (char*)lds;
    double* cvals = (double*)(base + L.cache_vals);
    uint32_t* ckeys = (uint32_t*)(base + L.cache_keys);
    if (SLDS) {
        copy_words(base + L.vols, P.vols_f, P.n_vols * (int)sizeof(VolT<float>));
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
    const SceneT<float> S =
        SLDS ? SceneT<float>{(const VolT<float>*)(base + L.vols), (const MatT<float>*)(base + L.mats),
                             (const FamT<float>*)(base + L.fams), (const int32_t*)(base + L.children),
                             (const GridT<float>*)(base + L.grids), (const int32_t*)(base + L.cell_start),
                             (const int32_t*)(base + L.cell_items)}
             : SceneT<float>{P.vols_f, P.mats_f, P.fams_f, P.children, P.grids_f, P.cell_start, P.cell_items};

    Counters cnt = {};
    PState<float> s;
    s.term = 1;            // idle, no history
    bool pending = false;  // finished history not yet scored
    bool exhausted = false;
    // the wave's current chunk of history indices [cnext, cend), claimed with one
    // atomic per chunk; values are wave-uniform
    unsigned long long cnext = 0, cend = 0;
    const unsigned long long chunk = (unsigned long long)P.chunk;
    const int lane = lane_id();
    for (;;) {
        const bool idle = s.term != 0;
        const unsigned long long idle_mask = __ballot(idle);
        const int n_idle = __popcll(idle_mask);
        if (n_idle >= P.refill_threshold || n_idle == kWave) {
            // score the histories that ended since the last refill, all together
            if (pending) {
                if (s.term == PR_END_ESCAPE || s.term == PR_END_ABSORB || s.term == PR_END_DETECT) {
                    for (int t = 0; t < P.n_tallies; ++t) {
                        const TallyDev& T = P.tallies[t];
                        int64_t b = tally_bin<float>(T, s);
                        if (b >= 0) score_mixed(T, b, s.w, lds, cvals, ckeys);
                    }
                }
                if (REC) write_record<float>(P.records + (s.h - P.first), s);
                count_end<float>(cnt, s);
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
                if (idle) {
                    const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(idle_mask >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)idle_mask, 0u));
                    if ((unsigned long long)rank < take) {
                        source<float, REC>(s, P.src, S, P.seed, P.first + cnext + (unsigned long long)rank, 0);
                        pending = s.term != 0;   // born outside the world: counted at the next refill
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
        if (s.term == 0) {
            step<float, REC>(s, S, P.seed);
            pending = s.term != 0;
        }
    }
    flush_counters(cnt, P.stats);
    __syncthreads();
    // merge the block's privatised tallies and cached bins (non-zero bins only)
    for (int t = 0; t < P.n_tallies; ++t) {
        const TallyDev& T = P.tallies[t];
        if (T.cache_base >= 0) {
            const int ns = 1 << T.cache_bits;
            for (int i = threadIdx.x; i < ns; i += blockDim.x) {
                const int slot = T.cache_base + i;
                const uint32_t key = ckeys[slot];
                if (key != kEmptyKey) {
                    atomicAdd(T.sw + key, cvals[2 * slot]);
                    atomicAdd(T.sw2 + key, cvals[2 * slot + 1]);
                }
            }
        }
        if (T.lds_offset < 0) continue;
        for (int64_t i = threadIdx.x; i < T.total; i += blockDim.x) {
            double a = lds[T.lds_offset + i];
            double b = lds[T.lds_offset + T.total + i];
            if (a != 0.0 || b != 0.0) {
                atomicAdd(T.sw + i, a);
                atomicAdd(T.sw2 + i, b);
            }
        }
    }
}

// ------------------------------------------------------------------------
// Batched FP32 mixed: many simulations in one persistent launch
// ------------------------------------------------------------------------

// tally whose key range [base[t], base[t+1]) holds key
__device__ __forceinline__ int tally_of_key(const uint64_t* base, int nt, uint64_t key) {
    int lo = 0, hi = nt - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= key) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ void score_batch(const BatchParams& B, int t, int64_t b, double w, double* cvals,
                                            uint32_t* ckeys) {
    const TallyDev& T = B.tallies[t];
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
                atomicAdd(cvals + 2 * slot, w);
                atomicAdd(cvals + 2 * slot + 1, w * w);
                return;
            }
        }
    }
    atomicAdd(T.sw + b, w);
    atomicAdd(T.sw2 + b, w * w);
}

__global__ __launch_bounds__(256) void k_batch(BatchParams B) {
    extern __shared__ double lds[];
    const int nslots = B.cache_bits > 0 ? (1 << B.cache_bits) : 0;
    double* cvals = lds;
    uint32_t* ckeys = (uint32_t*)(lds + 2 * nslots);
    for (int i = threadIdx.x; i < 2 * nslots; i += blockDim.x) cvals[i] = 0.0;
    for (int i = threadIdx.x; i < nslots; i += blockDim.x) ckeys[i] = kEmptyKey;
    __syncthreads();
    const SceneT<float> S{B.vols, B.mats, B.fams, B.children, B.grids, B.cell_start, B.cell_items};

    Counters cnt = {};
    PState<float> s;
    s.term = 1;
    int sim = 0;            // simulation of this lane's history
    bool pending = false;
    bool exhausted = false;
    // wave-uniform: the claimed chunk's simulation and its local history range
    int csim = 0;
    unsigned long long cnext = 0, cend = 0;
    const int lane = lane_id();
    for (;;) {
        const bool idle = s.term != 0;
        const unsigned long long idle_mask = __ballot(idle);
        const int n_idle = __popcll(idle_mask);
        if (n_idle >= B.refill_threshold || n_idle == kWave) {
            if (pending) {
                if (s.term == PR_END_ESCAPE || s.term == PR_END_ABSORB || s.term == PR_END_DETECT) {
                    const SimDev& sd = B.sims[sim];
                    for (int t = sd.tally_begin; t < sd.tally_begin + sd.tally_count; ++t) {
                        int64_t b = tally_bin<float>(B.tallies[t], s);
                        if (b >= 0) score_batch(B, t, b, s.w, cvals, ckeys);
                    }
                }
                count_end<float>(cnt, s);
                pending = false;
            }
            if (!exhausted && cnext >= cend) {
                const int leader = __ffsll((long long)idle_mask) - 1;
                unsigned long long got = 0;
                if (lane == leader) got = atomicAdd(B.counter, 1ull);
                got = __shfl(got, leader, kWave);
                if (got >= B.total_chunks) {
                    exhausted = true;
                } else {
                    // simulation owning chunk `got`: last with chunk_begin <= got
                    int lo = 0, hi = B.nsims - 1;
                    while (lo < hi) {
                        int mid = (lo + hi + 1) >> 1;
                        if (B.sims[mid].chunk_begin <= got) lo = mid; else hi = mid - 1;
                    }
                    csim = lo;
                    const unsigned long long l0 = (got - B.sims[lo].chunk_begin) * B.chunk;
                    cnext = l0;
                    cend = l0 + B.chunk < B.sims[lo].n ? l0 + B.chunk : B.sims[lo].n;
                }
            }
            if (!exhausted && cnext < cend) {
                const unsigned long long avail = cend - cnext;
                const unsigned long long take = (unsigned long long)n_idle < avail ? (unsigned long long)n_idle : avail;
                if (idle) {
                    const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(idle_mask >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)idle_mask, 0u));
                    if ((unsigned long long)rank < take) {
                        const SimDev& sd = B.sims[csim];
                        sim = csim;
                        source<float, false>(s, sd.src, S, B.seed, sd.first + cnext + (unsigned long long)rank, sd.root);
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
            step<float, false>(s, S, B.seed);
            pending = s.term != 0;
        }
    }
    flush_counters(cnt, B.stats);
    __syncthreads();
    for (int i = threadIdx.x; i < nslots; i += blockDim.x) {
        const uint32_t key = ckeys[i];
        if (key == kEmptyKey) continue;
        const int t = tally_of_key(B.tally_key_base, B.ntallies, key);
        const TallyDev& T = B.tallies[t];
        const uint64_t b = key - B.tally_key_base[t];
        atomicAdd(T.sw + b, cvals[2 * i]);
        atomicAdd(T.sw2 + b, cvals[2 * i + 1]);
    }
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

hipError_t launch_plain(const Params& P, bool rec, hipStream_t st) {
    if (P.n == 0) return hipSuccess;
    const int block = 256;
    uint64_t grid = (P.n + block - 1) / block;
    if (rec)
        hipLaunchKernelGGL(k_plain<true>, dim3((unsigned)grid), dim3(block), 0, st, P);
    else
        hipLaunchKernelGGL(k_plain<false>, dim3((unsigned)grid), dim3(block), 0, st, P);
    return hipGetLastError();
}

hipError_t launch_mixed(const Params& P, bool rec, int grid, int block, hipStream_t st) {
    if (P.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, P.counter, 1);
    int lds = mixed_lds_bytes(P);
    if (P.scene_in_lds) {
        if (rec)
            hipLaunchKernelGGL((k_mixed<true, true>), dim3(grid), dim3(block), lds, st, P);
        else
            hipLaunchKernelGGL((k_mixed<false, true>), dim3(grid), dim3(block), lds, st, P);
    } else {
        if (rec)
            hipLaunchKernelGGL((k_mixed<true, false>), dim3(grid), dim3(block), lds, st, P);
        else
            hipLaunchKernelGGL((k_mixed<false, false>), dim3(grid), dim3(block), lds, st, P);
    }
    return hipGetLastError();
}

int mixed_occupancy(const Params& P, int block) {
    int nb = 0;
    int lds = mixed_lds_bytes(P);
    hipError_t e = P.scene_in_lds
                       ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_mixed<false, true>, block, lds)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_mixed<false, false>, block, lds);
    if (e != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

int batch_lds_bytes(const BatchParams& B) { return B.cache_bits > 0 ? (1 << B.cache_bits) * 20 : 0; }

hipError_t launch_batch(const BatchParams& B, int grid, int block, hipStream_t st) {
    if (B.total_chunks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, B.counter, 1);
    hipLaunchKernelGGL(k_batch, dim3(grid), dim3(block), batch_lds_bytes(B), st, B);
    return hipGetLastError();
}

int batch_occupancy(const BatchParams& B, int block) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch, block, batch_lds_bytes(B)) != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
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
