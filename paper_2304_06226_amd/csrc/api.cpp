// C-ABI of prompt_mi355x: object creation with validation, scene building,
// run orchestration and result readback.  See include/prompt_mi355x.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/prompt_mi355x.h"
#include "device.h"
#include "launch.h"

using namespace prk;

namespace {

struct Material {
    pr_material_desc desc;
    std::vector<double> d, f2;
    std::vector<int32_t> mult;
    std::vector<double> tl, ta, ti;   // tabulated lambda, sigma_abs, sigma_inc (empty: analytic)
};

struct Geometry {
    std::vector<pr_volume_desc> vols;
    bool esc = false;    // some volume is marked exit_escapes
    bool fold = false;   // no mirrors, and some material volume sits in a vacuum one (FP32 fold passes apply)
    // host copies of the device scene (batched runs concatenate them)
    std::vector<VolT<double>> vd;
    std::vector<VolT<float>> vf;
    std::vector<MatT<double>> md;
    std::vector<MatT<float>> mf;
    std::vector<FamT<double>> fd;
    std::vector<FamT<float>> ff;
    std::vector<int32_t> children, cell_start, cell_items;
    std::vector<GridT<double>> gd;
    std::vector<GridT<float>> gf;
    std::vector<BoxT<double>> bd;   // box bounds by volume index (grid navigation)
    std::vector<BoxT<float>> bf;
    int nv = 0, nm = 0, nf = 0, nc = 0;
    uint32_t kinds = 0;   // bit k: some volume has solid kind k
    void* vols_d = nullptr;
    void* mats_d = nullptr;
    void* fams_d = nullptr;
    void* vols_f = nullptr;
    void* mats_f = nullptr;
    void* fams_f = nullptr;
    void* children_d = nullptr;
    void* grids_d = nullptr;
    void* grids_f = nullptr;
    void* cell_start_d = nullptr;
    void* cell_items_d = nullptr;
    void* boxes_d = nullptr;
    void* boxes_f = nullptr;
    int scene_f_bytes = 0;   // FP32 scene size (LDS staging decision)
    int scene_lds_bytes = 0; // LDS the FP32 scene takes when staged (grid scenes: all but the volume table)
};

struct Tally {
    pr_tally_desc desc;
    uint64_t nbins = 0;
    double* dev = nullptr;   // (sum_w, sum_w2) interleaved per bin
    bool owned = true;       // false: the caller's storage (pr_create_tally_in), never freed here
    uint64_t n_hist = 0;     // histories of host-issued runs
    unsigned long long* dev_nhist = nullptr;   // histories counted on the device (prepared batches)
};

// Per-call batch descriptors (simulations, tallies, key bases): a small ring of
// device buffers filled from pinned host staging, each reused only after the
// event recorded behind its last launch has completed.
struct DescSlot {
    void* dev = nullptr;
    void* host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    bool used = false;
};

}  // namespace

// One class of a batched run, planned on the host: descriptors and launch shape.
struct ClassPlan {
    std::vector<SimDev> sd;
    std::vector<TallyDev> td;
    std::vector<uint64_t> kb;
    BatchParams B{};        // device pointers set by bind_plan
    bool slds = false, grid_nav = false;
    int grid = 1, block = 256;
    size_t b_sims = 0, b_tal = 0, b_kb = 0, total = 0;   // descriptor layout [sims | tallies | key bases | counters]
};

// A batch uploaded once for repeated, capturable runs.
struct PreparedBatch {
    bool live = false;
    std::vector<ClassPlan> plans;
    std::vector<void*> desc;                  // device descriptors per class
    unsigned long long* shift = nullptr;      // device: history-id offset of the next run
    uint64_t stride = 0;
    unsigned long long** hist_ptrs = nullptr; // device: history counters of the tallies involved
    unsigned long long* hist_add = nullptr;   // device: histories added to each per run
    int nh = 0;
};

// Device scratch of pr_run_batch_static: the staged descriptors of a batch
// (simulations, tally entries, bin-cache key bases) and its per-simulation
// claim counters.  Each GPU the library runs on holds its own copy until the
// process ends.  Host code never uses the array's name as an address: at
// pr_init the device copy's address is looked up once per device
// (hipGetSymbolAddress) and kept in g_scratch_dev.
constexpr size_t kStaticScratchBytes = 2u << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
static void* g_scratch_dev[kMaxDevices] = {};
static std::mutex g_scratch_mutex;

// History-claim counters of runs without a caller workspace: a ring of slots,
// each reused only after the stream of its next run has waited for the event
// recorded behind the last run that used it, so runs on different streams never
// share a counter while they overlap.
constexpr int kRunSlots = 64;
constexpr size_t kRunSlotBytes = 256;   // one counter per slot, slots 256 bytes apart

struct pr_ctx {
    int device = -1;
    uint64_t seed = 4096;
    std::string err;
    std::vector<Material> mats;
    std::vector<Geometry> geoms;
    std::vector<pr_source_desc> srcs;
    std::vector<Tally> tallies;
    unsigned long long* stats = nullptr;
    char* run_slots = nullptr;              // kRunSlots x kRunSlotBytes of device memory
    hipEvent_t run_done[kRunSlots] = {};
    bool run_used[kRunSlots] = {};
    int next_run_slot = 0;
    int num_cus = 256;
    // launch tuning of the mixed policy
    int mixed_block = 256;
    int mixed_blocks_per_cu = 0;        // 0 = occupancy limit
    int refill_threshold = 16;
    int lds_tally_budget = 32768;       // bytes of LDS per block for privatised tallies
    int bin_cache_slots = 1024;         // LDS bin-cache slots per non-privatised tally (power of two, 0 = off)
    int chunk = 256;                    // history indices a wave claims per atomic
    int grid_chunk = 0;                 // claim size for scenes with a daughter grid (0: chunk)
    int lds_scene_budget = 16384;       // FP32 scenes up to this size are staged into LDS
    int lds_grid_budget = 98304;        // grid scenes: staged part (grid, box bounds, tables) up to this size
    int grid_walk_cells = 0;            // FP32 grid walks pause after this many cells (0: never)
    int vacuum_steps = 1;               // take steps that draw nothing early where the scene allows (0: never)
    DescSlot slots[4];
    int waves_per_simd = 4;             // FP32 kernels without a grid: variant built for 4 or 5 waves per SIMD
    double* scratch = nullptr;          // autotuner: tally scratch (trial runs score here)
    uint64_t scratch_bins = 0;
    unsigned long long* scratch_stats = nullptr;
    int next_slot = 0;
    std::vector<PreparedBatch> prepared;
    void* static_scratch = nullptr;     // this device's copy of `scratch` (pr_run_batch_static)
    std::vector<char> static_host;      // host image of the descriptors staged there
};

namespace {

int fail(pr_ctx* c, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

int hipfail(pr_ctx* c, hipError_t e, const char* what) {
    return fail(c, PR_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(ctx, call)                                   \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hipfail(ctx, e_, #call); \
    } while (0)

bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

// ---- geometry helpers (host, double) ----

struct Box3 {
    double lo[3], hi[3];
};

Box3 aabb(const pr_volume_desc& v) {
    Box3 b;
    double e[3] = {0, 0, 0};
    switch (v.kind) {
    case PR_BOX: e[0] = 0.5 * v.size[0]; e[1] = 0.5 * v.size[1]; e[2] = 0.5 * v.size[2]; break;
    case PR_CYLINDER:
    case PR_CYL_SHELL: {
        double r = v.kind == PR_CYLINDER ? v.size[0] : v.size[1];
        double h = v.kind == PR_CYLINDER ? v.size[1] : v.size[2];
        e[0] = e[1] = e[2] = r;
        e[v.axis] = 0.5 * h;
        break;
    }
    case PR_SPHERE: e[0] = e[1] = e[2] = v.size[0]; break;
    default: e[0] = e[1] = e[2] = v.size[1]; break;
    }
    for (int k = 0; k < 3; ++k) {
        b.lo[k] = v.center[k] - e[k];
        b.hi[k] = v.center[k] + e[k];
    }
    return b;
}

// point inside the solid; strict excludes the boundary
bool inside(const pr_volume_desc& v, const double p[3], bool strict) {
    double q[3] = {p[0] - v.center[0], p[1] - v.center[1], p[2] - v.center[2]};
    auto le = [strict](double a, double b) { return strict ? a < b : a <= b; };
    switch (v.kind) {
    case PR_BOX:
        return le(std::fabs(q[0]), 0.5 * v.size[0]) && le(std::fabs(q[1]), 0.5 * v.size[1]) &&
               le(std::fabs(q[2]), 0.5 * v.size[2]);
    case PR_CYLINDER:
    case PR_CYL_SHELL: {
        int a = v.axis, b = (a + 1) % 3, c = (a + 2) % 3;
        double rho = std::sqrt(q[b] * q[b] + q[c] * q[c]);
        double ro = v.kind == PR_CYLINDER ? v.size[0] : v.size[1];
        double h = v.kind == PR_CYLINDER ? v.size[1] : v.size[2];
        bool in = le(rho, ro) && le(std::fabs(q[a]), 0.5 * h);
        if (v.kind == PR_CYL_SHELL) in = in && le(v.size[0], rho);
        return in;
    }
    case PR_SPHERE: return le(std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]), v.size[0]);
    default: {
        double r = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
        return le(r, v.size[1]) && le(v.size[0], r);
    }
    }
}

// deterministic sample of points on the solid's surfaces
void surface_points(const pr_volume_desc& v, std::vector<std::array<double, 3>>& out) {
    out.clear();
    const double PI = 3.14159265358979323846;
    auto add = [&](double x, double y, double z) { out.push_back({v.center[0] + x, v.center[1] + y, v.center[2] + z}); };
    if (v.kind == PR_BOX) {
        double h[3] = {0.5 * v.size[0], 0.5 * v.size[1], 0.5 * v.size[2]};
        const int g = 17;
        for (int f = 0; f < 3; ++f)
            for (int s = -1; s <= 1; s += 2)
                for (int i = 0; i < g; ++i)
                    for (int j = 0; j < g; ++j) {
                        double p[3];
                        int a = (f + 1) % 3, b = (f + 2) % 3;
                        p[f] = s * h[f];
                        p[a] = h[a] * (2.0 * i / (g - 1) - 1.0);
                        p[b] = h[b] * (2.0 * j / (g - 1) - 1.0);
                        add(p[0], p[1], p[2]);
                    }
        return;
    }
    auto cyl = [&](double r, double hh, bool caps_annulus_from) {
        int a = v.axis, b = (a + 1) % 3, c = (a + 2) % 3;
        for (int i = 0; i < 96; ++i)
            for (int j = 0; j < 17; ++j) {
                double p[3];
                double ph = 2 * PI * i / 96;
                p[b] = r * std::cos(ph);
                p[c] = r * std::sin(ph);
                p[a] = hh * (2.0 * j / 16 - 1.0);
                add(p[0], p[1], p[2]);
            }
        (void)caps_annulus_from;
    };
    if (v.kind == PR_CYLINDER || v.kind == PR_CYL_SHELL) {
        int a = v.axis, b = (a + 1) % 3, c = (a + 2) % 3;
        double rin = v.kind == PR_CYLINDER ? 0.0 : v.size[0];
        double rout = v.kind == PR_CYLINDER ? v.size[0] : v.size[1];
        double hh = 0.5 * (v.kind == PR_CYLINDER ? v.size[1] : v.size[2]);
        cyl(rout, hh, false);
        if (v.kind == PR_CYL_SHELL) cyl(rin, hh, false);
        for (int s = -1; s <= 1; s += 2)
            for (int i = 0; i < 9; ++i)
                for (int j = 0; j < 48; ++j) {
                    double p[3];
                    double r = rin + (rout - rin) * i / 8.0;
                    double ph = 2 * PI * j / 48;
                    p[b] = r * std::cos(ph);
                    p[c] = r * std::sin(ph);
                    p[a] = s * hh;
                    add(p[0], p[1], p[2]);
                }
        return;
    }
    auto sph = [&](double r) {
        for (int i = 0; i <= 32; ++i)
            for (int j = 0; j < 64; ++j) {
                double th = PI * i / 32, ph = 2 * PI * j / 64;
                add(r * std::sin(th) * std::cos(ph), r * std::sin(th) * std::sin(ph), r * std::cos(th));
            }
    };
    if (v.kind == PR_SPHERE) {
        sph(v.size[0]);
    } else {
        sph(v.size[0]);
        sph(v.size[1]);
    }
}

bool boxes_apart(const Box3& a, const Box3& b) {
    for (int k = 0; k < 3; ++k)
        if (a.hi[k] < b.lo[k] || b.hi[k] < a.lo[k]) return true;
    return false;
}

bool box_inside(const Box3& in, const Box3& out) {
    for (int k = 0; k < 3; ++k)
        if (!(in.lo[k] > out.lo[k] && in.hi[k] < out.hi[k])) return false;
    return true;
}

template <class T>
int upload(pr_ctx* c, void** dst, const std::vector<T>& v) {
    size_t bytes = std::max<size_t>(v.size() * sizeof(T), 16);
    HIPCHK(c, hipMalloc(dst, bytes));
    if (!v.empty()) HIPCHK(c, hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return PR_OK;
}

void free_prepared(PreparedBatch& pb) {
    for (void* d : pb.desc)
        if (d) (void)hipFree(d);
    pb.desc.clear();
    pb.plans.clear();
    if (pb.shift) (void)hipFree(pb.shift);
    if (pb.hist_ptrs) (void)hipFree(pb.hist_ptrs);
    if (pb.hist_add) (void)hipFree(pb.hist_add);
    pb.shift = nullptr;
    pb.hist_ptrs = nullptr;
    pb.hist_add = nullptr;
    pb.nh = 0;
    pb.live = false;
}

void free_geometry(Geometry& g) {
    void** ps[] = {&g.vols_d, &g.mats_d, &g.fams_d, &g.vols_f, &g.mats_f, &g.fams_f, &g.children_d,
                   &g.grids_d, &g.grids_f, &g.cell_start_d, &g.cell_items_d, &g.boxes_d, &g.boxes_f};
    for (void** p : ps) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
}

// Uniform grid over the daughters of volume `v` (bounding boxes padded so that
// cell assignment is conservative against rounding of the cell index).
void build_grid(const pr_volume_desc* vols, const std::vector<int32_t>& kids, Geometry& g, int v) {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    std::vector<Box3> bb;
    for (int c : kids) {
        Box3 b = aabb(vols[c]);
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], b.lo[k]);
            hi[k] = std::max(hi[k], b.hi[k]);
        }
        bb.push_back(b);
    }
    double ext[3], vol = 1.0;
    for (int k = 0; k < 3; ++k) {
        ext[k] = std::max(hi[k] - lo[k], 1e-6);
        vol *= ext[k];
    }
    const double target = 4.0 * (double)kids.size();
    const double h = std::cbrt(vol / target);
    GridT<double> G{};
    for (int k = 0; k < 3; ++k) {
        int n = (int)std::ceil(ext[k] / h);
        n = std::max(1, std::min(n, 128));
        G.n[k] = n;
        G.cell[k] = ext[k] / n;
        G.inv_cell[k] = 1.0 / G.cell[k];
        G.lo[k] = lo[k];
        G.hi[k] = lo[k] + n * G.cell[k];
    }
    const int ncell = G.n[0] * G.n[1] * G.n[2];
    std::vector<std::vector<int32_t>> cells(ncell);
    for (size_t i = 0; i < kids.size(); ++i) {
        int r0[3], r1[3];
        for (int k = 0; k < 3; ++k) {
            const double pad = 1e-4 * G.cell[k];
            r0[k] = std::max(0, std::min(G.n[k] - 1, (int)std::floor((bb[i].lo[k] - pad - G.lo[k]) * G.inv_cell[k])));
            r1[k] = std::max(0, std::min(G.n[k] - 1, (int)std::floor((bb[i].hi[k] + pad - G.lo[k]) * G.inv_cell[k])));
        }
        for (int a = r0[0]; a <= r1[0]; ++a)
            for (int b = r0[1]; b <= r1[1]; ++b)
                for (int c = r0[2]; c <= r1[2]; ++c)
                    cells[(a * G.n[1] + b) * G.n[2] + c].push_back(
                        (int32_t)((uint32_t)kids[i] | ((uint32_t)vols[kids[i]].kind << kItemKindShift) |
                                  (vols[kids[i]].is_detector ? kItemDet : 0u)));
    }
    if (g.cell_start.empty()) g.cell_start.push_back(0);
    G.cells_off = (int32_t)g.cell_start.size() - 1;
    for (auto& cl : cells) {
        g.cell_items.insert(g.cell_items.end(), cl.begin(), cl.end());
        g.cell_start.push_back((int32_t)g.cell_items.size());
    }
    g.gd.push_back(G);
    GridT<float> F{};
    for (int k = 0; k < 3; ++k) {
        F.lo[k] = (float)G.lo[k];
        F.hi[k] = (float)G.hi[k];
        F.cell[k] = (float)G.cell[k];
        F.inv_cell[k] = (float)G.inv_cell[k];
        F.n[k] = G.n[k];
    }
    F.cells_off = G.cells_off;
    g.gf.push_back(F);
    g.vd[v].grid = (int32_t)g.gd.size() - 1;
    g.vf[v].grid = g.vd[v].grid;
}

constexpr int kGridMinDaughters = 8;   // at most 7 daughters are scanned as step candidates

int set_device(pr_ctx* c) {
    if (c->device < 0) return fail(c, PR_EDEVICE, "context has no device (created with hip_device = -1)");
    int cur = -1;
    HIPCHK(c, hipGetDevice(&cur));
    if (cur != c->device) HIPCHK(c, hipSetDevice(c->device));
    return PR_OK;
}

// E = h^2 / (2 m_n lambda^2): the constant in eV A^2 from CODATA 2018
double ev_angstrom2() {
    const double h = 6.62607015e-34, mn = 1.67492749804e-27, ev = 1.602176634e-19;
    return h * h / (2.0 * mn) / ev * 1e20;
}

}  // namespace

// =========================================================================
// context
// =========================================================================

extern "C" int pr_init(pr_ctx** out, int hip_device, uint64_t seed) {
    if (!out) return PR_EINVAL;
    *out = nullptr;
    pr_ctx* c = new (std::nothrow) pr_ctx();
    if (!c) return PR_ENOMEM;
    c->seed = seed;
    c->device = hip_device;
    if (hip_device >= 0) {
        int n = 0;
        hipError_t e = hipGetDeviceCount(&n);
        if (e != hipSuccess || hip_device >= n) {
            delete c;
            return PR_EDEVICE;
        }
        bool ok = hipSetDevice(hip_device) == hipSuccess &&
                  hipMalloc((void**)&c->stats, ST_N * sizeof(unsigned long long)) == hipSuccess &&
                  hipMalloc((void**)&c->run_slots, kRunSlots * kRunSlotBytes) == hipSuccess &&
                  hipMemset(c->stats, 0, ST_N * sizeof(unsigned long long)) == hipSuccess;
        for (int i = 0; ok && i < kRunSlots; ++i)
            ok = hipEventCreateWithFlags(&c->run_done[i], hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            for (int i = 0; i < kRunSlots; ++i)
                if (c->run_done[i]) (void)hipEventDestroy(c->run_done[i]);
            if (c->stats) (void)hipFree(c->stats);
            if (c->run_slots) (void)hipFree(c->run_slots);
            delete c;
            return PR_EDEVICE;
        }
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, hip_device) == hipSuccess && cus > 0)
            c->num_cus = cus;
        // this device's copy of the static scratch, looked up once per device
        if (hip_device < kMaxDevices) {
            std::lock_guard<std::mutex> lock(g_scratch_mutex);
            if (!g_scratch_dev[hip_device]) {
                void* ptr = nullptr;
                if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess && ptr) g_scratch_dev[hip_device] = ptr;
            }
            c->static_scratch = g_scratch_dev[hip_device];
        }
    }
    *out = c;
    return PR_OK;
}

extern "C" void pr_destroy(pr_ctx* c) {
    if (!c) return;
    if (c->device >= 0) {
        (void)hipSetDevice(c->device);
        (void)hipDeviceSynchronize();
        for (auto& g : c->geoms) free_geometry(g);
        for (auto& t : c->tallies) {
            if (t.dev && t.owned) (void)hipFree(t.dev);
            if (t.dev_nhist) (void)hipFree(t.dev_nhist);
        }
        for (auto& pb : c->prepared) free_prepared(pb);
        if (c->stats) (void)hipFree(c->stats);
        if (c->run_slots) (void)hipFree(c->run_slots);
        for (int i = 0; i < kRunSlots; ++i)
            if (c->run_done[i]) (void)hipEventDestroy(c->run_done[i]);
        if (c->scratch) (void)hipFree(c->scratch);
        if (c->scratch_stats) (void)hipFree(c->scratch_stats);
        for (auto& sl : c->slots) {
            if (sl.dev) (void)hipFree(sl.dev);
            if (sl.host) (void)hipHostFree(sl.host);
            if (sl.done) (void)hipEventDestroy(sl.done);
        }
    }
    delete c;
}

extern "C" const char* pr_last_error(const pr_ctx* c) { return c ? c->err.c_str() : "null context"; }

extern "C" int pr_set_seed(pr_ctx* c, uint64_t seed) {
    if (!c) return PR_EINVAL;
    c->seed = seed;
    return PR_OK;
}

// =========================================================================
// materials
// =========================================================================

extern "C" int pr_create_material(pr_ctx* c, const pr_material_desc* d, int32_t* id) {
    if (!c || !d || !id) return fail(c, PR_EINVAL, "null argument");
    if (!(std::isfinite(d->number_density) && d->number_density > 0))
        return fail(c, PR_EINVAL, "material.number_density must be > 0");
    if (!finite_nonneg(d->sigma_inc)) return fail(c, PR_EINVAL, "material.sigma_inc must be >= 0");
    if (!finite_nonneg(d->sigma_abs_ref)) return fail(c, PR_EINVAL, "material.sigma_abs_ref must be >= 0");
    if (!finite_nonneg(d->scatter_bias)) return fail(c, PR_EINVAL, "material.scatter_bias must be >= 0");
    if (!finite_nonneg(d->abs_bias)) return fail(c, PR_EINVAL, "material.abs_bias must be >= 0");
    if (d->n_families < 0 || d->n_families > 1024) return fail(c, PR_EINVAL, "material.n_families must be in [0, 1024]");
    if (d->n_families > 0) {
        if (!(std::isfinite(d->cell_volume) && d->cell_volume > 0))
            return fail(c, PR_EINVAL, "material.cell_volume must be > 0 with Bragg families");
        if (d->atoms_per_cell <= 0) return fail(c, PR_EINVAL, "material.atoms_per_cell must be > 0 with Bragg families");
        if (!d->d || !d->mult || !d->f2) return fail(c, PR_EINVAL, "material family arrays must not be null");
        for (int j = 0; j < d->n_families; ++j) {
            if (!(std::isfinite(d->d[j]) && d->d[j] > 0)) return fail(c, PR_EINVAL, "material.d[%d] must be > 0", j);
            if (j > 0 && d->d[j] > d->d[j - 1])
                return fail(c, PR_EINVAL, "material.d must be non-increasing (d[%d] > d[%d])", j, j - 1);
            if (d->mult[j] <= 0) return fail(c, PR_EINVAL, "material.mult[%d] must be > 0", j);
            if (!finite_nonneg(d->f2[j])) return fail(c, PR_EINVAL, "material.f2[%d] must be >= 0", j);
        }
    }
    if (d->n_table != 0) {
        if (d->n_table < 2 || d->n_table > 4096) return fail(c, PR_EINVAL, "material.n_table must be 0 or in [2, 4096]");
        if (!d->table_lambda || !d->table_sigma_abs || !d->table_sigma_inc)
            return fail(c, PR_EINVAL, "material table arrays must not be null");
        for (int j = 0; j < d->n_table; ++j) {
            if (!(std::isfinite(d->table_lambda[j]) && d->table_lambda[j] > 0))
                return fail(c, PR_EINVAL, "material.table_lambda[%d] must be > 0", j);
            if (j > 0 && !(d->table_lambda[j] > d->table_lambda[j - 1]))
                return fail(c, PR_EINVAL, "material.table_lambda must increase strictly (row %d)", j);
            if (!finite_nonneg(d->table_sigma_abs[j]) || !finite_nonneg(d->table_sigma_inc[j]))
                return fail(c, PR_EINVAL, "material table cross sections must be >= 0 (row %d)", j);
        }
    }
    Material m;
    m.desc = *d;
    if (d->n_table > 0) {
        m.tl.assign(d->table_lambda, d->table_lambda + d->n_table);
        m.ta.assign(d->table_sigma_abs, d->table_sigma_abs + d->n_table);
        m.ti.assign(d->table_sigma_inc, d->table_sigma_inc + d->n_table);
    }
    m.desc.table_lambda = m.desc.table_sigma_abs = m.desc.table_sigma_inc = nullptr;
    m.d.assign(d->d, d->d + d->n_families);
    m.mult.assign(d->mult, d->mult + d->n_families);
    m.f2.assign(d->f2, d->f2 + d->n_families);
    m.desc.d = nullptr;
    m.desc.mult = nullptr;
    m.desc.f2 = nullptr;
    c->mats.push_back(std::move(m));
    *id = (int32_t)c->mats.size() - 1;
    return PR_OK;
}

// =========================================================================
// geometry
// =========================================================================

static int validate_volume(pr_ctx* c, const pr_volume_desc& v, int i, int nmat) {
    if (v.kind < PR_BOX || v.kind > PR_SPH_SHELL) return fail(c, PR_EINVAL, "volume[%d].kind invalid", i);
    if ((v.kind == PR_CYLINDER || v.kind == PR_CYL_SHELL) && (v.axis < 0 || v.axis > 2))
        return fail(c, PR_EINVAL, "volume[%d].axis must be 0, 1 or 2", i);
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(v.center[k])) return fail(c, PR_EINVAL, "volume[%d].center not finite", i);
    int ns = v.kind == PR_BOX ? 3 : v.kind == PR_CYLINDER ? 2 : v.kind == PR_CYL_SHELL ? 3 : v.kind == PR_SPHERE ? 1 : 2;
    for (int k = 0; k < ns; ++k)
        if (!(std::isfinite(v.size[k]) && v.size[k] > 0)) return fail(c, PR_EINVAL, "volume[%d].size[%d] must be > 0", i, k);
    if ((v.kind == PR_CYL_SHELL || v.kind == PR_SPH_SHELL) && !(v.size[0] < v.size[1]))
        return fail(c, PR_EINVAL, "volume[%d]: shell needs r_in < r_out", i);
    if (v.material < -1 || v.material >= nmat) return fail(c, PR_ENOTFOUND, "volume[%d].material %d unknown", i, v.material);
    if (i == 0 && v.parent != -1) return fail(c, PR_EINVAL, "volume[0] is the world and needs parent -1");
    if (i > 0 && (v.parent < 0 || v.parent >= i)) return fail(c, PR_EINVAL, "volume[%d].parent must be in [0, %d)", i, i);
    if (i == 0 && v.is_detector) return fail(c, PR_EINVAL, "the world cannot be a detector");
    if (v.mirror_mask < 0 || v.mirror_mask > 63) return fail(c, PR_EINVAL, "volume[%d].mirror_mask out of range", i);
    if (v.mirror_mask) {
        const pr_mirror_desc& m = v.mirror;
        if (m.model != PR_MIRROR_LINEAR && m.model != PR_MIRROR_TANH)
            return fail(c, PR_EINVAL, "volume[%d].mirror.model invalid", i);
        if (!(finite_nonneg(m.R0) && m.R0 <= 1.0)) return fail(c, PR_EINVAL, "volume[%d].mirror.R0 must be in [0,1]", i);
        if (!finite_nonneg(m.Qc) || !finite_nonneg(m.alpha) || !finite_nonneg(m.m))
            return fail(c, PR_EINVAL, "volume[%d].mirror parameters must be >= 0", i);
        if (m.model == PR_MIRROR_TANH && !(std::isfinite(m.W) && m.W > 0))
            return fail(c, PR_EINVAL, "volume[%d].mirror.W must be > 0", i);
    }
    const pr_chopper_desc& ch = v.chopper;
    if (ch.n != 0) {
        if (v.kind != PR_CYLINDER) return fail(c, PR_EINVAL, "volume[%d]: a chopper needs a cylinder", i);
        if (i == 0 || v.is_detector) return fail(c, PR_EINVAL, "volume[%d]: a chopper cannot be the world or a detector", i);
        if (ch.n < 1 || ch.n > 1024) return fail(c, PR_EINVAL, "volume[%d].chopper.n must be in [1, 1024]", i);
        if (!finite_nonneg(ch.r) || !std::isfinite(ch.rot_freq) || !std::isfinite(ch.phase))
            return fail(c, PR_EINVAL, "volume[%d].chopper r, rot_freq, phase must be finite (r >= 0)", i);
        if (!(ch.theta0 > 0 && ch.theta0 <= 360.0 / ch.n))
            return fail(c, PR_EINVAL, "volume[%d].chopper.theta0 must be in (0, 360/n]", i);
    }
    return PR_OK;
}

extern "C" int pr_create_geometry(pr_ctx* c, const pr_volume_desc* vols, int32_t n, int32_t* id) {
    if (!c || !vols || !id) return fail(c, PR_EINVAL, "null argument");
    if (n < 1 || n > 100000) return fail(c, PR_EINVAL, "geometry needs 1..100000 volumes");
    const int nmat = (int)c->mats.size();
    for (int i = 0; i < n; ++i) {
        int rc = validate_volume(c, vols[i], i, nmat);
        if (rc) return rc;
    }
    // containment in the mother and separation from sisters
    std::vector<Box3> bb(n);
    for (int i = 0; i < n; ++i) bb[i] = aabb(vols[i]);
    std::vector<std::array<double, 3>> pts, pts2;
    for (int i = 1; i < n; ++i) {
        const pr_volume_desc& mo = vols[vols[i].parent];
        bool ok = box_inside(bb[i], bb[vols[i].parent]);
        if (ok && !(mo.kind == PR_BOX && vols[i].kind == PR_BOX)) {
            surface_points(vols[i], pts);
            for (auto& p : pts)
                if (!inside(mo, p.data(), true)) { ok = false; break; }
        }
        if (!ok) return fail(c, PR_EOVERLAP, "volume[%d] is not strictly inside its mother volume[%d]", i, vols[i].parent);
    }
    // sisters: group by parent, sort by x to prune the pair scan
    std::vector<int> order(n > 0 ? n - 1 : 0);
    for (int i = 1; i < n; ++i) order[i - 1] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return bb[a].lo[0] < bb[b].lo[0]; });
    for (size_t ia = 0; ia < order.size(); ++ia) {
        int a = order[ia];
        for (size_t ib = ia + 1; ib < order.size(); ++ib) {
            int b = order[ib];
            if (bb[b].lo[0] > bb[a].hi[0]) break;
            if (vols[a].parent != vols[b].parent || boxes_apart(bb[a], bb[b])) continue;
            bool clash = vols[a].kind == PR_BOX && vols[b].kind == PR_BOX;   // AABBs of boxes are exact
            if (!clash) {
                surface_points(vols[a], pts);
                for (auto& p : pts)
                    if (inside(vols[b], p.data(), false)) { clash = true; break; }
            }
            if (!clash) {
                surface_points(vols[b], pts2);
                for (auto& p : pts2)
                    if (inside(vols[a], p.data(), false)) { clash = true; break; }
            }
            if (clash) return fail(c, PR_EOVERLAP, "volumes %d and %d overlap or touch", a, b);
        }
    }

    Geometry g;
    g.vols.assign(vols, vols + n);
    // children lists
    std::vector<std::vector<int32_t>> kids(n);
    for (int i = 1; i < n; ++i) kids[vols[i].parent].push_back(i);
    std::vector<int32_t> children;
    std::vector<int32_t> cbeg(n), ccnt(n);
    for (int i = 0; i < n; ++i) {
        cbeg[i] = (int32_t)children.size();
        ccnt[i] = (int32_t)kids[i].size();
        children.insert(children.end(), kids[i].begin(), kids[i].end());
    }
    // materials used, re-indexed in order of first use
    std::vector<int> mat_map(nmat, -1), used;
    for (int i = 0; i < n; ++i) {
        int m = vols[i].material;
        if (m >= 0 && mat_map[m] < 0) { mat_map[m] = (int)used.size(); used.push_back(m); }
    }
    std::vector<VolT<double>> vd(n);
    std::vector<VolT<float>> vf(n);
    for (int i = 0; i < n; ++i) {
        const pr_volume_desc& v = vols[i];
        VolT<double> o{};
        for (int k = 0; k < 3; ++k) o.c[k] = v.center[k];
        switch (v.kind) {
        case PR_BOX: o.s[0] = 0.5 * v.size[0]; o.s[1] = 0.5 * v.size[1]; o.s[2] = 0.5 * v.size[2]; break;
        case PR_CYLINDER: o.s[0] = v.size[0]; o.s[1] = 0.5 * v.size[1]; break;
        case PR_CYL_SHELL: o.s[0] = v.size[0]; o.s[1] = v.size[1]; o.s[2] = 0.5 * v.size[2]; break;
        case PR_SPHERE: o.s[0] = v.size[0]; break;
        default: o.s[0] = v.size[0]; o.s[1] = v.size[1]; break;
        }
        o.kind = v.kind;
        o.axis = v.axis;
        o.parent = v.parent;
        o.mat = v.material >= 0 ? mat_map[v.material] : -1;
        o.detector = v.is_detector ? 1 : 0;
        o.mirror_mask = v.mirror_mask;
        o.child_begin = cbeg[i];
        o.child_count = ccnt[i];
        o.mirror_model = v.mirror.model;
        o.grid = -1;
        o.R0 = v.mirror.R0;
        o.Qc = v.mirror.Qc;
        o.alpha = v.mirror.alpha;
        o.mQc = v.mirror.m * v.mirror.Qc;
        o.W = v.mirror.W > 0 ? v.mirror.W : 1.0;
        o.chop_n = v.chopper.n;
        if (v.chopper.n > 0) {
            // the same expressions as the definition: phase pi / 180, 2 pi f, 2 pi / n
            o.chop_r = v.chopper.r;
            o.chop_omega = 2.0 * 3.14159265358979323846 * v.chopper.rot_freq;
            o.chop_theta0 = v.chopper.theta0 * 3.14159265358979323846 / 180.0;
            o.chop_phase = v.chopper.phase * 3.14159265358979323846 / 180.0;
            o.chop_period = 2.0 * 3.14159265358979323846 / v.chopper.n;
        }
        vd[i] = o;
        VolT<float> f{};
        for (int k = 0; k < 3; ++k) { f.c[k] = (float)o.c[k]; f.s[k] = (float)o.s[k]; }
        f.kind = o.kind; f.axis = o.axis; f.parent = o.parent; f.mat = o.mat; f.detector = o.detector;
        f.mirror_mask = o.mirror_mask; f.child_begin = o.child_begin; f.child_count = o.child_count;
        f.mirror_model = o.mirror_model;
        f.grid = -1;
        f.R0 = (float)o.R0; f.Qc = (float)o.Qc; f.alpha = (float)o.alpha; f.mQc = (float)o.mQc; f.W = (float)o.W;
        f.chop_n = o.chop_n;
        f.chop_r = (float)o.chop_r; f.chop_omega = (float)o.chop_omega; f.chop_theta0 = (float)o.chop_theta0;
        f.chop_phase = (float)o.chop_phase; f.chop_period = (float)o.chop_period;
        vf[i] = f;
    }
    std::vector<MatT<double>> md;
    std::vector<MatT<float>> mf;
    std::vector<FamT<double>> fd;
    std::vector<FamT<float>> ff;
    for (int m : used) {
        const Material& M = c->mats[m];
        const pr_material_desc& d = M.desc;
        MatT<double> o{};
        o.sa_per_lambda = 0.1 * d.number_density * d.sigma_abs_ref / 1.798;
        o.si = 0.1 * d.number_density * d.sigma_inc;
        o.sc_k = d.n_families > 0 ? 0.1 * d.number_density / (2.0 * d.cell_volume * d.atoms_per_cell) : 0.0;
        o.ga = d.abs_bias;
        o.gs = d.scatter_bias;
        o.fam_begin = (int32_t)fd.size();
        o.nfam = d.n_families;
        o.inv_ga = 1.0 / o.ga;
        o.inv_gs = 1.0 / o.gs;
        double cum = 0.0;
        for (int j = 0; j < d.n_families; ++j) {
            cum += M.mult[j] * M.d[j] * M.f2[j];
            FamT<double> f{2.0 * M.d[j], cum, 1.0 / (2.0 * M.d[j] * M.d[j]), 0.0};
            fd.push_back(f);
            ff.push_back(FamT<float>{(float)f.edge, (float)f.cum, (float)f.inv2d2, 0.0f});
        }
        // tabulated cross sections: rows (lambda, sigma_abs, sigma_inc) after the families
        o.tab_begin = (int32_t)fd.size();
        o.tab_n = (int32_t)M.tl.size();
        o.tab_k = d.number_density * (1e-8 * 1e7);
        for (size_t j = 0; j < M.tl.size(); ++j) {
            fd.push_back(FamT<double>{M.tl[j], M.ta[j], M.ti[j], 0.0});
            ff.push_back(FamT<float>{(float)M.tl[j], (float)M.ta[j], (float)M.ti[j], 0.0f});
        }
        md.push_back(o);
        // the FP32 policy divides by its own (float) factors, in FP64
        mf.push_back(MatT<float>{(float)o.sa_per_lambda, (float)o.si, (float)o.sc_k, (float)o.ga, (float)o.gs,
                                 o.fam_begin, o.nfam, 1.0 / (double)(float)o.ga, 1.0 / (double)(float)o.gs,
                                 o.tab_begin, o.tab_n, (float)o.tab_k});
    }
    g.vd = std::move(vd);
    g.vf = std::move(vf);
    g.md = std::move(md);
    g.mf = std::move(mf);
    g.fd = std::move(fd);
    g.ff = std::move(ff);
    g.children = std::move(children);
    for (int i = 0; i < n; ++i)
        if ((int)kids[i].size() >= kGridMinDaughters) build_grid(vols, kids[i], g, i);
    // boundary candidates per solid kind: the volume itself (bit 0) and, unless a
    // grid serves them, its daughters (bits 1..7; fewer than kGridMinDaughters)
    for (int i = 0; i < n; ++i) {
        uint64_t m = 1ull << (8 * g.vd[i].kind);
        uint32_t det = 0;
        if (g.vd[i].grid < 0)
            for (size_t j = 0; j < kids[i].size(); ++j) {
                m |= 1ull << (8 * g.vd[kids[i][j]].kind + 1 + (int)j);
                if (g.vd[kids[i][j]].detector) det |= 1u << (1 + (int)j);
            }
        g.vd[i].kind_items = g.vf[i].kind_items = (uint32_t)m;
        g.vd[i].kind_items4 = g.vf[i].kind_items4 = (uint32_t)(m >> 32);
        g.vd[i].det_items = g.vf[i].det_items = det;
    }
    // the only, convex daughter of a vacuum world without mirrors: leaving it ends in
    // the world's boundary (the step that leaves it takes the world crossing too)
    for (int i = 1; i < n; ++i) {
        const int w = g.vd[i].parent;
        const int k = g.vd[i].kind, wk = g.vd[w].kind;
        const bool convex = k == PR_BOX || k == PR_CYLINDER || k == PR_SPHERE;
        const bool plain_world = g.vd[w].parent < 0 && g.vd[w].mat < 0 && g.vd[w].mirror_mask == 0 &&
                                 g.vd[w].chop_n == 0 && g.vd[w].grid < 0 && kids[w].size() == 1 &&
                                 (wk == PR_BOX || wk == PR_CYLINDER || wk == PR_SPHERE);
        if (convex && plain_world) {
            const uint32_t mark = (uint32_t)(1 + wk) << 24;   // byte 3 of kind_items4: exit_escapes
            g.vd[i].kind_items4 |= mark;
            g.vf[i].kind_items4 |= mark;
            g.esc = true;
        }
    }
    // FP32 fold passes: worth it where histories go in and out of material volumes
    // that sit in vacuum; scenes with mirrors (guides) mostly step through vacuum,
    // and the extra pass there costs more than it saves
    if (!g.esc) {
        bool mirrors = false, mat_in_vacuum = false;
        for (int i = 0; i < n; ++i) {
            mirrors = mirrors || g.vd[i].mirror_mask != 0;
            if (i > 0 && g.vd[i].mat >= 0 && g.vd[g.vd[i].parent].mat < 0) mat_in_vacuum = true;
        }
        g.fold = !mirrors && mat_in_vacuum;
    }
    g.kinds = 0;
    for (int i = 0; i < n; ++i) {
        g.kinds |= 1u << g.vd[i].kind;
        if (g.vd[i].chop_n > 0) g.kinds |= 1u << kChopperBit;
    }
    g.bd.assign(n, BoxT<double>{});
    g.bf.assign(n, BoxT<float>{});
    for (int i = 0; i < n; ++i) {
        if (g.vd[i].kind != PR_BOX) continue;
        for (int k = 0; k < 3; ++k) {
            g.bd[i].c[k] = g.vd[i].c[k];
            g.bd[i].s[k] = g.vd[i].s[k];
            g.bf[i].c[k] = g.vf[i].c[k];
            g.bf[i].s[k] = g.vf[i].s[k];
        }
    }
    g.nv = n;
    g.nm = (int)g.md.size();
    g.nf = (int)g.fd.size();
    g.nc = (int)g.children.size();
    g.scene_f_bytes = (int)(g.vf.size() * sizeof(VolT<float>) + g.mf.size() * sizeof(MatT<float>) +
                            g.ff.size() * sizeof(FamT<float>) + g.children.size() * 4 +
                            g.gf.size() * sizeof(GridT<float>) + g.cell_start.size() * 4 + g.cell_items.size() * 4) +
                      7 * 16;
    g.scene_lds_bytes = batch_scene_lds_bytes(g.nv, g.nm, g.nf, g.nc, (int)g.gf.size(), (int)g.cell_start.size(),
                                              (int)g.cell_items.size(), g.gd.empty() ? 0 : 1);
    if (c->device >= 0) {
        int rc = set_device(c);
        if (rc) return rc;
        if ((rc = upload(c, &g.vols_d, g.vd)) || (rc = upload(c, &g.vols_f, g.vf)) || (rc = upload(c, &g.mats_d, g.md)) ||
            (rc = upload(c, &g.mats_f, g.mf)) || (rc = upload(c, &g.fams_d, g.fd)) || (rc = upload(c, &g.fams_f, g.ff)) ||
            (rc = upload(c, &g.children_d, g.children)) || (rc = upload(c, &g.grids_d, g.gd)) ||
            (rc = upload(c, &g.grids_f, g.gf)) || (rc = upload(c, &g.cell_start_d, g.cell_start)) ||
            (rc = upload(c, &g.cell_items_d, g.cell_items)) || (rc = upload(c, &g.boxes_d, g.bd)) ||
            (rc = upload(c, &g.boxes_f, g.bf))) {
            free_geometry(g);
            return rc;
        }
    }
    c->geoms.push_back(std::move(g));
    *id = (int32_t)c->geoms.size() - 1;
    return PR_OK;
}

// =========================================================================
// source
// =========================================================================

extern "C" int pr_create_source(pr_ctx* c, const pr_source_desc* d, int32_t* id) {
    if (!c || !d || !id) return fail(c, PR_EINVAL, "null argument");
    if (d->kind < PR_PENCIL || d->kind > PR_MODERATOR) return fail(c, PR_EINVAL, "source.kind invalid");
    if (d->spectrum < PR_MONO || d->spectrum > PR_MAXWELL) return fail(c, PR_EINVAL, "source.spectrum invalid");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(d->origin[k]) || !std::isfinite(d->dir[k])) return fail(c, PR_EINVAL, "source origin/dir not finite");
    double nd = std::sqrt(d->dir[0] * d->dir[0] + d->dir[1] * d->dir[1] + d->dir[2] * d->dir[2]);
    if (!(nd > 0)) return fail(c, PR_EINVAL, "source.dir must be non-zero");
    if (d->kind != PR_PENCIL && !(finite_nonneg(d->size[0]) && finite_nonneg(d->size[1])))
        return fail(c, PR_EINVAL, "source.size must be >= 0");
    if (d->kind == PR_RECT_DIVERGENT) {
        if (!(d->dir[0] == 0 && d->dir[1] == 0 && d->dir[2] > 0))
            return fail(c, PR_EINVAL, "PR_RECT_DIVERGENT needs dir = +z");
        for (int k = 0; k < 2; ++k)
            if (!(finite_nonneg(d->div_deg[k]) && d->div_deg[k] < 89.0))
                return fail(c, PR_EINVAL, "source.div_deg must be in [0, 89)");
    }
    if (d->kind == PR_MODERATOR) {
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(d->slit_center[k])) return fail(c, PR_EINVAL, "source.slit_center not finite");
        if (!(finite_nonneg(d->slit_size[0]) && finite_nonneg(d->slit_size[1])))
            return fail(c, PR_EINVAL, "source.slit_size must be >= 0");
        if (!(d->slit_center[2] != d->origin[2])) return fail(c, PR_EINVAL, "source slit must lie off the source plane");
    }
    if (d->spectrum == PR_MONO && !(std::isfinite(d->lam0) && d->lam0 > 0)) return fail(c, PR_EINVAL, "source.lam0 must be > 0");
    if (d->spectrum != PR_MONO && !(std::isfinite(d->lam_lo) && d->lam_lo > 0 && d->lam_hi > d->lam_lo && std::isfinite(d->lam_hi)))
        return fail(c, PR_EINVAL, "source needs 0 < lam_lo < lam_hi");
    if (d->spectrum == PR_MAXWELL && !(std::isfinite(d->kT) && d->kT > 0)) return fail(c, PR_EINVAL, "source.kT must be > 0");
    c->srcs.push_back(*d);
    *id = (int32_t)c->srcs.size() - 1;
    return PR_OK;
}

// =========================================================================
// tallies
// =========================================================================

// validates a tally description; *nbins receives its bin count
static int check_tally_desc(pr_ctx* c, const pr_tally_desc* d, uint64_t* nbins) {
    if (d->trigger < PR_TRIG_ESCAPE || d->trigger > PR_TRIG_FIRST_COLLISION)
        return fail(c, PR_EINVAL, "tally.trigger invalid");
    if (d->filter < PR_FILT_ALL || d->filter > PR_FILT_NSCAT_EQ) return fail(c, PR_EINVAL, "tally.filter invalid");
    if (d->naxes < 0 || d->naxes > 4) return fail(c, PR_EINVAL, "tally.naxes must be in [0, 4]");
    if (d->accumulator == PR_ACC_KAHAN_FP32)
        return fail(c, PR_EINVAL, "tally.accumulator: PR_ACC_KAHAN_FP32 is not supported (tallies accumulate in FP64)");
    if (d->accumulator != PR_ACC_FP64) return fail(c, PR_EINVAL, "tally.accumulator invalid");
    uint64_t nb = 1;
    for (int a = 0; a < d->naxes; ++a) {
        const pr_tally_axis& x = d->axes[a];
        if (x.quantity < PR_Q_THETA2 || x.quantity > PR_Q_TOF) return fail(c, PR_EINVAL, "tally.axes[%d].quantity invalid", a);
        if (x.nbins < 1) return fail(c, PR_EINVAL, "tally.axes[%d].nbins must be >= 1", a);
        if (!(std::isfinite(x.lo) && std::isfinite(x.hi) && x.hi > x.lo))
            return fail(c, PR_EINVAL, "tally.axes[%d] needs lo < hi", a);
        nb *= (uint64_t)x.nbins;
        if (nb > (1ull << 36)) return fail(c, PR_EINVAL, "tally has too many bins");
    }
    double bn = std::sqrt(d->beam[0] * d->beam[0] + d->beam[1] * d->beam[1] + d->beam[2] * d->beam[2]);
    for (int a = 0; a < d->naxes; ++a)
        if ((d->axes[a].quantity == PR_Q_THETA2 || d->axes[a].quantity == PR_Q_Q) && !(bn > 0))
            return fail(c, PR_EINVAL, "tally.beam must be non-zero");
    *nbins = nb;
    return PR_OK;
}

extern "C" int pr_tally_storage_size(pr_ctx* c, const pr_tally_desc* d, size_t* bytes) {
    if (!c || !d || !bytes) return fail(c, PR_EINVAL, "null argument");
    uint64_t nb = 0;
    int rc = check_tally_desc(c, d, &nb);
    if (rc) return rc;
    *bytes = (size_t)(2 * nb * sizeof(double));
    return PR_OK;
}

// storage: the caller's device buffer, or nullptr to allocate it
static int create_tally(pr_ctx* c, const pr_tally_desc* d, void* storage, size_t storage_bytes, int32_t* id) {
    if (!c || !d || !id) return fail(c, PR_EINVAL, "null argument");
    uint64_t nb = 0;
    int rc = check_tally_desc(c, d, &nb);
    if (rc) return rc;
    Tally t;
    t.desc = *d;
    t.nbins = nb;
    if (storage) {
        if (storage_bytes < 2 * nb * sizeof(double))
            return fail(c, PR_EWORKSPACE, "tally storage holds %zu bytes, %llu needed", storage_bytes,
                        (unsigned long long)(2 * nb * sizeof(double)));
        if ((uintptr_t)storage % 16 != 0) return fail(c, PR_EINVAL, "tally storage must be 16-byte aligned");
        if (c->device < 0) return fail(c, PR_EDEVICE, "caller tally storage needs a device context");
    }
    if (c->device >= 0) {
        if ((rc = set_device(c))) return rc;
        if (storage) {
            t.dev = (double*)storage;
            t.owned = false;
        } else if (hipMalloc((void**)&t.dev, 2 * nb * sizeof(double)) != hipSuccess) {
            return fail(c, PR_ENOMEM, "cannot allocate %llu tally bins on the device", (unsigned long long)nb);
        }
        hipError_t e = zero_f64(t.dev, 2 * nb, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            if (t.owned) (void)hipFree(t.dev);
            return hipfail(c, e, "zeroing tally");
        }
    }
    c->tallies.push_back(t);
    *id = (int32_t)c->tallies.size() - 1;
    return PR_OK;
}

extern "C" int pr_create_tally(pr_ctx* c, const pr_tally_desc* d, int32_t* id) {
    return create_tally(c, d, nullptr, 0, id);
}

extern "C" int pr_create_tally_in(pr_ctx* c, const pr_tally_desc* d, void* dev_storage, size_t storage_bytes,
                                  int32_t* id) {
    if (!dev_storage) return fail(c, PR_EINVAL, "dev_storage is null");
    return create_tally(c, d, dev_storage, storage_bytes, id);
}

extern "C" int pr_tally_nbins(pr_ctx* c, int32_t tally, uint64_t* nbins) {
    if (!c || !nbins) return fail(c, PR_EINVAL, "null argument");
    if (tally < 0 || tally >= (int)c->tallies.size()) return fail(c, PR_ENOTFOUND, "tally %d unknown", tally);
    *nbins = c->tallies[tally].nbins;
    return PR_OK;
}

// =========================================================================
// run
// =========================================================================

static void make_source_dev(const pr_source_desc& s, SourceDev& d) {
    memset(&d, 0, sizeof(d));
    d.kind = s.kind;
    d.spectrum = s.spectrum;
    double nd = std::sqrt(s.dir[0] * s.dir[0] + s.dir[1] * s.dir[1] + s.dir[2] * s.dir[2]);
    for (int k = 0; k < 3; ++k) {
        d.o[k] = s.origin[k];
        d.u[k] = s.dir[k] / nd;
    }
    d.size[0] = s.size[0];
    d.size[1] = s.size[1];
    d.div_rad[0] = s.div_deg[0] * 3.14159265358979323846 / 180.0;
    d.div_rad[1] = s.div_deg[1] * 3.14159265358979323846 / 180.0;
    d.lam0 = s.lam0;
    d.lam_lo = s.lam_lo;
    d.lam_hi = s.lam_hi;
    d.kT = s.kT;
    d.e_const = ev_angstrom2();
    for (int k = 0; k < 3; ++k) d.slit[k] = s.slit_center[k];
    d.slit_size[0] = s.slit_size[0];
    d.slit_size[1] = s.slit_size[1];
}

static uint32_t tally_qmask(const pr_tally_desc& td);

static void make_tally_dev(const Tally& T, int vol_offset, TallyDev& o) {
    memset(&o, 0, sizeof(o));
    const pr_tally_desc& td = T.desc;
    TallyHead& h = o.head;
    h.term_mask = td.trigger == PR_TRIG_ESCAPE   ? 1u << PR_END_ESCAPE
                  : td.trigger == PR_TRIG_ABSORB ? 1u << PR_END_ABSORB
                  : td.trigger == PR_TRIG_DETECT ? 1u << PR_END_DETECT
                                                 : 1u << kTermFirstCollision;
    h.fix_axis = -1;
    h.fix_bin = 0;
    h.volume = td.trigger == PR_TRIG_DETECT && td.trigger_volume >= 0 ? td.trigger_volume + vol_offset : -1;
    const int32_t big = std::numeric_limits<int32_t>::max();
    h.nscat_lo = td.filter == PR_FILT_SCATTERED ? 1 : td.filter == PR_FILT_NSCAT_EQ ? td.filter_arg : 0;
    h.nscat_hi = td.filter == PR_FILT_UNSCATTERED ? 0 : td.filter == PR_FILT_NSCAT_EQ ? td.filter_arg : big;
    h.naxes = td.naxes;
    h.qmask = tally_qmask(td);
    for (int a = 0; a < td.naxes; ++a) {
        TallyAxis& A = o.ax[a];
        A.quantity = td.axes[a].quantity;
        A.nbins = td.axes[a].nbins;
        A.lo = td.axes[a].lo;
        A.hi = td.axes[a].hi;
        A.scale = td.axes[a].nbins / (td.axes[a].hi - td.axes[a].lo);
        A.lo_f = (float)A.lo;
        A.hi_f = (float)A.hi;
        A.scale_f = (float)A.scale;
    }
    double bn = std::sqrt(td.beam[0] * td.beam[0] + td.beam[1] * td.beam[1] + td.beam[2] * td.beam[2]);
    for (int k = 0; k < 3; ++k) {
        o.beam[k] = bn > 0 ? td.beam[k] / bn : 0.0;
        o.beam_f[k] = (float)o.beam[k];
    }
    o.sw = T.dev;
    o.sw2 = T.dev ? T.dev + 1 : nullptr;
    o.total = (int64_t)T.nbins;
    o.lds_bins = 0;
    o.lds_offset = -1;
    o.cache_base = -1;
    o.cache_bits = 0;
}

// quantities a tally bins, one bit per PR_Q_* value
static uint32_t tally_qmask(const pr_tally_desc& td) {
    uint32_t m = 0;
    for (int a = 0; a < td.naxes; ++a) m |= 1u << td.axes[a].quantity;
    return m;
}

constexpr int kLdsPerCu = 160 * 1024;

// Block size for kernels that stage a grid scene into LDS: the staged copy is
// large, so fewer, larger blocks share it; take the size (256 or 512 threads)
// that keeps the most waves resident per CU, the smallest among equals.  A
// block count per CU set by the tuning keeps the tuned block size.
template <class Occ>
static int grid_block(const pr_ctx* c, Occ occupancy) {
    if (c->mixed_blocks_per_cu > 0) return std::min(c->mixed_block, 512);
    int best = std::min(c->mixed_block, 512), best_waves = occupancy(best) * (best / 64);
    for (int b = 256; b <= 512; b += 256) {
        const int w = occupancy(b) * (b / 64);
        if (w > best_waves) { best = b; best_waves = w; }
    }
    return best;
}

// Bin of value x on axis A computed as the device computes it in precision R
// (the FP32 range and scale are the axis's FP32 copies); -1 outside the axis.
template <class R>
static int axis_bin(const TallyAxis& A, R x) {
    const R lo = sizeof(R) == 4 ? (R)A.lo_f : (R)A.lo, hi = sizeof(R) == 4 ? (R)A.hi_f : (R)A.hi;
    const R scale = sizeof(R) == 4 ? (R)A.scale_f : (R)A.scale;
    if (!(x >= lo && x <= hi)) return -1;
    const R prod = (x - lo) * scale;
    int b = (int)std::floor((double)prod);
    if (x == hi || b >= A.nbins) b = A.nbins - 1;
    if (b < 0) b = 0;
    return b;
}

static int build_params(pr_ctx* c, int32_t geom, int32_t src, const int32_t* tallies, int32_t nt, uint64_t first,
                        uint64_t n, int32_t precision, void* records, Params& P) {
    if (geom < 0 || geom >= (int)c->geoms.size()) return fail(c, PR_ENOTFOUND, "geometry %d unknown", geom);
    if (src < 0 || src >= (int)c->srcs.size()) return fail(c, PR_ENOTFOUND, "source %d unknown", src);
    if (nt < 0 || nt > kMaxTallies) return fail(c, PR_EINVAL, "n_tallies must be in [0, %d]", kMaxTallies);
    if (nt > 0 && !tallies) return fail(c, PR_EINVAL, "tallies is null");
    if (precision != PR_FP64_PLAIN && precision != PR_FP32_MIXED && precision != PR_FP64_PERSISTENT)
        return fail(c, PR_EINVAL, "precision invalid");
    if (n > (1ull << 48) || first > (1ull << 62)) return fail(c, PR_EINVAL, "history range too large");
    const Geometry& g = c->geoms[geom];
    memset(&P, 0, sizeof(P));
    P.vols_d = (const VolT<double>*)g.vols_d;
    P.mats_d = (const MatT<double>*)g.mats_d;
    P.fams_d = (const FamT<double>*)g.fams_d;
    P.vols_f = (const VolT<float>*)g.vols_f;
    P.mats_f = (const MatT<float>*)g.mats_f;
    P.fams_f = (const FamT<float>*)g.fams_f;
    P.boxes_d = (const BoxT<double>*)g.boxes_d;
    P.boxes_f = (const BoxT<float>*)g.boxes_f;
    P.children = (const int32_t*)g.children_d;
    P.grids_d = (const GridT<double>*)g.grids_d;
    P.grids_f = (const GridT<float>*)g.grids_f;
    P.cell_start = (const int32_t*)g.cell_start_d;
    P.cell_items = (const int32_t*)g.cell_items_d;
    P.n_vols = g.nv;
    P.n_mats = g.nm;
    P.n_fams = g.nf;
    P.n_children = g.nc;
    P.n_grids = (int)g.gd.size();
    P.n_cell_start = (int)g.cell_start.size();
    P.n_cell_items = (int)g.cell_items.size();
    P.has_grid = g.gd.empty() ? 0 : 1;
    // the FP32 scene may be staged into LDS; the FP64 one is read from global memory
    P.scene_in_lds = precision == PR_FP32_MIXED &&
                     g.scene_lds_bytes <= (P.has_grid ? c->lds_grid_budget : c->lds_scene_budget);
    P.fp64 = precision == PR_FP64_PERSISTENT ? 1 : 0;
    P.kinds = g.kinds;
    // 1: the lone-daughter world crossing (and the newborn step); 2: FP32 fold
    // passes (and the newborn step); 0: neither
    P.esc = !c->vacuum_steps ? 0 : g.esc ? 1 : (precision != PR_FP64_PLAIN && g.fold && !P.has_grid) ? 2 : 0;
    make_source_dev(c->srcs[src], P.src);
    P.n_tallies = nt;
    int lds_doubles = 0;
    const int budget = precision != PR_FP64_PLAIN ? c->lds_tally_budget / 8 : 0;
    const pr_source_desc& sdesc = c->srcs[src];
    for (int i = 0; i < nt; ++i) {
        int t = tallies[i];
        if (t < 0 || t >= (int)c->tallies.size()) return fail(c, PR_ENOTFOUND, "tally %d unknown", t);
        for (int j = 0; j < i; ++j)
            if (tallies[j] == t) return fail(c, PR_EINVAL, "tally %d listed twice", t);
        const Tally& T = c->tallies[t];
        const pr_tally_desc& td = T.desc;
        if (td.trigger == PR_TRIG_DETECT && td.trigger_volume >= g.nv)
            return fail(c, PR_EINVAL, "tally %d: trigger_volume beyond the geometry", t);
        if (td.trigger == PR_TRIG_FIRST_COLLISION) {
            if (precision == PR_FP32_MIXED)
                return fail(c, PR_EINVAL, "tally %d: first-collision tallies run with the FP64 policies only", t);
            P.has_fc = 1;
        }
        TallyDev& o = P.tallies[i];
        make_tally_dev(T, 0, o);
        P.qmask |= tally_qmask(td);
        // Privatise the whole tally when it fits the block's LDS budget; else, under
        // a monochromatic source (elastic physics keeps lambda), the slice at the
        // source wavelength's bin of a wavelength axis, when that fits.
        int64_t bins = (int64_t)T.nbins;
        if ((int64_t)lds_doubles + 2 * bins > budget && sdesc.spectrum == PR_MONO) {
            for (int a = 0; a < td.naxes && o.head.fix_axis < 0; ++a) {
                if (td.axes[a].quantity != PR_Q_LAMBDA) continue;
                const int b = precision == PR_FP32_MIXED ? axis_bin<float>(o.ax[a], (float)sdesc.lam0)
                                                         : axis_bin<double>(o.ax[a], sdesc.lam0);
                const int64_t slice = bins / td.axes[a].nbins;
                if (b >= 0 && (int64_t)lds_doubles + 2 * slice <= budget) {
                    o.head.fix_axis = a;
                    o.head.fix_bin = b;
                    bins = slice;
                }
            }
        }
        if ((int64_t)lds_doubles + 2 * bins <= budget) {
            o.lds_offset = lds_doubles;
            o.lds_bins = (int32_t)bins;
            lds_doubles += 2 * (int)bins;
        }
    }
    // tallies too large to privatise get an LDS bin cache (persistent policies)
    int slots = 0;
    if (precision != PR_FP64_PLAIN && c->bin_cache_slots > 0) {
        int bits = 0;
        while ((1 << (bits + 1)) <= c->bin_cache_slots) ++bits;
        for (int i = 0; i < nt; ++i) {
            TallyDev& o = P.tallies[i];
            if (o.lds_offset >= 0 || o.total >= (int64_t)0xFFFFFFFFll) continue;
            o.cache_base = slots;
            o.cache_bits = bits;
            slots += 1 << bits;
        }
    }
    P.cache_slots = slots;
    // FP32 runs with a tally scoring straight into global memory (neither
    // privatised nor cached) score as a wave, with paired-lane atomics
    P.paired = 0;
    if (precision == PR_FP32_MIXED)
        for (int i = 0; i < nt; ++i)
            if (P.tallies[i].lds_offset < 0 && P.tallies[i].cache_base < 0) P.paired = 1;
    // the time of flight is tracked only when a chopper or a TOF axis needs it
    bool need_time = (g.kinds >> kChopperBit) & 1u;
    for (int i = 0; i < nt; ++i)
        for (int a = 0; a < P.tallies[i].head.naxes; ++a) need_time = need_time || P.tallies[i].ax[a].quantity == PR_Q_TOF;
    if (need_time) P.kinds |= 1u << kTimeBit;
    P.lds_tally_doubles = lds_doubles;
    P.seed = c->seed;
    P.first = first;
    P.n = n;
    P.records = (pr_history_record*)records;
    P.stats = c->stats;
    P.counter = nullptr;   // set by the caller: a run slot or the caller's workspace
    P.refill_threshold = c->refill_threshold;
    P.chunk = P.has_grid && c->grid_chunk > 0 ? c->grid_chunk : c->chunk;
    P.waves = c->waves_per_simd;
    P.walk_cells = precision == PR_FP32_MIXED ? c->grid_walk_cells : 0;
    return PR_OK;
}

// Launch one history range.  trial: autotuner run scoring into scratch.
// workspace: the caller's device workspace (pr_workspace_size bytes) holding
// the run's history-claim counter, or nullptr to take a slot of the context's
// ring (the stream then waits for the last run that used the slot).
static int run_single(pr_ctx* c, int32_t geom, int32_t src, const int32_t* tallies, int32_t nt, uint64_t first,
                      uint64_t n, int32_t precision, void* records, void* workspace, size_t ws_bytes, hipStream_t st,
                      bool trial) {
    Params P;
    int rc = build_params(c, geom, src, tallies, nt, first, n, precision, records, P);
    if (rc) return rc;
    if ((rc = set_device(c))) return rc;
    if (workspace) {
        if (ws_bytes < kRunSlotBytes)
            return fail(c, PR_EWORKSPACE, "workspace holds %zu bytes, %zu needed", ws_bytes, kRunSlotBytes);
        if ((uintptr_t)workspace % 8 != 0) return fail(c, PR_EINVAL, "workspace must be 8-byte aligned");
    }
    if (trial) {
        for (int i = 0; i < nt; ++i) {
            P.tallies[i].sw = c->scratch;
            P.tallies[i].sw2 = c->scratch + 1;
        }
        P.stats = c->scratch_stats;
    }
    if (n == 0) return PR_OK;
    hipError_t e;
    if (precision == PR_FP64_PLAIN) {
        e = launch_plain(P, records != nullptr, st);
    } else {
        if (P.scene_in_lds && mixed_lds_bytes(P) > kLdsPerCu) P.scene_in_lds = 0;   // tallies leave no room
        int lds = mixed_lds_bytes(P);
        if (lds > kLdsPerCu) return fail(c, PR_EINVAL, "scene and tallies need %d bytes of LDS", lds);
        int block = std::min(c->mixed_block, mixed_max_block(P));
        if (P.has_grid && P.scene_in_lds) block = grid_block(c, [&](int b) { return mixed_occupancy(P, b); });
        int per_cu = c->mixed_blocks_per_cu > 0 ? c->mixed_blocks_per_cu : mixed_occupancy(P, block);
        uint64_t want = (n + block - 1) / block;
        uint64_t grid = std::min<uint64_t>((uint64_t)per_cu * (uint64_t)c->num_cus, want);
        if (grid < 1) grid = 1;
        int slot = -1;
        if (workspace) {
            P.counter = (unsigned long long*)workspace;
        } else {
            slot = c->next_run_slot;
            c->next_run_slot = (slot + 1) % kRunSlots;
            if (c->run_used[slot]) HIPCHK(c, hipStreamWaitEvent(st, c->run_done[slot], 0));
            P.counter = (unsigned long long*)(c->run_slots + slot * kRunSlotBytes);
        }
        e = launch_mixed(P, records != nullptr, (int)grid, block, st);
        if (e == hipSuccess && slot >= 0) {
            e = hipEventRecord(c->run_done[slot], st);
            if (e == hipSuccess) c->run_used[slot] = true;
        }
    }
    if (e != hipSuccess) return hipfail(c, e, "kernel launch");
    return PR_OK;
}

extern "C" int pr_workspace_size(pr_ctx* c, int32_t precision, size_t* bytes) {
    if (!c || !bytes) return fail(c, PR_EINVAL, "null argument");
    if (precision != PR_FP64_PLAIN && precision != PR_FP32_MIXED && precision != PR_FP64_PERSISTENT)
        return fail(c, PR_EINVAL, "precision invalid");
    *bytes = kRunSlotBytes;
    return PR_OK;
}

extern "C" int pr_run_histories(pr_ctx* c, int32_t geom, int32_t src, const int32_t* tallies, int32_t nt,
                                uint64_t first, uint64_t n, int32_t precision, void* records, void* workspace,
                                size_t ws_bytes, void* stream) {
    if (!c) return PR_EINVAL;
    int rc = run_single(c, geom, src, tallies, nt, first, n, precision, records, workspace, ws_bytes,
                        (hipStream_t)stream, false);
    if (rc) return rc;
    for (int i = 0; i < nt; ++i) c->tallies[tallies[i]].n_hist += n;
    return PR_OK;
}

// =========================================================================
// results
// =========================================================================

extern "C" int pr_read_tally_range(pr_ctx* c, int32_t tally, uint64_t offset, uint64_t count, double* sw, double* sw2,
                                   void* stream) {
    if (!c) return PR_EINVAL;
    if (tally < 0 || tally >= (int)c->tallies.size()) return fail(c, PR_ENOTFOUND, "tally %d unknown", tally);
    const Tally& T = c->tallies[tally];
    if (offset > T.nbins || count > T.nbins - offset) return fail(c, PR_EWORKSPACE, "range beyond the tally's bins");
    int rc = set_device(c);
    if (rc) return rc;
    (void)stream;   // reads wait for the whole device: runs may be on any stream
    HIPCHK(c, hipDeviceSynchronize());
    if (count == 0) return PR_OK;
    // device layout is (sum w, sum w^2) interleaved per bin: copy in slices and split
    const uint64_t slice = 1ull << 22;
    std::vector<double> tmp;
    try {
        tmp.resize(2 * std::min(slice, count));
    } catch (...) {
        return fail(c, PR_ENOMEM, "host buffer for tally readback");
    }
    for (uint64_t done = 0; done < count; done += slice) {
        const uint64_t m = std::min(slice, count - done);
        HIPCHK(c, hipMemcpy(tmp.data(), T.dev + 2 * (offset + done), 2 * m * sizeof(double), hipMemcpyDeviceToHost));
        for (uint64_t i = 0; i < m; ++i) {
            if (sw) sw[done + i] = tmp[2 * i];
            if (sw2) sw2[done + i] = tmp[2 * i + 1];
        }
    }
    return PR_OK;
}

extern "C" int pr_read_tally(pr_ctx* c, int32_t tally, double* sw, double* sw2, uint64_t* n_hist, size_t nbins,
                             void* stream) {
    if (!c) return PR_EINVAL;
    if (tally < 0 || tally >= (int)c->tallies.size()) return fail(c, PR_ENOTFOUND, "tally %d unknown", tally);
    const Tally& T = c->tallies[tally];
    if ((sw || sw2) && nbins < T.nbins)
        return fail(c, PR_EWORKSPACE, "tally %d has %llu bins, buffer holds %zu", tally, (unsigned long long)T.nbins, nbins);
    int rc = set_device(c);
    if (rc) return rc;
    (void)stream;   // reads wait for the whole device: runs may be on any stream
    HIPCHK(c, hipDeviceSynchronize());
    if (n_hist) {
        unsigned long long d = 0;
        if (T.dev_nhist) HIPCHK(c, hipMemcpy(&d, T.dev_nhist, sizeof(d), hipMemcpyDeviceToHost));
        *n_hist = T.n_hist + d;
    }
    return pr_read_tally_range(c, tally, 0, (sw || sw2) ? T.nbins : 0, sw, sw2, stream);
}

extern "C" int pr_reset_tally(pr_ctx* c, int32_t tally, void* stream) {
    if (!c) return PR_EINVAL;
    if (tally < 0 || tally >= (int)c->tallies.size()) return fail(c, PR_ENOTFOUND, "tally %d unknown", tally);
    Tally& T = c->tallies[tally];
    int rc = set_device(c);
    if (rc) return rc;
    hipError_t e = zero_f64(T.dev, 2 * T.nbins, (hipStream_t)stream);
    if (e == hipSuccess && T.dev_nhist) e = zero_u64(T.dev_nhist, 1, (hipStream_t)stream);
    if (e != hipSuccess) return hipfail(c, e, "zeroing tally");
    T.n_hist = 0;
    return PR_OK;
}

extern "C" int pr_read_stats(pr_ctx* c, pr_run_stats* out, void* stream) {
    if (!c || !out) return fail(c, PR_EINVAL, "null argument");
    int rc = set_device(c);
    if (rc) return rc;
    unsigned long long h[ST_N];
    (void)stream;   // reads wait for the whole device: runs may be on any stream
    HIPCHK(c, hipDeviceSynchronize());
    HIPCHK(c, hipMemcpy(h, c->stats, sizeof(h), hipMemcpyDeviceToHost));
    out->histories = h[ST_HIST];
    out->escaped = h[ST_ESC];
    out->absorbed = h[ST_ABS];
    out->killed = h[ST_KILL];
    out->detected = h[ST_DET];
    out->capped = h[ST_CAP];
    out->outside = h[ST_OUT];
    out->steps = h[ST_STEPS];
    out->draws = h[ST_DRAWS];
    out->scatters = h[ST_SCAT];
    if (out->capped > 0)
        return fail(c, PR_ECAPPED, "%llu histories reached the step cap (%d); they are counted and scored as ended",
                    (unsigned long long)out->capped, PR_MAX_STEPS);
    return PR_OK;
}

extern "C" int pr_reset_stats(pr_ctx* c, void* stream) {
    if (!c) return PR_EINVAL;
    int rc = set_device(c);
    if (rc) return rc;
    hipError_t e = zero_u64(c->stats, ST_N, (hipStream_t)stream);
    if (e != hipSuccess) return hipfail(c, e, "zeroing stats");
    return PR_OK;
}

// =========================================================================
// launch tuning of the mixed policy
// =========================================================================

extern "C" int pr_set_tuning(pr_ctx* c, const pr_tuning* t) {
    if (!c || !t) return fail(c, PR_EINVAL, "null argument");
    if (t->block < 64 || t->block > 1024 || t->block % 64)
        return fail(c, PR_EINVAL, "tuning.block must be a multiple of 64 in [64, 1024]");
    if (t->blocks_per_cu < 0 || t->blocks_per_cu > 64) return fail(c, PR_EINVAL, "tuning.blocks_per_cu must be 0..64");
    if (t->refill_threshold < 1 || t->refill_threshold > 64) return fail(c, PR_EINVAL, "tuning.refill_threshold must be 1..64");
    if (t->lds_tally_bytes < 0 || t->lds_tally_bytes > 131072) return fail(c, PR_EINVAL, "tuning.lds_tally_bytes must be 0..131072");
    if (t->bin_cache_slots < 0 || t->bin_cache_slots > 4096 || (t->bin_cache_slots & (t->bin_cache_slots - 1)))
        return fail(c, PR_EINVAL, "tuning.bin_cache_slots must be 0 or a power of two up to 4096");
    if (t->chunk < 1 || t->chunk > (1 << 20)) return fail(c, PR_EINVAL, "tuning.chunk must be 1..2^20");
    if (t->grid_chunk < 0 || t->grid_chunk > (1 << 20)) return fail(c, PR_EINVAL, "tuning.grid_chunk must be 0..2^20");
    if (t->waves_per_simd != 0 && t->waves_per_simd != 4 && t->waves_per_simd != 5)
        return fail(c, PR_EINVAL, "tuning.waves_per_simd must be 0, 4 or 5");
    if (t->grid_walk_cells != 0 && (t->grid_walk_cells < 2 || t->grid_walk_cells > 1024))
        return fail(c, PR_EINVAL, "tuning.grid_walk_cells must be 0 or 2..1024");
    if (t->vacuum_steps != 0 && t->vacuum_steps != 1) return fail(c, PR_EINVAL, "tuning.vacuum_steps must be 0 or 1");
    c->vacuum_steps = t->vacuum_steps;
    c->grid_walk_cells = t->grid_walk_cells;
    c->waves_per_simd = t->waves_per_simd == 5 ? 5 : 4;
    c->chunk = t->chunk;
    c->grid_chunk = t->grid_chunk;
    c->mixed_block = t->block;
    c->mixed_blocks_per_cu = t->blocks_per_cu;
    c->refill_threshold = t->refill_threshold;
    c->lds_tally_budget = t->lds_tally_bytes;
    c->bin_cache_slots = t->bin_cache_slots;
    return PR_OK;
}

extern "C" int pr_get_tuning(pr_ctx* c, pr_tuning* t) {
    if (!c || !t) return fail(c, PR_EINVAL, "null argument");
    t->block = c->mixed_block;
    t->blocks_per_cu = c->mixed_blocks_per_cu;
    t->refill_threshold = c->refill_threshold;
    t->lds_tally_bytes = c->lds_tally_budget;
    t->bin_cache_slots = c->bin_cache_slots;
    t->chunk = c->chunk;
    t->waves_per_simd = c->waves_per_simd;
    t->grid_chunk = c->grid_chunk;
    t->grid_walk_cells = c->grid_walk_cells;
    t->vacuum_steps = c->vacuum_steps;
    return PR_OK;
}

// =========================================================================
// batched runs
// =========================================================================

// Plan one class of simulations idx: per-simulation descriptors, tally
// entries, bin-cache key bases, LDS budget and launch shape.
static int plan_batch_class(pr_ctx* c, const pr_sim* sims, const std::vector<int>& idx, bool slds, bool grid_nav,
                            bool trial, ClassPlan& P) {
    // LDS budgets: a simulation's tallies are privatised when they fit the tally
    // region, else they go through the bin cache whose values share that region
    const int priv_cap = c->lds_tally_budget / 8;
    int cache_bits = 0;
    if (c->bin_cache_slots > 0)
        while ((1 << (cache_bits + 1)) <= c->bin_cache_slots) ++cache_bits;
    const int nslots = c->bin_cache_slots > 0 ? (1 << cache_bits) : 0;
    const int ns = (int)idx.size();
    P.sd.assign(ns, SimDev{});
    P.td.clear();
    P.kb.clear();
    P.slds = slds;
    P.grid_nav = grid_nav;
    uint64_t total = 0;
    int tally_doubles = 0, scene_bytes = 0;
    bool any_cache = false;
    for (int q = 0; q < ns; ++q) {
        const pr_sim& sm = sims[idx[q]];
        const Geometry& g = c->geoms[sm.geom];
        SimDev& o = P.sd[q];
        memset(&o, 0, sizeof(o));
        o.vols = (const VolT<float>*)g.vols_f;
        o.mats = (const MatT<float>*)g.mats_f;
        o.fams = (const FamT<float>*)g.fams_f;
        o.children = (const int32_t*)g.children_d;
        o.grids = (const GridT<float>*)g.grids_f;
        o.cell_start = (const int32_t*)g.cell_start_d;
        o.cell_items = (const int32_t*)g.cell_items_d;
        o.boxes = (const BoxT<float>*)g.boxes_f;
        o.n_vols = g.nv;
        o.n_mats = g.nm;
        o.n_fams = g.nf;
        o.n_children = g.nc;
        o.n_grids = (int)g.gf.size();
        o.n_cell_start = (int)g.cell_start.size();
        o.n_cell_items = (int)g.cell_items.size();
        o.scene_in_lds = slds ? 1 : 0;
        o.kinds = g.kinds;
        for (int t = 0; t < sm.n_tallies; ++t) {
            const pr_tally_desc& tdsc = c->tallies[sm.tallies[t]].desc;
            for (int a = 0; a < tdsc.naxes; ++a)
                if (tdsc.axes[a].quantity == PR_Q_TOF) o.kinds |= 1u << kTimeBit;
        }
        if ((g.kinds >> kChopperBit) & 1u) o.kinds |= 1u << kTimeBit;
        if (slds) scene_bytes = std::max(scene_bytes, g.scene_lds_bytes);
        o.tally_begin = (int32_t)P.td.size();
        o.tally_count = sm.n_tallies;
        int64_t need = 0;
        for (int t = 0; t < sm.n_tallies; ++t) need += 2 * (int64_t)c->tallies[sm.tallies[t]].nbins;
        o.privatised = need <= priv_cap ? 1 : 0;
        if (o.privatised) tally_doubles = std::max<int>(tally_doubles, (int)need);
        else any_cache = true;
        uint64_t key = 0;
        int64_t loff = 0;
        for (int t = 0; t < sm.n_tallies; ++t) {
            TallyDev T;
            make_tally_dev(c->tallies[sm.tallies[t]], 0, T);
            if (trial) {   // autotuner trials score into scratch, never into the caller's tallies
                T.sw = c->scratch;
                T.sw2 = c->scratch + 1;
            }
            if (o.privatised) {
                T.lds_offset = (int32_t)loff;
                loff += 2 * T.total;
            }
            P.td.push_back(T);
            P.kb.push_back(key);
            key += (uint64_t)T.total;
        }
        o.first = sm.first_history;
        o.n = sm.n;
        o.hist_begin = total;
        total += sm.n;
        make_source_dev(c->srcs[sm.src], o.src);
    }
    if (any_cache) tally_doubles = std::max(tally_doubles, 2 * nslots);
    if (P.td.empty()) P.kb.push_back(0);
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    P.b_sims = al(P.sd.size() * sizeof(SimDev));
    P.b_tal = al(std::max<size_t>(1, P.td.size()) * sizeof(TallyDev));
    P.b_kb = al(P.kb.size() * sizeof(uint64_t));
    P.total = P.b_sims + P.b_tal + P.b_kb + al(P.sd.size() * sizeof(uint64_t));   // + per-simulation claim counters

    BatchParams& B = P.B;
    memset(&B, 0, sizeof(B));
    B.nsims = ns;
    B.ntallies = (int32_t)P.td.size();
    B.lds_tally_doubles = tally_doubles;
    B.cache_bits = any_cache ? cache_bits : 0;
    B.lds_scene_bytes = scene_bytes;
    B.refill_threshold = c->refill_threshold;
    B.waves = c->waves_per_simd;
    B.walk_cells = c->grid_walk_cells;
    B.total_histories = total;
    B.chunk = (uint64_t)(grid_nav && c->grid_chunk > 0 ? c->grid_chunk : c->chunk);
    B.seed = c->seed;
    B.stats = trial ? c->scratch_stats : c->stats;
    B.sim_next = nullptr;
    B.shift = nullptr;
    const int lds = batch_lds_bytes(B);
    if (lds > kLdsPerCu) return fail(c, PR_EINVAL, "batch needs %d bytes of LDS per block", lds);
    P.block = std::min(c->mixed_block, batch_max_block(grid_nav));
    if (grid_nav && slds) P.block = grid_block(c, [&](int b) { return batch_occupancy(B, slds, grid_nav, b); });
    const int per_cu =
        c->mixed_blocks_per_cu > 0 ? c->mixed_blocks_per_cu : batch_occupancy(B, slds, grid_nav, P.block);
    uint64_t grid = std::min<uint64_t>((uint64_t)per_cu * (uint64_t)c->num_cus, (total + 255) / 256);
    P.grid = (int)std::max<uint64_t>(grid, 1);
    return PR_OK;
}

// host image of a plan's descriptors, laid out as on the device
static void pack_plan(const ClassPlan& P, char* h) {
    memset(h, 0, P.total);
    memcpy(h, P.sd.data(), P.sd.size() * sizeof(SimDev));
    if (!P.td.empty()) memcpy(h + P.b_sims, P.td.data(), P.td.size() * sizeof(TallyDev));
    memcpy(h + P.b_sims + P.b_tal, P.kb.data(), P.kb.size() * sizeof(uint64_t));
}

static void bind_plan(ClassPlan& P, void* dev) {
    P.B.sims = (const SimDev*)dev;
    P.B.tallies = (const TallyDev*)((char*)dev + P.b_sims);
    P.B.tally_key_base = (const uint64_t*)((char*)dev + P.b_sims + P.b_tal);
    P.B.sim_next = (unsigned long long*)((char*)dev + P.b_sims + P.b_tal + P.b_kb);
}

// One persistent launch over the simulations idx of one class.
static int run_batch_class(pr_ctx* c, const pr_sim* sims, const std::vector<int>& idx, bool slds, bool grid_nav,
                           hipStream_t st, bool trial = false) {
    ClassPlan P;
    int rc = plan_batch_class(c, sims, idx, slds, grid_nav, trial, P);
    if (rc) return rc;
    if (P.B.total_histories == 0) return PR_OK;
    // descriptors go through a ring slot: pinned staging, then one async copy
    DescSlot& sl = c->slots[c->next_slot];
    c->next_slot = (c->next_slot + 1) % 4;
    if (sl.used) HIPCHK(c, hipEventSynchronize(sl.done));
    if (sl.bytes < P.total) {
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.host) (void)hipHostFree(sl.host);
        sl.dev = sl.host = nullptr;
        sl.bytes = 0;
        HIPCHK(c, hipMalloc(&sl.dev, P.total));
        HIPCHK(c, hipHostMalloc(&sl.host, P.total, hipHostMallocDefault));
        sl.bytes = P.total;
    }
    if (!sl.done) HIPCHK(c, hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    pack_plan(P, (char*)sl.host);
    HIPCHK(c, hipMemcpyAsync(sl.dev, sl.host, P.total, hipMemcpyHostToDevice, st));
    bind_plan(P, sl.dev);
    hipError_t e = launch_batch(P.B, slds, grid_nav, P.grid, P.block, st);
    if (e != hipSuccess) return hipfail(c, e, "batch kernel launch");
    HIPCHK(c, hipEventRecord(sl.done, st));
    sl.used = true;
    return PR_OK;
}

static int run_batch_all(pr_ctx* c, const pr_sim* sims, int32_t nsims, hipStream_t stream, bool trial);
static std::vector<int> batch_classes(const pr_ctx* c, const pr_sim* sims, int32_t nsims);

static int validate_sims(pr_ctx* c, const pr_sim* sims, int32_t nsims) {
    for (int i = 0; i < nsims; ++i) {
        const pr_sim& sm = sims[i];
        if (sm.geom < 0 || sm.geom >= (int)c->geoms.size()) return fail(c, PR_ENOTFOUND, "sims[%d].geom unknown", i);
        if (sm.src < 0 || sm.src >= (int)c->srcs.size()) return fail(c, PR_ENOTFOUND, "sims[%d].src unknown", i);
        if (sm.n_tallies < 0 || sm.n_tallies > PR_MAX_TALLIES) return fail(c, PR_EINVAL, "sims[%d].n_tallies out of range", i);
        if (sm.n > (1ull << 48) || sm.first_history > (1ull << 62)) return fail(c, PR_EINVAL, "sims[%d] history range too large", i);
        for (int t = 0; t < sm.n_tallies; ++t) {
            const int tid = sm.tallies[t];
            if (tid < 0 || tid >= (int)c->tallies.size()) return fail(c, PR_ENOTFOUND, "sims[%d].tallies[%d] unknown", i, t);
            for (int u = 0; u < t; ++u)
                if (sm.tallies[u] == tid) return fail(c, PR_EINVAL, "sims[%d] lists tally %d twice", i, tid);
            const pr_tally_desc& td = c->tallies[tid].desc;
            if (td.trigger == PR_TRIG_DETECT && td.trigger_volume >= c->geoms[sm.geom].nv)
                return fail(c, PR_EINVAL, "sims[%d]: tally %d trigger_volume beyond its geometry", i, tid);
            if (td.trigger == PR_TRIG_FIRST_COLLISION)
                return fail(c, PR_EINVAL, "sims[%d]: first-collision tallies run with the FP64 policies only", i);
        }
    }
    return PR_OK;
}

extern "C" int pr_run_batch(pr_ctx* c, const pr_sim* sims, int32_t nsims, int32_t precision, void* stream) {
    if (!c || !sims) return fail(c, PR_EINVAL, "null argument");
    if (nsims < 1 || nsims > (1 << 20)) return fail(c, PR_EINVAL, "nsims must be in [1, 2^20]");
    if (precision != PR_FP32_MIXED) return fail(c, PR_EINVAL, "batched runs use the PR_FP32_MIXED policy");
    int rc = set_device(c);
    if (rc) return rc;
    if ((rc = validate_sims(c, sims, nsims))) return rc;
    if ((rc = run_batch_all(c, sims, nsims, (hipStream_t)stream, false))) return rc;
    for (int i = 0; i < nsims; ++i)
        for (int t = 0; t < sims[i].n_tallies; ++t) c->tallies[sims[i].tallies[t]].n_hist += sims[i].n;
    return PR_OK;
}

extern "C" int pr_run_batch_static(pr_ctx* c, const pr_sim* sims, int32_t nsims, int32_t precision, void* stream) {
    if (!c || !sims) return fail(c, PR_EINVAL, "null argument");
    if (nsims < 1 || nsims > (1 << 20)) return fail(c, PR_EINVAL, "nsims must be in [1, 2^20]");
    if (precision != PR_FP32_MIXED) return fail(c, PR_EINVAL, "batched runs use the PR_FP32_MIXED policy");
    int rc = set_device(c);
    if (rc) return rc;
    if (!c->static_scratch) return fail(c, PR_EDEVICE, "the static scratch of device %d is not available", c->device);
    if ((rc = validate_sims(c, sims, nsims))) return rc;
    // plan every class, then place their descriptors side by side in the scratch
    const std::vector<int> cls = batch_classes(c, sims, nsims);
    ClassPlan plans[4];
    size_t offs[4] = {0, 0, 0, 0}, total = 0;
    bool used[4] = {false, false, false, false};
    for (int k = 0; k < 4; ++k) {
        std::vector<int> idx;
        for (int i = 0; i < nsims; ++i)
            if (cls[i] == k) idx.push_back(i);
        if (idx.empty()) continue;
        if ((rc = plan_batch_class(c, sims, idx, (k & 1) != 0, (k & 2) != 0, false, plans[k]))) return rc;
        if (plans[k].B.total_histories == 0) continue;
        offs[k] = total;
        total += (plans[k].total + 255) & ~(size_t)255;
        used[k] = true;
    }
    if (total > kStaticScratchBytes)
        return fail(c, PR_EWORKSPACE, "batch descriptors need %zu bytes; the static scratch holds %zu", total,
                    kStaticScratchBytes);
    if (total == 0) return PR_OK;
    if (c->static_host.size() < total) c->static_host.resize(total);
    for (int k = 0; k < 4; ++k)
        if (used[k]) pack_plan(plans[k], c->static_host.data() + offs[k]);
    const hipStream_t st = (hipStream_t)stream;
    // pageable source: the copy has consumed it when the call returns
    HIPCHK(c, hipMemcpyAsync(c->static_scratch, c->static_host.data(), total, hipMemcpyHostToDevice, st));
    for (int k = 0; k < 4; ++k) {
        if (!used[k]) continue;
        bind_plan(plans[k], (char*)c->static_scratch + offs[k]);
        hipError_t e = launch_batch(plans[k].B, plans[k].slds, plans[k].grid_nav, plans[k].grid, plans[k].block, st);
        if (e != hipSuccess) return hipfail(c, e, "batch kernel launch");
    }
    for (int i = 0; i < nsims; ++i)
        for (int t = 0; t < sims[i].n_tallies; ++t) c->tallies[sims[i].tallies[t]].n_hist += sims[i].n;
    return PR_OK;
}

// simulations fall into classes by scene placement (LDS or global) and grid
// navigation (class = staged + 2 * grid); each non-empty class runs as one
// persistent launch
static std::vector<int> batch_classes(const pr_ctx* c, const pr_sim* sims, int32_t nsims) {
    std::vector<int> cls(nsims);
    for (int i = 0; i < nsims; ++i) {
        const Geometry& g = c->geoms[sims[i].geom];
        const bool grid = !g.gd.empty();
        cls[i] = (g.scene_lds_bytes <= (grid ? c->lds_grid_budget : c->lds_scene_budget) ? 1 : 0) + (grid ? 2 : 0);
    }
    return cls;
}

static int run_batch_all(pr_ctx* c, const pr_sim* sims, int32_t nsims, hipStream_t stream, bool trial) {
    int rc;
    const std::vector<int> cls = batch_classes(c, sims, nsims);
    for (int k = 0; k < 4; ++k) {
        std::vector<int> idx;
        for (int i = 0; i < nsims; ++i)
            if (cls[i] == k) idx.push_back(i);
        if (idx.empty()) continue;
        if ((rc = run_batch_class(c, sims, idx, (k & 1) != 0, (k & 2) != 0, stream, trial))) return rc;
    }
    return PR_OK;
}

// =========================================================================
// prepared batches
// =========================================================================

extern "C" int pr_prepare_batch(pr_ctx* c, const pr_sim* sims, int32_t nsims, int32_t precision, uint64_t stride,
                                int32_t* batch) {
    if (!c || !sims || !batch) return fail(c, PR_EINVAL, "null argument");
    if (nsims < 1 || nsims > (1 << 20)) return fail(c, PR_EINVAL, "nsims must be in [1, 2^20]");
    if (precision != PR_FP32_MIXED) return fail(c, PR_EINVAL, "batched runs use the PR_FP32_MIXED policy");
    if (c->device < 0) return fail(c, PR_EDEVICE, "context has no device");
    int rc = set_device(c);
    if (rc) return rc;
    if ((rc = validate_sims(c, sims, nsims))) return rc;
    PreparedBatch pb;
    pb.stride = stride;
    auto bail = [&](int code) {
        free_prepared(pb);
        return code;
    };
    const std::vector<int> cls = batch_classes(c, sims, nsims);
    for (int k = 0; k < 4; ++k) {
        std::vector<int> idx;
        for (int i = 0; i < nsims; ++i)
            if (cls[i] == k) idx.push_back(i);
        if (idx.empty()) continue;
        ClassPlan P;
        if ((rc = plan_batch_class(c, sims, idx, (k & 1) != 0, (k & 2) != 0, false, P))) return bail(rc);
        if (P.B.total_histories == 0) continue;
        std::vector<char> host(P.total, 0);
        pack_plan(P, host.data());
        void* dev = nullptr;
        hipError_t e = hipMalloc(&dev, P.total);
        if (e != hipSuccess) return bail(hipfail(c, e, "prepared batch descriptors"));
        pb.desc.push_back(dev);
        if ((e = hipMemcpy(dev, host.data(), P.total, hipMemcpyHostToDevice)) != hipSuccess)
            return bail(hipfail(c, e, "prepared batch descriptors"));
        bind_plan(P, dev);
        pb.plans.push_back(std::move(P));
    }
    // history-id offset and per-tally history counts live on the device
    hipError_t e = hipMalloc(&pb.shift, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemset(pb.shift, 0, sizeof(unsigned long long));
    if (e != hipSuccess) return bail(hipfail(c, e, "prepared batch offset"));
    std::map<int32_t, unsigned long long> per_tally;
    for (int i = 0; i < nsims; ++i)
        for (int t = 0; t < sims[i].n_tallies; ++t) per_tally[sims[i].tallies[t]] += sims[i].n;
    std::vector<unsigned long long*> ptrs;
    std::vector<unsigned long long> adds;
    for (auto& kv : per_tally) {
        Tally& T = c->tallies[kv.first];
        if (!T.dev_nhist) {
            if ((e = hipMalloc(&T.dev_nhist, sizeof(unsigned long long))) != hipSuccess ||
                (e = hipMemset(T.dev_nhist, 0, sizeof(unsigned long long))) != hipSuccess) {
                T.dev_nhist = nullptr;
                return bail(hipfail(c, e, "tally history counter"));
            }
        }
        ptrs.push_back(T.dev_nhist);
        adds.push_back(kv.second);
    }
    pb.nh = (int)ptrs.size();
    if (pb.nh > 0) {
        if ((e = hipMalloc(&pb.hist_ptrs, ptrs.size() * sizeof(void*))) != hipSuccess ||
            (e = hipMalloc(&pb.hist_add, adds.size() * sizeof(unsigned long long))) != hipSuccess ||
            (e = hipMemcpy(pb.hist_ptrs, ptrs.data(), ptrs.size() * sizeof(void*), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(pb.hist_add, adds.data(), adds.size() * sizeof(unsigned long long), hipMemcpyHostToDevice)) !=
                hipSuccess)
            return bail(hipfail(c, e, "prepared batch history counters"));
    }
    for (auto& P : pb.plans) P.B.shift = pb.shift;
    pb.live = true;
    int id = -1;
    for (size_t i = 0; i < c->prepared.size(); ++i)
        if (!c->prepared[i].live) { id = (int)i; break; }
    if (id < 0) {
        id = (int)c->prepared.size();
        c->prepared.emplace_back();
    }
    c->prepared[id] = std::move(pb);
    *batch = id;
    return PR_OK;
}

extern "C" int pr_run_prepared(pr_ctx* c, int32_t batch, void* stream) {
    if (!c) return PR_EINVAL;
    if (batch < 0 || batch >= (int)c->prepared.size() || !c->prepared[batch].live)
        return fail(c, PR_ENOTFOUND, "prepared batch %d unknown", batch);
    int rc = set_device(c);
    if (rc) return rc;
    PreparedBatch& pb = c->prepared[batch];
    const hipStream_t st = (hipStream_t)stream;
    for (const ClassPlan& P : pb.plans) {
        hipError_t e = launch_batch(P.B, P.slds, P.grid_nav, P.grid, P.block, st);
        if (e != hipSuccess) return hipfail(c, e, "batch kernel launch");
    }
    hipError_t e = prepared_tail(pb.hist_ptrs, pb.hist_add, pb.nh, pb.shift, pb.stride, st);
    if (e != hipSuccess) return hipfail(c, e, "prepared batch tail");
    return PR_OK;
}

extern "C" int pr_release_batch(pr_ctx* c, int32_t batch) {
    if (!c) return PR_EINVAL;
    if (batch < 0 || batch >= (int)c->prepared.size() || !c->prepared[batch].live)
        return fail(c, PR_ENOTFOUND, "prepared batch %d unknown", batch);
    int rc = set_device(c);
    if (rc) return rc;
    HIPCHK(c, hipDeviceSynchronize());
    free_prepared(c->prepared[batch]);
    return PR_OK;
}

// =========================================================================
// autotuner
// =========================================================================

// Time `reps` runs of the sampled workload with the context's current tuning
// (after one warm-up); returns the fastest, in ms.
static int trial_ms(pr_ctx* c, const std::vector<pr_sim>& sample, bool batched, hipStream_t st, hipEvent_t e0,
                    hipEvent_t e1, int reps, float* best) {
    *best = 1e30f;
    for (int r = 0; r <= reps; ++r) {
        HIPCHK(c, hipEventRecord(e0, st));
        int rc;
        if (batched) {
            rc = run_batch_all(c, sample.data(), (int32_t)sample.size(), st, true);
        } else {
            const pr_sim& s = sample[0];
            rc = run_single(c, s.geom, s.src, s.tallies, s.n_tallies, s.first_history, s.n, PR_FP32_MIXED, nullptr,
                            nullptr, 0, st, true);
        }
        if (rc) return rc;
        HIPCHK(c, hipEventRecord(e1, st));
        HIPCHK(c, hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
        if (r > 0 && ms < *best) *best = ms;
    }
    return PR_OK;
}

extern "C" int pr_autotune(pr_ctx* c, const pr_sim* sims, int32_t nsims, double sample_fraction, pr_tuning* best,
                           void* stream) {
    if (!c || !sims || !best) return fail(c, PR_EINVAL, "null argument");
    if (nsims < 1 || nsims > (1 << 20)) return fail(c, PR_EINVAL, "nsims must be in [1, 2^20]");
    if (!(sample_fraction > 0.0 && sample_fraction <= 1.0)) return fail(c, PR_EINVAL, "sample_fraction must be in (0, 1]");
    int rc = set_device(c);
    if (rc) return rc;
    if ((rc = validate_sims(c, sims, nsims))) return rc;
    const bool batched = nsims > 1;
    std::vector<pr_sim> sample(sims, sims + nsims);
    uint64_t maxbins = 1;
    for (auto& s : sample) {
        s.n = std::max<uint64_t>(1, (uint64_t)std::llround((double)s.n * sample_fraction));
        for (int t = 0; t < s.n_tallies; ++t) maxbins = std::max(maxbins, c->tallies[s.tallies[t]].nbins);
    }
    if (c->scratch_bins < maxbins) {
        if (c->scratch) (void)hipFree(c->scratch);
        c->scratch = nullptr;
        c->scratch_bins = 0;
        HIPCHK(c, hipMalloc((void**)&c->scratch, 2 * maxbins * sizeof(double)));
        c->scratch_bins = maxbins;
    }
    if (!c->scratch_stats) HIPCHK(c, hipMalloc((void**)&c->scratch_stats, ST_N * sizeof(unsigned long long)));
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    // coordinate descent over the launch parameters, two passes
    struct Knob {
        int* field;
        std::vector<int> values;
    };
    std::vector<Knob> knobs = {
        {&c->refill_threshold, {4, 8, 16, 24, 32, 48}},
        {&c->chunk, {64, 128, 256, 512, 1024}},
        {&c->mixed_blocks_per_cu, {0, 2, 3}},
        {&c->bin_cache_slots, {0, 256, 1024, 2048}},
        {&c->waves_per_simd, {4, 5}},
        {&c->mixed_block, {64, 128, 256, 512, 1024}},
    };
    // scenes with a daughter grid get their own claim size
    bool any_grid = false;
    for (const auto& s : sample) any_grid = any_grid || !c->geoms[s.geom].gd.empty();
    if (any_grid) {
        knobs.push_back({&c->grid_chunk, {0, 64, 128, 256}});
        knobs.push_back({&c->grid_walk_cells, {0, 2, 3, 4, 6, 8, 16}});
    }
    // single runs of scenes where steps that draw nothing can be taken early
    bool any_vac = false;
    for (const auto& s : sample) any_vac = any_vac || c->geoms[s.geom].esc || c->geoms[s.geom].fold;
    if (!batched && any_vac) knobs.push_back({&c->vacuum_steps, {1, 0}});

    float cur = 0.f;
    rc = trial_ms(c, sample, batched, st, e0, e1, 2, &cur);
    for (int pass = 0; pass < 2 && rc == PR_OK; ++pass) {
        for (auto& k : knobs) {
            const int keep = *k.field;
            int bestv = keep;
            float bestt = cur;
            for (int v : k.values) {
                if (v == keep) continue;
                *k.field = v;
                float t = 0.f;
                if ((rc = trial_ms(c, sample, batched, st, e0, e1, 2, &t))) break;
                if (t < bestt * 0.98f) {
                    bestt = t;
                    bestv = v;
                }
            }
            *k.field = bestv;
            cur = bestt;
            if (rc) break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    return pr_get_tuning(c, best);
}
