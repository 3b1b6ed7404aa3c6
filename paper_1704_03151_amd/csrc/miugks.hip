// Host driver and C ABI of the MIUGKS library (see include/miugks.h).
//
// The outer iteration follows Steps 1-8 of Sec. II D: UGKS residuals, FAS
// V-cycle of the macroscopic prediction, Shakhov equilibrium and micro
// residual, CS V-cycle of the correction, update and moments.  All work is
// enqueued on one HIP stream; the only host round trips are the four
// residual norms of each cycle (Step 8) and the closed-domain mass check
// (kept on the device).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "adjoint.hpp"
#include "kernels.hpp"
#include "miugks.h"
#include "setup.hpp"

using namespace miugks;

namespace {

std::string g_create_error;
// device allocator for the contexts created next (null: hipMalloc / hipFree)
miugks_alloc_fn g_alloc = nullptr;
miugks_free_fn g_free = nullptr;
void* g_alloc_user = nullptr;

struct DevLevel {
    Geo geo;
    std::vector<void*> owned;
};

}  // namespace

// Fixed device scratch of the allocation-free entry point
// (miugks_get_f_noalloc): every GPU the library runs on holds its own copy
// until the process ends.  Host code never passes this name to a kernel or a
// copy: it is a host-side stand-in; the device address comes from
// hipGetSymbolAddress (scratch_address below).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// Device address of the scratch array on `device`, looked up once per device
// with that device current.
int scratch_address(int device, void** out, std::string& err) {
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) {
        err = "device index beyond the scratch table";
        return MIUGKS_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) {
            err = "hipGetDevice failed";
            return MIUGKS_EDEVICE;
        }
        if (cur != device && hipSetDevice(device) != hipSuccess) {
            err = "hipSetDevice failed";
            return MIUGKS_EDEVICE;
        }
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) {
            err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return MIUGKS_EDEVICE;
        }
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return MIUGKS_OK;
}

}  // namespace

struct miugks_timing_state;

struct miugks_ctx {
    std::string err;
    // the device allocator of this context (null: hipMalloc / hipFree)
    miugks_alloc_fn alloc = nullptr;
    miugks_free_fn free_fn = nullptr;
    void* alloc_user = nullptr;
    hipStream_t stream = nullptr;
    int device = 0;
    void* scratch = nullptr;   // device address of this GPU's allocation-free scratch
    int prec = MIUGKS_FP64;
    size_t esize = 8;
    int nk = 0, nu = 0, nv = 0, L = 1;
    int nu1 = 2, nu2 = 1, nuc = 10;
    int nuc_cs = 10;   // smoothings of the CS cycle on its coarsest level
    int gamma = 1;     // coarse corrections per level visit (1: V-cycle, 2: W-cycle,
                       // MIUGKS_CYCLE_F: F-cycle), FAS
    int gamma_cs = 1;  // the same for the CS cycle
    int FL = 1;   // levels of the FAS prediction, counted from the finest one in use
    // finest level the cycles run on: 0, except during a full-multigrid start,
    // whose stages treat a coarse level as the finest (f then holds that level)
    int top = 0;
    int kch_force = 0;   // > 0: velocities per block of the chunked reductions (chunk_len)
    int flux_mk_force = 0;   // 16 or 24: velocities per thread of the flux (flux_mk)
    // set around a correction whose result is applied at once (Step 6): the
    // finest level's last sweep, if in bands, adds df to f itself (fused)
    void* fuse_f = nullptr;
    bool fused = false;
    bool no_fuse = false;   // MIUGKS_NO_FUSED_UPDATE: keep Step 6 in the moments kernel
    bool wall_sliced = false;   // MIUGKS_WALL_SLICED: wall densities by slices for any velocity count
    double dtn_growth = 0.0;
    double dtn_max = 0.0;   // cap of a^n (0: none)
    double cfl = 0.5;
    bool renorm = false;
    // symmetry faces present: the cycles take the general CS path, whose
    // sweep reads the mirror ghosts from a snapshot of the correction (msnap)
    bool has_sym = false;
    std::vector<void*> msnap;
    HostVel hv;
    std::vector<HostLevel> hl;
    std::vector<Geo> geo;
    Vel vel{};
    Gas gas{};
    std::vector<void*> allocs;
    // level 0
    void *f = nullptr, *div = nullptr, *finf = nullptr;
    double *W = nullptr, *q = nullptr, *R = nullptr, *Wt = nullptr, *fp = nullptr, *cp = nullptr;
    double *part = nullptr, *norms = nullptr, *rho_w = nullptr, *mass = nullptr, *msum = nullptr;
    double* loads = nullptr;   // [4][n_wall] wall loads of level 0
    // explicit time-accurate steps: cell records of W^n, the global step per
    // cell (the level-0 geometry points at it during those steps), W^n scratch
    double *cp0 = nullptr, *dt_glob = nullptr, *Wtmp = nullptr, *tau_tmp = nullptr;
    double dt_global = 0.0;
    size_t part_bytes = 0;
    // per level
    std::vector<void*> r, df;
    std::vector<double*> tau_inv, dtn_inv, drho;
    std::vector<double*> fW, fW0, fR, fP, fE, fGam, fRm, fW2;
    double* h_norms = nullptr;   // pinned
    double M0 = 1.0;
    int cycle = 0;
    bool have_div = false;
    struct miugks_timing_state* timing = nullptr;
    // ordered-sweep support per level
    std::vector<unsigned*> flags;
    std::vector<double*> wbuf, wbuf_alt;   // wall-product partial sums; sweeps alternate between the two
    std::vector<double*> wdpart;           // partial sums of the wall densities per velocity slice
    std::vector<char> sweep_lds;
    // wavefront sweep (k_sweep_wave): side types and launch shape per level
    // (W = 0: not used on that level)
    // (stream: k_sweep_stream, one velocity per wavefront, instead)
    struct WaveCfg {
        int W = 0, I = 1, R = 1, blocks = 0;
        size_t lds = 0;
        bool stream = false;
        // per-cell data read through the caches (the tile alone fills the
        // LDS); split: the G and H planes as separate blocks of a one-plane sweep
        bool gc = false, split = false;
        int strips = 0;   // > 0: k_sweep_strips over that many strips of columns
        int bands = 0, bh = 0;   // > 0: k_sweep_band, that many bands of bh rows (one launch each)
    };
    std::vector<unsigned char*> stype;   // per cell, the side predicates of the LDS sweeps
    std::vector<void*> coefT;   // 1/tau + 1/dt_n per level in the distribution's type
    // restricted defect after an ordered sweep: per coarse cell the ranges of
    // the fine wall list under it and its inverse fluid volume; the change of
    // the wall densities since the last sweep
    std::vector<int4*> cwall;
    // number of wall-product partial sums the last sweep of each level left
    std::vector<int> wparts;
    std::vector<double*> civol, ddrho;
    std::vector<char> last_from_zero;
    CoefSet coefset{};
    std::vector<WaveCfg> wave, wave1;   // sweeping G and H, G only
    // graphs of Step 1 and Steps 2-7; pseudo-step factor a^{-n}
    bool use_graphs = true;
    bool own_stream = false;
    hipGraphExec_t g_step1 = nullptr, g_rest = nullptr;
    double* d_factor = nullptr;
    double* h_factor = nullptr;
    // FAS levels run inside one workgroup from this level on
    int fas_block_l0 = 1 << 30;
    std::vector<size_t> fas_block_lds;   // LDS of the one-workgroup FAS kernel starting at level l
    FasSet fasset{};
    // adjoint (allocated on first use): lam, residual, preconditioned step,
    // right-hand side, product, per-(k, cell) gathers, cell / face / wall
    // records, objective weights and partial sums
    double *a_lam = nullptr, *a_res = nullptr, *a_y = nullptr, *a_b = nullptr, *a_out = nullptr;
    double *a_gbd = nullptr, *a_sb = nullptr, *a_crec = nullptr, *a_fa = nullptr, *a_rws = nullptr;
    double *a_objw = nullptr, *a_Qj = nullptr, *a_rhow = nullptr, *a_part = nullptr, *a_grad = nullptr;
    double *a_fsave = nullptr, *a_fsum = nullptr;
    int* a_sides = nullptr;
    int a_nparts = 0;
    // Krylov basis (m + 1 vectors), Hessenberg column, dot-product partials
    double *a_V = nullptr, *a_h = nullptr, *a_dpart = nullptr;
    int a_m = 0;
};

namespace {

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) {                                                                \
            ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);                      \
            return MIUGKS_EDEVICE;                                                             \
        }                                                                                      \
    } while (0)

// device memory through the context's allocator; not recorded for destroy
int raw_alloc(miugks_ctx* ctx, void** p, size_t bytes) {
    if (bytes == 0) bytes = 8;
    if (ctx->alloc) {
        *p = ctx->alloc(bytes, ctx->alloc_user);
        if (!*p) {
            ctx->err = "the caller's allocator returned no memory";
            return MIUGKS_ENOMEM;
        }
        return MIUGKS_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        ctx->err = std::string("hipMalloc: ") + hipGetErrorString(e);
        return MIUGKS_ENOMEM;
    }
    return MIUGKS_OK;
}

void raw_free(miugks_ctx* ctx, void* p) {
    if (!p) return;
    if (ctx->free_fn)
        ctx->free_fn(p, ctx->alloc_user);
    else
        (void)hipFree(p);
}

int dev_alloc(miugks_ctx* ctx, void** p, size_t bytes) {
    int rc = raw_alloc(ctx, p, bytes);
    if (rc) return rc;
    ctx->allocs.push_back(*p);
    return MIUGKS_OK;
}

template <typename P>
int upload(miugks_ctx* ctx, P** dst, const std::vector<P>& src) {
    int rc = dev_alloc(ctx, (void**)dst, src.size() * sizeof(P));
    if (rc) return rc;
    if (!src.empty()) HIP_TRY(hipMemcpy(*dst, src.data(), src.size() * sizeof(P), hipMemcpyHostToDevice));
    return MIUGKS_OK;
}

inline int nchunks(int nk, int kch = KCH) { return (nk + kch - 1) / kch; }
inline int ntiles(int n) { return (n + TILE - 1) / TILE; }
// Velocities per block of the kernels that reduce over the velocities into
// per-chunk partial sums (moments, face moments, time slopes): KCH
// doubled while the launch keeps at least 2048 blocks (eight per CU), up to
// 8 KCH.  Longer chunks write fewer partial sums (NRAW doubles per cell and
// chunk) and spread each block's per-face set-up over more velocities; below
// about 2048 blocks the last round of blocks leaves CUs idle.  Measured on
// the 160x160 square (10 000 velocities: 8 KCH, 19.3 ms per cycle against
// 20.8 with KCH) and the 128x96 plate (1600 velocities: 4 KCH, 2.01 against
// 2.10 ms); the 64x64 cavity (784 velocities) keeps KCH.  A chunk's rows of one
// plane stay below 2^31 bytes (the range of a buffer resource).  force > 0
// (MIUGKS_CHUNK_LEN, at least KCH) sets the length instead, within that range.
inline int chunk_len(int nc, int nk, int force) {
    if (force > 0) {
        int kch = force;
        while (kch > KCH && (size_t)kch * nc * sizeof(double) >= (size_t(1) << 31)) kch /= 2;
        return std::max(kch, KCH);
    }
    int kch = KCH;
    while (kch < 8 * KCH && (long)ntiles(nc) * nchunks(nk, 2 * kch) >= 2048 &&
           (size_t)2 * kch * nc * sizeof(double) < (size_t(1) << 31))
        kch *= 2;
    return kch;
}
inline int nblk(int n, int b = 256) { return (n + b - 1) / b; }

int check_launch(miugks_ctx* ctx) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        ctx->err = std::string("kernel launch: ") + hipGetErrorString(e);
        return MIUGKS_EDEVICE;
    }
    return MIUGKS_OK;
}

// ---------------------------------------------------------------------------
// per-kernel timing: HIP events around each launch on the library's stream,
// aggregated by kernel label together with the launch's algorithmic bytes

struct TimingRec {
    const char* name;
    double bytes;
    hipEvent_t a, b;
};

struct TimingAgg {
    std::string name;
    long launches = 0;
    double ms = 0.0, bytes = 0.0;
};

}  // namespace

struct miugks_timing_state {
    bool on = false;
    std::vector<hipEvent_t> pool;
    std::vector<TimingRec> pending;
    std::vector<TimingAgg> agg;
};

namespace {

miugks_timing_state& timing(miugks_ctx* c) {
    if (!c->timing) c->timing = new miugks_timing_state();
    return *c->timing;
}

TimingRec* timing_begin(miugks_ctx* c, const char* name, double bytes) {
    miugks_timing_state& t = timing(c);
    if (!t.on) return nullptr;
    hipEvent_t e[2];
    for (int i = 0; i < 2; ++i) {
        if (t.pool.empty()) {
            if (hipEventCreate(&e[i]) != hipSuccess) return nullptr;
        } else {
            e[i] = t.pool.back();
            t.pool.pop_back();
        }
    }
    t.pending.push_back({name, bytes, e[0], e[1]});
    (void)hipEventRecord(e[0], c->stream);
    return &t.pending.back();
}

void timing_end(miugks_ctx* c, TimingRec* r) {
    if (r) (void)hipEventRecord(r->b, c->stream);
}

// fold completed records into the aggregate (call after a stream sync)
void timing_harvest(miugks_ctx* c) {
    miugks_timing_state& t = timing(c);
    for (auto& r : t.pending) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            TimingAgg* a = nullptr;
            for (auto& x : t.agg)
                if (x.name == r.name) a = &x;
            if (!a) {
                t.agg.push_back(TimingAgg());
                a = &t.agg.back();
                a->name = r.name;
            }
            a->launches += 1;
            a->ms += ms;
            a->bytes += r.bytes;
        }
        t.pool.push_back(r.a);
        t.pool.push_back(r.b);
    }
    t.pending.clear();
}

#define LAUNCH_SH(c, name, bytes, shmem, kernel, grid, block, ...)                \
    do {                                                                          \
        TimingRec* rec_ = timing_begin((c), (name), (double)(bytes));             \
        hipLaunchKernelGGL(kernel, grid, block, shmem, (c)->stream, __VA_ARGS__); \
        timing_end((c), rec_);                                                    \
    } while (0)
#define LAUNCH(c, name, bytes, kernel, grid, block, ...) \
    LAUNCH_SH(c, name, bytes, 0, kernel, grid, block, __VA_ARGS__)

// A kernel's limit on dynamic LDS (hipFuncAttributeMaxDynamicSharedMemorySize)
// belongs to the kernel, not to a context: contexts only ever raise it, so a
// context created later with smaller tiles never sets it below the size an
// earlier context launches with.
hipError_t raise_lds_limit(const void* f, int bytes) {
    static std::mutex m;
    static std::vector<std::pair<const void*, int>> limits;
    std::lock_guard<std::mutex> lock(m);
    int* cur = nullptr;
    for (auto& p : limits)
        if (p.first == f) cur = &p.second;
    if (cur && *cur >= bytes) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    if (cur)
        *cur = bytes;
    else
        limits.emplace_back(f, bytes);
    return hipSuccess;
}

// LDS bytes of the staged sweep on a level: r/df tile (G, H), 1/tau + 1/dt_n,
// 1/dx, side flags
template <typename T>
size_t sweep_lds_bytes(const Geo& g, int P) {
    size_t b = ((size_t)P * g.nc + g.nc + g.nx + (size_t)P * g.n_wall) * sizeof(T) + 4 * (size_t)g.nc;
    return (b + 15) & ~(size_t)15;
}

template <typename T, int NP, bool GC>
hipError_t set_wave_lds_t(int R, int bytes) {
    auto set = [bytes](const void* f) {
        return raise_lds_limit(f, bytes);
    };
    switch (R) {
        case 1: return set((const void*)k_sweep_wave<T, 1, NP, GC>);
        case 2: return set((const void*)k_sweep_wave<T, 2, NP, GC>);
        case 3: return set((const void*)k_sweep_wave<T, 3, NP, GC>);
        default: return set((const void*)k_sweep_wave<T, 4, NP, GC>);
    }
}

template <typename T, int NP>
hipError_t set_stream_lds_t(int R, int bytes) {
    auto set = [bytes](const void* f) {
        return raise_lds_limit(f, bytes);
    };
    switch (R) {
        case 1: return set((const void*)k_sweep_stream<T, 1, NP>);
        case 2: return set((const void*)k_sweep_stream<T, 2, NP>);
        case 3: return set((const void*)k_sweep_stream<T, 3, NP>);
        default: return set((const void*)k_sweep_stream<T, 4, NP>);
    }
}

hipError_t set_stream_lds(int prec, int R, int np, int bytes) {
    if (prec == MIUGKS_FP64)
        return np == 1 ? set_stream_lds_t<double, 1>(R, bytes) : set_stream_lds_t<double, 2>(R, bytes);
    return np == 1 ? set_stream_lds_t<float, 1>(R, bytes) : set_stream_lds_t<float, 2>(R, bytes);
}

template <typename T>
hipError_t set_strips_lds_t(int R, int bytes) {
    auto set = [bytes](const void* f) {
        return raise_lds_limit(f, bytes);
    };
    switch (R) {
        case 1: return set((const void*)k_sweep_strips<T, 1>);
        case 2: return set((const void*)k_sweep_strips<T, 2>);
        case 3: return set((const void*)k_sweep_strips<T, 3>);
        default: return set((const void*)k_sweep_strips<T, 4>);
    }
}

hipError_t set_strips_lds(int prec, int R, int bytes) {
    return prec == MIUGKS_FP64 ? set_strips_lds_t<double>(R, bytes) : set_strips_lds_t<float>(R, bytes);
}

hipError_t set_band_lds(int prec, int bytes) {
    return raise_lds_limit(prec == MIUGKS_FP64 ? (const void*)k_sweep_band<double> : (const void*)k_sweep_band<float>,
                           bytes);
}

hipError_t set_wave_lds(int prec, int R, int np, int bytes) {
    hipError_t e;
    if (prec == MIUGKS_FP64) {
        e = np == 1 ? set_wave_lds_t<double, 1, false>(R, bytes) : set_wave_lds_t<double, 2, false>(R, bytes);
        if (e == hipSuccess && np == 1) e = set_wave_lds_t<double, 1, true>(R, bytes);
        return e;
    }
    e = np == 1 ? set_wave_lds_t<float, 1, false>(R, bytes) : set_wave_lds_t<float, 2, false>(R, bytes);
    if (e == hipSuccess && np == 1) e = set_wave_lds_t<float, 1, true>(R, bytes);
    return e;
}

// Coarse-level cycles that one visit of a level makes (Sec. II D): gamma > 0
// gives gamma cycles of the same kind (1: V-cycle, 2: W-cycle), each from the
// level's current iterate; MIUGKS_CYCLE_F gives an F-cycle then a V-cycle.
int coarse_visits(int gamma) { return gamma == MIUGKS_CYCLE_F ? 2 : gamma; }
int visit_kind(int gamma, int i) { return gamma == MIUGKS_CYCLE_F ? (i == 0 ? MIUGKS_CYCLE_F : 1) : gamma; }

// ---------------------------------------------------------------------------
// the hot path, per precision

template <typename T>
struct Path {
    static T* F(miugks_ctx* c) { return (T*)c->f; }
    // bytes of one distribution-shaped array on level l
    static double arr(miugks_ctx* c, int l) { return 2.0 * c->nk * c->geo[l].nc * sizeof(T); }

    // Step 7: W, q of f (optionally after f += df, Step 6)
    static void moments(miugks_ctx* c, const T* df) {
        const Geo& g = c->geo[c->top];
        const int kch = chunk_len(g.nc, c->nk, c->kch_force), nkc = nchunks(c->nk, kch);
        double nc8 = g.nc * 8.0;
        LAUNCH(c, df ? "update_moments" : "moments", (df ? 3 : 1) * arr(c, c->top) + NRAW * nkc * nc8,
               k_moments_partial<T>, dim3(ntiles(g.nc), nkc), dim3(256), g, c->vel, F(c), df, c->part, kch);
        LAUNCH(c, "chunk_sum", NRAW * (nkc + 1.0) * nc8, k_chunk_sum, dim3(nblk(NRAW * g.nc)), dim3(256),
               (const double*)c->part, nkc, NRAW, g.nc, 1.0, (const unsigned char*)nullptr, c->msum);
        LAUNCH(c, "moments_records", (NRAW + 6.0) * nc8, k_moments_records, dim3(nblk(g.nc)), dim3(256), g,
               (const double*)c->msum, c->W, c->q);
    }

    static void wall_sums(miugks_ctx* c, int l, const T* G, double* out) {
        const Geo& g = c->geo[l];
        if (g.n_wall == 0) return;
        if (c->nk <= WD_WAVE_MAX_NK && !c->wall_sliced) {
            LAUNCH(c, "wall_density", (double)g.n_wall * c->nk * sizeof(T), (k_wall_density_wave<T, false>),
                   dim3((g.n_wall + 3) / 4), dim3(256), g, c->vel, G, g.nc, (const T*)nullptr, out);
            return;
        }
        const int ns = wall_density_slices(c->nk);
        LAUNCH(c, "wall_density", (double)g.n_wall * c->nk * sizeof(T), (k_wall_density_part<T, false>),
               dim3((g.n_wall + 63) / 64, ns), dim3(64), g, c->vel, G, g.nc, (const T*)nullptr, c->wdpart[l]);
        LAUNCH(c, "wall_density", (double)g.n_wall * ns * 8.0, k_wall_density_fin, dim3((g.n_wall + 3) / 4),
               dim3(256), g, ns, (const double*)c->wdpart[l], out);
    }

    // Step 1: interface records, div, R and the RMS norms (into c->norms)
    static void residual(miugks_ctx* c) {
        const int top = c->top;
        const Geo& g = c->geo[top];
        const int kch = chunk_len(g.nc, c->nk, c->kch_force), nkc = nchunks(c->nk, kch), nt = ntiles(g.nc);
        double nc8 = g.nc * 8.0;
        // raw moments of the upwind interface distributions, per velocity
        // chunk, summed in chunk order; interface records
        LAUNCH(c, "face_moments", arr(c, top) + 2.0 * NRAW * nkc * nc8, k_face_moments_partial<T>, dim3(nt, nkc),
               dim3(256), g, c->vel, F(c), c->part, kch);
        LAUNCH(c, "chunk_sum", 2.0 * NRAW * (nkc + 1) * nc8, k_chunk_sum, dim3(nblk(2 * NRAW * g.nc)), dim3(256),
               (const double*)c->part, nkc, 2 * NRAW, g.nc, 1.0, (const unsigned char*)nullptr, c->msum);
        LAUNCH(c, "face_records", (2.0 * NRAW + 8 + 2 * NFP) * nc8, k_face_records, dim3(nblk(2 * g.nc)),
               dim3(256), g, c->gas, (const double*)c->msum, (const double*)c->W, c->fp);
        // time slopes from the discrete compatibility condition
        LAUNCH(c, "face_timeslope", (2.0 * NFP + 8.0 * nkc) * nc8, k_face_timeslope_partial<T>, dim3(nt, nkc),
               dim3(256), g, c->vel, c->gas, (const double*)c->fp, c->part, kch);
        LAUNCH(c, "chunk_sum", 8.0 * (nkc + 1) * nc8, k_chunk_sum, dim3(nblk(8 * g.nc)), dim3(256),
               (const double*)c->part, nkc, 8, g.nc, 1.0, (const unsigned char*)nullptr, c->msum);
        LAUNCH(c, "timeslope_records", (8.0 + 2 * 8) * nc8, k_face_timeslope_records, dim3(nblk(2 * g.nc)),
               dim3(256), g, c->gas, (const double*)c->msum, c->fp);
        wall_sums(c, top, F(c), c->rho_w);
        // the flux takes chunks of WAVES * mk velocities: a thread holds its mk
        // velocities of div in registers, and the partial sums are 4 per cell
        const int mk = flux_mk(sizeof(T) == 4, flux_tiles(g), c->nk, c->flux_mk_force);
        const int nkf = nchunks(c->nk, WAVES * mk);
        const double fbytes = 2 * arr(c, top) + (2.0 * NFP + 4.0 * nkf) * nc8;
        bool launched = false;
        if constexpr (sizeof(T) == 4) {
            if (mk == 24) {
                LAUNCH(c, "flux_div", fbytes, (k_flux_div<T, 24>), dim3(flux_tiles(g), nkf), dim3(256), g, c->vel,
                       c->gas, F(c), c->fp, c->rho_w, (const T*)c->finf, (T*)c->div, c->part, flux_stride(g));
                launched = true;
            }
        }
        if (!launched)
            LAUNCH(c, "flux_div", fbytes, (k_flux_div<T, 16>), dim3(flux_tiles(g), nkf), dim3(256), g, c->vel, c->gas,
                   F(c), c->fp, c->rho_w, (const T*)c->finf, (T*)c->div, c->part, flux_stride(g));
        LAUNCH(c, "chunk_sum", 4.0 * (nkf + 1) * nc8, k_chunk_sum, dim3(nblk(4 * g.nc)), dim3(256),
               (const double*)c->part, nkf, 4, g.nc, -1.0, g.solid, c->R);
        LAUNCH(c, "residual_norm", 4 * nc8, k_residual_norm, dim3(1), dim3(256), g, c->hl[top].n_fluid, c->R,
               c->norms);
        c->have_div = true;
    }

    // Steps 3-4 (with the positivity guard on c->Wt)
    static void micro_residual(miugks_ctx* c) {
        const int top = c->top;
        const Geo& g = c->geo[top];
        LAUNCH(c, "cell_prep", (14.0 + NCP) * g.nc * 8, k_cell_prep, dim3(nblk(g.nc)), dim3(256), g, c->gas, c->Wt,
               c->W, c->q, c->cp, c->tau_inv[top]);
        LAUNCH(c, "micro_residual", 3 * arr(c, top) + NCP * g.nc * 8.0, k_micro_residual<T>,
               dim3(ntiles(g.nc), nchunks(c->nk)), dim3(256), g, c->vel, c->gas, F(c), (const T*)c->div, c->cp,
               (T*)c->r[top]);
    }

    // one smoothing on level l: wall densities from the current correction
    // (skipped when drho is already current), then the ordered sweep, which
    // also leaves the wall products of its result in wbuf
    static void smooth(miugks_ctx* c, int l, bool drho_current, bool from_zero = false, int np = 2) {
        const Geo& g = c->geo[l];
        c->last_from_zero[l] = from_zero && c->wave[l].W;
        const miugks_ctx::WaveCfg& wc = np == 1 ? c->wave1[l] : c->wave[l];
        // the wall densities from the last sweep's partial sums: inside the
        // wavefront sweep where they are few, else by k_drho
        // (the sweep's prologue takes one thread per wall side)
        const bool in_sweep = !drho_current && g.n_wall && wc.W && !wc.bands && g.n_wall <= 64 * wc.W &&
                              (long)c->wparts[l] * g.n_wall <= 16L * 64 * wc.W && !getenv("MIUGKS_DRHO_KERNEL");
        if (!drho_current && g.n_wall && !in_sweep)
            LAUNCH(c, "drho", (double)g.n_wall * c->wparts[l] * 8, k_drho, dim3((g.n_wall + 3) / 4), dim3(256), g,
                   c->wparts[l], c->wbuf[l], c->drho[l]);
        static const char* const names[] = {"sweep/l0", "sweep/l1", "sweep/l2", "sweep/l3",
                                            "sweep/l4", "sweep/l5", "sweep/l6", "sweep/l7"};
        const char* name = names[l < 8 ? l : 7];
        // the sweep leaves its partial sums in the other buffer
        std::swap(c->wbuf[l], c->wbuf_alt[l]);
        if (wc.W && wc.stream) {
#define MIUGKS_STREAM_LAUNCH(RR, NP)                                                                            \
    LAUNCH_SH(c, name, (NP) * arr(c, l), wc.lds, (k_sweep_stream<T, RR, NP>), dim3(wc.blocks), dim3(64 * wc.W),   \
              g, c->vel, c->gas.K_int, (const T*)c->r[l], (T*)c->df[l], (const T*)c->coefT[l],                 \
              (const unsigned*)c->flags[l], from_zero ? (const double*)nullptr : (const double*)c->drho[l],    \
              c->wbuf[l], in_sweep ? (const double*)c->wbuf_alt[l] : (const double*)nullptr, c->wparts[l],      \
              c->drho[l])
            if (np == 1) {
                switch (wc.R) {
                    case 1: MIUGKS_STREAM_LAUNCH(1, 1); break;
                    case 2: MIUGKS_STREAM_LAUNCH(2, 1); break;
                    case 3: MIUGKS_STREAM_LAUNCH(3, 1); break;
                    default: MIUGKS_STREAM_LAUNCH(4, 1); break;
                }
            } else {
                switch (wc.R) {
                    case 1: MIUGKS_STREAM_LAUNCH(1, 2); break;
                    case 2: MIUGKS_STREAM_LAUNCH(2, 2); break;
                    case 3: MIUGKS_STREAM_LAUNCH(3, 2); break;
                    default: MIUGKS_STREAM_LAUNCH(4, 2); break;
                }
            }
#undef MIUGKS_STREAM_LAUNCH
            c->wparts[l] = wc.blocks;
        } else if (wc.W && wc.bands) {
            // one launch per band, in every velocity's upwind order; each
            // reads the last row of the band before from df.  The finest
            // level's last sweep of a correction applied at once adds df to
            // f instead of storing it (then Step 6 only takes the moments).
            const int nblk = wc.split ? wc.blocks / 2 : wc.blocks;
            T* fout = (np == 2 && l == c->top && c->fuse_f) ? (T*)c->fuse_f : nullptr;
            const double planes = (wc.split ? 2 : 1) * (fout ? 1.5 : 1.0);
            for (int b = 0; b < wc.bands; ++b) {
                const int hb = std::min(wc.bh, g.ny - b * wc.bh);
                LAUNCH_SH(c, name, planes * arr(c, l) * hb / g.ny, wc.lds, k_sweep_band<T>,
                          dim3(wc.blocks), dim3(64 * wc.W), g, c->vel, c->gas.K_int, (const T*)c->r[l],
                          (T*)c->df[l], (const T*)c->coefT[l], c->stype[l],
                          from_zero ? (const double*)nullptr : (const double*)c->drho[l], c->wbuf[l], wc.I, wc.bh,
                          b, c->nv, wc.split ? 1 : 0, fout);
            }
            c->wparts[l] = nblk;
            if (fout) c->fused = true;
        } else if (wc.W && wc.strips) {
#define MIUGKS_STRIPS_LAUNCH(RR)                                                                                 \
    LAUNCH_SH(c, name, (wc.split ? 2 : 1) * arr(c, l), wc.lds, (k_sweep_strips<T, RR>), dim3(wc.blocks),           \
              dim3(64 * wc.W), g, c->vel, c->gas.K_int, (const T*)c->r[l], (T*)c->df[l], (const T*)c->coefT[l],      \
              c->stype[l], from_zero ? (const double*)nullptr : (const double*)c->drho[l], c->wbuf[l], wc.strips,    \
              in_sweep ? (const double*)c->wbuf_alt[l] : (const double*)nullptr, c->wparts[l], c->drho[l],          \
              wc.split ? 1 : 0, c->nv)
            switch (wc.R) {
                case 1: MIUGKS_STRIPS_LAUNCH(1); break;
                case 2: MIUGKS_STRIPS_LAUNCH(2); break;
                case 3: MIUGKS_STRIPS_LAUNCH(3); break;
                default: MIUGKS_STRIPS_LAUNCH(4); break;
            }
#undef MIUGKS_STRIPS_LAUNCH
            c->wparts[l] = wc.split ? wc.blocks / 2 : wc.blocks;
        } else if (wc.W) {
#define MIUGKS_WAVE_LAUNCH_G(RR, NP, GC)                                                                        \
    LAUNCH_SH(c, name, (wc.split ? 2 : (NP)) * arr(c, l), wc.lds, (k_sweep_wave<T, RR, NP, GC>), dim3(wc.blocks),   \
              dim3(64 * wc.W), g, c->vel, c->gas.K_int, (const T*)c->r[l], (T*)c->df[l], (const T*)c->coefT[l],      \
              c->stype[l], from_zero ? (const double*)nullptr : (const double*)c->drho[l], c->wbuf[l], wc.I,         \
              in_sweep ? (const double*)c->wbuf_alt[l] : (const double*)nullptr, c->wparts[l], c->drho[l],          \
              wc.split ? 1 : 0)
#define MIUGKS_WAVE_LAUNCH(RR, NP)                \
    if (wc.gc)                                    \
        MIUGKS_WAVE_LAUNCH_G(RR, 1, true);        \
    else                                          \
        MIUGKS_WAVE_LAUNCH_G(RR, NP, false)
            if (np == 1 || wc.split) {
                switch (wc.R) {
                    case 1: MIUGKS_WAVE_LAUNCH(1, 1); break;
                    case 2: MIUGKS_WAVE_LAUNCH(2, 1); break;
                    case 3: MIUGKS_WAVE_LAUNCH(3, 1); break;
                    default: MIUGKS_WAVE_LAUNCH(4, 1); break;
                }
            } else {
                switch (wc.R) {
                    case 1: MIUGKS_WAVE_LAUNCH(1, 2); break;
                    case 2: MIUGKS_WAVE_LAUNCH(2, 2); break;
                    case 3: MIUGKS_WAVE_LAUNCH(3, 2); break;
                    default: MIUGKS_WAVE_LAUNCH(4, 2); break;
                }
            }
#undef MIUGKS_WAVE_LAUNCH
#undef MIUGKS_WAVE_LAUNCH_G
            c->wparts[l] = wc.split ? wc.blocks / 2 : wc.blocks;
        } else if (c->sweep_lds[l]) {
            c->wparts[l] = c->nk;
            int npad = ((g.ny + 63) / 64) * 64, P = c->sweep_lds[l];
            int blocks = (2 * c->nk + P - 1) / P;
            LAUNCH_SH(c, name, 2 * arr(c, l), sweep_lds_bytes<T>(g, P), k_sweep_lds<T>, dim3(blocks), dim3(P * npad),
                      g, c->vel, c->gas.K_int, (const T*)c->r[l], (T*)c->df[l], c->tau_inv[l], c->dtn_inv[l],
                      c->flags[l], c->drho[l], c->wbuf[l], npad, P);
        } else {
            c->wparts[l] = c->nk;
            int threads = ((g.ny + 63) / 64) * 64;
            const T* ms = nullptr;
            if (c->has_sym) {   // the mirror ghosts read the correction before the sweep
                size_t n = 2 * (size_t)c->nk * g.nc;
                if (from_zero)
                    LAUNCH(c, "zero", arr(c, l), k_zero<T>, dim3(nblk((int)std::min<size_t>(n, 1 << 24))), dim3(256),
                           (T*)c->msnap[l], n);
                else
                    LAUNCH(c, "copy", 2 * arr(c, l), k_copy_t<T>, dim3(nblk((int)std::min<size_t>(n, 1 << 24))),
                           dim3(256), (const T*)c->df[l], (T*)c->msnap[l], n);
                ms = (const T*)c->msnap[l];
            }
            LAUNCH(c, name, 2 * arr(c, l), k_sweep<T>, dim3(c->nk), dim3(threads), g, c->vel, c->gas.K_int,
                   (const T*)c->r[l], (T*)c->df[l], c->tau_inv[l], c->dtn_inv[l], c->flags[l], c->drho[l],
                   c->wbuf[l], ms);
        }
    }

    // dF_l = CS(l, r_l) (Sec. II D); r_l, tau_inv_l, dtn_inv_l in place.  The
    // correction starts at zero: zero wall densities for the first sweep (the
    // sweep itself needs no initial correction).
    static void cs(miugks_ctx* c, int l, int gamma) {
        const Geo& g = c->geo[l];
        int pre = l == c->L - 1 ? c->nuc_cs : c->nu1;
        // the wavefront sweep starts from zero wall densities by itself
        if (g.n_wall && (!c->wave[l].W || pre == 0))
            LAUNCH(c, "zero", (double)g.n_wall * 8, k_zero<double>, dim3(1), dim3(256), c->drho[l],
                   (size_t)g.n_wall);
        for (int i = 0; i < pre; ++i) smooth(c, l, i == 0, i == 0);
        if (l == c->L - 1) return;
        if (pre == 0) {
            size_t n = 2 * (size_t)c->nk * g.nc;
            LAUNCH(c, "zero", arr(c, l), k_zero<T>, dim3(nblk((int)std::min<size_t>(n, 1 << 24))), dim3(256),
                   (T*)c->df[l], n);
        } else if (g.n_wall) {
            LAUNCH(c, "drho", (double)g.n_wall * c->wparts[l] * 8, k_drho_delta, dim3((g.n_wall + 3) / 4),
                   dim3(256), g, c->wparts[l], c->wbuf[l], c->drho[l], c->ddrho[l], (int)c->last_from_zero[l]);
        }
        const Geo& gc = c->geo[l + 1];
        const int nvis = coarse_visits(gamma);
        for (int gi = 0; gi < nvis; ++gi) {
            if (gi == 0 && pre > 0 && !c->has_sym) {
                // after an ordered sweep the defect lives on the wall cells only
                if (!g.n_wall)
                    LAUNCH(c, "zero", arr(c, l + 1), k_zero<T>,
                           dim3(nblk((int)std::min<size_t>(2 * (size_t)c->nk * gc.nc, 1 << 24))), dim3(256),
                           (T*)c->r[l + 1], 2 * (size_t)c->nk * gc.nc);
                else
                    LAUNCH(c, "defect_walls", arr(c, l + 1), k_defect_walls<T>, dim3(ntiles(gc.nc), nchunks(c->nk)),
                           dim3(256), g, gc, c->vel, c->gas.K_int, (const int4*)c->cwall[l + 1],
                           (const double*)c->civol[l + 1], (const double*)c->ddrho[l], (T*)c->r[l + 1], 2);
            } else {
                LAUNCH(c, "defect_restrict", 2 * arr(c, l) + arr(c, l + 1), k_defect_restrict<T>,
                       dim3(ntiles(gc.nc), nchunks(c->nk)), dim3(256), g, gc, c->vel, c->gas.K_int,
                       (const T*)c->r[l], (const T*)c->df[l], c->tau_inv[l], c->dtn_inv[l], c->drho[l],
                       (T*)c->r[l + 1]);
            }
            cs(c, l + 1, visit_kind(gamma, gi));
            LAUNCH(c, "prolong_add", 2 * arr(c, l) + arr(c, l + 1), k_prolong_add<T>,
                   dim3(ntiles(g.nc), nchunks(c->nk)), dim3(256), g, c->vel, gc.nc, (const T*)c->df[l + 1],
                   (T*)c->df[l]);
            // the prolongation changed the correction: wall densities from it
            if (c->nu2 > 0 || gi + 1 < nvis) wall_sums(c, l, (const T*)c->df[l], c->drho[l]);
        }
        for (int i = 0; i < c->nu2; ++i) smooth(c, l, i == 0);
    }

    // The same V-cycle when every level smooths before and after its coarse
    // correction.  An ordered sweep recomputes the correction from r and the
    // wall densities alone, so (i) a sweep whose result is overwritten by a
    // later sweep needs only its G plane (the wall densities depend on G),
    // which leaves the final sweep of the finest level as the only one that
    // sweeps H; (ii) the coarse levels need the G plane of r only; (iii) the
    // prolonged coarse correction enters only the wall densities of the next
    // sweep, so it is evaluated at the wall cells only.
    static bool cs_reduced_ok(miugks_ctx* c) {
        if (c->nu1 < 1 || c->nu2 < 1 || c->nuc_cs < 1 || c->gamma_cs != 1 || c->has_sym || getenv("MIUGKS_FULL_CS"))
            return false;
        for (int l = 0; l < c->L; ++l)
            if (!c->wave[l].W) return false;
        return true;
    }

    static void cs_reduced(miugks_ctx* c, int l) {
        const Geo& g = c->geo[l];
        const bool coarsest = l == c->L - 1;
        int pre = coarsest ? c->nuc_cs : c->nu1;
        for (int i = 0; i < pre; ++i) {
            // the finest level's last sweep is final only if it is also the coarsest
            int np = (l == c->top && coarsest && i == pre - 1) ? 2 : 1;
            smooth(c, l, i == 0, i == 0, np);
        }
        if (coarsest) return;
        const Geo& gc = c->geo[l + 1];
        if (g.n_wall) {
            LAUNCH(c, "drho", (double)g.n_wall * c->wparts[l] * 8, k_drho_delta, dim3((g.n_wall + 3) / 4),
                   dim3(256), g, c->wparts[l], c->wbuf[l], c->drho[l], c->ddrho[l], (int)c->last_from_zero[l]);
            LAUNCH(c, "defect_walls", arr(c, l + 1) / 2, k_defect_walls<T>, dim3(ntiles(gc.nc), nchunks(c->nk)),
                   dim3(256), g, gc, c->vel, c->gas.K_int, (const int4*)c->cwall[l + 1],
                   (const double*)c->civol[l + 1], (const double*)c->ddrho[l], (T*)c->r[l + 1], 1);
        } else {
            size_t n = (size_t)c->nk * gc.nc;
            LAUNCH(c, "zero", arr(c, l + 1) / 2, k_zero<T>, dim3(nblk((int)std::min<size_t>(n, 1 << 24))), dim3(256),
                   (T*)c->r[l + 1], n);
        }
        cs_reduced(c, l + 1);
        if (g.n_wall && c->nk <= WD_WAVE_MAX_NK && !c->wall_sliced) {
            LAUNCH(c, "wall_density", (double)g.n_wall * c->nk * 5 * sizeof(T), (k_wall_density_wave<T, true>),
                   dim3((g.n_wall + 3) / 4), dim3(256), g, c->vel, (const T*)c->df[l], gc.nc,
                   (const T*)c->df[l + 1], c->drho[l]);
        } else if (g.n_wall) {
            const int ns = wall_density_slices(c->nk);
            LAUNCH(c, "wall_density", (double)g.n_wall * c->nk * 5 * sizeof(T), (k_wall_density_part<T, true>),
                   dim3((g.n_wall + 63) / 64, ns), dim3(64), g, c->vel, (const T*)c->df[l], gc.nc,
                   (const T*)c->df[l + 1], c->wdpart[l]);
            LAUNCH(c, "wall_density", (double)g.n_wall * ns * 8.0, k_wall_density_fin, dim3((g.n_wall + 3) / 4),
                   dim3(256), g, ns, (const double*)c->wdpart[l], c->drho[l]);
        }
        for (int i = 0; i < c->nu2; ++i) smooth(c, l, i == 0, false, (l == c->top && i == c->nu2 - 1) ? 2 : 1);
    }

    static void correct(miugks_ctx* c) {
        for (int l = c->top; l + 1 < c->L; ++l)
            LAUNCH(c, "restrict_cells", (c->geo[l].nc + c->geo[l + 1].nc) * 8.0, k_restrict_cells,
                   dim3(nblk(c->geo[l + 1].nc)), dim3(256), c->geo[l], c->geo[l + 1], 1, c->tau_inv[l],
                   c->tau_inv[l + 1]);
        LAUNCH(c, "sweep_coef", 0.0, k_sweep_coef<T>, dim3(nblk(c->geo[0].nc)), dim3(256), c->coefset);
        if (cs_reduced_ok(c))
            cs_reduced(c, c->top);
        else
            cs(c, c->top, c->gamma_cs);
    }

    // Steps 6-7 and the closed-domain renormalisation (f += df already done
    // if the correction's last sweep was fused with it)
    static void update(miugks_ctx* c) {
        moments(c, c->fused ? (const T*)nullptr : (const T*)c->df[c->top]);
        c->fused = false;
        if (c->renorm) {
            const Geo& g = c->geo[c->top];
            LAUNCH(c, "mass", 4.0 * g.nc * 8, k_mass, dim3(1), dim3(1024), g, c->W, c->mass);
            size_t n = 2 * (size_t)c->nk * g.nc;
            LAUNCH(c, "scale_f", 2 * arr(c, c->top), k_scale_f<T>, dim3(nblk((int)std::min<size_t>(n, 1 << 24))),
                   dim3(256), F(c), n, c->mass, c->M0);
            LAUNCH(c, "scale_moments", 12.0 * g.nc * 8, k_scale_d, dim3(nblk(6 * g.nc)), dim3(256), c->W,
                   4 * (size_t)g.nc, c->mass, c->M0);
            LAUNCH(c, "scale_moments", 4.0 * g.nc * 8, k_scale_d, dim3(nblk(2 * g.nc)), dim3(256), c->q,
                   2 * (size_t)g.nc, c->mass, c->M0);
        }
    }
};

// ---------------------------------------------------------------------------
// FAS cycle (precision independent, FP64)

// one smoothing of Sec. II C 2: renewed residual with the first half-sweep
// (colour 0 from E = 0), red-black half-sweeps of colours 1 and 0, the last
// one with W += E into the other W buffer (four lanes per cell in every
// phase); W and Walt swap
void fas_smooth(miugks_ctx* c, int l, double*& W, double*& Walt) {
    const Geo& g = c->geo[l];
    int nb = nblk(4 * g.nc);
    double nc8 = g.nc * 8.0;
    LAUNCH(c, "fas_rsplit", 22 * nc8, k_fas4_rsplit_first, dim3(nb), dim3(256), g, c->gas, (const double*)W,
           (const double*)c->fGam[l], (const double*)c->fP[l], (const double*)c->dtn_inv[l], c->fRm[l], c->fE[l]);
    LAUNCH(c, "fas_halfsweep", 18 * nc8, k_fas4_halfsweep, dim3(nb), dim3(256), g, c->gas, (const double*)W,
           c->fE[l], (const double*)c->fRm[l], (const double*)c->fGam[l], (const double*)c->dtn_inv[l], 1);
    LAUNCH(c, "fas_halfsweep", 26 * nc8, k_fas4_halfsweep_apply, dim3(nb), dim3(256), g, c->gas, (const double*)W,
           (const double*)c->fE[l], (const double*)c->fRm[l], (const double*)c->fGam[l],
           (const double*)c->dtn_inv[l], Walt);
    std::swap(W, Walt);
}

// W_l^{n+1} = FAS(l, W_l^n, R_l^n): fW[l] holds W_l^n on entry and the result
// on exit; fR[l] holds the target residual
// coarsest level the FAS prediction visits
int fas_last(const miugks_ctx* c) { return std::min(c->top + c->FL, c->L) - 1; }

void fas(miugks_ctx* c, int l, int gamma) {
    if (gamma == 1 && l >= c->fas_block_l0 && fas_last(c) == c->fasset.L - 1) {
        FasSet F = c->fasset;
        F.l0 = l;
        double cells = 0;
        for (int q = l; q < c->L; ++q) cells += c->geo[q].nc;
        LAUNCH_SH(c, "fas_cycle_block", 60 * cells * 8.0, c->fas_block_lds[l], k_fas_cycle_block, dim3(1),
                  dim3(1024), F, c->gas);
        return;
    }
    const Geo& g = c->geo[l];
    int nb = nblk(4 * g.nc);
    double nc8 = g.nc * 8.0;
    double *W = c->fW[l], *Walt = c->fW2[l];
    // W0 := W, the frozen Gamma, the forcing P = R - R_split(W0)
    LAUNCH(c, "fas_enter", 28 * nc8, k_fas4_enter, dim3(nb), dim3(256), g, c->gas, (const double*)W, c->fW0[l],
           c->fGam[l], (const double*)c->fR[l], c->fP[l]);
    if (l == fas_last(c)) {
        for (int i = 0; i < c->nuc; ++i) fas_smooth(c, l, W, Walt);
    } else {
        for (int i = 0; i < c->nu1; ++i) fas_smooth(c, l, W, Walt);
        const Geo& gc = c->geo[l + 1];
        const int nvis = coarse_visits(gamma);
        for (int gi = 0; gi < nvis; ++gi) {
            LAUNCH(c, "fas_rsplit", 20 * nc8, k_fas4_rsplit, dim3(nb), dim3(256), g, c->gas, (const double*)W,
                   (const double*)c->fGam[l], (const double*)c->fP[l], 1.0, c->fRm[l], (double*)nullptr);
            LAUNCH(c, "fas_restrict", 10 * nc8, k_fas4_restrict, dim3(nblk(4 * gc.nc)), dim3(256), g, gc,
                   (const double*)W, (const double*)c->fRm[l], c->fW[l + 1], c->fR[l + 1]);
            fas(c, l + 1, visit_kind(gamma, gi));
            LAUNCH(c, "fas_prolong", 10 * nc8, k_fas4_prolong, dim3(nb), dim3(256), g, gc.nc,
                   (const double*)c->fW[l + 1], (const double*)c->fW0[l + 1], (const double*)W, Walt);
            std::swap(W, Walt);
        }
        for (int i = 0; i < c->nu2; ++i) fas_smooth(c, l, W, Walt);
    }
    if (W != c->fW[l])
        LAUNCH(c, "copy", 8 * nc8, k_copy2, dim3(nblk(4 * g.nc)), dim3(256), (const double*)W, c->fW[l],
               (double*)nullptr, (const double*)nullptr, (double*)nullptr, 4 * (size_t)g.nc);
}

// pseudo step of the current cycle: the host writes a^{-n} to device memory
// (outside any graph), the dtn kernels scale it by each level's 1/dt_p
void set_dtn_factor(miugks_ctx* c) {
    if (!(c->dtn_growth > 0.0)) return;
    double f = std::pow(c->dtn_growth, -(double)c->cycle);
    if (c->dtn_max > 0.0) f = std::fmax(f, 1.0 / c->dtn_max);
    c->h_factor[0] = f;
    (void)hipMemcpyAsync(c->d_factor, c->h_factor, sizeof(double), hipMemcpyHostToDevice, c->stream);
}

void set_dtn(miugks_ctx* c) {
    if (!(c->dtn_growth > 0.0)) return;
    for (int l = 0; l < c->L; ++l)
        LAUNCH(c, "dtn", 2.0 * c->geo[l].nc * 8, k_dtn, dim3(nblk(c->geo[l].nc)), dim3(256), c->geo[l],
               (const double*)c->d_factor, c->dtn_inv[l]);
}

// Step 2 on the device arrays: fW[0] := W^n, fR[0] := R, result into Wt
void predict(miugks_ctx* c) {
    const int top = c->top;
    size_t n = 4 * (size_t)c->geo[top].nc;
    LAUNCH(c, "copy", 24.0 * n, k_copy2, dim3(nblk((int)n)), dim3(256), (const double*)c->W, c->fW[top],
           (double*)nullptr, (const double*)c->R, c->fR[top], n);
    fas(c, top, c->gamma);
    LAUNCH(c, "copy", 16.0 * n, k_copy2, dim3(nblk((int)n)), dim3(256), (const double*)c->fW[top], c->Wt,
           (double*)nullptr, (const double*)nullptr, (double*)nullptr, n);
}

// Steps 2-7 of one cycle
template <typename T>
void cycle_rest(miugks_ctx* c) {
    set_dtn(c);
    predict(c);
    Path<T>::micro_residual(c);
    c->fuse_f = c->no_fuse ? nullptr : c->f;
    c->fused = false;
    Path<T>::correct(c);
    c->fuse_f = nullptr;
    Path<T>::update(c);
}

// capture Step 1 and Steps 2-7 as two graphs (once per context); timing
// runs stay eager because each launch is bracketed by events
// forget the captured graphs (they hold launch arguments by value, such as
// the reference mass); the next run captures them again
void drop_graphs(miugks_ctx* c) {
    if (c->g_step1) (void)hipGraphExecDestroy(c->g_step1);
    if (c->g_rest) (void)hipGraphExecDestroy(c->g_rest);
    c->g_step1 = c->g_rest = nullptr;
}

template <typename T>
int ensure_graphs(miugks_ctx* c) {
    if (c->g_step1 && c->g_rest) return MIUGKS_OK;
    hipGraph_t gr;
    for (int which = 0; which < 2; ++which) {
        hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            c->err = std::string("hipStreamBeginCapture: ") + hipGetErrorString(e);
            return MIUGKS_EDEVICE;
        }
        if (which == 0)
            Path<T>::residual(c);
        else
            cycle_rest<T>(c);
        e = hipStreamEndCapture(c->stream, &gr);
        if (e == hipSuccess) e = hipGraphInstantiate(which == 0 ? &c->g_step1 : &c->g_rest, gr, nullptr, nullptr, 0);
        if (e == hipSuccess) e = hipGraphDestroy(gr);
        if (e != hipSuccess) {
            c->err = std::string("graph capture: ") + hipGetErrorString(e);
            return MIUGKS_EDEVICE;
        }
    }
    return MIUGKS_OK;
}

template <typename T>
int run_cycles(miugks_ctx* c, int max_cycles, double tol, int* done, double* res) {
    int n = 0;
    double last[4] = {0, 0, 0, 0};
    double first_max = -1.0;
    int rc = MIUGKS_ENOTCONVERGED;
    bool graphs = c->use_graphs && !timing(c).on && c->top == 0;
    if (graphs && (rc = ensure_graphs<T>(c))) return rc;
    for (int it = 0; it < max_cycles; ++it) {
        if (graphs) {
            hipError_t ge = hipGraphLaunch(c->g_step1, c->stream);
            if (ge != hipSuccess) {
                c->err = std::string("hipGraphLaunch: ") + hipGetErrorString(ge);
                return MIUGKS_EDEVICE;
            }
        } else {
            Path<T>::residual(c);
        }
        (void)hipMemcpyAsync(c->h_norms, c->norms, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            c->err = std::string("hipStreamSynchronize: ") + hipGetErrorString(e);
            return MIUGKS_EDEVICE;
        }
        if ((rc = check_launch(c))) return rc;
        timing_harvest(c);
        double mx = 0.0;
        bool finite = true;
        for (int m = 0; m < 4; ++m) {
            last[m] = c->h_norms[m];
            finite = finite && std::isfinite(last[m]);
            mx = std::fmax(mx, last[m]);
        }
        if (first_max < 0) first_max = mx;
        if (!finite || mx > 1e6 * std::fmax(first_max, 1e-300)) {
            c->err = "residual diverged";
            rc = MIUGKS_EDIVERGED;
            break;
        }
        if (mx < tol) {
            rc = MIUGKS_OK;
            break;
        }
        set_dtn_factor(c);
        if (graphs) {
            hipError_t ge = hipGraphLaunch(c->g_rest, c->stream);
            if (ge != hipSuccess) {
                c->err = std::string("hipGraphLaunch: ") + hipGetErrorString(ge);
                return MIUGKS_EDEVICE;
            }
        } else {
            cycle_rest<T>(c);
        }
        ++c->cycle;
        ++n;
        rc = MIUGKS_ENOTCONVERGED;
    }
    hipError_t se = hipStreamSynchronize(c->stream);
    if (se != hipSuccess) {
        c->err = std::string("hipStreamSynchronize: ") + hipGetErrorString(se);
        return MIUGKS_EDEVICE;
    }
    if (int e = check_launch(c)) return e;
    timing_harvest(c);
    if (done) *done = n;
    if (res)
        for (int m = 0; m < 4; ++m) res[m] = last[m];
    return rc;
}

// Full-multigrid start (Sec. III C): the state is restricted to the coarsest
// level; each level from there up to level 1 runs the outer cycles as the
// finest level of its own sub-hierarchy, and the distribution it reaches is
// interpolated to the next finer level.  The div buffer is the scratch of
// the transfers (f holds one level at a time, in that level's layout).
template <typename T>
int run_fmg(miugks_ctx* c, int cycles, double tol, int* done) {
    T* f = (T*)c->f;
    T* tmp = (T*)c->div;
    const size_t nk = c->nk;
    for (int l = 0; l + 1 < c->L; ++l) {
        const Geo &g = c->geo[l], &gc = c->geo[l + 1];
        hipLaunchKernelGGL(k_restrict_full<T>, dim3(ntiles(gc.nc), nchunks(c->nk)), dim3(256), 0, c->stream, g, gc,
                           c->vel, (const T*)f, tmp);
        (void)hipMemcpyAsync(f, tmp, 2 * nk * gc.nc * sizeof(T), hipMemcpyDeviceToDevice, c->stream);
    }
    int total = 0, rc = MIUGKS_OK;
    for (int top = c->L - 1; top >= 1; --top) {
        c->top = top;
        c->cycle = 0;
        c->have_div = false;
        Path<T>::moments(c, nullptr);
        int n = 0;
        double res[4];
        rc = run_cycles<T>(c, cycles, tol, &n, res);
        total += n;
        if (rc != MIUGKS_OK && rc != MIUGKS_ENOTCONVERGED) break;
        rc = MIUGKS_OK;
        const Geo& gf = c->geo[top - 1];
        (void)hipMemcpyAsync(tmp, f, 2 * nk * c->geo[top].nc * sizeof(T), hipMemcpyDeviceToDevice, c->stream);
        hipLaunchKernelGGL(k_prolong_full<T>, dim3(ntiles(gf.nc), nchunks(c->nk)), dim3(256), 0, c->stream, gf,
                           c->vel, c->geo[top].nc, (const T*)tmp, f);
    }
    c->top = 0;
    c->cycle = 0;
    c->have_div = false;
    if (done) *done = total;
    if (rc != MIUGKS_OK) return rc;
    Path<T>::moments(c, nullptr);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        c->err = std::string("fmg: ") + hipGetErrorString(e);
        return MIUGKS_EDEVICE;
    }
    return check_launch(c);
}

// Explicit time-accurate UGKS steps (Sec. II A: the scheme whose fluxes the
// residuals use): one global step, the smallest CFL step of the mesh, for
// every cell and face.  Per step: Step 1 with that step, W* = W^n + dt R,
// the Shakhov equilibria of W^n and W* (heat flux q^n), the trapezoidal
// update of f, and the moments of the new f.
template <typename T>
int run_explicit(miugks_ctx* c, int steps, double* res) {
    const Geo g0 = c->geo[0];
    const Geo& g = c->geo[0];
    const double dt = c->dt_global;
    int rc = MIUGKS_OK;
    c->geo[0].dt = c->dt_glob;
    for (int s = 0; s < steps; ++s) {
        Path<T>::residual(c);
        size_t n = 4 * (size_t)g.nc;
        LAUNCH(c, "copy", 16.0 * n, k_copy2, dim3(nblk((int)n)), dim3(256), (const double*)c->W, c->Wtmp,
               (double*)nullptr, (const double*)nullptr, (double*)nullptr, n);
        LAUNCH(c, "cell_prep", (14.0 + NCP) * g.nc * 8, k_cell_prep, dim3(nblk(g.nc)), dim3(256), g, c->gas,
               c->Wtmp, (const double*)c->W, (const double*)c->q, c->cp0, c->tau_tmp);
        LAUNCH(c, "macro_step", 12.0 * n, k_macro_step, dim3(nblk((int)n)), dim3(256), g, (const double*)c->W,
               (const double*)c->R, dt, c->Wt);
        LAUNCH(c, "cell_prep", (14.0 + NCP) * g.nc * 8, k_cell_prep, dim3(nblk(g.nc)), dim3(256), g, c->gas, c->Wt,
               (const double*)c->W, (const double*)c->q, c->cp, c->tau_inv[0]);
        LAUNCH(c, "explicit_update", 3 * Path<T>::arr(c, 0) + 2 * NCP * g.nc * 8.0, k_explicit_update<T>,
               dim3(ntiles(g.nc), nchunks(c->nk)), dim3(256), g, c->vel, c->gas, (T*)c->f, (const T*)c->div,
               (const double*)c->cp0, (const double*)c->cp, dt);
        Path<T>::moments(c, nullptr);
        if (c->renorm) {
            LAUNCH(c, "mass", 4.0 * g.nc * 8, k_mass, dim3(1), dim3(1024), g, c->W, c->mass);
            size_t nf = 2 * (size_t)c->nk * g.nc;
            LAUNCH(c, "scale_f", 2 * Path<T>::arr(c, 0), k_scale_f<T>,
                   dim3(nblk((int)std::min<size_t>(nf, 1 << 24))), dim3(256), (T*)c->f, nf, c->mass, c->M0);
            LAUNCH(c, "scale_moments", 12.0 * g.nc * 8, k_scale_d, dim3(nblk(6 * g.nc)), dim3(256), c->W,
                   4 * (size_t)g.nc, c->mass, c->M0);
            LAUNCH(c, "scale_moments", 4.0 * g.nc * 8, k_scale_d, dim3(nblk(2 * g.nc)), dim3(256), c->q,
                   2 * (size_t)g.nc, c->mass, c->M0);
        }
    }
    c->geo[0] = g0;
    c->have_div = false;
    if (res) {
        hipError_t e = hipMemcpyAsync(c->h_norms, c->norms, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            c->err = std::string("explicit: ") + hipGetErrorString(e);
            return MIUGKS_EDEVICE;
        }
        for (int m = 0; m < 4; ++m) res[m] = c->h_norms[m];
    }
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        c->err = std::string("explicit: ") + hipGetErrorString(e);
        return MIUGKS_EDEVICE;
    }
    if ((rc = check_launch(c))) return rc;
    timing_harvest(c);
    return MIUGKS_OK;
}

int build_device(miugks_ctx* ctx) {
    int rc;
    ctx->geo.resize(ctx->L);
    for (int l = 0; l < ctx->L; ++l) {
        HostLevel& h = ctx->hl[l];
        Geo& g = ctx->geo[l];
        g.nx = h.nx;
        g.ny = h.ny;
        g.nc = h.nc;
        g.n_wall = (int)h.w_cell.size();
        double *xc, *yc, *dx, *dy, *dcent, *dt, *wT, *wU, *wV, *wden, *pw, *winvd, *wvol;
        std::vector<double> hinvd(h.w_cell.size()), hvol(h.w_cell.size());
        for (size_t j = 0; j < h.w_cell.size(); ++j) {
            int cc = h.w_cell[j];
            double ddx = h.dx[cc % h.nx], ddy = h.dy[cc / h.nx];
            hinvd[j] = 1.0 / (h.w_side[j] < 2 ? ddx : ddy);
            hvol[j] = ddx * ddy;
        }
        int *nb, *wc, *ws, *pidx;
        unsigned char* solid;
        if ((rc = upload(ctx, &xc, h.xc)) || (rc = upload(ctx, &yc, h.yc)) || (rc = upload(ctx, &dx, h.dx)) ||
            (rc = upload(ctx, &dy, h.dy)) || (rc = upload(ctx, &dcent, h.dcent)) || (rc = upload(ctx, &dt, h.dt)) ||
            (rc = upload(ctx, &nb, h.nb)) || (rc = upload(ctx, &solid, h.solid)) ||
            (rc = upload(ctx, &wc, h.w_cell)) || (rc = upload(ctx, &ws, h.w_side)) ||
            (rc = upload(ctx, &wT, h.w_T)) || (rc = upload(ctx, &wU, h.w_U)) || (rc = upload(ctx, &wV, h.w_V)) ||
            (rc = upload(ctx, &wden, h.w_den)) || (rc = upload(ctx, &pidx, h.p_idx)) || (rc = upload(ctx, &pw, h.p_w)) ||
            (rc = upload(ctx, &winvd, hinvd)) || (rc = upload(ctx, &wvol, hvol)))
            return rc;
        g.w_invd = winvd;
        g.w_vol = wvol;
        g.xc = xc;
        g.yc = yc;
        g.dx = dx;
        g.dy = dy;
        g.dcent = dcent;
        g.dt = dt;
        g.nb = nb;
        g.solid = solid;
        g.w_cell = wc;
        g.w_side = ws;
        g.w_T = wT;
        g.w_U = wU;
        g.w_V = wV;
        g.w_den = wden;
        g.p_idx = pidx;
        g.p_w = pw;
    }
    // side flags per level, wall-product buffers, sweep variant
    int dev = 0, max_lds = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    ctx->flags.resize(ctx->L);
    ctx->wbuf.resize(ctx->L);
    ctx->wbuf_alt.resize(ctx->L);
    ctx->wdpart.resize(ctx->L);
    ctx->sweep_lds.assign(ctx->L, 0);
    ctx->stype.assign(ctx->L, nullptr);
    ctx->wave.assign(ctx->L, miugks_ctx::WaveCfg());
    ctx->wave1.assign(ctx->L, miugks_ctx::WaveCfg());
    size_t need_max = 0, wave_need_max = 0;
    for (int l = 0; l < ctx->L; ++l) {
        HostLevel& h = ctx->hl[l];
        std::vector<unsigned> fl(h.nc, 0);
        for (int c = 0; c < h.nc; ++c) {
            if (h.solid[c]) {
                fl[c] = FLAG_SOLID;
                continue;
            }
            unsigned f = 0;
            int first_wall = -1;
            for (int s = 0; s < 4; ++s) {
                int code = h.nb[s * h.nc + c];
                // symmetry sides count as zero-ghost sides here; the general
                // sweep adds their mirror ghosts itself
                int t = code >= 0 ? 0
                                  : (code <= NB_WALL0 ? 1 : (code == NB_FARFIELD || code == NB_SYMMETRY ? 2 : 3));
                if (t == 1 && first_wall < 0) first_wall = NB_WALL0 - code;
                f |= (unsigned)(t << (2 * s));
            }
            if (first_wall >= (1 << (32 - FLAG_WALL_SHIFT))) {
                ctx->err = "too many wall sides";
                return MIUGKS_EINVAL;
            }
            if (first_wall > 0) f |= (unsigned)first_wall << FLAG_WALL_SHIFT;
            fl[c] = f;
        }
        unsigned* p;
        if ((rc = upload(ctx, &p, fl))) return rc;
        ctx->flags[l] = p;
        {
            std::vector<unsigned char> st(h.nc);
            // the side predicates of the LDS sweeps: per side s, bit 2s = an
            // interior face (type 0), bit 2s + 1 = not an outflow (type 3)
            for (int c = 0; c < h.nc; ++c) {
                unsigned bits = 0;
                for (int sd = 0; sd < 4; ++sd) {
                    const unsigned t = (fl[c] >> (2 * sd)) & 3u;
                    bits |= (t == 0u ? 1u : 0u) << (2 * sd);
                    bits |= (t != 3u ? 1u : 0u) << (2 * sd + 1);
                }
                st[c] = (unsigned char)bits;
            }
            unsigned char* sp;
            if ((rc = upload(ctx, &sp, st))) return rc;
            ctx->stype[l] = sp;
        }
        void *wb, *wb2;
        if ((rc = dev_alloc(ctx, &wb, std::max<size_t>(1, h.w_cell.size()) * ctx->nk * sizeof(double))) ||
            (rc = dev_alloc(ctx, &wb2, std::max<size_t>(1, h.w_cell.size()) * ctx->nk * sizeof(double))))
            return rc;
        ctx->wbuf[l] = (double*)wb;
        ctx->wbuf_alt[l] = (double*)wb2;
        void* wdp;
        if ((rc = dev_alloc(ctx, &wdp, std::max<size_t>(1, h.w_cell.size()) * wall_density_slices(ctx->nk) *
                                           sizeof(double))))
            return rc;
        ctx->wdpart[l] = (double*)wdp;
        // pipelines per block: as many as fit in LDS and 1024 threads, but
        // no more than needed to cover every item in one round of blocks
        int npad = ((h.ny + 63) / 64) * 64;
        int cus = 256;
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        int best = 0;
        for (int P = 1; P * npad <= 1024; ++P) {
            size_t need = ctx->prec == MIUGKS_FP64 ? sweep_lds_bytes<double>(ctx->geo[l], P)
                                                    : sweep_lds_bytes<float>(ctx->geo[l], P);
            if (need > (size_t)max_lds) break;
            best = P;
            if ((2 * ctx->nk + P - 1) / P <= cus) break;
        }
        if (const char* e = getenv("MIUGKS_SWEEP_P")) best = std::min(best, atoi(e));
        if (best > 0 && !getenv("MIUGKS_NO_LDS_SWEEP")) {
            ctx->sweep_lds[l] = (char)best;
            size_t need = ctx->prec == MIUGKS_FP64 ? sweep_lds_bytes<double>(ctx->geo[l], best)
                                                    : sweep_lds_bytes<float>(ctx->geo[l], best);
            need_max = std::max(need_max, need);
        }
        // wavefront sweep: W wavefronts of I velocities per block, W taken
        // for the fewest rounds of blocks over the chip (ties: smaller W)
        if (!getenv("MIUGKS_NO_WAVE_SWEEP") && h.ny <= 256 && (int)h.w_cell.size() <= SWEEP_WAVE_MAX_WALLS) {
            for (int np = 1; np <= 2; ++np) {
                miugks_ctx::WaveCfg wc;
                wc.I = h.ny <= 32 ? 64 / h.ny : 1;
                wc.R = (h.ny + 63) / 64;
                int nwaves = (ctx->nk + wc.I - 1) / wc.I;
                long best_rounds = 0;
                int force_w = getenv("MIUGKS_WAVE_W") ? atoi(getenv("MIUGKS_WAVE_W")) : 0;
                for (int W : {1, 2, 4}) {
                    if (force_w && W != force_w) continue;
                    size_t need =
                        ctx->prec == MIUGKS_FP64
                            ? sweep_wave_lds_bytes<double>(h.nc, h.nx, (int)h.w_cell.size(), W, wc.I, np)
                            : sweep_wave_lds_bytes<float>(h.nc, h.nx, (int)h.w_cell.size(), W, wc.I, np);
                    if (need > (size_t)max_lds) continue;
                    long per_cu = std::min<long>((long)max_lds / (long)need, 8);
                    long cap = (long)cus * per_cu * W;
                    long rounds = (nwaves + cap - 1) / cap;
                    // ties: more wavefronts per block (fewer blocks, smaller partial sums)
                    if (!wc.W || rounds <= best_rounds) {
                        wc.W = W;
                        wc.lds = need;
                        best_rounds = rounds;
                    }
                }
                // where the tile and the per-cell data do not fit together:
                // the sweep in strips of columns (one velocity per
                // wavefront, a row of the velocity grid per block), the
                // configuration with the most wavefronts per CU (at most 8),
                // then the fewest steps.  Each step is bound by instruction
                // issue, and a narrow strip wastes more lanes on the
                // pipeline's fill and drain, but more wavefronts keep every
                // SIMD busy (measured on the 160-row level: 8 strips of 4
                // wavefronts 4.9 ms per launch, the whole tile at one
                // wavefront per CU 6.7 ms).  Without any strip that fits (or
                // MIUGKS_GC_SWEEP=1): the whole tile, the per-cell data read
                // through the caches.  MIUGKS_SWEEP_STRIPS=n and
                // MIUGKS_STRIP_W=w force a strip count and block width.
                const char* gce = getenv("MIUGKS_GC_SWEEP");
                const bool force_gc = gce && atoi(gce) == 1;
                const char* se2 = getenv("MIUGKS_SWEEP_STRIPS");
                const int force_s = se2 ? atoi(se2) : 0;
                const char* sw2 = getenv("MIUGKS_STRIP_W");
                const int force_sw = sw2 ? atoi(sw2) : 0;
                if ((!wc.W || force_gc) && !(gce && atoi(gce) == 0)) {
                    miugks_ctx::WaveCfg gw = wc;
                    gw.W = 0;
                    gw.gc = true;
                    gw.split = np == 2;
                    gw.I = 1;
                    long best_waves = 0, best_steps = 0;
                    for (int S = 2; S <= 8 && (!force_gc || force_s > 0); ++S) {
                        if (force_s > 0 && S != force_s) continue;
                        const int sw = ctx->prec == MIUGKS_FP64 ? sweep_strip_width<double>(h.nx, S)
                                                                : sweep_strip_width<float>(h.nx, S);
                        if (force_s <= 0 && (S - 1) * sw >= h.nx) continue;   // fewer strips than S
                        long steps = 0;
                        for (int x0 = 0; x0 < h.nx; x0 += sw) steps += std::min(sw, h.nx - x0) + h.ny - 1;
                        for (int W : {4, 2, 1}) {
                            if (force_sw && W != force_sw) continue;
                            size_t need = ctx->prec == MIUGKS_FP64
                                              ? sweep_strip_lds_bytes<double>(h.nx, h.ny, (int)h.w_cell.size(), W, S)
                                              : sweep_strip_lds_bytes<float>(h.nx, h.ny, (int)h.w_cell.size(), W, S);
                            if (need > (size_t)max_lds) continue;
                            long waves = std::min<long>(8, (long)(max_lds / need) * W);
                            if (!gw.W || waves > best_waves || (waves == best_waves && steps < best_steps)) {
                                gw.W = W;
                                gw.lds = need;
                                gw.strips = S;
                                best_waves = waves;
                                best_steps = steps;
                            }
                        }
                    }
                    if (!gw.W && force_s <= 0) {
                        // the whole tile, per-cell data through the caches
                        gw.I = wc.I;
                        const long items = gw.split ? 2L * nwaves : nwaves;
                        long best = 0;
                        for (int W : {1, 2, 4}) {
                            if (force_w && W != force_w) continue;
                            size_t need =
                                ctx->prec == MIUGKS_FP64
                                    ? sweep_wave_lds_bytes<double>(h.nc, h.nx, (int)h.w_cell.size(), W, gw.I, 1, true)
                                    : sweep_wave_lds_bytes<float>(h.nc, h.nx, (int)h.w_cell.size(), W, gw.I, 1, true);
                            if (need > (size_t)max_lds) continue;
                            long per_cu = std::min<long>((long)max_lds / (long)need, 8);
                            long cap = (long)cus * per_cu * W;
                            long rounds = (items + cap - 1) / cap;
                            if (!gw.W || rounds <= best) {
                                gw.W = W;
                                gw.lds = need;
                                best = rounds;
                            }
                        }
                    }
                    if (gw.W) wc = gw;
                }
                // tall levels: the sweep in bands of rows (k_sweep_band, one
                // launch per band), I = 64 / bh velocities per wavefront, one
                // wavefront per block.  Measured on the three workloads: the
                // tallest band whose tile leaves room for at least three
                // blocks per CU in FP32 (two in FP64) is the fastest (a taller
                // band means fewer launches and fewer steps per velocity, but
                // fewer resident wavefronts); levels of at most 64 rows sweep
                // faster as one tile in FP32 (in FP64 from 64 rows the bands
                // win).  MIUGKS_SWEEP_BANDS=0 keeps the forms above, =h forces
                // the band height on every level of more than h rows (forcing
                // strips or the cached whole tile keeps those).
                const char* be = getenv("MIUGKS_SWEEP_BANDS");
                const int force_h = be ? atoi(be) : -1;
                const int band_min_ny = ctx->prec == MIUGKS_FP64 ? 64 : 65;
                if (((h.ny >= band_min_ny && force_h != 0) || (force_h > 0 && force_h <= 64 && h.ny > force_h)) &&
                    !force_gc && force_s <= 0) {
                    miugks_ctx::WaveCfg bw;
                    long best_per_cu = 0;
                    const long want_per_cu = ctx->prec == MIUGKS_FP64 ? 2 : 3;
                    std::vector<int> heights = {32, 21, 16, 13, 12, 10, 8};
                    if (force_h > 0) heights = {force_h};
                    for (int bh : heights) {
                        if (bh >= h.ny) continue;
                        const int I = 64 / bh, nb = (h.ny + bh - 1) / bh;
                        const long wpr = (ctx->nv + I - 1) / I;
                        const int W = force_w ? force_w : 1;
                        size_t need = ctx->prec == MIUGKS_FP64
                                          ? sweep_band_lds_bytes<double>(h.nx, bh, (int)h.w_cell.size(), W, I)
                                          : sweep_band_lds_bytes<float>(h.nx, bh, (int)h.w_cell.size(), W, I);
                        if (need > (size_t)max_lds) continue;
                        const long per_cu = (long)max_lds / (long)need;
                        if (!bw.W || per_cu > best_per_cu) {
                            bw = miugks_ctx::WaveCfg();
                            bw.W = W;
                            bw.I = I;
                            bw.R = 1;
                            bw.gc = true;
                            bw.split = np == 2;
                            bw.bands = nb;
                            bw.bh = bh;
                            bw.lds = need;
                            bw.blocks = (int)((long)ctx->nu * ((wpr + W - 1) / W) * (np == 2 ? 2 : 1));
                            best_per_cu = per_cu;
                        }
                        if (per_cu >= want_per_cu) break;
                    }
                    if (bw.W) wc = bw;
                }
                if (wc.W) {
                    // strips: one row of the velocity grid per block
                    if (!wc.bands)
                        wc.blocks = wc.strips ? ctx->nu * ((ctx->nv + wc.W - 1) / wc.W) * (wc.split ? 2 : 1)
                                              : (nwaves + wc.W - 1) / wc.W * (wc.split ? 2 : 1);
                    (np == 2 ? ctx->wave : ctx->wave1)[l] = wc;
                    wave_need_max = std::max(wave_need_max, wc.lds);
                }
            }
            // both forms or neither
            if (!ctx->wave[l].W || !ctx->wave1[l].W) ctx->wave[l].W = ctx->wave1[l].W = 0;
            // the streamed sweep where the tiles do not fit in LDS (reading
            // rows lane by lane misses the L1 cache, so an LDS tile is faster
            // even at one wavefront per CU; MIUGKS_SWEEP_STREAM=1/0 forces it
            // on/off for every level of more than 32 rows)
            const char* se = getenv("MIUGKS_SWEEP_STREAM");
            if (h.ny > 32 && (!se || atoi(se) != 0)) {
                int sw = getenv("MIUGKS_STREAM_W") ? atoi(getenv("MIUGKS_STREAM_W")) : 4;
                sw = std::max(1, std::min(sw, 8));
                for (int np = 1; np <= 2; ++np) {
                    miugks_ctx::WaveCfg& wc = (np == 2 ? ctx->wave : ctx->wave1)[l];
                    if (!se && wc.W) continue;
                    miugks_ctx::WaveCfg sc;
                    sc.stream = true;
                    sc.W = sw;
                    sc.I = 1;
                    sc.R = (h.ny + 63) / 64;
                    sc.lds = ctx->prec == MIUGKS_FP64
                                 ? sweep_stream_lds_bytes<double>(h.nx, (int)h.w_cell.size(), sw, np)
                                 : sweep_stream_lds_bytes<float>(h.nx, (int)h.w_cell.size(), sw, np);
                    sc.blocks = (ctx->nk + sw - 1) / sw;
                    if (sc.lds > (size_t)max_lds) continue;
                    wc = sc;
                }
                if (!ctx->wave[l].W || !ctx->wave1[l].W) ctx->wave[l].W = ctx->wave1[l].W = 0;
            }
        }
    }
    size_t stream_need_max = 0;
    for (int l = 0; l < ctx->L; ++l) {
        if (ctx->wave[l].stream) stream_need_max = std::max(stream_need_max, ctx->wave[l].lds);
        if (ctx->wave1[l].stream) stream_need_max = std::max(stream_need_max, ctx->wave1[l].lds);
    }
    if (wave_need_max > 65536) {
        hipError_t e = hipSuccess;
        for (int R = 1; R <= 4 && e == hipSuccess; ++R) {
            for (int np = 1; np <= 2 && e == hipSuccess; ++np) e = set_wave_lds(ctx->prec, R, np, (int)wave_need_max);
            if (e == hipSuccess) e = set_strips_lds(ctx->prec, R, (int)wave_need_max);
        }
        if (e == hipSuccess) e = set_band_lds(ctx->prec, (int)wave_need_max);
        if (e != hipSuccess)
            for (int l = 0; l < ctx->L; ++l)
                if ((!ctx->wave[l].stream && ctx->wave[l].lds > 65536) ||
                    (!ctx->wave1[l].stream && ctx->wave1[l].lds > 65536))
                    ctx->wave[l].W = ctx->wave1[l].W = 0;
    }
    if (stream_need_max > 65536) {
        hipError_t e = hipSuccess;
        for (int R = 1; R <= 4 && e == hipSuccess; ++R)
            for (int np = 1; np <= 2 && e == hipSuccess; ++np)
                e = set_stream_lds(ctx->prec, R, np, (int)stream_need_max);
        if (e != hipSuccess)
            for (int l = 0; l < ctx->L; ++l)
                if ((ctx->wave[l].stream && ctx->wave[l].lds > 65536) ||
                    (ctx->wave1[l].stream && ctx->wave1[l].lds > 65536))
                    ctx->wave[l].W = ctx->wave1[l].W = 0;
    }
    if (need_max > 65536) {
        hipError_t e = ctx->prec == MIUGKS_FP64 ? raise_lds_limit((const void*)k_sweep_lds<double>, (int)need_max)
                                                : raise_lds_limit((const void*)k_sweep_lds<float>, (int)need_max);
        if (e != hipSuccess)
            for (int l = 0; l < ctx->L; ++l)
                if (ctx->sweep_lds[l] &&
                    (ctx->prec == MIUGKS_FP64 ? sweep_lds_bytes<double>(ctx->geo[l], ctx->sweep_lds[l])
                                              : sweep_lds_bytes<float>(ctx->geo[l], ctx->sweep_lds[l])) > 65536)
                    ctx->sweep_lds[l] = 0;
    }
    if (ctx->has_sym)   // the mirror ghosts are read by the general sweep only
        for (int l = 0; l < ctx->L; ++l) {
            ctx->wave[l].W = ctx->wave1[l].W = 0;
            ctx->sweep_lds[l] = 0;
        }
    if (getenv("MIUGKS_DEBUG"))
        for (int l = 0; l < ctx->L; ++l)
            fprintf(stderr,
                    "[miugks] level %d: %dx%d cells, %d wall sides, sweep: %s (wavefronts/block %d, velocities/"
                    "wavefront %d, rows/lane %d, blocks %d, LDS %zu; pipelines/block %d)\n",
                    l, ctx->hl[l].nx, ctx->hl[l].ny, (int)ctx->hl[l].w_cell.size(),
                    ctx->wave[l].W ? (ctx->wave[l].stream ? "streamed wavefront" : "wavefront")
                                   : (ctx->sweep_lds[l] ? "LDS pipelines" : "global memory"),
                    ctx->wave[l].W, ctx->wave[l].I, ctx->wave[l].R, ctx->wave[l].blocks, ctx->wave[l].lds,
                    (int)ctx->sweep_lds[l]);
    {
        void* df;
        if ((rc = dev_alloc(ctx, &df, sizeof(double)))) return rc;
        ctx->d_factor = (double*)df;
        HIP_TRY(hipMemset(ctx->d_factor, 0, sizeof(double)));
        HIP_TRY(hipHostMalloc((void**)&ctx->h_factor, sizeof(double), hipHostMallocDefault));
    }
    // velocities
    std::vector<float> uf(ctx->hv.u.begin(), ctx->hv.u.end()), vf(ctx->hv.v.begin(), ctx->hv.v.end()),
        wf(ctx->hv.w.begin(), ctx->hv.w.end());
    double *u, *v, *w;
    float *uu, *vv, *ww;
    int *mxd, *myd;
    if ((rc = upload(ctx, &u, ctx->hv.u)) || (rc = upload(ctx, &v, ctx->hv.v)) || (rc = upload(ctx, &w, ctx->hv.w)) ||
        (rc = upload(ctx, &uu, uf)) || (rc = upload(ctx, &vv, vf)) || (rc = upload(ctx, &ww, wf)) ||
        (rc = upload(ctx, &mxd, ctx->hv.mx)) || (rc = upload(ctx, &myd, ctx->hv.my)))
        return rc;
    ctx->vel.mx = mxd;
    ctx->vel.my = myd;
    ctx->vel.nk = ctx->nk;
    ctx->vel.u = u;
    ctx->vel.v = v;
    ctx->vel.w = w;
    ctx->vel.uf = uu;
    ctx->vel.vf = vv;
    ctx->vel.wf = ww;
    // freestream distribution (farfield faces)
    {
        int nk = ctx->nk;
        std::vector<double> fi(2 * nk);
        double lam = ctx->gas.lam_inf;
        for (int k = 0; k < nk; ++k) {
            double du = ctx->hv.u[k] - ctx->gas.U_inf, dv = ctx->hv.v[k] - ctx->gas.V_inf;
            fi[k] = ctx->gas.rho_inf * lam / M_PI * std::exp(-lam * (du * du + dv * dv));
            fi[nk + k] = ctx->gas.K_int / (2.0 * lam) * fi[k];
        }
        if (ctx->prec == MIUGKS_FP64) {
            double* p;
            if ((rc = upload(ctx, &p, fi))) return rc;
            ctx->finf = p;
        } else {
            std::vector<float> ff(fi.begin(), fi.end());
            float* p;
            if ((rc = upload(ctx, &p, ff))) return rc;
            ctx->finf = p;
        }
    }
    size_t nc0 = ctx->hl[0].nc, nk = ctx->nk, es = ctx->esize;
    size_t fbytes = 2 * nk * nc0 * es;
    if ((rc = dev_alloc(ctx, &ctx->f, fbytes)) || (rc = dev_alloc(ctx, &ctx->div, fbytes))) return rc;
    void* p;
    auto dalloc = [&](double** d, size_t n) -> int {
        int r2 = dev_alloc(ctx, &p, n * sizeof(double));
        *d = (double*)p;
        return r2;
    };
    if ((rc = dalloc(&ctx->W, 4 * nc0)) || (rc = dalloc(&ctx->q, 2 * nc0)) || (rc = dalloc(&ctx->R, 4 * nc0)) ||
        (rc = dalloc(&ctx->Wt, 4 * nc0)) || (rc = dalloc(&ctx->fp, NFP * 2 * nc0)) ||
        (rc = dalloc(&ctx->cp, NCP * nc0)) || (rc = dalloc(&ctx->norms, 4)) ||
        (rc = dalloc(&ctx->cp0, NCP * nc0)) || (rc = dalloc(&ctx->dt_glob, nc0)) ||
        (rc = dalloc(&ctx->Wtmp, 4 * nc0)) || (rc = dalloc(&ctx->tau_tmp, nc0)) ||
        (rc = dalloc(&ctx->rho_w, ctx->hl[0].w_cell.size() + 1)) || (rc = dalloc(&ctx->mass, 1)) ||
        (rc = dalloc(&ctx->loads, 4 * ctx->hl[0].w_cell.size() + 1)) ||
        (rc = dalloc(&ctx->msum, 2 * NRAW * nc0)))
        return rc;
    {
        // the global explicit step: the smallest CFL step of the finest level
        const std::vector<double>& dt0 = ctx->hl[0].dt;
        double m = dt0.empty() ? 0.0 : *std::min_element(dt0.begin(), dt0.end());
        ctx->dt_global = m;
        std::vector<double> all(nc0, m);
        HIP_TRY(hipMemcpy(ctx->dt_glob, all.data(), nc0 * sizeof(double), hipMemcpyHostToDevice));
    }
    if (const char* e = getenv("MIUGKS_CHUNK_LEN")) ctx->kch_force = std::max(KCH, atoi(e));
    ctx->no_fuse = getenv("MIUGKS_NO_FUSED_UPDATE") != nullptr;
    ctx->wall_sliced = getenv("MIUGKS_WALL_SLICED") != nullptr;
    if (const char* e = getenv("MIUGKS_FLUX_MK")) ctx->flux_mk_force = atoi(e);
    // partial sums: the largest is 2 * NRAW per cell per chunk of KCH (the shortest)
    size_t maxw = 1;
    for (auto& h : ctx->hl) maxw = std::max(maxw, h.w_cell.size());
    ctx->part_bytes = (size_t)nchunks(ctx->nk) * std::max<size_t>(2 * NRAW * nc0, maxw) * sizeof(double);
    if ((rc = dev_alloc(ctx, &p, ctx->part_bytes))) return rc;
    ctx->part = (double*)p;
    ctx->r.resize(ctx->L);
    ctx->df.resize(ctx->L);
    ctx->msnap.assign(ctx->L, nullptr);
    for (auto* v2 : {&ctx->tau_inv, &ctx->dtn_inv, &ctx->drho, &ctx->fW, &ctx->fW0, &ctx->fR, &ctx->fP, &ctx->fE,
                     &ctx->fGam, &ctx->fRm, &ctx->fW2})
        v2->resize(ctx->L);
    for (int l = 0; l < ctx->L; ++l) {
        size_t nc = ctx->hl[l].nc;
        if ((rc = dev_alloc(ctx, &ctx->r[l], 2 * nk * nc * es)) || (rc = dev_alloc(ctx, &ctx->df[l], 2 * nk * nc * es)))
            return rc;
        if (ctx->has_sym && (rc = dev_alloc(ctx, &ctx->msnap[l], 2 * nk * nc * es))) return rc;
        if ((rc = dalloc(&ctx->tau_inv[l], nc)) || (rc = dalloc(&ctx->dtn_inv[l], nc)) ||
            (rc = dalloc(&ctx->drho[l], ctx->hl[l].w_cell.size() + 1)) || (rc = dalloc(&ctx->fW[l], 4 * nc)) ||
            (rc = dalloc(&ctx->fW0[l], 4 * nc)) || (rc = dalloc(&ctx->fR[l], 4 * nc)) ||
            (rc = dalloc(&ctx->fP[l], 4 * nc)) || (rc = dalloc(&ctx->fE[l], 4 * nc)) ||
            (rc = dalloc(&ctx->fGam[l], 4 * nc)) || (rc = dalloc(&ctx->fRm[l], 4 * nc)) ||
            (rc = dalloc(&ctx->fW2[l], 4 * nc)))
            return rc;
        HIP_TRY(hipMemset(ctx->fE[l], 0, 4 * nc * sizeof(double)));
        HIP_TRY(hipMemset(ctx->dtn_inv[l], 0, nc * sizeof(double)));
    }
    ctx->cwall.assign(ctx->L, nullptr);
    ctx->civol.assign(ctx->L, nullptr);
    ctx->ddrho.assign(ctx->L, nullptr);
    ctx->last_from_zero.assign(ctx->L, 0);
    for (int l = 0; l < ctx->L; ++l) {
        const HostLevel& h = ctx->hl[l];
        if ((rc = dalloc(&ctx->ddrho[l], h.w_cell.size() + 1))) return rc;
        if (l == 0) continue;
        // coarse level l, fine level l - 1
        const HostLevel& f = ctx->hl[l - 1];
        std::vector<int> first(f.nc + 1, 0);
        for (size_t j = 0; j < f.w_cell.size(); ++j) first[f.w_cell[j] + 1] += 1;
        for (int c = 0; c < f.nc; ++c) first[c + 1] += first[c];
        std::vector<int4> cw(h.nc);
        std::vector<double> iv(h.nc);
        for (int J = 0; J < h.ny; ++J)
            for (int I = 0; I < h.nx; ++I) {
                int C = J * h.nx + I, c0 = (2 * J) * f.nx + 2 * I, c1 = (2 * J + 1) * f.nx + 2 * I;
                cw[C] = make_int4(first[c0], first[c0 + 2], first[c1], first[c1 + 2]);
                double vol = 0.0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) {
                        int c = (2 * J + a) * f.nx + 2 * I + b;
                        if (!f.solid[c]) vol += f.dx[c % f.nx] * f.dy[c / f.nx];
                    }
                iv[C] = vol > 0.0 ? 1.0 / vol : 0.0;
            }
        int4* cwp;
        double* ivp;
        if ((rc = upload(ctx, &cwp, cw)) || (rc = upload(ctx, &ivp, iv))) return rc;
        ctx->cwall[l] = cwp;
        ctx->civol[l] = ivp;
    }
    ctx->wparts.assign(ctx->L, ctx->nk);
    ctx->coefT.assign(ctx->L, nullptr);
    ctx->coefset.L = std::min(ctx->L, FAS_MAXL);
    for (int l = 0; l < ctx->L; ++l) {
        if ((rc = dev_alloc(ctx, &ctx->coefT[l], ctx->hl[l].nc * es))) return rc;
        if (l < FAS_MAXL) {
            ctx->coefset.nc[l] = ctx->hl[l].nc;
            ctx->coefset.solid[l] = ctx->geo[l].solid;
            ctx->coefset.tau[l] = ctx->tau_inv[l];
            ctx->coefset.dtn[l] = ctx->dtn_inv[l];
            ctx->coefset.out[l] = ctx->coefT[l];
        } else {
            ctx->wave[l].W = 0;
        }
    }
    // FAS in one workgroup for the trailing levels of at most this many cells
    {
        int lim = 256;
        if (const char* e = getenv("MIUGKS_FAS_BLOCK_CELLS")) lim = atoi(e);
        // the levels it takes must also fit in LDS
        int max_lds = 65536;
        (void)hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device);
        ctx->fas_block_lds.assign(ctx->L, 0);
        size_t acc = 0;
        if (ctx->FL <= FAS_MAXL)
            for (int l = ctx->FL - 1; l >= 0 && ctx->hl[l].nc <= lim; --l) {
                size_t need = acc + fas_level_lds_bytes(ctx->hl[l].nx, ctx->hl[l].ny);
                if (need + sizeof(FasSet) + 1024 > (size_t)max_lds) break;   // static LDS beside it
                acc = need;
                ctx->fas_block_lds[l] = acc;
                ctx->fas_block_l0 = l;
            }
        if (acc > 65536 && raise_lds_limit((const void*)k_fas_cycle_block, (int)acc) != hipSuccess)
            for (int l = 0; l < ctx->L; ++l)
                if (ctx->fas_block_lds[l] > 65536) ctx->fas_block_l0 = std::max(ctx->fas_block_l0, l + 1);
        FasSet& F = ctx->fasset;
        F.L = ctx->FL;
        F.nu1 = ctx->nu1;
        F.nu2 = ctx->nu2;
        F.nuc = ctx->nuc;
        for (int l = 0; l < ctx->L && l < FAS_MAXL; ++l) {
            F.geo[l] = ctx->geo[l];
            F.W[l] = ctx->fW[l];
            F.W0[l] = ctx->fW0[l];
            F.R[l] = ctx->fR[l];
            F.P[l] = ctx->fP[l];
            F.E[l] = ctx->fE[l];
            F.Gam[l] = ctx->fGam[l];
            F.Rm[l] = ctx->fRm[l];
            F.dtn[l] = ctx->dtn_inv[l];
            F.W2[l] = ctx->fW2[l];
        }
    }
    HIP_TRY(hipHostMalloc((void**)&ctx->h_norms, 4 * sizeof(double), hipHostMallocDefault));
    return MIUGKS_OK;
}

template <typename T>
void init_f(miugks_ctx* c, const double* dprim) {
    const Geo& g = c->geo[0];
    hipLaunchKernelGGL(k_init<T>, dim3(ntiles(g.nc), nchunks(c->nk)), dim3(256), 0, c->stream, g, c->vel, c->gas,
                       dprim, (T*)c->f);
    Path<T>::moments(c, nullptr);
}

int reset_mass(miugks_ctx* c) {
    hipLaunchKernelGGL(k_mass, dim3(1), dim3(1024), 0, c->stream, c->geo[c->top], c->W, c->mass);
    double m = 0;
    hipError_t e = hipMemcpyAsync(&m, c->mass, sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        c->err = std::string("mass: ") + hipGetErrorString(e);
        return MIUGKS_EDEVICE;
    }
    c->M0 = m;
    drop_graphs(c);   // the renormalisation kernels take M0 by value
    return MIUGKS_OK;
}

// copy a distribution-shaped device array out / in with conversion
int copy_out(miugks_ctx* ctx, const void* src, void* dst, int dtype, int on_device) {
    size_t n = 2 * (size_t)ctx->nk * ctx->hl[0].nc;
    size_t des = dtype == MIUGKS_FP64 ? 8 : 4;
    if (dtype != MIUGKS_FP64 && dtype != MIUGKS_FP32F) {
        ctx->err = "dtype must be MIUGKS_FP64 or MIUGKS_FP32F";
        return MIUGKS_EINVAL;
    }
    if (!dst) {
        ctx->err = "null destination";
        return MIUGKS_EINVAL;
    }
    void* tmp = nullptr;
    void* target = dst;
    if (!on_device) {
        if (int r = raw_alloc(ctx, &tmp, n * des)) return r;
        target = tmp;
    }
    if (dtype == ctx->prec) {
        hipMemcpyAsync(target, src, n * des, hipMemcpyDeviceToDevice, ctx->stream);
    } else if (ctx->prec == MIUGKS_FP64) {
        hipLaunchKernelGGL((k_convert<double, float>), dim3(1024), dim3(256), 0, ctx->stream, (const double*)src,
                           (float*)target, n);
    } else {
        hipLaunchKernelGGL((k_convert<float, double>), dim3(1024), dim3(256), 0, ctx->stream, (const float*)src,
                           (double*)target, n);
    }
    if (!on_device) hipMemcpyAsync(dst, tmp, n * des, hipMemcpyDeviceToHost, ctx->stream);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    raw_free(ctx, tmp);
    if (e != hipSuccess) {
        ctx->err = std::string("copy: ") + hipGetErrorString(e);
        return MIUGKS_EDEVICE;
    }
    return check_launch(ctx);
}

int copy_in(miugks_ctx* ctx, const void* src, void* dst, int dtype, int on_device) {
    size_t n = 2 * (size_t)ctx->nk * ctx->hl[0].nc;
    size_t des = dtype == MIUGKS_FP64 ? 8 : 4;
    if (dtype != MIUGKS_FP64 && dtype != MIUGKS_FP32F) {
        ctx->err = "dtype must be MIUGKS_FP64 or MIUGKS_FP32F";
        return MIUGKS_EINVAL;
    }
    if (!src) {
        ctx->err = "null source";
        return MIUGKS_EINVAL;
    }
    void* tmp = nullptr;
    const void* from = src;
    if (!on_device) {
        if (int r = raw_alloc(ctx, &tmp, n * des)) return r;
        hipMemcpyAsync(tmp, src, n * des, hipMemcpyHostToDevice, ctx->stream);
        from = tmp;
    }
    if (dtype == ctx->prec) {
        hipMemcpyAsync(dst, from, n * des, hipMemcpyDeviceToDevice, ctx->stream);
    } else if (ctx->prec == MIUGKS_FP64) {
        hipLaunchKernelGGL((k_convert<float, double>), dim3(1024), dim3(256), 0, ctx->stream, (const float*)from,
                           (double*)dst, n);
    } else {
        hipLaunchKernelGGL((k_convert<double, float>), dim3(1024), dim3(256), 0, ctx->stream, (const double*)from,
                           (float*)dst, n);
    }
    hipError_t e = hipStreamSynchronize(ctx->stream);
    raw_free(ctx, tmp);
    if (e != hipSuccess) {
        ctx->err = std::string("copy: ") + hipGetErrorString(e);
        return MIUGKS_EDEVICE;
    }
    return check_launch(ctx);
}

int upload_cells(miugks_ctx* ctx, double* dst, const double* src, int m) {
    if (!src) {
        ctx->err = "null input";
        return MIUGKS_EINVAL;
    }
    HIP_TRY(hipMemcpyAsync(dst, src, (size_t)m * ctx->hl[0].nc * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    return MIUGKS_OK;
}

int download_cells(miugks_ctx* ctx, double* dst, const double* src, int m) {
    HIP_TRY(hipMemcpyAsync(dst, src, (size_t)m * ctx->hl[0].nc * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return check_launch(ctx);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

int miugks_quadrature(int kind, int n, double lo, double hi, double* nodes, double* weights) {
    return quadrature_rule(kind, n, lo, hi, nodes, weights) ? MIUGKS_OK : MIUGKS_EINVAL;
}

const char* miugks_last_error(const miugks_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

void miugks_destroy(miugks_ctx* ctx) {
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->timing) {
        timing_harvest(ctx);
        for (hipEvent_t e : ctx->timing->pool) (void)hipEventDestroy(e);
        delete ctx->timing;
    }
    if (ctx->g_step1) (void)hipGraphExecDestroy(ctx->g_step1);
    if (ctx->g_rest) (void)hipGraphExecDestroy(ctx->g_rest);
    for (void* p : ctx->allocs) raw_free(ctx, p);
    if (ctx->h_norms) (void)hipHostFree(ctx->h_norms);
    if (ctx->h_factor) (void)hipHostFree(ctx->h_factor);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

int miugks_set_allocator(miugks_alloc_fn alloc, miugks_free_fn free_fn, void* user) {
    if ((alloc == nullptr) != (free_fn == nullptr)) return MIUGKS_EINVAL;
    g_alloc = alloc;
    g_free = free_fn;
    g_alloc_user = user;
    return MIUGKS_OK;
}

int miugks_create(miugks_ctx** out, const miugks_mesh_desc* m, const miugks_vgrid_desc* v, const miugks_gas_desc* g,
                  const miugks_solver_desc* s, void* hip_stream) {
    g_create_error.clear();
    if (!out || !m || !v || !g || !s) {
        g_create_error = "null argument";
        return MIUGKS_EINVAL;
    }
    *out = nullptr;
    miugks_ctx* ctx = new (std::nothrow) miugks_ctx();
    if (!ctx) {
        g_create_error = "out of host memory";
        return MIUGKS_ENOMEM;
    }
    ctx->stream = (hipStream_t)hip_stream;
    ctx->alloc = g_alloc;
    ctx->free_fn = g_free;
    ctx->alloc_user = g_alloc_user;
    ctx->use_graphs = getenv("MIUGKS_NO_GRAPH") == nullptr;
    if (s->precision != MIUGKS_FP64 && s->precision != MIUGKS_FP32F) {
        g_create_error = "precision must be MIUGKS_FP64 or MIUGKS_FP32F";
        delete ctx;
        return MIUGKS_EINVAL;
    }
    if (v->nu < 1 || v->nv < 1 || !v->u || !v->v || !v->wu || !v->wv || s->nu1 < 0 || s->nu2 < 0 ||
        s->nu_coarse < 1 || s->nu_coarse_cs < 0 || s->fas_levels < 0 || s->cycle_gamma < MIUGKS_CYCLE_F ||
        s->cycle_gamma > 3 || s->cycle_gamma_cs < MIUGKS_CYCLE_F || s->cycle_gamma_cs > 3 ||
        !(s->cfl > 0) || !(s->dtn_max >= 0) || g->K_int < 0 || !(g->Kn > 0) || !(g->T_inf > 0)) {
        g_create_error = "bad velocity grid, gas or solver description";
        delete ctx;
        return MIUGKS_EINVAL;
    }
    if (m->ny > 1024) {
        g_create_error = "ny > 1024 is not supported by the ordered sweep";
        delete ctx;
        return MIUGKS_EINVAL;
    }
    // the interface flux addresses a velocity chunk's rows with 32-bit byte offsets
    if (m->nx < 1 || m->ny < 1 || (size_t)m->nx * m->ny * miugks::KCH * sizeof(double) >= (size_t(1) << 31)) {
        g_create_error = "mesh too large: nx * ny must stay below 2^23 cells";
        delete ctx;
        return MIUGKS_EINVAL;
    }
    ctx->prec = s->precision;
    ctx->esize = s->precision == MIUGKS_FP64 ? 8 : 4;
    ctx->nu = v->nu;
    ctx->nv = v->nv;
    ctx->nk = v->nu * v->nv;
    ctx->L = m->n_levels;
    ctx->FL = s->fas_levels > 0 ? std::min(s->fas_levels, m->n_levels) : m->n_levels;
    ctx->nu1 = s->nu1;
    ctx->nu2 = s->nu2;
    ctx->nuc = s->nu_coarse;
    ctx->nuc_cs = s->nu_coarse_cs > 0 ? s->nu_coarse_cs : s->nu_coarse;
    ctx->gamma = s->cycle_gamma != 0 ? s->cycle_gamma : 1;
    ctx->gamma_cs = s->cycle_gamma_cs != 0 ? s->cycle_gamma_cs : ctx->gamma;
    ctx->dtn_growth = s->dtn_growth;
    ctx->dtn_max = s->dtn_max;
    ctx->cfl = s->cfl;
    HostVel& hv = ctx->hv;
    hv.nu = v->nu;
    hv.nv = v->nv;
    hv.nk = ctx->nk;
    hv.u.resize(hv.nk);
    hv.v.resize(hv.nk);
    hv.w.resize(hv.nk);
    for (int a = 0; a < v->nu; ++a)
        for (int b = 0; b < v->nv; ++b) {
            int k = a * v->nv + b;
            hv.u[k] = v->u[a];
            hv.v[k] = v->v[b];
            hv.w[k] = v->wu[a] * v->wv[b];
        }
    for (int a = 0; a < v->nu; ++a) hv.umax = std::fmax(hv.umax, std::fabs(v->u[a]));
    for (int b = 0; b < v->nv; ++b) hv.vmax = std::fmax(hv.vmax, std::fabs(v->v[b]));
    // mirror velocities of the symmetry faces (-1 where the grid lacks the reversed node)
    {
        bool symu = true, symv = true;
        for (int a = 0; a < v->nu; ++a)
            symu = symu && std::fabs(v->u[v->nu - 1 - a] + v->u[a]) <= 1e-12 * std::fmax(1.0, hv.umax);
        for (int b = 0; b < v->nv; ++b)
            symv = symv && std::fabs(v->v[v->nv - 1 - b] + v->v[b]) <= 1e-12 * std::fmax(1.0, hv.vmax);
        hv.mx.assign(hv.nk, -1);
        hv.my.assign(hv.nk, -1);
        for (int a = 0; a < v->nu; ++a)
            for (int b = 0; b < v->nv; ++b) {
                if (symu) hv.mx[a * v->nv + b] = (v->nu - 1 - a) * v->nv + b;
                if (symv) hv.my[a * v->nv + b] = a * v->nv + (v->nv - 1 - b);
            }
        bool symx = false, symy = false;
        for (int i = 0; i < (m->nx + 1) * m->ny; ++i) symx = symx || m->face_type_x[i] == MIUGKS_FACE_SYMMETRY;
        for (int i = 0; i < m->nx * (m->ny + 1); ++i) symy = symy || m->face_type_y[i] == MIUGKS_FACE_SYMMETRY;
        if ((symx && !symu) || (symy && !symv)) {
            g_create_error = "symmetry faces need a velocity grid symmetric in the normal component";
            delete ctx;
            return MIUGKS_EINVAL;
        }
        ctx->has_sym = symx || symy;
    }
    // gas constants; mu_ref from the VHS mean free path (alpha = 1)
    Gas& gas = ctx->gas;
    gas.K_int = g->K_int;
    gas.K = g->K_int + 2.0;
    gas.gamma = (gas.K + 2.0) / gas.K;
    gas.Pr = g->Pr;
    gas.omega = g->omega;
    gas.mu_ref = 15.0 * std::sqrt(M_PI) * g->Kn / (2.0 * (5.0 - 2.0 * g->omega) * (7.0 - 2.0 * g->omega));
    gas.rho_inf = g->rho_inf;
    gas.U_inf = g->U_inf;
    gas.V_inf = g->V_inf;
    gas.lam_inf = 1.0 / g->T_inf;
    gas.W_inf[0] = g->rho_inf;
    gas.W_inf[1] = g->rho_inf * g->U_inf;
    gas.W_inf[2] = g->rho_inf * g->V_inf;
    gas.W_inf[3] = 0.5 * g->rho_inf * (g->U_inf * g->U_inf + g->V_inf * g->V_inf) +
                   gas.K * g->rho_inf * g->T_inf / 4.0;
    std::string err;
    if (!build_levels(m->nx, m->ny, m->n_levels, m->x, m->y, m->face_type_x, m->face_type_y, m->wall_x, m->wall_y,
                      m->solid, hv, s->cfl, ctx->hl, err)) {
        g_create_error = err;
        delete ctx;
        return MIUGKS_EINVAL;
    }
    bool closed = true;
    for (auto t : ctx->hl[0].ftx) closed = closed && t != MIUGKS_FACE_FARFIELD && t != MIUGKS_FACE_OUTFLOW;
    for (auto t : ctx->hl[0].fty) closed = closed && t != MIUGKS_FACE_FARFIELD && t != MIUGKS_FACE_OUTFLOW;
    ctx->renorm = s->mass_renorm < 0 ? closed : s->mass_renorm != 0;
    (void)hipGetDevice(&ctx->device);
    {
        std::string serr;
        if (int src = scratch_address(ctx->device, &ctx->scratch, serr)) {
            g_create_error = serr;
            delete ctx;
            return src;
        }
    }
    if (!ctx->stream) {
        // the legacy default stream cannot be captured into graphs
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            g_create_error = "hipStreamCreateWithFlags failed";
            delete ctx;
            return MIUGKS_EDEVICE;
        }
        ctx->own_stream = true;
    }
    int rc = build_device(ctx);
    if (rc) {
        g_create_error = ctx->err;
        miugks_destroy(ctx);
        return rc;
    }
    // start from the rest state
    size_t nc = ctx->hl[0].nc;
    std::vector<double> prim(4 * nc, 0.0);
    for (size_t c = 0; c < nc; ++c) {
        prim[c] = 1.0;
        prim[3 * nc + c] = 1.0;
    }
    rc = miugks_init_macro(ctx, prim.data(), prim.data() + nc, prim.data() + 2 * nc, prim.data() + 3 * nc);
    if (rc) {
        g_create_error = ctx->err;
        miugks_destroy(ctx);
        return rc;
    }
    *out = ctx;
    return MIUGKS_OK;
}

int miugks_init_macro(miugks_ctx* ctx, const double* rho, const double* U, const double* V, const double* T) {
    if (!ctx) return MIUGKS_EINVAL;
    if (!rho || !U || !V || !T) {
        ctx->err = "null field";
        return MIUGKS_EINVAL;
    }
    size_t nc = ctx->hl[0].nc;
    for (size_t c = 0; c < nc; ++c)
        if (!ctx->hl[0].solid[c] && !(rho[c] > 0 && T[c] > 0)) {
            ctx->err = "density and temperature must be positive";
            return MIUGKS_EINVAL;
        }
    std::vector<double> prim(4 * nc);
    std::memcpy(prim.data(), rho, nc * 8);
    std::memcpy(prim.data() + nc, U, nc * 8);
    std::memcpy(prim.data() + 2 * nc, V, nc * 8);
    std::memcpy(prim.data() + 3 * nc, T, nc * 8);
    for (size_t c = 0; c < nc; ++c)
        if (ctx->hl[0].solid[c]) prim[3 * nc + c] = 1.0;
    HIP_TRY(hipMemcpy(ctx->Wt, prim.data(), 4 * nc * sizeof(double), hipMemcpyHostToDevice));
    ctx->top = 0;
    if (ctx->prec == MIUGKS_FP64)
        init_f<double>(ctx, ctx->Wt);
    else
        init_f<float>(ctx, ctx->Wt);
    ctx->cycle = 0;
    ctx->have_div = false;
    return reset_mass(ctx);
}

int miugks_explicit(miugks_ctx* ctx, int steps, double* dt, double res[4]) {
    if (!ctx) return MIUGKS_EINVAL;
    if (steps < 0) {
        ctx->err = "steps must be >= 0";
        return MIUGKS_EINVAL;
    }
    if (ctx->top != 0) {
        ctx->err = "the state is not on the finest level";
        return MIUGKS_ESTATE;
    }
    if (dt) *dt = ctx->dt_global;
    if (ctx->prec == MIUGKS_FP64) return run_explicit<double>(ctx, steps, res);
    return run_explicit<float>(ctx, steps, res);
}

int miugks_fmg(miugks_ctx* ctx, int cycles_per_level, double tol, int* cycles_done) {
    if (!ctx) return MIUGKS_EINVAL;
    if (cycles_per_level < 0) {
        ctx->err = "cycles_per_level must be >= 0";
        return MIUGKS_EINVAL;
    }
    if (ctx->prec == MIUGKS_FP64) return run_fmg<double>(ctx, cycles_per_level, tol, cycles_done);
    return run_fmg<float>(ctx, cycles_per_level, tol, cycles_done);
}

int miugks_iterate(miugks_ctx* ctx, int max_cycles, double tol, int* cycles_done, double res[4]) {
    if (!ctx) return MIUGKS_EINVAL;
    if (max_cycles < 0) {
        ctx->err = "max_cycles must be >= 0";
        return MIUGKS_EINVAL;
    }
    if (ctx->prec == MIUGKS_FP64) return run_cycles<double>(ctx, max_cycles, tol, cycles_done, res);
    return run_cycles<float>(ctx, max_cycles, tol, cycles_done, res);
}

int miugks_get_macro(miugks_ctx* ctx, double* rho, double* U, double* V, double* T, double* qx, double* qy) {
    if (!ctx) return MIUGKS_EINVAL;
    size_t nc = ctx->hl[0].nc;
    std::vector<double> W(4 * nc), q(2 * nc);
    int rc = download_cells(ctx, W.data(), ctx->W, 4);
    if (rc) return rc;
    if ((rc = download_cells(ctx, q.data(), ctx->q, 2))) return rc;
    double K = ctx->gas.K;
    for (size_t c = 0; c < nc; ++c) {
        double r = W[c], u = 0, v = 0, t = 0;
        if (r != 0.0) {
            u = W[nc + c] / r;
            v = W[2 * nc + c] / r;
            double e = W[3 * nc + c] - 0.5 * r * (u * u + v * v);
            t = 4.0 * e / (K * r);
        }
        if (rho) rho[c] = r;
        if (U) U[c] = u;
        if (V) V[c] = v;
        if (T) T[c] = t;
        if (qx) qx[c] = q[c];
        if (qy) qy[c] = q[nc + c];
    }
    return MIUGKS_OK;
}

int miugks_wall_list(miugks_ctx* ctx, int* cell, int* side, int* n_walls) {
    if (!ctx || !n_walls) return MIUGKS_EINVAL;
    const HostLevel& h = ctx->hl[0];
    *n_walls = (int)h.w_cell.size();
    for (size_t j = 0; j < h.w_cell.size(); ++j) {
        if (cell) cell[j] = h.w_cell[j];
        if (side) side[j] = h.w_side[j];
    }
    return MIUGKS_OK;
}

// pressure, shear, heat flux and area of every wall side of level 0 into the
// host array out[4][n_wall]
static int wall_loads_host(miugks_ctx* ctx, std::vector<double>& out) {
    const Geo& g = ctx->geo[0];
    out.assign(4 * (size_t)g.n_wall, 0.0);
    if (g.n_wall == 0) return MIUGKS_OK;
    double* d = ctx->loads;
    if (ctx->prec == MIUGKS_FP64)
        k_wall_loads<double><<<dim3((g.n_wall + 3) / 4), dim3(256), 0, ctx->stream>>>(g, ctx->vel, ctx->gas.K_int,
                                                                                    (const double*)ctx->f, d);
    else
        k_wall_loads<float><<<dim3((g.n_wall + 3) / 4), dim3(256), 0, ctx->stream>>>(g, ctx->vel, ctx->gas.K_int,
                                                                                   (const float*)ctx->f, d);
    int rc = check_launch(ctx);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(out.data(), d, out.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return MIUGKS_OK;
}

int miugks_wall_loads(miugks_ctx* ctx, double* p, double* tau, double* q, double* S, int* n_walls) {
    if (!ctx || !n_walls) return MIUGKS_EINVAL;
    int nw = ctx->geo[0].n_wall;
    *n_walls = nw;
    if (!p && !tau && !q && !S) return MIUGKS_OK;
    std::vector<double> ld;
    int rc = wall_loads_host(ctx, ld);
    if (rc) return rc;
    double* dst[4] = {p, tau, q, S};
    for (int m = 0; m < 4; ++m)
        if (dst[m]) std::copy(ld.begin() + (size_t)m * nw, ld.begin() + (size_t)(m + 1) * nw, dst[m]);
    return MIUGKS_OK;
}

int miugks_objective(miugks_ctx* ctx, int kind, const int* walls, int n, double* J) {
    if (!ctx || !J || n < 0 || (n > 0 && !walls)) return MIUGKS_EINVAL;
    if (kind < MIUGKS_LOAD_PRESSURE || kind > MIUGKS_LOAD_HEAT) {
        ctx->err = "objective kind must be MIUGKS_LOAD_PRESSURE, MIUGKS_LOAD_SHEAR or MIUGKS_LOAD_HEAT";
        return MIUGKS_EINVAL;
    }
    int nw = ctx->geo[0].n_wall;
    for (int i = 0; i < n; ++i)
        if (walls[i] < 0 || walls[i] >= nw) {
            ctx->err = "wall index out of range";
            return MIUGKS_EINVAL;
        }
    std::vector<double> ld;
    int rc = wall_loads_host(ctx, ld);
    if (rc) return rc;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += ld[3 * (size_t)nw + walls[i]] * ld[(size_t)kind * nw + walls[i]];
    *J = s;
    return MIUGKS_OK;
}

int miugks_set_wall_T(miugks_ctx* ctx, const int* faces, const double* Tw, int n) {
    if (!ctx || n < 0 || (n > 0 && (!faces || !Tw))) return MIUGKS_EINVAL;
    const HostLevel& h0 = ctx->hl[0];
    const int nfx = (h0.nx + 1) * h0.ny, nfy = h0.nx * (h0.ny + 1);
    std::vector<double> wx = h0.wallx, wy = h0.wally;
    for (int i = 0; i < n; ++i) {
        int f = faces[i];
        if (f < 0 || f >= nfx + nfy || (f < nfx ? h0.ftx[f] : h0.fty[f - nfx]) != MIUGKS_FACE_WALL) {
            ctx->err = "face index out of range or not a wall";
            return MIUGKS_EINVAL;
        }
        if (!(Tw[i] > 0)) {
            ctx->err = "wall temperature must be positive";
            return MIUGKS_EINVAL;
        }
        (f < nfx ? wx[3 * (size_t)f] : wy[3 * (size_t)(f - nfx)]) = Tw[i];
    }
    // the coarse levels take area-weighted means of the new fine walls, as at creation
    std::vector<HostLevel> nh;
    std::string err;
    if (!build_levels(h0.nx, h0.ny, ctx->L, h0.xn.data(), h0.yn.data(), h0.ftx.data(), h0.fty.data(), wx.data(),
                      wy.data(), h0.solid.data(), ctx->hv, ctx->cfl, nh, err)) {
        ctx->err = err;
        return MIUGKS_EINVAL;
    }
    for (int l = 0; l < ctx->L; ++l) {
        HostLevel& h = ctx->hl[l];
        h.wallx = nh[l].wallx;
        h.wally = nh[l].wally;
        h.w_T = nh[l].w_T;
        h.w_den = nh[l].w_den;
        if (h.w_T.empty()) continue;
        HIP_TRY(hipMemcpyAsync((double*)ctx->geo[l].w_T, h.w_T.data(), h.w_T.size() * sizeof(double),
                               hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(hipMemcpyAsync((double*)ctx->geo[l].w_den, h.w_den.data(), h.w_den.size() * sizeof(double),
                               hipMemcpyHostToDevice, ctx->stream));
    }
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return MIUGKS_OK;
}

// ---------------------------------------------------------------------------
// adjoint of the steady state (FP64 contexts)

constexpr int DOT_BLOCKS = 1024;   // blocks of the Krylov dot products (4 per CU)

static int adj_alloc(miugks_ctx* c) {
    if (c->a_lam) return MIUGKS_OK;
    const size_t nc = c->hl[0].nc, n = (size_t)c->nk * nc, nw = c->hl[0].w_cell.size() + 1;
    auto da = [c](double** p, size_t cnt) { return dev_alloc(c, (void**)p, cnt * sizeof(double)); };
    c->a_nparts = 1024;
    int rc;
    if ((rc = da(&c->a_lam, 2 * n)) || (rc = da(&c->a_res, 2 * n)) || (rc = da(&c->a_y, 2 * n)) ||
        (rc = da(&c->a_b, 2 * n)) || (rc = da(&c->a_out, 2 * n)) || (rc = da(&c->a_gbd, 2 * n)) ||
        (rc = da(&c->a_sb, 4 * n)) || (rc = da(&c->a_crec, NCA * nc)) || (rc = da(&c->a_fa, NFA * 2 * nc)) ||
        (rc = da(&c->a_rws, nw)) || (rc = da(&c->a_objw, nw)) || (rc = da(&c->a_Qj, nw)) ||
        (rc = da(&c->a_rhow, nw)) || (rc = da(&c->a_part, c->a_nparts)) || (rc = da(&c->a_grad, 2 * nw)) ||
        (rc = da(&c->a_fsave, 2 * n)) || (rc = da(&c->a_fsum, NFS * 2 * nc)) ||
        (rc = dev_alloc(c, (void**)&c->a_sides, 2 * nw * sizeof(int))))
        return rc;
    return MIUGKS_OK;
}

static int adj_check(miugks_ctx* c) {
    if (c->prec != MIUGKS_FP64) {
        c->err = "the adjoint needs an FP64 context";
        return MIUGKS_EINVAL;
    }
    if (c->top != 0) {
        c->err = "not during a full-multigrid start";
        return MIUGKS_ESTATE;
    }
    return adj_alloc(c);
}

extern "C++" {
// out = (dr/df)^T v at the current f; Step 1 (interface records) and the
// moments must be those of f.  v and out are stored as VT
template <typename VT>
static void adj_product(miugks_ctx* c, const VT* v, VT* out) {
    const Geo& g = c->geo[0];
    const size_t n = (size_t)c->nk * g.nc;
    const double* f = (const double*)c->f;
    // algorithmic bytes: one pass = one distribution-shaped array (2 planes);
    // cell and face kernels read f and v, the gather reads v and writes 6
    // planes, the assembly reads f, v and 6 gathered planes and writes out
    const double pass = 2.0 * n * 8, vpass = 2.0 * n * sizeof(VT);
    LAUNCH(c, "adj_cell", pass + vpass, k_adj_cell<VT>, dim3((g.nc + 3) / 4), dim3(256), g, c->vel, c->gas, f,
           (const double*)c->W, (const double*)c->q, v, c->a_crec);
    LAUNCH(c, "adj_face_sums", pass + vpass, (k_adj_face<0, VT>), dim3((2 * g.nc + 3) / 4), dim3(256), g, c->vel,
           c->gas, f, (const double*)c->W, (const double*)c->fp, v, c->a_fsum, c->a_fa);
    LAUNCH(c, "adj_face", pass + vpass, (k_adj_face<1, VT>), dim3((2 * g.nc + 3) / 4), dim3(256), g, c->vel, c->gas,
           f, (const double*)c->W, (const double*)c->fp, v, c->a_fsum, c->a_fa);
    if (g.n_wall)
        LAUNCH(c, "adj_wall", 0.0, k_adj_wall<VT>, dim3((g.n_wall + 3) / 4), dim3(256), g, c->vel, c->gas.K_int, v,
               c->a_rws);
    dim3 nb((unsigned)((n + 255) / 256));
    LAUNCH(c, "adj_gather", 3 * pass + vpass, k_adj_gather<VT>, nb, dim3(256), g, c->vel, (const double*)c->fp,
           (const double*)c->a_fa, v, c->a_gbd, c->a_sb);
    LAUNCH(c, "adj_assemble", 5 * pass + 2 * vpass, k_adj_assemble<VT>, nb, dim3(256), g, c->vel, f, v,
           (const double*)c->a_crec, (const double*)c->a_fa, (const double*)c->a_rws, (const double*)c->a_gbd,
           (const double*)c->a_sb, out);
}
}  // extern "C++"

int miugks_residual_adjoint(miugks_ctx* ctx, const void* v, void* out, int dtype, int on_device) {
    if (!ctx) return MIUGKS_EINVAL;
    int rc;
    if ((rc = adj_check(ctx))) return rc;
    if ((rc = copy_in(ctx, v, ctx->a_y, dtype, on_device))) return rc;
    Path<double>::residual(ctx);
    adj_product<double>(ctx, ctx->a_y, ctx->a_out);
    if ((rc = copy_out(ctx, ctx->a_out, out, dtype, on_device))) return rc;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return check_launch(ctx);
}

// mesh face of wall side j of level 0 (x-faces first, then y-faces)
static int wall_face(const HostLevel& h, int j) {
    int c = h.w_cell[j], s = h.w_side[j], ix = c % h.nx, iy = c / h.nx, nfx = (h.nx + 1) * h.ny;
    switch (s) {
        case 0: return iy * (h.nx + 1) + ix;
        case 1: return iy * (h.nx + 1) + ix + 1;
        case 2: return nfx + iy * h.nx + ix;
        default: return nfx + (iy + 1) * h.nx + ix;
    }
}

extern "C++" {
// (dr/df)^T lam = b (b in ctx->a_b) by restarted GMRES with the Krylov basis
// and the preconditioner's vectors stored as VT; every product, dot product
// and the Hessenberg arithmetic in double.  lam itself is double: each
// restart forms the true residual b - (dr/df)^T lam in double and solves for
// a correction in VT, so with float vectors the restarts refine lam like
// mixed-precision iterative refinement rather than stalling at the float
// rounding of lam.  Then dJ/dT_w per parameter face from the sides (wall
// side, owning parameter) listed.
template <typename VT>
static int adj_gmres(miugks_ctx* ctx, int kind, double tol, int max_iter, const std::vector<int>& sides,
                     const std::vector<int>& owner, int n_param, double* dJ_dTw, int* iters, double* res_out) {
    const Geo& g = ctx->geo[0];
    const size_t N = 2 * (size_t)ctx->nk * g.nc;
    int rc;
    const double vs = sizeof(VT);
    double* lam = ctx->a_lam;
    VT* a_out = (VT*)ctx->a_out;
    VT* a_y = (VT*)ctx->a_y;
    VT* a_res = (VT*)ctx->a_res;
    LAUNCH(ctx, "zero", N * 8.0, k_zero<double>, dim3((unsigned)std::min<size_t>((N + 255) / 256, 1 << 16)),
           dim3(256), lam, N);
    // (dr/df)^T lam = b by restarted GMRES, right-preconditioned with
    // M^-1 = -A^-T (A the velocity-diagonal correction operator, solved by one
    // downwind sweep per velocity); classical Gram-Schmidt applied twice, the
    // dot products of a step in one launch
    const int threads = ((g.ny + 63) / 64) * 64;
    const size_t lds = 2 * (size_t)g.ny * sizeof(double);
    const double vb = (double)N * 8;
    int m = (int)std::min<double>(30.0, std::max(4.0, std::floor(32e9 / vb) - 1.0));
    if (!ctx->a_V || ctx->a_m != m) {
        if ((rc = dev_alloc(ctx, (void**)&ctx->a_V, (size_t)(m + 1) * N * sizeof(double))) ||
            (rc = dev_alloc(ctx, (void**)&ctx->a_h, (size_t)(m + 1) * sizeof(double))) ||
            (rc = dev_alloc(ctx, (void**)&ctx->a_dpart, (size_t)(m + 1) * DOT_BLOCKS * sizeof(double))))
            return rc;
        ctx->a_m = m;
    }
    VT* V = (VT*)ctx->a_V;
    auto vec = [&](int i) { return V + (size_t)i * N; };
    const dim3 nbv((unsigned)((N + 255) / 256));
    auto sweep = [&](const VT* in, VT* out) {
        LAUNCH_SH(ctx, "adj_sweep", 2.0 * N * vs, lds, k_adj_sweep<VT>, dim3(ctx->nk), dim3(threads), g, ctx->vel,
                  (const double*)ctx->a_crec, in, out);
    };
    std::vector<double> dpart((size_t)(m + 1) * DOT_BLOCKS), hv(m + 1);
    // dot products of w with vec(0..k)
    auto dots = [&](const VT* w, const VT* base, int k, double* outd) -> int {
        // model bytes: the k vectors and w once per group of eight
        LAUNCH(ctx, "adj_dots", (k + (k + 7) / 8) * (double)N * vs, k_adj_dots<VT>, dim3(DOT_BLOCKS), dim3(256), w,
               base, N, k, N, ctx->a_dpart);
        HIP_TRY(hipMemcpyAsync(dpart.data(), ctx->a_dpart, (size_t)k * DOT_BLOCKS * sizeof(double),
                               hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        for (int i = 0; i < k; ++i) {
            double t = 0.0;
            for (int b2 = 0; b2 < DOT_BLOCKS; ++b2) t += dpart[(size_t)i * DOT_BLOCKS + b2];
            outd[i] = t;
        }
        return check_launch(ctx);
    };
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), yv(m);
    std::vector<double> part(ctx->a_nparts);
    double r0 = 0.0, rn = 0.0;
    int it = 0;
    for (bool first = true;; first = false) {
        // true residual b - (dr/df)^T lam into vec(0)
        adj_product<double>(ctx, lam, ctx->a_out);
        LAUNCH(ctx, "adj_residual", N * (16.0 + vs), k_adj_residual<VT>, dim3(ctx->a_nparts), dim3(256),
               (const double*)ctx->a_b, (const double*)ctx->a_out, vec(0), N, ctx->a_part);
        HIP_TRY(hipMemcpyAsync(part.data(), ctx->a_part, part.size() * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        if ((rc = check_launch(ctx))) return rc;
        double ss = 0.0;
        for (double x : part) ss += x;
        rn = std::sqrt(ss);
        if (first) r0 = rn;
        if (!std::isfinite(rn)) {
            ctx->err = "adjoint iteration diverged";
            return MIUGKS_EDIVERGED;
        }
        if (rn <= tol * r0 || r0 == 0.0 || it >= max_iter) break;
        LAUNCH(ctx, "adj_scale", 2.0 * N * vs, k_adj_scale<VT>, nbv, dim3(256), vec(0), (const VT*)vec(0), 1.0 / rn,
               N);
        std::fill(gv.begin(), gv.end(), 0.0);
        gv[0] = rn;
        int k = 0;
        for (; k < m && it < max_iter; ++k) {
            // w = (dr/df)^T M^-1 v_k = -(dr/df)^T A^-T v_k
            sweep(vec(k), a_y);
            adj_product<VT>(ctx, a_y, a_out);
            LAUNCH(ctx, "adj_scale", 2.0 * N * vs, k_adj_scale<VT>, nbv, dim3(256), vec(k + 1), (const VT*)a_out,
                   -1.0, N);
            for (int i = 0; i <= k; ++i) H[(size_t)i * m + k] = 0.0;
            // two projections; the second also takes |w|^2 (w is vec(k + 1),
            // the next vector of the block), and |w - sum h v|^2 = |w|^2 - sum h^2
            // for the small second-pass coefficients
            double nn = 0.0;
            for (int pass = 0; pass < 2; ++pass) {
                if ((rc = dots(vec(k + 1), V, k + 1 + pass, hv.data()))) return rc;
                for (int i = 0; i <= k; ++i) H[(size_t)i * m + k] += hv[i];
                if (pass == 1) {
                    nn = hv[k + 1];
                    for (int i = 0; i <= k; ++i) nn -= hv[i] * hv[i];
                }
                HIP_TRY(hipMemcpyAsync(ctx->a_h, hv.data(), (k + 1) * sizeof(double), hipMemcpyHostToDevice,
                                       ctx->stream));
                LAUNCH(ctx, "adj_lincomb", (k + 3.0) * N * vs, k_adj_lincomb<VT>, nbv, dim3(256), vec(k + 1),
                       (const VT*)V, N, (const double*)ctx->a_h, k + 1, -1.0, N);
            }
            double hn = std::sqrt(std::max(nn, 0.0));
            H[(size_t)(k + 1) * m + k] = hn;
            if (hn > 0.0)
                LAUNCH(ctx, "adj_scale", 2.0 * N * vs, k_adj_scale<VT>, nbv, dim3(256), vec(k + 1),
                       (const VT*)vec(k + 1), 1.0 / hn, N);
            // Givens rotations of the Hessenberg column
            for (int i = 0; i < k; ++i) {
                double a = H[(size_t)i * m + k], b2 = H[(size_t)(i + 1) * m + k];
                H[(size_t)i * m + k] = cs[i] * a + sn[i] * b2;
                H[(size_t)(i + 1) * m + k] = -sn[i] * a + cs[i] * b2;
            }
            double a = H[(size_t)k * m + k], b2 = H[(size_t)(k + 1) * m + k];
            double rr = std::hypot(a, b2);
            cs[k] = rr > 0.0 ? a / rr : 1.0;
            sn[k] = rr > 0.0 ? b2 / rr : 0.0;
            H[(size_t)k * m + k] = rr;
            H[(size_t)(k + 1) * m + k] = 0.0;
            gv[k + 1] = -sn[k] * gv[k];
            gv[k] = cs[k] * gv[k];
            ++it;
            if (std::fabs(gv[k + 1]) <= tol * r0 || hn == 0.0) {
                ++k;
                break;
            }
        }
        // y from the triangular system, u = V y, lam += M^-1 u = -A^-T u
        for (int i = k - 1; i >= 0; --i) {
            double t = gv[i];
            for (int j = i + 1; j < k; ++j) t -= H[(size_t)i * m + j] * yv[j];
            yv[i] = H[(size_t)i * m + i] != 0.0 ? t / H[(size_t)i * m + i] : 0.0;
        }
        HIP_TRY(hipMemcpyAsync(ctx->a_h, yv.data(), k * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        LAUNCH(ctx, "zero", N * vs, k_zero<VT>, dim3((unsigned)std::min<size_t>((N + 255) / 256, 1 << 16)),
               dim3(256), a_res, N);
        LAUNCH(ctx, "adj_lincomb", (k + 2.0) * N * vs, k_adj_lincomb<VT>, nbv, dim3(256), a_res, (const VT*)V, N,
               (const double*)ctx->a_h, k, 1.0, N);
        sweep(a_res, a_y);
        LAUNCH(ctx, "adj_axpy", N * (16.0 + vs), (k_adj_axpy<double, VT>), nbv, dim3(256), lam, (const VT*)a_y,
               -1.0, N);
    }
    // dJ/dT_w = dJ/dT_w|_f - lam^T dr/dT_w, summed over the sides of each face
    if (!sides.empty()) {
        LAUNCH(ctx, "adj_paramgrad", 0.0, k_adj_paramgrad<double>, dim3(((int)sides.size() + 3) / 4), dim3(256),
               g, ctx->vel, ctx->gas.K_int, kind, (const double*)ctx->a_objw, (const double*)ctx->a_Qj,
               (const double*)ctx->a_rhow, (const double*)lam, (const int*)ctx->a_sides, (int)sides.size(),
               ctx->a_grad);
        std::vector<double> gs(sides.size());
        HIP_TRY(hipMemcpyAsync(gs.data(), ctx->a_grad, gs.size() * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        for (int p = 0; p < n_param; ++p) dJ_dTw[p] = 0.0;
        for (size_t i = 0; i < sides.size(); ++i) dJ_dTw[owner[i]] += gs[i];
    }
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if ((rc = check_launch(ctx))) return rc;
    if (iters) *iters = it;
    if (res_out) *res_out = r0 > 0.0 ? rn / r0 : 0.0;
    return (r0 == 0.0 || rn <= tol * r0) ? MIUGKS_OK : MIUGKS_ENOTCONVERGED;
}
}  // extern "C++"

int miugks_adjoint_ex(miugks_ctx* ctx, int kind, const int* walls, int n, const int* param_faces, int n_param,
                      double tol, int max_iter, int krylov_dtype, double* dJ_dTw, int* iters, double* res_out) {
    if (!ctx || n < 0 || n_param < 0 || (n > 0 && !walls) || (n_param > 0 && (!param_faces || !dJ_dTw)) ||
        max_iter < 0)
        return MIUGKS_EINVAL;
    int rc;
    if ((rc = adj_check(ctx))) return rc;
    if (krylov_dtype != MIUGKS_FP64 && krylov_dtype != MIUGKS_FP32F) {
        ctx->err = "krylov_dtype must be MIUGKS_FP64 or MIUGKS_FP32F";
        return MIUGKS_EINVAL;
    }
    if (kind < MIUGKS_LOAD_PRESSURE || kind > MIUGKS_LOAD_HEAT) {
        ctx->err = "objective kind must be MIUGKS_LOAD_PRESSURE, MIUGKS_LOAD_SHEAR or MIUGKS_LOAD_HEAT";
        return MIUGKS_EINVAL;
    }
    const HostLevel& h0 = ctx->hl[0];
    const Geo& g = ctx->geo[0];
    const int nw = g.n_wall;
    const size_t N = 2 * (size_t)ctx->nk * g.nc;
    std::vector<double> objw(nw + 1, 0.0);
    for (int i = 0; i < n; ++i) {
        if (walls[i] < 0 || walls[i] >= nw) {
            ctx->err = "wall index out of range";
            return MIUGKS_EINVAL;
        }
        objw[walls[i]] += 1.0;
    }
    // parameter faces -> wall sides
    std::vector<int> sides, owner;
    for (int p = 0; p < n_param; ++p) {
        int found = 0;
        for (int j = 0; j < nw; ++j)
            if (wall_face(h0, j) == param_faces[p]) {
                sides.push_back(j);
                owner.push_back(p);
                ++found;
            }
        if (!found) {
            ctx->err = "parameter face is not a wall of a fluid cell";
            return MIUGKS_EINVAL;
        }
    }
    HIP_TRY(hipMemcpyAsync(ctx->a_objw, objw.data(), objw.size() * sizeof(double), hipMemcpyHostToDevice,
                           ctx->stream));
    if (!sides.empty())
        HIP_TRY(hipMemcpyAsync(ctx->a_sides, sides.data(), sides.size() * sizeof(int), hipMemcpyHostToDevice,
                               ctx->stream));
    auto objective = [&](double& J) {
        std::vector<double> ld;
        int r = wall_loads_host(ctx, ld);
        if (r) return r;
        J = 0.0;
        for (int i = 0; i < n; ++i) J += ld[3 * (size_t)nw + walls[i]] * ld[(size_t)kind * nw + walls[i]];
        return (int)MIUGKS_OK;
    };
    // a closed domain's steady states form a family in the total mass M and
    // the residual's Jacobian is singular (the mass row is its left null
    // vector): the adjoint equation takes the term mu m with mu = dJ/dM along
    // the family, from two steady states at masses M0 (1 +- delta)
    double mu = 0.0;
    if (ctx->renorm) {
        // the perturbed states are converged as far as the given one is
        // (twice its residual, and no further than 1e-13)
        double nb[4];
        Path<double>::residual(ctx);
        HIP_TRY(hipMemcpyAsync(nb, ctx->norms, 4 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        const double tol_mu = std::max(1e-13, 2.0 * std::max(std::max(nb[0], nb[1]), std::max(nb[2], nb[3])));
        const double delta = 1e-4, M0 = ctx->M0;
        double Jpm[2];
        HIP_TRY(hipMemcpyAsync(ctx->a_fsave, ctx->f, N * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
        for (int sgn = 0; sgn < 2; ++sgn) {
            double sc = sgn == 0 ? delta : -delta;
            const dim3 nbN((unsigned)((N + 255) / 256));
            if (sgn == 0) {   // start from the scaled state
                HIP_TRY(hipMemcpyAsync(ctx->f, ctx->a_fsave, N * sizeof(double), hipMemcpyDeviceToDevice,
                                       ctx->stream));
                LAUNCH(ctx, "adj_axpy", 3.0 * N * 8, (k_adj_axpy<double, double>), nbN, dim3(256), (double*)ctx->f,
                       (const double*)ctx->f, sc, N);
            } else {          // 2 f* - f+: the reflection of the first state, of mass M0 (1 - delta)
                HIP_TRY(hipMemcpyAsync(ctx->a_res, ctx->f, N * sizeof(double), hipMemcpyDeviceToDevice,
                                       ctx->stream));
                LAUNCH(ctx, "adj_scale", 2.0 * N * 8, k_adj_scale<double>, nbN, dim3(256), (double*)ctx->f,
                       (const double*)ctx->a_fsave, 2.0, N);
                LAUNCH(ctx, "adj_axpy", 3.0 * N * 8, (k_adj_axpy<double, double>), nbN, dim3(256), (double*)ctx->f,
                       (const double*)ctx->a_res, -1.0, N);
            }
            ctx->M0 = M0 * (1.0 + sc);
            drop_graphs(ctx);
            Path<double>::moments(ctx, nullptr);
            int done = 0;
            double res[4];
            rc = run_cycles<double>(ctx, 300, tol_mu, &done, res);
            if (rc == MIUGKS_OK || rc == MIUGKS_ENOTCONVERGED) rc = objective(Jpm[sgn]);
            if (rc) break;
        }
        HIP_TRY(hipMemcpyAsync(ctx->f, ctx->a_fsave, N * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
        ctx->M0 = M0;
        drop_graphs(ctx);
        Path<double>::moments(ctx, nullptr);
        if (rc) return rc;
        mu = (Jpm[0] - Jpm[1]) / (2.0 * delta * M0);
    }
    Path<double>::residual(ctx);
    // right-hand side b = dJ/df - mu m
    if (nw)
        LAUNCH(ctx, "adj_objwall", 0.0, k_adj_objwall, dim3((nw + 3) / 4), dim3(256), g, ctx->vel, ctx->gas.K_int,
               kind, (const double*)ctx->f, ctx->a_Qj, ctx->a_rhow);
    dim3 nbN((unsigned)((N / 2 + 255) / 256));
    LAUNCH(ctx, "adj_objgrad", N * 8.0, k_adj_objgrad, nbN, dim3(256), g, ctx->vel, kind,
           (const double*)ctx->a_objw, (const double*)ctx->a_Qj, mu, ctx->a_b);
    if (krylov_dtype == MIUGKS_FP32F)
        return adj_gmres<float>(ctx, kind, tol, max_iter, sides, owner, n_param, dJ_dTw, iters, res_out);
    return adj_gmres<double>(ctx, kind, tol, max_iter, sides, owner, n_param, dJ_dTw, iters, res_out);
}

int miugks_adjoint(miugks_ctx* ctx, int kind, const int* walls, int n, const int* param_faces, int n_param,
                   double tol, int max_iter, double* dJ_dTw, int* iters, double* res_out) {
    return miugks_adjoint_ex(ctx, kind, walls, n, param_faces, n_param, tol, max_iter, MIUGKS_FP64, dJ_dTw, iters,
                             res_out);
}

int miugks_get_f(miugks_ctx* ctx, void* dst, int dtype, int on_device) {
    if (!ctx) return MIUGKS_EINVAL;
    return copy_out(ctx, ctx->f, dst, dtype, on_device);
}

int miugks_get_f_noalloc(miugks_ctx* ctx, void* dst, int dtype) {
    if (!ctx) return MIUGKS_EINVAL;
    if (dtype != MIUGKS_FP64 && dtype != MIUGKS_FP32F) {
        ctx->err = "dtype must be MIUGKS_FP64 or MIUGKS_FP32F";
        return MIUGKS_EINVAL;
    }
    if (!dst) {
        ctx->err = "null destination";
        return MIUGKS_EINVAL;
    }
    if (!ctx->scratch) {
        ctx->err = "no device scratch for this context";
        return MIUGKS_ESTATE;
    }
    const size_t n = 2 * (size_t)ctx->nk * ctx->hl[0].nc;
    const size_t des = dtype == MIUGKS_FP64 ? 8 : 4;
    if (dtype == ctx->prec) {
        HIP_TRY(hipMemcpyAsync(dst, ctx->f, n * des, hipMemcpyDeviceToHost, ctx->stream));
    } else {
        // converted in pieces of at most the scratch's size; on one stream each
        // piece's conversion starts after the previous piece left the scratch
        const size_t per = NOALLOC_SCRATCH_BYTES / des;
        for (size_t off = 0; off < n; off += per) {
            const size_t m = std::min(per, n - off);
            if (ctx->prec == MIUGKS_FP64)
                hipLaunchKernelGGL((k_convert<double, float>), dim3(1024), dim3(256), 0, ctx->stream,
                                   (const double*)ctx->f + off, (float*)ctx->scratch, m);
            else
                hipLaunchKernelGGL((k_convert<float, double>), dim3(1024), dim3(256), 0, ctx->stream,
                                   (const float*)ctx->f + off, (double*)ctx->scratch, m);
            HIP_TRY(hipMemcpyAsync((char*)dst + off * des, ctx->scratch, m * des, hipMemcpyDeviceToHost,
                                   ctx->stream));
        }
    }
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return check_launch(ctx);
}

int miugks_set_f(miugks_ctx* ctx, const void* src, int dtype, int on_device) {
    if (!ctx) return MIUGKS_EINVAL;
    int rc = copy_in(ctx, src, ctx->f, dtype, on_device);
    if (rc) return rc;
    ctx->top = 0;
    if (ctx->prec == MIUGKS_FP64)
        Path<double>::moments(ctx, nullptr);
    else
        Path<float>::moments(ctx, nullptr);
    ctx->have_div = false;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return check_launch(ctx);
}

int miugks_residual(miugks_ctx* ctx, double* R, double res[4]) {
    if (!ctx) return MIUGKS_EINVAL;
    if (ctx->prec == MIUGKS_FP64)
        Path<double>::residual(ctx);
    else
        Path<float>::residual(ctx);
    int rc;
    if (R && (rc = download_cells(ctx, R, ctx->R, 4))) return rc;
    double nrm[4];
    HIP_TRY(hipMemcpyAsync(nrm, ctx->norms, 4 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if ((rc = check_launch(ctx))) return rc;
    if (res)
        for (int m = 0; m < 4; ++m) res[m] = nrm[m];
    return MIUGKS_OK;
}

int miugks_get_div(miugks_ctx* ctx, void* dst, int dtype, int on_device) {
    if (!ctx) return MIUGKS_EINVAL;
    if (!ctx->have_div) {
        ctx->err = "no div: call miugks_residual first";
        return MIUGKS_ESTATE;
    }
    return copy_out(ctx, ctx->div, dst, dtype, on_device);
}

int miugks_predict(miugks_ctx* ctx, const double* W, const double* R, double* W_out) {
    if (!ctx) return MIUGKS_EINVAL;
    if (!W_out) {
        ctx->err = "null output";
        return MIUGKS_EINVAL;
    }
    int rc;
    if ((rc = upload_cells(ctx, ctx->fW[0], W, 4)) || (rc = upload_cells(ctx, ctx->fR[0], R, 4))) return rc;
    set_dtn_factor(ctx);
    set_dtn(ctx);
    fas(ctx, 0, ctx->gamma);
    return download_cells(ctx, W_out, ctx->fW[0], 4);
}

int miugks_micro_residual(miugks_ctx* ctx, const double* Wt, void* r_out, double* tau_inv_out, int dtype,
                          int on_device) {
    if (!ctx) return MIUGKS_EINVAL;
    if (!ctx->have_div) {
        ctx->err = "no div: call miugks_residual first";
        return MIUGKS_ESTATE;
    }
    int rc;
    if ((rc = upload_cells(ctx, ctx->Wt, Wt, 4))) return rc;
    if (ctx->prec == MIUGKS_FP64)
        Path<double>::micro_residual(ctx);
    else
        Path<float>::micro_residual(ctx);
    if (tau_inv_out && (rc = download_cells(ctx, tau_inv_out, ctx->tau_inv[0], 1))) return rc;
    if (r_out) return copy_out(ctx, ctx->r[0], r_out, dtype, on_device);
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return check_launch(ctx);
}

int miugks_correct(miugks_ctx* ctx, const void* r, const double* tau_inv, void* df_out, int dtype, int on_device) {
    if (!ctx) return MIUGKS_EINVAL;
    int rc;
    if ((rc = copy_in(ctx, r, ctx->r[0], dtype, on_device))) return rc;
    if ((rc = upload_cells(ctx, ctx->tau_inv[0], tau_inv, 1))) return rc;
    set_dtn_factor(ctx);
    set_dtn(ctx);
    if (ctx->prec == MIUGKS_FP64)
        Path<double>::correct(ctx);
    else
        Path<float>::correct(ctx);
    if (df_out) return copy_out(ctx, ctx->df[0], df_out, dtype, on_device);
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return check_launch(ctx);
}

int miugks_set_timing(miugks_ctx* ctx, int on) {
    if (!ctx) return MIUGKS_EINVAL;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    miugks_timing_state& t = timing(ctx);
    timing_harvest(ctx);
    t.agg.clear();
    t.on = on != 0;
    return MIUGKS_OK;
}

int miugks_timing(miugks_ctx* ctx, int cap, const char** names, int* launches, double* ms, double* bytes) {
    if (!ctx) return -MIUGKS_EINVAL;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
        ctx->err = "hipStreamSynchronize failed";
        return -MIUGKS_EDEVICE;
    }
    miugks_timing_state& t = timing(ctx);
    timing_harvest(ctx);
    int n = (int)t.agg.size();
    for (int i = 0; i < n && i < cap; ++i) {
        if (names) names[i] = t.agg[i].name.c_str();
        if (launches) launches[i] = (int)t.agg[i].launches;
        if (ms) ms[i] = t.agg[i].ms;
        if (bytes) bytes[i] = t.agg[i].bytes;
    }
    return n;
}

int miugks_sizes(const miugks_ctx* ctx, int* nc, int* n_fluid, int* nk, int* n_levels) {
    if (!ctx) return MIUGKS_EINVAL;
    if (nc) *nc = ctx->hl[0].nc;
    if (n_fluid) *n_fluid = ctx->hl[0].n_fluid;
    if (nk) *nk = ctx->nk;
    if (n_levels) *n_levels = ctx->L;
    return MIUGKS_OK;
}

}  // extern "C"
