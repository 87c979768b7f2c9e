// Host side of the MI355X level-set grain-growth library: the C ABI declared
// in include/gg.h, device memory ownership, and the launch sequence of a step
//   corrector (global tiles) -> box plan, coverage lists of the new boxes ->
//   re-initialization march (phi^c -> f, new boxes) -> predictor march
//   (f -> psi, phi, volumes)
// Every launch of a step has a fixed grid (one work group per grain or per
// global tile) and the step's bookkeeping stays on the device: buffers are
// sized with headroom, a step whose new layout does not fit raises a sticky
// flag in a device control block that makes the rest of the step (and of the
// batch) skip, and the host grows the buffers and takes the step again.  The
// host therefore reads nothing back between steps, and a step can be captured
// once in a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "../../include/gg.h"
#include "gg_kernels.hpp"
#include "gg_march.hpp"
#include "gg_closest.hpp"

// Rows per column unit of the FP64 predictor march: 3 (boxes up to 39 cells
// wide in one tile; with 2 rows those from 33 on split into tiles, whose halo
// work made the march 40% slower); 2 with the correction epilogue, whose
// registers spill at 3.
#ifndef GG_PREDICT_YB64
#define GG_PREDICT_YB64 3
#endif
#ifndef GG_PREDICT_YB64_PH
#define GG_PREDICT_YB64_PH 2
#endif

// Corrector tile of the 3D grid (powers of two, 512 voxels).  Rows of 16 FP32
// values write half cache lines of each box row; 8-wide rows (a cube, the
// fewest covering boxes per voxel) were 2% faster but wrote 2.1x the bytes,
// 32- and 64-wide rows cover more boxes per voxel and were 23-80% slower.
#ifndef GG_CMP_TILE_X
#define GG_CMP_TILE_X 16
#define GG_CMP_TILE_Y 8
#define GG_CMP_TILE_Z 4
#endif

// Partial sums per grain of the interface areas (blocks per grain box).
constexpr int kAreaSplit = 8;

// Device scratch of gg_grain_areas_noalloc: the per-block partial sums of the
// interface areas for up to kNoAllocMaxGrains grains (8 MiB on every device the
// library runs on, held until the process ends).  Host code reaches it only
// through the device address taken once per device at set-up (g_scratch).
constexpr int kNoAllocMaxGrains = 65536;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) double scratch[2 * kAreaSplit * kNoAllocMaxGrains];

namespace {

using gg::Boxes;
using gg::Ctl;
using gg::Totals;

struct HipError {
    hipError_t err;
    std::string where;
};

#define HIPCHECK(x)                                                    \
    do {                                                               \
        hipError_t e_ = (x);                                           \
        if (e_ != hipSuccess) throw HipError{e_, std::string(#x)};     \
    } while (0)

struct ArgError {
    std::string msg;
};
struct CapError {
    std::string msg;
};
struct MemError {
    std::string msg;
};

// The caller's allocator of the simulation being served on this thread (set
// around every library call; NULL: hipMalloc / hipFree) and its stream.
thread_local const gg_allocator *t_alloc = nullptr;
thread_local void *t_alloc_stream = nullptr;

// A device buffer with a capacity in bytes, owned (freed when it goes out of
// scope) and freed through the allocator that allocated it.
struct DBuf {
    void *p = nullptr;
    size_t cap = 0;
    const gg_allocator *al = nullptr;
    void *al_stream = nullptr;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { release(); }
    void ensure(size_t bytes) {
        if (bytes <= cap && p) return;
        if (p) (void)hipDeviceSynchronize();  // no pending work may still use the old buffer
        release();
        size_t b = std::max<size_t>(bytes, 256);
        if (t_alloc) {
            p = t_alloc->alloc(b, t_alloc_stream, t_alloc->user);
            if (!p) throw MemError{"the caller's allocator returned NULL for " + std::to_string(b) + " bytes"};
            al = t_alloc;
            al_stream = t_alloc_stream;
        } else {
            hipError_t e = hipMalloc(&p, b);
            if (e != hipSuccess) {
                p = nullptr;
                cap = 0;
                (void)hipGetLastError();
                throw MemError{"device allocation of " + std::to_string(b) + " bytes failed"};
            }
            al = nullptr;
        }
        cap = b;
    }
    void release() {
        if (p) {
            if (al) al->free(p, al_stream, al->user);
            else (void)hipFree(p);
        }
        p = nullptr;
        cap = 0;
        al = nullptr;
    }
    void swap(DBuf &o) {
        std::swap(p, o.p);
        std::swap(cap, o.cap);
        std::swap(al, o.al);
        std::swap(al_stream, o.al_stream);
    }
    template <typename U> U *as() const { return reinterpret_cast<U *>(p); }
};

int pow2_divisor(int N, int target) {
    int t = target;
    while (t > 1 && N % t) t >>= 1;
    return t;
}

// Roles of the value arenas: the predicted function psi; the corrected function
// phi^c (and the materialised phi in 3D); f, the forward-spread distances (3D)
// or phi (2D) or the Euclidean sweeps' result; the Euclidean sweeps' second
// buffer.
enum { A_PSI = 0, A_PHIC = 1, A_F = 2, A_SCR = 3 };

struct Tuning {
    int order_size, lds_bytes, small_bytes, candidates;
    double ns_per_gv[8];
    int cand_order[8], cand_lds[8], cand_small[8];
};

struct SimBase {
    virtual ~SimBase() = default;
    virtual void step(double dt, int n) = 0;
    virtual void volumes(double *out) = 0;
    virtual void labels(int32_t *out, bool device) = 0;
    virtual void boxes(int32_t *lo, int32_t *ext, int32_t *alive, int64_t *off, bool prev) = 0;
    virtual long long values(double *out, long long cap, int which) = 0;
    virtual long long iota(int32_t *out, long long cap) = 0;
    virtual void load_state(const int32_t *lo, const int32_t *ext, const uint8_t *alive, const double *vals,
                            const int32_t *iota) = 0;
    virtual void coarsen(const int32_t *np) = 0;
    virtual void areas(double *area, double *weighted) = 0;
    virtual bool areas_noalloc(double *part, double *area, double *weighted) = 0;
    virtual long long grain_sdf(int k, int32_t *lo, int32_t *ext, double *out, long long cap) = 0;
    virtual void save(FILE *f) = 0;
    virtual void load(FILE *f) = 0;
    virtual void grid(int32_t *n) const = 0;
    virtual void autotune(double dt, int per, Tuning *out) = 0;
    virtual void sync() = 0;
    virtual int alive_count() = 0;
    virtual gg_step_stats stats() = 0;
    virtual void profile(bool on) = 0;
    virtual gg_kernel_times kernel_times() = 0;
    virtual void set_keep(bool on) = 0;
};

template <typename T> struct Sim final : SimBase {
    // configuration
    int dim, G, n[3], P, K;
    int redist, K_euclid;  // re-initialization scheme of the steps; its Jacobi sweep count
    T W;
    double band_d;  // W as given
    // LDS budget of a work group and limit of the small launch class of the
    // Euclidean variant's item tilings (FP32 bytes; FP64 tiles get the same
    // values), tunable (gg_autotune)
    int lds_bytes = gg::kLdsBytes, small_bytes = gg::kSmallLdsBytes;
    int physics;
    double theta_c, voxel_m, gamma_max, headroom;
    bool exact = false;  // capacities without slack
    bool batched;
    int order_size;  // per-grain kernels take the largest boxes first
    bool closest = false;  // correction weights from the closest boundary point (A_SCR)
    int tdim[3], nt[3], ntiles, occ_words;
    hipStream_t stream = nullptr;
    bool own_stream = false;

    // layouts 0/1: box tables (+ the Euclidean variant's work items)
    DBuf lo[2], ext[2], alive[2], off[2];
    DBuf ipref[2], iowner[2][gg::kKinds * gg::kClasses], itile[2];
    Totals tot[2];
    int cur = 0;

    // per step accumulators and scratch
    DBuf bmin, bmax, occ, sizes, cnt, ldsmax, vol, vol_part;
    DBuf cov_cnt, cov_off, cov_cur, cov_list, cov_total;
    DBuf taps_d, quat_d, energy_d, totals_d, ctl_d, order_d;
    Totals *totals_h = nullptr;
    Ctl *ctl_h = nullptr;
    long long cap_arena = 0, cap_cov = 0;  // values per arena, coverage entries
    DBuf arena[4];  // value arenas, roles A_PSI .. A_SCR
    DBuf iota_a[2];
    int iota_cur = 0;  // ID-field of the current layout
    bool psi_ok = false;  // arena A_PSI holds psi of the current layout and taps
    int f_chain = 1;      // arena A_F: forward-spread distances (1) or a final function (0)
    int a_phi = -1;       // arena holding phi of the current layout (-1: not materialised)
    // kept intermediates (test hook)
    bool keep = false;
    DBuf keep_psi, keep_phic, keep_lo, keep_ext, keep_alive, keep_off;
    Totals keep_tot{};
    bool have_keep = false;

    // current Gaussian
    double sigma = -1.0;
    int R = 0;
    long long taps_epoch = 0;
    std::vector<T> taps_h;

    // host mirrors of the device counters (valid when nothing is pending)
    long long steps_done = 0, total_gv = 0, last_gv = 0;
    int alive_n = 0;
    double last_ms = 0.0;

    // the steps queued by the last gg_step call
    bool pending = false;
    long long call_steps0 = 0;
    int call_n = 0, call_cur0 = 0, call_ic0 = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;

    // captured steps: one graph per (layout parity, ID-field parity)
    struct GSlot {
        bool valid = false;
        int cur = 0, ic = 0;
        long long epoch = -1, taps = -1;
        hipGraphExec_t exec = nullptr;
    } gslot[4];
    long long epoch = 0;  // bumped whenever a buffer the step uses moves
    int gnext = 0;

    // per-kernel timing: HIP event pairs on the simulation's stream
    struct Span {
        hipEvent_t a, b;
        int cls;
        long long vox;
        int vmode;  // voxel count: 0 as given, 1 the step's input layout, 2 its new layout
        int n;      // kernel dispatches in the span
    };
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<Span> spans;
    size_t spans_step0 = 0;
    gg_kernel_times ktimes{};

    hipEvent_t next_event() {
        if (ev_used == ev_pool.size()) {
            hipEvent_t e;
            HIPCHECK(hipEventCreate(&e));
            ev_pool.push_back(e);
        }
        return ev_pool[ev_used++];
    }
    void tbegin(int cls, long long vox, int vmode = 0) {
        if (!prof) return;
        Span sp{next_event(), nullptr, cls, vox, vmode, 1};
        HIPCHECK(hipEventRecord(sp.a, stream));
        spans.push_back(sp);
    }
    void tend(int dispatches = 1) {
        if (!prof) return;
        spans.back().n = dispatches;
        spans.back().b = next_event();
        HIPCHECK(hipEventRecord(spans.back().b, stream));
    }
    void resolve_spans() {
        if (spans.empty()) return;
        HIPCHECK(hipStreamSynchronize(stream));
        for (const Span &sp : spans) {
            float ms = 0.f;
            HIPCHECK(hipEventElapsedTime(&ms, sp.a, sp.b));
            ktimes.ms[sp.cls] += ms;
            ktimes.launches[sp.cls] += sp.n;
            ktimes.voxels[sp.cls] += sp.vox;
        }
        spans.clear();
        spans_step0 = 0;
        ev_used = 0;
    }
    void profile(bool on) override {
        settle();
        resolve_spans();
        prof = on;
        std::memset(&ktimes, 0, sizeof(ktimes));
    }
    gg_kernel_times kernel_times() override {
        settle();
        resolve_spans();
        return ktimes;
    }
    void set_keep(bool on) override {
        settle();
        keep = on;
    }

    Boxes boxes_of(int l) {
        return Boxes{lo[l].as<int>(), ext[l].as<int>(), alive[l].as<int>(), off[l].as<long long>()};
    }
    gg::TileArgs tile_args() const {
        gg::TileArgs t;
        for (int a = 0; a < 3; ++a) {
            t.n[a] = n[a];
            t.t[a] = tdim[a];
            t.nt[a] = nt[a];
        }
        t.occ_words = occ_words;
        return t;
    }
    gg::GridArgs grid_args() const {
        gg::GridArgs g;
        for (int a = 0; a < 3; ++a) g.n[a] = n[a];
        g.dim = dim;
        return g;
    }
    Ctl *ctl() const { return ctl_d.as<Ctl>(); }

    Sim(const gg_config &c, int G_, hipStream_t s) {
        dim = c.dim;
        G = G_;
        for (int a = 0; a < 3; ++a) n[a] = c.n[a];
        W = (T)c.band;
        band_d = c.band;
        P = (int)std::ceil(c.band);
        K = P;
        redist = c.redistance;
        // a Godunov value exceeds its smallest neighbour by >= 1/sqrt(dim): values
        // up to W settle after ceil(sqrt(dim) W) + 1 sweeps, taken as an even count
        K_euclid = (int)std::ceil(std::sqrt((double)dim) * c.band) + 1;
        K_euclid += K_euclid & 1;
        physics = c.physics;
        theta_c = c.theta_c_deg;
        voxel_m = c.voxel_m;
        gamma_max = c.gamma_max;
        // 0: default slack; 1: buffers hold exactly the current layout
        headroom = c.capacity_headroom >= 1.0 ? c.capacity_headroom : 1.25;
        exact = c.capacity_headroom == 1.0;
        batched = c.batched != 0;
        order_size = (c.flags & GG_FLAG_ORDER_ID) ? 0 : 1;
        closest = (c.flags & GG_FLAG_CLOSEST_POINT) != 0;
        set_tiles();
        occ_words = (std::max(n[0], std::max(n[1], n[2])) + 31) / 32;
        if (s) {
            stream = s;
        } else {
            HIPCHECK(hipStreamCreate(&stream));
            own_stream = true;
        }
        try {
            allocate_tables();
        } catch (...) {
            // a throwing constructor runs no destructor: hand back what is not a member buffer
            free_host();
            if (own_stream && stream) (void)hipStreamDestroy(stream);
            stream = nullptr;
            throw;
        }
    }

    void free_host() {
        if (totals_h) (void)hipHostFree(totals_h);
        if (ctl_h) (void)hipHostFree(ctl_h);
        totals_h = nullptr;
        ctl_h = nullptr;
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        ev0 = ev1 = nullptr;
    }

    void allocate_tables() {
        HIPCHECK(hipHostMalloc((void **)&totals_h, sizeof(Totals), hipHostMallocDefault));
        HIPCHECK(hipHostMalloc((void **)&ctl_h, sizeof(Ctl), hipHostMallocDefault));
        std::memset(totals_h, 0, sizeof(Totals));
        std::memset(ctl_h, 0, sizeof(Ctl));
        HIPCHECK(hipEventCreate(&ev0));
        HIPCHECK(hipEventCreate(&ev1));
        for (int l = 0; l < 2; ++l) {
            lo[l].ensure(sizeof(int) * 3 * G);
            ext[l].ensure(sizeof(int) * 3 * G);
            alive[l].ensure(sizeof(int) * G);
            off[l].ensure(sizeof(long long) * (G + 1));
            if (redist == GG_REDIST_EUCLID) {
                ipref[l].ensure(sizeof(long long) * 3 * gg::kKinds * (size_t)(G + 1));
                itile[l].ensure(sizeof(int4) * 2 * gg::kKinds * (size_t)G);
            }
        }
        bmin.ensure(sizeof(int) * 3 * G);
        bmax.ensure(sizeof(int) * 3 * G);
        occ.ensure(sizeof(unsigned) * 3 * (size_t)G * occ_words);
        HIPCHECK(hipMemsetAsync(occ.p, 0, occ.cap, stream));
        std::vector<int> init_min(3 * G, 0x7fffffff), init_max(3 * G, -1);
        HIPCHECK(hipMemcpyAsync(bmin.p, init_min.data(), sizeof(int) * 3 * G, hipMemcpyHostToDevice, stream));
        HIPCHECK(hipMemcpyAsync(bmax.p, init_max.data(), sizeof(int) * 3 * G, hipMemcpyHostToDevice, stream));
        sizes.ensure(sizeof(long long) * G);
        if (redist == GG_REDIST_EUCLID) {
            cnt.ensure(sizeof(long long) * 3 * gg::kKinds * (size_t)G);
            ldsmax.ensure(sizeof(unsigned long long) * gg::kKinds * gg::kClasses);
        }
        vol.ensure(sizeof(double) * G);
        HIPCHECK(hipMemsetAsync(vol.p, 0, sizeof(double) * G, stream));
        cov_cnt.ensure(sizeof(int) * ntiles);
        cov_off.ensure(sizeof(int) * (ntiles + 1));
        cov_cur.ensure(sizeof(int) * (ntiles + 1));
        cov_total.ensure(sizeof(long long));
        taps_d.ensure(sizeof(T) * (2 * gg::kMaxRadius + 1));
        totals_d.ensure(sizeof(Totals));
        ctl_d.ensure(sizeof(Ctl));
        order_d.ensure(sizeof(int) * G);
        HIPCHECK(hipMemcpyAsync(ctl_d.p, ctl_h, sizeof(Ctl), hipMemcpyHostToDevice, stream));
        HIPCHECK(hipStreamSynchronize(stream));
    }

    // Global corrector / label tiles of the current grid.
    void set_tiles() {
        if (dim == 3) {
            tdim[0] = pow2_divisor(n[0], GG_CMP_TILE_X);
            tdim[1] = pow2_divisor(n[1], GG_CMP_TILE_Y);
            tdim[2] = pow2_divisor(n[2], GG_CMP_TILE_Z);
        } else {
            tdim[0] = pow2_divisor(n[0], 32);
            tdim[1] = pow2_divisor(n[1], gg::kTileVox / 32);
            tdim[2] = 1;
        }
        ntiles = 1;
        for (int a = 0; a < 3; ++a) {
            nt[a] = n[a] / tdim[a];
            ntiles *= nt[a];
        }
    }

    // Switch to the periodic grid np (coarsening, checkpoint of another grid):
    // corrector tiles, coverage counters and the occupancy rows of whole-axis
    // boxes (one bit per voxel of an axis), grown for a finer grid.
    void set_grid(const int *np) {
        for (int a = 0; a < 3; ++a) n[a] = np[a];
        set_tiles();
        cov_cnt.ensure(sizeof(int) * ntiles);
        cov_off.ensure(sizeof(int) * (ntiles + 1));
        cov_cur.ensure(sizeof(int) * (ntiles + 1));
        const int words = (std::max(n[0], std::max(n[1], n[2])) + 31) / 32;
        if (words > occ_words) {
            occ.ensure(sizeof(unsigned) * 3 * (size_t)G * words);
            HIPCHECK(hipMemsetAsync(occ.p, 0, occ.cap, stream));
            occ_words = words;
        }
        ++epoch;
    }
    void grid(int32_t *out) const override {
        for (int a = 0; a < 3; ++a) out[a] = n[a];
    }

    ~Sim() override {
        if (stream) (void)hipStreamSynchronize(stream);
        for (GSlot &g : gslot)
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
        DBuf *all[] = {&bmin,     &bmax,     &occ,      &sizes,   &ldsmax,   &vol,       &vol_part, &cov_cnt,
                       &cov_off,  &cov_cur,  &cov_list, &cov_total, &taps_d, &quat_d,    &energy_d, &totals_d,
                       &ctl_d,    &order_d,  &keep_psi, &keep_phic, &keep_lo, &keep_ext, &keep_alive, &keep_off,
                       &cnt};
        for (DBuf *b : all) b->release();
        for (int l = 0; l < 2; ++l) {
            lo[l].release();
            ext[l].release();
            alive[l].release();
            off[l].release();
            iota_a[l].release();
            itile[l].release();
            ipref[l].release();
            for (int q = 0; q < gg::kKinds * gg::kClasses; ++q) iowner[l][q].release();
        }
        for (int a = 0; a < 4; ++a) arena[a].release();
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        free_host();
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }

    void sync() override {
        settle();
        HIPCHECK(hipStreamSynchronize(stream));
    }

    // ------------------------------------------------------------ capacities

    long long grow_to(long long need) const {
        return exact ? std::max<long long>(need, 1) : (long long)((double)need * headroom) + 1024;
    }
    int n_arenas() const { return (redist == GG_REDIST_EUCLID || closest) ? 4 : 3; }

    // Grow a buffer to `bytes`, keeping its first `keep_bytes`.
    void grow_keep(DBuf &b, size_t bytes, size_t keep_bytes) {
        if (b.p && bytes <= b.cap) return;
        DBuf nb;
        nb.ensure(bytes);
        if (b.p && keep_bytes) {
            HIPCHECK(hipMemcpyAsync(nb.p, b.p, std::min(keep_bytes, b.cap), hipMemcpyDeviceToDevice, stream));
            HIPCHECK(hipStreamSynchronize(stream));
        }
        b.swap(nb);
        ++epoch;
    }

    // Value arenas (and ID-fields) for `need` values; arenas in `keep_mask`
    // keep their contents.
    void ensure_arenas(long long need, unsigned keep_mask) {
        if (need <= cap_arena && arena[0].p) return;
        const long long old = cap_arena;
        if (exact) cap_arena = 0;
        cap_arena = std::max(grow_to(need), cap_arena);
        for (int a = 0; a < n_arenas(); ++a)
            grow_keep(arena[a], sizeof(T) * (size_t)cap_arena, (keep_mask >> a & 1u) ? sizeof(T) * (size_t)old : 0);
        if (physics)
            for (int l = 0; l < 2; ++l) grow_keep(iota_a[l], sizeof(int) * (size_t)cap_arena, 0);
        ++epoch;
    }

    void ensure_cov(long long need) {
        if (need > 0x7fffffffLL) throw CapError{"coverage list exceeds 2^31 entries"};
        if (need <= cap_cov && cov_list.p) return;
        if (exact) cap_cov = 0;
        cap_cov = std::min<long long>(std::max(grow_to(need), cap_cov), 0x7fffffffLL);
        cov_list.ensure(sizeof(int) * (size_t)cap_cov);
        ++epoch;
    }

    // Coverage lists of layout l, sized on the host (synchronous).
    void build_coverage(int l) {
        tbegin(GG_K_PLAN, 0);
        HIPCHECK(hipMemsetAsync(cov_cnt.p, 0, sizeof(int) * ntiles, stream));
        hipLaunchKernelGGL(gg::k_coverage, dim3(G), dim3(64), 0, stream, boxes_of(l), cov_cnt.as<int>(), (int *)nullptr,
                           tile_args(), G, 0, (const Ctl *)nullptr);
        hipLaunchKernelGGL(gg::k_scan_int, dim3(1), dim3(1024), 0, stream, cov_cnt.as<int>(), cov_off.as<int>(),
                           cov_cur.as<int>(), ntiles, cov_total.as<long long>(), (Ctl *)nullptr, 0LL);
        tend();
        HIPCHECK(hipGetLastError());
        long long total = 0;
        HIPCHECK(hipMemcpyAsync(&total, cov_total.p, sizeof(long long), hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
        ensure_cov(total);
        tbegin(GG_K_PLAN, 0);
        hipLaunchKernelGGL(gg::k_coverage, dim3(G), dim3(64), 0, stream, boxes_of(l), cov_cur.as<int>(),
                           cov_list.as<int>(), tile_args(), G, 1, (const Ctl *)nullptr);
        tend();
        HIPCHECK(hipGetLastError());
        tot[l].cov = total;
    }

    // Arena size and alive count of layout l (synchronous).
    void read_totals(int l) {
        hipLaunchKernelGGL(gg::k_totals, dim3(1), dim3(256), 0, stream, (const long long *)off[l].as<long long>(),
                           (const long long *)nullptr, (const long long *)nullptr, (const int *)alive[l].as<int>(), G,
                           (const unsigned long long *)nullptr, totals_d.as<Totals>());
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipMemcpyAsync(totals_h, totals_d.p, sizeof(Totals), hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
        tot[l].arena = totals_h->arena;
        tot[l].alive = totals_h->alive;
    }

    // Work items of the Euclidean variant's kinds on layout l (synchronous).
    void layout_items(int l) {
        Boxes L = boxes_of(l);
        tbegin(GG_K_PLAN, 0);
        HIPCHECK(hipMemsetAsync(ldsmax.p, 0, sizeof(unsigned long long) * gg::kKinds * gg::kClasses, stream));
        const int tb = 256, gb = (G + tb - 1) / tb;
        hipLaunchKernelGGL(gg::k_item_counts, dim3(gb, gg::kKinds), dim3(tb), 0, stream, L, cnt.as<long long>(),
                           itile[l].as<int4>(), ldsmax.as<unsigned long long>(), G,
                           gg::budget_values<T>(lds_bytes), gg::budget_values<T>(small_bytes));
        hipLaunchKernelGGL(gg::k_scan_multi, dim3(3 * gg::kKinds), dim3(1024), 0, stream, cnt.as<long long>(),
                           ipref[l].as<long long>(), G);
        hipLaunchKernelGGL(gg::k_totals, dim3(1), dim3(256), 0, stream, (const long long *)L.off,
                           (const long long *)ipref[l].as<long long>(), (const long long *)nullptr,
                           (const int *)L.alive, G, (const unsigned long long *)ldsmax.as<unsigned long long>(),
                           totals_d.as<Totals>());
        HIPCHECK(hipGetLastError());
        tend();
        HIPCHECK(hipMemcpyAsync(totals_h, totals_d.p, sizeof(Totals), hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
        for (int q = 0; q < gg::kKinds; ++q) {
            for (int j = 0; j < 3; ++j) tot[l].items[q][j] = totals_h->items[q][j];
            for (int c = 0; c < gg::kClasses; ++c) {
                tot[l].lds[q][c] = totals_h->lds[q][c];
                if (tot[l].lds[q][c] < 0 || tot[l].lds[q][c] > gg::budget_values<T>(lds_bytes))
                    throw CapError{"a box is too large for the stencil tiling"};
            }
        }
        gg::OwnerMaps om;
        for (int q = 0; q < gg::kKinds; ++q)
            for (int c = 0; c < gg::kClasses; ++c) {
                DBuf &b = iowner[l][q * gg::kClasses + c];
                b.ensure(sizeof(int) * (size_t)std::max<long long>(tot[l].items[q][1 + c], 1) * 5 / 4);
                om.owner[q * gg::kClasses + c] = b.as<int>();
            }
        tbegin(GG_K_PLAN, 0);
        hipLaunchKernelGGL(gg::k_fill_owner, dim3(G, gg::kKinds * gg::kClasses), dim3(64), 0, stream,
                           ipref[l].as<long long>(), om, G);
        HIPCHECK(hipGetLastError());
        tend();
    }

    const long long *pref_of(int l, int kind, int j) const {
        return ipref[l].as<long long>() + ((size_t)kind * 3 + j) * (size_t)(G + 1);
    }
    gg::ItemRefs refs(int l, int kind, int cls) const {
        gg::ItemRefs r;
        r.owner = iowner[l][kind * gg::kClasses + cls].as<int>();
        r.pref = pref_of(l, kind, 1 + cls);
        r.pref_all = pref_of(l, kind, 0);
        r.tilings = itile[l].as<int4>() + (size_t)kind * 2 * G;
        r.n = tot[l].items[kind][1 + cls];
        return r;
    }

    // New taps when sigma changes; a cached predicted function is then stale.
    void set_gaussian(double dt) {
        double s = std::sqrt(2.0 * dt) * (double)n[0];
        if (s == sigma) return;
        int r = (int)std::ceil(4.0 * s - 1e-9);
        if (r < 1) r = 1;
        if (r > gg::kMaxRadius || r > 2 * P) throw ArgError{"kernel radius R = ceil(4 sigma) exceeds min(12, 2P)"};
        std::vector<double> t(2 * r + 1);
        double s2 = 2.0 * s * s, sum = 0.0;
        for (int i = -r; i <= r; ++i) {
            t[i + r] = std::exp(-(double)(i * i) / s2);
            sum = sum + t[i + r];
        }
        taps_h.assign(2 * r + 1, T(0));
        for (int i = 0; i < 2 * r + 1; ++i) taps_h[i] = (T)(t[i] / sum);
        HIPCHECK(hipMemcpyAsync(taps_d.p, taps_h.data(), sizeof(T) * taps_h.size(), hipMemcpyHostToDevice, stream));
        HIPCHECK(hipStreamSynchronize(stream));
        sigma = s;
        R = r;
        psi_ok = false;
        ++taps_epoch;
    }

    gg::Physics<T> physics_args(const int *iota_p) const {
        gg::Physics<T> ph;
        ph.mode = physics;
        ph.quat = quat_d.as<T>();
        ph.energy = energy_d.as<T>();
        ph.theta_c_deg = (T)theta_c;
        ph.bulk_scale = (physics & 2) ? (T)(sigma * sigma * voxel_m / (2.0 * gamma_max)) : T(0);
        ph.phi = nullptr;
        ph.iota = iota_p;
        ph.wcp = nullptr;
        return ph;
    }

    gg::MarchArgs march_args(bool in_step) const {
        gg::MarchArgs ma;
        for (int a = 0; a < 3; ++a) ma.n[a] = n[a];
        ma.dim = dim;
        ma.G = G;
        ma.K = K;
        ma.R = R;
        ma.order = (in_step && order_size) ? order_d.as<int>() : nullptr;
        ma.phi_always = 0;
        ma.ctl = in_step ? ctl() : nullptr;
        return ma;
    }

    // ------------------------------------------------------------ launches

    // Re-initialization march: phi^c on layout lo_l -> f on layout ln_l (2D:
    // the final function and the volumes).
    void launch_reinit(int lo_l, int ln_l, const T *phic, T *out, const int *io_old, int *io_new, bool in_step) {
        const gg::MarchArgs ma = march_args(in_step);
        const size_t lds = (size_t)gg::reinit_cells<T>() * sizeof(T);
        double *v = dim == 2 ? vol.as<double>() : nullptr;
        tbegin(GG_K_REINIT, in_step ? 0 : tot[ln_l].arena, in_step ? 1 : 0);
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(G), dim3(gg::kMT), lds, stream, boxes_of(lo_l), boxes_of(ln_l), ma, phic,
                               out, io_old, io_new, v, W);
        };
        constexpr int YB = gg::kReinitYB;
        auto pick = [&](auto ks) {
            constexpr int KS = decltype(ks)::value;
            const bool io = io_new != nullptr && io_old != nullptr;
            if (dim == 3) {
                if (io) go(gg::k_reinit_march<T, KS, YB, true, true>);
                else go(gg::k_reinit_march<T, KS, YB, true, false>);
            } else {
                if (io) go(gg::k_reinit_march<T, KS, YB, false, true>);
                else go(gg::k_reinit_march<T, KS, YB, false, false>);
            }
        };
        if (K == 8) pick(std::integral_constant<int, 8>{});
        else if (K == 6) pick(std::integral_constant<int, 6>{});
        else pick(std::integral_constant<int, 0>{});
        tend();
        HIPCHECK(hipGetLastError());
    }

    // Predictor march on layout l: in (f when chain, else a final function) ->
    // psi (when given) with the correction epilogue, phi (when given), volumes.
    void launch_predict(int l, T *in, int chain, T *psi, T *phi_out, const int *iota_l, bool in_step,
                        const T *wcp = nullptr, bool phi_always = false) {
        gg::MarchArgs ma = march_args(in_step);
        ma.phi_always = phi_always ? 1 : 0;
        gg::Physics<T> ph = physics_args(iota_l);
        ph.wcp = wcp;
        double *v = dim == 3 ? vol.as<double>() : nullptr;
        const int Rk = psi ? R : 8;
        tbegin(GG_K_PREDICT, in_step ? 0 : tot[l].arena, in_step ? 2 : 0);
        auto go = [&](auto kern, int yb) {
            const size_t lds = (size_t)gg::predict_cells<T>() * sizeof(T);
            (void)yb;
            hipLaunchKernelGGL(kern, dim3(G), dim3(gg::kMT), lds, stream, boxes_of(l), ma, in, psi, phi_out, v,
                               (const T *)taps_d.as<T>(), ph, W, chain);
        };
        const bool phys = physics != 0 && psi != nullptr;
        // rows per column unit: FP64 keeps its register window (2R + 1 planes of
        // YB rows) small enough not to spill
        constexpr int YB = sizeof(T) == 8 ? GG_PREDICT_YB64 : 4;
        constexpr int YBP = sizeof(T) == 8 ? GG_PREDICT_YB64_PH : 4;
        if (Rk == 8) {
            if (phys) go(gg::k_predict_march<T, 8, YBP, true>, YBP);
            else go(gg::k_predict_march<T, 8, YB, false>, YB);
        } else if (Rk == 6) {
            if (phys) go(gg::k_predict_march<T, 6, YBP, true>, YBP);
            else go(gg::k_predict_march<T, 6, YB, false>, YB);
        } else {
            if (phys) go(gg::k_predict_march<T, 0, 2, true>, 2);
            else go(gg::k_predict_march<T, 0, 2, false>, 2);
        }
        tend();
        HIPCHECK(hipGetLastError());
    }

    void launch_compare(int L, const T *psi, T *phic, int *iota_out, int mode, bool in_step) {
        tbegin(GG_K_COMPARE, 0, 1);
        auto kern = iota_out ? gg::k_compare<T, true> : gg::k_compare<T, false>;
        hipLaunchKernelGGL(kern, dim3((unsigned)gg::xcd_grid(ntiles)), dim3(gg::kBlock), 0, stream, boxes_of(L), (const int *)cov_off.as<int>(), (const int *)cov_list.as<int>(), psi, phic,
                           iota_out, bmin.as<int>(), bmax.as<int>(), occ.as<unsigned>(), tile_args(), W, mode,
                           in_step ? (const Ctl *)ctl() : (const Ctl *)nullptr);
        tend();
        HIPCHECK(hipGetLastError());
    }

    const int *iota_of(int ic) const { return physics ? iota_a[ic].as<int>() : nullptr; }
    int *iota_w(int ic) { return physics ? iota_a[ic].as<int>() : nullptr; }

    // ----------------------------------------------------------------- create
    void create(const int32_t *labels, const double *quat, const double *energy) {
        // initial boxes on the host: per axis the covered cyclic interval of the
        // grain's projection, padded by P (a box within 2P of the axis takes it all)
        const long long nt3 = (long long)n[0] * n[1] * n[2];
        const int nsum = n[0] + n[1] + n[2];
        std::vector<unsigned char> occh((size_t)G * nsum, 0);
        for (long long i = 0; i < nt3; ++i) {
            const int x = (int)(i % n[0]), y = (int)((i / n[0]) % n[1]), z = (int)(i / ((long long)n[0] * n[1]));
            unsigned char *o = &occh[(size_t)labels[i] * nsum];
            o[x] = 1;
            o[n[0] + y] = 1;
            o[n[0] + n[1] + z] = 1;
        }
        std::vector<int> hlo(3 * G, 0), hext(3 * G, 0), hal(G, 0);
        std::vector<long long> hoff(G + 1, 0);
        for (int k = 0; k < G; ++k) {
            const unsigned char *o = &occh[(size_t)k * nsum];
            bool ok = true;
            int base = 0;
            for (int a = 0; a < 3 && ok; ++a) {
                const int N = n[a];
                int first = -1, ones = 0;
                for (int i = 0; i < N; ++i)
                    if (o[base + i]) {
                        if (first < 0) first = i;
                        ++ones;
                    }
                if (first < 0) {
                    ok = false;
                    break;
                }
                int st = 0, ln = N;
                if (ones < N) {
                    int best_s = -1, best_l = -1, run_s = -1, run_l = 0;
                    for (int t = 1; t <= N; ++t) {
                        const int i = (first + t) % N;
                        if (!o[base + i]) {
                            if (run_l == 0) run_s = i;
                            ++run_l;
                        } else if (run_l > 0) {
                            if (run_l > best_l || (run_l == best_l && run_s < best_s)) {
                                best_l = run_l;
                                best_s = run_s;
                            }
                            run_l = 0;
                        }
                    }
                    st = (best_s + best_l) % N;
                    ln = N - best_l;
                }
                const long long e = (long long)ln + 2LL * P;
                if (e > (long long)N - 2LL * P) {
                    hlo[3 * k + a] = 0;
                    hext[3 * k + a] = N;
                } else {
                    hlo[3 * k + a] = gg::imod((long long)st - P, N);
                    hext[3 * k + a] = (int)e;
                }
                base += N;
            }
            hal[k] = ok ? 1 : 0;
            if (!ok)
                for (int a = 0; a < 3; ++a) hlo[3 * k + a] = hext[3 * k + a] = 0;
        }
        int nalive = 0;
        for (int k = 0; k < G; ++k) {
            hoff[k + 1] = hoff[k] + (hal[k] ? (long long)hext[3 * k] * hext[3 * k + 1] * hext[3 * k + 2] : 0);
            nalive += hal[k];
        }
        upload_table(0, hlo.data(), hext.data(), hal.data(), hoff.data());
        cur = 0;
        iota_cur = 0;
        tot[0].arena = hoff[G];
        alive_n = nalive;
        if (physics & 1) {
            std::vector<T> q(4 * (size_t)G);
            for (size_t i = 0; i < q.size(); ++i) q[i] = (T)quat[i];
            quat_d.ensure(sizeof(T) * q.size());
            HIPCHECK(hipMemcpyAsync(quat_d.p, q.data(), sizeof(T) * q.size(), hipMemcpyHostToDevice, stream));
            HIPCHECK(hipStreamSynchronize(stream));
        }
        if (physics & 2) {
            std::vector<T> e(G);
            for (int k = 0; k < G; ++k) e[k] = (T)energy[k];
            energy_d.ensure(sizeof(T) * G);
            HIPCHECK(hipMemcpyAsync(energy_d.p, e.data(), sizeof(T) * G, hipMemcpyHostToDevice, stream));
            HIPCHECK(hipStreamSynchronize(stream));
        }
        ensure_arenas(hoff[G], 0u);
        build_coverage(0);
        // initial function: the re-initialised +-1/2 indicator on the same boxes
        DBuf lab;
        lab.ensure(sizeof(int32_t) * nt3);
        HIPCHECK(hipMemcpyAsync(lab.p, labels, sizeof(int32_t) * nt3, hipMemcpyHostToDevice, stream));
        hipLaunchKernelGGL(gg::k_init_indicator<T>, dim3(G), dim3(gg::kBlock), 0, stream, boxes_of(0),
                           lab.as<int>(), arena[A_PHIC].as<T>(), grid_args());
        HIPCHECK(hipGetLastError());
        reinit_in_place(0, A_PHIC);
        HIPCHECK(hipStreamSynchronize(stream));
        lab.release();
        if (physics) initial_iota();
    }

    // Re-initialization of the values in arena `src` on layout l (creation,
    // coarsening): phi into a_phi, f (3D) or phi (2D) into A_F, volumes.
    void reinit_in_place(int l, int src) {
        launch_reinit(l, l, arena[src].as<T>(), arena[A_F].as<T>(), nullptr, nullptr, false);
        if (dim == 3) {
            launch_predict(l, arena[A_F].as<T>(), 1, nullptr, arena[A_PHIC].as<T>(), nullptr, false);
            a_phi = A_PHIC;
            f_chain = 1;
        } else {
            a_phi = A_F;
            f_chain = 0;
        }
        psi_ok = false;
    }

    // ID-field of the current phi: argmax of the other grains' functions.
    void initial_iota() {
        iota_cur = 0;
        launch_compare(cur, arena[a_phi].as<T>(), (T *)nullptr, iota_a[0].as<int>(), 1, false);
        HIPCHECK(hipStreamSynchronize(stream));
    }

    void upload_table(int l, const int *hlo, const int *hext, const int *hal, const long long *hoff) {
        HIPCHECK(hipMemcpyAsync(lo[l].p, hlo, sizeof(int) * 3 * G, hipMemcpyHostToDevice, stream));
        HIPCHECK(hipMemcpyAsync(ext[l].p, hext, sizeof(int) * 3 * G, hipMemcpyHostToDevice, stream));
        HIPCHECK(hipMemcpyAsync(alive[l].p, hal, sizeof(int) * G, hipMemcpyHostToDevice, stream));
        HIPCHECK(hipMemcpyAsync(off[l].p, hoff, sizeof(long long) * (G + 1), hipMemcpyHostToDevice, stream));
        HIPCHECK(hipStreamSynchronize(stream));
    }

    // ------------------------------------------------------------------ step

    // psi of the current layout from the state in A_F.
    void predict_state() {
        const T *wcp = closest_weights(cur, f_chain, iota_of(iota_cur), false);
        launch_predict(cur, arena[A_F].as<T>(), f_chain, arena[A_PSI].as<T>(), nullptr, iota_of(iota_cur), false, wcp);
        psi_ok = true;
    }

    // Correction weights from the closest boundary point (sec. 3.2) of layout l
    // into A_SCR, from the layout's function (A_F; with a pending z chain,
    // finished into A_PHIC first) and ID-field; NULL when the mode is off.
    const T *closest_weights(int l, int chain, const int *iota_l, bool in_step) {
        if (!closest) return nullptr;
        const T *phi_src = arena[A_F].as<T>();
        if (chain) {
            launch_predict(l, arena[A_F].as<T>(), chain, nullptr, arena[A_PHIC].as<T>(), nullptr, in_step, nullptr,
                           true);
            phi_src = arena[A_PHIC].as<T>();
        }
        tbegin(GG_K_CLOSEST, in_step ? 0 : tot[l].arena, in_step ? 2 : 0);
        hipLaunchKernelGGL(gg::k_closest_weight<T>, dim3(G), dim3(gg::kBlock), 0, stream, boxes_of(l), phi_src,
                           iota_l, physics_args(iota_l), arena[A_SCR].as<T>(), grid_args(),
                           (const int *)((in_step && order_size) ? order_d.as<int>() : nullptr),
                           in_step ? (const Ctl *)ctl() : (const Ctl *)nullptr);
        tend();
        HIPCHECK(hipGetLastError());
        return arena[A_SCR].as<T>();
    }

    // The kernels of one step from layout L (ID-field parity ic) to layout
    // 1 - L (1 - ic).  No host synchronisation: the step can be captured.
    void issue_step(int L, int ic) {
        const int Ln = 1 - L, icn = 1 - ic;
        Ctl *c = ctl();
        // 1. corrector: psi -> phi^c, ID-field, bounding boxes of phi^c > 0
        launch_compare(L, arena[A_PSI].as<T>(), arena[A_PHIC].as<T>(), iota_w(ic), 0, true);
        if (keep) keep_copy(L, arena[A_PSI].as<T>(), arena[A_PHIC].as<T>());
        // 2. new boxes, offsets (capacity check), coverage lists (capacity check), launch order
        gg::PlanArgs pa;
        for (int a = 0; a < 3; ++a) pa.n[a] = n[a];
        pa.P = P;
        pa.occ_words = occ_words;
        pa.G = G;
        const int tb = 256, gb = (G + tb - 1) / tb;
        tbegin(GG_K_PLAN, 0);
        hipLaunchKernelGGL(gg::k_plan, dim3(gb), dim3(tb), 0, stream, boxes_of(L), boxes_of(Ln), bmin.as<int>(),
                           bmax.as<int>(), occ.as<unsigned>(), sizes.as<long long>(), pa, (const Ctl *)c);
        hipLaunchKernelGGL(gg::k_scan, dim3(1), dim3(1024), 0, stream, (const long long *)sizes.as<long long>(),
                           off[Ln].as<long long>(), G, c, cap_arena);
        hipLaunchKernelGGL(gg::k_zero_int, dim3((ntiles + 255) / 256), dim3(256), 0, stream, cov_cnt.as<int>(), ntiles,
                           (const Ctl *)c);
        hipLaunchKernelGGL(gg::k_coverage, dim3(G), dim3(64), 0, stream, boxes_of(Ln), cov_cnt.as<int>(),
                           (int *)nullptr, tile_args(), G, 0, (const Ctl *)c);
        hipLaunchKernelGGL(gg::k_scan_int, dim3(1), dim3(1024), 0, stream, (const int *)cov_cnt.as<int>(),
                           cov_off.as<int>(), cov_cur.as<int>(), ntiles, cov_total.as<long long>(), c, cap_cov);
        hipLaunchKernelGGL(gg::k_coverage, dim3(G), dim3(64), 0, stream, boxes_of(Ln), cov_cur.as<int>(),
                           cov_list.as<int>(), tile_args(), G, 1, (const Ctl *)c);
        if (order_size)
            hipLaunchKernelGGL(gg::k_order_size, dim3(1), dim3(1024), 0, stream,
                               (const long long *)off[Ln].as<long long>(), (const int *)alive[Ln].as<int>(),
                               order_d.as<int>(), G, (const Ctl *)c);
        tend(order_size ? 7 : 6);
        HIPCHECK(hipGetLastError());
        // 3. re-initialization into the new boxes, 4. the next predictor
        if (redist == GG_REDIST_EUCLID) {
            euclid_reinit(L, Ln, ic, icn);
        } else {
            launch_reinit(L, Ln, arena[A_PHIC].as<T>(), arena[A_F].as<T>(), iota_of(ic), iota_w(icn), true);
        }
        const int chain = (dim == 3 && redist != GG_REDIST_EUCLID) ? 1 : 0;
        const T *wcp = closest_weights(Ln, chain, iota_of(icn), true);
        launch_predict(Ln, arena[A_F].as<T>(), chain, arena[A_PSI].as<T>(),
                       dim == 3 ? arena[A_PHIC].as<T>() : (T *)nullptr, iota_of(icn), true, wcp);
        tbegin(GG_K_PLAN, 0);
        hipLaunchKernelGGL(gg::k_step_end, dim3(1), dim3(1024), 0, stream, c, (const int *)alive[Ln].as<int>(),
                           (const long long *)off[L].as<long long>(), (const long long *)off[Ln].as<long long>(),
                           (const long long *)cov_total.as<long long>(), G);
        tend();
        HIPCHECK(hipGetLastError());
    }

    // The Euclidean variant's re-initialization (synchronous: its work items
    // are sized on the host).  A step whose layout failed the capacity checks
    // is left to the caller.
    void euclid_reinit(int L, int Ln, int ic, int icn) {
        HIPCHECK(hipMemcpyAsync(ctl_h, ctl_d.p, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
        if (ctl_h->fail) return;
        layout_items(Ln);
        const Totals &t = tot[Ln];
        const gg::GridArgs g = grid_args();
        T *u = arena[A_F].as<T>(), *v2 = arena[A_SCR].as<T>();
        if (t.items[gg::KIND_RXY][0] > 0) {
            tbegin(GG_K_REINIT, 0, 2);
            int nd = 0;
            for (int c = 0; c < gg::kClasses; ++c) {
                const gg::ItemRefs ir = refs(Ln, gg::KIND_RXY, c);
                if (ir.n <= 0) continue;
                ++nd;
                hipLaunchKernelGGL(gg::k_reinit_xy<T>, dim3((unsigned)gg::xcd_grid(ir.n)), dim3(gg::kBlock),
                                   sizeof(T) * t.lds[gg::KIND_RXY][c], stream, boxes_of(L), boxes_of(Ln), ir,
                                   (const T *)arena[A_PHIC].as<T>(), u, iota_of(ic), iota_w(icn), W, g);
            }
            tend(nd);
            HIPCHECK(hipGetLastError());
        }
        vol_part.ensure(sizeof(double) * (size_t)std::max<long long>(t.items[gg::KIND_JAC][0], 1) * 5 / 4);
        tbegin(GG_K_REINIT_SWEEP, 0, 2);
        int nd = 0;
        T *a = u, *b = v2;
        for (int s = 0; s < K_euclid; ++s) {
            const bool fin = dim == 2 && s == K_euclid - 1;  // K_euclid is even: the last sweep writes u
            T *dst = fin ? u : b;
            for (int c = 0; c < gg::kClasses; ++c) {
                const gg::ItemRefs ir = refs(Ln, gg::KIND_JAC, c);
                if (ir.n <= 0) continue;
                ++nd;
                hipLaunchKernelGGL(gg::k_jacobi<T>, dim3((unsigned)gg::xcd_grid(ir.n)), dim3(gg::kBlock),
                                   sizeof(T) * t.lds[gg::KIND_JAC][c], stream, boxes_of(Ln), ir, (const T *)a, dst,
                                   vol_part.as<double>(), W, fin ? 1 : 0, g);
            }
            std::swap(a, b);
        }
        tend(nd);
        HIPCHECK(hipGetLastError());
        if (dim == 2) {
            tbegin(GG_K_PLAN, 0);
            hipLaunchKernelGGL(gg::k_volumes, dim3(G), dim3(64), 0, stream, boxes_of(Ln), pref_of(Ln, gg::KIND_JAC, 0),
                               (const double *)vol_part.as<double>(), vol.as<double>(), G);
            tend();
            HIPCHECK(hipGetLastError());
        }
    }

    hipGraphExec_t graph_for(int c, int ic) {
        for (GSlot &g : gslot)
            if (g.valid && g.cur == c && g.ic == ic && g.epoch == epoch && g.taps == taps_epoch) return g.exec;
        GSlot &g = gslot[gnext];
        gnext = (gnext + 1) % 4;
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g.exec = nullptr;
        g.valid = false;
        hipGraph_t graph = nullptr;
        HIPCHECK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        try {
            issue_step(c, ic);
        } catch (...) {
            (void)hipStreamEndCapture(stream, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
        }
        HIPCHECK(hipStreamEndCapture(stream, &graph));
        hipGraphExec_t ex = nullptr;
        hipError_t e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHECK(e);
        g.valid = true;
        g.cur = c;
        g.ic = ic;
        g.epoch = epoch;
        g.taps = taps_epoch;
        g.exec = ex;
        return ex;
    }

    // Queue `nsteps` steps from the current layout (no synchronisation).
    void run_steps(int nsteps, bool use_graphs) {
        for (int s = 0; s < nsteps; ++s) {
            if (use_graphs) {
                HIPCHECK(hipGraphLaunch(graph_for(cur, iota_cur), stream));
            } else {
                if (prof) spans_step0 = spans.size();
                issue_step(cur, iota_cur);
                if (prof) resolve_step_voxels();
                if (redist == GG_REDIST_EUCLID && ctl_h->fail) {  // read back by euclid_reinit
                    grow_after_failure();
                    --s;
                    continue;
                }
            }
            cur = 1 - cur;
            iota_cur = 1 - iota_cur;
        }
    }

    // Profiling: the voxel counts of the last step's spans (synchronous).
    void resolve_step_voxels() {
        HIPCHECK(hipMemcpyAsync(ctl_h, ctl_d.p, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
        for (size_t i = spans_step0; i < spans.size(); ++i) {
            if (spans[i].vmode == 1) spans[i].vox = ctl_h->fail ? 0 : ctl_h->last_gv;
            if (spans[i].vmode == 2) spans[i].vox = ctl_h->fail ? 0 : ctl_h->arena_now;
        }
    }

    void upload_ctl(int phi_at) {
        ctl_h->fail = 0;
        ctl_h->fail_step = 0;
        ctl_h->steps = (int)steps_done;
        ctl_h->alive = alive_n;
        ctl_h->phi_at = phi_at;
        ctl_h->total_gv = total_gv;
        ctl_h->last_gv = last_gv;
        ctl_h->arena_now = tot[cur].arena;
        ctl_h->cov_now = tot[cur].cov;
        HIPCHECK(hipMemcpyAsync(ctl_d.p, ctl_h, sizeof(Ctl), hipMemcpyHostToDevice, stream));
    }

    void step(double dt, int nsteps) override {
        settle();
        if (nsteps <= 0) return;
        set_gaussian(dt);
        if (!psi_ok) predict_state();
        call_steps0 = steps_done;
        call_n = nsteps;
        call_cur0 = cur;
        call_ic0 = iota_cur;
        upload_ctl((int)(steps_done + nsteps - 1));
        const bool graphs = batched && !prof && !keep && redist != GG_REDIST_EUCLID;
        HIPCHECK(hipEventRecord(ev0, stream));
        run_steps(nsteps, graphs);
        HIPCHECK(hipEventRecord(ev1, stream));
        pending = true;
        a_phi = dim == 3 ? A_PHIC : A_F;
        f_chain = (dim == 3 && redist != GG_REDIST_EUCLID) ? 1 : 0;
        psi_ok = true;
        have_keep = keep;
        if (!batched) settle();
    }

    // Wait for the queued steps, take over the device counters, and finish the
    // steps a capacity failure stopped.
    void settle() {
        if (!pending) return;
        pending = false;
        HIPCHECK(hipMemcpyAsync(ctl_h, ctl_d.p, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
        float ms = 0.f;
        HIPCHECK(hipEventElapsedTime(&ms, ev0, ev1));
        if (call_n > 0) last_ms = ms / call_n;
        if (ctl_h->fail) recover();
        steps_done = ctl_h->steps;
        total_gv = ctl_h->total_gv;
        last_gv = ctl_h->last_gv;
        alive_n = ctl_h->alive;
        tot[cur].arena = ctl_h->arena_now;
        tot[cur].cov = ctl_h->cov_now;
        resolve_spans();
    }

    // A step failed its capacity check (ctl_h read back); the state it started
    // from (psi in A_PSI on layout cur) is intact.  Grow the buffer that was too
    // small and rebuild the coverage lists of that layout when the failing step
    // overwrote them; the counters of the completed steps stand.
    void grow_after_failure() {
        const int why = ctl_h->fail;
        if (why == 1) ensure_arenas(ctl_h->need_arena, 1u << A_PSI);
        if (why == 2) ensure_cov(ctl_h->need_cov);
        steps_done = ctl_h->steps;
        total_gv = ctl_h->total_gv;
        last_gv = ctl_h->last_gv;
        alive_n = ctl_h->alive;
        if (why == 2) build_coverage(cur);
        upload_ctl(ctl_h->phi_at);
    }

    // Take again the queued steps from the one that failed.
    void recover() {
        for (int round = 0; ctl_h->fail; ++round) {
            if (round > 8) throw CapError{"the step layout keeps outgrowing the device buffers"};
            const int completed = (int)(ctl_h->steps - call_steps0);
            const int remaining = call_n - completed;
            cur = call_cur0 ^ (completed & 1);
            iota_cur = call_ic0 ^ (completed & 1);
            grow_after_failure();
            call_steps0 = steps_done;
            call_n = remaining;
            call_cur0 = cur;
            call_ic0 = iota_cur;
            run_steps(remaining, false);
            HIPCHECK(hipMemcpyAsync(ctl_h, ctl_d.p, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
            HIPCHECK(hipStreamSynchronize(stream));
        }
    }

    // phi of the current layout (materialised from A_F when needed).
    void ensure_phi() {
        settle();
        if (a_phi >= 0) return;
        if (dim == 3) {
            launch_predict(cur, arena[A_F].as<T>(), f_chain, nullptr, arena[A_PHIC].as<T>(), nullptr, false);
            a_phi = A_PHIC;
        } else {
            a_phi = A_F;
        }
        HIPCHECK(hipStreamSynchronize(stream));
    }

    // Grid coarsening onto np (validated by the caller): projection of the
    // current phi, new boxes from its positive nodes (the box plan over a
    // virtual layout that takes every axis whole), re-initialization as at
    // creation, the ID-field rebuilt when the correction is on.
    void coarsen(const int32_t *np_in) override {
        int np[3] = {np_in[0], np_in[1], np_in[2]};
        ensure_phi();
        HIPCHECK(hipStreamSynchronize(stream));
        const int L = cur, Ln = 1 - cur;
        gg::CoarsenArgs<T> ca;
        for (int a = 0; a < 3; ++a) {
            ca.n[a] = n[a];
            ca.np[a] = np[a];
        }
        ca.dim = dim;
        ca.W = W;
        const double r = (double)n[0] / (double)np[0];
        ca.r = (T)r;
        const int split = 8;  // blocks per grain
        // virtual layout on the new grid: every axis whole, liveness of layout L
        DBuf vlo, vext;
        vlo.ensure(sizeof(int) * 3 * G);
        vext.ensure(sizeof(int) * 3 * G);
        std::vector<int> hz(3 * G, 0), he(3 * G);
        for (int k = 0; k < G; ++k)
            for (int a = 0; a < 3; ++a) he[3 * k + a] = np[a];
        HIPCHECK(hipMemcpyAsync(vlo.p, hz.data(), sizeof(int) * 3 * G, hipMemcpyHostToDevice, stream));
        HIPCHECK(hipMemcpyAsync(vext.p, he.data(), sizeof(int) * 3 * G, hipMemcpyHostToDevice, stream));
        Boxes Lv{vlo.as<int>(), vext.as<int>(), alive[L].as<int>(), off[L].as<long long>()};
        HIPCHECK(hipMemsetAsync(occ.p, 0, occ.cap, stream));
        tbegin(GG_K_PLAN, 0);
        hipLaunchKernelGGL(gg::k_coarsen_mark<T>, dim3(G, split), dim3(gg::kBlock), 0, stream, boxes_of(L),
                           (const T *)arena[a_phi].as<T>(), ca, bmax.as<int>(), occ.as<unsigned>(), occ_words);
        gg::PlanArgs pa;
        for (int a = 0; a < 3; ++a) pa.n[a] = np[a];
        pa.P = P;
        pa.occ_words = occ_words;
        pa.G = G;
        const int tb = 256, gb = (G + tb - 1) / tb;
        hipLaunchKernelGGL(gg::k_plan, dim3(gb), dim3(tb), 0, stream, Lv, boxes_of(Ln), bmin.as<int>(),
                           bmax.as<int>(), occ.as<unsigned>(), sizes.as<long long>(), pa, (const Ctl *)nullptr);
        hipLaunchKernelGGL(gg::k_scan, dim3(1), dim3(1024), 0, stream, (const long long *)sizes.as<long long>(),
                           off[Ln].as<long long>(), G, (Ctl *)nullptr, 0LL);
        tend();
        HIPCHECK(hipGetLastError());
        // the new grid
        set_grid(np);
        voxel_m *= r;
        have_keep = false;
        read_totals(Ln);
        ensure_arenas(tot[Ln].arena, 1u << a_phi);
        const int a_src = A_PSI;  // psi is stale from here on
        tbegin(GG_K_PLAN, 0);
        hipLaunchKernelGGL(gg::k_coarsen_values<T>, dim3(G, split), dim3(gg::kBlock), 0, stream, boxes_of(L),
                           (const T *)arena[a_phi].as<T>(), boxes_of(Ln), arena[a_src].as<T>(), ca);
        tend();
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipStreamSynchronize(stream));
        cur = Ln;
        build_coverage(Ln);
        reinit_in_place(Ln, a_src);
        alive_n = (int)tot[Ln].alive;
        if (physics) initial_iota();
        HIPCHECK(hipStreamSynchronize(stream));
        resolve_spans();
        vlo.release();
        vext.release();
    }

    // Interface areas of the current phi (FP64 per-grain sums, fixed order).
    // k_areas into `part` (2 G kAreaSplit doubles), then the per-grain sums into
    // area_out and weighted_out (NULL: not written), ordered on the stream.
    void areas_launch(double *part, double *area_out, double *weighted_out) {
        gg::AreaArgs aa;
        aa.mode = physics;
        aa.theta_c_deg = theta_c;
        aa.split = kAreaSplit;
        aa.G = G;
        hipLaunchKernelGGL(gg::k_areas<T>, dim3(G, kAreaSplit), dim3(gg::kBlock), 0, stream, boxes_of(cur),
                           (const T *)arena[a_phi].as<T>(), iota_of(iota_cur), (const T *)quat_d.as<T>(), aa, part,
                           W, grid_args());
        hipLaunchKernelGGL(gg::k_sum_rows, dim3((2 * G + 255) / 256), dim3(256), 0, stream, (const double *)part,
                           area_out, weighted_out, G, kAreaSplit);
        HIPCHECK(hipGetLastError());
    }
    void areas(double *area, double *weighted) override {
        ensure_phi();
        DBuf part, sums;
        part.ensure(sizeof(double) * 2 * (size_t)G * kAreaSplit);
        sums.ensure(sizeof(double) * 2 * (size_t)G);
        areas_launch(part.as<double>(), sums.as<double>(), sums.as<double>() + G);
        std::vector<double> h(2 * (size_t)G);
        HIPCHECK(hipMemcpyAsync(h.data(), sums.p, sizeof(double) * 2 * G, hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
        std::memcpy(area, h.data(), sizeof(double) * G);
        if (weighted) std::memcpy(weighted, h.data() + G, sizeof(double) * G);
    }
    // The same launches with the caller's partial-sum memory and device outputs,
    // allocating nothing: queued steps are taken over only when none of them
    // failed its capacity check (false: one did; it stays queued, and the next
    // other call grows the buffers and takes it again), and no timing spans are
    // recorded (they take events).
    bool areas_noalloc(double *part, double *area, double *weighted) override {
        if (pending) {
            HIPCHECK(hipMemcpyAsync(ctl_h, ctl_d.p, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
            HIPCHECK(hipStreamSynchronize(stream));
            if (ctl_h->fail) return false;
        }
        struct ProfOff {
            bool &p, was;
            explicit ProfOff(bool &q) : p(q), was(q) { p = false; }
            ~ProfOff() { p = was; }
        } off(prof);
        ensure_phi();
        areas_launch(part, area, weighted);
        return true;
    }

    // One grain's box and values (as doubles); returns the value count, or
    // -count when cap is too small (nothing written), 0 for an extinct grain.
    long long grain_sdf(int k, int32_t *lo_o, int32_t *ext_o, double *out, long long cap) override {
        ensure_phi();
        int l[3], e[3], al = 0;
        long long o = 0;
        HIPCHECK(hipMemcpyAsync(l, lo[cur].as<int>() + 3 * k, sizeof(int) * 3, hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipMemcpyAsync(e, ext[cur].as<int>() + 3 * k, sizeof(int) * 3, hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipMemcpyAsync(&al, alive[cur].as<int>() + k, sizeof(int), hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipMemcpyAsync(&o, off[cur].as<long long>() + k, sizeof(long long), hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
        if (!al) {
            for (int a = 0; a < 3; ++a) lo_o[a] = ext_o[a] = 0;
            return 0;
        }
        for (int a = 0; a < 3; ++a) {
            lo_o[a] = l[a];
            ext_o[a] = e[a];
        }
        const long long m = (long long)e[0] * e[1] * e[2];
        if (cap < m || !out) return -m;
        DBuf tmp;
        tmp.ensure(sizeof(double) * m);
        hipLaunchKernelGGL((gg::k_convert<T, double>), dim3(256), dim3(256), 0, stream, arena[a_phi].as<T>() + o,
                           tmp.as<double>(), m);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipMemcpyAsync(out, tmp.p, sizeof(double) * m, hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
        return m;
    }

    // ---------------------------------------------------------- checkpoint
    struct CkptHeader {
        char magic[8];
        int32_t version, dim, n[3], G, precision, redistance, physics, has_iota, pad;
        double band, theta_c, voxel_m, gamma_max;
        int64_t steps, total_gv, values;
    };
    static constexpr char kMagic[8] = {'G', 'G', 'C', 'K', 'P', 'T', 0, 1};
    int precision_code() const { return sizeof(T) == 8 ? GG_FP64 : GG_FP32; }

    static void put(FILE *f, const void *p, size_t bytes) {
        if (bytes && std::fwrite(p, 1, bytes, f) != bytes) throw ArgError{"checkpoint write failed"};
    }
    static void get(FILE *f, void *p, size_t bytes) {
        if (bytes && std::fread(p, 1, bytes, f) != bytes) throw ArgError{"checkpoint is truncated"};
    }

    void save(FILE *f) override {
        ensure_phi();
        HIPCHECK(hipStreamSynchronize(stream));
        const long long m = tot[cur].arena;
        CkptHeader h{};
        std::memcpy(h.magic, kMagic, 8);
        h.version = 1;
        h.dim = dim;
        for (int a = 0; a < 3; ++a) h.n[a] = n[a];
        h.G = G;
        h.precision = precision_code();
        h.redistance = redist;
        h.physics = physics;
        h.has_iota = physics ? 1 : 0;
        h.band = band_d;
        h.theta_c = theta_c;
        h.voxel_m = voxel_m;
        h.gamma_max = gamma_max;
        h.steps = steps_done;
        h.total_gv = total_gv;
        h.values = m;
        std::vector<int> l(3 * G), e(3 * G), al(G), io;
        std::vector<T> v(std::max<long long>(m, 1));
        std::vector<double> vo(G);
        HIPCHECK(hipMemcpyAsync(l.data(), lo[cur].p, sizeof(int) * 3 * G, hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipMemcpyAsync(e.data(), ext[cur].p, sizeof(int) * 3 * G, hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipMemcpyAsync(al.data(), alive[cur].p, sizeof(int) * G, hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipMemcpyAsync(v.data(), arena[a_phi].p, sizeof(T) * m, hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipMemcpyAsync(vo.data(), vol.p, sizeof(double) * G, hipMemcpyDeviceToHost, stream));
        if (h.has_iota) {
            io.resize(std::max<long long>(m, 1));
            HIPCHECK(hipMemcpyAsync(io.data(), iota_of(iota_cur), sizeof(int) * m, hipMemcpyDeviceToHost, stream));
        }
        HIPCHECK(hipStreamSynchronize(stream));
        put(f, &h, sizeof(h));
        put(f, l.data(), sizeof(int) * 3 * G);
        put(f, e.data(), sizeof(int) * 3 * G);
        put(f, al.data(), sizeof(int) * G);
        put(f, v.data(), sizeof(T) * m);
        if (h.has_iota) put(f, io.data(), sizeof(int) * m);
        put(f, vo.data(), sizeof(double) * G);
    }

    void load(FILE *f) override {
        settle();
        CkptHeader h;
        get(f, &h, sizeof(h));
        if (std::memcmp(h.magic, kMagic, 8) != 0 || h.version != 1) throw ArgError{"not a checkpoint of this library"};
        if (h.dim != dim || h.G != G || h.precision != precision_code() || h.band != band_d ||
            h.physics != physics || h.redistance != redist)
            throw ArgError{"checkpoint of a different configuration (dim, grains, precision, band, physics, "
                           "re-initialization)"};
        long long ntot = 1;
        for (int a = 0; a < 3; ++a) {
            const bool active = a < dim;
            if (active ? (h.n[a] < 4 * P + 2 || h.n[a] > 4096) : h.n[a] != 1)
                throw ArgError{"checkpoint grid out of range"};
            ntot *= h.n[a];
        }
        if (ntot > 2147483647LL || h.values < 0 || h.has_iota != (physics ? 1 : 0)) throw ArgError{"corrupt checkpoint"};
        std::vector<int> l(3 * G), e(3 * G), al(G);
        get(f, l.data(), sizeof(int) * 3 * G);
        get(f, e.data(), sizeof(int) * 3 * G);
        get(f, al.data(), sizeof(int) * G);
        long long m = 0;
        for (int k = 0; k < G; ++k)
            if (al[k]) {
                for (int a = 0; a < 3; ++a)
                    if (e[3 * k + a] < 1 || e[3 * k + a] > h.n[a]) throw ArgError{"corrupt checkpoint box"};
                m += (long long)e[3 * k] * e[3 * k + 1] * e[3 * k + 2];
            }
        if (m != h.values) throw ArgError{"corrupt checkpoint: box volumes and value count differ"};
        std::vector<T> v(std::max<long long>(m, 1));
        std::vector<int> io;
        std::vector<double> vo(G);
        get(f, v.data(), sizeof(T) * m);
        if (h.has_iota) {
            io.resize(std::max<long long>(m, 1));
            get(f, io.data(), sizeof(int) * m);
        }
        get(f, vo.data(), sizeof(double) * G);
        std::vector<uint8_t> a8(G);
        for (int k = 0; k < G; ++k) a8[k] = al[k] ? 1 : 0;
        // the grid of the checkpoint, then the state (validated by the box rule)
        const int keep_n[3] = {n[0], n[1], n[2]};
        const double keep_h = voxel_m;
        set_grid(h.n);
        voxel_m = h.voxel_m;
        try {
            load_state_core(l.data(), e.data(), a8.data(), v.data(), h.has_iota ? io.data() : nullptr);
        } catch (const ArgError &) {
            set_grid(keep_n);
            voxel_m = keep_h;
            throw;
        }
        HIPCHECK(hipMemcpyAsync(vol.p, vo.data(), sizeof(double) * G, hipMemcpyHostToDevice, stream));
        HIPCHECK(hipStreamSynchronize(stream));
        steps_done = h.steps;
        total_gv = h.total_gv;
        have_keep = false;
    }

    // Try the candidate schedules for `per` steps each (the simulation
    // advances), keep the one with the least device time per grain voxel.
    void autotune(double dt, int per, Tuning *out) override {
        settle();
        std::vector<std::array<int, 3>> cand;
        if (redist == GG_REDIST_EUCLID) {
            static const int b[][2] = {{40960, 26624}, {32768, 20480}, {40960, 20480}, {49152, 26624}, {49152, 32768}};
            for (const auto &c : b) cand.push_back({order_size, c[0], c[1]});
        } else {
            cand.push_back({0, lds_bytes, small_bytes});
            cand.push_back({1, lds_bytes, small_bytes});
        }
        double best = 1e300;
        std::array<int, 3> pick = cand[0];
        Tuning t{};
        t.candidates = (int)cand.size();
        for (size_t i = 0; i < cand.size(); ++i) {
            order_size = cand[i][0];
            lds_bytes = cand[i][1];
            small_bytes = cand[i][2];
            ++epoch;
            const long long gv0 = total_gv;
            step(dt, per);
            settle();
            const double per_gv = 1e6 * last_ms * per / (double)std::max<long long>(total_gv - gv0, 1);
            t.ns_per_gv[i] = per_gv;
            t.cand_order[i] = cand[i][0];
            t.cand_lds[i] = cand[i][1];
            t.cand_small[i] = cand[i][2];
            if (per_gv < best) {
                best = per_gv;
                pick = cand[i];
            }
        }
        order_size = pick[0];
        lds_bytes = pick[1];
        small_bytes = pick[2];
        ++epoch;
        t.order_size = order_size;
        t.lds_bytes = lds_bytes;
        t.small_bytes = small_bytes;
        *out = t;
    }

    void keep_copy(int L, const T *psi, const T *phic) {
        long long m = 0;  // the step's layout size (the host mirror is per call)
        HIPCHECK(hipMemcpyAsync(&m, off[L].as<long long>() + G, sizeof(long long), hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
        keep_psi.ensure(sizeof(T) * (size_t)std::max<long long>(cap_arena, 1));
        keep_phic.ensure(sizeof(T) * (size_t)std::max<long long>(cap_arena, 1));
        keep_lo.ensure(sizeof(int) * 3 * G);
        keep_ext.ensure(sizeof(int) * 3 * G);
        keep_alive.ensure(sizeof(int) * G);
        keep_off.ensure(sizeof(long long) * (G + 1));
        HIPCHECK(hipMemcpyAsync(keep_psi.p, psi, sizeof(T) * m, hipMemcpyDeviceToDevice, stream));
        HIPCHECK(hipMemcpyAsync(keep_phic.p, phic, sizeof(T) * m, hipMemcpyDeviceToDevice, stream));
        HIPCHECK(hipMemcpyAsync(keep_lo.p, lo[L].p, sizeof(int) * 3 * G, hipMemcpyDeviceToDevice, stream));
        HIPCHECK(hipMemcpyAsync(keep_ext.p, ext[L].p, sizeof(int) * 3 * G, hipMemcpyDeviceToDevice, stream));
        HIPCHECK(hipMemcpyAsync(keep_alive.p, alive[L].p, sizeof(int) * G, hipMemcpyDeviceToDevice, stream));
        HIPCHECK(hipMemcpyAsync(keep_off.p, off[L].p, sizeof(long long) * (G + 1), hipMemcpyDeviceToDevice, stream));
        keep_tot = tot[L];
        keep_tot.arena = m;
    }

    // ---------------------------------------------------------------- queries
    void volumes(double *out) override {
        settle();
        HIPCHECK(hipMemcpyAsync(out, vol.p, sizeof(double) * G, hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
    }

    void labels(int32_t *out, bool device) override {
        ensure_phi();
        const long long nt3 = (long long)n[0] * n[1] * n[2];
        DBuf tmp;
        int32_t *dst = out;
        if (!device) {
            tmp.ensure(sizeof(int32_t) * nt3);
            dst = tmp.as<int32_t>();
        }
        hipLaunchKernelGGL(gg::k_labels<T>, dim3(ntiles), dim3(gg::kBlock), 0, stream, boxes_of(cur),
                           (const int *)cov_off.as<int>(), (const int *)cov_list.as<int>(),
                           (const T *)arena[a_phi].as<T>(), dst, tile_args());
        HIPCHECK(hipGetLastError());
        if (!device) {
            HIPCHECK(hipMemcpyAsync(out, dst, sizeof(int32_t) * nt3, hipMemcpyDeviceToHost, stream));
            HIPCHECK(hipStreamSynchronize(stream));
        }
    }

    void boxes(int32_t *hlo, int32_t *hext, int32_t *hal, int64_t *hoff, bool prev) override {
        settle();
        std::vector<int> a(G);
        std::vector<long long> o(G + 1);
        const void *plo = prev ? keep_lo.p : lo[cur].p, *pext = prev ? keep_ext.p : ext[cur].p;
        const void *pal = prev ? keep_alive.p : alive[cur].p, *poff = prev ? keep_off.p : off[cur].p;
        if (hlo) HIPCHECK(hipMemcpyAsync(hlo, plo, sizeof(int) * 3 * G, hipMemcpyDeviceToHost, stream));
        if (hext) HIPCHECK(hipMemcpyAsync(hext, pext, sizeof(int) * 3 * G, hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipMemcpyAsync(a.data(), pal, sizeof(int) * G, hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipMemcpyAsync(o.data(), poff, sizeof(long long) * (G + 1), hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
        for (int k = 0; k < G; ++k) {
            if (hal) hal[k] = a[k];
            if (hoff) hoff[k] = a[k] ? o[k] : -1;
        }
    }

    long long values(double *out, long long cap, int which) override {
        const T *src;
        long long m;
        if (which < 0) {
            ensure_phi();
            src = arena[a_phi].as<T>();
            m = tot[cur].arena;
        } else if (which == 2) {
            settle();
            if (!closest) throw ArgError{"closest-point weights need GG_FLAG_CLOSEST_POINT"};
            if (!psi_ok) predict_state();  // the weights of the state's next correction
            src = arena[A_SCR].as<T>();
            m = tot[cur].arena;
        } else {
            settle();
            if (!have_keep) throw ArgError{"no intermediates kept"};
            src = which == 0 ? keep_psi.as<T>() : keep_phic.as<T>();
            m = keep_tot.arena;
        }
        if (cap < m) return -m;
        DBuf tmp;
        tmp.ensure(sizeof(double) * std::max<long long>(m, 1));
        if (m > 0) {
            hipLaunchKernelGGL((gg::k_convert<T, double>), dim3(1024), dim3(256), 0, stream, src, tmp.as<double>(), m);
            HIPCHECK(hipGetLastError());
            HIPCHECK(hipMemcpyAsync(out, tmp.p, sizeof(double) * m, hipMemcpyDeviceToHost, stream));
        }
        HIPCHECK(hipStreamSynchronize(stream));
        return m;
    }

    long long iota(int32_t *out, long long cap) override {
        settle();
        const long long m = tot[cur].arena;
        if (cap < m) return -m;
        if (!physics) {
            for (long long i = 0; i < m; ++i) out[i] = -1;
            return m;
        }
        HIPCHECK(hipMemcpyAsync(out, iota_a[iota_cur].p, sizeof(int) * m, hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
        return m;
    }

    void load_state(const int32_t *hlo, const int32_t *hext, const uint8_t *hal, const double *vals,
                    const int32_t *hiota) override {
        settle();
        load_state_core(hlo, hext, hal, vals, hiota);
    }

    // State from host tables: values as doubles (any precision) or in the
    // stored type T (a checkpoint of this precision, taken over unchanged).
    template <typename V>
    void load_state_core(const int32_t *hlo, const int32_t *hext, const uint8_t *hal, const V *vals,
                         const int32_t *hiota) {
        std::vector<int> l(3 * G), e(3 * G), a(G);
        std::vector<long long> o(G + 1, 0);
        std::vector<double> vh(G, 0.0);
        int nalive = 0;
        for (int k = 0; k < G; ++k) {
            a[k] = hal[k] ? 1 : 0;
            nalive += a[k];
            for (int q = 0; q < 3; ++q) {
                l[3 * k + q] = a[k] ? hlo[3 * k + q] : 0;
                e[3 * k + q] = a[k] ? hext[3 * k + q] : 0;
            }
            if (a[k])
                for (int q = 0; q < 3; ++q) {
                    const int N = n[q], ex = e[3 * k + q];
                    if (l[3 * k + q] < 0 || l[3 * k + q] >= N || ex < 1 || ex > N ||
                        (ex != N && ex > N - 2 * P))
                        throw ArgError{"box of grain " + std::to_string(k) + " violates the box rule"};
                }
            o[k + 1] = o[k] + (a[k] ? (long long)e[3 * k] * e[3 * k + 1] * e[3 * k + 2] : 0);
        }
        const long long m = o[G];
        for (long long i = 0; i < m; ++i)
            if (!std::isfinite((double)vals[i])) throw ArgError{"non-finite value in the state"};
        for (int k = 0; k < G; ++k)
            if (a[k]) {
                double s = 0.0;
                for (long long i = o[k]; i < o[k + 1]; ++i) {
                    double c = (double)vals[i] + 0.5;
                    c = c < 0.0 ? 0.0 : (c > 1.0 ? 1.0 : c);
                    s += c;
                }
                vh[k] = s;
            }
        HIPCHECK(hipStreamSynchronize(stream));
        cur = 0;
        upload_table(0, l.data(), e.data(), a.data(), o.data());
        tot[0].arena = m;
        alive_n = nalive;
        ensure_arenas(m, 0u);
        std::vector<T> tv;
        const T *up;
        if constexpr (std::is_same<V, T>::value) {
            up = vals;
        } else {
            tv.resize(std::max<long long>(m, 1));
            for (long long i = 0; i < m; ++i) tv[i] = (T)vals[i];
            up = tv.data();
        }
        HIPCHECK(hipMemcpyAsync(arena[A_F].p, up, sizeof(T) * m, hipMemcpyHostToDevice, stream));
        HIPCHECK(hipMemcpyAsync(vol.p, vh.data(), sizeof(double) * G, hipMemcpyHostToDevice, stream));
        a_phi = A_F;
        f_chain = 0;
        psi_ok = false;
        have_keep = false;
        iota_cur = 0;
        if (physics) {
            std::vector<int> io(std::max<long long>(m, 1), -1);
            if (hiota)
                for (long long i = 0; i < m; ++i) io[i] = hiota[i];
            HIPCHECK(hipMemcpyAsync(iota_a[0].p, io.data(), sizeof(int) * m, hipMemcpyHostToDevice, stream));
        }
        HIPCHECK(hipStreamSynchronize(stream));
        build_coverage(0);
        HIPCHECK(hipStreamSynchronize(stream));
    }

    int alive_count() override {
        settle();
        return alive_n;
    }

    gg_step_stats stats() override {
        settle();
        gg_step_stats s;
        s.steps = steps_done;
        s.total_grain_voxels = total_gv;
        s.alive = alive_n;
        s.kernel_radius = R;
        s.grain_voxels = last_gv;
        s.capacity = cap_arena;
        s.superposition = (double)last_gv / ((double)n[0] * n[1] * n[2]);
        s.last_step_ms = last_ms;
        for (int a = 0; a < 3; ++a) s.n[a] = n[a];
        s.dim = dim;
        return s;
    }
};

}  // namespace

struct gg_sim {
    bool has_alloc = false;
    gg_allocator alloc{};  // the caller's allocator (has_alloc); declared before impl, so it outlives it
    void *stream = nullptr;
    std::unique_ptr<SimBase> impl;
    std::string err;
    bool poisoned = false;
    int G = 0;
    int n[3] = {0, 0, 0};
    int dim = 3, P = 1;
    int device = 0;
};

namespace {

thread_local std::string g_create_error;

// Device address of `scratch` on each device, taken once per device at set-up.
std::mutex g_scratch_mu;
double *g_scratch[kScratchDevices] = {};

// With `dev` current: take the device address of the scratch array (once).
hipError_t scratch_setup(int dev) {
    if (dev < 0 || dev >= kScratchDevices) return hipSuccess;  // no no-alloc calls there
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[dev]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = static_cast<double *>(p);
    return hipSuccess;
}

double *scratch_of(int dev) {
    if (dev < 0 || dev >= kScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch[dev];
}

gg_status fail(gg_sim *s, gg_status st, const std::string &msg) {
    if (s) {
        s->err = msg;
        if (st == GG_E_HIP) s->poisoned = true;
    } else {
        g_create_error = msg;
    }
    return st;
}

// Routes the thread's device allocations to the simulation's allocator for the
// duration of a call.
struct AllocScope {
    const gg_allocator *pa;
    void *ps;
    explicit AllocScope(gg_sim *s) : pa(t_alloc), ps(t_alloc_stream) {
        t_alloc = s && s->has_alloc ? &s->alloc : nullptr;
        t_alloc_stream = s ? s->stream : nullptr;
    }
    ~AllocScope() {
        t_alloc = pa;
        t_alloc_stream = ps;
    }
};

template <typename F> gg_status guarded(gg_sim *s, F &&f) {
    if (!s) return GG_E_ARG;
    if (s->poisoned) return fail(s, GG_E_POISONED, "simulation poisoned by an earlier HIP error: " + s->err);
    AllocScope scope(s);
    try {
        HIPCHECK(hipSetDevice(s->device));
        return f();
    } catch (const ArgError &e) {
        return fail(s, GG_E_ARG, e.msg);
    } catch (const CapError &e) {
        return fail(s, GG_E_CAPACITY, e.msg);
    } catch (const MemError &e) {
        return fail(s, GG_E_NOMEM, e.msg);
    } catch (const HipError &e) {
        return fail(s, GG_E_HIP, std::string(hipGetErrorString(e.err)) + " in " + e.where);
    } catch (const std::bad_alloc &) {
        return fail(s, GG_E_NOMEM, "host allocation failed");
    }
}

// Calls that wait for queued steps report their failures as state-changing
// failures: memory or capacity errors poison the simulation.
gg_status settled(gg_sim *sim, gg_status st) {
    if (st == GG_E_NOMEM || st == GG_E_CAPACITY) sim->poisoned = true;
    return st;
}

}  // namespace

extern "C" {

const char *gg_version(void) { return "gg-mi355x 0.2 (gfx950)"; }

const char *gg_status_str(gg_status st) {
    switch (st) {
    case GG_OK: return "ok";
    case GG_E_ARG: return "invalid argument";
    case GG_E_NOMEM: return "out of memory";
    case GG_E_HIP: return "HIP runtime error";
    case GG_E_CAPACITY: return "capacity exceeded";
    case GG_E_SMALLBUF: return "output buffer too small";
    case GG_E_NUMERIC: return "non-finite value";
    case GG_E_POISONED: return "simulation poisoned";
    case GG_E_UNSUPPORTED: return "unsupported";
    case GG_E_NODEVICE: return "no usable device";
    }
    return "unknown status";
}

const char *gg_last_error(const gg_sim *sim) { return sim ? sim->err.c_str() : g_create_error.c_str(); }

gg_status gg_create(const gg_config *cfg, const int32_t *labels, int32_t n_grains, const double *quat,
                    const double *energy_density, void *hip_stream, const gg_allocator *allocator,
                    gg_sim **out) {
    g_create_error.clear();
    if (!out) return fail(nullptr, GG_E_ARG, "out is NULL");
    *out = nullptr;
    if (!cfg || !labels) return fail(nullptr, GG_E_ARG, "cfg or labels is NULL");
    if (cfg->dim != 2 && cfg->dim != 3) return fail(nullptr, GG_E_ARG, "dim must be 2 or 3");
    for (int a = 0; a < 3; ++a)
        if (cfg->n[a] < 1 || cfg->n[a] > 4096) return fail(nullptr, GG_E_ARG, "grid size out of range [1, 4096]");
    if (cfg->dim == 2 && cfg->n[2] != 1) return fail(nullptr, GG_E_ARG, "2D requires n[2] == 1");
    if (!(cfg->band >= 1.0 && cfg->band <= gg::kMaxBand)) return fail(nullptr, GG_E_ARG, "band must be in [1, 16]");
    const int P = (int)std::ceil(cfg->band);
    for (int a = 0; a < cfg->dim; ++a)
        if (cfg->n[a] < 4 * P + 2) return fail(nullptr, GG_E_ARG, "grid must have at least 4P + 2 voxels per axis");
    if (cfg->precision == GG_MIXED_BF16 || cfg->precision == GG_MIXED_FP16)
        return fail(nullptr, GG_E_UNSUPPORTED, "BF16 / FP16 convolution operands are not built: use GG_FP32");
    if (cfg->precision != GG_FP64 && cfg->precision != GG_FP32)
        return fail(nullptr, GG_E_ARG, "precision must be a gg_precision value");
    if (cfg->physics < 0 || cfg->physics > 3) return fail(nullptr, GG_E_ARG, "unknown physics bits");
    if (cfg->redistance != GG_REDIST_TAXICAB && cfg->redistance != GG_REDIST_EUCLID)
        return fail(nullptr, GG_E_ARG, "redistance must be GG_REDIST_TAXICAB or GG_REDIST_EUCLID");
    if (cfg->batched != 0 && cfg->batched != 1) return fail(nullptr, GG_E_ARG, "batched must be 0 or 1");
    if (cfg->flags & ~(uint32_t)(GG_FLAG_ORDER_ID | GG_FLAG_CLOSEST_POINT))
        return fail(nullptr, GG_E_ARG, "unknown flag bits");
    if ((cfg->flags & GG_FLAG_CLOSEST_POINT) && !(cfg->physics & GG_PHYS_MISORIENTATION))
        return fail(nullptr, GG_E_ARG, "GG_FLAG_CLOSEST_POINT needs GG_PHYS_MISORIENTATION");
    if ((cfg->physics & GG_PHYS_MISORIENTATION) && (!quat || !(cfg->theta_c_deg > 0.0)))
        return fail(nullptr, GG_E_ARG, "misorientation weights need quat and theta_c_deg > 0");
    if ((cfg->physics & GG_PHYS_BULK) && (!energy_density || !(cfg->voxel_m > 0.0) || !(cfg->gamma_max > 0.0)))
        return fail(nullptr, GG_E_ARG, "bulk energy needs energy_density, voxel_m > 0 and gamma_max > 0");
    if (n_grains < 1) return fail(nullptr, GG_E_ARG, "n_grains must be >= 1");
    const long long nt3 = (long long)cfg->n[0] * cfg->n[1] * cfg->n[2];
    // box offsets inside a grain's arena are 32-bit
    if (nt3 > 2147483647LL) return fail(nullptr, GG_E_ARG, "grid must have fewer than 2^31 voxels");
    for (long long i = 0; i < nt3; ++i)
        if (labels[i] < 0 || labels[i] >= n_grains) return fail(nullptr, GG_E_ARG, "label out of [0, n_grains)");
    if (quat && (cfg->physics & GG_PHYS_MISORIENTATION))
        for (long long i = 0; i < 4LL * n_grains; ++i)
            if (!std::isfinite(quat[i])) return fail(nullptr, GG_E_ARG, "non-finite quaternion");
    if (energy_density && (cfg->physics & GG_PHYS_BULK))
        for (int k = 0; k < n_grains; ++k)
            if (!std::isfinite(energy_density[k])) return fail(nullptr, GG_E_ARG, "non-finite energy density");
    if (allocator && (!allocator->alloc || !allocator->free))
        return fail(nullptr, GG_E_ARG, "allocator needs both alloc and free");
    if (allocator && !hip_stream) return fail(nullptr, GG_E_ARG, "an allocator needs the caller's stream");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return fail(nullptr, GG_E_NODEVICE, "no HIP device");
    }
    std::unique_ptr<gg_sim> s(new (std::nothrow) gg_sim());
    if (!s) return fail(nullptr, GG_E_NOMEM, "host allocation failed");
    if (allocator) {
        s->has_alloc = true;
        s->alloc = *allocator;
    }
    s->G = n_grains;
    for (int a = 0; a < 3; ++a) s->n[a] = cfg->n[a];
    s->dim = cfg->dim;
    s->P = (int)std::ceil(cfg->band);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    s->device = dev;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail(nullptr, GG_E_NODEVICE, "device query failed");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, GG_E_NODEVICE, std::string("device is ") + prop.gcnArchName + ", not gfx950");
    {
        const hipError_t e = scratch_setup(dev);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(nullptr, GG_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
    }
    s->stream = hip_stream;
    AllocScope scope(s.get());
    try {
        if (cfg->precision == GG_FP64) {
            auto *p = new Sim<double>(*cfg, n_grains, (hipStream_t)hip_stream);
            s->impl.reset(p);
            p->create(labels, quat, energy_density);
        } else {
            auto *p = new Sim<float>(*cfg, n_grains, (hipStream_t)hip_stream);
            s->impl.reset(p);
            p->create(labels, quat, energy_density);
        }
    } catch (const ArgError &e) {
        return fail(nullptr, GG_E_ARG, e.msg);
    } catch (const CapError &e) {
        return fail(nullptr, GG_E_CAPACITY, e.msg);
    } catch (const MemError &e) {
        return fail(nullptr, GG_E_NOMEM, e.msg);
    } catch (const HipError &e) {
        return fail(nullptr, GG_E_HIP, std::string(hipGetErrorString(e.err)) + " in " + e.where);
    } catch (const std::bad_alloc &) {
        return fail(nullptr, GG_E_NOMEM, "host allocation failed");
    }
    *out = s.release();
    return GG_OK;
}

gg_status gg_step(gg_sim *sim, double dt, int32_t n_steps) {
    if (!sim) return GG_E_ARG;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(sim, GG_E_ARG, "dt must be finite and positive");
    if (n_steps < 0) return fail(sim, GG_E_ARG, "n_steps must be >= 0");
    return settled(sim, guarded(sim, [&]() {
                       sim->impl->step(dt, n_steps);
                       return GG_OK;
                   }));
}

gg_status gg_sync(gg_sim *sim) {
    return settled(sim, guarded(sim, [&]() {
                       sim->impl->sync();
                       return GG_OK;
                   }));
}

gg_status gg_grain_count(gg_sim *sim, int32_t *alive) {
    if (!alive) return fail(sim, GG_E_ARG, "alive is NULL");
    return settled(sim, guarded(sim, [&]() {
                       *alive = sim->impl->alive_count();
                       return GG_OK;
                   }));
}

gg_status gg_grain_volumes(gg_sim *sim, double *out, int64_t cap) {
    if (!sim || !out) return fail(sim, GG_E_ARG, "NULL argument");
    if (cap < sim->G) return fail(sim, GG_E_SMALLBUF, "cap < n_grains");
    return settled(sim, guarded(sim, [&]() {
                       sim->impl->volumes(out);
                       return GG_OK;
                   }));
}

gg_status gg_labels(gg_sim *sim, int32_t *out, int64_t cap, int32_t out_is_device) {
    if (!sim || !out) return fail(sim, GG_E_ARG, "NULL argument");
    if (cap < (int64_t)sim->n[0] * sim->n[1] * sim->n[2]) return fail(sim, GG_E_SMALLBUF, "cap < prod(n)");
    return settled(sim, guarded(sim, [&]() {
                       sim->impl->labels(out, out_is_device != 0);
                       return GG_OK;
                   }));
}

gg_status gg_stats(gg_sim *sim, gg_step_stats *out) {
    if (!sim || !out) return fail(sim, GG_E_ARG, "NULL argument");
    return settled(sim, guarded(sim, [&]() {
                       *out = sim->impl->stats();
                       return GG_OK;
                   }));
}

gg_status gg_get_boxes(gg_sim *sim, int32_t *lo, int32_t *ext, int32_t *alive, int64_t *offset, int64_t cap) {
    if (!sim) return GG_E_ARG;
    if (cap < sim->G) return fail(sim, GG_E_SMALLBUF, "cap < n_grains");
    return settled(sim, guarded(sim, [&]() {
                       sim->impl->boxes(lo, ext, alive, offset, false);
                       return GG_OK;
                   }));
}

gg_status gg_get_values(gg_sim *sim, double *out, int64_t cap) {
    if (!sim || !out) return fail(sim, GG_E_ARG, "NULL argument");
    return settled(sim, guarded(sim, [&]() {
                       long long m = sim->impl->values(out, cap, -1);
                       if (m < 0)
                           return fail(sim, GG_E_SMALLBUF, "cap < sum of box volumes (" + std::to_string(-m) + ")");
                       return GG_OK;
                   }));
}

gg_status gg_get_iota(gg_sim *sim, int32_t *out, int64_t cap) {
    if (!sim || !out) return fail(sim, GG_E_ARG, "NULL argument");
    return settled(sim, guarded(sim, [&]() {
                       long long m = sim->impl->iota(out, cap);
                       if (m < 0) return fail(sim, GG_E_SMALLBUF, "cap < sum of box volumes");
                       return GG_OK;
                   }));
}

gg_status gg_load_state(gg_sim *sim, const int32_t *lo, const int32_t *ext, const uint8_t *alive,
                        const double *values, const int32_t *iota) {
    if (!sim || !lo || !ext || !alive || !values) return fail(sim, GG_E_ARG, "NULL argument");
    return settled(sim, guarded(sim, [&]() {
                       sim->impl->load_state(lo, ext, alive, values, iota);
                       return GG_OK;
                   }));
}

gg_status gg_grain_areas(gg_sim *sim, double *area, double *weighted, int64_t cap) {
    if (!sim || !area) return fail(sim, GG_E_ARG, "NULL argument");
    if (cap < sim->G) return fail(sim, GG_E_SMALLBUF, "cap < n_grains");
    return settled(sim, guarded(sim, [&]() {
                       sim->impl->areas(area, weighted);
                       return GG_OK;
                   }));
}

gg_status gg_grain_areas_noalloc(gg_sim *sim, double *area_dev, double *weighted_dev, int64_t cap) {
    if (!sim || !area_dev) return fail(sim, GG_E_ARG, "NULL argument");
    if (cap < sim->G) return fail(sim, GG_E_SMALLBUF, "cap < n_grains");
    if (sim->G > kNoAllocMaxGrains)
        return fail(sim, GG_E_CAPACITY, "n_grains exceeds the 65536 grains of the no-alloc scratch");
    double *part = scratch_of(sim->device);
    if (!part) return fail(sim, GG_E_UNSUPPORTED, "no no-alloc scratch on this device (index >= 64)");
    return guarded(sim, [&]() {
        if (!sim->impl->areas_noalloc(part, area_dev, weighted_dev))
            return fail(sim, GG_E_CAPACITY,
                        "a queued step awaits a retake with larger buffers: call gg_sync first");
        return GG_OK;
    });
}

gg_status gg_grain_sdf(gg_sim *sim, int32_t id, int32_t lo[3], int32_t ext[3], double *out, int64_t cap) {
    if (!sim || !lo || !ext) return fail(sim, GG_E_ARG, "NULL argument");
    if (id < 0 || id >= sim->G) return fail(sim, GG_E_ARG, "grain id out of range");
    return settled(sim, guarded(sim, [&]() {
                       const long long m = sim->impl->grain_sdf(id, lo, ext, out, cap);
                       if (m < 0 && out) return fail(sim, GG_E_SMALLBUF, "cap too small (" + std::to_string(-m) + ")");
                       return GG_OK;
                   }));
}

gg_status gg_autotune(gg_sim *sim, double dt, int32_t steps_per_candidate, gg_tuning *out) {
    if (!sim || !out) return fail(sim, GG_E_ARG, "NULL argument");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(sim, GG_E_ARG, "dt must be finite and positive");
    if (steps_per_candidate < 1) return fail(sim, GG_E_ARG, "steps_per_candidate must be >= 1");
    return settled(sim, guarded(sim, [&]() {
                       Tuning t{};
                       sim->impl->autotune(dt, steps_per_candidate, &t);
                       std::memset(out, 0, sizeof(*out));
                       out->order_size = t.order_size;
                       out->lds_bytes = t.lds_bytes;
                       out->small_bytes = t.small_bytes;
                       out->candidates = t.candidates;
                       for (int i = 0; i < 8; ++i) {
                           out->ns_per_gv[i] = t.ns_per_gv[i];
                           out->cand_order[i] = t.cand_order[i];
                           out->cand_lds[i] = t.cand_lds[i];
                           out->cand_small[i] = t.cand_small[i];
                       }
                       return GG_OK;
                   }));
}

gg_status gg_save(gg_sim *sim, const char *path) {
    if (!sim || !path) return fail(sim, GG_E_ARG, "NULL argument");
    return settled(sim, guarded(sim, [&]() {
                       FILE *f = std::fopen(path, "wb");
                       if (!f) return fail(sim, GG_E_ARG, std::string("cannot open ") + path + " for writing");
                       try {
                           sim->impl->save(f);
                       } catch (...) {
                           std::fclose(f);
                           throw;
                       }
                       if (std::fclose(f) != 0) return fail(sim, GG_E_ARG, std::string("write to ") + path + " failed");
                       return GG_OK;
                   }));
}

gg_status gg_load(gg_sim *sim, const char *path) {
    if (!sim || !path) return fail(sim, GG_E_ARG, "NULL argument");
    return settled(sim, guarded(sim, [&]() {
                       FILE *f = std::fopen(path, "rb");
                       if (!f) return fail(sim, GG_E_ARG, std::string("cannot open ") + path);
                       try {
                           sim->impl->load(f);
                       } catch (...) {
                           std::fclose(f);
                           throw;
                       }
                       std::fclose(f);
                       sim->impl->grid(sim->n);
                       return GG_OK;
                   }));
}

gg_status gg_coarsen(gg_sim *sim, const int32_t n_new[3]) {
    if (!sim || !n_new) return fail(sim, GG_E_ARG, "NULL argument");
    const int dim = sim->dim;
    if (dim == 2 && n_new[2] != 1) return fail(sim, GG_E_ARG, "2D requires n_new[2] == 1");
    for (int a = 0; a < dim; ++a) {
        if (n_new[a] < 4 * sim->P + 2 || n_new[a] > sim->n[a])
            return fail(sim, GG_E_ARG, "n_new must lie in [4P + 2, n] on every axis");
        if ((long long)n_new[a] * sim->n[0] != (long long)n_new[0] * sim->n[a])
            return fail(sim, GG_E_ARG, "n_new must keep the ratio n / n_new equal on every axis");
    }
    gg_status st = guarded(sim, [&]() {
        sim->impl->coarsen(n_new);
        return GG_OK;
    });
    if (st == GG_OK)
        for (int a = 0; a < 3; ++a) sim->n[a] = n_new[a];
    return settled(sim, st);
}

gg_status gg_keep_intermediates(gg_sim *sim, int32_t on) {
    return settled(sim, guarded(sim, [&]() {
                       sim->impl->set_keep(on != 0);
                       return GG_OK;
                   }));
}

gg_status gg_get_intermediate(gg_sim *sim, int32_t which, double *out, int64_t cap, int32_t *lo, int32_t *ext,
                              int32_t *alive, int64_t *offset, int64_t cap_grains) {
    if (!sim || !out || which < 0 || which > 2) return fail(sim, GG_E_ARG, "bad argument");
    if ((lo || ext || alive || offset) && cap_grains < sim->G) return fail(sim, GG_E_SMALLBUF, "cap_grains < n_grains");
    return settled(sim, guarded(sim, [&]() {
                       long long m = sim->impl->values(out, cap, which);
                       if (m < 0) return fail(sim, GG_E_SMALLBUF, "cap too small (" + std::to_string(-m) + ")");
                       if (lo || ext || alive || offset) sim->impl->boxes(lo, ext, alive, offset, which != 2);
                       return GG_OK;
                   }));
}

gg_status gg_profile(gg_sim *sim, int32_t on) {
    return settled(sim, guarded(sim, [&]() {
                       sim->impl->profile(on != 0);
                       return GG_OK;
                   }));
}

gg_status gg_get_kernel_times(gg_sim *sim, gg_kernel_times *out) {
    if (!sim || !out) return fail(sim, GG_E_ARG, "NULL argument");
    return settled(sim, guarded(sim, [&]() {
                       *out = sim->impl->kernel_times();
                       return GG_OK;
                   }));
}

void gg_destroy(gg_sim *sim) {
    if (!sim) return;
    (void)hipSetDevice(sim->device);
    delete sim;
}

}  // extern "C"
