// Host side of the MI355X level-set grain-growth library: the C ABI declared
// in include/gg.h, device memory ownership, and the per-step launch sequence
//   predictor (xy, z) -> corrector (global tiles) -> box plan + item/coverage
//   bookkeeping -> re-initialization (xy, z) into the new box layout -> volumes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <type_traits>
#include <memory>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/gg.h"
#include "gg_kernels.hpp"

// Corrector tile of the 3D grid (powers of two, 512 voxels).
#ifndef GG_CMP_TILE_X
#define GG_CMP_TILE_X 16
#define GG_CMP_TILE_Y 8
#define GG_CMP_TILE_Z 4
#endif

namespace {

using gg::Boxes;
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
    template <typename U> U *as() const { return reinterpret_cast<U *>(p); }
};

int pow2_divisor(int N, int target) {
    int t = target;
    while (t > 1 && N % t) t >>= 1;
    return t;
}

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
    virtual long long grain_sdf(int k, int32_t *lo, int32_t *ext, double *out, long long cap) = 0;
    virtual void save(FILE *f) = 0;
    virtual void load(FILE *f) = 0;
    virtual void grid(int32_t *n) const = 0;
    virtual void autotune(double dt, int per, int32_t *best_lds, int32_t *best_small) = 0;
    virtual void sync() = 0;
    virtual int alive_count() const = 0;
    virtual gg_step_stats stats() const = 0;
    virtual long long arena_total(bool prev) const = 0;
    virtual void profile(bool on) = 0;
    virtual gg_kernel_times kernel_times() const = 0;
    bool keep = false;
};

template <typename T> struct Sim final : SimBase {
    // configuration
    int dim, G, n[3], P, K;
    int redist, K_euclid;  // re-initialization scheme of the steps; its Jacobi sweep count
    T W;
    double band_d;  // W as given
    // LDS budget of a work group and limit of the small launch class (FP32
    // bytes; FP64 tiles get the same values), tunable (gg_autotune)
    int lds_bytes = gg::kLdsBytes, small_bytes = gg::kSmallLdsBytes;
    int physics;
    double theta_c, voxel_m, gamma_max, headroom;
    int tdim[3], nt[3], ntiles, occ_words;
    hipStream_t stream = nullptr;
    bool own_stream = false;

    // layouts 0/1: box tables and work items
    DBuf lo[2], ext[2], alive[2], off[2];
    DBuf ipref[2], iowner[2][gg::kKinds * gg::kClasses], itile[2];
    int items_R[2] = {-1, -1};
    Totals tot[2];
    int cur = 0;

    // per step accumulators and scratch
    DBuf bmin, bmax, occ, sizes, cnt, ldsmax, vol, vol_part;
    DBuf cov_cnt, cov_off, cov_cur, cov_list;
    DBuf taps_d, quat_d, energy_d, totals_d;
    Totals *totals_h = nullptr;
    // value arenas and their roles for the current layout (-1: not held)
    DBuf arena[4], iota_a[2];
    int a_state = -1;  // phi, materialised
    int a_T = -1;      // z pass of the predictor applied to phi (3D), radius T_R
    int a_psi = -1;    // predicted function psi, radius psi_R
    int T_R = -1, psi_R = -1;
    int iota_cur = 0;  // ID-field of the current layout
    // kept intermediates (test hook)
    DBuf keep_psi, keep_phic, keep_lo, keep_ext, keep_alive, keep_off;
    Totals keep_tot{};
    bool have_keep = false;

    // current Gaussian
    double sigma = -1.0;
    int R = 0;
    std::vector<T> taps_h;

    long long steps_done = 0;
    double last_ms = 0.0;
    long long last_gv = 0;
    long long total_gv = 0;

    // per-kernel timing: HIP event pairs on the simulation's stream
    struct Span {
        hipEvent_t a, b;
        int cls;
        long long vox;
        int n;  // kernel dispatches in the span
    };
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<Span> spans;
    gg_kernel_times ktimes{};

    hipEvent_t next_event() {
        if (ev_used == ev_pool.size()) {
            hipEvent_t e;
            HIPCHECK(hipEventCreate(&e));
            ev_pool.push_back(e);
        }
        return ev_pool[ev_used++];
    }
    void tbegin(int cls, long long vox) {
        if (!prof) return;
        Span sp{next_event(), nullptr, cls, vox, 1};
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
        ev_used = 0;
    }
    void profile(bool on) override {
        resolve_spans();
        prof = on;
        std::memset(&ktimes, 0, sizeof(ktimes));
    }
    gg_kernel_times kernel_times() const override { return ktimes; }

    const int4 *tiles_of(int l, int kind) const { return itile[l].as<int4>() + (size_t)kind * 2 * G; }
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
        headroom = c.capacity_headroom > 1.0 ? c.capacity_headroom : 1.25;
        set_tiles();
        // occupancy rows keep this width when the grid is coarsened
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
            if (totals_h) (void)hipHostFree(totals_h);
            totals_h = nullptr;
            if (own_stream && stream) (void)hipStreamDestroy(stream);
            stream = nullptr;
            throw;
        }
    }

    void allocate_tables() {
        HIPCHECK(hipHostMalloc((void **)&totals_h, sizeof(Totals), hipHostMallocDefault));
        std::memset(totals_h, 0, sizeof(Totals));
        for (int l = 0; l < 2; ++l) {
            lo[l].ensure(sizeof(int) * 3 * G);
            ext[l].ensure(sizeof(int) * 3 * G);
            alive[l].ensure(sizeof(int) * G);
            off[l].ensure(sizeof(long long) * (G + 1));
            ipref[l].ensure(sizeof(long long) * 3 * gg::kKinds * (size_t)(G + 1));
            itile[l].ensure(sizeof(int4) * 2 * gg::kKinds * (size_t)G);
        }
        bmin.ensure(sizeof(int) * 3 * G);
        bmax.ensure(sizeof(int) * 3 * G);
        occ.ensure(sizeof(unsigned) * 3 * (size_t)G * occ_words);
        HIPCHECK(hipMemsetAsync(occ.p, 0, occ.cap, stream));
        std::vector<int> init_min(3 * G, 0x7fffffff), init_max(3 * G, -1);
        HIPCHECK(hipMemcpyAsync(bmin.p, init_min.data(), sizeof(int) * 3 * G, hipMemcpyHostToDevice, stream));
        HIPCHECK(hipMemcpyAsync(bmax.p, init_max.data(), sizeof(int) * 3 * G, hipMemcpyHostToDevice, stream));
        sizes.ensure(sizeof(long long) * G);
        cnt.ensure(sizeof(long long) * 3 * gg::kKinds * (size_t)G);
        ldsmax.ensure(sizeof(unsigned long long) * gg::kKinds * gg::kClasses);
        vol.ensure(sizeof(double) * G);
        cov_cnt.ensure(sizeof(int) * ntiles);
        cov_off.ensure(sizeof(int) * (ntiles + 1));
        cov_cur.ensure(sizeof(int) * (ntiles + 1));
        taps_d.ensure(sizeof(T) * (2 * gg::kMaxRadius + 1));
        totals_d.ensure(sizeof(Totals));
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
            tdim[1] = pow2_divisor(n[1], 16);
            tdim[2] = 1;
        }
        ntiles = 1;
        for (int a = 0; a < 3; ++a) {
            nt[a] = n[a] / tdim[a];
            ntiles *= nt[a];
        }
    }

    // Switch to the periodic grid np (coarsening, checkpoint of a coarsened run).
    void set_grid(const int *np) {
        for (int a = 0; a < 3; ++a) n[a] = np[a];
        set_tiles();
        cov_cnt.ensure(sizeof(int) * ntiles);
        cov_off.ensure(sizeof(int) * (ntiles + 1));
        cov_cur.ensure(sizeof(int) * (ntiles + 1));
    }
    void grid(int32_t *out) const override {
        for (int a = 0; a < 3; ++a) out[a] = n[a];
    }

    ~Sim() override {
        if (stream) (void)hipStreamSynchronize(stream);
        DBuf *all[] = {&bmin, &bmax, &occ, &sizes, &ldsmax, &vol, &vol_part, &cov_cnt, &cov_off, &cov_cur,
                       &cov_list, &taps_d, &quat_d, &energy_d, &totals_d, &keep_psi, &keep_phic, &keep_lo,
                       &keep_ext, &keep_alive, &keep_off};
        for (DBuf *b : all) b->release();
        cnt.release();
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
        if (totals_h) (void)hipHostFree(totals_h);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }

    void sync() override { HIPCHECK(hipStreamSynchronize(stream)); }

    // Arena capacity for a layout of `need` values (with headroom).
    size_t grow_to(long long need) const { return (size_t)((double)need * headroom) + 1024; }

    void ensure_arena(int a, long long need) {
        if ((size_t)need * sizeof(T) <= arena[a].cap && arena[a].p) return;
        arena[a].ensure(grow_to(need) * sizeof(T));
    }
    // First arena outside `excl` (bit mask of arenas holding live data) with room
    // for `need` values; grows a dead one when none has room.
    int pick(unsigned excl, long long need) {
        for (int a = 0; a < 4; ++a)
            if (!(excl >> a & 1u) && arena[a].p && (size_t)need * sizeof(T) <= arena[a].cap) return a;
        for (int a = 0; a < 4; ++a)
            if (!(excl >> a & 1u)) {
                ensure_arena(a, need);
                return a;
            }
        throw CapError{"no free value arena"};
    }
    static unsigned bit(int a) { return a >= 0 ? 1u << a : 0u; }

    void ensure_iota(int a, long long need) {
        if ((size_t)need * sizeof(int) <= iota_a[a].cap && iota_a[a].p) return;
        iota_a[a].ensure(grow_to(need) * sizeof(int));
    }

    // Offsets, work items and coverage counts of layout l; fills tot[l] (syncs).
    // Then the item maps and the coverage lists.
    void layout_meta_count(int l, bool coverage) {
        Boxes L = boxes_of(l);
        tbegin(GG_K_PLAN, 0);
        HIPCHECK(hipMemsetAsync(ldsmax.p, 0, sizeof(unsigned long long) * gg::kKinds * gg::kClasses, stream));
        const int tb = 256, gb = (G + tb - 1) / tb;
        hipLaunchKernelGGL(gg::k_item_counts, dim3(gb, gg::kKinds), dim3(tb), 0, stream, L, cnt.as<long long>(), itile[l].as<int4>(),
                           ldsmax.as<unsigned long long>(), R, K, G, gg::budget_values<T>(lds_bytes),
                           gg::budget_values<T>(small_bytes), redist == GG_REDIST_EUCLID ? 1 : 0);
        hipLaunchKernelGGL(gg::k_scan_multi, dim3(3 * gg::kKinds), dim3(1024), 0, stream, cnt.as<long long>(),
                           ipref[l].as<long long>(), G);
        if (coverage) {
            HIPCHECK(hipMemsetAsync(cov_cnt.p, 0, sizeof(int) * ntiles, stream));
            hipLaunchKernelGGL(gg::k_coverage, dim3(G), dim3(64), 0, stream, L, cov_cnt.as<int>(), (int *)nullptr,
                               tile_args(), G, 0);
            hipLaunchKernelGGL(gg::k_scan_int, dim3(1), dim3(1024), 0, stream, cov_cnt.as<int>(), cov_off.as<int>(),
                               ntiles);
        }
        hipLaunchKernelGGL(gg::k_totals, dim3(1), dim3(256), 0, stream, L.off, ipref[l].as<long long>(),
                           coverage ? cov_off.as<int>() : (const int *)nullptr, ntiles, L.alive, G,
                           ldsmax.as<unsigned long long>(), totals_d.as<Totals>());
        HIPCHECK(hipGetLastError());
        tend();
        HIPCHECK(hipMemcpyAsync(totals_h, totals_d.p, sizeof(Totals), hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
        const long long keep_cov = tot[l].cov;
        tot[l] = *totals_h;
        if (!coverage) tot[l].cov = keep_cov;
        for (int q = 0; q < gg::kKinds; ++q)
            for (int c = 0; c < gg::kClasses; ++c)
                if (tot[l].lds[q][c] < 0 || tot[l].lds[q][c] > gg::budget_values<T>(lds_bytes))
                    throw CapError{"a box is too large for the stencil tiling"};
        items_R[l] = R;
    }

    void layout_meta_fill(int l, bool coverage) {
        gg::OwnerMaps om;
        for (int q = 0; q < gg::kKinds; ++q)
            for (int c = 0; c < gg::kClasses; ++c) {
                DBuf &b = iowner[l][q * gg::kClasses + c];
                b.ensure(sizeof(int) * (size_t)std::max<long long>(tot[l].items[q][1 + c], 1) * 5 / 4);
                om.owner[q * gg::kClasses + c] = b.as<int>();
            }
        if (coverage) {
            if (tot[l].cov > 0x7fffffffLL) throw CapError{"coverage list exceeds 2^31 entries"};
            cov_list.ensure(sizeof(int) * (size_t)std::max<long long>(tot[l].cov, 1) * 5 / 4);
        }
        tbegin(GG_K_PLAN, 0);
        hipLaunchKernelGGL(gg::k_fill_owner, dim3(G, gg::kKinds * gg::kClasses), dim3(64), 0, stream,
                           ipref[l].as<long long>(), om, G);
        if (coverage) {
            HIPCHECK(hipMemcpyAsync(cov_cur.p, cov_off.p, sizeof(int) * (ntiles + 1), hipMemcpyDeviceToDevice,
                                    stream));
            hipLaunchKernelGGL(gg::k_coverage, dim3(G), dim3(64), 0, stream, boxes_of(l), cov_cur.as<int>(),
                               cov_list.as<int>(), tile_args(), G, 1);
        }
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
        r.tilings = tiles_of(l, kind);
        r.n = tot[l].items[kind][1 + cls];
        return r;
    }

    void set_gaussian(double dt) {
        double s = std::sqrt(2.0 * dt) * (double)n[0];
        if (s == sigma) return;
        int r = (int)std::ceil(4.0 * s - 1e-9);
        if (r < 1) r = 1;
        if (r > gg::kMaxRadius || r > 2 * P) throw ArgError{"kernel radius R = ceil(4 sigma) exceeds min(24, 2P)"};
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
    }

    gg::Physics<T> physics_args(const T *phi, const int *iota_p) const {
        gg::Physics<T> ph;
        ph.mode = physics;
        ph.quat = quat_d.as<T>();
        ph.energy = energy_d.as<T>();
        ph.theta_c_deg = (T)theta_c;
        ph.bulk_scale = (physics & 2) ? (T)(sigma * sigma * voxel_m / (2.0 * gamma_max)) : T(0);
        ph.phi = phi;
        ph.iota = iota_p;
        return ph;
    }

    static unsigned grid_of(long long items) { return (unsigned)items; }

    // Predictor x and y passes (+ correction epilogue) on layout l: src -> dst.
    void launch_conv_xy(int l, const T *src, T *dst, const gg::Physics<T> &ph) {
        const Totals &t = tot[l];
        if (t.items[gg::KIND_CXY][0] <= 0) return;
        tbegin(GG_K_CONV_XY, t.arena);
        int nd = 0;
        for (int c = 0; c < gg::kClasses; ++c) {
            const gg::ItemRefs ir = refs(l, gg::KIND_CXY, c);
            if (ir.n <= 0) continue;
            ++nd;
            const dim3 gr(grid_of(gg::xcd_grid(ir.n))), bl(gg::kBlock);
            const size_t lds = sizeof(T) * t.lds[gg::KIND_CXY][c];
            auto args = std::make_tuple(boxes_of(l), ir, src, dst, (const T *)taps_d.as<T>(), R, W, grid_args(), ph);
            auto go = [&](auto kern) {
                std::apply([&](auto... a) { hipLaunchKernelGGL(kern, gr, bl, lds, stream, a...); }, args);
            };
            if (ph.mode) {
                if (R == 6) go(gg::k_conv_xy<T, 6, true>);
                else if (R == 8) go(gg::k_conv_xy<T, 8, true>);
                else go(gg::k_conv_xy<T, 0, true>);
            } else if (R == 6) go(gg::k_conv_xy<T, 6, false>);
            else if (R == 8) go(gg::k_conv_xy<T, 8, false>);
            else go(gg::k_conv_xy<T, 0, false>);
        }
        tend(nd);
        HIPCHECK(hipGetLastError());
    }

    // Predictor z pass alone on layout l (3D): src -> dst.
    void launch_conv_z(int l, const T *src, T *dst) {
        const Totals &t = tot[l];
        if (t.items[gg::KIND_CZ][0] <= 0) return;
        tbegin(GG_K_CONV_Z, t.arena);
        int nd = 0;
        for (int c = 0; c < gg::kClasses; ++c) {
            const gg::ItemRefs ir = refs(l, gg::KIND_CZ, c);
            if (ir.n <= 0) continue;
            ++nd;
            hipLaunchKernelGGL(gg::k_conv_z<T>, dim3(grid_of(gg::xcd_grid(ir.n))), dim3(gg::kBlock),
                               sizeof(T) * t.lds[gg::KIND_CZ][c], stream, boxes_of(l), ir, src, dst, taps_d.as<T>(), R,
                               W, grid_args());
        }
        tend(nd);
        HIPCHECK(hipGetLastError());
    }

    // Re-initialization of phi^c (layout lo_l) into layout ln_l.  2D: the final
    // function goes to `phi`.  3D: partial distances to `d2`, then the fused z
    // sweep writes phi (when `phi` is not null) and the predictor z pass to `t`.
    // Euclidean variant: reference values to `d2`, then K_euclid Jacobi sweeps
    // between `d2` and `tz` (an even count: the result is back in `d2`; 2D: the
    // last sweep writes `phi`), and in 3D the fused kernel without its z sweep.
    void launch_reinit(int lo_l, int ln_l, const T *phic, T *d2, T *phi, T *tz, const int *iota_old, int *iota_new,
                       bool euclid) {
        const Totals &t = tot[ln_l];
        const gg::GridArgs g = grid_args();
        const int vk = dim == 3 ? gg::KIND_ZF : (euclid ? gg::KIND_JAC : gg::KIND_RXY);
        vol_part.ensure(sizeof(double) * (size_t)std::max<long long>(t.items[vk][0], 1) * 5 / 4);
        if (t.items[gg::KIND_RXY][0] > 0) {
            tbegin(GG_K_REINIT_XY, t.arena);
            int nd = 0;
            T *out = dim == 3 || euclid ? d2 : phi;
            for (int c = 0; c < gg::kClasses; ++c) {
                const gg::ItemRefs ir = refs(ln_l, gg::KIND_RXY, c);
                if (ir.n <= 0) continue;
                ++nd;
                hipLaunchKernelGGL(gg::k_reinit_xy<T>, dim3(grid_of(gg::xcd_grid(ir.n))), dim3(gg::kBlock),
                                   sizeof(T) * t.lds[gg::KIND_RXY][c], stream, boxes_of(lo_l), boxes_of(ln_l), ir,
                                   phic, out, iota_old, iota_new, vol_part.as<double>(), euclid ? 0 : K, W,
                                   euclid ? 1 : 0, g);
            }
            tend(nd);
            if (euclid) {
                tbegin(GG_K_REINIT_SWEEP, t.arena);
                nd = 0;
                T *a = d2, *b = tz;
                for (int s = 0; s < K_euclid; ++s) {
                    const bool fin = dim == 2 && s == K_euclid - 1;
                    T *dst = fin ? phi : b;
                    for (int c = 0; c < gg::kClasses; ++c) {
                        const gg::ItemRefs ir = refs(ln_l, gg::KIND_JAC, c);
                        if (ir.n <= 0) continue;
                        ++nd;
                        hipLaunchKernelGGL(gg::k_jacobi<T>, dim3(grid_of(gg::xcd_grid(ir.n))), dim3(gg::kBlock),
                                           sizeof(T) * t.lds[gg::KIND_JAC][c], stream, boxes_of(ln_l), ir,
                                           (const T *)a, dst, vol_part.as<double>(), W, fin ? 1 : 0, g);
                    }
                    std::swap(a, b);
                }
                tend(nd);
            }
        }
        if (dim == 3 && t.items[gg::KIND_ZF][0] > 0) {
            tbegin(GG_K_REINIT_Z, t.arena);
            int nd = 0;
            for (int c = 0; c < gg::kClasses; ++c) {
                const gg::ItemRefs ir = refs(ln_l, gg::KIND_ZF, c);
                if (ir.n <= 0) continue;
                ++nd;
                const dim3 gr(grid_of(gg::xcd_grid(ir.n))), bl(gg::kBlock);
                const size_t lds = sizeof(T) * t.lds[gg::KIND_ZF][c];
                auto args = std::make_tuple(boxes_of(ln_l), ir, (const T *)d2, phi, tz, vol_part.as<double>(),
                                            (const T *)taps_d.as<T>(), euclid ? 0 : K, R, W, euclid ? 0 : 1, g);
                auto go = [&](auto kern) {
                    std::apply([&](auto... a) { hipLaunchKernelGGL(kern, gr, bl, lds, stream, a...); }, args);
                };
                if (R == 6) go(gg::k_zfused<T, 6>);
                else if (R == 8) go(gg::k_zfused<T, 8>);
                else go(gg::k_zfused<T, 0>);
            }
            tend(nd);
        }
        tbegin(GG_K_VOLUME, t.arena);
        hipLaunchKernelGGL(gg::k_volumes, dim3(G), dim3(64), 0, stream, boxes_of(ln_l), pref_of(ln_l, vk, 0),
                           vol_part.as<double>(), vol.as<double>(), G);
        tend();
        HIPCHECK(hipGetLastError());
    }

    // ---------------------------------------------------------------- create
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
        for (int k = 0; k < G; ++k)
            hoff[k + 1] = hoff[k] + (hal[k] ? (long long)hext[3 * k] * hext[3 * k + 1] * hext[3 * k + 2] : 0);
        upload_table(0, hlo.data(), hext.data(), hal.data(), hoff.data());
        cur = 0;
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
        // initial function: re-initialised +-1/2 indicator, on the same boxes
        // (the item bookkeeping needs a radius: R = 1 with identity taps; the
        // z-convolved output of this pass is discarded)
        set_identity_taps();
        layout_meta_count(0, true);
        layout_meta_fill(0, true);
        const long long need = tot[0].arena;
        for (int a = 0; a < 4; ++a) ensure_arena(a, need);
        DBuf lab;
        lab.ensure(sizeof(int32_t) * nt3);
        HIPCHECK(hipMemcpyAsync(lab.p, labels, sizeof(int32_t) * nt3, hipMemcpyHostToDevice, stream));
        hipLaunchKernelGGL(gg::k_init_indicator<T>, dim3(G), dim3(gg::kBlock), 0, stream, boxes_of(0),
                           lab.as<int>(), arena[0].as<T>(), grid_args());
        HIPCHECK(hipGetLastError());
        launch_reinit(0, 0, arena[0].as<T>(), arena[1].as<T>(), arena[2].as<T>(), arena[3].as<T>(), nullptr,
                      nullptr, false);
        a_state = 2;
        a_T = a_psi = -1;
        T_R = psi_R = -1;
        HIPCHECK(hipStreamSynchronize(stream));
        lab.release();
        if (physics) {
            ensure_iota(0, need);
            ensure_iota(1, need);
            iota_cur = 0;
            hipLaunchKernelGGL(gg::k_compare<T>, dim3(grid_of(gg::xcd_grid(ntiles))), dim3(gg::kBlock), 0, stream, boxes_of(0),
                               cov_off.as<int>(), cov_list.as<int>(), arena[a_state].as<T>(), (T *)nullptr,
                               iota_a[0].as<int>(), bmin.as<int>(), bmax.as<int>(), occ.as<unsigned>(),
                               tile_args(), W, 1);
            HIPCHECK(hipGetLastError());
            HIPCHECK(hipStreamSynchronize(stream));
        }
    }

    void set_identity_taps() {
        std::vector<T> t = {T(0), T(1), T(0)};
        HIPCHECK(hipMemcpyAsync(taps_d.p, t.data(), sizeof(T) * 3, hipMemcpyHostToDevice, stream));
        HIPCHECK(hipStreamSynchronize(stream));
        R = 1;
        sigma = -1.0;
    }

    void upload_table(int l, const int *hlo, const int *hext, const int *hal, const long long *hoff) {
        HIPCHECK(hipMemcpyAsync(lo[l].p, hlo, sizeof(int) * 3 * G, hipMemcpyHostToDevice, stream));
        HIPCHECK(hipMemcpyAsync(ext[l].p, hext, sizeof(int) * 3 * G, hipMemcpyHostToDevice, stream));
        HIPCHECK(hipMemcpyAsync(alive[l].p, hal, sizeof(int) * G, hipMemcpyHostToDevice, stream));
        HIPCHECK(hipMemcpyAsync(off[l].p, hoff, sizeof(long long) * (G + 1), hipMemcpyHostToDevice, stream));
        HIPCHECK(hipStreamSynchronize(stream));
    }

    // ------------------------------------------------------------------ step
    void step(double dt, int nsteps) override {
        set_gaussian(dt);
        hipEvent_t e0, e1;
        HIPCHECK(hipEventCreate(&e0));
        HIPCHECK(hipEventCreate(&e1));
        HIPCHECK(hipEventRecord(e0, stream));
        for (int s = 0; s < nsteps; ++s) step_once(s == nsteps - 1);
        HIPCHECK(hipEventRecord(e1, stream));
        HIPCHECK(hipEventSynchronize(e1));
        resolve_spans();
        float ms = 0.f;
        HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (nsteps > 0) last_ms = ms / nsteps;
    }

    const int *iota_now() { return physics ? iota_a[iota_cur].as<int>() : nullptr; }

    // psi of the current layout from phi (or from the kept z pass of phi).
    void predict(int l) {
        const long long m = tot[l].arena;
        int src = a_state;
        if (dim == 3) {
            if (a_T < 0 || T_R != R) {
                a_T = pick(bit(a_state), m);
                launch_conv_z(l, arena[a_state].as<T>(), arena[a_T].as<T>());
                T_R = R;
            }
            src = a_T;
        }
        a_psi = pick(bit(a_state) | bit(src), m);
        const T *phi = a_state >= 0 ? arena[a_state].as<T>() : nullptr;
        launch_conv_xy(l, arena[src].as<T>(), arena[a_psi].as<T>(), physics_args(phi, iota_now()));
        psi_R = R;
    }

    void step_once(bool last) {
        const int L = cur, Ln = 1 - cur;
        if (items_R[L] != R) {
            layout_meta_count(L, false);
            layout_meta_fill(L, false);
        }
        const Totals &t = tot[L];
        last_gv = t.arena;
        total_gv += t.arena;
        // 1. predictor (already issued at the end of the previous step when possible)
        if (a_psi < 0 || psi_R != R) predict(L);
        // 2. corrector: psi -> phi^c (phi, its z pass and psi are dead afterwards)
        const int a_phic = pick(bit(a_psi), t.arena);
        T *psi = arena[a_psi].as<T>(), *phic = arena[a_phic].as<T>();
        const int iota_old = 1 - iota_cur;
        if (physics) ensure_iota(iota_old, t.arena);
        tbegin(GG_K_COMPARE, t.arena);
        hipLaunchKernelGGL(gg::k_compare<T>, dim3(grid_of(gg::xcd_grid(ntiles))), dim3(gg::kBlock), 0, stream, boxes_of(L), cov_off.as<int>(),
                           cov_list.as<int>(), psi, phic, physics ? iota_a[iota_old].as<int>() : (int *)nullptr,
                           bmin.as<int>(), bmax.as<int>(), occ.as<unsigned>(), tile_args(), W, 0);
        tend();
        HIPCHECK(hipGetLastError());
        if (keep) keep_copy(L, psi, phic);
        a_state = a_T = a_psi = -1;
        // 3. new boxes, offsets, items and coverage of the new layout
        gg::PlanArgs pa;
        for (int a = 0; a < 3; ++a) pa.n[a] = n[a];
        pa.P = P;
        pa.occ_words = occ_words;
        pa.G = G;
        const int tb = 256, gb = (G + tb - 1) / tb;
        tbegin(GG_K_PLAN, 0);
        hipLaunchKernelGGL(gg::k_plan, dim3(gb), dim3(tb), 0, stream, boxes_of(L), boxes_of(Ln), bmin.as<int>(),
                           bmax.as<int>(), occ.as<unsigned>(), sizes.as<long long>(), pa);
        hipLaunchKernelGGL(gg::k_scan, dim3(1), dim3(1024), 0, stream, sizes.as<long long>(), off[Ln].as<long long>(), G);
        tend();
        HIPCHECK(hipGetLastError());
        layout_meta_count(Ln, true);
        const long long need = tot[Ln].arena;
        for (int a = 0; a < 4; ++a)
            if (a != a_phic) ensure_arena(a, need);  // all dead: grow before the writes
        if (physics) ensure_iota(iota_cur, need);
        layout_meta_fill(Ln, true);
        // 4. re-initialization into the new layout (+ the next predictor's z pass)
        const int *io_old = physics ? iota_a[iota_old].as<int>() : nullptr;
        int *io_new = physics ? iota_a[iota_cur].as<int>() : nullptr;
        if (dim == 3) {
            const int a_d2 = pick(bit(a_phic), need);
            const int a_t = pick(bit(a_phic) | bit(a_d2), need);
            const bool write_phi = last || physics;
            const int a_phi = write_phi ? pick(bit(a_phic) | bit(a_d2) | bit(a_t), need) : -1;
            launch_reinit(L, Ln, phic, arena[a_d2].as<T>(), write_phi ? arena[a_phi].as<T>() : nullptr,
                          arena[a_t].as<T>(), io_old, io_new, redist == GG_REDIST_EUCLID);
            a_T = a_t;
            T_R = R;
            a_state = a_phi;
        } else {
            const int a_phi = pick(bit(a_phic), need);
            if (redist == GG_REDIST_EUCLID) {
                // the Jacobi sweeps alternate between two more arenas
                const int a_u = pick(bit(a_phic) | bit(a_phi), need);
                const int a_v = pick(bit(a_phic) | bit(a_phi) | bit(a_u), need);
                launch_reinit(L, Ln, phic, arena[a_u].as<T>(), arena[a_phi].as<T>(), arena[a_v].as<T>(), io_old,
                              io_new, true);
            } else {
                launch_reinit(L, Ln, phic, nullptr, arena[a_phi].as<T>(), nullptr, io_old, io_new, false);
            }
            a_state = a_phi;
        }
        cur = Ln;
        ++steps_done;
        // 5. the next step's predictor
        if (!last) predict(Ln);
    }

    // Grid coarsening onto np (validated by the caller): projection of the
    // current phi, new boxes from its positive nodes (the box plan over a
    // virtual layout that takes every axis whole), re-initialization as at
    // creation, the ID-field rebuilt when the correction is on.
    void coarsen(const int32_t *np_in) override {
        int np[3] = {np_in[0], np_in[1], np_in[2]};
        if (a_state < 0) throw ArgError{"no materialised state to coarsen"};
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
                           (const T *)arena[a_state].as<T>(), ca, bmax.as<int>(), occ.as<unsigned>(), occ_words);
        gg::PlanArgs pa;
        for (int a = 0; a < 3; ++a) pa.n[a] = np[a];
        pa.P = P;
        pa.occ_words = occ_words;
        pa.G = G;
        const int tb = 256, gb = (G + tb - 1) / tb;
        hipLaunchKernelGGL(gg::k_plan, dim3(gb), dim3(tb), 0, stream, Lv, boxes_of(Ln), bmin.as<int>(),
                           bmax.as<int>(), occ.as<unsigned>(), sizes.as<long long>(), pa);
        hipLaunchKernelGGL(gg::k_scan, dim3(1), dim3(1024), 0, stream, sizes.as<long long>(), off[Ln].as<long long>(), G);
        tend();
        HIPCHECK(hipGetLastError());
        // the new grid
        set_grid(np);
        voxel_m *= r;
        items_R[0] = items_R[1] = -1;
        have_keep = false;
        set_identity_taps();
        layout_meta_count(Ln, true);
        const long long need = tot[Ln].arena;
        const int a_f = pick(bit(a_state), need);
        tbegin(GG_K_PLAN, 0);
        hipLaunchKernelGGL(gg::k_coarsen_values<T>, dim3(G, split), dim3(gg::kBlock), 0, stream, boxes_of(L),
                           (const T *)arena[a_state].as<T>(), boxes_of(Ln), arena[a_f].as<T>(), ca);
        tend();
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipStreamSynchronize(stream));  // the old phi is dead only now
        for (int a = 0; a < 4; ++a)
            if (a != a_f) ensure_arena(a, need);
        layout_meta_fill(Ln, true);
        int others[3], m = 0;
        for (int a = 0; a < 4; ++a)
            if (a != a_f) others[m++] = a;
        launch_reinit(Ln, Ln, arena[a_f].as<T>(), arena[others[0]].as<T>(), arena[others[1]].as<T>(),
                      arena[others[2]].as<T>(), nullptr, nullptr, false);
        cur = Ln;
        a_state = others[1];
        a_T = a_psi = -1;
        T_R = psi_R = -1;
        if (physics) {
            ensure_iota(0, need);
            ensure_iota(1, need);
            iota_cur = 0;
            hipLaunchKernelGGL(gg::k_compare<T>, dim3(grid_of(gg::xcd_grid(ntiles))), dim3(gg::kBlock), 0, stream,
                               boxes_of(Ln), cov_off.as<int>(), cov_list.as<int>(), arena[a_state].as<T>(),
                               (T *)nullptr, iota_a[0].as<int>(), bmin.as<int>(), bmax.as<int>(),
                               occ.as<unsigned>(), tile_args(), W, 1);
            HIPCHECK(hipGetLastError());
        }
        HIPCHECK(hipStreamSynchronize(stream));
        resolve_spans();
        vlo.release();
        vext.release();
    }

    // Interface areas of the current phi (FP64 per-grain sums, fixed order).
    void areas(double *area, double *weighted) override {
        if (a_state < 0) throw ArgError{"no materialised state"};
        const int split = 8;
        DBuf part, sums;
        part.ensure(sizeof(double) * 2 * (size_t)G * split);
        sums.ensure(sizeof(double) * 2 * (size_t)G);
        gg::AreaArgs aa;
        aa.mode = physics;
        aa.theta_c_deg = theta_c;
        aa.split = split;
        aa.G = G;
        hipLaunchKernelGGL(gg::k_areas<T>, dim3(G, split), dim3(gg::kBlock), 0, stream, boxes_of(cur),
                           (const T *)arena[a_state].as<T>(), iota_now(), (const T *)quat_d.as<T>(), aa,
                           part.as<double>(), W, grid_args());
        hipLaunchKernelGGL(gg::k_sum_rows, dim3((2 * G + 255) / 256), dim3(256), 0, stream, part.as<double>(),
                           sums.as<double>(), 2 * G, split);
        HIPCHECK(hipGetLastError());
        std::vector<double> h(2 * (size_t)G);
        HIPCHECK(hipMemcpyAsync(h.data(), sums.p, sizeof(double) * 2 * G, hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
        std::memcpy(area, h.data(), sizeof(double) * G);
        if (weighted) std::memcpy(weighted, h.data() + G, sizeof(double) * G);
    }

    // One grain's box and values (as doubles); returns the value count, or
    // -count when cap is too small (nothing written), 0 for an extinct grain.
    long long grain_sdf(int k, int32_t *lo_o, int32_t *ext_o, double *out, long long cap) override {
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
        if (a_state < 0) throw ArgError{"no materialised state"};
        DBuf tmp;
        tmp.ensure(sizeof(double) * m);
        hipLaunchKernelGGL((gg::k_convert<T, double>), dim3(256), dim3(256), 0, stream, arena[a_state].as<T>() + o,
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
        if (a_state < 0) throw ArgError{"no materialised state"};
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
        HIPCHECK(hipMemcpyAsync(v.data(), arena[a_state].p, sizeof(T) * m, hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipMemcpyAsync(vo.data(), vol.p, sizeof(double) * G, hipMemcpyDeviceToHost, stream));
        if (h.has_iota) {
            io.resize(std::max<long long>(m, 1));
            HIPCHECK(hipMemcpyAsync(io.data(), iota_now(), sizeof(int) * m, hipMemcpyDeviceToHost, stream));
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
        CkptHeader h;
        get(f, &h, sizeof(h));
        if (std::memcmp(h.magic, kMagic, 8) != 0 || h.version != 1) throw ArgError{"not a checkpoint of this library"};
        if (h.dim != dim || h.G != G || h.precision != precision_code() || h.band != band_d ||
            h.physics != physics || h.redistance != redist)
            throw ArgError{"checkpoint of a different configuration (dim, grains, precision, band, physics, "
                           "re-initialization)"};
        long long nt = 1;
        for (int a = 0; a < 3; ++a) {
            const bool active = a < dim;
            if (active ? (h.n[a] < 4 * P + 2 || h.n[a] > 4096) : h.n[a] != 1) throw ArgError{"checkpoint grid out of range"};
            nt *= h.n[a];
        }
        if (nt > 2147483647LL || h.values < 0 || h.has_iota != (physics ? 1 : 0)) throw ArgError{"corrupt checkpoint"};
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

    // Try the candidate (budget, small-class limit) pairs for `per` steps each
    // (the simulation advances), keep the one with the least device time per
    // grain voxel.  Tile shapes follow the budgets; the functions do not.
    void autotune(double dt, int per, int32_t *best_lds, int32_t *best_small) override {
        static const int cand[][2] = {{40960, 26624}, {32768, 20480}, {40960, 20480}, {40960, 32768},
                                      {49152, 26624}, {49152, 32768}, {32768, 26624}};
        double best = 1e300;
        int bl = lds_bytes, bs = small_bytes;
        for (const auto &c : cand) {
            lds_bytes = c[0];
            small_bytes = c[1];
            items_R[0] = items_R[1] = -1;  // re-tile the current layout (its predicted values stand)
            const long long gv0 = total_gv;
            step(dt, per);
            const double per_gv = last_ms * per / (double)std::max<long long>(total_gv - gv0, 1);
            if (per_gv < best) {
                best = per_gv;
                bl = c[0];
                bs = c[1];
            }
        }
        lds_bytes = bl;
        small_bytes = bs;
        items_R[0] = items_R[1] = -1;
        *best_lds = bl;
        *best_small = bs;
    }

    void keep_copy(int L, const T *psi, const T *phic) {
        const long long m = tot[L].arena;
        keep_psi.ensure(sizeof(T) * std::max<long long>(m, 1));
        keep_phic.ensure(sizeof(T) * std::max<long long>(m, 1));
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
        have_keep = true;
    }

    // ---------------------------------------------------------------- queries
    void volumes(double *out) override {
        HIPCHECK(hipMemcpyAsync(out, vol.p, sizeof(double) * G, hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
    }

    void labels(int32_t *out, bool device) override {
        const long long nt3 = (long long)n[0] * n[1] * n[2];
        DBuf tmp;
        int32_t *dst = out;
        if (!device) {
            tmp.ensure(sizeof(int32_t) * nt3);
            dst = tmp.as<int32_t>();
        }
        hipLaunchKernelGGL(gg::k_labels<T>, dim3(ntiles), dim3(gg::kBlock), 0, stream, boxes_of(cur), cov_off.as<int>(),
                           cov_list.as<int>(), arena[a_state].as<T>(), dst, tile_args());
        HIPCHECK(hipGetLastError());
        if (!device) {
            HIPCHECK(hipMemcpyAsync(out, dst, sizeof(int32_t) * nt3, hipMemcpyDeviceToHost, stream));
            HIPCHECK(hipStreamSynchronize(stream));
        }
    }

    void boxes(int32_t *hlo, int32_t *hext, int32_t *hal, int64_t *hoff, bool prev) override {
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

    long long arena_total(bool prev) const override { return prev ? keep_tot.arena : tot[cur].arena; }

    long long values(double *out, long long cap, int which) override {
        const T *src;
        long long m;
        if (which < 0) {
            src = arena[a_state].as<T>();
            m = tot[cur].arena;
        } else {
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
        for (int k = 0; k < G; ++k) {
            a[k] = hal[k] ? 1 : 0;
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
        for (int q = 0; q < 4; ++q) ensure_arena(q, m);
        a_state = 0;
        a_T = a_psi = -1;
        T_R = psi_R = -1;
        std::vector<T> tv;
        const T *up;
        if constexpr (std::is_same<V, T>::value) {
            up = vals;
        } else {
            tv.resize(std::max<long long>(m, 1));
            for (long long i = 0; i < m; ++i) tv[i] = (T)vals[i];
            up = tv.data();
        }
        HIPCHECK(hipMemcpyAsync(arena[0].p, up, sizeof(T) * m, hipMemcpyHostToDevice, stream));
        HIPCHECK(hipMemcpyAsync(vol.p, vh.data(), sizeof(double) * G, hipMemcpyHostToDevice, stream));
        if (physics) {
            ensure_iota(0, m);
            ensure_iota(1, m);
            iota_cur = 0;
            std::vector<int> io(std::max<long long>(m, 1), -1);
            if (hiota)
                for (long long i = 0; i < m; ++i) io[i] = hiota[i];
            HIPCHECK(hipMemcpyAsync(iota_a[0].p, io.data(), sizeof(int) * m, hipMemcpyHostToDevice, stream));
        }
        HIPCHECK(hipStreamSynchronize(stream));
        items_R[0] = items_R[1] = -1;
        const int keepR = R;
        R = R > 0 ? R : 1;
        layout_meta_count(0, true);
        layout_meta_fill(0, true);
        R = keepR;
        if (R <= 0) items_R[0] = -1;
        HIPCHECK(hipStreamSynchronize(stream));
    }

    int alive_count() const override { return (int)tot[cur].alive; }

    gg_step_stats stats() const override {
        gg_step_stats s;
        s.steps = steps_done;
        s.total_grain_voxels = total_gv;
        s.alive = (int)tot[cur].alive;
        s.kernel_radius = R;
        s.grain_voxels = last_gv;
        s.capacity = (int64_t)(arena[a_state >= 0 ? a_state : 0].cap / sizeof(T));
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

}  // namespace

extern "C" {

const char *gg_version(void) { return "gg-mi355x 0.1 (gfx950)"; }

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

// The calls that advance or replace the state check their arguments before they
// change anything (GG_E_ARG).  A later failure (memory, capacity) can leave the
// state part way replaced: it poisons the simulation, as a HIP error does.
static gg_status state_changed(gg_sim *sim, gg_status st) {
    if (st == GG_E_NOMEM || st == GG_E_CAPACITY) sim->poisoned = true;
    return st;
}

gg_status gg_step(gg_sim *sim, double dt, int32_t n_steps) {
    if (!sim) return GG_E_ARG;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(sim, GG_E_ARG, "dt must be finite and positive");
    if (n_steps < 0) return fail(sim, GG_E_ARG, "n_steps must be >= 0");
    return state_changed(sim, guarded(sim, [&]() {
                             sim->impl->step(dt, n_steps);
                             return GG_OK;
                         }));
}

gg_status gg_sync(gg_sim *sim) {
    return guarded(sim, [&]() {
        sim->impl->sync();
        return GG_OK;
    });
}

gg_status gg_grain_count(gg_sim *sim, int32_t *alive) {
    if (!alive) return fail(sim, GG_E_ARG, "alive is NULL");
    return guarded(sim, [&]() {
        *alive = sim->impl->alive_count();
        return GG_OK;
    });
}

gg_status gg_grain_volumes(gg_sim *sim, double *out, int64_t cap) {
    if (!sim || !out) return fail(sim, GG_E_ARG, "NULL argument");
    if (cap < sim->G) return fail(sim, GG_E_SMALLBUF, "cap < n_grains");
    return guarded(sim, [&]() {
        sim->impl->volumes(out);
        return GG_OK;
    });
}

gg_status gg_labels(gg_sim *sim, int32_t *out, int64_t cap, int32_t out_is_device) {
    if (!sim || !out) return fail(sim, GG_E_ARG, "NULL argument");
    if (cap < (int64_t)sim->n[0] * sim->n[1] * sim->n[2]) return fail(sim, GG_E_SMALLBUF, "cap < prod(n)");
    return guarded(sim, [&]() {
        sim->impl->labels(out, out_is_device != 0);
        return GG_OK;
    });
}

gg_status gg_stats(gg_sim *sim, gg_step_stats *out) {
    if (!sim || !out) return fail(sim, GG_E_ARG, "NULL argument");
    return guarded(sim, [&]() {
        *out = sim->impl->stats();
        return GG_OK;
    });
}

gg_status gg_get_boxes(gg_sim *sim, int32_t *lo, int32_t *ext, int32_t *alive, int64_t *offset, int64_t cap) {
    if (!sim) return GG_E_ARG;
    if (cap < sim->G) return fail(sim, GG_E_SMALLBUF, "cap < n_grains");
    return guarded(sim, [&]() {
        sim->impl->boxes(lo, ext, alive, offset, false);
        return GG_OK;
    });
}

gg_status gg_get_values(gg_sim *sim, double *out, int64_t cap) {
    if (!sim || !out) return fail(sim, GG_E_ARG, "NULL argument");
    return guarded(sim, [&]() {
        long long m = sim->impl->values(out, cap, -1);
        if (m < 0) return fail(sim, GG_E_SMALLBUF, "cap < sum of box volumes (" + std::to_string(-m) + ")");
        return GG_OK;
    });
}

gg_status gg_get_iota(gg_sim *sim, int32_t *out, int64_t cap) {
    if (!sim || !out) return fail(sim, GG_E_ARG, "NULL argument");
    return guarded(sim, [&]() {
        long long m = sim->impl->iota(out, cap);
        if (m < 0) return fail(sim, GG_E_SMALLBUF, "cap < sum of box volumes");
        return GG_OK;
    });
}

gg_status gg_load_state(gg_sim *sim, const int32_t *lo, const int32_t *ext, const uint8_t *alive,
                        const double *values, const int32_t *iota) {
    if (!sim || !lo || !ext || !alive || !values) return fail(sim, GG_E_ARG, "NULL argument");
    return state_changed(sim, guarded(sim, [&]() {
                             sim->impl->load_state(lo, ext, alive, values, iota);
                             return GG_OK;
                         }));
}

gg_status gg_grain_areas(gg_sim *sim, double *area, double *weighted, int64_t cap) {
    if (!sim || !area) return fail(sim, GG_E_ARG, "NULL argument");
    if (cap < sim->G) return fail(sim, GG_E_SMALLBUF, "cap < n_grains");
    return guarded(sim, [&]() {
        sim->impl->areas(area, weighted);
        return GG_OK;
    });
}

gg_status gg_grain_sdf(gg_sim *sim, int32_t id, int32_t lo[3], int32_t ext[3], double *out, int64_t cap) {
    if (!sim || !lo || !ext) return fail(sim, GG_E_ARG, "NULL argument");
    if (id < 0 || id >= sim->G) return fail(sim, GG_E_ARG, "grain id out of range");
    return guarded(sim, [&]() {
        const long long m = sim->impl->grain_sdf(id, lo, ext, out, cap);
        if (m < 0 && out) return fail(sim, GG_E_SMALLBUF, "cap too small (" + std::to_string(-m) + ")");
        return GG_OK;
    });
}

gg_status gg_autotune(gg_sim *sim, double dt, int32_t steps_per_candidate, int32_t *lds_bytes,
                      int32_t *small_bytes) {
    if (!sim || !lds_bytes || !small_bytes) return fail(sim, GG_E_ARG, "NULL argument");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(sim, GG_E_ARG, "dt must be finite and positive");
    if (steps_per_candidate < 1) return fail(sim, GG_E_ARG, "steps_per_candidate must be >= 1");
    return state_changed(sim, guarded(sim, [&]() {
                             sim->impl->autotune(dt, steps_per_candidate, lds_bytes, small_bytes);
                             return GG_OK;
                         }));
}

gg_status gg_save(gg_sim *sim, const char *path) {
    if (!sim || !path) return fail(sim, GG_E_ARG, "NULL argument");
    return guarded(sim, [&]() {
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
    });
}

gg_status gg_load(gg_sim *sim, const char *path) {
    if (!sim || !path) return fail(sim, GG_E_ARG, "NULL argument");
    return state_changed(sim, guarded(sim, [&]() {
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
    return state_changed(sim, st);
}

gg_status gg_keep_intermediates(gg_sim *sim, int32_t on) {
    return guarded(sim, [&]() {
        sim->impl->keep = on != 0;
        return GG_OK;
    });
}

gg_status gg_get_intermediate(gg_sim *sim, int32_t which, double *out, int64_t cap, int32_t *lo, int32_t *ext,
                              int32_t *alive, int64_t *offset, int64_t cap_grains) {
    if (!sim || !out || (which != 0 && which != 1)) return fail(sim, GG_E_ARG, "bad argument");
    if ((lo || ext || alive || offset) && cap_grains < sim->G) return fail(sim, GG_E_SMALLBUF, "cap_grains < n_grains");
    return guarded(sim, [&]() {
        long long m = sim->impl->values(out, cap, which);
        if (m < 0) return fail(sim, GG_E_SMALLBUF, "cap too small (" + std::to_string(-m) + ")");
        if (lo || ext || alive || offset) sim->impl->boxes(lo, ext, alive, offset, true);
        return GG_OK;
    });
}

gg_status gg_profile(gg_sim *sim, int32_t on) {
    return guarded(sim, [&]() {
        sim->impl->profile(on != 0);
        return GG_OK;
    });
}

gg_status gg_get_kernel_times(gg_sim *sim, gg_kernel_times *out) {
    if (!sim || !out) return fail(sim, GG_E_ARG, "NULL argument");
    return guarded(sim, [&]() {
        *out = sim->impl->kernel_times();
        return GG_OK;
    });
}

void gg_destroy(gg_sim *sim) {
    if (!sim) return;
    (void)hipSetDevice(sim->device);
    delete sim;
}

}  // extern "C"
