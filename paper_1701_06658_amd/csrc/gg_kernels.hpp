// Device code of the level-set grain-growth step for gfx950 (MI355X): shared
// helpers, the corrector, the Euclidean re-initialization variant, grid
// coarsening, interface areas and the box / coverage bookkeeping.  The two
// z-marching kernels of the step are in gg_march.hpp.
//
// Data layout in HBM: every alive grain's box is stored contiguously, x
// fastest, in grain-id order ("packed arena"); a box table (lo, ext, alive,
// offset) per layout describes it.  The corrector and the labels work over
// fixed tiles of the global grid with per-tile coverage lists of grains.
//
// One step is three sweeps over the packed boxes:
//   k_compare        psi (layout L)      -> phi^c (L)   top-2 of the covering grains per global tile
//   k_reinit_march   phi^c (L)           -> f (L')      reference values, taxicab spreading x, y, forward z
//   k_predict_march  f (L')              -> psi (L')    backward z spreading, band clamp, volume,
//                                                       Gaussian z, x, y (+ correction epilogue)
// with the box plan and coverage lists of the new layout L' between the first
// two.  The Euclidean variant replaces k_reinit_march by k_reinit_xy (reference
// values) and k_jacobi (Godunov sweeps).
//
// Along an axis a box is either the whole periodic axis (indices wrap) or at
// most n - 2P long (indices outside the box read the fill value): a stencil of
// reach <= 2P never wraps into a partial box.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gg {

constexpr int kBlock = 256;       // threads per work group of the tile kernels
constexpr int kWaves = kBlock / 64;
// Jacobi sweep work items: at most this many planes per item, marched through
// a ring of three LDS planes; values per lane of the next plane held in registers.
#ifndef GG_JAC_PLANES
#define GG_JAC_PLANES 16
#endif
constexpr int kJacPlanes = GG_JAC_PLANES;
constexpr int kJacQ = 16;
#ifndef GG_LDS_BYTES
#define GG_LDS_BYTES 40960
#endif
constexpr int kLdsBytes = GG_LDS_BYTES;  // dynamic LDS budget per work group (FP32)
constexpr int kMaxRadius = 12;    // largest Gaussian radius R
constexpr int kMaxBand = 16;      // largest band half width W
// item kinds of the Euclidean variant: reference values (xy tiles of z planes),
// Jacobi sweeps
constexpr int kKinds = 2;
enum { KIND_RXY = 0, KIND_JAC = 1 };

// Box table of one layout.
struct Boxes {
    int *lo;         // 3 per grain
    int *ext;        // 3 per grain (0 when extinct)
    int *alive;      // 1 per grain
    long long *off;  // G + 1: exclusive prefix of box volumes
};

// Work items of every kind come in two launch classes by their LDS need, so
// that the many small boxes are not launched with the LDS of the largest one.
#ifndef GG_SMALL_LDS_BYTES
#define GG_SMALL_LDS_BYTES 26624
#endif
constexpr int kSmallLdsBytes = GG_SMALL_LDS_BYTES;
constexpr int kClasses = 2;

struct Totals {
    long long arena;                  // sum of box volumes
    long long items[kKinds][3];       // all, class 0, class 1
    long long cov;                    // coverage list entries
    long long alive;                  // alive grains
    long long lds[kKinds][kClasses];  // largest LDS need per class, in values
};

// ------------------------------------------------------------------ helpers

__host__ __device__ inline int imod(long long v, int N) {
    long long r = v % N;
    return (int)(r < 0 ? r + N : r);
}

// Local index along an axis for a stencil read at local coordinate c, with
// -N < c < 2N: a whole axis wraps, a partial box clips (-1 = outside).
__device__ __forceinline__ int axis_map(int c, int e, int N) {
    if (e == N) return c < 0 ? c + N : (c >= N ? c - N : c);
    return (c >= 0 && c < e) ? c : -1;
}

// (a - b) mod N for a, b in [0, N).
__device__ __forceinline__ int wrap_diff(int a, int b, int N) {
    const int d = a - b;
    return d < 0 ? d + N : d;
}

// LDS budgets in values: the FP64 path gets twice the bytes (the same number of
// values per tile as FP32), so that its boxes split no more often.
#ifndef GG_F64_LDS_SCALE
#define GG_F64_LDS_SCALE 2
#endif
template <typename T> constexpr int lds_scale() { return sizeof(T) == 8 ? GG_F64_LDS_SCALE : 1; }
template <typename T> constexpr int lds_budget() { return kLdsBytes * lds_scale<T>() / (int)sizeof(T); }
template <typename T> constexpr int small_budget() { return kSmallLdsBytes * lds_scale<T>() / (int)sizeof(T); }
// The largest LDS budget a simulation may be tuned to (FP32 bytes; FP64 scaled
// alike), and the budget in values for a byte figure.
constexpr int kLdsBytesMax = 49152;
template <typename T> constexpr int budget_values(int bytes) { return bytes * lds_scale<T>() / (int)sizeof(T); }

template <typename T> __device__ __forceinline__ T mac(T acc, T a, T b);
template <> __device__ __forceinline__ double mac<double>(double acc, double a, double b) {
    return acc + a * b;  // built without contraction: product and sum rounded separately
}
template <> __device__ __forceinline__ float mac<float>(float acc, float a, float b) {
    return __builtin_fmaf(a, b, acc);
}

template <typename T> __device__ __forceinline__ T tinf();
template <> __device__ __forceinline__ double tinf<double>() { return __builtin_inf(); }
template <> __device__ __forceinline__ float tinf<float>() { return __builtin_inff(); }

// Hardware min / max.  No value on the path is NaN (device code is built
// without NaN semantics); of +0 and -0 either may come back, which no result
// depends on (a reference value fc / (fc - 0) is the same for both).
__device__ __forceinline__ float vmin(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double vmin(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float vmax(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double vmax(double a, double b) { return fmax(a, b); }

// a / b: correctly rounded in FP64; in FP32 (the mixed path) the product with
// the hardware reciprocal (about 1 ulp).
__device__ __forceinline__ double ratio(double a, double b) { return a / b; }
__device__ __forceinline__ float ratio(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// a / sqrt(b), b > 0: correctly rounded steps in FP64; in FP32 the product with
// the hardware reciprocal square root.
__device__ __forceinline__ double grad_dist(double a, double b) { return a / sqrt(b); }
__device__ __forceinline__ float grad_dist(float a, float b) { return a * __builtin_amdgcn_rsqf(b); }

// LDS values needed by an output tile tx * ty of nz planes.  Reference-value
// kind: per plane an f tile and a reference tile of (ty + 2) rows of pitch
// (tx + 2) | 1 (one ring of stencil neighbours) and int offset tables (counted
// as one value each).  Jacobi kind: three planes of the tile with one ring of
// neighbours, row and column tables.
__host__ __device__ inline long long lds_need(int kind, int tx, int ty, int nz = 1) {
    const long long FW = tx + 2, FH = ty + 2;
    if (kind == KIND_RXY) return (long long)nz * (2 * (FW | 1) * FH + FH) + 2 * FH + FW;
    return 3 * FW * FH + FW + FH;
}

// nb: planes per work item.
struct Tiling {
    int nxs, nys, tx, ty, nb;
};

// Split a box cross-section ex * ey into the fewest near-equal tiles whose LDS
// need fits the budget; then take as many of the `planes` z planes per work item
// as fit `target` values of LDS (reference kind) or kJacPlanes (Jacobi kind), in
// near-equal chunks.
__host__ __device__ inline Tiling choose_tiling(int kind, int ex, int ey, int planes, int budget, int target) {
    Tiling t = {0, 0, 0, 0, 1};
    for (int nxs = (ex + 127) / 128; nxs <= ex; ++nxs) {
        const int tx = (ex + nxs - 1) / nxs;
        if (lds_need(kind, tx, ey) <= budget) {
            t.nxs = nxs;
            t.nys = 1;
            t.tx = tx;
            t.ty = ey;
            break;
        }
        const long long b = lds_need(kind, tx, 0);  // the need is affine in ty
        const long long a = lds_need(kind, tx, 1) - b;
        if (budget - b < a) continue;
        const int tymax = (int)((budget - b) / a);
        if (tymax < 1) continue;
        const int nys = (ey + tymax - 1) / tymax;
        t.nxs = nxs;
        t.nys = nys;
        t.tx = tx;
        t.ty = (ey + nys - 1) / nys;
        break;
    }
    if (t.nxs > 0 && planes > 1) {
        long long nb = kJacPlanes;
        if (kind == KIND_RXY) {
            const long long one = lds_need(kind, t.tx, t.ty, 1);
            const long long per = lds_need(kind, t.tx, t.ty, 2) - one;
            const long long tg = target < budget ? target : budget;
            nb = (tg - (one - per)) / per;
        }
        nb = nb < 1 ? 1 : (nb > planes ? planes : nb);
        const int chunks = (int)((planes + nb - 1) / nb);
        t.nb = (planes + chunks - 1) / chunks;
    }
    return t;
}

__host__ __device__ inline Tiling kind_tiling(int kind, const int *e, int budget, int target) {
    return choose_tiling(kind, e[0], e[1], e[2], budget, target);
}

__host__ __device__ inline long long tiling_need(int kind, const Tiling &t) {
    return lds_need(kind, t.tx, t.ty, t.nb);
}

// Number of work items of one kind for a box.
__host__ __device__ inline long long tiling_items(const int *e, const Tiling &t) {
    return (long long)((e[2] + t.nb - 1) / t.nb) * t.nxs * t.nys;
}

// contiguous run of items, so that neighbouring planes of a box, or
// neighbouring tiles of the grid, are processed by the same L2.
constexpr int kXcds = 8;
__host__ __device__ inline long long xcd_grid(long long n) { return kXcds * ((n + kXcds - 1) / kXcds); }
__device__ __forceinline__ long long xcd_item(long long n) {
    const long long chunk = (n + kXcds - 1) / kXcds;
    const long long b = blockIdx.x;
    return (b % kXcds) * chunk + b / kXcds;
}

// Work item -> (grain, first plane, planes, tile origin, tile size).
struct ItemTile {
    long long item;
    int k, plane, np, x0, y0, wx, wy, nxs, nys;
};

// The tiling of every grain and kind is computed once per layout (k_item_counts)
// and stored as two int4: (nxs, nys, tx, ty), (nb, 0, 0, 0).
// Items of one class: owner[item] is the grain, pref the class prefix over
// grains; pref_all (all items of the kind) gives the item's global index.
struct ItemRefs {
    const int *owner;
    const long long *pref;
    const long long *pref_all;
    const int4 *tilings;
    long long n;
};

__device__ __forceinline__ ItemTile decode_item(long long item, int kind, const Boxes &L, const ItemRefs &ir) {
    ItemTile it;
    it.k = ir.owner[item];
    const int sub = (int)(item - ir.pref[it.k]);
    it.item = ir.pref_all[it.k] + sub;
    const int4 *tilings = ir.tilings;
    const int e[3] = {L.ext[3 * it.k], L.ext[3 * it.k + 1], L.ext[3 * it.k + 2]};
    const int4 t4 = tilings[2 * it.k];
    const Tiling tl = {t4.x, t4.y, t4.z, t4.w, 1};
    it.nxs = tl.nxs;
    it.nys = tl.nys;
    const int per = tl.nxs * tl.nys;
    const int chunk = sub / per;
    const int rem = sub - chunk * per;
    const int nb = tilings[2 * it.k + 1].x;
    it.plane = chunk * nb;
    it.np = min(nb, e[2] - it.plane);
    const int ys = rem / tl.nxs, xs = rem - ys * tl.nxs;
    it.x0 = xs * tl.tx;
    it.y0 = ys * tl.ty;
    it.wx = min(tl.tx, e[0] - it.x0);
    it.wy = min(tl.ty, e[1] - it.y0);
    return it;
}

__device__ inline double block_sum(double v, double *scratch) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += scratch[w];
    return s;  // valid in thread 0
}

// Wave-wide min / max (device library reductions over the active lanes, by
// lane permutations within rows and across them); the result is uniform.
extern "C" __device__ int __ockl_wfred_min_i32(int);
extern "C" __device__ int __ockl_wfred_max_i32(int);
__device__ __forceinline__ int wave_min(int v) { return __ockl_wfred_min_i32(v); }
__device__ __forceinline__ int wave_max(int v) { return __ockl_wfred_max_i32(v); }

// HBM latency.
constexpr int kLoadBatch = 8;

// ------------------------------------------------ predictor correction terms

template <typename T> struct Physics {
    int mode;           // bit 1 misorientation weights, bit 2 bulk energy
    const T *quat;      // 4 per grain (w, x, y, z)
    const T *energy;    // 1 per grain, J/m^3
    T theta_c_deg;
    T bulk_scale;       // sigma^2 h / (2 gamma_max): voxels per (J/m^3) and step
    const T *phi;       // the step's input function (same layout as psi)
    const int *iota;    // ID-field of the previous corrector (same layout)
    const T *wcp;       // per-voxel correction weights (same layout), or NULL: the pair (k, iota)
};

template <typename T> __device__ inline T dev_acos(T c);
template <> __device__ inline double dev_acos<double>(double c) { return acos(c); }
template <> __device__ inline float dev_acos<float>(float c) { return acosf(c); }
template <typename T> __device__ inline T dev_exp(T c);
template <> __device__ inline double dev_exp<double>(double c) { return exp(c); }
template <> __device__ inline float dev_exp<float>(float c) { return expf(c); }
template <typename T> __device__ inline T dev_log(T c);
template <> __device__ inline double dev_log<double>(double c) { return log(c); }
template <> __device__ inline float dev_log<float>(float c) { return logf(c); }

// Misorientation angle (degrees) under the hexagonal 622 rotation group: the
// smallest rotation angle of dq * S over the 12 proper symmetry operations S,
// i.e. 2 acos of the largest |scalar part|.
template <typename T> __device__ inline T misorientation_deg(const T *qa, const T *qb) {
    const T aw = qa[0], ax = -qa[1], ay = -qa[2], az = -qa[3];
    const T bw = qb[0], bx = qb[1], by = qb[2], bz = qb[3];
    const T dw = aw * bw - ax * bx - ay * by - az * bz;
    const T dx = aw * bx + ax * bw + ay * bz - az * by;
    const T dy = aw * by - ax * bz + ay * bw + az * bx;
    const T dz = aw * bz + ax * by - ay * bx + az * bw;
    // cos and sin of k*30 degrees, k = 0..5
    const T c6[6] = {T(1), T(0.86602540378443864676), T(0.5), T(0), T(-0.5), T(-0.86602540378443864676)};
    const T s6[6] = {T(0), T(0.5), T(0.86602540378443864676), T(1), T(0.86602540378443864676), T(0.5)};
    T best = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const T w1 = dw * c6[k] - dz * s6[k];   // rotation about c by 60k degrees
        const T w2 = -dx * c6[k] - dy * s6[k];  // 2-fold axis in the basal plane at 30k degrees
        const T m1 = w1 < 0 ? -w1 : w1;
        const T m2 = w2 < 0 ? -w2 : w2;
        best = m1 > best ? m1 : best;
        best = m2 > best ? m2 : best;
    }
    if (best > T(1)) best = T(1);
    return T(2) * dev_acos(best) * T(57.295779513082320877);
}

// Read-Shockley boundary energy, normalised to 1 at and above theta_c.
template <typename T> __device__ inline T read_shockley(T theta, T theta_c) {
    if (theta >= theta_c) return T(1);
    if (theta <= T(0)) return T(0);
    const T r = theta / theta_c;
    return r * (T(1) - dev_log(r));
}

// Pair weight w = mobility * Read-Shockley energy (both normalised to (0, 1]).
template <typename T> __device__ inline T pair_weight(T theta, T theta_c, T *mob) {
    const T g = read_shockley(theta, theta_c);
    const T u = theta / T(15);
    const T u3 = u * u * u;
    const T mu = T(1) - T(0.99) * dev_exp(T(-5) * (u3 * u3 * u3));
    *mob = mu;
    return mu * g;
}

template <typename T> struct PairCache {
    int j = -2;
    T w = 1, b = 0;
};


// --------------------------------------------------------- predictor kernels

// Position (r, c) of element e of an array of rows of W values, advanced by
// kBlock elements per step without division.
struct Walk2 {
    int r, c, W, dq, dm;
    __device__ __forceinline__ Walk2(int e, int W_) : W(W_) {
        dq = kBlock / W;
        dm = kBlock - dq * W;
        r = e / W;
        c = e - r * W;
    }
    __device__ __forceinline__ void step() {
        c += dm;
        r += dq;
        if (c >= W) {
            c -= W;
            ++r;
        }
    }
};

struct GridArgs {
    int n[3];
    int dim;
};

// x and y passes of the Gaussian on one tile of nz consecutive z planes of a

// Device control block of the step sequence.  Every kernel of a step returns
// at once when `fail` is set, so that a step whose new layout does not fit the
// buffers leaves the state it started from untouched (the library then grows
// the buffers and runs the step again).
struct Ctl {
    int fail;             // sticky: 0 none, 1 value arenas too small, 2 coverage list too small
    int fail_step;        // completed steps when the failure was raised
    int steps;            // completed steps since creation
    int alive;            // alive grains after the last completed step
    int phi_at;           // the step (value of `steps` while it runs) whose predictor stores phi
    int pad;
    long long need_arena; // values the failing layout needs
    long long need_cov;   // coverage entries the failing layout needs
    long long total_gv;   // grain voxels summed over completed steps
    long long last_gv;    // grain voxels of the last completed step
    long long arena_now;  // values of the layout after the last completed step
    long long cov_now;    // coverage entries of that layout
};

__device__ __forceinline__ bool ctl_failed(const Ctl *c) { return c != nullptr && c->fail != 0; }

// ------------------------------------------------------------ corrector (a3)

struct TileArgs {
    int n[3];
    int t[3];    // tile dims
    int nt[3];   // tiles per axis
    int occ_words;
};

// Top-2 of (value, id) in the order: larger value first, then lower id.
template <typename T> struct Top2 {
    T m1, m2;
    int i1, i2;
    __device__ void init() {
        m1 = m2 = -tinf<T>();
        i1 = i2 = -1;
    }
    // v (from grain j) joins when `in` holds, branch-free.  IDS: equal values
    // are ordered by id, lowest first, so that the argmax over the others is
    // unique; otherwise the first pushed stays first, which changes no value
    // the corrector takes from the pair.
    template <bool IDS> __device__ void push(T v, int j, bool in) {
        bool a1, a2;
        if constexpr (IDS) {
            a1 = in && (v > m1 || (v == m1 && j < i1));
            a2 = in && (v > m2 || (v == m2 && (i2 < 0 || j < i2)));
        } else {
            a1 = in && v > m1;
            a2 = in && v > m2;
        }
        m2 = a1 ? m1 : (a2 ? v : m2);
        i2 = a1 ? i1 : (a2 ? j : i2);
        m1 = a1 ? v : m1;
        i1 = a1 ? j : i1;
    }
};

// Values a corrector group keeps in LDS between its two passes: per voxel its
// first NS values from boxes met linearly, in coverage-list order (the k-th in
// slot k); the others are read again in the second pass.
#ifndef GG_CMP_LDS_BYTES
#define GG_CMP_LDS_BYTES 16384
#endif
#ifndef GG_CMP_LDS_BYTES_F64
#define GG_CMP_LDS_BYTES_F64 16384
#endif

#ifndef GG_CMP_TILE_VOX
#define GG_CMP_TILE_VOX 512
#endif
constexpr int kTileVox = GG_CMP_TILE_VOX;  // voxels of a corrector tile (at most)
constexpr int kVpt = kTileVox / kBlock;
template <typename T> constexpr int cmp_slots() {
    return (sizeof(T) == 8 ? GG_CMP_LDS_BYTES_F64 : GG_CMP_LDS_BYTES) / (kTileVox * (int)sizeof(T));
}

// Where a global tile meets box j.  Per axis s = (tile origin - box start) mod
// n.  The box coordinate of the tile voxel at offset v is linear, d + v, when
// no voxel of the tile reaches the box a second time around the axis: when
// ext + t <= n (then d = s, or s - n if s >= ext, the box starting inside the
// tile), or when s + t <= n (d = s).  The voxel lies in the box exactly when
// 0 <= d + v < ext, and its value is then at base + v_x + ext_x (v_y + ext_y
// v_z).  Otherwise ("wrapped") the coordinate is (s + v) mod n per voxel.
struct TileBox {
    long long off, base;
    int j, s[3], d[3], e[3];
    int lin;
};

// The TileBox of coverage entry c (c < end), computed by one lane.
__device__ __forceinline__ TileBox tile_box(const Boxes &L, const int *cov_list, int c, int end, const int (&t0)[3],
                                            const TileArgs &ta) {
    TileBox b;
    const int j = c < end ? cov_list[c] : 0;
    b.j = j;
    b.off = L.off[j];
    b.lin = 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int lo = L.lo[3 * j + a], ex = L.ext[3 * j + a], n = ta.n[a];
        int s = t0[a] - lo;
        s += s < 0 ? n : 0;
        b.s[a] = s;
        b.e[a] = ex;
        const int once = ex + ta.t[a] <= n;
        b.lin &= once | (s + ta.t[a] <= n);
        b.d[a] = (once && s >= ex) ? s - n : s;
    }
    b.base = b.off + b.d[0] + (long long)b.e[0] * (b.d[1] + (long long)b.e[1] * b.d[2]);
    return b;
}

// Uniform copies of lane `lane`'s TileBox (the fields of the linear case, or
// all of them).
__device__ __forceinline__ long long readlane64(long long v, int lane) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), lane);
    return (long long)(((unsigned long long)hi << 32) | lo);
}
template <bool ALL> __device__ __forceinline__ TileBox box_of_lane(const TileBox &w, int lane) {
    TileBox b;
    b.j = __builtin_amdgcn_readlane(w.j, lane);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        b.e[a] = __builtin_amdgcn_readlane(w.e[a], lane);
        if constexpr (ALL) b.s[a] = __builtin_amdgcn_readlane(w.s[a], lane);
        else b.d[a] = __builtin_amdgcn_readlane(w.d[a], lane);
    }
    if constexpr (ALL) b.off = readlane64(w.off, lane);
    else b.base = readlane64(w.base, lane);
    return b;
}

// An element of an array at a byte offset from a base pointer.
template <typename U, typename O> __device__ __forceinline__ U &at_bytes(U *base, O bo) {
    return *reinterpret_cast<U *>(reinterpret_cast<char *>(base) + bo);
}
template <typename U, typename O> __device__ __forceinline__ const U &at_bytes(const U *base, O bo) {
    return *reinterpret_cast<const U *>(reinterpret_cast<const char *>(base) + bo);
}

#ifndef GG_CMP_U
#define GG_CMP_U 8
#endif

// One global tile: the top-2 of the predicted functions of every grain whose
// box covers the tile, then for each of those grains
//   phi^c = (psi - max over the other grains) / 2   (-W if no other grain),
// its ID-field (argmax of the others; IDS: iota_out given), and the bounding
// box of phi^c > 0.  mode 0: corrector; mode 1: ID-field only.
template <typename T, bool IDS>
__global__ void __launch_bounds__(kBlock)
    k_compare(Boxes L, const int *__restrict__ cov_off, const int *__restrict__ cov_list, const T *__restrict__ psi,
              T *__restrict__ phic, int *__restrict__ iota_out, int *bmin, int *bmax, unsigned *occ, TileArgs ta,
              T W, int mode, const Ctl *ctl) {
    constexpr int NS = cmp_slots<T>();
    static_assert(NS >= 1, "corrector LDS holds at least one value per voxel");
    __shared__ T cache[NS][kTileVox];
    if (ctl_failed(ctl)) return;
    const int ntiles = ta.nt[0] * ta.nt[1] * ta.nt[2];
    const int tile = (int)xcd_item(ntiles);
    if (tile >= ntiles) return;
    const int t0[3] = {(tile % ta.nt[0]) * ta.t[0], ((tile / ta.nt[0]) % ta.nt[1]) * ta.t[1],
                       (tile / (ta.nt[0] * ta.nt[1])) * ta.t[2]};
    const int tvol = ta.t[0] * ta.t[1] * ta.t[2];
    // the thread's voxels: offsets in the tile, and the x offset in bytes
    int vc[kVpt][3];
    unsigned bx[kVpt];
    bool valid[kVpt];
#pragma unroll
    for (int i = 0; i < kVpt; ++i) {
        const int v = threadIdx.x + i * kBlock;
        valid[i] = v < tvol;
        vc[i][0] = v % ta.t[0];
        vc[i][1] = (v / ta.t[0]) % ta.t[1];
        vc[i][2] = v / (ta.t[0] * ta.t[1]);
        bx[i] = (unsigned)vc[i][0] * (unsigned)sizeof(T);
    }
    const int b = cov_off[tile], e = cov_off[tile + 1];
    // Linear case: membership, box coordinates, and the byte offset of the
    // value from base (below 2^32: ext <= 4096, tile offsets below 32).
    auto probe_lin = [&](const TileBox &tb, bool (&hit)[kVpt], int (&l)[kVpt][3], unsigned (&bo)[kVpt]) {
#pragma unroll
        for (int i = 0; i < kVpt; ++i) {
#pragma unroll
            for (int a = 0; a < 3; ++a) l[i][a] = tb.d[a] + vc[i][a];
            hit[i] = valid[i] && (unsigned)l[i][0] < (unsigned)tb.e[0] && (unsigned)l[i][1] < (unsigned)tb.e[1] &&
                     (unsigned)l[i][2] < (unsigned)tb.e[2];
            const unsigned r = (unsigned)vc[i][1] + (unsigned)__umul24(tb.e[1], vc[i][2]);
            bo[i] = bx[i] + (unsigned)__umul24(tb.e[0] * (int)sizeof(T), r);
        }
    };
    // Wrapped case: the same with the element index of the value.
    auto probe_wrap = [&](const TileBox &tb, bool (&hit)[kVpt], int (&l)[kVpt][3], long long (&ix)[kVpt]) {
#pragma unroll
        for (int i = 0; i < kVpt; ++i) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int q = tb.s[a] + vc[i][a];
                l[i][a] = q >= ta.n[a] ? q - ta.n[a] : q;
            }
            hit[i] = valid[i] && l[i][0] < tb.e[0] && l[i][1] < tb.e[1] && l[i][2] < tb.e[2];
            ix[i] = tb.off + l[i][0] + (long long)tb.e[0] * (l[i][1] + (long long)tb.e[1] * l[i][2]);
        }
    };
    Top2<T> top[kVpt];
#pragma unroll
    for (int i = 0; i < kVpt; ++i) top[i].init();
    // values kept per voxel (pass 1), then values taken back (pass 2)
    int kept[kVpt];
#pragma unroll
    for (int i = 0; i < kVpt; ++i) kept[i] = 0;
    auto keep = [&](int i, T v) {
        if (kept[i] < NS) cache[kept[i] < NS ? kept[i] : 0][threadIdx.x + i * kBlock] = v;
        ++kept[i];
    };
    // Each wave holds the TileBoxes of 64 coverage entries, one per lane.
    const int lane_id = (int)(threadIdx.x & 63);
    TileBox wb;
    int held = -1;
    auto hold = [&](int cb) {
        if (held != cb) wb = tile_box(L, cov_list, cb + lane_id, e, t0, ta);
        held = cb;
    };
    // pass 1: top-2 over the covering grains, U linear boxes' loads issued
    // together.  The values of the first U boxes stay in registers (v0) for
    // pass 2, those of later ones in the LDS cache.
    constexpr int U = GG_CMP_U;
    auto load_group = [&](int c0, int cb, int ce, unsigned long long wrapped, T (&v)[U][kVpt], bool (&hit)[U][kVpt],
                          int (&jj)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = c0 + u;
#pragma unroll
            for (int i = 0; i < kVpt; ++i) hit[u][i] = false;
            jj[u] = -1;
            if (c >= ce || ((wrapped >> (c - cb)) & 1ull)) continue;
            const TileBox tb = box_of_lane<false>(wb, c - cb);
            jj[u] = tb.j;
            int l[kVpt][3];
            unsigned bo[kVpt];
            probe_lin(tb, hit[u], l, bo);
            const T *pb = psi + tb.base;
#pragma unroll
            for (int i = 0; i < kVpt; ++i)
                if (hit[u][i]) v[u][i] = at_bytes(pb, bo[i]);
        }
    };
    T v0[U][kVpt];
    for (int cb = b; cb < e; cb += 64) {
        hold(cb);
        const int ce = min(e, cb + 64);
        const unsigned long long wrapped = __ballot(cb + lane_id < e && !wb.lin);
        int c0 = cb;
        if (cb == b) {
            bool hit[U][kVpt];
            int jj[U];
            load_group(b, cb, ce, wrapped, v0, hit, jj);
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int i = 0; i < kVpt; ++i) top[i].template push<IDS>(v0[u][i], jj[u], hit[u][i]);
            c0 += U;
        }
        for (; c0 < ce; c0 += U) {
            T v[U][kVpt];
            bool hit[U][kVpt];
            int jj[U];
            load_group(c0, cb, ce, wrapped, v, hit, jj);
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int i = 0; i < kVpt; ++i) {
                    top[i].template push<IDS>(v[u][i], jj[u], hit[u][i]);
                    if (hit[u][i]) keep(i, v[u][i]);
                }
        }
        for (unsigned long long m = wrapped; m; m &= m - 1) {
            const int lane = __builtin_ctzll(m);
            const TileBox tb = box_of_lane<true>(wb, lane);
            bool hit[kVpt];
            int l[kVpt][3];
            long long ix[kVpt];
            probe_wrap(tb, hit, l, ix);
#pragma unroll
            for (int i = 0; i < kVpt; ++i) {
                const T v = hit[i] ? psi[ix[i]] : T(0);
                top[i].template push<IDS>(v, tb.j, hit[i]);
            }
        }
    }
    // pass 2: the corrected function of every covering grain
#pragma unroll
    for (int i = 0; i < kVpt; ++i) kept[i] = 0;
    // REG: the values come from rv (a linear box among the first U)
    auto emit = [&](auto lin, auto reg, const TileBox &tb, const T (&rv)[kVpt]) {
        constexpr bool LIN = decltype(lin)::value, REG = decltype(reg)::value;
        const int j = tb.j;
        bool hit[kVpt];
        int l[kVpt][3];
        unsigned bo[kVpt];
        long long ix[kVpt];
        if constexpr (LIN) probe_lin(tb, hit, l, bo);
        else probe_wrap(tb, hit, l, ix);
        T val[kVpt];
#pragma unroll
        for (int i = 0; i < kVpt; ++i) {
            if constexpr (REG) {
                val[i] = rv[i];
            } else if constexpr (LIN) {
                // the LDS slot is read for every lane (clamped), HBM only for
                // the values that were not kept
                const int k = kept[i];
                val[i] = cache[k < NS ? k : NS - 1][threadIdx.x + i * kBlock];
                if (hit[i] && k >= NS) val[i] = at_bytes(psi + tb.base, bo[i]);
                kept[i] += hit[i] ? 1 : 0;
            } else if (hit[i]) {
                val[i] = psi[ix[i]];
            }
        }
        int mn[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, mx[3] = {-1, -1, -1};
#pragma unroll
        for (int i = 0; i < kVpt; ++i) {
            if (!hit[i]) continue;
            const bool first = top[i].i1 == j;
            if constexpr (IDS) {
                const int other = first ? top[i].i2 : top[i].i1;
                if constexpr (LIN) at_bytes(iota_out + tb.base, bo[i] / (unsigned)(sizeof(T) / sizeof(int))) = other;
                else iota_out[ix[i]] = other;
            }
            if (mode != 0) continue;
            const T m = first ? (top[i].i2 < 0 ? -W : top[i].m2) : top[i].m1;
            const T pc = T(0.5) * (val[i] - m);
            if constexpr (LIN) at_bytes(phic + tb.base, bo[i]) = pc;
            else phic[ix[i]] = pc;
            if (pc > T(0)) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    mn[a] = min(mn[a], l[i][a]);
                    mx[a] = max(mx[a], l[i][a]);
                    if (tb.e[a] == ta.n[a])
                        atomicOr(&occ[((long long)j * 3 + a) * ta.occ_words + (l[i][a] >> 5)], 1u << (l[i][a] & 31));
                }
            }
        }
        if (mode != 0) return;
        if (__ballot(mx[0] >= 0) == 0) return;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            mn[a] = wave_min(mn[a]);
            mx[a] = wave_max(mx[a]);
        }
        if ((threadIdx.x & 63) == 0 && mx[0] >= 0) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                atomicMin(&bmin[3 * j + a], mn[a]);
                atomicMax(&bmax[3 * j + a], mx[a]);
            }
        }
    };
    using Lin = std::integral_constant<bool, true>;
    using Wrap = std::integral_constant<bool, false>;
    using Reg = std::integral_constant<bool, true>;
    using Mem = std::integral_constant<bool, false>;
    for (int cb = b; cb < e; cb += 64) {
        hold(cb);
        const int ce = min(e, cb + 64);
        int c = cb;
        if (cb == b) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (b + u >= ce) continue;
                if (__builtin_amdgcn_readlane(wb.lin, u)) emit(Lin{}, Reg{}, box_of_lane<false>(wb, u), v0[u]);
                else emit(Wrap{}, Mem{}, box_of_lane<true>(wb, u), v0[u]);
            }
            c += U;
        }
        for (; c < ce; ++c) {
            if (__builtin_amdgcn_readlane(wb.lin, c - cb)) emit(Lin{}, Mem{}, box_of_lane<false>(wb, c - cb), v0[0]);
            else emit(Wrap{}, Mem{}, box_of_lane<true>(wb, c - cb), v0[0]);
        }
    }
}
// Voxel labels: argmax over the covering grains (ties to the lowest id).
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_labels(Boxes L, const int *__restrict__ cov_off, const int *__restrict__ cov_list, const T *__restrict__ phi,
             int *__restrict__ labels, TileArgs ta) {
    const int tile = blockIdx.x;
    const int tx = tile % ta.nt[0], ty = (tile / ta.nt[0]) % ta.nt[1], tz = tile / (ta.nt[0] * ta.nt[1]);
    const int tvol = ta.t[0] * ta.t[1] * ta.t[2];
    const int b = cov_off[tile], e = cov_off[tile + 1];
    for (int v = threadIdx.x; v < tvol; v += kBlock) {
        const int gx = tx * ta.t[0] + v % ta.t[0], gy = ty * ta.t[1] + (v / ta.t[0]) % ta.t[1],
                  gz = tz * ta.t[2] + v / (ta.t[0] * ta.t[1]);
        T best = -tinf<T>();
        int id = -1;
        for (int c = b; c < e; ++c) {
            const int j = cov_list[c];
            const int lx = wrap_diff(gx, L.lo[3 * j], ta.n[0]), ly = wrap_diff(gy, L.lo[3 * j + 1], ta.n[1]),
                      lz = wrap_diff(gz, L.lo[3 * j + 2], ta.n[2]);
            const int ex = L.ext[3 * j], ey = L.ext[3 * j + 1], ez = L.ext[3 * j + 2];
            if (lx < ex && ly < ey && lz < ez) {
                const T v2 = phi[L.off[j] + lx + (long long)ex * (ly + (long long)ey * lz)];
                if (v2 > best || (v2 == best && j < id)) {
                    best = v2;
                    id = j;
                }
            }
        }
        labels[gx + (long long)ta.n[0] * (gy + (long long)ta.n[1] * gz)] = id;
    }
}

// ------------------------------------------------------ re-initialization (a4)

// phi^c of the old layout read at new-layout local coordinates (x, y, z):
// outside the new box or outside the old box the value is -W.
template <typename T> struct Carry {
    const T *src;
    int nex[3], oex[3], d[3], n[3];  // d = (new lo - old lo) mod n
    long long ooff;
    T W;
    __device__ __forceinline__ long long old_index(int x, int y, int z) const {
        const int xm = axis_map(x, nex[0], n[0]), ym = axis_map(y, nex[1], n[1]), zm = axis_map(z, nex[2], n[2]);
        if (xm < 0 || ym < 0 || zm < 0) return -1;
        int ox = xm + d[0], oy = ym + d[1], oz = zm + d[2];
        ox -= ox >= n[0] ? n[0] : 0;
        oy -= oy >= n[1] ? n[1] : 0;
        oz -= oz >= n[2] ? n[2] : 0;
        if (ox >= oex[0] || oy >= oex[1] || oz >= oex[2]) return -1;
        return ooff + ox + (long long)oex[0] * (oy + (long long)oex[1] * oz);
    }
    __device__ __forceinline__ T value(int x, int y, int z) const {
        const long long i = old_index(x, y, z);
        return i >= 0 ? src[i] : -W;
    }
    // Offsets relative to the old box start, for per-tile tables: >= 0 inside
    // both boxes, -1 inside the new box only, -2 outside the new box.
    __device__ __forceinline__ int row_code(int y, int z) const {
        const int ym = axis_map(y, nex[1], n[1]), zm = axis_map(z, nex[2], n[2]);
        if (ym < 0 || zm < 0) return -2;
        int oy = ym + d[1], oz = zm + d[2];
        oy -= oy >= n[1] ? n[1] : 0;
        oz -= oz >= n[2] ? n[2] : 0;
        if (oy >= oex[1] || oz >= oex[2]) return -1;
        return oex[0] * (oy + oex[1] * oz);
    }
    __device__ __forceinline__ int col_code(int x) const {
        const int xm = axis_map(x, nex[0], n[0]);
        if (xm < 0) return -2;
        int ox = xm + d[0];
        ox -= ox >= n[0] ? n[0] : 0;
        return ox < oex[0] ? ox : -1;
    }
    // Separable form of old_index: old_row(y, z) + old_col(x), each -1 outside.
    __device__ __forceinline__ long long old_row(int y, int z) const {
        const int ym = axis_map(y, nex[1], n[1]), zm = axis_map(z, nex[2], n[2]);
        if (ym < 0 || zm < 0) return -1;
        int oy = ym + d[1], oz = zm + d[2];
        oy -= oy >= n[1] ? n[1] : 0;
        oz -= oz >= n[2] ? n[2] : 0;
        if (oy >= oex[1] || oz >= oex[2]) return -1;
        return ooff + (long long)oex[0] * (oy + (long long)oex[1] * oz);
    }
    __device__ __forceinline__ int old_col(int x) const {
        const int xm = axis_map(x, nex[0], n[0]);
        if (xm < 0) return -1;
        int ox = xm + d[0];
        ox -= ox >= n[0] ? n[0] : 0;
        return ox < oex[0] ? ox : -1;
    }
};


// Reference values next to the sign change, then the x and y spreading sweeps,
// on one tile of nz consecutive z planes of the new box.  3D: writes the partial
// distance with the inside flag as its sign bit; 2D: writes the final function
// and the tile's volume.  Also carries the ID-field over to the new layout.
//
// LDS: nz f planes and nz reference planes, each FH rows of pitch FP (the tile
// with one ring of stencil neighbours), then int tables of offsets relative to
// the old box start: f rows of every plane, the rows of the planes just below
// and above the batch (whose z neighbours are read from memory; the batch's
// Reference values of the Euclidean re-initialization variant on one tile of
// nz consecutive z planes of the new box: |phi| / |grad phi| (central
// differences summed in axis order) capped by the axis intercept theta = phi /
// (phi - phi_n), at cells with a face neighbour across the sign change, +inf
// elsewhere; written with the inside flag as the sign bit.  Also carries the
// ID-field over to the new layout.
//
// LDS: nz f planes and nz reference planes, each FH rows of pitch FP (the tile
// with one ring of stencil neighbours), then int tables of offsets relative to
// the old box start: f rows of every plane, the rows of the planes just below
// and above the batch (whose z neighbours are read from memory; the batch's
// inner planes take theirs from LDS), and the f columns.
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_reinit_xy(Boxes Lo, Boxes Ln, ItemRefs ir, const T *__restrict__ phic, T *__restrict__ out,
                const int *__restrict__ iota_old, int *__restrict__ iota_new, T W, GridArgs g) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);
    const long long cls_item = xcd_item(ir.n);
    if (cls_item >= ir.n) return;
    const ItemTile it = decode_item(cls_item, KIND_RXY, Ln, ir);
    const int k = it.k, z0 = it.plane, nz = it.np, x0 = it.x0, y0 = it.y0, wx = it.wx, wy = it.wy;
    Carry<T> cr;
    cr.src = phic;
    cr.W = W;
    cr.ooff = Lo.off[k];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cr.nex[a] = Ln.ext[3 * k + a];
        cr.oex[a] = Lo.ext[3 * k + a];
        cr.n[a] = g.n[a];
        const int dd = Ln.lo[3 * k + a] - Lo.lo[3 * k + a];  // both in [0, n)
        cr.d[a] = dd < 0 ? dd + g.n[a] : dd;
    }
    const int ex = cr.nex[0], ey = cr.nex[1];
    const int RW = wx, RH = wy;
    const int FW = RW + 2, FP = FW | 1, FH = RH + 2, PS = FH * FP;
    T *f = sm, *ref = sm + nz * PS;
    int *rtab = reinterpret_cast<int *>(ref + nz * PS), *rzm = rtab + nz * FH, *rzp = rzm + FH, *ctab = rzp + FH;
    const T *src = phic + cr.ooff;
    const T inf = tinf<T>();
    const bool d3 = g.dim == 3;
    for (int i = threadIdx.x; i < nz * FH; i += kBlock) {
        const int p = i / FH;
        rtab[i] = cr.row_code(y0 - 1 + i - p * FH, z0 + p);
    }
    if (d3)
        for (int i = threadIdx.x; i < FH; i += kBlock) {
            rzm[i] = cr.row_code(y0 - 1 + i, z0 - 1);
            rzp[i] = cr.row_code(y0 - 1 + i, z0 + nz);
        }
    for (int i = threadIdx.x; i < FW; i += kBlock) ctab[i] = cr.col_code(x0 - 1 + i);
    __syncthreads();
    // stage the f planes (their rows are consecutive: row R = p * FH + r);
    // kLoadBatch loads in flight per lane: all table reads first, then the
    // loads without branches (a position off the old box loads the box's
    // first value and keeps -W), then the LDS stores
    const int NR = nz * FH;
    for (Walk2 w(threadIdx.x, FW); w.r < NR;) {
        int ro[kLoadBatch], co[kLoadBatch], at[kLoadBatch];
#pragma unroll
        for (int j = 0; j < kLoadBatch; ++j) {
            const bool ok = w.r < NR;
            ro[j] = rtab[ok ? w.r : 0];
            co[j] = ctab[ok ? w.c : 0];
            at[j] = ok ? w.r * FP + w.c : -1;
            w.step();
        }
        T v[kLoadBatch];
#pragma unroll
        for (int j = 0; j < kLoadBatch; ++j) {
            const bool hit = (ro[j] | co[j]) >= 0;
            const T x = src[hit ? ro[j] + co[j] : 0];
            v[j] = hit ? x : -W;
        }
#pragma unroll
        for (int j = 0; j < kLoadBatch; ++j)
            if (at[j] >= 0) f[at[j]] = v[j];
    }
    __syncthreads();
    // reference values: each lane takes cell positions of the tile and walks
    // them through the nz planes, so that the z neighbours of a cell are the
    // previous and next centre values (memory only below the first and above
    // the last plane, fetched one position ahead).  Over all neighbours, the
    // smallest value is <= 0 exactly when an inside cell has an outside
    // neighbour, and then it is the extreme one; likewise the largest for an
    // outside cell.  theta = fc / (fc - fn) is monotone in fn on that side, and
    // so are the rounded operations, so the extreme neighbour gives the
    // smallest theta.
    {
        Walk2 w(threadIdx.x, RW);
        T zm_n = -W, zp_n = -W;
        auto fetch = [&](int r, int c) {
            zm_n = zp_n = -W;
            if (d3 && r < RH) {
                const int co = ctab[c + 1], rm = rzm[r + 1], rp = rzp[r + 1];
                if (rm >= 0 && co >= 0) zm_n = src[rm + co];
                if (rp >= 0 && co >= 0) zp_n = src[rp + co];
            }
        };
        fetch(w.r, w.c);
        while (w.r < RH) {
            const int r = w.r + 1, c = w.c + 1;
            T zm = zm_n;
            const T zlast = zp_n;
            w.step();
            fetch(w.r, w.c);
            const bool colin = ctab[c] != -2;
            int a = r * FP + c;
            T cur = f[a];
            for (int p = 0; p < nz; ++p, a += PS) {
                const T nxt = p + 1 < nz ? f[a + PS] : zlast;
                T rv = inf;
                if (colin && rtab[p * FH + r] != -2) {
                    const T n0 = f[a - 1], n1 = f[a + 1], n2 = f[a - FP], n3 = f[a + FP];
                    T lo = vmin(vmin(n0, n1), vmin(n2, n3)), hi = vmax(vmax(n0, n1), vmax(n2, n3));
                    if (d3) {
                        lo = vmin(lo, vmin(zm, nxt));
                        hi = vmax(hi, vmax(zm, nxt));
                    }
                    const bool in = cur > T(0);
                    const T ext = in ? lo : hi;
                    if ((ext > T(0)) != in) {
                        rv = ratio(cur, cur - ext);
                        // |phi| / |grad phi|, central differences summed in
                        // axis order, capped by the axis intercept above
                        const T gx = (n1 - n0) * T(0.5), gy = (n3 - n2) * T(0.5);
                        T gg = gx * gx;
                        gg = gg + gy * gy;
                        if (d3) {
                            const T gz = (nxt - zm) * T(0.5);
                            gg = gg + gz * gz;
                        }
                        if (gg > T(0)) {
                            const T r = grad_dist(fabs(cur), gg);
                            rv = rv < r ? rv : r;
                        }
                    }
                }
                ref[a] = rv;
                zm = cur;
                cur = nxt;
            }
        }
    }
    __syncthreads();
    T *outk = out + Ln.off[k];
    int *io_new = iota_new ? iota_new + Ln.off[k] : nullptr;
    const int *io_old = iota_old ? iota_old + cr.ooff : nullptr;
    const int plane_vals = ex * ey;
    for (Walk2 w(threadIdx.x, wx); w.r < wy; w.step()) {
        int a = (w.r + 1) * FP + w.c + 1;
        int idx = (z0 * ey + y0 + w.r) * ex + x0 + w.c;
        const int co = ctab[w.c + 1];
        for (int p = 0; p < nz; ++p, a += PS, idx += plane_vals) {
            // reference value (+inf elsewhere) for the Jacobi sweeps, the
            // inside flag in the sign bit (a zero value keeps it as well)
            const T m = fabs(ref[a]);
            outk[idx] = f[a] > T(0) ? m : -m;
            if (io_new) {
                const int ro = rtab[p * FH + w.r + 1];
                io_new[idx] = (ro >= 0 && co >= 0) ? io_old[ro + co] : -1;
            }
        }
    }
}


// Godunov's upwind update on a unit grid: the largest root u of
// sum over the a_i below u of (u - a_i)^2 = 1, for neighbour values a1..a3
// (+inf: no neighbour along that axis).  The three are sorted first; one
// neighbour gives a + 1, two the quadratic's root, three the cubic's.
// Square root and division by 3 for the update: correctly rounded in FP64; in
// FP32 (the mixed path) the hardware square root (1 ulp) and the product with
// the rounded 1/3.
__device__ __forceinline__ double upd_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float upd_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double upd_third(double x) { return x / 3.0; }
__device__ __forceinline__ float upd_third(float x) { return x * (1.0f / 3.0f); }
// A 32-bit word whose bit 31 is the sign bit of x.
__device__ __forceinline__ int sign_word(float x) { return __float_as_int(x); }
__device__ __forceinline__ int sign_word(double x) { return __double2hiint(x); }

template <typename T> __device__ __forceinline__ T godunov(T a1, T a2, T a3) {
    T t;
    if (a2 < a1) { t = a1; a1 = a2; a2 = t; }
    if (a3 < a2) { t = a2; a2 = a3; a3 = t; }
    if (a2 < a1) { t = a1; a1 = a2; a2 = t; }
    T u = a1 + T(1);
    if (u > a2) {
        const T d = a1 - a2;
        u = (a1 + a2 + upd_sqrt(T(2) - d * d)) * T(0.5);
        if (u > a3) {
            const T s1 = a1 + a2 + a3, s2 = a1 * a1 + a2 * a2 + a3 * a3;
            u = upd_third(s1 + upd_sqrt(s1 * s1 - T(3) * (s2 - T(1))));
        }
    }
    return u;
}

// One Jacobi sweep of the Euclidean re-initialization over a work item (an xy
// tile of consecutive z planes) of the new box: src -> dst, distances with the
// inside flag in the sign bit.  A cell with a face neighbour on the other side
// of the interface (a cell outside the box counts as outside the grain) keeps
// its reference value; every other cell takes min(u, godunov(a_x, a_y, a_z)),
// a_i the smaller magnitude of its two neighbours along axis i that lie in the
// box.  `final2d` (the last sweep in 2D) stores the band-clamped function and
// the tile's volume instead.
//
// The item marches through its planes with a ring of three LDS planes, each the
// tile and one ring of neighbours (FW x FH, -inf where the neighbour is not in
// the box: outside the grain, magnitude +inf).  While one plane is updated from
// LDS, the lanes' loads of the plane two ahead are in flight in registers.
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_jacobi(Boxes Ln, ItemRefs ir, const T *__restrict__ src, T *__restrict__ dst, double *__restrict__ vol_part,
             T W, int final2d, GridArgs g) {
    static_assert(budget_values<T>(kLdsBytesMax) / 3 <= kJacQ * kBlock, "a Jacobi plane must fit the lanes' registers");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);
    __shared__ double red[kBlock / 64];
    const long long cls_item = xcd_item(ir.n);
    if (cls_item >= ir.n) return;
    const ItemTile it = decode_item(cls_item, KIND_JAC, Ln, ir);
    const int k = it.k, z0 = it.plane, nz = it.np, x0 = it.x0, y0 = it.y0, wx = it.wx, wy = it.wy;
    const int ex = Ln.ext[3 * k], ey = Ln.ext[3 * k + 1], ez = Ln.ext[3 * k + 2];
    const T *u = src + Ln.off[k];
    T *v = dst + Ln.off[k];
    const T inf = tinf<T>();
    const bool d3 = g.dim == 3;
    const int plane = ex * ey;
    const int FW = wx + 2, FH = wy + 2, PS = FW * FH;
    int *ctab = reinterpret_cast<int *>(sm + 3 * PS), *rtab = ctab + FW;
    for (int i = threadIdx.x; i < FW; i += kBlock) ctab[i] = axis_map(x0 - 1 + i, ex, g.n[0]);
    for (int i = threadIdx.x; i < FH; i += kBlock) {
        const int yy = axis_map(y0 - 1 + i, ey, g.n[1]);
        rtab[i] = yy < 0 ? -1 : yy * ex;
    }
    __syncthreads();
    // in-plane offsets of this lane's ring positions (-1: not in the box)
    int qo[kJacQ];
#pragma unroll
    for (int j = 0; j < kJacQ; ++j) {
        const int q = j * kBlock + threadIdx.x;
        qo[j] = -1;
        if (q < PS) {
            const int r = q / FW, c = q - r * FW;
            const int ro = rtab[r], co = ctab[c];
            if (ro >= 0 && co >= 0) qo[j] = ro + co;
        }
    }
    T nx[kJacQ];
    auto fetch = [&](int z) {  // plane z (any integer) into registers
        const int zz = d3 ? axis_map(z, ez, g.n[2]) : (z == 0 ? 0 : -1);
        const T *pz = u + (zz < 0 ? 0 : zz) * plane;
#pragma unroll
        for (int j = 0; j < kJacQ; ++j) {
            nx[j] = -inf;
            if (zz >= 0 && qo[j] >= 0) nx[j] = pz[qo[j]];
        }
    };
    auto stash = [&](int slot) {
        T *d = sm + slot * PS;
#pragma unroll
        for (int j = 0; j < kJacQ; ++j) {
            const int q = j * kBlock + threadIdx.x;
            if (q < PS) d[q] = nx[j];
        }
    };
    fetch(z0 - 1);
    stash(0);
    fetch(z0);
    stash(1);
    fetch(z0 + 1);
    double vsum = 0.0;
    for (int p = 0; p < nz; ++p) {
        stash((p + 2) % 3);
        __syncthreads();
        if (p + 1 < nz) fetch(z0 + p + 2);
        const T *lo = sm + (p % 3) * PS, *mid = sm + ((p + 1) % 3) * PS, *hi = sm + ((p + 2) % 3) * PS;
        const int zoff = (z0 + p) * plane;
        for (Walk2 w(threadIdx.x, wx); w.r < wy; w.step()) {
            const int a = (w.r + 1) * FW + w.c + 1;
            const T cur = mid[a], nxm = mid[a - 1], nxp = mid[a + 1], nym = mid[a - FW], nyp = mid[a + FW];
            const T zlo = lo[a], zhi = hi[a];
            // a neighbour on the other side: a sign bit that differs from the cell's
            const int wc = sign_word(cur);
            int diff = (sign_word(nxm) ^ wc) | (sign_word(nxp) ^ wc) | (sign_word(nym) ^ wc) | (sign_word(nyp) ^ wc);
            if (d3) diff |= (sign_word(zlo) ^ wc) | (sign_word(zhi) ^ wc);
            const bool sc = wc < 0, fixed = diff < 0;
            const T mc = fabs(cur);
            T res = mc;
            if (!fixed) {
                const T ax = vmin(fabs(nxm), fabs(nxp)), ay = vmin(fabs(nym), fabs(nyp));
                const T az = d3 ? vmin(fabs(zlo), fabs(zhi)) : inf;
                const T gv = godunov(ax, ay, az);
                res = gv < mc ? gv : mc;
            }
            const int idx = zoff + (y0 + w.r) * ex + x0 + w.c;
            if (final2d) {
                const T dc = res < W ? res : W;
                const T pv = sc ? -dc : dc;
                v[idx] = pv;
                double cl = (double)pv + 0.5;
                cl = cl < 0.0 ? 0.0 : (cl > 1.0 ? 1.0 : cl);
                vsum += cl;
            } else {
                v[idx] = fixed ? cur : (sc ? -res : res);
            }
        }
        __syncthreads();
    }
    if (final2d) {
        const double s = block_sum(vsum, red);
        if (threadIdx.x == 0) vol_part[it.item] = s;
    }
}

// ------------------------------------------------------------ grid coarsening
//
// Projection onto a coarser periodic grid np (the ratio r = n / np on every
// axis): new node i' sits at old position i' n / np = i0 + rem / np (exact
// integer split).  A grain's value there is its old function (-W outside the
// old box) interpolated linearly along x, then y, then z, divided by r.
template <typename T> struct CoarsenArgs {
    int n[3], np[3];
    int dim;
    T W, r;
};

template <typename T>
__device__ T coarse_value(const T *__restrict__ f, const int *lo, const int *e, const CoarsenArgs<T> &ca, int gx,
                          int gy, int gz) {
    const int g[3] = {gx, gy, gz};
    int i0[3] = {0, 0, 0};
    T t[3] = {T(0), T(0), T(0)};
    for (int a = 0; a < ca.dim; ++a) {
        const long long num = (long long)g[a] * ca.n[a];
        const long long q = num / ca.np[a];
        i0[a] = (int)q;
        t[a] = (T)(num - q * ca.np[a]) / (T)ca.np[a];
    }
    auto at = [&](int x, int y, int z) -> T {
        const int lx = imod((long long)x - lo[0], ca.n[0]), ly = imod((long long)y - lo[1], ca.n[1]),
                  lz = imod((long long)z - lo[2], ca.n[2]);
        if (lx >= e[0] || ly >= e[1] || lz >= e[2]) return -ca.W;
        return f[lx + (long long)e[0] * (ly + (long long)e[1] * lz)];
    };
    T c[2][2];
    const int nzc = ca.dim == 3 ? 2 : 1;
    for (int dz = 0; dz < nzc; ++dz)
        for (int dy = 0; dy < 2; ++dy) {
            const T v0 = at(i0[0], i0[1] + dy, i0[2] + dz), v1 = at(i0[0] + 1, i0[1] + dy, i0[2] + dz);
            c[dz][dy] = (T(1) - t[0]) * v0 + t[0] * v1;
        }
    T v[2];
    for (int dz = 0; dz < nzc; ++dz) v[dz] = (T(1) - t[1]) * c[dz][0] + t[1] * c[dz][1];
    const T u = ca.dim == 3 ? (T(1) - t[2]) * v[0] + t[2] * v[1] : v[0];
    return u / ca.r;
}

// New nodes whose value can be positive: along an axis the old box covers only
// partly, those with old position in [lo - 1, lo + ext] (a superset); along a
// whole axis, all.  Returns the first node (unwrapped) and the count.
__device__ __forceinline__ void coarse_region(int lo, int ext, int N, int Np, int *first, int *count) {
    if (ext == N) {
        *first = 0;
        *count = Np;
        return;
    }
    const long long a = (long long)(lo - 1) * Np, b = (long long)(lo + ext) * Np;
    const long long f0 = a >= 0 ? a / N : -((-a + N - 1) / N);  // floor
    const long long l0 = b / N + 1;
    long long c = l0 - f0 + 1;
    *first = (int)f0;
    *count = (int)(c < Np ? c : Np);
}

// Positive nodes of every grain's projection: occupancy bits per axis over the
// new grid (the box plan's whole-axis rule then gives the new box) and a
// positive flag in bmax.  Grid (G, y): the y blocks of a grain stride over its
// region.
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_coarsen_mark(Boxes L, const T *__restrict__ phi, CoarsenArgs<T> ca, int *bmax, unsigned *occ, int occ_words) {
    const int k = blockIdx.x;
    if (!L.alive[k]) return;
    const int *lo = L.lo + 3 * k, *e = L.ext + 3 * k;
    const T *f = phi + L.off[k];
    int first[3], cnt[3];
    for (int a = 0; a < 3; ++a) coarse_region(lo[a], e[a], ca.n[a], ca.np[a], &first[a], &cnt[a]);
    // at most the new grid's voxel count (< 2^31)
    const int total = cnt[0] * cnt[1] * cnt[2];
    bool any = false;
    for (int i = blockIdx.y * kBlock + threadIdx.x; i < total; i += gridDim.y * kBlock) {
        const int yz = i / cnt[0], x = i - yz * cnt[0];
        const int z = yz / cnt[1], y = yz - z * cnt[1];
        const int gx = imod((long long)first[0] + x, ca.np[0]), gy = imod((long long)first[1] + y, ca.np[1]),
                  gz = imod((long long)first[2] + z, ca.np[2]);
        if (coarse_value(f, lo, e, ca, gx, gy, gz) > T(0)) {
            any = true;
            const int g[3] = {gx, gy, gz};
            for (int a = 0; a < 3; ++a)
                atomicOr(&occ[((long long)k * 3 + a) * occ_words + (g[a] >> 5)], 1u << (g[a] & 31));
        }
    }
    if (any) atomicMax(&bmax[3 * k], 0);
}

// Projected values on the new boxes (layout Ln), before re-initialization.
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_coarsen_values(Boxes Lo, const T *__restrict__ phi, Boxes Ln, T *__restrict__ out, CoarsenArgs<T> ca) {
    const int k = blockIdx.x;
    if (!Ln.alive[k]) return;
    const int *lo = Lo.lo + 3 * k, *e = Lo.ext + 3 * k, *nlo = Ln.lo + 3 * k, *ne = Ln.ext + 3 * k;
    const T *f = phi + Lo.off[k];
    T *o = out + Ln.off[k];
    const int total = ne[0] * ne[1] * ne[2];  // a box volume: < 2^31
    for (int i = blockIdx.y * kBlock + threadIdx.x; i < total; i += gridDim.y * kBlock) {
        const int yz = i / ne[0], x = i - yz * ne[0];
        const int z = yz / ne[1], y = yz - z * ne[1];
        o[i] = coarse_value(f, lo, e, ca, imod((long long)nlo[0] + x, ca.np[0]), imod((long long)nlo[1] + y, ca.np[1]),
                            imod((long long)nlo[2] + z, ca.np[2]));
    }
}

// ---------------------------------------------------------- interface areas
//
// Interface area of grain k: the sum over its box of |grad H(phi_k)|, H =
// clamp(phi + 1/2, 0, 1) (the volume's smoothed Heaviside), central
// differences with -W outside the box, squares summed over the axes in order,
// all in FP64; `weighted` multiplies each voxel by the Read-Shockley energy of
// the pair (k, iota) when the misorientation weights are on.  Grid (G, split):
// block y of grain k writes its partial sums to part[k * split + y] (areas) and
// part[(G + k) * split + y] (weighted).
struct AreaArgs {
    int mode;             // GG_PHYS_* bits
    double theta_c_deg;
    int split, G;
};

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_areas(Boxes L, const T *__restrict__ phi, const int *__restrict__ iota, const T *__restrict__ quat, AreaArgs aa,
            double *__restrict__ part, T W, GridArgs g) {
    __shared__ double red[kBlock / 64];
    const int k = blockIdx.x;
    double acc = 0.0, accw = 0.0;
    if (L.alive[k]) {
        const int ex = L.ext[3 * k], ey = L.ext[3 * k + 1], ez = L.ext[3 * k + 2];
        const T *f = phi + L.off[k];
        const int *io = iota ? iota + L.off[k] : nullptr;
        const int total = ex * ey * ez;  // a box volume: < 2^31
        const int e3[3] = {ex, ey, ez};
        int jc = -2;
        double gam_c = 1.0;
        for (int i = blockIdx.y * kBlock + threadIdx.x; i < total; i += gridDim.y * kBlock) {
            const int yz = i / ex, x = i - yz * ex;
            const int z = yz / ey, y = yz - z * ey;
            const int c[3] = {x, y, z};
            double gg = 0.0;
            for (int a = 0; a < g.dim; ++a) {
                double h2[2];
                for (int s = 0; s < 2; ++s) {
                    int q[3] = {c[0], c[1], c[2]};
                    q[a] = axis_map(c[a] + (s ? 1 : -1), e3[a], g.n[a]);
                    const double v = q[a] < 0 ? -(double)W : (double)f[q[0] + ex * (q[1] + ey * q[2])];
                    const double hv = v + 0.5;
                    h2[s] = hv < 0.0 ? 0.0 : (hv > 1.0 ? 1.0 : hv);
                }
                const double gd = (h2[1] - h2[0]) * 0.5;
                gg = gg + gd * gd;
            }
            const double m = sqrt(gg);
            acc = acc + m;
            double gam = 1.0;
            if (io && (aa.mode & 1) && m > 0.0) {
                const int j = io[i];
                if (j >= 0) {
                    if (j != jc) {
                        jc = j;
                        gam_c = (double)read_shockley<T>(misorientation_deg<T>(quat + 4LL * k, quat + 4LL * j),
                                                         (T)aa.theta_c_deg);
                    }
                    gam = gam_c;
                }
            }
            accw = accw + m * gam;
        }
    }
    const double s0 = block_sum(acc, red);
    if (threadIdx.x == 0) part[(long long)k * aa.split + blockIdx.y] = s0;
    const double s1 = block_sum(accw, red);
    if (threadIdx.x == 0) part[((long long)aa.G + k) * aa.split + blockIdx.y] = s1;
}

// Sum of the `split` partials of row i, in order, for the 2G rows of k_areas:
// rows [0, G) into out0, rows [G, 2G) into out1 (skipped when out1 is NULL).
__global__ void k_sum_rows(const double *__restrict__ part, double *__restrict__ out0, double *__restrict__ out1,
                           int G, int split) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * G || (i >= G && !out1)) return;
    double s = 0.0;
    for (int j = 0; j < split; ++j) s += part[(long long)i * split + j];
    if (i < G) out0[i] = s;
    else out1[i - G] = s;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_init_indicator(Boxes L, const int *__restrict__ labels, T *__restrict__ out,
                                                           GridArgs g) {
    const int k = blockIdx.x;
    if (!L.alive[k]) return;
    const int ex = L.ext[3 * k], ey = L.ext[3 * k + 1], ez = L.ext[3 * k + 2];
    const long long m = (long long)ex * ey * ez;
    for (long long v = threadIdx.x; v < m; v += kBlock) {
        const int x = (int)(v % ex), y = (int)((v / ex) % ey), z = (int)(v / ((long long)ex * ey));
        const int gx = imod((long long)L.lo[3 * k] + x, g.n[0]);
        const int gy = imod((long long)L.lo[3 * k + 1] + y, g.n[1]);
        const int gz = imod((long long)L.lo[3 * k + 2] + z, g.n[2]);
        const int lab = labels[gx + (long long)g.n[0] * (gy + (long long)g.n[1] * gz)];
        out[L.off[k] + v] = lab == k ? T(0.5) : T(-0.5);
    }
}
// -------------------------------------------------------------- bookkeeping

// Covered cyclic interval of a bit row: complement of the largest run of zeros
// (ties to the run with the smallest start).  Returns false if no bit is set.
__device__ inline bool cyclic_cover_bits(const unsigned *w, int N, int *start, int *len) {
    int first = -1, ones = 0;
    for (int i = 0; i < N; ++i)
        if ((w[i >> 5] >> (i & 31)) & 1u) {
            if (first < 0) first = i;
            ++ones;
        }
    if (first < 0) return false;
    if (ones == N) {
        *start = 0;
        *len = N;
        return true;
    }
    int best_s = -1, best_l = -1, run_s = -1, run_l = 0;
    for (int t = 1; t <= N; ++t) {
        const int i = (first + t) % N;
        const bool set = (w[i >> 5] >> (i & 31)) & 1u;
        if (!set) {
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
    *start = (best_s + best_l) % N;
    *len = N - best_l;
    return true;
}

struct PlanArgs {
    int n[3];
    int P;
    int occ_words;
    int G;
};

// New boxes from the positive set of phi^c (sec. 3.1: size-adaptive boxes;
// extinction when the set is empty).  Resets the bounding-box accumulators.
__global__ void k_plan(Boxes Lo, Boxes Ln, int *bmin, int *bmax, unsigned *occ, long long *sizes, PlanArgs pa,
                       const Ctl *ctl) {
    if (ctl_failed(ctl)) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= pa.G) return;
    const bool alive = Lo.alive[k] && bmax[3 * k] >= 0;
    long long size = 0;
    if (alive) {
        size = 1;
        for (int a = 0; a < 3; ++a) {
            const int N = pa.n[a];
            int st, ln;
            if (Lo.ext[3 * k + a] == N) {
                cyclic_cover_bits(occ + ((long long)k * 3 + a) * pa.occ_words, N, &st, &ln);
                st = imod((long long)Lo.lo[3 * k + a] + st, N);
            } else {
                st = imod((long long)Lo.lo[3 * k + a] + bmin[3 * k + a], N);
                ln = bmax[3 * k + a] - bmin[3 * k + a] + 1;
            }
            const long long e = (long long)ln + 2LL * pa.P;
            int lo, ex;
            if (e > (long long)N - 2LL * pa.P) {
                lo = 0;
                ex = N;
            } else {
                lo = imod((long long)st - pa.P, N);
                ex = (int)e;
            }
            Ln.lo[3 * k + a] = lo;
            Ln.ext[3 * k + a] = ex;
            size *= ex;
        }
    } else {
        for (int a = 0; a < 3; ++a) {
            Ln.lo[3 * k + a] = 0;
            Ln.ext[3 * k + a] = 0;
        }
    }
    Ln.alive[k] = alive ? 1 : 0;
    sizes[k] = size;
    if (Lo.alive[k])
        for (int a = 0; a < 3; ++a)
            if (Lo.ext[3 * k + a] == pa.n[a]) {
                unsigned *w = occ + ((long long)k * 3 + a) * pa.occ_words;
                for (int i = 0; i < pa.occ_words; ++i) w[i] = 0u;
            }
    for (int a = 0; a < 3; ++a) {
        bmin[3 * k + a] = 0x7fffffff;
        bmax[3 * k + a] = -1;
    }
}

// Per-grain work item counts of the Euclidean variant's kinds, split into the
// two launch classes, the stored tilings, and the largest LDS need per class.
// cnt holds 3 arrays of G per kind: all items, class 0, class 1.
// One thread per (grain, kind); grid (ceil(G / 256), kKinds).  The per-class
// LDS maxima are reduced over the wave before one atomic per wave and class.
__global__ void k_item_counts(Boxes L, long long *cnt, int4 *tilings, unsigned long long *lds_max, int G, int budget,
                              int small) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x, q = blockIdx.y;
    unsigned long long need_c[kClasses] = {0, 0};
    if (k < G) {
        long long *c = cnt + (long long)q * 3 * G;
        c[k] = c[G + k] = c[2LL * G + k] = 0;
        int4 *rec = tilings + 2 * ((long long)q * G + k);
        rec[0] = rec[1] = make_int4(0, 0, 0, 0);
        if (L.alive[k]) {
            const int *e = L.ext + 3 * k;
            const Tiling t = kind_tiling(q, e, budget, small);
            rec[0] = make_int4(t.nxs, t.nys, t.tx, t.ty);
            rec[1] = make_int4(t.nb, 0, 0, 0);
            if (t.nxs == 0) {
                need_c[1] = 0xffffffffffffffffULL;  // infeasible tiling
            } else {
                const long long n = tiling_items(e, t);
                const long long need = tiling_need(q, t);
                const int cls = need <= small ? 0 : 1;
                c[k] = n;
                c[(1LL + cls) * G + k] = n;
                need_c[cls] = (unsigned long long)need;
            }
        }
    }
#pragma unroll
    for (int cl = 0; cl < kClasses; ++cl) {
        unsigned long long v = need_c[cl];
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long u = __shfl_xor(v, o, 64);
            v = u > v ? u : v;
        }
        if ((threadIdx.x & 63) == 0 && v) atomicMax(&lds_max[q * kClasses + cl], v);
    }
}

// Exclusive prefix sums of several arrays of n values (one work group each):
// array m is in[m * n ..], its prefix out[m * (n + 1) ..].
__global__ void __launch_bounds__(1024) k_scan_multi(const long long *in, long long *out, int n) {
    __shared__ long long part[1024];
    const long long *src = in + (long long)blockIdx.x * n;
    long long *dst = out + (long long)blockIdx.x * (n + 1);
    const int t = threadIdx.x;
    const int chunk = (n + 1023) / 1024;
    const int b = min(t * chunk, n), e = min(b + chunk, n);
    long long s = 0;
    for (int i = b; i < e; ++i) s += src[i];
    part[t] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const long long v = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    long long base = t ? part[t - 1] : 0;
    for (int i = b; i < e; ++i) {
        dst[i] = base;
        base += src[i];
    }
    if (t == 1023) dst[n] = part[1023];
}

// Exclusive prefix sum of n values (out has n + 1 entries), one work group.
// With a control block: a total above `cap` raises fail = 1 (the value arenas
// are too small for the new layout) and records the need.
__global__ void __launch_bounds__(1024) k_scan(const long long *in, long long *out, int n, Ctl *ctl, long long cap) {
    if (ctl_failed(ctl)) return;
    __shared__ long long part[1024];
    const int t = threadIdx.x;
    const int chunk = (n + 1023) / 1024;
    const int b = min(t * chunk, n), e = min(b + chunk, n);
    long long s = 0;
    for (int i = b; i < e; ++i) s += in[i];
    part[t] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const long long v = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    long long base = t ? part[t - 1] : 0;
    for (int i = b; i < e; ++i) {
        out[i] = base;
        base += in[i];
    }
    if (t == 1023) {
        out[n] = part[1023];
        if (ctl && part[1023] > cap) {
            ctl->need_arena = part[1023];
            ctl->fail_step = ctl->steps;
            ctl->fail = 1;
        }
    }
}

// Exclusive prefix sum of n coverage counts into `out` and `cur` (the fill
// kernel's cursors), one work group; the 64-bit total goes to *total.  A total
// above `cap` (or beyond 32-bit offsets) raises fail = 2 in the control block.
__global__ void __launch_bounds__(1024) k_scan_int(const int *in, int *out, int *cur, int n, long long *total, Ctl *ctl,
                                                   long long cap) {
    if (ctl_failed(ctl)) return;
    __shared__ long long part[1024];
    const int t = threadIdx.x;
    const int chunk = (n + 1023) / 1024;
    const int b = min(t * chunk, n), e = min(b + chunk, n);
    long long s = 0;
    int i = b;
    for (; i + 8 <= e; i += 8) {  // 8 loads in flight
        int v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = in[i + j];
#pragma unroll
        for (int j = 0; j < 8; ++j) s += v[j];
    }
    for (; i < e; ++i) s += in[i];
    part[t] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const long long v = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    long long base = t ? part[t - 1] : 0;
    i = b;
    for (; i + 8 <= e; i += 8) {
        int v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = in[i + j];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            out[i + j] = (int)base;
            cur[i + j] = (int)base;
            base += v[j];
        }
    }
    for (; i < e; ++i) {
        out[i] = (int)base;
        cur[i] = (int)base;
        base += in[i];
    }
    if (t == 1023) {
        const long long tot = part[1023];
        out[n] = (int)tot;
        cur[n] = (int)tot;
        *total = tot;
        if (ctl && (tot > cap || tot > 0x7fffffffLL)) {
            ctl->need_cov = tot;
            ctl->fail_step = ctl->steps;
            ctl->fail = 2;
        }
    }
}

// item -> grain maps, one per (kind, class) = blockIdx.y; pref holds the
// prefixes of one layout (3 per kind: all, class 0, class 1).
struct OwnerMaps {
    int *owner[kKinds * kClasses];
};
__global__ void k_fill_owner(const long long *pref, OwnerMaps om, int G) {
    const int k = blockIdx.x, q = blockIdx.y / kClasses, c = blockIdx.y % kClasses;
    const long long *p = pref + ((long long)q * 3 + 1 + c) * (G + 1);
    int *owner = om.owner[blockIdx.y];
    const long long b = p[k], e = p[k + 1];
    for (long long i = b + threadIdx.x; i < e; i += blockDim.x) owner[i] = k;
}

// Tiles of the global grid covered by a box along one axis: start tile and count.
__device__ inline void axis_tiles(int lo, int ext, int N, int T, int nt, int *t0, int *cnt) {
    if (ext == N) {
        *t0 = 0;
        *cnt = nt;
        return;
    }
    const int s = lo / T, l = (lo + ext - 1) / T;
    *t0 = s;
    *cnt = min(l - s + 1, nt);
}

// Coverage lists: for every global tile, the alive grains whose box covers it.
// mode 0 counts, mode 1 fills (cursor = running positions).
__global__ void k_coverage(Boxes L, int *cnt_or_cursor, int *list, TileArgs ta, int G, int mode, const Ctl *ctl) {
    if (ctl_failed(ctl)) return;
    const int k = blockIdx.x;
    if (!L.alive[k]) return;
    int t0[3], c[3];
    for (int a = 0; a < 3; ++a)
        axis_tiles(L.lo[3 * k + a], L.ext[3 * k + a], ta.n[a], ta.t[a], ta.nt[a], &t0[a], &c[a]);
    const int total = c[0] * c[1] * c[2];
    for (int q = threadIdx.x; q < total; q += blockDim.x) {
        const int ix = q % c[0], iy = (q / c[0]) % c[1], iz = q / (c[0] * c[1]);
        const int tx = (t0[0] + ix) % ta.nt[0], ty = (t0[1] + iy) % ta.nt[1], tz = (t0[2] + iz) % ta.nt[2];
        const int tile = tx + ta.nt[0] * (ty + ta.nt[1] * tz);
        if (mode == 0) {
            atomicAdd(&cnt_or_cursor[tile], 1);
        } else {
            const int p = atomicAdd(&cnt_or_cursor[tile], 1);
            list[p] = k;
        }
    }
}

// Per-grain volume from per-item partial sums, in item order (the Euclidean
// variant's last 2D sweep).  One wave per grain: lane-strided partial sums,
// then a butterfly (fixed order).
__global__ void __launch_bounds__(64) k_volumes(const Boxes L, const long long *pref, const double *vol_part,
                                                double *vol, int G) {
    const int k = blockIdx.x;
    if (k >= G) return;
    double s = 0.0;
    if (L.alive[k])
        for (long long i = pref[k] + threadIdx.x; i < pref[k + 1]; i += 64) s += vol_part[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (threadIdx.x == 0) vol[k] = s;
}

// Layout totals for the host: arena size, item counts and LDS maxima of the
// Euclidean kinds (when pref is given), coverage entries, alive grains.
__global__ void k_totals(const long long *arena_pref, const long long *pref, const long long *cov_total,
                         const int *alive, int G, const unsigned long long *lds_max, Totals *t) {
    if (threadIdx.x == 0) {
        t->arena = arena_pref[G];
        for (int q = 0; q < kKinds; ++q)
            for (int j = 0; j < 3; ++j) t->items[q][j] = pref ? pref[((long long)q * 3 + j) * (G + 1) + G] : 0;
        t->cov = cov_total ? *cov_total : 0;
        for (int q = 0; q < kKinds; ++q)
            for (int c = 0; c < kClasses; ++c) t->lds[q][c] = pref ? (long long)lds_max[q * kClasses + c] : 0;
    }
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int local = 0;
    for (int k = threadIdx.x; k < G; k += blockDim.x) local += alive[k] != 0;
    atomicAdd(&cnt, local);
    __syncthreads();
    if (threadIdx.x == 0) t->alive = cnt;
}

// Copy between value types (state download / upload).
template <typename A, typename B> __global__ void k_convert(const A *in, B *out, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        out[i] = (B)in[i];
}

}  // namespace gg
