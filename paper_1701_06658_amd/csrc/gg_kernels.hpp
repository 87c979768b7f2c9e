// Device code of the level-set grain-growth step for gfx950 (MI355X).
//
// Data layout in HBM: every alive grain's box is stored contiguously, x
// fastest, in grain-id order ("packed arena"); a box table (lo, ext, alive,
// offset) per layout describes it.  All per-voxel work is expressed as work
// items over boxes (predictor, re-initialization) or over fixed tiles of the
// global grid (corrector, labels); per-item grain lookups are O(1) maps.
//
// Stencil kernels stage one output tile plus its halo in LDS, so every HBM
// value of a box plane is read once per pass and written once.  Along an axis
// a box is either the whole periodic axis (indices wrap) or at most n - 2P long
// (indices outside the box read the fill value): a stencil of reach <= 2P then
// never wraps into a partial box.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gg {

constexpr int kBlock = 256;       // threads per work group of the stencil/tile kernels
constexpr int kLdsBytes = 61440;  // dynamic LDS budget per work group (stays below 64 KB)
constexpr int kMaxRadius = 24;    // largest Gaussian radius R
constexpr int kMaxBand = 16;      // largest band half width W
constexpr int kKinds = 4;         // item kinds: predictor xy, predictor z, reinit xy, reinit z
enum { KIND_CXY = 0, KIND_CZ = 1, KIND_RXY = 2, KIND_RZ = 3 };

// Box table of one layout.
struct Boxes {
    int *lo;         // 3 per grain
    int *ext;        // 3 per grain (0 when extinct)
    int *alive;      // 1 per grain
    long long *off;  // G + 1: exclusive prefix of box volumes
};

// Work items of one layout: per kind, prefix counts over grains (G + 1) and the
// item -> grain map.
struct Items {
    long long *pref[kKinds];
    int *owner[kKinds];
};

struct Totals {
    long long arena;      // sum of box volumes
    long long items[kKinds];
    long long cov;        // coverage list entries
    long long alive;      // alive grains
    long long lds[kKinds];  // largest LDS need of any item, in values
};

// ------------------------------------------------------------------ helpers

__host__ __device__ inline int imod(long long v, int N) {
    long long r = v % N;
    return (int)(r < 0 ? r + N : r);
}

// Local index along an axis for a stencil read at local coordinate c: a whole
// axis wraps, a partial box clips (-1 = outside).
__device__ inline int axis_map(int c, int e, int N) {
    if (e == N) {
        int r = c % N;
        return r < 0 ? r + N : r;
    }
    return (c >= 0 && c < e) ? c : -1;
}

template <typename T> constexpr int lds_budget() { return kLdsBytes / (int)sizeof(T); }

template <typename T> __device__ inline T mac(T acc, T a, T b);
template <> __device__ inline double mac<double>(double acc, double a, double b) {
    return acc + a * b;  // built without contraction: product and sum rounded separately
}
template <> __device__ inline float mac<float>(float acc, float a, float b) {
    return __builtin_fmaf(a, b, acc);
}

template <typename T> __device__ inline T tinf();
template <> __device__ inline double tinf<double>() { return __builtin_inf(); }
template <> __device__ inline float tinf<float>() { return __builtin_inff(); }

// LDS values needed by an output tile tx * ty with halo h.
__host__ __device__ inline long long lds_need(int kind, int tx, int ty, int h) {
    if (kind == KIND_CXY) return (long long)(tx + 2 * h) * (ty + 2 * h) + (long long)tx * (ty + 2 * h);
    if (kind == KIND_RXY)
        return (long long)(tx + 2 * h + 2) * (ty + 2 * h + 2) + (long long)(tx + 2 * h) * (ty + 2 * h) +
               (long long)tx * (ty + 2 * h);
    return (long long)tx * (ty + 2 * h);  // z passes: tx lines of ty + 2h planes
}

struct Tiling {
    int nxs, nys, tx, ty;
};

// Split a box cross-section ex * ey (second axis y for xy kernels, z for z
// kernels) into the fewest near-equal tiles whose LDS need fits the budget.
__host__ __device__ inline Tiling choose_tiling(int kind, int ex, int ey, int h, int budget) {
    Tiling t = {0, 0, 0, 0};
    for (int nxs = (ex + 127) / 128; nxs <= ex; ++nxs) {
        int tx = (ex + nxs - 1) / nxs;
        long long a, b;  // lds_need = a * ty + b
        if (kind == KIND_CXY) {
            a = 2LL * tx + 2 * h;
            b = a * 2 * h;
        } else if (kind == KIND_RXY) {
            long long p = tx + 2 * h + 2, q = tx + 2 * h, r = tx;
            a = p + q + r;
            b = p * (2 * h + 2) + (q + r) * 2 * h;
        } else {
            a = tx;
            b = (long long)tx * 2 * h;
        }
        long long tymax = (budget - b) / a;
        if (tymax < 1) continue;
        int nys = (int)((ey + tymax - 1) / tymax);
        t.nxs = nxs;
        t.nys = nys;
        t.tx = tx;
        t.ty = (ey + nys - 1) / nys;
        return t;
    }
    return t;  // infeasible: nxs == 0
}

// Number of work items of one kind for a box.
__host__ __device__ inline long long kind_items(int kind, const int *e, int h, int budget) {
    if (kind == KIND_CXY || kind == KIND_RXY) {
        Tiling t = choose_tiling(kind, e[0], e[1], h, budget);
        return (long long)e[2] * t.nxs * t.nys;
    }
    Tiling t = choose_tiling(kind, e[0], e[2], h, budget);
    return (long long)e[1] * t.nxs * t.nys;
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

__device__ inline int wave_min(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline int wave_max(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// ------------------------------------------------ predictor correction terms

template <typename T> struct Physics {
    int mode;           // bit 1 misorientation weights, bit 2 bulk energy
    const T *quat;      // 4 per grain (w, x, y, z)
    const T *energy;    // 1 per grain, J/m^3
    T theta_c_deg;
    T bulk_scale;       // sigma^2 h / (2 gamma_max): voxels per (J/m^3) and step
    const T *phi;       // the step's input function (same layout as psi)
    const int *iota;    // ID-field of the previous corrector (same layout)
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
    for (int k = 0; k < 6; ++k) {
        T w1 = dw * c6[k] - dz * s6[k];       // rotation about c by 60k degrees
        T w2 = -dx * c6[k] - dy * s6[k];      // 2-fold axis in the basal plane at 30k degrees
        T m = w1 < 0 ? -w1 : w1;
        T m2 = w2 < 0 ? -w2 : w2;
        best = m > best ? m : best;
        best = m2 > best ? m2 : best;
    }
    if (best > T(1)) best = T(1);
    return T(2) * dev_acos(best) * T(57.295779513082320877);
}

// Pair weight w = mobility * Read-Shockley energy (both normalised to (0, 1]).
template <typename T> __device__ inline T pair_weight(T theta, T theta_c, T *mob) {
    T g;
    if (theta >= theta_c) g = T(1);
    else if (theta <= T(0)) g = T(0);
    else {
        T r = theta / theta_c;
        g = r * (T(1) - dev_log(r));
    }
    T u = theta / T(15);
    T u3 = u * u * u;
    T mu = T(1) - T(0.99) * dev_exp(T(-5) * (u3 * u3 * u3));
    *mob = mu;
    return mu * g;
}

template <typename T> struct PairCache {
    int j = -2;
    T w = 1, b = 0;
};

// d^p = phi + w (psi - phi) + mob (E_j - E_k) * bulk_scale, clamped to [-W, W].
template <typename T>
__device__ inline T correct_prediction(const Physics<T> &ph, int k, long long idx, T psi, T W,
                                       PairCache<T> &pc) {
    const int j = ph.iota[idx];
    if (j != pc.j) {
        pc.j = j;
        pc.w = 1;
        pc.b = 0;
        if (j >= 0) {
            T mob = 1;
            if (ph.mode & 1) {
                T th = misorientation_deg<T>(ph.quat + 4LL * k, ph.quat + 4LL * j);
                pc.w = pair_weight<T>(th, ph.theta_c_deg, &mob);
            }
            if (ph.mode & 2) pc.b = mob * (ph.energy[j] - ph.energy[k]) * ph.bulk_scale;
        }
    }
    const T p = ph.phi[idx];
    T d = p + pc.w * (psi - p) + pc.b;
    d = d > W ? W : d;
    d = d < -W ? -W : d;
    return d;
}

// --------------------------------------------------------- predictor kernels

struct GridArgs {
    int n[3];
    int dim;
};

// x and y passes of the Gaussian on one tile of one z plane (2D: the whole
// predictor, with the optional correction epilogue).
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_conv_xy(Boxes L, const int *__restrict__ owner, const long long *__restrict__ pref,
              const T *__restrict__ in, T *__restrict__ out, const T *__restrict__ taps, int R, T W,
              GridArgs g, Physics<T> ph) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);
    const long long item = blockIdx.x;
    const int k = owner[item];
    const int sub = (int)(item - pref[k]);
    const int ex = L.ext[3 * k], ey = L.ext[3 * k + 1];
    const Tiling tl = choose_tiling(KIND_CXY, ex, ey, R, lds_budget<T>());
    const int per_z = tl.nxs * tl.nys;
    const int z = sub / per_z, rem = sub - z * per_z, ys = rem / tl.nxs, xs = rem - ys * tl.nxs;
    const int x0 = xs * tl.tx, y0 = ys * tl.ty;
    const int wx = min(tl.tx, ex - x0), wy = min(tl.ty, ey - y0);
    const int RW = wx + 2 * R, RH = wy + 2 * R;
    const long long base = L.off[k] + (long long)z * ex * ey;
    const T *src = in + base;
    T *raw = sm, *xp = sm + RW * RH;
    for (int e = threadIdx.x; e < RW * RH; e += kBlock) {
        const int rr = e / RW, cc = e - rr * RW;
        const int yy = axis_map(y0 - R + rr, ey, g.n[1]);
        const int xx = axis_map(x0 - R + cc, ex, g.n[0]);
        raw[e] = (yy >= 0 && xx >= 0) ? src[(long long)yy * ex + xx] : -W;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < wx * RH; e += kBlock) {
        const int rr = e / wx, c = e - rr * wx;
        T acc;
        if (axis_map(y0 - R + rr, ey, g.n[1]) < 0) {
            acc = -W;  // rows outside the box read the fill value in the y pass
        } else {
            acc = 0;
            const T *rp = raw + rr * RW + c;
            for (int i = 0; i <= 2 * R; ++i) acc = mac<T>(acc, taps[i], rp[i]);
        }
        xp[e] = acc;
    }
    __syncthreads();
    T *dst = out + base;
    PairCache<T> pc;
    for (int e = threadIdx.x; e < wx * wy; e += kBlock) {
        const int r = e / wx, c = e - r * wx;
        T acc = 0;
        const T *cp = xp + r * wx + c;
        for (int j = 0; j <= 2 * R; ++j) acc = mac<T>(acc, taps[j], cp[j * wx]);
        const long long idx = (long long)(y0 + r) * ex + x0 + c;
        if (g.dim == 2 && ph.mode) acc = correct_prediction<T>(ph, k, base + idx, acc, W, pc);
        dst[idx] = acc;
    }
}

// z pass of the Gaussian on one tile (x chunk * z range) of one y row, with the
// optional correction epilogue.
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_conv_z(Boxes L, const int *__restrict__ owner, const long long *__restrict__ pref,
             const T *__restrict__ in, T *__restrict__ out, const T *__restrict__ taps, int R, T W,
             GridArgs g, Physics<T> ph) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *col = reinterpret_cast<T *>(smem_raw);
    const long long item = blockIdx.x;
    const int k = owner[item];
    const int sub = (int)(item - pref[k]);
    const int ex = L.ext[3 * k], ey = L.ext[3 * k + 1], ez = L.ext[3 * k + 2];
    const Tiling tl = choose_tiling(KIND_CZ, ex, ez, R, lds_budget<T>());
    const int per_y = tl.nxs * tl.nys;
    const int y = sub / per_y, rem = sub - y * per_y, zs = rem / tl.nxs, xs = rem - zs * tl.nxs;
    const int x0 = xs * tl.tx, z0 = zs * tl.ty;
    const int wx = min(tl.tx, ex - x0), wz = min(tl.ty, ez - z0);
    const int CH = wz + 2 * R;
    const long long plane = (long long)ex * ey;
    const long long rowbase = L.off[k] + (long long)y * ex + x0;
    for (int e = threadIdx.x; e < wx * CH; e += kBlock) {
        const int rr = e / wx, c = e - rr * wx;
        const int zz = axis_map(z0 - R + rr, ez, g.n[2]);
        col[e] = zz >= 0 ? in[rowbase + zz * plane + c] : -W;
    }
    __syncthreads();
    PairCache<T> pc;
    for (int e = threadIdx.x; e < wx * wz; e += kBlock) {
        const int r = e / wx, c = e - r * wx;
        T acc = 0;
        const T *cp = col + r * wx + c;
        for (int j = 0; j <= 2 * R; ++j) acc = mac<T>(acc, taps[j], cp[j * wx]);
        const long long idx = rowbase + (long long)(z0 + r) * plane + c;
        if (ph.mode) acc = correct_prediction<T>(ph, k, idx, acc, W, pc);
        out[idx] = acc;
    }
}

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
    __device__ void push(T v, int j) {
        if (v > m1 || (v == m1 && j < i1)) {
            m2 = m1;
            i2 = i1;
            m1 = v;
            i1 = j;
        } else if (v > m2 || (v == m2 && (i2 < 0 || j < i2))) {
            m2 = v;
            i2 = j;
        }
    }
};

constexpr int kTileVox = 512;
constexpr int kVpt = kTileVox / kBlock;

// One global tile: the top-2 of the predicted functions of every grain whose
// box covers the tile, then for each of those grains
//   phi^c = (psi - max over the other grains) / 2   (-W if no other grain),
// its ID-field (argmax of the others), and the bounding box of phi^c > 0.
// mode 0: corrector; mode 1: ID-field only (argmax of the others' values).
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_compare(Boxes L, const int *__restrict__ cov_off, const int *__restrict__ cov_list,
              const T *__restrict__ psi, T *__restrict__ phic, int *__restrict__ iota_out, int *bmin,
              int *bmax, unsigned *occ, TileArgs ta, T W, int mode) {
    const int tile = blockIdx.x;
    const int tx = tile % ta.nt[0], ty = (tile / ta.nt[0]) % ta.nt[1], tz = tile / (ta.nt[0] * ta.nt[1]);
    const int tvol = ta.t[0] * ta.t[1] * ta.t[2];
    int gx[kVpt], gy[kVpt], gz[kVpt];
    bool valid[kVpt];
#pragma unroll
    for (int i = 0; i < kVpt; ++i) {
        const int v = threadIdx.x + i * kBlock;
        valid[i] = v < tvol;
        const int vx = v % ta.t[0], vy = (v / ta.t[0]) % ta.t[1], vz = v / (ta.t[0] * ta.t[1]);
        gx[i] = tx * ta.t[0] + vx;
        gy[i] = ty * ta.t[1] + vy;
        gz[i] = tz * ta.t[2] + vz;
    }
    const int b = cov_off[tile], e = cov_off[tile + 1];
    Top2<T> top[kVpt];
#pragma unroll
    for (int i = 0; i < kVpt; ++i) top[i].init();
    for (int c = b; c < e; ++c) {
        const int j = cov_list[c];
        const int lx0 = L.lo[3 * j], ly0 = L.lo[3 * j + 1], lz0 = L.lo[3 * j + 2];
        const int ex = L.ext[3 * j], ey = L.ext[3 * j + 1], ez = L.ext[3 * j + 2];
        const long long off = L.off[j];
#pragma unroll
        for (int i = 0; i < kVpt; ++i) {
            const int lx = imod(gx[i] - lx0, ta.n[0]), ly = imod(gy[i] - ly0, ta.n[1]),
                      lz = imod(gz[i] - lz0, ta.n[2]);
            if (valid[i] && lx < ex && ly < ey && lz < ez)
                top[i].push(psi[off + lx + (long long)ex * (ly + (long long)ey * lz)], j);
        }
    }
    for (int c = b; c < e; ++c) {
        const int j = cov_list[c];
        const int lx0 = L.lo[3 * j], ly0 = L.lo[3 * j + 1], lz0 = L.lo[3 * j + 2];
        const int ex = L.ext[3 * j], ey = L.ext[3 * j + 1], ez = L.ext[3 * j + 2];
        const long long off = L.off[j];
        int mn[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, mx[3] = {-1, -1, -1};
#pragma unroll
        for (int i = 0; i < kVpt; ++i) {
            const int lx = imod(gx[i] - lx0, ta.n[0]), ly = imod(gy[i] - ly0, ta.n[1]),
                      lz = imod(gz[i] - lz0, ta.n[2]);
            if (!(valid[i] && lx < ex && ly < ey && lz < ez)) continue;
            const long long idx = off + lx + (long long)ex * (ly + (long long)ey * lz);
            const bool first = top[i].i1 == j;
            const int other = first ? top[i].i2 : top[i].i1;
            if (iota_out) iota_out[idx] = other;
            if (mode != 0) continue;
            const T m = first ? (top[i].i2 < 0 ? -W : top[i].m2) : top[i].m1;
            const T pc = T(0.5) * (psi[idx] - m);
            phic[idx] = pc;
            if (pc > T(0)) {
                const int l3[3] = {lx, ly, lz};
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    mn[a] = min(mn[a], l3[a]);
                    mx[a] = max(mx[a], l3[a]);
                }
                const int e3[3] = {ex, ey, ez};
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    if (e3[a] == ta.n[a])
                        atomicOr(&occ[((long long)j * 3 + a) * ta.occ_words + (l3[a] >> 5)],
                                 1u << (l3[a] & 31));
            }
        }
        if (mode != 0) continue;
        if (__ballot(mx[0] >= 0) == 0) continue;
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
    }
}

// Voxel labels: argmax over the covering grains (ties to the lowest id).
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_labels(Boxes L, const int *__restrict__ cov_off, const int *__restrict__ cov_list,
             const T *__restrict__ phi, int *__restrict__ labels, TileArgs ta) {
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
            const int lx = imod(gx - L.lo[3 * j], ta.n[0]), ly = imod(gy - L.lo[3 * j + 1], ta.n[1]),
                      lz = imod(gz - L.lo[3 * j + 2], ta.n[2]);
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
    int nlo[3], nex[3], olo[3], oex[3];
    long long ooff;
    int n[3];
    T W;
    __device__ inline long long old_index(int x, int y, int z) const {
        const int xm = axis_map(x, nex[0], n[0]), ym = axis_map(y, nex[1], n[1]),
                  zm = axis_map(z, nex[2], n[2]);
        if (xm < 0 || ym < 0 || zm < 0) return -1;
        const int ox = imod((long long)nlo[0] + xm - olo[0], n[0]);
        const int oy = imod((long long)nlo[1] + ym - olo[1], n[1]);
        const int oz = imod((long long)nlo[2] + zm - olo[2], n[2]);
        if (ox >= oex[0] || oy >= oex[1] || oz >= oex[2]) return -1;
        return ooff + ox + (long long)oex[0] * (oy + (long long)oex[1] * oz);
    }
    __device__ inline T value(int x, int y, int z) const {
        const long long i = old_index(x, y, z);
        return i >= 0 ? src[i] : -W;
    }
};

// Reference values next to the sign change and the x and y min-plus passes on
// one tile of one z plane of the new box.  3D: writes the partial distance
// with the inside flag as its sign bit; 2D: writes the final function and the
// tile's volume.  Also carries the ID-field over to the new layout.
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_reinit_xy(Boxes Lo, Boxes Ln, const int *__restrict__ owner, const long long *__restrict__ pref,
                const T *__restrict__ phic, T *__restrict__ out, const int *__restrict__ iota_old,
                int *__restrict__ iota_new, double *__restrict__ vol_part, int K, T W, GridArgs g) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);
    __shared__ double red[kBlock / 64];
    const long long item = blockIdx.x;
    const int k = owner[item];
    const int sub = (int)(item - pref[k]);
    Carry<T> cr;
    cr.src = phic;
    cr.W = W;
    cr.ooff = Lo.off[k];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cr.nlo[a] = Ln.lo[3 * k + a];
        cr.nex[a] = Ln.ext[3 * k + a];
        cr.olo[a] = Lo.lo[3 * k + a];
        cr.oex[a] = Lo.ext[3 * k + a];
        cr.n[a] = g.n[a];
    }
    const int ex = cr.nex[0], ey = cr.nex[1];
    const Tiling tl = choose_tiling(KIND_RXY, ex, ey, K, lds_budget<T>());
    const int per_z = tl.nxs * tl.nys;
    const int z = sub / per_z, rem = sub - z * per_z, ys = rem / tl.nxs, xs = rem - ys * tl.nxs;
    const int x0 = xs * tl.tx, y0 = ys * tl.ty;
    const int wx = min(tl.tx, ex - x0), wy = min(tl.ty, ey - y0);
    const int FW = wx + 2 * K + 2, FH = wy + 2 * K + 2, RW = wx + 2 * K, RH = wy + 2 * K;
    T *f = sm, *ref = sm + FW * FH, *d1 = ref + RW * RH;
    const T inf = tinf<T>();
    for (int e = threadIdx.x; e < FW * FH; e += kBlock) {
        const int rr = e / FW, cc = e - rr * FW;
        f[e] = cr.value(x0 - K - 1 + cc, y0 - K - 1 + rr, z);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < RW * RH; e += kBlock) {
        const int rr = e / RW, cc = e - rr * RW;
        const int x = x0 - K + cc, y = y0 - K + rr;
        T r = inf;
        if (axis_map(x, ex, g.n[0]) >= 0 && axis_map(y, ey, g.n[1]) >= 0) {
            const T fc = f[(rr + 1) * FW + cc + 1];
            const bool in = fc > T(0);
            T nb[6];
            nb[0] = f[(rr + 1) * FW + cc];
            nb[1] = f[(rr + 1) * FW + cc + 2];
            nb[2] = f[rr * FW + cc + 1];
            nb[3] = f[(rr + 2) * FW + cc + 1];
            int nn = 4;
            if (g.dim == 3) {
                nb[4] = cr.value(x, y, z - 1);
                nb[5] = cr.value(x, y, z + 1);
                nn = 6;
            }
            for (int q = 0; q < nn; ++q) {
                const T fn = nb[q];
                if ((fn > T(0)) != in) {
                    const T th = fc / (fc - fn);
                    if (th < r) r = th;
                }
            }
        }
        ref[e] = r;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < wx * RH; e += kBlock) {
        const int rr = e / wx, c = e - rr * wx;
        T best = inf;
        if (axis_map(y0 - K + rr, ey, g.n[1]) >= 0) {
            const T *rp = ref + rr * RW + c;
            for (int i = 0; i <= 2 * K; ++i) {
                const T t = rp[i] + T(i < K ? K - i : i - K);
                if (t < best) best = t;
            }
        }
        d1[e] = best;
    }
    __syncthreads();
    const long long base = Ln.off[k] + (long long)z * ex * ey;
    double vsum = 0.0;
    for (int e = threadIdx.x; e < wx * wy; e += kBlock) {
        const int r = e / wx, c = e - r * wx;
        T best = inf;
        const T *cp = d1 + r * wx + c;
        for (int j = 0; j <= 2 * K; ++j) {
            const T t = cp[j * wx] + T(j < K ? K - j : j - K);
            if (t < best) best = t;
        }
        const bool in = f[(r + K + 1) * FW + c + K + 1] > T(0);
        const long long idx = base + (long long)(y0 + r) * ex + x0 + c;
        if (g.dim == 2) {
            const T d = best < W ? best : W;
            const T p = in ? d : -d;
            out[idx] = p;
            double cl = (double)p + 0.5;
            cl = cl < 0.0 ? 0.0 : (cl > 1.0 ? 1.0 : cl);
            vsum += cl;
        } else {
            out[idx] = in ? best : -best;
        }
        if (iota_new) {
            const long long oi = cr.old_index(x0 + c, y0 + r, z);
            iota_new[idx] = oi >= 0 ? iota_old[oi] : -1;
        }
    }
    if (g.dim == 2) {
        const double s = block_sum(vsum, red);
        if (threadIdx.x == 0) vol_part[item] = s;
    }
}

// z min-plus pass, sign and band clamp, and the tile's volume (3D).
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_reinit_z(Boxes Ln, const int *__restrict__ owner, const long long *__restrict__ pref,
               const T *__restrict__ d2, T *__restrict__ out, double *__restrict__ vol_part, int K,
               T W, GridArgs g) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *col = reinterpret_cast<T *>(smem_raw);
    __shared__ double red[kBlock / 64];
    const long long item = blockIdx.x;
    const int k = owner[item];
    const int sub = (int)(item - pref[k]);
    const int ex = Ln.ext[3 * k], ey = Ln.ext[3 * k + 1], ez = Ln.ext[3 * k + 2];
    const Tiling tl = choose_tiling(KIND_RZ, ex, ez, K, lds_budget<T>());
    const int per_y = tl.nxs * tl.nys;
    const int y = sub / per_y, rem = sub - y * per_y, zs = rem / tl.nxs, xs = rem - zs * tl.nxs;
    const int x0 = xs * tl.tx, z0 = zs * tl.ty;
    const int wx = min(tl.tx, ex - x0), wz = min(tl.ty, ez - z0);
    const int CH = wz + 2 * K;
    const long long plane = (long long)ex * ey;
    const long long rowbase = Ln.off[k] + (long long)y * ex + x0;
    const T inf = tinf<T>();
    for (int e = threadIdx.x; e < wx * CH; e += kBlock) {
        const int rr = e / wx, c = e - rr * wx;
        const int zz = axis_map(z0 - K + rr, ez, g.n[2]);
        col[e] = zz >= 0 ? d2[rowbase + zz * plane + c] : inf;
    }
    __syncthreads();
    double vsum = 0.0;
    for (int e = threadIdx.x; e < wx * wz; e += kBlock) {
        const int r = e / wx, c = e - r * wx;
        T best = inf;
        const T *cp = col + r * wx + c;
        for (int j = 0; j <= 2 * K; ++j) {
            const T t = fabs(cp[j * wx]) + T(j < K ? K - j : j - K);
            if (t < best) best = t;
        }
        const bool in = !signbit(cp[K * wx]);
        const T d = best < W ? best : W;
        const T p = in ? d : -d;
        out[rowbase + (long long)(z0 + r) * plane + c] = p;
        double cl = (double)p + 0.5;
        cl = cl < 0.0 ? 0.0 : (cl > 1.0 ? 1.0 : cl);
        vsum += cl;
    }
    const double s = block_sum(vsum, red);
    if (threadIdx.x == 0) vol_part[item] = s;
}

// Initial function before re-initialization: +1/2 on the grain's labelled
// voxels, -1/2 elsewhere in its box.
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_init_indicator(Boxes L, const int *__restrict__ labels, T *__restrict__ out, GridArgs g) {
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
__global__ void k_plan(Boxes Lo, Boxes Ln, int *bmin, int *bmax, unsigned *occ, long long *sizes,
                       PlanArgs pa) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= pa.G) return;
    bool alive = Lo.alive[k] && bmax[3 * k] >= 0;
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

// Box volumes of a layout (for layouts set from the host).
__global__ void k_box_sizes(Boxes L, long long *sizes, int G) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= G) return;
    sizes[k] = L.alive[k] ? (long long)L.ext[3 * k] * L.ext[3 * k + 1] * L.ext[3 * k + 2] : 0;
}

// Per-grain work item counts of the four stencil kinds.
__global__ void k_item_counts(Boxes L, long long *c0, long long *c1, long long *c2, long long *c3,
                              unsigned long long *lds_max, int R, int K, int G, int budget) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= G) return;
    long long *cs[4] = {c0, c1, c2, c3};
    if (!L.alive[k]) {
        for (int q = 0; q < 4; ++q) cs[q][k] = 0;
        return;
    }
    const int *e = L.ext + 3 * k;
    const int h[4] = {R, R, K, K};
    for (int q = 0; q < 4; ++q) {
        cs[q][k] = kind_items(q, e, h[q], budget);
        const int sa = (q == KIND_CXY || q == KIND_RXY) ? e[1] : e[2];
        const Tiling t = choose_tiling(q, e[0], sa, h[q], budget);
        if (t.nxs == 0) {
            atomicMax(&lds_max[q], 0xffffffffffffffffULL);  // infeasible tiling
        } else {
            atomicMax(&lds_max[q], (unsigned long long)lds_need(q, t.tx, t.ty, h[q]));
        }
    }
}

// Exclusive prefix sum of n values (out has n + 1 entries), one work group.
__global__ void __launch_bounds__(1024) k_scan(const long long *in, long long *out, int n) {
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
    if (t == 1023) out[n] = part[1023];
}

__global__ void k_scan_int(const int *in, int *out, int n) {
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
        out[i] = (int)base;
        base += in[i];
    }
    if (t == 1023) out[n] = (int)part[1023];
}

// item -> grain maps of one kind.
__global__ void k_fill_owner(const long long *pref, int *owner, int G) {
    const int k = blockIdx.x;
    const long long b = pref[k], e = pref[k + 1];
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
__global__ void k_coverage(Boxes L, int *cnt_or_cursor, int *list, TileArgs ta, int G, int mode) {
    const int k = blockIdx.x;
    if (!L.alive[k]) return;
    int t0[3], c[3];
    for (int a = 0; a < 3; ++a) axis_tiles(L.lo[3 * k + a], L.ext[3 * k + a], ta.n[a], ta.t[a], ta.nt[a], &t0[a], &c[a]);
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

// Per-grain volume from the per-item partial sums, in item order.
__global__ void k_volumes(const Boxes L, const long long *pref, const double *vol_part, double *vol, int G) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= G) return;
    double s = 0.0;
    if (L.alive[k])
        for (long long i = pref[k]; i < pref[k + 1]; ++i) s += vol_part[i];
    vol[k] = s;
}

__global__ void k_totals(const long long *arena_pref, const long long *p0, const long long *p1,
                         const long long *p2, const long long *p3, const int *cov_off, int ntiles,
                         const int *alive, int G, const unsigned long long *lds_max, Totals *t) {
    if (threadIdx.x == 0) {
        t->arena = arena_pref[G];
        t->items[0] = p0[G];
        t->items[1] = p1[G];
        t->items[2] = p2[G];
        t->items[3] = p3[G];
        t->cov = cov_off ? cov_off[ntiles] : 0;
        for (int q = 0; q < 4; ++q) t->lds[q] = (long long)lds_max[q];
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
template <typename A, typename B>
__global__ void k_convert(const A *in, B *out, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        out[i] = (B)in[i];
}

}  // namespace gg
