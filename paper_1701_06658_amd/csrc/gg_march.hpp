// Z-marching kernels of the level-set step for gfx950 (MI355X): one work group
// per grain box walks through the box plane by plane, so every value of the box
// is read once from HBM and written once, in contiguous plane-sized chunks.
//
//   k_reinit_march   phi^c (old box) -> f    reference values next to the sign
//                    change, taxicab spreading along x and y inside the plane,
//                    forward spreading along z (ascending march); 2D: the final
//                    function and the grain volume
//   k_predict_march  f -> psi (+ phi)        backward spreading along z, band
//                    clamp, grain volume (3D), then the separable Gaussian: the
//                    z pass from a register window of 2R + 1 planes, the x and y
//                    passes inside the plane (descending march); the optional
//                    predictor-correction epilogue
//
// Together with the corrector these are the three sweeps of a step.  The
// spreading (sec. 2.1.6) is the running minimum c <- min(v, c + 1) along each
// line: forward and backward chains inside a window of +-K cells give the same
// value as sweeps over the whole line wherever the distance is below the band
// (a source farther than K cells is more than K away), and the band clamp makes
// every larger value W; along z the chains run over the whole column, forward in
// the first kernel, backward in the second, in the order of the sequential
// sweeps.
//
// Threads of a group own column units: one x position and YB consecutive rows
// of a plane tile, whose values of successive planes stay in registers.  In-plane
// passes go through LDS.  A box cross-section larger than the group is cut into
// tiles with halos (the stencil reach) on every side inside the box; a box axis
// that spans the whole periodic grid wraps its halos around.
#pragma once

#include "gg_kernels.hpp"

namespace gg {

#ifndef GG_MT
#define GG_MT 512
#endif
constexpr int kMT = GG_MT;  // threads per march group
#ifndef GG_REINIT_QX
#define GG_REINIT_QX 8
#endif
#ifndef GG_PREDICT_QX
#define GG_PREDICT_QX 4
#endif
#ifndef GG_REINIT_YB
#define GG_REINIT_YB 4
#endif
constexpr int kQXR = GG_REINIT_QX;   // outputs per thread of the re-initialization's x spreading
constexpr int kQXP = GG_PREDICT_QX;  // outputs per thread of the predictor's x pass
constexpr int kReinitYB = GG_REINIT_YB;  // rows per column unit of the re-initialization
#ifndef GG_ROW_REVERSE
#define GG_ROW_REVERSE 1
#endif
#ifndef GG_ROW_REVERSE_P
#define GG_ROW_REVERSE_P 1
#endif
// First row unit of the thread: row units are dealt from the last thread down,
// column units from the first thread up, so that in a tile smaller than the
// group the two kinds of work fall on different waves.
template <bool REV> __device__ __forceinline__ int row_unit0() { return REV ? kMT - 1 - (int)threadIdx.x : (int)threadIdx.x; }

// The row units (kQ consecutive cells of one row) a thread takes in a tile of
// EY rows: unit r = threadIdx.x + i kMT has row r % EY and x block r / EY,
// stepped without division.
struct RowWalk {
    int ry, xq, dq, dr;
    __device__ RowWalk(int EY, int t) {
        ry = t % EY;
        xq = t / EY;
        dq = kMT / EY;
        dr = kMT - dq * EY;
    }
    __device__ void next(int EY) {
        ry += dr;
        xq += dq;
        if (ry >= EY) {
            ry -= EY;
            ++xq;
        }
    }
};

// LDS layouts of the march kernels for an extended tile of EX x EY cells.
// Every in-plane window pass reads from a buffer whose frame (wide enough for
// the window) holds the fill value, so window reads need no bounds checks; the
// frames are written once per tile and never overwritten by plane data.
//
// Both kernels are software-pipelined over the planes of a box: each stage
// reads the buffer its predecessor wrote in the previous iteration, so every
// buffer comes twice (for planes of even and odd index) and one barrier per
// plane separates the stages.
//
// Re-initialization: F, phi^c with a one-cell frame of -W; Rf, reference values
// with x frames of KW cells of +inf (and kQXR more on the right); Dx, the x-spread
// values with y frames of KW rows of +inf (and YB more below).
template <int KW, int YB> struct ReinitLds {
    int pf, pr, pd, sF, sR, sD, oR, oD, total;
    __host__ __device__ constexpr ReinitLds(int EX, int EY)
        : pf((EX + 2) | 1), pr((EX + 2 * KW + kQXR) | 1), pd(EX | 1), sF(pf * (EY + 2)), sR(pr * EY),
          sD(pd * (EY + 2 * KW + YB)), oR(2 * sF), oD(oR + 2 * sR), total(oD + 2 * sD) {}
};
// Predictor: Cz, the z-convolved plane with x frames of RM cells of -W (and kQXP
// more on the right); Cx, the x-convolved plane with y frames of RM rows of -W
// (and YB more below).
template <int RM, int YB> struct PredictLds {
    int pz, px, sZ, sX, oX, total;
    __host__ __device__ constexpr PredictLds(int EX, int EY)
        : pz((EX + 2 * RM + kQXP) | 1), px(EX | 1), sZ(pz * EY), sX(px * (EY + 2 * RM + YB)), oX(2 * sZ),
          total(oX + 2 * sX) {}
};

// Tiles at most kPitchW wide may run with the LDS pitches of that width fixed
// at compile time (the |1 of the pitches makes 44 and 45 alike).
#ifndef GG_PITCH_W
#define GG_PITCH_W 45
#endif
constexpr int kPitchW = GG_PITCH_W;

// LDS cells a march kernel may use (its dynamic allocation).
#ifndef GG_REINIT_CELLS_F32
#define GG_REINIT_CELLS_F32 16384
#endif
#ifndef GG_REINIT_WAVES
#define GG_REINIT_WAVES 1
#endif
#ifndef GG_MARCH_CELLS_F64
#define GG_MARCH_CELLS_F64 19968
#endif
// FP64 marches run one group per CU (their registers allow no more), so they
// take nearly the whole 160 KB of the CU's LDS: larger tiles, fewer halos.
template <typename T> constexpr int reinit_cells() { return sizeof(T) == 8 ? GG_MARCH_CELLS_F64 : GG_REINIT_CELLS_F32; }
template <typename T> constexpr int predict_cells() { return sizeof(T) == 8 ? GG_MARCH_CELLS_F64 : 12288; }

// Every box has a tiling: the smallest extended tile (one interior cell and
// halos of the largest reach on both sides of both axes) fits the group's
// column units and each kernel's LDS.
constexpr int kReinitMinTile = 2 * (kMaxBand + 1) + 1;
constexpr int kPredictMinTile = 2 * kMaxRadius + 1;
static_assert(ReinitLds<kMaxBand, kReinitYB>(kReinitMinTile, kReinitMinTile).total <= reinit_cells<double>() &&
                  ReinitLds<kMaxBand, kReinitYB>(kReinitMinTile, kReinitMinTile).total <= reinit_cells<float>(),
              "re-initialization LDS too small for the largest band");
static_assert(PredictLds<kMaxRadius, 2>(kPredictMinTile, kPredictMinTile).total <= predict_cells<double>() &&
                  PredictLds<kMaxRadius, 2>(kPredictMinTile, kPredictMinTile).total <= predict_cells<float>(),
              "predictor LDS too small for the largest radius");
static_assert(kReinitYB * (kMT / kReinitMinTile) >= kReinitMinTile && 2 * (kMT / kPredictMinTile) >= kPredictMinTile,
              "too few threads per group for the smallest tiles");

struct MarchArgs {
    int n[3];
    int dim;
    int G;
    int K;              // taxicab spreading reach P (k_reinit_march)
    int R;              // Gaussian radius (k_predict_march)
    const int *order;   // grain processed by each block (NULL: block index)
    const Ctl *ctl;     // NULL outside the step sequence
    int phi_always;     // k_predict_march: write phi at every step of a batch
};

// Tiling of a box cross-section (x, y) for a march group.
struct MSplit {
    int e[2], nt[2], w[2], h;
    bool ring[2];
};

// The fewest tiles whose extended tile (interior plus a halo of h cells on each
// side that lies inside the box, or wraps around a whole periodic axis) has
// EX * ceil(EY / YB) <= kMT column units and a layout Lay(EX, EY) of at most
// `cells` LDS cells (the layout's size is affine in EY).
template <int YB, typename Lay>
__device__ inline MSplit march_split(int e0, int e1, int N0, int N1, int h, int cells) {
    MSplit s;
    s.e[0] = e0;
    s.e[1] = e1;
    s.h = h;
    s.ring[0] = e0 == N0;
    s.ring[1] = e1 == N1;
    s.nt[0] = s.nt[1] = 0;
    int best = 0x7fffffff;
    for (int tx = 1; tx <= e0 && tx < best; ++tx) {
        const int wx = (e0 + tx - 1) / tx;
        const int EX = wx + ((tx > 1 || s.ring[0]) ? 2 * h : 0);
        if (EX > kMT) continue;
        const int b = Lay(EX, 0).total, a = Lay(EX, 1).total - b;
        const int rows = min(YB * (kMT / EX), cells >= b ? (cells - b) / a : 0);
        if (rows < 1) continue;
        int ty;
        if (!s.ring[1] && e1 <= rows) {
            ty = 1;
        } else {
            const int avail = rows - 2 * h;
            if (avail < 1) continue;
            ty = (e1 + avail - 1) / avail;
        }
        if (tx * ty < best) {
            best = tx * ty;
            s.nt[0] = tx;
            s.nt[1] = ty;
        }
    }
    for (int a = 0; a < 2; ++a) {
        if (s.nt[a] < 1) s.nt[a] = 1;  // unreachable for boxes of at most 4096 cells per axis
        s.w[a] = (s.e[a] + s.nt[a] - 1) / s.nt[a];
        s.nt[a] = (s.e[a] + s.w[a] - 1) / s.w[a];  // no empty tile
    }
    return s;
}

// Fill n LDS cells with v (all threads of the group).
template <typename T> __device__ __forceinline__ void lds_fill(T *p, int n, T v) {
    for (int i = threadIdx.x; i < n; i += kMT) p[i] = v;
}

// Extended tile `t` of a split: first cell in box coordinates (below 0 or past
// the box only on a whole periodic axis), size, and interior [in0, in1) in
// extended coordinates.
struct MTile {
    int org[2], ext[2], in0[2], in1[2];
};

__device__ inline MTile march_tile(const MSplit &s, int t) {
    MTile m;
    const int i[2] = {t % s.nt[0], t / s.nt[0]};
    for (int a = 0; a < 2; ++a) {
        const int b = i[a] * s.w[a], e = min(s.e[a], b + s.w[a]);
        const int hl = s.ring[a] ? s.h : min(s.h, b), hr = s.ring[a] ? s.h : min(s.h, s.e[a] - e);
        m.org[a] = b - hl;
        m.ext[a] = hl + (e - b) + hr;
        m.in0[a] = hl;
        m.in1[a] = hl + (e - b);
    }
    return m;
}

// Taxicab chains over a window: forward c <- min(v_i, c + 1) and backward, each
// from the window's end; o[q] = the smaller of the two at window position KW + q.
template <typename T, int NV, int KW, int NO>
__device__ __forceinline__ void taxicab_chains(const T (&v)[NV], T (&o)[NO]) {
    static_assert(KW >= 1 && KW + NO <= NV, "window");
    T c = v[0];
#pragma unroll
    for (int i = 1; i < NV; ++i) {
        c = vmin(v[i], c + T(1));
        if (i >= KW && i < KW + NO) o[i - KW] = c;
    }
    c = v[NV - 1];
#pragma unroll
    for (int i = NV - 2; i >= 0; --i) {
        c = vmin(v[i], c + T(1));
        if (i >= KW && i < KW + NO) o[i - KW] = vmin(o[i - KW], c);
    }
}

// Gaussian pass over NO consecutive outputs from a register window v (first
// entry at output 0 - R): o[q] = sum over t = 0..2R of tp[t] v[q + t], summed in
// increasing t.  RM: static window radius (>= R).
template <typename T, int RM, int NO>
__device__ __forceinline__ void gauss_window(const T (&v)[NO + 2 * RM], const T *tp, int R, T (&o)[NO]) {
#pragma unroll
    for (int q = 0; q < NO; ++q) o[q] = T(0);
#pragma unroll
    for (int t = 0; t <= 2 * RM; ++t) {
        if (t > 2 * R) break;
        const T g = tp[t];
#pragma unroll
        for (int q = 0; q < NO; ++q) o[q] = mac<T>(o[q], g, v[q + t]);
    }
}

// Column geometry of a thread in an extended tile: the column unit's x, its
// first row, the box coordinates and interior flags of its YB cells.
template <int YB> struct MCol {
    bool act;          // the thread owns a column unit
    int cx, ry0;       // extended-tile column and first row
    int bx;            // box x of the column
    bool colint;       // the column lies in the interior
    bool rv[YB];       // the row exists in the tile
    bool rint[YB];     // the cell lies in the interior
    int by[YB];        // box y of the row
};

template <int YB>
__device__ inline MCol<YB> march_col(const MTile &tl, int ex, int ey, int N0, int N1) {
    MCol<YB> c;
    const int EX = tl.ext[0], EY = tl.ext[1];
    const int nyb = (EY + YB - 1) / YB;
    const int u = threadIdx.x;
    c.act = u < EX * nyb;
    c.cx = c.act ? u % EX : 0;
    c.ry0 = c.act ? (u / EX) * YB : 0;
    c.bx = axis_map(tl.org[0] + c.cx, ex, N0);
    c.colint = c.act && c.cx >= tl.in0[0] && c.cx < tl.in1[0];
#pragma unroll
    for (int j = 0; j < YB; ++j) {
        const int ry = c.ry0 + j;
        c.rv[j] = c.act && ry < EY;
        c.by[j] = c.rv[j] ? axis_map(tl.org[1] + ry, ey, N1) : 0;
        c.rint[j] = c.rv[j] && c.colint && ry >= tl.in0[1] && ry < tl.in1[1];
    }
    return c;
}

// ------------------------------------------------------- k_reinit_march (a4)

// Re-initialization of phi^c (old layout Lo) into the new layout Ln (sec.
// 2.1.6, taxicab scheme): reference values theta = phi / (phi - phi_n) at cells
// with a face neighbour across the sign change, spreading along x and y by
// windowed chains inside each plane, forward spreading along z.  3D: writes the
// partially spread distance with the inside flag as its sign bit; 2D: writes
// phi = +-min(d, W) and the grain's volume.  Carries the ID-field over to the
// new layout.  KS: static reach (0: runtime ma.K <= kMaxBand); D3: a 3D grid;
// IO: the ID-field is carried (iota_old and iota_new given).
template <typename T, int KS, int YB, bool D3, bool IO>
__global__ void __launch_bounds__(kMT, sizeof(T) == 4 ? GG_REINIT_WAVES : 1)
    k_reinit_march(Boxes Lo, Boxes Ln, MarchArgs ma, const T *__restrict__ phic, T *__restrict__ out,
                   const int *__restrict__ iota_old, int *__restrict__ iota_new, double *__restrict__ vol, T W) {
    constexpr int KW = KS ? KS : kMaxBand;
    using Lay = ReinitLds<KW, YB>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);
    __shared__ double red[kMT / 64];
    if (ctl_failed(ma.ctl) || (int)blockIdx.x >= ma.G) return;
    const int k = ma.order ? ma.order[blockIdx.x] : (int)blockIdx.x;
    constexpr bool d3 = D3;
    if (!Ln.alive[k]) {
        if (!d3 && vol && threadIdx.x == 0) vol[k] = 0.0;
        return;
    }
    const int K = KS ? KS : ma.K;
    int ne[3], oe[3], dd[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        ne[a] = Ln.ext[3 * k + a];
        oe[a] = Lo.ext[3 * k + a];
        const int t = Ln.lo[3 * k + a] - Lo.lo[3 * k + a];  // both in [0, n)
        dd[a] = t < 0 ? t + ma.n[a] : t;
    }
    const T *src = phic + Lo.off[k];
    T *dst = out + Ln.off[k];
    const int *io_src = IO ? iota_old + Lo.off[k] : nullptr;
    int *io_dst = IO ? iota_new + Ln.off[k] : nullptr;
    const int osz = oe[0] * oe[1];  // box volumes are below 2^31
    const int nplane = ne[0] * ne[1];
    const int ez = d3 ? ne[2] : 1;
    const bool ringz = d3 && ne[2] == ma.n[2];
    const T inf = tinf<T>();
    const MSplit sp = march_split<YB, Lay>(ne[0], ne[1], ma.n[0], ma.n[1], K + 1, reinit_cells<T>());
    double vsum = 0.0;
    for (int tile = 0; tile < sp.nt[0] * sp.nt[1]; ++tile) {
        const MTile tl = march_tile(sp, tile);
        const int EX = tl.ext[0], EY = tl.ext[1];
        // The tile body comes twice: with the LDS pitches of a tile kPitchW
        // wide, fixed at compile time (window reads then take immediate
        // offsets), when the tile is at most that wide and that layout fits;
        // else with the tile's own pitches.
        auto body = [&](auto wc) {
        constexpr int WC = decltype(wc)::value;
        const Lay ly(WC ? WC : EX, EY);
        // frames: -W around phi^c, +inf around the spreading inputs
        lds_fill(sm, ly.oR, -W);
        lds_fill(sm + ly.oR, ly.total - ly.oR, inf);
        __syncthreads();
        const MCol<YB> c = march_col<YB>(tl, ne[0], ne[1], ma.n[0], ma.n[1]);
        // old-box offsets of the column's cells within a plane (-1: outside the old box)
        int ocol = c.bx + dd[0];
        ocol -= ocol >= ma.n[0] ? ma.n[0] : 0;
        int orow[YB], nrow[YB];
#pragma unroll
        for (int j = 0; j < YB; ++j) {
            int oy = c.by[j] + dd[1];
            oy -= oy >= ma.n[1] ? ma.n[1] : 0;
            orow[j] = (c.rv[j] && ocol < oe[0] && oy < oe[1]) ? oy * oe[0] + ocol : -1;
            nrow[j] = c.by[j] * ne[0] + c.bx;
        }
        // the same as byte offsets inside a plane (below 2^32: a plane has at
        // most 4096^2 cells), for addressing from a uniform plane base
        unsigned orb[YB], nrb[YB];
#pragma unroll
        for (int j = 0; j < YB; ++j) {
            orb[j] = orow[j] >= 0 ? (unsigned)orow[j] * (unsigned)sizeof(T) : 0u;
            nrb[j] = (unsigned)nrow[j] * (unsigned)sizeof(T);
        }
        auto oplane = [&](int z) -> int {  // old-box offset of new plane z, -1 outside either box
            int zm = d3 ? axis_map(z, ne[2], ma.n[2]) : (z == 0 ? 0 : -1);
            if (zm < 0) return -1;
            int oz = zm + dd[2];
            oz -= oz >= ma.n[2] ? ma.n[2] : 0;
            return oz < oe[2] ? oz * osz : -1;
        };
        // Loads are issued for every row (outside the old box from its first
        // value), and which of them stand for -W is kept in `okp` (bit YB slot + j)
        // until the plane is settled where it is first used, so that the number
        // of loads in flight is the same on every path.
        static_assert(5 * YB <= 32, "validity bits of the plane ring");
        unsigned okp = 0;
        auto load = [&](int z, int slot, T (&v)[YB]) {
            const int po = oplane(z);
            const T *sp = src + (po >= 0 ? po : 0);
#pragma unroll
            for (int j = 0; j < YB; ++j) {
                const bool ok = po >= 0 && orow[j] >= 0;
                v[j] = at_bytes(sp, ok ? orb[j] : 0u);
                const unsigned bit = 1u << (YB * slot + j);
                okp = ok ? (okp | bit) : (okp & ~bit);
            }
        };
        auto settle = [&](int slot, T (&v)[YB]) {
#pragma unroll
            for (int j = 0; j < YB; ++j) v[j] = ((okp >> (YB * slot + j)) & 1u) ? v[j] : -W;
        };
        // planes in a ring of five buffers, plane p in P[(p + 2) % 5]: at
        // iteration z the planes z - 2, z - 1, z are used and z + 1, z + 2 are on
        // their way.  The plane loop is unrolled by five so that every buffer has
        // a fixed register home (a loaded plane is never moved, and its load is
        // waited for only where it is used, three iterations later).
        T P[5][YB], car[YB];
#pragma unroll
        for (int i = 0; i < 5; ++i) load(i - 2, i, P[i]);
        settle(0, P[0]);
        settle(1, P[1]);
#pragma unroll
        for (int j = 0; j < YB; ++j) car[j] = inf;
        unsigned ins = 0;  // inside flags: bit 4 j + (plane & 3)
        const int nxq = (EX + kQXR - 1) / kQXR;
        const RowWalk rw0(EY, row_unit0<GG_ROW_REVERSE>());
        const int fc = (c.ry0 + 1) * ly.pf + c.cx + 1;  // the unit's first cell in F
        // stages of iteration z: A plane z (phi^c into F), B plane z - 1
        // (reference values into Rf), C plane z - 2 (x spreading into Dx), D and
        // E plane z - 3 (y spreading, forward z spreading, output)
        // (the last group of five may run past plane ez + 2: its stages are off)
        for (int zb = 0; zb < ez + 3; zb += 5)
#pragma unroll
        for (int r = 0; r < 5; ++r) {
            const int z = zb + r;
            T(&q0)[YB] = P[r];
            T(&q1)[YB] = P[(r + 1) % 5];
            T(&q2)[YB] = P[(r + 2) % 5];
            settle((r + 2) % 5, q2);
            if (z < ez && c.act) {
                T *Fb = sm + (z & 1) * ly.sF;
#pragma unroll
                for (int j = 0; j < YB; ++j) {
                    if (!c.rv[j]) continue;
                    Fb[fc + j * ly.pf] = q2[j];
                    const unsigned bit = 1u << (4 * j + (z & 3));
                    ins = q2[j] > T(0) ? (ins | bit) : (ins & ~bit);
                }
            }
            if (z >= 1 && z - 1 < ez && c.act) {
                // reference values.  Over all neighbours the smallest value is <= 0
                // exactly when an inside cell has an outside neighbour, and then it
                // is the extreme one (likewise the largest for an outside cell);
                // theta = fc / (fc - fn) is monotone in fn on that side, and so are
                // the rounded operations, so the extreme neighbour gives the
                // smallest theta.
                const T *Fb = sm + ((z - 1) & 1) * ly.sF;
                T *Rb = sm + ly.oR + ((z - 1) & 1) * ly.sR;
#pragma unroll
                for (int j = 0; j < YB; ++j) {
                    if (!c.rv[j]) continue;
                    const int a = fc + j * ly.pf;
                    const T xm = Fb[a - 1], xp = Fb[a + 1];
                    const T ym = j > 0 ? q1[j > 0 ? j - 1 : 0] : Fb[a - ly.pf];
                    const T yp = (j + 1 < YB && c.rv[j + 1 < YB ? j + 1 : j]) ? q1[j + 1 < YB ? j + 1 : j] : Fb[a + ly.pf];
                    T lo = vmin(vmin(xm, xp), vmin(ym, yp)), hi = vmax(vmax(xm, xp), vmax(ym, yp));
                    if (d3) {
                        lo = vmin(lo, vmin(q0[j], q2[j]));
                        hi = vmax(hi, vmax(q0[j], q2[j]));
                    }
                    const T cur = q1[j];
                    const bool in = cur > T(0);
                    const T ext = in ? lo : hi;
                    T r = inf;
                    if ((ext > T(0)) != in) r = ratio(cur, cur - ext);
                    Rb[(c.ry0 + j) * ly.pr + c.cx + KW] = r;
                }
            }
            if (z >= 2 && z - 2 < ez) {
                // spreading along x (row units, rows fastest across lanes); the
                // window [x0 - KW, x0 + kQXR + KW) reads the +inf frame beyond the tile
                const T *Rb = sm + ly.oR + ((z - 2) & 1) * ly.sR;
                T *Db = sm + ly.oD + ((z - 2) & 1) * ly.sD;
                for (RowWalk rw = rw0; rw.xq < nxq; rw.next(EY)) {
                    const int ry = rw.ry, x0 = rw.xq * kQXR;
                    const T *row = Rb + ry * ly.pr + x0;
                    T v[kQXR + 2 * KW];
#pragma unroll
                    for (int i = 0; i < kQXR + 2 * KW; ++i) v[i] = row[i];
                    T o[kQXR];
                    taxicab_chains<T, kQXR + 2 * KW, KW, kQXR>(v, o);
                    T *drow = Db + (ry + KW) * ly.pd + x0;
#pragma unroll
                    for (int q = 0; q < kQXR; ++q)
                        if (x0 + q < EX) drow[q] = o[q];
                }
            }
            if (z >= 3 && z - 3 < ez && c.act) {
                // spreading along y for the column unit (rows [ry0 - KW, ry0 + YB + KW)),
                // forward spreading along z, output of the interior cells
                const int zz = z - 3;
                const T *col = sm + ly.oD + (zz & 1) * ly.sD + c.ry0 * ly.pd + c.cx;
                T v[YB + 2 * KW], d[YB];
#pragma unroll
                for (int i = 0; i < YB + 2 * KW; ++i) v[i] = col[i * ly.pd];
                taxicab_chains<T, YB + 2 * KW, KW, YB>(v, d);
                const int po = oplane(zz);
                T *dp = dst + (long long)zz * nplane;
#pragma unroll
                for (int j = 0; j < YB; ++j) {
                    if (!c.rint[j]) continue;
                    const bool in = (ins >> (4 * j + (zz & 3))) & 1u;
                    const int idx = zz * nplane + nrow[j];
                    if (d3) {
                        car[j] = vmin(d[j], car[j] + T(1));
                        at_bytes(dp, nrb[j]) = in ? car[j] : -car[j];
                    } else {
                        const T dc = d[j] < W ? d[j] : W;
                        const T pv = in ? dc : -dc;
                        at_bytes(dp, nrb[j]) = pv;
                        double cl = (double)pv + 0.5;
                        cl = cl < 0.0 ? 0.0 : (cl > 1.0 ? 1.0 : cl);
                        vsum += cl;
                    }
                    if constexpr (IO) io_dst[idx] = (po >= 0 && orow[j] >= 0) ? io_src[po + orow[j]] : -1;
                }
            }
            if (d3) load(z + 3, r, q0);  // plane z + 3 takes the place of plane z - 2
            __syncthreads();
        }
        if (ringz) {
            // a whole periodic z axis is a ring: the forward chain goes around a
            // second time from plane 0, over the values of the first lap
            __threadfence();
            for (int z = 0; z < ez; ++z)
#pragma unroll
                for (int j = 0; j < YB; ++j) {
                    if (!c.rint[j]) continue;
                    const int idx = z * nplane + nrow[j];
                    const T v = dst[idx];
                    car[j] = vmin(T(fabs(v)), car[j] + T(1));
                    dst[idx] = copysign(car[j], v);
                }
        }
        __syncthreads();  // the next tile refills the frames
        };
        if (EX <= kPitchW && Lay(kPitchW, EY).total <= reinit_cells<T>()) body(std::integral_constant<int, kPitchW>{});
        else body(std::integral_constant<int, 0>{});
    }
    if (!d3) {
        const double s = block_sum(vsum, red);
        if (threadIdx.x == 0 && vol) vol[k] = s;
    }
}

// ------------------------------------------------------ k_predict_march (a1, a2)

// d^p = phi + w (psi - phi) + mob (E_j - E_k) * bulk_scale, clamped to [-W, W],
// for a cell whose ID-field entry is j and whose function value is p; w from
// the pair (k, j), or wc when wc >= 0 (closest-boundary-point weights).
template <typename T>
__device__ inline T correct_prediction_v(const Physics<T> &ph, int k, int j, T p, T psi, T W, PairCache<T> &pc,
                                         T wc) {
    if (j != pc.j) {
        pc.j = j;
        pc.w = 1;
        pc.b = 0;
        if (j >= 0) {
            T mob = 1;
            if (ph.mode & 1) {
                const T th = misorientation_deg<T>(ph.quat + 4LL * k, ph.quat + 4LL * j);
                pc.w = pair_weight<T>(th, ph.theta_c_deg, &mob);
            }
            if (ph.mode & 2) pc.b = mob * (ph.energy[j] - ph.energy[k]) * ph.bulk_scale;
        }
    }
    T d = p + (wc >= T(0) ? wc : pc.w) * (psi - p) + pc.b;
    d = d > W ? W : d;
    d = d < -W ? -W : d;
    return d;
}

// The in-plane Gaussian passes of one plane: Cz (the z-convolved plane, x
// frames of RM cells of -W) -> Cx (x pass, row units; y frames of RM rows of
// -W) -> the column unit's y pass in `acc`.  Two barriers: Cz is complete
// before the x pass, Cx before the y pass.
template <typename T, int RM, int YB>
__device__ __forceinline__ void plane_xy_pass(const T *Cz, T *Cx, const PredictLds<RM, YB> &ly, int EX, int EY,
                                              const MCol<YB> &c, const T *tp, int R, T (&acc)[YB]) {
    __syncthreads();
    const int nxq = (EX + kQXP - 1) / kQXP;
    for (int r = row_unit0<GG_ROW_REVERSE_P>(); r < EY * nxq; r += kMT) {
        const int ry = r % EY, x0 = (r / EY) * kQXP;
        const T *row = Cz + ry * ly.pz + x0 + (RM - R);
        T v[kQXP + 2 * RM];
#pragma unroll
        for (int i = 0; i < kQXP + 2 * RM; ++i) v[i] = (i < kQXP + 2 * R) ? row[i] : T(0);
        T o[kQXP];
        gauss_window<T, RM, kQXP>(v, tp, R, o);
        T *xrow = Cx + (ry + RM) * ly.px + x0;
#pragma unroll
        for (int q = 0; q < kQXP; ++q)
            if (x0 + q < EX) xrow[q] = o[q];
    }
    __syncthreads();
    if (c.act) {
        const T *col = Cx + (c.ry0 + RM - R) * ly.px + c.cx;
        T v[YB + 2 * RM];
#pragma unroll
        for (int i = 0; i < YB + 2 * RM; ++i) v[i] = (i < YB + 2 * R) ? col[i * ly.px] : T(0);
        gauss_window<T, RM, YB>(v, tp, R, acc);
    }
}

// Backward spreading along z of the forward-spread distances f (sign bit: the
// inside flag), band clamp phi = +-min(d, W), the grain volume sum of clamp(phi
// + 1/2, 0, 1) (3D), and the predictor psi = G_sigma * phi (passes z, x, y; a
// sample outside the box reads -W), with the correction epilogue when PH.
// chain = 0: the input is already a final function (the identity on it).
// psi == NULL: phi and the volume only.  phi_out: phi is stored when given and
// the step is the one ma.ctl->phi_at names (always without a control block).
// RS: static radius (0: runtime ma.R <= kMaxRadius).
#ifndef GG_PREDICT_WAVES
#define GG_PREDICT_WAVES 4
#endif
template <typename T, int RS, int YB, bool PH>
__global__ void __launch_bounds__(kMT, sizeof(T) == 4 && !PH ? GG_PREDICT_WAVES : 1)
    k_predict_march(Boxes L, MarchArgs ma, T *__restrict__ in, T *__restrict__ psi, T *__restrict__ phi_out,
                    double *__restrict__ vol, const T *__restrict__ taps, Physics<T> ph, T W, int chain) {
    constexpr int RM = RS ? RS : kMaxRadius;
    constexpr int NW = 2 * RM + 1;
    using Lay = PredictLds<RM, YB>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);
    __shared__ double red[kMT / 64];
    if (ctl_failed(ma.ctl) || (int)blockIdx.x >= ma.G) return;
    const int k = ma.order ? ma.order[blockIdx.x] : (int)blockIdx.x;
    const bool d3 = ma.dim == 3;
    if (!L.alive[k]) {
        if (d3 && vol && threadIdx.x == 0) vol[k] = 0.0;
        return;
    }
    const int R = RS ? RS : ma.R;
    const bool want_psi = psi != nullptr;
    const bool write_phi =
        phi_out != nullptr && (ma.ctl == nullptr || ma.phi_always || ma.ctl->steps == ma.ctl->phi_at);
    const int ex = L.ext[3 * k], ey = L.ext[3 * k + 1], ez = d3 ? L.ext[3 * k + 2] : 1;
    const int plane = ex * ey;  // box volumes are below 2^31
    T *f = in + L.off[k];
    T *pp = want_psi ? psi + L.off[k] : nullptr;
    T *po = write_phi ? phi_out + L.off[k] : nullptr;
    const int *io = PH ? ph.iota + L.off[k] : nullptr;
    const T *wcb = (PH && ph.wcp) ? ph.wcp + L.off[k] : nullptr;
    T tp[NW];
#pragma unroll
    for (int t = 0; t < NW; ++t) tp[t] = (want_psi && t <= 2 * R) ? taps[t] : T(0);
    const MSplit sp = march_split<YB, Lay>(ex, ey, ma.n[0], ma.n[1], want_psi ? R : 0, predict_cells<T>());
    const bool ringz = d3 && ez == ma.n[2];
    const T inf = tinf<T>();
    double vsum = 0.0;
    PairCache<T> pc;

    auto emit = [&](const MCol<YB> &c, int q, const T (&acc)[YB], const T (&phv)[YB]) {
#pragma unroll
        for (int j = 0; j < YB; ++j) {
            if (!c.rint[j]) continue;
            const int idx = q * plane + c.by[j] * ex + c.bx;
            T val = acc[j];
            if constexpr (PH) val = correct_prediction_v<T>(ph, k, io[idx], phv[j], val, W, pc, wcb ? wcb[idx] : T(-1));
            pp[idx] = val;
        }
    };
    // frames of -W around both buffers (the next tile refills after a barrier)
    auto frames = [&](const Lay &ly) {
        __syncthreads();
        lds_fill(sm, ly.total, -W);
        __syncthreads();
    };

    if (!d3) {
        // 2D: the input is the final function; x and y passes only
        for (int tile = 0; tile < sp.nt[0] * sp.nt[1] && want_psi; ++tile) {
            const MTile tl = march_tile(sp, tile);
            const int EX = tl.ext[0], EY = tl.ext[1];
            const Lay ly(EX, EY);
            frames(ly);
            T *Cz = sm, *Cx = sm + ly.oX;
            const MCol<YB> c = march_col<YB>(tl, ex, ey, ma.n[0], ma.n[1]);
            T phv[YB];
#pragma unroll
            for (int j = 0; j < YB; ++j) {
                phv[j] = c.rv[j] ? f[c.by[j] * ex + c.bx] : -W;
                if (c.rv[j]) Cz[(c.ry0 + j) * ly.pz + c.cx + RM] = phv[j];
            }
            T acc[YB];
            plane_xy_pass<T, RM, YB>(Cz, Cx, ly, EX, EY, c, tp, R, acc);
            emit(c, 0, acc, phv);
        }
        return;
    }

    if (ringz) {
        // A whole periodic z axis: the backward chain goes around twice (from
        // the last plane), then the final function is convolved with wrapped
        // planes.  Phase 1 writes phi of every interior cell (to phi_out, or in
        // place); phase 2 reads it back after a fence.
        T *tgt = po ? po : f;
        for (int tile = 0; tile < sp.nt[0] * sp.nt[1]; ++tile) {
            const MTile tl = march_tile(sp, tile);
            const MCol<YB> c = march_col<YB>(tl, ex, ey, ma.n[0], ma.n[1]);
            T car[YB];
#pragma unroll
            for (int j = 0; j < YB; ++j) car[j] = inf;
            for (int lap = 0; lap < 2; ++lap) {
                for (int z = ez - 1; z >= 0; --z)
#pragma unroll
                    for (int j = 0; j < YB; ++j) {
                        if (!c.rint[j]) continue;
                        const int idx = z * plane + c.by[j] * ex + c.bx;
                        const T v = lap ? tgt[idx] : f[idx];
                        const T a = fabs(v);
                        T b = a;
                        if (chain) b = (lap == 0 && z == ez - 1) ? a : vmin(a, car[j] + T(1));
                        car[j] = b;
                        if (lap == 0) {
                            tgt[idx] = copysign(b, v);
                        } else {
                            const T dc = b < W ? b : W;
                            const T pv = signbit(v) ? -dc : dc;
                            tgt[idx] = pv;
                            double cl = (double)pv + 0.5;
                            cl = cl < 0.0 ? 0.0 : (cl > 1.0 ? 1.0 : cl);
                            vsum += cl;
                        }
                    }
                __threadfence();
            }
        }
        __syncthreads();
        for (int tile = 0; tile < sp.nt[0] * sp.nt[1] && want_psi; ++tile) {
            const MTile tl = march_tile(sp, tile);
            const int EX = tl.ext[0], EY = tl.ext[1];
            const Lay ly(EX, EY);
            frames(ly);
            T *Cz = sm, *Cx = sm + ly.oX;
            const MCol<YB> c = march_col<YB>(tl, ex, ey, ma.n[0], ma.n[1]);
            T win[NW][YB];
#pragma unroll
            for (int i = 0; i < NW; ++i)
#pragma unroll
                for (int j = 0; j < YB; ++j) win[i][j] = -W;
            for (int p = ez - 1 + R; p >= -R; --p) {
                const int pz = p < 0 ? p + ez : (p >= ez ? p - ez : p);
#pragma unroll
                for (int i = NW - 1; i > 0; --i)
#pragma unroll
                    for (int j = 0; j < YB; ++j) win[i][j] = win[i - 1][j];
#pragma unroll
                for (int j = 0; j < YB; ++j) win[0][j] = c.rv[j] ? tgt[pz * plane + c.by[j] * ex + c.bx] : -W;
                const int q = p + R;
                if (q > ez - 1 || q < 0) continue;
                T phv[YB];
#pragma unroll
                for (int j = 0; j < YB; ++j) {
                    phv[j] = win[R][j];
                    if (!c.rv[j]) continue;
                    T a = T(0);
#pragma unroll
                    for (int t = 0; t < NW; ++t)
                        if (t <= 2 * R) a = mac<T>(a, tp[t], win[t][j]);
                    Cz[(c.ry0 + j) * ly.pz + c.cx + RM] = a;
                }
                T acc[YB];
                plane_xy_pass<T, RM, YB>(Cz, Cx + 0, ly, EX, EY, c, tp, R, acc);
                emit(c, q, acc, phv);
            }
        }
    } else {
        for (int tile = 0; tile < sp.nt[0] * sp.nt[1]; ++tile) {
            const MTile tl = march_tile(sp, tile);
            const int EX = tl.ext[0], EY = tl.ext[1];
            // as in the re-initialization: compile-time LDS pitches for tiles at
            // most kPitchW wide whose layout at that width fits
            auto body = [&](auto wc) {
            constexpr int WC = decltype(wc)::value;
            const Lay ly(WC ? WC : EX, EY);
            if (want_psi) frames(ly);
            const MCol<YB> c = march_col<YB>(tl, ex, ey, ma.n[0], ma.n[1]);
            int cell[YB];
#pragma unroll
            for (int j = 0; j < YB; ++j) cell[j] = c.by[j] * ex + c.bx;
            // Input planes in a ring of PR buffers: iteration i (plane p = ez - 1
            // - i) uses PF[i % PR] and loads the plane of iteration i + PR - 1 into
            // the buffer of iteration i - 1.  The plane loop is unrolled by PR so
            // that every buffer has a fixed register home (a loaded plane is never
            // moved).  Every load is issued (rows and planes outside the box read
            // plane 0 and are not used), so that the number in flight is the same
            // on every path.
            constexpr int PR = 3;
            T win[NW][YB], bcar[YB], PF[PR][YB];
            auto load = [&](int pz, T(&v)[YB]) {
#pragma unroll
                for (int j = 0; j < YB; ++j) v[j] = f[(pz > 0 ? pz : 0) * plane + cell[j]];
            };
#pragma unroll
            for (int j = 0; j < YB; ++j) {
                bcar[j] = inf;
#pragma unroll
                for (int i = 0; i < NW; ++i) win[i][j] = -W;
            }
#pragma unroll
            for (int d = 0; d + 1 < PR; ++d) load(ez - 1 - d, PF[d]);
            const int nxq = (EX + kQXP - 1) / kQXP;
            // stages of the iteration for input plane p (descending): the z pass
            // of plane p + R into Cz, the x pass of plane p + R + 1 (Cz -> Cx), the
            // y pass and output of plane p + R + 2 (from Cx); the last group of PR
            // may run past plane pend, with every stage off
            const int pend = want_psi ? -R - 2 : 0;
            for (int pb = ez - 1; pb >= pend; pb -= PR)
#pragma unroll
            for (int u = 0; u < PR; ++u) {
                const int p = pb - u;
                load(p - (PR - 1), PF[(u + PR - 1) % PR]);
                T phv[YB];
                if (p >= 0) {
                    T(&cur)[YB] = PF[u];
#pragma unroll
                    for (int j = 0; j < YB; ++j) {
                        if (!c.rv[j]) {
                            phv[j] = -W;
                            continue;
                        }
                        const T a = fabs(cur[j]);
                        const T b = chain ? vmin(a, bcar[j] + T(1)) : a;
                        bcar[j] = b;
                        const T dc = b < W ? b : W;
                        phv[j] = signbit(cur[j]) ? -dc : dc;
                        if (c.rint[j]) {
                            double cl = (double)phv[j] + 0.5;
                            cl = cl < 0.0 ? 0.0 : (cl > 1.0 ? 1.0 : cl);
                            vsum += cl;
                            if (po) po[p * plane + cell[j]] = phv[j];
                        }
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < YB; ++j) phv[j] = -W;
                }
                if (!want_psi) continue;
                // window: win[i] holds plane p + i
#pragma unroll
                for (int i = NW - 1; i > 0; --i)
#pragma unroll
                    for (int j = 0; j < YB; ++j) win[i][j] = win[i - 1][j];
#pragma unroll
                for (int j = 0; j < YB; ++j) win[0][j] = phv[j];
                const int qz = p + R, qx = qz + 1, qy = qz + 2;
                if (qy >= 0 && qy <= ez - 1 && c.act) {
                    // y pass and output of plane qy (its phi: window entry R + 2)
                    const T *col = sm + ly.oX + (qy & 1) * ly.sX + (c.ry0 + RM - R) * ly.px + c.cx;
                    T v[YB + 2 * RM], acc[YB], phy[YB];
#pragma unroll
                    for (int i = 0; i < YB + 2 * RM; ++i) v[i] = (i < YB + 2 * R) ? col[i * ly.px] : T(0);
                    gauss_window<T, RM, YB>(v, tp, R, acc);
#pragma unroll
                    for (int j = 0; j < YB; ++j) phy[j] = win[R + 2][j];
                    emit(c, qy, acc, phy);
                }
                if (qx >= 0 && qx <= ez - 1) {
                    // x pass of plane qx (row units, rows fastest across lanes)
                    const T *Zb = sm + (qx & 1) * ly.sZ;
                    T *Xb = sm + ly.oX + (qx & 1) * ly.sX;
                    for (int r = row_unit0<GG_ROW_REVERSE_P>(); r < EY * nxq; r += kMT) {
                        const int ry = r % EY, x0 = (r / EY) * kQXP;
                        const T *row = Zb + ry * ly.pz + x0 + (RM - R);
                        T v[kQXP + 2 * RM];
#pragma unroll
                        for (int i = 0; i < kQXP + 2 * RM; ++i) v[i] = (i < kQXP + 2 * R) ? row[i] : T(0);
                        T o[kQXP];
                        gauss_window<T, RM, kQXP>(v, tp, R, o);
                        T *xrow = Xb + (ry + RM) * ly.px + x0;
#pragma unroll
                        for (int q = 0; q < kQXP; ++q)
                            if (x0 + q < EX) xrow[q] = o[q];
                    }
                }
                if (qz >= 0 && qz <= ez - 1 && c.act) {
                    // z pass of plane qz from the window (ascending taps)
                    T *Zb = sm + (qz & 1) * ly.sZ;
#pragma unroll
                    for (int j = 0; j < YB; ++j) {
                        if (!c.rv[j]) continue;
                        T a = T(0);
#pragma unroll
                        for (int t = 0; t < NW; ++t)
                            if (t <= 2 * R) a = mac<T>(a, tp[t], win[t][j]);
                        Zb[(c.ry0 + j) * ly.pz + c.cx + RM] = a;
                    }
                }
                // the stages of the next iteration read what this one wrote (the z
                // stage writes from qz = ez - 1 on, one iteration before the first
                // x stage reads it), and write what this one read
                if (qz <= ez - 1) __syncthreads();
            }
            };
            if (EX <= kPitchW && Lay(kPitchW, EY).total <= predict_cells<T>()) body(std::integral_constant<int, kPitchW>{});
            else body(std::integral_constant<int, 0>{});
        }
    }
    const double s = block_sum(vsum, red);
    if (threadIdx.x == 0 && vol) vol[k] = s;
}

// ------------------------------------------------------ step bookkeeping

// Zero n ints (graph-safe replacement of a memset).
__global__ void k_zero_int(int *p, int n, const Ctl *ctl) {
    if (ctl_failed(ctl)) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// End of a completed step: alive count and sizes of the new layout, grain
// voxels of the step (the box volumes of its input layout), step counter.
__global__ void __launch_bounds__(1024) k_step_end(Ctl *ctl, const int *alive_new, const long long *off_in,
                                                   const long long *off_new, const long long *cov_total, int G) {
    if (ctl->fail) return;
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int local = 0;
    for (int k = threadIdx.x; k < G; k += blockDim.x) local += alive_new[k] != 0;
    atomicAdd(&cnt, local);
    __syncthreads();
    if (threadIdx.x == 0) {
        ctl->alive = cnt;
        ctl->last_gv = off_in[G];
        ctl->total_gv += off_in[G];
        ctl->arena_now = off_new[G];
        ctl->cov_now = *cov_total;
        ctl->steps += 1;
    }
}

// Launch order of the march kernels: grains by box volume, largest first
// (classes of equal floor(log2 volume); the order within a class is
// arbitrary), extinct grains last.  One work group.
__global__ void __launch_bounds__(1024) k_order_size(const long long *off, const int *alive, int *order, int G,
                                                     const Ctl *ctl) {
    if (ctl_failed(ctl)) return;
    __shared__ int cnt[64], cur[64];
    const int t = threadIdx.x;
    if (t < 64) cnt[t] = 0;
    __syncthreads();
    auto bucket = [&](int k) {
        const long long v = alive[k] ? off[k + 1] - off[k] : 0;
        return v > 0 ? __clzll(v) : 63;  // larger volume: fewer leading zeros
    };
    for (int k = t; k < G; k += blockDim.x) atomicAdd(&cnt[bucket(k)], 1);
    __syncthreads();
    if (t == 0) {
        int s = 0;
        for (int b = 0; b < 64; ++b) {
            cur[b] = s;
            s += cnt[b];
        }
    }
    __syncthreads();
    for (int k = t; k < G; k += blockDim.x) order[atomicAdd(&cur[bucket(k)], 1)] = k;
}

}  // namespace gg
