// Correction weights from the closest grain-boundary point (sec. 3.2, with the
// correction of sec. 2.1.4).
//
// Every voxel of grain k's box inside the narrow tube |phi| < kClosestTube
// adopts the boundary character of the closest point of the linearised zero
// level set of phi_k:
//   - each cell (nodes c + {0,1}^D inside the box; on an axis the box takes
//     whole, cells wrap around the periodic grid) is cut along its main
//     diagonal into simplices -- triangles (0,1,3), (0,2,3) in 2D, the six
//     tetrahedra (0, e_a, e_a + e_b, 7) in 3D (corner bit 0 = x, 1 = y, 2 = z);
//     the zero set of the linear interpolant on a simplex is a segment (2D) or
//     one or two triangles (3D);
//   - a crossing vertex on the simplex edge from node u to node v (u <= v
//     componentwise) lies at u + t (v - u), t = phi_u / (phi_u - phi_v), in
//     coordinates relative to the voxel (integers plus t);
//   - a piece's character is the set of distinct ID-field entries j >= 0 at its
//     cell's nodes (one: the boundary with grain j; more: a junction), its
//     weight the mean of w(k, j) over the set (1 when empty);
//   - the voxel takes the weight of the piece of smallest squared distance,
//     ties to the lowest cell (linear box index of its lower node), then the
//     lowest piece; outside the tube the ID-field pair (k, iota) decides.
// Distances follow one fixed sequence of FP64 operations (segment: endpoints in
// node-key order, clamped projection; triangle: the plane distance when the
// projection falls inside, else the nearest edge), so that a voxel equally far
// from two pieces sharing a vertex or an edge gets the same value from both.
//
// Search per tube voxel: rings of cells around it ([-r-1, r] per axis, r = 0,
// 1, ...) until a piece is found, then every cell within the found distance
// (cells whose integer box distance exceeds it are skipped).  On a whole
// periodic axis a cell is taken at the image whose offset lies in
// [-floor(e/2), ceil(e/2) - 1], and the search never leaves that range.
#pragma once

#include "gg_kernels.hpp"

namespace gg {

constexpr double kClosestTube = 2.0;

struct CVtx {
    int u[3];  // node u relative to the voxel
    int d[3];  // v - u, 0 or 1
    double t;
};

__device__ inline void cv_pos(const CVtx &a, double p[3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) p[i] = (double)a.u[i] + a.t * (double)a.d[i];
}

// node-key order (u_z, u_y, u_x, v_z, v_y, v_x)
__device__ inline bool cv_less(const CVtx &a, const CVtx &b) {
    const int ka[6] = {a.u[2], a.u[1], a.u[0], a.u[2] + a.d[2], a.u[1] + a.d[1], a.u[0] + a.d[0]};
    const int kb[6] = {b.u[2], b.u[1], b.u[0], b.u[2] + b.d[2], b.u[1] + b.d[1], b.u[0] + b.d[0]};
#pragma unroll
    for (int i = 0; i < 6; ++i)
        if (ka[i] != kb[i]) return ka[i] < kb[i];
    return false;
}

__device__ inline double v3dot(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

__device__ inline void v3cross(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// squared distance from the voxel (the origin) to the segment PQ
__device__ inline double cv_seg2(const CVtx &P0, const CVtx &Q0) {
    const bool sw = cv_less(Q0, P0);
    const CVtx &P = sw ? Q0 : P0, &Q = sw ? P0 : Q0;
    double p[3], q[3], d[3], c[3];
    cv_pos(P, p);
    cv_pos(Q, q);
#pragma unroll
    for (int i = 0; i < 3; ++i) d[i] = q[i] - p[i];
    const double dd = v3dot(d, d);
    double s = 0.0;
    if (dd > 0.0) {
        s = -v3dot(p, d) / dd;
        s = s < 0.0 ? 0.0 : s;
        s = s > 1.0 ? 1.0 : s;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) c[i] = p[i] + s * d[i];
    return v3dot(c, c);
}

// squared distance from the origin to the triangle ABC
__device__ inline double cv_tri2(const CVtx &A, const CVtx &B, const CVtx &C) {
    double a[3], b[3], c[3], ab[3], ac[3], bc[3], ca[3], n[3];
    cv_pos(A, a);
    cv_pos(B, b);
    cv_pos(C, c);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        ab[i] = b[i] - a[i];
        ac[i] = c[i] - a[i];
        bc[i] = c[i] - b[i];
        ca[i] = a[i] - c[i];
    }
    v3cross(ab, ac, n);
    const double nn = v3dot(n, n);
    if (nn > 0.0) {
        const double ma[3] = {-a[0], -a[1], -a[2]}, mb[3] = {-b[0], -b[1], -b[2]}, mc[3] = {-c[0], -c[1], -c[2]};
        double e0[3], e1[3], e2[3];
        v3cross(ab, ma, e0);
        v3cross(bc, mb, e1);
        v3cross(ca, mc, e2);
        if (v3dot(n, e0) >= 0.0 && v3dot(n, e1) >= 0.0 && v3dot(n, e2) >= 0.0) {
            const double h = v3dot(n, ma);
            return h * h / nn;
        }
    }
    double m = cv_seg2(A, B);
    const double m1 = cv_seg2(B, C), m2 = cv_seg2(C, A);
    m = m1 < m ? m1 : m;
    m = m2 < m ? m2 : m;
    return m;
}

// crossing vertex on the edge between cell corners bu <= bv (corner bits); o:
// the cell's lower node relative to the voxel
__device__ inline CVtx cv_edge(const int o[3], int bu, int bv, const double *f) {
    CVtx r;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.u[a] = o[a] + ((bu >> a) & 1);
        r.d[a] = ((bv >> a) & 1) - ((bu >> a) & 1);
    }
    r.t = f[bu] / (f[bu] - f[bv]);
    return r;
}

// The best piece so far: smallest d2, then cell, then piece.
struct CBest {
    double d2;
    int cell, piece;
    __device__ void take(double v, int c, int p) {
        if (v < d2 || (v == d2 && (c < cell || (c == cell && p < piece)))) {
            d2 = v;
            cell = c;
            piece = p;
        }
    }
};

// Every piece of one cell (lower node at offset o, node values f by corner
// bits) against the best so far.  Pieces: 2D triangle i -> piece i; 3D
// tetrahedron i -> piece 2i (and 2i + 1 for a quadrilateral zero set).
__device__ inline void cell_pieces(int dim, const int o[3], const double *f, int cell, CBest &best) {
    if (dim == 2) {
        constexpr int tris[2][3] = {{0, 1, 3}, {0, 2, 3}};
        for (int ti = 0; ti < 2; ++ti) {
            const int *tv = tris[ti];
            const bool i0 = f[tv[0]] > 0.0, i1 = f[tv[1]] > 0.0, i2 = f[tv[2]] > 0.0;
            const int nin = (int)i0 + (int)i1 + (int)i2;
            if (nin == 0 || nin == 3) continue;
            // the lone vertex: inside when one is inside, outside when two are
            const bool want = nin == 1;
            const int lone = i0 == want ? 0 : (i1 == want ? 1 : 2);
            const int a = lone == 0 ? 1 : 0, b = lone == 2 ? 1 : 2;  // the other two, increasing
            const CVtx va = cv_edge(o, tv[min(lone, a)], tv[max(lone, a)], f);
            const CVtx vb = cv_edge(o, tv[min(lone, b)], tv[max(lone, b)], f);
            best.take(cv_seg2(va, vb), cell, ti);
        }
        return;
    }
    constexpr int tets[6][4] = {{0, 1, 3, 7}, {0, 1, 5, 7}, {0, 2, 3, 7}, {0, 2, 6, 7}, {0, 4, 5, 7}, {0, 4, 6, 7}};
    for (int ti = 0; ti < 6; ++ti) {
        const int *tv = tets[ti];
        bool in[4];
        int nin = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            in[i] = f[tv[i]] > 0.0;
            nin += in[i];
        }
        if (nin == 0 || nin == 4) continue;
        if (nin != 2) {
            const bool want = nin == 1;
            int lone = 0;
#pragma unroll
            for (int i = 3; i >= 0; --i)
                if (in[i] == want) lone = i;
            CVtx v[3];
            int m = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (i == lone) continue;
                v[m++] = cv_edge(o, tv[min(lone, i)], tv[max(lone, i)], f);
            }
            best.take(cv_tri2(v[0], v[1], v[2]), cell, 2 * ti);
        } else {
            int I0 = -1, I1 = -1, O0 = -1, O1 = -1;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (in[i]) {
                    if (I0 < 0) I0 = i;
                    else I1 = i;
                } else {
                    if (O0 < 0) O0 = i;
                    else O1 = i;
                }
            }
            const CVtx vac = cv_edge(o, tv[min(I0, O0)], tv[max(I0, O0)], f);
            const CVtx vad = cv_edge(o, tv[min(I0, O1)], tv[max(I0, O1)], f);
            const CVtx vbd = cv_edge(o, tv[min(I1, O1)], tv[max(I1, O1)], f);
            const CVtx vbc = cv_edge(o, tv[min(I1, O0)], tv[max(I1, O0)], f);
            best.take(cv_tri2(vac, vad, vbd), cell, 2 * ti);
            best.take(cv_tri2(vac, vbd, vbc), cell, 2 * ti + 1);
        }
    }
}

// Pair weight w(k, j) (the correction's misorientation weight), FP64 for
// double, else in T.
template <typename T> __device__ inline double pair_w(const Physics<T> &ph, int k, int j) {
    T mob;
    return (double)pair_weight<T>(misorientation_deg<T>(ph.quat + 4LL * k, ph.quat + 4LL * j), ph.theta_c_deg, &mob);
}

// Correction weights of every voxel of the layout L's boxes (one group per
// grain, launch order `order` or grain id): the closest piece's weight inside
// the tube, the ID-field pair outside; written as T into wout (same layout).
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_closest_weight(Boxes L, const T *__restrict__ phi, const int *__restrict__ iota, Physics<T> ph,
                     T *__restrict__ wout, GridArgs g, const int *__restrict__ order, const Ctl *ctl) {
    if (ctl_failed(ctl)) return;
    const int k = order ? order[blockIdx.x] : (int)blockIdx.x;
    if (!L.alive[k]) return;
    const int dim = g.dim;
    const int e[3] = {L.ext[3 * k], L.ext[3 * k + 1], dim == 3 ? L.ext[3 * k + 2] : 1};
    bool ring[3] = {false, false, false};
    int lo_lim[3] = {0, 0, 0}, hi_ring[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) {
        ring[a] = e[a] == g.n[a];
        lo_lim[a] = -(e[a] / 2);
        hi_ring[a] = e[a] - e[a] / 2 - 1;
    }
    const int nc = 1 << dim;
    const T *f = phi + L.off[k];
    const int *io = iota + L.off[k];
    T *w = wout + L.off[k];
    const int plane = e[0] * e[1];
    const int total = plane * e[2];  // a box volume: below 2^31
    int cj = -2;
    double cw = 1.0;
    for (int i = threadIdx.x; i < total; i += kBlock) {
        const int z = i / plane, r = i - z * plane, y = r / e[0], x = r - y * e[0];
        const int xv[3] = {x, y, z};
        const double p = (double)f[i];
        int cell = -1;
        if (fabs(p) < kClosestTube) {
            CBest best{__builtin_inf(), 0x7fffffff, 0x7fffffff};
            // cells with offsets in [-r-1, r] on each axis (clamped to the box,
            // or to the canonical image range on a whole periodic axis);
            // prune: skip cells farther than the best piece
            auto scan = [&](int rr, bool prune) -> bool {
                int ol[3], oh[3];
                bool full = true;
                for (int a = 0; a < 3; ++a) {
                    if (a >= dim) {
                        ol[a] = oh[a] = 0;
                        continue;
                    }
                    const int L0 = ring[a] ? lo_lim[a] : -xv[a];
                    const int H0 = ring[a] ? hi_ring[a] : e[a] - 2 - xv[a];
                    ol[a] = max(-rr - 1, L0);
                    oh[a] = min(rr, H0);
                    full = full && ol[a] == L0 && oh[a] == H0;
                }
                for (int oz = ol[2]; oz <= oh[2]; ++oz)
                    for (int oy = ol[1]; oy <= oh[1]; ++oy)
                        for (int ox = ol[0]; ox <= oh[0]; ++ox) {
                            const int o[3] = {ox, oy, oz};
                            if (prune) {
                                int s = 0;
#pragma unroll
                                for (int a = 0; a < 3; ++a) {
                                    const int d = o[a] > 0 ? o[a] : (o[a] < -1 ? -(o[a] + 1) : 0);
                                    s += d * d;
                                }
                                if ((double)s > best.d2) continue;
                            }
                            int c[3];
#pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                int v = xv[a] + o[a];
                                if (ring[a]) v = v < 0 ? v + e[a] : (v >= e[a] ? v - e[a] : v);
                                c[a] = v;
                            }
                            double fv[8];
                            int pos = 0;
                            for (int b = 0; b < nc; ++b) {
                                int q[3];
#pragma unroll
                                for (int a = 0; a < 3; ++a) {
                                    q[a] = c[a] + ((b >> a) & 1);
                                    if (q[a] >= e[a]) q[a] -= e[a];  // whole periodic axes only
                                }
                                fv[b] = (double)f[q[0] + e[0] * (q[1] + e[1] * q[2])];
                                pos += fv[b] > 0.0;
                            }
                            if (pos == 0 || pos == nc) continue;
                            cell_pieces(dim, o, fv, c[0] + e[0] * (c[1] + e[1] * c[2]), best);
                        }
                return full;
            };
            int rr = 0;
            for (;; ++rr)
                if (scan(rr, false) || best.cell != 0x7fffffff) break;
            if (best.cell != 0x7fffffff) {
                const int r2 = (int)floor(sqrt(best.d2)) + 1;
                if (r2 > rr) scan(r2, true);
                cell = best.cell;
            }
        }
        double wv;
        if (cell >= 0) {
            // the cell's character: distinct ID-field entries at its nodes
            const int c[3] = {cell % e[0], (cell / e[0]) % e[1], cell / plane};
            int js[8], nj = 0;
            for (int b = 0; b < nc; ++b) {
                int q[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    q[a] = c[a] + ((b >> a) & 1);
                    if (q[a] >= e[a]) q[a] -= e[a];
                }
                const int j = io[q[0] + e[0] * (q[1] + e[1] * q[2])];
                if (j < 0) continue;
                bool seen = false;
                for (int t = 0; t < nj; ++t) seen = seen || js[t] == j;
                if (!seen) {
                    int t = nj++;  // insertion in increasing j
                    while (t > 0 && js[t - 1] > j) {
                        js[t] = js[t - 1];
                        --t;
                    }
                    js[t] = j;
                }
            }
            double s = 0.0;
            for (int t = 0; t < nj; ++t) s += pair_w<T>(ph, k, js[t]);
            wv = nj ? s / (double)nj : 1.0;
        } else {
            const int j = io[i];
            if (j != cj) {
                cj = j;
                cw = j >= 0 ? pair_w<T>(ph, k, j) : 1.0;
            }
            wv = cw;
        }
        w[i] = (T)wv;
    }
}

}  // namespace gg
