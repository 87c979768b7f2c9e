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
// (cells whose integer box distance exceeds it are skipped, and cells the
// rings took are not taken again).  On a whole periodic axis a cell is taken at
// the image whose offset lies in [-floor(e/2), ceil(e/2) - 1], and the search
// never leaves that range.  A group queues the tube voxels of its box in LDS,
// in bands of |phi|, and searches them a group's width at a time; a cell's
// node values sit in the thread's LDS column while its simplices are taken in
// a rolled loop.
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

// crossing vertex on the edge between cell corners bu <= bv, node values read
// from the thread's LDS column f (stride kBlock per corner)
__device__ inline CVtx cv_edge_l(const int o[3], int bu, int bv, const double *f) {
    CVtx r;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.u[a] = o[a] + ((bu >> a) & 1);
        r.d[a] = ((bv >> a) & 1) - ((bu >> a) & 1);
    }
    const double fu = f[bu * kBlock], fv = f[bv * kBlock];
    r.t = fu / (fu - fv);
    return r;
}

__device__ inline CVtx cv_pick(bool s, const CVtx &a, const CVtx &b) {
    CVtx r;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        r.u[i] = s ? a.u[i] : b.u[i];
        r.d[i] = s ? a.d[i] : b.d[i];
    }
    r.t = s ? a.t : b.t;
    return r;
}

// Every piece of one cell (lower node at offset o, node values in the
// thread's LDS column f, by corner bits) against the best so far.  Pieces: 2D
// triangle i -> piece i; 3D tetrahedron i -> piece 2i (and 2i + 1 for a
// quadrilateral zero set, cut along the diagonal from its first vertex).  The
// simplices are taken in a rolled loop: tetrahedron i = (0, e_a, e_a + e_b, 7)
// with a = i / 2 and b the smaller (i even) or larger (i odd) other axis.
__device__ inline void cell_pieces(int dim, const int o[3], const double *f, int cell, CBest &best) {
    if (dim == 2) {
#pragma unroll 1
        for (int ti = 0; ti < 2; ++ti) {
            const int tv[3] = {0, ti ? 2 : 1, 3};
            bool in[3];
            int nin = 0;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                in[i] = f[tv[i] * kBlock] > 0.0;
                nin += in[i];
            }
            if (nin == 0 || nin == 3) continue;
            // the lone vertex: inside when one is inside, outside when two are
            const bool want = nin == 1;
            const int lone = in[0] == want ? 0 : (in[1] == want ? 1 : 2);
            const int a = lone == 0 ? 1 : 0, b = lone == 2 ? 1 : 2;  // the other two, increasing
            const CVtx va = cv_edge_l(o, tv[min(lone, a)], tv[max(lone, a)], f);
            const CVtx vb = cv_edge_l(o, tv[min(lone, b)], tv[max(lone, b)], f);
            best.take(cv_seg2(va, vb), cell, ti);
        }
        return;
    }
#pragma unroll 1
    for (int ti = 0; ti < 6; ++ti) {
        const int a1 = ti >> 1;
        const int lo = a1 == 0 ? 1 : 0, hi = a1 == 2 ? 1 : 2;
        const int v1 = 1 << a1, v2 = v1 | (1 << ((ti & 1) ? hi : lo));
        const int tv[4] = {0, v1, v2, 7};
        bool in[4];
        int nin = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            in[i] = f[tv[i] * kBlock] > 0.0;
            nin += in[i];
        }
        if (nin == 0 || nin == 4) continue;
        CVtx V0, V1, V2, V3;
        int ntri;
        if (nin != 2) {
            // one triangle: the edges from the lone vertex to the others, in order
            const bool want = nin == 1;
            const int l = in[0] == want ? 0 : (in[1] == want ? 1 : (in[2] == want ? 2 : 3));
            const int p0 = l == 0 ? 1 : 0, p1 = l <= 1 ? 2 : 1, p2 = l <= 2 ? 3 : 2;
            V0 = cv_edge_l(o, tv[min(l, p0)], tv[max(l, p0)], f);
            V1 = cv_edge_l(o, tv[min(l, p1)], tv[max(l, p1)], f);
            V2 = cv_edge_l(o, tv[min(l, p2)], tv[max(l, p2)], f);
            V3 = V2;
            ntri = 1;
        } else {
            // a quadrilateral: inside corners I0 < I1, outside O0 < O1
            const int I0 = in[0] ? 0 : (in[1] ? 1 : 2);
            const int I1 = in[3] ? 3 : (in[2] ? 2 : 1);
            const int O0 = !in[0] ? 0 : (!in[1] ? 1 : 2);
            const int O1 = !in[3] ? 3 : (!in[2] ? 2 : 1);
            V0 = cv_edge_l(o, tv[min(I0, O0)], tv[max(I0, O0)], f);  // ac
            V1 = cv_edge_l(o, tv[min(I0, O1)], tv[max(I0, O1)], f);  // ad
            V2 = cv_edge_l(o, tv[min(I1, O1)], tv[max(I1, O1)], f);  // bd
            V3 = cv_edge_l(o, tv[min(I1, O0)], tv[max(I1, O0)], f);  // bc
            ntri = 2;
        }
#pragma unroll 1
        for (int t = 0; t < ntri; ++t) {
            // triangles (V0, V1, V2) and (V0, V2, V3)
            const CVtx B = cv_pick(t != 0, V2, V1), C = cv_pick(t != 0, V3, V2);
            best.take(cv_tri2(V0, B, C), cell, 2 * ti + t);
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
    // the node values of the cell being searched, one LDS column per thread
    __shared__ double corners[8 * kBlock];
    double *corner = corners + threadIdx.x;
    int cj = -2;
    double cw = 1.0;
    // ID-field weight of voxel i (outside the tube)
    auto id_weight = [&](int i) -> double {
        const int j = io[i];
        if (j != cj) {
            cj = j;
            cw = j >= 0 ? pair_w<T>(ph, k, j) : 1.0;
        }
        return cw;
    };
    // The closest piece's weight of tube voxel i (the ID-field weight when
    // the box holds no piece).
    auto tube_weight = [&](int i) -> double {
        const int z = i / plane, r = i - z * plane, y = r / e[0], x = r - y * e[0];
        const int xv[3] = {x, y, z};
        CBest best{__builtin_inf(), 0x7fffffff, 0x7fffffff};
        // one region per round: offsets [-rr-1, rr] per axis (clamped to the
        // box, or to the canonical image range on a whole periodic axis)
        // without [-sk-1, sk] (scanned before); once a piece is found, cells
        // farther than the best piece are skipped (their pieces are at least
        // their box distance away).  Rings rr = 0, 1, ... until a piece is
        // found, then one round out to the found distance.
        int rr = 0, sk = -1;
        bool prune = false;
        for (;;) {
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
                        if (sk >= 0 && ox >= -sk - 1 && ox <= sk && oy >= -sk - 1 && oy <= sk && oz >= -sk - 1 &&
                            oz <= sk)
                            continue;
                        const int o[3] = {ox, oy, oz};
                        if (best.cell != 0x7fffffff) {
                            int sq = 0;
#pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                const int d = o[a] > 0 ? o[a] : (o[a] < -1 ? -(o[a] + 1) : 0);
                                sq += d * d;
                            }
                            if ((double)sq > best.d2) continue;
                        }
                        int c[3];
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            int v = xv[a] + o[a];
                            if (ring[a]) v = v < 0 ? v + e[a] : (v >= e[a] ? v - e[a] : v);
                            c[a] = v;
                        }
                        const int ci = c[0] + e[0] * (c[1] + e[1] * c[2]);
                        int pos = 0;
#pragma unroll
                        for (int bb = 0; bb < 8; ++bb) {
                            if (bb >= nc) continue;
                            int q[3];
#pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                q[a] = c[a] + ((bb >> a) & 1);
                                if (q[a] >= e[a]) q[a] -= e[a];  // whole periodic axes only
                            }
                            const double v = (double)f[q[0] + e[0] * (q[1] + e[1] * q[2])];
                            corner[bb * kBlock] = v;
                            pos += v > 0.0;
                        }
                        if (pos == 0 || pos == nc) continue;
                        cell_pieces(dim, o, corner, ci, best);
                    }
            if (!prune && best.cell != 0x7fffffff) {
                const int r2 = (int)floor(sqrt(best.d2)) + 1;
                if (r2 <= rr || full) break;
                prune = true;
                sk = rr;
                rr = r2;
                continue;
            }
            if (prune || full) break;
            sk = rr;
            ++rr;
        }
        if (best.cell == 0x7fffffff) return id_weight(i);
        // the cell's character: distinct ID-field entries at its nodes
        const int cell = best.cell;
        const int c[3] = {cell % e[0], (cell / e[0]) % e[1], cell / plane};
        int js[8], nj = 0;
        for (int bb = 0; bb < nc; ++bb) {
            int q[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                q[a] = c[a] + ((bb >> a) & 1);
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
        double sum = 0.0;
        for (int t = 0; t < nj; ++t) sum += pair_w<T>(ph, k, js[t]);
        return nj ? sum / (double)nj : 1.0;
    };
    // Tube voxels are gathered into queues by |phi| (kQueues bands of the
    // tube) and searched a group's width at a time, so that no lane idles on a
    // voxel outside the tube and the lanes of a wave need searches of about the
    // same extent (the search grows with the distance to the boundary).
#ifndef GG_CLOSEST_QUEUES
#define GG_CLOSEST_QUEUES 4
#endif
    constexpr int kQueues = GG_CLOSEST_QUEUES;
    __shared__ int queue[kQueues][2 * kBlock];
    __shared__ int qn[kQueues];
    if (threadIdx.x < kQueues) qn[threadIdx.x] = 0;
    __syncthreads();
    for (int base = 0; base < total; base += kBlock) {
        const int i = base + (int)threadIdx.x;
        if (i < total) {
            const double a = fabs((double)f[i]);
            if (a < kClosestTube) {
                const int qb = min(kQueues - 1, (int)(a * (kQueues / kClosestTube)));
                queue[qb][atomicAdd(&qn[qb], 1)] = i;
            } else {
                w[i] = (T)id_weight(i);
            }
        }
        __syncthreads();
        const bool last = base + kBlock >= total;
        for (int qb = 0; qb < kQueues; ++qb) {
            int n = qn[qb];
            while (n >= kBlock || (last && n > 0)) {
                const int take = min(n, kBlock);
                if ((int)threadIdx.x < take) {
                    const int v = queue[qb][n - take + threadIdx.x];
                    w[v] = (T)tube_weight(v);
                }
                n -= take;
                __syncthreads();
                if (threadIdx.x == 0) qn[qb] = n;
                __syncthreads();
            }
        }
    }
}

}  // namespace gg
