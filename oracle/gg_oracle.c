/*
 * FP64 CPU oracle of the local level-set grain-growth timestep
 * (Miessen et al., arXiv:1701.06658, section 2.1 "Simulation model").
 *
 * TEST INFRASTRUCTURE ONLY -- see gg_oracle.h.  Plain, grain-major and slow on
 * purpose: every step below follows the method's definition directly, with no
 * tiling, fusion or reordering, so that it can be checked against the paper by
 * eye.  Built with -ffp-contract=off so that each product and sum is rounded
 * separately, in the order written.
 *
 * The step (Algorithm 1 of the paper: predictor, corrector, re-initialization):
 *   1. predictor  (sec. 2.1.4, Eqs. Heatequation/Gaussian/solution):
 *        psi_k = G_sigma * phi_k, separable (passes z, x, y in 3D; x, y in 2D), taps
 *        g_i = exp(-i^2 / (2 sigma^2)) / sum_j exp(-j^2 / (2 sigma^2)), |i| <= R,
 *        R = ceil(4 sigma), sigma = sqrt(2 dt) * n voxels (heat kernel variance
 *        2t per axis); samples outside the box read -W;
 *      optional correction (Eq. eq:velocorrect):
 *        d^p = phi + w (psi - phi) + mob (E_iota - E_k) sigma^2 h / (2 gamma_max),
 *        clamped to [-W, W], with (w, mob) from the misorientation of the pair
 *        (k, iota_k(x)), iota the ID-field of the previous corrector;
 *   2. corrector (sec. 2.1.5): phi^c_k = (psi_k - max_{j != k} psi_j) / 2, the
 *      max over the other alive grains whose box covers the voxel (-W if none);
 *      the ID-field iota_k = that argmax (ties to the lowest id, -1 if none);
 *   3. extinction: grain k dies when no voxel has phi^c_k > 0;
 *   4. box update (sec. 3.1, size-adaptive boxes): new box = bounding box of
 *      {phi^c_k > 0} padded by P = ceil(W); a box longer than n - 2P on an axis
 *      takes the whole periodic axis; phi^c and iota are carried over through
 *      the sampling rule (new cells read -W / -1);
 *   5. re-initialization (sec. 2.1.6, the fast "taxicab" scheme): reference
 *      values at voxels next to a sign change, theta = phi(x)/(phi(x)-phi(n))
 *      over face neighbours n of opposite sign, ref = min theta (the exact L1
 *      distance to a locally planar interface); then the values are spread
 *      through the box one voxel at a time (+1 per voxel, forward and backward
 *      sweeps along x, y, z), which gives the L1 distance min_p ref(p) + |x - p|_1,
 *      and phi = +-min(dist, W) with the sign of phi^c > 0;
 *   6. volume V_k = sum over the box of clamp(phi + 1/2, 0, 1).
 *
 * Sampling rule (periodic grid): global voxel g is covered by box k iff
 * l = (g - lo_k) mod n satisfies l_a < ext_a on every axis; then the value is
 * the stored one at l, otherwise the fill value (-W for level-set values).
 */
#include "gg_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

struct orc_sim {
    int dim;
    int n[3];
    double W;
    int P;
    int G;
    int *alive;
    int *lo;  /* 3*G */
    int *ext; /* 3*G */
    double **phi;
    int **iota;
    double *vol;
    /* predictor correction */
    int mode;
    double *quat;
    double theta_c;
    double *energy;
    double h_phys;
    double gamma_max;
    /* re-initialization scheme of the steps: 0 taxicab spreading, 1 Euclidean */
    int redist;
    /* misorientation weight from the closest boundary point inside the tube
     * |phi| < cp_tube (sec. 3.2); otherwise from the ID-field */
    int closest;
    double cp_tube;
    /* intermediates of the last step */
    int keep;
    int *plo, *pext, *palive;
    double **psi;
    double **phic;
};

/* ------------------------------------------------------------------ helpers */

static int wrapi(long v, int N) {
    long r = v % N;
    if (r < 0) r += N;
    return (int)r;
}

static long nvox(const int *e) { return (long)e[0] * e[1] * e[2]; }

static long lidx(const int *e, int x, int y, int z) {
    return x + (long)e[0] * (y + (long)e[1] * z);
}

/* Value of a box field at local coordinates that may lie outside the box:
 * wrap modulo the grid, then test against the extent. */
static double sample(const double *f, const int *e, const int *n, long x, long y, long z,
                     double fill) {
    int lx = wrapi(x, n[0]), ly = wrapi(y, n[1]), lz = wrapi(z, n[2]);
    if (lx >= e[0] || ly >= e[1] || lz >= e[2]) return fill;
    return f[lidx(e, lx, ly, lz)];
}

static int kernel_radius(double sigma) {
    int R = (int)ceil(4.0 * sigma - 1e-9);
    return R < 1 ? 1 : R;
}

static double *gaussian_taps(double sigma, int R) {
    double *t = (double *)malloc(sizeof(double) * (2 * R + 1));
    double s2 = 2.0 * sigma * sigma, sum = 0.0;
    for (int i = -R; i <= R; i++) {
        t[i + R] = exp(-(double)(i * i) / s2);
        sum = sum + t[i + R];
    }
    for (int i = 0; i < 2 * R + 1; i++) t[i] = t[i] / sum;
    return t;
}

/* One 1D convolution pass along axis a over a box. */
static void conv_axis(const double *in, double *out, const int *e, const int *n, int a,
                      const double *taps, int R, double W) {
    for (int z = 0; z < e[2]; z++)
        for (int y = 0; y < e[1]; y++)
            for (int x = 0; x < e[0]; x++) {
                double acc = 0.0;
                for (int i = -R; i <= R; i++) {
                    long c[3] = {x, y, z};
                    c[a] += i;
                    acc = acc + taps[i + R] * sample(in, e, n, c[0], c[1], c[2], -W);
                }
                out[lidx(e, x, y, z)] = acc;
            }
}

/* Gaussian predictor on one box.  The kernel is a product of 1D kernels, so
 * the passes commute; they are applied z (3D), then x, then y. */
static void predictor_box(int dim, const int *n, double W, const int *e, const double *f,
                          double *out, const double *taps, int R) {
    long m = nvox(e);
    double *t1 = (double *)malloc(sizeof(double) * m);
    if (dim == 2) {
        conv_axis(f, t1, e, n, 0, taps, R, W);
        conv_axis(t1, out, e, n, 1, taps, R, W);
    } else {
        double *t2 = (double *)malloc(sizeof(double) * m);
        conv_axis(f, t1, e, n, 2, taps, R, W);
        conv_axis(t1, t2, e, n, 0, taps, R, W);
        conv_axis(t2, out, e, n, 1, taps, R, W);
        free(t2);
    }
    free(t1);
}

/* One axis of the L1 spreading on a box: along every line the distance grows
 * by one per voxel travelled, carried forward then backward.  A line that spans
 * a whole periodic axis is a ring: each direction goes around it twice, so that
 * paths across the periodic seam are included. */
static void sweep_axis(double *d, const int *e, const int *n, int a) {
    const int len = e[a];
    const long stride = a == 0 ? 1 : (a == 1 ? (long)e[0] : (long)e[0] * e[1]);
    const int o1 = a == 0 ? 1 : 0, o2 = a == 2 ? 1 : 2; /* the two other axes */
    for (int v = 0; v < e[o2]; v++)
        for (int u = 0; u < e[o1]; u++) {
            int c[3] = {0, 0, 0};
            c[o1] = u;
            c[o2] = v;
            double *line = d + lidx(e, c[0], c[1], c[2]);
            if (len == n[a]) {
                for (int t = 1; t < 2 * len; t++) {
                    const int i = t % len, p = (t - 1) % len;
                    const double w = line[p * stride] + 1.0;
                    if (w < line[i * stride]) line[i * stride] = w;
                }
                for (int t = 1; t < 2 * len; t++) {
                    const int i = wrapi((long)len - 1 - t, len), p = (i + 1) % len;
                    const double w = line[p * stride] + 1.0;
                    if (w < line[i * stride]) line[i * stride] = w;
                }
            } else {
                for (int i = 1; i < len; i++) {
                    const double w = line[(i - 1) * stride] + 1.0;
                    if (w < line[i * stride]) line[i * stride] = w;
                }
                for (int i = len - 2; i >= 0; i--) {
                    const double w = line[(i + 1) * stride] + 1.0;
                    if (w < line[i * stride]) line[i * stride] = w;
                }
            }
        }
}

/* Re-initialization on one box (sec. 2.1.6): exact distances at the voxels
 * next to the sign change, then spread along x, y (and z), one voxel per step;
 * the result is min over reference voxels p of ref(p) + |x - p|_1. */
static void redistance_box(int dim, const int *n, double W, const int *e, const double *f,
                           double *out) {
    long m = nvox(e);
    double *ref = (double *)malloc(sizeof(double) * m);
    for (int z = 0; z < e[2]; z++)
        for (int y = 0; y < e[1]; y++)
            for (int x = 0; x < e[0]; x++) {
                double fx = f[lidx(e, x, y, z)];
                int in = fx > 0.0;
                double r = INFINITY;
                for (int a = 0; a < dim; a++)
                    for (int s = -1; s <= 1; s += 2) {
                        long c[3] = {x, y, z};
                        c[a] += s;
                        double fn = sample(f, e, n, c[0], c[1], c[2], -W);
                        if ((fn > 0.0) != in) {
                            double th = fx / (fx - fn);
                            if (th < r) r = th;
                        }
                    }
                ref[lidx(e, x, y, z)] = r;
            }
    for (int a = 0; a < dim; a++) sweep_axis(ref, e, n, a);
    for (long v = 0; v < m; v++) {
        double d = fmin(ref[v], W);
        out[v] = f[v] > 0.0 ? d : -d;
    }
    free(ref);
}

/* ---- Euclidean variant of the re-initialization (fast sweeping with
 * Godunov's upwind update, the scheme the paper cites for its redistancing,
 * taken with Euclidean instead of taxicab distances).
 * Reference cells: cells with a face neighbour of the opposite sign.  Their
 * value is |phi| / |grad phi| with the central-difference gradient (exact for
 * a planar interface whatever the slope of phi), at most the smallest axis
 * intercept phi / (phi - phi_n) (the taxicab reference value).
 * Every other cell starts at +inf and takes K Jacobi sweeps of
 * u <- min(u, g(a_1, .., a_D)), where a_a is the smaller magnitude of its two
 * neighbours along axis a inside the box and g solves
 * sum over the a_j below it of (g - a_j)^2 = 1.  A Godunov value exceeds its
 * smallest neighbour by at least 1/sqrt(D), so a value at most W depends only
 * on cells within sqrt(D) W steps: K = ceil(sqrt(D) W) + 1 sweeps (rounded up
 * to an even count) reach the fixed point on the band. */
static double godunov_update(double a1, double a2, double a3) {
    double t;
    if (a2 < a1) { t = a1; a1 = a2; a2 = t; }
    if (a3 < a2) { t = a2; a2 = a3; a3 = t; }
    if (a2 < a1) { t = a1; a1 = a2; a2 = t; }
    double u = a1 + 1.0;
    if (u > a2) {
        const double d = a1 - a2;
        u = (a1 + a2 + sqrt(2.0 - d * d)) * 0.5;
        if (u > a3) {
            const double s1 = a1 + a2 + a3, s2 = a1 * a1 + a2 * a2 + a3 * a3;
            u = (s1 + sqrt(s1 * s1 - 3.0 * (s2 - 1.0))) / 3.0;
        }
    }
    return u;
}

static int euclid_sweeps(int dim, double W) {
    int K = (int)ceil(sqrt((double)dim) * W) + 1;
    return K + (K & 1);
}

static void redistance_box_euclid(int dim, const int *n, double W, const int *e, const double *f,
                                  double *out) {
    long m = nvox(e);
    double *u = (double *)malloc(sizeof(double) * m);
    double *v = (double *)malloc(sizeof(double) * m);
    unsigned char *fixed = (unsigned char *)malloc(m);
    for (int z = 0; z < e[2]; z++)
        for (int y = 0; y < e[1]; y++)
            for (int x = 0; x < e[0]; x++) {
                const long i = lidx(e, x, y, z);
                const double fx = f[i];
                const int in = fx > 0.0;
                double th = INFINITY, gg = 0.0;
                for (int a = 0; a < dim; a++) {
                    long cm[3] = {x, y, z}, cp[3] = {x, y, z};
                    cm[a] -= 1;
                    cp[a] += 1;
                    const double fm = sample(f, e, n, cm[0], cm[1], cm[2], -W);
                    const double fp = sample(f, e, n, cp[0], cp[1], cp[2], -W);
                    if ((fm > 0.0) != in) {
                        const double t = fx / (fx - fm);
                        if (t < th) th = t;
                    }
                    if ((fp > 0.0) != in) {
                        const double t = fx / (fx - fp);
                        if (t < th) th = t;
                    }
                    const double g = (fp - fm) * 0.5;
                    gg = gg + g * g;
                }
                fixed[i] = th < INFINITY;
                double r = INFINITY;
                if (fixed[i]) {
                    r = gg > 0.0 ? fabs(fx) / sqrt(gg) : INFINITY;
                    if (th < r) r = th;
                }
                u[i] = r;
            }
    const int K = euclid_sweeps(dim, W);
    for (int it = 0; it < K; it++) {
        for (int z = 0; z < e[2]; z++)
            for (int y = 0; y < e[1]; y++)
                for (int x = 0; x < e[0]; x++) {
                    const long i = lidx(e, x, y, z);
                    if (fixed[i]) {
                        v[i] = u[i];
                        continue;
                    }
                    double a[3] = {INFINITY, INFINITY, INFINITY};
                    for (int ax = 0; ax < dim; ax++) {
                        long cm[3] = {x, y, z}, cp[3] = {x, y, z};
                        cm[ax] -= 1;
                        cp[ax] += 1;
                        const double um = sample(u, e, n, cm[0], cm[1], cm[2], INFINITY);
                        const double up = sample(u, e, n, cp[0], cp[1], cp[2], INFINITY);
                        a[ax] = um < up ? um : up;
                    }
                    const double g = godunov_update(a[0], a[1], a[2]);
                    v[i] = g < u[i] ? g : u[i];
                }
        double *t = u;
        u = v;
        v = t;
    }
    for (long i = 0; i < m; i++) {
        const double d = fmin(u[i], W);
        out[i] = f[i] > 0.0 ? d : -d;
    }
    free(u);
    free(v);
    free(fixed);
}

static double volume_box(const double *phi, long m) {
    double v = 0.0;
    for (long i = 0; i < m; i++) {
        double c = phi[i] + 0.5;
        if (c < 0.0) c = 0.0;
        if (c > 1.0) c = 1.0;
        v = v + c;
    }
    return v;
}

/* Covered cyclic interval of an occupancy row: the complement of the largest
 * cyclic run of empty cells (ties to the run with the smallest start).
 * Returns 0 if nothing is occupied; len == N when nothing is empty. */
static int cyclic_cover(const unsigned char *occ, int N, int *start, int *len) {
    int any = 0, full = 1;
    for (int i = 0; i < N; i++) {
        if (occ[i]) any = 1;
        else full = 0;
    }
    if (!any) return 0;
    if (full) {
        *start = 0;
        *len = N;
        return 1;
    }
    int best_s = -1, best_l = -1;
    for (int s = 0; s < N; s++) {
        if (occ[s] || !occ[wrapi(s - 1, N)]) continue; /* a run of empties starts at s */
        int l = 0;
        while (l < N && !occ[wrapi(s + l, N)]) l++;
        if (l > best_l) {
            best_l = l;
            best_s = s;
        }
    }
    *start = wrapi(best_s + best_l, N);
    *len = N - best_l;
    return 1;
}

/* New (lo, ext) along one axis from a covered interval (start, len): pad by P
 * on both sides; a box that would come within 2P of the whole axis takes the
 * whole (periodic) axis instead, so that no stencil of reach <= 2P ever wraps
 * around a partial box. */
static void pad_interval(int start, int len, int P, int N, int *lo, int *ext) {
    long e = (long)len + 2L * P;
    if (e > (long)N - 2L * P) {
        *ext = N;
        *lo = 0;
    } else {
        *ext = (int)e;
        *lo = wrapi((long)start - P, N);
    }
}

static int boxes_overlap(const int *loa, const int *ea, const int *lob, const int *eb,
                         const int *n) {
    for (int a = 0; a < 3; a++) {
        if (!(wrapi((long)lob[a] - loa[a], n[a]) < ea[a] || wrapi((long)loa[a] - lob[a], n[a]) < eb[a]))
            return 0;
    }
    return 1;
}

/* ------------------------------------------------------------- physics (a2) */

double orc_misorientation_deg(const double qa[4], const double qb[4]) {
    /* dq = conj(qa) * qb */
    double aw = qa[0], ax = -qa[1], ay = -qa[2], az = -qa[3];
    double bw = qb[0], bx = qb[1], by = qb[2], bz = qb[3];
    double dw = aw * bw - ax * bx - ay * by - az * bz;
    double dx = aw * bx + ax * bw + ay * bz - az * by;
    double dy = aw * by - ax * bz + ay * bw + az * bx;
    double dz = aw * bz + ax * by - ay * bx + az * bw;
    double best = 4.0;
    /* proper rotations of the hexagonal 622 group: 6-fold about c (z) and six
     * 2-fold axes in the basal plane */
    for (int k = 0; k < 6; k++) {
        double h = 0.5 * (M_PI / 3.0) * k;
        double sw[2] = {cos(h), 0.0}, sx[2] = {0.0, cos(h)}, sy[2] = {0.0, sin(h)},
               sz[2] = {sin(h), 0.0};
        for (int t = 0; t < 2; t++) {
            double w = dw * sw[t] - dx * sx[t] - dy * sy[t] - dz * sz[t];
            double c = fabs(w);
            if (c > 1.0) c = 1.0;
            double ang = 2.0 * acos(c);
            if (ang < best) best = ang;
        }
    }
    return best * 180.0 / M_PI;
}

/* Read-Shockley boundary energy normalised to 1 at and above theta_c. */
static double read_shockley(double theta_deg, double theta_c_deg) {
    if (theta_deg >= theta_c_deg) return 1.0;
    if (theta_deg <= 0.0) return 0.0;
    double r = theta_deg / theta_c_deg;
    return r * (1.0 - log(r));
}

double orc_pair_weight(double theta_deg, double theta_c_deg, double *mobility) {
    double g = read_shockley(theta_deg, theta_c_deg);
    double mu = 1.0 - 0.99 * exp(-5.0 * pow(theta_deg / 15.0, 9.0));
    if (mobility) *mobility = mu;
    return mu * g;
}

/* ---------------------------------------- closest grain-boundary point (a2) */
/*
 * Sec. 2.1.4 lets every grid point of grain k adopt the boundary properties of
 * the closest point of the boundary; sec. 3.2 finds that point on an explicit
 * linear representation of the zero level set (marching squares / cubes), with
 * the pieces clustered by the number of neighbouring grains (ID-field) and the
 * search restricted to a narrow tube.  Reading taken here:
 *  - cells: the 2^D nodes c + {0,1}^D of the box (on an axis the box takes
 *    whole, cells wrap around the periodic grid); each cell is cut along its
 *    main diagonal into simplices -- triangles (0,1,3), (0,2,3) in 2D, the six
 *    tetrahedra (0, e_a, e_a + e_b, 7) in 3D, corner bit 0 = x, 1 = y, 2 = z --
 *    and the zero set of the linear interpolant of phi on a simplex is a
 *    segment (2D) or one or two triangles (3D);
 *  - a crossing vertex on the simplex edge from node u to node v (u <= v
 *    componentwise) lies at u + t (v - u), t = phi_u / (phi_u - phi_v), in
 *    coordinates relative to the voxel x (exact integers plus t);
 *  - the piece's character: the distinct ID-field entries j >= 0 at the cell's
 *    nodes (one: the boundary with grain j; more: a triple or higher junction);
 *    its weight is the mean of w(k, j) over them, 1 with none;
 *  - every voxel with |phi(x)| < tube takes the weight of the piece of smallest
 *    squared Euclidean distance, ties to the lowest cell (linear index of its
 *    lower node) and then the lowest piece; other voxels keep the ID-field.
 * The distances follow one fixed sequence of operations (segment: endpoints in
 * the order of their node keys, clamped projection; triangle: projection when
 * it falls inside, else the nearest edge), so that a voxel equally far from
 * two pieces that share a vertex or an edge sees the same value from both.
 */
static int valid_grid(int dim, const int32_t n[3]);

typedef struct {
    int u[3];  /* node u relative to the voxel */
    int d[3];  /* v - u, 0 or 1 per axis */
    double t;
} cp_vtx;

static void cp_pos(const cp_vtx *a, double p[3]) {
    for (int i = 0; i < 3; i++) p[i] = (double)a->u[i] + a->t * (double)a->d[i];
}

/* node key order: (u_z, u_y, u_x, v_z, v_y, v_x) */
static int cp_less(const cp_vtx *a, const cp_vtx *b) {
    int ka[6] = {a->u[2], a->u[1], a->u[0], a->u[2] + a->d[2], a->u[1] + a->d[1], a->u[0] + a->d[0]};
    int kb[6] = {b->u[2], b->u[1], b->u[0], b->u[2] + b->d[2], b->u[1] + b->d[1], b->u[0] + b->d[0]};
    for (int i = 0; i < 6; i++)
        if (ka[i] != kb[i]) return ka[i] < kb[i];
    return 0;
}

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* squared distance from the voxel (the origin) to the segment PQ */
static double cp_seg2(const cp_vtx *P, const cp_vtx *Q) {
    if (cp_less(Q, P)) {
        const cp_vtx *t = P;
        P = Q;
        Q = t;
    }
    double p[3], q[3], d[3], c[3];
    cp_pos(P, p);
    cp_pos(Q, q);
    for (int i = 0; i < 3; i++) d[i] = q[i] - p[i];
    double dd = dot3(d, d), s = 0.0;
    if (dd > 0.0) {
        s = -dot3(p, d) / dd;
        if (s < 0.0) s = 0.0;
        if (s > 1.0) s = 1.0;
    }
    for (int i = 0; i < 3; i++) c[i] = p[i] + s * d[i];
    return dot3(c, c);
}

/* squared distance from the origin to the triangle ABC */
static double cp_tri2(const cp_vtx *A, const cp_vtx *B, const cp_vtx *C) {
    double a[3], b[3], c[3], ab[3], ac[3], bc[3], ca[3], n[3];
    cp_pos(A, a);
    cp_pos(B, b);
    cp_pos(C, c);
    for (int i = 0; i < 3; i++) {
        ab[i] = b[i] - a[i];
        ac[i] = c[i] - a[i];
        bc[i] = c[i] - b[i];
        ca[i] = a[i] - c[i];
    }
    cross3(ab, ac, n);
    double nn = dot3(n, n);
    if (nn > 0.0) {
        double ma[3] = {-a[0], -a[1], -a[2]}, mb[3] = {-b[0], -b[1], -b[2]}, mc[3] = {-c[0], -c[1], -c[2]};
        double e0[3], e1[3], e2[3];
        cross3(ab, ma, e0);
        cross3(bc, mb, e1);
        cross3(ca, mc, e2);
        if (dot3(n, e0) >= 0.0 && dot3(n, e1) >= 0.0 && dot3(n, e2) >= 0.0) {
            double h = dot3(n, ma);
            return h * h / nn;
        }
    }
    double m = cp_seg2(A, B), m1 = cp_seg2(B, C), m2 = cp_seg2(C, A);
    if (m1 < m) m = m1;
    if (m2 < m) m = m2;
    return m;
}

static const int cp_tets[6][4] = {{0, 1, 3, 7}, {0, 1, 5, 7}, {0, 2, 3, 7}, {0, 2, 6, 7}, {0, 4, 5, 7}, {0, 4, 6, 7}};
static const int cp_tris[2][3] = {{0, 1, 3}, {0, 2, 3}};

/* crossing vertex on the edge between simplex corners bu <= bv (corner bits) */
static void cp_edge(const int o[3], int bu, int bv, const double *f, cp_vtx *out) {
    for (int a = 0; a < 3; a++) {
        out->u[a] = o[a] + ((bu >> a) & 1);
        out->d[a] = ((bv >> a) & 1) - ((bu >> a) & 1);
    }
    out->t = f[bu] / (f[bu] - f[bv]);
}

/* Every piece of one cell (lower node at offset o from the voxel, node values
 * f by corner bits): squared distances into d2[piece], -1 where the piece does
 * not exist.  Pieces: 2D triangle i -> piece i; 3D tetrahedron i -> pieces
 * 2i (and 2i + 1 when the zero set is a quadrilateral). */
static void cp_cell(int dim, const int o[3], const double *f, double d2[12]) {
    for (int i = 0; i < 12; i++) d2[i] = -1.0;
    if (dim == 2) {
        for (int ti = 0; ti < 2; ti++) {
            const int *tv = cp_tris[ti];
            int nin = 0, in[3];
            for (int i = 0; i < 3; i++) {
                in[i] = f[tv[i]] > 0.0;
                nin += in[i];
            }
            if (nin == 0 || nin == 3) continue;
            int lone = -1;
            for (int i = 0; i < 3; i++)
                if (in[i] == (nin == 1)) lone = i;
            cp_vtx v[2];
            int m = 0;
            for (int i = 0; i < 3; i++) {
                if (i == lone) continue;
                int lo = lone < i ? lone : i, hi = lone < i ? i : lone;
                cp_edge(o, tv[lo], tv[hi], f, &v[m++]);
            }
            d2[ti] = cp_seg2(&v[0], &v[1]);
        }
        return;
    }
    for (int ti = 0; ti < 6; ti++) {
        const int *tv = cp_tets[ti];
        int nin = 0, in[4];
        for (int i = 0; i < 4; i++) {
            in[i] = f[tv[i]] > 0.0;
            nin += in[i];
        }
        if (nin == 0 || nin == 4) continue;
        if (nin == 1 || nin == 3) {
            int lone = -1;
            for (int i = 0; i < 4; i++)
                if (in[i] == (nin == 1)) lone = i;
            cp_vtx v[3];
            int m = 0;
            for (int i = 0; i < 4; i++) {
                if (i == lone) continue;
                int lo = lone < i ? lone : i, hi = lone < i ? i : lone;
                cp_edge(o, tv[lo], tv[hi], f, &v[m++]);
            }
            d2[2 * ti] = cp_tri2(&v[0], &v[1], &v[2]);
        } else {
            int I[2], O[2], ni = 0, no = 0;
            for (int i = 0; i < 4; i++) {
                if (in[i]) I[ni++] = i;
                else O[no++] = i;
            }
            /* edge (i, j) with i < j in simplex order */
#define CP_E(i, j, out) cp_edge(o, tv[(i) < (j) ? (i) : (j)], tv[(i) < (j) ? (j) : (i)], f, out)
            cp_vtx vac, vad, vbd, vbc;
            CP_E(I[0], O[0], &vac);
            CP_E(I[0], O[1], &vad);
            CP_E(I[1], O[1], &vbd);
            CP_E(I[1], O[0], &vbc);
#undef CP_E
            d2[2 * ti] = cp_tri2(&vac, &vad, &vbd);
            d2[2 * ti + 1] = cp_tri2(&vac, &vbd, &vbc);
        }
    }
}

/* offset of cell coordinate c from voxel coordinate x on an axis of extent e
 * (whole periodic axis when ring: the image in [-floor(e/2), ceil(e/2) - 1]) */
static int cp_offset(int c, int x, int e, int ring) {
    int o = c - x;
    if (ring) {
        if (o < -(e / 2)) o += e;
        else if (o >= e - e / 2) o -= e;
    }
    return o;
}

/* The closest piece of every box voxel with |phi| < tube, by brute force over
 * all cells of the box: d2 (-1 outside the tube or when the box has no
 * piece), cell (linear index of the lower node), piece. */
static void closest_pieces(int dim, const int *n, const int *e, const double *phi, double tube, double *d2o,
                           long *cello, int *pieceo) {
    int ring[3] = {0, 0, 0}, ce[3] = {1, 1, 1};
    for (int a = 0; a < dim; a++) {
        ring[a] = e[a] == n[a];
        ce[a] = ring[a] ? e[a] : e[a] - 1;  /* cells per axis */
    }
    const int nc = 1 << dim;
    long m = nvox(e);
    for (long v = 0; v < m; v++) {
        d2o[v] = -1.0;
        cello[v] = -1;
        pieceo[v] = -1;
    }
    if (ce[0] < 1 || ce[1] < 1 || ce[2] < 1) return;
    /* the cells the zero set crosses, in increasing linear index, with their node values */
    long ncell = (long)ce[0] * ce[1] * ce[2], nx = 0;
    int *xc = (int *)malloc(sizeof(int) * 3 * ncell);
    double *xf = (double *)malloc(sizeof(double) * 8 * ncell);
    for (int cz = 0; cz < ce[2]; cz++)
        for (int cy = 0; cy < ce[1]; cy++)
            for (int cx = 0; cx < ce[0]; cx++) {
                int c[3] = {cx, cy, cz}, pos = 0, neg = 0;
                double *f = xf + 8 * nx;
                for (int b = 0; b < nc; b++) {
                    int g[3];
                    for (int a = 0; a < 3; a++) {
                        g[a] = c[a] + ((b >> a) & 1);
                        if (g[a] >= e[a]) g[a] -= e[a]; /* ring axes only */
                    }
                    f[b] = phi[lidx(e, g[0], g[1], g[2])];
                    if (f[b] > 0.0) pos++;
                    else neg++;
                }
                if (!pos || !neg) continue;
                for (int a = 0; a < 3; a++) xc[3 * nx + a] = c[a];
                nx++;
            }
#pragma omp parallel for schedule(dynamic)
    for (int z = 0; z < e[2]; z++)
        for (int y = 0; y < e[1]; y++)
            for (int x = 0; x < e[0]; x++) {
                long v = lidx(e, x, y, z);
                if (!(fabs(phi[v]) < tube)) continue;
                int xv[3] = {x, y, z};
                double best = -1.0;
                long bc = -1;
                int bp = -1;
                for (long i = 0; i < nx; i++) { /* cells and pieces in increasing order: the first wins ties */
                    const int *c = xc + 3 * i;
                    int o[3] = {0, 0, 0};
                    for (int a = 0; a < dim; a++) o[a] = cp_offset(c[a], xv[a], e[a], ring[a]);
                    double d2[12];
                    cp_cell(dim, o, xf + 8 * i, d2);
                    for (int pc = 0; pc < 12; pc++) {
                        if (d2[pc] < 0.0) continue;
                        if (best < 0.0 || d2[pc] < best) {
                            best = d2[pc];
                            bc = lidx(e, c[0], c[1], c[2]);
                            bp = pc;
                        }
                    }
                }
                d2o[v] = best;
                cello[v] = bc;
                pieceo[v] = bp;
            }
    free(xc);
    free(xf);
}

/* weight of a piece of grain k in the cell with lower node `cell` (linear
 * box index): mean of w(k, j) over the distinct ID-field entries j >= 0 at
 * the cell's nodes, in increasing j; 1 with none */
static double cell_weight(const orc_sim *s, int k, const int *e, long cell) {
    int dim = s->dim, nc = 1 << dim;
    int c[3] = {(int)(cell % e[0]), (int)((cell / e[0]) % e[1]), (int)(cell / ((long)e[0] * e[1]))};
    int js[8], nj = 0;
    for (int b = 0; b < nc; b++) {
        int g[3];
        for (int a = 0; a < 3; a++) {
            g[a] = c[a] + ((b >> a) & 1);
            if (g[a] >= e[a]) g[a] -= e[a];
        }
        int j = s->iota[k][lidx(e, g[0], g[1], g[2])];
        if (j < 0) continue;
        int seen = 0;
        for (int i = 0; i < nj; i++) seen |= js[i] == j;
        if (!seen) js[nj++] = j;
    }
    if (!nj) return 1.0;
    for (int i = 1; i < nj; i++) /* increasing j */
        for (int q = i; q > 0 && js[q - 1] > js[q]; q--) {
            int t = js[q];
            js[q] = js[q - 1];
            js[q - 1] = t;
        }
    double sum = 0.0;
    for (int i = 0; i < nj; i++)
        sum += orc_pair_weight(orc_misorientation_deg(&s->quat[4 * k], &s->quat[4 * js[i]]), s->theta_c, NULL);
    return sum / (double)nj;
}

/* The correction weight of every voxel of grain k's box for the next step:
 * the closest piece's weight inside the tube, the pair (k, iota) outside
 * (1 where iota < 0); out[v] also on extinct-free boxes only. */
static void closest_weight_map(const orc_sim *s, int k, double *w) {
    const int *e = &s->ext[3 * k];
    long m = nvox(e);
    double *d2 = (double *)malloc(sizeof(double) * m);
    long *cell = (long *)malloc(sizeof(long) * m);
    int *piece = (int *)malloc(sizeof(int) * m);
    closest_pieces(s->dim, s->n, e, s->phi[k], s->cp_tube, d2, cell, piece);
    for (long v = 0; v < m; v++) {
        if (d2[v] >= 0.0) {
            w[v] = cell_weight(s, k, e, cell[v]);
        } else {
            int j = s->iota[k][v];
            w[v] = j >= 0 ? orc_pair_weight(orc_misorientation_deg(&s->quat[4 * k], &s->quat[4 * j]), s->theta_c, NULL)
                          : 1.0;
        }
    }
    free(d2);
    free(cell);
    free(piece);
}

int orc_set_closest_point(orc_sim *s, int on, double tube) {
    if (!s || (on && !(tube > 0.0))) return -1;
    s->closest = on != 0;
    s->cp_tube = tube;
    return 0;
}

int orc_closest_weights(const orc_sim *s, int k, double *out, int64_t cap) {
    if (!s || k < 0 || k >= s->G || !out || !(s->mode & 1)) return -1;
    if (!s->alive[k]) return 0;
    if (nvox(&s->ext[3 * k]) > cap) return -1;
    closest_weight_map(s, k, out);
    return 1;
}

int orc_closest_box(int dim, const int32_t n[3], const int32_t ext[3], const double *phi, double tube,
                    double *d2, int64_t *cell, int32_t *piece) {
    if (!valid_grid(dim, n) || !phi || !d2 || !cell || !piece) return -1;
    int nn[3] = {n[0], n[1], n[2]}, e[3] = {ext[0], ext[1], ext[2]};
    for (int a = 0; a < 3; a++)
        if (e[a] < 1 || e[a] > nn[a]) return -1;
    long m = nvox(e);
    long *c = (long *)malloc(sizeof(long) * m);
    int *p = (int *)malloc(sizeof(int) * m);
    closest_pieces(dim, nn, e, phi, tube, d2, c, p);
    for (long v = 0; v < m; v++) {
        cell[v] = c[v];
        piece[v] = p[v];
    }
    free(c);
    free(p);
    return 0;
}

/* --------------------------------------------------------------- lifecycle */

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

void orc_keep_intermediates(orc_sim *s, int on) {
    if (s) s->keep = on;
}

static void free_intermediates(orc_sim *s) {
    if (s->psi)
        for (int k = 0; k < s->G; k++) {
            free(s->psi[k]);
            s->psi[k] = NULL;
        }
    if (s->phic)
        for (int k = 0; k < s->G; k++) {
            free(s->phic[k]);
            s->phic[k] = NULL;
        }
}

void orc_destroy(orc_sim *s) {
    if (!s) return;
    for (int k = 0; k < s->G; k++) {
        free(s->phi[k]);
        free(s->iota[k]);
    }
    free_intermediates(s);
    free(s->psi);
    free(s->phic);
    free(s->phi);
    free(s->iota);
    free(s->alive);
    free(s->lo);
    free(s->ext);
    free(s->vol);
    free(s->quat);
    free(s->energy);
    free(s->plo);
    free(s->pext);
    free(s->palive);
    free(s);
}

static int valid_grid(int dim, const int32_t n[3]) {
    if (dim != 2 && dim != 3) return 0;
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) return 0;
    if (dim == 2 && n[2] != 1) return 0;
    return 1;
}

/* Corrector argmax on the current phi (no halving): the initial ID-field. */
static void initial_iota(orc_sim *s);

orc_sim *orc_create(int dim, const int32_t n[3], double band, const int32_t *labels, int32_t G) {
    if (!valid_grid(dim, n) || !labels || G < 1 || !(band >= 1.0) || !isfinite(band)) return NULL;
    long nt = (long)n[0] * n[1] * n[2];
    for (long i = 0; i < nt; i++)
        if (labels[i] < 0 || labels[i] >= G) return NULL;
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    s->dim = dim;
    memcpy(s->n, n, sizeof(int) * 3);
    s->W = band;
    s->P = (int)ceil(band);
    s->G = G;
    s->alive = (int *)calloc(G, sizeof(int));
    s->lo = (int *)calloc(3L * G, sizeof(int));
    s->ext = (int *)calloc(3L * G, sizeof(int));
    s->phi = (double **)calloc(G, sizeof(double *));
    s->iota = (int **)calloc(G, sizeof(int *));
    s->vol = (double *)calloc(G, sizeof(double));
    s->psi = (double **)calloc(G, sizeof(double *));
    s->phic = (double **)calloc(G, sizeof(double *));
    s->plo = (int *)calloc(3L * G, sizeof(int));
    s->pext = (int *)calloc(3L * G, sizeof(int));
    s->palive = (int *)calloc(G, sizeof(int));

    /* initial boxes: per axis, the covered cyclic interval of the grain's
     * projection, padded by P */
    long ntot_axis = (long)n[0] + n[1] + n[2];
    unsigned char *occ = (unsigned char *)calloc((size_t)G * ntot_axis, 1);
    for (int z = 0; z < n[2]; z++)
        for (int y = 0; y < n[1]; y++)
            for (int x = 0; x < n[0]; x++) {
                int k = labels[x + (long)n[0] * (y + (long)n[1] * z)];
                unsigned char *o = occ + (size_t)k * ntot_axis;
                o[x] = 1;
                o[n[0] + y] = 1;
                o[n[0] + n[1] + z] = 1;
            }
    for (int k = 0; k < G; k++) {
        unsigned char *o = occ + (size_t)k * ntot_axis;
        int ok = 1, off = 0;
        for (int a = 0; a < 3; a++) {
            int st = 0, ln = 0;
            if (!cyclic_cover(o + off, n[a], &st, &ln)) {
                ok = 0;
                break;
            }
            pad_interval(st, ln, s->P, n[a], &s->lo[3 * k + a], &s->ext[3 * k + a]);
            off += n[a];
        }
        s->alive[k] = ok;
    }
    free(occ);

    /* initial phi: +1/2 on the grain's voxels, -1/2 elsewhere, redistanced */
#pragma omp parallel for schedule(dynamic)
    for (int k = 0; k < G; k++) {
        if (!s->alive[k]) continue;
        const int *lo = &s->lo[3 * k], *e = &s->ext[3 * k];
        long m = nvox(e);
        double *f0 = (double *)malloc(sizeof(double) * m);
        for (int z = 0; z < e[2]; z++)
            for (int y = 0; y < e[1]; y++)
                for (int x = 0; x < e[0]; x++) {
                    int gx = wrapi((long)lo[0] + x, n[0]), gy = wrapi((long)lo[1] + y, n[1]),
                        gz = wrapi((long)lo[2] + z, n[2]);
                    int lab = labels[gx + (long)n[0] * (gy + (long)n[1] * gz)];
                    f0[lidx(e, x, y, z)] = lab == k ? 0.5 : -0.5;
                }
        s->phi[k] = (double *)malloc(sizeof(double) * m);
        redistance_box(dim, s->n, s->W, e, f0, s->phi[k]);
        free(f0);
        s->iota[k] = (int *)malloc(sizeof(int) * m);
        for (long v = 0; v < m; v++) s->iota[k][v] = -1;
        s->vol[k] = volume_box(s->phi[k], m);
    }
    return s;
}

/* ----------------------------------------------------------------- corrector */

/* For each alive grain, the alive grains whose boxes overlap its box. */
static int **candidate_lists(const orc_sim *s, int *counts) {
    int G = s->G;
    int **lists = (int **)calloc(G, sizeof(int *));
#pragma omp parallel for schedule(dynamic, 16)
    for (int k = 0; k < G; k++) {
        counts[k] = 0;
        if (!s->alive[k]) continue;
        int cap = 16, c = 0;
        int *l = (int *)malloc(sizeof(int) * cap);
        for (int j = 0; j < G; j++) {
            if (j == k || !s->alive[j]) continue;
            if (!boxes_overlap(&s->lo[3 * k], &s->ext[3 * k], &s->lo[3 * j], &s->ext[3 * j], s->n))
                continue;
            if (c == cap) {
                cap *= 2;
                l = (int *)realloc(l, sizeof(int) * cap);
            }
            l[c++] = j; /* ascending id order */
        }
        lists[k] = l;
        counts[k] = c;
    }
    return lists;
}

/* max over the other covering grains of field[j] at global voxel g, with its
 * argmax (ties to the lowest id); returns 0 (and leaves m, id) if none covers */
static int max_other(const orc_sim *s, double *const *field, const int *cand, int nc,
                     const int g[3], double *m, int *id) {
    int have = 0;
    for (int c = 0; c < nc; c++) {
        int j = cand[c];
        const int *lo = &s->lo[3 * j], *e = &s->ext[3 * j];
        int lx = wrapi((long)g[0] - lo[0], s->n[0]);
        int ly = wrapi((long)g[1] - lo[1], s->n[1]);
        int lz = wrapi((long)g[2] - lo[2], s->n[2]);
        if (lx >= e[0] || ly >= e[1] || lz >= e[2]) continue;
        double v = field[j][lidx(e, lx, ly, lz)];
        if (!have || v > *m) {
            *m = v;
            *id = j;
            have = 1;
        }
    }
    return have;
}

static void initial_iota(orc_sim *s) {
    int *counts = (int *)calloc(s->G, sizeof(int));
    int **cand = candidate_lists(s, counts);
#pragma omp parallel for schedule(dynamic)
    for (int k = 0; k < s->G; k++) {
        if (!s->alive[k]) continue;
        const int *lo = &s->lo[3 * k], *e = &s->ext[3 * k];
        for (int z = 0; z < e[2]; z++)
            for (int y = 0; y < e[1]; y++)
                for (int x = 0; x < e[0]; x++) {
                    int g[3] = {wrapi((long)lo[0] + x, s->n[0]), wrapi((long)lo[1] + y, s->n[1]),
                                wrapi((long)lo[2] + z, s->n[2])};
                    double m = 0.0;
                    int id = -1;
                    max_other(s, s->phi, cand[k], counts[k], g, &m, &id);
                    s->iota[k][lidx(e, x, y, z)] = id;
                }
    }
    for (int k = 0; k < s->G; k++) free(cand[k]);
    free(cand);
    free(counts);
}

int orc_set_physics(orc_sim *s, int mode, const double *quat, double theta_c_deg,
                    const double *energy, double h_phys, double gamma_max) {
    if (!s || mode < 0 || mode > 3) return -1;
    if ((mode & 1) && (!quat || !(theta_c_deg > 0.0))) return -1;
    if ((mode & 2) && (!energy || !(h_phys > 0.0) || !(gamma_max > 0.0))) return -1;
    s->mode = mode;
    free(s->quat);
    free(s->energy);
    s->quat = NULL;
    s->energy = NULL;
    if (mode & 1) {
        s->quat = (double *)malloc(sizeof(double) * 4 * s->G);
        memcpy(s->quat, quat, sizeof(double) * 4 * s->G);
        s->theta_c = theta_c_deg;
    }
    if (mode & 2) {
        s->energy = (double *)malloc(sizeof(double) * s->G);
        memcpy(s->energy, energy, sizeof(double) * s->G);
        s->h_phys = h_phys;
        s->gamma_max = gamma_max;
    }
    if (mode) initial_iota(s);
    return 0;
}

/* ---------------------------------------------------------------------- step */

int orc_step(orc_sim *s, double dt) {
    if (!s || !(dt > 0.0) || !isfinite(dt)) return -1;
    const int G = s->G, dim = s->dim;
    const int *n = s->n;
    const double W = s->W;
    double sigma = sqrt(2.0 * dt) * (double)n[0];
    int R = kernel_radius(sigma);
    double *taps = gaussian_taps(sigma, R);
    double bulk_scale = (s->mode & 2) ? sigma * sigma * s->h_phys / (2.0 * s->gamma_max) : 0.0;
    free_intermediates(s);
    double **psi = s->psi, **phic = s->phic;
    int **niota = (int **)calloc(G, sizeof(int *));

    /* 1. predictor (+ correction) */
#pragma omp parallel for schedule(dynamic)
    for (int k = 0; k < G; k++) {
        if (!s->alive[k]) continue;
        const int *e = &s->ext[3 * k];
        long m = nvox(e);
        psi[k] = (double *)malloc(sizeof(double) * m);
        predictor_box(dim, n, W, e, s->phi[k], psi[k], taps, R);
        if (s->mode) {
            double *wcp = NULL;
            if (s->closest && (s->mode & 1)) {
                wcp = (double *)malloc(sizeof(double) * m);
                closest_weight_map(s, k, wcp);
            }
            for (long v = 0; v < m; v++) {
                int j = s->iota[k][v];
                double w = 1.0, mob = 1.0, b = 0.0;
                if (j >= 0) {
                    if (s->mode & 1) {
                        double th = orc_misorientation_deg(&s->quat[4 * k], &s->quat[4 * j]);
                        w = orc_pair_weight(th, s->theta_c, &mob);
                    }
                    if (s->mode & 2) b = mob * (s->energy[j] - s->energy[k]) * bulk_scale;
                }
                if (wcp) w = wcp[v]; /* closest boundary point: the weight only */
                double p = s->phi[k][v];
                double d = p + w * (psi[k][v] - p) + b;
                if (d > W) d = W;
                if (d < -W) d = -W;
                psi[k][v] = d;
            }
            free(wcp);
        }
    }

    /* 2. corrector */
    int *counts = (int *)calloc(G, sizeof(int));
    int **cand = candidate_lists(s, counts);
#pragma omp parallel for schedule(dynamic)
    for (int k = 0; k < G; k++) {
        if (!s->alive[k]) continue;
        const int *lo = &s->lo[3 * k], *e = &s->ext[3 * k];
        long m = nvox(e);
        phic[k] = (double *)malloc(sizeof(double) * m);
        niota[k] = (int *)malloc(sizeof(int) * m);
        for (int z = 0; z < e[2]; z++)
            for (int y = 0; y < e[1]; y++)
                for (int x = 0; x < e[0]; x++) {
                    int g[3] = {wrapi((long)lo[0] + x, n[0]), wrapi((long)lo[1] + y, n[1]),
                                wrapi((long)lo[2] + z, n[2])};
                    double mx = 0.0;
                    int id = -1;
                    if (!max_other(s, psi, cand[k], counts[k], g, &mx, &id)) mx = -W;
                    long v = lidx(e, x, y, z);
                    phic[k][v] = 0.5 * (psi[k][v] - mx);
                    niota[k][v] = id;
                }
    }
    for (int k = 0; k < G; k++) free(cand[k]);
    free(cand);
    free(counts);

    memcpy(s->plo, s->lo, sizeof(int) * 3 * G);
    memcpy(s->pext, s->ext, sizeof(int) * 3 * G);
    memcpy(s->palive, s->alive, sizeof(int) * G);

    /* 3.-6. extinction, box update, re-initialization, volume */
#pragma omp parallel for schedule(dynamic)
    for (int k = 0; k < G; k++) {
        if (!s->alive[k]) continue;
        int *lo = &s->lo[3 * k], *e = &s->ext[3 * k];
        int olo[3] = {lo[0], lo[1], lo[2]}, oe[3] = {e[0], e[1], e[2]};
        /* bounding box of the positive set (cyclic rule on full-grid axes) */
        int mn[3] = {1 << 30, 1 << 30, 1 << 30}, mx[3] = {-1, -1, -1};
        unsigned char *occ[3] = {NULL, NULL, NULL};
        for (int a = 0; a < 3; a++)
            if (oe[a] == n[a]) occ[a] = (unsigned char *)calloc(n[a], 1);
        int any = 0;
        for (int z = 0; z < oe[2]; z++)
            for (int y = 0; y < oe[1]; y++)
                for (int x = 0; x < oe[0]; x++) {
                    if (!(phic[k][lidx(oe, x, y, z)] > 0.0)) continue;
                    int c[3] = {x, y, z};
                    any = 1;
                    for (int a = 0; a < 3; a++) {
                        if (c[a] < mn[a]) mn[a] = c[a];
                        if (c[a] > mx[a]) mx[a] = c[a];
                        if (occ[a]) occ[a][c[a]] = 1;
                    }
                }
        if (!any) {
            s->alive[k] = 0;
            s->vol[k] = 0.0;
            free(s->phi[k]);
            free(s->iota[k]);
            s->phi[k] = NULL;
            s->iota[k] = NULL;
            for (int a = 0; a < 3; a++) free(occ[a]);
            continue;
        }
        int nlo[3], ne[3];
        for (int a = 0; a < 3; a++) {
            int st = 0, ln = 0;
            if (occ[a]) {
                cyclic_cover(occ[a], n[a], &st, &ln);
                st = wrapi((long)olo[a] + st, n[a]);
                free(occ[a]);
            } else {
                st = wrapi((long)olo[a] + mn[a], n[a]);
                ln = mx[a] - mn[a] + 1;
            }
            pad_interval(st, ln, s->P, n[a], &nlo[a], &ne[a]);
        }
        /* carry phi^c and iota over to the new box through the sampling rule */
        long m = nvox(ne);
        double *f = (double *)malloc(sizeof(double) * m);
        int *io = (int *)malloc(sizeof(int) * m);
        for (int z = 0; z < ne[2]; z++)
            for (int y = 0; y < ne[1]; y++)
                for (int x = 0; x < ne[0]; x++) {
                    long g0 = (long)nlo[0] + x, g1 = (long)nlo[1] + y, g2 = (long)nlo[2] + z;
                    int ox = wrapi(g0 - olo[0], n[0]), oy = wrapi(g1 - olo[1], n[1]),
                        oz = wrapi(g2 - olo[2], n[2]);
                    long v = lidx(ne, x, y, z);
                    if (ox < oe[0] && oy < oe[1] && oz < oe[2]) {
                        f[v] = phic[k][lidx(oe, ox, oy, oz)];
                        io[v] = niota[k][lidx(oe, ox, oy, oz)];
                    } else {
                        f[v] = -W;
                        io[v] = -1;
                    }
                }
        free(s->phi[k]);
        free(s->iota[k]);
        s->phi[k] = (double *)malloc(sizeof(double) * m);
        if (s->redist == 1)
            redistance_box_euclid(dim, n, W, ne, f, s->phi[k]);
        else
            redistance_box(dim, n, W, ne, f, s->phi[k]);
        s->iota[k] = io;
        memcpy(lo, nlo, sizeof(nlo));
        memcpy(e, ne, sizeof(ne));
        s->vol[k] = volume_box(s->phi[k], m);
        free(f);
    }
    for (int k = 0; k < G; k++) free(niota[k]);
    free(niota);
    if (!s->keep) free_intermediates(s);
    free(taps);
    return 0;
}

/* ------------------------------------------------------------------- queries */

int orc_grain_count(const orc_sim *s) { return s ? s->G : -1; }

int orc_alive_count(const orc_sim *s) {
    if (!s) return -1;
    int c = 0;
    for (int k = 0; k < s->G; k++) c += s->alive[k] != 0;
    return c;
}

int orc_get_box(const orc_sim *s, int k, int32_t lo[3], int32_t ext[3]) {
    if (!s || k < 0 || k >= s->G) return -1;
    for (int a = 0; a < 3; a++) {
        lo[a] = s->lo[3 * k + a];
        ext[a] = s->ext[3 * k + a];
    }
    return s->alive[k] ? 1 : 0;
}

int orc_get_prev_box(const orc_sim *s, int k, int32_t lo[3], int32_t ext[3]) {
    if (!s || k < 0 || k >= s->G) return -1;
    for (int a = 0; a < 3; a++) {
        lo[a] = s->plo[3 * k + a];
        ext[a] = s->pext[3 * k + a];
    }
    return s->palive[k] ? 1 : 0;
}

static int copy_field(const double *src, const int *e, double *out, int64_t cap) {
    if (!src) return -1;
    long m = nvox(e);
    if (cap < m) return -1;
    memcpy(out, src, sizeof(double) * m);
    return 0;
}

int orc_get_phi(const orc_sim *s, int k, double *out, int64_t cap) {
    if (!s || k < 0 || k >= s->G || !s->alive[k]) return -1;
    return copy_field(s->phi[k], &s->ext[3 * k], out, cap);
}

int orc_get_iota(const orc_sim *s, int k, int32_t *out, int64_t cap) {
    if (!s || k < 0 || k >= s->G || !s->alive[k]) return -1;
    long m = nvox(&s->ext[3 * k]);
    if (cap < m) return -1;
    memcpy(out, s->iota[k], sizeof(int) * m);
    return 0;
}

int orc_get_psi(const orc_sim *s, int k, double *out, int64_t cap) {
    if (!s || k < 0 || k >= s->G || !s->palive[k]) return -1;
    return copy_field(s->psi[k], &s->pext[3 * k], out, cap);
}

int orc_get_phic(const orc_sim *s, int k, double *out, int64_t cap) {
    if (!s || k < 0 || k >= s->G || !s->palive[k]) return -1;
    return copy_field(s->phic[k], &s->pext[3 * k], out, cap);
}

int orc_set_grain(orc_sim *s, int k, int alive, const int32_t lo[3], const int32_t ext[3],
                  const double *phi, const int32_t *iota) {
    if (!s || k < 0 || k >= s->G) return -1;
    free(s->phi[k]);
    free(s->iota[k]);
    s->phi[k] = NULL;
    s->iota[k] = NULL;
    s->alive[k] = 0;
    s->vol[k] = 0.0;
    if (!alive) return 0;
    for (int a = 0; a < 3; a++) {
        if (ext[a] < 1 || ext[a] > s->n[a] || lo[a] < 0 || lo[a] >= s->n[a]) return -1;
    }
    if (!phi) return -1;
    for (int a = 0; a < 3; a++) {
        s->lo[3 * k + a] = lo[a];
        s->ext[3 * k + a] = ext[a];
    }
    long m = nvox(&s->ext[3 * k]);
    s->phi[k] = (double *)malloc(sizeof(double) * m);
    memcpy(s->phi[k], phi, sizeof(double) * m);
    s->iota[k] = (int *)malloc(sizeof(int) * m);
    for (long v = 0; v < m; v++) s->iota[k][v] = iota ? iota[v] : -1;
    s->alive[k] = 1;
    s->vol[k] = volume_box(s->phi[k], m);
    return 0;
}

int orc_volumes(const orc_sim *s, double *out) {
    if (!s || !out) return -1;
    for (int k = 0; k < s->G; k++) out[k] = s->alive[k] ? s->vol[k] : 0.0;
    return 0;
}

/* Interface areas (energy functional, Eq. Energyfunctional): with the smoothed
 * Heaviside H = clamp(phi + 1/2, 0, 1) of the volume, grain k's interface
 * area is A_k = sum over its box of |grad H(phi_k)|, central differences (H =
 * 0 outside the box) summed over the axes in order; by the coarea formula
 * this is the area of the interface, whatever the slope of phi.  weighted[k]
 * weighs each voxel by the Read-Shockley energy of the pair (k, iota_k) when
 * the misorientation weights are on (1 where iota is -1 or they are off):
 * the boundary energy is (1/2) sum_k weighted_k in units of gamma_max h^(D-1)
 * (each boundary is seen from both grains). */
int orc_grain_areas(const orc_sim *s, double *area, double *weighted) {
    if (!s || !area) return -1;
    const int *n = s->n;
#pragma omp parallel for schedule(dynamic)
    for (int k = 0; k < s->G; k++) {
        area[k] = 0.0;
        if (weighted) weighted[k] = 0.0;
        if (!s->alive[k]) continue;
        const int *e = &s->ext[3 * k];
        const double *f = s->phi[k];
        double acc = 0.0, accw = 0.0;
        for (int z = 0; z < e[2]; z++)
            for (int y = 0; y < e[1]; y++)
                for (int x = 0; x < e[0]; x++) {
                    double gg = 0.0;
                    for (int a = 0; a < s->dim; a++) {
                        long cm[3] = {x, y, z}, cp[3] = {x, y, z};
                        cm[a] -= 1;
                        cp[a] += 1;
                        double hm = sample(f, e, n, cm[0], cm[1], cm[2], -s->W) + 0.5;
                        double hp = sample(f, e, n, cp[0], cp[1], cp[2], -s->W) + 0.5;
                        hm = hm < 0.0 ? 0.0 : (hm > 1.0 ? 1.0 : hm);
                        hp = hp < 0.0 ? 0.0 : (hp > 1.0 ? 1.0 : hp);
                        const double g = (hp - hm) * 0.5;
                        gg = gg + g * g;
                    }
                    const double m = sqrt(gg);
                    acc = acc + m;
                    double gam = 1.0;
                    const int j = s->iota[k] ? s->iota[k][lidx(e, x, y, z)] : -1;
                    if ((s->mode & 1) && j >= 0 && m > 0.0)
                        gam = read_shockley(orc_misorientation_deg(&s->quat[4 * k], &s->quat[4 * j]), s->theta_c);
                    accw = accw + m * gam;
                }
        area[k] = acc;
        if (weighted) weighted[k] = accw;
    }
    return 0;
}

int orc_labels(const orc_sim *s, int32_t *out) {
    if (!s || !out) return -1;
    const int *n = s->n;
    long nt = (long)n[0] * n[1] * n[2];
    double *best = (double *)malloc(sizeof(double) * nt);
    for (long i = 0; i < nt; i++) {
        best[i] = -INFINITY;
        out[i] = -1;
    }
    for (int k = 0; k < s->G; k++) { /* ascending id, strict '>' : ties -> lowest id */
        if (!s->alive[k]) continue;
        const int *lo = &s->lo[3 * k], *e = &s->ext[3 * k];
        for (int z = 0; z < e[2]; z++)
            for (int y = 0; y < e[1]; y++)
                for (int x = 0; x < e[0]; x++) {
                    long g = wrapi((long)lo[0] + x, n[0]) +
                             (long)n[0] * (wrapi((long)lo[1] + y, n[1]) +
                                           (long)n[1] * wrapi((long)lo[2] + z, n[2]));
                    double v = s->phi[k][lidx(e, x, y, z)];
                    if (v > best[g]) {
                        best[g] = v;
                        out[g] = k;
                    }
                }
    }
    free(best);
    return 0;
}

/* ------------------------------------------------------- stand-alone pieces */

int orc_convolve_box(int dim, const int32_t n[3], double band, double sigma,
                     const int32_t lo[3], const int32_t ext[3], const double *f, double *out) {
    (void)lo;
    if (!valid_grid(dim, n) || !(sigma > 0.0) || !f || !out) return -1;
    int e[3] = {ext[0], ext[1], ext[2]}, nn[3] = {n[0], n[1], n[2]};
    int R = kernel_radius(sigma);
    double *taps = gaussian_taps(sigma, R);
    predictor_box(dim, nn, band, e, f, out, taps, R);
    free(taps);
    return R;
}

/* ------------------------------------------------------- grid coarsening
 * (sec. 3, sequential optimizations): the grid spacing grows as grains vanish,
 * so that a grain keeps about the same number of voxels, and each function is
 * projected onto the coarser grid by trilinear interpolation.
 *
 * Reading: the periodic grid n becomes n' with the same ratio r = n / n' on
 * every axis of the model (r >= 1, any rational value).  New node i' sits at
 * old position i' r (node 0 on node 0), and the new voxel edge is r old edges.
 * A grain's remapped function at i' is its old function, by the sampling rule
 * (-W outside the old box), interpolated linearly along x, then y, then z
 * between the two old nodes that enclose i' r, and divided by r (distances in
 * new voxels).  The new box is the covered cyclic interval of the positive
 * nodes on each axis, padded by P (the creation rule); a grain without a
 * positive node vanishes.  The function is then re-initialised on the new box
 * with the taxicab scheme (as at creation), which restores the band [-W, W].
 * The voxel edge h used by the bulk term grows by r; the ID-field is rebuilt
 * as at creation when the predictor correction is on. */

/* Old node below new node i' and the interpolation weight of the node above:
 * i' n / n' = i0 + rem / n' in exact integer arithmetic. */
static void coarse_coord(int ip, int N, int Np, long *i0, double *t) {
    const long num = (long)ip * N;
    *i0 = num / Np;
    *t = (double)(num - *i0 * Np) / (double)Np;
}

/* Remapped value (before re-initialization) of a grain's old function at new
 * global node g' (n: old grid, np: new grid, r = n[0] / np[0]). */
static double coarse_sample(const double *f, const int *lo, const int *e, const int *n, const int *np,
                            int dim, double W, double r, const int gp[3]) {
    long i0[3] = {0, 0, 0};
    double t[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < dim; a++) coarse_coord(gp[a], n[a], np[a], &i0[a], &t[a]);
    double c[2][2]; /* (y, z) corners after the x interpolation, then y */
    const int nz = dim == 3 ? 2 : 1;
    for (int dz = 0; dz < nz; dz++)
        for (int dy = 0; dy < 2; dy++) {
            const long y = i0[1] + dy - lo[1], z = i0[2] + dz - lo[2];
            const double v0 = sample(f, e, n, i0[0] - lo[0], y, z, -W);
            const double v1 = sample(f, e, n, i0[0] + 1 - lo[0], y, z, -W);
            c[dz][dy] = (1.0 - t[0]) * v0 + t[0] * v1;
        }
    double v[2];
    for (int dz = 0; dz < nz; dz++) v[dz] = (1.0 - t[1]) * c[dz][0] + t[1] * c[dz][1];
    const double u = dim == 3 ? (1.0 - t[2]) * v[0] + t[2] * v[1] : v[0];
    return u / r;
}

int orc_coarsen(orc_sim *s, const int32_t np_in[3]) {
    if (!s || !np_in) return -1;
    const int dim = s->dim;
    int np[3] = {np_in[0], np_in[1], np_in[2]};
    const int *n = s->n;
    if (dim == 2 && np[2] != 1) return -1;
    for (int a = 0; a < dim; a++) {
        if (np[a] < 4 * s->P + 2 || np[a] > n[a]) return -1;
        if ((long)np[a] * n[0] != (long)np[0] * n[a]) return -1; /* one ratio on every axis */
    }
    const double r = (double)n[0] / (double)np[0];
    const double W = s->W;
    const int G = s->G;
    int *nlo = (int *)calloc(3L * G, sizeof(int)), *next = (int *)calloc(3L * G, sizeof(int));
    int *nalive = (int *)calloc(G, sizeof(int));
    double **nphi = (double **)calloc(G, sizeof(double *));
#pragma omp parallel for schedule(dynamic)
    for (int k = 0; k < G; k++) {
        if (!s->alive[k]) continue;
        const int *lo = &s->lo[3 * k], *e = &s->ext[3 * k];
        /* positive nodes of the remapped function over the whole new grid */
        unsigned char *occ[3];
        for (int a = 0; a < 3; a++) occ[a] = (unsigned char *)calloc(np[a], 1);
        int any = 0;
        for (int z = 0; z < np[2]; z++)
            for (int y = 0; y < np[1]; y++)
                for (int x = 0; x < np[0]; x++) {
                    const int gp[3] = {x, y, z};
                    if (!(coarse_sample(s->phi[k], lo, e, n, np, dim, W, r, gp) > 0.0)) continue;
                    any = 1;
                    occ[0][x] = occ[1][y] = occ[2][z] = 1;
                }
        if (any) {
            nalive[k] = 1;
            for (int a = 0; a < 3; a++) {
                int st = 0, ln = 0;
                cyclic_cover(occ[a], np[a], &st, &ln);
                pad_interval(st, ln, s->P, np[a], &nlo[3 * k + a], &next[3 * k + a]);
            }
            const int *ne = &next[3 * k], *nl = &nlo[3 * k];
            const long m = nvox(ne);
            double *f = (double *)malloc(sizeof(double) * m);
            for (int z = 0; z < ne[2]; z++)
                for (int y = 0; y < ne[1]; y++)
                    for (int x = 0; x < ne[0]; x++) {
                        const int gp[3] = {wrapi((long)nl[0] + x, np[0]), wrapi((long)nl[1] + y, np[1]),
                                           wrapi((long)nl[2] + z, np[2])};
                        f[lidx(ne, x, y, z)] = coarse_sample(s->phi[k], lo, e, n, np, dim, W, r, gp);
                    }
            nphi[k] = (double *)malloc(sizeof(double) * m);
            redistance_box(dim, np, W, ne, f, nphi[k]);
            free(f);
        }
        for (int a = 0; a < 3; a++) free(occ[a]);
    }
    for (int k = 0; k < G; k++) {
        free(s->phi[k]);
        free(s->iota[k]);
        s->phi[k] = nphi[k];
        s->iota[k] = NULL;
        s->alive[k] = nalive[k];
        s->vol[k] = 0.0;
        for (int a = 0; a < 3; a++) {
            s->lo[3 * k + a] = nlo[3 * k + a];
            s->ext[3 * k + a] = next[3 * k + a];
        }
        if (nalive[k]) {
            const long m = nvox(&next[3 * k]);
            s->vol[k] = volume_box(nphi[k], m);
            s->iota[k] = (int *)malloc(sizeof(int) * m);
            for (long v = 0; v < m; v++) s->iota[k][v] = -1;
        }
    }
    free(nlo);
    free(next);
    free(nalive);
    free(nphi);
    memcpy(s->n, np, sizeof(np));
    s->h_phys = s->h_phys * r;
    free_intermediates(s);
    if (s->mode) initial_iota(s);
    return 0;
}

/* Stand-alone remap of one box function (before re-initialization), for the
 * pinning tests: values at the new nodes of box (nlo, next) on grid np. */
int orc_coarse_sample_box(int dim, const int32_t n[3], const int32_t np[3], double band, const int32_t lo[3],
                          const int32_t ext[3], const double *f, const int32_t nlo[3], const int32_t next[3],
                          double *out) {
    const int nn[3] = {n[0], n[1], n[2]}, npp[3] = {np[0], np[1], np[2]};
    const int l[3] = {lo[0], lo[1], lo[2]}, e[3] = {ext[0], ext[1], ext[2]};
    const int ne[3] = {next[0], next[1], next[2]};
    const double r = (double)n[0] / (double)np[0];
    for (int z = 0; z < ne[2]; z++)
        for (int y = 0; y < ne[1]; y++)
            for (int x = 0; x < ne[0]; x++) {
                const int gp[3] = {wrapi((long)nlo[0] + x, npp[0]), wrapi((long)nlo[1] + y, npp[1]),
                                   wrapi((long)nlo[2] + z, npp[2])};
                out[lidx(ne, x, y, z)] = coarse_sample(f, l, e, nn, npp, dim, band, r, gp);
            }
    return 0;
}

int orc_set_redistance(orc_sim *s, int mode) {
    if (!s || mode < 0 || mode > 1) return -1;
    s->redist = mode;
    return 0;
}

int orc_redistance_box_euclid(int dim, const int32_t n[3], double band, const int32_t lo[3],
                              const int32_t ext[3], const double *f, double *out) {
    (void)lo;
    if (!valid_grid(dim, n) || !f || !out) return -1;
    int e[3] = {ext[0], ext[1], ext[2]}, nn[3] = {n[0], n[1], n[2]};
    redistance_box_euclid(dim, nn, band, e, f, out);
    return 0;
}

int orc_euclid_sweeps(int dim, double band) { return euclid_sweeps(dim, band); }

int orc_redistance_box(int dim, const int32_t n[3], double band,
                       const int32_t lo[3], const int32_t ext[3], const double *f, double *out) {
    (void)lo;
    if (!valid_grid(dim, n) || !f || !out) return -1;
    int e[3] = {ext[0], ext[1], ext[2]}, nn[3] = {n[0], n[1], n[2]};
    redistance_box(dim, nn, band, e, f, out);
    return 0;
}
