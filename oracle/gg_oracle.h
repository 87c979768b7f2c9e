/*
 * FP64 CPU oracle of the local level-set grain-growth timestep
 * (Miessen, Velinov, Gottstein, Barrales-Mora, arXiv:1701.06658).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no source,
 * header, table or helper with the HIP library under paper_1701_06658_amd/.
 *
 * Units: one voxel = one length unit.  The grid is periodic with n[a] voxels
 * per axis (n[2] == 1 in 2D).  Every grain k owns a box (lo_k, ext_k) and a
 * level-set function phi_k stored x-fastest on that box.
 */
#ifndef GG_ORACLE_H
#define GG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_sim orc_sim;

/* Build the grains from a label field (x fastest, values in [0, G)).
 * Returns NULL on bad arguments or out of memory. */
orc_sim *orc_create(int dim, const int32_t n[3], double band, const int32_t *labels, int32_t G);
void orc_destroy(orc_sim *s);

/* Predictor correction inputs (row a2).  mode bit 1: misorientation weights
 * (hexagonal 622 symmetry, Read-Shockley energy with cutoff theta_c_deg and the
 * sigmoidal mobility law); mode bit 2: per-grain bulk energy density.
 * quat: 4*G (w,x,y,z) or NULL; energy: G values in J/m^3 or NULL;
 * h_phys: voxel edge in metres; gamma_max in J/m^2.  Call after create. */
int orc_set_physics(orc_sim *s, int mode, const double *quat, double theta_c_deg,
                    const double *energy, double h_phys, double gamma_max);

/* Re-initialization scheme of the following steps (creation always uses the
 * taxicab one): 0 = the paper's fast scheme (exact reference values spread by
 * one per voxel: taxicab distances), 1 = Euclidean fast sweeping (Godunov
 * upwind update in Jacobi form from gradient-normalised reference values). */
int orc_set_redistance(orc_sim *s, int mode);

/* Closest grain-boundary point (sec. 3.2, with the correction of sec. 2.1.4):
 * with on != 0 and the misorientation weights on, every voxel with |phi| <
 * tube takes its correction weight from the closest piece of the linearised
 * zero level set of its grain (simplices cut along each cell's main diagonal;
 * the piece's weight is the mean pair weight over the distinct ID-field
 * entries at its cell's nodes); other voxels keep the ID-field pair. */
int orc_set_closest_point(orc_sim *s, int on, double tube);
/* The weight map the next step's correction uses for grain k (needs mode bit
 * 1); returns 1, 0 if extinct, -1 on error. */
int orc_closest_weights(const orc_sim *s, int k, double *out, int64_t cap);

/* Grid coarsening (sec. 3, sequential optimizations): project every grain onto
 * the coarser periodic grid np (same ratio r = n / np >= 1 on every axis of the
 * model, each axis >= 4P + 2) by trilinear interpolation at old position i' r,
 * values divided by r; new boxes from the positive nodes; re-initialised with
 * the taxicab scheme.  The voxel edge of the bulk term grows by r. */
int orc_coarsen(orc_sim *s, const int32_t np[3]);

/* One timestep of normalised length dt (sigma = sqrt(2 dt) * n[0] voxels). */
int orc_step(orc_sim *s, double dt);
/* Keep the predictor output and the corrector output of the last step. */
void orc_keep_intermediates(orc_sim *s, int on);

int orc_grain_count(const orc_sim *s);
int orc_alive_count(const orc_sim *s);
/* Box and liveness of grain k; returns 1 if alive, 0 if extinct, -1 on error. */
int orc_get_box(const orc_sim *s, int k, int32_t lo[3], int32_t ext[3]);
int orc_get_phi(const orc_sim *s, int k, double *out, int64_t cap);
int orc_get_iota(const orc_sim *s, int k, int32_t *out, int64_t cap);
/* Last step's predictor output psi and corrector output phi^c, on the box the
 * step started from (orc_get_prev_box). */
int orc_get_prev_box(const orc_sim *s, int k, int32_t lo[3], int32_t ext[3]);
int orc_get_psi(const orc_sim *s, int k, double *out, int64_t cap);
int orc_get_phic(const orc_sim *s, int k, double *out, int64_t cap);
/* Replace grain k's state (alive=0 removes it).  iota may be NULL (all -1). */
int orc_set_grain(orc_sim *s, int k, int alive, const int32_t lo[3], const int32_t ext[3],
                  const double *phi, const int32_t *iota);

int orc_volumes(const orc_sim *s, double *out);      /* G values, 0 if extinct */
int orc_labels(const orc_sim *s, int32_t *out);       /* prod(n) values */
/* Interface area of every grain, sum of |grad clamp(phi + 1/2, 0, 1)| (central
 * differences), and the same weighted by the Read-Shockley energy of the pair
 * (k, iota) when the misorientation weights are on (weighted may be NULL). */
int orc_grain_areas(const orc_sim *s, double *area, double *weighted);

/* Stand-alone pieces used by the pinning tests. */
int orc_convolve_box(int dim, const int32_t n[3], double band, double sigma,
                     const int32_t lo[3], const int32_t ext[3], const double *f, double *out);
int orc_redistance_box(int dim, const int32_t n[3], double band,
                       const int32_t lo[3], const int32_t ext[3], const double *f, double *out);
int orc_redistance_box_euclid(int dim, const int32_t n[3], double band,
                              const int32_t lo[3], const int32_t ext[3], const double *f, double *out);
int orc_euclid_sweeps(int dim, double band);   /* Jacobi sweeps of the Euclidean scheme */
/* The coarsening's remap of one box function before re-initialization. */
int orc_coarse_sample_box(int dim, const int32_t n[3], const int32_t np[3], double band, const int32_t lo[3],
                          const int32_t ext[3], const double *f, const int32_t nlo[3], const int32_t next[3],
                          double *out);
/* Closest piece of every voxel of a stand-alone box with |phi| < tube (the
 * box may take a whole periodic axis): squared distance (-1 outside the tube),
 * cell (linear box index of its lower node) and piece index. */
int orc_closest_box(int dim, const int32_t n[3], const int32_t ext[3], const double *phi, double tube,
                    double *d2, int64_t *cell, int32_t *piece);
double orc_misorientation_deg(const double qa[4], const double qb[4]);
double orc_pair_weight(double theta_deg, double theta_c_deg, double *mobility);
int orc_num_threads(void);
void orc_set_num_threads(int n);   /* threads of the following calls (n > 0) */

#ifdef __cplusplus
}
#endif
#endif
