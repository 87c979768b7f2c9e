/*
 * gg.h -- C ABI of the MI355X (gfx950) level-set grain-growth library.
 *
 * One timestep of the local level-set method of Miessen, Velinov, Gottstein and
 * Barrales-Mora (arXiv:1701.06658, sec. 2.1, Algorithm 1): every grain carries a
 * signed-distance function on its own padded bounding box; a step is the
 * Gaussian predictor (sec. 2.1.4), the comparison corrector (sec. 2.1.5), the
 * taxicab re-initialization in the narrow band (sec. 2.1.6; a Euclidean
 * fast-sweeping variant on request) and the box / neighbour update (sec. 3.1).
 * Around the step: grid coarsening (sec. 3), interface areas for the energy
 * bookkeeping (Eq. Energyfunctional), checkpoint / resume and a tiling
 * autotuner.
 *
 * Conventions
 *  - Lengths are in voxels.  The grid is periodic with n[0] x n[1] x n[2] voxels
 *    (n[2] == 1 in 2D); field arrays are x fastest: index x + n0*(y + n1*z).
 *  - Grain ids are the label values 0 .. n_grains-1 given to gg_create; they
 *    never change.  Extinct grains keep their id and report volume 0.
 *  - A grain's box is (lo[3], ext[3]); global voxel g lies in it iff
 *    (g - lo) mod n < ext on every axis.  Box values are stored x fastest.
 *  - Every call returns gg_status; nothing throws across the boundary.  After
 *    an error the text is available from gg_last_error.  A HIP runtime error
 *    poisons the simulation: later calls return GG_E_POISONED (gg_destroy
 *    still works).  Argument errors leave the simulation unchanged.  The calls
 *    that advance or replace the state (gg_step, gg_autotune, gg_coarsen,
 *    gg_load_state, gg_load) check their arguments before they change
 *    anything; when one fails later, for memory (GG_E_NOMEM) or a size limit
 *    (GG_E_CAPACITY), its state may be part way replaced, and the simulation
 *    is poisoned as by a HIP error.
 *  - Host pointers are read or written only during the call; the library
 *    copies inputs and owns all device memory it allocates.
 *  - Work is issued on the HIP stream given to gg_create (NULL: the library
 *    creates its own).  A step's launch geometry is fixed (one work group per
 *    grain or per global tile) and its bookkeeping stays on the device, so the
 *    host reads nothing back between steps.  With gg_config.batched == 0,
 *    gg_step returns when its steps have finished; with batched != 0 it
 *    returns once the steps have been queued (as replays of captured HIP
 *    graphs, one per step) and the next call on the simulation waits for them.
 *    Query calls synchronise the stream.
 */
#ifndef GG_H
#define GG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gg_sim gg_sim;

typedef enum {
    GG_OK = 0,
    GG_E_ARG = 1,         /* invalid argument; nothing changed                     */
    GG_E_NOMEM = 2,       /* host or device allocation failed                     */
    GG_E_HIP = 3,         /* HIP runtime error; the simulation is now poisoned     */
    GG_E_CAPACITY = 4,    /* a size limit of the library was exceeded             */
    GG_E_SMALLBUF = 5,    /* caller's output buffer is too small                  */
    GG_E_NUMERIC = 6,     /* reserved: non-finite inputs are argument errors      */
    GG_E_POISONED = 7,    /* an earlier HIP error poisoned this simulation         */
    GG_E_UNSUPPORTED = 8, /* valid request the library does not implement         */
    GG_E_NODEVICE = 9     /* no usable gfx950 device                              */
} gg_status;

typedef enum {
    GG_FP64 = 0,       /* plain path: FP64 storage and arithmetic                */
    GG_FP32 = 1,       /* mixed path: FP32 storage/arithmetic, FP64 reductions   */
    GG_MIXED_BF16 = 2, /* BF16 convolution operands with FP32 accumulation: not
                          built (GG_E_UNSUPPORTED): the convolution is a
                          17-tap stencil on the vector ALUs, not a dense
                          contraction, and its operands are already read once
                          per step in FP32                                      */
    GG_MIXED_FP16 = 3  /* FP16 likewise: GG_E_UNSUPPORTED                        */
} gg_precision;

/* Re-initialization scheme of gg_step (gg_create always uses the taxicab one
 * for the initial function). */
typedef enum {
    GG_REDIST_TAXICAB = 0, /* the method's scheme (sec. 2.1.6): reference values
                              next to the sign change spread as taxicab
                              distances, exact min over reference cells        */
    GG_REDIST_EUCLID = 1   /* variant: Euclidean fast sweeping with Godunov's
                              upwind update (the redistancing scheme the paper
                              cites), K = ceil(sqrt(dim) W) + 1 (rounded up to
                              even) Jacobi sweeps from gradient-normalised
                              reference values |phi| / |grad phi| (at most the
                              taxicab reference value) on the cells next to the
                              sign change; cells outside the box are absent    */
} gg_redistance;

/* Predictor-correction terms (sec. 2.1.4, Eq. eq:velocorrect). */
enum {
    GG_PHYS_NONE = 0,
    GG_PHYS_MISORIENTATION = 1, /* per-pair weight w = mobility * energy from the
                                   misorientation of the two grains (hexagonal 622
                                   symmetry; Read-Shockley energy below theta_c,
                                   mobility law Eq. eq:GB_mob); needs quat       */
    GG_PHYS_BULK = 2            /* per-grain bulk energy density driving force
                                   (Eqs. magneticE/magneticF, normalised with
                                   Eq. bulk normalization); needs energy_density */
};

typedef struct {
    int32_t dim;            /* 2 or 3                                               */
    int32_t n[3];           /* periodic grid size, each in [4P + 2, 4096] with       */
                            /* P = ceil(band); n[2] == 1 when dim == 2; at most      */
                            /* 2^31 - 1 voxels in all                                */
    double band;            /* narrow-band half width W in voxels (1 <= W <= 16);
                               the box pad is P = ceil(W) (Fig. 1a: >= 7 points)   */
    int32_t precision;      /* gg_precision                                         */
    int32_t physics;        /* GG_PHYS_* bits                                       */
    double theta_c_deg;     /* Read-Shockley cutoff angle (GG_PHYS_MISORIENTATION)   */
    double voxel_m;         /* voxel edge h in metres (GG_PHYS_BULK)                 */
    double gamma_max;       /* maximal boundary energy, J/m^2 (GG_PHYS_BULK)         */
    double capacity_headroom; /* device buffer slack factor (0: default 1.25); 1:
                               no slack, the buffers hold exactly the current
                               layout (every step whose boxes grow is then taken
                               again after the buffers grow)                   */
    int32_t redistance;     /* gg_redistance: re-initialization scheme of the steps  */
    int32_t batched;        /* 0: gg_step launches its kernels and waits for them;
                               1: gg_step replays captured HIP graphs and returns
                               at once (the Euclidean variant, per-kernel timing
                               and kept intermediates use plain launches)       */
    uint32_t flags;         /* GG_FLAG_* bits                                       */
} gg_config;

/* gg_config.flags */
enum {
    GG_FLAG_ORDER_ID = 1u,  /* launch the per-grain kernels in grain-id order
                               (the default is largest box first, which keeps
                               the longest boxes off the end of each launch);
                               results do not depend on the order               */
    GG_FLAG_CLOSEST_POINT = 2u /* correction weight from the closest point of
                               the grain boundary (sec. 3.2, with the
                               correction of sec. 2.1.4; needs
                               GG_PHYS_MISORIENTATION): every voxel with
                               |phi| < 2 takes the weight of the closest piece
                               of its grain's linearised zero level set (cells
                               cut along the main diagonal into triangles /
                               tetrahedra; a piece's weight is the mean pair
                               weight over the distinct ID-field entries at
                               its cell's nodes: boundary or junction; ties to
                               the lowest cell, then piece); other voxels keep
                               the ID-field pair.  Adds a pass that finishes
                               phi (3D) and the search to every step      */
};

typedef struct {
    int64_t steps;          /* steps taken since gg_create                          */
    int64_t total_grain_voxels; /* sum over all steps taken of the grain voxels    */
    int32_t alive;          /* alive grains                                         */
    int32_t kernel_radius;  /* R of the last step                                   */
    int64_t grain_voxels;   /* sum of box volumes at the start of the last step    */
    int64_t capacity;       /* device arena capacity in values                      */
    double superposition;   /* grain_voxels / prod(n)                               */
    double last_step_ms;    /* device time of the last gg_step call / its n_steps   */
    int32_t n[3];           /* current periodic grid (changes with gg_coarsen)      */
    int32_t dim;
} gg_step_stats;

/* Device memory of a simulation through the caller's allocator (e.g. a caching
 * allocator): alloc(bytes, stream, user) returns device memory on the
 * simulation's device, usable in stream order on `stream`, or NULL; free(p,
 * stream, user) takes back a block alloc returned.  No work that uses a block
 * is pending on the device when the library frees it.  Used for every device
 * buffer of the simulation, from gg_create to gg_destroy. */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *user);
    void (*free)(void *p, void *stream, void *user);
    void *user;
} gg_allocator;

/* Create a simulation from a label field (host, prod(n) int32, x fastest, values
 * in [0, n_grains)); sec. 3.1: one grain object per cell of the input tessellation.
 * Each grain's box is the covered cyclic interval of its projection on every
 * axis, padded by P; its function is the re-initialised +-1/2 indicator.
 * quat: 4*n_grains doubles (w,x,y,z) or NULL; energy_density: n_grains doubles
 * in J/m^3 or NULL (required by the matching physics bits).
 * hip_stream: a hipStream_t or NULL (the library creates its own).  allocator:
 * NULL (hipMalloc / hipFree) or the caller's allocator, copied; it needs a
 * non-NULL hip_stream.  On success *out owns the simulation.
 * Errors: GG_E_ARG (bad config/labels/allocator), GG_E_UNSUPPORTED (a
 * precision the library does not implement), GG_E_NODEVICE, GG_E_NOMEM,
 * GG_E_HIP. */
gg_status gg_create(const gg_config *cfg, const int32_t *labels, int32_t n_grains,
                    const double *quat, const double *energy_density, void *hip_stream,
                    const gg_allocator *allocator, gg_sim **out);

/* Advance n_steps timesteps of normalised length dt (Algorithm 1, sec. 2.1.3):
 * Gaussian width sigma = sqrt(2 dt) * n[0] voxels (heat kernel of Eq.
 * Heatequation), kernel radius R = ceil(4 sigma).  Requires R <= 2*ceil(W) and
 * R <= 12.  Each step is the predictor, the corrector, the box plan with the
 * coverage lists of the new boxes, and the re-initialization into the new
 * boxes; a step whose new boxes or coverage lists do not fit the device
 * buffers leaves its starting state untouched, and the library grows the
 * buffers and takes the step again.  batched != 0: the call returns once the
 * steps are queued; errors of the queued steps (GG_E_NOMEM, GG_E_CAPACITY,
 * GG_E_HIP) are reported by the next call.
 * Errors: GG_E_ARG (dt not finite/positive, n_steps < 0, R too large; nothing
 * changed), GG_E_CAPACITY / GG_E_NOMEM / GG_E_HIP (poisoned), GG_E_POISONED. */
gg_status gg_step(gg_sim *sim, double dt, int32_t n_steps);

/* Wait for all issued work. */
gg_status gg_sync(gg_sim *sim);

/* Number of alive grains. */
gg_status gg_grain_count(gg_sim *sim, int32_t *alive);

/* Grain volumes (sec. 3.1: the size of each grain object), read as the smoothed
 * Heaviside sum V_k = sum over the box of clamp(phi + 1/2, 0, 1) in FP64 and
 * voxels (exact across a planar two-grain boundary, where the two functions are
 * opposite), indexed by grain id (0 for extinct grains); out: host, cap >=
 * n_grains.  Errors: GG_E_ARG, GG_E_SMALLBUF. */
gg_status gg_grain_volumes(gg_sim *sim, double *out, int64_t cap);

/* Interface areas for the energy bookkeeping (energy functional, Eq.
 * Energyfunctional): area[k] = sum over grain k's box of |grad H(phi_k)|, H =
 * clamp(phi + 1/2, 0, 1) (the volume's smoothed Heaviside), central differences
 * with -W outside the box, in FP64 and voxel^(D-1) units (by the coarea formula
 * the interface area, whatever the slope of phi).  weighted (may be NULL): the
 * same sum with each voxel weighted by the Read-Shockley energy of the pair
 * (k, ID-field) under GG_PHYS_MISORIENTATION (1 otherwise).  The boundary
 * energy is (1/2) sum_k weighted[k] gamma_max h^(D-1); the bulk energy is
 * sum_k E_k V_k h^D.  Host arrays, cap >= n_grains (0 for extinct grains). */
gg_status gg_grain_areas(gg_sim *sim, double *area, double *weighted, int64_t cap);

/* gg_grain_areas for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and summation order, so the same values, written into device memory
 * of the simulation's device (area_dev, weighted_dev: cap >= n_grains doubles
 * each; weighted_dev may be NULL), ordered on the simulation's stream; the call
 * does not wait for the write.  It allocates nothing: the per-block partial
 * sums go to a static device array of the library (partials of at most 65536
 * grains, 8 MiB on every device the library runs on, held until the process
 * ends).  Every call on one device shares that array: calls whose streams
 * overlap on one device (different simulations, different streams) race on
 * it.  Queued batched steps are taken over only if none of them failed its
 * capacity check; otherwise the call returns GG_E_CAPACITY, writes nothing and
 * leaves the steps queued (gg_sync, which may allocate, takes them again).
 * Errors: GG_E_ARG (NULL area_dev), GG_E_SMALLBUF, GG_E_CAPACITY (n_grains >
 * 65536, or a queued step that needs larger buffers), GG_E_UNSUPPORTED
 * (device index above 63). */
gg_status gg_grain_areas_noalloc(gg_sim *sim, double *area_dev, double *weighted_dev, int64_t cap);

/* Voxel labels (the tessellation the grains define, sec. 2.1.1: a voxel belongs
 * to the grain whose function is largest there, i.e. inside its zero level
 * set): argmax over the grains whose box covers the voxel of their function
 * (ties to the lowest id); out: prod(n) int32, x fastest, host memory, or
 * device memory on the simulation's device when out_is_device != 0 (then the
 * write is ordered on the simulation's stream and the call does not wait for
 * it).  Errors: GG_E_ARG, GG_E_SMALLBUF. */
gg_status gg_labels(gg_sim *sim, int32_t *out, int64_t cap, int32_t out_is_device);

/* Step statistics: the counters of the metric (grain voxels per step, the
 * box voxels of the size-adaptive boxes of sec. 3.1), the superposition of
 * the boxes (sec. 5.2.3) and the device time of the last gg_step call.
 * Errors: GG_E_ARG. */
gg_status gg_stats(gg_sim *sim, gg_step_stats *out);

/* Per-kernel device time, for roofline accounting.  Kernel classes: */
enum {
    GG_K_PREDICT = 0,   /* backward z spreading, band clamp, volume, Gaussian z/x/y
                           (+ correction epilogue): f -> psi (+ phi)              */
    GG_K_COMPARE = 1,   /* corrector over global tiles: psi -> phi^c              */
    GG_K_REINIT = 2,    /* reference values, x/y spreading, forward z spreading:
                           phi^c -> f (Euclidean variant: reference values)       */
    GG_K_REINIT_SWEEP = 3, /* Jacobi sweeps of GG_REDIST_EUCLID                   */
    GG_K_PLAN = 4,      /* box plan, scans, coverage lists, launch order, step
                           counters; coarsening                                   */
    GG_K_CLOSEST = 5,   /* closest-boundary-point weights (GG_FLAG_CLOSEST_POINT) */
    GG_K_CLASSES = 6
};
typedef struct {
    double ms[GG_K_CLASSES];          /* summed device time (HIP events)            */
    int64_t launches[GG_K_CLASSES];   /* timed kernel dispatches                    */
    int64_t voxels[GG_K_CLASSES];     /* grain voxels the timed spans covered       */
} gg_kernel_times;

/* Turn per-kernel timing on (resets the sums) or off.  While on, every launch
 * of the step is bracketed by HIP events on the simulation's stream. */
gg_status gg_profile(gg_sim *sim, int32_t on);
gg_status gg_get_kernel_times(gg_sim *sim, gg_kernel_times *out);

/* State access (host memory).  gg_get_boxes fills cap >= n_grains entries:
 * lo/ext 3 per grain, alive 1 per grain, offset 1 per grain (start of the
 * grain's values in the packed order used by gg_get_values, -1 if extinct).
 * gg_get_values writes all alive grains' values as doubles in that packed
 * order (cap >= sum of box volumes); gg_get_iota does the same for the
 * ID-field (argmax neighbour of the last corrector, -1 where none). */
gg_status gg_get_boxes(gg_sim *sim, int32_t *lo, int32_t *ext, int32_t *alive, int64_t *offset,
                       int64_t cap);
gg_status gg_get_values(gg_sim *sim, double *out, int64_t cap);
gg_status gg_get_iota(gg_sim *sim, int32_t *out, int64_t cap);

/* Replace the whole state (host memory): boxes and liveness for every grain,
 * values packed grain after grain in id order over the alive grains, and an
 * optional ID-field in the same order (NULL: all -1).  Boxes must satisfy the
 * library's box rule: 1 <= ext[a] <= n[a] - 2P or ext[a] == n[a], 0 <= lo < n.
 * Errors: GG_E_ARG (a box breaks the rule, a value is not finite; nothing
 * changed), GG_E_NOMEM / GG_E_HIP (poisoned). */
gg_status gg_load_state(gg_sim *sim, const int32_t *lo, const int32_t *ext, const uint8_t *alive,
                        const double *values, const int32_t *iota);

/* Grid coarsening (sec. 3, sequential optimizations: the grid spacing grows as
 * grains vanish, keeping about the same voxels per grain; each function is
 * projected by trilinear interpolation).  The periodic grid becomes n_new with
 * one ratio r = n[a] / n_new[a] >= 1 on every axis of the model; new voxel i'
 * sits at old position i' r (voxel 0 on voxel 0).  Each grain's function (-W
 * outside its box) is interpolated linearly along x, y, z there and divided by
 * r (lengths in new voxels); the new box is the covered cyclic interval of the
 * positive voxels on each axis, padded by P (grains without one vanish); the
 * function is re-initialised on it with the taxicab scheme, as in gg_create.
 * voxel_m (the bulk term's h) grows by r; the ID-field is rebuilt as at
 * creation.  Later steps take sigma = sqrt(2 dt) * n_new[0] voxels, so the
 * same normalised dt is a shorter stencil.  Intermediates kept for
 * gg_get_intermediate are dropped.
 * Errors: GG_E_ARG (n_new outside [4P + 2, n] on an axis, ratios differ,
 * n_new[2] != 1 in 2D; nothing changed), GG_E_CAPACITY / GG_E_NOMEM / GG_E_HIP
 * (the state was replaced part way: the simulation is poisoned). */
gg_status gg_coarsen(gg_sim *sim, const int32_t n_new[3]);

/* One grain's box (lo, ext; all 0 for an extinct grain) and its values as
 * doubles, x fastest (host memory).  With out == NULL (or cap too small) only
 * the box is written: the call then returns GG_OK (out == NULL) or
 * GG_E_SMALLBUF, and prod(ext) values are needed.  Errors: GG_E_ARG (id out of
 * range). */
gg_status gg_grain_sdf(gg_sim *sim, int32_t id, int32_t lo[3], int32_t ext[3], double *out, int64_t cap);

/* Autotuning of the launch schedule: the order in which the per-grain kernels
 * take the boxes (largest box first, or grain id: GG_FLAG_ORDER_ID) and, for
 * the Euclidean variant, the LDS budgets of its work-item tilings (the work
 * group's, default 40 KB, and the small launch class's, default 26 KB).
 * gg_autotune takes steps_per_candidate steps (normalised length dt) with
 * each candidate, keeps the one with the least device time per grain voxel
 * and reports every candidate's time.  The simulation advances by those steps;
 * the functions do not depend on the schedule (bit-identical).
 * Errors: GG_E_ARG (dt not finite/positive, steps_per_candidate < 1; nothing
 * changed), GG_E_CAPACITY / GG_E_NOMEM / GG_E_HIP (poisoned). */
typedef struct {
    int32_t order_size;        /* chosen: 1 largest box first, 0 grain id       */
    int32_t lds_bytes;         /* chosen Euclidean work-group LDS budget        */
    int32_t small_bytes;       /* chosen Euclidean small-class LDS limit        */
    int32_t candidates;        /* candidates timed                              */
    double ns_per_gv[8];       /* device time per grain voxel of each candidate */
    int32_t cand_order[8], cand_lds[8], cand_small[8];
} gg_tuning;
gg_status gg_autotune(gg_sim *sim, double dt, int32_t steps_per_candidate, gg_tuning *out);

/* Checkpoint / resume.  gg_save writes the state to a file: grid, boxes,
 * liveness, values in the stored precision, the ID-field (with the predictor
 * correction), volumes and step counters.  gg_load replaces the state of a
 * simulation created with the same dim, n_grains, precision, band, physics
 * and re-initialization scheme (the grid may differ: a coarsened run); per-grain
 * physics inputs stay those given to gg_create.  The steps that follow a
 * gg_load are identical to those that would have followed the gg_save.
 * Errors: GG_E_ARG (cannot open or write the file, not a checkpoint of this
 * library, a different configuration, a corrupt file; nothing changed),
 * GG_E_NOMEM / GG_E_HIP (gg_load: poisoned). */
gg_status gg_save(gg_sim *sim, const char *path);
gg_status gg_load(gg_sim *sim, const char *path);

/* Test hook: when on, each step keeps its predictor output (which = 0) and its
 * corrector output (which = 1) on the box layout the step started from; read
 * them with gg_get_intermediate (same packing as gg_get_values, with the boxes
 * of that layout written to lo/ext/alive/offset when not NULL).  which = 2
 * (GG_FLAG_CLOSEST_POINT, no keeping needed): the correction weights of the
 * current state's next predictor, on the current boxes. */
gg_status gg_keep_intermediates(gg_sim *sim, int32_t on);
gg_status gg_get_intermediate(gg_sim *sim, int32_t which, double *out, int64_t cap, int32_t *lo,
                              int32_t *ext, int32_t *alive, int64_t *offset, int64_t cap_grains);

const char *gg_status_str(gg_status st);
const char *gg_last_error(const gg_sim *sim);
void gg_destroy(gg_sim *sim);

/* Library version string. */
const char *gg_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GG_H */
