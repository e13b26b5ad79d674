/*
 * sph4he.h: C ABI of the MI355X two-fluid SPH step (liquid helium-4 with spin angular
 * momentum, explicit weakly-compressible SPH).
 *
 * The library advances particles under the paper's Eqs. 1-2 (inviscid and viscous
 * components with pressure gradient, interfacial/temperature-gradient force, shear and
 * rotational viscosity with the spin term, local interaction force F_sn = C_l v_sn) and
 * the Tait equation of state, Eq. 4, by velocity Verlet (Sec. 2.3, Algorithm 1), with a
 * cell-linked-list neighbour search and a rotating wall-particle layer (Sec. 3).
 *
 * Conventions shared by every call:
 *   - All entry points return sph_status; none aborts, throws or prints.
 *   - Particle arrays are structure-of-arrays: a "[3][n]" array of doubles holds the
 *     x components of all n particles, then all y, then all z.  Per-particle arrays are
 *     indexed by particle id = position in the array given to *_init.
 *   - Array pointers are DEVICE pointers unless stated otherwise.  The caller owns all
 *     device memory, including the workspace; the library never allocates or frees
 *     device memory and never creates streams.  Work is enqueued on the stream given at
 *     creation (a hipStream_t passed as void*; NULL = the null stream); calls return
 *     before the work finishes unless they say they synchronise.
 *   - Argument and state errors are detected on the host before anything is enqueued.
 *     Device-side anomalies (non-finite values, particles leaving a non-periodic grid,
 *     overfull cells) set a sticky error word that the next synchronising call reports.
 *   - One handle must not be used from two host threads at once.  Two handles on one
 *     device are independent.
 */
#ifndef SPH4HE_H
#define SPH4HE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPH_ABI_VERSION 3u

typedef enum {
    SPH_OK = 0,
    SPH_E_INVALID = 1,     /* bad argument or parameter value                            */
    SPH_E_WORKSPACE = 2,   /* workspace NULL, misaligned (256 B) or too small             */
    SPH_E_HIP = 3,         /* a HIP runtime call failed (no device, launch failure ...)   */
    SPH_E_STATE = 4,       /* call out of order (e.g. step before init)                   */
    SPH_E_DOMAIN = 5,      /* a particle left the cell grid along a non-periodic axis      */
    SPH_E_NONFINITE = 6,   /* NaN/Inf in positions, velocities, spins or accelerations    */
    SPH_E_UNSUPPORTED = 7, /* valid but not implemented (e.g. gamma != 7)                 */
    SPH_E_CAPACITY = 8     /* a cell holds more particles than the search supports, or an */
                           /* output capacity is too small                               */
} sph_status;

/* Smoothing kernels (support radius 2h).  The paper's kernel list is an appendix figure;
 * these are the two standard 3D kernels used by the workloads. */
typedef enum { SPH_KERNEL_CUBIC = 0, SPH_KERNEL_WENDLAND_C2 = 1 } sph_kernel;

/* SPH_FP64: every quantity in double precision.
 * SPH_FP32_MIXED: positions, velocities, spins, the integrator and global sums in
 * double; pair interactions in single precision with compensated (Kahan) per-particle
 * accumulation; density, pressure and accelerations stored in single precision. */
typedef enum { SPH_FP64 = 0, SPH_FP32_MIXED = 1 } sph_precision;

/* SPH_GEOM_PERIODIC_BOX: all three axes periodic on [lo, hi).
 * SPH_GEOM_CYLINDER_Z:   x and y bounded (walls are particles), z periodic on
 *                        [lo[2], hi[2]) (the paper's slip top and bottom, Sec. 3).  Every
 *                        particle stays within 2h of the cylinder about the z axis
 *                        inscribed in the box's x-y extent: x^2 + y^2 <= (r + 2h)^2,
 *                        r = min(-lo[0], hi[0], -lo[1], hi[1]).  A particle beyond is a
 *                        domain error (SPH_E_DOMAIN), like one that leaves the box.
 * SPH_GEOM_OPEN:         no periodic axis (free clusters). */
typedef enum { SPH_GEOM_PERIODIC_BOX = 0, SPH_GEOM_CYLINDER_Z = 1, SPH_GEOM_OPEN = 2 } sph_geometry;

/* Per-particle kind (uint8): fluid particles move under the forces; wall particles turn
 * rigidly about the z axis at the imposed rate.  The inner wall layer gets its density
 * and pressure from the kernel sum like fluid; outer layers keep rho0 and P = 0
 * (wall and dummy particles, Sec. 3). */
typedef enum { SPH_FLUID = 0, SPH_WALL_INNER = 1, SPH_WALL_OUTER = 2 } sph_kind;

/* Per-particle species (uint8): inviscid (superfluid-like) or viscous (normal-like)
 * component of the mixture (Sec. 2.1).  Wall particles must be SPH_VISCOUS. */
typedef enum { SPH_INVISCID = 0, SPH_VISCOUS = 1 } sph_species;

typedef struct {
    uint32_t abi_version;   /* must be SPH_ABI_VERSION                                    */
    int32_t kernel;         /* sph_kernel                                                 */
    int32_t precision;      /* sph_precision                                              */
    int32_t geometry;       /* sph_geometry                                               */
    double dx;              /* lattice spacing: sets the spin inertia and default masses  */
    double h;               /* smoothing length; interaction radius 2h                    */
    double lo[3], hi[3];    /* domain box; periodic axes wrap on [lo, hi)                 */
    double rho0;            /* reference density of Eq. 4                                 */
    double c0;              /* sound speed: Tait stiffness B = rho0 c0^2 / gamma          */
    double gamma;           /* Tait exponent alpha_P of Eq. 4; only 7 is supported        */
    double mass[2];         /* particle mass per species; <= 0 selects rho0 dx^3 / lambda,*/
                            /* lambda = dx^3 sum over the cubic lattice of W(|n| dx), so   */
                            /* that a perfect lattice has density rho0                    */
    double eta;             /* shear = rotational viscosity eta_n (Sec. 3)                */
    double sigma_T;         /* interfacial (temperature-gradient) force coefficient       */
    double C_l;             /* local-interaction (mutual friction) coefficient            */
    double kappa_I;         /* spin inertia I = kappa_I m dx^2                            */
    int32_t cell_factor;    /* cells per interaction radius along each axis (1..4)        */
    int32_t pressure_filter;/* 1: pressure filter of Algorithm 1 after the EOS; 0: none.   */
                            /* Reading (the paper cites the filter without its formula):   */
                            /* P_i <- (V_i P_i W(0) + sum_j V_j P_j W_ij)                  */
                            /*       / (V_i W(0) + sum_j V_j W_ij), V = m/rho, over fluid   */
                            /* and inner-wall particles and neighbours; outer walls keep   */
                            /* P = 0 and are not sources.  The forces and the P returned   */
                            /* by sph_read_fields use the filtered pressure.               */
    double coll_alpha;      /* collision step of Algorithm 1: distance coll_alpha * dx,    */
                            /* 0 <= coll_alpha * dx < 2h; 0 switches it off.  Reading (the */
                            /* paper cites the model without its formula): after each      */
                            /* drift, every fluid particle i closer than that to a         */
                            /* neighbour j it approaches ((v_i - v_j).(x_i - x_j) < 0)     */
                            /* takes v_i -= (1 + coll_e) mu ((v_ij . r_ij) / r^2) r_ij,    */
                            /* mu = m_j / (m_i + m_j) (1 for a wall neighbour), all pairs  */
                            /* from the velocities before the step; walls are unchanged    */
    double coll_e;          /* restitution of the collision step, in [0, 1]               */
} sph_params;

/* Launch shape of the kernels (performance only; results do not depend on it).
 * Zero fields keep the current value.  Block sizes must be multiples of 64 in
 * [64, 1024]. */
typedef struct {
    int32_t block_density;  /* threads per block of the density sweep                     */
    int32_t block_force;    /* threads per block of the force sweep                       */
    int32_t block_stream;   /* threads per block of the streaming kernels                 */
    int32_t use_graph;      /* 1: replay steps from a captured hipGraph (needs a non-null */
                            /* stream); 0: launch eagerly; -1: keep                        */
    int32_t sweep;          /* FP32-mixed density/force sweeps: 1 one thread per particle; */
                            /* 3 (default) one workgroup per 2x2x2-cell brick staged in    */
                            /* LDS, lanes over candidates for the neighbour test; needs    */
                            /* cell_factor 1 on every instance (else 1 is used); 0: keep;  */
                            /* any other value is SPH_E_INVALID                            */
    int32_t xcd_run;        /* brick sweeps: consecutive bricks (in Morton order) given to   */
                            /* each of the 8 XCDs in turn, 1..256 (default 8); 0: keep       */
    int32_t list_targets;   /* brick density sweep: targets tested per round, 16 or 32        */
                            /* (default 32); 0: keep                                          */
} sph_tuning;

typedef struct sph_sim sph_sim;      /* one SPH instance (opaque, host memory)            */
typedef struct sph_batch sph_batch;  /* an ensemble of independent instances              */

/* Defaults: abi_version, Wendland C2, FP32_MIXED, periodic unit box, rho0 = 1, gamma = 7,
 * default masses, kappa_I = 0.4, cell_factor = 1, no pressure filter, no collision step;
 * dx, h, c0 must still be set. */
sph_status sph_params_init(sph_params *p);

/* Cells per axis of the search grid for these parameters (host only).
 * Periodic axis: n = floor(cf (hi-lo) / (2h)), edge (hi-lo)/n, n >= 2 cf + 1 required.
 * Bounded axis:  n = ceil(cf (hi-lo) / (2h)), edge 2h / cf.  n <= 1024 per axis. */
sph_status sph_grid_dims(const sph_params *p, int32_t dims[3]);

/* Device workspace needed for n particles (host only, no device access).  The
 * workspace must be 256-byte aligned and stay alive and untouched until sph_destroy. */
sph_status sph_workspace_bytes(const sph_params *p, int64_t n, size_t *bytes);

/* Validate parameters, take the workspace and stream, and upload the per-instance
 * tables.  n >= 1.  Synchronises the stream once.  *out is set only on SPH_OK. */
sph_status sph_create(const sph_params *p, int64_t n, void *workspace, size_t ws_bytes,
                      void *hip_stream, sph_sim **out);

/* Load particle state by id (x, v, omega: [3][n] doubles; species, kind: [n] uint8) and
 * evaluate density, pressure and accelerations at it: the evaluation that precedes the
 * first half-kick of velocity Verlet (Algorithm 1).  Inputs are read by enqueued kernels:
 * keep them alive until the stream reaches this point.  Also used to resume from a
 * checkpoint written by sph_read_fields. */
sph_status sph_init_particles(sph_sim *s, const double *x, const double *v,
                              const double *omega, const uint8_t *species,
                              const uint8_t *kind);

/* Advance nsteps >= 0 velocity-Verlet steps of size dt > 0 with walls turning at Omega
 * (rad per unit time, about the z axis through x = y = 0; ignored when there are no wall
 * particles).  Per step: half kick and drift (walls rotated exactly), cell list, the
 * collision step (if enabled), density and EOS, the pressure filter (if enabled), pair
 * forces and torques, closing half kick (Algorithm 1).  The collision step changes only
 * velocities, which the density and the filter do not read, so it is executed after them
 * with the same result.  The closing half kick is folded into the next step's opening
 * kick; reads apply it. */
sph_status sph_step(sph_sim *s, double dt, double Omega, int32_t nsteps);

/* Write the current fields by id; any pointer may be NULL to skip it.
 * x, v, omega, acc, alpha: [3][n] doubles; rho, P: [n] doubles.  v and omega are the
 * full-step values (pending half kick applied).  Returns the sticky device error, if
 * any, after synchronising the stream. */
sph_status sph_read_fields(sph_sim *s, double *x, double *v, double *omega, double *rho,
                           double *P, double *acc, double *alpha);

/* FP64 global sums over fluid particles (host output, synchronises):
 * out[0..2] = sum m v, out[3..5] = sum (m x × v + I omega), out[6] = kinetic + spin energy. */
sph_status sph_diagnostics(sph_sim *s, double out[7]);

/* Vortex diagnostic (the image analysis of Sec. 3: vortices are counted on the z = 0
 * section of the rotational-force intensity, the fifth term of Eq. 2).
 * sph_vortex_dims: pixels per row (nx) and rows (ny) of the image, squares of side dx over
 * [lo, hi) in x and y, n = ceil((hi - lo) / dx - 1e-9).  Host only.
 * sph_vortex_image: for the fluid particles with -dx <= z - z0 < dx (z taken periodic),
 * the intensity I = |sum over viscous neighbours j (walls included) of
 * 2 eta V_j F_ij (w_i + w_j) x r_ij| (FP64, from the current state and density), which is
 * the spin part of the viscous pair force per unit volume; image[iy][ix] = the largest I
 * in the pixel (0 if none).  Pixels with a positive value of at least theta times the
 * largest are on; labels[iy][ix] = the smallest pixel index iy nx + ix of the pixel's
 * 8-connected component of on pixels, -1 when off; *count (host) = the number of
 * components with at least min_pixels pixels.  image (double, nx ny), labels (int32,
 * nx ny) and scratch (int32, nx ny + 8, 8-byte aligned) are caller-owned device buffers
 * on the simulation's stream; the call synchronises.  SPH_E_INVALID for a missing
 * buffer, an unaligned scratch, non-finite z0 or theta, theta < 0 or min_pixels < 1;
 * SPH_E_STATE before init.  The labels and the count do not depend on the order of any
 * floating-point sum other than the intensities'. */
sph_status sph_vortex_dims(const sph_params *p, int32_t *nx, int32_t *ny);
sph_status sph_vortex_image(sph_sim *s, double z0, double theta, int32_t min_pixels,
                            double *image, int32_t *labels, int32_t *scratch, int32_t *count);

/* sph_vortex_image without the scratch argument, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid allocation).
 * It calls no hipMalloc, hipFree or other allocating routine: its scratch is a static
 * device array of the library, 2^20 + 8 int32 (4 MiB) per device, held by each device the
 * library runs on until the process ends.  image and labels stay caller-owned as in
 * sph_vortex_image; images of more than 2^20 pixels (nx ny from sph_vortex_dims) return
 * SPH_E_CAPACITY before anything is enqueued.  Results equal sph_vortex_image's.  Calls
 * on one device share that array, so two calls that overlap on one device (two host
 * threads, or two streams without ordering) race; calls one after the other are safe, the
 * array is cleared at the start of each call. */
sph_status sph_vortex_image_noalloc(sph_sim *s, double z0, double theta, int32_t min_pixels,
                                    double *image, int32_t *labels, int32_t *count);

/* Cell list of the last neighbour search (device outputs).  key_by_id[n]: Morton code of
 * the particle's cell (bit 0 = x); perm[n]: particle ids sorted by (key, id);
 * cell_start[ncell + 1]: CSR offsets of the cells taken in Morton order, ncell being the
 * product of sph_grid_dims.  Any pointer may be NULL. */
sph_status sph_debug_cells(sph_sim *s, uint32_t *key_by_id, uint32_t *perm,
                           uint32_t *cell_start);

/* Neighbour sets of the last search as CSR by id, columns ascending (device outputs
 * row_ptr[n+1], cols[cap]).  *nnz (host) receives the entry count; SPH_E_CAPACITY if it
 * exceeds cap (row_ptr is then still valid).  Synchronises.  Meant for small n. */
sph_status sph_debug_neighbors(sph_sim *s, int64_t *row_ptr, int32_t *cols, int64_t cap,
                               int64_t *nnz);

/* The neighbour sets the FP32-mixed brick sweeps used at the last evaluation (Sec. 2.3
 * neighbour particle lists), in the CSR of sph_debug_neighbors (same outputs, capacity
 * rule and synchronisation): for the particles of bricks the density sweep staged, the hit
 * masks it wrote and the pressure filter and the force sweep replay, decoded; for the
 * particles it evaluated one by one, their FP64 cell walk.  The masks come from a single
 * precision test in expanded form, |c|^2 - 2 c.t < (2h)^2 - |t|^2 on positions relative to
 * the brick centre in units of h, so a pair may differ from the FP64 test only when
 * |r^2 - (2h)^2| <= 1e-5 (2h)^2.  SPH_E_STATE before init, on the FP64 path, or when the
 * last density sweep was not the brick sweep.  Meant for small n. */
sph_status sph_debug_masks(sph_sim *s, int64_t *row_ptr, int32_t *cols, int64_t cap,
                           int64_t *nnz);

/* Near neighbours the brick density sweep listed for the collision step of Algorithm 1
 * (pairs closer than coll_alpha dx, listed with a relative margin of 1e-4 on the squared
 * distance; the step then tests each listed pair exactly in FP64).  Device outputs by id:
 * count[n] (uint8: 0..6 listed, 255: not listed, the step walks the cells) and ids[n][6]
 * (int32: the listed neighbours' ids ascending, -1 in unused places).  Synchronises.
 * SPH_E_STATE when the collision step is off, before init, or when the last density sweep
 * was not the brick sweep. */
sph_status sph_debug_near(sph_sim *s, uint8_t *count, int32_t *ids);

sph_status sph_set_tuning(sph_sim *s, const sph_tuning *t);
sph_status sph_get_tuning(const sph_sim *s, sph_tuning *t);

/* Per-kernel timing (measurement support, not part of the method).  Between begin and
 * end, steps are launched eagerly with a HIP event recorded on the library's stream
 * before and after each kernel group; end synchronises and returns, for each group, the
 * summed milliseconds over the profiled steps (ms[SPH_K_COUNT]) and the step count.
 * Events are created on first use and kept until destroy. */
typedef enum {
    SPH_K_KEYS = 0,     /* kick, drift, cell key and histogram                            */
    SPH_K_SCAN = 1,     /* exclusive scan of the cell histogram                           */
    SPH_K_SCATTER = 2,  /* counting-sort scatter                                          */
    SPH_K_REORDER = 3,  /* in-cell ordering and state move                                */
    SPH_K_DENSITY = 4,  /* density, EOS                                                   */
    SPH_K_FORCE = 5,    /* pair forces and torques                                        */
    SPH_K_COLLIDE = 6,  /* collision step (when enabled)                                   */
    SPH_K_FILTER = 7,   /* pressure filter (when enabled)                                  */
    SPH_K_COUNT = 8
} sph_kernel_group;
sph_status sph_profile_begin(sph_sim *s);
sph_status sph_profile_end(sph_sim *s, double ms[SPH_K_COUNT], int32_t *nsteps);
sph_status sph_batch_profile_begin(sph_batch *b);
sph_status sph_batch_profile_end(sph_batch *b, double ms[SPH_K_COUNT], int32_t *nsteps);

/* Wait for the stream and return the sticky device error (then cleared). */
sph_status sph_sync(sph_sim *s);

const char *sph_status_str(sph_status st);
/* Text of the last error on this handle ("" if none); valid until the next call. */
const char *sph_last_error(const sph_sim *s);
/* Release the handle (host memory only; the workspace stays the caller's). */
void sph_destroy(sph_sim *s);

/* ---------------------------------------------------------------------------------
 * Ensembles: n_inst independent instances of different sizes and parameters advanced
 * together, each kernel launch covering every instance.  All instances share the
 * precision.  Particle arrays are the instances' arrays concatenated (instance i owns
 * ids [off_i, off_i + counts[i]), off_i = sum of earlier counts), so x is [3][N] with
 * N = sum counts.  Steps are replayed from a captured hipGraph when the stream is not
 * the null stream.
 * --------------------------------------------------------------------------------- */
sph_status sph_batch_workspace_bytes(int32_t n_inst, const sph_params *params,
                                     const int64_t *counts, size_t *bytes);
sph_status sph_batch_create(int32_t n_inst, const sph_params *params, const int64_t *counts,
                            void *workspace, size_t ws_bytes, void *hip_stream,
                            sph_batch **out);
sph_status sph_batch_init(sph_batch *b, const double *x, const double *v, const double *omega,
                          const uint8_t *species, const uint8_t *kind);
/* Omega: host array [n_inst], the wall rate of each instance for these steps. */
sph_status sph_batch_step(sph_batch *b, double dt, const double *Omega, int32_t nsteps);
sph_status sph_batch_read_fields(sph_batch *b, double *x, double *v, double *omega,
                                 double *rho, double *P, double *acc, double *alpha);
/* out: host [n_inst][7], as sph_diagnostics per instance. */
sph_status sph_batch_diagnostics(sph_batch *b, double *out);
sph_status sph_batch_set_tuning(sph_batch *b, const sph_tuning *t);
sph_status sph_batch_sync(sph_batch *b);
const char *sph_batch_last_error(const sph_batch *b);
void sph_batch_destroy(sph_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* SPH4HE_H */
