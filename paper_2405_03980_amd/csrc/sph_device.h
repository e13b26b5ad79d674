// Device-side data layout of the SPH step: per-instance descriptors, workspace views and
// kernel launchers shared by the runtime (runtime.hip) and the kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace sph {

// Largest cell population the search walks; fuller cells raise the capacity error and
// are skipped, so that a collapsed state cannot turn a sweep into an O(N^2) loop.
constexpr int kMaxCell = 1024;
constexpr int kWave = 64;
constexpr int kDiagChunks = 64;  // diagnostics partial sums per instance

enum : uint32_t { ERR_NONFINITE = 1u, ERR_DOMAIN = 2u, ERR_CAPACITY = 4u, ERR_INPUT = 8u };
enum { KIND_FLUID = 0, KIND_WALL_INNER = 1, KIND_WALL_OUTER = 2 };
enum { KERNEL_CUBIC = 0, KERNEL_WENDLAND = 1 };

// Everything a kernel needs to know about one instance.  Lives in device memory; all
// lanes of a wavefront always belong to the same instance (particle ranges are padded to
// whole wavefronts), so the fields are read with scalar loads.
struct InstDesc {
    double lo[3], hi[3], L[3], halfL[3], edge[3];
    double h, inv_h, cut2;      // cut2 = (2h)^2: pair test r^2 < cut2
    double wnorm;               // kernel normalisation constant
    double W0;                  // W(0)
    double mass[2], inertia[2]; // per species; inertia = kappa_I m dx^2
    double inv_mass[2], inv_inertia[2];
    double rho0, B;             // Tait: P = B ((rho/rho0)^7 - 1)
    double eta, sigma_T, C_l;
    double coll_rc, coll_rc2;   // collision step: distance coll_alpha dx and its square
    double coll_e1;             // 1 + restitution
    double rxy2;                // cylinder geometry: x^2 + y^2 of every particle stays within
                                // rxy2 (the inscribed cylinder about the z axis widened by
                                // 2h); +inf for the other geometries
    int32_t pfilter, coll;      // pressure filter on; collision step on
    int32_t n[3], periodic[3];
    int32_t cf, kernel;
    uint32_t cell_off, n_cells; // this instance's cells in the global cell range
    uint32_t part_off, n_part;  // this instance's particles in the global particle range
    uint32_t wave_off, n_waves; // this instance's wavefronts in particle-parallel launches
};

// Per-instance values that change between step calls (wall rotation).
struct StepParams {
    double cosw, sinw, Omega, pad;
};

// Device views of the workspace.  Particle arrays are in cell-sorted order; "cur" selects
// the buffer holding the current state of the double-buffered arrays.
struct DevState {
    int precision;          // 0: FP64, 1: FP32-mixed
    int n_inst;
    int cur;                // buffer (0/1) holding the current state
    uint32_t N, C, n_waves; // particles, cells, wavefronts over all instances
    int any_filter;         // some instance has the pressure filter on
    int any_coll;           // some instance has the collision step on
    InstDesc *desc;
    StepParams *steptab;
    double *x[2], *v[2], *w[2];   // [3][N] each
    uint32_t *id[2];              // global particle id
    uint8_t *sk[2];               // bit 0 species, bits 1-2 kind
    void *acc, *alpha;            // [3][N], float or double
    void *aux;                    // [N][4]: V = m/rho, P/rho^2, 1/rho^2, V/S (0 if S = 0)
    void *rhoP;                   // [N][2]: rho, P (P before the pressure filter)
    void *pf;                     // [N]: filtered pressure (instances with the filter on)
    uint8_t *cflag;               // [N]: near neighbours listed by the brick density sweep
                                  // (0..kNearCap, kNearOverflow: walk the cells)
    uint32_t *nearq;              // [N][kNearCap]: their sorted indices
    uint32_t *key, *slot, *tmp, *pcell;
    uint32_t *idt;                // id of the particle at each scatter position (= id[tmp[.]])
    uint32_t *bframe;             // [n_bricks][128]: slot first indices, inclusive slot-count prefix
    uint32_t *count, *start, *bsum;
    uint32_t *cell_xyz;           // global cell rank -> packed (cx | cy << 10 | cz << 20)
    uint32_t *rank_of_lin;        // cell_off + linear cell index -> global cell rank
    uint32_t *err;
    double *diag_part;            // [n_inst][kDiagChunks][14]
    double *diag_out;             // [n_inst][7]
    // Bricks of 2x2x2 cells (instances with one cell per interaction radius):
    // packed (bx | by << 10 | bz << 20) and instance index, in Morton order per instance.
    uint32_t *brick_xyz, *brick_inst;
    uint32_t n_bricks;
    // Neighbour hit masks of the brick sweeps, kMaskSlots per particle: the density sweep
    // records the windows of candidate tests, the pressure filter and the force sweep
    // replay them.
    uint64_t *masks;
    uint32_t xcd_run;  // consecutive bricks per XCD in the brick sweeps' workgroup order
};

constexpr int kMaskSlots = 16;
// Near neighbours (within the collision distance) listed per particle for the collision step.
constexpr int kNearCap = 6;
constexpr int kNearOverflow = 255;

// Sweep implementations: one thread per particle walking its own cell stencil, or one
// workgroup per 2x2x2-cell brick with the brick's neighbourhood staged in LDS and the
// neighbour test done by wave ballots over candidates.  (Value 2 is not used.)
enum { SWEEP_THREAD = 1, SWEEP_CAND = 3 };

struct Launch {
    int bs_density = 256, bs_force = 256, bs_stream = 256;
    int sweep = SWEEP_CAND;  // brick sweeps when every instance allows them (FP32-mixed, cf = 1)
    int list_targets = 32;   // targets per round of the brick density sweep: 16 or 32
};
constexpr uint32_t kDefaultXcdRun = 8;

// Launchers (kernels.hip).  All enqueue on `st` and return hipGetLastError().
// mode 0: load/initial evaluation (no kick or drift); mode 1: time step.
hipError_t launch_keys(const DevState &d, const Launch &L, hipStream_t st, int mode,
                       double kick, double dt);
hipError_t launch_scan(const DevState &d, const Launch &L, hipStream_t st);
hipError_t launch_scatter(const DevState &d, const Launch &L, hipStream_t st);
hipError_t launch_reorder(const DevState &d, const Launch &L, hipStream_t st, int mode,
                          double kick, double dt);
hipError_t launch_density(const DevState &d, const Launch &L, hipStream_t st);
hipError_t launch_force(const DevState &d, const Launch &L, hipStream_t st);
// Pressure filter after launch_density, for the instances that have it on.
hipError_t launch_filter(const DevState &d, const Launch &L, hipStream_t st);
// Collision step on the current (drifted, cell-ordered) state, for the instances that
// have it on; after launch_density (whose brick sweep lists the near neighbours); uses the
// other velocity buffer as scratch.
hipError_t launch_collide(const DevState &d, const Launch &L, hipStream_t st);
hipError_t launch_load(const DevState &d, const Launch &L, hipStream_t st, const double *x,
                       const double *v, const double *w, const uint8_t *species,
                       const uint8_t *kind);
hipError_t launch_read(const DevState &d, const Launch &L, hipStream_t st, double pend,
                       double *x, double *v, double *w, double *rho, double *P, double *acc,
                       double *alpha);
hipError_t launch_diag(const DevState &d, const Launch &L, hipStream_t st, double pend);
hipError_t launch_debug_keys(const DevState &d, const Launch &L, hipStream_t st,
                             uint32_t *key_by_id, uint32_t *perm);
hipError_t launch_debug_nbr(const DevState &d, const Launch &L, hipStream_t st, int phase,
                            int64_t *row_ptr, int32_t *cols);
// The neighbour sets of the last brick density sweep (its decoded hit masks; the FP64 walk
// where it evaluated per particle), same two phases and CSR as launch_debug_nbr.
hipError_t launch_debug_masks(const DevState &d, hipStream_t st, int phase, int64_t *row_ptr,
                              int32_t *cols);
// The near-neighbour lists of the last brick density sweep (collision step), by id.
hipError_t launch_debug_near(const DevState &d, const Launch &L, hipStream_t st, uint8_t *count,
                             int32_t *ids);
hipError_t launch_fill_u32(uint32_t *p, uint32_t value, size_t n, hipStream_t st);

// Vortex diagnostic of one instance (the first): section z0, pixel grid nx x ny of side
// dx from (lox, loy), z period Lz; pend = half the last step's dt (the pending half kick).
struct VortexArgs {
    double z0, Lz, dx, lox, loy, pend;
    int32_t nx, ny;
};
// masks: the brick density sweep's masks hold the neighbours of the current positions
// (FP32-mixed path), so the brick intensity kernel may replay them.
hipError_t launch_vortex_intensity(const DevState &d, const Launch &L, hipStream_t st,
                                   const VortexArgs &a, bool masks, unsigned long long *img,
                                   unsigned long long *vmax);
hipError_t launch_vortex_label_init(hipStream_t st, const unsigned long long *img,
                                    const unsigned long long *vmax, double theta, uint32_t n,
                                    int32_t *lab);
hipError_t launch_vortex_relax(hipStream_t st, int32_t *lab, int nx, int ny, uint32_t *changed);
hipError_t launch_vortex_count(hipStream_t st, const int32_t *lab, int32_t *size, uint32_t n,
                               int32_t min_pixels, int32_t *count);

}  // namespace sph
