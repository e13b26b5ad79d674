// Host side of the C ABI (include/sph4he.h): parameter validation, workspace carving,
// per-instance tables, step sequencing, hipGraph replay and error reporting.
// A single instance (sph_sim) is an ensemble of one (sph_batch).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "sph4he.h"
#include "sph_device.h"

using namespace sph;

namespace {

constexpr size_t kAlign = 256;
constexpr uint32_t kMaxParticles = 1u << 30;

// ------------------------------------------------------------ kernels (host copy) ---
// The runtime needs W on the host only for the lattice normalisation of the default
// particle mass.

double host_W(int kernel, double h, double r)
{
    double q = r / h;
    if (q >= 2.0) return 0.0;
    if (kernel == KERNEL_CUBIC) {
        double s = 1.0 / (M_PI * h * h * h);
        if (q < 1.0) return s * (1.0 - 1.5 * q * q + 0.75 * q * q * q);
        double t = 2.0 - q;
        return s * 0.25 * t * t * t;
    }
    double s = 21.0 / (16.0 * M_PI * h * h * h);
    double t = 1.0 - 0.5 * q;
    return s * t * t * t * t * (2.0 * q + 1.0);
}

double kernel_norm(int kernel, double h)
{
    return kernel == KERNEL_CUBIC ? 1.0 / (M_PI * h * h * h) : 21.0 / (16.0 * M_PI * h * h * h);
}

// dx^3 times the sum of W over the infinite cubic lattice of spacing dx (origin
// included): the density of a perfect lattice of unit masses.
double lattice_norm(int kernel, double h, double dx)
{
    int m = (int)ceil(2.0 * h / dx) + 1;
    double s = 0.0;
    for (int a = -m; a <= m; a++)
        for (int b = -m; b <= m; b++)
            for (int c = -m; c <= m; c++)
                s += host_W(kernel, h, dx * sqrt((double)(a * a + b * b + c * c)));
    return s * dx * dx * dx;
}

uint32_t morton3_host(uint32_t x, uint32_t y, uint32_t z)
{
    uint32_t k = 0;
    for (int b = 0; b < 10; b++) {
        k |= ((x >> b) & 1u) << (3 * b);
        k |= ((y >> b) & 1u) << (3 * b + 1);
        k |= ((z >> b) & 1u) << (3 * b + 2);
    }
    return k;
}

bool is_periodic(int geometry, int a)
{
    if (geometry == SPH_GEOM_PERIODIC_BOX) return true;
    if (geometry == SPH_GEOM_CYLINDER_Z) return a == 2;
    return false;
}

sph_status grid_of(const sph_params *p, int32_t n[3], double edge[3], std::string &msg)
{
    double two_h = 2.0 * p->h;
    for (int a = 0; a < 3; a++) {
        double L = p->hi[a] - p->lo[a];
        if (!(L > 0.0) || !isfinite(L)) { msg = "hi must exceed lo on every axis"; return SPH_E_INVALID; }
        double cells = (double)p->cell_factor * L / two_h;
        if (is_periodic(p->geometry, a)) {
            double nf = floor(cells);
            if (nf < 2.0 * p->cell_factor + 1.0) {
                msg = "periodic axis shorter than (2 cell_factor + 1) cells of edge 2h/cell_factor";
                return SPH_E_INVALID;
            }
            if (nf > 1024.0) { msg = "more than 1024 cells along an axis"; return SPH_E_INVALID; }
            n[a] = (int32_t)nf;
            edge[a] = L / (double)n[a];
        } else {
            double nf = ceil(cells);
            if (nf < 1.0) nf = 1.0;
            if (nf > 1024.0) { msg = "more than 1024 cells along an axis"; return SPH_E_INVALID; }
            n[a] = (int32_t)nf;
            edge[a] = two_h / (double)p->cell_factor;
        }
    }
    return SPH_OK;
}

sph_status validate(const sph_params *p, std::string &msg)
{
    if (!p) { msg = "params is NULL"; return SPH_E_INVALID; }
    if (p->abi_version != SPH_ABI_VERSION) { msg = "abi_version mismatch"; return SPH_E_INVALID; }
    if (p->kernel != SPH_KERNEL_CUBIC && p->kernel != SPH_KERNEL_WENDLAND_C2) { msg = "unknown kernel"; return SPH_E_INVALID; }
    if (p->precision != SPH_FP64 && p->precision != SPH_FP32_MIXED) { msg = "unknown precision"; return SPH_E_INVALID; }
    if (p->geometry < SPH_GEOM_PERIODIC_BOX || p->geometry > SPH_GEOM_OPEN) { msg = "unknown geometry"; return SPH_E_INVALID; }
    if (!(p->dx > 0.0) || !isfinite(p->dx)) { msg = "dx must be positive"; return SPH_E_INVALID; }
    if (!(p->h > 0.0) || !isfinite(p->h)) { msg = "h must be positive"; return SPH_E_INVALID; }
    if (!(p->rho0 > 0.0) || !isfinite(p->rho0)) { msg = "rho0 must be positive"; return SPH_E_INVALID; }
    if (!(p->c0 >= 0.0) || !isfinite(p->c0)) { msg = "c0 must be >= 0"; return SPH_E_INVALID; }
    if (p->gamma != 7.0) { msg = "only the Tait exponent gamma = 7 is implemented"; return SPH_E_UNSUPPORTED; }
    for (int s = 0; s < 2; s++)
        if (!isfinite(p->mass[s])) { msg = "mass must be finite"; return SPH_E_INVALID; }
    if (!(p->eta >= 0.0) || !isfinite(p->eta)) { msg = "eta must be >= 0"; return SPH_E_INVALID; }
    if (!isfinite(p->sigma_T) || !isfinite(p->C_l)) { msg = "sigma_T and C_l must be finite"; return SPH_E_INVALID; }
    if (!(p->kappa_I > 0.0) || !isfinite(p->kappa_I)) { msg = "kappa_I must be positive"; return SPH_E_INVALID; }
    if (p->cell_factor < 1 || p->cell_factor > 4) { msg = "cell_factor must be in 1..4"; return SPH_E_INVALID; }
    if (p->pressure_filter != 0 && p->pressure_filter != 1) { msg = "pressure_filter must be 0 or 1"; return SPH_E_INVALID; }
    if (!(p->coll_alpha >= 0.0) || !isfinite(p->coll_alpha) || !(p->coll_alpha * p->dx < 2.0 * p->h)) {
        msg = "coll_alpha must satisfy 0 <= coll_alpha dx < 2h";
        return SPH_E_INVALID;
    }
    if (!(p->coll_e >= 0.0 && p->coll_e <= 1.0)) { msg = "coll_e must be in [0, 1]"; return SPH_E_INVALID; }
    for (int a = 0; a < 3; a++)
        if (!isfinite(p->lo[a]) || !isfinite(p->hi[a])) { msg = "lo/hi must be finite"; return SPH_E_INVALID; }
    int32_t n[3];
    double e[3];
    return grid_of(p, n, e, msg);
}

// ------------------------------------------------------------ workspace layout ------

struct Carver {
    char *base = nullptr;
    size_t off = 0;
    template <class T>
    T *take(size_t count)
    {
        off = (off + kAlign - 1) / kAlign * kAlign;
        T *p = base ? (T *)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

void carve(Carver &c, DevState &d, int n_inst, uint32_t N, uint32_t C, uint32_t NB, int precision,
           bool filter, bool coll)
{
    size_t rs = precision == SPH_FP64 ? sizeof(double) : sizeof(float);
    size_t n3 = 3 * (size_t)N;
    d.desc = c.take<InstDesc>(n_inst);
    d.steptab = c.take<StepParams>(n_inst);
    for (int b = 0; b < 2; b++) {
        d.x[b] = c.take<double>(n3);
        d.v[b] = c.take<double>(n3);
        d.w[b] = c.take<double>(n3);
        d.id[b] = c.take<uint32_t>(N);
        d.sk[b] = c.take<uint8_t>(N);
    }
    d.acc = c.take<char>(n3 * rs);
    d.alpha = c.take<char>(n3 * rs);
    d.aux = c.take<char>(4 * (size_t)N * rs);
    d.rhoP = c.take<char>(2 * (size_t)N * rs);
    d.pf = c.take<char>((filter ? (size_t)N : 1) * rs);
    d.cflag = c.take<uint8_t>(coll ? (size_t)N : 1);
    d.nearq = c.take<uint32_t>(coll ? (size_t)N * kNearCap : 1);
    d.key = c.take<uint32_t>(N);
    d.slot = c.take<uint32_t>(N);
    d.tmp = c.take<uint32_t>(N);
    d.idt = c.take<uint32_t>(N);
    d.pcell = c.take<uint32_t>(N);
    d.count = c.take<uint32_t>(C);
    d.start = c.take<uint32_t>((size_t)C + 1);
    d.bsum = c.take<uint32_t>(((size_t)C + 1023) / 1024 + 1);
    d.cell_xyz = c.take<uint32_t>(C);
    d.rank_of_lin = c.take<uint32_t>(C);
    d.err = c.take<uint32_t>(4);
    d.diag_part = c.take<double>((size_t)n_inst * kDiagChunks * 14);
    d.diag_out = c.take<double>((size_t)n_inst * 7);
    d.brick_xyz = c.take<uint32_t>(NB ? NB : 1);
    d.brick_inst = c.take<uint32_t>(NB ? NB : 1);
    d.n_bricks = NB;
    d.masks = c.take<uint64_t>((NB && precision == SPH_FP32_MIXED) ? (size_t)N * kMaskSlots : 1);
    d.bframe = c.take<uint32_t>((NB && precision == SPH_FP32_MIXED) ? (size_t)NB * 128 : 1);
}

struct Plan {
    std::vector<InstDesc> desc;
    uint32_t N = 0, C = 0, n_waves = 0;
    uint32_t n_bricks = 0;  // 0 unless every instance has cell_factor 1
    std::vector<uint32_t> bxyz, binst;  // the bricks: packed coordinates and instance
    bool any_filter = false, any_coll = false;
};

void brick_tables(const Plan &pl, std::vector<uint32_t> &xyz, std::vector<uint32_t> &inst);

sph_status plan(int32_t n_inst, const sph_params *params, const int64_t *counts, Plan &pl,
                std::string &msg)
{
    if (n_inst < 1 || n_inst > 65536) { msg = "n_inst must be in 1..65536"; return SPH_E_INVALID; }
    if (!params || !counts) { msg = "params/counts is NULL"; return SPH_E_INVALID; }
    pl.desc.assign(n_inst, InstDesc{});
    uint64_t N = 0, C = 0, W = 0;
    for (int i = 0; i < n_inst; i++) {
        const sph_params *p = params + i;
        sph_status st = validate(p, msg);
        if (st != SPH_OK) { msg = "instance " + std::to_string(i) + ": " + msg; return st; }
        if (p->precision != params[0].precision) { msg = "all instances must share the precision"; return SPH_E_INVALID; }
        if (counts[i] < 1) { msg = "every instance needs at least one particle"; return SPH_E_INVALID; }
        InstDesc &d = pl.desc[i];
        int32_t n[3];
        double edge[3];
        grid_of(p, n, edge, msg);
        for (int a = 0; a < 3; a++) {
            d.lo[a] = p->lo[a];
            d.hi[a] = p->hi[a];
            d.L[a] = p->hi[a] - p->lo[a];
            // bounded axes: an infinite half period disables the minimum image
            d.halfL[a] = is_periodic(p->geometry, a) ? 0.5 * d.L[a] : INFINITY;
            d.edge[a] = edge[a];
            d.n[a] = n[a];
            d.periodic[a] = is_periodic(p->geometry, a) ? 1 : 0;
        }
        d.h = p->h;
        d.inv_h = 1.0 / p->h;
        d.cut2 = (2.0 * p->h) * (2.0 * p->h);
        d.wnorm = kernel_norm(p->kernel, p->h);
        d.W0 = host_W(p->kernel, p->h, 0.0);
        double dflt = p->rho0 * p->dx * p->dx * p->dx / lattice_norm(p->kernel, p->h, p->dx);
        for (int s = 0; s < 2; s++) {
            d.mass[s] = p->mass[s] > 0.0 ? p->mass[s] : dflt;
            d.inertia[s] = p->kappa_I * d.mass[s] * p->dx * p->dx;
            d.inv_mass[s] = 1.0 / d.mass[s];
            d.inv_inertia[s] = 1.0 / d.inertia[s];
        }
        d.rho0 = p->rho0;
        d.B = p->rho0 * p->c0 * p->c0 / p->gamma;
        d.eta = p->eta;
        d.sigma_T = p->sigma_T;
        d.C_l = p->C_l;
        d.coll_rc = p->coll_alpha * p->dx;
        d.coll_rc2 = d.coll_rc * d.coll_rc;
        d.coll_e1 = 1.0 + p->coll_e;
        // the cylinder about the z axis inscribed in the box's x-y extent, widened by the
        // kernel support 2h (fluid pressed into the wall layers may pass the outermost one
        // by a fraction of dx): no particle of a cylinder instance may leave it, so bricks
        // wholly outside it are left out of the brick sweeps
        d.rxy2 = INFINITY;
        if (p->geometry == SPH_GEOM_CYLINDER_Z) {
            const double r = fmin(fmin(-p->lo[0], p->hi[0]), fmin(-p->lo[1], p->hi[1]));
            if (r > 0.0) d.rxy2 = (r + 2.0 * p->h) * (r + 2.0 * p->h);
        }
        d.pfilter = p->pressure_filter;
        d.coll = p->coll_alpha > 0.0 ? 1 : 0;
        pl.any_filter = pl.any_filter || d.pfilter;
        pl.any_coll = pl.any_coll || d.coll;
        d.cf = p->cell_factor;
        d.kernel = p->kernel;
        uint64_t nc = (uint64_t)n[0] * n[1] * n[2];
        d.cell_off = (uint32_t)C;
        d.n_cells = (uint32_t)nc;
        d.part_off = (uint32_t)N;
        d.n_part = (uint32_t)counts[i];
        d.wave_off = (uint32_t)W;
        d.n_waves = (uint32_t)((counts[i] + kWave - 1) / kWave);
        N += (uint64_t)counts[i];
        C += nc;
        W += d.n_waves;
        if (N > kMaxParticles) { msg = "too many particles (max 2^30)"; return SPH_E_INVALID; }
        if (C > (1ull << 31)) { msg = "too many cells"; return SPH_E_INVALID; }
    }
    pl.N = (uint32_t)N;
    pl.C = (uint32_t)C;
    pl.n_waves = (uint32_t)W;
    uint64_t NB = 0;
    bool bricks = true;
    for (const InstDesc &d : pl.desc) {
        if (d.cf != 1) bricks = false;
        NB += (uint64_t)((d.n[0] + 1) / 2) * ((d.n[1] + 1) / 2) * ((d.n[2] + 1) / 2);
    }
    pl.n_bricks = bricks ? (uint32_t)NB : 0u;
    if (pl.n_bricks) {
        brick_tables(pl, pl.bxyz, pl.binst);
        pl.n_bricks = (uint32_t)pl.bxyz.size();
    }
    return SPH_OK;
}

// Morton order of each instance's cells: rank_of_lin[cell_off + lin] = global rank and
// its inverse as packed coordinates.
void cell_tables(const Plan &pl, std::vector<uint32_t> &rank_of_lin, std::vector<uint32_t> &xyz)
{
    rank_of_lin.resize(pl.C);
    xyz.resize(pl.C);
    std::vector<uint64_t> keys;
    for (const InstDesc &d : pl.desc) {
        keys.resize(d.n_cells);
        size_t q = 0;
        for (int z = 0; z < d.n[2]; z++)
            for (int y = 0; y < d.n[1]; y++)
                for (int x = 0; x < d.n[0]; x++, q++)
                    keys[q] = ((uint64_t)morton3_host(x, y, z) << 32) | (uint64_t)q;
        std::sort(keys.begin(), keys.end());
        for (uint32_t r = 0; r < d.n_cells; r++) {
            uint32_t lin = (uint32_t)(keys[r] & 0xffffffffu);
            uint32_t x = lin % (uint32_t)d.n[0];
            uint32_t y = (lin / (uint32_t)d.n[0]) % (uint32_t)d.n[1];
            uint32_t z = lin / ((uint32_t)d.n[0] * (uint32_t)d.n[1]);
            rank_of_lin[d.cell_off + lin] = d.cell_off + r;
            xyz[d.cell_off + r] = x | (y << 10) | (z << 20);
        }
    }
}

// Bricks of 2x2x2 cells, Morton order within each instance.
void brick_tables(const Plan &pl, std::vector<uint32_t> &xyz, std::vector<uint32_t> &inst)
{
    xyz.clear();
    inst.clear();
    if (!pl.n_bricks) return;
    std::vector<uint64_t> keys;
    for (size_t i = 0; i < pl.desc.size(); i++) {
        const InstDesc &d = pl.desc[i];
        const uint32_t nb[3] = {(uint32_t)(d.n[0] + 1) / 2, (uint32_t)(d.n[1] + 1) / 2, (uint32_t)(d.n[2] + 1) / 2};
        keys.clear();
        for (uint32_t z = 0; z < nb[2]; z++)
            for (uint32_t y = 0; y < nb[1]; y++)
                for (uint32_t x = 0; x < nb[0]; x++)
                    keys.push_back(((uint64_t)morton3_host(x, y, z) << 32) | (x | (y << 10) | (z << 20)));
        std::sort(keys.begin(), keys.end());
        const double ex = 2.0 * d.edge[0], ey = 2.0 * d.edge[1];
        for (uint64_t k : keys) {
            const uint32_t v = (uint32_t)(k & 0xffffffffu);
            // a brick whose x-y footprint lies wholly outside the cylinder holds no particle
            const double x0 = d.lo[0] + (double)(v & 1023u) * ex;
            const double y0 = d.lo[1] + (double)((v >> 10) & 1023u) * ey;
            const double cx = fmin(fmax(0.0, x0), x0 + ex), cy = fmin(fmax(0.0, y0), y0 + ey);
            if (cx * cx + cy * cy > d.rxy2) continue;
            xyz.push_back(v);
            inst.push_back((uint32_t)i);
        }
    }
}

sph_status hip_fail(hipError_t e, std::string &msg, const char *what)
{
    msg = std::string(what) + ": " + hipGetErrorString(e);
    return SPH_E_HIP;
}

}  // namespace

// ------------------------------------------------------------ handles ---------------

struct GraphCache {
    hipGraphExec_t exec = nullptr;
    double dt = 0.0;
    int parity = -1;
};

// HIP events bracketing each kernel group of profiled steps.
struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> pool;
    std::vector<int> tag;  // kernel group measured from event k to event k + 1; -1: none
    size_t used = 0;
    int steps = 0;
};

struct sph_batch {
    DevState ds{};
    Launch L;
    Profiler prof;
    hipStream_t stream = nullptr;
    int n_inst = 0;
    std::vector<InstDesc> desc;
    std::vector<sph_params> params;  // as given at creation
    std::vector<StepParams> steptab;
    bool loaded = false;
    bool masks_current = false;  // the last density launch was the brick sweep (its masks
                                 // hold the neighbours of the current positions)
    double pending_dt = 0.0;  // closing half kick of this dt still to apply
    bool use_graph = true;
    int device = 0;           // device current at creation (the workspace's)
    GraphCache graphs[2];
    std::string err;
    uint32_t host_err = 0;
};

struct sph_sim {
    sph_batch *b = nullptr;
};

namespace {

void drop_graphs(sph_batch *b)
{
    for (GraphCache &g : b->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = GraphCache{};
    }
}

sph_status check_launch(sph_batch *b, hipError_t e, const char *what)
{
    if (e != hipSuccess) return hip_fail(e, b->err, what);
    return SPH_OK;
}

// Records a profiling event that closes the previous group and opens group `tag`.
sph_status prof_mark(sph_batch *b, int tag)
{
    Profiler &P = b->prof;
    if (!P.on) return SPH_OK;
    if (P.used == P.pool.size()) {
        hipEvent_t ev;
        hipError_t e = hipEventCreate(&ev);
        if (e != hipSuccess) return hip_fail(e, b->err, "event create");
        P.pool.push_back(ev);
        P.tag.push_back(-1);
    }
    hipError_t e = hipEventRecord(P.pool[P.used], b->stream);
    if (e != hipSuccess) return hip_fail(e, b->err, "event record");
    P.tag[P.used] = tag;
    P.used++;
    return SPH_OK;
}

// One velocity Verlet step: opening kick + drift, cell list, density, pressure filter,
// collision step, forces (the filter and the collision step for instances that have
// them on; mode 0, the evaluation at load, has no collision step).
sph_status enqueue_step(sph_batch *b, int mode, double kick, double dt)
{
    DevState &d = b->ds;
    hipStream_t st = b->stream;
    sph_status s;
    if ((s = prof_mark(b, SPH_K_KEYS)) != SPH_OK) return s;
    if ((s = check_launch(b, launch_keys(d, b->L, st, mode, kick, dt), "keys")) != SPH_OK) return s;
    if ((s = prof_mark(b, SPH_K_SCAN)) != SPH_OK) return s;
    if ((s = check_launch(b, launch_scan(d, b->L, st), "scan")) != SPH_OK) return s;
    if ((s = prof_mark(b, SPH_K_SCATTER)) != SPH_OK) return s;
    if ((s = check_launch(b, launch_scatter(d, b->L, st), "scatter")) != SPH_OK) return s;
    if ((s = prof_mark(b, SPH_K_REORDER)) != SPH_OK) return s;
    if ((s = check_launch(b, launch_reorder(d, b->L, st, mode, kick, dt), "reorder")) != SPH_OK) return s;
    d.cur ^= 1;
    if ((s = prof_mark(b, SPH_K_DENSITY)) != SPH_OK) return s;
    if ((s = check_launch(b, launch_density(d, b->L, st), "density")) != SPH_OK) return s;
    b->masks_current = d.precision != 0 && b->L.sweep == SWEEP_CAND && d.n_bricks != 0;
    if (d.any_filter) {
        if ((s = prof_mark(b, SPH_K_FILTER)) != SPH_OK) return s;
        if ((s = check_launch(b, launch_filter(d, b->L, st), "pressure filter")) != SPH_OK) return s;
    }
    // The collision step changes velocities only, which neither the density nor the
    // filter reads: after them it gives the same state as before them, and the brick
    // density sweep has flagged its candidates by then.
    if (mode == 1 && d.any_coll) {
        if ((s = prof_mark(b, SPH_K_COLLIDE)) != SPH_OK) return s;
        if ((s = check_launch(b, launch_collide(d, b->L, st), "collide")) != SPH_OK) return s;
    }
    if ((s = prof_mark(b, SPH_K_FORCE)) != SPH_OK) return s;
    if ((s = check_launch(b, launch_force(d, b->L, st), "force")) != SPH_OK) return s;
    if ((s = prof_mark(b, -1)) != SPH_OK) return s;
    if (b->prof.on) b->prof.steps++;
    return SPH_OK;
}

sph_status profile_begin(sph_batch *b)
{
    if (!b->loaded) { b->err = "profile before init"; return SPH_E_STATE; }
    b->prof.on = true;
    b->prof.used = 0;
    b->prof.steps = 0;
    return SPH_OK;
}

sph_status profile_end(sph_batch *b, double ms[SPH_K_COUNT], int32_t *nsteps)
{
    if (!ms || !nsteps) { b->err = "NULL output"; return SPH_E_INVALID; }
    Profiler &P = b->prof;
    if (!P.on) { b->err = "profile_end without profile_begin"; return SPH_E_STATE; }
    P.on = false;
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, b->err, "sync");
    for (int k = 0; k < SPH_K_COUNT; k++) ms[k] = 0.0;
    for (size_t k = 0; k + 1 < P.used; k++) {
        if (P.tag[k] < 0) continue;
        float t = 0.0f;
        e = hipEventElapsedTime(&t, P.pool[k], P.pool[k + 1]);
        if (e != hipSuccess) return hip_fail(e, b->err, "elapsed time");
        ms[P.tag[k]] += (double)t;
    }
    *nsteps = P.steps;
    P.used = 0;
    P.steps = 0;
    return SPH_OK;
}

sph_status status_of_flags(uint32_t f, std::string &msg)
{
    if (f & ERR_INPUT) { msg = "invalid species/kind values in the particle input"; return SPH_E_INVALID; }
    if (f & ERR_NONFINITE) { msg = "non-finite value in the particle state"; return SPH_E_NONFINITE; }
    if (f & ERR_DOMAIN) {
        msg = "a particle left the cell grid along a bounded axis, or the cylinder of a cylinder instance";
        return SPH_E_DOMAIN;
    }
    if (f & ERR_CAPACITY) { msg = "a cell holds more particles than the search supports"; return SPH_E_CAPACITY; }
    return SPH_OK;
}

sph_status batch_sync(sph_batch *b)
{
    uint32_t f = 0;
    hipError_t e = hipMemcpyAsync(&f, b->ds.err, sizeof(uint32_t), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, b->err, "sync");
    if (f) {
        e = launch_fill_u32(b->ds.err, 0u, 1, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return hip_fail(e, b->err, "clear error word");
        return status_of_flags(f, b->err);
    }
    return SPH_OK;
}

sph_status batch_step(sph_batch *b, double dt, const double *Omega, int32_t nsteps)
{
    if (!b->loaded) { b->err = "step before init"; return SPH_E_STATE; }
    if (!(dt > 0.0) || !isfinite(dt)) { b->err = "dt must be positive"; return SPH_E_INVALID; }
    if (nsteps < 0) { b->err = "nsteps must be >= 0"; return SPH_E_INVALID; }
    if (!Omega) { b->err = "Omega is NULL"; return SPH_E_INVALID; }
    for (int i = 0; i < b->n_inst; i++) {
        if (!isfinite(Omega[i])) { b->err = "Omega must be finite"; return SPH_E_INVALID; }
        b->steptab[i].cosw = cos(Omega[i] * dt);
        b->steptab[i].sinw = sin(Omega[i] * dt);
        b->steptab[i].Omega = Omega[i];
    }
    if (nsteps == 0) return SPH_OK;
    hipError_t e = hipMemcpyAsync(b->ds.steptab, b->steptab.data(), sizeof(StepParams) * b->n_inst,
                                  hipMemcpyHostToDevice, b->stream);
    if (e != hipSuccess) return hip_fail(e, b->err, "upload step table");
    int remaining = nsteps;
    sph_status s;
    if (b->pending_dt != dt) {
        if ((s = enqueue_step(b, 1, 0.5 * b->pending_dt + 0.5 * dt, dt)) != SPH_OK) return s;
        b->pending_dt = dt;
        remaining--;
    }
    if (b->use_graph && !b->prof.on && b->stream != nullptr && remaining >= 2) {
        GraphCache &g = b->graphs[b->ds.cur];
        if (!g.exec || g.dt != dt) {
            if (g.exec) { (void)hipGraphExecDestroy(g.exec); g.exec = nullptr; }
            hipGraph_t graph = nullptr;
            e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_fail(e, b->err, "begin capture");
            int cur0 = b->ds.cur;
            sph_status s1 = enqueue_step(b, 1, dt, dt);
            sph_status s2 = s1 == SPH_OK ? enqueue_step(b, 1, dt, dt) : s1;
            e = hipStreamEndCapture(b->stream, &graph);
            b->ds.cur = cur0;
            if (s2 != SPH_OK) { if (graph) (void)hipGraphDestroy(graph); return s2; }
            if (e != hipSuccess) return hip_fail(e, b->err, "end capture");
            e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) { g.exec = nullptr; return hip_fail(e, b->err, "instantiate graph"); }
            g.dt = dt;
            g.parity = cur0;
        }
        while (remaining >= 2) {
            e = hipGraphLaunch(g.exec, b->stream);
            if (e != hipSuccess) return hip_fail(e, b->err, "graph launch");
            remaining -= 2;
        }
    }
    while (remaining > 0) {
        if ((s = enqueue_step(b, 1, dt, dt)) != SPH_OK) return s;
        remaining--;
    }
    return SPH_OK;
}

// Pixel grid of the vortex image: squares of side dx over the x-y extent of the domain.
void vortex_grid(const sph_params &p, int32_t &nx, int32_t &ny)
{
    nx = (int32_t)std::ceil((p.hi[0] - p.lo[0]) / p.dx - 1e-9);
    ny = (int32_t)std::ceil((p.hi[1] - p.lo[1]) / p.dx - 1e-9);
}

}  // namespace


// ------------------------------------------------------------ C ABI -----------------

extern "C" {

const char *sph_status_str(sph_status st)
{
    switch (st) {
    case SPH_OK: return "ok";
    case SPH_E_INVALID: return "invalid argument";
    case SPH_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case SPH_E_HIP: return "HIP runtime error";
    case SPH_E_STATE: return "call out of order";
    case SPH_E_DOMAIN: return "particle left the cell grid";
    case SPH_E_NONFINITE: return "non-finite value";
    case SPH_E_UNSUPPORTED: return "unsupported parameter value";
    case SPH_E_CAPACITY: return "capacity exceeded";
    }
    return "unknown status";
}

sph_status sph_params_init(sph_params *p)
{
    if (!p) return SPH_E_INVALID;
    memset(p, 0, sizeof(*p));
    p->abi_version = SPH_ABI_VERSION;
    p->kernel = SPH_KERNEL_WENDLAND_C2;
    p->precision = SPH_FP32_MIXED;
    p->geometry = SPH_GEOM_PERIODIC_BOX;
    for (int a = 0; a < 3; a++) { p->lo[a] = 0.0; p->hi[a] = 1.0; }
    p->rho0 = 1.0;
    p->gamma = 7.0;
    p->kappa_I = 0.4;
    p->cell_factor = 1;
    return SPH_OK;
}

sph_status sph_grid_dims(const sph_params *p, int32_t dims[3])
{
    std::string msg;
    if (!dims) return SPH_E_INVALID;
    sph_status st = validate(p, msg);
    if (st != SPH_OK) return st;
    double e[3];
    return grid_of(p, dims, e, msg);
}

sph_status sph_batch_workspace_bytes(int32_t n_inst, const sph_params *params,
                                     const int64_t *counts, size_t *bytes)
{
    if (!bytes) return SPH_E_INVALID;
    Plan pl;
    std::string msg;
    sph_status st = plan(n_inst, params, counts, pl, msg);
    if (st != SPH_OK) return st;
    Carver c;
    DevState d{};
    carve(c, d, n_inst, pl.N, pl.C, pl.n_bricks, params[0].precision, pl.any_filter, pl.any_coll);
    *bytes = c.off;
    return SPH_OK;
}

sph_status sph_workspace_bytes(const sph_params *p, int64_t n, size_t *bytes)
{
    return sph_batch_workspace_bytes(1, p, &n, bytes);
}

sph_status sph_batch_create(int32_t n_inst, const sph_params *params, const int64_t *counts,
                            void *workspace, size_t ws_bytes, void *hip_stream, sph_batch **out)
{
    if (!out) return SPH_E_INVALID;
    Plan pl;
    std::string msg;
    sph_status st = plan(n_inst, params, counts, pl, msg);
    if (st != SPH_OK) return st;
    Carver c;
    DevState d{};
    carve(c, d, n_inst, pl.N, pl.C, pl.n_bricks, params[0].precision, pl.any_filter, pl.any_coll);
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0 || ws_bytes < c.off) return SPH_E_WORKSPACE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SPH_E_HIP;
    sph_batch *b = new (std::nothrow) sph_batch();
    if (!b) return SPH_E_INVALID;
    b->device = dev;
    b->stream = (hipStream_t)hip_stream;
    b->n_inst = n_inst;
    b->desc = pl.desc;
    b->params.assign(params, params + n_inst);
    b->steptab.assign(n_inst, StepParams{1.0, 0.0, 0.0, 0.0});
    Carver c2;
    c2.base = (char *)workspace;
    carve(c2, b->ds, n_inst, pl.N, pl.C, pl.n_bricks, params[0].precision, pl.any_filter, pl.any_coll);
    b->ds.precision = params[0].precision;
    b->ds.n_inst = n_inst;
    b->ds.cur = 0;
    b->ds.N = pl.N;
    b->ds.C = pl.C;
    b->ds.n_waves = pl.n_waves;
    b->ds.any_filter = pl.any_filter ? 1 : 0;
    b->ds.any_coll = pl.any_coll ? 1 : 0;
    b->ds.xcd_run = kDefaultXcdRun;
    std::vector<uint32_t> rank_of_lin, xyz;
    const std::vector<uint32_t> &bxyz = pl.bxyz, &binst = pl.binst;
    cell_tables(pl, rank_of_lin, xyz);
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemcpyAsync(b->ds.desc, pl.desc.data(), sizeof(InstDesc) * n_inst, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->ds.steptab, b->steptab.data(), sizeof(StepParams) * n_inst, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->ds.rank_of_lin, rank_of_lin.data(), sizeof(uint32_t) * pl.C, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->ds.cell_xyz, xyz.data(), sizeof(uint32_t) * pl.C, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && pl.n_bricks) e = hipMemcpyAsync(b->ds.brick_xyz, bxyz.data(), sizeof(uint32_t) * pl.n_bricks, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && pl.n_bricks) e = hipMemcpyAsync(b->ds.brick_inst, binst.data(), sizeof(uint32_t) * pl.n_bricks, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = launch_fill_u32(b->ds.count, 0u, pl.C, b->stream);
    if (e == hipSuccess) e = launch_fill_u32(b->ds.start + pl.C, pl.N, 1, b->stream);
    if (e == hipSuccess) e = launch_fill_u32(b->ds.err, 0u, 4, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        delete b;
        return SPH_E_HIP;
    }
    *out = b;
    return SPH_OK;
}

sph_status sph_batch_init(sph_batch *b, const double *x, const double *v, const double *omega,
                          const uint8_t *species, const uint8_t *kind)
{
    if (!b) return SPH_E_INVALID;
    if (!x || !v || !omega || !species || !kind) { b->err = "NULL particle array"; return SPH_E_INVALID; }
    drop_graphs(b);
    b->loaded = false;
    DevState &d = b->ds;
    d.cur = 0;
    sph_status s = check_launch(b, launch_load(d, b->L, b->stream, x, v, omega, species, kind), "load");
    if (s != SPH_OK) return s;
    if ((s = enqueue_step(b, 0, 0.0, 0.0)) != SPH_OK) return s;
    b->pending_dt = 0.0;
    b->loaded = true;
    return SPH_OK;
}

sph_status sph_batch_step(sph_batch *b, double dt, const double *Omega, int32_t nsteps)
{
    if (!b) return SPH_E_INVALID;
    return batch_step(b, dt, Omega, nsteps);
}

sph_status sph_batch_read_fields(sph_batch *b, double *x, double *v, double *omega, double *rho,
                                 double *P, double *acc, double *alpha)
{
    if (!b) return SPH_E_INVALID;
    if (!b->loaded) { b->err = "read before init"; return SPH_E_STATE; }
    sph_status s = check_launch(b, launch_read(b->ds, b->L, b->stream, 0.5 * b->pending_dt, x, v,
                                               omega, rho, P, acc, alpha), "read");
    if (s != SPH_OK) return s;
    return batch_sync(b);
}

sph_status sph_batch_diagnostics(sph_batch *b, double *out)
{
    if (!b || !out) return SPH_E_INVALID;
    if (!b->loaded) { b->err = "diagnostics before init"; return SPH_E_STATE; }
    sph_status s = check_launch(b, launch_diag(b->ds, b->L, b->stream, 0.5 * b->pending_dt), "diagnostics");
    if (s != SPH_OK) return s;
    hipError_t e = hipMemcpyAsync(out, b->ds.diag_out, sizeof(double) * 7 * b->n_inst,
                                  hipMemcpyDeviceToHost, b->stream);
    if (e != hipSuccess) return hip_fail(e, b->err, "diagnostics copy");
    return batch_sync(b);
}

sph_status sph_batch_set_tuning(sph_batch *b, const sph_tuning *t)
{
    if (!b || !t) return SPH_E_INVALID;
    const int32_t bs[3] = {t->block_density, t->block_force, t->block_stream};
    for (int k = 0; k < 3; k++)
        if (bs[k] != 0 && (bs[k] < 64 || bs[k] > 1024 || bs[k] % 64 != 0)) {
            b->err = "block sizes must be multiples of 64 in [64, 1024]";
            return SPH_E_INVALID;
        }
    if (t->use_graph < -1 || t->use_graph > 1) { b->err = "use_graph must be -1, 0 or 1"; return SPH_E_INVALID; }
    if (t->sweep != 0 && t->sweep != 1 && t->sweep != 3) {
        b->err = "sweep must be 0 (keep), 1 (per particle) or 3 (brick, candidate ballots)";
        return SPH_E_INVALID;
    }
    if (t->xcd_run < 0 || t->xcd_run > 256) { b->err = "xcd_run must be in 0..256"; return SPH_E_INVALID; }
    if (t->list_targets != 0 && t->list_targets != 16 && t->list_targets != 32) {
        b->err = "list_targets must be 0 (keep), 16 or 32";
        return SPH_E_INVALID;
    }
    if (t->xcd_run) b->ds.xcd_run = (uint32_t)t->xcd_run;
    if (t->list_targets) b->L.list_targets = t->list_targets;
    if (t->sweep) b->L.sweep = t->sweep;
    if (t->block_density) b->L.bs_density = t->block_density;
    if (t->block_force) b->L.bs_force = t->block_force;
    if (t->block_stream) b->L.bs_stream = t->block_stream;
    if (t->use_graph >= 0) b->use_graph = t->use_graph == 1;
    drop_graphs(b);
    return SPH_OK;
}

sph_status sph_batch_sync(sph_batch *b)
{
    if (!b) return SPH_E_INVALID;
    return batch_sync(b);
}

const char *sph_batch_last_error(const sph_batch *b)
{
    return b ? b->err.c_str() : "";
}

void sph_batch_destroy(sph_batch *b)
{
    if (!b) return;
    drop_graphs(b);
    for (hipEvent_t ev : b->prof.pool) (void)hipEventDestroy(ev);
    delete b;
}

sph_status sph_batch_profile_begin(sph_batch *b)
{
    if (!b) return SPH_E_INVALID;
    return profile_begin(b);
}

sph_status sph_batch_profile_end(sph_batch *b, double ms[SPH_K_COUNT], int32_t *nsteps)
{
    if (!b) return SPH_E_INVALID;
    return profile_end(b, ms, nsteps);
}

sph_status sph_profile_begin(sph_sim *s)
{
    if (!s) return SPH_E_INVALID;
    return profile_begin(s->b);
}

sph_status sph_profile_end(sph_sim *s, double ms[SPH_K_COUNT], int32_t *nsteps)
{
    if (!s) return SPH_E_INVALID;
    return profile_end(s->b, ms, nsteps);
}

// ---- single instance ----

sph_status sph_create(const sph_params *p, int64_t n, void *workspace, size_t ws_bytes,
                      void *hip_stream, sph_sim **out)
{
    if (!out) return SPH_E_INVALID;
    sph_batch *b = nullptr;
    sph_status st = sph_batch_create(1, p, &n, workspace, ws_bytes, hip_stream, &b);
    if (st != SPH_OK) return st;
    sph_sim *s = new (std::nothrow) sph_sim();
    if (!s) { sph_batch_destroy(b); return SPH_E_INVALID; }
    s->b = b;
    *out = s;
    return SPH_OK;
}

sph_status sph_init_particles(sph_sim *s, const double *x, const double *v, const double *omega,
                              const uint8_t *species, const uint8_t *kind)
{
    if (!s) return SPH_E_INVALID;
    return sph_batch_init(s->b, x, v, omega, species, kind);
}

sph_status sph_step(sph_sim *s, double dt, double Omega, int32_t nsteps)
{
    if (!s) return SPH_E_INVALID;
    return batch_step(s->b, dt, &Omega, nsteps);
}

sph_status sph_read_fields(sph_sim *s, double *x, double *v, double *omega, double *rho, double *P,
                           double *acc, double *alpha)
{
    if (!s) return SPH_E_INVALID;
    return sph_batch_read_fields(s->b, x, v, omega, rho, P, acc, alpha);
}

sph_status sph_diagnostics(sph_sim *s, double out[7])
{
    if (!s) return SPH_E_INVALID;
    return sph_batch_diagnostics(s->b, out);
}

sph_status sph_debug_cells(sph_sim *s, uint32_t *key_by_id, uint32_t *perm, uint32_t *cell_start)
{
    if (!s) return SPH_E_INVALID;
    sph_batch *b = s->b;
    if (!b->loaded) { b->err = "debug before init"; return SPH_E_STATE; }
    if (key_by_id || perm) {
        sph_status st = check_launch(b, launch_debug_keys(b->ds, b->L, b->stream, key_by_id, perm), "debug keys");
        if (st != SPH_OK) return st;
    }
    if (cell_start) {
        hipError_t e = hipMemcpyAsync(cell_start, b->ds.start, sizeof(uint32_t) * ((size_t)b->ds.C + 1),
                                      hipMemcpyDeviceToDevice, b->stream);
        if (e != hipSuccess) return hip_fail(e, b->err, "copy cell_start");
    }
    return SPH_OK;
}

}  // extern "C"

namespace {

// Neighbour CSR by id in two launches (counts, then columns), with the host prefix sum in
// between; `launch(phase, row_ptr, cols)` enqueues one phase.
template <class Launcher>
sph_status neighbour_csr(sph_batch *b, int64_t *row_ptr, int32_t *cols, int64_t cap, int64_t *nnz,
                         Launcher &&launch)
{
    const size_t n = b->ds.N;
    hipError_t e = hipMemsetAsync(row_ptr, 0, sizeof(int64_t), b->stream);
    if (e != hipSuccess) return hip_fail(e, b->err, "clear row_ptr");
    sph_status st = check_launch(b, launch(0, row_ptr, cols), "neighbour count");
    if (st != SPH_OK) return st;
    std::vector<int64_t> h(n + 1);
    e = hipMemcpyAsync(h.data(), row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, b->err, "neighbour counts");
    h[0] = 0;
    for (size_t i = 0; i < n; i++) h[i + 1] += h[i];
    *nnz = h[n];
    e = hipMemcpyAsync(row_ptr, h.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, b->err, "row_ptr upload");
    if (h[n] > cap) { b->err = "neighbour capacity too small"; return SPH_E_CAPACITY; }
    st = check_launch(b, launch(1, row_ptr, cols), "neighbour fill");
    if (st != SPH_OK) return st;
    return batch_sync(b);
}

sph_status neighbour_args(sph_batch *b, int64_t *row_ptr, int32_t *cols, int64_t cap, int64_t *nnz)
{
    if (!row_ptr || !nnz || cap < 0 || (cap > 0 && !cols)) { b->err = "bad neighbour output"; return SPH_E_INVALID; }
    if (!b->loaded) { b->err = "debug before init"; return SPH_E_STATE; }
    return SPH_OK;
}

}  // namespace

extern "C" {

sph_status sph_debug_neighbors(sph_sim *s, int64_t *row_ptr, int32_t *cols, int64_t cap, int64_t *nnz)
{
    if (!s) return SPH_E_INVALID;
    sph_batch *b = s->b;
    sph_status st = neighbour_args(b, row_ptr, cols, cap, nnz);
    if (st != SPH_OK) return st;
    return neighbour_csr(b, row_ptr, cols, cap, nnz, [&](int phase, int64_t *r, int32_t *c) {
        return launch_debug_nbr(b->ds, b->L, b->stream, phase, r, c);
    });
}

sph_status sph_debug_masks(sph_sim *s, int64_t *row_ptr, int32_t *cols, int64_t cap, int64_t *nnz)
{
    if (!s) return SPH_E_INVALID;
    sph_batch *b = s->b;
    sph_status st = neighbour_args(b, row_ptr, cols, cap, nnz);
    if (st != SPH_OK) return st;
    if (!b->masks_current) {
        b->err = "the last density sweep was not the brick sweep: no hit masks";
        return SPH_E_STATE;
    }
    return neighbour_csr(b, row_ptr, cols, cap, nnz, [&](int phase, int64_t *r, int32_t *c) {
        return launch_debug_masks(b->ds, b->stream, phase, r, c);
    });
}

sph_status sph_debug_near(sph_sim *s, uint8_t *count, int32_t *ids)
{
    if (!s) return SPH_E_INVALID;
    sph_batch *b = s->b;
    if (!count || !ids) { b->err = "bad near-list output"; return SPH_E_INVALID; }
    if (!b->loaded) { b->err = "debug before init"; return SPH_E_STATE; }
    if (!b->masks_current || !b->ds.any_coll) {
        b->err = "no near lists: the collision step is off or the last density sweep was not "
                 "the brick sweep";
        return SPH_E_STATE;
    }
    sph_status st = check_launch(b, launch_debug_near(b->ds, b->L, b->stream, count, ids), "near lists");
    if (st != SPH_OK) return st;
    return batch_sync(b);
}

sph_status sph_set_tuning(sph_sim *s, const sph_tuning *t)
{
    if (!s) return SPH_E_INVALID;
    return sph_batch_set_tuning(s->b, t);
}

sph_status sph_get_tuning(const sph_sim *s, sph_tuning *t)
{
    if (!s || !t) return SPH_E_INVALID;
    t->block_density = s->b->L.bs_density;
    t->block_force = s->b->L.bs_force;
    t->block_stream = s->b->L.bs_stream;
    t->use_graph = s->b->use_graph ? 1 : 0;
    t->sweep = s->b->L.sweep;
    t->xcd_run = (int32_t)s->b->ds.xcd_run;
    t->list_targets = s->b->L.list_targets;
    return SPH_OK;
}

sph_status sph_sync(sph_sim *s)
{
    if (!s) return SPH_E_INVALID;
    return batch_sync(s->b);
}

sph_status sph_vortex_dims(const sph_params *p, int32_t *nx, int32_t *ny)
{
    if (!p || !nx || !ny) return SPH_E_INVALID;
    std::string msg;
    sph_status st = validate(p, msg);
    if (st != SPH_OK) return st;
    vortex_grid(*p, *nx, *ny);
    return SPH_OK;
}

}  // extern "C"

namespace {

sph_status vortex_args(sph_batch *b, double z0, double theta, int32_t min_pixels, double *image,
                       int32_t *labels, int32_t *count)
{
    if (!image || !labels || !count || !std::isfinite(z0) || !std::isfinite(theta) ||
        theta < 0.0 || min_pixels < 1) {
        b->err = "vortex image: needs image, labels and count, finite z0, theta >= 0 and "
                 "min_pixels >= 1";
        return SPH_E_INVALID;
    }
    if (!b->loaded) { b->err = "vortex image before init"; return SPH_E_STATE; }
    return SPH_OK;
}

// The vortex image, labels and count with the given scratch (int32, nx ny + 8, 8-byte
// aligned, device memory; cleared here before use).
sph_status vortex_image(sph_batch *b, double z0, double theta, int32_t min_pixels, double *image,
                        int32_t *labels, int32_t *scr, int32_t *count)
{
    const sph_params &p = b->params[0];
    int32_t nx, ny;
    vortex_grid(p, nx, ny);
    const uint32_t n = (uint32_t)nx * (uint32_t)ny;
    VortexArgs a;
    a.z0 = z0;
    a.Lz = p.hi[2] - p.lo[2];
    a.dx = p.dx;
    a.lox = p.lo[0];
    a.loy = p.lo[1];
    a.pend = 0.5 * b->pending_dt;
    a.nx = nx;
    a.ny = ny;
    // scratch: size[n] | changed | count | (8-byte aligned) image maximum
    int32_t *size = scr;
    uint32_t *changed = (uint32_t *)(scr + n);
    int32_t *cnt = scr + n + 1;
    unsigned long long *vmax = (unsigned long long *)(scr + ((n + 3) & ~1u));
    unsigned long long *img = (unsigned long long *)image;
    hipError_t e = launch_fill_u32((uint32_t *)image, 0u, 2 * (size_t)n, b->stream);
    if (e == hipSuccess) e = launch_fill_u32((uint32_t *)scr, 0u, ((n + 3) & ~1u) + 2, b->stream);
    if (e == hipSuccess) e = launch_vortex_intensity(b->ds, b->L, b->stream, a, b->masks_current, img, vmax);
    if (e == hipSuccess) e = launch_vortex_label_init(b->stream, img, vmax, theta, n, labels);
    if (e != hipSuccess) return hip_fail(e, b->err, "vortex image");
    // Relax until a pass changes nothing.  Each pass carries a component's smallest label
    // at least one pixel further, so diameter + 1 <= n passes end it.
    bool settled = false;
    for (uint32_t it = 0; it <= n && !settled; it++) {
        uint32_t flag = 0;
        e = launch_fill_u32(changed, 0u, 1, b->stream);
        if (e == hipSuccess) e = launch_vortex_relax(b->stream, labels, nx, ny, changed);
        if (e == hipSuccess) e = hipMemcpyAsync(&flag, changed, sizeof(flag), hipMemcpyDeviceToHost, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return hip_fail(e, b->err, "vortex labels");
        settled = flag == 0;
    }
    if (!settled) {
        b->err = "vortex labels did not settle";
        return SPH_E_STATE;
    }
    e = launch_vortex_count(b->stream, labels, size, n, min_pixels, cnt);
    if (e == hipSuccess) e = hipMemcpyAsync(count, cnt, sizeof(int32_t), hipMemcpyDeviceToHost, b->stream);
    if (e != hipSuccess) return hip_fail(e, b->err, "vortex count");
    return batch_sync(b);
}

// Scratch of sph_vortex_image_noalloc: one array per device, held until the process ends.
constexpr uint32_t kVortexPixelsMax = 1u << 20;
constexpr size_t kVortexScratchInts = (size_t)kVortexPixelsMax + 8;
__device__ __align__(256) int32_t scratch[kVortexScratchInts];

// Device address of `scratch` on each device, looked up once per device with that device
// current (in host code the array's name is not a device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t *g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_on(int dev, int32_t **out)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (int32_t *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

sph_status sph_vortex_image(sph_sim *s, double z0, double theta, int32_t min_pixels,
                            double *image, int32_t *labels, int32_t *scratch_buf, int32_t *count)
{
    if (!s) return SPH_E_INVALID;
    sph_batch *b = s->b;
    sph_status st = vortex_args(b, z0, theta, min_pixels, image, labels, count);
    if (st != SPH_OK) return st;
    if (!scratch_buf || ((uintptr_t)scratch_buf & 7u)) {
        b->err = "vortex image: needs an 8-byte aligned scratch buffer";
        return SPH_E_INVALID;
    }
    return vortex_image(b, z0, theta, min_pixels, image, labels, scratch_buf, count);
}

sph_status sph_vortex_image_noalloc(sph_sim *s, double z0, double theta, int32_t min_pixels,
                                    double *image, int32_t *labels, int32_t *count)
{
    if (!s) return SPH_E_INVALID;
    sph_batch *b = s->b;
    sph_status st = vortex_args(b, z0, theta, min_pixels, image, labels, count);
    if (st != SPH_OK) return st;
    int32_t nx, ny;
    vortex_grid(b->params[0], nx, ny);
    if ((uint64_t)nx * (uint64_t)ny > (uint64_t)kVortexPixelsMax) {
        b->err = "vortex image (no-alloc): more than 2^20 pixels";
        return SPH_E_CAPACITY;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, b->err, "current device");
    const bool other = dev != b->device;
    if (other && (e = hipSetDevice(b->device)) != hipSuccess) return hip_fail(e, b->err, "set device");
    int32_t *scr = nullptr;
    e = scratch_on(b->device, &scr);
    if (e == hipSuccess) st = vortex_image(b, z0, theta, min_pixels, image, labels, scr, count);
    else st = hip_fail(e, b->err, "scratch address");
    if (other) (void)hipSetDevice(dev);
    return st;
}

const char *sph_last_error(const sph_sim *s)
{
    return s ? s->b->err.c_str() : "";
}

void sph_destroy(sph_sim *s)
{
    if (!s) return;
    sph_batch_destroy(s->b);
    delete s;
}

}  // extern "C"
