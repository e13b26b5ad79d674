// HIP kernels (gfx950) of the two-fluid SPH step.
//
// Per time step (velocity Verlet, Algorithm 1 of the paper, single device):
//   k_keys     half kick + drift of each particle (walls: exact rotation), its cell in
//              Morton order, and its slot in that cell (atomic histogram);
//   k_scan_*   exclusive scan of the cell histogram -> cell_start (CSR of the cell list);
//   k_scatter  counting-sort scatter (and the ids in scatter order);
//   k_reorder  orders each cell by particle id and moves the advanced state into the new
//              cell-sorted order (the paper's periodic defragmentation, done every step);
//   density    kernel-summed density, Tait EOS (Eq. 4) and the per-particle factors the
//              force sweep needs;
//   filter     pressure filter of Algorithm 1 (when enabled);
//   collide    collision step of Algorithm 1 (when enabled; it changes velocities only,
//              which the density and the filter do not read, so it runs after them);
//   force      pair forces of Eqs. 1-2 and the spin torques.
// The density, filter and force sweeps come in two forms: one thread per particle
// (k_density, k_filter, k_force; the FP64 path), and one that stages a 2x2x2-cell brick's
// neighbourhood in LDS and tests candidates with wave ballots (k_density_cand,
// k_filter_cand, k_force_cand, after k_brick_frames; the FP32-mixed default with cell
// factor 1).  The closing half kick is folded into the next k_keys / k_reorder.
#include <math.h>
#include <type_traits>

#include "sph_device.h"

namespace sph {
namespace {

// ---------------------------------------------------------------- thread mapping ----

struct PIdx {
    const InstDesc *d;
    uint32_t p;
    bool active;
};

__device__ __forceinline__ int find_inst(const InstDesc *desc, int n_inst, uint32_t wave)
{
    int lo = 0, hi = n_inst - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (desc[mid].wave_off <= wave) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Each instance's particle range is covered by whole wavefronts, so a wavefront never
// straddles two instances and its descriptor is wave-uniform.
__device__ __forceinline__ PIdx map_thread(const DevState &s)
{
    uint32_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    wave = __builtin_amdgcn_readfirstlane(wave);
    int inst = find_inst(s.desc, s.n_inst, wave);
    const InstDesc *d = s.desc + inst;
    uint32_t local = (wave - d->wave_off) * (uint32_t)kWave + (threadIdx.x & (kWave - 1));
    PIdx r;
    r.d = d;
    r.p = d->part_off + local;
    r.active = wave < s.n_waves && local < d->n_part;
    return r;
}

__host__ __device__ inline unsigned grid_for(uint32_t n_waves, int block)
{
    uint32_t wpb = (uint32_t)block / kWave;
    return (n_waves + wpb - 1) / wpb;
}

// ---------------------------------------------------------------- geometry ----------

// floor((x - lo) / edge) with IEEE division; periodic axes clamp, bounded axes flag.
__device__ __forceinline__ int cell_coord(const InstDesc *d, int a, double x, uint32_t &err)
{
    double t = (x - d->lo[a]) / d->edge[a];
    double f = floor(t);
    int n = d->n[a];
    if (!(f >= 0.0)) {
        if (f != f) err |= ERR_NONFINITE;
        else if (!d->periodic[a]) err |= ERR_DOMAIN;
        return 0;
    }
    if (f > (double)(n - 1)) {
        if (!d->periodic[a]) err |= ERR_DOMAIN;
        return n - 1;
    }
    return (int)f;
}

// Minimum image along one axis, branch-free: halfL is +inf on bounded axes, so neither
// correction applies there.
__device__ __forceinline__ double min_img(const InstDesc *d, int a, double dd)
{
    const double h = d->halfL[a], L = d->L[a];
    double up = dd - L, dn = dd + L;
    return dd > h ? up : (dd < -h ? dn : dd);
}

// (dx*dx + dy*dy) + dz*dz with every product and sum rounded separately (no fused
// multiply-add): the neighbour test is bit-identical to a plain double-precision
// evaluation in this order.
__device__ __forceinline__ double r2_exact(double a, double b, double c)
{
#pragma clang fp contract(off)
    double xx = a * a;
    double yy = b * b;
    double zz = c * c;
    return (xx + yy) + zz;
}

__device__ __forceinline__ uint32_t morton3(uint32_t x, uint32_t y, uint32_t z)
{
    uint32_t k = 0;
    for (int b = 0; b < 10; b++) {
        k |= ((x >> b) & 1u) << (3 * b);
        k |= ((y >> b) & 1u) << (3 * b + 1);
        k |= ((z >> b) & 1u) << (3 * b + 2);
    }
    return k;
}

// Calls fn(begin, end) for the sorted-particle range of every cell at offsets
// [lo[a], hi[a]] (within +-cf) from (cx, cy, cz), wrapping periodic axes and skipping cells
// off a bounded axis.
template <class Fn>
__device__ __forceinline__ void for_cells_in(const DevState &s, const InstDesc *d, int cx, int cy,
                                             int cz, const int lo[3], const int hi[3],
                                             uint32_t &err, Fn &&fn)
{
    const int n0 = d->n[0], n1 = d->n[1], n2 = d->n[2];
    for (int oz = lo[2]; oz <= hi[2]; ++oz) {
        int z = cz + oz;
        if (d->periodic[2]) { z += z < 0 ? n2 : 0; z -= z >= n2 ? n2 : 0; }
        else if (z < 0 || z >= n2) continue;
        for (int oy = lo[1]; oy <= hi[1]; ++oy) {
            int y = cy + oy;
            if (d->periodic[1]) { y += y < 0 ? n1 : 0; y -= y >= n1 ? n1 : 0; }
            else if (y < 0 || y >= n1) continue;
            for (int ox = lo[0]; ox <= hi[0]; ++ox) {
                int x = cx + ox;
                if (d->periodic[0]) { x += x < 0 ? n0 : 0; x -= x >= n0 ? n0 : 0; }
                else if (x < 0 || x >= n0) continue;
                uint32_t lin = (uint32_t)x + (uint32_t)n0 * ((uint32_t)y + (uint32_t)n1 * (uint32_t)z);
                uint32_t r = s.rank_of_lin[d->cell_off + lin];
                uint32_t b = s.start[r], e = s.start[r + 1];
                if (e - b > (uint32_t)kMaxCell) { err |= ERR_CAPACITY; continue; }
                fn(b, e);
            }
        }
    }
}

// The same over the whole stencil, +-cf cells on every axis.
template <class Fn>
__device__ __forceinline__ void for_each_cell(const DevState &s, const InstDesc *d, int cx,
                                              int cy, int cz, uint32_t &err, Fn &&fn)
{
    const int cf = d->cf;
    const int lo[3] = {-cf, -cf, -cf}, hi[3] = {cf, cf, cf};
    for_cells_in(s, d, cx, cy, cz, lo, hi, err, fn);
}

// ------------------------------------------------------------ integrator pieces -----

// New state of one particle.  mode 0 copies (initial evaluation); mode 1 applies the
// opening kick `kick` (= dt/2, or dt when the previous closing half kick is folded in)
// and the drift; walls are turned by the step's rotation.  Fused multiply-adds are
// spelled out so that k_keys and k_reorder produce bit-identical positions.
template <typename R>
__device__ __forceinline__ void advance(const DevState &s, const InstDesc *d, int kind,
                                        uint32_t op, int mode, double kick, double dt,
                                        double xo[3], double vo[3], double wo[3])
{
    const uint32_t N = s.N;
    const int cur = s.cur;
    const double *x = s.x[cur], *v = s.v[cur], *w = s.w[cur];
    if (mode == 0) {
        for (int a = 0; a < 3; a++) {
            xo[a] = x[a * N + op]; vo[a] = v[a * N + op]; wo[a] = w[a * N + op];
        }
        return;
    }
    if (kind == KIND_FLUID) {
        const R *acc = (const R *)s.acc, *alpha = (const R *)s.alpha;
        for (int a = 0; a < 3; a++) {
            double vh = __fma_rn(kick, (double)acc[a * N + op], v[a * N + op]);
            double wh = __fma_rn(kick, (double)alpha[a * N + op], w[a * N + op]);
            double xn = __fma_rn(dt, vh, x[a * N + op]);
            if (d->periodic[a]) {
                if (xn >= d->hi[a]) xn -= d->L[a];
                else if (xn < d->lo[a]) xn += d->L[a];
            }
            xo[a] = xn; vo[a] = vh; wo[a] = wh;
        }
    } else {
        const StepParams *sp = s.steptab + (d - s.desc);
        double c = sp->cosw, sn = sp->sinw, Om = sp->Omega;
        double x0 = x[op], y0 = x[N + op];
        double xr = __dsub_rn(__dmul_rn(c, x0), __dmul_rn(sn, y0));
        double yr = __dadd_rn(__dmul_rn(sn, x0), __dmul_rn(c, y0));
        xo[0] = xr; xo[1] = yr; xo[2] = x[2 * N + op];
        vo[0] = -Om * yr; vo[1] = Om * xr; vo[2] = 0.0;
        wo[0] = 0.0; wo[1] = 0.0; wo[2] = Om;
    }
}

// ---------------------------------------------------------------- kernels -----------

template <typename R>
__global__ void k_keys(DevState s, int mode, double kick, double dt)
{
    PIdx t = map_thread(s);
    if (!t.active) return;
    const InstDesc *d = t.d;
    const uint32_t p = t.p;
    uint32_t err = 0;
    int kind = s.sk[s.cur][p] >> 1;
    // only the new position is needed here (the spin and its acceleration are not loaded);
    // k_reorder checks the advanced velocity and spin when it stores them
    double xo[3], vo[3], wo[3];
    advance<R>(s, d, kind, p, mode, kick, dt, xo, vo, wo);
    for (int a = 0; a < 3; a++)
        if (!isfinite(xo[a])) err |= ERR_NONFINITE;
    int c0 = cell_coord(d, 0, xo[0], err);
    int c1 = cell_coord(d, 1, xo[1], err);
    int c2 = cell_coord(d, 2, xo[2], err);
    if (xo[0] * xo[0] + xo[1] * xo[1] > d->rxy2) err |= ERR_DOMAIN;  // beyond the cylinder
    uint32_t lin = (uint32_t)c0 + (uint32_t)d->n[0] * ((uint32_t)c1 + (uint32_t)d->n[1] * (uint32_t)c2);
    uint32_t key = s.rank_of_lin[d->cell_off + lin];
    s.key[p] = key;
    // One atomic per distinct key of the wavefront: particles arrive nearly cell-sorted, so
    // neighbouring lanes mostly share a cell.  Lanes of a key take consecutive slots in lane
    // order (the final in-cell order is fixed by id in k_reorder).
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t below = (1ull << lane) - 1ull;
    uint64_t todo = __ballot(1);
    while (todo) {
        const int leader = __builtin_ctzll(todo);
        const uint32_t lk = __shfl(key, leader);
        const uint64_t same = __ballot(key == lk) & todo;
        uint32_t base = 0;
        if ((int)lane == leader) base = atomicAdd(&s.count[lk], (uint32_t)__popcll(same));
        base = __shfl(base, leader);
        if (key == lk) s.slot[p] = base + (uint32_t)__popcll(same & below);
        todo &= ~same;
    }
    if (err) atomicOr(s.err, err);
}

constexpr int kScanBlock = 256;
constexpr int kScanPer = 4;
constexpr int kScanTile = kScanBlock * kScanPer;

// Exclusive block scan of one value per thread (Hillis-Steele in LDS); returns the
// exclusive prefix and writes the block total to *total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh, uint32_t *total)
{
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        uint32_t add = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    uint32_t incl = sh[t];
    *total = sh[kScanBlock - 1];
    __syncthreads();
    return incl - v;
}

__global__ void k_scan_tiles(const uint32_t *count, uint32_t C, uint32_t *bsum)
{
    __shared__ uint32_t sh[kScanBlock];
    uint32_t base = blockIdx.x * (uint32_t)kScanTile + threadIdx.x * (uint32_t)kScanPer;
    uint32_t v = 0;
    for (int k = 0; k < kScanPer; k++)
        if (base + k < C) v += count[base + k];
    uint32_t tot;
    block_exclusive_scan(v, sh, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void k_scan_bsum(uint32_t *bsum, uint32_t nb)
{
    __shared__ uint32_t sh[kScanBlock];
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nb; base += kScanBlock) {
        uint32_t i = base + threadIdx.x;
        uint32_t v = i < nb ? bsum[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_exclusive_scan(v, sh, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
}

// cell_start[c] = exclusive prefix of the histogram; the histogram is cleared for the
// next step (no memset node is needed inside a captured step).
__global__ void k_scan_apply(uint32_t *count, uint32_t C, const uint32_t *bsum, uint32_t *start)
{
    __shared__ uint32_t sh[kScanBlock];
    uint32_t base = blockIdx.x * (uint32_t)kScanTile + threadIdx.x * (uint32_t)kScanPer;
    uint32_t vals[kScanPer];
    uint32_t v = 0;
    for (int k = 0; k < kScanPer; k++) {
        vals[k] = base + k < C ? count[base + k] : 0u;
        v += vals[k];
    }
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(v, sh, &tot) + bsum[blockIdx.x];
    for (int k = 0; k < kScanPer; k++) {
        if (base + k < C) {
            start[base + k] = ex;
            count[base + k] = 0u;
        }
        ex += vals[k];
    }
}

__global__ void k_scatter(DevState s)
{
    PIdx t = map_thread(s);
    if (!t.active) return;
    uint32_t p = t.p;
    uint32_t pos = s.start[s.key[p]] + s.slot[p];
    s.tmp[pos] = p;
    s.idt[pos] = s.id[s.cur][p];
}

// Final position = cell start + rank of the particle id within its cell, so the order is
// (cell in Morton order, id) whatever order the atomics produced.
template <typename R>
__global__ void k_reorder(DevState s, int mode, double kick, double dt)
{
    PIdx t = map_thread(s);
    if (!t.active) return;
    const InstDesc *d = t.d;
    const uint32_t q = t.p, N = s.N;
    const int cur = s.cur, nxt = cur ^ 1;
    uint32_t op = s.tmp[q];
    uint32_t c = s.key[op];
    uint32_t b = s.start[c], e = s.start[c + 1];
    uint32_t myid = s.idt[q];
    uint32_t dst = q;
    if (e - b <= (uint32_t)kMaxCell) {
        // the cell's ids in scatter order are contiguous: one independent load per member
        uint32_t rank = 0;
        for (uint32_t k = b; k < e; k++) rank += s.idt[k] < myid ? 1u : 0u;
        dst = b + rank;
    } else {
        atomicOr(s.err, (uint32_t)ERR_CAPACITY);
    }
    uint8_t skv = s.sk[cur][op];
    double xo[3], vo[3], wo[3];
    advance<R>(s, d, skv >> 1, op, mode, kick, dt, xo, vo, wo);
    bool finite = true;
    for (int a = 0; a < 3; a++) {
        s.x[nxt][a * N + dst] = xo[a];
        s.v[nxt][a * N + dst] = vo[a];
        s.w[nxt][a * N + dst] = wo[a];
        finite = finite && isfinite(vo[a]) && isfinite(wo[a]);
    }
    if (!finite) atomicOr(s.err, (uint32_t)ERR_NONFINITE);
    s.id[nxt][dst] = myid;
    s.sk[nxt][dst] = skv;
    s.pcell[dst] = c;
}

// ----------------------------------------------------------- kernel functions ------

// W(r) and F(r) = -W'(r)/r for r^2 < (2h)^2.  Cubic spline and Wendland C2, q = r/h.
template <typename R>
__device__ __forceinline__ void kernel_WF(int kernel, R r2, R inv_h, R wnorm, R &W, R &F)
{
    R r = sqrt(r2);
    R q = r * inv_h;
    R ih2 = inv_h * inv_h;
    if (kernel == KERNEL_WENDLAND) {
        R t = (R)1 - (R)0.5 * q;
        R t3 = t * t * t;
        W = wnorm * t3 * t * ((R)2 * q + (R)1);
        F = (R)5 * wnorm * t3 * ih2;
    } else {
        if (q < (R)1) {
            W = wnorm * ((R)1 - (R)1.5 * q * q + (R)0.75 * q * q * q);
            F = wnorm * ((R)3 - (R)2.25 * q) * ih2;
        } else {
            R t = (R)2 - q;
            W = wnorm * (R)0.25 * t * t * t;
            F = wnorm * (R)0.75 * t * t * ih2 / q;
        }
    }
}

template <typename R>
__device__ __forceinline__ R kernel_W(int kernel, R r2, R inv_h, R wnorm)
{
    R r = sqrt(r2);
    R q = r * inv_h;
    if (kernel == KERNEL_WENDLAND) {
        R t = (R)1 - (R)0.5 * q;
        R t2 = t * t;
        return wnorm * t2 * t2 * ((R)2 * q + (R)1);
    }
    if (q < (R)1) return wnorm * ((R)1 - (R)1.5 * q * q + (R)0.75 * q * q * q);
    R t = (R)2 - q;
    return wnorm * (R)0.25 * t * t * t;
}

// Compensated (Kahan) accumulation; plain addition when KAHAN is false.
template <typename R, bool KAHAN>
struct Acc {
    R s = 0, c = 0;
    __device__ __forceinline__ void add(R x)
    {
        if (KAHAN) {
            R y = x - c;
            R t = s + y;
            c = (t - s) - y;
            s = t;
        } else {
            s += x;
        }
    }
    __device__ __forceinline__ double value() const
    {
        return KAHAN ? (double)s - (double)c : (double)s;
    }
};

// Writes rho, P and the per-particle factors of the force sweep from the kernel sums.
// Inner wall and fluid: rho = m (W(0) + sum W); outer wall: rho0, P = 0 (kept at their
// initial values); Tait EOS P = B ((rho/rho0)^7 - 1).
template <typename R>
__device__ __forceinline__ uint32_t density_finish(const DevState &s, const InstDesc *d, uint32_t p,
                                                   int spi, int kind, double sumW, double S)
{
    double mi = d->mass[spi];
    double rho, P;
    if (kind == KIND_WALL_OUTER) {
        rho = d->rho0;
        P = 0.0;
    } else {
        rho = mi * (d->W0 + sumW);
        double r = rho / d->rho0;
        double r2 = r * r;
        P = d->B * ((r2 * r2) * (r2 * r) - 1.0);
    }
    const double irho = 1.0 / rho;
    double V = mi * irho;
    double ir2 = irho * irho;
    R *aux = (R *)s.aux + 4 * (size_t)p;
    aux[0] = (R)V;
    aux[1] = (R)(P * ir2);
    aux[2] = (R)ir2;
    aux[3] = (R)(S > 0.0 ? V / S : 0.0);
    R *rp = (R *)s.rhoP + 2 * (size_t)p;
    rp[0] = (R)rho;
    rp[1] = (R)P;
    return (!isfinite(rho) || !isfinite(P)) ? (uint32_t)ERR_NONFINITE : 0u;
}

// Density (kernel summation), unlike-neighbour kernel sum S and Tait EOS of particle p,
// walking its cell stencil.
template <typename R, bool KAHAN>
__device__ __forceinline__ uint32_t density_one(const DevState &s, const InstDesc *d, uint32_t p)
{
    const uint32_t N = s.N;
    const int cur = s.cur;
    const double *X = s.x[cur];
    const uint8_t *SK = s.sk[cur];
    const double xi0 = X[p], xi1 = X[N + p], xi2 = X[2 * N + p];
    const uint8_t ski = SK[p];
    const int spi = ski & 1, kind = ski >> 1;
    const uint32_t cxyz = s.cell_xyz[s.pcell[p]];
    const int kernel = d->kernel;
    const double cut2 = d->cut2;
    const R inv_h = (R)d->inv_h, wnorm = (R)d->wnorm;
    uint32_t err = 0;
    Acc<R, KAHAN> sw, su;
    for_each_cell(s, d, cxyz & 1023, (cxyz >> 10) & 1023, cxyz >> 20, err,
                  [&](uint32_t b, uint32_t e) {
        for (uint32_t q = b; q < e; ++q) {
            const double xq0 = X[q], xq1 = X[N + q], xq2 = X[2 * N + q];
            const int spq = SK[q] & 1;
            double r2 = r2_exact(min_img(d, 0, xi0 - xq0), min_img(d, 1, xi1 - xq1),
                                 min_img(d, 2, xi2 - xq2));
            if (r2 < cut2 && q != p) {
                R W = kernel_W<R>(kernel, (R)r2, inv_h, wnorm);
                sw.add(W);
                su.add(spq != spi ? W : (R)0);
            }
        }
    });
    return err | density_finish<R>(s, d, p, spi, kind, sw.value(), su.value());
}

template <typename R, bool KAHAN>
__global__ void k_density(DevState s)
{
    PIdx t = map_thread(s);
    if (!t.active) return;
    uint32_t err = density_one<R, KAHAN>(s, t.d, t.p);
    if (err) atomicOr(s.err, err);
}

// Coefficients of the pair force, in the pair precision.
template <typename R>
struct ForceK {
    R m0, m1, sigT, eta4, Cl, inv_h, wnorm;
    int kernel;
    __device__ explicit ForceK(const InstDesc *d)
        : m0((R)d->mass[0]), m1((R)d->mass[1]), sigT((R)d->sigma_T), eta4((R)(4.0 * d->eta)),
          Cl((R)d->C_l), inv_h((R)d->inv_h), wnorm((R)d->wnorm), kernel(d->kernel) {}
};

// Per-particle inputs of the pair force: species, mass, V = m/rho, P/rho^2, 1/rho^2, V/S.
template <typename R>
struct ForceP {
    int sp;
    R m, V, Pr, ir2, VS;
};

// Force f on particle i from neighbour j and the spin torque n that both receive.
//   pressure     m_i m_j (P_i/rho_i^2 + P_j/rho_j^2) F r
//   interfacial  g_T (r_x, r_y, 0), g_T = -sigma_T m_i m_j (1/rho_i^2 + 1/rho_j^2) F, unlike
//   viscous      -4 eta V_i V_j F (v_ij - (w_i + w_j)/2 × r), viscous-viscous pairs
//   friction     -C_l W (V_i/S_i + V_j/S_j) v_ij, unlike pairs
//   torque       -1/2 r × (non-central force)
// r = x_i - x_j (r2 its squared length), v = v_i - v_j, hs = (w_i + w_j)/2.
template <typename R>
__device__ __forceinline__ void pair_force(const ForceK<R> &k, const ForceP<R> &I, const ForceP<R> &J,
                                           R r0, R r1, R r2, R rsq, R v0, R v1, R v2,
                                           R hs0, R hs1, R hs2, R f[3], R n[3])
{
    R W, Fk;
    kernel_WF<R>(k.kernel, rsq, k.inv_h, k.wnorm, W, Fk);
    const R mm = I.m * J.m;
    const R gp = mm * (I.Pr + J.Pr) * Fk;
    R f0 = gp * r0, f1 = gp * r1, f2 = gp * r2;
    R n0 = 0, n1 = 0;
    R c0 = 0, c1 = 0, c2 = 0;  // non-central part
    if (I.sp != J.sp) {
        R gT = -k.sigT * mm * (I.ir2 + J.ir2) * Fk;
        f0 += gT * r0;
        f1 += gT * r1;
        n0 = (R)0.5 * gT * r2 * r1;
        n1 = (R)-0.5 * gT * r2 * r0;
        R gm = -k.Cl * W * (I.VS + J.VS);
        c0 = gm * v0; c1 = gm * v1; c2 = gm * v2;
    }
    if ((I.sp & J.sp) != 0) {
        R u0 = v0 - (hs1 * r2 - hs2 * r1);
        R u1 = v1 - (hs2 * r0 - hs0 * r2);
        R u2 = v2 - (hs0 * r1 - hs1 * r0);
        R gv = -k.eta4 * I.V * J.V * Fk;
        c0 += gv * u0; c1 += gv * u1; c2 += gv * u2;
    }
    f[0] = f0 + c0; f[1] = f1 + c1; f[2] = f2 + c2;
    n[0] = n0 + (R)-0.5 * (r1 * c2 - r2 * c1);
    n[1] = n1 + (R)-0.5 * (r2 * c0 - r0 * c2);
    n[2] = (R)-0.5 * (r0 * c1 - r1 * c0);
}

template <typename R>
__device__ __forceinline__ uint32_t force_finish(const DevState &s, const InstDesc *d, uint32_t p,
                                                 int spi, const double F[3], const double T[3])
{
    R *acc = (R *)s.acc, *alpha = (R *)s.alpha;
    const uint32_t N = s.N;
    const double im = d->inv_mass[spi], iI = d->inv_inertia[spi];
    uint32_t err = 0;
    for (int a = 0; a < 3; a++) {
        double av = F[a] * im, al = T[a] * iI;
        acc[a * N + p] = (R)av;
        alpha[a * N + p] = (R)al;
        if (!isfinite(av) || !isfinite(al)) err |= ERR_NONFINITE;
    }
    return err;
}

template <typename R>
__device__ __forceinline__ ForceP<R> force_particle_in(const DevState &s, const InstDesc *d,
                                                       uint32_t q, int sp)
{
    const R *A = (const R *)s.aux + 4 * (size_t)q;
    ForceP<R> P;
    P.sp = sp;
    P.m = (R)d->mass[sp];
    P.V = A[0];
    P.Pr = A[1];
    P.ir2 = A[2];
    P.VS = A[3];
    return P;
}

// Pair forces and spin torques on particle p (walls get zero: their motion is imposed),
// walking its cell stencil.
template <typename R, bool KAHAN>
__device__ __forceinline__ uint32_t force_one(const DevState &s, const InstDesc *d, uint32_t p)
{
    const uint32_t N = s.N;
    const int cur = s.cur;
    const uint8_t *SK = s.sk[cur];
    const uint8_t ski = SK[p];
    if ((ski >> 1) != KIND_FLUID) {
        const double z[3] = {0.0, 0.0, 0.0};
        return force_finish<R>(s, d, p, ski & 1, z, z);
    }
    const double *X = s.x[cur], *Vv = s.v[cur], *Ww = s.w[cur];
    const double xi0 = X[p], xi1 = X[N + p], xi2 = X[2 * N + p];
    const double vi0 = Vv[p], vi1 = Vv[N + p], vi2 = Vv[2 * N + p];
    const double wi0 = Ww[p], wi1 = Ww[N + p], wi2 = Ww[2 * N + p];
    const ForceK<R> K(d);
    const ForceP<R> I = force_particle_in<R>(s, d, p, ski & 1);
    const double cut2 = d->cut2;
    const uint32_t cxyz = s.cell_xyz[s.pcell[p]];
    uint32_t err = 0;
    Acc<R, KAHAN> F0, F1, F2, T0, T1, T2;
    for_each_cell(s, d, cxyz & 1023, (cxyz >> 10) & 1023, cxyz >> 20, err,
                  [&](uint32_t b, uint32_t e) {
        for (uint32_t q = b; q < e; ++q) {
            const double xq0 = X[q], xq1 = X[N + q], xq2 = X[2 * N + q];
            double dx0 = min_img(d, 0, xi0 - xq0);
            double dx1 = min_img(d, 1, xi1 - xq1);
            double dx2 = min_img(d, 2, xi2 - xq2);
            double r2d = r2_exact(dx0, dx1, dx2);
            if (!(r2d < cut2) || q == p) continue;
            const ForceP<R> J = force_particle_in<R>(s, d, q, SK[q] & 1);
            R f[3], n[3];
            pair_force<R>(K, I, J, (R)dx0, (R)dx1, (R)dx2, (R)r2d,
                          (R)(vi0 - Vv[q]), (R)(vi1 - Vv[N + q]), (R)(vi2 - Vv[2 * N + q]),
                          (R)(0.5 * (wi0 + Ww[q])), (R)(0.5 * (wi1 + Ww[N + q])),
                          (R)(0.5 * (wi2 + Ww[2 * N + q])), f, n);
            F0.add(f[0]); F1.add(f[1]); F2.add(f[2]);
            T0.add(n[0]); T1.add(n[1]); T2.add(n[2]);
        }
    });
    const double F[3] = {F0.value(), F1.value(), F2.value()};
    const double T[3] = {T0.value(), T1.value(), T2.value()};
    return err | force_finish<R>(s, d, p, ski & 1, F, T);
}

template <typename R, bool KAHAN>
__global__ void k_force(DevState s)
{
    PIdx t = map_thread(s);
    if (!t.active) return;
    uint32_t err = force_one<R, KAHAN>(s, t.d, t.p);
    if (err) atomicOr(s.err, err);
}

// Pressure filter of particle p (Algorithm 1, after the EOS): the volume-weighted Shepard
// average of the pressure over p and its fluid and inner-wall neighbours,
//   P~ = (V_p P_p W(0) + sum V_q P_q W_pq) / (V_p W(0) + sum V_q W_pq).
// Outer walls are not averaged and are not sources.  Reads V (aux) and P (rhoP), writes
// P~ to pf and P~/rho^2 to aux, which the filter itself does not read.
template <typename R, bool KAHAN>
__device__ __forceinline__ uint32_t filter_one(const DevState &s, const InstDesc *d, uint32_t p)
{
    const uint32_t N = s.N;
    const int cur = s.cur;
    const uint8_t *SK = s.sk[cur];
    R *AUX = (R *)s.aux;
    const R *RP = (const R *)s.rhoP;
    R *PF = (R *)s.pf;
    if ((SK[p] >> 1) == KIND_WALL_OUTER) {
        PF[p] = RP[2 * (size_t)p + 1];
        return 0u;
    }
    const double *X = s.x[cur];
    const double xi0 = X[p], xi1 = X[N + p], xi2 = X[2 * N + p];
    const uint32_t cxyz = s.cell_xyz[s.pcell[p]];
    const int kernel = d->kernel;
    const double cut2 = d->cut2;
    const R inv_h = (R)d->inv_h, wnorm = (R)d->wnorm;
    uint32_t err = 0;
    Acc<R, KAHAN> num, den;
    for_each_cell(s, d, cxyz & 1023, (cxyz >> 10) & 1023, cxyz >> 20, err,
                  [&](uint32_t b, uint32_t e) {
        for (uint32_t q = b; q < e; ++q) {
            const double xq0 = X[q], xq1 = X[N + q], xq2 = X[2 * N + q];
            double r2 = r2_exact(min_img(d, 0, xi0 - xq0), min_img(d, 1, xi1 - xq1),
                                 min_img(d, 2, xi2 - xq2));
            if (!(r2 < cut2) || q == p || (SK[q] >> 1) == KIND_WALL_OUTER) continue;
            const R W = kernel_W<R>(kernel, (R)r2, inv_h, wnorm);
            const R Vq = AUX[4 * (size_t)q];
            num.add(Vq * RP[2 * (size_t)q + 1] * W);
            den.add(Vq * W);
        }
    });
    const double Vp = (double)AUX[4 * (size_t)p], Pp = (double)RP[2 * (size_t)p + 1];
    const double Pt = (Vp * Pp * d->W0 + num.value()) / (Vp * d->W0 + den.value());
    PF[p] = (R)Pt;
    AUX[4 * (size_t)p + 1] = (R)(Pt * (double)AUX[4 * (size_t)p + 2]);
    return err | (isfinite(Pt) ? 0u : (uint32_t)ERR_NONFINITE);
}

template <typename R, bool KAHAN>
__global__ void k_filter(DevState s)
{
    PIdx t = map_thread(s);
    if (!t.active || !t.d->pfilter) return;
    uint32_t err = filter_one<R, KAHAN>(s, t.d, t.p);
    if (err) atomicOr(s.err, err);
}

// Collision step (Algorithm 1), decided and computed in FP64 on both paths, for the
// instances that have it on.  A fluid particle i closer than rc to a neighbour j that it
// approaches ((v_i - v_j).(x_i - x_j) < 0) takes
//   dv_i = -(1 + e) mu (v_ij . r_ij) / |r_ij|^2 r_ij,  mu = m_j / (m_i + m_j), 1 for walls,
// summed over all such neighbours from the velocities before the step; the new velocities
// go to the other velocity buffer (free between the reorder and the next step's) and
// k_collide_apply copies them back.  Neither the density nor the pressure filter reads
// velocities, so the step may run after them.  A particle takes either the near
// neighbours the brick density sweep listed for it, or a walk over the cells within rc
// (rc < 2h; the test on each axis keeps a margin, so pruning never drops a pair).

// Impulse on fluid particle i (mass mi, velocity vi) from neighbour q at r = x_i - x_q
// (minimum image, r2 = |r|^2 < rc^2), added to dv when the pair approaches.
__device__ __forceinline__ void collide_term(const InstDesc *d, double mi, const double vi[3],
                                             const double *Vv, uint32_t N, uint32_t q,
                                             uint8_t skq, double r0, double r1, double r2,
                                             double rr, double dv[3])
{
    double vn;
    {
#pragma clang fp contract(off)
        vn = (vi[0] - Vv[q]) * r0;
        vn = vn + (vi[1] - Vv[N + q]) * r1;
        vn = vn + (vi[2] - Vv[2 * N + q]) * r2;
    }
    if (!(vn < 0.0)) return;
    const double mu = (skq >> 1) == KIND_FLUID ? d->mass[skq & 1] / (mi + d->mass[skq & 1]) : 1.0;
    const double g = -d->coll_e1 * mu * vn / rr;
    dv[0] += g * r0;
    dv[1] += g * r1;
    dv[2] += g * r2;
}

// The collision step of fluid particle p, walking the cells within rc; writes its new
// velocity to the other velocity buffer.
__device__ __forceinline__ uint32_t collide_one(const DevState &s, const InstDesc *d, uint32_t p)
{
    const uint32_t N = s.N;
    const int cur = s.cur;
    const uint8_t *SK = s.sk[cur];
    const uint8_t ski = SK[p];
    if ((ski >> 1) != KIND_FLUID) return 0u;
    const double *X = s.x[cur], *Vv = s.v[cur];
    double *VN = s.v[cur ^ 1];
    const double xi[3] = {X[p], X[N + p], X[2 * N + p]};
    const double vi[3] = {Vv[p], Vv[N + p], Vv[2 * N + p]};
    const uint32_t cxyz = s.cell_xyz[s.pcell[p]];
    const int c[3] = {(int)(cxyz & 1023), (int)((cxyz >> 10) & 1023), (int)(cxyz >> 20)};
    // cell offsets on each axis whose slab lies within rc of the particle
    int olo[3], ohi[3];
    for (int a = 0; a < 3; a++) {
        const double e = d->edge[a], reach = d->coll_rc + 1e-6 * e;
        const double below = xi[a] - (d->lo[a] + (double)c[a] * e);  // to the cell's lower face
        const double above = e - below;                                // to its upper face
        olo[a] = 0;
        ohi[a] = 0;
        for (int o = 1; o <= d->cf; o++) {
            if (below + (double)(o - 1) * e < reach) olo[a] = -o;
            if (above + (double)(o - 1) * e < reach) ohi[a] = o;
        }
    }
    const double mi = d->mass[ski & 1], rc2 = d->coll_rc2;
    uint32_t err = 0;
    double dv[3] = {0.0, 0.0, 0.0};
    for_cells_in(s, d, c[0], c[1], c[2], olo, ohi, err, [&](uint32_t b, uint32_t e) {
        for (uint32_t q = b; q < e; ++q) {
            if (q == p) continue;
            const double r0 = min_img(d, 0, xi[0] - X[q]);
            const double r1 = min_img(d, 1, xi[1] - X[N + q]);
            const double r2 = min_img(d, 2, xi[2] - X[2 * N + q]);
            const double rr = r2_exact(r0, r1, r2);
            if (rr < rc2) collide_term(d, mi, vi, Vv, N, q, SK[q], r0, r1, r2, rr, dv);
        }
    });
    for (int a = 0; a < 3; a++) {
        const double vnew = vi[a] + dv[a];
        VN[(size_t)a * N + p] = vnew;
        if (!isfinite(vnew)) err |= ERR_NONFINITE;
    }
    return err;
}

// The collision step of fluid particle p over the near neighbours the brick density sweep
// listed for it (n of them, in sorted-index order so that the sum does not depend on the
// order the lanes listed them).
__device__ __forceinline__ uint32_t collide_listed(const DevState &s, const InstDesc *d, uint32_t p,
                                                   uint32_t n)
{
    const uint32_t N = s.N;
    const int cur = s.cur;
    const uint8_t *SK = s.sk[cur];
    const uint8_t ski = SK[p];
    if ((ski >> 1) != KIND_FLUID) return 0u;
    const double *X = s.x[cur], *Vv = s.v[cur];
    double *VN = s.v[cur ^ 1];
    uint32_t q[kNearCap];
    for (uint32_t a = 0; a < n; a++) {
        uint32_t v = s.nearq[(size_t)p * kNearCap + a], b = a;
        for (; b > 0 && q[b - 1] > v; b--) q[b] = q[b - 1];
        q[b] = v;
    }
    const double xi[3] = {X[p], X[N + p], X[2 * N + p]};
    const double vi[3] = {Vv[p], Vv[N + p], Vv[2 * N + p]};
    const double mi = d->mass[ski & 1], rc2 = d->coll_rc2;
    double dv[3] = {0.0, 0.0, 0.0};
    for (uint32_t a = 0; a < n; a++) {
        const uint32_t j = q[a];
        const double r0 = min_img(d, 0, xi[0] - X[j]);
        const double r1 = min_img(d, 1, xi[1] - X[N + j]);
        const double r2 = min_img(d, 2, xi[2] - X[2 * N + j]);
        const double rr = r2_exact(r0, r1, r2);
        if (rr < rc2) collide_term(d, mi, vi, Vv, N, j, SK[j], r0, r1, r2, rr, dv);
    }
    uint32_t err = 0;
    for (int a = 0; a < 3; a++) {
        const double vnew = vi[a] + dv[a];
        VN[(size_t)a * N + p] = vnew;
        if (!isfinite(vnew)) err |= ERR_NONFINITE;
    }
    return err;
}

// listed: the brick density sweep of this step left cflag = number of listed near
// neighbours (0: none, kNearOverflow: more than kNearCap, or not listed: walk the cells).
__global__ void k_collide(DevState s, int listed)
{
    PIdx t = map_thread(s);
    if (!t.active || !t.d->coll) return;
    const uint32_t f = listed ? s.cflag[t.p] : (uint32_t)kNearOverflow;
    if (f == 0) return;
    const uint32_t err = f == (uint32_t)kNearOverflow ? collide_one(s, t.d, t.p)
                                                      : collide_listed(s, t.d, t.p, f);
    if (err) atomicOr(s.err, err);
}

__global__ void k_collide_apply(DevState s, int listed)
{
    PIdx t = map_thread(s);
    if (!t.active || !t.d->coll) return;
    const uint32_t N = s.N, p = t.p;
    const int cur = s.cur;
    if ((listed && !s.cflag[p]) || (s.sk[cur][p] >> 1) != KIND_FLUID) return;
    for (int a = 0; a < 3; a++) s.v[cur][(size_t)a * N + p] = s.v[cur ^ 1][(size_t)a * N + p];
}

// ------------------------------------------------------------ brick sweeps ----------
//
// One workgroup per brick of 2x2x2 cells (edge >= 2h each).  The 4x4x4 cells around the
// brick (its neighbourhood, periodic images shifted into the brick's frame) are staged in
// LDS in slot order, x fastest, so the 27-cell stencil of a target cell is 9 contiguous
// runs ("rows").  Wave w serves brick cell w.  Positions and velocities are staged in
// single precision relative to the brick centre (and to one particle's velocity), in units
// of h (FP32-mixed path); neighbourhoods too large to stage fall back to the per-particle
// code.

constexpr int kBrickThreads = 512;
constexpr int kStageDensity = 2048;
constexpr int kStageForce = 1408;
// The force sweep and the pressure filter replay masks only for bricks the density sweep
// could stage: a brick too large for the density stage must be too large for theirs.
static_assert(kStageForce <= kStageDensity, "mask replay needs the density sweep's masks");

struct BrickFrame {
    uint32_t begin[64];   // sorted index of each slot's first particle
    uint32_t off[65];     // staged index of each slot's first particle (prefix of counts)
    double shift[64][3];  // periodic image shift of each slot
    double origin[3];     // brick centre
    uint32_t ok;          // 0: too many particles to stage (per-thread fallback)
};

__device__ __forceinline__ int slot_index(int x, int y, int z) { return x + 4 * (y + 4 * z); }

// Hands LDS data written by some lanes of a wave to other lanes of the same wave.  A bare
// wave barrier orders execution only: the compiler may still move or overlap the LDS
// accesses around it.  Here the fences keep LDS accesses on their side, and the wave waits
// until its own LDS writes are complete (lgkmcnt 0; vector memory counters untouched).
__device__ __forceinline__ void wave_lds_handoff()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0), vmcnt(63), expcnt(7)
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Slot t (x + 4y + 16z over the 4x4x4 neighbourhood) of brick bxyz: its cell (wrapped on
// periodic axes, with the image shift in sh) and whether the cell lies in the grid.
__device__ __forceinline__ bool slot_cell(const InstDesc *d, uint32_t bxyz, int t, int c[3], double sh[3])
{
    const int b[3] = {(int)(bxyz & 1023), (int)((bxyz >> 10) & 1023), (int)(bxyz >> 20)};
    const int i[3] = {t & 3, (t >> 2) & 3, t >> 4};
    bool valid = true;
    for (int a = 0; a < 3; a++) {
        c[a] = 2 * b[a] + i[a] - 1;
        sh[a] = 0.0;
        if (d->periodic[a]) {
            if (c[a] < 0) { c[a] += d->n[a]; sh[a] = -d->L[a]; }
            else if (c[a] >= d->n[a]) { c[a] -= d->n[a]; sh[a] = d->L[a]; }
        } else if (c[a] < 0 || c[a] >= d->n[a]) {
            valid = false;
        }
    }
    return valid;
}

// The frames of all bricks, once per step (after the cell list): per brick, the sorted index
// of each slot's first particle and the inclusive prefix of the slot counts, [64] + [64]
// words.  The brick sweeps then set up a brick with one coalesced load instead of a chain
// of dependent loads through the cell tables.
__global__ void __launch_bounds__(64) k_brick_frames(DevState s)
{
    const uint32_t brick = blockIdx.x;
    const int t = threadIdx.x;
    const InstDesc *d = s.desc + s.brick_inst[brick];
    int c[3];
    double sh[3];
    uint32_t beg = 0, cnt = 0;
    if (slot_cell(d, s.brick_xyz[brick], t, c, sh)) {
        const uint32_t lin = (uint32_t)c[0] +
                             (uint32_t)d->n[0] * ((uint32_t)c[1] + (uint32_t)d->n[1] * (uint32_t)c[2]);
        const uint32_t r = s.rank_of_lin[d->cell_off + lin];
        beg = s.start[r];
        cnt = s.start[r + 1] - beg;
    }
    uint32_t inc = cnt;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o);
        if (t >= o) inc += y;
    }
    s.bframe[(size_t)brick * 128 + t] = beg;
    s.bframe[(size_t)brick * 128 + 64 + t] = inc;
}

// Fills the frame from the brick's precomputed slots (wave 0: one lane per slot) and returns
// the staged particle count; F.ok tells whether they fit stage_max.  With Vv, the lane of
// slot (1,1,1), the brick's first cell, also loads the velocity of that cell's first
// particle into vref.
__device__ __forceinline__ uint32_t brick_frame(const DevState &s, const InstDesc *d, uint32_t brick,
                                            uint32_t bxyz, BrickFrame &F, int stage_max,
                                            const double *Vv = nullptr, double *vref = nullptr)
{
    const int t = threadIdx.x;
    if (t < 64) {
        const uint32_t beg = s.bframe[(size_t)brick * 128 + t];
        const uint32_t inc = s.bframe[(size_t)brick * 128 + 64 + t];
        int c[3];
        double sh[3];
        slot_cell(d, bxyz, t, c, sh);
        for (int a = 0; a < 3; a++) F.shift[t][a] = sh[a];
        const uint32_t below = __shfl_up(inc, 1);
        const uint32_t cnt = inc - (t ? below : 0u);
        F.begin[t] = beg;
        F.off[t + 1] = inc;
        if (t == 0) F.off[0] = 0;
        const bool over = __any(cnt > (uint32_t)kMaxCell);
        if (t == 63) F.ok = !over && inc <= (uint32_t)stage_max;
        if (t < 3) F.origin[t] = d->lo[t] + (double)(2 * (int)((bxyz >> (10 * t)) & 1023) + 1) * d->edge[t];
        if (Vv && t == slot_index(1, 1, 1))
            for (int a = 0; a < 3; a++) vref[a] = cnt ? Vv[(size_t)a * s.N + beg] : 0.0;
    }
    __syncthreads();
    return F.off[64];
}

// Slot of staged particle k (largest slot whose first staged index is <= k).
__device__ __forceinline__ int slot_of(const BrickFrame &F, uint32_t k)
{
    int lo = 0, hi = 63;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (F.off[mid] <= k) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The brick cell served by wave w: its slot, and whether it lies in the grid.
__device__ __forceinline__ bool brick_target(const InstDesc *d, uint32_t bxyz, int w, int ts[3])
{
    const int b[3] = {(int)(bxyz & 1023), (int)((bxyz >> 10) & 1023), (int)(bxyz >> 20)};
    const int o[3] = {w & 1, (w >> 1) & 1, w >> 2};
    bool in = true;
    for (int a = 0; a < 3; a++) {
        ts[a] = 1 + o[a];
        if (2 * b[a] + o[a] >= d->n[a]) in = false;
    }
    return in;
}


// Particles in the brick's own cells that lie in the grid (every thread, from the frame in
// LDS, so the same value on the whole workgroup).  The brick list covers the instance's box,
// so a brick outside a curved container holds none and its workgroup has nothing to do.
__device__ __forceinline__ uint32_t brick_own_count(const BrickFrame &F, const InstDesc *d, uint32_t bxyz)
{
    uint32_t n = 0;
    for (int w = 0; w < 8; w++) {
        int ts[3];
        if (brick_target(d, bxyz, w, ts)) {
            const int sl = slot_index(ts[0], ts[1], ts[2]);
            n += F.off[sl + 1] - F.off[sl];
        }
    }
    return n;
}

// Sum of the G partial sums of a target, held by lanes t, t + ntc, ... (t < ntc): a tree
// over the groups in a fixed order, in FP64; the total is valid on lane t.  group_total
// takes a Kahan pair (s, c).
__device__ __forceinline__ double group_total_d(double v, int lane, int ntc, int G)
{
    const int g = lane / ntc;
    for (int off = 1; off < G; off <<= 1) {
        const int src = lane + off * ntc;
        const double o = __shfl(v, src < 64 ? src : lane);
        if ((g & (2 * off - 1)) == 0 && g + off < G) v += o;
    }
    return v;
}

__device__ __forceinline__ double group_total(float s_, float c_, int lane, int ntc, int G)
{
    return group_total_d((double)s_ - (double)c_, lane, ntc, G);
}

// Clears the k lowest set bits of m (k < popcount(m)): a binary search for the position of
// set bit k, halving the span six times.
__device__ __forceinline__ uint64_t drop_low_bits(uint64_t m, uint32_t k)
{
    uint32_t pos = 0;
    for (uint32_t w = 32; w >= 1; w >>= 1) {
        const uint32_t n = (uint32_t)__popcll((m >> pos) & ((1ull << w) - 1ull));
        if (n <= k) {
            k -= n;
            pos += w;
        }
    }
    return m & ~((1ull << pos) - 1ull);
}

// Density staging walks the 64 slots of the neighbourhood with kSlotThreads threads each:
// thread `sub` of a slot takes its particles sub, sub + kSlotThreads, ..., two at a time
// so that their loads are in flight together.
constexpr int kSlotThreads = kBrickThreads / 64;
static_assert(kSlotThreads * 64 == kBrickThreads, "staging assigns whole slots to threads");

// Stages the positions of the brick's neighbourhood particles relative to the brick centre
// in units of h (FP64 difference and scaling, then FP32) and their species.
__device__ __forceinline__ void stage_density(const DevState &s, const BrickFrame &F, double ih,
                                              float4 *stage)
{
    const uint32_t N = s.N;
    const double *X = s.x[s.cur];
    const uint8_t *SK = s.sk[s.cur];
    const int sl = (int)threadIdx.x / kSlotThreads;
    const uint32_t sub = threadIdx.x % kSlotThreads;
    const uint32_t off = F.off[sl], cnt = F.off[sl + 1] - off, beg = F.begin[sl];
    for (uint32_t k0 = sub; k0 < cnt; k0 += 2 * kSlotThreads) {
        double px[2][3];
        uint8_t sk[2];
        for (int u = 0; u < 2; u++) {
            const uint32_t q = beg + min(k0 + (uint32_t)(u * kSlotThreads), cnt - 1);
            for (int a = 0; a < 3; a++) px[u][a] = X[(size_t)a * N + q];
            sk[u] = SK[q];
        }
        for (int u = 0; u < 2; u++) {
            const uint32_t k = k0 + (uint32_t)(u * kSlotThreads);
            if (k >= cnt) break;
            float4 v;
            v.x = (float)(((px[u][0] + F.shift[sl][0]) - F.origin[0]) * ih);
            v.y = (float)(((px[u][1] + F.shift[sl][1]) - F.origin[1]) * ih);
            v.z = (float)(((px[u][2] + F.shift[sl][2]) - F.origin[2]) * ih);
            v.w = (float)(sk[u] & 1);
            stage[off + k] = v;
        }
    }
}

// Spreads the brick's M staged particles over the workgroup, up to three per thread (k,
// k + 512, k + 1024 from threadIdx.x), spaced evenly over the neighbourhood: load(u, q)
// issues the loads of particle u (sorted index q) for all three first, so that they are in
// flight together, then store(u, k, slot) writes staged particle k of that slot.
template <class Load, class Store>
__device__ __forceinline__ void stage_spread(const BrickFrame &F, uint32_t M, Load &&load,
                                             Store &&store)
{
    for (uint32_t k0 = threadIdx.x; k0 < M; k0 += 3 * kBrickThreads) {
        uint32_t kk[3], qq[3];
        int sl[3];
        for (int u = 0; u < 3; u++) {
            kk[u] = k0 + (uint32_t)u * kBrickThreads;
            sl[u] = slot_of(F, min(kk[u], M - 1));
            qq[u] = F.begin[sl[u]] + (min(kk[u], M - 1) - F.off[sl[u]]);
        }
        for (int u = 0; u < 3; u++) load(u, qq[u]);
        for (int u = 0; u < 3; u++) {
            if (kk[u] >= M) break;
            store(u, kk[u], sl[u]);
        }
    }
}

// Stages what the force sweep reads of the brick's M neighbourhood particles: position
// relative to the brick centre and P/rho^2; velocity relative to vref and V (negative for
// the viscous species); half the spin (exact, so (w_i + w_j)/2 takes one add) and V/S.
// Positions and velocities are in units of h (ih = 1/h, applied in FP64).  Particles are
// spread over the threads by stage_spread (the heavier force staging prefers this to
// whole slots).
__device__ __forceinline__ void stage_force(const DevState &s, const BrickFrame &F, uint32_t M,
                                            const double *vref, double ih, float4 *SA, float4 *SB,
                                            float4 *SC)
{
    const uint32_t N = s.N;
    const int cur = s.cur;
    const double *X = s.x[cur], *Vv = s.v[cur], *Ww = s.w[cur];
    const uint8_t *SK = s.sk[cur];
    const float *AUX = (const float *)s.aux;
    double px[3][3], pv[3][3], pw[3][3];
    float4 aq[3];
    uint8_t sk[3];
    stage_spread(F, M, [&](int u, uint32_t q) {
        for (int a = 0; a < 3; a++) {
            px[u][a] = X[(size_t)a * N + q];
            pv[u][a] = Vv[(size_t)a * N + q];
            pw[u][a] = Ww[(size_t)a * N + q];
        }
        aq[u] = *(const float4 *)(AUX + 4 * (size_t)q);
        sk[u] = SK[q];
    }, [&](int u, uint32_t k, int sl) {
        SA[k] = make_float4((float)(((px[u][0] + F.shift[sl][0]) - F.origin[0]) * ih),
                            (float)(((px[u][1] + F.shift[sl][1]) - F.origin[1]) * ih),
                            (float)(((px[u][2] + F.shift[sl][2]) - F.origin[2]) * ih), aq[u].y);
        SB[k] = make_float4((float)((pv[u][0] - vref[0]) * ih), (float)((pv[u][1] - vref[1]) * ih),
                            (float)((pv[u][2] - vref[2]) * ih), (sk[u] & 1) ? -aq[u].x : aq[u].x);
        SC[k] = make_float4((float)(0.5 * pw[u][0]), (float)(0.5 * pw[u][1]), (float)(0.5 * pw[u][2]),
                            aq[u].w);
    });
}

__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ---------------------------------------------------------- staged FP32 pair terms ---
// The brick sweeps stage positions and velocities in units of h (r_s = r/h, v_s = v/h), so
// that q = |r_s|.  The kernels enter through their shapes: W = wnorm What(q) and
// F = -W'/r = wnorm cF Fhat(q) / h^2, cF = 5 for Wendland C2 (What = t^4 (2q + 1),
// Fhat = t^3, t = 1 - q/2) and 1 for the cubic spline (Sec. 2.2 kernels).  The constant
// factors go into per-brick and per-target coefficients, once.

// What(q) alone (density sweep), q = sqrt(r2s).
template <int KT>
__device__ __forceinline__ float shape_W(float r2s)
{
    const float q = fast_sqrt(r2s);
    if (KT == KERNEL_WENDLAND) {
        const float t = 1.0f - 0.5f * q;
        const float t2 = t * t;
        return t2 * t2 * (2.0f * q + 1.0f);
    }
    if (q < 1.0f) return 1.0f - 1.5f * q * q + 0.75f * q * q * q;
    const float t = 2.0f - q;
    return 0.25f * t * t * t;
}

// What(q) and Fhat(q) (force sweep), q = sqrt(r2s).
template <int KT>
__device__ __forceinline__ void shape_WF(float r2s, float &W, float &F)
{
    const float q = fast_sqrt(r2s);
    if (KT == KERNEL_WENDLAND) {
        const float t = 1.0f - 0.5f * q;
        const float t3 = t * t * t;
        F = t3;
        W = t3 * t * (2.0f * q + 1.0f);
    } else if (q < 1.0f) {
        W = 1.0f - 1.5f * q * q + 0.75f * q * q * q;
        F = 3.0f - 2.25f * q;
    } else {
        const float t = 2.0f - q;
        W = 0.25f * t * t * t;
        F = 0.75f * t * t * fast_rcp(q);
    }
}

// Per-brick coefficients of the staged force terms.  With r = h r_s and v = h v_s every
// coefficient that multiplies r_s or v_s carries one factor h, so the force comes out in
// true units and the accumulated torque n' gives the true one as -(h/2) n'.
struct PairK {
    float kM;        // h m0^2 F / Fhat = m0^2 wnorm cF / h
    float mu1;       // m1 / m0
    float ks0, ks1;  // -sigma_T / m_s^2, so -sigma_T / rho_j^2 = ks_j V_j^2
    float kC;        // -C_l h wnorm
    float ke;        // -4 eta / (m0 m1)
    __device__ explicit PairK(const InstDesc *d)
    {
        const double cF = d->kernel == KERNEL_WENDLAND ? 5.0 : 1.0;
        kM = (float)(d->mass[0] * d->mass[0] * d->wnorm * cF * d->inv_h);
        mu1 = (float)(d->mass[1] / d->mass[0]);
        ks0 = (float)(-d->sigma_T / (d->mass[0] * d->mass[0]));
        ks1 = (float)(-d->sigma_T / (d->mass[1] * d->mass[1]));
        kC = (float)(-d->C_l * d->h * d->wnorm);
        ke = (float)(-4.0 * d->eta / (d->mass[0] * d->mass[1]));
    }
};

// Target-side factors, from the target's staged values (SA.w = P/rho^2, SB.w = V with the
// sign of the species, SC.w = V/S).
struct PairI {
    float kM;   // kM m_i / m0
    float Pr;   // P_i / rho_i^2
    float sT;   // -sigma_T / rho_i^2
    float cVS;  // kC V_i / S_i
    float ev;   // viscous target: ke V_i m0 / m_i; 0 for the other species
    bool sp;    // viscous species
};

__device__ __forceinline__ PairI pair_target(const PairK &k, float4 A, float4 B, float4 C)
{
    PairI I;
    const bool sp = B.w < 0.0f;
    const float V = fabsf(B.w);
    I.kM = sp ? k.kM * k.mu1 : k.kM;
    I.Pr = A.w;
    I.sT = V * V * (sp ? k.ks1 : k.ks0);
    I.cVS = k.kC * C.w;
    I.ev = sp ? k.ke * V / k.mu1 : 0.0f;
    I.sp = sp;
    return I;
}

// Force f on target i from staged neighbour j (A, B, C) and the torque term n' that both
// receive, the pair terms of Sec. 2.1:
//   pressure     m_i m_j (P_i/rho_i^2 + P_j/rho_j^2) F r
//   interfacial  g_T (r_x, r_y, 0), g_T = -sigma_T m_i m_j (1/rho_i^2 + 1/rho_j^2) F, unlike
//   viscous      -4 eta V_i V_j F (v - hs x r), viscous-viscous pairs
//   friction     -C_l W (V_i/S_i + V_j/S_j) v, unlike pairs
//   torque       -1/2 r x (non-central force), returned as n' with torque = -(h/2) n'
// r = r_s (units of h) = x_i - x_j, v = v_s = v_i - v_j, hs = (w_i + w_j)/2.  No branch on
// the species: the unlike terms are selected, the viscous-viscous one vanishes through
// I.ev and V_j taken only for a viscous neighbour (B.w = -V_j).  EQM: equal species masses.
template <int KT, bool EQM, bool VISC = true>
__device__ __forceinline__ void pair_force_f32(const PairK &k, const PairI &I, float4 A, float4 B,
                                               float4 C, float r0, float r1, float r2, float v0,
                                               float v1, float v2, float hs0, float hs1, float hs2,
                                               float f[3], float n[3])
{
    float W, Fh;
    shape_WF<KT>(r0 * r0 + r1 * r1 + r2 * r2, W, Fh);
    const bool spj = B.w < 0.0f;
    const bool unl = spj != I.sp;  // a scalar xor of lane masks
    const float mF = (EQM ? I.kM : I.kM * (spj ? k.mu1 : 1.0f)) * Fh;
    const float gp = mF * (I.Pr + A.w);
    const float sT = fmaf(B.w * B.w, EQM ? k.ks0 : (spj ? k.ks1 : k.ks0), I.sT);
    const float gT = unl ? mF * sT : 0.0f;
    const float gm = unl ? W * fmaf(C.w, k.kC, I.cVS) : 0.0f;
    // non-central part c = gm v + gv u, u = v - hs x r; without VISC (an inviscid target,
    // I.ev = 0) gv is zero and c = gm v, the same value the full form gives
    float c0, c1, c2;
    if (VISC) {
        const float gv = I.ev * (spj ? -B.w : 0.0f) * mF;
        const float u0 = fmaf(hs2, r1, fmaf(-hs1, r2, v0));
        const float u1 = fmaf(hs0, r2, fmaf(-hs2, r0, v1));
        const float u2 = fmaf(hs1, r0, fmaf(-hs0, r1, v2));
        c0 = fmaf(gm, v0, gv * u0);
        c1 = fmaf(gm, v1, gv * u1);
        c2 = fmaf(gm, v2, gv * u2);
    } else {
        c0 = gm * v0;
        c1 = gm * v1;
        c2 = gm * v2;
    }
    const float gh = gp + gT;
    f[0] = fmaf(gh, r0, c0);
    f[1] = fmaf(gh, r1, c1);
    f[2] = fmaf(gp, r2, c2);
    // n' = r x c - gT r_z (r_y, -r_x, 0)
    const float dz = fmaf(-gT, r2, c2);
    n[0] = fmaf(r1, dz, -r2 * c1);
    n[1] = fmaf(r2, c0, -r0 * dz);
    n[2] = fmaf(r0, c1, -r1 * c0);
}

// ------------------------------------------------------ candidate-major brick sweeps ---
// The wave of a target cell lays the candidates of its 27-cell stencil (nine rows of three
// x-adjacent cells, each a contiguous run of the staged particles) out as one list, held
// in registers as windows of 64 candidates, one per lane.  Testing one target against a
// window is then one 64-lane comparison whose ballot is the window's hit mask, so targets
// are tested one after another with every lane busy.  The density sweep stores the masks
// (one word per window and target); the pressure filter and the force sweep replay them.
// Pair terms are evaluated with lanes = (target, group g of G): group g takes the g-th of
// G equal consecutive shares of the target's hits in list order.

constexpr int kCandWin = 10;      // windows per wave: stencils of up to 640 candidates
constexpr int kListTargets = 32;  // largest number of targets per round of the density sweep
static_assert(kCandWin <= kMaskSlots, "a target's masks must fit its mask slots");
static_assert(kStageDensity <= 32767 && kStageForce <= 32767, "staged indices are int16");

// The nine stencil rows of a target cell as one list: writes the staged index of every
// list position below kCandWin * 64 into the wave's table (row by row, lanes along the
// row) and returns the list length, its windows of 64 and the offset from list position
// to staged index in row 4, whose middle cell is the target's own.
struct StencilList {
    uint32_t C, NW;
    int32_t self_off;
};

__device__ __forceinline__ StencilList stencil_list(const BrickFrame &F, const int ts[3], int lane,
                                                    int16_t *tbl)
{
    StencilList S;
    uint32_t acc = 0;
    S.self_off = 0;
#pragma unroll
    for (int r = 0; r < 9; r++) {
        const int s0 = slot_index(ts[0] - 1, ts[1] - 1 + r % 3, ts[2] - 1 + r / 3);
        const uint32_t b = __builtin_amdgcn_readfirstlane(F.off[s0]);
        const uint32_t e = __builtin_amdgcn_readfirstlane(F.off[s0 + 3]);
        if (r == 4) S.self_off = (int32_t)b - (int32_t)acc;
        for (uint32_t i = (uint32_t)lane; i < e - b && acc + i < (uint32_t)(kCandWin * 64); i += 64)
            tbl[acc + i] = (int16_t)(b + i);
        acc += e - b;
    }
    S.C = acc;
    S.NW = (acc + 63) / 64;
    wave_lds_handoff();
    return S;
}

// List position of the target with staged index kt.
__device__ __forceinline__ uint32_t stencil_self(const StencilList &S, uint32_t kt)
{
    return (uint32_t)((int32_t)kt - S.self_off);
}

// Workgroups are dealt to the XCDs in turn (workgroup i runs on XCD i mod kXcd).  Giving
// each XCD runs of `run` consecutive bricks of the Morton order (a tuning parameter, 1..256)
// makes the neighbourhoods that its resident workgroups stage overlap, so more staging
// loads hit that XCD's own L2, while the runs stay short enough to spread uneven work over
// all XCDs.
constexpr uint32_t kXcd = 8;
__device__ __forceinline__ uint32_t brick_of_workgroup(uint32_t wg, uint32_t nb, uint32_t run)
{
    const uint32_t P = kXcd * run, base = wg / P * P, T = min(P, nb - base), in = wg - base;
    const uint32_t q = T / kXcd, r = T % kXcd, x = in % kXcd;
    return base + x * q + min(x, r) + in / kXcd;
}

// Share g of G of a target's H hits (mask words word(0..)): hits [H g / G, H (g+1) / G) in
// list order.  Returns their count, the window c of the first and the bits of that window
// from the first on.
template <class Word>
__device__ __forceinline__ void hit_share(Word &&word, uint32_t H, int g, int G, uint32_t &cnt,
                                          int &c, uint64_t &mc)
{
    const uint32_t lo = (H * (uint32_t)g) / (uint32_t)G;
    cnt = (H * (uint32_t)(g + 1)) / (uint32_t)G - lo;
    c = 0;
    mc = 0;
    if (cnt == 0) return;
    uint32_t skip = lo;
    mc = word(0);
    uint32_t pc = (uint32_t)__popcll(mc);
    while (skip >= pc) {
        skip -= pc;
        mc = word(++c);
        pc = (uint32_t)__popcll(mc);
    }
    mc = drop_low_bits(mc, skip);
}


// A lane's share of one target's hits, replayed from the mask words the density sweep
// stored: share g of G takes hits [H g / G, H (g + 1) / G) of the H hits, in list order.
// All of the target's words are loaded at once (no chain of dependent loads); next()
// walks the share's hits in order.
struct HitReplay {
    const uint64_t *gm;
    int NW, c;
    uint32_t cnt;
    uint64_t mc, nxt;  // bits of window c still to walk; window c + 1

    __device__ __forceinline__ HitReplay(const uint64_t *gm_, int NW_, bool target, int g, int G)
        : gm(gm_), NW(NW_), c(0), mc(0), nxt(0)
    {
        uint64_t mw[kCandWin];
        uint32_t H = 0;
#pragma unroll
        for (int cc = 0; cc < kCandWin; cc++) {
            mw[cc] = (target && cc < NW) ? gm[cc] : 0ull;
            H += (uint32_t)__popcll(mw[cc]);
        }
        const uint32_t lo = (H * (uint32_t)g) / (uint32_t)G;
        cnt = (H * (uint32_t)(g + 1)) / (uint32_t)G - lo;
        uint32_t pre = 0, before = 0;
#pragma unroll
        for (int cc = 0; cc < kCandWin; cc++) {
            pre += (uint32_t)__popcll(mw[cc]);
            if (pre <= lo) {
                c = cc + 1;
                before = pre;
            }
        }
#pragma unroll
        for (int cc = 0; cc < kCandWin; cc++) {
            if (cc == c) mc = mw[cc];
            if (cc == c + 1) nxt = mw[cc];
        }
        if (cnt) mc = drop_low_bits(mc, lo - before);
    }

    // Staged index of the next hit, from the wave's list table.
    __device__ __forceinline__ uint32_t next(const int16_t (*tbl)[64])
    {
        while (mc == 0) {
            mc = nxt;
            ++c;
            nxt = c + 1 < NW ? gm[c + 1] : 0ull;
        }
        const int j = __builtin_ctzll(mc);
        mc &= mc - 1;
        return (uint32_t)tbl[c][j];
    }
};

// Ballot tests of targets kbase .. kbase + ntc - 1 (staged indices) against the first NWc
// candidate windows, NWc fixed at compile time so that the windows need no branch per
// target.  The ballots of one target stay in scalar registers until lane t copies them
// into mw, one 64-bit move per window.
// The test is |c - t|^2 < cut2 expanded as |c|^2 - 2 c.t < cut2 - |t|^2, with the
// candidate's -2c (px, py, pz) and |c|^2 (cc) precomputed: three FMAs and a compare per
// target and window.  Positions are relative to the brick centre in units of h
// (|c|^2 <= 48), so the expanded form can misjudge only pairs within a few 1e-6 of the
// support radius, where W and F are below 1e-17 of their scale.
template <int NWc>
__device__ __forceinline__ void test_targets(const float4 *stage, const float *px, const float *py,
                                             const float *pz, const float *cc, uint32_t kbase,
                                             uint32_t ntc, float cut2, int lane, uint64_t *mw)
{
    for (uint32_t t = 0; t < ntc; t++) {
        const float4 T = stage[kbase + t];
        const float thr = cut2 - (T.x * T.x + T.y * T.y + T.z * T.z);
        uint64_t m[NWc];
#pragma unroll
        for (int c = 0; c < NWc; c++) {
            const float e = fmaf(pz[c], T.z, fmaf(py[c], T.y, fmaf(px[c], T.x, cc[c])));
            m[c] = __ballot(e < thr);
        }
        if ((uint32_t)lane == t) {
#pragma unroll
            for (int c = 0; c < NWc; c++) mw[c] = m[c];
        }
    }
}

// With COLL, the sweep also lists, per target, the neighbours within the collision distance
// (plus a relative margin of 1e-4 on its square, far above the FP32 rounding of the staged
// distances): up to kNearCap sorted indices in nearq and their number in cflag, so that
// the collision step tests only those, exactly.  Targets with more, targets evaluated per
// particle (fallbacks) and collision distances near 2h get kNearOverflow: the collision
// step walks their cells.
template <bool KAHAN, bool COLL, int LT>
__global__ void __launch_bounds__(kBrickThreads) k_density_cand(DevState s)
{
    static_assert(LT >= 1 && LT <= kListTargets, "targets per round");
    __shared__ BrickFrame F;
    __shared__ float4 stage[kStageDensity];
    __shared__ int16_t tbl[kBrickThreads / 64][kCandWin][64];
    __shared__ uint64_t msk[kBrickThreads / 64][LT][kCandWin];
    __shared__ uint32_t ncnt[kBrickThreads / 64][LT];  // near neighbours listed (COLL)
    __shared__ int16_t nearl[kBrickThreads][kNearCap + 1];        // a lane's near hits (COLL;
                                                                  // the last is a spare)
    const uint32_t brick = brick_of_workgroup(blockIdx.x, gridDim.x, s.xcd_run);
    const uint32_t bxyz = s.brick_xyz[brick];
    const InstDesc *d = s.desc + s.brick_inst[brick];
    const uint8_t *SK = s.sk[s.cur];
    brick_frame(s, d, brick, bxyz, F, kStageDensity);
    if (brick_own_count(F, d, bxyz) == 0) return;  // the same for the whole workgroup
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int ts[3];
    const bool has_cell = brick_target(d, bxyz, w, ts);
    const int tslot = slot_index(ts[0], ts[1], ts[2]);
    uint32_t err = 0;
    if (!F.ok) {
        if (has_cell) {
            const uint32_t nt = F.off[tslot + 1] - F.off[tslot];
            for (uint32_t i = lane; i < nt; i += 64) {
                err |= density_one<float, KAHAN>(s, d, F.begin[tslot] + i);
                if (COLL) s.cflag[F.begin[tslot] + i] = kNearOverflow;
            }
        }
        if (err) atomicOr(s.err, err);
        return;
    }
    stage_density(s, F, d->inv_h, stage);
    __syncthreads();
    if (!has_cell) return;
    const uint32_t toff = __builtin_amdgcn_readfirstlane(F.off[tslot]);
    const uint32_t pbase = __builtin_amdgcn_readfirstlane(F.begin[tslot]);
    const uint32_t nt = __builtin_amdgcn_readfirstlane(F.off[tslot + 1]) - toff;
    if (nt == 0) return;
    const StencilList S = stencil_list(F, ts, lane, &tbl[w][0][0]);
    if (S.NW > (uint32_t)kCandWin) {
        for (uint32_t i = lane; i < nt; i += 64) {
            err |= density_one<float, KAHAN>(s, d, pbase + i);
            if (COLL) s.cflag[pbase + i] = kNearOverflow;
        }
        if (err) atomicOr(s.err, err);
        return;
    }
    float px[kCandWin], py[kCandWin], pz[kCandWin], cc[kCandWin];
#pragma unroll
    for (int c = 0; c < kCandWin; c++) {
        px[c] = py[c] = pz[c] = 0.0f;
        cc[c] = __builtin_inff();  // never within reach
        if (c < (int)S.NW && 64u * (uint32_t)c + (uint32_t)lane < S.C) {
            const float4 q = stage[tbl[w][c][lane]];
            px[c] = -2.0f * q.x;
            py[c] = -2.0f * q.y;
            pz[c] = -2.0f * q.z;
            cc[c] = q.x * q.x + q.y * q.y + q.z * q.z;
        }
    }
    const float cut2 = (float)(d->cut2 * d->inv_h * d->inv_h);  // positions in units of h
    const float rc2m = (float)(d->coll_rc2 * d->inv_h * d->inv_h * (1.0 + 1e-4));
    const bool list_ok = d->coll_rc2 < 0.9 * d->cut2;  // well inside the masks' reach
    const int kernel = d->kernel;
    // compiled once per smoothing kernel, chosen per brick (as in the force sweep)
    auto sweep = [&](auto kt) {
        constexpr int KT = decltype(kt)::value;
        for (uint32_t t0 = 0; t0 < nt; t0 += LT) {
            const uint32_t ntc = min((uint32_t)LT, nt - t0);
            // test: one target at a time against every window; lane t collects target t's
            // masks
            uint64_t mw[kCandWin];
#pragma unroll
            for (int c = 0; c < kCandWin; c++) mw[c] = 0ull;
            switch (S.NW) {
            case 1: test_targets<1>(stage, px, py, pz, cc, toff + t0, ntc, cut2, lane, mw); break;
            case 2: test_targets<2>(stage, px, py, pz, cc, toff + t0, ntc, cut2, lane, mw); break;
            case 3: test_targets<3>(stage, px, py, pz, cc, toff + t0, ntc, cut2, lane, mw); break;
            case 4: test_targets<4>(stage, px, py, pz, cc, toff + t0, ntc, cut2, lane, mw); break;
            case 5: test_targets<5>(stage, px, py, pz, cc, toff + t0, ntc, cut2, lane, mw); break;
            case 6: test_targets<6>(stage, px, py, pz, cc, toff + t0, ntc, cut2, lane, mw); break;
            case 7: test_targets<7>(stage, px, py, pz, cc, toff + t0, ntc, cut2, lane, mw); break;
            case 8: test_targets<8>(stage, px, py, pz, cc, toff + t0, ntc, cut2, lane, mw); break;
            case 9: test_targets<9>(stage, px, py, pz, cc, toff + t0, ntc, cut2, lane, mw); break;
            default: test_targets<10>(stage, px, py, pz, cc, toff + t0, ntc, cut2, lane, mw); break;
            }
            static_assert(kCandWin == 10, "one case per window count");
            // a target is not its own neighbour: its lane clears the bit of its list position
            if ((uint32_t)lane < ntc) {
                const uint32_t vs = stencil_self(S, toff + t0 + (uint32_t)lane);
                const uint64_t keep = ~(1ull << (vs & 63));
#pragma unroll
                for (int c = 0; c < kCandWin; c++)
                    if ((vs >> 6) == (uint32_t)c) mw[c] &= keep;
            }
            if ((uint32_t)lane < ntc) {
                if (COLL) ncnt[w][lane] = 0u;
                uint64_t *gm = s.masks + (size_t)(pbase + t0 + lane) * kMaskSlots;
#pragma unroll
                for (int c = 0; c < kCandWin; c++) {
                    if (c < (int)S.NW) {
                        msk[w][lane][c] = mw[c];
                        gm[c] = mw[c];
                    }
                }
            }
            wave_lds_handoff();
            // kernel sums: lanes (target tt, group g)
            const int G = 64 / (int)ntc;
            const int g = lane / (int)ntc, tt = lane % (int)ntc;
            const bool act = g < G;
            const uint64_t *mrow = msk[w][tt];
            uint32_t H = 0;
            for (int c = 0; c < (int)S.NW; c++) H += (uint32_t)__popcll(mrow[c]);
            uint32_t cnt;
            int c;
            uint64_t mc;
            hit_share([&](int cc) { return mrow[cc]; }, act ? H : 0u, g, G, cnt, c, mc);
            const float4 me = stage[toff + t0 + tt];
            Acc<float, KAHAN> sw, su;
            uint32_t nloc = 0;  // near hits of this lane (COLL)
            auto next_k = [&]() {
                while (mc == 0) mc = mrow[++c];
                const int j = __builtin_ctzll(mc);
                mc &= mc - 1;
                return (uint32_t)tbl[w][c][j];
            };
            // one hit's kernel value and unlike-species share; with COLL, the hit is listed
            // branch-free: written to the next free slot (the spare once the list is full),
            // and only a near one advances the count
            auto hit = [&](float &W, float &U) {
                const uint32_t kq = next_k();
                const float4 qc = stage[kq];
                const float d0 = me.x - qc.x, d1 = me.y - qc.y, d2 = me.z - qc.z;
                const float r2s = d0 * d0 + d1 * d1 + d2 * d2;
                W = shape_W<KT>(r2s);
                U = qc.w != me.w ? W : 0.0f;
                if (COLL) {
                    nearl[threadIdx.x][min(nloc, (uint32_t)kNearCap)] = (int16_t)kq;
                    nloc += r2s < rc2m ? 1u : 0u;
                }
            };
            // a per-lane trip count (lanes leave as they finish), two hits per trip: their
            // values are added in FP32, then into the compensated sums; the loop body is
            // unrolled twice (0.05 ms faster here, 0.1 ms slower in the force sweep)
#pragma unroll 2
            for (uint32_t i = 1; i < cnt; i += 2) {
                float Wa, Ua, Wb, Ub;
                hit(Wa, Ua);
                hit(Wb, Ub);
                sw.add(Wa + Wb);
                su.add(Ua + Ub);
            }
            if (cnt & 1u) {
                float W, U;
                hit(W, U);
                sw.add(W);
                su.add(U);
            }
            if (COLL && nloc) {
                // after the loop: reserve the lane's slots of the target's list, then store
                // their sorted indices
                const uint32_t base = atomicAdd(&ncnt[w][tt], nloc);
                for (uint32_t j = 0; j < nloc && j < (uint32_t)kNearCap && base + j < (uint32_t)kNearCap; j++) {
                    const uint32_t kq = (uint32_t)nearl[threadIdx.x][j];
                    const int sl = slot_of(F, kq);
                    s.nearq[(size_t)(pbase + t0 + tt) * kNearCap + base + j] = F.begin[sl] + (kq - F.off[sl]);
                }
            }
            const double SW = d->wnorm * group_total(sw.s, KAHAN ? sw.c : 0.0f, lane, (int)ntc, G);
            const double SU = d->wnorm * group_total(su.s, KAHAN ? su.c : 0.0f, lane, (int)ntc, G);
            if (act && g == 0) {
                const uint32_t p = pbase + t0 + tt;
                const uint8_t ski = SK[p];
                err |= density_finish<float>(s, d, p, ski & 1, ski >> 1, SW, SU);
            }
            if (COLL) {
                wave_lds_handoff();  // the counts of all of a target's lanes
                if (act && g == 0) {
                    const uint32_t nn = ncnt[w][tt];
                    s.cflag[pbase + t0 + tt] =
                        (uint8_t)(!list_ok || nn > (uint32_t)kNearCap ? (uint32_t)kNearOverflow : nn);
                }
            }
            wave_lds_handoff();  // the masks are rewritten by the next round
        }
    };
    if (kernel == KERNEL_WENDLAND) sweep(std::integral_constant<int, KERNEL_WENDLAND>());
    else sweep(std::integral_constant<int, KERNEL_CUBIC>());
    if (err) atomicOr(s.err, err);
}

// The fluid targets of a brick (the inviscid ones, then the viscous ones, each in cell
// order) are dealt to its eight waves in contiguous shares of equal cost, so that the waves
// finish together whatever the cells' populations (a workgroup holds its LDS until its last
// wave ends, and on a lattice the cells of one brick hold 8 to 27 particles).  Each wave
// builds its own cell's stencil list first; a target then replays its masks through the
// list of its own cell.
template <bool KAHAN>
__global__ void __launch_bounds__(kBrickThreads, 4) k_force_cand(DevState s)
{
    __shared__ BrickFrame F;
    __shared__ float4 SA[kStageForce];   // position (brick frame), P/rho^2
    __shared__ float4 SB[kStageForce];   // velocity - v_ref, V (negative: viscous species)
    __shared__ float4 SC[kStageForce];   // half the spin, V/S
    __shared__ double vref[3];
    __shared__ int16_t tbl[kBrickThreads / 64][kCandWin][64];
    __shared__ uint64_t tmask[2][kBrickThreads / 64];  // fluid targets of each cell, by species
    __shared__ int32_t cellnw[kBrickThreads / 64];     // windows of each cell's stencil list
    const uint32_t brick = brick_of_workgroup(blockIdx.x, gridDim.x, s.xcd_run);
    const uint32_t bxyz = s.brick_xyz[brick];
    const InstDesc *d = s.desc + s.brick_inst[brick];
    const uint8_t *SK = s.sk[s.cur];
    const uint32_t M = brick_frame(s, d, brick, bxyz, F, kStageForce, s.v[s.cur], vref);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int ts[3];
    const bool has_cell = brick_target(d, bxyz, w, ts);
    const int tslot = slot_index(ts[0], ts[1], ts[2]);
    uint32_t err = 0;
    if (!F.ok) {
        if (has_cell) {
            const uint32_t nt = F.off[tslot + 1] - F.off[tslot];
            for (uint32_t i = lane; i < nt; i += 64) err |= force_one<float, KAHAN>(s, d, F.begin[tslot] + i);
        }
        if (err) atomicOr(s.err, err);
        return;
    }
    if (brick_own_count(F, d, bxyz) == 0) return;  // the same for the whole workgroup
    stage_force(s, F, M, vref, d->inv_h, SA, SB, SC);
    __syncthreads();
    // Cell w: its stencil list and fluid targets; wall targets are finished here (zero force
    // and torque), and a cell of more than 64 particles or a stencil longer than the windows
    // is evaluated per particle by its wave.
    {
        const uint32_t toff = F.off[tslot], pbase = F.begin[tslot];
        const uint32_t nt = has_cell ? F.off[tslot + 1] - toff : 0u;
        uint64_t fl0 = 0, fl1 = 0;
        int nw = 0;
        if (nt) {
            const StencilList S = stencil_list(F, ts, lane, &tbl[w][0][0]);
            if (S.NW > (uint32_t)kCandWin || nt > 64u) {
                for (uint32_t i = lane; i < nt; i += 64) err |= force_one<float, KAHAN>(s, d, pbase + i);
            } else {
                nw = (int)S.NW;
                uint32_t sk_t = 0;
                if ((uint32_t)lane < nt) sk_t = SK[pbase + lane];
                const bool fluid = (uint32_t)lane < nt && (sk_t >> 1) == KIND_FLUID;
                if ((uint32_t)lane < nt && !fluid) {
                    const double z[3] = {0.0, 0.0, 0.0};
                    err |= force_finish<float>(s, d, pbase + lane, sk_t & 1, z, z);
                }
                fl0 = __ballot(fluid && !(sk_t & 1));
                fl1 = __ballot(fluid && (sk_t & 1));
            }
        }
        if (lane == 0) {
            tmask[0][w] = fl0;
            tmask[1][w] = fl1;
            cellnw[w] = nw;
        }
    }
    __syncthreads();
    // Flat target order: the inviscid targets of cells 0..7, then the viscous ones.  Shares
    // are balanced by cost, an inviscid target (no viscous term) counting 7 and a viscous
    // one 8, so that a wave whose share is all inviscid runs the shorter hit loop.
    uint32_t TS[2] = {0u, 0u};
    for (int c = 0; c < 8; c++) {
        TS[0] += (uint32_t)__popcll(tmask[0][c]);
        TS[1] += (uint32_t)__popcll(tmask[1][c]);
    }
    const uint32_t T = TS[0] + TS[1], C7 = 7u * TS[0], Ctot = C7 + 8u * TS[1];
    auto share_start = [&](uint32_t ww) {
        const uint32_t cw = (Ctot * ww) / 8u;
        return cw <= C7 ? (cw + 6u) / 7u : TS[0] + (cw - C7 + 7u) / 8u;
    };
    const uint32_t b0 = share_start((uint32_t)w), b1 = share_start((uint32_t)w + 1u);
    const PairK K(d);
    const double th = -0.5 * d->h;  // torque = -(h/2) n'
    // Per block of up to 64 of the wave's targets: they share the lanes as (target, group g
    // of G).  Compiled once per smoothing kernel and for equal or unequal species masses,
    // chosen per brick (a batch may mix them), so that the hit loop carries no branch on them.
    auto sweep = [&](auto kt, auto eqm, auto visc) {
        constexpr int KT = decltype(kt)::value;
        constexpr bool EQM = decltype(eqm)::value;
        constexpr bool VISC = decltype(visc)::value;
        for (uint32_t f0 = b0; f0 < b1; f0 += 64) {
            const int n = (int)min(64u, b1 - f0);
            const int G = 64 / n;
            const int g = lane / n;
            const bool target = g < G;
            // this lane's target: flat index f, the rank-th target of species sp in cell c
            const uint32_t f = f0 + (uint32_t)(lane % n);
            const int sp = f < TS[0] ? 0 : 1;
            const uint32_t fs = sp ? f - TS[0] : f;
            int c = 0;
            uint32_t rank = 0, before = 0;
            for (int cc = 0; cc < 8; cc++) {
                if (fs >= before) {
                    c = cc;
                    rank = fs - before;
                }
                before += (uint32_t)__popcll(tmask[sp][cc]);
            }
            const uint32_t local = (uint32_t)__builtin_ctzll(drop_low_bits(tmask[sp][c], rank));
            const int cs = slot_index(1 + (c & 1), 1 + ((c >> 1) & 1), 1 + (c >> 2));
            const uint32_t p = F.begin[cs] + local;
            const uint32_t ki = F.off[cs] + local;
            const float4 Ai = SA[ki], Bi = SB[ki], Ci = SC[ki];
            const PairI I = pair_target(K, Ai, Bi, Ci);
            HitReplay hr(s.masks + (size_t)p * kMaskSlots, cellnw[c], target, g, G);
            const uint32_t cnt = hr.cnt;
            Acc<float, KAHAN> F0, F1, F2, T0, T1, T2;
            auto term = [&](uint32_t k, float fo[3], float nn[3]) {
                const float4 A = SA[k], B = SB[k], C = SC[k];
                pair_force_f32<KT, EQM, VISC>(K, I, A, B, C, Ai.x - A.x, Ai.y - A.y, Ai.z - A.z,
                                              Bi.x - B.x, Bi.y - B.y, Bi.z - B.z, Ci.x + C.x,
                                              Ci.y + C.y, Ci.z + C.z, fo, nn);
            };
            // per-lane trip count, two hits per trip: the two terms are added in FP32, then
            // into the compensated sums (one compensated add per two hits)
            for (uint32_t i = 1; i < cnt; i += 2) {
                const uint32_t ka = hr.next(tbl[c]);
                const uint32_t kb = hr.next(tbl[c]);
                float fa[3], na[3], fb[3], nb[3];
                term(ka, fa, na);
                term(kb, fb, nb);
                F0.add(fa[0] + fb[0]); F1.add(fa[1] + fb[1]); F2.add(fa[2] + fb[2]);
                T0.add(na[0] + nb[0]); T1.add(na[1] + nb[1]); T2.add(na[2] + nb[2]);
            }
            if (cnt & 1u) {
                float fo[3], nn[3];
                term(hr.next(tbl[c]), fo, nn);
                F0.add(fo[0]); F1.add(fo[1]); F2.add(fo[2]);
                T0.add(nn[0]); T1.add(nn[1]); T2.add(nn[2]);
            }
            const double f0d = group_total(F0.s, KAHAN ? F0.c : 0.0f, lane, n, G);
            const double f1d = group_total(F1.s, KAHAN ? F1.c : 0.0f, lane, n, G);
            const double f2d = group_total(F2.s, KAHAN ? F2.c : 0.0f, lane, n, G);
            const double q0 = group_total(T0.s, KAHAN ? T0.c : 0.0f, lane, n, G);
            const double q1 = group_total(T1.s, KAHAN ? T1.c : 0.0f, lane, n, G);
            const double q2 = group_total(T2.s, KAHAN ? T2.c : 0.0f, lane, n, G);
            if (target && g == 0) {
                const double FF[3] = {f0d, f1d, f2d};
                const double TT[3] = {th * q0, th * q1, th * q2};
                err |= force_finish<float>(s, d, p, I.sp ? 1 : 0, FF, TT);
            }
        }
    };
    using Wend = std::integral_constant<int, KERNEL_WENDLAND>;
    using Cub = std::integral_constant<int, KERNEL_CUBIC>;
    using Eq = std::integral_constant<bool, true>;
    using Uneq = std::integral_constant<bool, false>;
    using Visc = std::integral_constant<bool, true>;
    using Inv = std::integral_constant<bool, false>;
    const bool eq = d->mass[0] == d->mass[1];
    const bool inv = b1 <= TS[0];  // the wave's share holds inviscid targets only
    if (d->kernel == KERNEL_WENDLAND) {
        if (eq) {
            if (inv) sweep(Wend(), Eq(), Inv());
            else sweep(Wend(), Eq(), Visc());
        } else {
            if (inv) sweep(Wend(), Uneq(), Inv());
            else sweep(Wend(), Uneq(), Visc());
        }
    } else {
        if (eq) {
            if (inv) sweep(Cub(), Eq(), Inv());
            else sweep(Cub(), Eq(), Visc());
        } else {
            if (inv) sweep(Cub(), Uneq(), Inv());
            else sweep(Cub(), Uneq(), Visc());
        }
    }
    if (err) atomicOr(s.err, err);
}

// Stages what the pressure filter reads of the brick's M neighbourhood particles: the
// position relative to the brick centre in units of h with the source volume V (0 for an
// outer wall, which is not a source), and V P.
__device__ __forceinline__ void stage_filter(const DevState &s, const BrickFrame &F, uint32_t M,
                                             double ih, float4 *SA, float *SP)
{
    const uint32_t N = s.N;
    const int cur = s.cur;
    const double *X = s.x[cur];
    const uint8_t *SK = s.sk[cur];
    const float *AUX = (const float *)s.aux;
    const float *RP = (const float *)s.rhoP;
    double px[3][3];
    float vq[3], pq[3];
    uint8_t sk[3];
    stage_spread(F, M, [&](int u, uint32_t q) {
        for (int a = 0; a < 3; a++) px[u][a] = X[(size_t)a * N + q];
        vq[u] = AUX[4 * (size_t)q];
        pq[u] = RP[2 * (size_t)q + 1];
        sk[u] = SK[q];
    }, [&](int u, uint32_t k, int sl) {
        const float Vs = (sk[u] >> 1) == KIND_WALL_OUTER ? 0.0f : vq[u];
        SA[k] = make_float4((float)(((px[u][0] + F.shift[sl][0]) - F.origin[0]) * ih),
                            (float)(((px[u][1] + F.shift[sl][1]) - F.origin[1]) * ih),
                            (float)(((px[u][2] + F.shift[sl][2]) - F.origin[2]) * ih), Vs);
        SP[k] = Vs * pq[u];
    });
}

// Pressure filter over the brick sweeps' neighbour masks (the density sweep's, replayed as
// in the force sweep).  Each wave first builds its cell's stencil list, copies the fixed
// pressure of the cell's outer walls, and marks its targets (fluid and inner walls); a cell
// of more than 64 particles or with a stencil longer than the windows is filtered per
// particle by its wave.  After a barrier the brick's targets, in cell order, are dealt to
// the eight waves in equal contiguous shares with lanes = (target, group g of G), as in
// the force sweep.  The kernel shape sums are scaled by the normalisation in FP64, where
// the self term joins the denominator; the stage capacity is the force sweep's, so a brick
// the density sweep could not stage (and left without masks) is filtered per particle here
// too.
template <bool KAHAN>
__global__ void __launch_bounds__(kBrickThreads, 4) k_filter_cand(DevState s)
{
    __shared__ BrickFrame F;
    __shared__ float4 SA[kStageForce];  // position (brick frame), source volume
    __shared__ float SP[kStageForce];   // source volume times pressure
    __shared__ int16_t tbl[kBrickThreads / 64][kCandWin][64];
    __shared__ uint64_t tmask[kBrickThreads / 64];  // filter targets of each cell
    __shared__ int32_t cellnw[kBrickThreads / 64];  // windows of each cell's stencil list
    const uint32_t brick = brick_of_workgroup(blockIdx.x, gridDim.x, s.xcd_run);
    const uint32_t bxyz = s.brick_xyz[brick];
    const InstDesc *d = s.desc + s.brick_inst[brick];
    if (!d->pfilter) return;  // the same for the whole workgroup
    const uint8_t *SK = s.sk[s.cur];
    float *AUX = (float *)s.aux;
    const float *RP = (const float *)s.rhoP;
    float *PF = (float *)s.pf;
    const uint32_t M = brick_frame(s, d, brick, bxyz, F, kStageForce);
    if (brick_own_count(F, d, bxyz) == 0) return;  // the same for the whole workgroup
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int ts[3];
    const bool has_cell = brick_target(d, bxyz, w, ts);
    const int tslot = slot_index(ts[0], ts[1], ts[2]);
    uint32_t err = 0;
    if (!F.ok) {
        if (has_cell) {
            const uint32_t nt = F.off[tslot + 1] - F.off[tslot];
            for (uint32_t i = lane; i < nt; i += 64) err |= filter_one<float, KAHAN>(s, d, F.begin[tslot] + i);
        }
        if (err) atomicOr(s.err, err);
        return;
    }
    stage_filter(s, F, M, d->inv_h, SA, SP);
    __syncthreads();
    {
        const uint32_t pbase = F.begin[tslot];
        const uint32_t nt = has_cell ? F.off[tslot + 1] - F.off[tslot] : 0u;
        uint64_t tm = 0;
        int nw = 0;
        if (nt) {
            const StencilList S = stencil_list(F, ts, lane, &tbl[w][0][0]);
            if (S.NW > (uint32_t)kCandWin || nt > 64u) {
                for (uint32_t i = lane; i < nt; i += 64) err |= filter_one<float, KAHAN>(s, d, pbase + i);
            } else {
                nw = (int)S.NW;
                uint32_t sk_t = 0;
                if ((uint32_t)lane < nt) sk_t = SK[pbase + lane];
                const bool tgt = (uint32_t)lane < nt && (sk_t >> 1) != KIND_WALL_OUTER;
                if ((uint32_t)lane < nt && !tgt) {
                    const uint32_t q = pbase + lane;
                    PF[q] = RP[2 * (size_t)q + 1];
                }
                tm = __ballot(tgt);
            }
        }
        if (lane == 0) {
            tmask[w] = tm;
            cellnw[w] = nw;
        }
    }
    __syncthreads();
    uint32_t T = 0;
    for (int c = 0; c < 8; c++) T += (uint32_t)__popcll(tmask[c]);
    const uint32_t b0 = (T * (uint32_t)w) / 8u, b1 = (T * (uint32_t)(w + 1)) / 8u;
    const double wn = d->wnorm, W0 = d->W0;
    auto sweep = [&](auto kt) {
        constexpr int KT = decltype(kt)::value;
        for (uint32_t f0 = b0; f0 < b1; f0 += 64) {
            const int n = (int)min(64u, b1 - f0);
            const int G = 64 / n;
            const int g = lane / n;
            const bool target = g < G;
            // this lane's target: flat index f, the rank-th target of cell c
            const uint32_t f = f0 + (uint32_t)(lane % n);
            int c = 0;
            uint32_t rank = 0, before = 0;
            for (int cc = 0; cc < 8; cc++) {
                if (f >= before) {
                    c = cc;
                    rank = f - before;
                }
                before += (uint32_t)__popcll(tmask[cc]);
            }
            const uint32_t local = (uint32_t)__builtin_ctzll(drop_low_bits(tmask[c], rank));
            const int cs = slot_index(1 + (c & 1), 1 + ((c >> 1) & 1), 1 + (c >> 2));
            const uint32_t p = F.begin[cs] + local;
            const float4 Ai = SA[F.off[cs] + local];
            const float Pi = RP[2 * (size_t)p + 1];
            HitReplay hr(s.masks + (size_t)p * kMaskSlots, cellnw[c], target, g, G);
            // P~ = P_i + sum V_j (P_j - P_i) W_ij / (V_i W(0) + sum V_j W_ij): the numerator
            // holds only pressure differences (compensated); the denominator's terms are all
            // positive and it scales only that difference, so it is summed plainly
            Acc<float, KAHAN> num;
            float den = 0.0f;
            auto hit = [&](float &nm) {
                const uint32_t k = hr.next(tbl[c]);
                const float4 A = SA[k];
                const float d0 = Ai.x - A.x, d1 = Ai.y - A.y, d2 = Ai.z - A.z;
                const float W = shape_W<KT>(d0 * d0 + d1 * d1 + d2 * d2);
                nm = fmaf(-A.w, Pi, SP[k]) * W;
                den = fmaf(A.w, W, den);
            };
            // two hits per trip, their numerator terms added in FP32 before the compensated add
            for (uint32_t i = 1; i < hr.cnt; i += 2) {
                float na, nb;
                hit(na);
                hit(nb);
                num.add(na + nb);
            }
            if (hr.cnt & 1u) {
                float nm;
                hit(nm);
                num.add(nm);
            }
            const double sn = group_total(num.s, KAHAN ? num.c : 0.0f, lane, n, G);
            const double sd = group_total(den, 0.0f, lane, n, G);
            if (target && g == 0) {
                const double Vp = (double)AUX[4 * (size_t)p], Pp = (double)Pi;
                const double Pt = Pp + wn * sn / (Vp * W0 + wn * sd);
                PF[p] = (float)Pt;
                AUX[4 * (size_t)p + 1] = (float)(Pt * (double)AUX[4 * (size_t)p + 2]);
                if (!isfinite(Pt)) err |= ERR_NONFINITE;
            }
        }
    };
    if (d->kernel == KERNEL_WENDLAND) sweep(std::integral_constant<int, KERNEL_WENDLAND>());
    else sweep(std::integral_constant<int, KERNEL_CUBIC>());
    if (err) atomicOr(s.err, err);
}

// ------------------------------------------------------------ load / read / debug ---

__global__ void k_load(DevState s, const double *x, const double *v, const double *w,
                       const uint8_t *species, const uint8_t *kind)
{
    PIdx t = map_thread(s);
    if (!t.active) return;
    const uint32_t p = t.p, N = s.N;
    const int cur = s.cur;
    for (int a = 0; a < 3; a++) {
        s.x[cur][a * N + p] = x[a * N + p];
        s.v[cur][a * N + p] = v[a * N + p];
        s.w[cur][a * N + p] = w[a * N + p];
    }
    uint8_t sp = species[p], kd = kind[p];
    if (sp > 1 || kd > 2 || (kd != KIND_FLUID && sp != 1)) {
        atomicOr(s.err, (uint32_t)ERR_INPUT);
        sp &= 1;
        kd = kd > 2 ? 2 : kd;
    }
    s.id[cur][p] = p;
    s.sk[cur][p] = (uint8_t)(sp | (kd << 1));
}

template <typename R>
__global__ void k_read(DevState s, double pend, double *x, double *v, double *w, double *rho,
                       double *P, double *acc, double *alpha)
{
    PIdx t = map_thread(s);
    if (!t.active) return;
    const uint32_t p = t.p, N = s.N;
    const int cur = s.cur;
    const uint32_t id = s.id[cur][p];
    const bool fluid = (s.sk[cur][p] >> 1) == KIND_FLUID;
    const R *A = (const R *)s.acc, *AL = (const R *)s.alpha;
    const double pk = fluid ? pend : 0.0;
    for (int a = 0; a < 3; a++) {
        if (x) x[a * N + id] = s.x[cur][a * N + p];
        if (v) v[a * N + id] = __fma_rn(pk, (double)A[a * N + p], s.v[cur][a * N + p]);
        if (w) w[a * N + id] = __fma_rn(pk, (double)AL[a * N + p], s.w[cur][a * N + p]);
        if (acc) acc[a * N + id] = (double)A[a * N + p];
        if (alpha) alpha[a * N + id] = (double)AL[a * N + p];
    }
    const R *rp = (const R *)s.rhoP + 2 * (size_t)p;
    if (rho) rho[id] = (double)rp[0];
    if (P) P[id] = (double)(t.d->pfilter ? ((const R *)s.pf)[p] : rp[1]);
}

__global__ void k_debug_keys(DevState s, uint32_t *key_by_id, uint32_t *perm)
{
    PIdx t = map_thread(s);
    if (!t.active) return;
    const uint32_t p = t.p;
    const uint32_t id = s.id[s.cur][p];
    const uint32_t c = s.cell_xyz[s.pcell[p]];
    if (key_by_id) key_by_id[id] = morton3(c & 1023, (c >> 10) & 1023, c >> 20);
    if (perm) perm[p] = id;
}

// Row of the neighbour CSR (by id): phase 0 writes the count to row_ptr[id + 1]; phase 1
// sorts the cnt columns already written from row_ptr[id] ascending.
__device__ __forceinline__ void nbr_row_finish(int phase, uint32_t id, int64_t cnt, int64_t *row_ptr,
                                               int32_t *cols)
{
    if (phase == 0) {
        row_ptr[id + 1] = cnt;
        return;
    }
    const int64_t base = row_ptr[id];
    for (int64_t i = 1; i < cnt; i++) {
        int32_t v = cols[base + i];
        int64_t j = i - 1;
        while (j >= 0 && cols[base + j] > v) { cols[base + j + 1] = cols[base + j]; j--; }
        cols[base + j + 1] = v;
    }
}

// Neighbour row of sorted particle p by its FP64 cell walk (the test of the per-particle
// sweeps).
__device__ __forceinline__ uint32_t nbr_walk(const DevState &s, const InstDesc *d, uint32_t p, int phase,
                                             int64_t *row_ptr, int32_t *cols)
{
    const uint32_t N = s.N;
    const int cur = s.cur;
    const double *X = s.x[cur];
    const uint32_t id = s.id[cur][p];
    const double xi0 = X[p], xi1 = X[N + p], xi2 = X[2 * N + p];
    const uint32_t cxyz = s.cell_xyz[s.pcell[p]];
    uint32_t err = 0;
    int64_t cnt = 0;
    const int64_t base = phase ? row_ptr[id] : 0;
    for_each_cell(s, d, cxyz & 1023, (cxyz >> 10) & 1023, cxyz >> 20, err,
                  [&](uint32_t b, uint32_t e) {
        for (uint32_t q = b; q < e; ++q) {
            if (q == p) continue;
            double dx0 = min_img(d, 0, xi0 - X[q]);
            double dx1 = min_img(d, 1, xi1 - X[N + q]);
            double dx2 = min_img(d, 2, xi2 - X[2 * N + q]);
            if (r2_exact(dx0, dx1, dx2) < d->cut2) {
                if (phase) cols[base + cnt] = (int32_t)s.id[cur][q];
                cnt++;
            }
        }
    });
    nbr_row_finish(phase, id, cnt, row_ptr, cols);
    return err;
}

// phase 0: row_ptr[id + 1] = neighbour count; phase 1: fill columns and sort each row.
__global__ void k_debug_nbr(DevState s, int phase, int64_t *row_ptr, int32_t *cols)
{
    PIdx t = map_thread(s);
    if (!t.active) return;
    const uint32_t err = nbr_walk(s, t.d, t.p, phase, row_ptr, cols);
    if (err) atomicOr(s.err, err);
}

// The neighbour sets the brick density sweep used at the last evaluation (FP32-mixed
// path), as the same CSR by id: its hit masks decoded through the stencil list of each
// target cell (the masks the force sweep and the pressure filter replay), and the FP64
// cell walk for the particles that sweep evaluated one by one (bricks too large to stage,
// stencils longer than its windows).  One workgroup per brick, laid out as in the sweep.
__global__ void __launch_bounds__(kBrickThreads) k_debug_masks(DevState s, int phase, int64_t *row_ptr,
                                                               int32_t *cols)
{
    __shared__ BrickFrame F;
    __shared__ int16_t tbl[kBrickThreads / 64][kCandWin][64];
    const uint32_t brick = blockIdx.x;
    const uint32_t bxyz = s.brick_xyz[brick];
    const InstDesc *d = s.desc + s.brick_inst[brick];
    brick_frame(s, d, brick, bxyz, F, kStageDensity);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int ts[3];
    if (!brick_target(d, bxyz, w, ts)) return;
    const int tslot = slot_index(ts[0], ts[1], ts[2]);
    const uint32_t pbase = F.begin[tslot], nt = F.off[tslot + 1] - F.off[tslot];
    uint32_t err = 0;
    bool walk = !F.ok;
    StencilList S{0, 0, 0};
    if (!walk && nt) {
        S = stencil_list(F, ts, lane, &tbl[w][0][0]);
        walk = S.NW > (uint32_t)kCandWin;
    }
    for (uint32_t i = lane; i < nt; i += 64) {
        const uint32_t p = pbase + i;
        if (walk) {
            err |= nbr_walk(s, d, p, phase, row_ptr, cols);
            continue;
        }
        const uint32_t id = s.id[s.cur][p];
        const int64_t base = phase ? row_ptr[id] : 0;
        int64_t cnt = 0;
        for (uint32_t c = 0; c < S.NW; c++) {
            uint64_t m = s.masks[(size_t)p * kMaskSlots + c];
            while (m) {
                const int j = __builtin_ctzll(m);
                m &= m - 1;
                if (phase) {
                    const uint32_t k = (uint32_t)tbl[w][c][j];
                    const int sl = slot_of(F, k);
                    cols[base + cnt] = (int32_t)s.id[s.cur][F.begin[sl] + (k - F.off[sl])];
                }
                cnt++;
            }
        }
        nbr_row_finish(phase, id, cnt, row_ptr, cols);
    }
    if (err) atomicOr(s.err, err);
}

// Near neighbours listed by the brick density sweep for the collision step, by id:
// count[id] = the number listed (kNearOverflow: not listed, the step walks the cells) and
// ids[id][0 .. count) their ids, ascending (-1 in the unused places).
__global__ void k_debug_near(DevState s, uint8_t *count, int32_t *ids)
{
    PIdx t = map_thread(s);
    if (!t.active) return;
    const uint32_t p = t.p;
    const uint32_t id = s.id[s.cur][p];
    const uint32_t n = s.cflag[p];
    count[id] = (uint8_t)n;
    int32_t v[kNearCap];
    for (int a = 0; a < kNearCap; a++) v[a] = -1;
    if (n <= (uint32_t)kNearCap) {
        for (uint32_t a = 0; a < n; a++) {
            int32_t x = (int32_t)s.id[s.cur][s.nearq[(size_t)p * kNearCap + a]];
            uint32_t b = a;
            for (; b > 0 && v[b - 1] > x; b--) v[b] = v[b - 1];
            v[b] = x;
        }
    }
    for (int a = 0; a < kNearCap; a++) ids[(size_t)id * kNearCap + a] = v[a];
}

// ------------------------------------------------------------ diagnostics -----------

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

struct DD {
    double hi = 0.0, lo = 0.0;
    __device__ __forceinline__ void add(double x)
    {
        double s, e;
        two_sum(hi, x, s, e);
        hi = s;
        lo += e;
    }
    __device__ __forceinline__ void add(const DD &o)
    {
        double s, e;
        two_sum(hi, o.hi, s, e);
        hi = s;
        lo += e + o.lo;
    }
};

template <typename R>
__global__ void k_diag_part(DevState s, double pend)
{
    __shared__ double sh[14][256];
    const int inst = blockIdx.x / kDiagChunks, chunk = blockIdx.x % kDiagChunks;
    const InstDesc *d = s.desc + inst;
    const uint32_t N = s.N;
    const int cur = s.cur;
    const uint32_t per = (d->n_part + kDiagChunks - 1) / kDiagChunks;
    const uint32_t b = d->part_off + chunk * per;
    uint32_t e = b + per;
    if (e > d->part_off + d->n_part) e = d->part_off + d->n_part;
    const R *A = (const R *)s.acc, *AL = (const R *)s.alpha;
    DD acc[7];
    for (uint32_t p = b + threadIdx.x; p < e; p += blockDim.x) {
        uint8_t sk = s.sk[cur][p];
        if ((sk >> 1) != KIND_FLUID) continue;
        double m = d->mass[sk & 1], I = d->inertia[sk & 1];
        double x[3], v[3], w[3];
        for (int a = 0; a < 3; a++) {
            x[a] = s.x[cur][a * N + p];
            v[a] = __fma_rn(pend, (double)A[a * N + p], s.v[cur][a * N + p]);
            w[a] = __fma_rn(pend, (double)AL[a * N + p], s.w[cur][a * N + p]);
        }
        double L0 = x[1] * v[2] - x[2] * v[1];
        double L1 = x[2] * v[0] - x[0] * v[2];
        double L2 = x[0] * v[1] - x[1] * v[0];
        acc[0].add(m * v[0]); acc[1].add(m * v[1]); acc[2].add(m * v[2]);
        acc[3].add(m * L0 + I * w[0]);
        acc[4].add(m * L1 + I * w[1]);
        acc[5].add(m * L2 + I * w[2]);
        acc[6].add(0.5 * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) +
                   0.5 * I * (w[0] * w[0] + w[1] * w[1] + w[2] * w[2]));
    }
    for (int k = 0; k < 7; k++) { sh[2 * k][threadIdx.x] = acc[k].hi; sh[2 * k + 1][threadIdx.x] = acc[k].lo; }
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            for (int k = 0; k < 7; k++) {
                DD a, o;
                a.hi = sh[2 * k][threadIdx.x]; a.lo = sh[2 * k + 1][threadIdx.x];
                o.hi = sh[2 * k][threadIdx.x + off]; o.lo = sh[2 * k + 1][threadIdx.x + off];
                a.add(o);
                sh[2 * k][threadIdx.x] = a.hi; sh[2 * k + 1][threadIdx.x] = a.lo;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 14) s.diag_part[(size_t)blockIdx.x * 14 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_diag_final(DevState s)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.n_inst * 7) return;
    int inst = i / 7, k = i % 7;
    DD a;
    for (int c = 0; c < kDiagChunks; c++) {
        DD o;
        const double *pp = s.diag_part + ((size_t)inst * kDiagChunks + c) * 14;
        o.hi = pp[2 * k];
        o.lo = pp[2 * k + 1];
        a.add(o);
    }
    s.diag_out[i] = a.hi + a.lo;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t value, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}


// ------------------------------------------------------------ vortex diagnostic -----
// The paper counts spinning vortices by image analysis of the rotational-force intensity
// (the fifth term of Eq. 2, 2 eta_r curl(omega_0)) on the z = 0 section (Sec. 3).  Here:
// the intensity of each fluid particle in the section -dx <= z - z0 < dx (z periodic) is
// I = |sum over viscous neighbours j of 2 eta V_j F_ij (w_i + w_j) x r_ij| in FP64 (the
// spin part of the viscous pair force per unit volume); a pixel of side dx holds the
// largest intensity of its particles; pixels with a positive value of at least theta
// times the largest are on; 8-connected sets of on pixels are labelled by their smallest
// pixel index; components of at least min_pixels pixels are counted.

// Deposits intensity I of the particle at (x0, x1) into its pixel: non-negative doubles
// order like their bit patterns, so the largest wins through an integer atomicMax.
__device__ __forceinline__ uint32_t vortex_deposit(const VortexArgs &a, double x0, double x1,
                                                   double I, unsigned long long *img)
{
    if (!isfinite(I)) return ERR_NONFINITE;
    int ix = (int)floor((x0 - a.lox) / a.dx), iy = (int)floor((x1 - a.loy) / a.dx);
    ix = min(max(ix, 0), a.nx - 1);
    iy = min(max(iy, 0), a.ny - 1);
    atomicMax(&img[(size_t)iy * a.nx + ix], (unsigned long long)__double_as_longlong(I));
    return 0u;
}

// Whether z lies in the section -dx <= z - z0 < dx (z periodic with period Lz).
__device__ __forceinline__ bool in_section(const VortexArgs &a, double z)
{
    double dz = z - a.z0;
    dz = dz - a.Lz * floor(dz / a.Lz + 0.5);
    return dz >= -a.dx && dz < a.dx;
}

// Intensity of fluid particle p of the section, walking its cell stencil in FP64.
template <typename R>
__device__ __forceinline__ uint32_t vortex_one(const DevState &s, const InstDesc *d,
                                               const VortexArgs &a, uint32_t p,
                                               unsigned long long *img)
{
#pragma clang fp contract(off)
    const uint32_t N = s.N;
    const int cur = s.cur;
    const double *X = s.x[cur], *Wv = s.w[cur];
    const uint8_t *SK = s.sk[cur];
    if ((SK[p] >> 1) != KIND_FLUID) return 0u;
    const double xi0 = X[p], xi1 = X[N + p], xi2 = X[2 * N + p];
    if (!in_section(a, xi2)) return 0u;
    // spins at the end of the step: the closing half kick is still pending for fluid
    // particles (as in k_read); walls hold their exact spin
    const R *AL = (const R *)s.alpha;
    auto spin = [&](uint32_t q, int c) {
        const double pk = (SK[q] >> 1) == KIND_FLUID ? a.pend : 0.0;
        return __fma_rn(pk, (double)AL[c * N + q], Wv[c * N + q]);
    };
    const double wi0 = spin(p, 0), wi1 = spin(p, 1), wi2 = spin(p, 2);
    const R *RP = (const R *)s.rhoP;
    const double m1 = d->mass[1], eta2 = 2.0 * d->eta, cut2 = d->cut2;
    const uint32_t cxyz = s.cell_xyz[s.pcell[p]];
    uint32_t err = 0;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for_each_cell(s, d, cxyz & 1023, (cxyz >> 10) & 1023, cxyz >> 20, err,
                  [&](uint32_t b, uint32_t e) {
        for (uint32_t q = b; q < e; ++q) {
            if ((SK[q] & 1) != 1 || q == p) continue;
            const double r0 = min_img(d, 0, xi0 - X[q]), r1 = min_img(d, 1, xi1 - X[N + q]),
                         r2 = min_img(d, 2, xi2 - X[2 * N + q]);
            const double rr2 = r2_exact(r0, r1, r2);
            if (!(rr2 < cut2)) continue;
            double Wk, Fk;
            kernel_WF<double>(d->kernel, rr2, d->inv_h, d->wnorm, Wk, Fk);
            const double g = eta2 * (m1 / (double)RP[2 * q]) * Fk;
            const double w0 = wi0 + spin(q, 0), w1 = wi1 + spin(q, 1), w2 = wi2 + spin(q, 2);
            s0 += g * (w1 * r2 - w2 * r1);
            s1 += g * (w2 * r0 - w0 * r2);
            s2 += g * (w0 * r1 - w1 * r0);
        }
    });
    return err | vortex_deposit(a, xi0, xi1, sqrt(s0 * s0 + s1 * s1 + s2 * s2), img);
}

// One thread per particle; threads of particles outside the section leave at once.
template <typename R>
__global__ void k_vortex_intensity(DevState s, VortexArgs a, unsigned long long *img)
{
    PIdx t = map_thread(s);
    if (!t.active) return;
    const uint32_t err = vortex_one<R>(s, t.d, a, t.p, img);
    if (err) atomicOr(s.err, err);
}

// Stages what the brick intensity reads of the neighbourhood: position relative to the
// brick centre in units of h with V = m/rho for a viscous particle (0 otherwise, so that
// the others drop out of the sum), and the spin at the end of the step.
__device__ __forceinline__ void stage_vortex(const DevState &s, const InstDesc *d, const BrickFrame &F,
                                             uint32_t M, double pend, float4 *SA, float4 *SW)
{
    const uint32_t N = s.N;
    const int cur = s.cur;
    const double *X = s.x[cur], *Wv = s.w[cur];
    const uint8_t *SK = s.sk[cur];
    const float *AL = (const float *)s.alpha;
    const float *RP = (const float *)s.rhoP;
    const double ih = d->inv_h, m1 = d->mass[1];
    double px[3][3], pw[3][3];
    float al[3][3], rq[3];
    uint8_t sk[3];
    stage_spread(F, M, [&](int u, uint32_t q) {
        for (int c = 0; c < 3; c++) {
            px[u][c] = X[(size_t)c * N + q];
            pw[u][c] = Wv[(size_t)c * N + q];
            al[u][c] = AL[(size_t)c * N + q];
        }
        rq[u] = RP[2 * (size_t)q];
        sk[u] = SK[q];
    }, [&](int u, uint32_t k, int sl) {
        const double pk = (sk[u] >> 1) == KIND_FLUID ? pend : 0.0;
        SA[k] = make_float4((float)(((px[u][0] + F.shift[sl][0]) - F.origin[0]) * ih),
                            (float)(((px[u][1] + F.shift[sl][1]) - F.origin[1]) * ih),
                            (float)(((px[u][2] + F.shift[sl][2]) - F.origin[2]) * ih),
                            (sk[u] & 1) ? (float)(m1 / (double)rq[u]) : 0.0f);
        SW[k] = make_float4((float)__fma_rn(pk, (double)al[u][0], pw[u][0]),
                            (float)__fma_rn(pk, (double)al[u][1], pw[u][1]),
                            (float)__fma_rn(pk, (double)al[u][2], pw[u][2]), 0.0f);
    });
}

// Intensity over the brick sweeps' neighbour masks (FP32-mixed path; the density sweep of
// the same positions stored them): one workgroup per brick whose cells reach the section,
// lanes = (target, group g of G) over the cell's fluid particles in the section.  With
// r_ij = h r_s and F_ij = (wnorm cF / h^2) Fhat, each term is V_j Fhat (w_i + w_j) x r_s
// (compensated FP32 sums) times 2 eta wnorm cF / h (FP64).  Bricks too large to stage, and
// stencils too long for the masks, use the per-particle walk.
__global__ void __launch_bounds__(kBrickThreads, 4) k_vortex_cand(DevState s, VortexArgs a,
                                                                unsigned long long *img)
{
    __shared__ BrickFrame F;
    __shared__ float4 SA[kStageForce];  // position (brick frame), V of a viscous particle
    __shared__ float4 SW[kStageForce];  // spin at the end of the step
    __shared__ int16_t tbl[kBrickThreads / 64][kCandWin][64];
    const uint32_t brick = brick_of_workgroup(blockIdx.x, gridDim.x, s.xcd_run);
    const uint32_t bxyz = s.brick_xyz[brick];
    const InstDesc *d = s.desc + s.brick_inst[brick];
    {
        // the brick's two cell layers span [zc - e, zc + e): leave unless the section is near
        const double e = d->edge[2];
        double dz = d->lo[2] + (double)(2 * (int)(bxyz >> 20) + 1) * e - a.z0;
        dz = dz - a.Lz * floor(dz / a.Lz + 0.5);
        if (!(fabs(dz) < e + a.dx + 1e-6 * e)) return;  // the same for the whole workgroup
    }
    const uint32_t N = s.N;
    const double *X = s.x[s.cur];
    const uint8_t *SK = s.sk[s.cur];
    const uint32_t M = brick_frame(s, d, brick, bxyz, F, kStageForce);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int ts[3];
    const bool has_cell = brick_target(d, bxyz, w, ts);
    const int tslot = slot_index(ts[0], ts[1], ts[2]);
    uint32_t err = 0;
    if (!F.ok) {
        if (has_cell) {
            const uint32_t nt = F.off[tslot + 1] - F.off[tslot];
            for (uint32_t i = lane; i < nt; i += 64) err |= vortex_one<float>(s, d, a, F.begin[tslot] + i, img);
        }
        if (err) atomicOr(s.err, err);
        return;
    }
    stage_vortex(s, d, F, M, a.pend, SA, SW);
    __syncthreads();
    if (!has_cell) return;
    const uint32_t toff = F.off[tslot], pbase = F.begin[tslot];
    const uint32_t nt = F.off[tslot + 1] - toff;
    if (nt == 0) return;
    const StencilList S = stencil_list(F, ts, lane, &tbl[w][0][0]);
    if (S.NW > (uint32_t)kCandWin) {
        for (uint32_t i = lane; i < nt; i += 64) err |= vortex_one<float>(s, d, a, pbase + i, img);
        if (err) atomicOr(s.err, err);
        return;
    }
    const int NW = (int)S.NW;
    const double kv = 2.0 * d->eta * d->wnorm * (d->kernel == KERNEL_WENDLAND ? 5.0 : 1.0) * d->inv_h;
    auto sweep = [&](auto kt) {
        constexpr int KT = decltype(kt)::value;
        for (uint32_t t0 = 0; t0 < nt; t0 += 64) {
            const uint32_t nb = min(64u, nt - t0);
            bool tgt = false;
            if ((uint32_t)lane < nb) {
                const uint32_t q = pbase + t0 + lane;
                tgt = (SK[q] >> 1) == KIND_FLUID && in_section(a, X[2 * (size_t)N + q]);
            }
            const uint64_t Mt = __ballot(tgt);
            if (Mt == 0) continue;
            const int n = __popcll(Mt);
            const int G = 64 / n;
            const int g = lane / n;
            const bool target = g < G;
            const uint32_t t = (uint32_t)__builtin_ctzll(drop_low_bits(Mt, (uint32_t)(lane % n)));
            const uint32_t p = pbase + t0 + t;
            const float4 Ai = SA[toff + t0 + t], Wi = SW[toff + t0 + t];
            HitReplay hr(s.masks + (size_t)p * kMaskSlots, NW, target, g, G);
            Acc<float, true> s0, s1, s2;
            for (uint32_t i = 0; i < hr.cnt; i++) {
                const uint32_t k = hr.next(tbl[w]);
                const float4 A = SA[k], Wj = SW[k];
                const float r0 = Ai.x - A.x, r1 = Ai.y - A.y, r2 = Ai.z - A.z;
                float Wk, Fh;
                shape_WF<KT>(r0 * r0 + r1 * r1 + r2 * r2, Wk, Fh);
                const float gv = A.w * Fh;
                const float w0 = Wi.x + Wj.x, w1 = Wi.y + Wj.y, w2 = Wi.z + Wj.z;
                s0.add(gv * (w1 * r2 - w2 * r1));
                s1.add(gv * (w2 * r0 - w0 * r2));
                s2.add(gv * (w0 * r1 - w1 * r0));
            }
            const double v0 = group_total(s0.s, s0.c, lane, n, G);
            const double v1 = group_total(s1.s, s1.c, lane, n, G);
            const double v2 = group_total(s2.s, s2.c, lane, n, G);
            if (target && g == 0)
                err |= vortex_deposit(a, X[p], X[(size_t)N + p], kv * sqrt(v0 * v0 + v1 * v1 + v2 * v2), img);
        }
    };
    if (d->kernel == KERNEL_WENDLAND) sweep(std::integral_constant<int, KERNEL_WENDLAND>());
    else sweep(std::integral_constant<int, KERNEL_CUBIC>());
    if (err) atomicOr(s.err, err);
}

// Largest pixel value (one block; max is exact in any order).
__global__ void k_vortex_max(const unsigned long long *img, uint32_t n, unsigned long long *vmax)
{
    __shared__ unsigned long long part[1024 / 64];
    unsigned long long m = 0;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) m = img[i] > m ? img[i] : m;
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(m, off);
        m = o > m ? o : m;
    }
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (uint32_t w = 1; w < blockDim.x / 64; w++) m = part[w] > m ? part[w] : m;
        *vmax = m;
    }
}

__global__ void k_vortex_label_init(const unsigned long long *img, const unsigned long long *vmax,
                                    double theta, uint32_t n, int32_t *lab)
{
#pragma clang fp contract(off)
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = __longlong_as_double((long long)img[i]);
    const double thr = theta * __longlong_as_double((long long)*vmax);
    lab[i] = (v > 0.0 && v >= thr) ? (int32_t)i : -1;
}

// One relaxation: every on pixel takes the smallest label among itself and its on
// 8-neighbours, then follows its label's own label while that decreases (labels only
// ever decrease and always name a pixel of the same component).
__global__ void k_vortex_relax(int32_t *lab, int nx, int ny, uint32_t *changed)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nx * ny) return;
    const int l0 = lab[i];
    if (l0 < 0) return;
    const int iy = i / nx, ix = i - iy * nx;
    int m = l0;
    for (int dy = -1; dy <= 1; dy++) {
        const int y = iy + dy;
        if (y < 0 || y >= ny) continue;
        for (int dx = -1; dx <= 1; dx++) {
            const int x = ix + dx;
            if (x < 0 || x >= nx) continue;
            const int l = lab[y * nx + x];
            if (l >= 0 && l < m) m = l;
        }
    }
    for (int l = lab[m]; l >= 0 && l < m; l = lab[m]) m = l;
    if (m < l0) {
        atomicMin(&lab[i], m);
        *changed = 1u;
    }
}

__global__ void k_vortex_sizes(const int32_t *lab, uint32_t n, int32_t *size)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && lab[i] >= 0) atomicAdd(&size[lab[i]], 1);
}

__global__ void k_vortex_count(const int32_t *lab, const int32_t *size, uint32_t n,
                               int32_t min_pixels, int32_t *count)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && lab[i] == (int32_t)i && size[i] >= min_pixels) atomicAdd(count, 1);
}

}  // namespace

// ---------------------------------------------------------------- launchers ---------

hipError_t launch_keys(const DevState &d, const Launch &L, hipStream_t st, int mode, double kick,
                       double dt)
{
    unsigned g = grid_for(d.n_waves, L.bs_stream);
    if (d.precision == 0) k_keys<double><<<g, L.bs_stream, 0, st>>>(d, mode, kick, dt);
    else k_keys<float><<<g, L.bs_stream, 0, st>>>(d, mode, kick, dt);
    return hipGetLastError();
}

hipError_t launch_scan(const DevState &d, const Launch &, hipStream_t st)
{
    uint32_t nb = (d.C + kScanTile - 1) / kScanTile;
    k_scan_tiles<<<nb, kScanBlock, 0, st>>>(d.count, d.C, d.bsum);
    k_scan_bsum<<<1, kScanBlock, 0, st>>>(d.bsum, nb);
    k_scan_apply<<<nb, kScanBlock, 0, st>>>(d.count, d.C, d.bsum, d.start);
    return hipGetLastError();
}

hipError_t launch_scatter(const DevState &d, const Launch &L, hipStream_t st)
{
    k_scatter<<<grid_for(d.n_waves, L.bs_stream), L.bs_stream, 0, st>>>(d);
    return hipGetLastError();
}

hipError_t launch_reorder(const DevState &d, const Launch &L, hipStream_t st, int mode,
                          double kick, double dt)
{
    unsigned g = grid_for(d.n_waves, L.bs_stream);
    if (d.precision == 0) k_reorder<double><<<g, L.bs_stream, 0, st>>>(d, mode, kick, dt);
    else k_reorder<float><<<g, L.bs_stream, 0, st>>>(d, mode, kick, dt);
    return hipGetLastError();
}

hipError_t launch_density(const DevState &d, const Launch &L, hipStream_t st)
{
    unsigned g = grid_for(d.n_waves, L.bs_density);
    if (d.precision == 0) k_density<double, false><<<g, L.bs_density, 0, st>>>(d);
    else if (L.sweep == SWEEP_CAND && d.n_bricks) {
        k_brick_frames<<<d.n_bricks, 64, 0, st>>>(d);
        if (L.list_targets == 16) {
            if (d.any_coll) k_density_cand<true, true, 16><<<d.n_bricks, kBrickThreads, 0, st>>>(d);
            else k_density_cand<true, false, 16><<<d.n_bricks, kBrickThreads, 0, st>>>(d);
        } else {
            if (d.any_coll) k_density_cand<true, true, 32><<<d.n_bricks, kBrickThreads, 0, st>>>(d);
            else k_density_cand<true, false, 32><<<d.n_bricks, kBrickThreads, 0, st>>>(d);
        }
    }
    else k_density<float, true><<<g, L.bs_density, 0, st>>>(d);
    return hipGetLastError();
}

hipError_t launch_force(const DevState &d, const Launch &L, hipStream_t st)
{
    unsigned g = grid_for(d.n_waves, L.bs_force);
    if (d.precision == 0) k_force<double, false><<<g, L.bs_force, 0, st>>>(d);
    else if (L.sweep == SWEEP_CAND && d.n_bricks) k_force_cand<true><<<d.n_bricks, kBrickThreads, 0, st>>>(d);
    else k_force<float, true><<<g, L.bs_force, 0, st>>>(d);
    return hipGetLastError();
}

hipError_t launch_filter(const DevState &d, const Launch &L, hipStream_t st)
{
    if (!d.any_filter) return hipSuccess;
    unsigned g = grid_for(d.n_waves, L.bs_density);
    if (d.precision == 0) k_filter<double, false><<<g, L.bs_density, 0, st>>>(d);
    else if (L.sweep == SWEEP_CAND && d.n_bricks) k_filter_cand<true><<<d.n_bricks, kBrickThreads, 0, st>>>(d);
    else k_filter<float, true><<<g, L.bs_density, 0, st>>>(d);
    return hipGetLastError();
}

hipError_t launch_collide(const DevState &d, const Launch &L, hipStream_t st)
{
    if (!d.any_coll) return hipSuccess;
    unsigned g = grid_for(d.n_waves, L.bs_stream);
    // the brick density sweep (chosen as in launch_density) lists the near neighbours
    const int listed = (d.precision != 0 && L.sweep == SWEEP_CAND && d.n_bricks) ? 1 : 0;
    k_collide<<<g, L.bs_stream, 0, st>>>(d, listed);
    k_collide_apply<<<g, L.bs_stream, 0, st>>>(d, listed);
    return hipGetLastError();
}

hipError_t launch_load(const DevState &d, const Launch &L, hipStream_t st, const double *x,
                       const double *v, const double *w, const uint8_t *species,
                       const uint8_t *kind)
{
    k_load<<<grid_for(d.n_waves, L.bs_stream), L.bs_stream, 0, st>>>(d, x, v, w, species, kind);
    return hipGetLastError();
}

hipError_t launch_read(const DevState &d, const Launch &L, hipStream_t st, double pend, double *x,
                       double *v, double *w, double *rho, double *P, double *acc, double *alpha)
{
    unsigned g = grid_for(d.n_waves, L.bs_stream);
    if (d.precision == 0) k_read<double><<<g, L.bs_stream, 0, st>>>(d, pend, x, v, w, rho, P, acc, alpha);
    else k_read<float><<<g, L.bs_stream, 0, st>>>(d, pend, x, v, w, rho, P, acc, alpha);
    return hipGetLastError();
}

hipError_t launch_diag(const DevState &d, const Launch &, hipStream_t st, double pend)
{
    unsigned g = (unsigned)d.n_inst * kDiagChunks;
    if (d.precision == 0) k_diag_part<double><<<g, 256, 0, st>>>(d, pend);
    else k_diag_part<float><<<g, 256, 0, st>>>(d, pend);
    unsigned nt = (unsigned)d.n_inst * 7;
    k_diag_final<<<(nt + 255) / 256, 256, 0, st>>>(d);
    return hipGetLastError();
}

hipError_t launch_debug_keys(const DevState &d, const Launch &L, hipStream_t st,
                             uint32_t *key_by_id, uint32_t *perm)
{
    k_debug_keys<<<grid_for(d.n_waves, L.bs_stream), L.bs_stream, 0, st>>>(d, key_by_id, perm);
    return hipGetLastError();
}

hipError_t launch_debug_nbr(const DevState &d, const Launch &L, hipStream_t st, int phase,
                            int64_t *row_ptr, int32_t *cols)
{
    k_debug_nbr<<<grid_for(d.n_waves, L.bs_stream), L.bs_stream, 0, st>>>(d, phase, row_ptr, cols);
    return hipGetLastError();
}

hipError_t launch_debug_masks(const DevState &d, hipStream_t st, int phase, int64_t *row_ptr,
                              int32_t *cols)
{
    if (!d.n_bricks) return hipErrorInvalidValue;
    k_debug_masks<<<d.n_bricks, kBrickThreads, 0, st>>>(d, phase, row_ptr, cols);
    return hipGetLastError();
}

hipError_t launch_debug_near(const DevState &d, const Launch &L, hipStream_t st, uint8_t *count,
                             int32_t *ids)
{
    k_debug_near<<<grid_for(d.n_waves, L.bs_stream), L.bs_stream, 0, st>>>(d, count, ids);
    return hipGetLastError();
}

hipError_t launch_vortex_intensity(const DevState &d, const Launch &L, hipStream_t st,
                                   const VortexArgs &a, bool masks, unsigned long long *img,
                                   unsigned long long *vmax)
{
    const unsigned g = grid_for(d.n_waves, L.bs_stream);
    if (d.precision == 0) k_vortex_intensity<double><<<g, L.bs_stream, 0, st>>>(d, a, img);
    else if (masks) k_vortex_cand<<<d.n_bricks, kBrickThreads, 0, st>>>(d, a, img);
    else k_vortex_intensity<float><<<g, L.bs_stream, 0, st>>>(d, a, img);
    k_vortex_max<<<1, 1024, 0, st>>>(img, (uint32_t)(a.nx * a.ny), vmax);
    return hipGetLastError();
}

hipError_t launch_vortex_label_init(hipStream_t st, const unsigned long long *img,
                                    const unsigned long long *vmax, double theta, uint32_t n,
                                    int32_t *lab)
{
    k_vortex_label_init<<<(n + 255) / 256, 256, 0, st>>>(img, vmax, theta, n, lab);
    return hipGetLastError();
}

hipError_t launch_vortex_relax(hipStream_t st, int32_t *lab, int nx, int ny, uint32_t *changed)
{
    const unsigned n = (unsigned)(nx * ny);
    k_vortex_relax<<<(n + 255) / 256, 256, 0, st>>>(lab, nx, ny, changed);
    return hipGetLastError();
}

hipError_t launch_vortex_count(hipStream_t st, const int32_t *lab, int32_t *size, uint32_t n,
                               int32_t min_pixels, int32_t *count)
{
    k_vortex_sizes<<<(n + 255) / 256, 256, 0, st>>>(lab, n, size);
    k_vortex_count<<<(n + 255) / 256, 256, 0, st>>>(lab, size, n, min_pixels, count);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, size_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    k_fill_u32<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, value, n);
    return hipGetLastError();
}

}  // namespace sph
