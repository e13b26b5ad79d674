// HIP kernels (gfx950) of the two-fluid SPH step.
//
// Per time step (velocity Verlet, Algorithm 1 of the paper, single device):
//   k_keys     half kick + drift of each particle (walls: exact rotation), its cell in
//              Morton order, and its slot in that cell (atomic histogram);
//   k_scan_*   exclusive scan of the cell histogram -> cell_start (CSR of the cell list);
//   k_scatter  counting-sort scatter;
//   k_reorder  orders each cell by particle id and moves the advanced state into the new
//              cell-sorted order (the paper's periodic defragmentation, done every step);
//   k_density  kernel-summed density, Tait EOS (Eq. 4) and the per-particle factors the
//              force sweep needs;
//   k_force    pair forces of Eqs. 1-2 and the spin torques.
// The closing half kick is folded into the next k_keys / k_reorder.
#include <math.h>

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

__device__ __forceinline__ double min_img(const InstDesc *d, int a, double dd)
{
    if (d->periodic[a]) {
        if (dd > d->halfL[a]) dd -= d->L[a];
        else if (dd < -d->halfL[a]) dd += d->L[a];
    }
    return dd;
}

// (dx*dx + dy*dy) + dz*dz, each operation rounded: the neighbour test is bit-identical
// to a plain double-precision evaluation in this order.
__device__ __forceinline__ double r2_exact(double a, double b, double c)
{
    return __dadd_rn(__dadd_rn(__dmul_rn(a, a), __dmul_rn(b, b)), __dmul_rn(c, c));
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

// Calls fn(begin, end) for the sorted-particle range of every cell within +-cf of
// (cx, cy, cz), wrapping periodic axes and skipping cells off a bounded axis.
template <class Fn>
__device__ __forceinline__ void for_each_cell(const DevState &s, const InstDesc *d, int cx,
                                              int cy, int cz, uint32_t &err, Fn &&fn)
{
    const int cf = d->cf;
    const int n0 = d->n[0], n1 = d->n[1], n2 = d->n[2];
    for (int oz = -cf; oz <= cf; ++oz) {
        int z = cz + oz;
        if (d->periodic[2]) { z += z < 0 ? n2 : 0; z -= z >= n2 ? n2 : 0; }
        else if (z < 0 || z >= n2) continue;
        for (int oy = -cf; oy <= cf; ++oy) {
            int y = cy + oy;
            if (d->periodic[1]) { y += y < 0 ? n1 : 0; y -= y >= n1 ? n1 : 0; }
            else if (y < 0 || y >= n1) continue;
            for (int ox = -cf; ox <= cf; ++ox) {
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
    double xo[3], vo[3], wo[3];
    advance<R>(s, d, kind, p, mode, kick, dt, xo, vo, wo);
    for (int a = 0; a < 3; a++)
        if (!isfinite(xo[a]) || !isfinite(vo[a]) || !isfinite(wo[a])) err |= ERR_NONFINITE;
    int c0 = cell_coord(d, 0, xo[0], err);
    int c1 = cell_coord(d, 1, xo[1], err);
    int c2 = cell_coord(d, 2, xo[2], err);
    uint32_t lin = (uint32_t)c0 + (uint32_t)d->n[0] * ((uint32_t)c1 + (uint32_t)d->n[1] * (uint32_t)c2);
    uint32_t key = s.rank_of_lin[d->cell_off + lin];
    s.key[p] = key;
    s.slot[p] = atomicAdd(&s.count[key], 1u);
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
    uint32_t myid = s.id[cur][op];
    uint32_t dst = q;
    if (e - b <= (uint32_t)kMaxCell) {
        uint32_t rank = 0;
        for (uint32_t k = b; k < e; k++) rank += s.id[cur][s.tmp[k]] < myid ? 1u : 0u;
        dst = b + rank;
    } else {
        atomicOr(s.err, (uint32_t)ERR_CAPACITY);
    }
    uint8_t skv = s.sk[cur][op];
    double xo[3], vo[3], wo[3];
    advance<R>(s, d, skv >> 1, op, mode, kick, dt, xo, vo, wo);
    for (int a = 0; a < 3; a++) {
        s.x[nxt][a * N + dst] = xo[a];
        s.v[nxt][a * N + dst] = vo[a];
        s.w[nxt][a * N + dst] = wo[a];
    }
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

// Density (kernel summation), unlike-neighbour kernel sum S and Tait EOS.
template <typename R, bool KAHAN>
__global__ void k_density(DevState s)
{
    PIdx t = map_thread(s);
    if (!t.active) return;
    const InstDesc *d = t.d;
    const uint32_t p = t.p, N = s.N;
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
            if (q == p) continue;
            double dx0 = min_img(d, 0, xi0 - X[q]);
            double dx1 = min_img(d, 1, xi1 - X[N + q]);
            double dx2 = min_img(d, 2, xi2 - X[2 * N + q]);
            double r2 = r2_exact(dx0, dx1, dx2);
            if (r2 < cut2) {
                R W = kernel_W<R>(kernel, (R)r2, inv_h, wnorm);
                sw.add(W);
                if ((SK[q] & 1) != spi) su.add(W);
            }
        }
    });
    double mi = d->mass[spi];
    double rho, P;
    if (kind == KIND_WALL_OUTER) {
        rho = d->rho0;
        P = 0.0;
    } else {
        rho = mi * (d->W0 + sw.value());
        double r = rho / d->rho0;
        double r2 = r * r;
        P = d->B * ((r2 * r2) * (r2 * r) - 1.0);
    }
    double S = su.value();
    double V = mi / rho;
    double ir2 = 1.0 / (rho * rho);
    R *aux = (R *)s.aux + 4 * (size_t)p;
    aux[0] = (R)V;
    aux[1] = (R)(P * ir2);
    aux[2] = (R)ir2;
    aux[3] = (R)(S > 0.0 ? V / S : 0.0);
    R *rp = (R *)s.rhoP + 2 * (size_t)p;
    rp[0] = (R)rho;
    rp[1] = (R)P;
    if (!isfinite(rho) || !isfinite(P)) err |= ERR_NONFINITE;
    if (err) atomicOr(s.err, err);
}

// Pair forces and spin torques on fluid particles (walls: zero, their motion is imposed).
//   pressure     m_i m_j (P_i/rho_i^2 + P_j/rho_j^2) F r
//   interfacial  g_T (r_x, r_y, 0), g_T = -sigma_T m_i m_j (1/rho_i^2 + 1/rho_j^2) F, unlike
//   viscous      -4 eta V_i V_j F (v_ij - (w_i + w_j)/2 × r), viscous-viscous pairs
//   friction     -C_l W (V_i/S_i + V_j/S_j) v_ij, unlike pairs
//   torque       -1/2 r × (non-central force), added to both particles of the pair
template <typename R, bool KAHAN>
__global__ void k_force(DevState s)
{
    PIdx t = map_thread(s);
    if (!t.active) return;
    const InstDesc *d = t.d;
    const uint32_t p = t.p, N = s.N;
    const int cur = s.cur;
    R *acc = (R *)s.acc, *alpha = (R *)s.alpha;
    const uint8_t *SK = s.sk[cur];
    const uint8_t ski = SK[p];
    if ((ski >> 1) != KIND_FLUID) {
        for (int a = 0; a < 3; a++) { acc[a * N + p] = (R)0; alpha[a * N + p] = (R)0; }
        return;
    }
    const double *X = s.x[cur], *Vv = s.v[cur], *Ww = s.w[cur];
    const R *AUX = (const R *)s.aux;
    const double xi0 = X[p], xi1 = X[N + p], xi2 = X[2 * N + p];
    const double vi0 = Vv[p], vi1 = Vv[N + p], vi2 = Vv[2 * N + p];
    const double wi0 = Ww[p], wi1 = Ww[N + p], wi2 = Ww[2 * N + p];
    const int spi = ski & 1;
    const R Vi = AUX[4 * (size_t)p], Pri = AUX[4 * (size_t)p + 1];
    const R ir2i = AUX[4 * (size_t)p + 2], VSi = AUX[4 * (size_t)p + 3];
    const R mi = (R)d->mass[spi];
    const R m0 = (R)d->mass[0], m1 = (R)d->mass[1];
    const R sigT = (R)d->sigma_T, eta4 = (R)(4.0 * d->eta), Cl = (R)d->C_l;
    const int kernel = d->kernel;
    const double cut2 = d->cut2;
    const R inv_h = (R)d->inv_h, wnorm = (R)d->wnorm;
    const uint32_t cxyz = s.cell_xyz[s.pcell[p]];
    uint32_t err = 0;
    Acc<R, KAHAN> F0, F1, F2, T0, T1, T2;
    for_each_cell(s, d, cxyz & 1023, (cxyz >> 10) & 1023, cxyz >> 20, err,
                  [&](uint32_t b, uint32_t e) {
        for (uint32_t q = b; q < e; ++q) {
            if (q == p) continue;
            double dx0 = min_img(d, 0, xi0 - X[q]);
            double dx1 = min_img(d, 1, xi1 - X[N + q]);
            double dx2 = min_img(d, 2, xi2 - X[2 * N + q]);
            double r2d = r2_exact(dx0, dx1, dx2);
            if (!(r2d < cut2)) continue;
            const int spj = SK[q] & 1;
            const R Vj = AUX[4 * (size_t)q], Prj = AUX[4 * (size_t)q + 1];
            const R ir2j = AUX[4 * (size_t)q + 2], VSj = AUX[4 * (size_t)q + 3];
            const R mj = spj ? m1 : m0;
            const R r0 = (R)dx0, r1 = (R)dx1, r2 = (R)dx2;
            R W, Fk;
            kernel_WF<R>(kernel, (R)r2d, inv_h, wnorm, W, Fk);
            const R v0 = (R)(vi0 - Vv[q]), v1 = (R)(vi1 - Vv[N + q]), v2 = (R)(vi2 - Vv[2 * N + q]);
            const R mm = mi * mj;
            // pressure (central)
            R gp = mm * (Pri + Prj) * Fk;
            R f0 = gp * r0, f1 = gp * r1, f2 = gp * r2;
            R n0 = 0, n1 = 0, n2 = 0;
            R c0 = 0, c1 = 0, c2 = 0;  // non-central force
            if (spj != spi) {
                R gT = -sigT * mm * (ir2i + ir2j) * Fk;
                f0 += gT * r0;
                f1 += gT * r1;
                n0 += (R)0.5 * gT * r2 * r1;
                n1 += (R)-0.5 * gT * r2 * r0;
                R gm = -Cl * W * (VSi + VSj);
                c0 += gm * v0; c1 += gm * v1; c2 += gm * v2;
            }
            if ((spi & spj) != 0) {
                const R s0 = (R)(0.5 * (wi0 + Ww[q])), s1 = (R)(0.5 * (wi1 + Ww[N + q])),
                        s2 = (R)(0.5 * (wi2 + Ww[2 * N + q]));
                R u0 = v0 - (s1 * r2 - s2 * r1);
                R u1 = v1 - (s2 * r0 - s0 * r2);
                R u2 = v2 - (s0 * r1 - s1 * r0);
                R gv = -eta4 * Vi * Vj * Fk;
                c0 += gv * u0; c1 += gv * u1; c2 += gv * u2;
            }
            f0 += c0; f1 += c1; f2 += c2;
            n0 += (R)-0.5 * (r1 * c2 - r2 * c1);
            n1 += (R)-0.5 * (r2 * c0 - r0 * c2);
            n2 += (R)-0.5 * (r0 * c1 - r1 * c0);
            F0.add(f0); F1.add(f1); F2.add(f2);
            T0.add(n0); T1.add(n1); T2.add(n2);
        }
    });
    double im = 1.0 / d->mass[spi];
    double iI = 1.0 / d->inertia[spi];
    double a0 = F0.value() * im, a1 = F1.value() * im, a2 = F2.value() * im;
    double al0 = T0.value() * iI, al1 = T1.value() * iI, al2 = T2.value() * iI;
    acc[p] = (R)a0; acc[N + p] = (R)a1; acc[2 * N + p] = (R)a2;
    alpha[p] = (R)al0; alpha[N + p] = (R)al1; alpha[2 * N + p] = (R)al2;
    if (!isfinite(a0) || !isfinite(a1) || !isfinite(a2) || !isfinite(al0) || !isfinite(al1) ||
        !isfinite(al2))
        err |= ERR_NONFINITE;
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
    if (P) P[id] = (double)rp[1];
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

// phase 0: row_ptr[id + 1] = neighbour count; phase 1: fill columns and sort each row.
__global__ void k_debug_nbr(DevState s, int phase, int64_t *row_ptr, int32_t *cols)
{
    PIdx t = map_thread(s);
    if (!t.active) return;
    const InstDesc *d = t.d;
    const uint32_t p = t.p, N = s.N;
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
    if (phase == 0) {
        row_ptr[id + 1] = cnt;
    } else {
        for (int64_t i = 1; i < cnt; i++) {
            int32_t v = cols[base + i];
            int64_t j = i - 1;
            while (j >= 0 && cols[base + j] > v) { cols[base + j + 1] = cols[base + j]; j--; }
            cols[base + j + 1] = v;
        }
    }
    if (err) atomicOr(s.err, err);
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
    else k_density<float, true><<<g, L.bs_density, 0, st>>>(d);
    return hipGetLastError();
}

hipError_t launch_force(const DevState &d, const Launch &L, hipStream_t st)
{
    unsigned g = grid_for(d.n_waves, L.bs_force);
    if (d.precision == 0) k_force<double, false><<<g, L.bs_force, 0, st>>>(d);
    else k_force<float, true><<<g, L.bs_force, 0, st>>>(d);
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

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, size_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    k_fill_u32<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, value, n);
    return hipGetLastError();
}

}  // namespace sph
