/*
 * oracle.c -- plain, slow, single-threaded FP64 reference for the per-timestep
 * update of the synthetic BRAMS-like application and for its load balancers,
 * after "Dynamic Load Balancing in GPU-Based Systems -- Early Experiments"
 * (Fazenda, Mendes, Kale, Panetta, Rodrigues; arXiv 1310.4218).
 *
 * TEST INFRASTRUCTURE ONLY.  The HIP library never links, loads or calls this
 * file; only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg do.  It shares no code, header, table or helper with the HIP path.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fno-fast-math -shared -fPIC
 *        oracle.c -o liboracle.so -lm
 * (-ffp-contract=off: every a*b+c below is a rounded multiply then a rounded
 * add, in the order written.)
 *
 * What the paper fixes and what is read here (each reading is listed with the
 * design notes of the repository):
 *  - Section IV: each time step applies a 3D Jacobi ("laminar diffusion")
 *    update, then a column "physics" loop (Fig. 2: JACOBI kernel, then PHYSIC).
 *    Jacobi here is the 7-point update s = cc*q + cn*(sum of the 6 neighbours),
 *    periodic in x and y, zero-flux (mirror ghost) in z.
 *  - Section VI, Fig. 4: the physics trip count per column comes from a
 *    load-control array that is moved across the domain over time.  Here that
 *    array is k_t(x,y) = kmin + floor((kmax-kmin) * max_h exp(-r_h^2/(2 sigma^2))),
 *    r_h^2 the integer minimum-image squared distance to hotspot h at step t.
 *  - The physics map per iteration is Phi(q) = q + eps*(q - (q*q)*q), applied
 *    k times to every cell of the column (a pointwise reading of Fig. 1); the
 *    vertical variant sweeps the column k times with a dependency on the
 *    level below (Fig. 1 / Fig. 4 as written).
 *  - Section V / Section VI: load is measured per virtual processor (chunk);
 *    here in deterministic work units w_c = sum over columns of nz*(alpha+k).
 *  - Section VI, Experiment A: GreedyLB places objects heaviest first, each on
 *    the processor with the least load so far.  Experiment B: RefineSwapLB
 *    moves objects off the most overloaded processors towards the average,
 *    swapping when no single move fits.  Refine is the move-only half.
 *
 * Parity status of each function: pinned by the CPU tests (closed-form
 * eigenmodes, constants, mass, symmetry, published generator outputs,
 * exhaustive search for the balancers).  The order inside a step (stencil,
 * then physics) is pinned by a delta field; the windowed runner and the
 * windowed initial field by the whole-grid run they must reproduce.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Initial field: uniform values in [-1, 1) from SplitMix64 (Steele, Lea and
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014).
 * The value of global cell n is the (n+1)-th output of a SplitMix64 stream
 * seeded with `seed`: gamma-increment the state, then the three-round mix. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t n)
{
    uint64_t z = seed + (n + 1u) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Top 24 bits of the output, centred: (m - 2^23) * 2^-23, exact in FP32/FP64. */
void orc_init_field(int64_t ncells, uint64_t seed, double *q)
{
    for (int64_t n = 0; n < ncells; ++n) {
        uint64_t m = orc_splitmix64(seed, (uint64_t)n) >> 40;
        q[n] = ((double)(int64_t)m - 8388608.0) * (1.0 / 8388608.0);
    }
}

/* ------------------------------------------------------------------------ */
/* Load-control array (Section VI, Fig. 4 and the moving array C). */
static int64_t wrap64(int64_t a, int64_t n)
{
    int64_t r = a % n;
    return r < 0 ? r + n : r;
}

static int64_t min_image(int64_t a, int64_t b, int64_t n)
{
    int64_t d = a - b;
    if (d < 0) d = -d;
    return (n - d < d) ? n - d : d;
}

/* Trip count of global column (x, y) of an NX x NY grid at absolute time t
 * (hotspot h sits at (hx0[h] + hvx[h]*t, hy0[h] + hvy[h]*t) modulo the grid). */
static int32_t k_at(int64_t x, int64_t y, int32_t NX, int32_t NY, int32_t nhot,
                    const int64_t *hx0, const int64_t *hy0, const int64_t *hvx,
                    const int64_t *hvy, int64_t t, double sigma, int32_t kmin, int32_t kmax)
{
    double g = 0.0;
    for (int32_t h = 0; h < nhot; ++h) {
        int64_t cx = wrap64(hx0[h] + hvx[h] * t, NX);
        int64_t cy = wrap64(hy0[h] + hvy[h] * t, NY);
        int64_t dx = min_image(x, cx, NX);
        int64_t dy = min_image(y, cy, NY);
        int64_t r2 = dx * dx + dy * dy;
        double e = exp(-(double)r2 / (2.0 * sigma * sigma));
        if (e > g) g = e;
    }
    return kmin + (int32_t)floor((double)(kmax - kmin) * g);
}

/* k[y*nx + x] over the whole grid at absolute time index t. */
void orc_kfield(int32_t nx, int32_t ny, int32_t nhot, const int64_t *hx0, const int64_t *hy0,
                const int64_t *hvx, const int64_t *hvy, int64_t t, double sigma,
                int32_t kmin, int32_t kmax, int32_t *k)
{
    for (int32_t y = 0; y < ny; ++y)
        for (int32_t x = 0; x < nx; ++x)
            k[(int64_t)y * nx + x] = k_at(x, y, nx, ny, nhot, hx0, hy0, hvx, hvy, t, sigma,
                                          kmin, kmax);
}

/* ------------------------------------------------------------------------ */
/* One 3D Jacobi update (Section IV): 7-point, periodic x/y, mirror ghost in z.
 * Layout: q[((y*nx)+x)*nz + z], the vertical index fastest as in Fig. 1. */
void orc_stencil(int32_t nx, int32_t ny, int32_t nz, double cc, double cn,
                 const double *q, double *s)
{
    for (int32_t y = 0; y < ny; ++y) {
        int32_t ym = (y == 0) ? ny - 1 : y - 1;
        int32_t yp = (y == ny - 1) ? 0 : y + 1;
        for (int32_t x = 0; x < nx; ++x) {
            int32_t xm = (x == 0) ? nx - 1 : x - 1;
            int32_t xp = (x == nx - 1) ? 0 : x + 1;
            const double *c = q + ((int64_t)y * nx + x) * nz;
            const double *cxm = q + ((int64_t)y * nx + xm) * nz;
            const double *cxp = q + ((int64_t)y * nx + xp) * nz;
            const double *cym = q + ((int64_t)ym * nx + x) * nz;
            const double *cyp = q + ((int64_t)yp * nx + x) * nz;
            double *o = s + ((int64_t)y * nx + x) * nz;
            for (int32_t z = 0; z < nz; ++z) {
                double zm = (z == 0) ? c[z] : c[z - 1];
                double zp = (z == nz - 1) ? c[z] : c[z + 1];
                double sum = cxm[z] + cxp[z];
                sum = sum + cym[z];
                sum = sum + cyp[z];
                sum = sum + zm;
                sum = sum + zp;
                o[z] = cc * c[z] + cn * sum;
            }
        }
    }
}

/* Column physics: k(x,y) applications of Phi(q) = q + eps*(q - (q*q)*q) to every
 * cell of column (x,y), in place (Section VI, Fig. 4 trip count; Fig. 1 column). */
void orc_physics(int32_t nx, int32_t ny, int32_t nz, double eps, const int32_t *k, double *s)
{
    for (int64_t col = 0; col < (int64_t)nx * ny; ++col) {
        double *c = s + col * nz;
        for (int32_t z = 0; z < nz; ++z) {
            double q = c[z];
            for (int32_t it = 0; it < k[col]; ++it) {
                double q3 = (q * q) * q;
                q = q + eps * (q - q3);
            }
            c[z] = q;
        }
    }
}

/* Column physics with a vertical dependency (Fig. 1: a(k) = f(b(k), a(k-1));
 * Fig. 4: the level loop repeated C(i,j) times).  For each column, k(x,y)
 * upward sweeps; within a sweep level z (1..nz-1, in order) becomes
 *   q[z] + eps*((q[z-1]*q[z-1])*q[z-1] - (q[z]*q[z])*q[z])
 * using level z-1 as already updated in the same sweep.  Level 0 is the
 * bottom boundary and is not updated. */
void orc_physics_vertical(int32_t nx, int32_t ny, int32_t nz, double eps, const int32_t *k,
                          double *s)
{
    for (int64_t col = 0; col < (int64_t)nx * ny; ++col) {
        double *c = s + col * nz;
        for (int32_t it = 0; it < k[col]; ++it) {
            for (int32_t z = 1; z < nz; ++z) {
                double below = (c[z - 1] * c[z - 1]) * c[z - 1];
                double here = (c[z] * c[z]) * c[z];
                c[z] = c[z] + eps * (below - here);
            }
        }
    }
}

/* Per-chunk work of one step: w_c = sum over the chunk's columns of nz*(alpha + k).
 * Chunk c = j*px + i covers [xs[i], xs[i+1]) x [ys[j], ys[j+1]). */
void orc_chunk_work(int32_t nx, int32_t nz, int32_t px, int32_t py, const int32_t *xs,
                    const int32_t *ys, int32_t alpha, const int32_t *k, double *w)
{
    for (int32_t j = 0; j < py; ++j) {
        for (int32_t i = 0; i < px; ++i) {
            double acc = 0.0;
            for (int32_t y = ys[j]; y < ys[j + 1]; ++y)
                for (int32_t x = xs[i]; x < xs[i + 1]; ++x)
                    acc += (double)nz * (double)(alpha + k[(int64_t)y * nx + x]);
            w[j * px + i] = acc;
        }
    }
}

double orc_sum(int64_t n, const double *q)
{
    double a = 0.0;
    for (int64_t i = 0; i < n; ++i) a += q[i];
    return a;
}

/* T steps of the whole update for nfields independent fields sharing one cost
 * field.  q holds nfields*ny*nx*nz values on entry and on exit.  For step
 * index s (0-based) the hotspots sit at time t0 + s.  Outputs, when non-NULL:
 * work[s*C + c] (work units of step s), cksum[s] (sum of all cells after step s),
 * kout (the cost field of the last step). */
int orc_run(int32_t nx, int32_t ny, int32_t nz, int32_t nfields, int32_t px, int32_t py,
            const int32_t *xs, const int32_t *ys, double cc, double cn, double eps,
            int32_t nhot, const int64_t *hx0, const int64_t *hy0, const int64_t *hvx,
            const int64_t *hvy, double sigma, int32_t kmin, int32_t kmax, int32_t alpha,
            int64_t t0, int32_t nsteps, double *q, double *work, double *cksum, int32_t *kout,
            int32_t vertical)
{
    int64_t ncol = (int64_t)nx * ny;
    int64_t nper = ncol * nz;
    double *s = (double *)malloc(sizeof(double) * (size_t)nper);
    int32_t *k = (int32_t *)malloc(sizeof(int32_t) * (size_t)ncol);
    if (!s || !k) {
        free(s);
        free(k);
        return -1;
    }
    for (int32_t step = 0; step < nsteps; ++step) {
        orc_kfield(nx, ny, nhot, hx0, hy0, hvx, hvy, t0 + step, sigma, kmin, kmax, k);
        for (int32_t f = 0; f < nfields; ++f) {
            double *qf = q + (int64_t)f * nper;
            orc_stencil(nx, ny, nz, cc, cn, qf, s);
            if (vertical)
                orc_physics_vertical(nx, ny, nz, eps, k, s);
            else
                orc_physics(nx, ny, nz, eps, k, s);
            memcpy(qf, s, sizeof(double) * (size_t)nper);
        }
        if (work) {
            orc_chunk_work(nx, nz, px, py, xs, ys, alpha, k, work + (int64_t)step * px * py);
            if (nfields > 1)
                for (int32_t c = 0; c < px * py; ++c)
                    work[(int64_t)step * px * py + c] *= (double)nfields;
        }
        if (cksum) cksum[step] = orc_sum(nper * nfields, q);
    }
    if (kout) memcpy(kout, k, sizeof(int32_t) * (size_t)ncol);
    free(s);
    free(k);
    return 0;
}

/* Same update restricted to a window of nxw x nyw columns whose local column
 * (x, y) is global column ((ox + x) mod NX, (oy + y) mod NY) of an NX x NY grid.
 * The window is advanced as if it were periodic, so after nsteps steps only
 * the columns at least nsteps away from its border hold the true values (the
 * 7-point update reaches one column further per step).  q (nyw*nxw*nz values,
 * one field) holds the window on entry and on exit. */
int orc_run_window(int32_t nxw, int32_t nyw, int32_t nz, int32_t ox, int32_t oy, int32_t NX,
                   int32_t NY, double cc, double cn, double eps, int32_t nhot,
                   const int64_t *hx0, const int64_t *hy0, const int64_t *hvx,
                   const int64_t *hvy, double sigma, int32_t kmin, int32_t kmax, int64_t t0,
                   int32_t nsteps, double *q, int32_t vertical)
{
    int64_t ncol = (int64_t)nxw * nyw;
    double *s = (double *)malloc(sizeof(double) * (size_t)(ncol * nz));
    int32_t *k = (int32_t *)malloc(sizeof(int32_t) * (size_t)ncol);
    if (!s || !k) {
        free(s);
        free(k);
        return -1;
    }
    for (int32_t step = 0; step < nsteps; ++step) {
        for (int32_t y = 0; y < nyw; ++y)
            for (int32_t x = 0; x < nxw; ++x)
                k[(int64_t)y * nxw + x] = k_at(wrap64((int64_t)ox + x, NX), wrap64((int64_t)oy + y, NY),
                                               NX, NY, nhot, hx0, hy0, hvx, hvy, t0 + step, sigma,
                                               kmin, kmax);
        orc_stencil(nxw, nyw, nz, cc, cn, q, s);
        if (vertical)
            orc_physics_vertical(nxw, nyw, nz, eps, k, s);
        else
            orc_physics(nxw, nyw, nz, eps, k, s);
        memcpy(q, s, sizeof(double) * (size_t)(ncol * nz));
    }
    free(s);
    free(k);
    return 0;
}

/* Initial values of a window of field f (see orc_init_field): global cell
 * ((f*NY + gy)*NX + gx)*nz + z with gx = (ox + x) mod NX, gy = (oy + y) mod NY. */
void orc_init_window(int32_t nxw, int32_t nyw, int32_t nz, int32_t ox, int32_t oy, int32_t NX,
                     int32_t NY, int32_t f, uint64_t seed, double *q)
{
    for (int32_t y = 0; y < nyw; ++y)
        for (int32_t x = 0; x < nxw; ++x) {
            int64_t gx = wrap64((int64_t)ox + x, NX), gy = wrap64((int64_t)oy + y, NY);
            int64_t base = (((int64_t)f * NY + gy) * NX + gx) * nz;
            for (int32_t z = 0; z < nz; ++z) {
                uint64_t m = orc_splitmix64(seed, (uint64_t)(base + z)) >> 40;
                q[((int64_t)y * nxw + x) * nz + z] = ((double)(int64_t)m - 8388608.0) * (1.0 / 8388608.0);
            }
        }
}

/* ------------------------------------------------------------------------ */
/* Balancers.  Loads w[C] >= 0; slots (the paper's processors) 0..S-1.       */

/* Chunk order used by both balancers: load descending, then id ascending. */
static const double *g_sort_w;
static int heavier_first(const void *a, const void *b)
{
    int32_t ia = *(const int32_t *)a, ib = *(const int32_t *)b;
    if (g_sort_w[ia] > g_sort_w[ib]) return -1;
    if (g_sort_w[ia] < g_sort_w[ib]) return 1;
    return (ia < ib) ? -1 : (ia > ib);
}

static void order_heavy_first(const double *w, int32_t C, int32_t *ord)
{
    for (int32_t c = 0; c < C; ++c) ord[c] = c;
    g_sort_w = w;
    qsort(ord, (size_t)C, sizeof(int32_t), heavier_first);
}

/* Least loaded slot, lowest index on ties (linear scan). */
static int32_t least_loaded(const double *L, int32_t S)
{
    int32_t best = 0;
    for (int32_t s = 1; s < S; ++s)
        if (L[s] < L[best]) best = s;
    return best;
}

/* GreedyLB (Section VI, Experiment A): heaviest chunk to the least loaded slot;
 * the previous placement is ignored. */
int orc_greedy(const double *w, int32_t C, int32_t S, int32_t *map)
{
    if (C < 0 || S < 1) return -1;
    int32_t *ord = (int32_t *)malloc(sizeof(int32_t) * (size_t)(C > 0 ? C : 1));
    double *L = (double *)calloc((size_t)S, sizeof(double));
    if (!ord || !L) {
        free(ord);
        free(L);
        return -1;
    }
    order_heavy_first(w, C, ord);
    for (int32_t i = 0; i < C; ++i) {
        int32_t c = ord[i];
        int32_t s = least_loaded(L, S);
        map[c] = s;
        L[s] += w[c];
    }
    free(ord);
    free(L);
    return 0;
}

/* RefineLB with threshold thr (the move-only half of RefineSwapLB, Section VI,
 * Experiment B): starting from old_map, repeatedly take the most loaded slot p
 * that is above limit = (W/S)*thr and move its heaviest chunk that fits under
 * the limit onto the least loaded slot q; a slot with no such chunk is left
 * as it is.  W sums the loads in chunk order; slot loads accumulate in chunk
 * order.  Ties: lowest slot index, then heavier chunk, then lower chunk id. */
int orc_refine(const double *w, const int32_t *old_map, int32_t C, int32_t S, double thr,
               int32_t *map)
{
    if (C < 0 || S < 1) return -1;
    double *L = (double *)calloc((size_t)S, sizeof(double));
    char *done = (char *)calloc((size_t)S, 1);
    int32_t *ord = (int32_t *)malloc(sizeof(int32_t) * (size_t)(C > 0 ? C : 1));
    if (!L || !done || !ord) {
        free(L);
        free(done);
        free(ord);
        return -1;
    }
    double W = 0.0;
    for (int32_t c = 0; c < C; ++c) W += w[c];
    double avg = W / (double)S;
    double limit = avg * thr;
    for (int32_t c = 0; c < C; ++c) {
        map[c] = old_map[c];
        L[map[c]] += w[c];
    }
    order_heavy_first(w, C, ord);
    for (;;) {
        int32_t p = -1;
        for (int32_t s = 0; s < S; ++s)
            if (!done[s] && (p < 0 || L[s] > L[p])) p = s;
        if (p < 0 || !(L[p] > limit)) break;
        int32_t q = least_loaded(L, S);
        int32_t moved = -1;
        for (int32_t i = 0; i < C; ++i) {
            int32_t c = ord[i];
            if (map[c] == p && L[q] + w[c] <= limit) {
                moved = c;
                break;
            }
        }
        if (moved < 0) {
            done[p] = 1;
            continue;
        }
        map[moved] = q;
        L[p] -= w[moved];
        L[q] += w[moved];
    }
    free(L);
    free(done);
    free(ord);
    return 0;
}

/* Chunk order light first: load ascending, then id ascending. */
static int lighter_first(const void *a, const void *b)
{
    int32_t ia = *(const int32_t *)a, ib = *(const int32_t *)b;
    if (g_sort_w[ia] < g_sort_w[ib]) return -1;
    if (g_sort_w[ia] > g_sort_w[ib]) return 1;
    return (ia < ib) ? -1 : (ia > ib);
}

/* RefineSwapLB with threshold thr (Section VI, Experiment B: move objects away
 * from the most overloaded processors towards the average, and swap objects
 * when no single move from an overloaded processor fits).  As orc_refine,
 * except that when no chunk of p fits on the least loaded slot, the first
 * swap that fits is made before p is given up: slots r != p in increasing
 * (load, index) order, chunks c of p heavy first, chunks d of r light first
 * (ties by id), with w[d] < w[c] and L[r] + (w[c] - w[d]) <= limit.  A swap
 * lowers L[p] and keeps r at or under the limit.  At most 4*C moves and
 * swaps are made in total. */
int orc_refineswap(const double *w, const int32_t *old_map, int32_t C, int32_t S, double thr,
                   int32_t *map)
{
    if (C < 0 || S < 1) return -1;
    size_t nc = (size_t)(C > 0 ? C : 1);
    double *L = (double *)calloc((size_t)S, sizeof(double));
    char *done = (char *)calloc((size_t)S, 1);
    int32_t *heavy = (int32_t *)malloc(sizeof(int32_t) * nc);
    int32_t *light = (int32_t *)malloc(sizeof(int32_t) * nc);
    int32_t *sl = (int32_t *)malloc(sizeof(int32_t) * (size_t)S);
    if (!L || !done || !heavy || !light || !sl) {
        free(L);
        free(done);
        free(heavy);
        free(light);
        free(sl);
        return -1;
    }
    double W = 0.0;
    for (int32_t c = 0; c < C; ++c) W += w[c];
    double limit = (W / (double)S) * thr;
    for (int32_t c = 0; c < C; ++c) {
        map[c] = old_map[c];
        L[map[c]] += w[c];
    }
    order_heavy_first(w, C, heavy);
    for (int32_t c = 0; c < C; ++c) light[c] = c;
    g_sort_w = w;
    qsort(light, (size_t)C, sizeof(int32_t), lighter_first);

    int64_t ops = 0;
    while (ops < 4 * (int64_t)C) {
        int32_t p = -1;
        for (int32_t s = 0; s < S; ++s)
            if (!done[s] && (p < 0 || L[s] > L[p])) p = s;
        if (p < 0 || !(L[p] > limit)) break;
        int32_t q = least_loaded(L, S);
        int32_t moved = -1;
        for (int32_t i = 0; i < C; ++i) {
            int32_t c = heavy[i];
            if (map[c] == p && L[q] + w[c] <= limit) {
                moved = c;
                break;
            }
        }
        if (moved >= 0) {
            map[moved] = q;
            L[p] -= w[moved];
            L[q] += w[moved];
            ++ops;
            continue;
        }
        /* slots in increasing (load, index) order (insertion sort) */
        for (int32_t s = 0; s < S; ++s) {
            int32_t i = s;
            while (i > 0 && (L[sl[i - 1]] > L[s] || (L[sl[i - 1]] == L[s] && sl[i - 1] > s))) {
                sl[i] = sl[i - 1];
                --i;
            }
            sl[i] = s;
        }
        int32_t sc = -1, sd = -1, sr = -1;
        for (int32_t ri = 0; ri < S && sc < 0; ++ri) {
            int32_t r = sl[ri];
            if (r == p) continue;
            for (int32_t i = 0; i < C && sc < 0; ++i) {
                int32_t c = heavy[i];
                if (map[c] != p) continue;
                for (int32_t j = 0; j < C; ++j) {
                    int32_t d = light[j];
                    if (map[d] == r && w[d] < w[c] && L[r] + (w[c] - w[d]) <= limit) {
                        sc = c;
                        sd = d;
                        sr = r;
                        break;
                    }
                }
            }
        }
        if (sc < 0) {
            done[p] = 1;
            continue;
        }
        map[sc] = sr;
        map[sd] = p;
        L[p] = (L[p] - w[sc]) + w[sd];
        L[sr] = (L[sr] - w[sd]) + w[sc];
        ++ops;
    }
    free(L);
    free(done);
    free(heavy);
    free(light);
    free(sl);
    return 0;
}
