// Device code of liblbgrid for gfx950 (CDNA4): the fused time-step kernel of
// the over-decomposed grid (3D Jacobi update + column physics, Section IV and
// Section VI Fig. 4 of the paper) with in-kernel per-chunk load measurement
// (Section V), in three launch forms:
//   - plain: one launch per chunk over that chunk's items, chunks in id order;
//   - persistent: one launch per step whose workgroups claim items from work
//     queues with atomic counters (the chunks of balancer slot s, the paper's
//     processors, feed queue s mod Q), optionally taking work from other
//     queues once their own is empty;
//   - one workgroup per item, in the queues' order, the hardware dispatcher
//     scheduling them; this form can also advance every item by two or three
//     steps per launch (temporal blocking: each item recomputes the earlier
//     steps on rings of cells around it, so that no intermediate step goes
//     through memory).
//
// Data layout: field[((f*ny + y)*nx + x)*nz + z] (z fastest).  Chunks are cut
// into tiles of up to TX x TY columns; a work item is a range of rows of one
// tile (the whole tile unless the host split a costly tile into row ranges).
// In the row pipelines a workgroup has TX*nz/V threads; thread t owns V
// consecutive levels of column t / (nz/V) of the current row (the column
// march, below, adds threads for the halo columns).  The item is swept row by
// row (along y) through a ring of LDS rows, each holding TX+2 columns (one halo
// column on either side) of all nz levels: rows y-1, y, y+1 are read by the stencil
// while later rows are in flight, either straight into the ring (direct
// global->LDS loads, B rows per batch) or through registers (2, 4 or 8 rows).
// Every cell is read from HBM once per item and written once; halo columns and
// halo rows are re-read by the neighbouring items, and the register pipeline
// re-reads an item's last halo row in place of rows past the item (mostly
// from L2 / MALL).
//
// Arithmetic per cell, with s the stencil value and k the column's trip count:
//   FP32:        q <- fma(eps, fma(-(q*q), q, q), q), k times
//   FP32 Kahan:  d = eps*(q - q^3); y = d - c; t = q + y; c = (t - q) - y; q = t
//   FP64:        q <- q + eps*(q - (q*q)*q) with every product and sum rounded
//                separately in the written order (no contraction), which makes
//                the FP64 path bit-identical to a plain sequential evaluation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <type_traits>

#include "lbgrid.h"
#include "lbgrid_internal.h"

namespace lbgrid {
namespace {

constexpr int kWave = 64;

// V levels of one thread, aligned to their size when V is a power of two (one
// wide LDS access); V = 5 is aligned to one element
template <typename T, int V>
struct alignas(sizeof(T) * ((V & (V - 1)) == 0 ? V : 1)) Vec {
    T v[V];
};

template <typename T, int V>
__device__ __forceinline__ Vec<T, V> ld(const T* p) {
    return *reinterpret_cast<const Vec<T, V>*>(p);
}
template <typename T, int V>
__device__ __forceinline__ void st(T* p, const Vec<T, V>& x) {
    *reinterpret_cast<Vec<T, V>*>(p) = x;
}

// ---- arithmetic of one cell ------------------------------------------------
__device__ __forceinline__ float combine(float cc, float cn, float c, float sum) {
    return cc * c + cn * sum;  // contracted to one fma
}
__device__ __forceinline__ double combine(double cc, double cn, double c, double sum) {
#pragma clang fp contract(off)
    return cc * c + cn * sum;
}

// Physics of the V cells of one thread (the per-cell arithmetic in the file
// header), with the V chains interleaved for ILP; each cell's operations and
// their order are those of a plain loop over its k iterations.
template <int V>
__device__ __forceinline__ void physics_vec_fp64(double eps, int k, double (&q)[V]) {
#pragma clang fp contract(off)
    for (int it = 0; it < k; ++it) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const double q3 = (q[v] * q[v]) * q[v];
            q[v] = q[v] + eps * (q[v] - q3);
        }
    }
}

template <int KAHAN, typename T, int V>
__device__ __forceinline__ void physics_vec(T eps, int k, T (&q)[V]) {
    if constexpr (sizeof(T) == 8) {
        physics_vec_fp64<V>(eps, k, q);
    } else if constexpr (KAHAN) {
        float comp[V];
#pragma unroll
        for (int v = 0; v < V; ++v) comp[v] = 0.0f;
        for (int it = 0; it < k; ++it) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const float d = eps * (q[v] - (q[v] * q[v]) * q[v]);
                const float y = d - comp[v];
                const float t = q[v] + y;
                comp[v] = (t - q[v]) - y;
                q[v] = t;
            }
        }
    } else {
        // two iterations per trip: half the loop-control instructions
        int it = 0;
        for (; it + 1 < k; it += 2) {
#pragma unroll
            for (int v = 0; v < V; ++v) q[v] = q[v] + eps * (q[v] - (q[v] * q[v]) * q[v]);
#pragma unroll
            for (int v = 0; v < V; ++v) q[v] = q[v] + eps * (q[v] - (q[v] * q[v]) * q[v]);
        }
        if (it < k) {
#pragma unroll
            for (int v = 0; v < V; ++v) q[v] = q[v] + eps * (q[v] - (q[v] * q[v]) * q[v]);
        }
    }
}

// ---- column physics with the vertical dependency ----------------------------------
// One update of level z from the level below (already updated in this sweep):
// q + eps*((b*b)*b - (q*q)*q).
__device__ __forceinline__ float vstep(float eps, float q, float b) {
    return q + eps * ((b * b) * b - (q * q) * q);
}
__device__ __forceinline__ double vstep(double eps, double q, double b) {
#pragma clang fp contract(off)
    const double below = (b * b) * b;
    const double here = (q * q) * q;
    return q + eps * (below - here);
}

// k upward sweeps over a column whose nz levels are spread over NQ consecutive
// lanes of one wave (V levels per lane), as a systolic wavefront: at time step
// tau lane j applies sweep tau - j to its levels, taking the level below from
// lane j - 1's result of the previous time step.  Level 0 is the fixed bottom
// boundary.  k + NQ - 1 time steps instead of k * nz.
template <typename T, int V>
__device__ __forceinline__ void physics_vertical(T eps, int k, int tzq, int NQ, T (&q)[V]) {
    T top = q[V - 1];
    const int lane = static_cast<int>(threadIdx.x) & (kWave - 1);
    const int from = tzq == 0 ? lane : lane - 1;    // the lane holding the levels below
    const int steps = k > 0 ? k + NQ - 1 : 0;
    for (int tau = 0; tau < steps; ++tau) {
        const T below = __shfl(top, from, kWave);
        const int sweep = tau - tzq;
        if (sweep >= 0 && sweep < k) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                if (v == 0 && tzq == 0) continue;
                q[v] = vstep(eps, q[v], v == 0 ? below : q[v - 1]);
            }
        }
        top = q[V - 1];
    }
}

// ---- cost field --------------------------------------------------------------
__device__ __forceinline__ int column_k(const DevArgs& a, const int* hcx, const int* hcy, int x,
                                        int y) {
    int k = a.kmin;
#pragma unroll
    for (int h = 0; h < kMaxHot; ++h) {  // fixed trip count keeps hcx/hcy in registers
        if (h < a.nhot) {
            int dx = abs(x - hcx[h]);
            dx = min(dx, a.nx - dx);
            int dy = abs(y - hcy[h]);
            dy = min(dy, a.ny - dy);
            const int r2 = dx * dx + dy * dy;
            k = max(k, a.ktab[min(r2, a.r2cut)]);
        }
    }
    return k;
}

// ---- block reduction in a fixed order (deterministic) -------------------------
__device__ __forceinline__ double wave_sum(double v, int active) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        double other = __shfl_xor(v, o, kWave);
        if ((lane ^ o) < active) v += other;
    }
    return v;
}

// Sum over the block; the result is valid in thread 0.  Uses red[0..nwaves).
__device__ double block_sum(double v, double* red, int bs) {
    const int wave = threadIdx.x / kWave;
    const int nwaves = (bs + kWave - 1) / kWave;
    const int active = min(kWave, bs - wave * kWave);
    v = wave_sum(v, active);
    if ((threadIdx.x & (kWave - 1)) == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < nwaves; ++w) s += red[w];
    __syncthreads();
    return s;
}

// Two sums at once (same fixed order); results valid in thread 0.  Uses red[0..2*nwaves).
__device__ void block_sum2(double& a, double& b, double* red, int bs) {
    const int wave = threadIdx.x / kWave;
    const int nwaves = (bs + kWave - 1) / kWave;
    const int active = min(kWave, bs - wave * kWave);
    a = wave_sum(a, active);
    b = wave_sum(b, active);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        red[wave] = a;
        red[kMaxBlock / kWave + wave] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0;
        for (int w = 0; w < nwaves; ++w) {
            sa += red[w];
            sb += red[kMaxBlock / kWave + w];
        }
        a = sa;
        b = sb;
    }
    __syncthreads();
}

// Three block-wide sums (valid in thread 0); red must hold 3 * kMaxBlock / 64
// doubles of LDS.
__device__ void block_sum3(double& a, double& b, double& c, double* red, int bs) {
    constexpr int kW = kMaxBlock / kWave;
    const int wave = threadIdx.x / kWave;
    const int nwaves = (bs + kWave - 1) / kWave;
    const int active = min(kWave, bs - wave * kWave);
    a = wave_sum(a, active);
    b = wave_sum(b, active);
    c = wave_sum(c, active);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        red[wave] = a;
        red[kW + wave] = b;
        red[2 * kW + wave] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0, sc = 0.0;
        for (int w = 0; w < nwaves; ++w) {
            sa += red[w];
            sb += red[kW + w];
            sc += red[2 * kW + w];
        }
        a = sa;
        b = sb;
        c = sc;
    }
    __syncthreads();
}

// ---- one work item ----------------------------------------------------------------
constexpr int kPipeDma = 1;   // pipeline template value of the direct global->LDS path

// Largest workgroup of a pipeline.  The deeper register pipelines keep 4 or 8
// rows in registers, and FP64 rows take twice the registers; both need more
// than the 128 VGPRs a 1024-thread workgroup allows (the FP64 depth-2 kernel
// spilled at that bound), so they are limited to 512 threads (up to 256 VGPRs).
template <typename T>
constexpr int max_block(int pipe) {
    if (pipe >= 100) return sizeof(T) == 8 ? kMaxBlockDeep : kMaxBlock;   // column march
    return pipe != kPipeDma && (pipe >= 4 || sizeof(T) == 8) ? kMaxBlockDeep : kMaxBlock;
}
struct ItemOut {
    double checksum;  // sum of the item's outputs over all fields (valid in thread 0)
    double work;      // work units of the item (valid in thread 0)
    int chunk;
};

// Result of an item that advances its cells by two steps in one pass.
struct ItemOut2 {
    double checksum1;  // sum of the item's outputs of the first step (thread 0)
    double checksum2;  // ... of the second step
    double work;       // work units of both steps (thread 0)
};

// Result of an item that advances its cells by three steps in one pass.
struct ItemOut3 {
    double checksum[3];  // sums of the item's outputs of each step (thread 0)
    double work;         // work units of the three steps (thread 0)
};

// Four block-wide sums (valid in thread 0); red must hold 4 * kMaxBlock / 64
// doubles of LDS.
__device__ void block_sum4(double (&v)[4], double* red, int bs) {
    constexpr int kW = kMaxBlock / kWave;
    const int wave = threadIdx.x / kWave;
    const int nwaves = (bs + kWave - 1) / kWave;
    const int active = min(kWave, bs - wave * kWave);
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = wave_sum(v[i], active);
    if ((threadIdx.x & (kWave - 1)) == 0)
#pragma unroll
        for (int i = 0; i < 4; ++i) red[i * kW + wave] = v[i];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double t = 0.0;
            for (int w = 0; w < nwaves; ++w) t += red[i * kW + w];
            v[i] = t;
        }
    }
    __syncthreads();
}

struct NoHook {
    __device__ void operator()() const {}
};

using lds_ptr = __attribute__((address_space(3))) unsigned char*;
using glb_ptr = const __attribute__((address_space(1))) unsigned char*;

// One 16-byte direct global->LDS load per active lane (gfx950 global_load_lds
// dwordx4): lane i of the wave writes LDS bytes [wave_base + 16 i, +16).
// wave_base must be the same in every lane of the wave.  The load counts in
// vmcnt like any vector load (see wait_vmem).
__device__ __forceinline__ void dma16(const void* g, lds_ptr wave_base) {
    __builtin_amdgcn_global_load_lds((glb_ptr)g, wave_base, 16, 0, 0);
}

// s_waitcnt vmcnt(0) (gfx9 encoding: expcnt and lgkmcnt fields at their maxima,
// i.e. not waited on).  The compiler does not track direct global->LDS loads,
// and a workgroup barrier's fence does not wait for vector memory on this
// target, so every barrier that publishes such loads is preceded by this.
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// One item; `hook` runs in every thread right after the first prologue barrier
// (the persistent kernel uses it to prefetch the next item's descriptor).
// PIPE = kPipeDma (V = 4 only): rows move HBM -> LDS directly, a.stage_rows
//   rows in flight per workgroup, through a ring of 2*stage_rows + 2 LDS rows.
// PIPE = 2, 4 or 8: rows move HBM -> registers -> LDS with PIPE rows in flight
//   per workgroup (row r + 2 .. r + 1 + PIPE while row r is computed); the
//   compiler's own wait counts order each row's registers before its LDS
//   store, so the pipeline needs no barrier-wide wait for memory.  Every lane
//   issues every row load (lanes without a halo column, and rows past the
//   item's last, read a valid duplicate): a load inside a divergent or
//   row-dependent branch makes the compiler wait for all outstanding loads
//   before the next one, which serialises the pipeline.
// What an item of the direct-load pipeline hands to the next item of its
// workgroup: during its last block it issues the next item's first rows into
// the free part of the ring and looks up the next item's trip counts, so that
// the next item starts with its data in flight or landed.
struct Carry {
    int base;   // ring slot of the next item's row -1
    int pre;    // rows of the next item already issued (rows -1 .. pre - 2); 0 = none
    int kb;     // trip-count buffer (0 or 1) of the next item
};

template <typename T, int V, int KAHAN, int PIPE, typename Hook>
__device__ ItemOut process_item(const DevArgs& a, const ItemDesc& d, const ItemDesc& nx_item,
                                const Carry& cin, Carry& cout, const T* __restrict__ src,
                                T* __restrict__ dst, const int* hcx, const int* hcy, T* lds,
                                double* red, Hook hook) {
    const int nz = a.nz, nx = a.nx, ny = a.ny;
    const int NQ = nz / V;
    const int TX = a.tile_x;
    const int BS = a.block;                   // == blockDim.x, kept in a register
    const int tcol = threadIdx.x / NQ;
    const int tzq = threadIdx.x - tcol * NQ;
    const int zoff = tzq * V;

    const int x0 = d.x0;
    const int y0 = d.y0;
    const int w = d.wh & 0xffff;
    const int h = d.wh >> 16;

    const int RL = (TX + 2) * nz;             // LDS row stride (elements)
    const bool has0 = tcol < w + 2;           // this thread fetches halo column tcol
    const bool has1 = tcol + TX < w + 2;      // ... and column tcol + TX
    const bool active = tcol < w;             // this thread computes column tcol
    int gx0 = x0 - 1 + tcol;
    gx0 = gx0 < 0 ? gx0 + nx : (gx0 >= nx ? gx0 - nx : gx0);
    int gx1 = x0 - 1 + tcol + TX;
    gx1 = gx1 >= nx ? gx1 - nx : gx1;
    // Register-path loads are issued by every lane; a lane without a halo
    // column reads the tile's left halo column instead (and does not store it).
    const int lx0 = has0 ? gx0 : (x0 == 0 ? nx - 1 : x0 - 1);
    const int lx1 = has1 ? gx1 : lx0;
    const T cc = static_cast<T>(a.cc), cn = static_cast<T>(a.cn), eps = static_cast<T>(a.eps);

    constexpr bool kDma = (PIPE == kPipeDma);
    const int RING = kDma ? 2 * a.stage_rows + 2 : kRingRows;
    const int KB = TX * a.tile_y;             // one trip-count buffer
    int* kbuf0 = reinterpret_cast<int*>(lds + RING * RL);
    int* kbuf = kbuf0 + (kDma ? cin.kb * KB : 0);
    const int rbase = kDma ? cin.base : 0;
    auto slot = [&](int i) -> T* {              // LDS row of tile-relative row i >= -1
        return kDma ? lds + ((rbase + i + 1) % RING) * RL : lds + (i & (kRingRows - 1)) * RL;
    };
    // Trip counts of an item's columns, looked up once per item; these table
    // loads are in flight together with row loads.
    auto fill_k_of = [&](const ItemDesc& it, int* kb) {
        const int iw = it.wh & 0xffff, ih = it.wh >> 16;
        for (int i = threadIdx.x; i < iw * ih; i += BS) {
            const int r = i / iw, c = i - r * iw;
            kb[r * TX + c] = column_k(a, hcx, hcy, it.x0 + c, it.y0 + r);
        }
    };
    auto fill_k = [&]() { fill_k_of(d, kbuf); };
    cout.base = 0;
    cout.pre = 0;
    cout.kb = kDma ? cin.kb : 0;

    double chk = 0.0, work = 0.0;
    for (int f = 0; f < a.nfields; ++f) {
        const T* fsrc = src + static_cast<int64_t>(f) * a.ncells;
        T* fdst = dst + static_cast<int64_t>(f) * a.ncells;

        auto fetch = [&](int i, Vec<T, V>& r0, Vec<T, V>& r1) {
            int gy = y0 + i;
            gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
            const T* row = fsrc + static_cast<int64_t>(gy) * nx * nz;
            r0 = ld<T, V>(row + static_cast<int64_t>(lx0) * nz + zoff);
            r1 = ld<T, V>(row + static_cast<int64_t>(lx1) * nz + zoff);
        };
        auto put = [&](int i, const Vec<T, V>& r0, const Vec<T, V>& r1) {
            T* row = slot(i);
            if (has0) st<T, V>(row + tcol * nz + zoff, r0);
            if (has1) st<T, V>(row + (tcol + TX) * nz + zoff, r1);
        };
        auto compute = [&](int r) {
            if (!active) return;
            const int gy = y0 + r;
            const int k = kbuf[r * TX + tcol];
            const T* Lm = slot(r - 1) + (tcol + 1) * nz + zoff;
            const T* Lc = slot(r) + (tcol + 1) * nz + zoff;
            const T* Lp = slot(r + 1) + (tcol + 1) * nz + zoff;
            const Vec<T, V> c = ld<T, V>(Lc);
            const Vec<T, V> xm = ld<T, V>(Lc - nz);
            const Vec<T, V> xp = ld<T, V>(Lc + nz);
            const Vec<T, V> ym = ld<T, V>(Lm);
            const Vec<T, V> yp = ld<T, V>(Lp);
            const T below = Lc[-1];  // neighbouring column's data when tzq == 0
            const T above = Lc[V];   // ... when tzq == NQ - 1 (ignored then)
            const T zlo = (tzq == 0) ? c.v[0] : below;
            const T zhi = (tzq == NQ - 1) ? c.v[V - 1] : above;
            T q[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const T zm = (v == 0) ? zlo : c.v[v - 1];
                const T zp = (v == V - 1) ? zhi : c.v[v + 1];
                T sum = xm.v[v] + xp.v[v];
                sum = sum + ym.v[v];
                sum = sum + yp.v[v];
                sum = sum + zm;
                sum = sum + zp;
                q[v] = combine(cc, cn, c.v[v], sum);
            }
            if (a.vertical)
                physics_vertical<T, V>(eps, k, tzq, NQ, q);
            else
                physics_vec<KAHAN, T, V>(eps, k, q);
            Vec<T, V> out;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                out.v[v] = q[v];
                chk += static_cast<double>(q[v]);
            }
            st<T, V>(fdst + (static_cast<int64_t>(gy) * nx + x0 + tcol) * nz + zoff, out);
            if (tzq == 0) work += static_cast<double>(nz) * static_cast<double>(a.alpha + k);
        };

        if constexpr (!kDma) {
            // Prologue: rows -1, 0, 1 go to the LDS ring; rows 2 .. 1 + PIPE stay in
            // registers, row r in buffer r % PIPE.
            constexpr int D = PIPE;
            Vec<T, V> m0, m1, c0, c1, n0, n1;
            Vec<T, V> R0[D], R1[D];
            fetch(-1, m0, m1);
            fetch(0, c0, c1);
            fetch(1, n0, n1);
#pragma unroll
            for (int j = 0; j < D; ++j) fetch(min(2 + j, h), R0[(2 + j) % D], R1[(2 + j) % D]);
            if (f == 0) fill_k();
            put(-1, m0, m1);
            put(0, c0, c1);
            put(1, n0, n1);
            __syncthreads();
            if (f == 0) hook();

            // Row r: compute r from the ring, move row r + 2 from its registers into
            // the ring (the slot of row r - 2, free since the last barrier) and fetch
            // row r + 2 + D into the same registers.  Unrolled by D so that every
            // register buffer keeps a fixed name.
            for (int r0 = 0; r0 < h; r0 += D) {
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const int r = r0 + j;
                    if (r < h) {
                        const int b = (j + 2) % D;   // == (r + 2) % D: r0 is a multiple of D
                        compute(r);
                        if (r + 2 <= h) put(r + 2, R0[b], R1[b]);
                        fetch(min(r + 2 + D, h), R0[b], R1[b]);
                        __syncthreads();
                    }
                }
            }
        } else {
            // Direct loads: a row of an item is (w+2) columns of nz*sizeof(T)
            // bytes, contiguous in LDS, moved as 16-byte chunks.  Chunk c of the
            // row is loaded by thread c mod blockDim; the lanes of one wave fill
            // 64 consecutive chunks, so the wave's LDS base is uniform.
            const int CPC = nz * static_cast<int>(sizeof(T)) / 16;   // chunks per column
            const int lane = threadIdx.x & (kWave - 1);
            const int wave_first0 = threadIdx.x - lane;
            const lds_ptr lds3 = (lds_ptr)lds;  // address-space cast: lds is LDS
            // row i of item (ix0, iw, iy0) of field fsrc into ring slot s
            auto issue_at = [&](const T* fs, int ix0, int iw, int iy0, int i, int s) {
                const int nchunk = (iw + 2) * CPC;
                int gy = iy0 + i;
                gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
                const unsigned char* row = reinterpret_cast<const unsigned char*>(
                    fs + static_cast<int64_t>(gy) * nx * nz);
                const int slot_byte = s * RL * static_cast<int>(sizeof(T));
                for (int c0 = 0; c0 < nchunk; c0 += BS) {
                    const int first = c0 + wave_first0;     // wave-uniform
                    if (first >= nchunk) break;
                    const int c = c0 + threadIdx.x;
                    const int wbase = __builtin_amdgcn_readfirstlane(slot_byte + first * 16);
                    if (c < nchunk) {
                        const int col = c / CPC, off = c - col * CPC;
                        int gx = ix0 - 1 + col;
                        gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
                        dma16(row + (static_cast<int64_t>(gx) * nz * sizeof(T) + off * 16), lds3 + wbase);
                    }
                }
            };
            auto issue = [&](int i) { issue_at(fsrc, x0, w, y0, i, (rbase + i + 1) % RING); };
            const int B = a.stage_rows;
            const bool last_field = (f == a.nfields - 1);
            // rows -1 .. B, less those the previous item already issued
            for (int i = (f == 0 ? cin.pre - 1 : -1); i <= min(B, h); ++i) issue(i);
            if (f == 0 && cin.pre == 0) fill_k();
            for (int r0 = 0; r0 < h; r0 += B) {
                wait_vmem();            // this thread's loads of rows <= r0 + B have landed
                __syncthreads();        // ... everyone's; and block r0 - B is done
                if (f == 0 && r0 == 0) hook();
                const bool last_block = r0 + B >= h;
                bool ahead = false;
                if (last_block && last_field && nx_item.id >= 0) {
                    // The ring slots this block does not read (at least B of the
                    // 2B + 2) take the next item's first rows, in the ring order the
                    // next item expects: its row -1 right after this item's row h.
                    const int nh = nx_item.wh >> 16;
                    const int nb = (rbase + h + 2) % RING;
                    const int np = min(RING - (h - r0 + 2), min(B, nh) + 2);
                    for (int i = -1; i <= np - 2; ++i)
                        issue_at(src, nx_item.x0, nx_item.wh & 0xffff, nx_item.y0, i, (nb + i + 1) % RING);
                    cout.base = nb;
                    cout.pre = np;
                    cout.kb = cin.kb ^ 1;
                    ahead = true;
                } else {
                    for (int i = r0 + B + 1; i <= min(r0 + 2 * B, h); ++i) issue(i);
                }
                for (int r = r0; r < min(r0 + B, h); ++r) compute(r);
                // after the compute, so that waiting for these table loads does not
                // hold up this block
                if (ahead) fill_k_of(nx_item, kbuf0 + cout.kb * KB);
            }
            __syncthreads();            // the ring rows of this item are free again
        }
    }
    block_sum2(chk, work, red, BS);
    ItemOut o;
    o.checksum = chk;
    o.work = work;
    o.chunk = d.chunk;
    return o;
}

// ---- one work item, column-march pipeline -----------------------------------------
// Template tag of the march pipeline with D rows in flight: kPipeMarch + D.
constexpr int kPipeMarch = 100;

// Raw buffer access to one field: 32-bit byte offsets from the field's base,
// range-checked by the hardware against the field's size.  A lane that must
// not touch memory passes kOutOfRange: its load returns zeros and its store is
// dropped, with no memory traffic, so every lane can issue every load and store
// and the compiler counts outstanding memory operations exactly (no divergent
// branch around them).
using rsrc_t = __amdgpu_buffer_rsrc_t;
// Far enough above every field (fields are limited to 0xFFFFFE00 bytes) that no
// part of a 40-byte access from it wraps round to a valid offset.
constexpr uint32_t kOutOfRange = 0xFFFFFF00u;
constexpr int kRsrcWord3 = 0x00020000;   // gfx9 buffer format word: 32-bit data, no swizzle

__device__ __forceinline__ rsrc_t field_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, static_cast<int>(bytes), kRsrcWord3);
}
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Raw loads and stores of 4, 8 or 16 bytes at byte offset off; group_load and
// group_store cover N bytes with the widest pieces first (so 20 bytes are 16 + 4).
template <int N>
__device__ __forceinline__ void group_load(rsrc_t r, uint32_t off, char* x) {
    if constexpr (N >= 16) {
        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, static_cast<int>(off), 0, 0);
        __builtin_memcpy(x, &v, 16);
        group_load<N - 16>(r, off + 16u, x + 16);
    } else if constexpr (N >= 8) {
        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, static_cast<int>(off), 0, 0);
        __builtin_memcpy(x, &v, 8);
        group_load<N - 8>(r, off + 8u, x + 8);
    } else if constexpr (N >= 4) {
        const unsigned v = __builtin_amdgcn_raw_buffer_load_b32(r, static_cast<int>(off), 0, 0);
        __builtin_memcpy(x, &v, 4);
        group_load<N - 4>(r, off + 4u, x + 4);
    } else {
        static_assert(N == 0, "element groups are whole multiples of 4 bytes");
    }
}
template <int N, int AUX>
__device__ __forceinline__ void group_store(rsrc_t r, uint32_t off, const char* x) {
    if constexpr (N >= 16) {
        u32x4 v;
        __builtin_memcpy(&v, x, 16);
        __builtin_amdgcn_raw_buffer_store_b128(v, r, static_cast<int>(off), 0, AUX);
        group_store<N - 16, AUX>(r, off + 16u, x + 16);
    } else if constexpr (N >= 8) {
        u32x2 v;
        __builtin_memcpy(&v, x, 8);
        __builtin_amdgcn_raw_buffer_store_b64(v, r, static_cast<int>(off), 0, AUX);
        group_store<N - 8, AUX>(r, off + 8u, x + 8);
    } else if constexpr (N >= 4) {
        unsigned v;
        __builtin_memcpy(&v, x, 4);
        __builtin_amdgcn_raw_buffer_store_b32(v, r, static_cast<int>(off), 0, AUX);
        group_store<N - 4, AUX>(r, off + 4u, x + 4);
    } else {
        static_assert(N == 0, "element groups are whole multiples of 4 bytes");
    }
}
template <typename T, int V>
__device__ __forceinline__ Vec<T, V> bload(rsrc_t r, uint32_t off) {
    static_assert(sizeof(T) * V <= 40, "at most 40 bytes per thread and row");
    Vec<T, V> x;
    group_load<static_cast<int>(sizeof(T)) * V>(r, off, reinterpret_cast<char*>(&x));
    return x;
}
// AUX: the store's cache policy; 2 marks it non-temporal (streamed past the
// caches), for output that is not read again before the whole field has gone by.
template <typename T, int V, int AUX>
__device__ __forceinline__ void bstore(rsrc_t r, uint32_t off, const Vec<T, V>& x) {
    group_store<static_cast<int>(sizeof(T)) * V, AUX>(r, off, reinterpret_cast<const char*>(&x));
}

// One cell group of the march: the 7-point update of this thread's V levels
// of the current row (x and z neighbours from the row in LDS at Lc, y
// neighbours ym and yp), then the column physics with k iterations.  PHYS:
// 0 pointwise, 1 vertical, -1 as a.vertical says.
template <typename T, int V, int KAHAN, int PHYS = -1>
__device__ __forceinline__ void cell_update(const DevArgs& a, const T* Lc, const Vec<T, V>& c,
                                            const Vec<T, V>& ym, const Vec<T, V>& yp, int tzq, int NQ,
                                            int nz, int k, T cc, T cn, T eps, T (&q)[V]) {
    const Vec<T, V> xm = ld<T, V>(Lc - nz);
    const Vec<T, V> xp = ld<T, V>(Lc + nz);
    const T below = Lc[-1];   // the column's level zoff - 1 when tzq > 0
    const T above = Lc[V];    // ... zoff + V when tzq < NQ - 1
    const T zlo = (tzq == 0) ? c.v[0] : below;
    const T zhi = (tzq == NQ - 1) ? c.v[V - 1] : above;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const T zm = (v == 0) ? zlo : c.v[v - 1];
        const T zp = (v == V - 1) ? zhi : c.v[v + 1];
        T sum = xm.v[v] + xp.v[v];
        sum = sum + ym.v[v];
        sum = sum + yp.v[v];
        sum = sum + zm;
        sum = sum + zp;
        q[v] = combine(cc, cn, c.v[v], sum);
    }
    if (PHYS == 1 || (PHYS < 0 && a.vertical))
        physics_vertical<T, V>(eps, k, tzq, NQ, q);
    else
        physics_vec<KAHAN, T, V>(eps, k, q);
}

// Thread -> (column tcol, lane tzq of the column) of a march workgroup whose
// thread columns 0 .. TX + 2 HALO - 1 stream grid columns x0 - HALO + tcol.
// Threads are grouped in column slots: dense, NQ consecutive threads per slot;
// with cpw > 0 (the vertical physics when NQ does not divide 64)
// every wave holds cpw whole slots in its first lanes and leaves the
// rest idle, so that a column's lanes never straddle two waves.  Slots 0 ..
// TX - 1 hold the item's own columns, the slots after them the halo columns,
// innermost first, alternating left and right.  The item's columns thus fill
// whole waves, and a wave that holds only halo columns skips the arithmetic
// of the cells it does not compute (a wave issues its vector instructions for
// all of its lanes, idle or not).  Returns whether the lane is used.
template <int HALO>
__device__ __forceinline__ bool march_lane(int cpw, int NQ, int TX, int& tcol, int& tzq) {
    int slot;
    bool used = true;
    if (cpw > 0) {
        const int lane = static_cast<int>(threadIdx.x) & (kWave - 1);
        const int cw = lane / NQ;
        slot = (static_cast<int>(threadIdx.x) >> 6) * cpw + cw;
        tzq = lane - cw * NQ;
        used = cw < cpw;
    } else {
        slot = threadIdx.x / NQ;
        tzq = threadIdx.x - slot * NQ;
    }
    const int h = slot - TX;                  // halo slot: ring h / 2, left when even
    if (h < 0)
        tcol = slot + HALO;
    else if (h < 2 * HALO)
        tcol = (h & 1) ? TX + HALO + (h >> 1) : HALO - 1 - (h >> 1);
    else
        tcol = slot + 2 * HALO;               // past every column: streams nothing
    return used;
}

// v mod n in [0, n) for v within a few multiples of n of the range
__device__ __forceinline__ int wrap_near(int v, int n) {
    while (v < 0) v += n;
    while (v >= n) v -= n;
    return v;
}

// One item with the column-march pipeline.  The workgroup has (TX+2)*NQ
// threads: thread column tcol (0..TX+1) streams grid column x0 - 1 + tcol of
// the item's rows -1 .. h (the item's own w columns and one halo column on
// either side), V levels per thread, and threads 1..w of each row compute.
// Each thread keeps rows y-1, y, y+1 of its column in registers and D more
// rows in flight; only the current row goes through LDS (double-buffered, one
// barrier per row), for the x neighbours and the z neighbours across lanes.
// Every cell is read once per item and written once; the halo columns and the
// two halo rows are re-read by the neighbouring items.
template <typename T, int V, int KAHAN, int D, typename Hook>
__device__ ItemOut process_item_march(const DevArgs& a, const ItemDesc& d, const T* __restrict__ src,
                                      T* __restrict__ dst, const int* hcx, const int* hcy, T* lds,
                                      double* red, Hook hook) {
    const int nz = a.nz, nx = a.nx, ny = a.ny;
    const int NQ = nz / V;
    const int TX = a.tile_x;
    const int BS = a.block;                   // == blockDim.x (at least (TX + 2) columns)
    int tcol, tzq;
    const bool lane_used = march_lane<1>(a.col_per_wave, NQ, TX, tcol, tzq);
    const int zoff = tzq * V;
    const int x0 = d.x0, y0 = d.y0;
    const int w = d.wh & 0xffff;
    const int h = d.wh >> 16;
    const bool streams = lane_used && tcol < w + 2;   // this thread loads grid column x0 - 1 + tcol
    const bool active = lane_used && tcol >= 1 && tcol <= w;
    int gx = x0 - 1 + tcol;
    gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
    const uint32_t rowbytes = static_cast<uint32_t>(nx) * static_cast<uint32_t>(nz) * sizeof(T);
    const uint32_t colbytes = (static_cast<uint32_t>(gx) * nz + zoff) * sizeof(T);
    const T cc = static_cast<T>(a.cc), cn = static_cast<T>(a.cn), eps = static_cast<T>(a.eps);
    const int RL = (TX + 2) * nz;             // LDS row (elements)
    int* kbuf = reinterpret_cast<int*>(lds + 2 * RL);
    // byte offset of row i (-1 .. h) of this thread's column; out of range for
    // threads without a column and for rows past the item's last halo row
    // items clear of the grid's y edges by the halo row need no wrap (uniform per item)
    const bool inner = y0 >= 1 && y0 + h + 1 <= ny;
    const uint32_t base = colbytes + static_cast<uint32_t>(inner ? y0 : 0) * rowbytes;
    auto row_off = [&](int i) -> uint32_t {
        if (!streams || i > h) return kOutOfRange;
        if (inner) return base + static_cast<uint32_t>(i) * rowbytes;
        int gy = y0 + i;
        gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
        return colbytes + static_cast<uint32_t>(gy) * rowbytes;
    };
    // trip counts of the item's columns, looked up once per item; the item's work
    // (k of every column, and the number of columns, each nz * nfields times) is
    // summed here as well
    int flat = 1;                             // every trip count this thread looked up is kmin
    int ksum = 0, kcols = 0;
    for (int i = threadIdx.x; i < w * h; i += BS) {
        const int r = i / w, cx = i - r * w;
        const int k = column_k(a, hcx, hcy, x0 + cx, y0 + r);
        kbuf[r * TX + cx] = k;
        flat &= k == a.kmin;
        ksum += k;
        ++kcols;
    }
    // all of the item's trip counts kmin: the physics loop runs on a scalar count
    // (the reduction also orders the table stores before their reads)
    const bool uniform = __builtin_amdgcn_readfirstlane(__syncthreads_and(flat)) != 0;
    const int ku = a.kmin;
    double chk = 0.0;
    int lpar = 0;                             // LDS buffer of the next row
    // Rows sit in a ring of U = D + 2 register rows, row r (-1 .. h) in slot
    // (r + 1) mod U: rows r - 1, r, r + 1 of the update and D rows in flight.  The
    // row loop is unrolled U times, so every slot is a constant register row and no
    // row is copied between registers; it is compiled once for each trip-count form
    // (uniform or per column) and physics.
    constexpr int U = D + 2;
    auto rows = [&](auto uni_c, auto phys_c) {
        constexpr bool UNI = decltype(uni_c)::value;
        constexpr int PHYS = decltype(phys_c)::value;
        for (int f = 0; f < a.nfields; ++f) {
            const rsrc_t in = field_rsrc(src + static_cast<int64_t>(f) * a.ncells, a.field_bytes);
            const rsrc_t out = field_rsrc(dst + static_cast<int64_t>(f) * a.ncells, a.field_bytes);
            Vec<T, V> R[U];                   // rows -1 .. D to start
#pragma unroll
            for (int j = 0; j < U; ++j) R[j] = bload<T, V>(in, row_off(j - 1));
            // row r: publish row r in the LDS buffer of this row's parity, compute
            // row r, store it, and refill the slot of row r - 1 with row r + 1 + D.
            // The parity runs on across fields, so consecutive rows always use
            // different buffers and one barrier per row suffices.
            for (int r0 = 0; r0 < h; r0 += U) {
#pragma unroll
                for (int j = 0; j < U; ++j) {
                    const int r = r0 + j;
                    if (r < h) {
                        Vec<T, V>& ym = R[j];                 // row r - 1
                        const Vec<T, V>& c = R[(j + 1) % U];  // row r
                        const Vec<T, V>& yp = R[(j + 2) % U]; // row r + 1
                        T* L = lds + lpar * RL;
                        lpar ^= 1;
                        if (streams) st<T, V>(L + tcol * nz + zoff, c);
                        __syncthreads();
                        if (f == 0 && r == 0) hook();
                        Vec<T, V> o;
                        uint32_t so = kOutOfRange;
                        if (active) {
                            T q[V];
                            cell_update<T, V, KAHAN, PHYS>(a, L + tcol * nz + zoff, c, ym, yp, tzq, NQ, nz,
                                                            UNI ? ku : kbuf[r * TX + tcol - 1], cc, cn, eps, q);
#pragma unroll
                            for (int v = 0; v < V; ++v) {
                                o.v[v] = q[v];
                                chk += static_cast<double>(q[v]);
                            }
                            int gy = y0 + r;
                            gy = gy >= ny ? gy - ny : gy;
                            so = colbytes + static_cast<uint32_t>(gy) * rowbytes;
                        }
                        ym = bload<T, V>(in, row_off(r + 1 + D));   // its slot takes row r + 1 + D
                        if (a.stream_store)
                            bstore<T, V, 2>(out, so, o);
                        else
                            bstore<T, V, 0>(out, so, o);
                    }
                }
            }
        }
    };
    using yes = std::true_type;
    using no = std::false_type;
    using pointwise = std::integral_constant<int, 0>;
    using vertical = std::integral_constant<int, 1>;
    if (uniform) {
        if (a.vertical)
            rows(yes{}, vertical{});
        else
            rows(yes{}, pointwise{});
    } else {
        if (a.vertical)
            rows(no{}, vertical{});
        else
            rows(no{}, pointwise{});
    }
    double work = static_cast<double>(nz) * static_cast<double>(a.nfields) *
                  (static_cast<double>(a.alpha) * static_cast<double>(kcols) + static_cast<double>(ksum));
    block_sum2(chk, work, red, BS);
    ItemOut o;
    o.checksum = chk;
    o.work = work;
    o.chunk = d.chunk;
    return o;
}

// Two steps of one item in one pass (temporal blocking): the values of step
// s + 2 on the item's w x h columns from those of step s, with the field read
// once and written once for both steps.  The workgroup has (TX + 4) * NQ
// threads (or whole columns per wave, as in the one-step march): thread
// column tcol streams grid column x0 - 2 + tcol, rows -2 .. h + 1 of the item.
// V is 4 or 5 levels per thread (NQ = nz / V threads per column): 5 where
// nz / 4 threads would leave a column's lanes straddling waves, e.g. nz = 80
// gives 16 threads per column and whole waves of columns.
// Threads 1 .. w + 2 compute step s + 1 on the columns -1 .. w and rows
// -1 .. h (the item and the ring of cells around it that the item's next
// update reads); threads 2 .. w + 1 compute step s + 2 on the item's own cells
// one row behind.  Each update is the same arithmetic as in the one-step
// march, so the fused steps give the same bits as two launches of one step.
// The ring's step s + 1 values are computed again by the neighbouring items;
// only the item's own cells count in the checksum and the work of each step.
// Both rows of a step go through LDS (step s values for step s + 1, step s + 1
// values for step s + 2), double-buffered, with one barrier per row.  hc1 are
// the hotspot centres of step s, hc2 those of step s + 1.
template <typename T, int V, int KAHAN, int D>
__device__ ItemOut2 process_item_march2(const DevArgs& a, const ItemDesc& d, const T* __restrict__ src,
                                        T* __restrict__ dst, const int* hc1x, const int* hc1y,
                                        const int* hc2x, const int* hc2y, T* lds, double* red) {
    const int nz = a.nz, nx = a.nx, ny = a.ny;
    const int NQ = nz / V;
    const int TX = a.tile_x;
    const int BS = a.block2;                  // == blockDim.x (at least (TX + 4) columns)
    int tcol, tzq;
    const bool lane_used = march_lane<2>(a.col_per_wave2, NQ, TX, tcol, tzq);
    const int zoff = tzq * V;
    const int x0 = d.x0, y0 = d.y0;
    const int w = d.wh & 0xffff;
    const int h = d.wh >> 16;
    const bool streams = lane_used && tcol < w + 4;                // loads grid column x0 - 2 + tcol
    const bool act1 = lane_used && tcol >= 1 && tcol <= w + 2;      // step s + 1 on column tcol - 2
    const bool act2 = lane_used && tcol >= 2 && tcol <= w + 1;      // step s + 2 on column tcol - 2
    const int gx = streams ? wrap_near(x0 - 2 + tcol, nx) : 0;
    const uint32_t rowbytes = static_cast<uint32_t>(nx) * static_cast<uint32_t>(nz) * sizeof(T);
    const uint32_t colbytes = (static_cast<uint32_t>(gx) * nz + zoff) * sizeof(T);
    const T cc = static_cast<T>(a.cc), cn = static_cast<T>(a.cn), eps = static_cast<T>(a.eps);
    const int RL = (TX + 4) * nz;             // LDS row (elements); buffers: 2 of step s, 2 of s + 1
    const int K1 = TX + 2;                    // row stride of the step s + 1 trip counts
    int* kb1 = reinterpret_cast<int*>(lds + 4 * RL);
    int* kb2 = kb1 + K1 * (a.tile_y + 2);
    // byte offset of row i (-2 .. h + 1) of this thread's column; out of range for
    // threads without a column and past the last row the item reads
    // items clear of the grid's y edges by the halo need no wrap (uniform per item)
    const bool inner = y0 >= 2 && y0 + h + 2 <= ny;
    const uint32_t base = colbytes + static_cast<uint32_t>(inner ? y0 : 0) * rowbytes;
    auto row_off = [&](int i) -> uint32_t {
        if (!streams || i > h + 1) return kOutOfRange;
        if (inner) return base + static_cast<uint32_t>(i) * rowbytes;
        return colbytes + static_cast<uint32_t>(wrap_near(y0 + i, ny)) * rowbytes;
    };
    // Trip counts of both steps, looked up once per item.  The item's work (its own
    // columns in both steps) is summed here as well: k of every own column, and
    // the number of own columns, each taken nz * nfields times.
    int flat = 1;                             // every trip count this thread looked up is kmin
    int ksum = 0, kcols = 0;
    for (int i = threadIdx.x; i < (w + 2) * (h + 2); i += BS) {
        const int r = i / (w + 2), cx = i - r * (w + 2);
        const int k = column_k(a, hc1x, hc1y, wrap_near(x0 - 1 + cx, nx), wrap_near(y0 - 1 + r, ny));
        kb1[r * K1 + cx] = k;
        flat &= k == a.kmin;
        if (r >= 1 && r <= h && cx >= 1 && cx <= w) {
            ksum += k;
            ++kcols;
        }
    }
    for (int i = threadIdx.x; i < w * h; i += BS) {
        const int r = i / w, cx = i - r * w;
        const int k = column_k(a, hc2x, hc2y, x0 + cx, y0 + r);
        kb2[r * TX + cx] = k;
        flat &= k == a.kmin;
        ksum += k;
        ++kcols;
    }
    // When every trip count of the item (both steps, ring included) is kmin, the
    // physics takes kmin as a workgroup-uniform scalar: a loop without per-lane
    // control.  (The reduction also orders the table stores before their reads.)
    const bool uniform = __builtin_amdgcn_readfirstlane(__syncthreads_and(flat)) != 0;
    const int ku = a.kmin;
    T* const lrow = lds + tcol * nz + zoff;   // this thread's V levels in LDS row buffer 0
    int par = 0;                              // LDS buffers of the next row (the parity runs on
                                              // across fields: consecutive rows never share one)
    double chk1 = 0.0, chk2 = 0.0;
    const int n_it = h + 2;                   // iteration n computes step s + 1 on row n - 1
    // Rows of step s sit in a ring of U = D + 2 register rows, row r in slot
    // (r + 2) mod U: rows r - 1, r, r + 1 of the update and D rows in flight.  Rows
    // of step s + 1 sit in a ring of P1 rows (the smallest divisor of U of at least
    // 3), row r in slot (r + 1) mod P1.  The row loop is unrolled U times, so every
    // slot is a constant register row and no row is ever copied between registers;
    // it is compiled once for each trip-count form (uniform or per column) and
    // physics, so no branch of the body merges values from another.
    constexpr int U = D + 2;
    constexpr int P1 = (U % 3 == 0) ? 3 : (U % 4 == 0) ? 4 : (U % 5 == 0) ? 5 : U;
    auto rows = [&](auto uni_c, auto phys_c) {
        constexpr bool UNI = decltype(uni_c)::value;
        constexpr int PHYS = decltype(phys_c)::value;
        for (int f = 0; f < a.nfields; ++f) {
            const rsrc_t in = field_rsrc(src + static_cast<int64_t>(f) * a.ncells, a.field_bytes);
            const rsrc_t out = field_rsrc(dst + static_cast<int64_t>(f) * a.ncells, a.field_bytes);
            Vec<T, V> R[U];                   // step s rows -2 .. D - 1 to start
#pragma unroll
            for (int j = 0; j < U; ++j) R[j] = bload<T, V>(in, row_off(j - 2));
            Vec<T, V> S[P1];                  // step s + 1 rows
#pragma unroll
            for (int j = 0; j < P1; ++j)
#pragma unroll
                for (int v = 0; v < V; ++v) S[j].v[v] = T(0);
            for (int n0 = 0; n0 < n_it; n0 += U) {
#pragma unroll
                for (int j = 0; j < U; ++j) {
                    const int n = n0 + j;
                    if (n < n_it) {
                        const int i = n - 1;
                        Vec<T, V>& ym = R[j];                 // step s row n - 2
                        const Vec<T, V>& c = R[(j + 1) % U];  // row n - 1
                        const Vec<T, V>& yp = R[(j + 2) % U]; // row n
                        Vec<T, V>& s1n = S[j % P1];           // step s + 1 row n - 1 (computed here)
                        const Vec<T, V>& s1c = S[(j + P1 - 1) % P1];   // row n - 2
                        const Vec<T, V>& s1m = S[(j + P1 - 2) % P1];   // row n - 3
                        T* const LA = lrow + par * RL;         // step s, row i
                        T* const LB = lrow + (2 + par) * RL;   // step s + 1, row i - 1
                        par ^= 1;
                        if (streams) st<T, V>(LA, c);
                        if (act1) st<T, V>(LB, s1c);
                        __syncthreads();
                        if (act1) {
                            T q[V];
                            cell_update<T, V, KAHAN, PHYS>(a, LA, c, ym, yp, tzq, NQ, nz,
                                                            UNI ? ku : kb1[n * K1 + tcol - 1], cc, cn, eps, q);
#pragma unroll
                            for (int v = 0; v < V; ++v) s1n.v[v] = q[v];
                        }
                        ym = bload<T, V>(in, row_off(n + D));  // its slot takes row n + D
                        if (i >= 1) {                     // step s + 2 on row i - 1
                            Vec<T, V> o;
                            uint32_t so = kOutOfRange;
                            if (act2) {
                                T q[V];
                                cell_update<T, V, KAHAN, PHYS>(a, LB, s1c, s1m, s1n, tzq, NQ, nz,
                                                                UNI ? ku : kb2[(i - 1) * TX + tcol - 2], cc, cn,
                                                                eps, q);
                                // the item's own cells: step s + 1 (row i - 1, as read here), step s + 2
#pragma unroll
                                for (int v = 0; v < V; ++v) {
                                    o.v[v] = q[v];
                                    chk1 += static_cast<double>(s1c.v[v]);
                                    chk2 += static_cast<double>(q[v]);
                                }
                                so = colbytes + static_cast<uint32_t>(y0 + i - 1) * rowbytes;
                            }
                            if (a.stream_store)
                                bstore<T, V, 2>(out, so, o);
                            else
                                bstore<T, V, 0>(out, so, o);
                        }
                    }
                }
            }
        }
    };
    using yes = std::true_type;
    using no = std::false_type;
    using pointwise = std::integral_constant<int, 0>;
    using vertical = std::integral_constant<int, 1>;
    if (uniform) {
        if (a.vertical)
            rows(yes{}, vertical{});
        else
            rows(yes{}, pointwise{});
    } else {
        if (a.vertical)
            rows(no{}, vertical{});
        else
            rows(no{}, pointwise{});
    }
    double work = static_cast<double>(nz) * static_cast<double>(a.nfields) *
                  (static_cast<double>(a.alpha) * static_cast<double>(kcols) + static_cast<double>(ksum));
    block_sum3(chk1, chk2, work, red, BS);
    ItemOut2 o;
    o.checksum1 = chk1;
    o.checksum2 = chk2;
    o.work = work;
    return o;
}

// Three steps of one item in one pass: the two-step march above with one more
// stage.  The workgroup streams grid columns x0 - 3 .. x0 + w + 2, rows -3 ..
// h + 2 of the item (thread column tcol holds grid column x0 - 3 + tcol);
// stage 1 computes step s + 1 on columns -2 .. w + 1 and rows -2 .. h + 1,
// stage 2 step s + 2 on columns -1 .. w and rows -1 .. h one row behind, and
// stage 3 step s + 3 on the item's own cells one row further behind.  Each
// stage's current row goes through LDS (double-buffered) for the next stage's
// x and z neighbours, one barrier per row; the same arithmetic as one step
// per launch, so the same bits.  Only the item's own cells count in each
// step's checksum and work.  hc1, hc2, hc3: hotspot centres of steps s, s + 1
// and s + 2.
template <typename T, int V, int KAHAN, int D>
__device__ ItemOut3 process_item_march3(const DevArgs& a, const ItemDesc& d, const T* __restrict__ src,
                                        T* __restrict__ dst, const int* hc1x, const int* hc1y,
                                        const int* hc2x, const int* hc2y, const int* hc3x, const int* hc3y,
                                        T* lds, double* red) {
    const int nz = a.nz, nx = a.nx, ny = a.ny;
    const int NQ = nz / V;
    const int TX = a.tile_x;
    const int BS = a.block3;                  // == blockDim.x (at least (TX + 6) columns)
    int tcol, tzq;
    const bool lane_used = march_lane<3>(a.col_per_wave, NQ, TX, tcol, tzq);
    const int zoff = tzq * V;
    const int x0 = d.x0, y0 = d.y0;
    const int w = d.wh & 0xffff;
    const int h = d.wh >> 16;
    const bool streams = lane_used && tcol < w + 6;                // loads grid column x0 - 3 + tcol
    const bool act1 = lane_used && tcol >= 1 && tcol <= w + 4;      // step s + 1 on column tcol - 3
    const bool act2 = lane_used && tcol >= 2 && tcol <= w + 3;      // step s + 2
    const bool act3 = lane_used && tcol >= 3 && tcol <= w + 2;      // step s + 3 (the item's columns)
    const int gx = streams ? wrap_near(x0 - 3 + tcol, nx) : 0;
    const uint32_t rowbytes = static_cast<uint32_t>(nx) * static_cast<uint32_t>(nz) * sizeof(T);
    const uint32_t colbytes = (static_cast<uint32_t>(gx) * nz + zoff) * sizeof(T);
    const T cc = static_cast<T>(a.cc), cn = static_cast<T>(a.cn), eps = static_cast<T>(a.eps);
    const int RL = (TX + 6) * nz;             // LDS row (elements); 2 buffers for each of 3 stages
    const int K1 = TX + 4, K2 = TX + 2;       // row strides of the stage 1 and 2 trip counts
    int* kb1 = reinterpret_cast<int*>(lds + 6 * RL);
    int* kb2 = kb1 + K1 * (a.tile_y + 4);
    int* kb3 = kb2 + K2 * (a.tile_y + 2);
    // byte offset of row i (-3 .. h + 2) of this thread's column; out of range for
    // threads without a column and past the last row the item reads
    // items clear of the grid's y edges by the halo need no wrap (uniform per item)
    const bool inner = y0 >= 3 && y0 + h + 3 <= ny;
    const uint32_t base = colbytes + static_cast<uint32_t>(inner ? y0 : 0) * rowbytes;
    auto row_off = [&](int i) -> uint32_t {
        if (!streams || i > h + 2) return kOutOfRange;
        if (inner) return base + static_cast<uint32_t>(i) * rowbytes;
        return colbytes + static_cast<uint32_t>(wrap_near(y0 + i, ny)) * rowbytes;
    };
    // trip counts of the three steps; the item's work (its own columns in each
    // step) is summed here as well
    int flat = 1;
    int ksum = 0, kcols = 0;
    for (int i = threadIdx.x; i < (w + 4) * (h + 4); i += BS) {
        const int r = i / (w + 4), cx = i - r * (w + 4);
        const int k = column_k(a, hc1x, hc1y, wrap_near(x0 - 2 + cx, nx), wrap_near(y0 - 2 + r, ny));
        kb1[r * K1 + cx] = k;
        flat &= k == a.kmin;
        if (r >= 2 && r <= h + 1 && cx >= 2 && cx <= w + 1) {
            ksum += k;
            ++kcols;
        }
    }
    for (int i = threadIdx.x; i < (w + 2) * (h + 2); i += BS) {
        const int r = i / (w + 2), cx = i - r * (w + 2);
        const int k = column_k(a, hc2x, hc2y, wrap_near(x0 - 1 + cx, nx), wrap_near(y0 - 1 + r, ny));
        kb2[r * K2 + cx] = k;
        flat &= k == a.kmin;
        if (r >= 1 && r <= h && cx >= 1 && cx <= w) {
            ksum += k;
            ++kcols;
        }
    }
    for (int i = threadIdx.x; i < w * h; i += BS) {
        const int r = i / w, cx = i - r * w;
        const int k = column_k(a, hc3x, hc3y, x0 + cx, y0 + r);
        kb3[r * TX + cx] = k;
        flat &= k == a.kmin;
        ksum += k;
        ++kcols;
    }
    // all trip counts kmin: the physics runs on a scalar count (the reduction also
    // orders the table stores before their reads)
    const bool uniform = __builtin_amdgcn_readfirstlane(__syncthreads_and(flat)) != 0;
    const int ku = a.kmin;
    T* const lrow = lds + tcol * nz + zoff;   // this thread's V levels in LDS row buffer 0
    int par = 0;                              // LDS buffers of the next row (runs on across fields)
    double chk[3] = {0.0, 0.0, 0.0};
    const int n_it = h + 4;                   // iteration n: stage 1 on row n - 2, 2 on n - 3, 3 on n - 4
    for (int f = 0; f < a.nfields; ++f) {
        const rsrc_t in = field_rsrc(src + static_cast<int64_t>(f) * a.ncells, a.field_bytes);
        const rsrc_t out = field_rsrc(dst + static_cast<int64_t>(f) * a.ncells, a.field_bytes);
        Vec<T, V> ym = bload<T, V>(in, row_off(-3));   // step s rows n - 3, n - 2, then n - 1 ..
        Vec<T, V> c = bload<T, V>(in, row_off(-2));
        Vec<T, V> R[D];
#pragma unroll
        for (int j = 0; j < D; ++j) R[j] = bload<T, V>(in, row_off(j - 1));
        Vec<T, V> s1m{}, s1c{}, s2m{}, s2c{};   // stage 1 rows n - 4, n - 3; stage 2 rows n - 5, n - 4
        for (int n0 = 0; n0 < n_it; n0 += D) {
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const int n = n0 + j;
                if (n < n_it) {
                    T* const LA = lrow + par * RL;         // step s, row n - 2
                    T* const LB = lrow + (2 + par) * RL;   // stage 1, row n - 3
                    T* const LC = lrow + (4 + par) * RL;   // stage 2, row n - 4
                    par ^= 1;
                    if (streams) st<T, V>(LA, c);
                    if (act1) st<T, V>(LB, s1c);
                    if (act2) st<T, V>(LC, s2c);
                    __syncthreads();
                    const Vec<T, V> yp = R[j];
                    R[j] = bload<T, V>(in, row_off(n - 1 + D));
                    Vec<T, V> s1n, s2n;               // (used only where their stage sets them)
                    if (act1) {                       // stage 1, row n - 2
                        T q[V];
                        if (uniform)
                            cell_update<T, V, KAHAN>(a, LA, c, ym, yp, tzq, NQ, nz, ku, cc, cn, eps, q);
                        else
                            cell_update<T, V, KAHAN>(a, LA, c, ym, yp, tzq, NQ, nz, kb1[n * K1 + tcol - 1], cc,
                                                     cn, eps, q);
#pragma unroll
                        for (int v = 0; v < V; ++v) s1n.v[v] = q[v];
                    }
                    if (n >= 2 && act2) {             // stage 2, row n - 3
                        T q[V];
                        if (uniform)
                            cell_update<T, V, KAHAN>(a, LB, s1c, s1m, s1n, tzq, NQ, nz, ku, cc, cn, eps, q);
                        else
                            cell_update<T, V, KAHAN>(a, LB, s1c, s1m, s1n, tzq, NQ, nz,
                                                     kb2[(n - 2) * K2 + tcol - 2], cc, cn, eps, q);
#pragma unroll
                        for (int v = 0; v < V; ++v) s2n.v[v] = q[v];
                    }
                    if (n >= 4) {                     // stage 3, row n - 4
                        Vec<T, V> o;
                        uint32_t so = kOutOfRange;
                        if (act3) {
                            T q[V];
                            if (uniform)
                                cell_update<T, V, KAHAN>(a, LC, s2c, s2m, s2n, tzq, NQ, nz, ku, cc, cn, eps, q);
                            else
                                cell_update<T, V, KAHAN>(a, LC, s2c, s2m, s2n, tzq, NQ, nz,
                                                         kb3[(n - 4) * TX + tcol - 3], cc, cn, eps, q);
                            // the item's own cells of row n - 4 in each step
#pragma unroll
                            for (int v = 0; v < V; ++v) {
                                o.v[v] = q[v];
                                chk[0] += static_cast<double>(s1m.v[v]);
                                chk[1] += static_cast<double>(s2c.v[v]);
                                chk[2] += static_cast<double>(q[v]);
                            }
                            so = colbytes + static_cast<uint32_t>(y0 + n - 4) * rowbytes;
                        }
                        if (a.stream_store)
                            bstore<T, V, 2>(out, so, o);
                        else
                            bstore<T, V, 0>(out, so, o);
                    }
                    ym = c;
                    c = yp;
                    s1m = s1c;
                    s1c = s1n;
                    s2m = s2c;
                    s2c = s2n;
                }
            }
        }
    }
    double sums[4] = {chk[0], chk[1], chk[2],
                      static_cast<double>(nz) * static_cast<double>(a.nfields) *
                          (static_cast<double>(a.alpha) * static_cast<double>(kcols) + static_cast<double>(ksum))};
    block_sum4(sums, red, BS);
    ItemOut3 o;
    o.checksum[0] = sums[0];
    o.checksum[1] = sums[1];
    o.checksum[2] = sums[2];
    o.work = sums[3];
    return o;
}

// ---- step context --------------------------------------------------------------
struct StepInfo {
    uint64_t step;
    int hcx[kMaxHot], hcy[kMaxHot];
};

__device__ __forceinline__ StepInfo step_info(const WgState& w) {
    StepInfo s;
    s.step = w.step;
#pragma unroll
    for (int h = 0; h < kMaxHot; ++h) {
        s.hcx[h] = w.hx[h];
        s.hcy[h] = w.hy[h];
    }
    return s;
}

// The state of the step after `w`: each hotspot moves by its velocity, wrapped.
__device__ __forceinline__ WgState next_state(const DevArgs& a, const WgState& w) {
    WgState n;
    n.step = w.step + 1;
    n.cur = w.cur ^ 1;
#pragma unroll
    for (int h = 0; h < kMaxHot; ++h) {
        int x = w.hx[h] + a.hvx[h], y = w.hy[h] + a.hvy[h];
        n.hx[h] = x >= a.nx ? x - a.nx : x;
        n.hy[h] = y >= a.ny ? y - a.ny : y;
    }
    return n;
}

// Called by every thread after an item.  Thread 0 writes the item's checksum
// partial, adds its work and ticks to the chunk's loads and its work to the
// tile's (from which the host cuts the next plan's items); the tile rows the
// item covered each get one visit, one thread per row.  None of these waits
// for a reply (stores and non-returning atomics), so an item's bookkeeping
// costs no memory latency.  Exactly one workgroup owns a row in a step, so a
// second claim or a missed row shows as a wrong visit count.
__device__ __forceinline__ void record_item(const DevArgs& a, double* partials, const ItemDesc& d,
                                            const ItemOut& o, double ticks) {
    if (threadIdx.x == 0) {
        partials[d.id] = o.checksum;
        unsafeAtomicAdd(&a.loads_work[d.chunk], o.work);
        unsafeAtomicAdd(&a.loads_time[d.chunk], ticks);
        unsafeAtomicAdd(&a.tile_work[d.tile], o.work);
    }
    for (int r = threadIdx.x; r < (d.wh >> 16); r += a.block)
        __hip_atomic_fetch_add(&a.visits[d.vbase + r], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Deterministic sum of n checksum partials, valid in every thread.  The shape is
// fixed whatever the block size: accumulator v (0..255) adds partials v,
// v + 256, v + 512, ... in that order, then the 256 accumulators are added as a
// pairwise tree (v + 128, then v + 64, ...), so every kernel that sums a step's
// partials gets the same bits.  acc must hold kSumThreads doubles of LDS.
// Loads go out 16 at a time so that one memory latency covers a batch.
constexpr int kSumThreads = 256;
constexpr int kRedLen = kSumThreads;  // LDS doubles for block sums and partial sums
static_assert(kRedLen >= 4 * kMaxBlock / 64, "block_sum2..4 need up to four entries per wave");
__device__ double sum_partials(const double* part, int n, double* acc, int bs) {
    constexpr int kBatch = 16;
    for (int v = threadIdx.x; v < kSumThreads; v += bs) {
        double s = 0.0;
        for (int i0 = 0; i0 < n; i0 += kBatch * kSumThreads) {
            double x[kBatch];
#pragma unroll
            for (int j = 0; j < kBatch; ++j) {
                const int i = i0 + j * kSumThreads + v;
                x[j] = i < n ? part[i] : 0.0;
            }
#pragma unroll
            for (int j = 0; j < kBatch; ++j) s += x[j];
        }
        acc[v] = s;
    }
    __syncthreads();
    for (int h = kSumThreads / 2; h > 0; h >>= 1) {
        for (int v = threadIdx.x; v < h; v += bs) acc[v] = acc[v] + acc[v + h];
        __syncthreads();
    }
    const double total = acc[0];
    __syncthreads();                  // acc may be reused at once
    return total;
}

// If partials buffer p holds a step whose sum is still pending, sum it into the
// checksum ring and mark it done.  Run by one whole workgroup, with no other
// workgroup touching buffer p.
__device__ void settle_partials(const DevArgs& a, int p, double* red, int bs) {
    const uint64_t ps = a.ctrl->pend_step[p];     // the same value in every thread
    if (ps == 0) return;
    const int n = static_cast<int>(a.ctrl->pend_n[p]);
    const double total = sum_partials(a.partials + static_cast<int64_t>(p) * a.part_stride, n, red, bs);
    if (threadIdx.x == 0) {
        a.hist[(ps - 1) % kHistLen] = total;
        a.ctrl->pend_step[p] = 0;
    }
}

// Sum every pending partials buffer other than those in `mine` (bit b: buffer
// b), which the calling launch writes.  Run by one whole workgroup.
__device__ void settle_others(const DevArgs& a, unsigned mine, double* red, int bs) {
    for (int b = 0; b < kStepSlots; ++b)
        if (!((mine >> b) & 1u)) settle_partials(a, b, red, bs);
}

// ---- claiming work ----------------------------------------------------------------
// Workgroups are dispatched to the eight XCDs round-robin (workgroup w runs on
// XCD w % 8).  When Q is a multiple of 8, queue q is served only by workgroups
// on XCD q % 8, so the items of a chunk share that XCD's L2.  Every queue has
// exactly G workgroups, with ranks 0..G-1 (rank (w >> 3) / (Q / 8), else w / Q);
// the host uses the same assignment to precompute each workgroup's first item.
__device__ __forceinline__ int home_queue(const DevArgs& a, int wg) {
    if (a.xcd_queues) {
        const int per_xcd = a.nqueues / 8;
        return (wg & 7) + 8 * ((wg >> 3) % per_xcd);
    }
    return wg % a.nqueues;
}

// Index (into the queue array) of a claimed item of queue q, or -1 if it is empty.
__device__ __forceinline__ int try_claim(const DevArgs& a, int* heads, int q) {
    const int beg = a.seg[q];
    const int n = a.seg[q + 1] - beg;
    if (__hip_atomic_load(&heads[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= n) return -1;
    const int i = atomicAdd(&heads[q], 1);
    return i < n ? beg + i : -1;
}

// Called by all lanes of wave 0.  Home queue first; then, if stealing is on,
// scan the other queues 64 at a time (same-XCD queues first) and claim from
// the one with the most work left among the first 64 with any.  Every failed
// claim means that queue is empty for good (heads only grow), so the scan
// ends after at most Q failures.
__device__ int claim(const DevArgs& a, int* heads, int home) {
    const int lane = threadIdx.x & (kWave - 1);
    int qi = -1;
    if (lane == 0) qi = try_claim(a, heads, home);
    qi = __shfl(qi, 0, kWave);
    if (qi >= 0 || !a.steal) return qi;
    const int Q = a.nqueues;
    const int per_xcd = a.xcd_queues ? Q / 8 : Q;
    int base = 0;
    while (base < Q) {
        const int j = base + lane;
        int q = -1, rem = 0;
        if (j < Q && lane < a.block) {
            q = a.xcd_queues ? (home + 8 * (j % per_xcd) + j / per_xcd) % Q : (home + j) % Q;
            rem = (a.seg[q + 1] - a.seg[q]) -
                  __hip_atomic_load(&heads[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (__ballot(rem > 0) == 0) {
            base += kWave;
            continue;
        }
        // the lane with the most remaining work (lowest lane on ties) picks the victim
        int best = rem, who = lane;
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) {
            const int ob = __shfl_xor(best, o, kWave);
            const int ow = __shfl_xor(who, o, kWave);
            if (ob > best || (ob == best && ow < who)) {
                best = ob;
                who = ow;
            }
        }
        const int victim = __shfl(q, who, kWave);
        int got = -1;
        if (lane == 0) got = try_claim(a, heads, victim);
        got = __shfl(got, 0, kWave);
        if (got >= 0) return got;
    }
    return -1;
}

__device__ __forceinline__ ItemDesc no_item() {
    ItemDesc d{};
    d.id = -1;
    return d;
}

// ---- kernels ----------------------------------------------------------------------
// One launch per step.  The first two rounds of every queue are assigned
// statically: workgroup (queue q, rank j) starts with item j of its queue and
// goes on with item 2G - 1 - j (the largest first items pair with the smallest
// second ones, as a longest-first schedule of two rounds would); both
// descriptors are precomputed, so the step starts with no atomic and no
// dependent load.  After that, claims run two items ahead: at the start of
// every item a workgroup claims one more item of its queue, so that during an
// item it always knows the item after it and the direct-load pipeline can
// issue that item's first rows from the current item's last block.  Once its
// queue is drained a workgroup claims through `claim` (stealing), one item at
// a time.  A step needs no
// end-of-launch work: the step number is kept per workgroup, the claim
// counters alternate between two sets by step parity (workgroup 0 resets the
// set of the next step), and the checksum partials of the step are summed by
// the last workgroup of the next step (or by k_flush), so workgroups simply
// exit and the launch boundary orders one step before the next.
template <typename T, int V, int KAHAN, int PIPE>
__global__ __launch_bounds__(max_block<T>(PIPE)) void k_persistent(DevArgs a) {
    extern __shared__ __align__(32) unsigned char smem[];
    T* lds = reinterpret_cast<T*>(smem);
    __shared__ double red[kRedLen];
    __shared__ ItemDesc s_cur, s_nxt;

    const uint64_t t_launch = wall_clock64();
    const int wg = blockIdx.x;
    const WgState ws = a.wstate[wg];            // equal in every workgroup of the launch
    const uint64_t step = ws.step;
    const int par = static_cast<int>(step & 1);  // claim-counter set
    const int b = static_cast<int>(step & kSlotMask);    // partials buffer and state slot
    const StepInfo si = step_info(ws);
    const T* src = static_cast<const T*>(ws.cur ? a.field1 : a.field0);
    T* dst = static_cast<T*>(ws.cur ? a.field0 : a.field1);
    int* heads = a.heads + par * a.nqueues;
    double* partials = a.partials + static_cast<int64_t>(b) * a.part_stride;
    const int home = home_queue(a, wg);
    const int hbeg = a.seg[home];
    const int hn = a.seg[home + 1] - hbeg;
    double busy = 0.0;

    uint64_t t_first = 0, t_last = 0;
    if (threadIdx.x == 0) {
        s_cur = a.firstd[2 * wg];
        s_nxt = a.firstd[2 * wg + 1];
    }
    if (wg == 0) {
        // the previous step, which used the other set, has ended; the next one uses it
        int* other = a.heads + (par ^ 1) * a.nqueues;
        for (int q = threadIdx.x; q < a.nqueues; q += a.block) other[q] = a.head0;
        if (threadIdx.x == 0) {
            a.ctrl->pend_n[b] = a.ctrl->nitems;
            a.ctrl->pend_step[b] = step + 1;
            a.pstate[(b + 1) & kSlotMask] = next_state(a, ws);
        }
    }
    if (wg == a.nwg - 1) settle_others(a, 1u << b, red, a.block);   // earlier steps' sums
    __syncthreads();
    Carry carry{0, 0, 0};
    bool drained = false;    // (thread 0) the home queue has nothing left to claim
    for (;;) {
        ItemDesc d = s_cur;
        ItemDesc nx = s_nxt;
        if (d.id < 0) {                      // nothing claimed ahead: claim with stealing
            __syncthreads();
            if (threadIdx.x < kWave) {
                const int qi = claim(a, heads, home);
                if (threadIdx.x == 0) s_cur = qi >= 0 ? a.queue[qi] : no_item();
            }
            __syncthreads();
            d = s_cur;
            nx = no_item();
            carry.pre = 0;
            drained = true;
            if (d.id < 0) break;
        }
        __syncthreads();                     // every thread holds d and nx before they change
        // claim one more item; its index is first used after the item's first
        // barrier, whose wait covers the atomic anyway
        int nidx = hn;
        if (threadIdx.x == 0 && !drained) nidx = atomicAdd(&heads[home], 1);
        ItemDesc na = no_item();
        auto ahead = [&]() {
            if (threadIdx.x == 0) {
                if (nidx < hn) na = a.queue[hbeg + nidx];
                drained = nidx + 1 >= hn;
            }
        };
        const uint64_t t_start = wall_clock64();
        if (t_first == 0) t_first = t_start;
        Carry next;
        const ItemOut o = process_item<T, V, KAHAN, PIPE>(a, d, nx, carry, next, src, dst, si.hcx, si.hcy,
                                                          lds, red, ahead);
        t_last = wall_clock64();
        const double ticks = static_cast<double>(t_last - t_start);  // used by thread 0
        record_item(a, partials, d, o, ticks);
        if (threadIdx.x == 0) {
            busy += ticks;
            s_cur = nx;
            s_nxt = na;
        }
        carry = next;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        unsafeAtomicAdd(&a.wg_busy[wg], busy);
        uint64_t* tl = a.wg_timeline + 4 * static_cast<size_t>(wg);
        tl[0] = t_launch;
        tl[1] = t_first ? t_first : t_launch;
        tl[2] = t_last ? t_last : t_launch;
        tl[3] = wall_clock64();
        a.wstate[wg] = next_state(a, ws);
    }
}

// Wave-uniform copies (scalar registers) of values every lane holds the same.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ ItemDesc uni(const ItemDesc& d) {
    ItemDesc u;
    u.x0 = uni(d.x0);
    u.y0 = uni(d.y0);
    u.wh = uni(d.wh);
    u.chunk = uni(d.chunk);
    u.id = uni(d.id);
    u.vbase = uni(d.vbase);
    u.tile = uni(d.tile);
    u.pad1 = 0;
    return u;
}

// The persistent launch with the column-march item body.  Same queues, static
// start, claims and stealing as k_persistent, arranged so that little state
// lives in vector registers across an item: the step's hotspot centres and the
// item's descriptor are wave-uniform (scalar registers), the next step's state
// is written before the first item, and a claim ahead keeps only its index
// during the item (thread 0 loads that item's descriptor at the item's end).
template <typename T, int V, int KAHAN, int D>
__global__ __launch_bounds__(max_block<T>(kPipeMarch + D)) void k_persistent_march(DevArgs a) {
    extern __shared__ __align__(32) unsigned char smem[];
    T* lds = reinterpret_cast<T*>(smem);
    __shared__ double red[kRedLen];
    __shared__ ItemDesc s_cur, s_nxt;

    const uint64_t t_launch = wall_clock64();
    const int wg = blockIdx.x;
    const WgState ws = a.wstate[wg];            // equal in every workgroup of the launch
    const uint64_t step = ws.step;
    const int par = uni(static_cast<int>(step & 1));   // claim-counter set
    const int b = uni(static_cast<int>(step & kSlotMask));     // partials buffer and state slot
    const int cur = uni(ws.cur);
    StepInfo si;
    si.step = step;
#pragma unroll
    for (int h = 0; h < kMaxHot; ++h) {
        si.hcx[h] = uni(ws.hx[h]);
        si.hcy[h] = uni(ws.hy[h]);
    }
    const T* src = static_cast<const T*>(cur ? a.field1 : a.field0);
    T* dst = static_cast<T*>(cur ? a.field0 : a.field1);
    int* heads = a.heads + par * a.nqueues;
    double* partials = a.partials + static_cast<int64_t>(b) * a.part_stride;
    const int home = uni(home_queue(a, wg));
    const int hbeg = uni(a.seg[home]);
    const int hn = uni(a.seg[home + 1]) - hbeg;

    if (threadIdx.x == 0) {
        s_cur = a.firstd[2 * wg];
        s_nxt = a.firstd[2 * wg + 1];
    }
    if (wg == 0) {
        int* other = a.heads + (par ^ 1) * a.nqueues;
        for (int q = threadIdx.x; q < a.nqueues; q += a.block) other[q] = a.head0;
        if (threadIdx.x == 0) {
            a.ctrl->pend_n[b] = a.ctrl->nitems;
            a.ctrl->pend_step[b] = step + 1;
            a.pstate[(b + 1) & kSlotMask] = next_state(a, ws);
        }
    }
    if (wg == a.nwg - 1) settle_others(a, 1u << b, red, a.block);   // earlier steps' sums
    __syncthreads();                             // every thread has read its step state
    if (threadIdx.x == 0) a.wstate[wg] = next_state(a, ws);
    double busy = 0.0;
    uint64_t t_first = 0, t_last = 0;
    bool drained = false;    // (thread 0) the home queue has nothing left to claim
    for (;;) {
        ItemDesc d = uni(s_cur);
        if (d.id < 0) {                      // nothing claimed ahead: claim with stealing
            __syncthreads();
            if (threadIdx.x < kWave) {
                const int qi = claim(a, heads, home);
                if (threadIdx.x == 0) {
                    s_cur = qi >= 0 ? a.queue[qi] : no_item();
                    s_nxt = no_item();
                }
            }
            __syncthreads();
            d = uni(s_cur);
            drained = true;
            if (d.id < 0) break;
        }
        __syncthreads();                     // every thread holds d before s_cur changes
        int nidx = hn;
        if (threadIdx.x == 0 && !drained) nidx = atomicAdd(&heads[home], 1);
        const uint64_t t_start = wall_clock64();
        if (t_first == 0) t_first = t_start;
        const ItemOut o = process_item_march<T, V, KAHAN, D>(a, d, src, dst, si.hcx, si.hcy, lds, red,
                                                             NoHook{});
        t_last = wall_clock64();
        const double ticks = static_cast<double>(t_last - t_start);  // used by thread 0
        record_item(a, partials, d, o, ticks);
        if (threadIdx.x == 0) {
            busy += ticks;
            s_cur = s_nxt;
            ItemDesc na = no_item();
            if (!drained) {
                if (nidx < hn) na = a.queue[hbeg + nidx];
                drained = nidx + 1 >= hn;
            }
            s_nxt = na;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        unsafeAtomicAdd(&a.wg_busy[wg], busy);
        uint64_t* tl = a.wg_timeline + 4 * static_cast<size_t>(wg);
        tl[0] = t_launch;
        tl[1] = t_first ? t_first : t_launch;
        tl[2] = t_last ? t_last : t_launch;
        tl[3] = wall_clock64();
    }
}

// Busy time per compute unit of a launch of one workgroup per item: the
// hardware's XCD id and the CU/array/engine bits 8..15 of its HW_ID register
// name the unit this workgroup ran on.
__device__ __forceinline__ void add_cu_busy(const DevArgs& a, double ticks) {
    const unsigned hw = __builtin_amdgcn_s_getreg((31 << 11) | 4);      // HW_ID, 32 bits
    const unsigned xcc = __builtin_amdgcn_s_getreg((3 << 11) | 20);     // XCC_ID, 4 bits
    unsafeAtomicAdd(&a.wg_busy[((xcc & 7u) << 8) | ((hw >> 8) & 0xffu)], ticks);
}

// One launch per step with one workgroup per item: workgroup b runs item b of
// the queue order (all queues in turn; with one queue, the global longest-first
// or hot-first-then-by-position order), and the hardware dispatcher starts each
// workgroup as soon as a previous one leaves the CU.  This keeps every CU full
// of short-lived workgroups whose loads cover neighbouring rows, the pattern a
// streaming kernel reads HBM fastest with, and needs no claims.  The step
// state is the shared copy in the step's slot (its number mod kStepSlots, from the
// host); workgroup 0 writes the next step's copy, resets the claim-counter set
// of the next step, records this step's pending checksum and sums the earlier
// steps'.
template <typename T, int V, int KAHAN, int D>
__global__ __launch_bounds__(max_block<T>(kPipeMarch + D)) void k_items(DevArgs a, int slot) {
    extern __shared__ __align__(32) unsigned char smem[];
    T* lds = reinterpret_cast<T*>(smem);
    __shared__ double red[kRedLen];

    const WgState ws = a.pstate[slot];
    StepInfo si;
    si.step = ws.step;
#pragma unroll
    for (int h = 0; h < kMaxHot; ++h) {
        si.hcx[h] = uni(ws.hx[h]);
        si.hcy[h] = uni(ws.hy[h]);
    }
    const int cur = uni(ws.cur);
    const T* src = static_cast<const T*>(cur ? a.field1 : a.field0);
    T* dst = static_cast<T*>(cur ? a.field0 : a.field1);
    double* partials = a.partials + static_cast<int64_t>(slot) * a.part_stride;
    if (blockIdx.x == 0) {
        settle_others(a, 1u << slot, red, a.block);   // earlier steps' sums
        int* other = a.heads + static_cast<int>((ws.step + 1) & 1) * a.nqueues;
        for (int q = threadIdx.x; q < a.nqueues; q += a.block) other[q] = a.head0;
        if (threadIdx.x == 0) {
            a.ctrl->pend_n[slot] = a.ctrl->nitems;
            a.ctrl->pend_step[slot] = ws.step + 1;
            a.pstate[(slot + 1) & kSlotMask] = next_state(a, ws);
        }
    }
    const ItemDesc d = uni(a.queue[blockIdx.x]);
    const uint64_t t_start = wall_clock64();
    const ItemOut o = process_item_march<T, V, KAHAN, D>(a, d, src, dst, si.hcx, si.hcy, lds, red, NoHook{});
    const double ticks = static_cast<double>(wall_clock64() - t_start);
    record_item(a, partials, d, o, ticks);
    if (threadIdx.x == 0) add_cu_busy(a, ticks);
}

// Two steps per launch, one workgroup per item (the launch form above with
// the fused two-step item body).  Step s's shared state is in slot; the
// state of step s + 1 follows from it.  The launch writes the checksum
// partials of steps s and s + 1 (buffers slot and slot + 1 mod kStepSlots), sums the
// other buffers, and leaves the state of step s + 2 in slot + 2 mod kStepSlots: two
// steps later, and the field copy flipped once (one launch, one write).
template <typename T, int V, int KAHAN, int D>
__global__ __launch_bounds__(max_block<T>(kPipeMarch + D)) void k_items2(DevArgs a, int slot) {
    extern __shared__ __align__(32) unsigned char smem[];
    T* lds = reinterpret_cast<T*>(smem);
    __shared__ double red[kRedLen];

    const WgState ws = a.pstate[slot];
    const WgState ws1 = next_state(a, ws);
    int h1x[kMaxHot], h1y[kMaxHot], h2x[kMaxHot], h2y[kMaxHot];
#pragma unroll
    for (int h = 0; h < kMaxHot; ++h) {
        h1x[h] = uni(ws.hx[h]);
        h1y[h] = uni(ws.hy[h]);
        h2x[h] = uni(ws1.hx[h]);
        h2y[h] = uni(ws1.hy[h]);
    }
    const int cur = uni(ws.cur);
    const T* src = static_cast<const T*>(cur ? a.field1 : a.field0);
    T* dst = static_cast<T*>(cur ? a.field0 : a.field1);
    const int slot1 = (slot + 1) & kSlotMask;
    if (blockIdx.x == 0) {
        settle_others(a, (1u << slot) | (1u << slot1), red, a.block2);   // earlier steps' sums
        for (int q = threadIdx.x; q < 2 * a.nqueues; q += a.block2) a.heads[q] = a.head0;
        if (threadIdx.x == 0) {
            a.ctrl->pend_n[slot] = a.ctrl->nitems;
            a.ctrl->pend_n[slot1] = a.ctrl->nitems;
            a.ctrl->pend_step[slot] = ws.step + 1;
            a.ctrl->pend_step[slot1] = ws.step + 2;
            WgState n2 = next_state(a, ws1);
            n2.cur = ws.cur ^ 1;
            a.pstate[(slot + 2) & kSlotMask] = n2;
        }
    }
    const ItemDesc d = uni(a.queue[blockIdx.x]);
    const uint64_t t_start = wall_clock64();
    const ItemOut2 o = process_item_march2<T, V, KAHAN, D>(a, d, src, dst, h1x, h1y, h2x, h2y, lds, red);
    const double ticks = static_cast<double>(wall_clock64() - t_start);
    if (threadIdx.x == 0) {
        a.partials[static_cast<int64_t>(slot) * a.part_stride + d.id] = o.checksum1;
        a.partials[static_cast<int64_t>(slot1) * a.part_stride + d.id] = o.checksum2;
        unsafeAtomicAdd(&a.loads_work[d.chunk], o.work);
        unsafeAtomicAdd(&a.loads_time[d.chunk], ticks);
        unsafeAtomicAdd(&a.tile_work[d.tile], o.work);
        add_cu_busy(a, ticks);
    }
    for (int r = threadIdx.x; r < (d.wh >> 16); r += a.block2)   // one visit per row and step
        __hip_atomic_fetch_add(&a.visits[d.vbase + r], 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Three steps per launch, one workgroup per item: as the two-step launch, with
// the partials of steps s, s + 1 and s + 2 (buffers slot .. slot + 2 mod
// kStepSlots) and the state of step s + 3 left in slot + 3.
template <typename T, int V, int KAHAN, int D>
__global__ __launch_bounds__(max_block<T>(kPipeMarch + D)) void k_items3(DevArgs a, int slot) {
    extern __shared__ __align__(32) unsigned char smem[];
    T* lds = reinterpret_cast<T*>(smem);
    __shared__ double red[kRedLen];

    const WgState ws = a.pstate[slot];
    const WgState ws1 = next_state(a, ws);
    const WgState ws2 = next_state(a, ws1);
    int h1x[kMaxHot], h1y[kMaxHot], h2x[kMaxHot], h2y[kMaxHot], h3x[kMaxHot], h3y[kMaxHot];
#pragma unroll
    for (int h = 0; h < kMaxHot; ++h) {
        h1x[h] = uni(ws.hx[h]);
        h1y[h] = uni(ws.hy[h]);
        h2x[h] = uni(ws1.hx[h]);
        h2y[h] = uni(ws1.hy[h]);
        h3x[h] = uni(ws2.hx[h]);
        h3y[h] = uni(ws2.hy[h]);
    }
    const int cur = uni(ws.cur);
    const T* src = static_cast<const T*>(cur ? a.field1 : a.field0);
    T* dst = static_cast<T*>(cur ? a.field0 : a.field1);
    int sl[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) sl[i] = (slot + i) & kSlotMask;
    if (blockIdx.x == 0) {
        settle_others(a, (1u << sl[0]) | (1u << sl[1]) | (1u << sl[2]), red, a.block3);   // earlier sums
        for (int q = threadIdx.x; q < 2 * a.nqueues; q += a.block3) a.heads[q] = a.head0;
        if (threadIdx.x == 0) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                a.ctrl->pend_n[sl[i]] = a.ctrl->nitems;
                a.ctrl->pend_step[sl[i]] = ws.step + 1 + i;
            }
            WgState n3 = next_state(a, ws2);
            n3.cur = ws.cur ^ 1;
            a.pstate[(slot + 3) & kSlotMask] = n3;
        }
    }
    const ItemDesc d = uni(a.queue[blockIdx.x]);
    const uint64_t t_start = wall_clock64();
    const ItemOut3 o =
        process_item_march3<T, V, KAHAN, D>(a, d, src, dst, h1x, h1y, h2x, h2y, h3x, h3y, lds, red);
    const double ticks = static_cast<double>(wall_clock64() - t_start);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < 3; ++i) a.partials[static_cast<int64_t>(sl[i]) * a.part_stride + d.id] = o.checksum[i];
        unsafeAtomicAdd(&a.loads_work[d.chunk], o.work);
        unsafeAtomicAdd(&a.loads_time[d.chunk], ticks);
        unsafeAtomicAdd(&a.tile_work[d.tile], o.work);
        add_cu_busy(a, ticks);
    }
    for (int r = threadIdx.x; r < (d.wh >> 16); r += a.block3)   // one visit per row and step
        __hip_atomic_fetch_add(&a.visits[d.vbase + r], 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T, int V, int KAHAN, int PIPE>
__global__ __launch_bounds__(max_block<T>(PIPE)) void k_plain(DevArgs a, int chunk) {
    extern __shared__ __align__(32) unsigned char smem[];
    T* lds = reinterpret_cast<T*>(smem);
    __shared__ double red[2 * kMaxBlock / kWave];

    const WgState ws = a.wstate[0];
    const uint64_t step = ws.step;
    const int b = static_cast<int>(step & kSlotMask);
    const StepInfo si = step_info(ws);
    const T* src = static_cast<const T*>(ws.cur ? a.field1 : a.field0);
    T* dst = static_cast<T*>(ws.cur ? a.field0 : a.field1);
    const int item = a.item_off[chunk] + blockIdx.x;
    if (item >= a.item_off[chunk + 1]) return;  // grid sized for a larger plan
    const ItemDesc d = a.items[item];
    const uint64_t t_start = wall_clock64();
    const Carry none{0, 0, 0};
    Carry unused;
    ItemOut o;
    if constexpr (PIPE >= kPipeMarch)
        o = process_item_march<T, V, KAHAN, PIPE - kPipeMarch>(a, d, src, dst, si.hcx, si.hcy, lds, red,
                                                             NoHook{});
    else
        o = process_item<T, V, KAHAN, PIPE>(a, d, no_item(), none, unused, src, dst, si.hcx, si.hcy, lds,
                                            red, NoHook{});
    record_item(a, a.partials + static_cast<int64_t>(b) * a.part_stride, d, o,
                static_cast<double>(wall_clock64() - t_start));
}

// End of a plain step (one workgroup): settle a persistent step still pending
// in the other buffer, sum this step's partials, reset both claim-counter
// sets, and move every workgroup's step number on.
__global__ __launch_bounds__(kSumThreads) void k_finish(DevArgs a) {
    __shared__ double red[kRedLen];
    const WgState ws = a.wstate[0];
    const uint64_t step = ws.step;
    const int b = static_cast<int>(step & kSlotMask);
    settle_others(a, 1u << b, red, kSumThreads);
    const double total = sum_partials(a.partials + static_cast<int64_t>(b) * a.part_stride,
                                      static_cast<int>(a.ctrl->nitems), red, kSumThreads);
    if (threadIdx.x == 0) {
        a.hist[step % kHistLen] = total;
        a.ctrl->pend_step[b] = 0;
    }
    for (int q = threadIdx.x; q < 2 * a.nqueues; q += kSumThreads) a.heads[q] = a.head0;
    __syncthreads();                  // every thread has read wstate[0]
    const WgState nx = next_state(a, ws);
    for (int w = threadIdx.x; w < a.nwg; w += kSumThreads) a.wstate[w] = nx;
    if (threadIdx.x == 0) a.pstate[(b + 1) & kSlotMask] = nx;
}

// Every workgroup's own copy of the step state from the shared copy in slot
// (after steps launched one workgroup per item, which keep only the shared
// copies, and before a form that reads its own copy).
__global__ __launch_bounds__(256) void k_seed_state(DevArgs a, int slot) {
    const WgState s = a.pstate[slot];
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < a.nwg; w += gridDim.x * blockDim.x)
        a.wstate[w] = s;
}

// Sums the checksum of any persistent step still pending (one workgroup).
__global__ __launch_bounds__(kSumThreads) void k_flush(DevArgs a) {
    __shared__ double red[kRedLen];
    settle_others(a, 0u, red, kSumThreads);
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t n) {
    uint64_t z = seed + (n + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename T>
__global__ void k_init(T* q, int64_t n, uint64_t seed) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t m = static_cast<int64_t>(splitmix64(seed, static_cast<uint64_t>(i)) >> 40);
        q[i] = static_cast<T>(static_cast<double>(m - 8388608) * (1.0 / 8388608.0));
    }
}

__global__ void k_zero(uint32_t* p, size_t nwords) {
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < nwords;
         i += static_cast<size_t>(gridDim.x) * blockDim.x)
        p[i] = 0u;
}

__global__ void k_reset_control(DevArgs a) {
    for (int q = threadIdx.x; q < 2 * a.nqueues; q += blockDim.x) a.heads[q] = a.head0;
    WgState first;
    first.step = 0;
    first.cur = 0;
#pragma unroll
    for (int h = 0; h < kMaxHot; ++h) {
        first.hx[h] = a.hx_first[h];
        first.hy[h] = a.hy_first[h];
    }
    for (int w = threadIdx.x; w < a.nwg; w += blockDim.x) a.wstate[w] = first;
    if (threadIdx.x < kStepSlots) {
        a.pstate[threadIdx.x] = first;
        a.ctrl->pend_step[threadIdx.x] = 0;
    }
}

// Table upload: segment blockIdx.y copied by the blocks of row y, grid-stride,
// so that the reads over the bus of all segments are in flight together.
struct GatherArgs {
    GatherSeg seg[kMaxGather];
    int n;
};
__global__ __launch_bounds__(256) void k_gather(GatherArgs g) {
    const uint32_t stride = gridDim.x * blockDim.x;
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const GatherSeg sg = g.seg[blockIdx.y];
    // 16-byte words where both ends allow it (every table but the item count)
    const bool wide = ((reinterpret_cast<uintptr_t>(sg.src) | reinterpret_cast<uintptr_t>(sg.dst)) & 15) == 0;
    const uint32_t nv = wide ? sg.words / 4 : 0;
    const uint4* src4 = reinterpret_cast<const uint4*>(sg.src);
    uint4* dst4 = reinterpret_cast<uint4*>(sg.dst);
    for (uint32_t i = tid; i < nv; i += stride) dst4[i] = src4[i];
    for (uint32_t i = 4 * nv + tid; i < sg.words; i += stride) sg.dst[i] = sg.src[i];
}

// End of a measurement window: the chosen chunk loads and the tile work go to
// pinned host memory (the device address of the staging area), and with
// `reset` the window's counters (chunk work and time, tile work, workgroup
// busy time: one contiguous range [clear, clear + clear_words)) start again
// from zero.  A counter that is copied is cleared by the thread that read it,
// after the read; the others are only cleared.  So any grid works.
__global__ __launch_bounds__(256) void k_measure_out(double* loads, double* tiles, int C, int ntiles,
                                                    double* out_loads, double* out_tiles, uint32_t* clear,
                                                    size_t clear_words) {
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    const size_t tid = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool reset = clear_words > 0;
    for (size_t i = tid; i < static_cast<size_t>(C); i += stride) {
        out_loads[i] = loads[i];
        if (reset) loads[i] = 0.0;
    }
    for (size_t i = tid; i < static_cast<size_t>(ntiles); i += stride) {
        out_tiles[i] = tiles[i];
        if (reset) tiles[i] = 0.0;
    }
    const uint32_t* lo = reinterpret_cast<const uint32_t*>(loads);
    const uint32_t* to = reinterpret_cast<const uint32_t*>(tiles);
    for (size_t i = tid; i < clear_words; i += stride) {
        const uint32_t* w = clear + i;
        const bool copied = (w >= lo && w < lo + 2 * static_cast<size_t>(C)) ||
                            (w >= to && w < to + 2 * static_cast<size_t>(ntiles));
        if (!copied) clear[i] = 0u;
    }
}

// Field sum, pass 1: block b sums the contiguous range [b*n/B, (b+1)*n/B).
template <typename T>
__global__ __launch_bounds__(256) void k_sum1(const T* q, int64_t n, double* partial) {
    __shared__ double red[256 / kWave];
    const int64_t b = blockIdx.x, B = gridDim.x;
    const int64_t lo = b * n / B, hi = (b + 1) * n / B;
    double acc = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) acc += static_cast<double>(q[i]);
    const double s = block_sum(acc, red, 256);
    if (threadIdx.x == 0) partial[b] = s;
}

__global__ __launch_bounds__(256) void k_sum2(const double* partial, int nb, double* out) {
    __shared__ double red[256 / kWave];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) acc += partial[i];
    const double s = block_sum(acc, red, 256);
    if (threadIdx.x == 0) *out = s;
}

// ---- dispatch ------------------------------------------------------------------
using PersistentFn = void (*)(DevArgs);
using PlainFn = void (*)(DevArgs, int);
using ItemsFn = void (*)(DevArgs, int);

// pipe: kPipeDma, or the register pipeline's depth (2, 4 or 8 with V = 4, where
// the host allows 8 in FP32 only: eight FP64 rows do not fit in registers; 2 otherwise)
template <typename T, int KAHAN>
PersistentFn persistent_for(int vec, int pipe) {
    if (vec == 4) {
        switch (pipe) {
            case kPipeMarch + 2: return k_persistent_march<T, 4, KAHAN, 2>;
            case kPipeMarch + 4: return k_persistent_march<T, 4, KAHAN, 4>;
            case kPipeMarch + 8: return k_persistent_march<T, 4, KAHAN, 6>;   // 6: a ring of 10 would spill
            case kPipeDma: return k_persistent<T, 4, KAHAN, kPipeDma>;
            case 8: return k_persistent<T, 4, KAHAN, sizeof(T) == 4 ? 8 : 4>;
            case 4: return k_persistent<T, 4, KAHAN, 4>;
            default: return k_persistent<T, 4, KAHAN, 2>;
        }
    }
    return vec == 2 ? k_persistent<T, 2, KAHAN, 2> : k_persistent<T, 1, KAHAN, 2>;
}
template <typename T, int KAHAN>
PlainFn plain_for(int vec, int pipe) {
    if (vec == 4) {
        switch (pipe) {
            case kPipeMarch + 2: return k_plain<T, 4, KAHAN, kPipeMarch + 2>;
            case kPipeMarch + 4: return k_plain<T, 4, KAHAN, kPipeMarch + 4>;
            case kPipeMarch + 8: return k_plain<T, 4, KAHAN, kPipeMarch + 8>;
            case kPipeDma: return k_plain<T, 4, KAHAN, kPipeDma>;
            case 8: return k_plain<T, 4, KAHAN, sizeof(T) == 4 ? 8 : 4>;
            case 4: return k_plain<T, 4, KAHAN, 4>;
            default: return k_plain<T, 4, KAHAN, 2>;
        }
    }
    return vec == 2 ? k_plain<T, 2, KAHAN, 2> : k_plain<T, 1, KAHAN, 2>;
}

template <typename T, int KAHAN>
ItemsFn items_for(int pipe) {
    switch (pipe) {
        case kPipeMarch + 4: return k_items<T, 4, KAHAN, 4>;
        case kPipeMarch + 8: return k_items<T, 4, KAHAN, 8>;
        default: return k_items<T, 4, KAHAN, 2>;
    }
}
ItemsFn pick_items(int prec, int pipe) {
    if (prec == 2) return items_for<double, 0>(pipe);
    if (prec == 1) return items_for<float, 1>(pipe);
    return items_for<float, 0>(pipe);
}
template <typename T, int KAHAN>
ItemsFn items2_for(int vec, int pipe) {
    if (vec == 5)   // rows in flight: 2 or 4
        return pipe == kPipeMarch + 4 ? k_items2<T, 5, KAHAN, 4> : k_items2<T, 5, KAHAN, 2>;
    // 8 rows in flight: 4 in the two-step launch, whose register rings of 8 + 2 rows
    // would spill
    return pipe >= kPipeMarch + 4 ? k_items2<T, 4, KAHAN, 4> : k_items2<T, 4, KAHAN, 2>;
}
ItemsFn pick_items2(int prec, int vec, int pipe) {
    if (prec == 2) return items2_for<double, 0>(vec, pipe);
    if (prec == 1) return items2_for<float, 1>(vec, pipe);
    return items2_for<float, 0>(vec, pipe);
}
template <typename T, int KAHAN>
ItemsFn items3_for(int pipe) {
    switch (pipe) {
        case kPipeMarch + 4: return k_items3<T, 4, KAHAN, 4>;
        case kPipeMarch + 8: return k_items3<T, 4, KAHAN, 8>;
        default: return k_items3<T, 4, KAHAN, 2>;
    }
}
ItemsFn pick_items3(int prec, int pipe) {
    if (prec == 2) return items3_for<double, 0>(pipe);
    if (prec == 1) return items3_for<float, 1>(pipe);
    return items3_for<float, 0>(pipe);
}

PersistentFn pick_persistent(int prec, int vec, int pipe) {
    if (prec == 2) return persistent_for<double, 0>(vec, pipe);
    if (prec == 1) return persistent_for<float, 1>(vec, pipe);
    return persistent_for<float, 0>(vec, pipe);
}
PlainFn pick_plain(int prec, int vec, int pipe) {
    if (prec == 2) return plain_for<double, 0>(vec, pipe);
    if (prec == 1) return plain_for<float, 1>(vec, pipe);
    return plain_for<float, 0>(vec, pipe);
}

// the pipeline a launch uses
int pipe_of(const DevArgs& a) {
    if (a.march > 0) return kPipeMarch + a.march;
    return a.stage_rows > 0 ? kPipeDma : a.reg_depth;
}

}  // namespace

int persistent_occupancy(const DevArgs& a, int prec, int vec, int block, size_t lds) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, reinterpret_cast<const void*>(pick_persistent(prec, vec, pipe_of(a))), block,
            lds) != hipSuccess)
        return -1;
    return n;
}

int launch_persistent(const DevArgs& a, int prec, int vec, int nwg, int block, size_t lds,
                      void* stream) {
    hipLaunchKernelGGL(pick_persistent(prec, vec, pipe_of(a)), dim3(nwg), dim3(block), lds,
                       static_cast<hipStream_t>(stream), a);
    return static_cast<int>(hipGetLastError());
}

int launch_plain_chunk(const DevArgs& a, int prec, int vec, int chunk, int nitems_chunk,
                       int block, size_t lds, void* stream) {
    hipLaunchKernelGGL(pick_plain(prec, vec, pipe_of(a)), dim3(nitems_chunk), dim3(block), lds,
                       static_cast<hipStream_t>(stream), a, chunk);
    return static_cast<int>(hipGetLastError());
}

int launch_items(const DevArgs& a, int prec, int vec, int nitems, int block, size_t lds, int slot,
                 void* stream) {
    if (vec != 4 || a.march <= 0 || nitems <= 0) return static_cast<int>(hipErrorInvalidValue);
    hipLaunchKernelGGL(pick_items(prec, pipe_of(a)), dim3(nitems), dim3(block), lds,
                       static_cast<hipStream_t>(stream), a, slot);
    return static_cast<int>(hipGetLastError());
}

int launch_items2(const DevArgs& a, int prec, int vec, int nitems, int block, size_t lds, int slot,
                  void* stream) {
    if ((vec != 4 && vec != 5) || (vec == 5 && a.march == 8) || a.march <= 0 || nitems <= 0 ||
        block != a.block2)
        return static_cast<int>(hipErrorInvalidValue);
    hipLaunchKernelGGL(pick_items2(prec, vec, pipe_of(a)), dim3(nitems), dim3(block), lds,
                       static_cast<hipStream_t>(stream), a, slot);
    return static_cast<int>(hipGetLastError());
}

int launch_items3(const DevArgs& a, int prec, int vec, int nitems, int block, size_t lds, int slot,
                  void* stream) {
    if (vec != 4 || a.march <= 0 || nitems <= 0 || block != a.block3)
        return static_cast<int>(hipErrorInvalidValue);
    hipLaunchKernelGGL(pick_items3(prec, pipe_of(a)), dim3(nitems), dim3(block), lds,
                       static_cast<hipStream_t>(stream), a, slot);
    return static_cast<int>(hipGetLastError());
}

int launch_seed_state(const DevArgs& a, int slot, void* stream) {
    const int blocks = (a.nwg + 255) / 256;
    hipLaunchKernelGGL(k_seed_state, dim3(blocks > 0 ? blocks : 1), dim3(256), 0,
                       static_cast<hipStream_t>(stream), a, slot);
    return static_cast<int>(hipGetLastError());
}

int launch_finish(const DevArgs& a, void* stream) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kSumThreads), 0, static_cast<hipStream_t>(stream), a);
    return static_cast<int>(hipGetLastError());
}

int launch_flush(const DevArgs& a, void* stream) {
    hipLaunchKernelGGL(k_flush, dim3(1), dim3(kSumThreads), 0, static_cast<hipStream_t>(stream), a);
    return static_cast<int>(hipGetLastError());
}

int launch_gather(const GatherSeg* segs, int n, void* stream) {
    if (n < 0 || n > kMaxGather) return static_cast<int>(hipErrorInvalidValue);
    GatherArgs g{};
    uint32_t most = 0;
    for (int s = 0; s < n; ++s) {
        g.seg[s] = segs[s];
        most = segs[s].words > most ? segs[s].words : most;
    }
    g.n = n;
    if (n == 0) return static_cast<int>(hipSuccess);
    const uint32_t want = (most / 4 + 255) / 256;   // blocks for the largest segment in 16-byte words
    const dim3 grid(want < 64 ? (want > 0 ? want : 1) : 64, n);
    hipLaunchKernelGGL(k_gather, grid, dim3(256), 0, static_cast<hipStream_t>(stream), g);
    return static_cast<int>(hipGetLastError());
}

int launch_measure_out(double* loads, double* tiles, int C, int ntiles, double* out_loads, double* out_tiles,
                       void* clear, size_t clear_bytes, void* stream) {
    const size_t most = std::max(static_cast<size_t>(std::max(C, ntiles)), clear_bytes / 4);
    const size_t want = (most + 255) / 256;
    const dim3 grid(static_cast<unsigned>(want < 256 ? (want > 0 ? want : 1) : 256));
    hipLaunchKernelGGL(k_measure_out, grid, dim3(256), 0, static_cast<hipStream_t>(stream), loads, tiles, C,
                       ntiles, out_loads, out_tiles, static_cast<uint32_t*>(clear), clear_bytes / 4);
    return static_cast<int>(hipGetLastError());
}

int launch_reset_control(const DevArgs& a, void* stream) {
    hipLaunchKernelGGL(k_reset_control, dim3(1), dim3(256), 0, static_cast<hipStream_t>(stream), a);
    return static_cast<int>(hipGetLastError());
}

int launch_init_field(void* q, int prec, int64_t n, uint64_t seed, void* stream) {
    const int64_t want = (n + 255) / 256;
    const dim3 grid(static_cast<unsigned>(want < 65536 ? (want > 0 ? want : 1) : 65536));
    if (prec == 2)
        hipLaunchKernelGGL(k_init<double>, grid, dim3(256), 0, static_cast<hipStream_t>(stream),
                           static_cast<double*>(q), n, seed);
    else
        hipLaunchKernelGGL(k_init<float>, grid, dim3(256), 0, static_cast<hipStream_t>(stream),
                           static_cast<float*>(q), n, seed);
    return static_cast<int>(hipGetLastError());
}

int launch_zero(void* p, size_t bytes, void* stream) {
    const size_t nwords = bytes / 4;
    if (nwords == 0) return 0;
    const size_t want = (nwords + 255) / 256;
    const dim3 grid(static_cast<unsigned>(want < 4096 ? want : 4096));
    hipLaunchKernelGGL(k_zero, grid, dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<uint32_t*>(p), nwords);
    return static_cast<int>(hipGetLastError());
}

int launch_field_sum(const void* q, int prec, int64_t n, double* partial, double* out,
                     void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (prec == 2)
        hipLaunchKernelGGL(k_sum1<double>, dim3(kSumBlocks), dim3(256), 0, s,
                           static_cast<const double*>(q), n, partial);
    else
        hipLaunchKernelGGL(k_sum1<float>, dim3(kSumBlocks), dim3(256), 0, s,
                           static_cast<const float*>(q), n, partial);
    hipLaunchKernelGGL(k_sum2, dim3(1), dim3(256), 0, s, partial, kSumBlocks, out);
    return static_cast<int>(hipGetLastError());
}

}  // namespace lbgrid

// ---- the checksum for callers that cannot allocate ----------------------------------
// The two-pass FP64 field sum of lb_fields (k_sum1 over kSumBlocks blocks, then
// k_sum2) with its partials in this file-scope array instead of a context's
// workspace.  Each GPU the library runs on holds its own copy until the process
// ends; host code reaches it only through the address hipGetSymbolAddress gives
// for the current device (the array's name is a host-side stand-in).
static __device__ __align__(256) double scratch[lbgrid::kSumBlocks];

namespace lbgrid {
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};
}  // namespace

int prepare_static_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return static_cast<int>(hipErrorInvalidDevice);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[device]) return static_cast<int>(hipSuccess);
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return static_cast<int>(e);
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return static_cast<int>(e);
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return static_cast<int>(e);
    g_scratch_dev[device] = static_cast<double*>(p);
    return static_cast<int>(hipSuccess);
}

}  // namespace lbgrid

extern "C" int lb_field_sum_noalloc(const void* field, int32_t precision, int64_t ncells, double* sum_out,
                                    void* hip_stream) {
    using namespace lbgrid;
    if (!sum_out) return report_error(LB_E_INVAL, "sum_out is NULL");
    if (!field && ncells > 0) return report_error(LB_E_INVAL, "field is NULL");
    if (precision != LB_FP32 && precision != LB_FP32_KAHAN && precision != LB_FP64)
        return report_error(LB_E_INVAL, "unknown precision");
    if (ncells < 0 || ncells > LB_NOALLOC_MAX_CELLS)
        return report_error(LB_E_INVAL, "ncells must be in [0, LB_NOALLOC_MAX_CELLS]");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return report_error(LB_E_HIP, hipGetErrorString(e));
    if ((e = static_cast<hipError_t>(prepare_static_scratch(dev))) != hipSuccess)
        return report_error(LB_E_HIP, hipGetErrorString(e));
    double* part = g_scratch_dev[dev];
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (precision == LB_FP64)
        hipLaunchKernelGGL(k_sum1<double>, dim3(kSumBlocks), dim3(256), 0, s, static_cast<const double*>(field),
                           ncells, part);
    else
        hipLaunchKernelGGL(k_sum1<float>, dim3(kSumBlocks), dim3(256), 0, s, static_cast<const float*>(field),
                           ncells, part);
    hipLaunchKernelGGL(k_sum2, dim3(1), dim3(256), 0, s, part, kSumBlocks, sum_out);
    if ((e = hipGetLastError()) != hipSuccess) return report_error(LB_E_HIP, hipGetErrorString(e));
    return LB_OK;
}
