/*
 * lbgrid.h -- C ABI of liblbgrid.so: an over-decomposed 3D grid update with
 * per-chunk GPU load measurement and chunk-to-slot rebalancing on one MI355X
 * (gfx950), after "Dynamic Load Balancing in GPU-Based Systems -- Early
 * Experiments" (Fazenda, Mendes, Kale, Panetta, Rodrigues; arXiv 1310.4218).
 *
 * The paper's synthetic application (Section IV, Fig. 2) advances a
 * 2D-decomposed grid of virtual processors (VPs) one time step at a time:
 * a 3D Jacobi update, then a column "physics" loop whose trip count is set by
 * a load-control array moved across the domain (Section VI, Fig. 4).  Loads
 * are measured per VP (Section V) and a balancer (GreedyLB, RefineSwapLB,
 * Section VI) migrates VPs between processors.  On one GPU:
 *   VP          -> chunk: a rectangle of grid columns with all nz levels
 *   processor   -> slot: a queue served by a group of workgroups of one
 *                  persistent kernel
 *   migration   -> an update of the chunk->slot table (no data moves)
 *   measurement -> in-kernel per-chunk work counts and wall-clock ticks
 *
 * One time step, for every cell (x, y, z) of every field:
 *   s = c_center*q + c_nbr*(((((q[x-1] + q[x+1]) + q[y-1]) + q[y+1]) + q[z-1]) + q[z+1])
 *       x and y periodic; z mirror ghost (q[-1] = q[0], q[nz] = q[nz-1]);
 *   k = kmin + floor((kmax-kmin) * max_h exp(-r_h^2 / (2 sigma^2))), r_h^2 the
 *       integer minimum-image squared distance from (x, y) to hotspot h, which
 *       sits at (hx0 + hvx*t, hy0 + hvy*t) mod (nx, ny) at time t = t0 + step;
 *   q' = Phi^k(s),  Phi(q) = q + eps*(q - (q*q)*q).
 * Chunk c = j*px + i covers columns [xsplit[i], xsplit[i+1]) x [ysplit[j], ysplit[j+1]).
 * Field layout: q[((f*ny + y)*nx + x)*nz + z], the vertical index fastest
 * (the column layout of Fig. 1).
 *
 * Conventions for every call:
 *  - Every call returns an lb_status; the library never aborts or throws.
 *    On failure lb_last_error(ctx) (or lb_last_error(NULL) for calls without a
 *    context) gives a message; HIP failures carry hipGetErrorString's text.
 *  - Device buffers are borrowed: the caller allocates them (lb_query gives the
 *    sizes) and keeps them alive and untouched until lb_destroy.
 *  - Host arrays passed in are copied before the call returns; host output
 *    arrays are caller-allocated.
 *  - A context is not thread-safe.  Separate contexts are independent.
 *  - GPU work is enqueued on the stream given to lb_grid_init; calls that
 *    return host data synchronize that stream first.
 */
#ifndef LBGRID_H
#define LBGRID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LB_ABI_VERSION 7
#define LB_MAX_HOT 4
#define LB_NBUF 3

typedef enum {
    LB_OK = 0,
    LB_E_INVAL = -1,       /* bad argument or configuration                   */
    LB_E_STATE = -2,       /* call not valid in the context's current state   */
    LB_E_HIP = -3,         /* a HIP runtime call failed                       */
    LB_E_NOMEM = -4,       /* host allocation failed or a buffer is too small */
    LB_E_UNSUPPORTED = -5  /* valid request this build does not implement     */
} lb_status;

/* Arithmetic of the fields. */
enum { LB_FP32 = 0, LB_FP32_KAHAN = 1, LB_FP64 = 2 };
/* How lb_step runs a step. */
enum {
    LB_PLAIN = 0,          /* one kernel launch per chunk, chunks in id order  */
    LB_PERSISTENT = 1,     /* the balanced launch (persistent workgroups, or
                              one workgroup per item, one step or fuse_steps
                              steps per launch), replayed from a captured HIP
                              graph                                            */
    LB_PLAIN_GRAPH = 2,    /* LB_PLAIN's launches replayed from a HIP graph    */
    LB_PERSISTENT_EAGER = 3 /* LB_PERSISTENT launched directly (no graph)      */
};
/* Column physics.  POINTWISE: every cell of column (x, y) gets k(x, y)
 * applications of Phi (a pointwise reading of Fig. 1).  VERTICAL: k(x, y)
 * upward sweeps, level z (1..nz-1, in order) becoming
 * q[z] + eps*((q[z-1]^3) - (q[z]^3)) from the level below as already updated
 * in the same sweep, level 0 fixed (Fig. 1 / Fig. 4 as written, with the
 * level wrap of Fig. 4 kept inside 1..nz-1). */
enum { LB_PHYS_POINTWISE = 0, LB_PHYS_VERTICAL = 1 };
/* Load source for lb_measure / lb_rebalance. */
enum { LB_LOAD_WORK = 0, LB_LOAD_TIME = 1 };
/* Balancer. */
enum { LB_GREEDY = 0, LB_REFINE = 1, LB_REFINESWAP = 2,
       LB_GREEDY_THEN_REFINESWAP = 3 /* Experiment C's policy: Greedy first, then RefineSwap */ };

typedef struct lb_ctx lb_ctx;

/* Problem and launch configuration.  lb_config_default fills every field with
 * the defaults shown. */
typedef struct {
    int32_t nx, ny, nz;      /* grid cells; nz levels per column (>= 1 each)    */
    int32_t nfields;         /* independent fields sharing one cost field (1)  */
    int32_t px, py;          /* chunks along x and y                          */
    const int32_t *xsplit;   /* px+1 strictly increasing split points, [0] = 0,
                                [px] = nx; NULL = equal split floor(i*nx/px)   */
    const int32_t *ysplit;   /* likewise for y                                */
    int32_t precision;       /* LB_FP32 | LB_FP32_KAHAN | LB_FP64              */
    double c_center;         /* 0.4                                           */
    double c_nbr;            /* 0.1                                           */
    double eps;              /* 0.01                                          */
    int32_t nhot;            /* 0..LB_MAX_HOT hotspots (0: k = kmin)           */
    int32_t hx0[LB_MAX_HOT], hy0[LB_MAX_HOT];   /* start cell of each hotspot  */
    int32_t hvx[LB_MAX_HOT], hvy[LB_MAX_HOT];   /* cells per step              */
    double sigma;            /* Gaussian width in cells (> 0)                 */
    int32_t kmin, kmax;      /* 0 <= kmin <= kmax: column-loop trip range      */
    int32_t alpha_work;      /* work units per cell for the stencil (32)       */
    int32_t nslots;          /* S, the balancer's processors (256)            */
    int32_t nqueues;         /* Q work queues of the persistent kernel; slot s
                                feeds queue s mod Q; 0 = 8 when S is a
                                multiple of 8 (one queue per XCD), else S     */
    int32_t wg_per_queue;    /* G workgroups per queue; 0 = as many as can be
                                resident on the device, divided by Q          */
    int32_t tile_x, tile_y;  /* columns per work item along x, y; 0 = 16, 16   */
    int32_t steal;           /* 1: a workgroup whose slot queue is empty takes
                                items from other slots (default 1)            */
    int32_t graph_steps;     /* persistent steps per captured graph (10)      */
    int32_t item_split;      /* after a rebalance, tiles whose measured cost
                                exceeds W/(Q*G*item_split) are cut into row
                                ranges; 0 = never (2)                          */
    int32_t stage_rows;      /* > 0: rows per direct global->LDS batch (nz % 4
                                == 0 only); 0 = 4 when nz % 4 == 0, else the
                                register pipeline; -1 or -2: register pipeline
                                with 2 rows in flight; -4, -8: 4 or 8 rows in
                                flight (nz % 4 == 0, at most 512 threads per
                                workgroup; -8 in FP32 only).  In FP64 every
                                register pipeline allows at most 512 threads
                                per workgroup (tile_x * nz / V)              */
    int32_t physics;         /* LB_PHYS_POINTWISE | LB_PHYS_VERTICAL (the
                                latter needs nz/V to divide 64)               */
    int32_t tail_split;      /* in every queue, the cheapest tiles whose items
                                make up the final round of its G workgroups
                                (its last G items) are cut this many times
                                finer, so a step ends on small items;
                                0 or 1 = off (4)                              */
    int32_t item_alpha;      /* stencil weight per cell when measured tile work
                                sets item sizes (the balancer's loads keep
                                alpha_work); -1 = alpha_work (default). A
                                small value sizes items by their physics,
                                which one workgroup runs serially            */
    int32_t march;           /* > 0: the column-march pipeline with this many
                                rows in flight (2, 4 or 8; nz % 4 == 0, every
                                field below 4 GiB, (tile_x + 2) * nz / 4
                                threads per workgroup, at most 512 in FP64;
                                for 8 the persistent launch keeps 6 rows in
                                flight and the two-step launch 4); overrides
                                stage_rows.  0 = off (default)                */
    int32_t queue_order;     /* order of the items of a queue: 0 = longest
                                first (cost per item descending); 1 = the hot
                                items (cost per item above hot_cut percent of
                                the mean) longest first, then all others by their
                                position (first row, then first column), so
                                that workgroups running at the same time read
                                neighbouring rows (default 0)                 */
    int32_t hot_cut;         /* queue_order 1: an item is hot when its cost
                                exceeds hot_cut percent of the mean cost per
                                item (200)                                    */
    int32_t item_grid;       /* 1: a balanced step (LB_PERSISTENT,
                                LB_PERSISTENT_EAGER) launches one workgroup
                                per item, in queue order, and the hardware
                                dispatcher schedules them instead of claims on
                                the queues; needs march > 0.  0 = persistent
                                workgroups claiming from the queues (default) */
    int32_t fuse_steps;      /* item_grid 1 only: 2 = a balanced launch takes
                                two steps at once (temporal blocking): each
                                item reads its cells and a two-cell halo of
                                step s once, computes step s + 1 on the item
                                and a one-cell ring around it, and writes
                                step s + 2, with the same bits as two single
                                steps; an odd step count ends on a single
                                step.  (tile_x + 4) * nz / 4 threads per
                                workgroup, at most 512 in FP64.  3 = three
                                steps at once (a three-cell halo, rings of two
                                and one cells; (tile_x + 6) * nz / 4 threads),
                                a remainder ending on a two- or one-step
                                launch.  0 or 1 = one step per launch
                                (default)                                     */
    int32_t lane_levels;     /* levels per thread V of the two-step launch: 0
                                or 4 = 4 (default); 5 = 5, with nz / 5
                                threads per column, for nz whose nz / 4
                                threads per column would straddle waves (nz =
                                80: 16 threads, four whole columns per wave).
                                5 needs fuse_steps 2, march 2 or 4 and nz % 20
                                == 0 (the one-step launches keep 4 levels per
                                thread).  Same bits for either V.            */
    int32_t xcd_group;       /* item_grid 1 only: G > 1 deals the item queue to
                                the 8 XCDs in runs of G consecutive items (in
                                position order: neighbours along x, whose halo
                                columns overlap), so that one XCD runs each run
                                side by side and reads the shared halos from
                                its own L2; the queue order stands at a
                                granularity of 8 G items.  0 or 1 = off
                                (default); at most 64.  Same bits either way */
    int64_t t0;              /* time index of step 0 (hotspot phase)          */
    uint64_t seed;           /* seed of the SplitMix64 initial field           */
} lb_config;

/* Device buffers: ptr[0] and ptr[1] hold the two field copies (ping-pong),
 * ptr[2] the workspace (tables, queues, loads, counters). */
typedef struct {
    void *ptr[LB_NBUF];
    size_t bytes[LB_NBUF];
} lb_buffers;

/* Per-context counters, filled by lb_stats. */
typedef struct {
    int64_t steps;           /* steps enqueued since init                     */
    int32_t nchunks;         /* C                                             */
    int32_t ntiles;          /* tiles of chunks                               */
    int32_t nrows;           /* tile rows (the finest possible items)         */
    int32_t nitems;          /* work items of the installed plan              */
    int32_t nslots;          /* S                                             */
    int32_t nqueues;         /* Q                                             */
    int32_t nwg;             /* workgroups of the persistent launch (Q*G)     */
    int32_t block;           /* threads per workgroup                         */
    int32_t tile_x, tile_y;
    double clock_hz;         /* rate of the in-kernel wall clock              */
    double last_checksum;    /* FP64 sum of all cells after the last step     */
    int64_t measured_steps;  /* steps accumulated in the current load window  */
    double host_balance_us;  /* host time of every rebalance's balancer, summed */
    double host_plan_us;     /* host time of every plan (items, queue order,
                                staging, the upload launch), summed           */
    int32_t busy_slots;      /* entries lb_wg_busy returns: nwg (persistent
                                workgroups), or 2048 per-compute-unit slots
                                when balanced steps launch one workgroup per
                                item (keyed by XCD and CU id; unused ones 0)  */
    int32_t block2;          /* threads per workgroup of a two-step launch
                                (fuse_steps 2 or 3), else 0                   */
    int32_t block3;          /* ... of a three-step launch (fuse_steps 3)     */
    int32_t pad1;
} lb_stats_t;

/* Fill *cfg with the defaults listed in lb_config. */
void lb_config_default(lb_config *cfg);

/* Validate *cfg and report the device bytes each buffer needs in
 * sizes_out->bytes (ptr entries are set to NULL).  No GPU needed.
 * Errors: LB_E_INVAL (message names the field). */
int lb_query(const lb_config *cfg, lb_buffers *sizes_out);

/* Create a context over the caller's device buffers (sizes at least those of
 * lb_query) on the current HIP device.  hip_stream (a hipStream_t, may be
 * NULL for the null stream) orders all GPU work of the context.
 * init_field: NULL for the seeded SplitMix64 field (value of cell n is
 * ((splitmix64 output n+1) >> 40 - 2^23) * 2^-23), else nfields*ny*nx*nz
 * values of the precision's element type (float for LB_FP32 and
 * LB_FP32_KAHAN, double for LB_FP64), host or device memory.
 * The initial chunk->slot map is the block map floor(c*S/C) (c for C < S):
 * every slot holds a contiguous run of chunk ids, the starting placement of
 * the VPs in Section VI, Table V.  Returns LB_OK and *out, or an error with
 * *out = NULL. */
int lb_grid_init(const lb_config *cfg, const lb_buffers *bufs, void *hip_stream,
                 const void *init_field, lb_ctx **out);

/* The time-step loop of Fig. 2.  Enqueue nsteps >= 0 time steps in the given
 * mode (LB_PLAIN, LB_PERSISTENT, LB_PLAIN_GRAPH, LB_PERSISTENT_EAGER);
 * asynchronous.  Every mode gives bit-identical fields and loads.  With
 * fuse_steps 2 or 3 the balanced modes launch that many steps at once while
 * at least that many remain, and the rest in one shorter launch.  Loads of
 * every step are added to the current measurement window (Section V: the
 * measured time steps).  Errors: LB_E_INVAL (nsteps < 0, unknown mode),
 * LB_E_HIP (a capture or launch failed).  After LB_E_HIP the steps whose
 * launches were all enqueued count as done (lb_stats); if a plain step had
 * some of its per-chunk launches enqueued, the context is left unusable and
 * every later call but lb_stats, lb_destroy and lb_last_error returns
 * LB_E_STATE. */
int lb_step(lb_ctx *ctx, int32_t nsteps, int32_t mode);

/* The load measurement of Section V: the runtime's per-VP load database,
 * filled during the instrumented time steps of a migration window (Fig. 2
 * turns instrumentation on for the window's last steps, which Section V runs
 * synchronously so that GPU time is attributed to the right VP).  Here every
 * step is instrumented inside the kernel, with no serialisation.
 * Synchronize, copy the window's per-chunk loads (C doubles; LB_LOAD_WORK:
 * sum over steps of nz*nfields*(alpha_work + k) per column, exact integers;
 * LB_LOAD_TIME: in-kernel wall-clock ticks of the chunk's items) to loads_out
 * (may be NULL) and, when reset != 0, start a new window.  The copy is also
 * kept for lb_rebalance.  Errors: LB_E_INVAL (ctx NULL, unknown source),
 * LB_E_HIP (the synchronisation or the copy failed). */
int lb_measure(lb_ctx *ctx, int32_t source, double *loads_out, int32_t reset);

/* lb_measure in two halves, so that the host can enqueue more steps before it
 * waits (Section V's measured window, collected without draining the GPU).
 * lb_measure_begin enqueues the window's snapshot behind the steps enqueued so
 * far (and, when reset != 0, starts a new window, counting the steps enqueued
 * after it) and returns at once; lb_measure_end waits for that snapshot only
 * (steps enqueued after it keep running) and returns it as lb_measure does.
 * Errors: LB_E_STATE (begin while a snapshot is pending, end without one),
 * LB_E_INVAL, LB_E_HIP. */
int lb_measure_begin(lb_ctx *ctx, int32_t source, int32_t reset);
int lb_measure_end(lb_ctx *ctx, double *loads_out);

/* Compute a new chunk->slot map with strategy LB_GREEDY (Section VI,
 * Experiment A: heaviest chunk to the least loaded slot), LB_REFINE (move
 * chunks off slots above threshold*average, Experiment B without swaps),
 * LB_REFINESWAP (refine, then swap pairs where no move fits) or
 * LB_GREEDY_THEN_REFINESWAP (the policy of Experiment C: Greedy on the
 * context's first rebalance, RefineSwap on every later one) from loads
 * (C doubles, or NULL for the loads kept by the last lb_measure: LB_E_STATE
 * if there is none), install it and rebuild the per-slot work queues in
 * descending per-tile cost.  Outputs (each may be NULL): map_out[C],
 * *nmigrated, lambda_before_after[2] = max slot load / average slot load
 * under the old and the new map. */
int lb_rebalance(lb_ctx *ctx, int32_t strategy, double threshold, const double *loads,
                 int32_t *map_out, int32_t *nmigrated, double *lambda_before_after);

/* Install an explicit map (C slot indices in [0, S)) with per-chunk costs for
 * the queue order (NULL: equal costs, chunk id order). */
int lb_set_map(lb_ctx *ctx, const int32_t *map, const double *cost);

/* The full-data transfer of Fig. 2: before each migration call the
 * application copies its fields from the GPU to the host (and back after it).
 * On one GPU nothing has to move for a migration, so this is the checkpoint
 * and read-back path.
 * Synchronize and copy field `field` of the current step (native precision,
 * ny*nx*nz elements, layout [y][x][z]) to dst (host or device, dst_bytes at
 * least that) when dst is not NULL; *checksum_out (may be NULL) receives the
 * FP64 sum of its cells, computed on the device in a fixed order.  Errors:
 * LB_E_INVAL (field out of range), LB_E_NOMEM (dst_bytes too small),
 * LB_E_HIP. */
int lb_fields(lb_ctx *ctx, int32_t field, void *dst, size_t dst_bytes, double *checksum_out);

/* Synchronize and fill *out. */
int lb_stats(lb_ctx *ctx, lb_stats_t *out);

/* Synchronize and copy per-workgroup busy ticks of the persistent launches in
 * the current window (n >= nwg doubles).  max/avg of these is the workgroup
 * imbalance of the persistent kernel. */
int lb_wg_busy(lb_ctx *ctx, double *out, int32_t n);

/* Synchronize and copy the timeline of the last persistent launch: 4 doubles
 * per workgroup (n >= 4*nwg), in microseconds from the earliest workgroup
 * start: start, first item start, last item end, exit. */
int lb_wg_timeline(lb_ctx *ctx, double *out, int32_t n);

/* Synchronize and copy per-tile-row visit counts since the last reset (n >= nrows
 * int32, tiles in chunk order, rows top to bottom); every row is computed
 * exactly once per step.  reset != 0 zeroes them. */
int lb_visits(lb_ctx *ctx, int32_t *out, int32_t n, int32_t reset);

/* Synchronize and copy the per-step FP64 sums of all cells of the last
 * min(n, 1024, steps) steps, oldest first.  Returns the count in *got. */
int lb_checksums(lb_ctx *ctx, double *out, int32_t n, int32_t *got);

/* The balancers of Section VI (Experiment A: GreedyLB; Experiments B and C:
 * RefineSwapLB and the Greedy-then-RefineSwap policy) without a GPU or a
 * context: the same computation lb_rebalance uses.  loads: C doubles >= 0;
 * old_map: C slot indices in [0, S), or NULL for LB_GREEDY (then *nmigrated
 * counts chunks off the block map); map_out: C int32, caller-allocated.
 * LB_GREEDY_THEN_REFINESWAP runs Greedy when old_map is NULL (a first call)
 * and RefineSwap from old_map otherwise.  Errors: LB_E_INVAL (bad sizes,
 * loads, threshold or map entries). */
int lb_balance_host(const double *loads, const int32_t *old_map, int32_t C, int32_t S,
                    int32_t strategy, double threshold, int32_t *map_out, int32_t *nmigrated);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the FP64 checksum of
 * lb_fields (the same two-pass, fixed-order sum, so the same bits) of a field
 * the caller owns, without a context.  Its partial sums live in a fixed
 * 8 KiB device array of the library (1024 doubles per GPU, held until the
 * process ends), whose address is resolved at lb_grid_init or at this call's
 * first use on a device; the call itself allocates nothing and does not
 * synchronize.  field: ncells values (float for LB_FP32 and LB_FP32_KAHAN,
 * double for LB_FP64) in device memory; sum_out: one double the device can
 * write (device memory or mapped pinned host memory), written when the work
 * enqueued on hip_stream (NULL: the null stream) of the current device
 * completes.  Calls that overlap on one GPU share the array and race: order
 * them on one stream.  Errors: LB_E_INVAL (NULL pointers, unknown precision,
 * ncells < 0 or > LB_NOALLOC_MAX_CELLS), LB_E_HIP (launch failure). */
#define LB_NOALLOC_MAX_CELLS ((int64_t)1 << 40)
int lb_field_sum_noalloc(const void *field, int32_t precision, int64_t ncells, double *sum_out,
                         void *hip_stream);

/* Release the context (synchronizes its stream first).  NULL is a no-op. */
void lb_destroy(lb_ctx *ctx);

/* Last error message of ctx, or of the calling thread when ctx is NULL. */
const char *lb_last_error(const lb_ctx *ctx);

/* LB_ABI_VERSION of the built library. */
int lb_abi_version(void);

/* sizeof(lb_config) and sizeof(lb_stats_t) as compiled into the library, so that
 * bindings can check their struct layouts. */
size_t lb_config_bytes(void);
size_t lb_stats_bytes(void);

#ifdef __cplusplus
}
#endif
#endif /* LBGRID_H */
