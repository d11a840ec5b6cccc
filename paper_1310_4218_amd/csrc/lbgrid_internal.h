// Internal declarations shared by the kernels (kernels.hip), the host runtime
// (runtime.cpp) and the host balancer (balance.cpp).  Not part of the ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace lbgrid {

constexpr int kMaxHot = 4;
constexpr int kHistLen = 1024;      // per-step checksum ring
constexpr int kSumBlocks = 1024;    // first pass of the field sum
constexpr int kRingRows = 4;        // LDS row ring of the tile kernel
constexpr int kMaxBlock = 1024;
constexpr int kMaxBlockDeep = 512;  // workgroup limit of the 4- and 8-row register pipelines
constexpr size_t kMaxLds = 160 * 1024;  // gfx950: 160 KiB of LDS per CU
// Busy-time slots of a launch of one workgroup per item: one per compute unit,
// keyed by XCD (3 bits) and the unit's shader-engine/array/CU id (8 bits).
constexpr int kCuSlots = 2048;

// Checksum partial buffers and shared step-state copies are kept per step
// mod kStepSlots: a launch writes those of its own steps (one, or up to three
// when it fuses steps) and never those of the launch before it, so the slots
// must cover two launches of the most steps.
constexpr int kStepSlots = 8;
constexpr int kSlotMask = kStepSlots - 1;

// Device control block (first bytes of the workspace).
struct Ctrl {
    uint32_t nitems;        // work items of the installed plan
    uint32_t pad0;
    // The checksum partials of a step are summed during a later launch (or by
    // k_flush): pend_step[b] = 1 + the step whose partials buffer b holds, 0
    // once they are summed; pend_n[b] = the items that wrote it.
    uint64_t pend_step[kStepSlots];
    uint32_t pend_n[kStepSlots];
    uint64_t pad1[2];
};

// What each workgroup of the persistent launch carries from one step to the
// next (all workgroups hold the same values between launches): the steps done
// and the hotspot centres of the next step, so that a launch needs one small
// load and no division to know its step.
struct alignas(64) WgState {
    uint64_t step;
    int32_t hx[kMaxHot], hy[kMaxHot];
    int32_t cur;            // field copy (0 or 1) holding the values this step reads
};

// One work item: a range of rows of one tile, self-contained so that a claim
// needs a single dependent load.
struct alignas(16) ItemDesc {
    int32_t x0, y0;         // first column and first row of the item
    int32_t wh;             // columns | rows << 16
    int32_t chunk;
    int32_t id;             // index in chunk order (its checksum partial); -1 = none
    int32_t vbase;          // visit counter of the item's first row
    int32_t tile;           // the tile the rows belong to (its measured work)
    int32_t pad1;
};

// Kernel arguments: every pointer is device memory inside the caller's buffers.
struct DevArgs {
    void* field0;
    void* field1;
    const int32_t* ktab;
    const ItemDesc* items;     // items in chunk order
    const int32_t* item_off;   // C + 1: items of chunk c are [item_off[c], item_off[c+1])
    const ItemDesc* queue;     // the same items grouped by queue, each queue's in cost order
    const int32_t* seg;        // Q + 1 offsets into queue
    const ItemDesc* firstd;    // 2 x nwg: the first two items of each workgroup in a step
                               // (id -1: none)
    int32_t* heads;            // 2 x Q claim counters, one set per step parity; a step finds
                               // its set at head0 and resets the other set for the next step
    WgState* wstate;           // nwg: step and hotspot centres, kept by each workgroup
    WgState* pstate;           // kStepSlots, by step mod kStepSlots: the state of a step whose launch
                               // form reads one shared copy (one workgroup per item); every
                               // form writes the copy of the step after its own
    Ctrl* ctrl;
    double* loads_work;        // C
    double* loads_time;        // C
    double* tile_work;         // ntiles: work units of each tile (rebuilds items from it)
    double* partials;          // kStepSlots x part_stride, by step mod kStepSlots: per item, the sum
                               // of its outputs in that step
    double* hist;              // kHistLen per-step sums
    double* wg_busy;           // nwg (persistent: per workgroup), or kCuSlots (one workgroup
                               // per item: per compute unit)
    uint64_t* wg_timeline;     // 4 per workgroup, last persistent launch: start, first item,
                               // end of last item, exit (wall-clock ticks)
    int32_t* visits;           // per tile row: times it was computed
    int64_t ncells;            // cells per field
    int32_t part_stride;       // items a partials buffer can hold
    int32_t nx, ny, nz, nfields;
    int32_t nqueues, nwg, steal;
    int32_t head0;             // 2G: the first 2G items of a queue go two to each of its workgroups
    int32_t tile_x;            // TX
    int32_t tile_y;            // TY (the trip-count buffers hold TX * TY entries)
    int32_t block;             // threads per workgroup = TX * nz / V (== blockDim.x)
    int32_t block2;            // threads per workgroup of the two-step item launch
    int32_t block3;            // ... of the three-step item launch
    int32_t stage_rows;        // > 0: rows per direct global->LDS batch (V = 4 only); 0: registers
    int32_t reg_depth;         // register pipeline: rows in flight (2, 4 or 8; 2 unless V = 4)
    int32_t march;             // > 0: column-march pipeline with this many rows in flight (2, 4, 8)
    int32_t item_grid;         // 1: a balanced step launches one workgroup per item (queue order)
    int32_t stream_store;      // 1: the march writes its output non-temporally (both field
                               // copies exceed the 256 MB last-level cache)
    uint32_t field_bytes;      // bytes of one field (< 4 GiB with the march pipeline)
    int32_t vertical;          // 1: column physics with the vertical dependency
    int32_t col_per_wave;      // > 0: the march puts this many whole columns in each wave
                               // (vertical physics with nz / V not dividing 64); 0: dense
    int32_t col_per_wave2;     // the same for the two-step launch, whose V may differ
    int32_t r2cut;
    int32_t kmin;
    int32_t alpha;
    int32_t nhot;
    int32_t xcd_queues;        // 1: queue q is served by workgroups on XCD q % 8
    int32_t hx_first[kMaxHot], hy_first[kMaxHot];  // hotspot centres at step 0 (t = t0)
    int32_t hvx[kMaxHot], hvy[kMaxHot];             // cells per step, reduced to [0, nx), [0, ny)
    double cc, cn, eps;
};

// One segment of a table upload: `words` 32-bit words from src (pinned host
// memory as the device addresses it) to dst (device memory).
struct GatherSeg {
    const uint32_t* src;
    uint32_t* dst;
    uint32_t words;
};
constexpr int kMaxGather = 8;

// Kernel launchers (kernels.hip).  prec: 0 FP32, 1 FP32 Kahan, 2 FP64.
int  launch_persistent(const DevArgs& a, int prec, int vec, int nwg, int block, size_t lds,
                       void* stream);
int  launch_plain_chunk(const DevArgs& a, int prec, int vec, int chunk, int nitems_chunk,
                        int block, size_t lds, void* stream);
// One workgroup per item of the installed plan (nitems of them, in queue order);
// slot is the step's number mod kStepSlots (steps enqueued so far).
int  launch_items(const DevArgs& a, int prec, int vec, int nitems, int block, size_t lds, int slot,
                  void* stream);
// The same with two steps per launch (temporal blocking): slot is the number mod kStepSlots
// of the first of them, block the threads of a two-step workgroup (a.block2).
int  launch_items2(const DevArgs& a, int prec, int vec, int nitems, int block, size_t lds, int slot,
                   void* stream);
// Three steps per launch.
int  launch_items3(const DevArgs& a, int prec, int vec, int nitems, int block, size_t lds, int slot,
                   void* stream);
// Copy the shared state of the step in slot (its number mod kStepSlots) into every
// workgroup's own copy.
int  launch_seed_state(const DevArgs& a, int slot, void* stream);
int  launch_finish(const DevArgs& a, void* stream);
int  launch_flush(const DevArgs& a, void* stream);
int  launch_gather(const GatherSeg* segs, int n, void* stream);   // n <= kMaxGather
// loads (C) and tile work (ntiles) to pinned host memory, then clear_bytes of
// counters from `clear` (0 bytes: keep them)
int  launch_measure_out(double* loads, double* tiles, int C, int ntiles, double* out_loads,
                        double* out_tiles, void* clear, size_t clear_bytes, void* stream);
int  launch_init_field(void* q, int prec, int64_t n, uint64_t seed, void* stream);
int  launch_zero(void* p, size_t bytes, void* stream);
int  launch_field_sum(const void* q, int prec, int64_t n, double* partial, double* out,
                      void* stream);
int  launch_reset_control(const DevArgs& a, void* stream);
int  persistent_occupancy(const DevArgs& a, int prec, int vec, int block, size_t lds);  // per CU

// The allocation-free checksum entry point's scratch (kernels.hip): resolve the
// device address of `device`'s copy (with that device current); 0 or a hipError_t.
int  prepare_static_scratch(int device);
// Record msg as the calling thread's last error and return code (runtime.cpp).
int  report_error(int code, const char* msg);

// Host balancer (balance.cpp).  Return 0 on success, -1 on bad arguments.
enum Strategy { kGreedy = 0, kRefine = 1, kRefineSwap = 2 };
int balance(const double* w, const int32_t* old_map, int32_t C, int32_t S, int strategy,
            double threshold, int32_t* map_out);
void block_map(int32_t C, int32_t S, int32_t* map_out);
double imbalance(const double* w, const int32_t* map, int32_t C, int32_t S);

}  // namespace lbgrid
