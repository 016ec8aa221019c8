// Launch interface of the HIP kernels (used by the C ABI in pc_host.cpp).
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>
#include "pc_entries.h"
#include "pc_internal.h"

namespace pc {

struct DevPlan {
    const Item* items;
    int n_items;
    const Item* items_ord[2];       // the items in the canonical summation order (forward, adjoint), d <= 2
    const Item3* items3;            // 3-D operators
    int n_items3;
    int rows, cols;                 // 2-D view of Omega (reduction)
    int planes, prow;               // Omega as planes x prow x cols
    const void* spec;               // complex dtype
    const void* wts;                // dtype
    const void* tw;                 // complex dtype
    const Tile* tiles_fwd;
    const Tile* tiles_adj;
    int n_tiles_fwd, n_tiles_adj;
    const Box* cboxes_fwd;          // staging box of every tile contributor
    const Box* cboxes_adj;
    int64_t slot_fwd, slot_adj;     // staging elements per vector
    int max_lds;
    int conv_threads;               // 1-D/2-D convolution workgroup size (1024 or 512)
    int max_lds_axis;               // 3-D axis-0 kernel
    int dtype;                      // 0 = f32, 1 = f64
    // staged FP32 launches in two parts: the items whose LDS fits twice in a
    // CU (kSmallItemLds) run as 512-thread workgroups, two per CU, after the
    // others; items_split holds the others, then those (n_big + n_small)
    const Item* items_split;
    int n_big, n_small;
    int lds_big, lds_small;         // LDS bytes of the two launches
    int* queue;                     // persistent launches: 8 XCD counters, 16 ints apart
    int n_cu;                       // compute units of the device
};

// One 3-D launch set (plane-forward, axis-0, plane-inverse) over items
// [item_lo, item_hi) and B vectors; the grids cover max_gather / max_write
// planes and max_tiles column tiles per item.
struct Conv3Launch {
    bool adjoint;
    int item_lo, item_hi, B;
    const void* in;
    int64_t ld_in;
    void* slots;
    int64_t slot_stride;
    void* scratch;
    int64_t scratch_base;
    int max_gather, max_write, max_tiles;
};

// Timing events of a launch, carried by its own dispatch packets (the start
// event by the first kernel, the stop event by the last), so that timing adds
// no marker packets to the stream; both null for an untimed launch.  A launch
// with no work records both as plain events on its stream.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};

// Convolution items (one workgroup per item and vector): items[item_lo,
// item_hi) of the given array (the plain mode launches one item at a time),
// B vectors starting at 'in'.  With out null the written boxes go to
// staging; otherwise they are added into the B outputs at out (stride ldo),
// which is only race-free and deterministic for items of one colour.
// item_major: staged launches deal the blocks item-major over the XCDs
// instead of whole items per XCD (the same results).
hipError_t launch_conv(const DevPlan& P, const Item* items, bool adjoint, int item_lo, int item_hi, int B,
                       const void* in, int64_t ld_in, void* slots, int64_t slot_stride, void* out, int64_t ldo,
                       hipStream_t s, bool item_major = false, LaunchEvents ev = {});

// Staged launch of all items in persistent form (fixed grid, per-XCD unit
// queues at P.queue, cleared on s first): the same staging boxes as
// launch_conv with out null.  persistent_fits: whether the item data leaves
// room in LDS for the queue slot (else launch_conv_persistent refuses).
bool persistent_fits(const DevPlan& P);
hipError_t launch_conv_persistent(const DevPlan& P, bool adjoint, int B, const void* in, int64_t ld_in, void* slots,
                                  int64_t slot_stride, hipStream_t s);

// Staged FP32 launch of all items in two parts (see DevPlan::items_split):
// the same staging boxes as launch_conv with out null.
hipError_t launch_conv_split(const DevPlan& P, bool adjoint, int B, const void* in, int64_t ld_in, void* slots,
                             int64_t slot_stride, hipStream_t s, LaunchEvents ev = {});

// out[b * ld + i] = 0 for b < B, i < N.
hipError_t launch_fill_zero(int dtype, void* out, int64_t ld, int64_t N, int B, hipStream_t s);

// 3-D convolution items -> staging (three kernels, see pc_phases3.h).
hipError_t launch_conv3(const DevPlan& P, const Conv3Launch& L, hipStream_t s);

// Deterministic reduction of the staging boxes into the outputs (out = sum,
// or out += alpha * sum with accumulate).
hipError_t launch_reduce(const DevPlan& P, bool adjoint, int B, const void* slots, int64_t slot_stride,
                         void* out, int64_t ldo, hipStream_t s, bool accumulate = false, double alpha = 1.0,
                         LaunchEvents ev = {});

// Estimator: per-leaf (leaf_box [L][6]) FP64 sums of squares of (Yt - Y) over q vectors into
// leaf_sq, and the totals sum (Yt - Y)^2 and sum Y^2 into totals[2] (through n_part
// row-block partials, summed in order).
hipError_t launch_est(int dtype, const int32_t* leaf_box, int n_leaves, int q,
                      const void* Yt, int64_t ldt, const void* Y, int64_t ldy,
                      int planes, int prow, int cols, double* leaf_sq, double* partials, int n_part,
                      double* totals, hipStream_t s);

// Matrix entries out[i] = A~[ys[i], xs[i]] (device int64 [n][d] coordinates).
hipError_t launch_entries(const EntryTables& E, int dtype, const void* wts, const void* phiE, int64_t n,
                          const int64_t* ys, const int64_t* xs, void* out, hipStream_t s);

hipError_t set_kernel_attributes();

// Work area of the allocation-free entry point (pc_apply_batch_noalloc):
// kNoAllocBytes of device memory per device, shared by every operator on
// that device.  noalloc_area_init(device) looks up the area's device
// address with 'device' current (once per device; later calls return at
// once); noalloc_area(device) returns it, or null before the lookup.
constexpr size_t kNoAllocBytes = size_t(128) << 20;
hipError_t noalloc_area_init(int device);
void* noalloc_area(int device);

}  // namespace pc
