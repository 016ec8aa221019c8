// C ABI of the product-convolution library (declared in include/pc.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/pc.h"
#include "pc_kernels.h"
#include "pc_phases3.h"
#include "pc_plan.h"

namespace {

thread_local std::string g_err;

pc_status fail(pc_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

pc_status hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? PC_ERR_OOM : PC_ERR_DEVICE;
}

// The staging buffer holds at most this many bytes (split in two halves when
// the reduction of one vector chunk overlaps the next chunk's convolution).
constexpr size_t kSlotCapBytes = size_t(2) << 30;
constexpr int64_t kMinChunks = 4;
// 3-D operators: default staging cap of one vector chunk (a 128^3 vector
// stages about 0.7 GB in FP32), and default scratch bytes of one item group
// (all vectors of a chunk), the plane spectra between the three kernels of
// the group, by dtype (the faster sizes on the 128^3 blur: 1 GiB in FP32,
// 256 MiB in FP64).
constexpr size_t kSlotCapBytes3 = size_t(8) << 30;
constexpr size_t kScratchCapBytesF32 = size_t(1) << 30;
constexpr size_t kScratchCapBytesF64 = size_t(256) << 20;
// Colour launches: most streams that vector chunks run on at once.
constexpr int kMaxLanes = 4;

}  // namespace

struct pc_op {
    pc::Plan plan;
    pc::DevPlan dev{};
    int device = 0;
    size_t esz = 4;
    std::vector<void*> allocs;
    size_t resident = 0;
    void* slots = nullptr;        // two staging buffers of slots_bytes / 2 each
    size_t slots_bytes = 0;
    int64_t tune_chunk = 0;       // 0: default chunking
    int64_t tune_scratch = 0;     // 3-D: scratch bytes per item group, 0: default
    void* scratch = nullptr;      // 3-D plane spectra of one item group
    size_t scratch_bytes = 0;
    bool tune_overlap = false;    // reduce on the aux stream while the next chunk convolves
    bool tune_direct = false;     // d <= 2: colour launches add into the outputs (no staging)
    int tune_streams = 4;         // colour launches: vector chunks run on this many streams at once
    bool tune_persistent = false; // staged 1-D/2-D applies: persistent convolution launches
    bool tune_item_major = false; // staged 1-D/2-D applies: item-major block order over the XCDs
    bool tune_split = true;       // staged FP32 applies: small items two workgroups per CU
    hipStream_t lanes[kMaxLanes] = {};       // the library's streams of the colour launches
    hipEvent_t lane_done[kMaxLanes] = {};    // end of each lane's work in the current call
    hipEvent_t fork = nullptr;               // start of the current call on the caller's stream
    hipStream_t aux = nullptr;    // reductions overlap the next chunk's convolution here
    hipEvent_t ev_conv[2] = {nullptr, nullptr};
    hipEvent_t ev_red[2] = {nullptr, nullptr};
    void* work = nullptr;     // estimator: Y~ and (if needed) Y
    size_t work_bytes = 0;
    double* est = nullptr;    // estimator sums
    size_t est_bytes = 0;
    int32_t* leaf_box = nullptr;   // [L][6] leaf boxes, device
    void* d_wts = nullptr;         // weight tables (dtype), device
    // block applies: per-call tables and the event of the last call using them
    void* blk = nullptr;
    size_t blk_bytes = 0;
    hipEvent_t blk_done = nullptr;
    // the end of the last call that used the work buffers above (stream order
    // for releasing a buffer that has to grow); budget: cap on their bytes
    hipEvent_t last_use = nullptr;
    bool last_use_set = false;
    size_t budget = 0;
    // matrix entries: tables uploaded on the first pc_entries call
    bool ent_ready = false;
    pc::EntryTables ent{};
    void* ent_phiE = nullptr;
    // profiling: event pairs of launches not yet read
    bool profiling = false;
    int64_t dbg_first = 0, dbg_count = 0, dbg_seen = 0;   // injected launch failures (test hook)
    struct Timed {
        hipEvent_t a, b;
        int kind;        // 0 conv, 1 reduce
        int vectors;
    };
    std::vector<Timed> timed;
    std::vector<hipEvent_t> event_pool;

    ~pc_op() {
        for (int i = 0; i < 2; ++i) {
            if (ev_conv[i]) hipEventDestroy(ev_conv[i]);
            if (ev_red[i]) hipEventDestroy(ev_red[i]);
        }
        if (aux) hipStreamDestroy(aux);
        for (auto& t : timed) {
            hipEventDestroy(t.a);
            hipEventDestroy(t.b);
        }
        for (hipEvent_t e : event_pool) hipEventDestroy(e);
        for (int i = 0; i < kMaxLanes; ++i) {
            if (lanes[i]) hipStreamDestroy(lanes[i]);
            if (lane_done[i]) hipEventDestroy(lane_done[i]);
        }
        if (fork) hipEventDestroy(fork);
        for (void* p : allocs) hipFree(p);
        if (slots) hipFree(slots);
        if (scratch) hipFree(scratch);
        if (blk) hipFree(blk);
        if (blk_done) hipEventDestroy(blk_done);
        if (last_use) hipEventDestroy(last_use);
        if (work) hipFree(work);
        if (est) hipFree(est);
    }
};

namespace {

// Operator data: allocated once, copied on stream s (finished before the
// host array may go away).
template <class V>
pc_status upload(pc_op* op, const V& host, void** dptr, hipStream_t s) {
    size_t bytes = host.size() * sizeof(host[0]);
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(dptr, bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc (operator data)");
    op->allocs.push_back(*dptr);
    op->resident += bytes;
    if (!host.empty()) {
        e = hipMemcpyAsync(*dptr, host.data(), host.size() * sizeof(host[0]), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync (operator data)");
    }
    return PC_OK;
}

pc_status upload_real(pc_op* op, const std::vector<double>& v, void** dptr, hipStream_t s) {
    if (op->plan.dtype == PC_F64) return upload(op, v, dptr, s);
    std::vector<float> f(v.size());
    for (size_t i = 0; i < v.size(); ++i) f[i] = (float)v[i];
    return upload(op, f, dptr, s);
}

// True while s records a graph (stream capture).
bool capturing(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

// Bytes of the work buffers the operator holds (grown by calls, kept until
// pc_destroy).
size_t work_buffer_bytes(const pc_op* op) {
    return op->slots_bytes + op->scratch_bytes + op->work_bytes + op->est_bytes + op->blk_bytes;
}

// Grows one of the operator's work buffers to at least 'need' bytes, in
// stream order on s: the old buffer is released on s after the end of the
// last call that used the work buffers (an event, so neither the host nor
// other streams wait) and the new one is allocated on s.  Refused under
// stream capture (PC_ERR_ARG) and beyond the operator's work-buffer budget
// (PC_ERR_BUDGET), in both cases before anything is enqueued.
pc_status ensure(pc_op* op, void** buf, size_t* have, size_t need, const char* what, hipStream_t s) {
    if (*have >= need) return PC_OK;
    if (capturing(s))   // growing would allocate inside the capture
        return fail(PC_ERR_ARG, std::string(what) + ": the buffer is smaller than this call needs; make one call "
                                                    "of at least this size before the stream capture");
    if (op->budget > 0 && work_buffer_bytes(op) - *have + need > op->budget)
        return fail(PC_ERR_BUDGET, std::string(what) + ": " + std::to_string(need) +
                                       " bytes would take the operator's work buffers to " +
                                       std::to_string(work_buffer_bytes(op) - *have + need) + " bytes, above its budget of " +
                                       std::to_string(op->budget));
    hipError_t e;
    if (*buf) {
        if (op->last_use_set) {
            e = hipStreamWaitEvent(s, op->last_use, 0);
            if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
        }
        e = hipFreeAsync(*buf, s);
        if (e != hipSuccess) return hip_fail(e, "hipFreeAsync");
        *buf = nullptr;
        *have = 0;
    }
    e = hipMallocAsync(buf, need, s);
    if (e != hipSuccess) return hip_fail(e, what);
    *have = need;
    return PC_OK;
}

// Records the end of a call that used the work buffers (not under capture:
// a replayed graph is ordered by its caller, as the header states).
pc_status mark_used(pc_op* op, hipStream_t s) {
    if (capturing(s)) return PC_OK;
    hipError_t e;
    if (!op->last_use) {
        e = hipEventCreateWithFlags(&op->last_use, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreateWithFlags");
    }
    e = hipEventRecord(op->last_use, s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    op->last_use_set = true;
    return PC_OK;
}

hipEvent_t get_event(pc_op* op) {
    if (!op->event_pool.empty()) {
        hipEvent_t e = op->event_pool.back();
        op->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records the start event of a timed launch (no-op when not profiling).
void prof_begin(pc_op* op, hipStream_t s, hipEvent_t* ev) {
    *ev = nullptr;
    if (!op->profiling || capturing(s)) return;   // no event nodes in a captured graph
    *ev = get_event(op);
    if (*ev) hipEventRecord(*ev, s);
}

void prof_end(pc_op* op, hipStream_t s, hipEvent_t start, int kind, int vectors) {
    if (!op->profiling || !start) return;
    hipEvent_t e = get_event(op);
    if (!e) return;
    hipEventRecord(e, s);
    op->timed.push_back({start, e, kind, vectors});
}

// Events for a launch that carries its own timing (pc::LaunchEvents: no
// marker packets between the kernels); both null when not profiling or
// under capture.  prof_take registers them once the launch is enqueued,
// prof_drop returns them to the pool when it failed.
pc::LaunchEvents prof_events(pc_op* op, hipStream_t s) {
    pc::LaunchEvents ev;
    if (!op->profiling || capturing(s)) return ev;
    ev.start = get_event(op);
    ev.stop = ev.start ? get_event(op) : nullptr;
    if (ev.start && !ev.stop) {
        op->event_pool.push_back(ev.start);
        ev.start = nullptr;
    }
    return ev;
}

void prof_take(pc_op* op, const pc::LaunchEvents& ev, int kind, int vectors) {
    if (ev.start && ev.stop) op->timed.push_back({ev.start, ev.stop, kind, vectors});
}

void prof_drop(pc_op* op, const pc::LaunchEvents& ev) {
    if (ev.start) op->event_pool.push_back(ev.start);
    if (ev.stop) op->event_pool.push_back(ev.stop);
}

// Test hook: the operator's convolution launches numbered dbg_first ..
// dbg_first + dbg_count - 1 (counted from the last pc_debug_fail_launches)
// fail before anything of theirs is enqueued.
bool injected_failure(pc_op* op) {
    if (op->dbg_count <= 0) return false;
    const int64_t k = ++op->dbg_seen;
    return k >= op->dbg_first && k < op->dbg_first + op->dbg_count;
}
pc_status injected(void) { return fail(PC_ERR_DEVICE, "injected launch failure (pc_debug_fail_launches)"); }

pc_status check_op(const pc_op* op) {
    if (!op) return fail(PC_ERR_ARG, "null operator");
    return PC_OK;
}

pc_status ensure_aux(pc_op* op) {
    if (op->aux) return PC_OK;
    hipError_t e = hipStreamCreateWithFlags(&op->aux, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
    for (int i = 0; i < 2; ++i) {
        e = hipEventCreateWithFlags(&op->ev_conv[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&op->ev_red[i], hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreateWithFlags");
    }
    return PC_OK;
}

// Caller-supplied work buffers (the allocation-free entry point): staging of
// 'chunk' vectors at 'slots', then 3-D scratch of at most scratch_cap bytes.
struct ExtBufs {
    void* slots;
    int64_t chunk;
    void* scratch;
    size_t scratch_cap;
};

// 3-D: vector chunks sized by the staging buffer; within a chunk, contiguous
// item groups sized by the scratch buffer each run the three kernels of
// pc_phases3.h; one reduction per chunk.  items: host copy of the items Dc
// points to (the operator's, or a block apply's); Dr: the reduction tables.
// ext: null, or buffers to use instead of the operator's (nothing is
// allocated then; PC_ERR_UNSUPPORTED if one item's scratch exceeds them).
pc_status run_3d(pc_op* op, const std::vector<pc::Item3>& items, const pc::DevPlan& Dc, const pc::DevPlan& Dr,
                 int64_t per, bool adj, bool plain, int64_t B, const void* U, int64_t ldu, void* OUT, int64_t ldo,
                 hipStream_t s, bool acc, double alpha, const ExtBufs* ext = nullptr) {
    const pc::Plan& P = op->plan;
    const size_t per_bytes = (size_t)std::max<int64_t>(per, 1) * op->esz;
    const size_t cx_bytes = 2 * op->esz;
    int64_t chunk = 1;
    if (ext) {
        chunk = std::min<int64_t>(ext->chunk, B);
    } else if (!plain) {
        // an explicit chunk overrides the default staging cap
        const int64_t cap = (int64_t)std::max<size_t>(1, kSlotCapBytes3 / per_bytes);
        chunk = op->tune_chunk > 0 ? std::min<int64_t>(op->tune_chunk, B) : std::min<int64_t>(cap, B);
    }
    const size_t scap_default = P.dtype == PC_F64 ? kScratchCapBytesF64 : kScratchCapBytesF32;
    const size_t scap = ext ? ext->scratch_cap : op->tune_scratch > 0 ? (size_t)op->tune_scratch : scap_default;
    const int n = (int)items.size();
    const int cols = pc::axis_cols(P.dtype);
    auto scratch_of = [&](int i) { return items[(size_t)i].scratch_off; };
    auto scratch_end = [&](int i) {
        const pc::Item3& I = items[(size_t)i];
        return I.scratch_off + (int64_t)I.nz * I.p.n0 * (I.p.m + 1);
    };
    // item groups for chunk vectors (smaller chunks reuse them)
    std::vector<pc::Conv3Launch> groups;
    size_t scratch_need = 0;
    for (int i = 0; i < n;) {
        int j = i + 1;
        if (!plain)
            while (j < n && (size_t)(scratch_end(j) - scratch_of(i)) * (size_t)chunk * cx_bytes <= scap) ++j;
        pc::Conv3Launch L{};
        L.adjoint = adj;
        L.item_lo = i;
        L.item_hi = j;
        L.scratch_base = scratch_of(i);
        for (int k = i; k < j; ++k) {
            const pc::Item3& I = items[(size_t)k];
            const pc::Planes pl = pc::planes_of(I, adj);
            L.max_gather = std::max(L.max_gather, pl.s_n);
            L.max_write = std::max(L.max_write, pl.d_n);
            L.max_tiles = std::max(L.max_tiles, (int)(((int64_t)I.p.n0 * (I.p.m + 1) + cols - 1) / cols));
        }
        scratch_need = std::max(scratch_need, (size_t)(scratch_end(j - 1) - scratch_of(i)) * (size_t)chunk * cx_bytes);
        groups.push_back(L);
        i = j;
    }
    void* slots = nullptr;
    void* scratch = nullptr;
    if (ext) {
        if (scratch_need > ext->scratch_cap)
            return fail(PC_ERR_UNSUPPORTED, "one 3-D work item needs " + std::to_string(scratch_need) +
                                                " bytes of plane scratch; the allocation-free work area leaves " +
                                                std::to_string(ext->scratch_cap));
        slots = ext->slots;
        scratch = ext->scratch;
    } else {
        pc_status st = ensure(op, &op->slots, &op->slots_bytes, (size_t)chunk * per_bytes, "hipMallocAsync (staging)", s);
        if (st != PC_OK) return st;
        st = ensure(op, &op->scratch, &op->scratch_bytes, std::max<size_t>(scratch_need, 16),
                    "hipMallocAsync (3-D scratch)", s);
        if (st != PC_OK) return st;
        slots = op->slots;
        scratch = op->scratch;
    }
    const char* u = static_cast<const char*>(U);
    char* o = static_cast<char*>(OUT);
    for (int64_t b0 = 0; b0 < B; b0 += chunk) {
        const int nb = (int)std::min<int64_t>(chunk, B - b0);
        const void* in = u + (size_t)b0 * ldu * op->esz;
        void* out = o + (size_t)b0 * ldo * op->esz;
        hipError_t e;
        hipEvent_t ev;
        for (size_t g = 0; g < groups.size(); ++g) {
            pc::Conv3Launch L = groups[g];
            L.B = nb;
            L.in = in;
            L.ld_in = ldu;
            L.slots = slots;
            L.slot_stride = per;
            L.scratch = scratch;
            if (injected_failure(op)) return injected();
            prof_begin(op, s, &ev);
            e = pc::launch_conv3(Dc, L, s);
            if (e != hipSuccess) return hip_fail(e, "3-D conv launch");
            prof_end(op, s, ev, 0, g == 0 ? nb : 0);
        }
        prof_begin(op, s, &ev);
        e = pc::launch_reduce(Dr, adj, nb, slots, per, out, ldo, s, acc, alpha);
        if (e != hipSuccess) return hip_fail(e, "reduce launch");
        prof_end(op, s, ev, 1, nb);
    }
    return PC_OK;
}

pc_status run_batch_3d(pc_op* op, bool adj, bool plain, int64_t B, const void* U, int64_t ldu, void* OUT, int64_t ldo,
                       hipStream_t s, bool acc, double alpha) {
    const int64_t per = adj ? op->plan.slot_adj : op->plan.slot_fwd;
    return run_3d(op, op->plan.items3, op->dev, op->dev, per, adj, plain, B, U, ldu, OUT, ldo, s, acc, alpha);
}

// d <= 2, colour launches: each vector chunk's outputs are zeroed, then the
// items of each colour (pairwise disjoint written boxes) add their boxes
// straight into the outputs, colour after colour, so every output point sums
// its contributions in the canonical (colour, item) order - the order the
// staged reduction uses.  The order only binds within a vector: chunks of
// vectors run their colour sequences on up to tune_streams library streams
// at once (forked from and joined back into s with events), so the tail of
// one chunk's colour launch overlaps the next launches of the others.  No
// work buffer is needed.
pc_status lane_streams(pc_op* op, int n) {
    for (int i = 0; i < n; ++i) {
        hipError_t e = hipSuccess;
        if (!op->lanes[i]) e = hipStreamCreateWithFlags(&op->lanes[i], hipStreamNonBlocking);
        if (e == hipSuccess && !op->lane_done[i]) e = hipEventCreateWithFlags(&op->lane_done[i], hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "library stream setup");
    }
    if (!op->fork) {
        hipError_t e = hipEventCreateWithFlags(&op->fork, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreateWithFlags");
    }
    return PC_OK;
}

pc_status run_direct(pc_op* op, bool adj, int64_t B, const void* U, int64_t ldu, void* OUT, int64_t ldo,
                     hipStream_t s, int max_lanes = kMaxLanes) {
    const pc::Plan& P = op->plan;
    const std::vector<int32_t>& cbeg = adj ? P.cbeg_adj : P.cbeg_fwd;
    const pc::Item* items = op->dev.items_ord[adj ? 1 : 0];
    const int lanes_want = std::max(1, std::min(op->tune_streams, max_lanes));
    int64_t chunk = op->tune_chunk > 0 ? op->tune_chunk : (B + lanes_want - 1) / lanes_want;
    chunk = std::max<int64_t>(1, std::min<int64_t>(chunk, B));
    const int64_t nchunks = (B + chunk - 1) / chunk;
    const int lanes = (int)std::min<int64_t>(lanes_want, nchunks);
    const bool cap = capturing(s);
    if (lanes > 1) {
        if (cap && !op->lanes[lanes - 1])
            return fail(PC_ERR_ARG, "make one call with this stream setting before the stream capture");
        pc_status st = lane_streams(op, lanes);
        if (st != PC_OK) return st;
    }
    hipEvent_t ev_all;
    prof_begin(op, s, &ev_all);   // one span: the colour launches of all lanes
    hipError_t e;
    if (lanes > 1) {
        e = hipEventRecord(op->fork, s);
        for (int i = 0; i < lanes && e == hipSuccess; ++i) e = hipStreamWaitEvent(op->lanes[i], op->fork, 0);
        if (e != hipSuccess) return hip_fail(e, "stream fork");
    }
    const char* u = static_cast<const char*>(U);
    char* o = static_cast<char*>(OUT);
    pc_status st = PC_OK;
    for (int64_t k = 0; k < nchunks && st == PC_OK; ++k) {
        const int64_t b0 = k * chunk;
        const int nb = (int)std::min<int64_t>(chunk, B - b0);
        hipStream_t ls = lanes > 1 ? op->lanes[k % lanes] : s;
        const void* in = u + (size_t)b0 * ldu * op->esz;
        void* out = o + (size_t)b0 * ldo * op->esz;
        e = pc::launch_fill_zero(P.dtype, out, ldo, P.N, nb, ls);
        if (e != hipSuccess) st = hip_fail(e, "fill launch");
        for (size_t c = 0; c + 1 < cbeg.size() && st == PC_OK; ++c) {
            if (injected_failure(op)) {
                st = injected();
                break;
            }
            e = pc::launch_conv(op->dev, items, adj, cbeg[c], cbeg[c + 1], nb, in, ldu, nullptr, 0, out, ldo, ls);
            if (e != hipSuccess) st = hip_fail(e, "conv launch");
        }
    }
    if (lanes > 1) {   // join every lane, also after a failure, so s orders all work enqueued
        for (int i = 0; i < lanes; ++i) {
            e = hipEventRecord(op->lane_done[i], op->lanes[i]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, op->lane_done[i], 0);
            if (e != hipSuccess && st == PC_OK) st = hip_fail(e, "stream join");
        }
    }
    if (st != PC_OK) return st;
    prof_end(op, s, ev_all, 0, (int)B);
    return mark_used(op, s);
}

// The staged FP32 launch runs in two parts (see DevPlan::items_split).
bool uses_split(const pc_op* op) { return op->dev.n_small > 0 && op->dev.dtype == 0; }

bool uses_direct(const pc_op* op) { return op->tune_direct && op->plan.d <= 2 && !op->plan.cbeg_fwd.empty(); }

pc_status run_batch(pc_op* op, bool adj, bool plain, int64_t B, const void* U, int64_t ldu, void* OUT, int64_t ldo,
                    hipStream_t s, bool acc = false, double alpha = 1.0) {
    pc_status st = check_op(op);
    if (st != PC_OK) return st;
    const int64_t N = op->plan.N;
    if (B < 0) return fail(PC_ERR_ARG, "negative batch size");
    if (B == 0) return PC_OK;
    if (!U || !OUT) return fail(PC_ERR_ARG, "null vector pointer");
    if (ldu < N || ldo < N) return fail(PC_ERR_ARG, "leading dimension smaller than N");
    if (B > 0x7fff) return fail(PC_ERR_ARG, "batch too large (B > 32767)");
    if (op->plan.d == 3) {
        st = run_batch_3d(op, adj, plain, B, U, ldu, OUT, ldo, s, acc, alpha);
        return st == PC_OK ? mark_used(op, s) : st;
    }
    if (!plain && !acc && uses_direct(op)) return run_direct(op, adj, B, U, ldu, OUT, ldo, s);
    const int64_t per = adj ? op->plan.slot_adj : op->plan.slot_fwd;
    const size_t per_bytes = (size_t)std::max<int64_t>(per, 1) * op->esz;
    int64_t chunk = 1;
    if (!plain) {
        const size_t cap_bytes = op->tune_overlap ? kSlotCapBytes / 2 : kSlotCapBytes;
        const int64_t cap = (int64_t)std::max<size_t>(1, cap_bytes / per_bytes);
        const int64_t want = op->tune_chunk > 0 ? op->tune_chunk
                             : (op->tune_overlap ? (B + kMinChunks - 1) / kMinChunks : B);
        chunk = std::min<int64_t>(cap, std::max<int64_t>(1, want));
    }
    const int64_t nchunks = (B + chunk - 1) / chunk;
    const bool overlap = !plain && op->tune_overlap && nchunks > 1;
    const size_t buf_bytes = (size_t)chunk * per_bytes;
    const bool cap = capturing(s);
    st = ensure(op, &op->slots, &op->slots_bytes, (overlap ? 2 : 1) * buf_bytes, "hipMallocAsync (staging)", s);
    if (st != PC_OK) return st;
    if (overlap && cap && !op->aux) return fail(PC_ERR_ARG, "make one overlapped call before the stream capture");
    if (overlap && (st = ensure_aux(op)) != PC_OK) return st;
    const char* u = static_cast<const char*>(U);
    char* o = static_cast<char*>(OUT);
    const int n_items = (int)op->plan.items.size();
    for (int64_t c = 0; c < nchunks; ++c) {
        const int64_t b0 = c * chunk;
        const int nb = (int)std::min<int64_t>(chunk, B - b0);
        const int pb = overlap ? (int)(c & 1) : 0;
        void* slots = static_cast<char*>(op->slots) + (size_t)pb * buf_bytes;
        const void* in = u + (size_t)b0 * ldu * op->esz;
        void* out = o + (size_t)b0 * ldo * op->esz;
        hipError_t e;
        hipEvent_t ev;
        if (overlap && c >= 2) {   // the reduction two chunks back still reads this buffer
            e = hipStreamWaitEvent(s, op->ev_red[pb], 0);
            if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
        }
        if (plain) {
            for (int it = 0; it < n_items; ++it) {
                if (injected_failure(op)) return injected();
                prof_begin(op, s, &ev);
                e = pc::launch_conv(op->dev, op->dev.items, adj, it, it + 1, 1, in, ldu, slots, per, nullptr, 0, s);
                if (e != hipSuccess) return hip_fail(e, "conv launch");
                prof_end(op, s, ev, 0, 1);
            }
        } else if (op->tune_persistent && pc::persistent_fits(op->dev)) {
            if (injected_failure(op)) return injected();
            prof_begin(op, s, &ev);   // a fill kernel, then the persistent kernel
            e = pc::launch_conv_persistent(op->dev, adj, nb, in, ldu, slots, per, s);
            if (e != hipSuccess) return hip_fail(e, "conv launch");
            prof_end(op, s, ev, 0, nb);
        } else {
            if (injected_failure(op)) return injected();
            const pc::LaunchEvents lev = prof_events(op, s);
            if (op->tune_split && !op->tune_item_major && uses_split(op))
                e = pc::launch_conv_split(op->dev, adj, nb, in, ldu, slots, per, s, lev);
            else
                e = pc::launch_conv(op->dev, op->dev.items, adj, 0, n_items, nb, in, ldu, slots, per, nullptr, 0, s,
                                    op->tune_item_major, lev);
            if (e != hipSuccess) {
                prof_drop(op, lev);
                return hip_fail(e, "conv launch");
            }
            prof_take(op, lev, 0, nb);
        }
        hipStream_t rs = s;
        if (overlap) {
            e = hipEventRecord(op->ev_conv[pb], s);
            if (e == hipSuccess) e = hipStreamWaitEvent(op->aux, op->ev_conv[pb], 0);
            if (e != hipSuccess) return hip_fail(e, "event chaining");
            rs = op->aux;
        }
        const pc::LaunchEvents rev = prof_events(op, rs);
        e = pc::launch_reduce(op->dev, adj, nb, slots, per, out, ldo, rs, acc, alpha, rev);
        if (e != hipSuccess) {
            prof_drop(op, rev);
            return hip_fail(e, "reduce launch");
        }
        prof_take(op, rev, 1, nb);
        if (overlap) {
            e = hipEventRecord(op->ev_red[pb], op->aux);
            if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        }
    }
    if (overlap) {   // the caller's stream sees the last reduction (the aux stream is in order)
        hipError_t e = hipStreamWaitEvent(s, op->ev_red[(nchunks - 1) & 1], 0);
        if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    }
    return mark_used(op, s);
}

pc_status create_impl(int d, const int64_t* shape, int64_t n_leaves, const int64_t* leaf_lo, const int64_t* leaf_hi,
                      int64_t r, const int64_t* points, const int64_t* radius, const double* phi,
                      const int64_t* phi_off, pc_dtype dtype, uint32_t flags, int64_t n_sel, const int64_t* sel,
                      hipStream_t s, pc_op** out) {
    if (!out) return fail(PC_ERR_ARG, "null output handle");
    *out = nullptr;
    pc_op* op = new (std::nothrow) pc_op();
    if (!op) return fail(PC_ERR_OOM, "host allocation failed");
    pc::CreateArgs a{d, shape, n_leaves, leaf_lo, leaf_hi, r, points, radius, phi, phi_off, (int)dtype, flags,
                     n_sel, sel};
    std::string err;
    pc_status st;
    try {
        st = pc::build_plan(a, op->plan, err);
    } catch (const std::bad_alloc&) {
        st = PC_ERR_OOM;
        err = "host allocation failed while planning";
    } catch (...) {
        st = PC_ERR_ARG;
        err = "unexpected error while planning";
    }
    if (st != PC_OK) {
        delete op;
        return fail(st, err);
    }
    hipError_t e = hipGetDevice(&op->device);
    if (e != hipSuccess) {
        delete op;
        return hip_fail(e, "hipGetDevice");
    }
    int lds_max = 0;
    e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, op->device);
    if (e != hipSuccess) {
        delete op;
        return hip_fail(e, "hipDeviceGetAttribute");
    }
    if (std::max(op->plan.max_lds, op->plan.max_lds_axis) > lds_max) {
        delete op;
        return fail(PC_ERR_UNSUPPORTED, "device LDS per workgroup (" + std::to_string(lds_max) +
                                            " B) is below the plan's need (" +
                                            std::to_string(std::max(op->plan.max_lds, op->plan.max_lds_axis)) + " B)");
    }
    e = pc::set_kernel_attributes();
    if (e != hipSuccess) {
        delete op;
        return hip_fail(e, "hipFuncSetAttribute");
    }
    e = pc::noalloc_area_init(op->device);   // once per device, this device current
    if (e != hipSuccess) {
        delete op;
        return hip_fail(e, "hipGetSymbolAddress (allocation-free work area)");
    }
    op->esz = (dtype == PC_F64) ? 8 : 4;
    pc::Plan& P = op->plan;
    void *d_items, *d_spec, *d_wts, *d_tw, *d_tf, *d_ta, *d_bf, *d_ba;
    if ((st = upload(op, P.items, &d_items, s)) != PC_OK || (st = upload_real(op, P.spec, &d_spec, s)) != PC_OK ||
        (st = upload_real(op, P.wts, &d_wts, s)) != PC_OK || (st = upload_real(op, P.tw, &d_tw, s)) != PC_OK ||
        (st = upload(op, P.tiles_fwd, &d_tf, s)) != PC_OK || (st = upload(op, P.tiles_adj, &d_ta, s)) != PC_OK ||
        (st = upload(op, P.cboxes_fwd, &d_bf, s)) != PC_OK || (st = upload(op, P.cboxes_adj, &d_ba, s)) != PC_OK) {
        delete op;
        return st;
    }
    void *d_leaf, *d_items3, *d_queue;
    if ((st = upload(op, P.leaf_box, &d_leaf, s)) != PC_OK || (st = upload(op, P.items3, &d_items3, s)) != PC_OK ||
        (st = upload(op, std::vector<int32_t>(128, 0), &d_queue, s)) != PC_OK) {
        delete op;
        return st;
    }
    int n_cu = 0;
    e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, op->device);
    if (e != hipSuccess) {
        delete op;
        return hip_fail(e, "hipDeviceGetAttribute");
    }
    void* d_ord[2] = {d_items, d_items};
    for (int dir = 0; dir < 2 && !P.items.empty(); ++dir) {
        const std::vector<int32_t>& ord = dir ? P.order_adj : P.order_fwd;
        if (ord.size() != P.items.size()) continue;
        std::vector<pc::Item> perm(ord.size());
        for (size_t j = 0; j < ord.size(); ++j) perm[j] = P.items[(size_t)ord[j]];
        if ((st = upload(op, perm, &d_ord[dir], s)) != PC_OK) {
            delete op;
            return st;
        }
    }
    // the items again, those above kSmallItemLds first (they run as 1024-
    // thread workgroups), then the others (two 512-thread workgroups per CU)
    void* d_split = d_items;
    int n_big = 0, n_small = 0, lds_big = 0, lds_small = 0;
    if (!P.items.empty()) {
        const int64_t csz = (dtype == PC_F64) ? 16 : 8;
        std::vector<pc::Item> big, small;
        for (const pc::Item& it : P.items) {
            const int lds = (int)(((int64_t)it.n0 * it.ld + pc::twiddle_elems(it.a0, it.b0, it.am, it.bm)) * csz);
            if (lds <= pc::kSmallItemLds) {
                small.push_back(it);
                lds_small = std::max(lds_small, lds);
            } else {
                big.push_back(it);
                lds_big = std::max(lds_big, lds);
            }
        }
        n_big = (int)big.size();
        n_small = (int)small.size();
        big.insert(big.end(), small.begin(), small.end());
        if ((st = upload(op, big, &d_split, s)) != PC_OK) {
            delete op;
            return st;
        }
    }
    pc::DevPlan& D = op->dev;
    D.items_split = static_cast<const pc::Item*>(d_split);
    D.n_big = n_big;
    D.n_small = n_small;
    D.lds_big = lds_big;
    D.lds_small = lds_small;
    D.items = static_cast<const pc::Item*>(d_items);
    D.n_items = (int)P.items.size();
    D.items_ord[0] = static_cast<const pc::Item*>(d_ord[0]);
    D.items_ord[1] = static_cast<const pc::Item*>(d_ord[1]);
    D.items3 = static_cast<const pc::Item3*>(d_items3);
    D.n_items3 = (int)P.items3.size();
    D.rows = P.rows;
    D.cols = P.cols;
    D.planes = P.planes;
    D.prow = P.prow;
    D.spec = d_spec;
    D.wts = d_wts;
    D.tw = d_tw;
    D.tiles_fwd = static_cast<const pc::Tile*>(d_tf);
    D.tiles_adj = static_cast<const pc::Tile*>(d_ta);
    D.n_tiles_fwd = (int)P.tiles_fwd.size();
    D.n_tiles_adj = (int)P.tiles_adj.size();
    D.cboxes_fwd = static_cast<const pc::Box*>(d_bf);
    D.cboxes_adj = static_cast<const pc::Box*>(d_ba);
    D.slot_fwd = P.slot_fwd;
    D.slot_adj = P.slot_adj;
    D.max_lds = P.max_lds;
    D.conv_threads = P.conv_threads;
    D.max_lds_axis = P.max_lds_axis;
    D.dtype = (int)dtype;
    D.queue = static_cast<int*>(d_queue);
    D.n_cu = n_cu;
    op->leaf_box = static_cast<int32_t*>(d_leaf);
    op->d_wts = d_wts;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        delete op;
        return hip_fail(e, "hipStreamSynchronize after upload");
    }
    // spectra are only needed on the device from now on
    std::vector<double>().swap(P.spec);
    if (const char* env = std::getenv("PC_DEBUG_FAIL_LAUNCH")) {   // test hook, as pc_debug_fail_launches(n, 1)
        const long long n = std::atoll(env);
        if (n > 0) {
            op->dbg_first = n;
            op->dbg_count = 1;
        }
    }
    *out = op;
    return PC_OK;
}

// Uploads the matrix-entry tables (once per operator).
pc_status ensure_entries(pc_op* op, hipStream_t s) {
    if (op->ent_ready) return PC_OK;
    const pc::Plan& P = op->plan;
    std::vector<int32_t> leaf_of((size_t)P.N, -1);
    for (int64_t c = 0; c < P.L; ++c) {
        const int32_t* b = &P.leaf_box[(size_t)c * 6];
        for (int32_t z = 0; z < b[3]; ++z)
            for (int32_t y = 0; y < b[4]; ++y) {
                int32_t* row = &leaf_of[(size_t)(((int64_t)(b[0] + z) * P.prow + b[1] + y) * P.cols + b[2])];
                for (int32_t x = 0; x < b[5]; ++x)
                    if (row[x] < 0) row[x] = (int32_t)c;
            }
    }
    void *d_leaf, *d_off, *d_lp, *d_wb, *d_ub, *d_eo, *d_eb, *d_phi;
    pc_status st;
    if ((st = upload(op, leaf_of, &d_leaf, s)) != PC_OK || (st = upload(op, P.leaf_pts_off, &d_off, s)) != PC_OK ||
        (st = upload(op, P.leaf_pts, &d_lp, s)) != PC_OK || (st = upload(op, P.pt_wbase, &d_wb, s)) != PC_OK ||
        (st = upload(op, P.pt_ubox, &d_ub, s)) != PC_OK || (st = upload(op, P.pt_eoff, &d_eo, s)) != PC_OK ||
        (st = upload(op, P.pt_ebox, &d_eb, s)) != PC_OK || (st = upload_real(op, P.phiE, &d_phi, s)) != PC_OK)
        return st;
    pc::EntryTables& E = op->ent;
    E.d = P.d;
    E.planes = P.planes;
    E.prow = P.prow;
    E.cols = P.cols;
    E.leaf_of = static_cast<const int32_t*>(d_leaf);
    E.lp_off = static_cast<const int32_t*>(d_off);
    E.lp = static_cast<const int32_t*>(d_lp);
    E.wbase = static_cast<const int64_t*>(d_wb);
    E.ubox = static_cast<const int32_t*>(d_ub);
    E.eoff = static_cast<const int64_t*>(d_eo);
    E.ebox = static_cast<const int32_t*>(d_eb);
    op->ent_phiE = d_phi;
    op->ent_ready = true;
    return PC_OK;
}

constexpr int kEstParts = 512;   // row-block partials of the estimator totals

// Estimator sums (Sec. 2.6) of Yt - Y over the operator's leaves, left on
// the device in stream order: sums[c] per leaf, sums[L] over Omega, sums[L+1]
// = sum Y^2.  The row-block partials live in the operator's estimator buffer.
pc_status est_sums_device(pc_op* op, int64_t q, const void* Yt, int64_t ldt, const void* Y, int64_t ldy,
                          double* sums, hipStream_t s) {
    const int L = (int)op->plan.L;
    void* est = op->est;
    pc_status st = ensure(op, &est, &op->est_bytes, sizeof(double) * (size_t)(L + 2 + 2 * kEstParts),
                          "hipMallocAsync (estimator sums)", s);
    op->est = static_cast<double*>(est);
    if (st != PC_OK) return st;
    double* leaf = sums ? sums : op->est;
    hipError_t e = pc::launch_est(op->plan.dtype, op->leaf_box, L, (int)q, Yt, ldt, Y, ldy, op->plan.planes,
                                  op->plan.prow, op->plan.cols, leaf, op->est + L + 2, kEstParts, leaf + L, s);
    if (e != hipSuccess) return hip_fail(e, "estimator launch");
    return mark_used(op, s);
}

// The same sums read back (synchronises s) and turned into eta_leaf, eta_abs
// and eta_rel.
pc_status est_sums(pc_op* op, int64_t q, const void* Yt, int64_t ldt, const void* Y, int64_t ldy, double* eta_leaf,
                   double* eta_abs, double* eta_rel, hipStream_t s) {
    const int L = (int)op->plan.L;
    pc_status st = est_sums_device(op, q, Yt, ldt, Y, ldy, nullptr, s);
    if (st != PC_OK) return st;
    std::vector<double> h((size_t)L + 2);
    hipError_t e = hipMemcpyAsync(h.data(), op->est, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync (estimator sums)");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize (estimator)");
    const double dd = h[(size_t)L], yy = h[(size_t)L + 1];
    if (eta_leaf)
        for (int c = 0; c < L; ++c) eta_leaf[c] = std::sqrt(h[(size_t)c] / (double)q);
    *eta_abs = std::sqrt(dd / (double)q);
    *eta_rel = yy > 0.0 ? std::sqrt(dd) / std::sqrt(yy) : INFINITY;
    return PC_OK;
}

}  // namespace

extern "C" {

pc_status pc_create(int d, const int64_t* shape, int64_t n_leaves, const int64_t* leaf_lo, const int64_t* leaf_hi,
                    int64_t r, const int64_t* points, const int64_t* radius, const double* phi,
                    const int64_t* phi_off, pc_dtype dtype, uint32_t flags, hipStream_t s, pc_op** out) {
    return create_impl(d, shape, n_leaves, leaf_lo, leaf_hi, r, points, radius, phi, phi_off, dtype, flags, -1,
                       nullptr, s, out);
}

pc_status pc_create_patches(int d, const int64_t* shape, int64_t n_leaves, const int64_t* leaf_lo,
                            const int64_t* leaf_hi, int64_t r, const int64_t* points, const int64_t* radius,
                            const double* phi, const int64_t* phi_off, pc_dtype dtype, uint32_t flags,
                            int64_t n_sel, const int64_t* sel, hipStream_t s, pc_op** out) {
    if (n_sel < 0) {
        if (out) *out = nullptr;
        return fail(PC_ERR_ARG, "negative selection size");
    }
    return create_impl(d, shape, n_leaves, leaf_lo, leaf_hi, r, points, radius, phi, phi_off, dtype, flags, n_sel,
                       sel, s, out);
}

pc_status pc_apply(pc_op* op, const void* u, void* out, hipStream_t s) {
    if (!op) return fail(PC_ERR_ARG, "null operator");
    return run_batch(op, false, false, 1, u, op->plan.N, out, op->plan.N, s);
}

pc_status pc_apply_batch(pc_op* op, int64_t B, const void* U, int64_t ldu, void* OUT, int64_t ldo, hipStream_t s) {
    return run_batch(op, false, false, B, U, ldu, OUT, ldo, s);
}

pc_status pc_apply_adjoint_batch(pc_op* op, int64_t B, const void* V, int64_t ldv, void* OUT, int64_t ldo,
                                 hipStream_t s) {
    return run_batch(op, true, false, B, V, ldv, OUT, ldo, s);
}

pc_status pc_apply_batch_plain(pc_op* op, int64_t B, const void* U, int64_t ldu, void* OUT, int64_t ldo,
                               hipStream_t s) {
    return run_batch(op, false, true, B, U, ldu, OUT, ldo, s);
}

pc_status pc_apply_batch_noalloc(pc_op* op, int64_t B, const void* U, int64_t ldu, void* OUT, int64_t ldo,
                                 hipStream_t s) {
    pc_status st = check_op(op);
    if (st != PC_OK) return st;
    const pc::Plan& P = op->plan;
    if (B < 0) return fail(PC_ERR_ARG, "negative batch size");
    if (B == 0) return PC_OK;
    if (!U || !OUT) return fail(PC_ERR_ARG, "null vector pointer");
    if (ldu < P.N || ldo < P.N) return fail(PC_ERR_ARG, "leading dimension smaller than N");
    if (B > 0x7fff) return fail(PC_ERR_ARG, "batch too large (B > 32767)");
    char* area = static_cast<char*>(pc::noalloc_area(op->device));
    if (!area) return fail(PC_ERR_DEVICE, "the allocation-free work area of this device was not set up");
    if (uses_direct(op)) {   // the colour launches need no work area
        struct NoProfiling {
            pc_op* op;
            bool was;
            ~NoProfiling() { op->profiling = was; }
        } guard{op, op->profiling};
        op->profiling = false;
        return run_direct(op, false, B, U, ldu, OUT, ldo, s, 1);   // the caller's stream only
    }
    const size_t per_bytes = (size_t)std::max<int64_t>(P.slot_fwd, 1) * op->esz;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    if (al(per_bytes) > pc::kNoAllocBytes)
        return fail(PC_ERR_UNSUPPORTED, "one vector needs " + std::to_string(per_bytes) +
                                            " bytes of staging; the allocation-free work area holds " +
                                            std::to_string(pc::kNoAllocBytes));
    struct NoProfiling {   // no event objects are created on this path
        pc_op* op;
        bool was;
        ~NoProfiling() { op->profiling = was; }
    } guard{op, op->profiling};
    op->profiling = false;
    if (P.d == 3) {
        // one vector at a time: its staging first, the plane scratch behind it
        ExtBufs ext{area, 1, area + al(per_bytes), pc::kNoAllocBytes - al(per_bytes)};
        return run_3d(op, P.items3, op->dev, op->dev, P.slot_fwd, false, false, B, U, ldu, OUT, ldo, s, false, 1.0,
                      &ext);
    }
    const int64_t chunk = std::min<int64_t>(B, (int64_t)(pc::kNoAllocBytes / per_bytes));
    const int n_items = (int)P.items.size();
    const char* u = static_cast<const char*>(U);
    char* o = static_cast<char*>(OUT);
    for (int64_t b0 = 0; b0 < B; b0 += chunk) {
        const int nb = (int)std::min<int64_t>(chunk, B - b0);
        if (injected_failure(op)) return injected();
        hipError_t e = pc::launch_conv(op->dev, op->dev.items, false, 0, n_items, nb, u + (size_t)b0 * ldu * op->esz,
                                       ldu, area, P.slot_fwd, nullptr, 0, s);
        if (e != hipSuccess) return hip_fail(e, "conv launch");
        e = pc::launch_reduce(op->dev, false, nb, area, P.slot_fwd, o + (size_t)b0 * ldo * op->esz, ldo, s);
        if (e != hipSuccess) return hip_fail(e, "reduce launch");
    }
    return PC_OK;
}

pc_status pc_apply_batch_axpy(pc_op* op, int64_t B, const void* U, int64_t ldu, double alpha, void* OUT, int64_t ldo,
                              hipStream_t s) {
    return run_batch(op, false, false, B, U, ldu, OUT, ldo, s, true, alpha);
}

pc_status pc_apply_adjoint_batch_axpy(pc_op* op, int64_t B, const void* V, int64_t ldv, double alpha, void* OUT,
                                      int64_t ldo, hipStream_t s) {
    return run_batch(op, true, false, B, V, ldv, OUT, ldo, s, true, alpha);
}

pc_status pc_apply_block(pc_op* op, int adjoint, const int64_t* tlo, const int64_t* thi, const int64_t* slo,
                         const int64_t* shi, int64_t B, const void* U, int64_t ldu, void* OUT, int64_t ldo,
                         hipStream_t s) {
    pc_status st = check_op(op);
    if (st != PC_OK) return st;
    if (capturing(s)) return fail(PC_ERR_ARG, "pc_apply_block copies its tables synchronously: not capturable");
    if (B < 0) return fail(PC_ERR_ARG, "negative batch size");
    pc::BlockPlan bp;
    std::string err;
    st = pc::build_block(op->plan, adjoint != 0, tlo, thi, slo, shi, bp, err);
    if (st != PC_OK) return fail(st, err);
    const int64_t nS = (int64_t)bp.s_planes * bp.s_rows * bp.s_cols, nT = (int64_t)bp.t_rows * bp.t_cols;
    if (B == 0) return PC_OK;
    if (!U || !OUT) return fail(PC_ERR_ARG, "null vector pointer");
    if (ldu < nS || ldo < nT) return fail(PC_ERR_ARG, "leading dimension smaller than the block box");
    if (B > 0x7fff) return fail(PC_ERR_ARG, "batch too large (B > 32767)");
    // per-call tables: items | tiles | contributor boxes
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const bool d3 = op->plan.d == 3;
    const size_t bi = d3 ? al(bp.items3.size() * sizeof(pc::Item3)) : al(bp.items.size() * sizeof(pc::Item)),
                 bt = al(bp.tiles.size() * sizeof(pc::Tile)), bc = al(bp.cboxes.size() * sizeof(pc::Box));
    hipError_t e;
    if (op->blk_done) {
        e = hipEventSynchronize(op->blk_done);   // the previous block call may still read the tables
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    } else {
        e = hipEventCreateWithFlags(&op->blk_done, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreateWithFlags");
    }
    st = ensure(op, &op->blk, &op->blk_bytes, std::max<size_t>(bi + bt + bc, 256), "hipMallocAsync (block tables)", s);
    if (st != PC_OK) return st;
    char* base = static_cast<char*>(op->blk);
    if (!bp.items.empty()) e = hipMemcpy(base, bp.items.data(), bp.items.size() * sizeof(pc::Item), hipMemcpyHostToDevice);
    if (e == hipSuccess && !bp.items3.empty())
        e = hipMemcpy(base, bp.items3.data(), bp.items3.size() * sizeof(pc::Item3), hipMemcpyHostToDevice);
    if (e == hipSuccess && !bp.tiles.empty())
        e = hipMemcpy(base + bi, bp.tiles.data(), bp.tiles.size() * sizeof(pc::Tile), hipMemcpyHostToDevice);
    if (e == hipSuccess && !bp.cboxes.empty())
        e = hipMemcpy(base + bi + bt, bp.cboxes.data(), bp.cboxes.size() * sizeof(pc::Box), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy (block tables)");
    pc::DevPlan Dc = op->dev;          // convolution: gather pitch of S
    Dc.items = reinterpret_cast<const pc::Item*>(base);
    Dc.n_items = (int)bp.items.size();
    Dc.cols = bp.s_cols;
    pc::DevPlan Dr = op->dev;          // reduction over T
    Dr.tiles_fwd = Dr.tiles_adj = reinterpret_cast<const pc::Tile*>(base + bi);
    Dr.n_tiles_fwd = Dr.n_tiles_adj = (int)bp.tiles.size();
    Dr.cboxes_fwd = Dr.cboxes_adj = reinterpret_cast<const pc::Box*>(base + bi + bt);
    Dr.rows = bp.t_rows;
    Dr.cols = bp.t_cols;
    if (d3) {
        Dc.items3 = reinterpret_cast<const pc::Item3*>(base);
        Dc.n_items3 = (int)bp.items3.size();
        Dc.prow = bp.s_rows;           // plane pitch of S = s_rows * s_cols
        st = run_3d(op, bp.items3, Dc, Dr, bp.per, adjoint != 0, false, B, U, ldu, OUT, ldo, s, false, 1.0);
        if (st != PC_OK) return st;
        e = hipEventRecord(op->blk_done, s);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        return mark_used(op, s);
    }
    const size_t per_bytes = (size_t)std::max<int64_t>(bp.per, 1) * op->esz;
    const int64_t chunk = std::min<int64_t>(B, std::max<int64_t>(1, (int64_t)(kSlotCapBytes / per_bytes)));
    st = ensure(op, &op->slots, &op->slots_bytes, (size_t)chunk * per_bytes, "hipMallocAsync (staging)", s);
    if (st != PC_OK) return st;
    const char* u = static_cast<const char*>(U);
    char* o = static_cast<char*>(OUT);
    for (int64_t b0 = 0; b0 < B; b0 += chunk) {
        const int nb = (int)std::min<int64_t>(chunk, B - b0);
        if (injected_failure(op)) return injected();
        e = pc::launch_conv(Dc, Dc.items, adjoint != 0, 0, Dc.n_items, nb, u + (size_t)b0 * ldu * op->esz, ldu,
                            op->slots, bp.per, nullptr, 0, s);
        if (e != hipSuccess) return hip_fail(e, "block conv launch");
        e = pc::launch_reduce(Dr, adjoint != 0, nb, op->slots, bp.per, o + (size_t)b0 * ldo * op->esz, ldo, s);
        if (e != hipSuccess) return hip_fail(e, "block reduce launch");
    }
    e = hipEventRecord(op->blk_done, s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    return mark_used(op, s);
}

pc_status pc_entries(pc_op* op, int64_t n, const int64_t* ys, const int64_t* xs, void* out, hipStream_t s) {
    pc_status st = check_op(op);
    if (st != PC_OK) return st;
    if (n < 0) return fail(PC_ERR_ARG, "negative entry count");
    if (n == 0) return PC_OK;
    if (!ys || !xs || !out) return fail(PC_ERR_ARG, "null coordinate or output pointer");
    if (!op->ent_phiE && capturing(s)) return fail(PC_ERR_ARG, "make one pc_entries call before the stream capture");
    if ((st = ensure_entries(op, s)) != PC_OK) return st;
    hipError_t e = pc::launch_entries(op->ent, op->plan.dtype, op->d_wts, op->ent_phiE, n, ys, xs, out, s);
    if (e != hipSuccess) return hip_fail(e, "entries launch");
    return PC_OK;
}

pc_status pc_estimate_sums(pc_op* op, int64_t q, const void* Yt, int64_t ldt, const void* Y, int64_t ldy,
                           double* eta_leaf, double* eta_abs, double* eta_rel, hipStream_t s) {
    pc_status st = check_op(op);
    if (st != PC_OK) return st;
    const int64_t N = op->plan.N;
    if (q < 1 || !Yt || !Y || ldt < N || ldy < N) return fail(PC_ERR_ARG, "invalid estimator blocks");
    if (!eta_abs || !eta_rel) return fail(PC_ERR_ARG, "null output scalar");
    if (capturing(s)) return fail(PC_ERR_ARG, "the estimator returns host scalars: not capturable");
    return est_sums(op, q, Yt, ldt, Y, ldy, eta_leaf, eta_abs, eta_rel, s);
}

pc_status pc_estimate_sums_device(pc_op* op, int64_t q, const void* Yt, int64_t ldt, const void* Y, int64_t ldy,
                                  double* sums, hipStream_t s) {
    pc_status st = check_op(op);
    if (st != PC_OK) return st;
    const int64_t N = op->plan.N;
    if (q < 1 || !Yt || !Y || ldt < N || ldy < N) return fail(PC_ERR_ARG, "invalid estimator blocks");
    if (!sums) return fail(PC_ERR_ARG, "null sums pointer");
    return est_sums_device(op, q, Yt, ldt, Y, ldy, sums, s);
}

pc_status pc_error_estimate(pc_op* op, int64_t q, const void* Z, int64_t ldz, const void* Y_or_null, int64_t ldy,
                            pc_matvec_fn exact_adjoint, void* user, double* eta_leaf, double* eta_abs,
                            double* eta_rel, hipStream_t s) {
    pc_status st = check_op(op);
    if (st != PC_OK) return st;
    const int64_t N = op->plan.N;
    if (q < 1 || !Z || ldz < N) return fail(PC_ERR_ARG, "invalid probe block");
    if (!eta_abs || !eta_rel) return fail(PC_ERR_ARG, "null output scalar");
    if (!Y_or_null && !exact_adjoint) return fail(PC_ERR_ARG, "need Y or an exact-adjoint callback");
    if (Y_or_null && ldy < N) return fail(PC_ERR_ARG, "ldy smaller than N");
    if (capturing(s)) return fail(PC_ERR_ARG, "the estimator returns host scalars: not capturable");
    const size_t vec = (size_t)N * op->esz;
    const size_t need = (size_t)q * vec * (Y_or_null ? 1 : 2);
    st = ensure(op, &op->work, &op->work_bytes, need, "hipMallocAsync (estimator work)", s);
    if (st != PC_OK) return st;
    char* Yt = static_cast<char*>(op->work);
    const void* Y = Y_or_null;
    int64_t ldY = ldy;
    if (!Y_or_null) {
        void* Ybuf = Yt + (size_t)q * vec;
        int rc = exact_adjoint(user, q, Z, ldz, Ybuf, N, s);
        if (rc != 0) return fail(PC_ERR_CALLBACK, "exact-adjoint callback returned " + std::to_string(rc));
        Y = Ybuf;
        ldY = N;
    }
    st = run_batch(op, true, false, q, Z, ldz, Yt, N, s);
    if (st != PC_OK) return st;
    return est_sums(op, q, Yt, N, Y, ldY, eta_leaf, eta_abs, eta_rel, s);
}

pc_status pc_get_stats(const pc_op* op, pc_stats* st) {
    if (!op || !st) return fail(PC_ERR_ARG, "null argument");
    const pc::Plan& P = op->plan;
    std::memset(st, 0, sizeof(*st));
    st->n = P.N;
    st->r = P.r;
    st->n_leaves = P.L;
    st->n_items = (int64_t)(P.d == 3 ? P.items3.size() : P.items.size());
    st->sum_fft_points = P.sum_fft_points;
    st->alg_flops_per_rhs = P.alg_flops;
    st->kernel_elems = P.kernel_elems;
    int64_t spec_elems = 0;
    for (const auto& I : P.items3) spec_elems += (int64_t)I.nz * I.p.n0 * (I.p.m + 1);
    {
        // one spectrum per patch: n0 x (m + 1) complex
        int last = -1;
        for (const auto& it : P.items)
            if (it.patch != last) {
                spec_elems += (int64_t)it.n0 * (it.m + 1);
                last = it.patch;
            }
    }
    st->spectrum_bytes = spec_elems * 2 * (int64_t)op->esz;
    st->weight_bytes = (int64_t)P.wts.size() * (int64_t)op->esz;
    st->slot_elems_fwd = P.slot_fwd;
    st->slot_elems_adj = P.slot_adj;
    st->device_bytes = (int64_t)op->resident;
    st->dtype = P.dtype;
    st->max_lds_bytes = P.max_lds;
    return PC_OK;
}

pc_status pc_debug_fail_launches(pc_op* op, int64_t first, int64_t count) {
    pc_status st = check_op(op);
    if (st != PC_OK) return st;
    if (count < 0 || (count > 0 && first < 1)) return fail(PC_ERR_ARG, "first must be >= 1 and count >= 0");
    op->dbg_first = first;
    op->dbg_count = count;
    op->dbg_seen = 0;
    return PC_OK;
}

pc_status pc_set_profiling(pc_op* op, int enable) {
    if (!op) return fail(PC_ERR_ARG, "null operator");
    op->profiling = enable != 0;
    return PC_OK;
}

pc_status pc_set_tuning(pc_op* op, int key, int64_t value) {
    if (!op) return fail(PC_ERR_ARG, "null operator");
    switch (key) {
        case PC_TUNE_CHUNK:
            if (value < 0 || value > 0x7fff) return fail(PC_ERR_ARG, "chunk out of range");
            op->tune_chunk = value;
            return PC_OK;
        case PC_TUNE_OVERLAP:
            op->tune_overlap = value != 0;
            return PC_OK;
        case PC_TUNE_SCRATCH:
            if (value < 0) return fail(PC_ERR_ARG, "scratch size out of range");
            op->tune_scratch = value;
            return PC_OK;
        case PC_TUNE_DIRECT:
            op->tune_direct = value != 0;
            return PC_OK;
        case PC_TUNE_STREAMS:
            if (value < 1 || value > kMaxLanes) return fail(PC_ERR_ARG, "streams out of range (1..4)");
            op->tune_streams = (int)value;
            return PC_OK;
        case PC_TUNE_PERSISTENT:
            op->tune_persistent = value != 0;
            return PC_OK;
        case PC_TUNE_XCD_ORDER:
            op->tune_item_major = value != 0;
            return PC_OK;
        case PC_TUNE_SPLIT:
            op->tune_split = value != 0;
            return PC_OK;
        case PC_TUNE_BUDGET:
            if (value < 0) return fail(PC_ERR_ARG, "budget out of range");
            op->budget = (size_t)value;
            return PC_OK;
        default:
            return fail(PC_ERR_ARG, "unknown tuning key");
    }
}

pc_status pc_read_profile(pc_op* op, pc_profile* out) {
    if (!op || !out) return fail(PC_ERR_ARG, "null argument");
    std::memset(out, 0, sizeof(*out));
    pc_status st = PC_OK;
    for (auto& t : op->timed) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(t.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.a, t.b);
        if (e != hipSuccess && st == PC_OK) st = hip_fail(e, "hipEventElapsedTime");
        if (t.kind == 0) {
            out->conv_ms += ms;
            out->conv_launches += 1;
            out->conv_vectors += t.vectors;
        } else {
            out->reduce_ms += ms;
            out->reduce_launches += 1;
        }
        op->event_pool.push_back(t.a);
        op->event_pool.push_back(t.b);
    }
    op->timed.clear();
    return st;
}

size_t pc_device_bytes(const pc_op* op) {
    if (!op) return 0;
    return op->resident + work_buffer_bytes(op);
}

pc_status pc_destroy(pc_op* op) {
    if (!op) return PC_OK;
    // the operator's last calls end before its memory is released
    if (op->last_use_set) hipEventSynchronize(op->last_use);
    if (op->blk_done) hipEventSynchronize(op->blk_done);
    delete op;
    return PC_OK;
}

const char* pc_status_string(pc_status st) {
    switch (st) {
        case PC_OK: return "PC_OK";
        case PC_ERR_ARG: return "PC_ERR_ARG";
        case PC_ERR_GRID: return "PC_ERR_GRID";
        case PC_ERR_OOM: return "PC_ERR_OOM";
        case PC_ERR_BUDGET: return "PC_ERR_BUDGET";
        case PC_ERR_DEVICE: return "PC_ERR_DEVICE";
        case PC_ERR_CALLBACK: return "PC_ERR_CALLBACK";
        case PC_ERR_UNSUPPORTED: return "PC_ERR_UNSUPPORTED";
    }
    return "PC_ERR_UNKNOWN";
}

const char* pc_last_error(void) { return g_err.c_str(); }

}  // extern "C"
