// HIP kernels of the product-convolution apply for gfx950.
#include <algorithm>
#include <mutex>

#include <hip/hip_ext.h>

#include "pc_kernels.h"
#include "pc_entries.h"
#include "pc_phases3.h"

namespace pc {

// A kernel launch that carries timing events in its dispatch when START or
// STOP is non-null (never under stream capture: the host does not time
// captured calls), else a plain launch.
#define PC_LAUNCH(K, G, BL, LDS, S, START, STOP, ...)                                                  \
    do {                                                                                               \
        if ((START) || (STOP))                                                                         \
            hipExtLaunchKernelGGL(K, G, BL, (std::uint32_t)(LDS), S, START, STOP, 0u, __VA_ARGS__);    \
        else                                                                                           \
            hipLaunchKernelGGL(K, G, BL, LDS, S, __VA_ARGS__);                                         \
    } while (0)

// The events of a timed launch that enqueued no kernel, recorded on s so
// that the caller can still read them.
static hipError_t record_unused(const LaunchEvents& ev, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (ev.start) e = hipEventRecord(ev.start, s);
    if (e == hipSuccess && ev.stop) e = hipEventRecord(ev.stop, s);
    return e;
}

// ------------------------------------------------- allocation-free work area
// Staging and 3-D scratch of pc_apply_batch_noalloc: a file-scope device
// array, one copy per device, held until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in for
// the symbol): the device address of each device's copy is looked up once,
// with that device current, and kept per device.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_area_mu;
void* g_area[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_area_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_area_mu);
    if (g_area[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;   // the caller makes the device current
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_area[device] = ptr;
    return hipSuccess;
}

void* noalloc_area(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_area_mu);
    return g_area[device];
}

template <class T>
struct ConvArgs {
    const Item* items;
    int item_lo, n_items;   // items [item_lo, item_lo + n_items)
    int B;
    int adj;
    const cx<T>* spec;
    const T* wts;
    const cx<T>* tw;
    const T* in;
    int64_t ld_in;
    T* slots;
    int64_t slot_stride;
    T* out;                 // non-null: add the written boxes into out (items of one colour)
    int64_t ldo;
    int64_t pitch;
    int item_major;         // staged launches: 1 = item-major block order (see conv_kernel)
};

// One (item, vector) unit of the convolution, phases A0 to H.  With
// load_tw false the item's twiddle tables are already in LDS (the previous
// unit of a persistent workgroup was the same item).
template <class T, int NT, bool ADD>
__device__ __forceinline__ void conv_unit(const ConvArgs<T>& A, cx<T>* buf, int item, int rhs, bool load_tw, int tid) {
    const Item it = A.items[A.item_lo + item];
    T* const slot_vec = A.slots + (ADD ? 0 : (int64_t)rhs * A.slot_stride);
    Ctx<T> c = make_ctx<T>(it, A.adj != 0, A.in + (int64_t)rhs * A.ld_in, slot_vec, A.wts, A.spec, A.tw, A.pitch,
                           ADD ? A.out + (int64_t)rhs * A.ldo : nullptr);
    twiddles_to_lds(c, buf + (int64_t)it.n0 * it.ld, tid, NT, load_tw);
    phA0(c, buf, tid, NT);
    __syncthreads();
    phA(c, buf, tid, NT);
    __syncthreads();
    phB(c, buf, tid, NT);
    __syncthreads();
    phC(c, buf, tid, NT);
    __syncthreads();
    phD(c, buf, tid, NT);
    __syncthreads();
    phE(c, buf, tid, NT);
    __syncthreads();
    phF(c, buf, tid, NT);
    __syncthreads();
    phG(c, buf, tid, NT);
    __syncthreads();
    phH<4, ADD ? kOutAdd : kOutStage>(c, buf, tid, NT);
}

// One workgroup per (item, vector).  Blocks are dealt round-robin to the 8
// XCDs (block id mod 8).  Staged launches (all items at once) give every
// XCD whole items with all their vectors in sequence, so a patch's spectrum
// is fetched into one XCD's L2 and reused there by every vector.  A colour
// launch holds a few dozen items of uneven size, and whole items per XCD
// would leave the XCD with the largest ones working alone at the end, so
// there the blocks of one item run through all XCDs (item-major order);
// staged launches take that order too when A.item_major is set (a tuning
// choice).
template <class T, int NT, bool ADD>
__global__ __launch_bounds__(NT) void conv_kernel(ConvArgs<T> A) {
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
    const int bid = blockIdx.x;
    int item, rhs;
    if (ADD || A.item_major) {
        item = bid / A.B;
        rhs = bid - item * A.B;
    } else {
        const int xcd = bid & 7, l = bid >> 3;
        item = xcd + 8 * (l / A.B);
        rhs = l % A.B;
    }
    if (item >= A.n_items) return;
    conv_unit<T, NT, ADD>(A, buf, item, rhs, true, threadIdx.x);
}

// Staged FP32 launch of the small items: 512-thread workgroups held to 128
// VGPRs, so that two fit in a CU (LDS, waves and registers), otherwise as
// conv_kernel<T, 512, false>.
template <class T>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void conv_kernel_small(ConvArgs<T> A) {
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
    const int bid = blockIdx.x;
    const int xcd = bid & 7, l = bid >> 3;
    const int item = xcd + 8 * (l / A.B);
    if (item >= A.n_items) return;
    conv_unit<T, 512, false>(A, buf, item, l % A.B, true, threadIdx.x);
}

// Persistent form of the staged launch: a fixed grid of workgroups (one per
// CU), each taking units from the queue of its XCD (block id mod 8).  Unit l
// of XCD x is item x + 8 (l / B) with vector l mod B: the same units on the
// same XCD as the block-per-unit launch, handed out as workgroups free up,
// and a workgroup whose next unit is the same item keeps the item's twiddle
// tables in LDS.  queue[16 x] counts the units handed out on XCD x (cleared
// before the launch); the int at byte q_off of LDS (behind the item data)
// passes a unit index to the workgroup.  Every workgroup leaves once its
// XCD's queue is empty.
template <class T, int NT>
__global__ __launch_bounds__(NT) void conv_persistent_kernel(ConvArgs<T> A, int* queue, int q_off) {
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
    int* const next = reinterpret_cast<int*>(smem + q_off);
    const int xcd = blockIdx.x & 7;
    int prev = -1;
    for (;;) {
        // the barrier also ends the previous unit's LDS reads (phase H)
        // before the next unit writes the box and the twiddle tables
        if (threadIdx.x == 0) *next = atomicAdd(queue + 16 * xcd, 1);
        __syncthreads();
        const int l = *next;
        const int item = xcd + 8 * (l / A.B);
        if (item >= A.n_items) return;
        // the thread index passes through an opaque move on every unit, so
        // no per-thread offset of the phases is hoisted out of this loop
        // (kept live across units, they would not fit in registers)
        int tid;
        asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"((int)threadIdx.x));
        conv_unit<T, NT, false>(A, buf, item, l % A.B, item != prev, tid);
        prev = item;
    }
}

// ------------------------------------------------------------------- 3-D
template <class T>
struct Conv3Args {
    const Item3* items;
    int item_lo, n_items;   // items [item_lo, item_lo + n_items)
    int B;
    int adj;
    int maxp;               // planes (plane kernels) or column tiles (axis kernel) per item in the grid
    const cx<T>* spec;
    const T* wts;
    const cx<T>* tw;
    const T* in;
    int64_t ld_in;
    T* slots;
    int64_t slot_stride;
    cx<T>* scratch;
    int64_t scratch_base;   // scratch offset of item item_lo
    int64_t pitch;          // Omega row pitch (n2)
    int64_t plane_pitch;    // n1 * n2
};

// One workgroup per (item, vector, gathered plane), plane fastest.
template <class T>
__global__ __launch_bounds__(kPlaneThreads) void plane_fwd_kernel(Conv3Args<T> A) {
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
    constexpr int NT = kPlaneThreads;
    const int q = blockIdx.x % A.maxp, l = blockIdx.x / A.maxp;
    const int rhs = l % A.B, item = l / A.B;
    if (item >= A.n_items) return;
    const Item3 I = A.items[A.item_lo + item];
    const bool adj = A.adj != 0;
    const Planes pl = planes_of(I, adj);
    if (q >= pl.s_n) return;
    Ctx<T> c = plane_ctx_gather<T>(I, adj, q, A.in + (int64_t)rhs * A.ld_in, A.slots + (int64_t)rhs * A.slot_stride,
                                   A.wts, A.spec, A.tw, A.pitch, A.plane_pitch);
    const int tid = threadIdx.x;
    twiddles_to_lds(c, buf + (int64_t)I.p.n0 * I.p.ld, tid, NT);
    phA0<16>(c, buf, tid, NT);
    __syncthreads();
    phA(c, buf, tid, NT);
    __syncthreads();
    phB(c, buf, tid, NT);
    __syncthreads();
    phC(c, buf, tid, NT);
    __syncthreads();
    phD_fwd(c, buf, tid, NT);
    __syncthreads();
    plane_store(c, buf, item_scratch(A.scratch, A.scratch_base, I, A.B, rhs) + (int64_t)(pl.s_off + q) * plane_elems(I),
                tid, NT);
}

// One workgroup per (item, column tile, vector); tiles are dealt to the
// XCDs whole, with all their vectors, so a tile's spectrum columns are
// fetched into one XCD's L2 and reused by every vector.
template <class T>
__global__ __launch_bounds__(kAxisThreads) void axis_kernel(Conv3Args<T> A) {
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
    constexpr int NT = kAxisThreads;
    constexpr int COLS = axis_cols(sizeof(T) == 8 ? 1 : 0);
    const int bid = blockIdx.x;
    const int xcd = bid & 7, l = bid >> 3;
    const int task = xcd + 8 * (l / A.B), rhs = l % A.B;
    const int item = task / A.maxp, tile = task - item * A.maxp;
    if (item >= A.n_items) return;
    const Item3 I = A.items[A.item_lo + item];
    const int64_t pe = plane_elems(I);
    const int c_lo = tile * COLS;
    if (c_lo >= pe) return;
    const int ncols = (int)(pe - c_lo < COLS ? pe - c_lo : COLS);
    Ctx<T> c = axis_ctx<T>(I, A.adj != 0, c_lo, ncols, axis_ld(COLS), A.spec, A.tw);
    cx<T>* sc = item_scratch(A.scratch, A.scratch_base, I, A.B, rhs) + c_lo;
    const int tid = threadIdx.x;
    axis_twiddles_to_lds(c, buf + (int64_t)I.nz * axis_ld(COLS), tid, NT);
    axis_load(c, buf, sc, pe, tid, NT);
    __syncthreads();
    phC(c, buf, tid, NT);
    __syncthreads();
    phD(c, buf, tid, NT);
    __syncthreads();
    phE(c, buf, tid, NT);
    __syncthreads();
    axis_store(c, buf, sc, pe, tid, NT);
}

// One workgroup per (item, vector, written plane), plane fastest.
template <class T>
__global__ __launch_bounds__(kPlaneThreads) void plane_inv_kernel(Conv3Args<T> A) {
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
    constexpr int NT = kPlaneThreads;
    const int q = blockIdx.x % A.maxp, l = blockIdx.x / A.maxp;
    const int rhs = l % A.B, item = l / A.B;
    if (item >= A.n_items) return;
    const Item3 I = A.items[A.item_lo + item];
    const bool adj = A.adj != 0;
    const Planes pl = planes_of(I, adj);
    if (q >= pl.d_n) return;
    Ctx<T> c = plane_ctx_write<T>(I, adj, q, A.in + (int64_t)rhs * A.ld_in, A.slots + (int64_t)rhs * A.slot_stride,
                                  A.wts, A.spec, A.tw, A.pitch);
    const int tid = threadIdx.x;
    twiddles_to_lds(c, buf + (int64_t)I.p.n0 * I.p.ld, tid, NT);
    plane_load(c, buf, item_scratch(A.scratch, A.scratch_base, I, A.B, rhs) + (int64_t)(pl.d_off + q) * plane_elems(I),
               tid, NT);
    __syncthreads();
    phD_inv(c, buf, tid, NT);
    __syncthreads();
    phE(c, buf, tid, NT);
    __syncthreads();
    phF(c, buf, tid, NT);
    __syncthreads();
    phG(c, buf, tid, NT);
    __syncthreads();
    phH<8>(c, buf, tid, NT);
}

template <class T>
static hipError_t conv3_t(const DevPlan& P, const Conv3Launch& L, hipStream_t s) {
    Conv3Args<T> A;
    A.items = P.items3;
    A.item_lo = L.item_lo;
    A.n_items = L.item_hi - L.item_lo;
    A.B = L.B;
    A.adj = L.adjoint ? 1 : 0;
    A.spec = static_cast<const cx<T>*>(P.spec);
    A.wts = static_cast<const T*>(P.wts);
    A.tw = static_cast<const cx<T>*>(P.tw);
    A.in = static_cast<const T*>(L.in);
    A.ld_in = L.ld_in;
    A.slots = static_cast<T*>(L.slots);
    A.slot_stride = L.slot_stride;
    A.scratch = static_cast<cx<T>*>(L.scratch);
    A.scratch_base = L.scratch_base;
    A.pitch = P.cols;
    A.plane_pitch = (int64_t)P.prow * P.cols;
    if (A.n_items <= 0 || A.B <= 0) return hipSuccess;
    const int64_t per = (int64_t)A.n_items * A.B;
    const int64_t g_fwd = per * L.max_gather, g_inv = per * L.max_write;
    const int64_t g_axis = 8 * (((int64_t)A.n_items * L.max_tiles + 7) / 8) * A.B;
    if (g_fwd > 0x7fffffff || g_inv > 0x7fffffff || g_axis > 0x7fffffff) return hipErrorInvalidValue;
    A.maxp = L.max_gather;
    hipLaunchKernelGGL(plane_fwd_kernel<T>, dim3((unsigned)g_fwd), dim3(kPlaneThreads), P.max_lds, s, A);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    A.maxp = L.max_tiles;
    hipLaunchKernelGGL(axis_kernel<T>, dim3((unsigned)g_axis), dim3(kAxisThreads), P.max_lds_axis, s, A);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    A.maxp = L.max_write;
    hipLaunchKernelGGL(plane_inv_kernel<T>, dim3((unsigned)g_inv), dim3(kPlaneThreads), P.max_lds, s, A);
    return hipGetLastError();
}

hipError_t launch_conv3(const DevPlan& P, const Conv3Launch& L, hipStream_t s) {
    if (P.dtype == 1) return conv3_t<double>(P, L, s);
    return conv3_t<float>(P, L, s);
}

template <class T>
__global__ __launch_bounds__(kReduceCols) void reduce_kernel(const Tile* tiles, const Box* cboxes, const T* slots,
                                                             int64_t slot_stride, T* out, int64_t ldo, int64_t pitch,
                                                             int accumulate, T alpha) {
    const Tile t = tiles[blockIdx.x];
    const int rhs = blockIdx.y;
    reduce_tile<T>(t, threadIdx.x, cboxes, slots + (int64_t)rhs * slot_stride, out + (int64_t)rhs * ldo, pitch,
                   accumulate != 0, alpha);
}

// ------------------------------------------------------------ matrix entries
template <class T>
__global__ __launch_bounds__(256) void entries_kernel(EntryTables E, const T* wts, const T* phiE, int64_t n,
                                                      const int64_t* ys, const int64_t* xs, T* out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    out[i] = (T)entry_value<T>(E, wts, phiE, ys + i * E.d, xs + i * E.d);
}

hipError_t launch_entries(const EntryTables& E, int dtype, const void* wts, const void* phiE, int64_t n,
                          const int64_t* ys, const int64_t* xs, void* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + 255) / 256;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    if (dtype == 1)
        hipLaunchKernelGGL(entries_kernel<double>, dim3((unsigned)nb), dim3(256), 0, s, E,
                           static_cast<const double*>(wts), static_cast<const double*>(phiE), n, ys, xs,
                           static_cast<double*>(out));
    else
        hipLaunchKernelGGL(entries_kernel<float>, dim3((unsigned)nb), dim3(256), 0, s, E,
                           static_cast<const float*>(wts), static_cast<const float*>(phiE), n, ys, xs,
                           static_cast<float*>(out));
    return hipGetLastError();
}

// ---------------------------------------------------------------- estimator
constexpr int kEstThreads = 256;

__device__ inline double block_sum(double v, double* sh) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int s = kEstThreads / 2; s > 0; s >>= 1) {
        if (tid < s) sh[tid] += sh[tid + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// One block per leaf: sum over probes i and leaf points x of (Yt - Y)^2, in
// FP64, in a fixed order (probe, plane, then a thread-strided loop over the
// plane's box, then a fixed tree).  Omega is planes x prow x cols.
template <class T>
__global__ __launch_bounds__(kEstThreads) void est_leaf_kernel(const int32_t* leaf_box, int q, const T* Yt, int64_t ldt,
                                                               const T* Y, int64_t ldy, int64_t prow, int64_t pitch,
                                                               double* leaf_sq) {
    __shared__ double sh[kEstThreads];
    const int c = blockIdx.x;
    const int32_t* b = leaf_box + 6 * c;
    const int lz = b[0], lo0 = b[1], lo1 = b[2], nz = b[3], n0 = b[4], n1 = b[5];
    const int64_t cnt = (int64_t)n0 * n1;
    double acc = 0.0;
    for (int i = 0; i < q; ++i) {
        const T* a = Yt + (int64_t)i * ldt;
        const T* y = Y + (int64_t)i * ldy;
        for (int z = 0; z < nz; ++z) {
            const int64_t base = ((int64_t)(lz + z) * prow + lo0) * pitch + lo1;
            for (int64_t e = threadIdx.x; e < cnt; e += kEstThreads) {
                const int64_t idx = base + (e / n1) * pitch + e % n1;
                const double dv = (double)a[idx] - (double)y[idx];
                acc += dv * dv;
            }
        }
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) leaf_sq[c] = s;
}

// Row blocks of Omega: partial sums of (Yt - Y)^2 and Y^2 (each point once).
template <class T>
__global__ __launch_bounds__(kEstThreads) void est_total_kernel(int q, const T* Yt, int64_t ldt, const T* Y, int64_t ldy,
                                                                int64_t n_total, int n_part, double* partials) {
    __shared__ double sh[kEstThreads];
    const int64_t chunk = (n_total + n_part - 1) / n_part;
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = beg + chunk < n_total ? beg + chunk : n_total;
    double dd = 0.0, yy = 0.0;
    for (int i = 0; i < q; ++i) {
        const T* a = Yt + (int64_t)i * ldt;
        const T* b = Y + (int64_t)i * ldy;
        for (int64_t e = beg + threadIdx.x; e < end; e += kEstThreads) {
            const double bv = (double)b[e];
            const double dv = (double)a[e] - bv;
            dd += dv * dv;
            yy += bv * bv;
        }
    }
    const double s0 = block_sum(dd, sh);
    const double s1 = block_sum(yy, sh);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s0;
        partials[2 * blockIdx.x + 1] = s1;
    }
}

// The totals from the row-block partials, one thread, partials in index
// order (FP64): totals[0] = sum (Yt - Y)^2, totals[1] = sum Y^2.
__global__ __launch_bounds__(64) void est_final_kernel(const double* partials, int n_part, double* totals) {
    if (threadIdx.x != 0) return;
    double dd = 0.0, yy = 0.0;
    for (int i = 0; i < n_part; ++i) {
        dd += partials[2 * i];
        yy += partials[2 * i + 1];
    }
    totals[0] = dd;
    totals[1] = yy;
}

// Zero fill of B vectors of N elements at stride ld (the outputs that the
// colour launches then add into; a kernel rather than a memset node, so the
// apply records into graphs safely).
template <class T>
__global__ __launch_bounds__(256) void fill_zero_kernel(T* out, int64_t ld, int64_t N, int B) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int b = 0; b < B; ++b) {
        T* o = out + (int64_t)b * ld;
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += stride) o[i] = T(0);
    }
}

hipError_t launch_fill_zero(int dtype, void* out, int64_t ld, int64_t N, int B, hipStream_t s) {
    if (N <= 0 || B <= 0) return hipSuccess;
    const int64_t want = (N + 255) / 256;
    const unsigned nb = (unsigned)(want < 8192 ? want : 8192);
    if (dtype == 1)
        hipLaunchKernelGGL(fill_zero_kernel<double>, dim3(nb), dim3(256), 0, s, static_cast<double*>(out), ld, N, B);
    else
        hipLaunchKernelGGL(fill_zero_kernel<float>, dim3(nb), dim3(256), 0, s, static_cast<float*>(out), ld, N, B);
    return hipGetLastError();
}

// ---------------------------------------------------------------- launchers
template <class T>
static hipError_t conv_t(const DevPlan& P, const Item* items, bool adj, int item_lo, int item_hi, int B,
                         const void* in, int64_t ld_in, void* slots, int64_t slot_stride, void* out, int64_t ldo,
                         hipStream_t s, bool item_major, LaunchEvents ev) {
    ConvArgs<T> A;
    A.items = items;
    A.item_lo = item_lo;
    A.n_items = item_hi - item_lo;
    A.B = B;
    A.adj = adj ? 1 : 0;
    A.spec = static_cast<const cx<T>*>(P.spec);
    A.wts = static_cast<const T*>(P.wts);
    A.tw = static_cast<const cx<T>*>(P.tw);
    A.in = static_cast<const T*>(in);
    A.ld_in = ld_in;
    A.slots = static_cast<T*>(slots);
    A.slot_stride = slot_stride;
    A.out = static_cast<T*>(out);
    A.ldo = ldo;
    A.pitch = P.cols;
    A.item_major = item_major ? 1 : 0;
    if (A.n_items <= 0 || B <= 0) return record_unused(ev, s);
    const int64_t nblk = (out || item_major) ? (int64_t)A.n_items * B : 8 * ((int64_t)((A.n_items + 7) / 8) * B);
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 grid((unsigned)nblk);
    if (P.conv_threads == 512) {
        if (out)
            PC_LAUNCH((conv_kernel<T, 512, true>), grid, dim3(512), P.max_lds, s, ev.start, ev.stop, A);
        else
            PC_LAUNCH((conv_kernel<T, 512, false>), grid, dim3(512), P.max_lds, s, ev.start, ev.stop, A);
    } else {
        if constexpr (sizeof(T) == 4) {
            if (out)
                PC_LAUNCH((conv_kernel<T, 1024, true>), grid, dim3(1024), P.max_lds, s, ev.start, ev.stop, A);
            else
                PC_LAUNCH((conv_kernel<T, 1024, false>), grid, dim3(1024), P.max_lds, s, ev.start, ev.stop, A);
        } else {
            return hipErrorInvalidValue;   // FP64 items always use 512 threads
        }
    }
    return hipGetLastError();
}

// LDS of a persistent launch: the item data, then the unit slot (16 B).
static int persistent_q_off(const DevPlan& P) { return (P.max_lds + 15) & ~15; }

bool persistent_fits(const DevPlan& P) {
    return P.queue != nullptr && persistent_q_off(P) + 16 <= kLdsBytes && (P.conv_threads == 512 || P.dtype == 0);
}

template <class T>
static hipError_t conv_persistent_t(const DevPlan& P, bool adj, int B, const void* in, int64_t ld_in, void* slots,
                                    int64_t slot_stride, hipStream_t s) {
    if (!persistent_fits(P)) return hipErrorInvalidValue;
    if (P.n_items <= 0 || B <= 0) return hipSuccess;
    ConvArgs<T> A;
    A.items = P.items;
    A.item_lo = 0;
    A.n_items = P.n_items;
    A.B = B;
    A.adj = adj ? 1 : 0;
    A.spec = static_cast<const cx<T>*>(P.spec);
    A.wts = static_cast<const T*>(P.wts);
    A.tw = static_cast<const cx<T>*>(P.tw);
    A.in = static_cast<const T*>(in);
    A.ld_in = ld_in;
    A.slots = static_cast<T*>(slots);
    A.slot_stride = slot_stride;
    A.out = nullptr;
    A.ldo = 0;
    A.pitch = P.cols;
    A.item_major = 0;
    const int q_off = persistent_q_off(P), lds = q_off + 16;
    // workgroups per CU that LDS and the 2048 threads of a CU allow
    const int per_cu = std::max(1, std::min(kLdsBytes / lds, 2048 / P.conv_threads));
    const int grid = std::max(8, (P.n_cu * per_cu) / 8 * 8);
    hipError_t e = launch_fill_zero(0, P.queue, 128, 128, 1, s);   // 128 int counters = zero floats
    if (e != hipSuccess) return e;
    if (P.conv_threads == 512)
        hipLaunchKernelGGL((conv_persistent_kernel<T, 512>), dim3((unsigned)grid), dim3(512), lds, s, A, P.queue, q_off);
    else if constexpr (sizeof(T) == 4)
        hipLaunchKernelGGL((conv_persistent_kernel<T, 1024>), dim3((unsigned)grid), dim3(1024), lds, s, A, P.queue,
                           q_off);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_conv_persistent(const DevPlan& P, bool adjoint, int B, const void* in, int64_t ld_in, void* slots,
                                  int64_t slot_stride, hipStream_t s) {
    if (P.dtype == 1) return conv_persistent_t<double>(P, adjoint, B, in, ld_in, slots, slot_stride, s);
    return conv_persistent_t<float>(P, adjoint, B, in, ld_in, slots, slot_stride, s);
}

hipError_t launch_conv_split(const DevPlan& P, bool adjoint, int B, const void* in, int64_t ld_in, void* slots,
                             int64_t slot_stride, hipStream_t s, LaunchEvents ev) {
    if (P.dtype != 0) return hipErrorInvalidValue;
    if (B <= 0 || (P.n_big <= 0 && P.n_small <= 0)) return record_unused(ev, s);
    ConvArgs<float> A;
    A.items = P.items_split;
    A.item_lo = 0;
    A.n_items = P.n_big;
    A.B = B;
    A.adj = adjoint ? 1 : 0;
    A.spec = static_cast<const cx<float>*>(P.spec);
    A.wts = static_cast<const float*>(P.wts);
    A.tw = static_cast<const cx<float>*>(P.tw);
    A.in = static_cast<const float*>(in);
    A.ld_in = ld_in;
    A.slots = static_cast<float*>(slots);
    A.slot_stride = slot_stride;
    A.out = nullptr;
    A.ldo = 0;
    A.pitch = P.cols;
    A.item_major = 0;
    const int64_t nblk_big = 8 * ((int64_t)((P.n_big + 7) / 8) * B);
    const int64_t nblk_small = 8 * ((int64_t)((P.n_small + 7) / 8) * B);
    if (nblk_big > 0x7fffffff || nblk_small > 0x7fffffff) return hipErrorInvalidValue;
    // timing: the start event rides on the first kernel, the stop event on the last
    if (P.n_big > 0) {
        const hipEvent_t stop = P.n_small > 0 ? nullptr : ev.stop;
        PC_LAUNCH((conv_kernel<float, 1024, false>), dim3((unsigned)nblk_big), dim3(1024), P.lds_big, s, ev.start,
                  stop, A);
    }
    if (P.n_small > 0) {
        A.item_lo = P.n_big;
        A.n_items = P.n_small;
        const hipEvent_t start = P.n_big > 0 ? nullptr : ev.start;
        PC_LAUNCH((conv_kernel_small<float>), dim3((unsigned)nblk_small), dim3(512), P.lds_small, s, start, ev.stop,
                  A);
    }
    return hipGetLastError();
}

hipError_t launch_conv(const DevPlan& P, const Item* items, bool adjoint, int item_lo, int item_hi, int B,
                       const void* in, int64_t ld_in, void* slots, int64_t slot_stride, void* out, int64_t ldo,
                       hipStream_t s, bool item_major, LaunchEvents ev) {
    if (P.dtype == 1)
        return conv_t<double>(P, items, adjoint, item_lo, item_hi, B, in, ld_in, slots, slot_stride, out, ldo, s,
                              item_major, ev);
    return conv_t<float>(P, items, adjoint, item_lo, item_hi, B, in, ld_in, slots, slot_stride, out, ldo, s,
                         item_major, ev);
}

hipError_t launch_reduce(const DevPlan& P, bool adjoint, int B, const void* slots, int64_t slot_stride, void* out,
                         int64_t ldo, hipStream_t s, bool accumulate, double alpha, LaunchEvents ev) {
    const int nt = adjoint ? P.n_tiles_adj : P.n_tiles_fwd;
    if (nt <= 0 || B <= 0) return record_unused(ev, s);
    const Tile* tiles = adjoint ? P.tiles_adj : P.tiles_fwd;
    const Box* cboxes = adjoint ? P.cboxes_adj : P.cboxes_fwd;
    dim3 grid((unsigned)nt, (unsigned)B);
    if (P.dtype == 1)
        PC_LAUNCH(reduce_kernel<double>, grid, dim3(kReduceCols), 0, s, ev.start, ev.stop, tiles, cboxes,
                  static_cast<const double*>(slots), slot_stride, static_cast<double*>(out), ldo, (int64_t)P.cols,
                  accumulate ? 1 : 0, alpha);
    else
        PC_LAUNCH(reduce_kernel<float>, grid, dim3(kReduceCols), 0, s, ev.start, ev.stop, tiles, cboxes,
                  static_cast<const float*>(slots), slot_stride, static_cast<float*>(out), ldo, (int64_t)P.cols,
                  accumulate ? 1 : 0, (float)alpha);
    return hipGetLastError();
}

hipError_t launch_est(int dtype, const int32_t* leaf_box, int n_leaves, int q, const void* Yt, int64_t ldt,
                      const void* Y, int64_t ldy, int planes, int prow, int cols, double* leaf_sq, double* partials,
                      int n_part, double* totals, hipStream_t s) {
    const int64_t n_total = (int64_t)planes * prow * cols;
    if (dtype == 1) {
        hipLaunchKernelGGL(est_leaf_kernel<double>, dim3(n_leaves), dim3(kEstThreads), 0, s, leaf_box, q,
                           static_cast<const double*>(Yt), ldt, static_cast<const double*>(Y), ldy, (int64_t)prow,
                           (int64_t)cols, leaf_sq);
        hipLaunchKernelGGL(est_total_kernel<double>, dim3(n_part), dim3(kEstThreads), 0, s, q,
                           static_cast<const double*>(Yt), ldt, static_cast<const double*>(Y), ldy, n_total, n_part,
                           partials);
    } else {
        hipLaunchKernelGGL(est_leaf_kernel<float>, dim3(n_leaves), dim3(kEstThreads), 0, s, leaf_box, q,
                           static_cast<const float*>(Yt), ldt, static_cast<const float*>(Y), ldy, (int64_t)prow,
                           (int64_t)cols, leaf_sq);
        hipLaunchKernelGGL(est_total_kernel<float>, dim3(n_part), dim3(kEstThreads), 0, s, q,
                           static_cast<const float*>(Yt), ldt, static_cast<const float*>(Y), ldy, n_total, n_part,
                           partials);
    }
    hipLaunchKernelGGL(est_final_kernel, dim3(1), dim3(64), 0, s, partials, n_part, totals);
    return hipGetLastError();
}

hipError_t set_kernel_attributes() {
    const void* fns[] = {
        reinterpret_cast<const void*>(&conv_kernel<float, 1024, false>),
        reinterpret_cast<const void*>(&conv_kernel<float, 512, false>),
        reinterpret_cast<const void*>(&conv_kernel<double, 512, false>),
        reinterpret_cast<const void*>(&conv_kernel<float, 1024, true>),
        reinterpret_cast<const void*>(&conv_kernel<float, 512, true>),
        reinterpret_cast<const void*>(&conv_kernel<double, 512, true>),
        reinterpret_cast<const void*>(&conv_kernel_small<float>),
        reinterpret_cast<const void*>(&conv_persistent_kernel<float, 1024>),
        reinterpret_cast<const void*>(&conv_persistent_kernel<float, 512>),
        reinterpret_cast<const void*>(&conv_persistent_kernel<double, 512>),
        reinterpret_cast<const void*>(&plane_fwd_kernel<float>), reinterpret_cast<const void*>(&plane_fwd_kernel<double>),
        reinterpret_cast<const void*>(&axis_kernel<float>),      reinterpret_cast<const void*>(&axis_kernel<double>),
        reinterpret_cast<const void*>(&plane_inv_kernel<float>), reinterpret_cast<const void*>(&plane_inv_kernel<double>)};
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace pc
