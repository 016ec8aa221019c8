// Host-side construction of the product-convolution operator: grid
// derivation (Sec. 2.2), harmonic weights (Sec. 2.4), extended impulse
// responses (Sec. 2.5), FFT planning and FP64 spectra.  Pure C++ (no HIP
// runtime calls) so the same planner serves the library and its CPU
// emulation build.
#pragma once
#include <map>
#include <utility>
#include <stdint.h>
#include <complex>
#include <string>
#include <vector>
#include "../../include/pc.h"
#include "pc_internal.h"

namespace pc {

struct CreateArgs {
    int d;
    const int64_t* shape;
    int64_t n_leaves;
    const int64_t* leaf_lo;
    const int64_t* leaf_hi;
    int64_t r;
    const int64_t* points;
    const int64_t* radius;
    const double* phi;
    const int64_t* phi_off;
    int dtype;
    uint32_t flags;
    int64_t n_sel = -1;              // >= 0: keep only the terms of these points
    const int64_t* sel = nullptr;
};

struct Plan {
    int d = 0;
    int64_t shape[3] = {1, 1, 1};
    int64_t N = 0;
    int rows = 1, cols = 1;          // 2-D view of Omega (d = 1: one row; d = 3: rows = n0 * n1)
    int planes = 1, prow = 1;        // Omega as planes x prow x cols (d < 3: one plane of 'rows' rows)
    int dtype = 0;
    uint32_t flags = 0;
    int64_t r = 0, L = 0;
    std::vector<char> sel;           // [r]: 1 if point k's term is part of the operator
    std::vector<Item> items;         // d = 1, 2
    std::vector<Item3> items3;       // d = 3
    int64_t scratch_per_vec = 0;     // d = 3: complex scratch elements per vector over all items
    int max_lds_axis = 0;            // d = 3: LDS of the axis-0 kernel
    std::vector<double> spec;        // interleaved complex, FP64, pre-scaled
    std::vector<double> wts;         // FP64 weight tables
    std::vector<double> tw;          // interleaved complex twiddle tables
    std::vector<Tile> tiles_fwd, tiles_adj;
    std::vector<int32_t> contrib_fwd, contrib_adj;
    // Canonical summation order of the contributions to an output point
    // (d <= 2): ascending (colour, item), where the items of one colour write
    // pairwise disjoint boxes (forward: output boxes, adjoint: input boxes).
    // order_*: item indices in that order; cbeg_*: colour c holds positions
    // [cbeg[c], cbeg[c + 1]) of order_*.  Empty for d = 3.
    std::vector<int32_t> order_fwd, order_adj, cbeg_fwd, cbeg_adj;
    std::vector<Box> boxes_fwd, boxes_adj;     // staging box of every item (canonical order)
    std::vector<Box> cboxes_fwd, cboxes_adj;   // staging box of every tile contributor
    std::vector<int32_t> leaf_box;   // [L][6]: plane, row, col origin and extents (planes x prow x cols view)
    // matrix entries (Sec. 3.1), in the planes x prow x cols view
    std::vector<int32_t> leaf_pts_off, leaf_pts;   // CSR: points on each closed leaf, ascending
    std::vector<int64_t> pt_wbase;   // [r] weight table offset of point k, -1 if its term is not kept
    std::vector<int32_t> pt_ubox;    // [r][6] bbox(U_k): origin, extents
    std::vector<int64_t> pt_eoff;    // [r] offset of phi_k^E in phiE, -1 if not kept
    std::vector<int32_t> pt_ebox;    // [r][6] box of phi_k^E: offset origin zlo, extents
    std::vector<double> phiE;        // extended kernels phi_k^E, FP64
    int64_t slot_fwd = 0, slot_adj = 0;   // staging elements per vector
    int max_lds = 0;
    int conv_threads = 1024;         // workgroup size of the 1-D/2-D convolution kernel
    // statistics
    int64_t sum_fft_points = 0;
    double alg_flops = 0.0;
    int64_t kernel_elems = 0;
};

// Builds the plan; returns PC_OK or an error status with a message.
pc_status build_plan(const CreateArgs& a, Plan& p, std::string& err);

// FFT lengths usable by the kernels: n = a * b with a, b radices.
bool fft_factor(int n, int* a, int* b);
int next_fft_size(int need);

// Twiddle tables in the layout the kernels read (interleaved complex FP64,
// appended to tw; the returned value is the table's complex offset).
// TwiddleTables keeps one table per (kind, a, b):
//   pass(a, b): the inter-pass twiddles of a length n = a b transform, one
//     run per pass-1 task: entry j0 (a - 1) + k1 - 1 = w_n^(j0 k1) for
//     j0 < b, 1 <= k1 < a (b (a - 1) entries);
//   pair(am, bm): the real-row post-/pre-processing twiddles of m = am bm,
//     one run per frequency group: entry k1 bm + k0 = w_2m^(k1 + am k0) for
//     k1 <= am / 2, k0 < bm.
// with w_n = exp(-2 pi i / n).
struct TwiddleTables {
    std::vector<double>* tw;
    std::map<std::pair<int, int>, int> pass_off, pair_off;
    int pass(int a, int b);
    int pair(int am, int bm);
};
// Complex elements of an item's three tables (column pass, row pass, pairs).
int64_t twiddle_elems(int a0, int b0, int am, int bm);

// ---- planner internals shared by the 2-D and 3-D planners
using cd = std::complex<double>;
constexpr double kPi = 3.14159265358979323846264338327950288;
// slot of frequency k in the two-pass order of a length a * b transform
int perm_slot(int k, int a, int b);
int smallest_7smooth(int64_t need);
// FP64 DFT of one length with prime factors <= 64:
// y[k] = sum_j x[j stride] w_n^(j k), w_n = exp(-2 pi i / n).
struct Dft64 {
    int n;
    std::vector<int> fac;          // prime factors
    std::vector<cd> W;             // w_n^e, e < n
    explicit Dft64(int n_);
    void run(const cd* x, int64_t stride, cd* y) const;

  private:
    void rec(const cd* x, int64_t stride, int len, int level, cd* y) const;
};
// cached plan of length n (per thread)
const Dft64& dft64(int n);
// Sine eigenbasis of the tridiagonal T_n = tridiag(-1, 2, -1):
// T_n = S diag(lambda) S with S symmetric orthogonal (row-major n x n).
struct SineBasis {
    int n = 0;
    std::vector<double> S, lam;
    explicit SineBasis(int n_);
};
// reduction tiles of a rows x cols view with, per tile, the boxes meeting it
// in ascending box order
bool build_tiles(const std::vector<Box>& boxes, int rows, int cols, std::vector<Tile>& tiles,
                 std::vector<int32_t>& contrib, std::string& err);
// Greedy colouring (first fit in the given order) of the boxes of a
// rows x cols view: boxes of one colour are pairwise disjoint.  Writes the
// order (ascending colour, then position) and the colour ranges.
void colour_boxes(const std::vector<Box>& boxes, int rows, int cols, std::vector<int32_t>& order,
                  std::vector<int32_t>& cbeg);
// reduction tiles and contributor boxes of both directions from the
// per-item staging boxes (given in the canonical summation order)
bool finish_tiles(Plan& p, std::vector<Box>& bf, std::vector<Box>& ba, std::string& err);
// Block apply (Sec. 3.3): OUT_T = A~[T, S] U_S or A~*[T, S] U_S, with U_S
// row-major over the box S and OUT_T over the box T (d <= 2).  Every work
// item whose gather box meets S and whose written box meets T takes part,
// both boxes clipped; the FFT of the whole item is kept, so the clipped
// convolution is exact.  Gather coordinates are S-local, reduction tiles
// T-local.
struct BlockPlan {
    std::vector<Item> items;         // d <= 2
    std::vector<Item3> items3;       // d = 3 (scratch offsets local to the call)
    std::vector<Tile> tiles;
    std::vector<Box> cboxes;
    int64_t per = 0;                 // staging elements per vector
    int t_rows = 0, t_cols = 0;      // T in the reduction view (d = 3: rows = T0 * T1)
    int s_rows = 0, s_cols = 0;      // S in the gather view (d = 3: rows per plane)
    int s_planes = 1, t_prow = 1;    // d = 3: planes of S, rows per plane of T
};
pc_status build_block(const Plan& P, bool adjoint, const int64_t* tlo, const int64_t* thi, const int64_t* slo,
                      const int64_t* shi, BlockPlan& B, std::string& err);

// 3-D operators (called by build_plan after the argument checks)
pc_status build_plan_3d(const CreateArgs& a, Plan& p, std::string& err);
// 3-D block plan (called by build_block)
pc_status build_block3(const Plan& P, bool adjoint, const int64_t* tlo, const int64_t* thi, const int64_t* slo,
                       const int64_t* shi, BlockPlan& B, std::string& err);

}  // namespace pc
