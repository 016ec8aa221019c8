// Host-side construction of the product-convolution operator: grid
// derivation (Sec. 2.2), harmonic weights (Sec. 2.4), extended impulse
// responses (Sec. 2.5), FFT planning and FP64 spectra.  Pure C++ (no HIP
// runtime calls) so the same planner serves the library and its CPU
// emulation build.
#pragma once
#include <stdint.h>
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
};

struct Plan {
    int d = 0;
    int64_t shape[3] = {1, 1, 1};
    int64_t N = 0;
    int rows = 1, cols = 1;          // 2-D view of Omega (d = 1: one row)
    int dtype = 0;
    uint32_t flags = 0;
    int64_t r = 0, L = 0;
    std::vector<Item> items;
    std::vector<double> spec;        // interleaved complex, FP64, pre-scaled
    std::vector<double> wts;         // FP64 weight tables
    std::vector<double> tw;          // interleaved complex twiddle tables
    std::vector<Tile> tiles_fwd, tiles_adj;
    std::vector<int32_t> contrib_fwd, contrib_adj;
    std::vector<Box> boxes_fwd, boxes_adj;     // staging box of every item
    std::vector<Box> cboxes_fwd, cboxes_adj;   // staging box of every tile contributor
    std::vector<int32_t> leaf_box;   // [L][4]: lo0, lo1, n0, n1 in the 2-D view
    int64_t slot_fwd = 0, slot_adj = 0;   // staging elements per vector
    int max_lds = 0;
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

}  // namespace pc
