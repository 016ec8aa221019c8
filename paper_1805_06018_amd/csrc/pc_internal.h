// Internal definitions shared by the host planner (pc_host.cpp) and the HIP
// kernels (pc_kernels.hip).  Not part of the public ABI.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

namespace pc {

// Largest radix handled by the register codelets; every FFT length used by
// the library is a * b with a, b in {1,2,3,4,5,6,7,8,9,10,12,14,15,16}.
constexpr int kMaxRadix = 16;
constexpr int kLdsBytes = 160 * 1024;  // LDS per CU on gfx950
// Largest item LDS (box and twiddles) that runs two workgroups per CU.
constexpr int kSmallItemLds = kLdsBytes / 2 - 1024;
constexpr int kReduceCols = 256;       // reduce tile width (threads)
constexpr int kReduceRows = 8;         // reduce tile height (accumulators per thread)
constexpr int kAxisThreads = 256;      // threads of the 3-D axis-0 kernel
constexpr int kPlaneThreads = 256;     // threads of the 3-D plane kernels (one plane per workgroup)

// Columns (flattened axis-1 x axis-2 frequencies) per block of the 3-D
// axis-0 kernel: the block holds nz x (cols + 1) complex values in LDS.
// FP32: 60 columns keep an 81-deep block (the 128^3 workload) with its
// twiddles under 40 KB, so four blocks share a CU (64: three; 22.2 against
// 23.3 ms per 16-vector apply).
constexpr int axis_cols(int dtype) { return dtype == 1 ? 32 : 60; }

// One convolution work item: a patch (or a row piece of a patch) of the
// 2-D product-convolution sum.  FFT index (i0, i1) <-> Omega point
// (g0 + i0, g1 + i1).  The input box of the forward sum (the patch's
// weighted gather box I) sits at FFT offset (in_off0, in_off1) with extent
// (in_n0, in_n1); the output box O = (I + kernel box) n Omega sits at FFT
// offset (out_off0, out_off1) with extent (out_n0, out_n1) (offset 0 for the
// whole operator; block applies clip both boxes).  The adjoint swaps the
// roles.
struct Item {
    int32_t n0;          // column FFT length (axis 0); 1 for 1-D problems
    int32_t a0, b0;      // n0 = a0 * b0
    int32_t m;           // row complex FFT length; the real row length is 2m
    int32_t am, bm;      // m = am * bm
    int32_t ld;          // LDS row stride (complex elements), >= m + 1, odd
    int32_t tw0, twm, tw2m;  // offsets of the twiddle tables for n0, m, 2m
    int32_t g0, g1;      // Omega coordinates of FFT index (0, 0)
    int32_t in_off0, in_off1, in_n0, in_n1;
    int32_t out_n0, out_n1;
    int32_t out_off0, out_off1;  // FFT offset of the output box (0 except in block applies)
    int32_t patch;       // k
    int32_t w_ld;        // row stride of the weight table (the patch's box width)
    int64_t w_off;       // weight table (in_n0 x in_n1 block, row stride w_ld)
    int64_t spec_off;    // spectrum (n0 x (m+1), slot-permuted)
    int64_t slot_fwd;    // forward staging offset (out_n0 x out_n1)
    int64_t slot_adj;    // adjoint staging offset (in_n0 x in_n1)
};

// 3-D work item: the patch's FFT box nz x n1 x n2 (n2 = 2m) is handled as
// 2-D FFTs of its planes along axes 1 and 2 (in LDS, described by 'p', whose
// boxes, weights strides and Omega origins refer to axes 1 and 2) plus an
// axis-0 pass over the planes' spectra, which sit in a global scratch area of
// nz x n1 x (m+1) complex values per vector.
struct Item3 {
    Item p;
    int32_t nz, az, bz, twz;                 // axis-0 FFT length, radices, twiddle table
    int32_t gz, in_offz, in_nz, out_nz;      // axis-0 origin, input box offset/extent, output extent
    int32_t w_plane;                         // weight table plane stride (m1 * m2)
    int32_t out_offz;                        // axis-0 FFT offset of the output box (0 except in block applies)
    int64_t scratch_off;                     // complex elements, per vector
};

// Output tile of the deterministic reduction and the staging boxes that
// overlap it (a CSR range into the contributor list, ascending item order).
struct Tile {
    int32_t r0, c0, nr, nc;
    int32_t beg, end;
};

// Staging box of one contributor: Omega box and staging offset per vector.
struct Box {
    int32_t lo0, lo1, n0, n1;
    int64_t off;
};

}  // namespace pc
