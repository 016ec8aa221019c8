// CPU emulation of the convolution and reduction kernels (test tool only).
//
// Built host-only into a separate library (libpc_emu.so), never linked into
// the product library.  It runs the same phase functions as the GPU kernel,
// one simulated thread after another with the phase boundary standing in for
// the barrier, on exact-size host buffers so that an address sanitizer build
// reports any out-of-range index.  It checks the kernels' indexing on the CPU
// before they run on a GPU.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "pc_entries.h"
#include "pc_phases3.h"
#include "pc_plan.h"

namespace {
thread_local std::string g_emu_err;

template <class T>
void reduce_all(const pc::Plan& P, bool adj, int64_t B, const std::vector<T>& slots, int64_t per, T* OUT, int64_t ldo);

// direct: the colour launches of the library (outputs zeroed, then every
// item in the canonical order adds its written box into the output);
// otherwise every item stages its box and the reduction sums them.
template <class T>
void emu_apply(const pc::Plan& P, bool adj, int64_t B, const T* U, int64_t ldu, T* OUT, int64_t ldo,
               bool direct = false) {
    using C = pc::cx<T>;
    const int64_t N = P.N;
    std::vector<T> spec(P.spec.begin(), P.spec.end());
    std::vector<T> wts(P.wts.begin(), P.wts.end());
    std::vector<T> tw(P.tw.begin(), P.tw.end());
    const int64_t per = adj ? P.slot_adj : P.slot_fwd;
    std::vector<T> in((size_t)(B * N));
    for (int64_t b = 0; b < B; ++b) std::memcpy(&in[(size_t)(b * N)], U + b * ldu, sizeof(T) * (size_t)N);
    std::vector<T> slots(direct ? 0 : (size_t)(B * per), T(0));
    std::vector<T> out(direct ? (size_t)(B * N) : 0, T(0));
    const std::vector<int32_t>& ord = adj ? P.order_adj : P.order_fwd;
    for (int64_t b = 0; b < B; ++b) {
        for (size_t pos = 0; pos < P.items.size(); ++pos) {
            const pc::Item& it = P.items[direct ? (size_t)ord[pos] : pos];
            std::vector<C> buf((size_t)(it.n0 * it.ld + pc::tw_lds_elems(it)));
            for (auto& v : buf) v = C{T(1e30), T(1e30)};   // poison: unwritten reads show up
            pc::Ctx<T> c = pc::make_ctx<T>(it, adj, &in[(size_t)(b * N)], direct ? nullptr : &slots[(size_t)(b * per)],
                                           wts.data(), reinterpret_cast<const C*>(spec.data()),
                                           reinterpret_cast<const C*>(tw.data()), P.cols,
                                           direct ? &out[(size_t)(b * N)] : nullptr);
            const int nth = P.conv_threads;
            {
                pc::Ctx<T> c0 = c;
                for (int t = 0; t < nth; ++t) {
                    c0 = c;
                    pc::twiddles_to_lds(c0, buf.data() + (int64_t)it.n0 * it.ld, t, nth);
                }
                c = c0;
            }
            for (int t = 0; t < nth; ++t) pc::phA0(c, buf.data(), t, nth);
            for (int t = 0; t < nth; ++t) pc::phA(c, buf.data(), t, nth);
            for (int t = 0; t < nth; ++t) pc::phB(c, buf.data(), t, nth);
            for (int t = 0; t < nth; ++t) pc::phC(c, buf.data(), t, nth);
            for (int t = 0; t < nth; ++t) pc::phD(c, buf.data(), t, nth);
            for (int t = 0; t < nth; ++t) pc::phE(c, buf.data(), t, nth);
            for (int t = 0; t < nth; ++t) pc::phF(c, buf.data(), t, nth);
            for (int t = 0; t < nth; ++t) pc::phG(c, buf.data(), t, nth);
            for (int t = 0; t < nth; ++t) pc::phH(c, buf.data(), t, nth);
        }
    }
    if (direct) {
        for (int64_t b = 0; b < B; ++b) std::memcpy(OUT + b * ldo, &out[(size_t)(b * N)], sizeof(T) * (size_t)N);
        return;
    }
    reduce_all(P, adj, B, slots, per, OUT, ldo);
}

template <class T>
void reduce_all(const pc::Plan& P, bool adj, int64_t B, const std::vector<T>& slots, int64_t per, T* OUT,
                int64_t ldo) {
    const int64_t N = P.N;
    std::vector<T> out((size_t)(B * N), T(0));
    const auto& tiles = adj ? P.tiles_adj : P.tiles_fwd;
    const auto& cboxes = adj ? P.cboxes_adj : P.cboxes_fwd;
    for (int64_t b = 0; b < B; ++b)
        for (const pc::Tile& t : tiles)
            for (int col = 0; col < pc::kReduceCols; ++col)
                pc::reduce_tile<T>(t, col, cboxes.data(), &slots[(size_t)(b * per)], &out[(size_t)(b * N)], P.cols);
    for (int64_t b = 0; b < B; ++b) std::memcpy(OUT + b * ldo, &out[(size_t)(b * N)], sizeof(T) * (size_t)N);
}

// 3-D: the three kernels of pc_phases3.h, one simulated block after another,
// on one scratch area holding every item and vector (the layout of a launch
// over all items with B vectors).  items/per/tiles/cboxes: the operator's or
// a block apply's; in_pitch, in_prow: gather view; out_cols: reduction pitch.
template <class T>
void emu_3d(const pc::Plan& P, const std::vector<pc::Item3>& items, int64_t per, const std::vector<pc::Tile>& tiles,
            const std::vector<pc::Box>& cboxes, int64_t n_in, int64_t in_pitch, int64_t in_prow, int64_t n_out,
            int out_cols, bool adj, int64_t B, const T* U, int64_t ldu, T* OUT, int64_t ldo) {
    using C = pc::cx<T>;
    std::vector<T> spec(P.spec.begin(), P.spec.end());
    std::vector<T> wts(P.wts.begin(), P.wts.end());
    std::vector<T> tw(P.tw.begin(), P.tw.end());
    const C* specc = reinterpret_cast<const C*>(spec.data());
    const C* twc = reinterpret_cast<const C*>(tw.data());
    std::vector<T> in((size_t)(B * n_in));
    for (int64_t b = 0; b < B; ++b) std::memcpy(&in[(size_t)(b * n_in)], U + b * ldu, sizeof(T) * (size_t)n_in);
    std::vector<T> slots((size_t)std::max<int64_t>(B * per, 1), T(0));
    int64_t sc_total = 0;
    for (const pc::Item3& I : items) sc_total = std::max(sc_total, I.scratch_off + I.nz * pc::plane_elems(I));
    std::vector<C> scratch((size_t)std::max<int64_t>(sc_total * B, 1), C{T(1e30), T(1e30)});
    const int NT = pc::kPlaneThreads;
    const int COLS = pc::axis_cols(P.dtype), LDA = pc::axis_ld(COLS);
    const int64_t plane_pitch = in_prow * in_pitch;
    for (const pc::Item3& I : items) {
        const pc::Planes pl = pc::planes_of(I, adj);
        const int64_t pe = pc::plane_elems(I);
        for (int64_t b = 0; b < B; ++b) {
            const T* iv = &in[(size_t)(b * n_in)];
            T* sv = &slots[(size_t)(b * per)];
            C* sc = pc::item_scratch(scratch.data(), 0, I, (int)B, (int)b);
            for (int q = 0; q < pl.s_n; ++q) {
                std::vector<C> buf((size_t)(I.p.n0 * I.p.ld + pc::tw_lds_elems(I.p)), C{T(1e30), T(1e30)});
                pc::Ctx<T> c =
                    pc::plane_ctx_gather<T>(I, adj, q, iv, sv, wts.data(), specc, twc, in_pitch, plane_pitch);
                {
                    pc::Ctx<T> c0 = c;
                    for (int t = 0; t < NT; ++t) {
                        c0 = c;
                        pc::twiddles_to_lds(c0, buf.data() + (int64_t)I.p.n0 * I.p.ld, t, NT);
                    }
                    c = c0;
                }
                for (int t = 0; t < NT; ++t) pc::phA0(c, buf.data(), t, NT);
                for (int t = 0; t < NT; ++t) pc::phA(c, buf.data(), t, NT);
                for (int t = 0; t < NT; ++t) pc::phB(c, buf.data(), t, NT);
                for (int t = 0; t < NT; ++t) pc::phC(c, buf.data(), t, NT);
                for (int t = 0; t < NT; ++t) pc::phD_fwd(c, buf.data(), t, NT);
                for (int t = 0; t < NT; ++t) pc::plane_store(c, buf.data(), sc + (int64_t)(pl.s_off + q) * pe, t, NT);
            }
            for (int64_t c_lo = 0; c_lo < pe; c_lo += COLS) {
                const int ncols = (int)std::min<int64_t>(COLS, pe - c_lo);
                std::vector<C> buf((size_t)(I.nz * LDA + I.nz), C{T(1e30), T(1e30)});
                pc::Ctx<T> c = pc::axis_ctx<T>(I, adj, (int)c_lo, ncols, LDA, specc, twc);
                const int AT = pc::kAxisThreads;
                {
                    pc::Ctx<T> c0 = c;
                    for (int t = 0; t < AT; ++t) {
                        c0 = c;
                        pc::axis_twiddles_to_lds(c0, buf.data() + (int64_t)I.nz * LDA, t, AT);
                    }
                    c = c0;
                }
                for (int t = 0; t < AT; ++t) pc::axis_load(c, buf.data(), sc + c_lo, pe, t, AT);
                for (int t = 0; t < AT; ++t) pc::phC(c, buf.data(), t, AT);
                for (int t = 0; t < AT; ++t) pc::phD(c, buf.data(), t, AT);
                for (int t = 0; t < AT; ++t) pc::phE(c, buf.data(), t, AT);
                for (int t = 0; t < AT; ++t) pc::axis_store(c, buf.data(), sc + c_lo, pe, t, AT);
            }
            for (int q = 0; q < pl.d_n; ++q) {
                std::vector<C> buf((size_t)(I.p.n0 * I.p.ld + pc::tw_lds_elems(I.p)), C{T(1e30), T(1e30)});
                pc::Ctx<T> c = pc::plane_ctx_write<T>(I, adj, q, iv, sv, wts.data(), specc, twc, in_pitch);
                {
                    pc::Ctx<T> c0 = c;
                    for (int t = 0; t < NT; ++t) {
                        c0 = c;
                        pc::twiddles_to_lds(c0, buf.data() + (int64_t)I.p.n0 * I.p.ld, t, NT);
                    }
                    c = c0;
                }
                for (int t = 0; t < NT; ++t) pc::plane_load(c, buf.data(), sc + (int64_t)(pl.d_off + q) * pe, t, NT);
                for (int t = 0; t < NT; ++t) pc::phD_inv(c, buf.data(), t, NT);
                for (int t = 0; t < NT; ++t) pc::phE(c, buf.data(), t, NT);
                for (int t = 0; t < NT; ++t) pc::phF(c, buf.data(), t, NT);
                for (int t = 0; t < NT; ++t) pc::phG(c, buf.data(), t, NT);
                for (int t = 0; t < NT; ++t) pc::phH(c, buf.data(), t, NT);
            }
        }
    }
    std::vector<T> out((size_t)(B * n_out), T(0));
    for (int64_t b = 0; b < B; ++b)
        for (const pc::Tile& t : tiles)
            for (int col = 0; col < pc::kReduceCols; ++col)
                pc::reduce_tile<T>(t, col, cboxes.data(), &slots[(size_t)(b * per)], &out[(size_t)(b * n_out)],
                                   out_cols);
    for (int64_t b = 0; b < B; ++b) std::memcpy(OUT + b * ldo, &out[(size_t)(b * n_out)], sizeof(T) * (size_t)n_out);
}

template <class T>
void emu_apply_3d(const pc::Plan& P, bool adj, int64_t B, const T* U, int64_t ldu, T* OUT, int64_t ldo) {
    emu_3d<T>(P, P.items3, adj ? P.slot_adj : P.slot_fwd, adj ? P.tiles_adj : P.tiles_fwd,
              adj ? P.cboxes_adj : P.cboxes_fwd, P.N, P.cols, P.prow, P.N, P.cols, adj, B, U, ldu, OUT, ldo);
}

}  // namespace

struct pc_emu {
    pc::Plan plan;
};

extern "C" {

int pc_emu_create(int d, const int64_t* shape, int64_t n_leaves, const int64_t* leaf_lo, const int64_t* leaf_hi,
                  int64_t r, const int64_t* points, const int64_t* radius, const double* phi, const int64_t* phi_off,
                  int dtype, uint32_t flags, pc_emu** out) {
    *out = nullptr;
    pc_emu* e = new pc_emu();
    pc::CreateArgs a{d, shape, n_leaves, leaf_lo, leaf_hi, r, points, radius, phi, phi_off, dtype, flags};
    std::string err;
    pc_status st = pc::build_plan(a, e->plan, err);
    if (st != PC_OK) {
        g_emu_err = err;
        delete e;
        return (int)st;
    }
    *out = e;
    return 0;
}

// As pc_emu_create, keeping only the terms of the selected points.
int pc_emu_create_patches(int d, const int64_t* shape, int64_t n_leaves, const int64_t* leaf_lo,
                          const int64_t* leaf_hi, int64_t r, const int64_t* points, const int64_t* radius,
                          const double* phi, const int64_t* phi_off, int dtype, uint32_t flags, int64_t n_sel,
                          const int64_t* sel, pc_emu** out) {
    *out = nullptr;
    pc_emu* e = new pc_emu();
    pc::CreateArgs a{d, shape, n_leaves, leaf_lo, leaf_hi, r, points, radius, phi, phi_off, dtype, flags,
                     n_sel, sel};
    std::string err;
    pc_status st = pc::build_plan(a, e->plan, err);
    if (st != PC_OK) {
        g_emu_err = err;
        delete e;
        return (int)st;
    }
    *out = e;
    return 0;
}

int pc_emu_apply(pc_emu* e, int adj, int64_t B, const void* U, int64_t ldu, void* OUT, int64_t ldo) {
    if (e->plan.d == 3) {
        if (e->plan.dtype == PC_F64)
            emu_apply_3d<double>(e->plan, adj != 0, B, static_cast<const double*>(U), ldu, static_cast<double*>(OUT),
                                 ldo);
        else
            emu_apply_3d<float>(e->plan, adj != 0, B, static_cast<const float*>(U), ldu, static_cast<float*>(OUT),
                                ldo);
        return 0;
    }
    if (e->plan.dtype == PC_F64)
        emu_apply<double>(e->plan, adj != 0, B, static_cast<const double*>(U), ldu, static_cast<double*>(OUT), ldo);
    else
        emu_apply<float>(e->plan, adj != 0, B, static_cast<const float*>(U), ldu, static_cast<float*>(OUT), ldo);
    return 0;
}

// The colour-launch path (d <= 2): items in the canonical order add their
// written boxes into zeroed outputs.  Returns -1 for d = 3.
int pc_emu_apply_direct(pc_emu* e, int adj, int64_t B, const void* U, int64_t ldu, void* OUT, int64_t ldo) {
    if (e->plan.d == 3) return -1;
    if (e->plan.dtype == PC_F64)
        emu_apply<double>(e->plan, adj != 0, B, static_cast<const double*>(U), ldu, static_cast<double*>(OUT), ldo,
                          true);
    else
        emu_apply<float>(e->plan, adj != 0, B, static_cast<const float*>(U), ldu, static_cast<float*>(OUT), ldo,
                         true);
    return 0;
}

// The canonical summation order of one direction (d <= 2): for each
// position, the item index, its colour and its written box in the 2-D view
// (row, column origin and extents), into out[6 * n_items]; returns the
// number of colours (0 for d = 3).
int64_t pc_emu_order(pc_emu* e, int adj, int32_t* out) {
    const pc::Plan& P = e->plan;
    const std::vector<int32_t>& ord = adj ? P.order_adj : P.order_fwd;
    const std::vector<int32_t>& cbeg = adj ? P.cbeg_adj : P.cbeg_fwd;
    if (cbeg.empty()) return 0;
    for (size_t c = 0; c + 1 < cbeg.size(); ++c)
        for (int32_t j = cbeg[c]; j < cbeg[c + 1]; ++j) {
            const pc::Item& it = P.items[(size_t)ord[(size_t)j]];
            const int32_t v[6] = {ord[(size_t)j], (int32_t)c,
                                  adj ? it.g0 + it.in_off0 : it.g0 + it.out_off0,
                                  adj ? it.g1 + it.in_off1 : it.g1 + it.out_off1,
                                  adj ? it.in_n0 : it.out_n0, adj ? it.in_n1 : it.out_n1};
            std::memcpy(out + 6 * (size_t)j, v, sizeof(v));
        }
    return (int64_t)cbeg.size() - 1;
}

int pc_emu_stats(pc_emu* e, int64_t* out8) {
    const pc::Plan& P = e->plan;
    out8[0] = (int64_t)(P.d == 3 ? P.items3.size() : P.items.size());
    out8[1] = P.sum_fft_points;
    out8[2] = P.slot_fwd;
    out8[3] = P.slot_adj;
    out8[4] = P.max_lds;
    out8[5] = (int64_t)P.tiles_fwd.size();
    out8[6] = (int64_t)P.contrib_fwd.size();
    out8[7] = P.kernel_elems;
    return 0;
}

// Block apply (same per-call plan and phases as the library): OUT_T over T
// from U_S over S, host arrays.
int pc_emu_apply_block(pc_emu* e, int adj, const int64_t* tlo, const int64_t* thi, const int64_t* slo,
                       const int64_t* shi, int64_t B, const double* U, int64_t ldu, double* OUT, int64_t ldo) {
    const pc::Plan& P = e->plan;
    if (P.dtype != PC_F64) return -1;
    pc::BlockPlan bp;
    std::string err;
    pc_status st = pc::build_block(P, adj != 0, tlo, thi, slo, shi, bp, err);
    if (st != PC_OK) {
        g_emu_err = err;
        return (int)st;
    }
    using C = pc::cx<double>;
    const C* spec = reinterpret_cast<const C*>(P.spec.data());
    const C* tw = reinterpret_cast<const C*>(P.tw.data());
    const int64_t nS = (int64_t)bp.s_planes * bp.s_rows * bp.s_cols, nT = (int64_t)bp.t_rows * bp.t_cols;
    if (P.d == 3) {
        emu_3d<double>(P, bp.items3, bp.per, bp.tiles, bp.cboxes, nS, bp.s_cols, bp.s_rows, nT, bp.t_cols, adj != 0,
                       B, U, ldu, OUT, ldo);
        return 0;
    }
    for (int64_t b = 0; b < B; ++b) {
        std::vector<double> in(U + b * ldu, U + b * ldu + nS);
        std::vector<double> slots((size_t)std::max<int64_t>(bp.per, 1), 0.0);
        for (const pc::Item& it : bp.items) {
            std::vector<C> buf((size_t)(it.n0 * it.ld + pc::tw_lds_elems(it)), C{1e30, 1e30});
            pc::Ctx<double> c = pc::make_ctx<double>(it, adj != 0, in.data(), slots.data(), P.wts.data(), spec, tw,
                                                     bp.s_cols);
            const int nth = P.conv_threads;
            {
                pc::Ctx<double> c0 = c;
                for (int t = 0; t < nth; ++t) {
                    c0 = c;
                    pc::twiddles_to_lds(c0, buf.data() + (int64_t)it.n0 * it.ld, t, nth);
                }
                c = c0;
            }
            for (int t = 0; t < nth; ++t) pc::phA0(c, buf.data(), t, nth);
            for (int t = 0; t < nth; ++t) pc::phA(c, buf.data(), t, nth);
            for (int t = 0; t < nth; ++t) pc::phB(c, buf.data(), t, nth);
            for (int t = 0; t < nth; ++t) pc::phC(c, buf.data(), t, nth);
            for (int t = 0; t < nth; ++t) pc::phD(c, buf.data(), t, nth);
            for (int t = 0; t < nth; ++t) pc::phE(c, buf.data(), t, nth);
            for (int t = 0; t < nth; ++t) pc::phF(c, buf.data(), t, nth);
            for (int t = 0; t < nth; ++t) pc::phG(c, buf.data(), t, nth);
            for (int t = 0; t < nth; ++t) pc::phH(c, buf.data(), t, nth);
        }
        std::vector<double> out((size_t)nT, 0.0);
        for (const pc::Tile& t : bp.tiles)
            for (int col = 0; col < pc::kReduceCols; ++col)
                pc::reduce_tile<double>(t, col, bp.cboxes.data(), slots.data(), out.data(), bp.t_cols);
        std::memcpy(OUT + b * ldo, out.data(), sizeof(double) * (size_t)nT);
    }
    return 0;
}

// Matrix entries on the host with the same entry function as the kernel
// (FP64 tables): out[i] = A~[ys[i], xs[i]], host int64 [n][d] coordinates.
int pc_emu_entries(pc_emu* e, int64_t n, const int64_t* ys, const int64_t* xs, double* out) {
    const pc::Plan& P = e->plan;
    std::vector<int32_t> leaf_of((size_t)P.N, -1);
    for (int64_t c = 0; c < P.L; ++c) {
        const int32_t* b = &P.leaf_box[(size_t)c * 6];
        for (int32_t z = 0; z < b[3]; ++z)
            for (int32_t y = 0; y < b[4]; ++y)
                for (int32_t x = 0; x < b[5]; ++x) {
                    int32_t& v = leaf_of[(size_t)(((int64_t)(b[0] + z) * P.prow + b[1] + y) * P.cols + b[2] + x)];
                    if (v < 0) v = (int32_t)c;
                }
    }
    pc::EntryTables E{P.d, P.planes, P.prow, P.cols, leaf_of.data(), P.leaf_pts_off.data(), P.leaf_pts.data(),
                      P.pt_wbase.data(), P.pt_ubox.data(), P.pt_eoff.data(), P.pt_ebox.data()};
    for (int64_t i = 0; i < n; ++i)
        out[i] = pc::entry_value<double>(E, P.wts.data(), P.phiE.data(), ys + i * P.d, xs + i * P.d);
    return 0;
}

// Per-item geometry (d <= 2): n0, m, ld, in_n0, in_n1, out_n0, out_n1, patch
// for each item, into out[8 * n_items]; returns the item count.
int64_t pc_emu_items(pc_emu* e, int32_t* out) {
    const auto& its = e->plan.items;
    if (out)
        for (size_t i = 0; i < its.size(); ++i) {
            const pc::Item& it = its[i];
            const int32_t v[8] = {it.n0, it.m, it.ld, it.in_n0, it.in_n1, it.out_n0, it.out_n1, it.patch};
            std::memcpy(out + 8 * i, v, sizeof(v));
        }
    return (int64_t)its.size();
}

void pc_emu_destroy(pc_emu* e) { delete e; }

const char* pc_emu_last_error(void) { return g_emu_err.c_str(); }

}  // extern "C"
