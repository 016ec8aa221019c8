// Host planner of 3-D product-convolution operators (see pc_plan.h).
//
// Weights (Sec. 2.4): on a leaf that carries only its 2^d' corners (d' the
// number of axes along which it has positive width) the harmonic weights are
// the trilinear hats.  On a leaf with hanging nodes they are built
// recursively in dimension: point values, linear interpolation on segments
// cut at the points on them, the 2-D harmonic extension on every facet (a
// broken facet replaced by the facets of the smaller leaves on its other
// side, clipped to it), then the 3-D harmonic extension of the facet values;
// the Dirichlet problems are solved exactly in the sine eigenbasis.
//
// One work item per patch, no pieces: the FFT box nz x n1 x 2m is processed
// plane by plane (2-D FFTs along axes 1, 2 in LDS) with an axis-0 pass over
// the planes' spectra in a global scratch area.
#include "pc_plan.h"
#include "pc_phases3.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <map>
#include <set>

namespace pc {

namespace {

// complex row length m of the real axis-2 transform: m <= 128 and the
// second radix at most 10 (row pass 2 of the kernels)
int next_row_len(int need) {
    for (int m = std::max(need, 1); m <= 128; ++m) {
        int a, b;
        if (fft_factor(m, &a, &b) && b <= 10) return m;
    }
    return -1;
}

struct IBox {
    int64_t lo[3], hi[3];
};

// Interior of the box (extents n, degenerate axes have n = 1) from its
// boundary values: L U = R with L the Kronecker sum of T_{n_i - 2} over the
// live axes, R the boundary neighbours; solved in the sine eigenbasis.
void dirichlet_interior(const int64_t n[3], std::vector<double>& V) {
    int64_t m[3], o[3];
    bool live[3];
    for (int i = 0; i < 3; ++i) {
        live[i] = n[i] > 1;
        m[i] = live[i] ? n[i] - 2 : 1;
        o[i] = live[i] ? 1 : 0;
        if (live[i] && m[i] <= 0) return;
    }
    auto at = [&](int64_t a, int64_t b, int64_t c) -> double& { return V[(size_t)((a * n[1] + b) * n[2] + c)]; };
    const int64_t M = m[0] * m[1] * m[2];
    std::vector<double> R((size_t)M, 0.0), T((size_t)M);
    for (int64_t a = 0; a < m[0]; ++a)
        for (int64_t b = 0; b < m[1]; ++b)
            for (int64_t c = 0; c < m[2]; ++c) {
                double s = 0.0;
                const int64_t A = a + o[0], B = b + o[1], Cc = c + o[2];
                if (live[0]) s += (a == 0 ? at(0, B, Cc) : 0.0) + (a == m[0] - 1 ? at(n[0] - 1, B, Cc) : 0.0);
                if (live[1]) s += (b == 0 ? at(A, 0, Cc) : 0.0) + (b == m[1] - 1 ? at(A, n[1] - 1, Cc) : 0.0);
                if (live[2]) s += (c == 0 ? at(A, B, 0) : 0.0) + (c == m[2] - 1 ? at(A, B, n[2] - 1) : 0.0);
                R[(size_t)((a * m[1] + b) * m[2] + c)] = s;
            }
    std::unique_ptr<SineBasis> SB[3];
    for (int i = 0; i < 3; ++i)
        if (live[i]) SB[i].reset(new SineBasis((int)m[i]));
    const int64_t stride[3] = {m[1] * m[2], m[2], 1};
    auto transform = [&](std::vector<double>& X) {   // X <- (S (x) S (x) S) X over the live axes
        for (int i = 0; i < 3; ++i) {
            if (!live[i]) continue;
            const SineBasis& B = *SB[i];
            std::fill(T.begin(), T.end(), 0.0);
            for (int64_t idx = 0; idx < M; ++idx) {
                const int64_t ai = (idx / stride[i]) % m[i];
                const int64_t base = idx - ai * stride[i];
                const double x = X[(size_t)idx];
                if (x == 0.0) continue;
                for (int64_t k = 0; k < m[i]; ++k) T[(size_t)(base + k * stride[i])] += B.S[(size_t)(k * m[i] + ai)] * x;
            }
            X.swap(T);
        }
    };
    transform(R);
    for (int64_t a = 0; a < m[0]; ++a)
        for (int64_t b = 0; b < m[1]; ++b)
            for (int64_t c = 0; c < m[2]; ++c) {
                double den = 0.0;
                if (live[0]) den += SB[0]->lam[(size_t)a];
                if (live[1]) den += SB[1]->lam[(size_t)b];
                if (live[2]) den += SB[2]->lam[(size_t)c];
                R[(size_t)((a * m[1] + b) * m[2] + c)] /= den;
            }
    transform(R);
    for (int64_t a = 0; a < m[0]; ++a)
        for (int64_t b = 0; b < m[1]; ++b)
            for (int64_t c = 0; c < m[2]; ++c) at(a + o[0], b + o[1], c + o[2]) = R[(size_t)((a * m[1] + b) * m[2] + c)];
}

// Harmonic extension on the box b of the values pv[i] at the points
// pts[i] lying on it (Sec. 2.4), recursively in dimension; parts(i, side)
// gives the boxes a 3-D facet is made of.  Values row-major over b.
void harmonic_box(const IBox& b, const int64_t* Pt, const std::vector<int64_t>& pts, const std::vector<double>& pv,
                  const std::function<std::vector<IBox>(int, int)>* parts, std::vector<double>& out) {
    int64_t n[3];
    int live = 0, ax = -1;
    for (int i = 0; i < 3; ++i) {
        n[i] = b.hi[i] - b.lo[i] + 1;
        if (n[i] > 1) {
            ++live;
            ax = i;
        }
    }
    out.assign((size_t)(n[0] * n[1] * n[2]), 0.0);
    auto inside = [&](int64_t k, const IBox& x) {
        for (int i = 0; i < 3; ++i)
            if (Pt[3 * k + i] < x.lo[i] || Pt[3 * k + i] > x.hi[i]) return false;
        return true;
    };
    if (live == 0) {
        for (size_t j = 0; j < pts.size(); ++j)
            if (inside(pts[j], b)) out[0] = pv[j];
        return;
    }
    if (live == 1) {   // linear between consecutive points on the segment
        std::vector<std::pair<int64_t, double>> cut;
        for (size_t j = 0; j < pts.size(); ++j)
            if (inside(pts[j], b)) cut.push_back({Pt[3 * pts[j] + ax], pv[j]});
        std::sort(cut.begin(), cut.end());
        for (size_t q = 0; q + 1 < cut.size(); ++q) {
            const int64_t x0 = cut[q].first, x1 = cut[q + 1].first;
            for (int64_t x = x0; x <= x1; ++x) {
                const double t = (double)(x - x0) / (double)(x1 - x0);
                out[(size_t)(x - b.lo[ax])] = cut[q].second * (1.0 - t) + cut[q + 1].second * t;
            }
        }
        return;
    }
    std::vector<double> fv;
    for (int i = 0; i < 3; ++i) {
        if (n[i] <= 1) continue;
        for (int side = 0; side < 2; ++side) {
            std::vector<IBox> fs;
            if (live == 3 && parts) {
                fs = (*parts)(i, side);
            } else {
                IBox f = b;
                f.lo[i] = f.hi[i] = side ? b.hi[i] : b.lo[i];
                fs.push_back(f);
            }
            for (const IBox& f : fs) {
                std::vector<int64_t> fp;
                std::vector<double> fval;
                for (size_t j = 0; j < pts.size(); ++j)
                    if (inside(pts[j], f)) {
                        fp.push_back(pts[j]);
                        fval.push_back(pv[j]);
                    }
                harmonic_box(f, Pt, fp, fval, nullptr, fv);
                const int64_t fn[3] = {f.hi[0] - f.lo[0] + 1, f.hi[1] - f.lo[1] + 1, f.hi[2] - f.lo[2] + 1};
                for (int64_t a = 0; a < fn[0]; ++a)
                    for (int64_t c = 0; c < fn[1]; ++c)
                        for (int64_t e = 0; e < fn[2]; ++e)
                            out[(size_t)(((f.lo[0] - b.lo[0] + a) * n[1] + (f.lo[1] - b.lo[1] + c)) * n[2] +
                                         (f.lo[2] - b.lo[2] + e))] = fv[(size_t)((a * fn[1] + c) * fn[2] + e)];
            }
        }
    }
    dirichlet_interior(n, out);
}

struct Geo3 {
    pc_status st = PC_OK;
    std::string err;
    Item3 it;
    int64_t I_lo[3], m[3], zlo[3], zhi[3];
    double flops = 0.0;
    int64_t kel = 0;
    int lds_plane = 0, lds_axis = 0;
};

}  // namespace

pc_status build_plan_3d(const CreateArgs& a, Plan& p, std::string& err) {
    const int64_t* n = a.shape;
    const int64_t L = a.n_leaves, r = a.r;
    if (n[0] * n[1] > INT32_MAX || n[2] > INT32_MAX) {
        err = "3-D domain too large for the reduction view";
        return PC_ERR_ARG;
    }
    p.rows = (int)(n[0] * n[1]);
    p.cols = (int)n[2];
    p.planes = (int)n[0];
    p.prow = (int)n[1];
    const int64_t* Pt = a.points;
    const int64_t* Rd = a.radius;
    auto lo = [&](int64_t c, int i) { return a.leaf_lo[c * 3 + i]; };
    auto hi = [&](int64_t c, int i) { return a.leaf_hi[c * 3 + i]; };
    // ------------------------------------------------ cells and neighbours
    std::vector<std::vector<int64_t>> leaf_pts(L), cells(r);
    for (int64_t c = 0; c < L; ++c)
        for (int64_t k = 0; k < r; ++k) {
            bool in = true;
            for (int i = 0; i < 3 && in; ++i) in = Pt[k * 3 + i] >= lo(c, i) && Pt[k * 3 + i] <= hi(c, i);
            if (in) {
                leaf_pts[c].push_back(k);
                cells[k].push_back(c);
            }
        }
    std::vector<std::vector<int64_t>> nbrs(r);
    std::vector<int64_t> Ulo(3 * r, INT64_MAX), Uhi(3 * r, INT64_MIN);
    for (int64_t k = 0; k < r; ++k) {
        std::set<int64_t> s;
        for (int64_t c : cells[k]) {
            for (int64_t j : leaf_pts[c]) s.insert(j);
            for (int i = 0; i < 3; ++i) {
                Ulo[3 * k + i] = std::min(Ulo[3 * k + i], lo(c, i));
                Uhi[3 * k + i] = std::max(Uhi[3 * k + i], hi(c, i));
            }
        }
        nbrs[k].assign(s.begin(), s.end());
    }
    p.leaf_pts_off.assign((size_t)L + 1, 0);
    for (int64_t c = 0; c < L; ++c) {
        p.leaf_pts_off[(size_t)c + 1] = p.leaf_pts_off[(size_t)c] + (int32_t)leaf_pts[c].size();
        for (int64_t k : leaf_pts[c]) p.leaf_pts.push_back((int32_t)k);
    }
    // ----------------------------------------- weights: trilinear hats
    std::vector<int64_t> w_base(r + 1, 0);
    for (int64_t k = 0; k < r; ++k) {
        int64_t v = 1;
        for (int i = 0; i < 3; ++i) v *= Uhi[3 * k + i] - Ulo[3 * k + i] + 1;
        w_base[k + 1] = w_base[k] + v;
    }
    p.pt_wbase.assign((size_t)r, -1);
    p.pt_ubox.assign((size_t)r * 6, 0);
    for (int64_t k = 0; k < r; ++k) {
        if (p.sel[(size_t)k]) p.pt_wbase[(size_t)k] = w_base[k];
        for (int i = 0; i < 3; ++i) {
            p.pt_ubox[(size_t)k * 6 + i] = (int32_t)Ulo[3 * k + i];
            p.pt_ubox[(size_t)k * 6 + 3 + i] = (int32_t)(Uhi[3 * k + i] - Ulo[3 * k + i] + 1);
        }
    }
    std::vector<double> W((size_t)w_base[r], 0.0);
    // leaves are independent: weights solved in parallel, scattered in leaf order
    std::vector<std::vector<std::vector<double>>> leaf_vals((size_t)L);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < L; ++c) {
        const std::vector<int64_t>& lp = leaf_pts[c];
        bool any = false;
        for (int64_t k : lp) any = any || p.sel[(size_t)k];
        if (!any) continue;
        int live = 0;
        for (int i = 0; i < 3; ++i) live += hi(c, i) > lo(c, i);
        const int64_t n0 = hi(c, 0) - lo(c, 0) + 1, n1 = hi(c, 1) - lo(c, 1) + 1, n2 = hi(c, 2) - lo(c, 2) + 1;
        std::vector<std::vector<double>>& vals = leaf_vals[(size_t)c];
        vals.assign(lp.size(), std::vector<double>());
        if ((int64_t)lp.size() == (int64_t)(1 << live)) {   // conforming leaf: trilinear hats
            double H[3];
            for (int i = 0; i < 3; ++i) H[i] = (double)(hi(c, i) - lo(c, i));
            for (size_t j = 0; j < lp.size(); ++j) {
                const int64_t k = lp[j];
                std::vector<double>& V = vals[j];
                V.resize((size_t)(n0 * n1 * n2));
                for (int64_t y0 = 0; y0 < n0; ++y0) {
                    const double f0 = H[0] > 0 ? 1.0 - std::fabs((double)(lo(c, 0) + y0 - Pt[k * 3])) / H[0] : 1.0;
                    for (int64_t y1 = 0; y1 < n1; ++y1) {
                        const double f1 =
                            H[1] > 0 ? 1.0 - std::fabs((double)(lo(c, 1) + y1 - Pt[k * 3 + 1])) / H[1] : 1.0;
                        for (int64_t y2 = 0; y2 < n2; ++y2) {
                            const double f2 =
                                H[2] > 0 ? 1.0 - std::fabs((double)(lo(c, 2) + y2 - Pt[k * 3 + 2])) / H[2] : 1.0;
                            V[(size_t)((y0 * n1 + y1) * n2 + y2)] = f0 * f1 * f2;
                        }
                    }
                }
            }
            continue;
        }
        // hanging nodes: the facets as the smaller leaves' facets (Sec. 2.4)
        IBox box;
        for (int i = 0; i < 3; ++i) {
            box.lo[i] = lo(c, i);
            box.hi[i] = hi(c, i);
        }
        std::function<std::vector<IBox>(int, int)> parts = [&](int axis, int side) {
            const int64_t v = side ? hi(c, axis) : lo(c, axis);
            IBox f = box;
            f.lo[axis] = f.hi[axis] = v;
            std::vector<IBox> out;
            for (int64_t e = 0; e < L; ++e) {
                if (e == c || (side ? lo(e, axis) : hi(e, axis)) != v) continue;
                IBox g;
                bool ok = true;
                for (int i = 0; i < 3; ++i) {
                    g.lo[i] = std::max(f.lo[i], lo(e, i));
                    g.hi[i] = std::min(f.hi[i], hi(e, i));
                    if (i != axis && f.hi[i] > f.lo[i] && g.hi[i] <= g.lo[i]) ok = false;
                }
                g.lo[axis] = g.hi[axis] = v;
                if (ok) out.push_back(g);
            }
            if (out.empty()) out.push_back(f);
            return out;
        };
        std::vector<double> pv(lp.size());
        for (size_t j = 0; j < lp.size(); ++j) {
            std::fill(pv.begin(), pv.end(), 0.0);
            pv[j] = 1.0;
            harmonic_box(box, Pt, lp, pv, &parts, vals[j]);
        }
    }
    for (int64_t c = 0; c < L; ++c) {
        const std::vector<std::vector<double>>& vals = leaf_vals[(size_t)c];
        if (vals.empty()) continue;
        const int64_t n1 = hi(c, 1) - lo(c, 1) + 1, n2 = hi(c, 2) - lo(c, 2) + 1;
        const std::vector<int64_t>& lp = leaf_pts[c];
        for (size_t j = 0; j < lp.size(); ++j) {
            const int64_t k = lp[j];
            if (!p.sel[(size_t)k]) continue;
            const int64_t um1 = Uhi[3 * k + 1] - Ulo[3 * k + 1] + 1, um2 = Uhi[3 * k + 2] - Ulo[3 * k + 2] + 1;
            for (int64_t y0 = lo(c, 0); y0 <= hi(c, 0); ++y0)
                for (int64_t y1 = lo(c, 1); y1 <= hi(c, 1); ++y1) {
                    double* row = &W[(size_t)(w_base[k] + ((y0 - Ulo[3 * k]) * um1 + (y1 - Ulo[3 * k + 1])) * um2)];
                    const double* src = &vals[j][(size_t)(((y0 - lo(c, 0)) * n1 + (y1 - lo(c, 1))) * n2)];
                    for (int64_t y2 = lo(c, 2); y2 <= hi(c, 2); ++y2) row[y2 - Ulo[3 * k + 2]] = src[y2 - lo(c, 2)];
                }
        }
        std::vector<std::vector<double>>().swap(leaf_vals[(size_t)c]);
    }
    p.wts = std::move(W);
    // ------------------------------------------- geometry of every patch
    const bool extend = !(a.flags & PC_NO_EXTEND);
    const size_t csz = (a.dtype == PC_F64) ? 16 : 8;
    const int acols = axis_cols(a.dtype);
    const int ld_axis = axis_ld(acols);
    std::vector<Geo3> geo((size_t)r);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < r; ++k) {
        Geo3& g = geo[(size_t)k];
        if (!p.sel[(size_t)k]) continue;
        int64_t K[3], Rm[3], olo[3], ohi[3];
        for (int i = 0; i < 3; ++i) {
            g.I_lo[i] = Ulo[3 * k + i];
            g.m[i] = Uhi[3 * k + i] - Ulo[3 * k + i] + 1;
            Rm[i] = Rd[k * 3 + i];
        }
        if (extend) {
            for (int64_t j : nbrs[k])
                for (int i = 0; i < 3; ++i) Rm[i] = std::max(Rm[i], Rd[j * 3 + i]);
            // phi_k^E differs from phi_k only at offsets z with p_k + z
            // outside Omega; if the neighbour-radius box around p_k stays in
            // Omega, phi_k^E is zero outside phi_k's own box, which is then
            // the kernel box (shorter FFTs, smaller output boxes, same sum)
            bool inside = true;
            for (int i = 0; i < 3; ++i)
                inside = inside && Pt[k * 3 + i] - Rm[i] >= 0 && Pt[k * 3 + i] + Rm[i] <= n[i] - 1;
            if (inside)
                for (int i = 0; i < 3; ++i) Rm[i] = Rd[k * 3 + i];
        }
        g.kel = 1;
        for (int i = 0; i < 3; ++i) {
            g.zlo[i] = std::max(-Rm[i], -(Uhi[3 * k + i]));
            g.zhi[i] = std::min(Rm[i], n[i] - 1 - g.I_lo[i]);
            K[i] = g.zhi[i] - g.zlo[i] + 1;
            olo[i] = std::max(g.I_lo[i] + g.zlo[i], (int64_t)0);
            ohi[i] = std::min(Uhi[3 * k + i] + g.zhi[i], n[i] - 1);
            g.kel *= 2 * Rd[k * 3 + i] + 1;
        }
        const int nz = next_fft_size((int)std::min<int64_t>(g.m[0] + K[0] - 1, 1 << 20));
        const int n1 = next_fft_size((int)std::min<int64_t>(g.m[1] + K[1] - 1, 1 << 20));
        const int M = next_row_len((int)std::min<int64_t>((g.m[2] + K[2]) / 2, 1 << 20));
        if (nz < 0 || n1 < 0 || M < 0) {
            g.st = PC_ERR_UNSUPPORTED;
            g.err = "patch " + std::to_string(k) + " needs an FFT longer than the kernels support";
            continue;
        }
        int ld = M + 1;
        if (ld % 2 == 0) ++ld;
        g.lds_plane = (int)(((size_t)n1 * ld + n1 + 3 * (size_t)M) * csz);   // plane box + twiddles
        g.lds_axis = (int)(((size_t)nz * ld_axis + nz) * csz);
        if (g.lds_plane > kLdsBytes || g.lds_axis > kLdsBytes) {
            g.st = PC_ERR_UNSUPPORTED;
            g.err = "patch " + std::to_string(k) + " does not fit the LDS-resident plane FFT";
            continue;
        }
        Item3& it = g.it;
        std::memset(&it, 0, sizeof(it));
        Item& q = it.p;
        q.n0 = n1;
        fft_factor(n1, &q.a0, &q.b0);
        q.m = M;
        fft_factor(M, &q.am, &q.bm);
        q.ld = ld;
        q.g0 = (int32_t)olo[1];
        q.g1 = (int32_t)olo[2];
        q.in_off0 = (int32_t)(g.I_lo[1] - olo[1]);
        q.in_off1 = (int32_t)(g.I_lo[2] - olo[2]);
        q.in_n0 = (int32_t)g.m[1];
        q.in_n1 = (int32_t)g.m[2];
        q.out_n0 = (int32_t)(ohi[1] - olo[1] + 1);
        q.out_n1 = (int32_t)(ohi[2] - olo[2] + 1);
        q.patch = (int32_t)k;
        q.w_ld = (int32_t)g.m[2];
        q.w_off = w_base[k];
        it.nz = nz;
        fft_factor(nz, &it.az, &it.bz);
        it.gz = (int32_t)olo[0];
        it.in_offz = (int32_t)(g.I_lo[0] - olo[0]);
        it.in_nz = (int32_t)g.m[0];
        it.out_nz = (int32_t)(ohi[0] - olo[0] + 1);
        it.w_plane = (int32_t)(g.m[1] * g.m[2]);
        if (it.in_offz < 0 || it.in_offz + it.in_nz > nz || it.out_nz > nz || q.in_off0 < 0 ||
            q.in_off0 + q.in_n0 > n1 || q.out_n0 > n1 || q.in_off1 < 0 || q.in_off1 + q.in_n1 > 2 * M ||
            q.out_n1 > 2 * M) {
            g.st = PC_ERR_ARG;
            g.err = "internal planning error (FFT box too small) at patch " + std::to_string(k);
            continue;
        }
        int64_t nn = 1, I = 1, O = 1;
        for (int i = 0; i < 3; ++i) {
            nn *= smallest_7smooth(g.m[i] + K[i] - 1);
            I *= g.m[i];
            O *= ohi[i] - olo[i] + 1;
        }
        g.flops = 5.0 * nn * std::log2((double)nn) + 3.0 * nn + (double)I + (double)O;
    }
    // ----------------------------------- offsets (patch order) and tables
    TwiddleTables twt{&p.tw, {}, {}};
    int64_t spec_total = 0;
    for (int64_t k = 0; k < r; ++k) {
        Geo3& g = geo[(size_t)k];
        if (g.st != PC_OK) {
            err = g.err;
            return g.st;
        }
        if (!p.sel[(size_t)k]) continue;
        Item3& it = g.it;
        Item& q = it.p;
        q.tw0 = twt.pass(q.a0, q.b0);
        q.twm = twt.pass(q.am, q.bm);
        q.tw2m = twt.pair(q.am, q.bm);
        it.twz = twt.pass(it.az, it.bz);
        const int64_t plane = (int64_t)q.n0 * (q.m + 1);
        q.spec_off = spec_total;
        spec_total += (int64_t)it.nz * plane;
        it.scratch_off = p.scratch_per_vec;
        p.scratch_per_vec += (int64_t)it.nz * plane;
        q.slot_fwd = p.slot_fwd;
        q.slot_adj = p.slot_adj;
        p.slot_fwd += (int64_t)it.out_nz * q.out_n0 * q.out_n1;
        p.slot_adj += (int64_t)it.in_nz * q.in_n0 * q.in_n1;
        p.sum_fft_points += (int64_t)it.nz * q.n0 * 2 * q.m;
        p.alg_flops += g.flops;
        p.kernel_elems += g.kel;
        p.max_lds = std::max(p.max_lds, g.lds_plane);
        p.max_lds_axis = std::max(p.max_lds_axis, g.lds_axis);
        p.items3.push_back(it);
    }
    // extended kernels kept for matrix entries
    p.pt_eoff.assign((size_t)r, -1);
    p.pt_ebox.assign((size_t)r * 6, 0);
    int64_t e_total = 0;
    for (const Item3& it : p.items3) {
        const int64_t k = it.p.patch;
        const Geo3& g = geo[(size_t)k];
        int64_t vol = 1;
        for (int i = 0; i < 3; ++i) {
            p.pt_ebox[(size_t)k * 6 + i] = (int32_t)g.zlo[i];
            p.pt_ebox[(size_t)k * 6 + 3 + i] = (int32_t)(g.zhi[i] - g.zlo[i] + 1);
            vol *= g.zhi[i] - g.zlo[i] + 1;
        }
        p.pt_eoff[(size_t)k] = e_total;
        e_total += vol;
    }
    p.phiE.assign((size_t)e_total, 0.0);
    // ------------------------------------------- FP64 spectra, in place
    p.spec.assign((size_t)(2 * spec_total), 0.0);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t ii = 0; ii < (int64_t)p.items3.size(); ++ii) {
        const Item3& it = p.items3[(size_t)ii];
        const int64_t k = it.p.patch;
        const Geo3& g = geo[(size_t)k];
        const int nz = it.nz, n1 = it.p.n0, M = it.p.m, n2 = 2 * M;
        // extended kernel phi_k^E (Sec. 2.5) on [zlo, zhi], placed circularly
        auto defined = [&](int64_t j, const int64_t* z) {
            for (int i = 0; i < 3; ++i) {
                const int64_t y = Pt[j * 3 + i] + z[i];
                if (y < 0 || y >= n[i]) return false;
            }
            return true;
        };
        auto val = [&](int64_t j, const int64_t* z) -> double {
            const int64_t R0 = Rd[j * 3], R1 = Rd[j * 3 + 1], R2 = Rd[j * 3 + 2];
            if (z[0] < -R0 || z[0] > R0 || z[1] < -R1 || z[1] > R1 || z[2] < -R2 || z[2] > R2) return 0.0;
            return a.phi[a.phi_off[j] + ((z[0] + R0) * (2 * R1 + 1) + (z[1] + R1)) * (2 * R2 + 1) + (z[2] + R2)];
        };
        std::vector<cd> G((size_t)nz * n1 * n2, cd(0.0));
        std::vector<char> live((size_t)nz * n1, 0);
        int64_t z[3];
        for (z[0] = g.zlo[0]; z[0] <= g.zhi[0]; ++z[0])
            for (z[1] = g.zlo[1]; z[1] <= g.zhi[1]; ++z[1])
                for (z[2] = g.zlo[2]; z[2] <= g.zhi[2]; ++z[2]) {
                    double v = 0.0;
                    if (defined(k, z)) {
                        v = val(k, z);
                    } else if (extend) {
                        int cnt = 0;
                        double s = 0.0;
                        for (int64_t j : nbrs[k]) {
                            if (j == k || !defined(j, z)) continue;
                            ++cnt;
                            s += val(j, z);
                        }
                        if (cnt) v = s / (double)cnt;
                    }
                    const int64_t i0 = ((z[0] % nz) + nz) % nz, i1 = ((z[1] % n1) + n1) % n1,
                                  i2 = ((z[2] % n2) + n2) % n2;
                    G[(size_t)((i0 * n1 + i1) * n2 + i2)] += v;
                    p.phiE[(size_t)(p.pt_eoff[(size_t)k] +
                                    ((z[0] - g.zlo[0]) * (g.zhi[1] - g.zlo[1] + 1) + (z[1] - g.zlo[1])) *
                                        (g.zhi[2] - g.zlo[2] + 1) +
                                    (z[2] - g.zlo[2]))] = v;
                    live[(size_t)(i0 * n1 + i1)] = 1;
                }
        // axis 2 (real length 2M, keep 0..M), axis 1, axis 0
        const int NC = M + 1;
        std::vector<cd> H((size_t)nz * n1 * NC, cd(0.0)), buf_in(std::max({n1, nz, n2})),
            buf_out(std::max({n1, nz, n2}));
        const Dft64& F2 = dft64(n2);
        const Dft64& F1 = dft64(n1);
        const Dft64& F0 = dft64(nz);
        for (int i0 = 0; i0 < nz; ++i0)
            for (int i1 = 0; i1 < n1; ++i1) {
                if (!live[(size_t)(i0 * n1 + i1)]) continue;
                F2.run(&G[(size_t)((i0 * n1 + i1) * n2)], 1, buf_out.data());
                for (int kk = 0; kk < NC; ++kk) H[(size_t)((i0 * n1 + i1) * NC + kk)] = buf_out[kk];
            }
        std::vector<cd>().swap(G);
        for (int i0 = 0; i0 < nz; ++i0)
            for (int kk = 0; kk < NC; ++kk) {
                for (int i1 = 0; i1 < n1; ++i1) buf_in[i1] = H[(size_t)((i0 * n1 + i1) * NC + kk)];
                F1.run(buf_in.data(), 1, buf_out.data());
                for (int k1 = 0; k1 < n1; ++k1) H[(size_t)((i0 * n1 + k1) * NC + kk)] = buf_out[k1];
            }
        // normalisation of the inverse transforms, and 1/4 for the factors
        // 1/2 that the real-row post- and pre-processing leave out
        const double sc = 0.25 / ((double)nz * (double)n1 * (double)M);
        double* out = &p.spec[(size_t)(2 * it.p.spec_off)];
        for (int k1 = 0; k1 < n1; ++k1)
            for (int kk = 0; kk < NC; ++kk) {
                for (int i0 = 0; i0 < nz; ++i0) buf_in[i0] = H[(size_t)((i0 * n1 + k1) * NC + kk)];
                F0.run(buf_in.data(), 1, buf_out.data());
                const int s1 = perm_slot(k1, it.p.a0, it.p.b0);
                const int s2 = (kk < M) ? perm_slot(kk, it.p.am, it.p.bm) : M;
                for (int kz = 0; kz < nz; ++kz) {
                    const int s0 = perm_slot(kz, it.az, it.bz);
                    const size_t e = (size_t)(((int64_t)s0 * n1 + s1) * NC + s2);
                    out[2 * e] = buf_out[kz].real() * sc;
                    out[2 * e + 1] = buf_out[kz].imag() * sc;
                }
            }
    }
    // ------------------------------------------------ reduction view boxes
    const int64_t N1 = n[1];
    std::vector<Box> bf, ba;
    for (const Item3& it : p.items3) {
        const Item& q = it.p;
        const int64_t pf = (int64_t)q.out_n0 * q.out_n1, pa = (int64_t)q.in_n0 * q.in_n1;
        for (int z = 0; z < it.out_nz; ++z)
            bf.push_back(Box{(int32_t)((it.gz + z) * N1 + q.g0), q.g1, q.out_n0, q.out_n1, q.slot_fwd + z * pf});
        for (int z = 0; z < it.in_nz; ++z)
            ba.push_back(Box{(int32_t)((it.gz + it.in_offz + z) * N1 + q.g0 + q.in_off0), q.g1 + q.in_off1, q.in_n0,
                             q.in_n1, q.slot_adj + z * pa});
    }
    if (!finish_tiles(p, bf, ba, err)) return PC_ERR_UNSUPPORTED;
    p.leaf_box.resize(6 * L);
    for (int64_t c = 0; c < L; ++c)
        for (int i = 0; i < 3; ++i) {
            p.leaf_box[6 * c + i] = (int32_t)lo(c, i);
            p.leaf_box[6 * c + 3 + i] = (int32_t)(hi(c, i) - lo(c, i) + 1);
        }
    return PC_OK;
}

}  // namespace pc

namespace pc {

pc_status build_block3(const Plan& P, bool adjoint, const int64_t* tlo, const int64_t* thi, const int64_t* slo,
                       const int64_t* shi, BlockPlan& B, std::string& err) {
    for (int i = 0; i < 3; ++i)
        if (tlo[i] < 0 || thi[i] >= P.shape[i] || tlo[i] > thi[i] || slo[i] < 0 || shi[i] >= P.shape[i] ||
            slo[i] > shi[i]) {
            err = "block boxes must be non-empty and inside Omega";
            return PC_ERR_ARG;
        }
    int64_t Tn[3], Sn[3];
    for (int i = 0; i < 3; ++i) {
        Tn[i] = thi[i] - tlo[i] + 1;
        Sn[i] = shi[i] - slo[i] + 1;
    }
    if (Tn[0] * Tn[1] > INT32_MAX || Sn[1] * Sn[2] > INT32_MAX) {
        err = "block boxes too large";
        return PC_ERR_ARG;
    }
    B = BlockPlan();
    B.t_rows = (int)(Tn[0] * Tn[1]);
    B.t_cols = (int)Tn[2];
    B.t_prow = (int)Tn[1];
    B.s_planes = (int)Sn[0];
    B.s_rows = (int)Sn[1];
    B.s_cols = (int)Sn[2];
    auto clip = [](int64_t alo, int64_t an, int64_t blo, int64_t bn, int64_t& lo, int64_t& n) {
        lo = std::max(alo, blo);
        n = std::min(alo + an, blo + bn) - lo;
        return n > 0;
    };
    std::vector<Box> boxes;
    int64_t scratch = 0;
    for (const Item3& I : P.items3) {
        const Item& q = I.p;
        // input box and output box in Omega coordinates (axis 0, 1, 2)
        const int64_t Ilo[3] = {I.gz + I.in_offz, q.g0 + q.in_off0, q.g1 + q.in_off1};
        const int64_t In[3] = {I.in_nz, q.in_n0, q.in_n1};
        const int64_t Olo[3] = {I.gz, q.g0, q.g1};
        const int64_t On[3] = {I.out_nz, q.out_n0, q.out_n1};
        const int64_t* glo = adjoint ? Olo : Ilo;
        const int64_t* gn = adjoint ? On : In;
        const int64_t* wlo = adjoint ? Ilo : Olo;
        const int64_t* wn = adjoint ? In : On;
        int64_t Gl[3], Gn[3], Wl[3], Wn[3];
        bool ok = true;
        for (int i = 0; i < 3 && ok; ++i)
            ok = clip(glo[i], gn[i], slo[i], Sn[i], Gl[i], Gn[i]) && clip(wlo[i], wn[i], tlo[i], Tn[i], Wl[i], Wn[i]);
        if (!ok) continue;
        Item3 c = I;
        Item& cp = c.p;
        const int64_t* Al = adjoint ? Wl : Gl;   // the clipped input (weighted) box
        const int64_t* An = adjoint ? Wn : Gn;
        const int64_t* Bl = adjoint ? Gl : Wl;   // the clipped output box
        const int64_t* Bn = adjoint ? Gn : Wn;
        c.in_offz = (int32_t)(Al[0] - I.gz);
        c.in_nz = (int32_t)An[0];
        cp.in_off0 = (int32_t)(Al[1] - q.g0);
        cp.in_n0 = (int32_t)An[1];
        cp.in_off1 = (int32_t)(Al[2] - q.g1);
        cp.in_n1 = (int32_t)An[2];
        cp.w_off = q.w_off + (Al[0] - Ilo[0]) * I.w_plane + (Al[1] - Ilo[1]) * q.w_ld + (Al[2] - Ilo[2]);
        c.out_offz = (int32_t)(Bl[0] - I.gz);
        c.out_nz = (int32_t)Bn[0];
        cp.out_off0 = (int32_t)(Bl[1] - q.g0);
        cp.out_n0 = (int32_t)Bn[1];
        cp.out_off1 = (int32_t)(Bl[2] - q.g1);
        cp.out_n1 = (int32_t)Bn[2];
        c.gz = (int32_t)(I.gz - slo[0]);        // gather in S-local coordinates
        cp.g0 = (int32_t)(q.g0 - slo[1]);
        cp.g1 = (int32_t)(q.g1 - slo[2]);
        cp.slot_fwd = cp.slot_adj = B.per;
        c.scratch_off = scratch;
        scratch += (int64_t)I.nz * q.n0 * (q.m + 1);
        const int64_t pa = Wn[1] * Wn[2];
        for (int64_t z = 0; z < Wn[0]; ++z)
            boxes.push_back(Box{(int32_t)((Wl[0] - tlo[0] + z) * Tn[1] + (Wl[1] - tlo[1])), (int32_t)(Wl[2] - tlo[2]),
                                (int32_t)Wn[1], (int32_t)Wn[2], B.per + z * pa});
        B.per += Wn[0] * pa;
        B.items3.push_back(c);
    }
    std::vector<int32_t> contrib;
    if (!build_tiles(boxes, B.t_rows, B.t_cols, B.tiles, contrib, err)) return PC_ERR_UNSUPPORTED;
    B.cboxes.resize(contrib.size());
    for (size_t i = 0; i < contrib.size(); ++i) B.cboxes[i] = boxes[(size_t)contrib[i]];
    return PC_OK;
}

}  // namespace pc
