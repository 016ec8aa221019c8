// Host planner of the product-convolution operator (see pc_plan.h).
#include "pc_plan.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <memory>
#include <set>
#include <tuple>

namespace pc {

namespace {


// ------------------------------------------------------------------ FFT sizes
const int kRadices[] = {1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 14, 15, 16};

}  // namespace

bool fft_factor(int n, int* a, int* b) {
    int best_a = 0, best_b = 0;
    for (int x : kRadices)
        for (int y : kRadices)
            if (x * y == n) {
                bool better = best_a == 0 || std::max(x, y) < std::max(best_a, best_b) ||
                              (std::max(x, y) == std::max(best_a, best_b) && x > best_a);
                if (better) {
                    best_a = x;
                    best_b = y;
                }
            }
    if (!best_a) return false;
    *a = best_a;
    *b = best_b;
    return true;
}

int next_fft_size(int need) {
    if (need < 1) need = 1;
    for (int n = need; n <= 256; ++n) {
        int a, b;
        if (fft_factor(n, &a, &b)) return n;
    }
    return -1;
}

int perm_slot(int k, int a, int b) { return b * (k % a) + k / a; }

int TwiddleTables::pass(int a, int b) {
    const auto key = std::make_pair(a, b);
    auto f = pass_off.find(key);
    if (f != pass_off.end()) return f->second;
    const int off = (int)(tw->size() / 2);
    pass_off[key] = off;
    const int n = a * b;
    for (int j0 = 0; j0 < b; ++j0)
        for (int k1 = 1; k1 < a; ++k1) {
            const double ang = 2.0 * kPi * (double)((int64_t)j0 * k1 % n) / (double)n;
            tw->push_back(std::cos(ang));
            tw->push_back(-std::sin(ang));
        }
    return off;
}

int TwiddleTables::pair(int am, int bm) {
    const auto key = std::make_pair(am, bm);
    auto f = pair_off.find(key);
    if (f != pair_off.end()) return f->second;
    const int off = (int)(tw->size() / 2);
    pair_off[key] = off;
    const int n2 = 2 * am * bm;
    for (int k1 = 0; k1 <= am / 2; ++k1)
        for (int k0 = 0; k0 < bm; ++k0) {
            const double ang = 2.0 * kPi * (double)(k1 + am * k0) / (double)n2;
            tw->push_back(std::cos(ang));
            tw->push_back(-std::sin(ang));
        }
    return off;
}

int64_t twiddle_elems(int a0, int b0, int am, int bm) {
    return (int64_t)b0 * (a0 - 1) + (int64_t)bm * (am - 1) + (int64_t)(am / 2 + 1) * bm;
}

// Estimated time of one convolution unit (one piece, one vector) on a CU,
// in cycles.  Each phase runs its tasks (t = thread, thread + NT, ...) on
// NT threads; waves go round-robin to the 4 SIMDs, a SIMD issues one wave64
// VALU instruction per 4 cycles, and a barrier ends every phase, so a phase
// costs 4 x (waves on the busiest SIMD) x (instructions per task).  The
// per-task counts are the vector instructions of each phase's task loop in
// the compiled gfx950 kernel, by radix (0 where the radix does not occur):
//   kRow: row pass 1 (phases A and G), kCol1: column pass 1 (C), kColInv:
//   inverse column pass 1 (E), kCol2: column pass 2, spectral product and
//   inverse column pass 2 (D), kPair: row pass 2 with the real-row post- or
//   pre-processing of two frequency groups (B and F).
// Gather (A0) and copy-out (H) take 94 and 43 instructions per batch of 8
// and 4 rows, and the reduction costs about 0.56 CU-cycles per staged
// element (measured on the 1024^2 blur: 7.9e8 elements in 0.72 ms on 256
// CUs).
double simd_rounds(int64_t ntask, int NT) {
    const int64_t full = ntask / NT, rem = ntask % NT;
    double r = (double)full * (NT / 256);
    if (rem) r += std::ceil(std::ceil(rem / 64.0) / 4.0);
    return r;
}

double unit_cycles(int NT, int n0, int a0, int b0, int M, int am, int bm, int64_t in0, int64_t out0, int64_t out1) {
    static const double kRow[17] = {0, 11, 28, 43, 50, 75, 92, 115, 108, 159, 172, 0, 194, 0, 268, 299, 250};
    static const double kCol1[17] = {0, 11, 35, 55, 65, 95, 115, 142, 139, 195, 212, 0, 242, 0, 324, 359, 314};
    static const double kColInv[17] = {0, 11, 29, 48, 56, 86, 104, 130, 126, 182, 196, 0, 224, 0, 304, 338, 292};
    static const double kCol2[17] = {0, 11, 44, 73, 88, 137, 171, 217, 204, 305, 331, 0, 375, 0, 523, 585, 488};
    static const double kPair[11] = {0, 50, 85, 127, 159, 221, 270, 331, 335, 449, 490};
    if (a0 > 16 || b0 > 16 || am > 16 || bm > 10) return 1e30;
    const int64_t NC = M + 1, H = am / 2 + 1;
    double c = simd_rounds(in0 * bm, NT) * kRow[am] + simd_rounds(in0 * H, NT) * kPair[bm] +
               simd_rounds(NC * b0, NT) * kCol1[a0] + simd_rounds(NC * a0, NT) * kCol2[b0] +
               simd_rounds(NC * b0, NT) * kColInv[a0] + simd_rounds(out0 * H, NT) * kPair[bm] +
               simd_rounds(out0 * bm, NT) * kRow[am];
    (void)n0;
    const int64_t rps_in = std::max<int64_t>(1, NT / (2 * M)), rps_out = std::max<int64_t>(1, NT / std::max<int64_t>(out1, 1));
    c += (NT / 256) * (double)((in0 + 8 * rps_in - 1) / (8 * rps_in)) * 94.0;
    c += (NT / 256) * (double)((out0 + 4 * rps_out - 1) / (4 * rps_out)) * 43.0;
    return 4.0 * c + 0.56 * (double)(out0 * out1);
}

int smallest_7smooth(int64_t need) {
    for (int64_t n = std::max<int64_t>(need, 1);; ++n) {
        int64_t m = n;
        for (int p : {2, 3, 5, 7})
            while (m % p == 0) m /= p;
        if (m == 1) return (int)n;
    }
}

// --------------------------------------------------------- FP64 host FFT
// Plan of one length: prime factors and the table w_n^e, e < n.
Dft64::Dft64(int n_) : n(n_), W((size_t)n_) {
    for (int e = 0; e < n; ++e) {
        const double ang = 2.0 * kPi * (double)e / (double)n;
        W[(size_t)e] = cd(std::cos(ang), -std::sin(ang));
    }
    int m = n;
    for (int f = 2; f * f <= m; ++f)
        while (m % f == 0) {
            fac.push_back(f);
            m /= f;
        }
    if (m > 1) fac.push_back(m);
}

// y[k] = sum_j x[j * stride] w_n^(j k) for a sub-length len = n / (product of
// the first 'level' factors): decimation in time over fac[level], then for
// every k < len/p an in-place DFT_p of the p twiddled sub-results.
void Dft64::rec(const cd* x, int64_t stride, int len, int level, cd* y) const {
    if (len == 1) {
        y[0] = x[0];
        return;
    }
    const int p = fac[(size_t)level], m = len / p;
    for (int q = 0; q < p; ++q) rec(x + q * stride, stride * p, m, level + 1, y + q * m);
    const int step = n / len, pstep = n / p;
    cd t[64];
    for (int k = 0; k < m; ++k) {
        for (int q = 0; q < p; ++q) t[q] = y[q * m + k] * W[(size_t)(q * k * step)];
        for (int sft = 0; sft < p; ++sft) {
            cd acc = t[0];
            for (int q = 1; q < p; ++q) acc += t[q] * W[(size_t)(((q * sft) % p) * pstep)];
            y[k + sft * m] = acc;
        }
    }
}

void Dft64::run(const cd* x, int64_t stride, cd* y) const { rec(x, stride, n, 0, y); }

const Dft64& dft64(int n) {
    thread_local std::map<int, std::unique_ptr<Dft64>> cache;
    auto& slot = cache[n];
    if (!slot) slot.reset(new Dft64(n));
    return *slot;
}

namespace {

// -------------------------------------------------------- harmonic weights
// Hat of point 'pos' among sorted cut positions, evaluated on [c0, c1].
void edge_hat(const std::vector<int64_t>& cuts, int64_t pos, int64_t c0, int64_t c1, double* out) {
    // cuts sorted, contain c0 and c1
    for (int64_t x = c0; x <= c1; ++x) {
        auto it = std::upper_bound(cuts.begin(), cuts.end(), x);
        double v;
        if (it == cuts.end()) {
            v = (x == pos) ? 1.0 : 0.0;
        } else {
            int64_t right = *it, left = *(it - 1);
            double fl = (left == pos) ? 1.0 : 0.0, fr = (right == pos) ? 1.0 : 0.0;
            double t = (double)(x - left) / (double)(right - left);
            v = fl * (1.0 - t) + fr * t;
        }
        out[x - c0] = v;
    }
}

// Dirichlet problem for the 5-point graph Laplacian on the interior (p x q)
// of a box, L U = R with L = T_p (x) I + I (x) T_q, solved exactly in the
// sine eigenbasis: U = Sp [(Sp R Sq) / (lambda_a + mu_b)] Sq.  R holds the
// boundary values next to the border only: R = e_0 t' + e_{p-1} b' + l e_0'
// + r e_{q-1}' (t, b: top and bottom rows; l, r: left and right columns), so
// Sp R Sq is a sum of four outer products.  Result in U (p x q, row-major).
}  // namespace

SineBasis::SineBasis(int n_) : n(n_), S((size_t)n_ * n_), lam((size_t)n_) {
    const double sc = std::sqrt(2.0 / (n + 1));
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < n; ++a) S[(size_t)i * n + a] = sc * std::sin(kPi * (i + 1) * (a + 1) / (n + 1));
    for (int a = 0; a < n; ++a) lam[(size_t)a] = 2.0 - 2.0 * std::cos(kPi * (a + 1) / (n + 1));
}

namespace {

void dst_solve_border(const SineBasis& P, const SineBasis& Q, const double* t, const double* b, const double* l,
                      const double* r, std::vector<double>& U) {
    const int p = P.n, q = Q.n;
    std::vector<double> St(q, 0.0), Sb(q, 0.0), Sl(p, 0.0), Sr(p, 0.0);
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j) {
            St[i] += Q.S[(size_t)i * q + j] * t[j];
            Sb[i] += Q.S[(size_t)i * q + j] * b[j];
        }
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) {
            Sl[i] += P.S[(size_t)i * p + j] * l[j];
            Sr[i] += P.S[(size_t)i * p + j] * r[j];
        }
    std::vector<double> H((size_t)p * q);
    for (int a = 0; a < p; ++a) {
        const double pa0 = P.S[(size_t)a * p], pa1 = P.S[(size_t)a * p + p - 1];
        for (int c = 0; c < q; ++c) {
            const double v = pa0 * St[c] + pa1 * Sb[c] + Sl[a] * Q.S[(size_t)c * q] + Sr[a] * Q.S[(size_t)c * q + q - 1];
            H[(size_t)a * q + c] = v / (P.lam[a] + Q.lam[c]);
        }
    }
    // U = Sp H Sq
    std::vector<double> T((size_t)p * q, 0.0);
    for (int i = 0; i < p; ++i)
        for (int k = 0; k < p; ++k) {
            const double s = P.S[(size_t)i * p + k];
            const double* h = &H[(size_t)k * q];
            double* o = &T[(size_t)i * q];
            for (int j = 0; j < q; ++j) o[j] += s * h[j];
        }
    U.assign((size_t)p * q, 0.0);
    for (int i = 0; i < p; ++i)
        for (int k = 0; k < q; ++k) {
            const double s = T[(size_t)i * q + k];
            const double* qs = &Q.S[(size_t)k * q];
            double* o = &U[(size_t)i * q];
            for (int j = 0; j < q; ++j) o[j] += s * qs[j];
        }
}

// Weights of every sample point lying on a 2-D leaf over the leaf box.
// pts: indices into the point list; returns vals[j][(y0-lo0)*(w1) + (y1-lo1)].
void leaf_weights_2d(const int64_t* lo, const int64_t* hi, const std::vector<int64_t>& pts,
                     const int64_t* P, std::vector<std::vector<double>>& vals) {
    const int64_t H0 = hi[0] - lo[0], H1 = hi[1] - lo[1];
    const int64_t w0 = H0 + 1, w1 = H1 + 1;
    vals.assign(pts.size(), std::vector<double>((size_t)(w0 * w1), 0.0));
    if (pts.size() == 4) {   // conforming leaf: bilinear hats
        for (size_t j = 0; j < pts.size(); ++j) {
            const int64_t* p = P + 2 * pts[j];
            for (int64_t y0 = 0; y0 < w0; ++y0) {
                double f0 = 1.0 - std::fabs((double)(lo[0] + y0 - p[0])) / (double)H0;
                for (int64_t y1 = 0; y1 < w1; ++y1) {
                    double f1 = 1.0 - std::fabs((double)(lo[1] + y1 - p[1])) / (double)H1;
                    vals[j][(size_t)(y0 * w1 + y1)] = f0 * f1;
                }
            }
        }
        return;
    }
    // cut positions on each edge
    std::vector<int64_t> top, bot, lef, rig;   // rows lo0 / hi0 (by col), cols lo1 / hi1 (by row)
    for (int64_t k : pts) {
        const int64_t* p = P + 2 * k;
        if (p[0] == lo[0]) top.push_back(p[1]);
        if (p[0] == hi[0]) bot.push_back(p[1]);
        if (p[1] == lo[1]) lef.push_back(p[0]);
        if (p[1] == hi[1]) rig.push_back(p[0]);
    }
    for (auto* v : {&top, &bot, &lef, &rig}) std::sort(v->begin(), v->end());
    const int p_in = (int)H0 - 1, q_in = (int)H1 - 1;
    std::vector<double> e(std::max(w0, w1));
    std::unique_ptr<SineBasis> Bp, Bq;
    if (p_in > 0 && q_in > 0) {
        Bp.reset(new SineBasis(p_in));
        Bq.reset(new SineBasis(q_in));
    }
    std::vector<double> t, b, l, r, U;
    for (size_t j = 0; j < pts.size(); ++j) {
        const int64_t* p = P + 2 * pts[j];
        std::vector<double>& V = vals[j];
        // edges (a point not on an edge contributes a zero hat there)
        edge_hat(top, p[0] == lo[0] ? p[1] : INT64_MIN, lo[1], hi[1], e.data());
        for (int64_t y1 = 0; y1 < w1; ++y1) V[(size_t)y1] = e[y1];
        edge_hat(bot, p[0] == hi[0] ? p[1] : INT64_MIN, lo[1], hi[1], e.data());
        for (int64_t y1 = 0; y1 < w1; ++y1) V[(size_t)(H0 * w1 + y1)] = e[y1];
        edge_hat(lef, p[1] == lo[1] ? p[0] : INT64_MIN, lo[0], hi[0], e.data());
        for (int64_t y0 = 0; y0 < w0; ++y0) V[(size_t)(y0 * w1)] = e[y0];
        edge_hat(rig, p[1] == hi[1] ? p[0] : INT64_MIN, lo[0], hi[0], e.data());
        for (int64_t y0 = 0; y0 < w0; ++y0) V[(size_t)(y0 * w1 + H1)] = e[y0];
        if (p_in <= 0 || q_in <= 0) continue;
        // boundary values next to the interior: rows 0 and H0, columns 0 and H1
        t.assign((size_t)q_in, 0.0);
        b.assign((size_t)q_in, 0.0);
        l.assign((size_t)p_in, 0.0);
        r.assign((size_t)p_in, 0.0);
        for (int jj = 0; jj < q_in; ++jj) {
            t[(size_t)jj] = V[(size_t)(0 * w1 + jj + 1)];
            b[(size_t)jj] = V[(size_t)(H0 * w1 + jj + 1)];
        }
        for (int i = 0; i < p_in; ++i) {
            l[(size_t)i] = V[(size_t)((i + 1) * w1)];
            r[(size_t)i] = V[(size_t)((i + 1) * w1 + H1)];
        }
        dst_solve_border(*Bp, *Bq, t.data(), b.data(), l.data(), r.data(), U);
        for (int i = 0; i < p_in; ++i)
            for (int jj = 0; jj < q_in; ++jj) V[(size_t)((i + 1) * w1 + jj + 1)] = U[(size_t)i * q_in + jj];
    }
}

}  // namespace

// Reduction tiles of the rows x cols view and, for every tile, the staging
// boxes that overlap it in ascending box order (boxes are listed in ascending
// item order, so every tile sums its contributors in ascending patch order).
bool build_tiles(const std::vector<Box>& boxes, int rows, int cols, std::vector<Tile>& tiles,
                 std::vector<int32_t>& contrib, std::string& err) {
    const int ntr = (rows + kReduceRows - 1) / kReduceRows, ntc = (cols + kReduceCols - 1) / kReduceCols;
    std::vector<std::vector<int32_t>> per((size_t)ntr * ntc);
    for (size_t i = 0; i < boxes.size(); ++i) {
        const Box& b = boxes[i];
        if (b.n0 <= 0 || b.n1 <= 0) continue;
        for (int tr = b.lo0 / kReduceRows; tr <= (b.lo0 + b.n0 - 1) / kReduceRows; ++tr)
            for (int tc = b.lo1 / kReduceCols; tc <= (b.lo1 + b.n1 - 1) / kReduceCols; ++tc)
                per[(size_t)tr * ntc + tc].push_back((int32_t)i);
    }
    tiles.clear();
    contrib.clear();
    size_t total = 0;
    for (const auto& v : per) total += v.size();
    if (total > (size_t)INT32_MAX) {
        err = "too many staging contributions for the reduction tables";
        return false;
    }
    contrib.reserve(total);
    for (int tr = 0; tr < ntr; ++tr)
        for (int tc = 0; tc < ntc; ++tc) {
            Tile t;
            t.r0 = tr * kReduceRows;
            t.c0 = tc * kReduceCols;
            t.nr = std::min(kReduceRows, rows - t.r0);
            t.nc = std::min(kReduceCols, cols - t.c0);
            t.beg = (int32_t)contrib.size();
            const auto& v = per[(size_t)tr * ntc + tc];
            contrib.insert(contrib.end(), v.begin(), v.end());
            t.end = (int32_t)contrib.size();
            tiles.push_back(t);
        }
    return true;
}

// Tiles, contributor lists and per-contributor boxes of both directions.
void colour_boxes(const std::vector<Box>& boxes, int rows, int cols, std::vector<int32_t>& order,
                  std::vector<int32_t>& cbeg) {
    constexpr int kCell = 64;   // bucket grid for the overlap queries
    const int gr = (rows + kCell - 1) / kCell, gc = (cols + kCell - 1) / kCell;
    std::vector<std::vector<int32_t>> bucket((size_t)gr * gc);
    const int n = (int)boxes.size();
    std::vector<int32_t> colour((size_t)n, 0), stamp((size_t)n, -1);
    std::vector<char> used;
    int n_colours = 0;
    for (int i = 0; i < n; ++i) {
        const Box& b = boxes[(size_t)i];
        if (b.n0 <= 0 || b.n1 <= 0) {
            colour[(size_t)i] = 0;
            n_colours = std::max(n_colours, 1);
            continue;
        }
        const int r0 = b.lo0 / kCell, r1 = (b.lo0 + b.n0 - 1) / kCell;
        const int c0 = b.lo1 / kCell, c1 = (b.lo1 + b.n1 - 1) / kCell;
        used.assign((size_t)n_colours + 1, 0);
        for (int r = r0; r <= r1; ++r)
            for (int c = c0; c <= c1; ++c)
                for (int32_t j : bucket[(size_t)r * gc + c]) {
                    if (stamp[(size_t)j] == i) continue;
                    stamp[(size_t)j] = i;
                    const Box& o = boxes[(size_t)j];
                    const bool meet = b.lo0 < o.lo0 + o.n0 && o.lo0 < b.lo0 + b.n0 && b.lo1 < o.lo1 + o.n1 &&
                                      o.lo1 < b.lo1 + b.n1;
                    if (meet) used[(size_t)colour[(size_t)j]] = 1;
                }
        int col = 0;
        while (used[(size_t)col]) ++col;
        colour[(size_t)i] = col;
        n_colours = std::max(n_colours, col + 1);
        for (int r = r0; r <= r1; ++r)
            for (int c = c0; c <= c1; ++c) bucket[(size_t)r * gc + c].push_back(i);
    }
    // counting sort by colour, stable in the given order
    cbeg.assign((size_t)n_colours + 1, 0);
    for (int i = 0; i < n; ++i) ++cbeg[(size_t)colour[(size_t)i] + 1];
    for (int c = 0; c < n_colours; ++c) cbeg[(size_t)c + 1] += cbeg[(size_t)c];
    order.assign((size_t)n, 0);
    std::vector<int32_t> fill(cbeg.begin(), cbeg.end() - 1);
    for (int i = 0; i < n; ++i) order[(size_t)fill[(size_t)colour[(size_t)i]]++] = i;
}

bool finish_tiles(Plan& p, std::vector<Box>& bf, std::vector<Box>& ba, std::string& err) {
    if (!build_tiles(bf, p.rows, p.cols, p.tiles_fwd, p.contrib_fwd, err) ||
        !build_tiles(ba, p.rows, p.cols, p.tiles_adj, p.contrib_adj, err))
        return false;
    p.boxes_fwd = std::move(bf);
    p.boxes_adj = std::move(ba);
    p.cboxes_fwd.resize(p.contrib_fwd.size());
    for (size_t i = 0; i < p.contrib_fwd.size(); ++i) p.cboxes_fwd[i] = p.boxes_fwd[(size_t)p.contrib_fwd[i]];
    p.cboxes_adj.resize(p.contrib_adj.size());
    for (size_t i = 0; i < p.contrib_adj.size(); ++i) p.cboxes_adj[i] = p.boxes_adj[(size_t)p.contrib_adj[i]];
    return true;
}

pc_status build_block(const Plan& P, bool adjoint, const int64_t* tlo, const int64_t* thi, const int64_t* slo,
                      const int64_t* shi, BlockPlan& B, std::string& err) {
    if (!tlo || !thi || !slo || !shi) {
        err = "null box pointer";
        return PC_ERR_ARG;
    }
    if (P.d == 3) return build_block3(P, adjoint, tlo, thi, slo, shi, B, err);
    const int d = P.d;
    for (int i = 0; i < d; ++i)
        if (tlo[i] < 0 || thi[i] >= P.shape[i] || tlo[i] > thi[i] || slo[i] < 0 || shi[i] >= P.shape[i] ||
            slo[i] > shi[i]) {
            err = "block boxes must be non-empty and inside Omega";
            return PC_ERR_ARG;
        }
    // boxes in the 2-D view (d = 1: one row)
    const int64_t T0 = d == 1 ? 0 : tlo[0], T1 = tlo[d - 1], Tn0 = d == 1 ? 1 : thi[0] - tlo[0] + 1,
                  Tn1 = thi[d - 1] - tlo[d - 1] + 1;
    const int64_t S0 = d == 1 ? 0 : slo[0], S1 = slo[d - 1], Sn0 = d == 1 ? 1 : shi[0] - slo[0] + 1,
                  Sn1 = shi[d - 1] - slo[d - 1] + 1;
    B = BlockPlan();
    B.t_rows = (int)Tn0;
    B.t_cols = (int)Tn1;
    B.s_rows = (int)Sn0;
    B.s_cols = (int)Sn1;
    auto clip = [](int64_t alo, int64_t an, int64_t blo, int64_t bn, int64_t& lo, int64_t& n) {
        lo = std::max(alo, blo);
        n = std::min(alo + an, blo + bn) - lo;
        return n > 0;
    };
    std::vector<Box> boxes;
    const std::vector<int32_t>& order = adjoint ? P.order_adj : P.order_fwd;
    for (size_t pos = 0; pos < P.items.size(); ++pos) {
        // the canonical summation order, so that every output point sums its
        // contributions as the full apply does
        const Item& it = P.items[order.empty() ? pos : (size_t)order[pos]];
        // input box I and output box O in Omega coordinates
        const int64_t I0 = it.g0 + it.in_off0, I1 = it.g1 + it.in_off1;
        const int64_t O0 = it.g0, O1 = it.g1;
        int64_t g0l, g0n, g1l, g1n, w0l, w0n, w1l, w1n;   // gathered and written boxes
        bool ok;
        if (!adjoint)
            ok = clip(I0, it.in_n0, S0, Sn0, g0l, g0n) && clip(I1, it.in_n1, S1, Sn1, g1l, g1n) &&
                 clip(O0, it.out_n0, T0, Tn0, w0l, w0n) && clip(O1, it.out_n1, T1, Tn1, w1l, w1n);
        else
            ok = clip(O0, it.out_n0, S0, Sn0, g0l, g0n) && clip(O1, it.out_n1, S1, Sn1, g1l, g1n) &&
                 clip(I0, it.in_n0, T0, Tn0, w0l, w0n) && clip(I1, it.in_n1, T1, Tn1, w1l, w1n);
        if (!ok) continue;
        Item c = it;
        if (!adjoint) {
            c.in_off0 = (int32_t)(g0l - it.g0);
            c.in_off1 = (int32_t)(g1l - it.g1);
            c.in_n0 = (int32_t)g0n;
            c.in_n1 = (int32_t)g1n;
            c.w_off = it.w_off + (g0l - I0) * it.w_ld + (g1l - I1);
            c.out_off0 = (int32_t)(w0l - it.g0);
            c.out_off1 = (int32_t)(w1l - it.g1);
            c.out_n0 = (int32_t)w0n;
            c.out_n1 = (int32_t)w1n;
        } else {
            c.out_off0 = (int32_t)(g0l - it.g0);
            c.out_off1 = (int32_t)(g1l - it.g1);
            c.out_n0 = (int32_t)g0n;
            c.out_n1 = (int32_t)g1n;
            c.in_off0 = (int32_t)(w0l - it.g0);
            c.in_off1 = (int32_t)(w1l - it.g1);
            c.in_n0 = (int32_t)w0n;
            c.in_n1 = (int32_t)w1n;
            c.w_off = it.w_off + (w0l - I0) * it.w_ld + (w1l - I1);
        }
        c.g0 = (int32_t)(it.g0 - S0);     // gather in S-local coordinates
        c.g1 = (int32_t)(it.g1 - S1);
        c.slot_fwd = c.slot_adj = B.per;
        boxes.push_back(Box{(int32_t)(w0l - T0), (int32_t)(w1l - T1), (int32_t)w0n, (int32_t)w1n, B.per});
        B.per += w0n * w1n;
        B.items.push_back(c);
    }
    std::vector<int32_t> contrib;
    if (!build_tiles(boxes, B.t_rows, B.t_cols, B.tiles, contrib, err)) return PC_ERR_UNSUPPORTED;
    B.cboxes.resize(contrib.size());
    for (size_t i = 0; i < contrib.size(); ++i) B.cboxes[i] = boxes[(size_t)contrib[i]];
    return PC_OK;
}

// ======================================================================
pc_status build_plan(const CreateArgs& a, Plan& p, std::string& err) {
    // ---------------------------------------------------------- arguments
    if (a.d < 1 || a.d > 3) {
        err = "d must be 1, 2 or 3";
        return PC_ERR_ARG;
    }
    if (!a.shape || !a.leaf_lo || !a.leaf_hi || !a.points || !a.radius || !a.phi || !a.phi_off) {
        err = "null host pointer";
        return PC_ERR_ARG;
    }
    if (a.n_leaves < 1 || a.r < 1) {
        err = "need at least one leaf and one point";
        return PC_ERR_ARG;
    }
    if (a.dtype != PC_F32 && a.dtype != PC_F64) {
        err = "dtype must be PC_F32 or PC_F64";
        return PC_ERR_ARG;
    }
    if (a.flags & ~(uint32_t)(PC_NO_EXTEND | PC_PLAN_HALF_LDS | PC_PLAN_SMALLEST_FFT)) {
        err = "unknown flag bits";
        return PC_ERR_ARG;
    }
    const int d = a.d;
    p.d = d;
    p.dtype = a.dtype;
    p.flags = a.flags;
    int64_t N = 1;
    for (int i = 0; i < d; ++i) {
        if (a.shape[i] < 1 || a.shape[i] > (1 << 20)) {
            err = "shape entries must be in [1, 2^20]";
            return PC_ERR_ARG;
        }
        p.shape[i] = a.shape[i];
        N *= a.shape[i];
    }
    if (N > ((int64_t)1 << 30)) {
        err = "domain too large (N > 2^30)";
        return PC_ERR_ARG;
    }
    p.N = N;
    const int64_t L = a.n_leaves, r = a.r;
    p.L = L;
    p.r = r;
    const int64_t* n = a.shape;
    // ------------------------------------------------------ tiling checks
    for (int64_t c = 0; c < L; ++c)
        for (int i = 0; i < d; ++i) {
            int64_t lo = a.leaf_lo[c * d + i], hi = a.leaf_hi[c * d + i];
            if (lo < 0 || hi > n[i] - 1 || lo > hi) {
                err = "leaf " + std::to_string(c) + " outside Omega or inverted";
                return PC_ERR_GRID;
            }
            if (n[i] > 1 && hi == lo) {
                err = "leaf " + std::to_string(c) + " is degenerate along a live axis";
                return PC_ERR_GRID;
            }
        }
    {
        long double vol = 0, tot = 1;
        for (int i = 0; i < d; ++i)
            if (n[i] > 1) tot *= (long double)(n[i] - 1);
        for (int64_t c = 0; c < L; ++c) {
            long double v = 1;
            for (int i = 0; i < d; ++i)
                if (n[i] > 1) v *= (long double)(a.leaf_hi[c * d + i] - a.leaf_lo[c * d + i]);
            vol += v;
        }
        if (std::fabs((double)(vol - tot)) > 0.5) {
            err = "leaf volumes do not add up to Omega";
            return PC_ERR_GRID;
        }
        // pairwise interiors: sort by lo along axis 0 and sweep
        std::vector<int64_t> ord(L);
        for (int64_t c = 0; c < L; ++c) ord[c] = c;
        std::sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) { return a.leaf_lo[x * d] < a.leaf_lo[y * d]; });
        for (int64_t ii = 0; ii < L; ++ii) {
            int64_t c = ord[ii];
            for (int64_t jj = ii + 1; jj < L; ++jj) {
                int64_t e = ord[jj];
                if (n[0] > 1 && a.leaf_lo[e * d] >= a.leaf_hi[c * d]) break;
                bool ov = true;
                for (int i = 0; i < d && ov; ++i) {
                    if (n[i] <= 1) continue;
                    int64_t lo = std::max(a.leaf_lo[c * d + i], a.leaf_lo[e * d + i]);
                    int64_t hi = std::min(a.leaf_hi[c * d + i], a.leaf_hi[e * d + i]);
                    ov = hi - lo > 0;
                }
                if (ov) {
                    err = "leaf interiors overlap (" + std::to_string(c) + ", " + std::to_string(e) + ")";
                    return PC_ERR_GRID;
                }
            }
        }
    }
    // ----------------------------------------------- points = leaf corners
    {
        std::set<std::vector<int64_t>> cs;
        std::vector<int64_t> v(d);
        for (int64_t c = 0; c < L; ++c)
            for (int bits = 0; bits < (1 << d); ++bits) {
                for (int i = 0; i < d; ++i)
                    v[i] = (bits >> (d - 1 - i)) & 1 ? a.leaf_hi[c * d + i] : a.leaf_lo[c * d + i];
                cs.insert(v);
            }
        if ((int64_t)cs.size() != r) {
            err = "point count " + std::to_string(r) + " != number of distinct leaf corners " +
                  std::to_string(cs.size());
            return PC_ERR_GRID;
        }
        int64_t k = 0;
        for (const auto& q : cs) {
            for (int i = 0; i < d; ++i)
                if (a.points[k * d + i] != q[i]) {
                    err = "points are not the sorted union of leaf corners (index " + std::to_string(k) + ")";
                    return PC_ERR_GRID;
                }
            ++k;
        }
    }
    // ------------------------------------------------- impulse responses
    {
        if (a.phi_off[0] != 0) {
            err = "phi_off[0] must be 0";
            return PC_ERR_ARG;
        }
        for (int64_t k = 0; k < r; ++k) {
            int64_t sz = 1;
            for (int i = 0; i < d; ++i) {
                int64_t R = a.radius[k * d + i];
                if (R < 0 || R > (1 << 16)) {
                    err = "radius of point " + std::to_string(k) + " out of range";
                    return PC_ERR_ARG;
                }
                sz *= 2 * R + 1;
            }
            if (a.phi_off[k + 1] - a.phi_off[k] != sz) {
                err = "phi_off does not match the radii at point " + std::to_string(k);
                return PC_ERR_ARG;
            }
        }
    }
    // ---------------------------------------------------- term selection
    p.sel.assign((size_t)r, a.n_sel < 0 ? 1 : 0);
    if (a.n_sel >= 0) {
        if (a.n_sel > 0 && !a.sel) {
            err = "null selection array";
            return PC_ERR_ARG;
        }
        for (int64_t i = 0; i < a.n_sel; ++i) {
            const int64_t k = a.sel[i];
            if (k < 0 || k >= r || p.sel[(size_t)k]) {
                err = "selected point indices must be distinct and in [0, r)";
                return PC_ERR_ARG;
            }
            p.sel[(size_t)k] = 1;
        }
    }
    if (d == 3) return build_plan_3d(a, p, err);

    // ------------------------------------------------------- 2-D view
    // d = 1 is handled as a single row: axis 0 of the view has extent 1.
    auto c0 = [&](const int64_t* v, int64_t k) -> int64_t { return d == 1 ? 0 : v[k * d + 0]; };
    auto c1 = [&](const int64_t* v, int64_t k) -> int64_t { return d == 1 ? v[k] : v[k * d + 1]; };
    const int64_t nr = (d == 1) ? 1 : n[0], nc = (d == 1) ? n[0] : n[1];
    p.rows = (int)nr;
    p.cols = (int)nc;
    std::vector<int64_t> P2(2 * r), R2(2 * r), LO(2 * L), HI(2 * L);
    for (int64_t k = 0; k < r; ++k) {
        P2[2 * k] = c0(a.points, k);
        P2[2 * k + 1] = c1(a.points, k);
        R2[2 * k] = d == 1 ? 0 : a.radius[k * d];
        R2[2 * k + 1] = c1(a.radius, k);
    }
    for (int64_t c = 0; c < L; ++c) {
        LO[2 * c] = c0(a.leaf_lo, c);
        LO[2 * c + 1] = c1(a.leaf_lo, c);
        HI[2 * c] = c0(a.leaf_hi, c);
        HI[2 * c + 1] = c1(a.leaf_hi, c);
    }
    // ------------------------------------------------ cells, nbrs, U_k
    std::vector<std::vector<int64_t>> leaf_pts(L), cells(r);
    for (int64_t c = 0; c < L; ++c)
        for (int64_t k = 0; k < r; ++k)
            if (P2[2 * k] >= LO[2 * c] && P2[2 * k] <= HI[2 * c] && P2[2 * k + 1] >= LO[2 * c + 1] &&
                P2[2 * k + 1] <= HI[2 * c + 1]) {
                leaf_pts[c].push_back(k);
                cells[k].push_back(c);
            }
    std::vector<std::vector<int64_t>> nbrs(r);
    std::vector<int64_t> Ulo(2 * r), Uhi(2 * r);
    for (int64_t k = 0; k < r; ++k) {
        std::set<int64_t> s;
        Ulo[2 * k] = Ulo[2 * k + 1] = INT64_MAX;
        Uhi[2 * k] = Uhi[2 * k + 1] = INT64_MIN;
        for (int64_t c : cells[k]) {
            for (int64_t j : leaf_pts[c]) s.insert(j);
            for (int i = 0; i < 2; ++i) {
                Ulo[2 * k + i] = std::min(Ulo[2 * k + i], LO[2 * c + i]);
                Uhi[2 * k + i] = std::max(Uhi[2 * k + i], HI[2 * c + i]);
            }
        }
        nbrs[k].assign(s.begin(), s.end());
    }
    p.leaf_pts_off.assign((size_t)L + 1, 0);
    for (int64_t c = 0; c < L; ++c) {
        p.leaf_pts_off[(size_t)c + 1] = p.leaf_pts_off[(size_t)c] + (int32_t)leaf_pts[c].size();
        for (int64_t k : leaf_pts[c]) p.leaf_pts.push_back((int32_t)k);
    }
    // ----------------------------------------------------------- weights
    // (only the selected points' tables are stored, only their leaves solved)
    std::vector<int64_t> w_base(r + 1, 0);
    for (int64_t k = 0; k < r; ++k)
        w_base[k + 1] = w_base[k] + (p.sel[(size_t)k] ? (Uhi[2 * k] - Ulo[2 * k] + 1) *
                                                            (Uhi[2 * k + 1] - Ulo[2 * k + 1] + 1)
                                                      : 0);
    p.pt_wbase.assign((size_t)r, -1);
    p.pt_ubox.assign((size_t)r * 6, 0);
    for (int64_t k = 0; k < r; ++k) {
        if (p.sel[(size_t)k]) p.pt_wbase[(size_t)k] = w_base[k];
        int32_t* u = &p.pt_ubox[(size_t)k * 6];
        u[0] = 0;
        u[1] = (int32_t)Ulo[2 * k];
        u[2] = (int32_t)Ulo[2 * k + 1];
        u[3] = 1;
        u[4] = (int32_t)(Uhi[2 * k] - Ulo[2 * k] + 1);
        u[5] = (int32_t)(Uhi[2 * k + 1] - Ulo[2 * k + 1] + 1);
    }
    std::vector<double> W((size_t)w_base[r], 0.0);
    // leaves are independent: weights are solved in parallel, then scattered
    // into the per-point tables in leaf order
    std::vector<std::vector<std::vector<double>>> leaf_vals((size_t)L);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < L; ++c) {
        bool any = false;
        for (int64_t k : leaf_pts[c]) any = any || p.sel[(size_t)k];
        if (!any) continue;
        std::vector<std::vector<double>>& vals = leaf_vals[(size_t)c];
        const int64_t lo[2] = {LO[2 * c], LO[2 * c + 1]}, hi[2] = {HI[2 * c], HI[2 * c + 1]};
        if (d == 1) {
            // two end points; linear hats
            vals.assign(leaf_pts[c].size(), std::vector<double>((size_t)(hi[1] - lo[1] + 1)));
            for (size_t j = 0; j < leaf_pts[c].size(); ++j) {
                int64_t pp = P2[2 * leaf_pts[c][j] + 1];
                for (int64_t y = lo[1]; y <= hi[1]; ++y)
                    vals[j][(size_t)(y - lo[1])] = 1.0 - std::fabs((double)(y - pp)) / (double)(hi[1] - lo[1]);
            }
        } else {
            leaf_weights_2d(lo, hi, leaf_pts[c], P2.data(), vals);
        }
    }
    for (int64_t c = 0; c < L; ++c) {
        const std::vector<std::vector<double>>& vals = leaf_vals[(size_t)c];
        if (vals.empty()) continue;
        const int64_t lo[2] = {LO[2 * c], LO[2 * c + 1]}, hi[2] = {HI[2 * c], HI[2 * c + 1]};
        const int64_t w1 = hi[1] - lo[1] + 1;
        for (size_t j = 0; j < leaf_pts[c].size(); ++j) {
            int64_t k = leaf_pts[c][j];
            if (!p.sel[(size_t)k]) continue;
            int64_t um1 = Uhi[2 * k + 1] - Ulo[2 * k + 1] + 1;
            for (int64_t y0 = lo[0]; y0 <= hi[0]; ++y0)
                for (int64_t y1 = lo[1]; y1 <= hi[1]; ++y1)
                    W[(size_t)(w_base[k] + (y0 - Ulo[2 * k]) * um1 + (y1 - Ulo[2 * k + 1]))] =
                        vals[j][(size_t)((y0 - lo[0]) * w1 + (y1 - lo[1]))];
        }
        std::vector<std::vector<double>>().swap(leaf_vals[(size_t)c]);
    }
    p.wts = std::move(W);
    // ------------------------------------------------ extension + planning
    const bool extend = !(a.flags & PC_NO_EXTEND);
    const size_t csz = (a.dtype == PC_F64) ? 16 : 8;
    const bool half = (a.flags & PC_PLAN_HALF_LDS) != 0;
    const int64_t lds_cap = half ? kLdsBytes / 2 : kLdsBytes;
    p.conv_threads = (half || a.dtype == PC_F64) ? 512 : 1024;
    TwiddleTables twt{&p.tw, {}, {}};
    p.items.clear();
    p.spec.clear();
    struct PatchOut {
        pc_status st = PC_OK;
        std::string err;
        std::vector<double> E;       // phi_k^E on [zlo, zhi] (until its spectrum is formed)
        int64_t zlo[2] = {0, 0}, zhi[2] = {0, 0};
        std::vector<Item> items;
        int n0 = 0, M = 0, a0 = 1, b0 = 1, am = 1, bm = 1;
        int64_t spec_off = 0;
        double flops = 0.0;
        int64_t kel = 0;
    };
    std::vector<PatchOut> outs((size_t)r);
    // every patch is independent: extension, sizes, spectrum and pieces are
    // computed in parallel, then assembled in patch order below
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < r; ++k) {
        PatchOut& po = outs[(size_t)k];
        if (!p.sel[(size_t)k]) continue;
        const int64_t I_lo[2] = {Ulo[2 * k], Ulo[2 * k + 1]}, I_hi[2] = {Uhi[2 * k], Uhi[2 * k + 1]};
        const int64_t m[2] = {I_hi[0] - I_lo[0] + 1, I_hi[1] - I_lo[1] + 1};
        int64_t Rm[2] = {R2[2 * k], R2[2 * k + 1]};
        if (extend)
            for (int64_t j : nbrs[k])
                for (int i = 0; i < 2; ++i) Rm[i] = std::max(Rm[i], R2[2 * j + i]);
        const int64_t ndom[2] = {nr, nc};
        int64_t zlo[2], zhi[2], K[2];
        for (int i = 0; i < 2; ++i) {
            zlo[i] = std::max(-Rm[i], -I_hi[i]);
            zhi[i] = std::min(Rm[i], ndom[i] - 1 - I_lo[i]);
            K[i] = zhi[i] - zlo[i] + 1;
        }
        po.kel = (2 * R2[2 * k] + 1) * (2 * R2[2 * k + 1] + 1);
        // extended kernel phi_k^E on the box [zlo, zhi]
        std::vector<double> E((size_t)(K[0] * K[1]), 0.0);
        auto defined = [&](int64_t j, int64_t z0, int64_t z1) {
            int64_t y0 = P2[2 * j] + z0, y1 = P2[2 * j + 1] + z1;
            return y0 >= 0 && y0 < nr && y1 >= 0 && y1 < nc;
        };
        auto val = [&](int64_t j, int64_t z0, int64_t z1) -> double {
            int64_t Ra = R2[2 * j], Rb = R2[2 * j + 1];
            if (z0 < -Ra || z0 > Ra || z1 < -Rb || z1 > Rb) return 0.0;
            return a.phi[a.phi_off[j] + (z0 + Ra) * (2 * Rb + 1) + (z1 + Rb)];
        };
        for (int64_t z0 = zlo[0]; z0 <= zhi[0]; ++z0)
            for (int64_t z1 = zlo[1]; z1 <= zhi[1]; ++z1) {
                double v = 0.0;
                if (defined(k, z0, z1)) {
                    v = val(k, z0, z1);
                } else if (extend) {
                    int cnt = 0;
                    double s = 0.0;
                    for (int64_t j : nbrs[k]) {
                        if (j == k || !defined(j, z0, z1)) continue;
                        ++cnt;
                        s += val(j, z0, z1);
                    }
                    if (cnt) v = s / (double)cnt;
                }
                E[(size_t)((z0 - zlo[0]) * K[1] + (z1 - zlo[1]))] = v;
            }
        // The box above allows for the largest neighbour radius, but phi_k^E
        // is zero wherever p_k + z lies in Omega and z is outside phi_k's own
        // box (the extension only fills offsets that leave Omega), so away
        // from the boundary most of that margin is zero.  The kernel box is
        // cut to the bounding box of the non-zero entries: the same sum,
        // with shorter FFTs and smaller output boxes.
        {
            int64_t lo0 = K[0], hi0 = -1, lo1 = K[1], hi1 = -1;
            for (int64_t i0 = 0; i0 < K[0]; ++i0)
                for (int64_t i1 = 0; i1 < K[1]; ++i1)
                    if (E[(size_t)(i0 * K[1] + i1)] != 0.0) {
                        lo0 = std::min(lo0, i0);
                        hi0 = std::max(hi0, i0);
                        lo1 = std::min(lo1, i1);
                        hi1 = std::max(hi1, i1);
                    }
            if (hi0 < 0) {   // an all-zero kernel: keep one (zero) entry at the smallest |z| in the box
                lo0 = hi0 = std::min(std::max<int64_t>(-zlo[0], 0), K[0] - 1);
                lo1 = hi1 = std::min(std::max<int64_t>(-zlo[1], 0), K[1] - 1);
            }
            if (lo0 > 0 || hi0 < K[0] - 1 || lo1 > 0 || hi1 < K[1] - 1) {
                const int64_t K0 = hi0 - lo0 + 1, K1 = hi1 - lo1 + 1;
                std::vector<double> T((size_t)(K0 * K1));
                for (int64_t i0 = 0; i0 < K0; ++i0)
                    for (int64_t i1 = 0; i1 < K1; ++i1)
                        T[(size_t)(i0 * K1 + i1)] = E[(size_t)((i0 + lo0) * K[1] + (i1 + lo1))];
                E.swap(T);
                zlo[0] += lo0;
                zlo[1] += lo1;
                zhi[0] = zlo[0] + K0 - 1;
                zhi[1] = zlo[1] + K1 - 1;
                K[0] = K0;
                K[1] = K1;
            }
        }
        // algorithmic flops by the unsplit 7-smooth convention
        {
            int64_t nn = (int64_t)smallest_7smooth(m[0] + K[0] - 1) * smallest_7smooth(m[1] + K[1] - 1);
            int64_t O = (std::min(I_hi[0] + zhi[0], nr - 1) - std::max(I_lo[0] + zlo[0], (int64_t)0) + 1) *
                        (std::min(I_hi[1] + zhi[1], nc - 1) - std::max(I_lo[1] + zlo[1], (int64_t)0) + 1);
            po.flops = 5.0 * nn * std::log2((double)nn) + 3.0 * nn + (double)(m[0] * m[1]) + (double)O;
        }
        // choose FFT lengths and the number of row pieces
        const int64_t need1 = m[1] + K[1] - 1;
        (void)need1;
        int M = 0, ldr = 0;
        // P0 x P1 pieces (rows x columns) and FFT lengths that fit LDS.
        // Default: the least estimated time over the pieces (unit_cycles:
        // whole SIMD rounds per phase at the measured per-task instruction
        // counts, the gather and copy-out, and the staged output box read
        // back by the reduction), at lengths up to 35 % above the needed
        // ones (a longer length with cheaper radices or fewer rounds can
        // win) and up to two more row pieces than the fewest that fit.
        // With PC_PLAN_SMALLEST_FFT: the smallest supported lengths, the
        // fewest row pieces that fit and the least n log n over the pieces.
        const bool smallest = (a.flags & PC_PLAN_SMALLEST_FFT) != 0;
        const int NT = p.conv_threads;
        int best_P0 = -1, best_P1 = -1, best_n0 = 0, best_M = 0;
        double best_cost = 1e300;
        const int maxP0 = (int)std::min<int64_t>(m[0], 64), maxP1 = (int)std::min<int64_t>(m[1], 64);
        for (int P1 = 1; P1 <= maxP1; ++P1) {
            const int64_t h1 = (m[1] + P1 - 1) / P1;
            const int need_m = (int)((h1 + K[1] - 1 + 1) / 2);
            const int Mlo = next_fft_size(need_m);
            if (Mlo < 0 || Mlo > 128) continue;
            const int Mhi = smallest ? Mlo : std::min(128, (int)std::ceil(need_m * 1.35));
            bool fit_any = false;
            for (int Mp = Mlo; Mp <= Mhi; ++Mp) {
                int ap, bp;
                if (!fft_factor(Mp, &ap, &bp) || bp > 10) continue;
                int ld_p = Mp + 1;
                if (ld_p % 2 == 0) ++ld_p;
                int first_fit = -1;
                for (int P0 = 1; P0 <= maxP0; ++P0) {
                    if (first_fit > 0 && (smallest || P0 > first_fit + 2)) break;
                    const int64_t h0 = (m[0] + P0 - 1) / P0;
                    const int need0 = (int)(h0 + K[0] - 1);
                    const int nlo = (d == 1) ? 1 : next_fft_size(need0);
                    if (nlo < 0) continue;
                    const int nhi = (d == 1 || smallest) ? nlo : std::min(256, (int)std::ceil(need0 * 1.35));
                    bool fit = false;
                    for (int n0p = nlo; n0p <= nhi; ++n0p) {
                        int a0p = 1, b0p = 1;
                        if (d != 1 && !fft_factor(n0p, &a0p, &b0p)) continue;
                        if (((int64_t)n0p * ld_p + twiddle_elems(a0p, b0p, ap, bp)) * (int64_t)csz > lds_cap)
                            continue;   // box + twiddles
                        fit = true;
                        double cost;
                        if (smallest) {
                            const double nn = (double)n0p * 2.0 * Mp;
                            cost = (double)P0 * P1 * nn * std::log2(std::max(nn, 2.0));
                        } else {
                            const int64_t out0 = std::min<int64_t>(n0p, h0 + K[0] - 1);
                            cost = (double)P0 * P1 *
                                   unit_cycles(NT, n0p, a0p, b0p, Mp, ap, bp, h0, out0, std::min<int64_t>(2 * Mp, h1 + K[1] - 1));
                            // FP32 items within half a CU's LDS run two workgroups per CU
                            // (measured: about 0.73 of their one-per-CU time)
                            const int64_t lds_item = ((int64_t)n0p * ld_p + twiddle_elems(a0p, b0p, ap, bp)) * (int64_t)csz;
                            if (a.dtype == PC_F32 && lds_item <= kSmallItemLds) cost *= 0.73;
                        }
                        if (cost < best_cost) {
                            best_cost = cost;
                            best_P0 = P0;
                            best_P1 = P1;
                            best_n0 = n0p;
                            best_M = Mp;
                        }
                    }
                    if (fit) {
                        fit_any = true;
                        if (first_fit < 0) first_fit = P0;
                    }
                }
            }
            (void)fit_any;
        }
        if (best_P0 < 0) {
            po.err = "patch " + std::to_string(k) + " does not fit the LDS-resident FFT";
            po.st = PC_ERR_UNSUPPORTED;
            continue;
        }
        M = best_M;
        ldr = M + 1;
        if (ldr % 2 == 0) ++ldr;
        const int n0 = best_n0;
        int a0, b0, am, bm;
        fft_factor(n0, &a0, &b0);
        fft_factor(M, &am, &bm);
        if (M > 128 || bm > 10) {
            po.err = "patch " + std::to_string(k) + " needs a row FFT outside the supported lengths";
            po.st = PC_ERR_UNSUPPORTED;
            continue;
        }
        po.n0 = n0;
        po.M = M;
        const int n1 = 2 * M;
        po.a0 = a0;
        po.b0 = b0;
        po.am = am;
        po.bm = bm;
        for (int i = 0; i < 2; ++i) {
            po.zlo[i] = zlo[i];
            po.zhi[i] = zhi[i];
        }
        po.E = std::move(E);
        // pieces: P0 row ranges x P1 column ranges of the patch box
        for (int i0 = 0; i0 < best_P0; ++i0)
            for (int i1 = 0; i1 < best_P1; ++i1) {
                const int64_t s0 = (m[0] * i0) / best_P0, e0 = (m[0] * (i0 + 1)) / best_P0;
                const int64_t s1 = (m[1] * i1) / best_P1, e1 = (m[1] * (i1 + 1)) / best_P1;
                if (e0 <= s0 || e1 <= s1) continue;
                const int64_t plo0 = I_lo[0] + s0, phi0 = I_lo[0] + e0 - 1;
                const int64_t plo1 = I_lo[1] + s1, phi1 = I_lo[1] + e1 - 1;
                const int64_t olo0 = std::max(plo0 + zlo[0], (int64_t)0), ohi0 = std::min(phi0 + zhi[0], nr - 1);
                const int64_t olo1 = std::max(plo1 + zlo[1], (int64_t)0), ohi1 = std::min(phi1 + zhi[1], nc - 1);
                Item it;
                std::memset(&it, 0, sizeof(it));
                it.n0 = n0;
                it.a0 = a0;
                it.b0 = b0;
                it.m = M;
                it.am = am;
                it.bm = bm;
                it.ld = ldr;
                it.g0 = (int32_t)olo0;
                it.g1 = (int32_t)olo1;
                it.in_off0 = (int32_t)(plo0 - olo0);
                it.in_off1 = (int32_t)(plo1 - olo1);
                it.in_n0 = (int32_t)(e0 - s0);
                it.in_n1 = (int32_t)(e1 - s1);
                it.out_n0 = (int32_t)(ohi0 - olo0 + 1);
                it.out_n1 = (int32_t)(ohi1 - olo1 + 1);
                it.patch = (int32_t)k;
                it.w_ld = (int32_t)m[1];
                it.w_off = w_base[k] + s0 * m[1] + s1;
                // the FFT box must hold input and output without wrap-around
                if (it.in_off0 < 0 || it.in_off1 < 0 || it.in_off0 + it.in_n0 > n0 || it.in_off1 + it.in_n1 > n1 ||
                    it.out_n0 > n0 || it.out_n1 > n1) {
                    po.err = "internal planning error (FFT box too small) at patch " + std::to_string(k);
                    po.st = PC_ERR_ARG;
                    continue;
                }
                po.items.push_back(it);
            }
    }
    // assembly in patch order: spectrum offsets, twiddle tables, staging offsets
    int64_t kernel_elems = 0;
    double alg_flops = 0.0;
    int64_t spec_total = 0;

    for (int64_t k = 0; k < r; ++k) {
        PatchOut& po = outs[(size_t)k];
        if (po.st != PC_OK) {
            err = po.err;
            return po.st;
        }
        if (!p.sel[(size_t)k]) continue;
        kernel_elems += po.kel;
        alg_flops += po.flops;
        const int64_t spec_off = spec_total;
        po.spec_off = spec_off;
        spec_total += (int64_t)po.n0 * (po.M + 1);
        const int t0 = twt.pass(po.a0, po.b0), tm = twt.pass(po.am, po.bm), t2m = twt.pair(po.am, po.bm);
        int ldr = po.M + 1;
        if (ldr % 2 == 0) ++ldr;
        for (Item it : po.items) {
            it.tw0 = t0;
            it.twm = tm;
            it.tw2m = t2m;
            it.spec_off = spec_off;
            it.slot_fwd = p.slot_fwd;
            it.slot_adj = p.slot_adj;
            p.slot_fwd += (int64_t)it.out_n0 * it.out_n1;
            p.slot_adj += (int64_t)it.in_n0 * it.in_n1;
            p.sum_fft_points += (int64_t)po.n0 * 2 * po.M;
            p.max_lds = std::max(p.max_lds, (int)(((int64_t)po.n0 * ldr + twiddle_elems(po.a0, po.b0, po.am, po.bm)) * csz));
            p.items.push_back(it);
        }
    }
    p.kernel_elems = kernel_elems;
    p.alg_flops = alg_flops;
    // extended kernels kept for matrix entries
    p.pt_eoff.assign((size_t)r, -1);
    p.pt_ebox.assign((size_t)r * 6, 0);
    int64_t e_total = 0;
    for (int64_t k = 0; k < r; ++k) {
        if (!p.sel[(size_t)k]) continue;
        const PatchOut& po = outs[(size_t)k];
        int32_t* e = &p.pt_ebox[(size_t)k * 6];
        e[0] = 0;
        e[1] = (int32_t)po.zlo[0];
        e[2] = (int32_t)po.zlo[1];
        e[3] = 1;
        e[4] = (int32_t)(po.zhi[0] - po.zlo[0] + 1);
        e[5] = (int32_t)(po.zhi[1] - po.zlo[1] + 1);
        p.pt_eoff[(size_t)k] = e_total;
        e_total += (int64_t)e[4] * e[5];
    }
    p.phiE.assign((size_t)e_total, 0.0);
    // spectra of phi_k^E placed circularly, FP64, half spectrum along axis 1,
    // written in place (patches in parallel)
    p.spec.assign((size_t)(2 * spec_total), 0.0);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < r; ++k) {
        PatchOut& po = outs[(size_t)k];
        if (!p.sel[(size_t)k]) continue;
        const int n0 = po.n0, M = po.M, n1 = 2 * M;
        const int64_t* zlo = po.zlo;
        const int64_t* zhi = po.zhi;
        const int64_t K1 = zhi[1] - zlo[1] + 1;
        std::vector<cd> G((size_t)n0 * n1, cd(0.0));
        for (int64_t z0 = zlo[0]; z0 <= zhi[0]; ++z0)
            for (int64_t z1 = zlo[1]; z1 <= zhi[1]; ++z1) {
                int64_t i0 = ((z0 % n0) + n0) % n0, i1 = ((z1 % n1) + n1) % n1;
                G[(size_t)(i0 * n1 + i1)] += po.E[(size_t)((z0 - zlo[0]) * K1 + (z1 - zlo[1]))];
            }
        std::copy(po.E.begin(), po.E.end(), p.phiE.begin() + p.pt_eoff[(size_t)k]);
        std::vector<double>().swap(po.E);
        std::vector<cd> rowout((size_t)n1), colin((size_t)n0), colout((size_t)n0);
        const Dft64& F1 = dft64(n1);
        const Dft64& F0 = dft64(n0);
        std::vector<cd> H((size_t)n0 * (M + 1), cd(0.0));
        std::vector<char> live((size_t)n0, 0);
        for (int64_t z0 = zlo[0]; z0 <= zhi[0]; ++z0) live[(size_t)(((z0 % n0) + n0) % n0)] = 1;
        for (int i0 = 0; i0 < n0; ++i0) {
            if (!live[(size_t)i0]) continue;      // rows outside the kernel box stay zero
            F1.run(&G[(size_t)i0 * n1], 1, rowout.data());
            for (int kk = 0; kk <= M; ++kk) H[(size_t)i0 * (M + 1) + kk] = rowout[kk];
        }
        // 1/(n0 M) normalises the inverse transforms; the extra 1/4 stands
        // for the factors 1/2 that the kernels' real-row post- and
        // pre-processing leave out
        const double sc = 0.25 / ((double)n0 * (double)M);
        double* out = &p.spec[(size_t)(2 * po.spec_off)];
        for (int kk = 0; kk <= M; ++kk) {
            for (int i0 = 0; i0 < n0; ++i0) colin[i0] = H[(size_t)i0 * (M + 1) + kk];
            F0.run(colin.data(), 1, colout.data());
            int s1 = (kk < M) ? perm_slot(kk, po.am, po.bm) : M;
            for (int k0 = 0; k0 < n0; ++k0) {
                int s0 = perm_slot(k0, po.a0, po.b0);
                out[2 * ((size_t)s0 * (M + 1) + s1)] = colout[k0].real() * sc;
                out[2 * ((size_t)s0 * (M + 1) + s1) + 1] = colout[k0].imag() * sc;
            }
        }
    }
    // ------------------------- summation order and reduction tiles
    std::vector<Box> bf(p.items.size()), ba(p.items.size());
    for (size_t i = 0; i < p.items.size(); ++i) {
        const Item& it = p.items[i];
        bf[i] = Box{it.g0, it.g1, it.out_n0, it.out_n1, it.slot_fwd};
        ba[i] = Box{it.g0 + it.in_off0, it.g1 + it.in_off1, it.in_n0, it.in_n1, it.slot_adj};
    }
    colour_boxes(bf, p.rows, p.cols, p.order_fwd, p.cbeg_fwd);
    colour_boxes(ba, p.rows, p.cols, p.order_adj, p.cbeg_adj);
    std::vector<Box> bfo(bf.size()), bao(ba.size());
    for (size_t j = 0; j < bf.size(); ++j) {
        bfo[j] = bf[(size_t)p.order_fwd[j]];
        bao[j] = ba[(size_t)p.order_adj[j]];
    }
    if (!finish_tiles(p, bfo, bao, err)) return PC_ERR_UNSUPPORTED;
    p.planes = 1;
    p.prow = p.rows;
    p.leaf_box.resize(6 * L);
    for (int64_t c = 0; c < L; ++c) {
        int32_t* b = &p.leaf_box[6 * c];
        b[0] = 0;
        b[1] = (int32_t)LO[2 * c];
        b[2] = (int32_t)LO[2 * c + 1];
        b[3] = 1;
        b[4] = (int32_t)(HI[2 * c] - LO[2 * c] + 1);
        b[5] = (int32_t)(HI[2 * c + 1] - LO[2 * c + 1] + 1);
    }
    return PC_OK;
}

}  // namespace pc
