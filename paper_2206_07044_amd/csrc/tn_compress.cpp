// One bond compression between two dense matrices (tn_compress_pair): the compression
// primitive of section II.C, Eq. (svd), on its own, through the same kernels the tree
// executor runs for bonds of size D <= 64 (narrow split-K Grams or explicit factors, the
// LDS-resident pivoted-Cholesky + Jacobi core, and the grouped GEMM for the re-absorption).
#include "tn_compress.hpp"

#include <algorithm>
#include <cstring>
#include <string>

#include "tn_kernels.hpp"
#include "tn_plan.hpp"

namespace tn {

namespace {

constexpr int64_t kAlignB = 256;
constexpr int64_t kGramRows = 512;   // rows per split of the narrow Gram kernel

int64_t up(int64_t x) { return (x + kAlignB - 1) / kAlignB * kAlignB; }

std::string dense(int64_t rows, int64_t rs, int64_t cols, int64_t cs, View* v) {
    ViewSpec s;
    s.row_dims = {(int32_t)rows};
    s.row_strides = {rs};
    s.col_dims = {(int32_t)cols};
    s.col_strides = {cs};
    return make_view(s, v);
}

}  // namespace

std::string pair_layout(int64_t ma, int64_t D, int64_t mb, int64_t chi, PairLayout* L) {
    if (ma < 1 || mb < 1 || D < 1 || chi < 1) return "m_a, D, m_b and chi must be >= 1";
    if (D > kCoreLdsMaxD) return "D must be at most 64";
    if (ma * D > INT32_MAX || mb * D > INT32_MAX) return "m_a * D and m_b * D must be below 2^31";
    PairLayout l{};
    l.ma = ma;
    l.D = D;
    l.mb = mb;
    l.nw = std::min<int64_t>(chi, std::min(std::min(ma, D), std::min(mb, D)));
    l.gram_a = ma > D;
    l.gram_b = mb > D;
    l.splits_a = l.gram_a ? (ma + kGramRows - 1) / kGramRows : 0;
    l.splits_b = l.gram_b ? (mb + kGramRows - 1) / kGramRows : 0;
    int64_t off = 0;
    l.off_desc = off;
    off = up(off + (int64_t)sizeof(PairDescs));
    l.off_side_a = off;
    off = up(off + 8 * (l.gram_a ? l.splits_a * D * D : ma * D));
    l.off_side_b = off;
    off = up(off + 8 * (l.gram_b ? l.splits_b * D * D : mb * D));
    l.off_work = off;
    off = up(off + 8 * (4 * D * D + 4 * D + 2 * D * l.nw));
    l.off_pl = off;
    off = up(off + 8 * D * l.nw);
    l.off_pr = off;
    off = up(off + 8 * l.nw * D);
    l.off_maxparts = off;
    l.n_maxparts = (ma + 63) / 64 + ((l.nw + 63) / 64) * ((mb + 63) / 64);
    off = up(off + 8 * l.n_maxparts);
    l.off_stats = off;   // discarded weight (double), tie (int32), sweeps (int32)
    off = up(off + 16);
    l.bytes = off;
    *L = l;
    return "";
}

std::string pair_enqueue(const PairLayout& L, const double* a, const double* b, double cutoff, int max_sweeps,
                         double* a_out, double* b_out, char* ws, PairDescs* h, hipStream_t s) {
    std::memset(h, 0, sizeof(*h));
    const int64_t D = L.D, ma = L.ma, mb = L.mb, nw = L.nw;
    PairDescs* dd = (PairDescs*)(ws + L.off_desc);
    double* side_a = (double*)(ws + L.off_side_a);
    double* side_b = (double*)(ws + L.off_side_b);
    double* maxparts = (double*)(ws + L.off_maxparts);
    double* disc = (double*)(ws + L.off_stats);
    int32_t* tie = (int32_t*)(ws + L.off_stats + 8);
    int32_t* sweeps = tie + 1;
    std::string err;
    // ---- side factors: split-K Grams A^T A and B B^T (D x D per split), or the explicit
    //      factors A (ma x D) and B^T (mb x D) when a side has no more rows than D
    int ngram = 0, ncopy = 0;
    for (int side = 0; side < 2; ++side) {
        const bool gram = side == 0 ? L.gram_a : L.gram_b;
        const int64_t m = side == 0 ? ma : mb;
        const double* src = side == 0 ? a : b;
        double* dst = side == 0 ? side_a : side_b;
        // side A: A is (ma x D) row-major; side B: B^T is (mb x D) with element (r, c) at c * mb + r
        const int64_t rs = side == 0 ? D : 1, cs = side == 0 ? 1 : mb;
        if (gram) {
            GemmDesc& g = h->gram[ngram++];
            if (err.empty()) err = dense(D, cs, m, rs, &g.va);   // X^T (D x m)
            if (err.empty()) err = dense(m, rs, D, cs, &g.vb);   // X   (m x D)
            g.A = src;
            g.B = src;
            g.C = dst;
            g.M = (int32_t)D;
            g.N = (int32_t)D;
            g.K = (int32_t)m;
            g.mode = GEMM_GRAM;
            g.tiles_m = 1;
            g.tiles_n = 1;
            g.splits = (int32_t)(side == 0 ? L.splits_a : L.splits_b);
            g.k_per_split = (int32_t)kGramRows;
            g.scale_a = g.scale_b = -1;
        } else {
            CopyDesc& c = h->copy[ncopy++];
            if (err.empty()) err = dense(m, rs, D, cs, &c.v);
            c.src = src;
            c.dst = dst;
            c.rows = (int32_t)m;
            c.cols = (int32_t)D;
            c.scale = -1;
        }
    }
    int64_t tiles = 0;
    for (int i = 0; i < ngram; ++i) {
        h->gram[i].tile_begin = tiles;
        tiles += h->gram[i].splits;
    }
    int64_t elems = 0;
    for (int i = 0; i < ncopy; ++i) {
        h->copy[i].elem_begin = elems;
        elems += (int64_t)h->copy[i].rows * h->copy[i].cols;
    }
    // ---- core: reduced factors, Jacobi SVD of R~_A R~_B^T, projectors (float64)
    CoreDesc& cd = h->core;
    cd.gram_a = L.gram_a ? side_a : nullptr;
    cd.fac_a = L.gram_a ? nullptr : side_a;
    cd.gram_b = L.gram_b ? side_b : nullptr;
    cd.fac_b = L.gram_b ? nullptr : side_b;
    cd.splits_a = (int32_t)std::max<int64_t>(1, L.splits_a);
    cd.splits_b = (int32_t)std::max<int64_t>(1, L.splits_b);
    cd.rows_a = L.gram_a ? 0 : (int32_t)ma;
    cd.rows_b = L.gram_b ? 0 : (int32_t)mb;
    cd.D = (int32_t)D;
    cd.chi_new = (int32_t)nw;
    cd.cutoff = cutoff;
    cd.work = (double*)(ws + L.off_work);
    cd.p_left = ws + L.off_pl;
    cd.p_right = ws + L.off_pr;
    cd.stat = 0;
    cd.kmin = (int32_t)std::min(std::min(ma, D), std::min(mb, D));
    // ---- re-absorption: a' = A P_L (ma x nw), b' = P_R B (nw x mb)
    for (int side = 0; side < 2; ++side) {
        GemmDesc& g = h->absorb[side];
        if (side == 0) {
            if (err.empty()) err = dense(ma, D, D, 1, &g.va);
            if (err.empty()) err = dense(D, nw, nw, 1, &g.vb);
            g.A = a;
            g.B = ws + L.off_pl;
            g.C = a_out;
            g.M = (int32_t)ma;
            g.N = (int32_t)nw;
            g.maxpart = 0;
        } else {
            if (err.empty()) err = dense(nw, D, D, 1, &g.va);
            if (err.empty()) err = dense(D, mb, mb, 1, &g.vb);
            g.A = ws + L.off_pr;
            g.B = b;
            g.C = b_out;
            g.M = (int32_t)nw;
            g.N = (int32_t)mb;
            g.maxpart = (int32_t)((ma + 63) / 64);
        }
        g.K = (int32_t)D;
        g.mode = GEMM_TENSOR;
        g.tiles_m = (int32_t)((g.M + 63) / 64);
        g.tiles_n = (int32_t)((g.N + 63) / 64);
        g.splits = 1;
        g.k_per_split = (int32_t)D;
        g.scale_a = g.scale_b = -1;
    }
    h->absorb[0].tile_begin = 0;
    h->absorb[1].tile_begin = (int64_t)h->absorb[0].tiles_m * h->absorb[0].tiles_n;
    const int64_t absorb_tiles = h->absorb[1].tile_begin + (int64_t)h->absorb[1].tiles_m * h->absorb[1].tiles_n;
    if (!err.empty()) return err;

    auto hip = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && err.empty()) err = std::string(what) + ": " + hipGetErrorString(e);
        return e == hipSuccess;
    };
    if (!hip(hipMemcpyAsync(dd, h, sizeof(PairDescs), hipMemcpyHostToDevice, s), "descriptor upload")) return err;
    if (ngram && !hip(launch_gemm(GEMM_GRAM_NARROW_F64, dd->gram, ngram, tiles, nullptr, nullptr, s), "Gram"))
        return err;
    if (ncopy && !hip(launch_copy(0, dd->copy, ncopy, elems, nullptr, s), "factor copy")) return err;
    if (!hip(launch_core(1, 0, &dd->core, 1, (int)D, max_sweeps, disc, tie, sweeps, s), "core")) return err;
    if (!hip(launch_gemm(GEMM_F64, dd->absorb, 2, absorb_tiles, nullptr, maxparts, s), "re-absorption")) return err;
    return err;
}

}  // namespace tn
