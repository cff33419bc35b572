// C ABI (include/tn.h): context, device arena, schedule upload and execution.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/tn.h"
#include "tn_compress.hpp"
#include "tn_kernels.hpp"
#include "tn_krylov.hpp"
#include "tn_plan.hpp"
#include "tn_tune.hpp"
#include "tn_static.hpp"

using namespace tn;

namespace {

// L_SPRE: the float64 products that form a Gram-Lanczos operator (key 0: T1, key 1: S = F_X T1)
// L_KRYLOV: the block-Krylov chains of a level (begin/count index the chain steps, KOp)
enum LaunchKind { L_GEMM = 0, L_COPY, L_CORE, L_SCALE, L_LANCZOS, L_GLANCZOS, L_REDUCE, L_CORE_BWD, L_SPRE, L_KRYLOV,
                  L_TSQR };

struct Launch {
    int kind = 0;
    int key = 0;          // GEMM instantiation / tensor precision / CORE lds flag
    int64_t begin = 0;    // first descriptor
    int count = 0;
    int64_t work = 0;     // tiles / elements
    int max_d = 0;
    int prof = 0;         // tn_kernel_kind for timing
    double flops = 0;     // algorithmic flops of the steps in this launch
    double bytes = 0;     // algorithmic bytes of the steps in this launch
    int level = 0;        // schedule level (forward or reverse numbering)
};

constexpr int kKinds = 12;   // >= number of tn_kernel_kind values
constexpr int kLanes = 4;    // streams per level: tensor GEMMs + scales, cores, Lanczos, Gram GEMMs + copies

}  // namespace

// Arena above which a plan is levelled in tree order (a third of an MI355X's 288 GB).
constexpr int64_t kArenaSoftCap = (int64_t)96 << 30;
// Forward schedules of more kernel launches than this are enqueued launch by launch on every
// evaluation instead of being captured into a hipGraph: a capture of some 230,000 launches (the
// 12^3 chi = 64 tree, ~1,700 block-Jacobi cores of up to 272 launches each) ended the process
// inside the runtime, while captures of up to ~11,000 launches run; such schedules are bound by
// their kernels, not by launch overhead, so replay gains nothing there.
constexpr int64_t kMaxCaptureKernels = 20000;

struct tn_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // independent kernel kinds of one level run concurrently on these (fork/join per level)
    hipStream_t aux[kLanes - 1] = {nullptr, nullptr, nullptr};
    std::vector<hipEvent_t> sync_ev;   // fork/join events (timing disabled)
    std::vector<hipEvent_t> rc_ev;     // the same, for re-runs of forward segments in the reverse pass
    std::string err;

    GraphSpec g;
    bool has_graph = false;
    // Ising coupling map (graphs whose edges all have dimension 2)
    bool ising_ok = false;
    IsingGraph ising{};
    int32_t* d_ising_i32 = nullptr;     // inc_off | inc_edge | edge_u | edge_v
    int64_t* d_ising_off = nullptr;
    int64_t n_input_elems = 0;
    double* d_staging = nullptr;

    Plan plan;
    bool has_plan = false;
    char* arena = nullptr;
    size_t arena_cap = 0;
    bool arena_owned = true;           // false: the arena is the caller's workspace (tn_set_workspace)
    char* workspace = nullptr;         // caller-owned device memory for the next plans, or null
    size_t workspace_bytes = 0;

    std::vector<GemmDesc> h_gemm;
    std::vector<CopyDesc> h_copy;
    std::vector<CoreDesc> h_core;
    std::vector<ScaleDesc> h_scale;
    std::vector<InputDesc> h_inputs;
    std::vector<LanczosDesc> h_lanczos;
    LanczosDesc* d_lanczos = nullptr;
    std::vector<GLanczosDesc> h_glanczos;
    GLanczosDesc* d_glanczos = nullptr;
    // block-Krylov chains: their steps, and the small-operation and block-factor descriptors
    std::vector<KOp> h_kops;
    std::vector<SmallDesc> h_small;
    SmallDesc* d_small = nullptr;
    std::vector<CholInvDesc> h_chol;
    CholInvDesc* d_chol = nullptr;
    std::vector<KrylovCheckDesc> h_kcheck;
    std::vector<TsqrDesc> h_tsqr;   // TSQR passes (r_factor = 1)
    TsqrDesc* d_tsqr = nullptr;
    KrylovCheckDesc* d_kcheck = nullptr;
    std::vector<Launch> launches;
    int64_t n_kernels = 0;            // kernel launches of one forward evaluation
    GemmDesc* d_gemm = nullptr;
    CopyDesc* d_copy = nullptr;
    CoreDesc* d_core = nullptr;
    ScaleDesc* d_scale = nullptr;
    InputDesc* d_inputs = nullptr;
    double* d_scales = nullptr;
    double* d_maxparts = nullptr;
    double* d_disc = nullptr;
    int32_t* d_tie = nullptr;
    int32_t* d_sweeps = nullptr;
    double* d_result = nullptr;
    double* h_result = nullptr;

    // reverse pass
    std::vector<GemmDesc> h_bgemm;
    std::vector<ReduceDesc> h_reduce;
    std::vector<CoreBwdDesc> h_cbwd;
    std::vector<InputDesc> h_gin;
    std::vector<Launch> blaunches;
    GemmDesc* d_bgemm = nullptr;
    ReduceDesc* d_reduce = nullptr;
    CoreBwdDesc* d_cbwd = nullptr;
    InputDesc* d_gin = nullptr;
    double* d_grad = nullptr;         // host-destined gradient staging (n_input float64)

    bool evaluated = false;
    // the forward arena holds what the last forward evaluation left there (no recomputation has
    // written over it since), so the reverse pass need not re-run the last segment
    bool fwd_fresh = false;
    double sign = 0, lnz = 0;
    int flags = 0;

    // per-kind launch timing with HIP events (tn_profile)
    uint32_t prof_mask = 0;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, size_t>> ev_used;   // (kind, index of the start event)
    double prof_ms[kKinds] = {0};
    int64_t prof_launches[kKinds] = {0};
    double prof_flops[kKinds] = {0}, prof_bytes[kKinds] = {0};

    // forward-pass timing: device stamps around each profiled launch (valid inside graphs)
    unsigned long long* d_stamps = nullptr;
    size_t stamps_cap = 0;                          // stamp pairs
    std::vector<std::pair<int, int>> st_used;       // (kind, stamp pair)
    // the forward schedule captured once per plan (and profiling mask) and replayed; the stamps and
    // counts that one evaluation adds to the profile, replayed with it
    hipGraph_t fgraph = nullptr;
    hipGraphExec_t fexec = nullptr;
    uint32_t fgraph_mask = 0;
    std::vector<std::pair<int, int>> fgraph_st;
    int64_t fgraph_launches[kKinds] = {0};
    double fgraph_flops[kKinds] = {0}, fgraph_bytes[kKinds] = {0};
};

namespace {

// GEMM instantiation for tensor operands (contractions, re-absorptions, adjoints) and for
// Gram / float64-partial outputs, by tensor precision (0 float64, 1 float32, 2 bfloat16).
int tensor_key(int prec) { return prec == 0 ? GEMM_F64 : prec == 1 ? GEMM_F32 : GEMM_BF16; }
int wide_key(int prec) { return prec == 0 ? GEMM_F64 : prec == 1 ? GEMM_F32_TO_F64 : GEMM_BF16_TO_F64; }
int narrow_gram_key(int prec) {
    return prec == 0 ? GEMM_GRAM_NARROW_F64 : prec == 1 ? GEMM_GRAM_NARROW_F32 : GEMM_GRAM_NARROW_BF16;
}

tn_status fail(tn_ctx* c, tn_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

#define HIP_TRY(ctx, expr)                                                                        \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(ctx, TN_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)

template <typename T>
void dfree(T*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

void free_forward_graph(tn_ctx* c) {
    if (c->fexec) (void)hipGraphExecDestroy(c->fexec);
    if (c->fgraph) (void)hipGraphDestroy(c->fgraph);
    c->fexec = nullptr;
    c->fgraph = nullptr;
    c->fgraph_st.clear();
}

void free_plan(tn_ctx* c) {
    free_forward_graph(c);
    if (c->arena_owned) dfree(c->arena);
    c->arena = nullptr;
    c->arena_owned = true;
    c->arena_cap = 0;
    dfree(c->d_gemm);
    dfree(c->d_copy);
    dfree(c->d_core);
    dfree(c->d_scale);
    dfree(c->d_inputs);
    dfree(c->d_lanczos);
    dfree(c->d_glanczos);
    dfree(c->d_small);
    dfree(c->d_chol);
    dfree(c->d_kcheck);
    c->h_kcheck.clear();
    dfree(c->d_tsqr);
    c->h_tsqr.clear();
    c->h_kops.clear();
    c->h_small.clear();
    c->h_chol.clear();
    dfree(c->d_scales);
    dfree(c->d_maxparts);
    dfree(c->d_disc);
    dfree(c->d_tie);
    dfree(c->d_sweeps);
    dfree(c->d_bgemm);
    dfree(c->d_reduce);
    dfree(c->d_cbwd);
    dfree(c->d_gin);
    dfree(c->d_grad);
    c->h_bgemm.clear();
    c->h_reduce.clear();
    c->h_cbwd.clear();
    c->h_gin.clear();
    c->blaunches.clear();
    c->h_gemm.clear();
    c->h_copy.clear();
    c->h_core.clear();
    c->h_scale.clear();
    c->h_inputs.clear();
    c->h_lanczos.clear();
    c->h_glanczos.clear();
    c->launches.clear();
    c->has_plan = false;
    c->evaluated = false;
}

template <typename T>
tn_status upload(tn_ctx* c, T** dst, const std::vector<T>& src) {
    dfree(*dst);
    if (src.empty()) return TN_OK;
    HIP_TRY(c, hipMalloc((void**)dst, src.size() * sizeof(T)));
    HIP_TRY(c, hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return TN_OK;
}

std::string fill_view(const ViewSpec& s, View* v) { return make_view(s, v); }

// Turn the plan's levelled steps into grouped launch descriptors.
// Within a level, the one-workgroup compression kernels are issued before the many-workgroup
// GEMMs: they need a whole compute unit each, which a GEMM launch issued first would occupy
// until its workgroups drain.  Stable: the order inside each stream is kept.
void order_for_issue(std::vector<Launch>& ls) {
    auto first = [](const Launch& l) {
        return l.kind == L_CORE || l.kind == L_LANCZOS || l.kind == L_GLANCZOS || l.kind == L_KRYLOV;
    };
    std::stable_sort(ls.begin(), ls.end(), [&](const Launch& a, const Launch& b) {
        if (a.level != b.level) return a.level < b.level;
        return first(a) && !first(b);
    });
}

tn_status build_launches(tn_ctx* c) {
    Plan& P = c->plan;
    const int prec = P.opts.precision;
    char* base = c->arena;
    auto buf_ptr = [&](int32_t b) -> char* { return base + P.bufs[b].off; };
    auto ten_ptr = [&](int32_t t) -> char* { return buf_ptr(P.tens[t].buf); };

    std::vector<std::vector<int32_t>> by_level(P.n_levels + 1);
    for (int32_t s = 0; s < (int32_t)P.steps.size(); ++s) by_level[P.steps[s].level].push_back(s);
    int64_t max_parts = 1;
    for (int L = 1; L <= P.n_levels; ++L) {
        std::map<int, std::vector<GemmDesc>> gemms;   // 2*dtype key + is_gram -> descs
        std::map<int, std::pair<double, double>> gemm_work;
        std::pair<double, double> copy_work{0, 0}, core_work[2] = {{0, 0}, {0, 0}};
        std::vector<CopyDesc> copies;
        std::vector<CoreDesc> cores_lds, cores_glb;
        std::vector<LanczosDesc> lanczos;
        std::vector<GLanczosDesc> glanczos;
        std::pair<double, double> glanczos_work{0, 0};
        std::vector<int32_t> krylov_steps;
        std::pair<double, double> krylov_work{0, 0};
        std::pair<double, double> lanczos_work{0, 0};
        int lanczos_smax = 1;
        std::vector<ScaleDesc> scales;
        std::vector<ReduceDesc> sums;
        std::vector<GemmDesc> spre[2];
        std::vector<std::vector<TsqrDesc>> tsqr_pass;   // per pass, over the level's TSQR steps
        std::pair<double, double> tsqr_work{0, 0};
        int64_t parts = 0;
        if (L < P.n_levels) {
            // Gram-Lanczos cores of the next level: their operator S = F_X G_Y F_X^T (or C1 C1^T,
            // C1 = F_X F_Y^T) is formed here, on the stream that wrote the side factors, after them
            for (int32_t si : by_level[L + 1]) {
                const Step& st = P.steps[si];
                if (st.kind != ST_CORE || !P.comps[st.comp].glanczos) continue;
                const Compression& cp = P.comps[st.comp];
                const int xb = cp.x_is_b;
                const int ygram = xb ? cp.gram_a : cp.gram_b;
                const double* fx = (const double*)buf_ptr(xb ? cp.side_b_buf : cp.side_a_buf);
                const double* y = (const double*)buf_ptr(xb ? cp.side_a_buf : cp.side_b_buf);
                const int64_t n = xb ? cp.mb : cp.ma, my = xb ? cp.ma : cp.mb, D = cp.D;
                double* S = (double*)buf_ptr(cp.work_buf);
                double* T1 = S + n * n;
                auto dense = [&](int64_t rows, int64_t rs, int64_t cols, int64_t cs, View* v) {
                    ViewSpec vs;
                    vs.row_dims = {(int32_t)rows};
                    vs.row_strides = {rs};
                    vs.col_dims = {(int32_t)cols};
                    vs.col_strides = {cs};
                    return make_view(vs, v);
                };
                auto product = [&](const double* A, int64_t M, int64_t K, int64_t ar, int64_t ac, const double* B,
                                   int64_t N, int64_t br, int64_t bc, double* C, GemmDesc* g) {
                    std::memset(g, 0, sizeof(*g));
                    std::string e = dense(M, ar, K, ac, &g->va);
                    if (e.empty()) e = dense(K, br, N, bc, &g->vb);
                    g->A = A;
                    g->B = B;
                    g->C = C;
                    g->M = (int32_t)M;
                    g->N = (int32_t)N;
                    g->K = (int32_t)K;
                    g->mode = GEMM_GRAM;
                    g->tiles_m = (int32_t)((M + 63) / 64);
                    g->tiles_n = (int32_t)((N + 63) / 64);
                    g->splits = 1;
                    g->k_per_split = (int32_t)K;
                    g->scale_a = g->scale_b = -1;
                    return e;
                };
                GemmDesc g1, g2;
                std::string err;
                if (ygram) {   // T1 = G_Y F_X^T (D x n), S = F_X T1
                    err = product(y, D, D, D, 1, fx, n, 1, D, T1, &g1);
                    if (err.empty()) err = product(fx, n, D, D, 1, T1, n, n, 1, S, &g2);
                } else {       // T1 = F_X F_Y^T (n x my), S = T1 T1^T
                    err = product(fx, n, D, D, 1, y, my, 1, D, T1, &g1);
                    if (err.empty()) err = product(T1, n, my, my, 1, T1, n, 1, my, S, &g2);
                }
                if (!err.empty()) return fail(c, TN_EINVAL, err);
                spre[0].push_back(g1);
                spre[1].push_back(g2);
            }
        }
        for (int32_t si : by_level[L]) {
            const Step& st = P.steps[si];
            if (st.kind == ST_CONTRACT || st.kind == ST_ABSORB || st.kind == ST_GRAM) {
                GemmDesc g;
                std::memset(&g, 0, sizeof(g));
                std::string err = fill_view(st.va, &g.va);
                if (err.empty()) err = fill_view(st.vb, &g.vb);
                if (!err.empty()) return fail(c, TN_EINVAL, err);
                g.M = (int32_t)st.M;
                g.N = (int32_t)st.N;
                g.K = (int32_t)st.K;
                g.tiles_m = (int32_t)((st.M + 63) / 64);
                g.tiles_n = (int32_t)((st.N + 63) / 64);
                g.scale_a = g.scale_b = -1;
                int key;
                if (st.kind == ST_GRAM) {
                    g.mode = GEMM_GRAM;
                    g.A = ten_ptr(st.in_a);
                    g.B = ten_ptr(st.in_a);
                    g.C = buf_ptr(st.out_buf);
                    g.splits = st.splits;
                    g.k_per_split = st.k_per_split;
                    g.scale_a = st.in_a;
                    g.square_a = 1;
                    key = 2 * (st.M <= kGramNarrowMaxD ? narrow_gram_key(prec) : wide_key(prec)) + 1;
                    if (st.splits > 1) {
                        // the split partials are summed in place right after the level's Gram
                        // GEMMs (same stream, many workgroups), so readers see one matrix
                        ReduceDesc r;
                        std::memset(&r, 0, sizeof(r));
                        ViewSpec vs;
                        vs.row_dims = {(int32_t)st.M};
                        vs.row_strides = {st.N};
                        vs.col_dims = {(int32_t)st.N};
                        vs.col_strides = {1};
                        std::string verr = make_view(vs, &r.vc);
                        if (!verr.empty()) return fail(c, TN_EINVAL, verr);
                        r.part = (const double*)g.C;
                        r.out = g.C;
                        r.M = (int32_t)st.M;
                        r.N = (int32_t)st.N;
                        r.splits = st.splits;
                        r.scale_a = r.scale_b = -1;
                        sums.push_back(r);
                    }
                } else {
                    g.mode = GEMM_TENSOR;
                    g.splits = 1;
                    g.k_per_split = (int32_t)st.K;
                    if (st.kind == ST_CONTRACT) {
                        g.A = ten_ptr(st.in_a);
                        g.B = ten_ptr(st.in_b);
                        g.scale_a = st.in_a;
                        g.scale_b = st.in_b;
                    } else if (st.proj_left) {
                        g.A = ten_ptr(st.in_a);
                        g.B = buf_ptr(st.proj_buf);
                        g.scale_a = st.in_a;
                    } else {
                        g.A = buf_ptr(st.proj_buf);
                        g.B = ten_ptr(st.in_a);
                        g.scale_b = st.in_a;
                    }
                    g.C = ten_ptr(st.out_t);
                    // tile shape by the GEMM's short side (per-tile maxima follow the tiling)
                    const int variant = pick_gemm_tile(prec, st.M, st.N, st.K, g.va.row_unit != 0, g.vb.col_unit != 0);
                    int bm = 64, bn = 64;
                    gemm_tile(variant, &bm, &bn);
                    g.tiles_m = (int32_t)((st.M + bm - 1) / bm);
                    g.tiles_n = (int32_t)((st.N + bn - 1) / bn);
                    g.maxpart = (int32_t)parts;
                    ScaleDesc sd{};
                    sd.maxpart = (int32_t)parts;
                    sd.nparts = g.tiles_m * g.tiles_n;
                    sd.tensor = st.out_t;
                    scales.push_back(sd);
                    parts += sd.nparts;
                    key = 2 * (tensor_key(prec) + kGemmVariantStride * variant);
                }
                gemms[key].push_back(g);
                gemm_work[key].first += st.flops;
                gemm_work[key].second += st.bytes;
            } else if (st.kind == ST_GAUGE) {
                // tree gauge: a metric applied on one bond (output through the tensor's layout), or a
                // metric-weighted Gram (split partials summed in place, as for the side Grams)
                GemmDesc g;
                std::memset(&g, 0, sizeof(g));
                const bool apply = st.gauge_mode == GAUGE_APPLY;
                std::string err = fill_view(st.va, &g.va);
                if (err.empty()) err = fill_view(st.vb, &g.vb);
                if (err.empty() && apply) err = fill_view(st.vc, &g.vc);
                if (!err.empty()) return fail(c, TN_EINVAL, err);
                g.M = (int32_t)st.M;
                g.N = (int32_t)st.N;
                g.K = (int32_t)st.K;
                g.tiles_m = (int32_t)((st.M + 63) / 64);
                g.tiles_n = (int32_t)((st.N + 63) / 64);
                g.A = st.in_a >= 0 ? ten_ptr(st.in_a) : buf_ptr(st.a_buf);
                g.B = buf_ptr(st.b_buf);
                g.C = buf_ptr(st.out_buf);
                g.scale_a = st.in_a >= 0 ? st.in_a : -1;   // the tensor's pending 1/s (a buffer has it applied)
                g.scale_b = -1;
                // the tensor operand in its storage precision against a float64 one
                const int k0 = st.in_a < 0 || prec == 0 ? GEMM_F64 : prec == 1 ? GEMM_F32_X_F64 : GEMM_BF16_X_F64;
                int key;
                if (apply) {
                    g.mode = GEMM_ADJ;
                    g.splits = 1;
                    g.k_per_split = (int32_t)st.K;
                    key = 2 * k0;
                } else {
                    g.mode = GEMM_GRAM;
                    g.splits = st.splits;
                    g.k_per_split = st.k_per_split;
                    key = 2 * k0 + 1;
                    if (st.splits > 1) {
                        ReduceDesc r;
                        std::memset(&r, 0, sizeof(r));
                        ViewSpec vs;
                        vs.row_dims = {(int32_t)st.M};
                        vs.row_strides = {st.N};
                        vs.col_dims = {(int32_t)st.N};
                        vs.col_strides = {1};
                        std::string verr = make_view(vs, &r.vc);
                        if (!verr.empty()) return fail(c, TN_EINVAL, verr);
                        r.part = (const double*)g.C;
                        r.out = g.C;
                        r.M = (int32_t)st.M;
                        r.N = (int32_t)st.N;
                        r.splits = st.splits;
                        r.scale_a = r.scale_b = -1;
                        sums.push_back(r);
                    }
                }
                gemms[key].push_back(g);
                gemm_work[key].first += st.flops;
                gemm_work[key].second += st.bytes;
            } else if (st.kind == ST_COPY) {
                CopyDesc cd;
                std::memset(&cd, 0, sizeof(cd));
                std::string err = fill_view(st.va, &cd.v);
                if (!err.empty()) return fail(c, TN_EINVAL, err);
                cd.src = ten_ptr(st.in_a);
                cd.dst = (double*)buf_ptr(st.out_buf);
                cd.rows = st.copy_rows;
                cd.cols = st.copy_cols;
                cd.scale = st.in_a;
                copies.push_back(cd);
                copy_work.first += st.flops;
                copy_work.second += st.bytes;
            } else if (st.kind == ST_LANCZOS) {
                const Compression& cp = P.comps[st.comp];
                LanczosDesc ld;
                std::memset(&ld, 0, sizeof(ld));
                std::string err = fill_view(st.va, &ld.va);
                if (err.empty()) err = fill_view(st.vb, &ld.vb);
                if (!err.empty()) return fail(c, TN_EINVAL, err);
                ld.A = ten_ptr(st.in_a);
                ld.B = ten_ptr(st.in_b);
                ld.work = (double*)buf_ptr(cp.work_buf);
                ld.p_left = buf_ptr(cp.pl_buf);
                ld.p_right = buf_ptr(cp.pr_buf);
                ld.cutoff = P.opts.cutoff;
                ld.ma = (int32_t)cp.ma;
                ld.mb = (int32_t)cp.mb;
                ld.D = (int32_t)cp.D;
                ld.chi_new = cp.chi_new;
                ld.s_min = cp.s_min;
                ld.s_max = cp.s_max;
                ld.scale_a = st.in_a;
                ld.scale_b = st.in_b;
                ld.stat = st.comp;
                ld.kmin = (int32_t)std::min(std::min(cp.ma, cp.D), std::min(cp.mb, cp.D));
                ld.gram_a = (const double*)buf_ptr(cp.side_a_buf);
                ld.gram_b = (const double*)buf_ptr(cp.side_b_buf);
                lanczos_smax = std::max(lanczos_smax, cp.s_max);
                lanczos.push_back(ld);
                lanczos_work.first += st.flops;
                lanczos_work.second += st.bytes;
            } else if (st.kind == ST_TSQR) {
                int64_t rows = st.K;
                for (size_t p = 0; p < st.tsqr_bufs.size(); ++p) {
                    TsqrDesc td;
                    std::memset(&td, 0, sizeof(td));
                    std::string err;
                    if (p == 0) {
                        err = fill_view(st.va, &td.v);
                        td.src = ten_ptr(st.in_a);
                        td.scale = st.in_a;
                    } else {
                        // the previous pass's stacked R's: (nb D) x D, row-major
                        ViewSpec vs;
                        vs.row_dims = {(int32_t)rows};
                        vs.row_strides = {st.M};
                        vs.col_dims = {(int32_t)st.M};
                        vs.col_strides = {1};
                        err = make_view(vs, &td.v);
                        td.src = buf_ptr(st.tsqr_bufs[p - 1]);
                        td.scale = -1;
                    }
                    if (!err.empty()) return fail(c, TN_EINVAL, err);
                    td.dst = (double*)buf_ptr(st.tsqr_bufs[p]);
                    td.rows = (int32_t)rows;
                    td.D = (int32_t)st.M;
                    td.nblk = st.tsqr_blocks[p];
                    if (tsqr_pass.size() <= p) tsqr_pass.resize(p + 1);
                    tsqr_pass[p].push_back(td);
                    rows = (int64_t)st.tsqr_blocks[p] * st.M;
                }
                tsqr_work.first += st.flops;
                tsqr_work.second += st.bytes;
            } else if (st.kind == ST_KRYLOV) {
                krylov_steps.push_back(si);
                krylov_work.first += st.flops;
                krylov_work.second += st.bytes;
            } else if (st.kind == ST_CORE && P.comps[st.comp].glanczos) {
                const Compression& cp = P.comps[st.comp];
                GLanczosDesc gd;
                std::memset(&gd, 0, sizeof(gd));
                const int xb = cp.x_is_b;
                const int32_t xbuf = xb ? cp.side_b_buf : cp.side_a_buf;
                const int32_t ybuf = xb ? cp.side_a_buf : cp.side_b_buf;
                const int ygram = xb ? cp.gram_a : cp.gram_b;
                gd.fx = (const double*)buf_ptr(xbuf);
                gd.gram_y = ygram ? (const double*)buf_ptr(ybuf) : nullptr;
                gd.fy = ygram ? nullptr : (const double*)buf_ptr(ybuf);
                gd.splits_y = 1;   // the Gram partials were summed in place
                gd.work = (double*)buf_ptr(cp.work_buf);
                gd.p_left = buf_ptr(cp.pl_buf);
                gd.p_right = buf_ptr(cp.pr_buf);
                gd.cutoff = P.opts.cutoff;
                gd.n = (int32_t)(xb ? cp.mb : cp.ma);
                gd.my = (int32_t)(xb ? cp.ma : cp.mb);
                gd.D = (int32_t)cp.D;
                gd.chi_new = cp.chi_new;
                gd.x_is_b = xb;
                gd.s_min = cp.s_min;
                gd.s_max = cp.s_max;
                gd.stat = st.comp;
                gd.kmin = (int32_t)std::min(std::min(cp.ma, cp.D), std::min(cp.mb, cp.D));
                glanczos.push_back(gd);
                glanczos_work.first += st.flops;
                glanczos_work.second += st.bytes;
            } else if (st.kind == ST_CORE) {
                const Compression& cp = P.comps[st.comp];
                CoreDesc cd;
                std::memset(&cd, 0, sizeof(cd));
                cd.gram_a = cp.gram_a ? (const double*)buf_ptr(cp.side_a_buf) : nullptr;
                cd.fac_a = cp.gram_a ? nullptr : (const double*)buf_ptr(cp.side_a_buf);
                cd.gram_b = cp.gram_b ? (const double*)buf_ptr(cp.side_b_buf) : nullptr;
                cd.fac_b = cp.gram_b ? nullptr : (const double*)buf_ptr(cp.side_b_buf);
                cd.splits_a = 1;   // the Gram partials were summed in place
                cd.splits_b = 1;
                cd.rows_a = cp.rows_a;
                cd.rows_b = cp.rows_b;
                cd.D = (int32_t)cp.D;
                cd.chi_new = cp.chi_new;
                cd.cutoff = P.opts.cutoff;
                cd.work = (double*)buf_ptr(cp.work_buf);
                cd.p_left = buf_ptr(cp.pl_buf);
                cd.p_right = buf_ptr(cp.pr_buf);
                cd.stat = st.comp;
                cd.kmin = (int32_t)std::min(std::min(cp.ma, cp.D), std::min(cp.mb, cp.D));
                cd.keep_out = P.opts.grad ? 1 : 0;
                (cp.D <= kCoreLdsMaxD ? cores_lds : cores_glb).push_back(cd);
                auto& cw = core_work[cp.D <= kCoreLdsMaxD ? 0 : 1];
                cw.first += st.flops;
                cw.second += st.bytes;
            }
        }
        max_parts = std::max(max_parts, parts);
        for (auto& kv : gemms) {
            Launch l;
            l.level = L;
            l.kind = L_GEMM;
            l.key = kv.first / 2;
            l.prof = (kv.first & 1) ? TN_KERNEL_GRAM : TN_KERNEL_GEMM;
            l.flops = gemm_work[kv.first].first;
            l.bytes = gemm_work[kv.first].second;
            l.begin = (int64_t)c->h_gemm.size();
            l.count = (int)kv.second.size();
            int64_t tiles = 0;
            for (auto& g : kv.second) {
                g.tile_begin = tiles;
                tiles += (int64_t)g.tiles_m * g.tiles_n * g.splits;
                c->h_gemm.push_back(g);
            }
            l.work = tiles;
            c->launches.push_back(l);
        }
        if (!sums.empty()) {
            Launch l;
            l.level = L;
            l.kind = L_REDUCE;
            l.key = 0;   // float64
            l.prof = TN_KERNEL_GRAM;
            l.begin = (int64_t)c->h_reduce.size();
            l.count = (int)sums.size();
            int64_t elems = 0;
            for (auto& r : sums) {
                r.elem_begin = elems;
                elems += (int64_t)r.M * r.N;
                c->h_reduce.push_back(r);
            }
            l.work = elems;
            c->launches.push_back(l);
        }
        for (size_t p = 0; p < tsqr_pass.size(); ++p) {
            // passes in order on one stream (the Gram lane); the first reads the tensors
            Launch l;
            l.level = L;
            l.kind = L_TSQR;
            l.key = p == 0 ? prec : 0;
            l.prof = TN_KERNEL_GRAM;
            if (p == 0) {
                l.flops = tsqr_work.first;
                l.bytes = tsqr_work.second;
            }
            l.begin = (int64_t)c->h_tsqr.size();
            l.count = (int)tsqr_pass[p].size();
            int64_t blocks = 0;
            for (auto& td : tsqr_pass[p]) {
                td.blk_begin = blocks;
                blocks += td.nblk;
                c->h_tsqr.push_back(td);
            }
            l.work = blocks;
            c->launches.push_back(l);
        }
        if (!copies.empty()) {
            Launch l;
            l.level = L;
            l.kind = L_COPY;
            l.key = prec;
            l.prof = TN_KERNEL_COPY;
            l.flops = copy_work.first;
            l.bytes = copy_work.second;
            l.begin = (int64_t)c->h_copy.size();
            l.count = (int)copies.size();
            int64_t elems = 0;
            for (auto& cd : copies) {
                cd.elem_begin = elems;
                elems += (int64_t)cd.rows * cd.cols;
                c->h_copy.push_back(cd);
            }
            l.work = elems;
            c->launches.push_back(l);
        }
        for (int stage = 0; stage < 2; ++stage) {
            if (spre[stage].empty()) continue;
            Launch l;
            l.level = L;
            l.kind = L_SPRE;
            l.key = stage;
            l.prof = TN_KERNEL_LANCZOS;   // part of the Lanczos compressions' cost
            l.begin = (int64_t)c->h_gemm.size();
            l.count = (int)spre[stage].size();
            int64_t tiles = 0;
            for (auto& g : spre[stage]) {
                g.tile_begin = tiles;
                tiles += (int64_t)g.tiles_m * g.tiles_n;
                c->h_gemm.push_back(g);
            }
            l.work = tiles;
            c->launches.push_back(l);
        }
        for (int pass = 0; pass < 2; ++pass) {
            auto& v = pass == 0 ? cores_lds : cores_glb;
            if (v.empty()) continue;
            Launch l;
            l.level = L;
            l.kind = L_CORE;
            l.key = pass == 0 ? 1 : 0;
            l.prof = pass == 0 ? TN_KERNEL_CORE_LDS : TN_KERNEL_CORE_GLOBAL;
            l.flops = core_work[pass].first;
            l.bytes = core_work[pass].second;
            l.begin = (int64_t)c->h_core.size();
            l.count = (int)v.size();
            for (auto& cd : v) {
                l.max_d = std::max(l.max_d, cd.D);
                c->h_core.push_back(cd);
            }
            c->launches.push_back(l);
        }
        if (!lanczos.empty()) {
            Launch l;
            l.level = L;
            l.kind = L_LANCZOS;
            l.key = prec;
            l.prof = TN_KERNEL_LANCZOS;
            l.begin = (int64_t)c->h_lanczos.size();
            l.count = (int)lanczos.size();
            l.max_d = lanczos_smax;
            l.flops = lanczos_work.first;
            l.bytes = lanczos_work.second;
            for (auto& ld : lanczos) c->h_lanczos.push_back(ld);
            c->launches.push_back(l);
        }
        if (!glanczos.empty()) {
            Launch l;
            l.level = L;
            l.kind = L_GLANCZOS;
            l.key = prec;
            l.prof = TN_KERNEL_LANCZOS;
            l.begin = (int64_t)c->h_glanczos.size();
            l.count = (int)glanczos.size();
            l.flops = glanczos_work.first;
            l.bytes = glanczos_work.second;
            for (auto& gd : glanczos) c->h_glanczos.push_back(gd);
            c->launches.push_back(l);
        }
        if (!krylov_steps.empty()) {
            // one chain per group of same-shape compressions (per compression in the plain form)
            std::map<std::vector<int64_t>, std::vector<KrylovJob>> groups;
            std::map<std::vector<int64_t>, KrylovShape> shapes;
            for (int32_t si : krylov_steps) {
                const Step& st = P.steps[si];
                const Compression& cp = P.comps[st.comp];
                KrylovShape sh;
                sh.n = cp.kr_n;
                sh.D = cp.D;
                sh.my = cp.kr_my;
                sh.nw = cp.chi_new;
                sh.b = cp.kr_b;
                sh.s = cp.kr_s;
                sh.k = cp.kr_k;
                sh.full = cp.kr_full;
                sh.splits = cp.kr_splits;
                sh.splits2 = cp.kr_splits2;
                KrylovJob job;
                std::string err = fill_view(st.va, &job.vy);
                if (err.empty()) err = fill_view(st.vb, &job.vyt);
                if (!err.empty()) return fail(c, TN_EINVAL, err);
                job.fx = (const double*)buf_ptr(cp.x_is_b ? cp.side_b_buf : cp.side_a_buf);
                job.y = ten_ptr(st.in_a);
                job.y_scale = st.in_a;
                job.ws = buf_ptr(cp.work_buf);
                job.p_left = buf_ptr(cp.pl_buf);
                job.p_right = buf_ptr(cp.pr_buf);
                job.x_is_b = cp.x_is_b;
                job.stat = st.comp;
                job.kmin = (int32_t)std::min(std::min(cp.ma, cp.D), std::min(cp.mb, cp.D));
                job.cutoff = P.opts.cutoff;
                std::vector<int64_t> key = {sh.n, sh.D, sh.my, sh.nw, sh.b, sh.s, sh.k, sh.full, sh.splits, sh.splits2};
                if (P.opts.plain) key.push_back(si);
                groups[key].push_back(job);
                shapes[key] = sh;
            }
            Launch l;
            l.level = L;
            l.kind = L_KRYLOV;
            l.prof = TN_KERNEL_LANCZOS;
            l.flops = krylov_work.first;
            l.bytes = krylov_work.second;
            l.begin = (int64_t)c->h_kops.size();
            KrylovSink sink{&c->h_gemm, &c->h_reduce, &c->h_small, &c->h_chol, &c->h_core, &c->h_kcheck, &c->h_kops};
            for (auto& kv : groups) {
                std::string err = krylov_chain(shapes[kv.first], prec, kv.second, sink);
                if (!err.empty()) return fail(c, TN_EINVAL, "block-Krylov chain: " + err);
            }
            l.count = (int)((int64_t)c->h_kops.size() - l.begin);
            c->launches.push_back(l);
        }
        if (!scales.empty()) {
            Launch l;
            l.level = L;
            l.kind = L_SCALE;
            l.prof = TN_KERNEL_SCALE;
            l.begin = (int64_t)c->h_scale.size();
            l.count = (int)scales.size();
            for (auto& sd : scales) c->h_scale.push_back(sd);
            c->launches.push_back(l);
        }
    }
    if (P.opts.plain) {
        // the plain form: every step of a level is its own launch (one descriptor each), issued in
        // order on one stream without graph capture, the way a host loop would run the ops
        std::vector<Launch> split;
        for (const Launch& l : c->launches) {
            for (int i = 0; i < l.count; ++i) {
                Launch x = l;
                x.begin = l.begin + i;
                x.count = 1;
                x.flops = l.flops / l.count;
                x.bytes = l.bytes / l.count;
                switch (l.kind) {
                    case L_GEMM:
                    case L_SPRE: {
                        GemmDesc& g = c->h_gemm[x.begin];
                        g.tile_begin = 0;
                        x.work = (int64_t)g.tiles_m * g.tiles_n * g.splits;
                        break;
                    }
                    case L_REDUCE: {
                        ReduceDesc& r = c->h_reduce[x.begin];
                        r.elem_begin = 0;
                        x.work = (int64_t)r.M * r.N;
                        break;
                    }
                    case L_COPY: {
                        CopyDesc& cd = c->h_copy[x.begin];
                        cd.elem_begin = 0;
                        x.work = (int64_t)cd.rows * cd.cols;
                        break;
                    }
                    case L_CORE: x.max_d = c->h_core[x.begin].D; break;
                    case L_LANCZOS: x.max_d = c->h_lanczos[x.begin].s_max; break;
                    case L_TSQR: {
                        TsqrDesc& td = c->h_tsqr[x.begin];
                        td.blk_begin = 0;
                        x.work = td.nblk;
                        break;
                    }
                    default: break;
                }
                split.push_back(x);
            }
        }
        c->launches.swap(split);
    }
    // inputs
    for (int v = 0; v < c->g.n; ++v) {
        InputDesc d{};
        d.dst = ten_ptr(v);
        d.src_off = c->g.offsets[v];
        d.count = c->g.offsets[v + 1] - c->g.offsets[v];
        d.tensor = v;
        c->h_inputs.push_back(d);
    }
    tn_status s;
    if ((s = upload(c, &c->d_gemm, c->h_gemm)) != TN_OK) return s;
    if ((s = upload(c, &c->d_copy, c->h_copy)) != TN_OK) return s;
    if ((s = upload(c, &c->d_core, c->h_core)) != TN_OK) return s;
    if ((s = upload(c, &c->d_scale, c->h_scale)) != TN_OK) return s;
    if ((s = upload(c, &c->d_inputs, c->h_inputs)) != TN_OK) return s;
    if ((s = upload(c, &c->d_lanczos, c->h_lanczos)) != TN_OK) return s;
    if ((s = upload(c, &c->d_glanczos, c->h_glanczos)) != TN_OK) return s;
    if ((s = upload(c, &c->d_reduce, c->h_reduce)) != TN_OK) return s;
    if ((s = upload(c, &c->d_small, c->h_small)) != TN_OK) return s;
    if ((s = upload(c, &c->d_chol, c->h_chol)) != TN_OK) return s;
    if ((s = upload(c, &c->d_kcheck, c->h_kcheck)) != TN_OK) return s;
    if ((s = upload(c, &c->d_tsqr, c->h_tsqr)) != TN_OK) return s;
    HIP_TRY(c, hipMalloc((void**)&c->d_scales, std::max<size_t>(1, P.tens.size()) * sizeof(double)));
    HIP_TRY(c, hipMalloc((void**)&c->d_maxparts, (size_t)max_parts * sizeof(double)));
    const size_t nc = std::max<size_t>(1, P.comps.size());
    HIP_TRY(c, hipMalloc((void**)&c->d_disc, nc * sizeof(double)));
    HIP_TRY(c, hipMalloc((void**)&c->d_tie, nc * sizeof(int32_t)));
    HIP_TRY(c, hipMalloc((void**)&c->d_sweeps, nc * sizeof(int32_t)));
    HIP_TRY(c, hipMemset(c->d_sweeps, 0, nc * sizeof(int32_t)));
    P.max_parts = max_parts;
    order_for_issue(c->launches);
    // kernel launches per evaluation (the capture budget)
    c->n_kernels = 2 + (int64_t)c->launches.size();
    for (const Launch& l : c->launches) {
        if (l.kind == L_CORE) c->n_kernels += core_launch_count(l.key, l.max_d, P.opts.jacobi_max_sweeps) - 1;
        if (l.kind == L_KRYLOV)
            for (int64_t i = l.begin; i < l.begin + l.count; ++i)
                c->n_kernels += c->h_kops[i].kind == KO_CORE
                                    ? core_launch_count(c->h_kops[i].key, c->h_kops[i].max_d, P.opts.jacobi_max_sweeps)
                                    : 1;
    }
    return TN_OK;
}

// Reverse-pass launches, grouped by level like the forward ones.
tn_status build_bwd_launches(tn_ctx* c) {
    Plan& P = c->plan;
    const int prec = P.opts.precision;
    char* base = c->arena;
    auto buf_ptr = [&](int32_t b) -> char* { return base + P.bufs[b].off; };
    std::vector<std::vector<int32_t>> by_level(P.n_blevels + 1);
    for (int32_t s = 0; s < (int32_t)P.bsteps.size(); ++s)
        if (P.bsteps[s].kind != BS_SEED) by_level[P.bsteps[s].level].push_back(s);
    for (int L = 1; L <= P.n_blevels; ++L) {
        std::map<int, std::vector<GemmDesc>> gemms;   // GemmKey -> descs
        std::map<int, std::pair<double, double>> gwork;
        std::vector<ReduceDesc> reds;
        std::vector<CoreBwdDesc> cores;
        double red_bytes = 0, core_flops = 0;
        for (int32_t si : by_level[L]) {
            const BStep& st = P.bsteps[si];
            if (st.kind == BS_GEMM) {
                GemmDesc g;
                std::memset(&g, 0, sizeof(g));
                std::string err = make_view(st.va, &g.va);
                if (err.empty()) err = make_view(st.vb, &g.vb);
                if (err.empty() && !st.partial) err = make_view(st.vc, &g.vc);
                if (!err.empty()) return fail(c, TN_EINVAL, err);
                g.A = buf_ptr(st.a_buf);
                g.B = buf_ptr(st.b_buf);
                g.C = buf_ptr(st.c_buf) + st.c_off;
                g.M = (int32_t)st.M;
                g.N = (int32_t)st.N;
                g.K = (int32_t)st.K;
                const int variant =
                    st.partial ? GV_64x64 : pick_gemm_tile(prec, st.M, st.N, st.K, g.va.row_unit != 0, g.vb.col_unit != 0);
                int bm = 64, bn = 64;
                gemm_tile(variant, &bm, &bn);
                g.tiles_m = (int32_t)((st.M + bm - 1) / bm);
                g.tiles_n = (int32_t)((st.N + bn - 1) / bn);
                g.splits = st.splits;
                g.k_per_split = st.k_per_split;
                g.scale_a = st.scale_a;
                g.scale_b = st.scale_b;
                g.accumulate = st.accumulate;
                g.mode = st.partial ? GEMM_GRAM : GEMM_ADJ;
                const int key = st.partial ? wide_key(prec) : tensor_key(prec) + kGemmVariantStride * variant;
                gemms[key].push_back(g);
                gwork[key].first += st.flops;
                gwork[key].second += st.bytes;
            } else if (st.kind == BS_REDUCE) {
                ReduceDesc r;
                std::memset(&r, 0, sizeof(r));
                std::string err = make_view(st.vc, &r.vc);
                if (!err.empty()) return fail(c, TN_EINVAL, err);
                r.part = (const double*)buf_ptr(st.a_buf);
                r.out = buf_ptr(st.c_buf);
                r.M = (int32_t)st.M;
                r.N = (int32_t)st.N;
                r.splits = st.splits;
                r.scale_a = st.scale_a;
                r.scale_b = st.scale_b;
                reds.push_back(r);
                red_bytes += st.bytes;
            } else if (st.kind == BS_CORE_BWD) {
                const Compression& cp = P.comps[st.comp];
                const CompBwd& cb = P.cbwd[st.comp];
                CoreBwdDesc d;
                std::memset(&d, 0, sizeof(d));
                d.work = (const double*)buf_ptr(cp.work_buf);
                d.h = (const double*)buf_ptr(cb.h_buf);
                d.ws = (double*)buf_ptr(cb.work_buf);
                d.n_a = buf_ptr(cb.na_buf);
                d.n_b = buf_ptr(cb.nb_buf);
                d.cutoff = P.opts.cutoff;
                d.splits_a = cb.splits_a;
                d.splits_b = cb.splits_b;
                d.D = (int32_t)cp.D;
                d.chi_new = cp.chi_new;
                cores.push_back(d);
                core_flops += st.flops;
            }
        }
        for (auto& kv : gemms) {
            Launch l;
            l.level = L;
            l.kind = L_GEMM;
            l.key = kv.first;
            l.prof = TN_KERNEL_BWD_GEMM;
            l.flops = gwork[kv.first].first;
            l.bytes = gwork[kv.first].second;
            l.begin = (int64_t)c->h_bgemm.size();
            l.count = (int)kv.second.size();
            int64_t tiles = 0;
            for (auto& g : kv.second) {
                g.tile_begin = tiles;
                tiles += (int64_t)g.tiles_m * g.tiles_n * g.splits;
                c->h_bgemm.push_back(g);
            }
            l.work = tiles;
            c->blaunches.push_back(l);
        }
        if (!reds.empty()) {
            Launch l;
            l.level = L;
            l.kind = L_REDUCE;
            l.key = prec;
            l.prof = TN_KERNEL_BWD_GEMM;
            l.bytes = red_bytes;
            l.begin = (int64_t)c->h_reduce.size();
            l.count = (int)reds.size();
            int64_t elems = 0;
            for (auto& r : reds) {
                r.elem_begin = elems;
                elems += (int64_t)r.M * r.N;
                c->h_reduce.push_back(r);
            }
            l.work = elems;
            c->blaunches.push_back(l);
        }
        if (!cores.empty()) {
            Launch l;
            l.level = L;
            l.kind = L_CORE_BWD;
            l.key = prec;
            l.prof = TN_KERNEL_BWD_CORE;
            l.flops = core_flops;
            l.begin = (int64_t)c->h_cbwd.size();
            l.count = (int)cores.size();
            for (auto& d : cores) {
                c->h_cbwd.push_back(d);
                l.max_d = std::max(l.max_d, (int)d.D);
            }
            c->blaunches.push_back(l);
        }
    }
    for (int v = 0; v < c->g.n; ++v) {
        InputDesc d{};
        d.dst = buf_ptr(P.adj_buf[v]);
        d.src_off = c->g.offsets[v];
        d.count = c->g.offsets[v + 1] - c->g.offsets[v];
        d.tensor = v;
        c->h_gin.push_back(d);
    }
    tn_status s;
    if ((s = upload(c, &c->d_bgemm, c->h_bgemm)) != TN_OK) return s;
    if ((s = upload(c, &c->d_reduce, c->h_reduce)) != TN_OK) return s;
    if ((s = upload(c, &c->d_cbwd, c->h_cbwd)) != TN_OK) return s;
    if ((s = upload(c, &c->d_gin, c->h_gin)) != TN_OK) return s;
    HIP_TRY(c, hipMalloc((void**)&c->d_grad, std::max<int64_t>(1, c->n_input_elems) * sizeof(double)));
    return TN_OK;
}

// Record HIP events around a launch of a profiled kind; returns the start-event slot or -1.
tn_status prof_begin(tn_ctx* c, const Launch& l, hipStream_t s, bool* timed) {
    *timed = (c->prof_mask >> l.prof) & 1u;
    if (!*timed) return TN_OK;
    const size_t i0 = c->ev_used.empty() ? 0 : c->ev_used.back().second + 2;
    while (c->ev_pool.size() < i0 + 2) {
        hipEvent_t e;
        HIP_TRY(c, hipEventCreate(&e));
        c->ev_pool.push_back(e);
    }
    HIP_TRY(c, hipEventRecord(c->ev_pool[i0], s));
    c->ev_used.push_back({l.prof, i0});
    c->prof_launches[l.prof] += 1;
    c->prof_flops[l.prof] += l.flops;
    c->prof_bytes[l.prof] += l.bytes;
    return TN_OK;
}

// Which stream of a level a launch runs on.  Launches of one level never depend on each other,
// except SCALE on the tensor GEMMs of its level, which share lane 0.
int lane_of(const Launch& l) {
    switch (l.kind) {
        case L_GEMM: return l.prof == TN_KERNEL_GRAM ? 3 : 0;
        case L_SCALE: return 0;
        case L_CORE: return 1;
        case L_LANCZOS:
        case L_GLANCZOS:
        case L_KRYLOV: return 2;
        default: return 3;
    }
}

// Enqueue launches [b, e) of one level: on `main` alone when they all share a lane, else forked
// onto the lanes' streams after an event on `main` and joined back with one event per lane.
// `run` enqueues one launch on a given stream.  `events` supplies timing-disabled events.
// The compression lanes (cores; Gram-Lanczos, unless a level holds other Lanczos launches) may be
// left unjoined (`allow_defer`): their events go to `pending`, and the next level makes `main`
// wait for them before its first tensor-GEMM launch (the re-absorptions that read the
// projectors) or, failing that, at its own join.  So a compression runs beside the next level's
// other compressions, Grams and copies; the planner keeps its inputs one level longer.
//
// `open` is a ledger of the lanes whose work `main` has not yet waited for (bit = lane): forks
// set bits, joins clear them, deferred joins keep them until the next level waits.  On a failed
// launch every forked lane is joined back before returning, so a capture can always be ended
// with no stream left forked; the caller checks the ledger is empty before ending a capture.
template <typename Run>
hipError_t run_level(const std::vector<Launch>& ls, size_t b, size_t e, hipStream_t main, hipStream_t* aux,
                     std::vector<hipEvent_t>& events, size_t& next_ev, Run&& run, hipEvent_t* pending,
                     bool allow_defer, int& open) {
    int used = 0;
    bool lane2_glanczos = true;
    for (size_t i = b; i < e; ++i) {
        used |= 1 << lane_of(ls[i]);
        if (lane_of(ls[i]) == 2 && ls[i].kind != L_GLANCZOS && ls[i].kind != L_KRYLOV) lane2_glanczos = false;
    }
    auto event = [&](hipEvent_t* out) -> hipError_t {
        if (next_ev == events.size()) {
            hipEvent_t ev;
            hipError_t err = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (err != hipSuccess) return err;
            events.push_back(ev);
        }
        *out = events[next_ev++];
        return hipSuccess;
    };
    auto wait_pending = [&]() -> hipError_t {
        for (int k = 0; k < 2; ++k)
            if (pending[k]) {
                hipError_t err = hipStreamWaitEvent(main, pending[k], 0);
                pending[k] = nullptr;
                if (err != hipSuccess) return err;
                open &= ~(1 << (k + 1));
            }
        return hipSuccess;
    };
    // failure inside a level: bring every lane with outstanding work back to `main` (best
    // effort: the first error is the one reported)
    auto join_all = [&](hipError_t first) -> hipError_t {
        for (int k = 0; k < 2; ++k)
            if (pending[k]) {
                (void)hipStreamWaitEvent(main, pending[k], 0);
                pending[k] = nullptr;
            }
        for (int lane = 1; lane < kLanes; ++lane)
            if (open & (1 << lane)) {
                hipEvent_t j = nullptr;
                if (event(&j) == hipSuccess && hipEventRecord(j, aux[lane - 1]) == hipSuccess &&
                    hipStreamWaitEvent(main, j, 0) == hipSuccess)
                    open &= ~(1 << lane);
            }
        return first;
    };
    hipError_t err = hipSuccess;
    if ((used & (used - 1)) == 0) {   // a single lane: no fork
        err = wait_pending();
        for (size_t i = b; i < e && err == hipSuccess; ++i) err = run(ls[i], main);
        return err == hipSuccess ? err : join_all(err);
    }
    hipEvent_t fork;
    err = event(&fork);
    if (err == hipSuccess) err = hipEventRecord(fork, main);
    for (int lane = 1; lane < kLanes && err == hipSuccess; ++lane)
        if (used & (1 << lane)) {
            err = hipStreamWaitEvent(aux[lane - 1], fork, 0);
            if (err == hipSuccess) open |= 1 << lane;
        }
    for (size_t i = b; i < e && err == hipSuccess; ++i) {
        const int lane = lane_of(ls[i]);
        if (lane == 0) err = wait_pending();   // the previous level's projectors
        if (err == hipSuccess) err = run(ls[i], lane == 0 ? main : aux[lane - 1]);
    }
    hipEvent_t deferred[2] = {nullptr, nullptr};
    for (int lane = 1; lane < kLanes && err == hipSuccess; ++lane)
        if (used & (1 << lane)) {
            hipEvent_t join;
            err = event(&join);
            if (err == hipSuccess) err = hipEventRecord(join, aux[lane - 1]);
            if (err != hipSuccess) break;
            const bool defer = allow_defer && (lane == 1 || (lane == 2 && lane2_glanczos));
            if (defer) {
                deferred[lane - 1] = join;
            } else {
                err = hipStreamWaitEvent(main, join, 0);
                if (err == hipSuccess) open &= ~(1 << lane);
            }
        }
    if (err == hipSuccess) err = wait_pending();   // never past one level
    if (err != hipSuccess) {
        for (int k = 0; k < 2; ++k)
            if (deferred[k] && !pending[k]) pending[k] = deferred[k];
        return join_all(err);
    }
    pending[0] = deferred[0];
    pending[1] = deferred[1];
    return err;
}

// Wait on `main` for the deferred joins of the last level and check the fork/join ledger.
template <typename Ctx, typename Fail>
tn_status join_tail(Ctx* x, hipStream_t main, hipEvent_t* pending, int& open, Fail&& failf) {
    for (int k = 0; k < 2; ++k)
        if (pending[k]) {
            hipError_t e = hipStreamWaitEvent(main, pending[k], 0);
            if (e != hipSuccess) return failf(x, TN_EDEVICE, std::string("join: ") + hipGetErrorString(e));
            pending[k] = nullptr;
            open &= ~(1 << (k + 1));
        }
    if (open != 0)
        return failf(x, TN_EDEVICE, "internal: a stream forked for a schedule level was never joined");
    return TN_OK;
}

}  // namespace

extern "C" {

tn_status tn_create(int device, void* hip_stream, tn_ctx** out) {
    if (!out) return TN_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return TN_EDEVICE;
    if (device < 0 || device >= n) return TN_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return TN_EDEVICE;
    tn_ctx* c = new tn_ctx();
    c->device = device;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return TN_EDEVICE;
        }
        c->own_stream = true;
    }
    if (hipHostMalloc((void**)&c->h_result, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void**)&c->d_result, 4 * sizeof(double)) != hipSuccess) {
        delete c;
        return TN_EDEVICE;
    }
    for (int i = 0; i < kLanes - 1; ++i)
        if (hipStreamCreateWithFlags(&c->aux[i], hipStreamNonBlocking) != hipSuccess) {
            tn_destroy(c);
            return TN_EDEVICE;
        }
    // the allocation-free entry point's scratch: its address on this device, looked up once
    if (!static_scratch_init(device).empty()) {
        tn_destroy(c);
        return TN_EDEVICE;
    }
    init_kernel_attrs();
    *out = c;
    return TN_OK;
}

void tn_destroy(tn_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_plan(c);
    dfree(c->d_staging);
    dfree(c->d_ising_i32);
    dfree(c->d_ising_off);
    dfree(c->d_result);
    dfree(c->d_stamps);
    if (c->h_result) (void)hipHostFree(c->h_result);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->sync_ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->rc_ev) (void)hipEventDestroy(e);
    for (hipStream_t a : c->aux)
        if (a) (void)hipStreamDestroy(a);
    delete c;
}

const char* tn_last_error(const tn_ctx* c) { return c ? c->err.c_str() : "null context"; }

tn_status tn_load_graph(tn_ctx* c, int32_t n_tensors, int32_t n_edges, const int32_t* edge_u, const int32_t* edge_v,
                        const int32_t* edge_dim, const int64_t* offsets, const double* data) {
    if (!c) return TN_EINVAL;
    if (n_tensors < 1 || n_edges < 0 || !offsets || !data || (n_edges > 0 && (!edge_u || !edge_v || !edge_dim)))
        return fail(c, TN_EINVAL, "missing graph arrays");
    (void)hipSetDevice(c->device);
    free_plan(c);
    GraphSpec g;
    g.n = n_tensors;
    g.ne = n_edges;
    g.eu.assign(edge_u, edge_u + n_edges);
    g.ev.assign(edge_v, edge_v + n_edges);
    g.ed.assign(edge_dim, edge_dim + n_edges);
    g.offsets.assign(offsets, offsets + n_tensors + 1);
    std::string err = check_graph(g);
    if (!err.empty()) {
        c->has_graph = false;
        return fail(c, TN_EINVAL, err);
    }
    c->g = g;
    c->has_graph = true;
    c->n_input_elems = g.offsets[n_tensors];
    dfree(c->d_staging);
    HIP_TRY(c, hipMalloc((void**)&c->d_staging, std::max<int64_t>(1, c->n_input_elems) * sizeof(double)));
    HIP_TRY(c, hipMemcpy(c->d_staging, data, c->n_input_elems * sizeof(double), hipMemcpyHostToDevice));
    // incidence lists for the Ising coupling map (only when every edge has dimension 2)
    dfree(c->d_ising_i32);
    dfree(c->d_ising_off);
    c->ising_ok = std::all_of(g.ed.begin(), g.ed.end(), [](int32_t d) { return d == 2; });
    if (c->ising_ok) {
        std::vector<std::vector<int32_t>> inc(g.n);
        for (int e = 0; e < g.ne; ++e) {
            inc[g.eu[e]].push_back(e);
            inc[g.ev[e]].push_back(e);
        }
        std::vector<int32_t> h;
        h.reserve(g.n + 1 + 4 * (size_t)g.ne);
        int32_t acc = 0;
        for (int v = 0; v < g.n; ++v) {
            h.push_back(acc);
            acc += (int32_t)inc[v].size();
        }
        h.push_back(acc);
        for (int v = 0; v < g.n; ++v) h.insert(h.end(), inc[v].begin(), inc[v].end());
        h.insert(h.end(), g.eu.begin(), g.eu.end());
        h.insert(h.end(), g.ev.begin(), g.ev.end());
        HIP_TRY(c, hipMalloc((void**)&c->d_ising_i32, h.size() * sizeof(int32_t)));
        HIP_TRY(c, hipMemcpy(c->d_ising_i32, h.data(), h.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        HIP_TRY(c, hipMalloc((void**)&c->d_ising_off, g.offsets.size() * sizeof(int64_t)));
        HIP_TRY(c, hipMemcpy(c->d_ising_off, g.offsets.data(), g.offsets.size() * sizeof(int64_t),
                             hipMemcpyHostToDevice));
        c->ising.inc_off = c->d_ising_i32;
        c->ising.inc_edge = c->d_ising_i32 + g.n + 1;
        c->ising.edge_u = c->ising.inc_edge + 2 * g.ne;
        c->ising.edge_v = c->ising.edge_u + g.ne;
        c->ising.data_off = c->d_ising_off;
        c->ising.n = g.n;
        c->ising.ne = g.ne;
    }
    return TN_OK;
}

tn_status tn_update_values(tn_ctx* c, const double* data) {
    if (!c) return TN_EINVAL;
    if (!c->has_graph) return fail(c, TN_ESTATE, "no graph loaded");
    if (!data) return fail(c, TN_EINVAL, "null data");
    (void)hipSetDevice(c->device);
    HIP_TRY(c, hipMemcpyAsync(c->d_staging, data, c->n_input_elems * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->evaluated = false;
    return TN_OK;
}

tn_status tn_update_values_device(tn_ctx* c, const void* dev_data) {
    if (!c) return TN_EINVAL;
    if (!c->has_graph) return fail(c, TN_ESTATE, "no graph loaded");
    if (!dev_data) return fail(c, TN_EINVAL, "null data");
    (void)hipSetDevice(c->device);
    HIP_TRY(c, hipMemcpyAsync(c->d_staging, dev_data, c->n_input_elems * sizeof(double), hipMemcpyDeviceToDevice,
                              c->stream));
    c->evaluated = false;
    return TN_OK;
}

tn_status tn_set_tree(tn_ctx* c, int32_t n_steps, const int32_t* pair_i, const int32_t* pair_j,
                      const tn_tree_opts* opts) {
    if (!c) return TN_EINVAL;
    if (!c->has_graph) return fail(c, TN_ESTATE, "tn_set_tree before tn_load_graph");
    if (!opts || (n_steps > 0 && (!pair_i || !pair_j))) return fail(c, TN_EINVAL, "missing tree arrays or options");
    if (opts->gauge_r < 0) return fail(c, TN_EINVAL, "gauge_r must be >= 0");
    if (opts->gauge_r > 0 && opts->grad) return fail(c, TN_EINVAL, "gauge_r >= 1 has no reverse pass (grad must be 0)");
    if (opts->compress_late != 0 && opts->compress_late != 1) return fail(c, TN_EINVAL, "compress_late must be 0 or 1");
    if (opts->checkpoint_segments < -1) return fail(c, TN_EINVAL, "checkpoint_segments must be >= -1");
    if (opts->r_factor != TN_RFACTOR_GRAM && opts->r_factor != TN_RFACTOR_TSQR)
        return fail(c, TN_EINVAL, "r_factor must be TN_RFACTOR_GRAM or TN_RFACTOR_TSQR");
    if (opts->r_factor == TN_RFACTOR_TSQR && opts->grad)
        return fail(c, TN_EINVAL, "r_factor TN_RFACTOR_TSQR has no reverse pass (grad must be 0)");
    if ((opts->checkpoint_segments > 1 || opts->checkpoint_segments == -1) && !opts->grad)
        return fail(c, TN_EINVAL, "checkpoint_segments is a reverse-pass option (grad must be 1)");
    if (opts->precision != TN_FP64 && opts->precision != TN_FP32 && opts->precision != TN_BF16)
        return fail(c, TN_EINVAL, "precision must be TN_FP64, TN_FP32 or TN_BF16");
    if (!(opts->cutoff >= 0.0)) return fail(c, TN_EINVAL, "cutoff must be >= 0");
    (void)hipSetDevice(c->device);
    free_plan(c);
    TreeOpts o;
    o.chi = opts->chi;
    o.cutoff = opts->cutoff;
    o.precision = opts->precision;
    o.jacobi_max_sweeps = opts->jacobi_max_sweeps > 0 ? opts->jacobi_max_sweeps : 40;
    o.budget = opts->device_budget_bytes;
    o.keep = opts->keep_intermediates;
    o.grad = opts->grad ? 1 : 0;
    o.plain = opts->plain ? 1 : 0;
    o.late = opts->compress_late;
    o.gauge_r = opts->gauge_r;
    o.segments = opts->checkpoint_segments;
    o.rfactor = opts->r_factor;
    if (o.plain && o.grad) return fail(c, TN_EINVAL, "the plain form has no reverse pass (grad must be 0)");
    std::string err = build_plan(c->g, pair_i, pair_j, n_steps, o, false, &c->plan);
    // level by level every independent branch advances at once; when that holds more than the
    // budget (or, without one, more than a third of the device), plan again with the levels in
    // tree order, which needs only the memory of a sequential run
    const int64_t soft_cap = o.budget > 0 ? o.budget : kArenaSoftCap;
    if (err.empty() && c->plan.arena_bytes > soft_cap) {
        o.ordered = 1;
        err = build_plan(c->g, pair_i, pair_j, n_steps, o, false, &c->plan);
    }
    if (!err.empty()) {
        const bool nomem = err.rfind("plan needs", 0) == 0;
        return fail(c, nomem ? TN_ENOMEM : TN_EINVAL, err);
    }
    const size_t bytes = (size_t)std::max<int64_t>(c->plan.arena_bytes, 256);
    if (c->workspace) {
        if (bytes > c->workspace_bytes) {
            const std::string msg = "plan needs an arena of " + std::to_string(bytes) + " bytes, the workspace holds " +
                                    std::to_string(c->workspace_bytes);
            free_plan(c);
            return fail(c, TN_ENOMEM, msg);
        }
        c->arena = c->workspace;
        c->arena_owned = false;
    } else {
        hipError_t e = hipMalloc((void**)&c->arena, bytes);
        if (e != hipSuccess) {
            c->arena = nullptr;
            return fail(c, TN_ENOMEM, std::string("arena of ") + std::to_string(bytes) + " bytes: " + hipGetErrorString(e));
        }
        c->arena_owned = true;
    }
    c->arena_cap = bytes;
    tn_status s = build_launches(c);
    if (s == TN_OK && o.grad) s = build_bwd_launches(c);
    if (s != TN_OK) {
        free_plan(c);
        return s;
    }
    c->has_plan = true;
    return TN_OK;
}

tn_status tn_set_workspace(tn_ctx* c, void* dev_ptr, size_t bytes) {
    if (!c) return TN_EINVAL;
    if (dev_ptr && ((uintptr_t)dev_ptr % 256) != 0) return fail(c, TN_EINVAL, "workspace must be 256-byte aligned");
    if (dev_ptr && bytes == 0) return fail(c, TN_EINVAL, "empty workspace");
    c->workspace = (char*)dev_ptr;
    c->workspace_bytes = dev_ptr ? bytes : 0;
    return TN_OK;
}

tn_status tn_compress_pair(tn_ctx* c, const double* a_dev, const double* b_dev, int64_t m_a, int32_t D, int64_t m_b,
                           int32_t chi, double cutoff, double* a_out, double* b_out, int32_t* chi_out) {
    if (!c) return TN_EINVAL;
    if (!a_dev || !b_dev || !a_out || !b_out) return fail(c, TN_EINVAL, "null matrix pointer");
    if (!(cutoff >= 0.0)) return fail(c, TN_EINVAL, "cutoff must be >= 0");
    PairLayout L;
    std::string err = pair_layout(m_a, D, m_b, chi, &L);
    if (!err.empty()) return fail(c, TN_EINVAL, err);
    (void)hipSetDevice(c->device);
    char* ws = nullptr;
    hipError_t e = hipMalloc((void**)&ws, (size_t)L.bytes);
    if (e != hipSuccess) return fail(c, TN_ENOMEM, std::string("compression workspace: ") + hipGetErrorString(e));
    PairDescs h;
    err = pair_enqueue(L, a_dev, b_dev, cutoff, 40, a_out, b_out, ws, &h, c->stream);
    int32_t sweeps = 0;
    if (err.empty()) {
        e = hipMemcpyAsync(&sweeps, ws + L.off_stats + 12, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
        if (e != hipSuccess) err = std::string("stats: ") + hipGetErrorString(e);
    }
    e = hipStreamSynchronize(c->stream);
    if (err.empty() && e != hipSuccess) err = std::string("compression: ") + hipGetErrorString(e);
    (void)hipFree(ws);
    if (!err.empty()) return fail(c, TN_EDEVICE, err);
    if (chi_out) *chi_out = (int32_t)L.nw;
    if (sweeps < 0) return fail(c, TN_ENUMERIC, "the Jacobi SVD did not converge within the sweep cap");
    return TN_OK;
}

tn_status tn_compress_pair_static(tn_ctx* c, const double* a_dev, const double* b_dev, int64_t m_a, int32_t D,
                                  int64_t m_b, int32_t chi, double cutoff, double* a_out, double* b_out,
                                  int32_t* chi_out) {
    if (!c) return TN_EINVAL;
    if (!a_dev || !b_dev || !a_out || !b_out) return fail(c, TN_EINVAL, "null matrix pointer");
    if (!(cutoff >= 0.0)) return fail(c, TN_EINVAL, "cutoff must be >= 0");
    PairLayout L;
    std::string err = pair_layout(m_a, D, m_b, chi, &L);
    if (!err.empty()) return fail(c, TN_EINVAL, err);
    if ((size_t)L.bytes > kStaticScratchBytes)
        return fail(c, TN_EINVAL, "the compression needs " + std::to_string(L.bytes) +
                                      " bytes of work memory, more than the static scratch of " +
                                      std::to_string(kStaticScratchBytes));
    char* ws = (char*)static_scratch(c->device);
    if (!ws) return fail(c, TN_ESTATE, "no static scratch address for this device");
    (void)hipSetDevice(c->device);
    PairDescs h;   // host copy of the descriptors: lives until the synchronisation below
    err = pair_enqueue(L, a_dev, b_dev, cutoff, 40, a_out, b_out, ws, &h, c->stream);
    int32_t sweeps = 0;
    hipError_t e = hipSuccess;
    if (err.empty()) {
        e = hipMemcpyAsync(&sweeps, ws + L.off_stats + 12, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
        if (e != hipSuccess) err = std::string("stats: ") + hipGetErrorString(e);
    }
    e = hipStreamSynchronize(c->stream);
    if (err.empty() && e != hipSuccess) err = std::string("compression: ") + hipGetErrorString(e);
    if (!err.empty()) return fail(c, TN_EDEVICE, err);
    if (chi_out) *chi_out = (int32_t)L.nw;
    if (sweeps < 0) return fail(c, TN_ENUMERIC, "the Jacobi SVD did not converge within the sweep cap");
    return TN_OK;
}

tn_status tn_plan_info(const tn_ctx* c, int64_t* arena_bytes, double* fwd_flops, double* fwd_bytes,
                       int32_t* n_steps) {
    if (!c) return TN_EINVAL;
    if (!c->has_plan) return TN_ESTATE;
    if (arena_bytes) *arena_bytes = c->plan.arena_bytes;
    if (fwd_flops) *fwd_flops = c->plan.fwd_flops;
    if (fwd_bytes) *fwd_bytes = c->plan.fwd_bytes;
    if (n_steps) *n_steps = (int32_t)c->plan.steps.size();
    return TN_OK;
}

// Add the stamped durations of the finished evaluation to the profile (stream synchronised).
tn_status collect_stamps(tn_ctx* c) {
    if (c->st_used.empty()) return TN_OK;
    int npairs = 0;
    for (auto& u : c->st_used) npairs = std::max(npairs, u.second + 1);
    std::vector<unsigned long long> h(2 * (size_t)npairs);
    HIP_TRY(c, hipMemcpy(h.data(), c->d_stamps, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    for (auto& u : c->st_used) c->prof_ms[u.first] += (double)(h[2 * u.second + 1] - h[2 * u.second]) * 1e-5;
    c->st_used.clear();
    return TN_OK;
}

// Enqueue one forward evaluation on the context's streams (eager, or inside a capture).
// Enqueue one forward launch of ctx c on stream st.
static hipError_t run_forward_launch(tn_ctx* c, const Launch& l, hipStream_t st) {
    const Plan& P = c->plan;
    const int prec = P.opts.precision;
    switch (l.kind) {
        case L_GEMM: return launch_gemm(l.key, c->d_gemm + l.begin, l.count, l.work, c->d_scales, c->d_maxparts, st);
        case L_COPY: return launch_copy(l.key, c->d_copy + l.begin, l.count, l.work, c->d_scales, st);
        case L_CORE:
            return launch_core(l.key, prec, c->d_core + l.begin, l.count, l.max_d, P.opts.jacobi_max_sweeps, c->d_disc,
                               c->d_tie, c->d_sweeps, st);
        case L_LANCZOS:
            return launch_lanczos(l.key, c->d_lanczos + l.begin, l.count, l.max_d, c->d_scales,
                                  P.opts.jacobi_max_sweeps, c->d_disc, c->d_tie, c->d_sweeps, st);
        case L_GLANCZOS:
            return launch_gram_lanczos(l.key, c->d_glanczos + l.begin, l.count, P.opts.jacobi_max_sweeps, c->d_disc,
                                       c->d_tie, c->d_sweeps, st);
        case L_SCALE: return launch_scale_finalize(c->d_scale + l.begin, l.count, c->d_maxparts, c->d_scales, st);
        case L_REDUCE: return launch_reduce(l.key, c->d_reduce + l.begin, l.count, l.work, c->d_scales, st);
        case L_SPRE: return launch_gemm(GEMM_F64, c->d_gemm + l.begin, l.count, l.work, c->d_scales, c->d_maxparts, st);
        case L_TSQR: return launch_tsqr(l.key, c->d_tsqr + l.begin, l.count, l.work, c->d_scales, st);
        case L_KRYLOV: {
            hipError_t err = hipSuccess;
            for (int64_t i = l.begin; i < l.begin + l.count && err == hipSuccess; ++i) {
                const KOp& o = c->h_kops[i];
                switch (o.kind) {
                    case KO_GEMM:
                        err = launch_gemm(o.key, c->d_gemm + o.begin, o.count, o.work, c->d_scales, c->d_maxparts, st);
                        break;
                    case KO_REDUCE: err = launch_reduce(0, c->d_reduce + o.begin, o.count, o.work, c->d_scales, st); break;
                    case KO_SMALL: err = launch_small(o.key, c->d_small + o.begin, o.count, o.work, st); break;
                    case KO_CHOL: err = launch_cholinv(c->d_chol + o.begin, o.count, st); break;
                    case KO_CORE:
                        err = launch_core(o.key, 0, c->d_core + o.begin, o.count, o.max_d, P.opts.jacobi_max_sweeps,
                                          c->d_disc, c->d_tie, c->d_sweeps, st);
                        break;
                    case KO_CHECK: err = launch_krylov_check(c->d_kcheck + o.begin, o.count, c->d_sweeps, st); break;
                }
            }
            return err;
        }
    }
    return hipSuccess;
}

tn_status enqueue_forward(tn_ctx* c) {
    Plan& P = c->plan;
    const int prec = P.opts.precision;
    hipStream_t s = c->stream;
    HIP_TRY(c, launch_inputs(prec, c->d_inputs, (int)c->h_inputs.size(), c->d_staging, c->d_scales, s));
    auto run = [&](const Launch& l, hipStream_t st) -> hipError_t {
        const bool timed = (c->prof_mask >> l.prof) & 1u;
        int pair = -1;
        if (timed) {
            pair = (int)c->st_used.size();
            if ((size_t)pair >= c->stamps_cap) return hipErrorInvalidValue;   // sized before enqueueing
            hipError_t err = launch_stamp(c->d_stamps + 2 * pair, st);
            if (err != hipSuccess) return err;
            c->st_used.push_back({l.prof, pair});
            c->prof_launches[l.prof] += 1;
            c->prof_flops[l.prof] += l.flops;
            c->prof_bytes[l.prof] += l.bytes;
        }
        hipError_t err = run_forward_launch(c, l, st);
        if (err == hipSuccess && timed) err = launch_stamp(c->d_stamps + 2 * pair + 1, st);
        return err;
    };
    size_t next_ev = 0;
    hipEvent_t pending[2] = {nullptr, nullptr};
    int open = 0;
    if (P.opts.plain) {   // one launch per step, in schedule order, on the context's stream
        for (const Launch& l : c->launches) HIP_TRY(c, run(l, s));
    }
    for (size_t b = 0; !P.opts.plain && b < c->launches.size();) {
        size_t e = b;
        while (e < c->launches.size() && c->launches[e].level == c->launches[b].level) ++e;
        HIP_TRY(c, run_level(c->launches, b, e, s, c->aux, c->sync_ev, next_ev, run, pending, e < c->launches.size(),
                             open));
        b = e;
    }
    if (tn_status st = join_tail(c, s, pending, open, fail); st != TN_OK) return st;
    const void* fin = c->arena + P.bufs[P.tens[P.final_tensor].buf].off;
    HIP_TRY(c, launch_result(prec, c->d_scales, (int)P.tens.size(), fin, c->d_sweeps, (int)P.comps.size(),
                             c->d_result, s));
    HIP_TRY(c, hipMemcpyAsync(c->h_result, c->d_result, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    return TN_OK;
}

tn_status tn_enqueue(tn_ctx* c) {
    if (!c) return TN_EINVAL;
    if (!c->has_plan) return fail(c, TN_ESTATE, "evaluate before tn_set_tree");
    (void)hipSetDevice(c->device);
    if (c->plan.opts.plain || c->n_kernels > kMaxCaptureKernels) {
        // the plain form, and schedules too long to capture, are enqueued launch by launch on every
        // evaluation (no graph)
        if (!c->st_used.empty()) {
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            if (tn_status st = collect_stamps(c); st != TN_OK) return st;
        }
        size_t timed = 0;
        for (const Launch& l : c->launches) timed += (c->prof_mask >> l.prof) & 1u;
        if (timed > c->stamps_cap) {
            dfree(c->d_stamps);
            c->stamps_cap = 0;
            HIP_TRY(c, hipMalloc((void**)&c->d_stamps, 2 * timed * sizeof(unsigned long long)));
            c->stamps_cap = timed;
        }
        return enqueue_forward(c);
    }
    if (!c->fexec || c->fgraph_mask != c->prof_mask) {
        // capture the schedule once (per profiling mask): replays skip the per-launch host work
        free_forward_graph(c);
        if (!c->st_used.empty()) {   // stamps of an unfetched evaluation: fold them in first
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            if (tn_status st = collect_stamps(c); st != TN_OK) return st;
        }
        size_t timed = 0;
        for (const Launch& l : c->launches) timed += (c->prof_mask >> l.prof) & 1u;
        if (timed > c->stamps_cap) {
            dfree(c->d_stamps);
            c->stamps_cap = 0;
            HIP_TRY(c, hipMalloc((void**)&c->d_stamps, 2 * timed * sizeof(unsigned long long)));
            c->stamps_cap = timed;
        }
        const auto st0 = c->st_used;
        int64_t l0[kKinds];
        double f0[kKinds], b0[kKinds];
        for (int k = 0; k < kKinds; ++k) {
            l0[k] = c->prof_launches[k];
            f0[k] = c->prof_flops[k];
            b0[k] = c->prof_bytes[k];
        }
        c->st_used.clear();
        HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        const tn_status es = enqueue_forward(c);
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(c->stream, &g);
        c->fgraph_st = c->st_used;
        c->st_used = st0;
        for (int k = 0; k < kKinds; ++k) {
            c->fgraph_launches[k] = c->prof_launches[k] - l0[k];
            c->fgraph_flops[k] = c->prof_flops[k] - f0[k];
            c->fgraph_bytes[k] = c->prof_bytes[k] - b0[k];
            c->prof_launches[k] = l0[k];
            c->prof_flops[k] = f0[k];
            c->prof_bytes[k] = b0[k];
        }
        if (es != TN_OK || ce != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            c->fgraph_st.clear();
            return es != TN_OK ? es : fail(c, TN_EDEVICE, std::string("forward capture: ") + hipGetErrorString(ce));
        }
        c->fgraph = g;
        HIP_TRY(c, hipGraphInstantiate(&c->fexec, c->fgraph, nullptr, nullptr, 0));
        c->fgraph_mask = c->prof_mask;
    }
    HIP_TRY(c, hipGraphLaunch(c->fexec, c->stream));
    // a replay re-writes the same stamp pairs: the totals read at tn_fetch are the last replay's
    c->st_used.insert(c->st_used.end(), c->fgraph_st.begin(), c->fgraph_st.end());
    for (int k = 0; k < kKinds; ++k) {
        c->prof_launches[k] += c->fgraph_launches[k];
        c->prof_flops[k] += c->fgraph_flops[k];
        c->prof_bytes[k] += c->fgraph_bytes[k];
    }
    return TN_OK;
}

tn_status tn_fetch(tn_ctx* c) {
    if (!c) return TN_EINVAL;
    if (!c->has_plan) return fail(c, TN_ESTATE, "no plan");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (tn_status st = collect_stamps(c); st != TN_OK) return st;
    c->sign = c->h_result[0];
    c->lnz = c->h_result[1];
    c->flags = (int)c->h_result[2];
    // only a finished evaluation counts: tn_result and tn_grad refuse a failed one
    c->evaluated = false;
    if (c->flags & 2) return fail(c, TN_ENUMERIC, "non-finite tensor entry");
    if (c->flags & 4)
        return fail(c, TN_ENUMERIC,
                    "a compression did not converge (Jacobi sweep cap, or a block-Krylov basis too small for a flat "
                    "core spectrum)");
    c->evaluated = true;
    c->fwd_fresh = true;
    if ((c->flags & 1) || c->sign == 0.0) {
        c->sign = 0.0;
        c->lnz = -INFINITY;
        return fail(c, TN_ZERO, "the network evaluates to zero");
    }
    return TN_OK;
}

tn_status tn_contract_compressed(tn_ctx* c, double* mantissa, double* log10_exponent) {
    tn_status s = tn_enqueue(c);
    if (s != TN_OK) return s;
    s = tn_fetch(c);
    if (s == TN_ZERO) {
        if (mantissa) *mantissa = 0.0;
        if (log10_exponent) *log10_exponent = -INFINITY;
        return s;
    }
    if (s != TN_OK) return s;
    const double l10 = c->lnz / std::log(10.0);
    const double ex = std::floor(l10);
    double m = std::pow(10.0, l10 - ex);
    if (m >= 10.0) m /= 10.0;   // guard against rounding at the boundary
    if (mantissa) *mantissa = c->sign * m;
    if (log10_exponent) *log10_exponent = ex;
    return TN_OK;
}

tn_status tn_result(const tn_ctx* c, double* sign, double* ln_abs_z) {
    if (!c) return TN_EINVAL;
    if (!c->evaluated) return TN_ESTATE;
    if (sign) *sign = c->sign;
    if (ln_abs_z) *ln_abs_z = c->lnz;
    return TN_OK;
}

tn_status tn_compress_stats(const tn_ctx* c0, int32_t cap, double* discarded, int32_t* tie, int32_t* sweeps,
                            int32_t* n_out) {
    tn_ctx* c = const_cast<tn_ctx*>(c0);
    if (!c) return TN_EINVAL;
    if (!c->evaluated) return fail(c, TN_ESTATE, "no evaluation yet");
    const int n = (int)c->plan.comps.size();
    if (n_out) *n_out = n;
    const int k = std::min(n, std::max(0, cap));
    if (k > 0) {
        if (discarded) HIP_TRY(c, hipMemcpy(discarded, c->d_disc, k * sizeof(double), hipMemcpyDeviceToHost));
        if (tie) HIP_TRY(c, hipMemcpy(tie, c->d_tie, k * sizeof(int32_t), hipMemcpyDeviceToHost));
        if (sweeps) HIP_TRY(c, hipMemcpy(sweeps, c->d_sweeps, k * sizeof(int32_t), hipMemcpyDeviceToHost));
    }
    return TN_OK;
}

tn_status tn_profile(tn_ctx* c, uint32_t kind_mask) {
    if (!c) return TN_EINVAL;
    c->prof_mask = kind_mask;
    for (int k = 0; k < kKinds; ++k) {
        c->prof_ms[k] = 0;
        c->prof_launches[k] = 0;
        c->prof_flops[k] = c->prof_bytes[k] = 0;
    }
    return TN_OK;
}

tn_status tn_profile_read(const tn_ctx* c, int32_t kind, double* ms, int64_t* launches, double* flops,
                          double* bytes) {
    if (!c) return TN_EINVAL;
    if (kind < 0 || kind >= kKinds) return TN_EINVAL;
    if (ms) *ms = c->prof_ms[kind];
    if (launches) *launches = c->prof_launches[kind];
    if (flops) *flops = c->prof_flops[kind];
    if (bytes) *bytes = c->prof_bytes[kind];
    return TN_OK;
}

tn_status tn_read_tensor(const tn_ctx* c0, int32_t index, double* out, int64_t cap, int64_t* n) {
    tn_ctx* c = const_cast<tn_ctx*>(c0);
    if (!c) return TN_EINVAL;
    if (!c->evaluated) return fail(c, TN_ESTATE, "no evaluation yet");
    const Plan& P = c->plan;
    if (index < 0 || index >= (int32_t)P.tens.size()) return fail(c, TN_EINVAL, "tensor index out of range");
    const TensorVer& t = P.tens[index];
    if (n) *n = t.size;
    const int64_t k = std::min<int64_t>(std::max<int64_t>(cap, 0), t.size);
    if (k == 0 || !out) return TN_OK;
    (void)hipSetDevice(c->device);
    double s = 0.0;
    HIP_TRY(c, hipMemcpy(&s, c->d_scales + index, sizeof(double), hipMemcpyDeviceToHost));
    const char* src = c->arena + P.bufs[t.buf].off;
    if (P.elem_size == 8) {
        HIP_TRY(c, hipMemcpy(out, src, k * sizeof(double), hipMemcpyDeviceToHost));
    } else if (P.elem_size == 4) {
        std::vector<float> tmp(k);
        HIP_TRY(c, hipMemcpy(tmp.data(), src, k * sizeof(float), hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < k; ++i) out[i] = tmp[i];
    } else {   // bfloat16: the upper half of a binary32
        std::vector<uint16_t> tmp(k);
        HIP_TRY(c, hipMemcpy(tmp.data(), src, k * sizeof(uint16_t), hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < k; ++i) {
            const uint32_t u = (uint32_t)tmp[i] << 16;
            float f;
            std::memcpy(&f, &u, sizeof(f));
            out[i] = f;
        }
    }
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    for (int64_t i = 0; i < k; ++i) out[i] *= inv;
    return TN_OK;
}

tn_status tn_read_projectors(const tn_ctx* c0, int32_t comp, double* p_left, double* p_right, int64_t cap,
                             int32_t* bond_edges, int32_t edge_cap, int32_t* info) {
    tn_ctx* c = const_cast<tn_ctx*>(c0);
    if (!c) return TN_EINVAL;
    if (!c->has_plan) return fail(c, TN_ESTATE, "no tree set");
    const Plan& P = c->plan;
    if (comp < 0 || comp >= (int32_t)P.comps.size()) return fail(c, TN_EINVAL, "compression index out of range");
    const Compression& cp = P.comps[comp];
    const int64_t D = cp.D, cn = cp.chi_new;
    if (info) {
        info[0] = (int32_t)D;
        info[1] = (int32_t)cn;
        info[2] = cp.e_new;
        info[3] = cp.node_a;
        info[4] = cp.node_b;
        info[5] = (int32_t)cp.bond_edges.size();
    }
    if (bond_edges)
        for (int32_t i = 0; i < std::min<int32_t>(edge_cap, (int32_t)cp.bond_edges.size()); ++i)
            bond_edges[i] = cp.bond_edges[i];
    if (!p_left && !p_right) return TN_OK;
    if (!c->evaluated) return fail(c, TN_ESTATE, "no evaluation yet");
    if (!P.opts.keep) return fail(c, TN_ESTATE, "projectors stay intact only with keep_intermediates = 1");
    if (cap < D * cn) return fail(c, TN_EINVAL, "output buffers hold fewer than D * chi' entries");
    (void)hipSetDevice(c->device);
    for (int side = 0; side < 2; ++side) {
        double* out = side == 0 ? p_left : p_right;
        if (!out) continue;
        const char* src = c->arena + P.bufs[side == 0 ? cp.pl_buf : cp.pr_buf].off;
        const int64_t k = D * cn;
        if (P.elem_size == 8) {
            HIP_TRY(c, hipMemcpy(out, src, k * sizeof(double), hipMemcpyDeviceToHost));
        } else if (P.elem_size == 4) {
            std::vector<float> tmp(k);
            HIP_TRY(c, hipMemcpy(tmp.data(), src, k * sizeof(float), hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < k; ++i) out[i] = tmp[i];
        } else {   // bfloat16: the upper half of a binary32
            std::vector<uint16_t> tmp(k);
            HIP_TRY(c, hipMemcpy(tmp.data(), src, k * sizeof(uint16_t), hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < k; ++i) {
                const uint32_t u = (uint32_t)tmp[i] << 16;
                float f;
                std::memcpy(&f, &u, sizeof(f));
                out[i] = f;
            }
        }
    }
    return TN_OK;
}

tn_status tn_grad_device(tn_ctx* c, void* out) {
    if (!c) return TN_EINVAL;
    if (!out) return fail(c, TN_EINVAL, "null gradient buffer");
    if (!c->has_plan || !c->plan.opts.grad) return fail(c, TN_ESTATE, "the tree was planned without opts.grad");
    if (!c->evaluated) return fail(c, TN_ESTATE, "tn_grad before an evaluation");
    if (c->sign == 0.0) return fail(c, TN_ZERO, "Z = 0: ln|Z| has no gradient");
    (void)hipSetDevice(c->device);
    Plan& P = c->plan;
    const int prec = P.opts.precision;
    hipStream_t s = c->stream;
    const int fin = P.final_tensor;
    // Segments last to first: re-run the forward launches of a segment, then its reverse levels.
    // The last segment is not re-run: the arena holds it from the evaluation.  A re-run of
    // segment s writes over buffers of later segments, including checkpoints that the re-runs of
    // later segments start from, so once any re-run has happened the arena no longer holds the
    // evaluation: a later tn_grad first re-runs the whole forward schedule (inputs and scale
    // slots are never written over).  The seed reads the final tensor, after those re-runs.
    const int S = P.n_segments;
    size_t bi = 0;
    size_t next_ev = 0;
    auto rerun_levels = [&](int32_t first, int32_t end) -> tn_status {
        Launch tl;
        tl.prof = TN_KERNEL_RECOMPUTE;
        size_t b = 0;
        while (b < c->launches.size() && c->launches[b].level < first) ++b;
        size_t e = b;
        while (e < c->launches.size() && c->launches[e].level < end) {
            tl.flops += c->launches[e].flops;
            tl.bytes += c->launches[e].bytes;
            ++e;
        }
        bool timed = false;
        if (tn_status st = prof_begin(c, tl, s, &timed); st != TN_OK) return st;
        auto run = [&](const Launch& l, hipStream_t st) { return run_forward_launch(c, l, st); };
        hipEvent_t pending[2] = {nullptr, nullptr};
        int open = 0;
        for (size_t i = b; i < e;) {
            size_t j = i;
            while (j < e && c->launches[j].level == c->launches[i].level) ++j;
            HIP_TRY(c, run_level(c->launches, i, j, s, c->aux, c->rc_ev, next_ev, run, pending, j < e, open));
            i = j;
        }
        if (tn_status st = join_tail(c, s, pending, open, fail); st != TN_OK) return st;
        if (timed) HIP_TRY(c, hipEventRecord(c->ev_pool[c->ev_used.back().second + 1], s));
        return TN_OK;
    };
    if (S > 1 && !c->fwd_fresh) {
        if (tn_status st = rerun_levels(1, P.seg_begin[S]); st != TN_OK) return st;
        c->fwd_fresh = true;
    }
    for (int seg = S - 1; seg >= 0; --seg) {
        if (S > 1 && seg < S - 1 && P.seg_recompute[seg]) {
            c->fwd_fresh = false;
            if (tn_status st = rerun_levels(P.seg_begin[seg], P.seg_begin[seg + 1]); st != TN_OK) return st;
        }
        if (seg == S - 1)
            HIP_TRY(c, launch_seed(prec, c->arena + P.bufs[P.tens[fin].buf].off,
                                   c->arena + P.bufs[P.adj_buf[fin]].off, c->d_scales, fin, s));
        for (; bi < c->blaunches.size() && c->blaunches[bi].level <= P.seg_bend[seg]; ++bi) {
            const Launch& l = c->blaunches[bi];
            bool timed = false;
            tn_status st = prof_begin(c, l, s, &timed);
            if (st != TN_OK) return st;
            switch (l.kind) {
                case L_GEMM:
                    HIP_TRY(c, launch_gemm(l.key, c->d_bgemm + l.begin, l.count, l.work, c->d_scales, c->d_maxparts, s));
                    break;
                case L_REDUCE:
                    HIP_TRY(c, launch_reduce(l.key, c->d_reduce + l.begin, l.count, l.work, c->d_scales, s));
                    break;
                case L_CORE_BWD:
                    HIP_TRY(c, launch_core_bwd(l.key, c->d_cbwd + l.begin, l.count, l.max_d, s));
                    break;
            }
            if (timed) HIP_TRY(c, hipEventRecord(c->ev_pool[c->ev_used.back().second + 1], s));
        }
    }
    if (bi != c->blaunches.size()) return fail(c, TN_EINVAL, "internal: reverse launches outside every segment");
    HIP_TRY(c, launch_grad_inputs(prec, c->d_gin, (int)c->h_gin.size(), c->d_scales, (double*)out, s));
    return TN_OK;
}

tn_status tn_grad(tn_ctx* c, double* dlnz_ddata) {
    if (!c) return TN_EINVAL;
    if (!dlnz_ddata) return fail(c, TN_EINVAL, "null gradient buffer");
    if (!c->has_plan || !c->plan.opts.grad) return fail(c, TN_ESTATE, "the tree was planned without opts.grad");
    tn_status st = tn_grad_device(c, c->d_grad);
    if (st != TN_OK) return st;
    HIP_TRY(c, hipMemcpyAsync(dlnz_ddata, c->d_grad, c->n_input_elems * sizeof(double), hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (auto& u : c->ev_used) {
        float ms = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&ms, c->ev_pool[u.second], c->ev_pool[u.second + 1]));
        c->prof_ms[u.first] += ms;
    }
    c->ev_used.clear();
    return TN_OK;
}

tn_status tn_sync(tn_ctx* c) {
    if (!c) return TN_EINVAL;
    (void)hipSetDevice(c->device);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TN_OK;
}

tn_status tn_ising_values_device(tn_ctx* c, double beta, const void* J_dev) {
    if (!c) return TN_EINVAL;
    if (!c->has_graph) return fail(c, TN_ESTATE, "no graph loaded");
    if (!c->ising_ok) return fail(c, TN_EINVAL, "the Ising map needs every edge of dimension 2");
    if (!J_dev) return fail(c, TN_EINVAL, "null couplings");
    (void)hipSetDevice(c->device);
    HIP_TRY(c, launch_ising_values(c->ising, beta, (const double*)J_dev, c->d_staging, c->n_input_elems, c->stream));
    c->evaluated = false;
    return TN_OK;
}

tn_status tn_ising_coupling_grad_device(tn_ctx* c, double beta, const void* J_dev, const void* dlnz_ddata_dev,
                                        void* dlnz_dJ_dev) {
    if (!c) return TN_EINVAL;
    if (!c->has_graph) return fail(c, TN_ESTATE, "no graph loaded");
    if (!c->ising_ok) return fail(c, TN_EINVAL, "the Ising map needs every edge of dimension 2");
    if (!J_dev || !dlnz_ddata_dev || !dlnz_dJ_dev) return fail(c, TN_EINVAL, "null device buffer");
    (void)hipSetDevice(c->device);
    HIP_TRY(c, launch_ising_grad(c->ising, beta, (const double*)J_dev, (const double*)dlnz_ddata_dev,
                                 (double*)dlnz_dJ_dev, c->stream));
    return TN_OK;
}

tn_status tn_grad_info(const tn_ctx* c, double* bwd_flops, double* bwd_bytes, int32_t* n_levels) {
    if (!c) return TN_EINVAL;
    if (!c->has_plan || !c->plan.opts.grad) return TN_ESTATE;
    if (bwd_flops) *bwd_flops = c->plan.bwd_flops;
    if (bwd_bytes) *bwd_bytes = c->plan.bwd_bytes;
    if (n_levels) *n_levels = c->plan.n_blevels;
    return TN_OK;
}

tn_status tn_grad_checkpoint_info(const tn_ctx* c, int32_t* segments, double* recompute_flops,
                                  int64_t* checkpoint_bytes) {
    if (!c) return TN_EINVAL;
    if (!c->has_plan || !c->plan.opts.grad) return TN_ESTATE;
    if (segments) *segments = c->plan.n_segments;
    if (recompute_flops) *recompute_flops = c->plan.recompute_flops;
    if (checkpoint_bytes) *checkpoint_bytes = c->plan.checkpoint_bytes;
    return TN_OK;
}

tn_status tn_plan_describe(int32_t n_tensors, int32_t n_edges, const int32_t* edge_u, const int32_t* edge_v,
                           const int32_t* edge_dim, int32_t n_steps, const int32_t* pair_i, const int32_t* pair_j,
                           const tn_tree_opts* opts, int64_t cap, int64_t* ops, int64_t* n_ops) {
    if (n_tensors < 1 || n_edges < 0 || !opts || !n_ops) return TN_EINVAL;
    if (n_edges > 0 && (!edge_u || !edge_v || !edge_dim)) return TN_EINVAL;
    if (n_steps > 0 && (!pair_i || !pair_j)) return TN_EINVAL;
    GraphSpec g;
    g.n = n_tensors;
    g.ne = n_edges;
    g.eu.assign(edge_u, edge_u + n_edges);
    g.ev.assign(edge_v, edge_v + n_edges);
    g.ed.assign(edge_dim, edge_dim + n_edges);
    // sizes from the graph itself (no data is involved)
    std::vector<int64_t> size(n_tensors, 1);
    for (int e = 0; e < n_edges; ++e)
        if (edge_u[e] >= 0 && edge_u[e] < n_tensors && edge_v[e] >= 0 && edge_v[e] < n_tensors) {
            size[edge_u[e]] *= edge_dim[e];
            size[edge_v[e]] *= edge_dim[e];
        }
    g.offsets.assign(n_tensors + 1, 0);
    for (int v = 0; v < n_tensors; ++v) g.offsets[v + 1] = g.offsets[v] + size[v];
    if (!check_graph(g).empty()) return TN_EINVAL;
    if (opts->gauge_r < 0 || (opts->compress_late != 0 && opts->compress_late != 1)) return TN_EINVAL;
    TreeOpts o;
    o.chi = opts->chi;
    o.cutoff = opts->cutoff;
    o.precision = opts->precision;
    o.late = opts->compress_late;
    Plan P;
    std::string err = build_plan(g, pair_i, pair_j, n_steps, o, true, &P);
    if (!err.empty()) return TN_EINVAL;
    *n_ops = (int64_t)P.ops.size();
    for (int64_t i = 0; i < std::min<int64_t>(cap, (int64_t)P.ops.size()); ++i) {
        const OpRec& r = P.ops[i];
        int64_t* q = ops + 8 * i;
        q[0] = r.kind;
        q[1] = r.a;
        q[2] = r.b;
        q[3] = r.out;
        q[4] = r.m;
        q[5] = r.n;
        q[6] = r.k;
        q[7] = r.new_dim;
    }
    return TN_OK;
}

}  // extern "C"

// ==========================================================================================
// Batches: several planned contexts merged level by level and captured in one hipGraph
// ==========================================================================================
struct tn_batch {
    int device = 0;
    int prec = 0;
    hipStream_t stream = nullptr;
    std::vector<tn_ctx*> ctxs;
    std::vector<int64_t> scale_off, comp_off;
    int64_t n_scales = 0, n_comps = 0;
    std::string err;
    // merged forward schedule
    std::vector<GemmDesc> h_gemm;
    std::vector<CopyDesc> h_copy;
    std::vector<CoreDesc> h_core;
    std::vector<ScaleDesc> h_scale;
    std::vector<LanczosDesc> h_lanczos;
    std::vector<GLanczosDesc> h_glanczos;
    std::vector<Launch> launches;
    GemmDesc* d_gemm = nullptr;
    CopyDesc* d_copy = nullptr;
    CoreDesc* d_core = nullptr;
    ScaleDesc* d_scale = nullptr;
    LanczosDesc* d_lanczos = nullptr;
    GLanczosDesc* d_glanczos = nullptr;
    int64_t max_parts = 1;
    // merged reverse schedule (when every context was planned with opts.grad)
    bool grad = false;
    std::vector<GemmDesc> h_bgemm;
    std::vector<ReduceDesc> h_reduce;
    std::vector<CoreBwdDesc> h_cbwd;
    std::vector<Launch> blaunches;
    GemmDesc* d_bgemm = nullptr;
    ReduceDesc* d_reduce = nullptr;
    CoreBwdDesc* d_cbwd = nullptr;
    // batch-wide state
    double* d_scales = nullptr;
    double* d_maxparts = nullptr;
    double* d_disc = nullptr;
    int32_t* d_tie = nullptr;
    int32_t* d_sweeps = nullptr;
    double* d_result = nullptr;      // 4 per context
    double* h_result = nullptr;      // pinned
    hipGraph_t graph = nullptr, bgraph = nullptr;
    hipGraphExec_t exec = nullptr, bexec = nullptr;
    hipStream_t aux[kLanes - 1] = {nullptr, nullptr, nullptr};
    std::vector<hipEvent_t> sync_ev;
    std::vector<void*> bgrad_ptrs;   // the device outputs the reverse graph was captured with
};

namespace {

tn_status bfail(tn_batch* b, tn_status s, const std::string& msg) {
    if (b) b->err = msg;
    return s;
}

#define BHIP_TRY(b, expr)                                                                         \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return bfail(b, TN_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)

template <typename T>
tn_status bupload(tn_batch* b, T** dst, const std::vector<T>& src) {
    dfree(*dst);
    if (src.empty()) return TN_OK;
    BHIP_TRY(b, hipMalloc((void**)dst, src.size() * sizeof(T)));
    BHIP_TRY(b, hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return TN_OK;
}

inline void shift(int32_t& idx, int64_t off) {
    if (idx >= 0) idx = (int32_t)(idx + off);
}

// Merge the contexts' launches of one level and kind/key into one grouped launch.
void merge_forward(tn_batch* b) {
    int max_level = 0;
    for (tn_ctx* c : b->ctxs) max_level = std::max(max_level, c->plan.n_levels);
    for (int L = 1; L <= max_level; ++L) {
        // per (kind, key): the launches of every context at this level, in context order
        std::map<std::pair<int, int>, std::vector<std::pair<int, const Launch*>>> groups;
        for (int i = 0; i < (int)b->ctxs.size(); ++i)
            for (const Launch& l : b->ctxs[i]->launches)
                if (l.level == L) groups[{l.kind, l.kind == L_GEMM ? l.key * 4 + l.prof : l.key}].push_back({i, &l});
        // per-tile max slots of this level: each context's block follows the previous ones
        std::vector<int64_t> part_off(b->ctxs.size(), 0);
        int64_t parts = 0;
        for (int i = 0; i < (int)b->ctxs.size(); ++i) {
            part_off[i] = parts;
            for (const Launch& l : b->ctxs[i]->launches)
                if (l.level == L && l.kind == L_SCALE)
                    for (int k = 0; k < l.count; ++k) parts += b->ctxs[i]->h_scale[l.begin + k].nparts;
        }
        b->max_parts = std::max(b->max_parts, parts);
        // GEMM and lanczos-type launches first, SCALE last (it reads the GEMMs' tile maxima)
        for (int pass = 0; pass < 2; ++pass)
            for (auto& kv : groups) {
                const int kind = kv.first.first;
                if ((kind == L_SCALE) != (pass == 1)) continue;
                Launch m = *kv.second.front().second;
                m.level = L;
                m.count = 0;
                m.work = 0;
                m.flops = m.bytes = 0;
                m.max_d = 0;
                switch (kind) {
                    case L_GEMM:
                    case L_SPRE: m.begin = (int64_t)b->h_gemm.size(); break;
                    case L_COPY: m.begin = (int64_t)b->h_copy.size(); break;
                    case L_CORE: m.begin = (int64_t)b->h_core.size(); break;
                    case L_LANCZOS: m.begin = (int64_t)b->h_lanczos.size(); break;
                    case L_GLANCZOS: m.begin = (int64_t)b->h_glanczos.size(); break;
                    case L_SCALE: m.begin = (int64_t)b->h_scale.size(); break;
                    case L_REDUCE: m.begin = (int64_t)b->h_reduce.size(); break;
                }
                for (auto& pr : kv.second) {
                    const int i = pr.first;
                    const Launch& l = *pr.second;
                    tn_ctx* c = b->ctxs[i];
                    const int64_t so = b->scale_off[i], co = b->comp_off[i], po = part_off[i];
                    m.count += l.count;
                    m.flops += l.flops;
                    m.bytes += l.bytes;
                    m.max_d = std::max(m.max_d, l.max_d);
                    for (int k = 0; k < l.count; ++k) {
                        switch (kind) {
                            case L_GEMM:
                            case L_SPRE: {
                                GemmDesc g = c->h_gemm[l.begin + k];
                                shift(g.scale_a, so);
                                shift(g.scale_b, so);
                                if (g.mode == GEMM_TENSOR) g.maxpart = (int32_t)(g.maxpart + po);
                                g.tile_begin = m.work;
                                m.work += (int64_t)g.tiles_m * g.tiles_n * g.splits;
                                b->h_gemm.push_back(g);
                                break;
                            }
                            case L_COPY: {
                                CopyDesc d = c->h_copy[l.begin + k];
                                shift(d.scale, so);
                                d.elem_begin = m.work;
                                m.work += (int64_t)d.rows * d.cols;
                                b->h_copy.push_back(d);
                                break;
                            }
                            case L_CORE: {
                                CoreDesc d = c->h_core[l.begin + k];
                                shift(d.stat, co);
                                b->h_core.push_back(d);
                                break;
                            }
                            case L_LANCZOS: {
                                LanczosDesc d = c->h_lanczos[l.begin + k];
                                shift(d.scale_a, so);
                                shift(d.scale_b, so);
                                shift(d.stat, co);
                                b->h_lanczos.push_back(d);
                                break;
                            }
                            case L_GLANCZOS: {
                                GLanczosDesc d = c->h_glanczos[l.begin + k];
                                shift(d.stat, co);
                                b->h_glanczos.push_back(d);
                                break;
                            }
                            case L_SCALE: {
                                ScaleDesc d = c->h_scale[l.begin + k];
                                d.maxpart = (int32_t)(d.maxpart + po);
                                shift(d.tensor, so);
                                b->h_scale.push_back(d);
                                break;
                            }
                            case L_REDUCE: {
                                ReduceDesc r = c->h_reduce[l.begin + k];
                                r.elem_begin = m.work;
                                m.work += (int64_t)r.M * r.N;
                                b->h_reduce.push_back(r);
                                break;
                            }
                        }
                    }
                }
                b->launches.push_back(m);
            }
    }
    order_for_issue(b->launches);
}

void merge_backward(tn_batch* b) {
    int max_level = 0;
    for (tn_ctx* c : b->ctxs) max_level = std::max(max_level, c->plan.n_blevels);
    for (int L = 1; L <= max_level; ++L) {
        std::map<std::pair<int, int>, std::vector<std::pair<int, const Launch*>>> groups;
        for (int i = 0; i < (int)b->ctxs.size(); ++i)
            for (const Launch& l : b->ctxs[i]->blaunches)
                if (l.level == L) groups[{l.kind, l.key}].push_back({i, &l});
        for (auto& kv : groups) {
            const int kind = kv.first.first;
            Launch m = *kv.second.front().second;
            m.count = 0;
            m.work = 0;
            m.flops = m.bytes = 0;
            m.max_d = 0;
            m.begin = kind == L_GEMM ? (int64_t)b->h_bgemm.size()
                                     : kind == L_REDUCE ? (int64_t)b->h_reduce.size() : (int64_t)b->h_cbwd.size();
            for (auto& pr : kv.second) {
                const Launch& l = *pr.second;
                tn_ctx* c = b->ctxs[pr.first];
                const int64_t so = b->scale_off[pr.first];
                m.count += l.count;
                m.flops += l.flops;
                m.bytes += l.bytes;
                m.max_d = std::max(m.max_d, l.max_d);
                for (int k = 0; k < l.count; ++k) {
                    if (kind == L_GEMM) {
                        GemmDesc g = c->h_bgemm[l.begin + k];
                        shift(g.scale_a, so);
                        shift(g.scale_b, so);
                        g.tile_begin = m.work;
                        m.work += (int64_t)g.tiles_m * g.tiles_n * g.splits;
                        b->h_bgemm.push_back(g);
                    } else if (kind == L_REDUCE) {
                        ReduceDesc r = c->h_reduce[l.begin + k];
                        shift(r.scale_a, so);
                        shift(r.scale_b, so);
                        r.elem_begin = m.work;
                        m.work += (int64_t)r.M * r.N;
                        b->h_reduce.push_back(r);
                    } else {
                        b->h_cbwd.push_back(c->h_cbwd[l.begin + k]);
                    }
                }
            }
            b->blaunches.push_back(m);
        }
    }
}

// Enqueue the merged forward schedule on the batch stream (captured into the graph).
tn_status enqueue_batch_forward(tn_batch* b) {
    hipStream_t s = b->stream;
    for (int i = 0; i < (int)b->ctxs.size(); ++i) {
        tn_ctx* c = b->ctxs[i];
        BHIP_TRY(b, launch_inputs(b->prec, c->d_inputs, (int)c->h_inputs.size(), c->d_staging,
                                  b->d_scales + b->scale_off[i], s));
    }
    auto run = [&](const Launch& l, hipStream_t st) -> hipError_t {
        switch (l.kind) {
            case L_GEMM: return launch_gemm(l.key, b->d_gemm + l.begin, l.count, l.work, b->d_scales, b->d_maxparts, st);
            case L_COPY: return launch_copy(l.key, b->d_copy + l.begin, l.count, l.work, b->d_scales, st);
            case L_CORE:
                return launch_core(l.key, b->prec, b->d_core + l.begin, l.count, l.max_d,
                                   b->ctxs[0]->plan.opts.jacobi_max_sweeps, b->d_disc, b->d_tie, b->d_sweeps, st);
            case L_LANCZOS:
                return launch_lanczos(l.key, b->d_lanczos + l.begin, l.count, l.max_d, b->d_scales,
                                      b->ctxs[0]->plan.opts.jacobi_max_sweeps, b->d_disc, b->d_tie, b->d_sweeps, st);
            case L_GLANCZOS:
                return launch_gram_lanczos(l.key, b->d_glanczos + l.begin, l.count,
                                           b->ctxs[0]->plan.opts.jacobi_max_sweeps, b->d_disc, b->d_tie, b->d_sweeps,
                                           st);
            case L_SCALE: return launch_scale_finalize(b->d_scale + l.begin, l.count, b->d_maxparts, b->d_scales, st);
            case L_REDUCE: return launch_reduce(l.key, b->d_reduce + l.begin, l.count, l.work, b->d_scales, st);
            case L_SPRE:
                return launch_gemm(GEMM_F64, b->d_gemm + l.begin, l.count, l.work, b->d_scales, b->d_maxparts, st);
        }
        return hipSuccess;
    };
    size_t next_ev = 0;
    hipEvent_t pending[2] = {nullptr, nullptr};
    int open = 0;
    for (size_t i = 0; i < b->launches.size();) {
        size_t e = i;
        while (e < b->launches.size() && b->launches[e].level == b->launches[i].level) ++e;
        BHIP_TRY(b, run_level(b->launches, i, e, s, b->aux, b->sync_ev, next_ev, run, pending, e < b->launches.size(),
                              open));
        i = e;
    }
    if (tn_status st = join_tail(b, s, pending, open, bfail); st != TN_OK) return st;
    for (int i = 0; i < (int)b->ctxs.size(); ++i) {
        tn_ctx* c = b->ctxs[i];
        const Plan& P = c->plan;
        const void* fin = c->arena + P.bufs[P.tens[P.final_tensor].buf].off;
        BHIP_TRY(b, launch_result(b->prec, b->d_scales + b->scale_off[i], (int)P.tens.size(), fin,
                                  b->d_sweeps + b->comp_off[i], (int)P.comps.size(), b->d_result + 4 * i, s));
    }
    return TN_OK;
}

tn_status enqueue_batch_backward(tn_batch* b, void* const* outs) {
    hipStream_t s = b->stream;
    for (int i = 0; i < (int)b->ctxs.size(); ++i) {
        tn_ctx* c = b->ctxs[i];
        const Plan& P = c->plan;
        const int fin = P.final_tensor;
        BHIP_TRY(b, launch_seed(b->prec, c->arena + P.bufs[P.tens[fin].buf].off, c->arena + P.bufs[P.adj_buf[fin]].off,
                                b->d_scales + b->scale_off[i], fin, s));
    }
    for (const Launch& l : b->blaunches) {
        switch (l.kind) {
            case L_GEMM:
                BHIP_TRY(b, launch_gemm(l.key, b->d_bgemm + l.begin, l.count, l.work, b->d_scales, b->d_maxparts, s));
                break;
            case L_REDUCE:
                BHIP_TRY(b, launch_reduce(l.key, b->d_reduce + l.begin, l.count, l.work, b->d_scales, s));
                break;
            case L_CORE_BWD:
                BHIP_TRY(b, launch_core_bwd(l.key, b->d_cbwd + l.begin, l.count, l.max_d, s));
                break;
        }
    }
    for (int i = 0; i < (int)b->ctxs.size(); ++i) {
        tn_ctx* c = b->ctxs[i];
        BHIP_TRY(b, launch_grad_inputs(b->prec, c->d_gin, (int)c->h_gin.size(), b->d_scales + b->scale_off[i],
                                       (double*)outs[i], s));
    }
    return TN_OK;
}

void free_batch(tn_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->bexec) (void)hipGraphExecDestroy(b->bexec);
    if (b->bgraph) (void)hipGraphDestroy(b->bgraph);
    b->exec = b->bexec = nullptr;
    b->graph = b->bgraph = nullptr;
    dfree(b->d_gemm);
    dfree(b->d_copy);
    dfree(b->d_core);
    dfree(b->d_scale);
    dfree(b->d_lanczos);
    dfree(b->d_glanczos);
    dfree(b->d_bgemm);
    dfree(b->d_reduce);
    dfree(b->d_cbwd);
    dfree(b->d_scales);
    dfree(b->d_maxparts);
    dfree(b->d_disc);
    dfree(b->d_tie);
    dfree(b->d_sweeps);
    dfree(b->d_result);
    if (b->h_result) (void)hipHostFree(b->h_result);
    b->h_result = nullptr;
    if (b->stream) (void)hipStreamDestroy(b->stream);
    b->stream = nullptr;
    for (hipStream_t& a : b->aux) {
        if (a) (void)hipStreamDestroy(a);
        a = nullptr;
    }
    for (hipEvent_t e : b->sync_ev) (void)hipEventDestroy(e);
    b->sync_ev.clear();
}

}  // namespace

extern "C" {

tn_status tn_batch_create(int32_t n, tn_ctx* const* ctxs, tn_batch** out) {
    if (!out || n < 1 || !ctxs) return TN_EINVAL;
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i]) return TN_EINVAL;
        if (!ctxs[i]->has_plan) return fail(ctxs[i], TN_ESTATE, "tn_batch_create: context without a plan");
    }
    const int dev = ctxs[0]->device, prec = ctxs[0]->plan.opts.precision;
    bool grad = true;
    for (int i = 0; i < n; ++i) {
        if (ctxs[i]->device != dev) return fail(ctxs[i], TN_EINVAL, "tn_batch_create: contexts on different devices");
        if (ctxs[i]->plan.opts.precision != prec)
            return fail(ctxs[i], TN_EINVAL, "tn_batch_create: contexts with different precisions");
        if (ctxs[i]->plan.opts.plain)
            return fail(ctxs[i], TN_EINVAL, "tn_batch_create: a context planned in the plain form");
        if (!ctxs[i]->h_kops.empty())
            return fail(ctxs[i], TN_EINVAL, "tn_batch_create: block-Krylov compressions are not merged into batches");
        if (!ctxs[i]->h_tsqr.empty())
            return fail(ctxs[i], TN_EINVAL, "tn_batch_create: TSQR R-factors are not merged into batches");
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return fail(ctxs[i], TN_EINVAL, "tn_batch_create: a context appears twice");
        grad = grad && ctxs[i]->plan.opts.grad && ctxs[i]->plan.n_segments <= 1;
    }
    (void)hipSetDevice(dev);
    tn_batch* b = new tn_batch();
    b->device = dev;
    b->prec = prec;
    b->grad = grad;
    b->ctxs.assign(ctxs, ctxs + n);
    for (tn_ctx* c : b->ctxs) {
        b->scale_off.push_back(b->n_scales);
        b->comp_off.push_back(b->n_comps);
        b->n_scales += (int64_t)c->plan.tens.size();
        b->n_comps += (int64_t)c->plan.comps.size();
        (void)hipStreamSynchronize(c->stream);
    }
    merge_forward(b);
    if (grad) merge_backward(b);
    auto bail = [&](tn_status s) {
        free_batch(b);
        delete b;
        return s;
    };
    tn_status s;
    if ((s = bupload(b, &b->d_gemm, b->h_gemm)) != TN_OK) return bail(s);
    if ((s = bupload(b, &b->d_copy, b->h_copy)) != TN_OK) return bail(s);
    if ((s = bupload(b, &b->d_core, b->h_core)) != TN_OK) return bail(s);
    if ((s = bupload(b, &b->d_scale, b->h_scale)) != TN_OK) return bail(s);
    if ((s = bupload(b, &b->d_lanczos, b->h_lanczos)) != TN_OK) return bail(s);
    if ((s = bupload(b, &b->d_glanczos, b->h_glanczos)) != TN_OK) return bail(s);
    if ((s = bupload(b, &b->d_bgemm, b->h_bgemm)) != TN_OK) return bail(s);
    if ((s = bupload(b, &b->d_reduce, b->h_reduce)) != TN_OK) return bail(s);
    if ((s = bupload(b, &b->d_cbwd, b->h_cbwd)) != TN_OK) return bail(s);
    const size_t nc = (size_t)std::max<int64_t>(1, b->n_comps);
    if (hipMalloc((void**)&b->d_scales, (size_t)std::max<int64_t>(1, b->n_scales) * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&b->d_maxparts, (size_t)b->max_parts * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&b->d_disc, nc * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&b->d_tie, nc * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void**)&b->d_sweeps, nc * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void**)&b->d_result, 4 * (size_t)n * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void**)&b->h_result, 4 * (size_t)n * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipMemset(b->d_sweeps, 0, nc * sizeof(int32_t)) != hipSuccess ||
        hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
        return bail(TN_ENOMEM);
    for (int i = 0; i < kLanes - 1; ++i)
        if (hipStreamCreateWithFlags(&b->aux[i], hipStreamNonBlocking) != hipSuccess) return bail(TN_EDEVICE);
    // capture the forward schedule once; replays evaluate every instance
    if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return bail(TN_EDEVICE);
    const tn_status es = enqueue_batch_forward(b);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(b->stream, &g);
    if (es != TN_OK || ce != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return bail(es != TN_OK ? es : TN_EDEVICE);
    }
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) return bail(TN_EDEVICE);
    *out = b;
    return TN_OK;
}

void tn_batch_destroy(tn_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    free_batch(b);
    delete b;
}

const char* tn_batch_last_error(const tn_batch* b) { return b ? b->err.c_str() : "null batch"; }

tn_status tn_batch_contract(tn_batch* b, double* mantissas, double* log10_exponents) {
    if (!b) return TN_EINVAL;
    (void)hipSetDevice(b->device);
    for (tn_ctx* c : b->ctxs) BHIP_TRY(b, hipStreamSynchronize(c->stream));
    BHIP_TRY(b, hipGraphLaunch(b->exec, b->stream));
    BHIP_TRY(b, hipMemcpyAsync(b->h_result, b->d_result, 4 * b->ctxs.size() * sizeof(double), hipMemcpyDeviceToHost,
                               b->stream));
    // hand each context its scales and compression statistics, so that tn_result, tn_grad and
    // tn_compress_stats work on it as after its own evaluation
    for (int i = 0; i < (int)b->ctxs.size(); ++i) {
        tn_ctx* c = b->ctxs[i];
        const size_t ns = c->plan.tens.size(), nc = c->plan.comps.size();
        BHIP_TRY(b, hipMemcpyAsync(c->d_scales, b->d_scales + b->scale_off[i], ns * sizeof(double),
                                   hipMemcpyDeviceToDevice, b->stream));
        if (nc) {
            BHIP_TRY(b, hipMemcpyAsync(c->d_disc, b->d_disc + b->comp_off[i], nc * sizeof(double),
                                       hipMemcpyDeviceToDevice, b->stream));
            BHIP_TRY(b, hipMemcpyAsync(c->d_tie, b->d_tie + b->comp_off[i], nc * sizeof(int32_t),
                                       hipMemcpyDeviceToDevice, b->stream));
            BHIP_TRY(b, hipMemcpyAsync(c->d_sweeps, b->d_sweeps + b->comp_off[i], nc * sizeof(int32_t),
                                       hipMemcpyDeviceToDevice, b->stream));
        }
    }
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    tn_status worst = TN_OK;
    for (int i = 0; i < (int)b->ctxs.size(); ++i) {
        tn_ctx* c = b->ctxs[i];
        const double* r = b->h_result + 4 * i;
        c->sign = r[0];
        c->lnz = r[1];
        c->flags = (int)r[2];
        c->evaluated = true;
        c->fwd_fresh = true;
        double m = 0.0, e = -INFINITY;
        tn_status st = TN_OK;
        if (c->flags & 2) st = fail(c, TN_ENUMERIC, "non-finite tensor entry");
        else if (c->flags & 4) st = fail(c, TN_ENUMERIC, "a Jacobi SVD did not converge within the sweep cap");
        else if ((c->flags & 1) || c->sign == 0.0) {
            c->sign = 0.0;
            c->lnz = -INFINITY;
            st = TN_ZERO;
        } else {
            const double l10 = c->lnz / std::log(10.0);
            e = std::floor(l10);
            m = std::pow(10.0, l10 - e);
            if (m >= 10.0) m /= 10.0;
            m *= c->sign;
        }
        if (mantissas) mantissas[i] = m;
        if (log10_exponents) log10_exponents[i] = e;
        if (st != TN_OK && st != TN_ZERO && worst == TN_OK) {
            worst = st;
            b->err = "instance " + std::to_string(i) + ": " + c->err;
        }
    }
    return worst;
}

tn_status tn_batch_grad(tn_batch* b, void* const* dlnz_ddata_dev) {
    if (!b) return TN_EINVAL;
    if (!b->grad)
        return bfail(b, TN_ESTATE,
                     "the batch's contexts were not all planned with opts.grad and a single segment "
                     "(a recomputed reverse pass runs per context: tn_grad)");
    if (!dlnz_ddata_dev) return bfail(b, TN_EINVAL, "null output array");
    for (size_t i = 0; i < b->ctxs.size(); ++i) {
        if (!dlnz_ddata_dev[i]) return bfail(b, TN_EINVAL, "null gradient buffer");
        if (!b->ctxs[i]->evaluated) return bfail(b, TN_ESTATE, "tn_batch_grad before tn_batch_contract");
        if (b->ctxs[i]->sign == 0.0) return bfail(b, TN_ZERO, "instance " + std::to_string(i) + " has Z = 0");
    }
    (void)hipSetDevice(b->device);
    std::vector<void*> want(dlnz_ddata_dev, dlnz_ddata_dev + b->ctxs.size());
    if (!b->bexec || want != b->bgrad_ptrs) {
        // (re)capture the reverse schedule for these output buffers
        if (b->bexec) (void)hipGraphExecDestroy(b->bexec);
        if (b->bgraph) (void)hipGraphDestroy(b->bgraph);
        b->bexec = nullptr;
        b->bgraph = nullptr;
        BHIP_TRY(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        const tn_status es = enqueue_batch_backward(b, want.data());
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(b->stream, &g);
        if (es != TN_OK || ce != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return es != TN_OK ? es : bfail(b, TN_EDEVICE, "graph capture of the reverse pass failed");
        }
        b->bgraph = g;
        BHIP_TRY(b, hipGraphInstantiate(&b->bexec, b->bgraph, nullptr, nullptr, 0));
        b->bgrad_ptrs = want;
    }
    BHIP_TRY(b, hipGraphLaunch(b->bexec, b->stream));
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    return TN_OK;
}

}  // extern "C"
