// Host planner: expands an ordered contraction tree into a static schedule.
//
// Algorithm 1 of arXiv:2206.07044 (section II.F) with early compression and
// r = 0 is traced on tensor shapes only: every CONTRACT and every COMPRESS
// it implies (section II.G: compressions follow from the contraction order)
// becomes a set of device steps with fixed shapes, fixed matricisation Views
// and fixed arena offsets.  Steps are levelled (a step's level is one more
// than the latest level of anything it reads) so that every level is a set
// of independent steps executed as a few grouped kernel launches.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "tn_internal.hpp"

namespace tn {

struct GraphSpec {
    int32_t n = 0, ne = 0;
    std::vector<int32_t> eu, ev, ed;
    std::vector<int64_t> offsets;   // n+1 element offsets of the input tensors
};

struct TreeOpts {
    int32_t chi = 0;
    double cutoff = 0.0;
    int32_t precision = 0;          // 0 = float64 tensors, 1 = float32, 2 = bfloat16
    int32_t jacobi_max_sweeps = 40;
    int64_t budget = 0;
    int32_t keep = 0;               // never reuse arena memory
    int32_t grad = 0;               // plan the reverse pass too
    int32_t plain = 0;              // one launch per step, no streams, no graph (the plain form)
    int32_t ordered = 0;            // contraction levels follow the tree order (memory of a sequential run)
    int32_t late = 0;               // late compression: bonds of i and j compressed before contracting them
    int32_t gauge_r = 0;            // tree-gauge distance r of every compression
    int32_t segments = 0;           // grad: forward levels in this many recomputed segments (<= 1: none;
                                    // -1: the count of smallest arena among a few candidates)
    int32_t rfactor = 0;            // R-factors of tall sides with D <= 64: 0 Gram + pivoted Cholesky, 1 TSQR
};

// One op of the Algorithm 1 expansion (same fields as the host-only describe call).
struct OpRec {
    int64_t kind, a, b, out, m, n, k, new_dim;
};

enum BufKind { BUF_INPUT = 0, BUF_TENSOR, BUF_GRAM, BUF_FACTOR, BUF_WORK, BUF_PROJ, BUF_BWD };

struct Buf {
    int64_t bytes = 0;
    int32_t lo = 0, hi = 0;         // first and last level that touch it
    int32_t kind = BUF_TENSOR;
    int64_t off = -1;               // byte offset in the arena
};

struct TensorVer {
    std::vector<int32_t> legs;      // edge ids, axis order (last = fastest)
    int64_t size = 1;
    int32_t buf = -1;
    int32_t level = 0;              // level of the producing step (0 = input)
    int32_t last_read = 0;
};

enum StepKind { ST_CONTRACT = 0, ST_GRAM, ST_COPY, ST_CORE, ST_ABSORB, ST_LANCZOS, ST_KRYLOV, ST_GAUGE, ST_TSQR };

// Tree-gauge steps (ST_GAUGE): 1 = apply a child's environment metric on one bond of a tensor (or of
// an earlier apply's output), W = X x_bond M, float64 into a buffer of the tensor's layout; 2 = the
// metric-weighted Gram X^T W over every leg but one bond (split-K partials, summed in place).
enum GaugeMode { GAUGE_APPLY = 1, GAUGE_GRAM = 2 };

// Gram steps of sides with D <= kGramNarrowMaxD run on the narrow-Gram kernel (512 rows per split)
constexpr int kGramNarrowMaxD = 64;

struct ViewSpec {                   // a View before arena addresses are known
    std::vector<int32_t> row_dims, col_dims;            // slowest..fastest
    std::vector<int64_t> row_strides, col_strides;
};

struct Step {
    int32_t kind = ST_CONTRACT;
    int32_t level = 0;
    // GEMM-like steps: A (M x K) . B (K x N) -> C
    int32_t in_a = -1, in_b = -1;   // tensor-version ids (or -1 for a projector operand)
    int32_t proj_buf = -1;          // ABSORB: projector buffer used as the dense operand
    int32_t proj_left = 0;          // ABSORB: 1 => A_mat . P_L, 0 => P_R . B_mat
    int32_t out_t = -1;             // produced tensor version (CONTRACT / ABSORB)
    int32_t out_buf = -1;           // GRAM partials / COPY factor
    int64_t M = 0, N = 0, K = 0;
    int32_t splits = 1, k_per_split = 0;
    ViewSpec va, vb;                // for COPY only va is used
    int32_t copy_rows = 0, copy_cols = 0;
    // GAUGE: mode, float64 operands held in buffers (A when it is an earlier apply's output, B the
    // metric or the applied tensor) and the output view of an apply
    int32_t gauge_mode = 0;
    int32_t a_buf = -1, b_buf = -1;
    ViewSpec vc;
    // TSQR: one output buffer and block count per pass (the last pass's buffer is out_buf, 1 block)
    std::vector<int32_t> tsqr_bufs, tsqr_blocks;
    // CORE
    int32_t comp = -1;              // compression index
    double flops = 0, bytes = 0;
};

struct Compression {
    int32_t a_ver_in, b_ver_in, a_ver_out, b_ver_out;
    // the bond: tree nodes a (P_L's side) and b, the edges it bundles in P_L's row order (slowest
    // first), the new edge that replaces them
    int32_t node_a, node_b, e_new;
    std::vector<int32_t> bond_edges;
    int64_t ma, D, mb;
    int32_t chi_new;
    int32_t side_a_buf, side_b_buf;     // Gram partials or explicit factor
    int32_t gram_a, gram_b;             // 1 if the side is a Gram
    int32_t splits_a, splits_b;
    int32_t rows_a, rows_b;             // explicit factor rows
    int32_t work_buf, pl_buf, pr_buf;
    int32_t core_step;
    int32_t lanczos;                    // 1: Golub-Kahan-Lanczos on A B (large D), 0: Gram + core
    int32_t glanczos;                   // 1: large D with an explicit side: Lanczos on F_X G_Y F_X^T
    int32_t x_is_b;                     // glanczos: the explicit side X is B
    int32_t s_min, s_max;               // Krylov steps (lanczos / glanczos)
    // block Krylov (large D with an explicit side X of n rows; the other side Y is read in place)
    int32_t krylov;
    int64_t kr_n, kr_my;                // rows of X and of Y
    int32_t kr_b, kr_s, kr_k, kr_full;  // block size, blocks, basis dimension, 1: the basis is all of R^n
    int32_t kr_splits, kr_splits2;      // split-K factors of Y^T U (b columns) and Y^T U2 (chi' columns)
};

// Large-D compressions with one explicit side use the block-Krylov path from this bond size on.
constexpr int64_t kKrylovMinD = 512;

// Byte offsets of a block-Krylov compression's workspace (see the chain in tn_krylov.cpp).
struct KrylovLayout {
    int64_t q, ws, wo, wx, t1, t1t, u, t2p, hc, g, m, h, ik, core, plc, prc, qp, px, pxt, pyp, nrm, e;
    int64_t bytes;
};
KrylovLayout krylov_layout(int64_t n, int64_t D, int64_t my, int64_t nw, int64_t b, int64_t k, int full,
                           int64_t splits, int64_t splits2, int64_t w);

// Compressions with D above this use Golub-Kahan-Lanczos on A B instead of Gram matrices,
// unless the matricised tensors are much taller than D.
constexpr int64_t kLanczosMinD = 65;
// Largest core the block Jacobi handles (the core kernel's kBJRows).
constexpr int64_t kBlockJacobiMaxD = 256;
constexpr int64_t kLanczosMaxRowsPerD = 256;

// One step of the reverse pass (levels count from the seed of the final scalar).
enum BStepKind { BS_GEMM = 0, BS_REDUCE, BS_CORE_BWD, BS_SEED };

struct BStep {
    int32_t kind = BS_GEMM;
    int32_t level = 0;
    // BS_GEMM: C(view vc) = [C +] f * A(view va) . B(view vb), f = 1/(s[scale_a] s[scale_b]);
    //          partial: split-K float64 partials (dense M x N per split) into c_buf instead
    // BS_REDUCE: C(view vc) = f * sum over splits of a_buf (float64 partials, dense M x N)
    int32_t a_buf = -1, b_buf = -1, c_buf = -1;   // arena buffers (forward ones or reverse-pass ones)
    int64_t c_off = 0;                             // byte offset of C inside c_buf
    int32_t scale_a = -1, scale_b = -1;
    int32_t accumulate = 0, partial = 0;
    int32_t splits = 1, k_per_split = 0;
    int64_t M = 0, N = 0, K = 0;
    ViewSpec va, vb, vc;
    // BS_CORE_BWD
    int32_t comp = -1;
    double flops = 0, bytes = 0;
};

// Reverse-pass buffers of one compression.
struct CompBwd {
    int32_t h_buf = -1;             // H_A partials then H_B partials (float64, D x chi' each)
    int32_t splits_a = 1, splits_b = 1;
    int32_t na_buf = -1, nb_buf = -1;   // N_A, N_B (D x D, compute precision)
    int32_t work_buf = -1;          // core-space workspace (float64)
};

struct Plan {
    GraphSpec g;
    TreeOpts opts;
    std::vector<TensorVer> tens;        // creation order == scale-slot order
    std::vector<Buf> bufs;
    std::vector<Step> steps;
    std::vector<Compression> comps;
    std::vector<OpRec> ops;
    int32_t n_levels = 0;
    int32_t final_tensor = -1;
    int64_t arena_bytes = 0;
    int64_t max_parts = 0;              // per-level per-tile max slots needed
    double fwd_flops = 0, fwd_bytes = 0;
    int32_t elem_size = 8;
    // reverse pass (opts.grad)
    std::vector<int32_t> adj_buf;       // per tensor version: its adjoint (compute precision)
    std::vector<BStep> bsteps;
    std::vector<CompBwd> cbwd;
    int32_t n_blevels = 0;
    double bwd_flops = 0, bwd_bytes = 0;
    // checkpointed recomputation (opts.segments): segment s holds forward levels
    // [seg_begin[s], seg_begin[s+1]); the reverse pass takes the segments last to first, re-running
    // the forward launches of a segment (all but the last, right after a forward evaluation) and
    // then its reverse levels up to seg_bend[s].  One segment: no recomputation.
    int32_t n_segments = 1;
    std::vector<int32_t> seg_begin, seg_bend;
    std::vector<uint8_t> seg_recompute;  // 1 if the segment has reverse steps, so is re-run
    double recompute_flops = 0;          // forward flops of segments 0 .. S-2 that are re-run
    int64_t checkpoint_bytes = 0;        // forward buffers kept across a segment boundary
};

// Validate the graph (returns "" or an error message).
std::string check_graph(const GraphSpec& g);
// Expand Algorithm 1 on shapes.  With `shapes_only` nothing but `ops` is built.
std::string build_plan(const GraphSpec& g, const int32_t* pi, const int32_t* pj, int32_t n_steps,
                       const TreeOpts& o, bool shapes_only, Plan* out);
// Convert a ViewSpec to a device View (merges adjacent legs, checks limits).
std::string make_view(const ViewSpec& s, View* v);

}  // namespace tn
