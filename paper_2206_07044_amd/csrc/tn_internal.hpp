// Internal structures shared by the host planner and the device kernels.
//
// A tensor lives in device memory as a dense row-major array whose axes are
// its edges in "leg order".  Every matrix that a kernel reads (a
// matricisation, Fig. "tensor primitives" A) is described by a View: the
// element (r, c) sits at  sum_l idx_l(r) * rstride_l + sum_l idx_l(c) * cstride_l,
// where idx_l(r) is the mixed-radix digit of r over the row legs (last leg
// fastest).  Gathers through Views fuse the permutation into the loads, so
// no tensor is ever transposed in memory.
#pragma once

#include <stdint.h>

#ifndef __HIPCC__
#define TN_HD
#else
#define TN_HD __host__ __device__
#endif

namespace tn {

constexpr int kMaxLegs = 16;

// 32-bit division by a runtime constant via multiply-high (round-up method):
// q = (umulhi(n, mul) + n) >> shr, exact for n < 2^31 and 1 <= d < 2^31.
struct FastDiv {
    uint32_t d;
    uint32_t mul;
    uint32_t shr;
};

inline FastDiv make_fastdiv(uint32_t d) {
    FastDiv f;
    f.d = d;
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    f.shr = l;
    f.mul = (uint32_t)((((1ull << 32) * ((1ull << l) - d)) / d) + 1);
    return f;
}

TN_HD inline uint32_t fd_div(uint32_t n, const FastDiv& f) {
#ifdef __HIP_DEVICE_COMPILE__
    uint32_t hi = __umulhi(n, f.mul);
#else
    uint32_t hi = (uint32_t)(((uint64_t)n * f.mul) >> 32);
#endif
    return (uint32_t)(((uint64_t)hi + n) >> f.shr);
}

// One side (rows or columns) of a matricisation.  Legs are stored fastest
// first: leg 0 is the least significant digit.
struct Axis {
    int32_t n;                   // number of legs (0 => single index 0)
    int32_t pad;
    FastDiv div[kMaxLegs];
    uint32_t stride[kMaxLegs];   // element stride of each leg in the tensor
};

TN_HD inline uint32_t axis_offset(const Axis& a, uint32_t r) {
    uint32_t off = 0;
    for (int l = 0; l < a.n; ++l) {
        uint32_t q = fd_div(r, a.div[l]);
        off += (r - q * a.div[l].d) * a.stride[l];
        r = q;
    }
    return off;
}

struct View {
    Axis row;
    Axis col;
    int32_t row_unit;            // 1 if the fastest row leg has stride 1
    int32_t col_unit;            // 1 if the fastest column leg has stride 1
};

enum GemmMode : int32_t {
    GEMM_TENSOR = 0,   // C (M x N, row-major) = fA*fB * A.B ; writes per-tile max |C|
    GEMM_GRAM = 1,     // C[split] (M x N, float64) = fA*fB * A.B over one K range
    GEMM_ADJ = 2,      // C(view vc) = [C +] fA*fB * A.B  (reverse pass; no tile max)
};

// C = op(A) . op(B) with A an (M x K) view and B a (K x N) view.
struct GemmDesc {
    const void* A;
    const void* B;
    void* C;
    int64_t tile_begin;          // first linear tile of this op in the grouped launch
    int32_t M, N, K;
    int32_t mode;                // GemmMode
    int32_t tiles_m, tiles_n, splits;
    int32_t k_per_split;         // K range per split (multiple of the K tile)
    int32_t scale_a, scale_b;    // indices into the tensor-scale array (-1: factor 1)
    int32_t square_a;            // GRAM: factor is 1/s_a^2 (A and B are the same tensor)
    int32_t maxpart;             // TENSOR: index of the first per-tile max slot
    int32_t accumulate;          // ADJ: add to C instead of overwriting it
    int32_t pad;
    View va;                     // A: rows = M, cols = K
    View vb;                     // B: rows = K, cols = N
    View vc;                     // ADJ: C, rows = M, cols = N
};

// Reverse pass: C(view vc) = f * sum over splits of dense float64 partials (M x N each).
struct ReduceDesc {
    const double* part;
    void* out;                   // compute precision
    int64_t elem_begin;          // first linear element of this op in the grouped launch
    int32_t M, N, splits;
    int32_t scale_a, scale_b;    // f = 1/(s[scale_a] s[scale_b]) (-1: factor 1)
    int32_t pad;
    View vc;
};

// Reverse pass of one compression in the space of its core (see core_bwd_kernel).
struct CoreBwdDesc {
    const double* work;          // the forward core workspace (R~_A, R~_B, W, V, sigma, order, ranks)
    const double* h;             // H_A partials (splits_a x D x chi'), then H_B partials (splits_b x D x chi')
    double* ws;                  // float64 workspace
    void* n_a;                   // N_A (D x D, compute precision)
    void* n_b;                   // N_B
    double cutoff;
    int32_t splits_a, splits_b;
    int32_t D, chi_new;
};

// Gather-copy: dst (rows x cols, row-major float64) = src(view) / s.
struct CopyDesc {
    const void* src;
    double* dst;
    int64_t elem_begin;          // first linear element of this op in the grouped launch
    int32_t rows, cols;
    int32_t scale;               // tensor-scale index
    int32_t transpose;           // 1: write dst as (cols x rows)
    View v;
};

// One bond compression's small dense part: reduced factors, core SVD, projectors.
struct CoreDesc {
    // Side A: either a split-K Gram (gram_a != null, D x D partials) or an explicit
    // factor R~_A (rows_a x D, row-major) with R~_A^T R~_A = A^T A.
    const double* gram_a;
    const double* gram_b;
    const double* fac_a;
    const double* fac_b;
    int32_t splits_a, splits_b;
    int32_t rows_a, rows_b;      // rows of the explicit factors (when no Gram)
    int32_t D;                   // bond size being compressed
    int32_t chi_new;             // static new bond dimension chi'
    double cutoff;
    double* work;                // float64 workspace (layout fixed by the kernel)
    void* p_left;                // D x chi' projector in the tensor dtype
    void* p_right;               // chi' x D projector in the tensor dtype
    int32_t stat;                // index into the per-compression stats arrays
    int32_t kmin;                // min(k_A, k_B): number of singular values of the structural core
    int32_t keep_out;            // LDS variant: leave R~_A, R~_B, W, V in the workspace (reverse pass)
    int32_t pad;
};

// One pass of a tall-skinny QR (TSQR) of a (rows x D) matrix read through a View: blocks of
// tsqr_block_rows(D) rows, each block's R (Householder, float64) written to dst as a D x D
// row-major matrix (upper triangular; rows beyond the block's own count are zero).  The next
// pass takes the stacked R's as its input, until one block remains.
struct TsqrDesc {
    const void* src;             // pass 0: the tensor (its dtype); later passes: float64
    double* dst;                 // nblk x D x D
    int64_t blk_begin;           // first block of this op in the grouped launch
    int32_t rows, D, nblk;
    int32_t scale;               // tensor-scale index applied as 1/s on load (-1: none)
    View v;                      // rows x D
};
constexpr int kTsqrElems = 16384;   // float64 entries of one block in LDS (128 KiB)
TN_HD inline int tsqr_block_rows(int D) { return kTsqrElems / (D > 0 ? D : 1); }

// Large-core compression by Golub-Kahan-Lanczos on M = (A/s_a)(B/s_b) read through Views.
struct LanczosDesc {
    const void* A;               // tensor a
    const void* B;               // tensor b
    double* work;                // float64 workspace (layout fixed by the kernel)
    void* p_left;                // D x chi' projector in the tensor dtype
    void* p_right;               // chi' x D projector in the tensor dtype
    double cutoff;
    int32_t ma, mb, D, chi_new;
    int32_t s_min, s_max;        // Krylov steps before the first convergence check / at most
    int32_t scale_a, scale_b;
    int32_t stat, kmin;
    View va;                     // A_mat: rows = free legs of a, cols = shared legs
    View vb;                     // B_mat: rows = shared legs, cols = free legs of b
    const double* gram_a;        // A_mat^T A_mat / s_a^2 (D x D), for ||A B||_F^2 = <G_A, G_B>
    const double* gram_b;        // B_mat B_mat^T / s_b^2 (D x D)
};

// Large-core compression with an explicit side X: symmetric Lanczos on F_X G_Y F_X^T.
struct GLanczosDesc {
    const double* fx;            // explicit factor of side X (n x D, row-major)
    const double* gram_y;        // summed Gram of side Y (D x D), or null
    const double* fy;            // explicit factor of side Y (my x D) when it has no Gram
    double* work;                // on entry: S (n x n) then T1 (D x n, or n x my), then scratch
    void* p_left;                // D x chi'
    void* p_right;               // chi' x D
    double cutoff;
    int32_t n, my, D, chi_new;
    int32_t splits_y, x_is_b;    // x_is_b: X is the B side (operator M^T M), else A (M M^T)
    int32_t s_min, s_max;
    int32_t stat, kmin;
};

// Small dense float64 operations of the block-Krylov compressions (one thread per element of
// the destination).
enum SmallOp : int32_t {
    SM_RANDOM = 0,     // dst = uniform in [-1, 1) from a counter-based hash of (seed, element)
    SM_COPY = 1,       // dst = src (transposed if `transpose`)
    SM_NEG = 2,        // dst = -src (in place allowed)
    SM_SYM = 3,        // dst (square) = (dst + dst^T) / 2, in place
    SM_COLNORM2 = 4,   // dst[0, c] = sum over src_rows rows of src[r, c]^2
    SM_COLSCALE = 5,   // dst[r, c] *= src[c]
    SM_IDENTITY = 6,   // dst = I
    SM_CAST = 7,       // dst (tensor dtype of the launch) = src (transposed if `transpose`)
};

struct SmallDesc {
    const double* src;
    void* dst;
    int64_t elem_begin;          // first linear element of this op in the grouped launch
    int32_t rows, cols;          // the destination's shape
    int32_t src_ld, dst_ld;      // row strides in elements
    int32_t op;                  // SmallOp
    int32_t transpose;
    uint32_t seed;
    int32_t src_rows;            // COLNORM2
};

// Convergence check of a block-Krylov compression's kept Ritz pairs: with QP = Z s^-1/2 (Z the
// Ritz vectors), nrm[i] = 1 / s_i (0 for a masked pair) and E = F_X P_Y = S Z s^-3/2, the
// residual of pair i is ||S z_i - s_i^2 z_i|| = ||E_i - s_i QP_i|| s_i^(3/2); a pair whose
// residual exceeds tol * s_1^2 marks the compression as not converged.
struct KrylovCheckDesc {
    const double* e;             // n x nw
    const double* qp;            // n x nw
    const double* nrm;           // nw
    int32_t n, nw;
    int32_t stat;
    int32_t pad;
    double tol;
};

// Orthonormalising factor of a block of b <= 64 columns from its Gram G = W^T W: pivoted
// Cholesky P^T G P = R^T R stopped at pivots <= 1e-14 of the largest diagonal entry, and
// M = P R^-1 (zero columns beyond the rank), so that W M has orthonormal columns.
struct CholInvDesc {
    const double* g;             // b x b, row-major
    double* m;                   // b x b, row-major
    int32_t b;
    int32_t pad;
};

// Upload of one input tensor: float64 staging -> arena (converted to the tensor dtype).
struct InputDesc {
    void* dst;
    int64_t src_off;
    int64_t count;
    int32_t tensor;
    int32_t pad;
};

// Ising model on a graph whose edges all have dimension 2 (coupling map and its adjoint).
struct IsingGraph {
    const int32_t* inc_off;      // n+1 offsets into inc_edge
    const int32_t* inc_edge;     // incident edges of each vertex, ascending (= its axis order)
    const int32_t* edge_u;       // lower endpoint of each edge
    const int32_t* edge_v;
    const int64_t* data_off;     // n+1 element offsets of the tensors
    int32_t n, ne;
};

// Per-tensor scale finalisation: s = max over the tensor's per-tile maxima.
struct ScaleDesc {
    int32_t maxpart;             // first per-tile max slot
    int32_t nparts;
    int32_t tensor;              // tensor-scale index to write
    int32_t pad;
};

}  // namespace tn
