// Block-Krylov truncated SVD of a large bond with one explicit side (see tn_krylov.cpp).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "tn_internal.hpp"
#include "tn_plan.hpp"

namespace tn {

// One step of a chain: a grouped launch of one kernel over the descriptors [begin, begin + count)
// of its kind's array.
enum KOpKind { KO_GEMM = 0, KO_REDUCE, KO_SMALL, KO_CHOL, KO_CORE, KO_CHECK };
struct KOp {
    int kind = 0;
    int key = 0;          // GEMM: GemmKey; SMALL: dtype of SM_CAST (0/1/2); CORE: 1 = LDS variant
    int64_t begin = 0;
    int count = 0;
    int64_t work = 0;     // tiles / elements
    int max_d = 0;        // CORE: largest D
};

struct KrylovShape {
    int64_t n, D, my, nw;
    int b, s, k, full, splits, splits2;
};

// One compression of a group that shares a shape.
struct KrylovJob {
    const double* fx;     // explicit factor of side X (n x D, row-major, float64, already divided by its scale)
    const void* y;        // the tensor of side Y (tensor dtype)
    View vy, vyt;         // Y (m_Y x D) and Y^T (D x m_Y) through the tensor's layout
    int32_t y_scale;      // scale index of Y
    char* ws;             // workspace (krylov_layout)
    void* p_left;         // D x chi' (tensor dtype)
    void* p_right;        // chi' x D
    int x_is_b;
    int32_t stat, kmin;
    double cutoff;
};

struct KrylovSink {
    std::vector<GemmDesc>* gemm;
    std::vector<ReduceDesc>* reduce;
    std::vector<SmallDesc>* small;
    std::vector<CholInvDesc>* chol;
    std::vector<CoreDesc>* core;
    std::vector<KrylovCheckDesc>* check;
    std::vector<KOp>* ops;
};

// Largest accepted Ritz-pair residual ||S z - s^2 z|| relative to s_1^2.
constexpr double kKrylovResidualTol = 1e-8;

// Append the chain of a group of same-shape compressions (prec: tensor dtype 0/1/2); "" or an error.
std::string krylov_chain(const KrylovShape& sh, int prec, const std::vector<KrylovJob>& jobs, const KrylovSink& out);

}  // namespace tn
