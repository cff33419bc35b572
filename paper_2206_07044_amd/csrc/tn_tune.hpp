// Tile selection of the tensor GEMMs: a table over shape classes, the built-in defaults, and the
// measurement primitive behind the autotuner (tn_gemm_tiles_get / _set, tn_gemm_tune).
#pragma once

#include <stdint.h>

namespace tn {

// Class of a tensor GEMM whose short side (M or N) is at most 32 and whose long side exceeds 64:
// (((prec * 2 + wide) * 2 + short32) * 3 + kclass) * 2 + long_unit.  -1 for other GEMMs (64 x 64).
int gemm_class(int prec, int64_t M, int64_t N, int64_t K, bool a_rows_unit, bool b_cols_unit);
constexpr int kGemmClasses = 72;
// 1 if tile variant v (GemmVariant) is correct and sensible for class c.
bool gemm_variant_allowed(int c, int v);
// The tile variant for a GEMM (the installed table for classed GEMMs, else 64 x 64).
int pick_gemm_tile(int prec, int64_t M, int64_t N, int64_t K, bool a_rows_unit, bool b_cols_unit);
// The representative shape a class is measured on.
void gemm_class_shape(int c, int* prec, int64_t* M, int64_t* N, int64_t* K, bool* a_rows_unit, bool* b_cols_unit);

}  // namespace tn
