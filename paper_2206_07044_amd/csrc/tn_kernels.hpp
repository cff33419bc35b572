// Launch wrappers for the device kernels (tn_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "tn_internal.hpp"
#include "../../include/tn.h"

namespace tn {

// GEMM_GRAM_NARROW_*: forward Gram X^T X of a side with D <= 64 (by input type), float64 result
// GEMM_*_X_F64: A in float32 / bfloat16, B in float64, product and result in float64
enum GemmKey { GEMM_F64 = 0, GEMM_F32 = 1, GEMM_F32_TO_F64 = 2, GEMM_BF16 = 3, GEMM_BF16_TO_F64 = 4,
               GEMM_GRAM_NARROW_F64 = 5, GEMM_GRAM_NARROW_F32 = 6, GEMM_GRAM_NARROW_BF16 = 7, GEMM_F32_X_F64 = 8,
               GEMM_BF16_X_F64 = 9 };

// Tile shapes of the tensor GEMMs (GEMM_F64 / GEMM_F32 / GEMM_BF16, single split): a launch key is
// GemmKey + kGemmVariantStride * variant.  The other keys take the 64 x 64 tile only.
// GV_TALL* / GV_WIDE*: the skinny kernel (no MFMA): N (resp. M) at most 16 or 32, K at most
// kSkinnyGemmMaxK, 256 rows (columns) of C per workgroup.
enum GemmVariant {
    GV_64x64 = 0, GV_256x16 = 1, GV_16x256 = 2, GV_128x32 = 3, GV_32x128 = 4,
    GV_TALL16 = 5, GV_TALL32 = 6, GV_WIDE16 = 7, GV_WIDE32 = 8, GV_COUNT = 9
};
constexpr int kGemmVariantStride = 16;
constexpr int kSkinnyGemmMaxK = 64;
inline void gemm_tile(int variant, int* bm, int* bn) {
    static const int dims[GV_COUNT][2] = {{64, 64}, {256, 16}, {16, 256}, {128, 32}, {32, 128},
                                          {256, 16}, {256, 32}, {16, 256}, {32, 256}};
    *bm = dims[variant][0];
    *bn = dims[variant][1];
}
// The variant of a tensor GEMM comes from the tile table (tn_tune.hpp).

constexpr int kCoreLdsMaxD = 64;
constexpr int kLanczosMaxSteps = 512;     // cap on Krylov steps per compression
constexpr int kLanczosLdsBytes = 150 * 1024;   // dynamic LDS for the small SVD (static use is ~4.3 KB)

void init_kernel_attrs();
hipError_t launch_gemm(int dtype_key, const GemmDesc* descs, int ndesc, int64_t tiles, const double* scales,
                       double* maxparts, hipStream_t s);
hipError_t launch_copy(int prec, const CopyDesc* descs, int ndesc, int64_t total, const double* scales,
                       hipStream_t s);
// One TSQR pass over `blocks` row blocks; prec is the input's dtype (0 float64, 1 float32, 2 bf16).
hipError_t launch_tsqr(int prec, const TsqrDesc* descs, int ndesc, int64_t blocks, const double* scales,
                       hipStream_t s);
size_t core_lds_bytes(int max_d);
hipError_t launch_core(int lds, int prec, const CoreDesc* descs, int ndesc, int max_d, int max_sweeps,
                       double* disc, int32_t* tie, int32_t* sweeps, hipStream_t s);
size_t lanczos_lds_bytes(int s_max);
// Kernel launches one launch_core call issues (the block-Jacobi cores issue one per tournament round).
int core_launch_count(int lds, int max_d, int max_sweeps);
hipError_t launch_lanczos(int prec, const LanczosDesc* descs, int ndesc, int s_max, const double* scales,
                          int max_sweeps, double* disc, int32_t* tie, int32_t* sweeps, hipStream_t s);
hipError_t launch_gram_lanczos(int prec, const GLanczosDesc* descs, int ndesc, int max_sweeps, double* disc,
                               int32_t* tie, int32_t* sweeps, hipStream_t s);
hipError_t launch_scale_finalize(const ScaleDesc* descs, int n, const double* maxparts, double* scales,
                                 hipStream_t s);
hipError_t launch_inputs(int prec, const InputDesc* descs, int n, const double* staging, double* scales,
                         hipStream_t s);
hipError_t launch_reduce(int prec, const ReduceDesc* descs, int ndesc, int64_t total, const double* scales,
                         hipStream_t s);
hipError_t launch_core_bwd(int prec, const CoreBwdDesc* descs, int ndesc, int max_d, hipStream_t s);
hipError_t launch_seed(int prec, const void* final_ptr, void* adj_final, const double* scales, int final_index,
                       hipStream_t s);
hipError_t launch_grad_inputs(int prec, const InputDesc* descs, int n, const double* scales, double* out,
                              hipStream_t s);
hipError_t launch_ising_values(const IsingGraph& g, double beta, const double* J, double* data, int64_t total,
                               hipStream_t s);
hipError_t launch_ising_grad(const IsingGraph& g, double beta, const double* J, const double* dlnz_ddata,
                             double* dlnz_dJ, hipStream_t s);
// Small dense float64 operations (SmallOp); `prec` is the dtype of SM_CAST destinations.
hipError_t launch_small(int prec, const SmallDesc* descs, int ndesc, int64_t total, hipStream_t s);
// One workgroup per compression: Ritz-pair residuals; non-converged compressions get a negative
// sweep count (the evaluation then reports TN_ENUMERIC).
hipError_t launch_krylov_check(const KrylovCheckDesc* descs, int ndesc, int32_t* sweeps, hipStream_t s);
// One 64-lane wave per block: the orthonormalising factor M of W from G = W^T W.
hipError_t launch_cholinv(const CholInvDesc* descs, int ndesc, hipStream_t s);
// One 8-byte wall-clock stamp (100 MHz) written by the device when the stream reaches it.
hipError_t launch_stamp(unsigned long long* dst, hipStream_t s);
hipError_t launch_result(int prec, const double* scales, int n_scales, const void* final_ptr, const int32_t* sweeps,
                         int n_comp, double* result, hipStream_t s);

}  // namespace tn
