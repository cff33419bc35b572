// Device kernels for gfx950 (MI355X).
//
// * gemm_grouped  — one launch runs every GEMM-shaped step of a schedule level:
//   pairwise contractions (Fig. "tensor primitives" B), the Gram matrices that
//   stand in for the R-factors of the QR-reduced compression (section II.C),
//   and the projector re-absorptions A P_L, P_R B (SI section B).  Operands are
//   read through Views, so the permutation of the matricisation is fused into
//   the LDS staging; the product runs on MFMA (v_mfma_f64_16x16x4f64 or
//   v_mfma_f32_16x16x4f32).  The epilogue applies the pending scales of the
//   inputs and records the tile's largest |value| for the running exponent.
// * core_kernel   — one workgroup per bond compression: reduced factors from
//   the Gram matrices (pivoted Cholesky), R_A R_B, its one-sided Jacobi SVD,
//   truncation to chi' and the projectors P_L = R_B V s^-1/2, P_R = s^-1/2 U^T R_A.
// * scale / result kernels — the running log-scale exponent.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "tn_internal.hpp"
#include "tn_kernels.hpp"

namespace tn {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

// bfloat16 storage: the upper 16 bits of an IEEE binary32 (8 exponent, 7 fraction bits).
// float -> bf16 rounds to nearest, ties to even; NaN stays NaN.
struct bf16 {
    uint16_t bits;
    bf16() = default;
    __device__ explicit bf16(float f) : bits(round(f)) {}
    __device__ explicit bf16(double d) : bits(round((float)d)) {}
    __device__ explicit bf16(int i) : bits(round((float)i)) {}
    __device__ explicit operator float() const { return __uint_as_float((uint32_t)bits << 16); }
    __device__ explicit operator double() const { return (double)__uint_as_float((uint32_t)bits << 16); }
    __device__ static uint16_t round(float f) {
        const uint32_t u = __float_as_uint(f);
        if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
        return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
    }
};

template <typename Tc>
struct Mma;
// Operands: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16].
// Result element r of lane l is D[row(l, r)][l % 16]; the row mapping differs
// between the float64 and float32 instructions (checked on gfx950).
template <>
struct Mma<double> {
    using acc = v4d;
    static constexpr int kK = 4;
    __device__ static inline acc run(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mma<float> {
    using acc = v4f;
    static constexpr int kK = 4;
    __device__ static inline acc run(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
// bfloat16 inputs, float32 accumulation, K = 16 per instruction: lane l supplies
// A[l % 16][4 (l / 16) + j] and B[4 (l / 16) + j][l % 16], j = 0..3; the result layout is the
// float32 one (checked on gfx950).
template <>
struct Mma<bf16> {
    using acc = v4f;
    static constexpr int kK = 16;
    __device__ static inline acc run(v4s a, v4s b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
    }
    __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

__device__ inline double inv_scale(const double* scales, int idx) {
    if (idx < 0) return 1.0;
    double s = scales[idx];
    return s > 0.0 ? 1.0 / s : 0.0;
}

// A pointer into LDS with its address space in the type, for helpers that are also called on
// global memory: the compiler then emits LDS instructions where a generic pointer would give flat
// ones.
typedef __attribute__((address_space(3))) double lds_double;
typedef lds_double* LdsPtr;

// Wave reductions with DPP: xor-1 and xor-2 quad permutes, then half-row and row mirrors
// leave every lane holding its 16-lane row's total; the four row totals are read with
// readlane and combined in a fixed order, so every lane gets the same, deterministic value.
template <int kCtrl>
__device__ inline double dpp_mov(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), kCtrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), kCtrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ inline double read_lane(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// value of v in lane src (src uniform across the wave)
__device__ inline double bcast(double v, int src) {
    const unsigned long long b = __double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, src);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), src);
    return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}

__device__ inline double wave_sum(double v) {
    v += dpp_mov<0xB1>(v);    // quad_perm(1,0,3,2)
    v += dpp_mov<0x4E>(v);    // quad_perm(2,3,0,1)
    v += dpp_mov<0x141>(v);   // row_half_mirror
    v += dpp_mov<0x140>(v);   // row_mirror
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

__device__ inline double wave_max(double v) {
    v = fmax(v, dpp_mov<0xB1>(v));
    v = fmax(v, dpp_mov<0x4E>(v));
    v = fmax(v, dpp_mov<0x141>(v));
    v = fmax(v, dpp_mov<0x140>(v));
    return fmax(fmax(read_lane(v, 0), read_lane(v, 16)), fmax(read_lane(v, 32), read_lane(v, 48)));
}

// ------------------------------------------------------------------------------------------
// Grouped gather GEMM
// ------------------------------------------------------------------------------------------
constexpr int kBK = 16, kGemmThreads = 256;

// Tile shapes (BM x BN) of the grouped GEMM; GemmVariant (tn_kernels.hpp) picks one per GEMM.
// Four waves; square tiles put them 2 x 2, tall or wide ones 4 x 1 or 1 x 4.  Each wave owns
// (BM / WGM) x (BN / WGN) of the tile as 16 x 16 MFMA blocks.  Skinny tiles (256 x 16, 16 x 256)
// give the re-absorptions by a chi-column projector and the contractions over one small bond
// whole 16-wide sides instead of a quarter of a 64-wide one, and four times the rows per
// workgroup.
template <int BM, int BN>
struct TileShape {
    static constexpr int WGM = BM == BN ? 2 : (BM > BN ? 4 : 1);
    static constexpr int WGN = 4 / WGM;
    static constexpr int FM = BM / WGM / 16, FN = BN / WGN / 16;   // MFMA blocks per wave
    static constexpr int EA = BM * kBK / kGemmThreads, EB = BN * kBK / kGemmThreads;   // staged per thread
    static_assert(FM >= 1 && FN >= 1 && EA >= 1 && EB >= 1, "tile shape");
};

// TinB: element type of B (the same as A's except for the block-Krylov passes, where a float32 or
// bfloat16 tensor meets float64 vectors and the product is formed in float64)
template <typename Tin, typename Tc, typename Tout, typename TinB = Tin, int BM = 64, int BN = 64>
__global__ __launch_bounds__(kGemmThreads) void gemm_grouped(const GemmDesc* __restrict__ descs, int ndesc,
                                                             const double* __restrict__ scales,
                                                             double* __restrict__ maxparts, int64_t tile0) {
    using TS = TileShape<BM, BN>;
    constexpr int EA = TS::EA, EB = TS::EB, FM = TS::FM, FN = TS::FN;
    __shared__ Tc As[kBK][BM + 2];
    __shared__ Tc Bs[kBK][BN + 2];
    __shared__ double wmax[kGemmThreads / 64];

    const int tid = threadIdx.x;
    const int64_t tile = tile0 + blockIdx.x;
    int lo = 0, hi = ndesc - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (descs[mid].tile_begin <= tile) lo = mid;
        else hi = mid - 1;
    }
    const GemmDesc& d = descs[lo];
    const int M = d.M, N = d.N, K = d.K;
    const int per_split = d.tiles_m * d.tiles_n;
    const int local = (int)(tile - d.tile_begin);
    const int split = local / per_split;
    const int rem = local - split * per_split;
    const int tm = rem / d.tiles_n;
    const int tn_ = rem - tm * d.tiles_n;
    const int m0 = tm * BM, n0 = tn_ * BN;
    const int k_begin = split * d.k_per_split;
    const int k_end = min(K, k_begin + d.k_per_split);

    const Tin* __restrict__ A = (const Tin*)d.A;
    const TinB* __restrict__ B = (const TinB*)d.B;

    // per-thread fixed coordinates of the EA A and EB B elements it stages
    const bool a_mfast = d.va.row_unit != 0;
    const bool b_nfast = d.vb.col_unit != 0;
    int a_m[EA], a_k[EA], b_k[EB], b_n[EB];
    uint32_t a_off[EA], b_off[EB];
    bool a_ok[EA], b_ok[EB];
#pragma unroll
    for (int i = 0; i < EA; ++i) {
        const int e = tid + kGemmThreads * i;
        if (a_mfast) { a_m[i] = e % BM; a_k[i] = e / BM; }
        else { a_k[i] = e % kBK; a_m[i] = e / kBK; }
        const int gm = m0 + a_m[i];
        a_ok[i] = gm < M;
        a_off[i] = a_ok[i] ? axis_offset(d.va.row, (uint32_t)gm) : 0u;
    }
#pragma unroll
    for (int i = 0; i < EB; ++i) {
        const int e = tid + kGemmThreads * i;
        if (b_nfast) { b_n[i] = e % BN; b_k[i] = e / BN; }
        else { b_k[i] = e % kBK; b_n[i] = e / kBK; }
        const int gn = n0 + b_n[i];
        b_ok[i] = gn < N;
        b_off[i] = b_ok[i] ? axis_offset(d.vb.col, (uint32_t)gn) : 0u;
    }

    // K offsets of the current and next chunk, decomposed once per chunk (not per element)
    __shared__ uint32_t koff_a[2][kBK], koff_b[2][kBK];
    auto fill_koff = [&](int buf, int kc) {
        if (tid < kBK) {
            const int gk = kc + tid;
            koff_a[buf][tid] = gk < k_end ? axis_offset(d.va.col, (uint32_t)gk) : 0u;
        } else if (tid < 2 * kBK) {
            const int gk = kc + tid - kBK;
            koff_b[buf][tid - kBK] = gk < k_end ? axis_offset(d.vb.row, (uint32_t)gk) : 0u;
        }
    };
    Tc ra[EA], rb[EB];
    auto load_chunk = [&](int buf, int kc) {
#pragma unroll
        for (int i = 0; i < EA; ++i) {
            const int gka = kc + a_k[i];
            ra[i] = (a_ok[i] && gka < k_end) ? (Tc)A[a_off[i] + koff_a[buf][a_k[i]]] : (Tc)0;
        }
#pragma unroll
        for (int i = 0; i < EB; ++i) {
            const int gkb = kc + b_k[i];
            rb[i] = (b_ok[i] && gkb < k_end) ? (Tc)B[b_off[i] + koff_b[buf][b_k[i]]] : (Tc)0;
        }
    };

    using acc_t = typename Mma<Tc>::acc;
    acc_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    const int lane = tid & 63, wave = tid >> 6;
    const int wm = (wave % TS::WGM) * (BM / TS::WGM), wn = (wave / TS::WGM) * (BN / TS::WGN);
    const int lrow = lane & 15, lk = lane >> 4;

    fill_koff(0, k_begin);
    __syncthreads();
    if (k_begin < k_end) load_chunk(0, k_begin);
    int buf = 0;
    for (int kc = k_begin; kc < k_end; kc += kBK) {
#pragma unroll
        for (int i = 0; i < EA; ++i) As[a_k[i]][a_m[i]] = ra[i];
#pragma unroll
        for (int i = 0; i < EB; ++i) Bs[b_k[i]][b_n[i]] = rb[i];
        if (kc + kBK < k_end) fill_koff(buf ^ 1, kc + kBK);
        __syncthreads();
        if (kc + kBK < k_end) load_chunk(buf ^ 1, kc + kBK);
        if constexpr (Mma<Tc>::kK == 4) {
#pragma unroll
            for (int kk = 0; kk < kBK; kk += 4) {
                Tc a[FM], b[FN];
#pragma unroll
                for (int i = 0; i < FM; ++i) a[i] = As[kk + lk][wm + 16 * i + lrow];
#pragma unroll
                for (int j = 0; j < FN; ++j) b[j] = Bs[kk + lk][wn + 16 * j + lrow];
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j) acc[i][j] = Mma<Tc>::run(a[i], b[j], acc[i][j]);
            }
        } else {   // one 16-deep instruction covers the whole K chunk
            v4s a[FM], b[FN];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
#pragma unroll
                for (int i = 0; i < FM; ++i) a[i][q] = (short)As[4 * lk + q][wm + 16 * i + lrow].bits;
#pragma unroll
                for (int j = 0; j < FN; ++j) b[j][q] = (short)Bs[4 * lk + q][wn + 16 * j + lrow].bits;
            }
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) acc[i][j] = Mma<Tc>::run(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
        buf ^= 1;
    }

    const double fa = inv_scale(scales, d.scale_a);
    const double factor = d.square_a ? fa * fa : fa * inv_scale(scales, d.scale_b);
    double local_max = 0.0;
    Tout* __restrict__ C = (Tout*)d.C;
    if (d.mode == GEMM_ADJ) {
        // reverse pass: scatter into the adjoint's own layout, optionally accumulating
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gm = m0 + wm + i * 16 + Mma<Tc>::row(lane, r);
                    const int gn = n0 + wn + j * 16 + lrow;
                    if (gm < M && gn < N) {
                        const uint32_t off = axis_offset(d.vc.row, (uint32_t)gm) + axis_offset(d.vc.col, (uint32_t)gn);
                        double v = (double)acc[i][j][r] * factor;
                        if (d.accumulate) v += (double)C[off];
                        C[off] = (Tout)v;
                    }
                }
        return;
    }
    const int64_t cbase = (d.mode == GEMM_GRAM) ? (int64_t)split * M * N : 0;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm + i * 16 + Mma<Tc>::row(lane, r);
                const int gn = n0 + wn + j * 16 + lrow;
                if (gm < M && gn < N) {
                    const double v = (double)acc[i][j][r] * factor;
                    const Tout o = (Tout)v;
                    C[cbase + (int64_t)gm * N + gn] = o;
                    local_max = fmax(local_max, fabs((double)o));
                }
            }
    if (d.mode == GEMM_TENSOR) {
        local_max = wave_max(local_max);
        if (lane == 0) wmax[wave] = local_max;
        __syncthreads();
        if (tid == 0) {
            double m = wmax[0];
            for (int w = 1; w < kGemmThreads / 64; ++w) m = fmax(m, wmax[w]);
            maxparts[d.maxpart + local] = m;
        }
    }
}

// ------------------------------------------------------------------------------------------
// Grouped skinny GEMM: one side of C is short (at most S = 16 or 32) and K <= kSkinnyMaxK.  These
// are the re-absorptions A P_L and P_R B of a chi'-column projector (section II.C, SI B) and the
// contractions over one small bond.  They move a long operand once and do 2 S K flops per element
// of it, so they are HBM-bound: instead of padding the short side to a 64-wide MFMA tile, a
// workgroup takes 256 indices of the long side, one per thread, keeps the small operand in LDS
// (read as broadcasts) and accumulates all S outputs of its index in registers (float32 for
// float32 / bfloat16 tensors, float64 for float64).  kTall: M long (each thread one row of C);
// else N long (each thread one column).  The long operand is read along K with 16-byte vector
// loads when K is its unit-stride axis, else one element per K with consecutive threads on
// consecutive indices.
// ------------------------------------------------------------------------------------------
constexpr int kSkinnyMaxK = kSkinnyGemmMaxK, kSkinnyThreads = 256;

template <typename T>
struct Vec16;   // 16 bytes of T
template <>
struct Vec16<float> {
    static constexpr int n = 4;
    typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct Vec16<double> {
    static constexpr int n = 2;
    typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct Vec16<bf16> {
    static constexpr int n = 8;
    typedef uint4 type;
};
__device__ inline double vec_elem(const Vec16<double>::type& v, int i) { return v[i]; }
__device__ inline float vec_elem(const Vec16<float>::type& v, int i) { return v[i]; }
__device__ inline float vec_elem(const uint4& v, int i) {   // bfloat16 i of 8, little-endian
    const uint32_t w = i < 2 ? v.x : i < 4 ? v.y : i < 6 ? v.z : v.w;
    return __uint_as_float((i & 1) ? (w & 0xffff0000u) : (w << 16));
}
// a stored element as the accumulation type's source: float64 stays float64, the rest float32
__device__ inline double float_or_double(double x) { return x; }
__device__ inline float float_or_double(float x) { return x; }
__device__ inline float float_or_double(bf16 x) { return (float)x; }
template <typename T>
struct SkinnyAcc {
    typedef float type;
};
template <>
struct SkinnyAcc<double> {
    typedef double type;
};

template <typename Tin, typename Tacc, int S, bool kTall>
__global__ __launch_bounds__(kSkinnyThreads) void gemm_skinny_grouped(const GemmDesc* __restrict__ descs, int ndesc,
                                                                      const double* __restrict__ scales,
                                                                      double* __restrict__ maxparts, int64_t tile0) {
    __shared__ Tacc small[kSkinnyMaxK][S];   // small operand, K-major, zero beyond the short side
    __shared__ uint32_t koff[kSkinnyMaxK];   // long operand: offset of each K index
    __shared__ double wmax[kSkinnyThreads / 64];
    const int tid = threadIdx.x;
    const int64_t tile = tile0 + blockIdx.x;
    int lo = 0, hi = ndesc - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (descs[mid].tile_begin <= tile) lo = mid;
        else hi = mid - 1;
    }
    const GemmDesc& d = descs[lo];
    const int M = d.M, N = d.N, K = d.K;
    const int local = (int)(tile - d.tile_begin);
    const int L = kTall ? M : N, SS = kTall ? N : M;   // long and short extents
    const View& vl = kTall ? d.va : d.vb;              // long operand
    const View& vs = kTall ? d.vb : d.va;              // small operand
    const Axis& lax = kTall ? vl.row : vl.col;         // long operand: long axis
    const Axis& kax = kTall ? vl.col : vl.row;         // long operand: K axis
    const Tin* __restrict__ Xl = (const Tin*)(kTall ? d.A : d.B);
    const Tin* __restrict__ Xs = (const Tin*)(kTall ? d.B : d.A);

    for (int e = tid; e < K * S; e += kSkinnyThreads) {
        const int k = e / S, j = e - k * S;
        Tacc v = (Tacc)0;
        if (j < SS) {
            // small operand element (k, j): B[k][j] when tall, A[j][k] when wide
            const uint32_t off = kTall ? axis_offset(vs.row, (uint32_t)k) + axis_offset(vs.col, (uint32_t)j)
                                       : axis_offset(vs.row, (uint32_t)j) + axis_offset(vs.col, (uint32_t)k);
            v = (Tacc)(float_or_double(Xs[off]));
        }
        small[k][j] = v;
    }
    for (int k = tid; k < K; k += kSkinnyThreads) koff[k] = axis_offset(kax, (uint32_t)k);
    __syncthreads();

    const int idx = local * kSkinnyThreads + tid;
    const bool ok = idx < L;
    const uint32_t base = ok ? axis_offset(lax, (uint32_t)idx) : 0u;
    Tacc acc[S];
#pragma unroll
    for (int j = 0; j < S; ++j) acc[j] = (Tacc)0;

    // 16-byte loads along K: K is one unit-stride leg, and every index's base offset is aligned
    constexpr int V = Vec16<Tin>::n;
    bool vec = kax.n == 1 && kax.stride[0] == 1 && K % V == 0 &&
               ((uintptr_t)Xl & 15u) == 0;
    for (int l = 0; l < lax.n && vec; ++l) vec = lax.stride[l] % V == 0;
    if (ok && vec) {
        const typename Vec16<Tin>::type* p = (const typename Vec16<Tin>::type*)(Xl + base);
        for (int k0 = 0; k0 < K; k0 += 4 * V) {
            typename Vec16<Tin>::type x[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (k0 + q * V < K) x[q] = p[(k0 >> (V == 8 ? 3 : V == 4 ? 2 : 1)) + q];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (k0 + q * V >= K) break;
#pragma unroll
                for (int i = 0; i < V; ++i) {
                    const Tacc xv = (Tacc)vec_elem(x[q], i);
                    const Tacc* sr = small[k0 + q * V + i];
#pragma unroll
                    for (int j = 0; j < S; ++j) acc[j] = fma(xv, sr[j], acc[j]);
                }
            }
        }
    } else if (ok) {
        for (int k0 = 0; k0 < K; k0 += 16) {
            Tacc x[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) x[q] = k0 + q < K ? (Tacc)float_or_double(Xl[base + koff[k0 + q]]) : (Tacc)0;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                if (k0 + q >= K) break;
                const Tacc* sr = small[k0 + q];
#pragma unroll
                for (int j = 0; j < S; ++j) acc[j] = fma(x[q], sr[j], acc[j]);
            }
        }
    }

    const double factor = inv_scale(scales, d.scale_a) * inv_scale(scales, d.scale_b);
    double local_max = 0.0;
    if (ok) {
        if (d.mode == GEMM_ADJ) {
            Tin* __restrict__ C = (Tin*)d.C;
            const uint32_t o_long = kTall ? axis_offset(d.vc.row, (uint32_t)idx) : axis_offset(d.vc.col, (uint32_t)idx);
#pragma unroll
            for (int j = 0; j < S; ++j) {
                if (j >= SS) break;
                const uint32_t off =
                    o_long + (kTall ? axis_offset(d.vc.col, (uint32_t)j) : axis_offset(d.vc.row, (uint32_t)j));
                double v = (double)acc[j] * factor;
                if (d.accumulate) v += (double)float_or_double(C[off]);
                C[off] = (Tin)v;
            }
        } else {
            Tin* __restrict__ C = (Tin*)d.C;
#pragma unroll
            for (int j = 0; j < S; ++j) {
                if (j >= SS) break;
                const Tin o = (Tin)((double)acc[j] * factor);
                if (kTall) C[(int64_t)idx * N + j] = o;
                else C[(int64_t)j * N + idx] = o;
                local_max = fmax(local_max, fabs((double)float_or_double(o)));
            }
        }
    }
    if (d.mode == GEMM_TENSOR) {
        local_max = wave_max(local_max);
        if ((tid & 63) == 0) wmax[tid >> 6] = local_max;
        __syncthreads();
        if (tid == 0) {
            double m = wmax[0];
            for (int w = 1; w < kSkinnyThreads / 64; ++w) m = fmax(m, wmax[w]);
            maxparts[d.maxpart + local] = m;
        }
    }
}

// ------------------------------------------------------------------------------------------
// Batched tall-skinny QR (TSQR) for the R-factors of section II.C, Eq. (svd): the rows of a
// matricised side are cut into blocks held in LDS (float64, column-major); a workgroup reduces
// its block to R by Householder reflections (one column per step: the column norm, the
// reflector's products with the columns to its right, their update), and the stacked R's of a
// pass are the next pass's rows.  R^T R = X^T X / s^2 without forming the Gram, so directions
// far below the largest (which the Gram route drops under 1e-15 of the first pivot) survive.
// ------------------------------------------------------------------------------------------
constexpr int kTsqrThreads = 256;

__device__ inline double tsqr_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

template <typename T>
__global__ __launch_bounds__(kTsqrThreads) void tsqr_blocks(const TsqrDesc* __restrict__ descs, int ndesc,
                                                             const double* __restrict__ scales, int64_t blk0) {
    extern __shared__ double X[];                 // block, column-major, leading dimension br
    __shared__ double wcol[kCoreLdsMaxD];         // v^T x_c for the columns right of the step
    __shared__ double red[kTsqrThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t blk = blk0 + blockIdx.x;
    int lo = 0, hi = ndesc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (descs[mid].blk_begin <= blk) lo = mid;
        else hi = mid - 1;
    }
    const TsqrDesc& d = descs[lo];
    const int D = d.D, br = tsqr_block_rows(D);
    const int b = (int)(blk - d.blk_begin);
    const int r0 = b * br, nr = min(br, d.rows - r0);
    const double f = inv_scale(scales, d.scale);
    const T* __restrict__ src = (const T*)d.src;
    const bool rows_fast = d.v.row_unit != 0;
    for (int idx = tid; idx < nr * D; idx += kTsqrThreads) {
        int i, c;
        if (rows_fast) {
            i = idx % nr;
            c = idx / nr;
        } else {
            c = idx % D;
            i = idx / D;
        }
        X[c * br + i] = (double)src[axis_offset(d.v.row, (uint32_t)(r0 + i)) + axis_offset(d.v.col, (uint32_t)c)] * f;
    }
    __syncthreads();
    const int kmax = min(nr, D);
    for (int j = 0; j < kmax; ++j) {
        double* xj = X + j * br;
        double part = 0.0;
        for (int i = j + tid; i < nr; i += kTsqrThreads) part += xj[i] * xj[i];
        const double nrm2 = tsqr_sum(part, red);
        if (!(nrm2 > 0.0)) continue;   // a zero column: R[j][j] = 0, nothing to reflect
        const double x0 = xj[j];
        const double nrm = sqrt(nrm2);
        const double alpha = x0 > 0.0 ? -nrm : nrm;   // reflect x onto alpha e_j (no cancellation)
        const double v0 = x0 - alpha;                  // v = x - alpha e_j
        const double tau = 2.0 / (nrm2 - x0 * x0 + v0 * v0);
        for (int c = j + 1 + wave; c < D; c += kTsqrThreads / 64) {
            const double* xc = X + c * br;
            double sdot = 0.0;
            for (int i = j + 1 + lane; i < nr; i += 64) sdot += xj[i] * xc[i];
            sdot = wave_sum(sdot);
            if (lane == 0) wcol[c] = sdot + v0 * xc[j];
        }
        __syncthreads();
        const int h = nr - j;
        for (int idx = tid; idx < (D - j - 1) * h; idx += kTsqrThreads) {
            const int c = j + 1 + idx / h, i = j + idx % h;
            X[c * br + i] -= tau * (i == j ? v0 : xj[i]) * wcol[c];
        }
        __syncthreads();
        if (tid == 0) xj[j] = alpha;
    }
    __syncthreads();
    double* dst = d.dst + (int64_t)b * D * D;
    for (int idx = tid; idx < D * D; idx += kTsqrThreads) {
        const int r = idx / D, c = idx - r * D;
        dst[idx] = (r < kmax && c >= r) ? X[c * br + r] : 0.0;
    }
}

// ------------------------------------------------------------------------------------------
// Grouped Gram of a narrow side: C[split] (D x D, float64) = f * X^T X over one row range, X the
// (K x D) matricisation of a tensor (view va: rows = D, cols = K), D <= 64.  A workgroup takes
// one split: chunks of kGramKC rows are staged through LDS as float64 (double buffered, one
// barrier per chunk), and each wave accumulates 16 x 16 blocks of the upper triangle on the
// float64 MFMA; the lower triangle is written by symmetry.
// ------------------------------------------------------------------------------------------
constexpr int kGramThreads = 256, kGramKC = 32;

template <typename Tin>
__global__ __launch_bounds__(kGramThreads) void gram_narrow_grouped(const GemmDesc* __restrict__ descs, int ndesc,
                                                                   const double* __restrict__ scales, int64_t tile0) {
    __shared__ double Xs[2][kGramKC][65];
    __shared__ uint32_t koff[2][kGramKC];
    __shared__ uint32_t doff[64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t tile = tile0 + blockIdx.x;
    int lo = 0, hi = ndesc - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (descs[mid].tile_begin <= tile) lo = mid;
        else hi = mid - 1;
    }
    const GemmDesc& d = descs[lo];
    const int D = d.M, K = d.K;
    const int split = (int)(tile - d.tile_begin);
    const int k_begin = split * d.k_per_split;
    const int k_end = min(K, k_begin + d.k_per_split);
    const Tin* __restrict__ X = (const Tin*)d.A;
    if (tid < D) doff[tid] = axis_offset(d.va.row, (uint32_t)tid);
    // staging map: 8 elements per thread, lanes along whichever index has unit stride
    const bool kfast = d.va.col_unit != 0;
    int st_k[8], st_d[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (kfast) {
            st_k[j] = tid & 31;
            st_d[j] = (tid >> 5) + 8 * j;
        } else {
            st_d[j] = tid & 63;
            st_k[j] = (tid >> 6) + 4 * j;
        }
    }
    auto fill_koff = [&](int buf, int kc) {
        if (tid < kGramKC) {
            const int gk = kc + tid;
            koff[buf][tid] = gk < k_end ? axis_offset(d.va.col, (uint32_t)gk) : 0u;
        }
    };
    double r[8];
    auto load_chunk = [&](int buf, int kc) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int kk = st_k[j], dd = st_d[j];
            r[j] = (dd < D && kc + kk < k_end) ? (double)X[doff[dd] + koff[buf][kk]] : 0.0;
        }
    };
    // upper-triangle 16 x 16 blocks (bi <= bj) dealt round-robin to the waves; a single block is
    // shared by all four waves, each taking every fourth step along K
    const int nbd = (D + 15) / 16, nblk = nbd * (nbd + 1) / 2;
    const bool shared_blk = nblk == 1;
    int bi[3] = {0, 0, 0}, bj[3] = {0, 0, 0}, nmine = 0;
    for (int b = shared_blk ? 0 : wave; b < nblk && nmine < 3; b += 4) {
        int row = 0, rem = b;
        while (rem >= nbd - row) {
            rem -= nbd - row;
            ++row;
        }
        bi[nmine] = row;
        bj[nmine] = row + rem;
        ++nmine;
    }
    v4d acc[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
    const int lr = lane & 15, lk = lane >> 4;

    __syncthreads();   // doff
    fill_koff(0, k_begin);
    __syncthreads();
    if (k_begin < k_end) load_chunk(0, k_begin);
    int buf = 0;
    for (int kc = k_begin; kc < k_end; kc += kGramKC) {
#pragma unroll
        for (int j = 0; j < 8; ++j) Xs[buf][st_k[j]][st_d[j]] = r[j];
        if (kc + kGramKC < k_end) fill_koff(buf ^ 1, kc + kGramKC);
        __syncthreads();
        if (kc + kGramKC < k_end) load_chunk(buf ^ 1, kc + kGramKC);
#pragma unroll
        for (int ks = 0; ks < kGramKC / 4; ++ks) {
            if (shared_blk && (ks & 3) != wave) continue;
            const int k = 4 * ks + lk;
#pragma unroll
            for (int q = 0; q < 3; ++q)
                if (q < nmine) {
                    const double a = Xs[buf][k][16 * bi[q] + lr];
                    const double b = Xs[buf][k][16 * bj[q] + lr];
                    acc[q] = Mma<double>::run(a, b, acc[q]);
                }
        }
        buf ^= 1;
    }
    const double fa = inv_scale(scales, d.scale_a);
    const double factor = fa * fa;
    double* C = (double*)d.C + (int64_t)split * D * D;
    if (shared_blk) {
        // the four waves' partial sums of the one block meet in LDS (staging is over)
        __syncthreads();
        double* red = &Xs[0][0][0];
#pragma unroll
        for (int q = 0; q < 4; ++q) red[(wave * 64 + lane) * 4 + q] = acc[0][q];
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                acc[0][q] = ((red[lane * 4 + q] + red[(64 + lane) * 4 + q]) + red[(128 + lane) * 4 + q]) +
                            red[(192 + lane) * 4 + q];
        } else {
            nmine = 0;
        }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q)
        if (q < nmine)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int gi = 16 * bi[q] + Mma<double>::row(lane, rr), gj = 16 * bj[q] + lr;
                if (gi < D && gj < D) {
                    const double v = acc[q][rr] * factor;
                    C[(int64_t)gi * D + gj] = v;
                    C[(int64_t)gj * D + gi] = v;
                }
            }
}

// ------------------------------------------------------------------------------------------
// Gather copy (explicit reduced factor when a side has no more rows than D)
// ------------------------------------------------------------------------------------------
template <typename Tin>
__global__ __launch_bounds__(256) void copy_grouped(const CopyDesc* __restrict__ descs, int ndesc,
                                                    const double* __restrict__ scales, int64_t total, int64_t e0) {
    const int64_t e = e0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    int lo = 0, hi = ndesc - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (descs[mid].elem_begin <= e) lo = mid;
        else hi = mid - 1;
    }
    const CopyDesc& d = descs[lo];
    const int local = (int)(e - d.elem_begin);
    const int r = local / d.cols, c = local - r * d.cols;
    const Tin* src = (const Tin*)d.src;
    const double v = (double)src[axis_offset(d.v.row, (uint32_t)r) + axis_offset(d.v.col, (uint32_t)c)];
    d.dst[(int64_t)r * d.cols + c] = v * inv_scale(scales, d.scale);
}

// ------------------------------------------------------------------------------------------
// Compression core: one workgroup per compression
// ------------------------------------------------------------------------------------------
constexpr int kCoreThreads = 1024;
constexpr double kNoiseRel = 1e-13;   // singular values below this * sigma_1 are zeros
constexpr double kZeroRel = 1e-14;    // Jacobi leaves columns below this * ||W||_F alone
constexpr double kLanczosBreak = 1e-13;   // Krylov breakdown relative to the largest alpha/beta
constexpr double kNoiseRelSq = 1e-13;     // eigenvalues sigma^2 of M^T M below this * sigma_1^2 are zeros
constexpr int kCoreWaves = kCoreThreads / 64;
// LDS-resident cores (D <= 64): four waves rotate the at most 32 column pairs of a round, and a
// small workgroup finds room on a compute unit while the GEMMs of the same level occupy it
constexpr int kCoreLdsThreads = 256;

struct CoreShared {
    double rv[kCoreWaves];
    int ri[kCoreWaves];
    int flag;
    int flag_big;                // a rotation of the sweep had |g| > 1e-8 sqrt(a b)
    double row[kCoreLdsMaxD];
};

// R (rows x D, row-major, original column order) with R^T R = G: pivoted Cholesky
// of the symmetric positive semidefinite D x D matrix G (destroyed).  Returns the rank.
// Wave 0 picks each pivot (largest remaining diagonal, lowest index on ties); two barriers
// per step.
__device__ int pivoted_cholesky(double* G, int D, double* R, int* chosen, CoreShared& sh) {
    const int tid = threadIdx.x, lane = tid & 63;
    for (int i = tid; i < D; i += kCoreThreads) chosen[i] = 0;
    __syncthreads();
    double tol = 0.0;
    int r = 0;
    for (int t = 0; t < D; ++t) {
        if (tid < 64) {
            double bv = -1.0;
            int bi = 0x7fffffff;
            for (int i = lane; i < D; i += 64) {
                if (chosen[i]) continue;
                const double v = G[(int64_t)i * D + i];
                if (v > bv || (v == bv && i < bi)) { bv = v; bi = i; }
            }
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                const double ov = __shfl_xor(bv, o, 64);
                const int oi = __shfl_xor(bi, o, 64);
                if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
            }
            if (lane == 0) { sh.rv[0] = bv; sh.ri[0] = bi; }
        }
        __syncthreads();
        const double piv = sh.rv[0];
        const int p = sh.ri[0];
        if (t == 0) tol = 1e-15 * piv;
        if (!(piv > tol) || !(piv > 0.0)) break;
        const double rp = sqrt(piv);
        double* Rt = R + (int64_t)t * D;
        double* rrow = D <= kCoreLdsMaxD ? sh.row : Rt;   // the row the update reads, in LDS when small
        for (int j = tid; j < D; j += kCoreThreads) {
            const double v = chosen[j] ? 0.0 : (j == p ? rp : G[(int64_t)p * D + j] / rp);
            Rt[j] = v;
            if (D <= kCoreLdsMaxD) sh.row[j] = v;
        }
        __syncthreads();
        const int64_t DD = (int64_t)D * D;
        for (int64_t idx = tid; idx < DD; idx += kCoreThreads) {
            const int i = (int)(idx / D), j = (int)(idx - (int64_t)i * D);
            if (i != p && j != p && !chosen[i] && !chosen[j]) G[idx] -= rrow[i] * rrow[j];
        }
        if (tid == 0) chosen[p] = 1;
        __syncthreads();
        r = t + 1;
    }
    return r;
}

// The same factorisation for 64 < D <= kCholBlkMaxD, blocked: pivots are taken kCholPanel at a
// time, the panel's rows of R kept in LDS (row t: R[t, j] = (G'[p, j] - sum over the panel's
// earlier rows of R[s, p] R[s, j]) / R[t, p], with G' the Gram updated by the previous panels),
// then one rank-kCholPanel update of the remaining rows and columns of G (destroyed).  The
// remaining diagonal is kept in LDS; the pivot is its largest entry (DPP maximum, lowest index
// among equals by ballot).  Same pivots, ties and stopping rule as pivoted_cholesky.
constexpr int kCholPanel = 16;
constexpr int kCholBlkMaxD = 384;
__device__ int pivoted_cholesky_blocked(double* __restrict__ G, int D, double* __restrict__ R, double* lds,
                                        CoreShared& sh) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double* diag = lds;
    double* pan = lds + D;                              // kCholPanel rows of length D
    int* chosen = (int*)(pan + kCholPanel * D);
    for (int j = tid; j < D; j += kCoreThreads) {
        diag[j] = G[(int64_t)j * D + j];
        chosen[j] = 0;
    }
    __syncthreads();
    double tol = 0.0;
    int r = 0;
    bool done = false;
    for (int t0 = 0; t0 < D && !done; t0 += kCholPanel) {
        int np = 0;
        for (int t = t0; t < D && t < t0 + kCholPanel; ++t) {
            if (wave == 0) {
                double bl = -1.0;
                for (int i = lane; i < D; i += 64)
                    if (!chosen[i]) bl = fmax(bl, diag[i]);
                const double bv = wave_max(bl);
                int bi = -1;
                for (int i0 = 0; i0 < D && bi < 0; i0 += 64) {
                    const int i = i0 + lane;
                    const unsigned long long m = __ballot(i < D && !chosen[i] && diag[i] == bv);
                    if (m) bi = i0 + __ffsll(m) - 1;
                }
                if (lane == 0) { sh.rv[0] = bv; sh.ri[0] = bi; }
            }
            __syncthreads();
            const double piv = sh.rv[0];
            const int p = sh.ri[0];
            if (t == 0) tol = 1e-15 * piv;
            if (!(piv > tol) || !(piv > 0.0)) { done = true; break; }
            const double rp = sqrt(piv);
            const int u = t - t0;
            for (int j = tid; j < D; j += kCoreThreads) {
                const bool ch = chosen[j] != 0;
                double v = 0.0;
                if (!ch) {
                    if (j == p) {
                        v = rp;
                    } else {
                        double a = G[(int64_t)p * D + j];
                        for (int q = 0; q < u; ++q) a = fma(-pan[q * D + p], pan[q * D + j], a);
                        v = a / rp;
                    }
                }
                R[(int64_t)t * D + j] = v;
                pan[u * D + j] = v;
                if (j == p) chosen[j] = 1;
                else if (!ch) diag[j] -= v * v;
            }
            __syncthreads();
            np = u + 1;
            r = t + 1;
        }
        if (done || t0 + kCholPanel >= D) break;
        // G -= Pᵀ P over the rows and columns not yet chosen (the panel P in LDS): a wave per
        // row, the lane's columns of P held in registers
        for (int j0 = 0; j0 < D; j0 += 64) {
            const int j = j0 + lane;
            const bool cj = j < D && !chosen[j];
            double pj[kCholPanel];
#pragma unroll
            for (int q = 0; q < kCholPanel; ++q) pj[q] = (cj && q < np) ? pan[q * D + j] : 0.0;
            for (int i = wave; i < D; i += kCoreWaves) {
                if (chosen[i]) continue;
                double a = 0.0;
#pragma unroll
                for (int q = 0; q < kCholPanel; ++q) a = fma(pan[q * D + i], pj[q], a);
                if (cj) G[(int64_t)i * D + j] -= a;
            }
        }
        __syncthreads();
    }
    return r;
}

// The same factorisation, left-looking, for large D: step t computes only the pivot's row,
// R[t, j] = (G[p, j] - sum_{s<t} R[s, p] R[s, j]) / R[t, p], from the rows already found, and keeps
// the remaining diagonal d_j = G[j, j] - sum_s R[s, j]^2 in LDS (same pivots, ties and stopping
// rule; G is read, not destroyed).  Four lanes share a column's sum.  LDS: 20 D bytes.
constexpr int kCholLLMaxD = 3072;
__device__ int pivoted_cholesky_ll(const double* __restrict__ G, int D, double* __restrict__ R, double* lds,
                                   CoreShared& sh) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double* diag = lds;
    double* rcol = lds + D;                 // R[s, p] of the current pivot, s < t
    int* chosen = (int*)(lds + 2 * D);
    for (int j = tid; j < D; j += kCoreThreads) {
        diag[j] = G[(int64_t)j * D + j];
        chosen[j] = 0;
    }
    __syncthreads();
    double tol = 0.0;
    int r = 0;
    for (int t = 0; t < D; ++t) {
        if (wave == 0) {
            double bv = -1.0;
            int bi = 0x7fffffff;
            for (int i = lane; i < D; i += 64) {
                if (chosen[i]) continue;
                const double v = diag[i];
                if (v > bv || (v == bv && i < bi)) { bv = v; bi = i; }
            }
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                const double ov = __shfl_xor(bv, o, 64);
                const int oi = __shfl_xor(bi, o, 64);
                if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
            }
            if (lane == 0) { sh.rv[0] = bv; sh.ri[0] = bi; }
        }
        __syncthreads();
        const double piv = sh.rv[0];
        const int p = sh.ri[0];
        if (t == 0) tol = 1e-15 * piv;
        if (!(piv > tol) || !(piv > 0.0)) break;
        for (int q = tid; q < t; q += kCoreThreads) rcol[q] = R[(int64_t)q * D + p];
        __syncthreads();
        const double rp = sqrt(piv);
        double* Rt = R + (int64_t)t * D;
        const int k = tid & 3;
        for (int j0 = 0; j0 < D; j0 += kCoreThreads / 4) {
            const int j = j0 + (tid >> 2);
            // eight independent loads in flight per lane (the rows come from L2)
            double acc8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            if (j < D) {
                int q = k;
                for (; q + 28 < t; q += 32) {
                    double x[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) x[u] = R[(int64_t)(q + 4 * u) * D + j];
#pragma unroll
                    for (int u = 0; u < 8; ++u) acc8[u] = fma(rcol[q + 4 * u], x[u], acc8[u]);
                }
                for (; q < t; q += 4) acc8[0] = fma(rcol[q], R[(int64_t)q * D + j], acc8[0]);
            }
            double acc = ((acc8[0] + acc8[1]) + (acc8[2] + acc8[3])) + ((acc8[4] + acc8[5]) + (acc8[6] + acc8[7]));
            acc += __shfl_xor(acc, 1, 64);
            acc += __shfl_xor(acc, 2, 64);
            if (j < D && k == 0) {
                const bool ch = chosen[j] != 0;
                const double v = ch ? 0.0 : (j == p ? rp : (G[(int64_t)p * D + j] - acc) / rp);
                Rt[j] = v;
                if (j == p) chosen[j] = 1;
                else if (!ch) diag[j] -= v * v;
            }
        }
        __syncthreads();
        r = t + 1;
    }
    return r;
}

// 1/x and 1/sqrt(x) (x > 0) from the hardware estimates refined by two Newton-Raphson steps
// each (every step doubles the correct bits), to within a few ulp in float64.
__device__ inline double rcp_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}
__device__ inline double rsq_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    return y * fma(-h * y, y, 1.5);
}

// Jacobi rotation annihilating the off-diagonal g of the 2 x 2 Gram [[a, g], [g, b]] of two
// columns, through the smaller angle theta with tan(2 theta) = 2g / (b - a): with d = b - a and
// r = sqrt(d^2 + 4 g^2), cos(2 theta) = |d| / r, so c = sqrt((1 + |d| / r) / 2) and
// s = sgn(d) g / (r c).  Two refined reciprocal square roots form the whole dependent chain
// (float64 latency rules here); squares out of range take the tangent form
// t = sgn(zeta) / (|zeta| + sqrt(1 + zeta^2)), zeta = (b - a) / 2g, c = 1 / sqrt(1 + t^2), s = c t.
__device__ inline void jacobi_rotation(double a, double b, double g, double* c, double* s) {
    const double d = b - a;
    const double q = fma(d, d, 4.0 * g * g);
    if (q > 1e-290 && q < 1e290) {
        const double y = rsq_nr(q);                       // 1 / r
        const double h = fma(0.5 * fabs(d), y, 0.5);      // c^2, in [1/2, 1]
        const double yc = rsq_nr(h);                      // 1 / c
        *c = h * yc;
        *s = (d >= 0.0 ? g : -g) * y * yc;
        return;
    }
    const double zeta = d * rcp_nr(2.0 * g);
    const double az = fabs(zeta);
    double root;
    if (az > 1e100) {
        root = az;
    } else {
        const double r2 = fma(zeta, zeta, 1.0);
        root = r2 * rsq_nr(r2);
    }
    const double t = (zeta >= 0.0 ? 1.0 : -1.0) * rcp_nr(az + root);
    const double cc = rsq_nr(fma(t, t, 1.0));
    *c = cc;
    *s = cc * t;
}

// pivoted_cholesky by a single wave for D <= 64: lane l owns index l, the pivot search is a
// wave butterfly, and the rank-1 update runs down each lane's own column of G (LDS, symmetric,
// destroyed).  Same pivot rule, stopping tolerance and output layout as pivoted_cholesky.
__device__ int pivoted_cholesky_wave(double* G, int D, double* R) {
    const int l = threadIdx.x & 63;
    const bool own = l < D;
    bool chosen = !own;
    double diag = own ? G[l * D + l] : 0.0;
    double tol = 0.0;
    int r = 0;
    for (int t = 0; t < D; ++t) {
        // pivot: the largest remaining diagonal (DPP maximum), lowest lane on ties (ballot)
        const double cand = chosen ? -1.0 : diag;
        const double bv = wave_max(cand);
        if (t == 0) tol = 1e-15 * bv;
        if (!(bv > tol) || !(bv > 0.0)) break;
        const int p = __ffsll((unsigned long long)__ballot(!chosen && cand == bv)) - 1;
        const double rp = sqrt(bv);
        double v = 0.0;
        if (!chosen) v = (l == p) ? rp : G[p * D + l] / rp;
        if (own) R[t * D + l] = v;
        if (!chosen && l != p) {
            double* col = G + l;
            int i = 0;
            for (; i + 4 <= D; i += 4) {
                const double v0 = bcast(v, i), v1 = bcast(v, i + 1), v2 = bcast(v, i + 2), v3 = bcast(v, i + 3);
                const double g0 = col[i * D], g1 = col[(i + 1) * D], g2 = col[(i + 2) * D], g3 = col[(i + 3) * D];
                col[i * D] = g0 - v0 * v;
                col[(i + 1) * D] = g1 - v1 * v;
                col[(i + 2) * D] = g2 - v2 * v;
                col[(i + 3) * D] = g3 - v3 * v;
            }
            for (; i < D; ++i) col[i * D] -= bcast(v, i) * v;
        }
        if (l == p) chosen = true;
        if (!chosen) diag = G[l * D + l];
        r = t + 1;
    }
    return r;
}

// pivoted_cholesky_wave for D <= KMAX with lane l's column of G held in registers (G is read,
// not destroyed): the pivot's entry G'[p][l] is picked by a select chain (p is the same on every
// lane), and the rank-1 update is one unrolled row of readlane + FMA (a zero multiplier on the
// lanes that keep their column).  Same pivot rule, stopping tolerance and output as
// pivoted_cholesky_wave.
template <int KMAX>
__device__ int pivoted_cholesky_wave_reg(const double* G, int D, double* R) {
    const int l = threadIdx.x & 63;
    const bool own = l < D;
    double g[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) g[i] = (own && i < D) ? G[i * D + l] : 0.0;
    bool chosen = !own;
    double diag = own ? G[l * D + l] : 0.0;
    double tol = 0.0;
    int r = 0;
    // not unrolled: two copies of the column would double the live registers
#pragma nounroll
    for (int t = 0; t < D; ++t) {
        const double cand = chosen ? -1.0 : diag;
        const double bv = wave_max(cand);
        if (t == 0) tol = 1e-15 * bv;
        if (!(bv > tol) || !(bv > 0.0)) break;
        const int p = __ffsll((unsigned long long)__ballot(!chosen && cand == bv)) - 1;
        const double rp = sqrt(bv);
        double gp = 0.0;
#pragma unroll
        for (int i = 0; i < KMAX; ++i) gp = i == p ? g[i] : gp;
        double v = 0.0;
        if (!chosen) v = (l == p) ? rp : gp / rp;
        if (own) R[t * D + l] = v;
        const double w = (!chosen && l != p) ? v : 0.0;
#pragma unroll
        for (int i = 0; i < KMAX; ++i) g[i] = fma(-bcast(v, i), w, g[i]);
        diag = fma(-w, v, diag);
        if (l == p) chosen = true;
        r = t + 1;
    }
    return r;
}

__device__ inline int rr_col(int pos, int round, int n) {
    int v = pos - 1 + round;   // pos - 1 and round are below n - 1: one wrap at most
    if (v >= n - 1) v -= n - 1;
    return pos == 0 ? 0 : 1 + v;
}

// A sweep whose rotations all had |g| <= 1e-8 sqrt(a b) ends the iteration: convergence is
// quadratic, so the off-diagonal it leaves is of order 1e-16 relative, and a confirming sweep
// would rotate nothing above the tolerance.
constexpr double kQuadRel2 = 1e-16;

// One-sided (Hestenes) Jacobi on the columns of W (rows x cols, column j at W + j*ld),
// accumulating the rotations in V (cols x cols, column j at V + j*ld, identity on entry).
// Pairs follow a round-robin tournament; one wave rotates one pair.  A pair is rotated
// while its columns are not orthogonal to relative precision tol; columns whose norm is
// at the rounding level of ||W||_F (rank-deficient matrices) are numerically zero and are
// left alone, else their noise would keep rotating forever.  Returns convergence.
__device__ bool jacobi_svd(double* W, double* V, int rows, int cols, int ld, int max_sweeps, CoreShared& sh,
                           int* sweeps_out) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nc = cols + (cols & 1);
    const double tol = 2.220446049250313e-16 * (double)max(rows, 16);
    {
        double f = 0.0;
        for (int64_t idx = tid; idx < (int64_t)rows * cols; idx += kCoreThreads) {
            const int j = (int)(idx / rows), i = (int)(idx - (int64_t)j * rows);
            const double x = W[(int64_t)j * ld + i];
            f += x * x;
        }
        f = wave_sum(f);
        if (lane == 0) sh.rv[wave] = f;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int w = 0; w < kCoreWaves; ++w) t += sh.rv[w];
            sh.rv[0] = t;
        }
        __syncthreads();
    }
    const double zero2 = kZeroRel * kZeroRel * sh.rv[0];
    __syncthreads();
    int sweeps = 0;
    bool converged = (cols <= 1);
    for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
        if (tid == 0) sh.flag = sh.flag_big = 0;
        __syncthreads();
        for (int round = 0; round < nc - 1; ++round) {
            for (int q = wave; q < nc / 2; q += kCoreWaves) {
                const int p1 = rr_col(q, round, nc), p2 = rr_col(nc - 1 - q, round, nc);
                if (p1 >= cols || p2 >= cols) continue;
                double* w1 = W + (int64_t)p1 * ld;
                double* w2 = W + (int64_t)p2 * ld;
                double a = 0.0, b = 0.0, g = 0.0;
                for (int i = lane; i < rows; i += 64) {
                    const double x = w1[i], y = w2[i];
                    a += x * x;
                    b += y * y;
                    g += x * y;
                }
                a = wave_sum(a);
                b = wave_sum(b);
                g = wave_sum(g);
                if (a > zero2 && b > zero2 && g * g > tol * tol * a * b) {
                    double c, s;
                    jacobi_rotation(a, b, g, &c, &s);
                    for (int i = lane; i < rows; i += 64) {
                        const double x = w1[i], y = w2[i];
                        w1[i] = c * x - s * y;
                        w2[i] = s * x + c * y;
                    }
                    double* v1 = V + (int64_t)p1 * ld;
                    double* v2 = V + (int64_t)p2 * ld;
                    for (int i = lane; i < cols; i += 64) {
                        const double x = v1[i], y = v2[i];
                        v1[i] = c * x - s * y;
                        v2[i] = s * x + c * y;
                    }
                    if (lane == 0) {
                        sh.flag = 1;
                        if (g * g > kQuadRel2 * a * b) sh.flag_big = 1;
                    }
                }
            }
            __syncthreads();
        }
        sweeps = sweep + 1;
        if (!sh.flag || !sh.flag_big) converged = true;
        __syncthreads();
    }
    *sweeps_out = sweeps;
    return converged;
}

// jacobi_svd for rows, cols <= 256 (W, V in global memory): a wave rotates two pairs at a time,
// one row of each per lane for four rows, every operand held in registers between the dot
// products and the update, the two pairs' reductions and rotations interleaved.  Same pair order,
// thresholds and result contract as jacobi_svd.
__device__ bool jacobi_svd_256(double* W, double* V, int rows, int cols, int ld, int max_sweeps, CoreShared& sh,
                               int* sweeps_out) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nc = cols + (cols & 1);
    const double tol = 2.220446049250313e-16 * (double)max(rows, 16);
    {
        double f = 0.0;
        for (int64_t idx = tid; idx < (int64_t)rows * cols; idx += kCoreThreads) {
            const int j = (int)(idx / rows), i = (int)(idx - (int64_t)j * rows);
            const double x = W[(int64_t)j * ld + i];
            f += x * x;
        }
        f = wave_sum(f);
        if (lane == 0) sh.rv[wave] = f;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int w = 0; w < kCoreWaves; ++w) t += sh.rv[w];
            sh.rv[0] = t;
        }
        __syncthreads();
    }
    const double zero2 = kZeroRel * kZeroRel * sh.rv[0];
    __syncthreads();
    int sweeps = 0;
    bool converged = (cols <= 1);
    for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
        if (tid == 0) sh.flag = sh.flag_big = 0;
        __syncthreads();
        for (int round = 0; round < nc - 1; ++round) {
            for (int q0 = 2 * wave; q0 < nc / 2; q0 += 2 * kCoreWaves) {
                double* w1[2];
                double* w2[2];
                double* v1[2];
                double* v2[2];
                double x[2][4], y[2][4], xv[2][4], yv[2][4], a[2], b[2], g[2];
                bool ok[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int q = q0 + u;
                    const int p1 = rr_col(q, round, nc), p2 = rr_col(nc - 1 - q, round, nc);
                    ok[u] = q < nc / 2 && p1 < cols && p2 < cols;
                    const int c1 = ok[u] ? p1 : 0, c2 = ok[u] ? p2 : 1;
                    w1[u] = W + (int64_t)c1 * ld;
                    w2[u] = W + (int64_t)c2 * ld;
                    v1[u] = V + (int64_t)c1 * ld;
                    v2[u] = V + (int64_t)c2 * ld;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int i = lane + 64 * k;
                        x[u][k] = i < rows ? w1[u][i] : 0.0;
                        y[u][k] = i < rows ? w2[u][i] : 0.0;
                        xv[u][k] = i < cols ? v1[u][i] : 0.0;
                        yv[u][k] = i < cols ? v2[u][i] : 0.0;
                    }
                }
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    a[u] = b[u] = g[u] = 0.0;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        a[u] = fma(x[u][k], x[u][k], a[u]);
                        b[u] = fma(y[u][k], y[u][k], b[u]);
                        g[u] = fma(x[u][k], y[u][k], g[u]);
                    }
                }
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    a[u] = wave_sum(a[u]);
                    b[u] = wave_sum(b[u]);
                    g[u] = wave_sum(g[u]);
                }
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    if (ok[u] && a[u] > zero2 && b[u] > zero2 && g[u] * g[u] > tol * tol * a[u] * b[u]) {
                        double c, s;
                        jacobi_rotation(a[u], b[u], g[u], &c, &s);
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const int i = lane + 64 * k;
                            if (i < rows) {
                                w1[u][i] = c * x[u][k] - s * y[u][k];
                                w2[u][i] = s * x[u][k] + c * y[u][k];
                            }
                            if (i < cols) {
                                v1[u][i] = c * xv[u][k] - s * yv[u][k];
                                v2[u][i] = s * xv[u][k] + c * yv[u][k];
                            }
                        }
                        if (lane == 0) {
                            sh.flag = 1;
                            if (g[u] * g[u] > kQuadRel2 * a[u] * b[u]) sh.flag_big = 1;
                        }
                    }
                }
            }
            __syncthreads();
        }
        sweeps = sweep + 1;
        if (!sh.flag || !sh.flag_big) converged = true;
        __syncthreads();
    }
    *sweeps_out = sweeps;
    return converged;
}

// Sum over the lane's 16-lane DPP row (every lane of the row gets the row total).  The four
// controls stay inside the row, so no lane reads out of bounds and the moves need no old value.
template <int kCtrl>
__device__ inline double dpp_in_row(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), kCtrl, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), kCtrl, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ inline double row16_sum(double v) {
    v += dpp_in_row<0xB1>(v);
    v += dpp_in_row<0x4E>(v);
    v += dpp_in_row<0x141>(v);
    v += dpp_in_row<0x140>(v);
    return v;
}

// One halving step of a transposed reduction over a 16-lane DPP row: the lanes l and l ^ W
// pair up, the one with that bit clear keeps v[0, W) and the other v[W, 2 W), and each adds the
// partner's copy of the half it keeps into v[0, W).  kFromUp / kFromDown: DPP controls that read
// lane l - W and l + W (row_ror moves data to higher lanes; or quad permutations).
template <int W, int kFromUp, int kFromDown>
__device__ inline void halve_rows(double* v, bool up) {
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const double send = up ? v[k] : v[k + W];
        const double keep = up ? v[k + W] : v[k];
        const double a = dpp_in_row<kFromUp>(send), b = dpp_in_row<kFromDown>(send);
        v[k] = keep + (up ? a : b);
    }
}

// jacobi_svd for rows, cols <= 16 KR (KR <= 4): each pair is rotated by one 16-lane row of a
// wave (KR rows of W per lane), so reductions stay inside DPP rows and a wave rotates four
// pairs at once.  Same pair order, thresholds and result contract as jacobi_svd.
// P: double* or an LDS-qualified pointer (LdsPtr), for callers whose W and V may live in either.
template <int NT = kCoreThreads, int KR = 4, typename P = double*>
__device__ bool jacobi_svd_small(P W, P V, int rows, int cols, int ld, int max_sweeps, CoreShared& sh,
                                 int* sweeps_out) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int quarter = lane >> 4, ql = lane & 15;
    const int nc = cols + (cols & 1);
    const double tol = 2.220446049250313e-16 * (double)max(rows, 16);
    double f = 0.0;
    for (int idx = tid; idx < rows * cols; idx += NT) {
        const int j = idx / rows, i = idx - j * rows;
        const double x = W[(int64_t)j * ld + i];
        f += x * x;
    }
    f = wave_sum(f);
    if (lane == 0) sh.rv[wave] = f;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < (NT / 64); ++w) t += sh.rv[w];
        sh.rv[0] = t;
    }
    __syncthreads();
    const double zero2 = kZeroRel * kZeroRel * sh.rv[0];
    __syncthreads();
    int sweeps = 0;
    bool converged = (cols <= 1);
    for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
        if (tid == 0) sh.flag = sh.flag_big = 0;
        __syncthreads();
        for (int round = 0; round < nc - 1; ++round) {
            for (int q = wave * 4 + quarter; q < nc / 2; q += (NT / 64) * 4) {
                const int p1 = rr_col(q, round, nc), p2 = rr_col(nc - 1 - q, round, nc);
                if (p1 >= cols || p2 >= cols) continue;
                const P w1 = W + (int64_t)p1 * ld;
                const P w2 = W + (int64_t)p2 * ld;
                const P v1 = V + (int64_t)p1 * ld;
                const P v2 = V + (int64_t)p2 * ld;
                // every load up front (clamped index, then zeroed), so their latencies overlap
                double x[KR], y[KR], xv[KR], yv[KR];
                double a = 0.0, b = 0.0, g = 0.0;
#pragma unroll
                for (int k = 0; k < KR; ++k) {
                    const int i = ql + 16 * k;
                    const int iw = min(i, max(rows, 1) - 1), iv = min(i, cols - 1);
                    x[k] = w1[iw];
                    y[k] = w2[iw];
                    xv[k] = v1[iv];
                    yv[k] = v2[iv];
                    if (i >= rows) x[k] = y[k] = 0.0;
                }
#pragma unroll
                for (int k = 0; k < KR; ++k) {
                    a = fma(x[k], x[k], a);
                    b = fma(y[k], y[k], b);
                    g = fma(x[k], y[k], g);
                }
                a = row16_sum(a);
                b = row16_sum(b);
                g = row16_sum(g);
                if (a > zero2 && b > zero2 && g * g > tol * tol * a * b) {
                    double c, s;
                    jacobi_rotation(a, b, g, &c, &s);
#pragma unroll
                    for (int k = 0; k < KR; ++k) {
                        const int i = ql + 16 * k;
                        if (i < rows) {
                            w1[i] = c * x[k] - s * y[k];
                            w2[i] = s * x[k] + c * y[k];
                        }
                        if (i < cols) {
                            v1[i] = c * xv[k] - s * yv[k];
                            v2[i] = s * xv[k] + c * yv[k];
                        }
                    }
                    if (ql == 0) {
                        sh.flag = 1;
                        if (g * g > kQuadRel2 * a * b) sh.flag_big = 1;
                    }
                }
            }
            __syncthreads();
        }
        sweeps = sweep + 1;
        if (!sh.flag || !sh.flag_big) converged = true;
        __syncthreads();
    }
    *sweeps_out = sweeps;
    return converged;
}

// The rotation of jacobi_rotation by a shorter dependent chain: with u = |d| + r,
// c = u / sqrt(u^2 + 4 g^2) and s = sgn(d) 2g / sqrt(u^2 + 4 g^2) (u^2 + 4 g^2 = 2 r u, so these
// are the same c and s).  r = sqrt(d^2 + 4 g^2) takes one Newton step from the hardware
// reciprocal square root (its error only perturbs the angle); 1 / sqrt(u^2 + 4 g^2) takes one
// third-order step, so c^2 + s^2 = 1 to rounding.
__device__ inline void jacobi_rotation_fast(double a, double b, double g, double* c, double* s) {
    const double d = b - a;
    const double g2 = g * (4.0 * g);
    const double q = fma(d, d, g2);
    if (q > 1e-290 && q < 1e290) {
        const double y0 = __builtin_amdgcn_rsq(q);
        const double r0 = q * y0, h0 = 0.5 * y0;
        const double r = fma(r0, fma(-r0, h0, 0.5), r0);
        const double u = fabs(d) + r;
        const double w = fma(u, u, g2);
        const double z0 = __builtin_amdgcn_rsq(w);
        const double e = fma(-w * z0, z0, 1.0);
        const double z = fma(z0 * e, fma(e, 0.375, 0.5), z0);
        *c = u * z;
        *s = (d >= 0.0 ? 2.0 * g : -2.0 * g) * z;
        return;
    }
    jacobi_rotation(a, b, g, c, s);
}

// three row16_sum reductions, stage by stage
__device__ inline void row16_sum3(double& a, double& b, double& g) {
    a += dpp_in_row<0xB1>(a); b += dpp_in_row<0xB1>(b); g += dpp_in_row<0xB1>(g);
    a += dpp_in_row<0x4E>(a); b += dpp_in_row<0x4E>(b); g += dpp_in_row<0x4E>(g);
    a += dpp_in_row<0x141>(a); b += dpp_in_row<0x141>(b); g += dpp_in_row<0x141>(g);
    a += dpp_in_row<0x140>(a); b += dpp_in_row<0x140>(b); g += dpp_in_row<0x140>(g);
}

// jacobi_svd_small for exactly 32 x 32 (rows = cols = 32, column stride ld), the D = 32 cores and
// the Lanczos tridiagonals of 32 steps.  The first 256 threads rotate the 16 pairs of a round
// (a 16-lane row per pair, rows i and i + 16 per lane); the rest only keep the barriers.  Round
// r pairs tournament positions q and 31 - q, whose columns advance by one each round (31 wraps
// to 1, position 0 keeps column 0), the order of rr_col.  Each round's rotation of V is applied
// during the next round (V is not read by the rotations), so its loads and stores overlap the
// next round's dependent chain; the last one is applied after the sweeps.  No row or column
// masks.  Same thresholds, stopping rule and result contract as jacobi_svd_small.
template <int NT, typename P>
__device__ bool jacobi32(P W, P V, int ld, int max_sweeps, CoreShared& sh, int* sweeps_out) {
    static_assert(NT >= 256 && NT % 64 == 0, "sixteen pairs need four waves");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q = wave * 4 + (lane >> 4), ql = lane & 15;
    const bool act = q < 16;
    const double tol2 = (2.220446049250313e-16 * 32.0) * (2.220446049250313e-16 * 32.0);
    double f = 0.0;
    for (int idx = tid; idx < 1024; idx += NT) {
        const double x = W[(idx >> 5) * ld + (idx & 31)];
        f = fma(x, x, f);
    }
    f = wave_sum(f);
    if (lane == 0) sh.rv[wave] = f;
    __syncthreads();
    double fro2 = 0.0;
    for (int w = 0; w < NT / 64; ++w) fro2 += sh.rv[w];
    const double zero2 = kZeroRel * kZeroRel * fro2;
    bool pend = false;
    int pv1 = 0, pv2 = 0;
    double pc = 1.0, ps = 0.0;
    int sweeps = 0;
    bool converged = false;
    for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
        __syncthreads();   // every thread has read sh.rv / the previous sweep's flags
        if (tid == 0) sh.flag = sh.flag_big = 0;
        __syncthreads();
        int p1 = q, p2 = 31 - q;
        for (int round = 0; round < 31; ++round) {
            if (act) {
                const auto w1 = W + p1 * ld + ql;
                const auto w2 = W + p2 * ld + ql;
                const double xa = w1[0], xb = w1[16], ya = w2[0], yb = w2[16];
                const auto u1 = V + pv1 * ld + ql;
                const auto u2 = V + pv2 * ld + ql;
                double vx0 = 0.0, vx1 = 0.0, vy0 = 0.0, vy1 = 0.0;
                if (pend) {
                    vx0 = u1[0];
                    vx1 = u1[16];
                    vy0 = u2[0];
                    vy1 = u2[16];
                }
                double a = fma(xa, xa, xb * xb), b = fma(ya, ya, yb * yb), g = fma(xa, ya, xb * yb);
                row16_sum3(a, b, g);
                if (pend) {
                    u1[0] = pc * vx0 - ps * vy0;
                    u2[0] = ps * vx0 + pc * vy0;
                    u1[16] = pc * vx1 - ps * vy1;
                    u2[16] = ps * vx1 + pc * vy1;
                    pend = false;
                }
                if (a > zero2 && b > zero2 && g * g > tol2 * a * b) {
                    double c, s;
                    jacobi_rotation_fast(a, b, g, &c, &s);
                    w1[0] = c * xa - s * ya;
                    w2[0] = s * xa + c * ya;
                    w1[16] = c * xb - s * yb;
                    w2[16] = s * xb + c * yb;
                    pend = true;
                    pv1 = p1;
                    pv2 = p2;
                    pc = c;
                    ps = s;
                    if (ql == 0) {
                        sh.flag = 1;
                        if (g * g > kQuadRel2 * a * b) sh.flag_big = 1;
                    }
                }
                p1 = q == 0 ? 0 : (p1 == 31 ? 1 : p1 + 1);
                p2 = p2 == 31 ? 1 : p2 + 1;
            }
            __syncthreads();
        }
        sweeps = sweep + 1;
        if (!sh.flag || !sh.flag_big) converged = true;
    }
    if (act && pend) {
        const auto u1 = V + pv1 * ld + ql;
        const auto u2 = V + pv2 * ld + ql;
        const double x0 = u1[0], x1 = u1[16], y0 = u2[0], y1 = u2[16];
        u1[0] = pc * x0 - ps * y0;
        u2[0] = ps * x0 + pc * y0;
        u1[16] = pc * x1 - ps * y1;
        u2[16] = ps * x1 + pc * y1;
    }
    __syncthreads();
    *sweeps_out = sweeps;
    return converged;
}

// Column norms of W (sig[j], j < cols) and their descending order (ties: lower column first).
// With stage (LDS, cols doubles) the ranking reads its copy of the norms instead of sig.
template <int NT = kCoreThreads, typename P = const double*>
__device__ void sorted_norms(P W, int rows, int cols, int ld, double* sig, int* order,
                             double* stage = nullptr) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int j = wave; j < cols; j += (NT / 64)) {
        double s = 0.0;
        for (int i = lane; i < rows; i += 64) s += W[(int64_t)j * ld + i] * W[(int64_t)j * ld + i];
        s = wave_sum(s);
        if (lane == 0) {
            sig[j] = sqrt(s);
            if (stage) stage[j] = sqrt(s);
        }
    }
    __syncthreads();
    const double* sv = stage ? stage : sig;
    for (int j = tid; j < cols; j += NT) {
        const double sj = sv[j];
        int rank = 0;
        for (int q = 0; q < cols; ++q) rank += (sv[q] > sj) || (sv[q] == sj && q < j);
        order[rank] = j;
    }
    __syncthreads();
}

// One 128 x 128 tile (rows i0.., columns j0..) of C (M x N, row-major, leading dimension ldc) =
// A (M x K) . B (K x N) + A2 (M x K2) . B2 (K2 x N), in float64 on MFMA, stored as TC, by the whole
// 1024-thread workgroup: each wave a 32 x 32 block (2 x 2 instructions of 16 x 16 x 4), K staged
// through LDS in chunks of 32 with the loads coalesced along whichever index has unit stride.
// A(i, k) = A[i * ar + k * ac], B(k, j) = B[k * br + j * bc] (likewise A2, B2); stage holds
// 2 * 32 * 128 doubles.
template <typename TC>
__device__ void wg_gemm_tile(const double* __restrict__ A, int64_t ar, int64_t ac, const double* __restrict__ B,
                             int64_t br, int64_t bc, int K, const double* __restrict__ A2, int64_t ar2,
                             int64_t ac2, const double* __restrict__ B2, int64_t br2, int64_t bc2, int K2,
                             TC* __restrict__ C, int64_t ldc, int M, int N, int i0, int j0,
                             double* __restrict__ stage) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 2) * 32, wc = (wave & 3) * 32;
    const int lrow = lane & 15, lk = lane >> 4;
    double* As = stage;              // As[k * 128 + i]
    double* Bs = stage + 32 * 128;   // Bs[k * 128 + j]
    v4d acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int part = 0; part < 2; ++part) {
        const double* PA = part == 0 ? A : A2;
        const double* PB = part == 0 ? B : B2;
        const int64_t pr = part == 0 ? ar : ar2, pc = part == 0 ? ac : ac2;
        const int64_t qr = part == 0 ? br : br2, qc = part == 0 ? bc : bc2;
        const int KK = part == 0 ? K : K2;
        const bool a_kfast = pc == 1, b_jfast = qc == 1;
        for (int k0 = 0; k0 < KK; k0 += 32) {
            for (int e = tid; e < 32 * 128; e += kCoreThreads) {
                const int kk = a_kfast ? (e & 31) : (e >> 7), ii = a_kfast ? (e >> 5) : (e & 127);
                const int gi = i0 + ii, gk = k0 + kk;
                As[kk * 128 + ii] = (gi < M && gk < KK) ? PA[gi * pr + gk * pc] : 0.0;
                const int kb = b_jfast ? (e >> 7) : (e & 31), jj = b_jfast ? (e & 127) : (e >> 5);
                const int gj = j0 + jj, gkb = k0 + kb;
                Bs[kb * 128 + jj] = (gj < N && gkb < KK) ? PB[gkb * qr + gj * qc] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < 32; kk += 4) {
                const int k = kk + lk;
                const double a0 = As[k * 128 + wr + lrow], a1 = As[k * 128 + wr + 16 + lrow];
                const double b0 = Bs[k * 128 + wc + lrow], b1 = Bs[k * 128 + wc + 16 + lrow];
                acc[0][0] = Mma<double>::run(a0, b0, acc[0][0]);
                acc[0][1] = Mma<double>::run(a0, b1, acc[0][1]);
                acc[1][0] = Mma<double>::run(a1, b0, acc[1][0]);
                acc[1][1] = Mma<double>::run(a1, b1, acc[1][1]);
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = i0 + wr + 16 * x + Mma<double>::row(lane, r);
                const int gj = j0 + wc + 16 * y + lrow;
                if (gi < M && gj < N) C[(int64_t)gi * ldc + gj] = (TC)acc[x][y][r];
            }
}

// C (M x N, row-major, leading dimension ldc) = A (M x K) . B (K x N): every 128 x 128 tile by
// the whole workgroup (wg_gemm_tile).  Ends with a barrier.
__device__ void wg_gemm_f64(const double* __restrict__ A, int64_t ar, int64_t ac, const double* __restrict__ B,
                            int64_t br, int64_t bc, double* __restrict__ C, int64_t ldc, int M, int N, int K,
                            double* __restrict__ stage) {
    for (int i0 = 0; i0 < M; i0 += 128)
        for (int j0 = 0; j0 < N; j0 += 128)
            wg_gemm_tile<double>(A, ar, ac, B, br, bc, K, nullptr, 0, 0, nullptr, 0, 0, 0, C, ldc, M, N, i0, j0, stage);
    __syncthreads();
}

// C (M x N) = A (M x K) . B (K x N) in float64 on MFMA for narrow N, operands read straight from
// memory: each wave owns 16 x 32 blocks of C (two 16 x 16 x 4 instructions per step of 4 along
// K).  A(i, k) = A[i * ar + k * ac], B(k, j) = B[k * br + j * bc], C(i, j) = C[i * cr + j * cc],
// stored as TC.  Ends with a barrier.
// PB: B's pointer type (const double*, or LdsPtr for a B staged in LDS)
template <typename TC, int NW = kCoreWaves, typename PB = const double*>
__device__ void wg_gemm_narrow_to(const double* __restrict__ A, int64_t ar, int64_t ac,
                                  PB __restrict__ B, int64_t br, int64_t bc, TC* __restrict__ C,
                                  int64_t cr, int64_t cc, int M, int N, int K) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int mb = (M + 15) / 16, nb = (N + 31) / 32;
    for (int blk = wave; blk < mb * nb; blk += NW) {
        const int i0 = (blk % mb) * 16, j0 = (blk / mb) * 32;
        const int gi = i0 + lr, gj0 = j0 + lr, gj1 = j0 + 16 + lr;
        const bool ri = gi < M, c0 = gj0 < N, c1 = gj1 < N;
        v4d acc0 = v4d{0.0, 0.0, 0.0, 0.0}, acc1 = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int k0 = 0; k0 < K; k0 += 4) {
            const int k = k0 + lk;
            const bool kk = k < K;
            const double a = (ri && kk) ? A[(int64_t)gi * ar + (int64_t)k * ac] : 0.0;
            const double b0 = (kk && c0) ? B[(int64_t)k * br + (int64_t)gj0 * bc] : 0.0;
            const double b1 = (kk && c1) ? B[(int64_t)k * br + (int64_t)gj1 * bc] : 0.0;
            acc0 = Mma<double>::run(a, b0, acc0);
            acc1 = Mma<double>::run(a, b1, acc1);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = i0 + Mma<double>::row(lane, r);
            if (row < M) {
                if (c0) C[(int64_t)row * cr + (int64_t)gj0 * cc] = (TC)acc0[r];
                if (c1) C[(int64_t)row * cr + (int64_t)gj1 * cc] = (TC)acc1[r];
            }
        }
    }
    __syncthreads();
}

// wg_gemm_narrow_to into a row-major float64 C with leading dimension ldc.
template <int NW = kCoreWaves, typename PB = const double*>
__device__ inline void wg_gemm_f64_narrow(const double* __restrict__ A, int64_t ar, int64_t ac,
                                          PB __restrict__ B, int64_t br, int64_t bc,
                                          double* __restrict__ C, int64_t ldc, int M, int N, int K) {
    wg_gemm_narrow_to<double, NW, PB>(A, ar, ac, B, br, bc, C, ldc, 1, M, N, K);
}

// Block one-sided Jacobi for the global cores (64 < D <= 256): the columns of the matrix it
// rotates (here called W; the core's transpose when kBJTransposed) are cut into blocks of kBJCols, and the blocks follow a round-robin tournament, one launch per round and one
// workgroup per block pair.  A workgroup stages its two blocks of W in LDS and rotates every cross
// pair once (16 steps of 16 disjoint pairs); in the first round of a sweep each block is met for
// the first time, so the workgroup also rotates the pairs inside its two blocks (a 32-column
// tournament, 31 steps).  Every column pair is thus rotated once per sweep, as in the
// one-workgroup Jacobi, with the same rotation, thresholds and stopping rule.  A pair is rotated
// by one 16-lane DPP row (16 rows of W per lane), four pairs per wave; the rotations of the
// launch are accumulated in a 32 x 32 matrix Q and applied to the two blocks of V (staged in LDS
// with W) once at the end, V <- V Q on the MFMA.
constexpr int kBJCols = 16;
constexpr int kBJRows = 256;
constexpr int kBJThreads = 256;
constexpr int kBJKR = kBJRows / 16;   // rows of W per lane
constexpr int kBJSweeps = 18;   // sweeps issued as block launches; a core still rotating after
                                // them finishes in the one-workgroup Jacobi
constexpr size_t kBJLdsBytes = (size_t)(4 * kBJCols * kBJRows + 4 * kBJCols * kBJCols) * sizeof(double);

// Per-core block-Jacobi state after the singular values: ranks (two ints), ||W||_F^2, and one
// flag per issued sweep (set when the sweep made a rotation above the quadratic-convergence level).
__device__ inline int* core_ranks(double* gsig, int D) { return (int*)(gsig + 2 * D); }
__device__ inline double* core_fro2(double* gsig, int D) { return gsig + 2 * D + 1; }
__device__ inline int* core_bigflags(double* gsig, int D) { return (int*)(gsig + 2 * D + 2); }
// rows and columns of the matrix the block launches rotate (after the sweep flags)
__device__ inline int* core_jdims(double* gsig, int D) { return core_bigflags(gsig, D) + kBJSweeps; }
// The block launches rotate the columns of W^T = R~_B R~_A^T (rb x ra) and accumulate U: on these
// graded cores that takes about 40% fewer sweeps than W's columns (same stopping rule).
constexpr bool kBJTransposed = true;

__global__ __launch_bounds__(kBJThreads) void block_jacobi_kernel(const CoreDesc* __restrict__ descs, int per_core,
                                                                  int sweep, int round) {
    extern __shared__ double lds[];
    __shared__ int s_big;
    constexpr int NC = 2 * kBJCols;
    const int ci = blockIdx.x / per_core, q = blockIdx.x - ci * per_core;
    const CoreDesc& d = descs[ci];
    const int D = d.D;
    const int64_t DD = (int64_t)D * D;
    double* W = d.work + 2 * DD;
    double* V = W + DD;
    double* gsig = d.work + 4 * DD;
    int* big = core_bigflags(gsig, D);
    if (sweep > 0 && big[sweep - 1] == 0) return;   // the previous sweep converged
    const int* jd = core_jdims(gsig, D);
    const int ra = jd[0], rb = jd[1];   // rows, columns of the rotated matrix
    int nb = (rb + kBJCols - 1) / kBJCols;
    nb += nb & 1;
    if (q >= nb / 2 || round >= nb - 1) return;
    const int b1 = rr_col(q, round, nb), b2 = rr_col(nb - 1 - q, round, nb);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int quarter = lane >> 4, ql = lane & 15;
    auto gcol = [&](int c) { return c < kBJCols ? b1 * kBJCols + c : b2 * kBJCols + c - kBJCols; };
    double* lw = lds;                    // local column c of W at lw + c * kBJRows
    double* lv = lw + NC * kBJRows;      // the same for V
    double* lq = lv + NC * kBJRows;      // Q, column c at lq + c * NC
    {
        // every load of the two blocks issued before the first LDS write (the columns were last
        // written by other workgroups, possibly on other dies: far memory latency)
        constexpr int kPer = NC * kBJRows / kBJThreads;
        double xw[kPer], xv[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int idx = tid + u * kBJThreads;
            const int c = idx / kBJRows, i = idx - c * kBJRows;
            const int g = gcol(c);
            xw[u] = (g < rb && i < ra) ? W[(int64_t)g * D + i] : 0.0;
            xv[u] = (g < rb && i < rb) ? V[(int64_t)g * D + i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            lw[tid + u * kBJThreads] = xw[u];
            lv[tid + u * kBJThreads] = xv[u];
        }
        for (int idx = tid; idx < NC * NC; idx += kBJThreads) lq[idx] = (idx / NC == idx % NC) ? 1.0 : 0.0;
    }
    if (tid == 0) s_big = 0;
    __syncthreads();
    const double zero2 = kZeroRel * kZeroRel * *core_fro2(gsig, D);
    const double tol = 2.220446049250313e-16 * (double)max(ra, 16);
    const int pi = wave * 4 + quarter;   // this 16-lane row's pair
    if (round > 0) {
        // cross pairs only: this row keeps its first-block column (and its column of Q) in
        // registers for the 16 steps, and meets the second block's columns in turn
        const int p1 = pi;
        const bool in1 = gcol(p1) < rb;
        double x[kBJKR], qx[NC / 16];
#pragma unroll
        for (int k = 0; k < kBJKR; ++k) x[k] = lw[p1 * kBJRows + ql + 16 * k];
#pragma unroll
        for (int k = 0; k < NC / 16; ++k) qx[k] = lq[p1 * NC + ql + 16 * k];
        double a = row16_sum([&] {
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int k = 0; k < kBJKR; k += 2) {
                s0 = fma(x[k], x[k], s0);
                s1 = fma(x[k + 1], x[k + 1], s1);
            }
            return s0 + s1;
        }());
        for (int t = 0; t < kBJCols; ++t) {
            const int p2 = kBJCols + ((pi + t) & (kBJCols - 1));
            double* w2 = lw + p2 * kBJRows;
            double y[kBJKR];
#pragma unroll
            for (int k = 0; k < kBJKR; ++k) y[k] = w2[ql + 16 * k];
            double b0 = 0.0, b1 = 0.0, g0 = 0.0, g1 = 0.0;
#pragma unroll
            for (int k = 0; k < kBJKR; k += 2) {
                b0 = fma(y[k], y[k], b0);
                g0 = fma(x[k], y[k], g0);
                b1 = fma(y[k + 1], y[k + 1], b1);
                g1 = fma(x[k + 1], y[k + 1], g1);
            }
            const double b = row16_sum(b0 + b1), g = row16_sum(g0 + g1);
            if (in1 && gcol(p2) < rb && a > zero2 && b > zero2 && g * g > tol * tol * a * b) {
                double c, sn;
                jacobi_rotation_fast(a, b, g, &c, &sn);
                if (ql == 0 && g * g > kQuadRel2 * a * b) s_big = 1;
                double a0 = 0.0, a1 = 0.0;
#pragma unroll
                for (int k = 0; k < kBJKR; ++k) {
                    const double xn = c * x[k] - sn * y[k];
                    w2[ql + 16 * k] = sn * x[k] + c * y[k];
                    x[k] = xn;
                    if (k & 1) a1 = fma(xn, xn, a1);
                    else a0 = fma(xn, xn, a0);
                }
                a = row16_sum(a0 + a1);
                double* q2 = lq + p2 * NC;
#pragma unroll
                for (int k = 0; k < NC / 16; ++k) {
                    const double u1 = qx[k], u2 = q2[ql + 16 * k];
                    qx[k] = c * u1 - sn * u2;
                    q2[ql + 16 * k] = sn * u1 + c * u2;
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < kBJKR; ++k) lw[p1 * kBJRows + ql + 16 * k] = x[k];
#pragma unroll
        for (int k = 0; k < NC / 16; ++k) lq[p1 * NC + ql + 16 * k] = qx[k];
        __syncthreads();
    }
    for (int t = 0; t < (round == 0 ? NC - 1 : 0); ++t) {
        const int p1 = rr_col(pi, t, NC), p2 = rr_col(NC - 1 - pi, t, NC);
        double* w1 = lw + p1 * kBJRows;
        double* w2 = lw + p2 * kBJRows;
        double x[kBJKR], y[kBJKR];
#pragma unroll
        for (int k = 0; k < kBJKR; ++k) {
            x[k] = w1[ql + 16 * k];
            y[k] = w2[ql + 16 * k];
        }
        double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0, g0 = 0.0, g1 = 0.0;
#pragma unroll
        for (int k = 0; k < kBJKR; k += 2) {
            a0 = fma(x[k], x[k], a0);
            b0 = fma(y[k], y[k], b0);
            g0 = fma(x[k], y[k], g0);
            a1 = fma(x[k + 1], x[k + 1], a1);
            b1 = fma(y[k + 1], y[k + 1], b1);
            g1 = fma(x[k + 1], y[k + 1], g1);
        }
        const double a = row16_sum(a0 + a1), b = row16_sum(b0 + b1), g = row16_sum(g0 + g1);
        if (gcol(p1) < rb && gcol(p2) < rb && a > zero2 && b > zero2 && g * g > tol * tol * a * b) {
            double c, sn;
            jacobi_rotation_fast(a, b, g, &c, &sn);
#pragma unroll
            for (int k = 0; k < kBJKR; ++k) {
                w1[ql + 16 * k] = c * x[k] - sn * y[k];
                w2[ql + 16 * k] = sn * x[k] + c * y[k];
            }
            double* q1 = lq + p1 * NC;
            double* q2 = lq + p2 * NC;
#pragma unroll
            for (int k = 0; k < NC / 16; ++k) {
                const double u1 = q1[ql + 16 * k], u2 = q2[ql + 16 * k];
                q1[ql + 16 * k] = c * u1 - sn * u2;
                q2[ql + 16 * k] = sn * u1 + c * u2;
            }
            if (ql == 0 && g * g > kQuadRel2 * a * b) s_big = 1;
        }
        __syncthreads();
    }
    for (int idx = tid; idx < NC * kBJRows; idx += kBJThreads) {
        const int c = idx / kBJRows, i = idx - c * kBJRows;
        const int g = gcol(c);
        if (g < rb && i < ra) W[(int64_t)g * D + i] = lw[idx];
    }
    // V <- V Q on the MFMA (16 x 16 x 4): a wave per 64 rows of V, Q's fragments held in registers,
    // a row block's fragments of V read from LDS before its products; the two 16-column halves
    // of the result are the two blocks of V
    {
        const int lr = lane & 15, lk = lane >> 4;
        double qb0[NC / 4], qb1[NC / 4];
#pragma unroll
        for (int u = 0; u < NC / 4; ++u) {
            qb0[u] = lq[lr * NC + 4 * u + lk];
            qb1[u] = lq[(kBJCols + lr) * NC + 4 * u + lk];
        }
        const int gA = b1 * kBJCols + lr, gB = b2 * kBJCols + lr;
        for (int i1 = wave * 64; i1 < wave * 64 + 64 && i1 < rb; i1 += 16) {
            double av[NC / 4];
#pragma unroll
            for (int u = 0; u < NC / 4; ++u) av[u] = lv[(4 * u + lk) * kBJRows + i1 + lr];
            v4d acc0 = v4d{0.0, 0.0, 0.0, 0.0}, acc1 = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int u = 0; u < NC / 4; ++u) {
                acc0 = Mma<double>::run(av[u], qb0[u], acc0);
                acc1 = Mma<double>::run(av[u], qb1[u], acc1);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = i1 + Mma<double>::row(lane, r);
                if (row < rb) {
                    if (gA < rb) V[(int64_t)gA * D + row] = acc0[r];
                    if (gB < rb) V[(int64_t)gB * D + row] = acc1[r];
                }
            }
        }
    }
    if (tid == 0 && s_big) big[sweep] = 1;
}

// phase 0: the whole compression.  Global variant only: phase 1 stops after the matrix for
// block_jacobi_kernel (the core W, or W^T when kBJTransposed) and V = I, with ranks, the rotated
// matrix's size, ||W||_F^2 and cleared sweep flags in the workspace; phase 2 starts from the
// rotated matrix and V, rebuilds W (columns u s) and V (columns v) from the transposed problem,
// and does the rest.
template <bool kLds, typename Tp>
__global__ __launch_bounds__(kLds ? kCoreLdsThreads : kCoreThreads) void core_kernel(const CoreDesc* __restrict__ descs, int max_sweeps,
                                                            double* __restrict__ stat_disc,
                                                            int32_t* __restrict__ stat_tie,
                                                            int32_t* __restrict__ stat_sweeps, int phase) {
    extern __shared__ double lds[];
    __shared__ CoreShared sh;
    constexpr int NT = kLds ? kCoreLdsThreads : kCoreThreads;
    const CoreDesc& d = descs[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int D = d.D;
    const int64_t DD = (int64_t)D * D;
    // LDS variant (D <= 64): W, V, R~_A, R~_B all in LDS; else all in the global workspace
    double* W = kLds ? lds : d.work + 2 * DD;    // column-major core, column j at W + j*D
    double* V = W + DD;                          // column-major right singular vectors
    double* Ra = kLds ? lds + 2 * DD : d.work;   // row-major R~_A, row t at Ra + t*D
    double* Rb = Ra + DD;
    double* gsig = d.work + 4 * DD;              // global copies read by the reverse pass
    int* gorder = (int*)(gsig + D);
    int* chosen = gorder + D;
    __shared__ double lsig[kLds ? kCoreLdsMaxD : 1];
    __shared__ int lorder[kLds ? kCoreLdsMaxD : 1];
    double* sig = kLds ? lsig : gsig;
    int* order = kLds ? lorder : gorder;

    // ---- reduced factors R~_A (ra x D), R~_B (rb x D)
    int ra, rb;
    if (!kLds && phase == 2) {
        ra = core_ranks(gsig, D)[0];
        rb = core_ranks(gsig, D)[1];
    } else if (kLds) {
        // split-K Gram partials summed into LDS (side A into W, side B into V), explicit
        // factors copied; then one wave per side runs its pivoted Cholesky
        const int DDi = D * D;
        for (int side = 0; side < 2; ++side) {
            const double* gram = side == 0 ? d.gram_a : d.gram_b;
            if (gram) {
                const int splits = side == 0 ? d.splits_a : d.splits_b;
                double* G = side == 0 ? W : V;
                for (int idx = tid; idx < DDi; idx += NT) {
                    const double* g = gram + idx;
                    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
                    int p = 0;
                    for (; p + 4 <= splits; p += 4) {
                        s0 += g[(int64_t)p * DD];
                        s1 += g[(int64_t)(p + 1) * DD];
                        s2 += g[(int64_t)(p + 2) * DD];
                        s3 += g[(int64_t)(p + 3) * DD];
                    }
                    for (; p < splits; ++p) s0 += g[(int64_t)p * DD];
                    G[idx] = (s0 + s1) + (s2 + s3);
                }
            } else {
                const int rows = side == 0 ? d.rows_a : d.rows_b;
                const double* fac = side == 0 ? d.fac_a : d.fac_b;
                double* R = side == 0 ? Ra : Rb;
                for (int idx = tid; idx < rows * D; idx += NT) R[idx] = fac[idx];
            }
        }
        __syncthreads();
        if (wave < 2) {
            const double* gram = wave == 0 ? d.gram_a : d.gram_b;
            int r = wave == 0 ? d.rows_a : d.rows_b;
            if (gram)
                r = D <= 32 ? pivoted_cholesky_wave_reg<32>(wave == 0 ? W : V, D, wave == 0 ? Ra : Rb)
                            : pivoted_cholesky_wave(wave == 0 ? W : V, D, wave == 0 ? Ra : Rb);
            if (lane == 0) sh.ri[wave] = r;
        }
        __syncthreads();
        ra = sh.ri[0];
        rb = sh.ri[1];
    } else {
        int rk[2];
        for (int side = 0; side < 2; ++side) {
            const double* gram = side == 0 ? d.gram_a : d.gram_b;
            const double* fac = side == 0 ? d.fac_a : d.fac_b;
            double* R = side == 0 ? Ra : Rb;
            if (gram) {
                const int splits = side == 0 ? d.splits_a : d.splits_b;
                for (int64_t idx = tid; idx < DD; idx += NT) {
                    double s = 0.0;
                    for (int p = 0; p < splits; ++p) s += gram[(int64_t)p * DD + idx];
                    W[idx] = s;
                }
                __syncthreads();
                rk[side] = D <= kCholBlkMaxD ? pivoted_cholesky_blocked(W, D, R, lds, sh)
                           : D <= kCholLLMaxD  ? pivoted_cholesky_ll(W, D, R, lds, sh)
                                               : pivoted_cholesky(W, D, R, chosen, sh);
            } else {
                const int rows = side == 0 ? d.rows_a : d.rows_b;
                for (int64_t idx = tid; idx < (int64_t)rows * D; idx += NT) R[idx] = fac[idx];
                rk[side] = rows;
            }
            __syncthreads();
        }
        ra = rk[0];
        rb = rk[1];
    }

    // ---- core W = R~_A R~_B^T  (ra x rb), V = I
    if constexpr (!kLds) {
        // column j of W is row j of R~_B R~_A^T: one workgroup GEMM on the MFMA (LDS staging);
        // for the block launches the transpose W^T (column i = row i of R~_A R~_B^T)
        if (phase == 1 && kBJTransposed) wg_gemm_f64(Ra, D, 1, Rb, 1, D, W, D, ra, rb, D, lds);
        else if (phase != 2) wg_gemm_f64(Rb, D, 1, Ra, 1, D, W, D, rb, ra, D, lds);
    } else
    for (int idx = tid; idx < ra * rb; idx += NT) {
        const int j = idx / ra, i = idx - j * ra;
        const double* x = Ra + (int64_t)i * D;
        const double* y = Rb + (int64_t)j * D;
        // start each thread at its own offset so neighbouring rows hit different LDS banks
        int q = i % D;
        double s = 0.0;
        for (int c = 0; c < D; ++c) {
            s += x[q] * y[q];
            q = q + 1 == D ? 0 : q + 1;
        }
        W[(int64_t)j * D + i] = s;
    }
    // V = I, the size of the rotated matrix's column count
    const int nv = (!kLds && phase == 1 && kBJTransposed) ? ra : rb;
    if (phase != 2)
        for (int idx = tid; idx < nv * nv; idx += NT) {
            const int j = idx / nv, i = idx - j * nv;
            V[(int64_t)j * D + i] = (i == j) ? 1.0 : 0.0;
        }
    __syncthreads();
    if (!kLds && phase == 1) {
        // ||W||_F^2 over the rotated matrix (rows fr, columns fc, column j at W + j * D)
        const int fr = kBJTransposed ? rb : ra, fc = kBJTransposed ? ra : rb;
        double f = 0.0;
        for (int idx = tid; idx < fr * fc; idx += NT) {
            const int j = idx / fr, i = idx - j * fr;
            const double x = W[(int64_t)j * D + i];
            f = fma(x, x, f);
        }
        f = wave_sum(f);
        if (lane == 0) sh.rv[wave] = f;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int w = 0; w < kCoreWaves; ++w) t += sh.rv[w];
            *core_fro2(gsig, D) = t;
            core_ranks(gsig, D)[0] = ra;
            core_ranks(gsig, D)[1] = rb;
            core_jdims(gsig, D)[0] = kBJTransposed ? rb : ra;
            core_jdims(gsig, D)[1] = kBJTransposed ? ra : rb;
        }
        for (int t = tid; t < kBJSweeps; t += NT) core_bigflags(gsig, D)[t] = 0;
        return;
    }

    // ---- one-sided (Hestenes) Jacobi on the columns of W, accumulating V
    int sweeps = 0;
    bool converged;
    if (!kLds && phase == 2) {
        // sweeps made by the block launches: the first one without a large rotation ended them
        const int* big = core_bigflags(gsig, D);
        const int jr = core_jdims(gsig, D)[0], jc = core_jdims(gsig, D)[1];
        const int issued = min(kBJSweeps, max_sweeps);
        converged = jc <= 1;
        sweeps = converged ? 0 : issued;
        for (int t = 0; t < issued && !converged; ++t)
            if (big[t] == 0) {
                sweeps = t + 1;
                converged = true;
            }
        if (!converged && max_sweeps > issued) {
            int more = 0;
            converged = jacobi_svd_256(W, V, jr, jc, D, max_sweeps - issued, sh, &more);
            sweeps += more;
        }
        if (kBJTransposed) {
            // W^T V = (V_W s) with V holding U: column j of the rotated W^T is v_j s_j, column j of
            // V is u_j.  Rebuild W (columns u_t s_t) and V (columns v_t) in descending order
            // through the scratch after the workspace's sorted projector columns.
            sorted_norms<NT>(W, jr, jc, D, sig, order, lds);
            double* Wn = d.work + 4 * DD + 4 * D + 2 * (int64_t)D * d.chi_new;
            double* Vn = Wn + DD;
            const int m = min(ra, rb);
            for (int idx = tid; idx < rb * D; idx += NT) {
                const int t = idx / D, i = idx - t * D;
                const int j = t < m ? order[t] : -1;
                const double sj = j >= 0 ? sig[j] : 0.0;
                const bool ok = sj > 0.0;
                Wn[idx] = (ok && i < ra) ? V[(int64_t)j * D + i] * sj : 0.0;
                Vn[idx] = (ok && i < rb) ? W[(int64_t)j * D + i] / sj : 0.0;
            }
            __syncthreads();
            for (int idx = tid; idx < rb * D; idx += NT) {
                W[idx] = Wn[idx];
                V[idx] = Vn[idx];
            }
            __syncthreads();
        }
    } else if constexpr (kLds)   // ra, rb <= D <= 64
        converged = (ra == 32 && rb == 32)   ? jacobi32<NT>(W, V, D, max_sweeps, sh, &sweeps)
                    : (ra <= 32 && rb <= 32) ? jacobi_svd_small<NT, 2>(W, V, ra, rb, D, max_sweeps, sh, &sweeps)
                                             : jacobi_svd_small<NT>(W, V, ra, rb, D, max_sweeps, sh, &sweeps);
    else
        converged = (ra <= 32 && rb <= 32)     ? jacobi_svd_small<NT, 2>(W, V, ra, rb, D, max_sweeps, sh, &sweeps)
                    : (ra <= 64 && rb <= 64)   ? jacobi_svd_small<NT>(W, V, ra, rb, D, max_sweeps, sh, &sweeps)
                    : (ra <= 256 && rb <= 256) ? jacobi_svd_256(W, V, ra, rb, D, max_sweeps, sh, &sweeps)
                                               : jacobi_svd(W, V, ra, rb, D, max_sweeps, sh, &sweeps);

    // ---- singular values and descending order (ties: lower column first)
    sorted_norms<NT>(W, ra, rb, D, sig, order, kLds ? nullptr : lds);
    double fro = 0.0;
    {
        double f4[4] = {0.0, 0.0, 0.0, 0.0};
        int j = 0;
        for (; j + 4 <= rb; j += 4)
#pragma unroll
            for (int e = 0; e < 4; ++e) f4[e] = fma(sig[j + e], sig[j + e], f4[e]);
        for (; j < rb; ++j) f4[0] = fma(sig[j], sig[j], f4[0]);
        fro = (f4[0] + f4[1]) + (f4[2] + f4[3]);
    }
    fro = sqrt(fro);

    // ---- projectors P_L (D x chi') and P_R (chi' x D)
    const int cn = d.chi_new;
    const double smax = rb > 0 ? sig[order[0]] : 0.0;
    Tp* PL = (Tp*)d.p_left;
    Tp* PR = (Tp*)d.p_right;
    if constexpr (!kLds) {
        // the kept columns of V and W, sorted and scaled by sigma^-1/2 and sigma^-3/2 (zero where
        // the projector column is zero), then P_L = R~_B^T Vs and P_R^T = R~_A^T Ws on the MFMA
        double* Vs = d.work + 4 * DD + 4 * D;
        double* Ws = Vs + (int64_t)D * cn;
        for (int idx = tid; idx < D * cn; idx += NT) {
            const int t = idx / D, i = idx - t * D;
            const int j = t < rb ? order[t] : -1;
            const double s = j >= 0 ? sig[j] : 0.0;
            const bool keep = s > kNoiseRel * smax && s > 4.0 * kZeroRel * fro && s >= d.cutoff * smax;
            const double rs = keep ? sqrt(s) : 1.0;
            Vs[idx] = (keep && i < rb) ? V[(int64_t)j * D + i] / rs : 0.0;
            Ws[idx] = (keep && i < ra) ? W[(int64_t)j * D + i] / (s * rs) : 0.0;
        }
        __syncthreads();
        wg_gemm_narrow_to<Tp>(Rb, 1, D, Vs, 1, D, PL, cn, 1, D, cn, rb);
        wg_gemm_narrow_to<Tp>(Ra, 1, D, Ws, 1, D, PR, 1, D, D, cn, ra);
    } else
    for (int idx = tid; idx < D * cn; idx += NT) {
        const int dd = idx / cn, t = idx - dd * cn;
        const int j = t < rb ? order[t] : -1;
        const double s = j >= 0 ? sig[j] : 0.0;
        double pl = 0.0, pr = 0.0;
        // singular values below kNoiseRel * sigma_1 are numerical zeros of an FP64 core: their
        // vectors are rounding noise, and dividing by them would amplify it (they change A B by
        // less than kNoiseRel relative when dropped)
        if (s > kNoiseRel * smax && s > 4.0 * kZeroRel * fro && s >= d.cutoff * smax) {
            const double* v = V + (int64_t)j * D;
            const double* u = W + (int64_t)j * D;
            // four partial sums per dot product, so that the LDS loads overlap
            double l4[4] = {0.0, 0.0, 0.0, 0.0}, r4[4] = {0.0, 0.0, 0.0, 0.0};
            int i = 0;
            for (; i + 4 <= rb; i += 4)
#pragma unroll
                for (int e = 0; e < 4; ++e) l4[e] = fma(Rb[(int64_t)(i + e) * D + dd], v[i + e], l4[e]);
            for (; i < rb; ++i) l4[0] = fma(Rb[(int64_t)i * D + dd], v[i], l4[0]);
            i = 0;
            for (; i + 4 <= ra; i += 4)
#pragma unroll
                for (int e = 0; e < 4; ++e) r4[e] = fma(u[i + e], Ra[(int64_t)(i + e) * D + dd], r4[e]);
            for (; i < ra; ++i) r4[0] = fma(u[i], Ra[(int64_t)i * D + dd], r4[0]);
            pl = (l4[0] + l4[1]) + (l4[2] + l4[3]);
            pr = (r4[0] + r4[1]) + (r4[2] + r4[3]);
            const double rs = sqrt(s);
            pl /= rs;
            pr /= (s * rs);
        }
        PL[(int64_t)dd * cn + t] = (Tp)pl;
        PR[(int64_t)t * D + dd] = (Tp)pr;
    }

    // ---- what the reverse pass reads back: factors, core, V, singular values, order (LDS
    // variant) and the ranks
    if (kLds && d.keep_out) {
        double* gw = d.work;
        for (int idx = tid; idx < 4 * D * D; idx += NT) {
            const int part = idx / (D * D), off = idx - part * D * D;
            const double* src = part == 0 ? Ra : part == 1 ? Rb : part == 2 ? W : V;
            gw[idx] = src[off];
        }
        for (int j = tid; j < rb; j += NT) {
            gsig[j] = sig[j];
            gorder[j] = order[j];
        }
    }
    if (tid == 0) {
        int* ranks = (int*)(gsig + 2 * D);
        ranks[0] = ra;
        ranks[1] = rb;
    }

    // ---- diagnostics
    if (tid == 0) {
        double tot = 0.0, disc = 0.0;
        for (int t = 0; t < rb; ++t) {
            const double s = sig[order[t]];
            tot += s * s;
            if (t >= cn) disc += s * s;
        }
        stat_disc[d.stat] = tot > 0.0 ? disc / tot : 0.0;
        const double s_last = (cn - 1 < rb) ? sig[order[cn - 1]] : 0.0;
        const double s_next = (cn < rb) ? sig[order[cn]] : 0.0;
        stat_tie[d.stat] = (d.kmin > cn && s_last > 1e-13 * smax && s_last - s_next <= 1e-12 * smax) ? 1 : 0;
        stat_sweeps[d.stat] = converged ? sweeps : -1 - sweeps;   // negative: not converged
    }
}


// ------------------------------------------------------------------------------------------
// Large cores: Golub-Kahan-Lanczos truncated SVD of M = (A/s_a)(B/s_b), one workgroup per
// compression, reading the two tensors through their matricisation Views.
// ------------------------------------------------------------------------------------------
__device__ double block_sum(double v, CoreShared& sh) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) sh.rv[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < kCoreWaves; ++w) t += sh.rv[w];
    __syncthreads();
    return t;
}

// x (n) -= Q[:, :k] (Q[:, :k]^T x), twice (classical Gram-Schmidt with reorthogonalisation).
__device__ void reorthogonalise(double* x, const double* Q, int n, int k, double* coef) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int pass = 0; pass < 2; ++pass) {
        for (int j = wave; j < k; j += kCoreWaves) {
            const double* q = Q + (int64_t)j * n;
            double c = 0.0;
            for (int i = lane; i < n; i += 64) c += q[i] * x[i];
            c = wave_sum(c);
            if (lane == 0) coef[j] = c;
        }
        __syncthreads();
        for (int i = tid; i < n; i += kCoreThreads) {
            double acc = x[i];
            for (int j = 0; j < k; ++j) acc -= Q[(int64_t)j * n + i] * coef[j];
            x[i] = acc;
        }
        __syncthreads();
    }
}


// y[r] = scale * sum_c X[ro[r] + co[c]] x[c]  (r < nrow): lanes run along the unit-stride side.
template <typename Tin>
__device__ void mv_rows(const Tin* __restrict__ X, const uint32_t* ro, const uint32_t* co, int nrow, int ncol,
                        bool col_unit, const double* x, double* y, double scale) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (col_unit) {   // a wave per row, lanes along the (contiguous) columns
        for (int r = wave; r < nrow; r += kCoreWaves) {
            const uint32_t base = ro[r];
            double acc = 0.0;
            for (int c = lane; c < ncol; c += 64) acc += (double)X[base + co[c]] * x[c];
            acc = wave_sum(acc);
            if (lane == 0) y[r] = acc * scale;
        }
    } else {          // a thread per row: neighbouring lanes read neighbouring rows
        for (int r = tid; r < nrow; r += kCoreThreads) {
            const uint32_t base = ro[r];
            double acc = 0.0;
            for (int c = 0; c < ncol; ++c) acc += (double)X[base + co[c]] * x[c];
            y[r] = acc * scale;
        }
    }
}

// y[c] = scale * sum_r X[ro[r] + co[c]] x[r]  (c < ncol)
template <typename Tin>
__device__ void mv_cols(const Tin* __restrict__ X, const uint32_t* ro, const uint32_t* co, int nrow, int ncol,
                        bool row_unit, const double* x, double* y, double scale) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (row_unit) {   // a wave per column, lanes along the (contiguous) rows
        for (int c = wave; c < ncol; c += kCoreWaves) {
            const uint32_t off = co[c];
            double acc = 0.0;
            for (int r = lane; r < nrow; r += 64) acc += (double)X[ro[r] + off] * x[r];
            acc = wave_sum(acc);
            if (lane == 0) y[c] = acc * scale;
        }
    } else {          // a thread per column: neighbouring lanes read neighbouring columns
        for (int c = tid; c < ncol; c += kCoreThreads) {
            const uint32_t off = co[c];
            double acc = 0.0;
            for (int r = 0; r < nrow; ++r) acc += (double)X[ro[r] + off] * x[r];
            y[c] = acc * scale;
        }
    }
}

// deterministic, generic start / restart vector
__device__ inline double probe_entry(int i, int r) {
    const double x = (double)i;
    return cos(0.7 * x + 0.3 + 1.1 * r) + 0.5 * sin(1.9 * x + 0.7 * r + 0.1);
}

template <typename Tin, typename Tp>
__global__ __launch_bounds__(kCoreThreads) void lanczos_kernel(const LanczosDesc* __restrict__ descs,
                                                               const double* __restrict__ scales, int max_sweeps,
                                                               double* __restrict__ stat_disc,
                                                               int32_t* __restrict__ stat_tie,
                                                               int32_t* __restrict__ stat_sweeps) {
    extern __shared__ double lds[];
    __shared__ CoreShared sh;
    __shared__ double coef[kLanczosMaxSteps + 1];
    const LanczosDesc& d = descs[blockIdx.x];
    const int tid = threadIdx.x;
    const int ma = d.ma, mb = d.mb, D = d.D, cn = d.chi_new, smax_steps = d.s_max, ls = d.s_max + 1;
    const Tin* __restrict__ A = (const Tin*)d.A;
    const Tin* __restrict__ B = (const Tin*)d.B;
    const double ia = inv_scale(scales, d.scale_a), ib = inv_scale(scales, d.scale_b);
    const bool a_col_unit = d.va.col_unit != 0, a_row_unit = d.va.row_unit != 0;
    const bool b_col_unit = d.vb.col_unit != 0, b_row_unit = d.vb.row_unit != 0;

    double* U = d.work;                                   // ma x s_max
    double* V = U + (int64_t)ma * smax_steps;             // mb x (s_max + 1)
    double* Ut = V + (int64_t)mb * (smax_steps + 1);      // ma x cn  Ritz vectors of M
    double* Vt = Ut + (int64_t)ma * cn;                   // mb x cn
    double* t1 = Vt + (int64_t)mb * cn;                   // D
    double* t2 = t1 + D;                                  // D
    double* alpha = t2 + D;                               // s_max
    double* beta = alpha + smax_steps;                    // s_max
    double* sig = beta + smax_steps;                      // s_max + 1
    double* Wg = sig + ls;                                // (s_max + 1)^2 (global fallback)
    double* Vg = Wg + (int64_t)ls * ls;                   // (s_max + 1)^2
    int* order = (int*)(Vg + (int64_t)ls * ls);           // s_max + 1
    uint32_t* roa = (uint32_t*)(order + ls);              // ma
    uint32_t* coa = roa + ma;                             // D
    uint32_t* rob = coa + D;                              // D
    uint32_t* cob = rob + D;                              // mb
    double* W = Wg;                                       // small bidiagonal -> its SVD (LDS when it fits)
    double* Vs = Vg;
    int lw = ls;                                          // their leading dimension

    for (int i = tid; i < ma; i += kCoreThreads) roa[i] = axis_offset(d.va.row, (uint32_t)i);
    for (int i = tid; i < D; i += kCoreThreads) {
        coa[i] = axis_offset(d.va.col, (uint32_t)i);
        rob[i] = axis_offset(d.vb.row, (uint32_t)i);
    }
    for (int i = tid; i < mb; i += kCoreThreads) cob[i] = axis_offset(d.vb.col, (uint32_t)i);
    // start vector
    for (int i = tid; i < mb; i += kCoreThreads) V[i] = probe_entry(i, 0);
    __syncthreads();
    {
        double nrm = 0.0;
        for (int i = tid; i < mb; i += kCoreThreads) nrm += V[i] * V[i];
        nrm = sqrt(block_sum(nrm, sh));
        for (int i = tid; i < mb; i += kCoreThreads) V[i] /= nrm;
        __syncthreads();
    }

    // ||A B||_F^2 = <G_A, G_B> (both Grams carry the scales' 1/s^2), for the completeness test
    double fro2 = 0.0;
    {
        double part = 0.0;
        for (int64_t idx = tid; idx < (int64_t)D * D; idx += kCoreThreads) part += d.gram_a[idx] * d.gram_b[idx];
        fro2 = block_sum(part, sh);
    }
    int s = 0, restarts = 0, extra_col = 0;
    bool exhausted = false, converged = false;
    double amax = 0.0;
    int target = d.s_min;
    int nsv = 0;
    for (;;) {
        for (; s < target && !exhausted; ++s) {
            const int j = s;
            const double* vj = V + (int64_t)j * mb;
            double* uj = U + (int64_t)j * ma;
            // t1 = B v_j ; u_j = A t1 - beta_{j-1} u_{j-1}
            mv_rows(B, rob, cob, D, mb, b_col_unit, vj, t1, ib);
            __syncthreads();
            mv_rows(A, roa, coa, ma, D, a_col_unit, t1, uj, ia);
            __syncthreads();
            if (j > 0) {
                const double bprev = beta[j - 1];
                const double* uprev = U + (int64_t)(j - 1) * ma;
                for (int i = tid; i < ma; i += kCoreThreads) uj[i] -= bprev * uprev[i];
                __syncthreads();
            }
            reorthogonalise(uj, U, ma, j, coef);
            double an = 0.0;
            for (int i = tid; i < ma; i += kCoreThreads) an += uj[i] * uj[i];
            an = sqrt(block_sum(an, sh));
            amax = fmax(amax, an);
            if (!(an > kLanczosBreak * amax)) {
                // M v_j lies in span(U): the range is exhausted.  v_j stays in the
                // factorisation M V_{j+1} = U_j B with B of size j x (j+1).
                exhausted = true;
                extra_col = 1;
                break;
            }
            alpha[j] = an;
            for (int i = tid; i < ma; i += kCoreThreads) uj[i] /= an;
            __syncthreads();
            // t2 = A^T u_j ; v_{j+1} = B^T t2 - alpha_j v_j
            mv_cols(A, roa, coa, ma, D, a_row_unit, uj, t2, ia);
            __syncthreads();
            double* w = V + (int64_t)(j + 1) * mb;
            mv_cols(B, rob, cob, D, mb, b_row_unit, t2, w, ib);
            __syncthreads();
            for (int f = tid; f < mb; f += kCoreThreads) w[f] -= an * vj[f];
            __syncthreads();
            reorthogonalise(w, V, mb, j + 1, coef);
            double bn = 0.0;
            for (int i = tid; i < mb; i += kCoreThreads) bn += w[i] * w[i];
            bn = sqrt(block_sum(bn, sh));
            amax = fmax(amax, bn);
            if (bn > kLanczosBreak * amax) {
                beta[j] = bn;
                for (int i = tid; i < mb; i += kCoreThreads) w[i] /= bn;
                __syncthreads();
            } else {
                // invariant Krylov space: restart with a fresh direction orthogonal to V
                beta[j] = 0.0;
                ++restarts;
                for (int i = tid; i < mb; i += kCoreThreads) w[i] = probe_entry(i, restarts);
                __syncthreads();
                reorthogonalise(w, V, mb, j + 1, coef);
                double rn = 0.0;
                for (int i = tid; i < mb; i += kCoreThreads) rn += w[i] * w[i];
                rn = sqrt(block_sum(rn, sh));
                if (!(rn > 1e-8)) {
                    exhausted = true;
                    s = j + 1;
                    break;
                }
                for (int i = tid; i < mb; i += kCoreThreads) w[i] /= rn;
                __syncthreads();
            }
        }
        // SVD of the s x nc upper bidiagonal (diag alpha, superdiag beta); nc = s + 1 after a
        // breakdown of alpha, whose last column holds beta_{s-1} only
        const int ncol = s + extra_col;
        if ((size_t)2 * ncol * ncol * sizeof(double) <= (size_t)kLanczosLdsBytes) {
            W = lds;
            Vs = lds + (int64_t)ncol * ncol;
            lw = ncol;
        } else {
            W = Wg;
            Vs = Vg;
            lw = ls;
        }
        for (int64_t idx = tid; idx < (int64_t)ncol * ncol; idx += kCoreThreads) {
            const int c = (int)(idx / ncol), r = (int)(idx - (int64_t)c * ncol);
            if (r < s) W[(int64_t)c * lw + r] = (r == c) ? alpha[c] : ((r + 1 == c) ? beta[r] : 0.0);
            Vs[(int64_t)c * lw + r] = (r == c) ? 1.0 : 0.0;
        }
        __syncthreads();
        int sw = 0;
        const bool jc = jacobi_svd(W, Vs, s, ncol, lw, max_sweeps, sh, &sw);
        sorted_norms(W, s, ncol, lw, sig, order);
        nsv = ncol;
        // residual of Ritz triplet t: beta_{s-1} |Ub[s-1, t]| (zero when the space is exhausted)
        const double smax_v = s > 0 ? sig[order[0]] : 0.0;
        const double bl = (exhausted || s == 0) ? 0.0 : beta[s - 1];
        bool ok = jc;
        for (int t = 0; t < min(cn, ncol); ++t) {
            const int c = order[t];
            const double sv = sig[c];
            if (!(sv > kNoiseRel * smax_v)) continue;
            const double res = bl * fabs(W[(int64_t)c * lw + (s - 1)]) / sv;
            if (res > 1e-13 * smax_v) ok = false;
        }
        if (ok && !exhausted && s < smax_steps) {
            // Completeness (see gram_lanczos_kernel): with M V_s = U_s B_s and
            // U_s^T M = B_s V_s^T + beta_s e_s v_{s+1}^T, M on the complement of the kept triplets
            // is [[diag(sigma_Y), c], [0, O]] with c of rank one, |c| = beta_s |last entries of
            // the other left vectors of B_s|, and |O|_F^2 = ||A B||_F^2 - |B_s|_F^2 - beta_s^2;
            // its largest singular value is at most that of [[a, |c|], [0, |O|_F]].  Below the
            // smallest kept value, nothing can join the kept set; else the iteration goes on.
            int keff = 0;
            double scut = 0.0, kept_last2 = 0.0;
            for (int t = 0; t < min(cn, ncol); ++t) {
                const int c = order[t];
                const double sv = sig[c];
                if (!(sv > kNoiseRel * smax_v)) break;
                scut = sv;
                const double u = W[(int64_t)c * lw + (s - 1)] / sv;   // left vector's last entry
                kept_last2 += u * u;
                ++keff;
            }
            double b2 = 0.0;
            for (int j = 0; j < s; ++j) b2 += alpha[j] * alpha[j] + (j + 1 < s ? beta[j] * beta[j] : 0.0);
            const double a = keff < ncol ? fmax(sig[order[keff]], 0.0) : 0.0;
            const double o2 = fmax(fro2 - b2 - bl * bl, 0.0);
            const double c2 = bl * bl * fmax(1.0 - kept_last2, 0.0);
            const double h = 0.5 * (a * a + c2 + o2);
            const double bound = sqrt(h + sqrt(fmax(h * h - a * a * o2, 0.0)));
            if (keff > 0 && !(bound < scut || scut * scut <= 1e-13 * fro2)) ok = false;
        }
        if (ok || exhausted || s >= smax_steps) {
            converged = ok || exhausted;
            break;
        }
        target = min(smax_steps, s + 8);
        __syncthreads();
    }

    // Ritz vectors of M: Ut = U Ub, Vt = V Vb for the kept columns
    const double smax_v = nsv > 0 ? sig[order[0]] : 0.0;
    const int nrow = nsv - extra_col;
    for (int64_t idx = tid; idx < (int64_t)(ma + mb) * cn; idx += kCoreThreads) {
        const int t = (int)(idx / (ma + mb)), i = (int)(idx - (int64_t)t * (ma + mb));
        double acc = 0.0;
        if (t < nsv) {
            const int c = order[t];
            const double sv = sig[c];
            if (sv > 0.0) {
                if (i < ma) {
                    for (int j = 0; j < nrow; ++j) acc += U[(int64_t)j * ma + i] * W[(int64_t)c * lw + j];
                    acc /= sv;
                } else {
                    const int f = i - ma;
                    for (int j = 0; j < nsv; ++j) acc += V[(int64_t)j * mb + f] * Vs[(int64_t)c * lw + j];
                }
            }
        }
        if (i < ma) Ut[(int64_t)t * ma + i] = acc;
        else Vt[(int64_t)t * mb + (i - ma)] = acc;
    }
    __syncthreads();
    // projectors P_L = (B/s_b) Vt S^-1/2 (D x cn), P_R = S^-1/2 Ut^T (A/s_a) (cn x D), one column
    // (row) at a time through the same matvecs; t1 / t2 hold the float64 results
    Tp* PL = (Tp*)d.p_left;
    Tp* PR = (Tp*)d.p_right;
    for (int t = 0; t < cn; ++t) {
        const double sv = t < nsv ? sig[order[t]] : 0.0;
        const bool keep = sv > kNoiseRel * smax_v && sv >= d.cutoff * smax_v;
        if (keep) {
            mv_rows(B, rob, cob, D, mb, b_col_unit, Vt + (int64_t)t * mb, t1, ib / sqrt(sv));
            mv_cols(A, roa, coa, ma, D, a_row_unit, Ut + (int64_t)t * ma, t2, ia / sqrt(sv));
            __syncthreads();
        }
        for (int dd = tid; dd < D; dd += kCoreThreads) {
            PL[(int64_t)dd * cn + t] = (Tp)(keep ? t1[dd] : 0.0);
            PR[(int64_t)t * D + dd] = (Tp)(keep ? t2[dd] : 0.0);
        }
        __syncthreads();
    }
    if (tid == 0) {
        // diagnostics within the Krylov space (the full spectrum of M is never formed)
        double tot = 0.0, disc = 0.0;
        for (int t = 0; t < nsv; ++t) {
            const double sv = sig[order[t]];
            tot += sv * sv;
            if (t >= cn) disc += sv * sv;
        }
        stat_disc[d.stat] = tot > 0.0 ? disc / tot : 0.0;
        const double s_last = (cn - 1 < nsv) ? sig[order[cn - 1]] : 0.0;
        const double s_next = (cn < nsv) ? sig[order[cn]] : 0.0;
        stat_tie[d.stat] = (d.kmin > cn && nsv > cn && s_last > 1e-13 * smax_v && s_last - s_next <= 1e-12 * smax_v) ? 1 : 0;
        stat_sweeps[d.stat] = converged ? nsv : -1 - nsv;
    }
}


// ------------------------------------------------------------------------------------------
// Large cores with at least one explicit side: symmetric Lanczos on S = F_X G_Y F_X^T, where
// F_X (n x D) is the explicit factor of side X (n <= D rows) and G_Y the D x D Gram matrix of
// side Y (or F_Y^T F_Y when Y is explicit too).  S = M^T M (X = B) or M M^T (X = A), so its
// eigenpairs are (sigma^2, right / left singular vectors of M).  Projectors:
//   side-X projector column t: F_X^T w_t / sqrt(sigma_t)
//   side-Y projector column t: G_Y F_X^T w_t / sigma_t^(3/2)
// (P_L = the B-side one as D x chi', P_R = the A-side one transposed).
// ------------------------------------------------------------------------------------------
// y[i] = scale * sum_d F[i*D + d] x[d]   (dense row-major F, n rows): a wave per group of
// four rows, lanes along the contiguous columns, four independent loads in flight per lane.
__device__ void dense_mv(const double* __restrict__ F, int n, int D, const double* __restrict__ x,
                         double* __restrict__ y, double scale) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i0 = wave * 4; i0 < n; i0 += kCoreWaves * 4) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        const int nr = min(4, n - i0);
        const double* f = F + (int64_t)i0 * D;
        for (int d = lane; d < D; d += 64) {
            const double xv = x[d];
            a0 += f[d] * xv;
            if (nr > 1) a1 += f[D + d] * xv;
            if (nr > 2) a2 += f[2 * D + d] * xv;
            if (nr > 3) a3 += f[3 * D + d] * xv;
        }
        a0 = wave_sum(a0);
        a1 = wave_sum(a1);
        a2 = wave_sum(a2);
        a3 = wave_sum(a3);
        if (lane == 0) {
            y[i0] = a0 * scale;
            if (nr > 1) y[i0 + 1] = a1 * scale;
            if (nr > 2) y[i0 + 2] = a2 * scale;
            if (nr > 3) y[i0 + 3] = a3 * scale;
        }
    }
}
// y[d] = scale * sum_i F[i*D + d] x[i]: waves split the rows, lanes run along the columns
// (four per lane per block of 256), then the per-wave partials are summed in fixed order.
// part: kCoreWaves * D doubles of scratch.  Ends with a barrier.
__device__ void dense_mvt(const double* __restrict__ F, int n, int D, const double* __restrict__ x,
                          double* __restrict__ y, double scale, double* __restrict__ part) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int d0 = 0; d0 < D; d0 += 256) {
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        for (int i = wave; i < n; i += kCoreWaves) {
            const double xv = x[i];
            const double* f = F + (int64_t)i * D + d0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int dd = lane + 64 * q;
                if (d0 + dd < D) a[q] += f[dd] * xv;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int dd = d0 + lane + 64 * q;
            if (dd < D) part[(int64_t)wave * D + dd] = a[q];
        }
    }
    __syncthreads();
    for (int dd = tid; dd < D; dd += kCoreThreads) {
        double acc = 0.0;
        for (int w = 0; w < kCoreWaves; ++w) acc += part[(int64_t)w * D + dd];
        y[dd] = acc * scale;
    }
    __syncthreads();
}


template <typename Tp>
__global__ __launch_bounds__(kCoreThreads) void gram_lanczos_kernel(const GLanczosDesc* __restrict__ descs,
                                                                    int max_sweeps, double* __restrict__ stat_disc,
                                                                    int32_t* __restrict__ stat_tie,
                                                                    int32_t* __restrict__ stat_sweeps) {
    extern __shared__ double lds[];
    __shared__ CoreShared sh;
    __shared__ double coef[kLanczosMaxSteps + 1];
    const GLanczosDesc& d = descs[blockIdx.x];
    const int tid = threadIdx.x;
    const int n = d.n, D = d.D, cn = d.chi_new, sm = d.s_max, ls = d.s_max + 1;

    double* S = d.work;                          // n x n operator F_X G_Y F_X^T
    double* T1 = S + (int64_t)n * n;             // D x n (G_Y F_X^T) or n x my (F_X F_Y^T)
    double* Q = T1 + (int64_t)min(D, d.my) * n;  // n x s_max Lanczos basis (T1 holds min(D, m_y) x n)
    double* Wt = Q + (int64_t)n * sm;            // n x cn Ritz vectors
    double* t1 = Wt + (int64_t)n * cn;           // D
    double* t2 = t1 + D;                         // D
    double* py = t2 + D;                         // max(n, m_y) scratch
    double* alpha = py + max(n, d.my);           // s_max
    double* beta = alpha + sm;                   // s_max
    double* sig = beta + sm;                     // ls
    double* Wg = sig + ls;                       // ls^2
    double* Vg = Wg + (int64_t)ls * ls;          // ls^2
    double* part = Vg + (int64_t)ls * ls;        // kCoreWaves x D partial sums
    double* P1 = part + (int64_t)kCoreWaves * D; // D x cn: F_X^T W
    double* P2 = P1 + (int64_t)D * cn;           // D x cn: G_Y F_X^T W
    double* PY = P2 + (int64_t)D * cn;           // m_y x cn (explicit Y)
    int* order = (int*)(PY + (int64_t)max(n, d.my) * cn);   // ls
    const double* FX = d.fx;
    // S and T1 were formed before this launch by grouped float64 GEMMs, so that a Lanczos step is
    // one matvec: Y a Gram: T1 = G_Y F_X^T (D x n), S = F_X T1; Y explicit: T1 = C1 = F_X F_Y^T
    // (n x my), S = C1 C1^T
    // y = S x for n <= 256.  S is symmetric up to the rounding of the GEMMs that formed it, so only
    // its upper 32 x 32 tiles are read (288 of 512 KB at n = 256, and the S of the cores sharing
    // an XCD then fit its L2): tile (I, J), I <= J, gives block J its column sums
    // sum_d S[d, i] x_d and, for I < J, block I its row sums sum_i S[d, i] x_i.  Wave w takes
    // tiles w, w + 16, ...; in a tile, lane (h, c) holds rows 16 h .. 16 h + 15 of column c.  The
    // row sums are reduced over the 32 columns of a half wave by halving exchanges inside each
    // 16-lane row (halve_rows over lane bits 3, 2, 1, 0) and one cross-row add, after which lane
    // c < 16 holds row c of its half.  Each tile's 32 column and 32 row sums go to their own LDS slots after
    // y (the room there is free while the steps run), and y_i adds its block's slots in a fixed
    // order
    static_assert(kCoreThreads == 1024, "16 waves over at most 36 upper tiles");
    auto apply_small = [&](const double* x, double* y) {
        const int nb = (n + 31) >> 5, ntile = nb * (nb + 1) / 2;
        double* slot = y + n;                          // ntile x 64: column sums, then row sums
        const int c = tid & 31, hf = (tid >> 5) & 1;
        for (int t = tid >> 6; t < ntile; t += kCoreWaves) {
            int I = 0, rem = t;
            while (rem >= nb - I) {
                rem -= nb - I;
                ++I;
            }
            const int J = I + rem;
            const int col = 32 * J + c, row0 = 32 * I + 16 * hf;
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u)
                v[u] = (col < n && row0 + u < n) ? S[(int64_t)(row0 + u) * n + col] : 0.0;
            double cs = 0.0;
#pragma unroll
            for (int u = 0; u < 16; ++u)
                if (row0 + u < n) cs = fma(v[u], x[row0 + u], cs);
            cs += __shfl_xor(cs, 32, 64);
            if (hf == 0) slot[t * 64 + c] = cs;
            if (I < J) {
                const double xc = col < n ? x[col] : 0.0;
#pragma unroll
                for (int u = 0; u < 16; ++u) v[u] *= xc;
                halve_rows<8, 0x128, 0x128>(v, (c & 8) != 0);
                halve_rows<4, 0x124, 0x12C>(v, (c & 4) != 0);
                halve_rows<2, 0x4E, 0x4E>(v, (c & 2) != 0);
                halve_rows<1, 0xB1, 0xB1>(v, (c & 1) != 0);
                const double r = v[0] + __shfl_xor(v[0], 16, 64);
                if (c < 16) slot[t * 64 + 32 + 16 * hf + c] = r;
            }
        }
        __syncthreads();
        if (tid < n) {
            const int J = tid >> 5, cc = tid & 31;
            double acc = 0.0;
            for (int I = 0; I <= J; ++I) acc += slot[(I * nb - I * (I - 1) / 2 + (J - I)) * 64 + cc];
            for (int K = J + 1; K < nb; ++K) acc += slot[(J * nb - J * (J - 1) / 2 + (K - J)) * 64 + 32 + cc];
            y[tid] = acc;
        }
        __syncthreads();
    };

    // Lanczos basis: its first jl columns live in LDS, after the room kept for the tridiagonal
    // solve (s <= kTriLdsS), the rest in the workspace
    constexpr int kTriLdsS = 48;
    static_assert(256 + 36 * 64 <= 2 * kTriLdsS * kTriLdsS, "the matvec slots fit in the room before the basis");
    double* lq = lds + 2 * kTriLdsS * kTriLdsS;
    const int jl = min(sm, (int)(((int64_t)kLanczosLdsBytes / 8 - 2 * kTriLdsS * kTriLdsS) / max(n, 1)));
    auto qcol = [&](int j) -> double* { return j < jl ? lq + (int64_t)j * n : Q + (int64_t)j * n; };
    // x -= Q[:, :k] (Q[:, :k]^T x), twice (classical Gram-Schmidt with reorthogonalisation).
    // Returns the sum of the two passes' coefficients of column k - 1 and ||x||^2 after them.
    const int wave = tid >> 6, lane = tid & 63;
    auto cgs2 = [&](double* x, int k, double* last_coef, bool x_lds) -> double {
        double lc = 0.0, nrm2 = 0.0;
        // basis in LDS and x the LDS vector lds[0, n), n <= 256, k <= 64: every wave's
        // coefficients (up to four columns) reduced together, the update split over four column
        // classes of 256 threads, all through LDS-derived pointers
        const bool fast = x_lds && n <= 256 && k <= 4 * kCoreWaves && k <= jl;
        for (int pass = 0; pass < 2; ++pass) {
            if (fast) {
                double v[4] = {0.0, 0.0, 0.0, 0.0};
                for (int i = lane; i < n; i += 64) {
                    const double xi = lds[i];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int c = wave + kCoreWaves * u;
                        if (c < k) v[u] = fma(lq[(int64_t)c * n + i], xi, v[u]);
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] = wave_sum(v[u]);
                if (lane == 0)
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (wave + kCoreWaves * u < k) coef[wave + kCoreWaves * u] = v[u];
            } else {
                for (int c = wave; c < k; c += kCoreWaves) {
                    const double* q = qcol(c);
                    double v = 0.0;
                    for (int i = lane; i < n; i += 64) v += q[i] * x[i];
                    v = wave_sum(v);
                    if (lane == 0) coef[c] = v;
                }
            }
            __syncthreads();
            if (k > 0) lc += coef[k - 1];
            double part = 0.0;
            if (fast) {
                const int i = tid & 255, h = tid >> 8;
                double a0 = 0.0, a1 = 0.0;
                if (i < n) {
                    int c = h;
                    for (; c + 4 < k; c += 8) {
                        a0 = fma(lq[(int64_t)c * n + i], coef[c], a0);
                        a1 = fma(lq[(int64_t)(c + 4) * n + i], coef[c + 4], a1);
                    }
                    if (c < k) a0 = fma(lq[(int64_t)c * n + i], coef[c], a0);
                }
                // x occupies at most lds[0, n) or the basis room: the partial sums go after it
                double* spart = lds + n;
                spart[tid] = a0 + a1;
                __syncthreads();
                if (tid < n) {
                    const double acc = lds[tid] - ((spart[tid] + spart[256 + tid]) + (spart[512 + tid] + spart[768 + tid]));
                    lds[tid] = acc;
                    part = acc * acc;
                }
            } else {
                for (int i = tid; i < n; i += kCoreThreads) {
                    // four interleaved partial sums keep the dependent chain a quarter as long
                    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
                    int c = 0;
                    for (; c + 4 <= k; c += 4) {
                        s0 = fma(qcol(c)[i], coef[c], s0);
                        s1 = fma(qcol(c + 1)[i], coef[c + 1], s1);
                        s2 = fma(qcol(c + 2)[i], coef[c + 2], s2);
                        s3 = fma(qcol(c + 3)[i], coef[c + 3], s3);
                    }
                    for (; c < k; ++c) s0 = fma(qcol(c)[i], coef[c], s0);
                    const double acc = x[i] - ((s0 + s1) + (s2 + s3));
                    x[i] = acc;
                    part += acc * acc;
                }
            }
            if (pass == 1) nrm2 = block_sum(part, sh);
            else __syncthreads();
        }
        if (last_coef) *last_coef = lc;
        return nrm2;
    };

    {
        double* q0 = qcol(0);
        for (int i = tid; i < n; i += kCoreThreads) q0[i] = probe_entry(i, 0);
        __syncthreads();
        double nrm = 0.0;
        for (int i = tid; i < n; i += kCoreThreads) nrm += q0[i] * q0[i];
        nrm = sqrt(block_sum(nrm, sh));
        for (int i = tid; i < n; i += kCoreThreads) q0[i] /= nrm;
        __syncthreads();
    }
    // ||S||_F^2 = the sum of the squared eigenvalues of S (the completeness test below)
    double fro2 = 0.0;
    {
        // sixteen loads in flight per thread
        double p4[4] = {0.0, 0.0, 0.0, 0.0};
        const int64_t nn = (int64_t)n * n;
        int64_t idx = tid;
        for (; idx + 15 * kCoreThreads < nn; idx += 16 * kCoreThreads) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = S[idx + (int64_t)u * kCoreThreads];
#pragma unroll
            for (int u = 0; u < 16; ++u) p4[u & 3] = fma(v[u], v[u], p4[u & 3]);
        }
        for (; idx < nn; idx += kCoreThreads) p4[0] = fma(S[idx], S[idx], p4[0]);
        fro2 = block_sum((p4[0] + p4[1]) + (p4[2] + p4[3]), sh);
    }
    int s = 0, restarts = 0, nev = 0;
    int s_prev = 0;   // size of the last tridiagonal solve (its eigenvectors are in Vs)
    bool exhausted = false, converged = false;
    double bmax = 0.0;
    int target = d.s_min;
    double* W = Wg;
    double* Vs = Vg;
    int lw = ls;
    // the next Lanczos vector candidate (length n): in LDS (the tridiagonal solve's room, free
    // between checks) when it fits
    double* qnext = n <= 2 * kTriLdsS * kTriLdsS ? lds : py;
    for (;;) {
        for (; s < target && !exhausted; ++s) {
            const int j = s;
            // the vector and the result in LDS (n <= 256) are read and written through
            // LDS-derived pointers, so the loops use LDS instructions rather than flat ones
            if (n > 256) {
                dense_mv(S, n, n, qcol(j), qnext, 1.0);
                __syncthreads();
            } else if (j < jl) {
                apply_small(lq + (int64_t)j * n, lds);
            } else {
                apply_small(Q + (int64_t)j * n, lds);
            }
            // full orthogonalisation against q_0..q_j: q_j's coefficient is alpha_j, the remaining
            // norm beta_j (the three-term recurrence in exact arithmetic)
            double a = 0.0;
            const double b = sqrt(cgs2(qnext, j + 1, &a, qnext == lds));
            alpha[j] = a;
            bmax = fmax(bmax, fmax(b, fabs(a)));
            if (j + 1 >= n) {   // the basis spans the whole space
                beta[j] = 0.0;
                exhausted = true;
                s = j + 1;
                break;
            }
            double* qn = qcol(j + 1);
            if (b > kLanczosBreak * bmax) {
                beta[j] = b;
                for (int i = tid; i < n; i += kCoreThreads) qn[i] = qnext[i] / b;
                __syncthreads();
            } else {
                beta[j] = 0.0;   // invariant subspace: restart orthogonally to the basis
                ++restarts;
                for (int i = tid; i < n; i += kCoreThreads) qn[i] = probe_entry(i, restarts);
                __syncthreads();
                const double rn = sqrt(cgs2(qn, j + 1, nullptr, false));
                if (!(rn > 1e-8)) {
                    exhausted = true;
                    s = j + 1;
                    break;
                }
                for (int i = tid; i < n; i += kCoreThreads) qn[i] /= rn;
                __syncthreads();
            }
        }
        // eigenpairs of the s x s tridiagonal T (symmetric positive semidefinite): the one-sided
        // Jacobi SVD of L^T V (T = L L^T) gives eigenvalues as squared column norms and
        // eigenvectors in Vs.
        // Warm start: T's leading s_prev x s_prev block is the previous check's T, whose
        // eigenvectors the previous solve left in Vs; V starts as those, extended by the
        // identity, and W = L^T V.  The rotations then only resolve the coupling to the new
        // steps, in a few sweeps instead of a full solve.
        // (a solve in LDS copied its V to Wg, since the next Lanczos vectors reuse that room; one
        // in the workspace left it in Vg, at the same stride as the next)
        const double* vp = s_prev <= kTriLdsS ? Wg : Vg;
        const int lwp = s_prev <= kTriLdsS ? s_prev : ls;
        // one body for both homes of W and V, inlined at each call so that the LDS one compiles
        // to LDS instructions
        auto tri_solve = [&](auto Wp, auto Vp, int lwv) __attribute__((always_inline)) -> bool {
            for (int64_t idx = tid; idx < (int64_t)s * s; idx += kCoreThreads) {
                const int c = (int)(idx / s), r = (int)(idx - (int64_t)c * s);
                Vp[(int64_t)c * lwv + r] = (c < s_prev && r < s_prev) ? vp[(int64_t)c * lwp + r] : (r == c ? 1.0 : 0.0);
            }
            // T = L L^T with L lower bidiagonal (diagonal ld_[i], subdiagonal le_[i] = L[i+1][i]),
            // by one thread; W = L^T V then has W^T W = V^T T V, so the one-sided Jacobi below
            // converges like a two-sided one on T (rather than on T^2, as on W = T V would) and
            // the eigenvalues of T are the squared column norms.  T is positive semidefinite: a
            // pivot at the rounding level of ||T|| is taken as zero, with its column of L.
            double* ld_ = t1;   // s <= n <= D: the explicit side has at most D rows
            double* le_ = t2;
            if (tid == 0) {
                double amax = 0.0;
                for (int i = 0; i < s; ++i) amax = fmax(amax, fabs(alpha[i]));
                const double floor_ = 1e-15 * amax;
                double prev = 0.0;   // L[i][i-1]
                for (int i = 0; i < s; ++i) {
                    const double piv = alpha[i] - prev * prev;
                    const double l = piv > floor_ ? sqrt(piv) : 0.0;
                    ld_[i] = l;
                    prev = (i + 1 < s && l > 0.0) ? beta[i] / l : 0.0;
                    if (i + 1 < s) le_[i] = prev;
                }
            }
            __syncthreads();
            for (int64_t idx = tid; idx < (int64_t)s * s; idx += kCoreThreads) {
                const int c = (int)(idx / s), r = (int)(idx - (int64_t)c * s);
                const auto vc = Vp + (int64_t)c * lwv;
                double v = ld_[r] * vc[r];
                if (r + 1 < s) v = fma(le_[r], vc[r + 1], v);
                Wp[(int64_t)c * lwv + r] = v;
            }
            __syncthreads();
            int sw = 0;
            const bool ok = s == 32 ? jacobi32<kCoreThreads>(Wp, Vp, lwv, max_sweeps, sh, &sw)
                            : s < 32 ? jacobi_svd_small<kCoreThreads, 2>(Wp, Vp, s, s, lwv, max_sweeps, sh, &sw)
                            : s <= 64 ? jacobi_svd_small(Wp, Vp, s, s, lwv, max_sweeps, sh, &sw)
                                      : jacobi_svd((double*)Wp, (double*)Vp, s, s, lwv, max_sweeps, sh, &sw);
            sorted_norms(Wp, s, s, lwv, sig, order);
            for (int j = tid; j < s; j += kCoreThreads) sig[j] = sig[j] * sig[j];
            __syncthreads();
            return ok;
        };
        bool jc;
        if (s <= kTriLdsS) {
            W = lds;
            Vs = lds + (int64_t)s * s;
            lw = s;
            jc = tri_solve((LdsPtr)lds, (LdsPtr)lds + (int64_t)s * s, s);
            // keep V for the next check's warm start (read after the barrier below)
            for (int64_t idx = tid; idx < (int64_t)s * s; idx += kCoreThreads) Wg[idx] = lds[(int64_t)s * s + idx];
        } else {
            W = Wg;   // written only after V has been read from Wg (barrier between)
            Vs = Vg;
            lw = ls;
            jc = tri_solve(Wg, Vg, ls);
        }
        s_prev = s;
        nev = s;
        const double lmax = s > 0 ? sig[order[0]] : 0.0;
        const double bl = (exhausted || s == 0) ? 0.0 : beta[s - 1];
        bool ok = jc;
        for (int t = 0; t < min(cn, s); ++t) {
            const int c = order[t];
            const double lv = sig[c];
            if (!(lv > kNoiseRelSq * lmax)) continue;
            // residual of the Ritz pair: beta_s |last entry of its eigenvector|
            if (bl * fabs(Vs[(int64_t)c * lw + (s - 1)]) > 1e-13 * lmax) ok = false;
        }
        if (ok && !exhausted && s < sm) {
            // Completeness.  A Krylov space from one start vector holds one direction of each
            // eigenspace, so converged Ritz pairs can miss further copies of a repeated kept
            // eigenvalue.  The eigenvalues of S other than the kept Ritz values are those of S on
            // the complement of the kept Ritz vectors W (an invariant subspace up to their
            // residuals).  In the basis (the other Ritz vectors Y, then the complement of Q) that
            // operator is [[diag(theta_Y), b], [b^T, O]] with b of rank one, |b| = beta_s |last
            // entries of Y| (S Q = Q T + beta_s q_s e^T), and O positive semidefinite with
            // |O|_F^2 = |S|_F^2 - |T|_F^2 - 2 beta_s^2.  Its largest eigenvalue is therefore at most
            // that of [[a, |b|], [|b|, |O|_F]] (a = the largest other Ritz value).  When that bound
            // is below the smallest kept value, nothing can join the kept set; else the iteration
            // goes on (to exhaustion at worst, where T holds every eigenvalue).  Kept values at the
            // rounding floor of |O|_F^2 (lambda^2 <= 1e-13 |S|_F^2) pass unchecked.
            int keff = 0;
            double lcut = 0.0, kept_last2 = 0.0;
            for (int t = 0; t < min(cn, s); ++t) {
                const int c = order[t];
                if (!(sig[c] > kNoiseRelSq * lmax)) break;
                lcut = sig[c];
                const double v = Vs[(int64_t)c * lw + (s - 1)];
                kept_last2 += v * v;
                ++keff;
            }
            double t2 = 0.0;
            for (int j = 0; j < s; ++j) t2 += alpha[j] * alpha[j] + (j + 1 < s ? 2.0 * beta[j] * beta[j] : 0.0);
            const double a = keff < s ? fmax(sig[order[keff]], 0.0) : 0.0;
            const double od = sqrt(fmax(fro2 - t2 - 2.0 * bl * bl, 0.0));
            const double bb = bl * sqrt(fmax(1.0 - kept_last2, 0.0));
            const double bound = 0.5 * (a + od) + sqrt(0.25 * (a - od) * (a - od) + bb * bb);
            if (keff > 0 && !(bound < lcut || lcut * lcut <= 1e-13 * fro2)) ok = false;
        }
        if (ok || exhausted || s >= sm) {
            converged = ok || exhausted;
            break;
        }
        target = min(sm, s + 4);
        __syncthreads();
    }
    // Ritz vectors w_t = Q Vs[:, order[t]]; when the basis and Vs are both in LDS (Vs right after
    // the last solve's W, stride nev) through LDS-typed pointers, two partial sums per output
    if (nev <= jl && nev <= kTriLdsS) {
        const LdsPtr qb = (LdsPtr)lq;
        const LdsPtr vb = (LdsPtr)lds + (int64_t)nev * nev;
        for (int64_t idx = tid; idx < (int64_t)n * cn; idx += kCoreThreads) {
            const int t = (int)(idx / n), i = (int)(idx - (int64_t)t * n);
            double a0 = 0.0, a1 = 0.0;
            if (t < nev) {
                const LdsPtr vc = vb + (int64_t)order[t] * nev;
                int j = 0;
                for (; j + 1 < nev; j += 2) {
                    a0 = fma(qb[(int64_t)j * n + i], vc[j], a0);
                    a1 = fma(qb[(int64_t)(j + 1) * n + i], vc[j + 1], a1);
                }
                if (j < nev) a0 = fma(qb[(int64_t)j * n + i], vc[j], a0);
            }
            Wt[(int64_t)t * n + i] = a0 + a1;
        }
    } else {
        for (int64_t idx = tid; idx < (int64_t)n * cn; idx += kCoreThreads) {
            const int t = (int)(idx / n), i = (int)(idx - (int64_t)t * n);
            double acc = 0.0;
            if (t < nev) {
                const int c = order[t];
                for (int j = 0; j < nev; ++j) acc += qcol(j)[i] * Vs[(int64_t)c * lw + j];
            }
            Wt[(int64_t)t * n + i] = acc;
        }
    }
    __syncthreads();
    const double lmax = nev > 0 ? sig[order[0]] : 0.0;
    Tp* PL = (Tp*)d.p_left;
    Tp* PR = (Tp*)d.p_right;
    // all kept columns at once: P1 = F_X^T W; Y a Gram: P2 = T1 W = G_Y F_X^T W; Y explicit: PY = C1^T W = F_Y F_X^T W, then
    // P2 = F_Y^T PY.  W is staged in LDS (free after the Ritz vectors) when it fits: every wave of
    // the products reads all of it
    if ((int64_t)n * cn <= (int64_t)kLanczosLdsBytes / 8) {
        for (int64_t idx = tid; idx < (int64_t)n * cn; idx += kCoreThreads) lds[idx] = Wt[idx];
        __syncthreads();
        const LdsPtr wl = (LdsPtr)lds;
        wg_gemm_f64_narrow<kCoreWaves, LdsPtr>(FX, 1, D, wl, 1, n, P1, cn, D, cn, n);
        if (d.gram_y) wg_gemm_f64_narrow<kCoreWaves, LdsPtr>(T1, n, 1, wl, 1, n, P2, cn, D, cn, n);
        else wg_gemm_f64_narrow<kCoreWaves, LdsPtr>(T1, 1, d.my, wl, 1, n, PY, cn, d.my, cn, n);
    } else {
        wg_gemm_f64_narrow(FX, 1, D, Wt, 1, n, P1, cn, D, cn, n);
        if (d.gram_y) wg_gemm_f64_narrow(T1, n, 1, Wt, 1, n, P2, cn, D, cn, n);
        else wg_gemm_f64_narrow(T1, 1, d.my, Wt, 1, n, PY, cn, d.my, cn, n);
    }
    if (!d.gram_y) wg_gemm_f64_narrow(d.fy, 1, D, PY, cn, 1, P2, cn, D, cn, d.my);
    for (int idx = tid; idx < D * cn; idx += kCoreThreads) {
        const int dd = idx / cn, t = idx - dd * cn;
        const double lv = t < nev ? sig[order[t]] : 0.0;   // eigenvalue = sigma^2
        const double sv = sqrt(fmax(lv, 0.0));
        const bool keep = lv > kNoiseRelSq * lmax && sv >= d.cutoff * sqrt(lmax);
        const double fx = keep ? 1.0 / sqrt(sv) : 0.0, fy = keep ? 1.0 / (sv * sqrt(sv)) : 0.0;
        const double px = P1[idx] * fx, pyv = P2[idx] * fy;
        // X = B: P_L column = side-X vector, P_R row = side-Y vector; X = A: the reverse
        PL[(int64_t)dd * cn + t] = (Tp)(d.x_is_b ? px : pyv);
        PR[(int64_t)t * D + dd] = (Tp)(d.x_is_b ? pyv : px);
    }
    if (tid == 0) {
        double tot = 0.0, disc = 0.0;
        for (int t = 0; t < nev; ++t) {
            const double lv = fmax(sig[order[t]], 0.0);
            tot += lv;
            if (t >= cn) disc += lv;
        }
        stat_disc[d.stat] = tot > 0.0 ? disc / tot : 0.0;
        const double l_last = (cn - 1 < nev) ? sig[order[cn - 1]] : 0.0;
        const double l_next = (cn < nev) ? sig[order[cn]] : 0.0;
        const double sl = sqrt(fmax(l_last, 0.0)), sn = sqrt(fmax(l_next, 0.0));
        stat_tie[d.stat] = (d.kmin > cn && nev > cn && sl > 1e-13 * sqrt(lmax) && sl - sn <= 1e-12 * sqrt(lmax)) ? 1 : 0;
        stat_sweeps[d.stat] = converged ? nev : -1 - nev;
    }
}

// ------------------------------------------------------------------------------------------
// Running exponent
// ------------------------------------------------------------------------------------------
__global__ void scale_finalize(const ScaleDesc* __restrict__ descs, int n, const double* __restrict__ maxparts,
                               double* __restrict__ scales) {
    const int gw = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (gw >= n) return;
    const ScaleDesc& d = descs[gw];
    double m = 0.0;
    for (int i = lane; i < d.nparts; i += 64) m = fmax(m, maxparts[d.maxpart + i]);
    m = wave_max(m);
    if (lane == 0) scales[d.tensor] = m;
}

template <typename T>
__global__ void input_scales(const InputDesc* __restrict__ descs, int n, double* __restrict__ scales) {
    const int gw = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (gw >= n) return;
    const InputDesc& d = descs[gw];
    const T* x = (const T*)d.dst;
    double m = 0.0;
    bool bad = false;
    for (int64_t i = lane; i < d.count; i += 64) {
        const double v = (double)x[i];
        if (!isfinite(v)) bad = true;
        m = fmax(m, fabs(v));
    }
    m = wave_max(m);
    const double b = wave_max(bad ? 1.0 : 0.0);
    if (lane == 0) scales[d.tensor] = b > 0.0 ? __builtin_nan("") : m;
}

template <typename T>
__global__ void input_scatter(const InputDesc* __restrict__ descs, int n, const double* __restrict__ src) {
    const int gw = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (gw >= n) return;
    const InputDesc& d = descs[gw];
    T* x = (T*)d.dst;
    for (int64_t i = lane; i < d.count; i += 64) x[i] = (T)src[d.src_off + i];
}

// ln|Z| = sum of ln s over every tensor in creation order (fixed-order reduction), sign of the
// final raw scalar; flags: 1 = a zero scale, 2 = non-finite scale, 4 = Jacobi not converged.
template <typename T>
__global__ __launch_bounds__(1024) void result_kernel(const double* __restrict__ scales, int n_scales,
                                                      const void* __restrict__ final_ptr,
                                                      const int32_t* __restrict__ sweeps, int n_comp,
                                                      double* __restrict__ result) {
    __shared__ double part[1024];
    __shared__ int fl[1024];
    const int tid = threadIdx.x;
    const int per = (n_scales + 1023) / 1024;
    const int b = tid * per, e = min(n_scales, b + per);
    double acc = 0.0;
    int flags = 0;
    for (int i = b; i < e; ++i) {
        const double s = scales[i];
        if (!isfinite(s)) flags |= 2;
        else if (s == 0.0) flags |= 1;
        else acc += log(s);
    }
    for (int c = tid; c < n_comp; c += 1024)
        if (sweeps[c] < 0) flags |= 4;
    part[tid] = acc;
    fl[tid] = flags;
    __syncthreads();
    for (int o = 512; o >= 1; o >>= 1) {
        if (tid < o) {
            part[tid] += part[tid + o];
            fl[tid] |= fl[tid + o];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double x = (double)((const T*)final_ptr)[0];
        result[0] = x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0);
        result[1] = part[0];
        result[2] = (double)fl[0];
    }
}

// ------------------------------------------------------------------------------------------
// Host-side launchers
// ------------------------------------------------------------------------------------------
// Runs f(T{}) with T the tensor storage type of precision 0 (float64), 1 (float32) or 2 (bfloat16).
template <typename F>
hipError_t by_prec(int prec, F&& f) {
    switch (prec) {
        case 0: f(double{}); break;
        case 1: f(float{}); break;
        case 2: f(bf16{}); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// A dispatch holds at most 2^32 - 1 work-items per dimension: grids beyond kMaxGridBlocks
// workgroups (of up to 256 work-items) are issued as several launches over consecutive ranges.
constexpr int64_t kMaxGridBlocks = (int64_t)1 << 23;

// One grouped GEMM launch in tile shape `variant`.
template <typename Tin, typename Tc, typename Tout, typename TinB = Tin>
hipError_t gemm_variant_launch(int variant, dim3 grid, hipStream_t s, const GemmDesc* descs, int ndesc,
                               const double* scales, double* maxparts, int64_t t0) {
    const dim3 block(kGemmThreads);
    switch (variant) {
        case GV_64x64:
            gemm_grouped<Tin, Tc, Tout, TinB, 64, 64><<<grid, block, 0, s>>>(descs, ndesc, scales, maxparts, t0);
            break;
        case GV_256x16:
            gemm_grouped<Tin, Tc, Tout, TinB, 256, 16><<<grid, block, 0, s>>>(descs, ndesc, scales, maxparts, t0);
            break;
        case GV_16x256:
            gemm_grouped<Tin, Tc, Tout, TinB, 16, 256><<<grid, block, 0, s>>>(descs, ndesc, scales, maxparts, t0);
            break;
        case GV_128x32:
            gemm_grouped<Tin, Tc, Tout, TinB, 128, 32><<<grid, block, 0, s>>>(descs, ndesc, scales, maxparts, t0);
            break;
        case GV_32x128:
            gemm_grouped<Tin, Tc, Tout, TinB, 32, 128><<<grid, block, 0, s>>>(descs, ndesc, scales, maxparts, t0);
            break;
        case GV_TALL16:
            gemm_skinny_grouped<Tin, typename SkinnyAcc<Tin>::type, 16, true>
                <<<grid, dim3(kSkinnyThreads), 0, s>>>(descs, ndesc, scales, maxparts, t0);
            break;
        case GV_TALL32:
            gemm_skinny_grouped<Tin, typename SkinnyAcc<Tin>::type, 32, true>
                <<<grid, dim3(kSkinnyThreads), 0, s>>>(descs, ndesc, scales, maxparts, t0);
            break;
        case GV_WIDE16:
            gemm_skinny_grouped<Tin, typename SkinnyAcc<Tin>::type, 16, false>
                <<<grid, dim3(kSkinnyThreads), 0, s>>>(descs, ndesc, scales, maxparts, t0);
            break;
        case GV_WIDE32:
            gemm_skinny_grouped<Tin, typename SkinnyAcc<Tin>::type, 32, false>
                <<<grid, dim3(kSkinnyThreads), 0, s>>>(descs, ndesc, scales, maxparts, t0);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gemm(int key, const GemmDesc* descs, int ndesc, int64_t tiles, const double* scales,
                       double* maxparts, hipStream_t s) {
    if (ndesc == 0 || tiles == 0) return hipSuccess;
    const int dtype_key = key % kGemmVariantStride, variant = key / kGemmVariantStride;
    if (variant != GV_64x64 && dtype_key != GEMM_F64 && dtype_key != GEMM_F32 && dtype_key != GEMM_BF16)
        return hipErrorInvalidValue;
    for (int64_t t0 = 0; t0 < tiles; t0 += kMaxGridBlocks) {
        const dim3 grid((unsigned)std::min<int64_t>(kMaxGridBlocks, tiles - t0)), block(kGemmThreads);
        hipError_t e = hipSuccess;
        switch (dtype_key) {
            case GEMM_F64:
                e = gemm_variant_launch<double, double, double>(variant, grid, s, descs, ndesc, scales, maxparts, t0);
                break;
            case GEMM_F32:
                e = gemm_variant_launch<float, float, float>(variant, grid, s, descs, ndesc, scales, maxparts, t0);
                break;
            case GEMM_BF16:
                e = gemm_variant_launch<bf16, bf16, bf16>(variant, grid, s, descs, ndesc, scales, maxparts, t0);
                break;
            case GEMM_F32_TO_F64:
                gemm_grouped<float, double, double><<<grid, block, 0, s>>>(descs, ndesc, scales, maxparts, t0);
                break;
            case GEMM_BF16_TO_F64:
                gemm_grouped<bf16, double, double><<<grid, block, 0, s>>>(descs, ndesc, scales, maxparts, t0);
                break;
            case GEMM_F32_X_F64:
                gemm_grouped<float, double, double, double><<<grid, block, 0, s>>>(descs, ndesc, scales, maxparts, t0);
                break;
            case GEMM_BF16_X_F64:
                gemm_grouped<bf16, double, double, double><<<grid, block, 0, s>>>(descs, ndesc, scales, maxparts, t0);
                break;
            case GEMM_GRAM_NARROW_F64:
                gram_narrow_grouped<double><<<grid, dim3(kGramThreads), 0, s>>>(descs, ndesc, scales, t0);
                break;
            case GEMM_GRAM_NARROW_F32:
                gram_narrow_grouped<float><<<grid, dim3(kGramThreads), 0, s>>>(descs, ndesc, scales, t0);
                break;
            case GEMM_GRAM_NARROW_BF16:
                gram_narrow_grouped<bf16><<<grid, dim3(kGramThreads), 0, s>>>(descs, ndesc, scales, t0);
                break;
            default: return hipErrorInvalidValue;
        }
        if (e == hipSuccess) e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_tsqr(int prec, const TsqrDesc* descs, int ndesc, int64_t blocks, const double* scales,
                       hipStream_t s) {
    if (ndesc == 0 || blocks == 0) return hipSuccess;
    const size_t lds = (size_t)kTsqrElems * sizeof(double);
    for (int64_t b0 = 0; b0 < blocks; b0 += kMaxGridBlocks) {
        const dim3 grid((unsigned)std::min<int64_t>(kMaxGridBlocks, blocks - b0)), block(kTsqrThreads);
        const hipError_t e = by_prec(prec, [&](auto t) {
            tsqr_blocks<decltype(t)><<<grid, block, lds, s>>>(descs, ndesc, scales, b0);
        });
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Elementwise grouped kernels take an element offset e0 for the same reason (256 work-items each).
constexpr int64_t kMaxGridElems = kMaxGridBlocks * 256;

hipError_t launch_copy(int prec, const CopyDesc* descs, int ndesc, int64_t total, const double* scales,
                       hipStream_t s) {
    if (ndesc == 0 || total == 0) return hipSuccess;
    for (int64_t e0 = 0; e0 < total; e0 += kMaxGridElems) {
        const dim3 grid((unsigned)((std::min(kMaxGridElems, total - e0) + 255) / 256)), block(256);
        const hipError_t e = by_prec(prec, [&](auto t) {
            copy_grouped<decltype(t)><<<grid, block, 0, s>>>(descs, ndesc, scales, total, e0);
        });
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ------------------------------------------------------------------------------------------
// Reverse pass
// ------------------------------------------------------------------------------------------
// C(view) = f * sum of split-K partials, converted to the compute precision (the partial GEMM
// normally carries the factor already, and f = 1).
template <typename Tout>
__global__ __launch_bounds__(256) void reduce_grouped(const ReduceDesc* __restrict__ descs, int ndesc,
                                                      const double* __restrict__ scales, int64_t total, int64_t e0) {
    const int64_t e = e0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    int lo = 0, hi = ndesc - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (descs[mid].elem_begin <= e) lo = mid;
        else hi = mid - 1;
    }
    const ReduceDesc& d = descs[lo];
    const int64_t local = e - d.elem_begin;
    const int64_t MN = (int64_t)d.M * d.N;
    const int r = (int)(local / d.N), c = (int)(local - (int64_t)r * d.N);
    double acc = 0.0;
    for (int p = 0; p < d.splits; ++p) acc += d.part[p * MN + local];
    const double f = inv_scale(scales, d.scale_a) * inv_scale(scales, d.scale_b);
    Tout* out = (Tout*)d.out;
    out[axis_offset(d.vc.row, (uint32_t)r) + axis_offset(d.vc.col, (uint32_t)c)] = (Tout)(acc * f);
}

// Adjoint of one compression in the space of its core.  With the core SVD
// R~_A R~_B^T = U s V^T (all singular triplets above the rounding level, the "+" set, r of them,
// the first nK kept), L = R~_B^T V s^-1 and M = R~_A^T U s^-1 (D x r), the inputs
// H_A = A^T G_a, H_B = B G_b^T (D x nK) give a = L^T H_A, b = M^T H_B (r x nK) and
//   Phi (r x r): the truncated-SVD adjoint in singular coordinates (full spectrum; kept pairs in
//                their gauge-invariant form),
//   N_A = L Psi_A L^T + sum_t L_t H_B,t^T / sqrt(s_t),   N_B = M Psi_B M^T + sum_t H_A,t M_t^T / sqrt(s_t),
//   Psi_A = Phi s - a s^1/2 E^T - E s^-1/2 b^T s,   Psi_B = s Phi - s a s^-1/2 E^T - E s^1/2 b^T,
// so that A_bar = G_a P_L^T + A N_A and B_bar = P_R^T G_b + N_B B need no inverse of R~.
constexpr size_t kCoreBwdLdsBytes = 2 * 32 * 128 * sizeof(double);

// Phases of core_bwd_kernel: 0 = the whole adjoint in one workgroup per compression; for large
// cores the same steps split over launches, the D x D products one 128 x 128 tile per workgroup:
// 1 = + set, H sums, sorted vectors; 2 = tiles of R~_B^T V_+ and R~_A^T W_+; 3 = scaling, a, b,
// Phi, Psi, scaled H; 4 = tiles of L Psi_A and M Psi_B; 5 = tiles of N_A and N_B.
constexpr int kBwdTile = 128;

template <typename Tp>
__global__ __launch_bounds__(kCoreThreads) void core_bwd_kernel(const CoreBwdDesc* __restrict__ descs, int phase,
                                                                int per_core) {
    extern __shared__ double lds[];   // GEMM staging, 2 x 32 x 128 doubles
    const int ci = blockIdx.x / per_core, q = blockIdx.x - ci * per_core;
    const CoreBwdDesc& d = descs[ci];
    const int tid = threadIdx.x;
    const int D = d.D, cn = d.chi_new, DD = D * D;
    const double* Ra = d.work;
    const double* Rb = Ra + DD;
    const double* W = Rb + DD;
    const double* V = W + DD;
    const double* sig = V + DD;
    const int* order = (const int*)(sig + D);
    const int* ranks = (const int*)(sig + 2 * D);
    const int ra = ranks[0], rb = ranks[1];
    double* L = d.ws;             // D x D, L[dd*D + p]
    double* Mm = L + DD;          // D x D
    double* Phi = Mm + DD;        // r x r (ld D)
    double* PsiA = Phi + DD;
    double* PsiB = PsiA + DD;
    double* T = PsiB + DD;        // D x D scratch
    double* HA = T + DD;          // D x cn
    double* HB = HA + D * cn;
    double* a = HB + D * cn;      // r x cn (ld cn)
    double* b = a + D * cn;
    double* sg = b + D * cn;      // sigma of the + set, descending
    double* sq = sg + D;          // sqrt(sigma)
    int* meta = (int*)(sq + D);   // r, nk (phase 1 -> later phases)
    // singular vectors of the + set in descending order (columns), into the Psi slots (free
    // until Psi is formed): Vs = V_+, Ws = W_+ = U_+ s; H_B, H_A scaled by s^-1/2 into the a, b
    // slots once Psi exists
    double* Vs = PsiA;
    double* Ws = PsiB;
    double* HBs = a;
    double* HAs = b;
    const bool all = phase == 0;
    const double smax = rb > 0 ? sig[order[0]] : 0.0;
    int r, nk;
    if (all || phase == 1) {
        __shared__ double sh_part[kCoreWaves];
        __shared__ int sh_cnt[2][kCoreWaves];
        const int lane = tid & 63, wave = tid >> 6;
        // ||sigma|| and, since order sorts sigma descending, the size r of the + set (sigma above
        // both zero thresholds) and the kept count nk as plain counts (block reductions)
        {
            double f = 0.0;
            for (int j = tid; j < rb; j += kCoreThreads) f = fma(sig[j], sig[j], f);
            f = wave_sum(f);
            if (lane == 0) sh_part[wave] = f;
            __syncthreads();
        }
        double fro = 0.0;
        for (int w = 0; w < kCoreWaves; ++w) fro += sh_part[w];
        fro = sqrt(fro);
        {
            int c1 = 0, c2 = 0;
            for (int j = tid; j < rb; j += kCoreThreads) {
                c1 += (sig[j] > kNoiseRel * smax && sig[j] > 4.0 * kZeroRel * fro) ? 1 : 0;
                c2 += sig[j] >= d.cutoff * smax ? 1 : 0;
            }
            c1 = (int)wave_sum((double)c1);
            c2 = (int)wave_sum((double)c2);
            if (lane == 0) {
                sh_cnt[0][wave] = c1;
                sh_cnt[1][wave] = c2;
            }
            __syncthreads();
        }
        int nc = 0;
        r = 0;
        for (int w = 0; w < kCoreWaves; ++w) {
            r += sh_cnt[0][w];
            nc += sh_cnt[1][w];
        }
        nk = min(min(cn, r), nc);
        if (tid == 0) {
            meta[0] = r;
            meta[1] = nk;
        }
        for (int p = tid; p < r; p += kCoreThreads) {
            sg[p] = sig[order[p]];
            sq[p] = sqrt(sg[p]);
        }
        const double* ha = d.h;
        const double* hb = d.h + (int64_t)d.splits_a * D * cn;
        for (int idx = tid; idx < D * cn; idx += kCoreThreads) {
            double x = 0.0, y = 0.0;
            for (int p = 0; p < d.splits_a; ++p) x += ha[(int64_t)p * D * cn + idx];
            for (int p = 0; p < d.splits_b; ++p) y += hb[(int64_t)p * D * cn + idx];
            HA[idx] = x;
            HB[idx] = y;
        }
        for (int idx = tid; idx < r * D; idx += kCoreThreads) {
            const int p = idx / D, i = idx - p * D;
            const int j = order[p];
            Vs[(int64_t)p * D + i] = i < rb ? V[(int64_t)j * D + i] : 0.0;
            Ws[(int64_t)p * D + i] = i < ra ? W[(int64_t)j * D + i] : 0.0;
        }
        __syncthreads();
        if (!all) return;
    } else {
        r = meta[0];
        nk = meta[1];
    }
    // tile q of the phase's two products (the first product's tiles, then the second's)
    const int tr = (r + kBwdTile - 1) / kBwdTile, td = (D + kBwdTile - 1) / kBwdTile;
    auto tile_of = [&](int ntile_cols, int* which, int* i0, int* j0) {
        const int per = td * ntile_cols;
        if (per == 0) return false;   // empty + set
        *which = q / per;
        const int t = q - *which * per;
        *i0 = (t / ntile_cols) * kBwdTile;
        *j0 = (t % ntile_cols) * kBwdTile;
        return *which < 2;
    };
    // L = R~_B^T V_+ s^-1, M = R~_A^T (W_+ s^-1) s^-1, on the MFMA (unscaled products first)
    if (all) {
        wg_gemm_f64(Rb, 1, D, Vs, 1, D, L, D, D, r, rb, lds);
        wg_gemm_f64(Ra, 1, D, Ws, 1, D, Mm, D, D, r, ra, lds);
    } else if (phase == 2) {
        int which, i0, j0;
        if (!tile_of(tr, &which, &i0, &j0)) return;
        if (which == 0)
            wg_gemm_tile<double>(Rb, 1, D, Vs, 1, D, rb, nullptr, 0, 0, nullptr, 0, 0, 0, L, D, D, r, i0, j0, lds);
        else
            wg_gemm_tile<double>(Ra, 1, D, Ws, 1, D, ra, nullptr, 0, 0, nullptr, 0, 0, 0, Mm, D, D, r, i0, j0, lds);
        return;
    }
    if (all || phase == 3) {
        for (int idx = tid; idx < D * r; idx += kCoreThreads) {
            const int dd = idx / r, p = idx - dd * r;
            L[dd * D + p] /= sg[p];
            Mm[dd * D + p] /= sg[p] * sg[p];
        }
        __syncthreads();
        // a = L^T H_A, b = M^T H_B  (r x nk, leading dimension cn)
        wg_gemm_f64_narrow(L, 1, D, HA, cn, 1, a, cn, r, nk, D);
        wg_gemm_f64_narrow(Mm, 1, D, HB, cn, 1, b, cn, r, nk, D);
        __syncthreads();
        // Phi[x][y].  Kept block (x, y < nk, the diagonal included): the gauge-invariant form
        // (s_y^1/2 a_xy + s_x^1/2 b_yx) / (s_x + s_y), equal to the textbook entry because ln|Z| is
        // invariant under an orthogonal change of basis of the new bond, and free of any division
        // by a gap between kept values.  A kept index against a discarded one: the textbook
        // 1 / (s_y^2 - s_x^2) terms (the gap of the truncation itself).
        for (int idx = tid; idx < r * r; idx += kCoreThreads) {
            const int x = idx / r, y = idx - x * r;
            const double sx = sg[x], sy = sg[y];
            double v = 0.0;
            if (x < nk && y < nk) {
                v = (a[x * cn + y] * sq[y] + b[y * cn + x] * sq[x]) / (sx + sy);
            } else if (y < nk) {   // i = y kept, j = x discarded
                v = (a[x * cn + y] * sq[y] * sy + b[x * cn + y] * sq[y] * sx) / (sy * sy - sx * sx);
            } else if (x < nk) {   // i = x kept, j = y discarded
                v = -(a[y * cn + x] * sq[x] * sy + b[y * cn + x] * sq[x] * sx) / (sy * sy - sx * sx);
            }
            Phi[x * D + y] = v;
        }
        __syncthreads();
        for (int idx = tid; idx < r * r; idx += kCoreThreads) {
            const int x = idx / r, y = idx - x * r;
            const double ph = Phi[x * D + y], sx = sg[x], sy = sg[y];
            double pa = ph * sy, pb = sx * ph;
            if (y < nk) {
                pa -= a[x * cn + y] * sq[y];
                pb -= sx * a[x * cn + y] / sq[y];
            }
            if (x < nk) {
                pa -= b[y * cn + x] * sy / sq[x];
                pb -= sq[x] * b[y * cn + x];
            }
            PsiA[x * D + y] = pa;
            PsiB[x * D + y] = pb;
        }
        __syncthreads();
        for (int idx = tid; idx < D * cn; idx += kCoreThreads) {
            const int t = idx % cn;
            HBs[idx] = t < nk ? HB[idx] / sq[t] : 0.0;
            HAs[idx] = t < nk ? HA[idx] / sq[t] : 0.0;
        }
        __syncthreads();
        if (!all) return;
    }
    // T_A = L Psi_A (T slot), T_B = M Psi_B (Phi slot: Phi is no longer needed)
    double* TA = T;
    double* TB = Phi;
    if (all) {
        wg_gemm_f64(L, D, 1, PsiA, D, 1, TA, D, D, r, r, lds);
        wg_gemm_f64(Mm, D, 1, PsiB, D, 1, TB, D, D, r, r, lds);
    } else if (phase == 4) {
        int which, i0, j0;
        if (!tile_of(tr, &which, &i0, &j0)) return;
        if (which == 0)
            wg_gemm_tile<double>(L, D, 1, PsiA, D, 1, r, nullptr, 0, 0, nullptr, 0, 0, 0, TA, D, D, r, i0, j0, lds);
        else
            wg_gemm_tile<double>(Mm, D, 1, PsiB, D, 1, r, nullptr, 0, 0, nullptr, 0, 0, 0, TB, D, D, r, i0, j0, lds);
        return;
    }
    // N_A = T_A L^T + sum_t L_t H_B,t^T / sqrt(s_t);  N_B = T_B M^T + sum_t H_A,t M_t^T / sqrt(s_t)
    Tp* na = (Tp*)d.n_a;
    Tp* nb = (Tp*)d.n_b;
    if (all) {
        for (int i0 = 0; i0 < D; i0 += kBwdTile)
            for (int j0 = 0; j0 < D; j0 += kBwdTile) {
                wg_gemm_tile<Tp>(TA, D, 1, L, 1, D, r, L, D, 1, HBs, 1, cn, nk, na, D, D, D, i0, j0, lds);
                wg_gemm_tile<Tp>(TB, D, 1, Mm, 1, D, r, HAs, cn, 1, Mm, 1, D, nk, nb, D, D, D, i0, j0, lds);
            }
    } else if (phase == 5) {
        int which, i0, j0;
        if (!tile_of(td, &which, &i0, &j0)) return;
        if (which == 0)
            wg_gemm_tile<Tp>(TA, D, 1, L, 1, D, r, L, D, 1, HBs, 1, cn, nk, na, D, D, D, i0, j0, lds);
        else
            wg_gemm_tile<Tp>(TB, D, 1, Mm, 1, D, r, HAs, cn, 1, Mm, 1, D, nk, nb, D, D, D, i0, j0, lds);
    }
}

// Adjoint of the final scalar: d ln|x| / d x^ = 1 / x^ with x^ = x / s the normalised value.
template <typename Tp>
__global__ void seed_kernel(const void* __restrict__ final_ptr, void* __restrict__ adj, const double* scales,
                            int final_index) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double x = (double)((const Tp*)final_ptr)[0];
        ((Tp*)adj)[0] = (Tp)(x != 0.0 ? scales[final_index] / x : 0.0);
    }
}

// d ln|Z| / d data_v = adj(T^_v) / s_v, in the input layout (float64).
template <typename Tp>
__global__ void grad_inputs_kernel(const InputDesc* __restrict__ descs, int n, const double* __restrict__ scales,
                                   double* __restrict__ out) {
    const int gw = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (gw >= n) return;
    const InputDesc& d = descs[gw];
    const Tp* x = (const Tp*)d.dst;
    const double inv = 1.0 / scales[d.tensor];
    for (int64_t i = lane; i < d.count; i += 64) out[d.src_off + i] = (double)x[i] * inv;
}

// ------------------------------------------------------------------------------------------
// Ising couplings (SI F.1): T_v[s_1..s_d] = sum_x prod_k W^(e_k)[x, s_k], with the bond matrix
// exp(beta J s s') split as W_lo W_hi, W = H diag(sqrt c, +-sqrt|sh|) H / sqrt 2, c = cosh(beta J),
// sh = sinh(beta J), the sign of sinh on the higher vertex id; so W[x][s] = (d0 + (x == s ? d1 : -d1)) / sqrt 2.
// ------------------------------------------------------------------------------------------
__device__ inline void ising_factor(double beta, double J, bool hi, bool deriv, double* w) {
    const double x = beta * J, c = cosh(x), sh = sinh(x);
    const double sg = sh < 0.0 ? -1.0 : 1.0;
    double d0, d1;
    if (!deriv) {
        d0 = sqrt(c);
        d1 = (hi ? sg : 1.0) * sqrt(fabs(sh));
    } else {   // d/dJ of (sqrt c, +-sqrt|sh|)
        d0 = beta * sh / (2.0 * sqrt(c));
        d1 = (hi ? 1.0 : sg) * beta * c / (2.0 * sqrt(fabs(sh)));
    }
    const double r = 0.70710678118654752440;   // 1 / sqrt 2
    w[0] = (d0 + d1) * r;   // [x][s] with x == s
    w[1] = (d0 - d1) * r;   // x != s
}

// One thread per tensor entry.
__global__ void ising_values_kernel(IsingGraph g, double beta, const double* __restrict__ J, double* __restrict__ data,
                                    int64_t total) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    int lo = 0, hi = g.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (g.data_off[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    const int v = lo;
    const int b = g.inc_off[v], d = g.inc_off[v + 1] - b;
    const int64_t idx = e - g.data_off[v];
    double acc = 0.0;
    for (int x = 0; x < 2; ++x) {
        double p = 1.0;
        for (int k = 0; k < d; ++k) {
            const int ed = g.inc_edge[b + k];
            const int s = (int)((idx >> (d - 1 - k)) & 1);
            double w[2];
            ising_factor(beta, J[ed], g.edge_v[ed] == v, false, w);
            p *= (x == s) ? w[0] : w[1];
        }
        acc += p;
    }
    data[e] = acc;
}

// d ln|Z| / d J_e = sum over both ends v of sum_s (d ln|Z| / d T_v[s]) (d T_v[s] / d J_e); one thread per edge.
__global__ void ising_grad_kernel(IsingGraph g, double beta, const double* __restrict__ J,
                                  const double* __restrict__ dT, double* __restrict__ dJ) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= g.ne) return;
    double total = 0.0;
    for (int end = 0; end < 2; ++end) {
        const int v = end == 0 ? g.edge_u[e] : g.edge_v[e];
        const int b = g.inc_off[v], d = g.inc_off[v + 1] - b;
        const double* gv = dT + g.data_off[v];
        for (int64_t idx = 0; idx < ((int64_t)1 << d); ++idx) {
            double acc = 0.0;
            for (int x = 0; x < 2; ++x) {
                double p = 1.0;
                for (int k = 0; k < d; ++k) {
                    const int ed = g.inc_edge[b + k];
                    const int s = (int)((idx >> (d - 1 - k)) & 1);
                    double w[2];
                    ising_factor(beta, J[ed], g.edge_v[ed] == v, ed == e, w);
                    p *= (x == s) ? w[0] : w[1];
                }
                acc += p;
            }
            total += gv[idx] * acc;
        }
    }
    dJ[e] = total;
}

hipError_t launch_ising_values(const IsingGraph& g, double beta, const double* J, double* data, int64_t total,
                               hipStream_t s) {
    if (total == 0) return hipSuccess;
    ising_values_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(g, beta, J, data, total);
    return hipGetLastError();
}

hipError_t launch_ising_grad(const IsingGraph& g, double beta, const double* J, const double* dlnz_ddata,
                             double* dlnz_dJ, hipStream_t s) {
    if (g.ne == 0) return hipSuccess;
    ising_grad_kernel<<<(g.ne + 127) / 128, 128, 0, s>>>(g, beta, J, dlnz_ddata, dlnz_dJ);
    return hipGetLastError();
}

size_t core_lds_bytes(int max_d) { return (size_t)4 * max_d * max_d * sizeof(double); }

void init_kernel_attrs() {
    const int tsqr_lds = kTsqrElems * (int)sizeof(double);
    (void)hipFuncSetAttribute((const void*)tsqr_blocks<double>, hipFuncAttributeMaxDynamicSharedMemorySize, tsqr_lds);
    (void)hipFuncSetAttribute((const void*)tsqr_blocks<float>, hipFuncAttributeMaxDynamicSharedMemorySize, tsqr_lds);
    (void)hipFuncSetAttribute((const void*)tsqr_blocks<bf16>, hipFuncAttributeMaxDynamicSharedMemorySize, tsqr_lds);
    (void)hipFuncSetAttribute((const void*)block_jacobi_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBJLdsBytes);
    (void)hipFuncSetAttribute((const void*)core_kernel<false, double>, hipFuncAttributeMaxDynamicSharedMemorySize, kCoreBwdLdsBytes);
    (void)hipFuncSetAttribute((const void*)core_kernel<false, float>, hipFuncAttributeMaxDynamicSharedMemorySize, kCoreBwdLdsBytes);
    (void)hipFuncSetAttribute((const void*)core_kernel<false, bf16>, hipFuncAttributeMaxDynamicSharedMemorySize, kCoreBwdLdsBytes);
    (void)hipFuncSetAttribute((const void*)core_bwd_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize, kCoreBwdLdsBytes);
    (void)hipFuncSetAttribute((const void*)core_bwd_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize, kCoreBwdLdsBytes);
    (void)hipFuncSetAttribute((const void*)core_bwd_kernel<bf16>, hipFuncAttributeMaxDynamicSharedMemorySize, kCoreBwdLdsBytes);
    (void)hipFuncSetAttribute((const void*)gram_lanczos_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize, kLanczosLdsBytes);
    (void)hipFuncSetAttribute((const void*)gram_lanczos_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize, kLanczosLdsBytes);
    (void)hipFuncSetAttribute((const void*)lanczos_kernel<float, float>, hipFuncAttributeMaxDynamicSharedMemorySize, kLanczosLdsBytes);
    (void)hipFuncSetAttribute((const void*)lanczos_kernel<double, double>, hipFuncAttributeMaxDynamicSharedMemorySize, kLanczosLdsBytes);
    const int bytes = (int)core_lds_bytes(kCoreLdsMaxD);
    (void)hipFuncSetAttribute((const void*)core_kernel<true, float>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute((const void*)core_kernel<true, double>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute((const void*)core_kernel<true, bf16>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute((const void*)gram_lanczos_kernel<bf16>, hipFuncAttributeMaxDynamicSharedMemorySize, kLanczosLdsBytes);
    (void)hipFuncSetAttribute((const void*)lanczos_kernel<bf16, bf16>, hipFuncAttributeMaxDynamicSharedMemorySize, kLanczosLdsBytes);
}

hipError_t launch_core(int lds, int prec, const CoreDesc* descs, int ndesc, int max_d, int max_sweeps,
                       double* disc, int32_t* tie, int32_t* sweeps, hipStream_t s) {
    if (ndesc == 0) return hipSuccess;
    dim3 grid(ndesc), block(lds ? kCoreLdsThreads : kCoreThreads);
    const size_t bytes = core_lds_bytes(max_d);
    return by_prec(prec, [&](auto t) {
        using Tp = decltype(t);
        if (lds) {
            core_kernel<true, Tp><<<grid, block, bytes, s>>>(descs, max_sweeps, disc, tie, sweeps, 0);
        } else if (max_d > 64 && max_d <= kBJRows) {
            // factors and core; block-Jacobi sweeps, one launch per tournament round; the rest
            core_kernel<false, Tp><<<grid, block, kCoreBwdLdsBytes, s>>>(descs, max_sweeps, disc, tie, sweeps, 1);
            int nb = (max_d + kBJCols - 1) / kBJCols;
            nb += nb & 1;
            const dim3 bgrid(ndesc * (nb / 2));
            const int issued = kBJSweeps < max_sweeps ? kBJSweeps : max_sweeps;
            for (int sw = 0; sw < issued; ++sw)
                for (int r = 0; r < nb - 1; ++r)
                    block_jacobi_kernel<<<bgrid, dim3(kBJThreads), kBJLdsBytes, s>>>(descs, nb / 2, sw, r);
            core_kernel<false, Tp><<<grid, block, kCoreBwdLdsBytes, s>>>(descs, max_sweeps, disc, tie, sweeps, 2);
        } else {
            core_kernel<false, Tp><<<grid, block, kCoreBwdLdsBytes, s>>>(descs, max_sweeps, disc, tie, sweeps, 0);
        }
    });
}

int core_launch_count(int lds, int max_d, int max_sweeps) {
    if (lds || max_d <= 64 || max_d > kBJRows) return 1;
    int nb = (max_d + kBJCols - 1) / kBJCols;
    nb += nb & 1;
    return 2 + std::min(kBJSweeps, max_sweeps) * (nb - 1);
}

size_t lanczos_lds_bytes(int s_max) { return (size_t)2 * (s_max + 1) * (s_max + 1) * sizeof(double); }

hipError_t launch_lanczos(int prec, const LanczosDesc* descs, int ndesc, int s_max, const double* scales,
                          int max_sweeps, double* disc, int32_t* tie, int32_t* sweeps, hipStream_t s) {
    (void)s_max;
    if (ndesc == 0) return hipSuccess;
    dim3 grid(ndesc), block(kCoreThreads);
    const size_t bytes = kLanczosLdsBytes;
    return by_prec(prec, [&](auto t) {
        using T = decltype(t);
        lanczos_kernel<T, T><<<grid, block, bytes, s>>>(descs, scales, max_sweeps, disc, tie, sweeps);
    });
}

hipError_t launch_gram_lanczos(int prec, const GLanczosDesc* descs, int ndesc, int max_sweeps, double* disc,
                               int32_t* tie, int32_t* sweeps, hipStream_t s) {
    if (ndesc == 0) return hipSuccess;
    dim3 grid(ndesc), block(kCoreThreads);
    const size_t bytes = kLanczosLdsBytes;
    return by_prec(prec, [&](auto t) {
        gram_lanczos_kernel<decltype(t)><<<grid, block, bytes, s>>>(descs, max_sweeps, disc, tie, sweeps);
    });
}

hipError_t launch_scale_finalize(const ScaleDesc* descs, int n, const double* maxparts, double* scales,
                                 hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int threads = 256;
    dim3 grid((unsigned)((n * 64 + threads - 1) / threads)), block(threads);
    scale_finalize<<<grid, block, 0, s>>>(descs, n, maxparts, scales);
    return hipGetLastError();
}

hipError_t launch_inputs(int prec, const InputDesc* descs, int n, const double* staging, double* scales,
                         hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int threads = 256;
    dim3 grid((unsigned)((n * 64 + threads - 1) / threads)), block(threads);
    return by_prec(prec, [&](auto t) {
        using T = decltype(t);
        input_scatter<T><<<grid, block, 0, s>>>(descs, n, staging);
        input_scales<T><<<grid, block, 0, s>>>(descs, n, scales);
    });
}

hipError_t launch_reduce(int prec, const ReduceDesc* descs, int ndesc, int64_t total, const double* scales,
                         hipStream_t s) {
    if (ndesc == 0 || total == 0) return hipSuccess;
    for (int64_t e0 = 0; e0 < total; e0 += kMaxGridElems) {
        const dim3 grid((unsigned)((std::min(kMaxGridElems, total - e0) + 255) / 256)), block(256);
        const hipError_t e = by_prec(prec, [&](auto t) {
            reduce_grouped<decltype(t)><<<grid, block, 0, s>>>(descs, ndesc, scales, total, e0);
        });
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_core_bwd(int prec, const CoreBwdDesc* descs, int ndesc, int max_d, hipStream_t s) {
    if (ndesc == 0) return hipSuccess;
    return by_prec(prec, [&](auto t) {
        using Tp = decltype(t);
        if (max_d <= kCoreLdsMaxD) {
            core_bwd_kernel<Tp><<<ndesc, kCoreThreads, kCoreBwdLdsBytes, s>>>(descs, 0, 1);
        } else {
            // the D x D products of large cores over many workgroups: two products per phase,
            // one 128 x 128 tile per workgroup
            const int td = (max_d + kBwdTile - 1) / kBwdTile, per = 2 * td * td;
            core_bwd_kernel<Tp><<<ndesc, kCoreThreads, kCoreBwdLdsBytes, s>>>(descs, 1, 1);
            core_bwd_kernel<Tp><<<ndesc * per, kCoreThreads, kCoreBwdLdsBytes, s>>>(descs, 2, per);
            core_bwd_kernel<Tp><<<ndesc, kCoreThreads, kCoreBwdLdsBytes, s>>>(descs, 3, 1);
            core_bwd_kernel<Tp><<<ndesc * per, kCoreThreads, kCoreBwdLdsBytes, s>>>(descs, 4, per);
            core_bwd_kernel<Tp><<<ndesc * per, kCoreThreads, kCoreBwdLdsBytes, s>>>(descs, 5, per);
        }
    });
}

hipError_t launch_seed(int prec, const void* final_ptr, void* adj_final, const double* scales, int final_index,
                       hipStream_t s) {
    return by_prec(prec, [&](auto t) { seed_kernel<decltype(t)><<<1, 64, 0, s>>>(final_ptr, adj_final, scales, final_index); });
}

hipError_t launch_grad_inputs(int prec, const InputDesc* descs, int n, const double* scales, double* out,
                              hipStream_t s) {
    if (n == 0) return hipSuccess;
    const dim3 grid((unsigned)((n * 64 + 255) / 256)), block(256);
    return by_prec(prec, [&](auto t) { grad_inputs_kernel<decltype(t)><<<grid, block, 0, s>>>(descs, n, scales, out); });
}

// ------------------------------------------------------------------------------------------
// Block-Krylov compressions: small dense float64 operations and the orthonormalising factor of
// a block (the products themselves run on gemm_grouped)
// ------------------------------------------------------------------------------------------

// SplitMix64 finaliser (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
// OOPSLA 2014): a counter-based generator for the Krylov start blocks.
__device__ inline double hash_uniform(uint32_t seed, uint64_t i) {
    uint64_t z = ((uint64_t)seed << 32) ^ i;
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;   // 53 bits -> [-1, 1)
}

template <typename Tp>
__global__ __launch_bounds__(256) void small_grouped(const SmallDesc* __restrict__ descs, int ndesc,
                                                     int64_t total, int64_t e0) {
    const int64_t e = e0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    int lo = 0, hi = ndesc - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (descs[mid].elem_begin <= e) lo = mid;
        else hi = mid - 1;
    }
    const SmallDesc& d = descs[lo];
    const int64_t local = e - d.elem_begin;
    const int r = (int)(local / d.cols), c = (int)(local - (int64_t)r * d.cols);
    double* dst = (double*)d.dst;
    const int64_t o = (int64_t)r * d.dst_ld + c;
    switch (d.op) {
        case SM_RANDOM: dst[o] = hash_uniform(d.seed, (uint64_t)local); break;
        case SM_COPY:
            dst[o] = d.transpose ? d.src[(int64_t)c * d.src_ld + r] : d.src[(int64_t)r * d.src_ld + c];
            break;
        case SM_NEG: dst[o] = -d.src[(int64_t)r * d.src_ld + c]; break;
        case SM_SYM:
            if (r < c) {
                const int64_t t = (int64_t)c * d.dst_ld + r;
                const double v = 0.5 * (dst[o] + dst[t]);
                dst[o] = v;
                dst[t] = v;
            }
            break;
        case SM_COLNORM2: {
            double acc = 0.0;
            for (int t = 0; t < d.src_rows; ++t) {
                const double v = d.src[(int64_t)t * d.src_ld + c];
                acc = fma(v, v, acc);
            }
            dst[o] = acc;
            break;
        }
        case SM_COLSCALE: dst[o] *= d.src[c]; break;
        case SM_IDENTITY: dst[o] = r == c ? 1.0 : 0.0; break;
        case SM_CAST: {
            const double v = d.transpose ? d.src[(int64_t)c * d.src_ld + r] : d.src[(int64_t)r * d.src_ld + c];
            ((Tp*)d.dst)[o] = (Tp)v;
            break;
        }
    }
}

hipError_t launch_small(int prec, const SmallDesc* descs, int ndesc, int64_t total, hipStream_t s) {
    if (ndesc == 0 || total == 0) return hipSuccess;
    for (int64_t e0 = 0; e0 < total; e0 += kMaxGridElems) {
        const dim3 grid((unsigned)((std::min(kMaxGridElems, total - e0) + 255) / 256)), block(256);
        const hipError_t e = by_prec(prec, [&](auto t) {
            small_grouped<decltype(t)><<<grid, block, 0, s>>>(descs, ndesc, total, e0);
        });
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

__global__ __launch_bounds__(256) void krylov_check_kernel(const KrylovCheckDesc* __restrict__ descs,
                                                           int32_t* __restrict__ stat_sweeps) {
    __shared__ double part[4];
    const KrylovCheckDesc& d = descs[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double s1 = d.nrm[0] > 0.0 ? 1.0 / d.nrm[0] : 0.0;
    bool bad = false;
    for (int i = 0; i < d.nw; ++i) {
        const double inv = d.nrm[i];
        if (!(inv > 0.0)) continue;   // masked pair
        const double si = 1.0 / inv;
        double acc = 0.0;
        for (int r = tid; r < d.n; r += 256) {
            const double v = d.e[(int64_t)r * d.nw + i] - si * d.qp[(int64_t)r * d.nw + i];
            acc = fma(v, v, acc);
        }
        acc = wave_sum(acc);
        if (lane == 0) part[wave] = acc;
        __syncthreads();
        const double tot = (part[0] + part[1]) + (part[2] + part[3]);
        __syncthreads();
        const double resid = sqrt(tot) * si * sqrt(si);
        if (!(resid <= d.tol * s1 * s1)) bad = true;
    }
    if (tid == 0 && bad) {
        const int32_t sw = stat_sweeps[d.stat];
        stat_sweeps[d.stat] = sw < 0 ? sw : -1 - sw;
    }
}

hipError_t launch_krylov_check(const KrylovCheckDesc* descs, int ndesc, int32_t* sweeps, hipStream_t s) {
    if (ndesc == 0) return hipSuccess;
    krylov_check_kernel<<<ndesc, 256, 0, s>>>(descs, sweeps);
    return hipGetLastError();
}

constexpr int kCholMaxB = 64;

// One wave per block; lane j owns column j.  Pivoted Cholesky on the full symmetric Gram in LDS
// (pivot: the largest remaining diagonal entry, lowest index on ties), then the inverse of the
// leading rank x rank triangle by back substitution, one column per lane.
__global__ __launch_bounds__(64) void cholinv_kernel(const CholInvDesc* __restrict__ descs) {
    __shared__ double A[kCholMaxB][kCholMaxB + 1];
    __shared__ double R[kCholMaxB][kCholMaxB + 1];
    __shared__ int perm[kCholMaxB];
    const CholInvDesc& d = descs[blockIdx.x];
    const int b = d.b, j = threadIdx.x;
    for (int i = 0; i < b; ++i)
        if (j < b) {
            A[i][j] = d.g[i * b + j];
            R[i][j] = 0.0;
        }
    if (j < b) perm[j] = j;
    __syncthreads();
    const double d0 = wave_max(j < b ? A[j][j] : 0.0);
    int rank = 0;
    for (int t = 0; t < b; ++t) {
        const double dj = (j >= t && j < b) ? A[j][j] : -1.0;
        const double dmax = wave_max(dj);
        if (!(dmax > 1e-14 * d0) || !(d0 > 0.0)) break;
        const unsigned long long hit = __ballot(dj == dmax);
        const int p = __ffsll((long long)hit) - 1;
        if (p != t) {   // symmetric swap of rows and columns t and p
            if (j < b) {
                const double x = A[t][j];
                A[t][j] = A[p][j];
                A[p][j] = x;
            }
            __syncthreads();
            if (j < b) {
                const double x = A[j][t];
                A[j][t] = A[j][p];
                A[j][p] = x;
            }
            if (j == 0) {
                const int x = perm[t];
                perm[t] = perm[p];
                perm[p] = x;
            }
            for (int i = 0; i < t; ++i)   // earlier rows of R follow the column swap
                if (j == 0) {
                    const double x = R[i][t];
                    R[i][t] = R[i][p];
                    R[i][p] = x;
                }
            __syncthreads();
        }
        const double rtt = sqrt(A[t][t]);
        if (j == t) R[t][t] = rtt;
        if (j > t && j < b) R[t][j] = A[t][j] / rtt;
        __syncthreads();
        if (j > t && j < b) {
            const double rj = R[t][j];
            for (int i = t + 1; i < b; ++i) A[i][j] = fma(-R[t][i], rj, A[i][j]);
        }
        __syncthreads();
        rank = t + 1;
    }
    // X = R[0:rank, 0:rank]^-1 (upper triangular), column j by back substitution into column j
    // of A (no longer needed; each lane touches only its own column)
    if (j < rank) {
        A[j][j] = 1.0 / R[j][j];
        for (int i = j - 1; i >= 0; --i) {
            double acc = 0.0;
            for (int l = i + 1; l <= j; ++l) acc = fma(R[i][l], A[l][j], acc);
            A[i][j] = -acc / R[i][i];
        }
    }
    // M[perm[i], j] = X[i, j] for i <= j < rank; zero elsewhere
    if (j < b)
        for (int i = 0; i < b; ++i) d.m[i * b + j] = 0.0;
    __syncthreads();
    if (j < rank)
        for (int i = 0; i <= j; ++i) d.m[perm[i] * b + j] = A[i][j];
}

hipError_t launch_cholinv(const CholInvDesc* descs, int ndesc, hipStream_t s) {
    if (ndesc == 0) return hipSuccess;
    cholinv_kernel<<<ndesc, 64, 0, s>>>(descs);
    return hipGetLastError();
}

// Device wall-clock stamp (100 MHz counter) on a stream, for timing the launches between two stamps
// also inside captured graphs.  One lane writes through a lane-indexed address (a vector store).
__global__ void stamp_kernel(unsigned long long* __restrict__ dst) { dst[threadIdx.x] = wall_clock64(); }

hipError_t launch_stamp(unsigned long long* dst, hipStream_t s) {
    stamp_kernel<<<1, 1, 0, s>>>(dst);
    return hipGetLastError();
}

hipError_t launch_result(int prec, const double* scales, int n_scales, const void* final_ptr, const int32_t* sweeps,
                         int n_comp, double* result, hipStream_t s) {
    return by_prec(prec, [&](auto t) {
        result_kernel<decltype(t)><<<1, 1024, 0, s>>>(scales, n_scales, final_ptr, sweeps, n_comp, result);
    });
}

}  // namespace tn
