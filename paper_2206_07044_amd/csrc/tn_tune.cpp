// Tile selection of the tensor GEMMs and its measurement (see tn_tune.hpp, include/tn.h).
#include "tn_tune.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "tn_internal.hpp"
#include "tn_kernels.hpp"
#include "tn_plan.hpp"
#include "../../include/tn.h"

namespace tn {

static_assert(TN_TILE_64x64 == GV_64x64 && TN_TILE_256x16 == GV_256x16 && TN_TILE_16x256 == GV_16x256 &&
                  TN_TILE_128x32 == GV_128x32 && TN_TILE_32x128 == GV_32x128 && TN_TILE_SKINNY_TALL16 == GV_TALL16 &&
                  TN_TILE_SKINNY_TALL32 == GV_TALL32 && TN_TILE_SKINNY_WIDE16 == GV_WIDE16 &&
                  TN_TILE_SKINNY_WIDE32 == GV_WIDE32 && GV_COUNT == 9 && TN_GEMM_CLASSES == kGemmClasses,
              "tile ids of the C ABI and the kernels");

namespace {

// Class fields: prec (0 float64, 1 float32, 2 bfloat16), wide (M is the short side), short32 (the
// short side is 17..32), kclass (0: K <= 4, 1: K <= 64, 2: larger), long_unit (the long operand's
// long axis has unit stride).
struct ClassFields {
    int prec, wide, short32, kclass, long_unit;
};
ClassFields fields(int c) {
    ClassFields f;
    f.long_unit = c % 2;
    c /= 2;
    f.kclass = c % 3;
    c /= 3;
    f.short32 = c % 2;
    c /= 2;
    f.wide = c % 2;
    f.prec = c / 2;
    return f;
}

// Built-in choices, from grouped launches of 8-12 GEMMs of these shapes on MI355X: the skinny
// kernel for a short side of 16 with K <= 64 (3.7-4.1 TB/s against 2.0-2.1 for 64 x 64 tiles); for
// a short side of 32, 128 x 32 / 32 x 128 MFMA tiles (4.0-4.2 TB/s at K = 64), except the
// float32 / bfloat16 outer products (K <= 4), where the skinny kernel writes C at 4.9 TB/s.
int default_variant(int c) {
    const ClassFields f = fields(c);
    if (!f.wide) {
        if (!f.short32) {
            if (f.kclass <= 1) return (f.prec == 0 && !f.long_unit) ? GV_256x16 : GV_TALL16;
            return f.prec == 0 ? GV_256x16 : GV_128x32;
        }
        if (f.kclass == 0 && f.prec != 0) return GV_TALL32;
        return GV_128x32;
    }
    if (!f.short32) return f.kclass <= 1 ? GV_WIDE16 : GV_16x256;
    if (f.kclass == 0 && f.prec != 0) return GV_WIDE32;
    return GV_32x128;
}

std::mutex g_mu;
int g_table[kGemmClasses];
bool g_init = false;

void ensure_init() {   // caller holds g_mu
    if (g_init) return;
    for (int c = 0; c < kGemmClasses; ++c) g_table[c] = default_variant(c);
    g_init = true;
}

}  // namespace

int gemm_class(int prec, int64_t M, int64_t N, int64_t K, bool a_rows_unit, bool b_cols_unit) {
    if (prec < 0 || prec > 2) return -1;
    const bool tall = N <= 32 && M > 64 && M >= N;
    const bool wide = !tall && M <= 32 && N > 64;
    if (!tall && !wide) return -1;
    const int64_t s = tall ? N : M;
    const int kclass = K <= 4 ? 0 : K <= kSkinnyGemmMaxK ? 1 : 2;
    const int long_unit = tall ? (a_rows_unit ? 1 : 0) : (b_cols_unit ? 1 : 0);
    return (((prec * 2 + (wide ? 1 : 0)) * 2 + (s > 16 ? 1 : 0)) * 3 + kclass) * 2 + long_unit;
}

bool gemm_variant_allowed(int c, int v) {
    if (c < 0 || c >= kGemmClasses || v < 0 || v >= GV_COUNT) return false;
    const ClassFields f = fields(c);
    const bool skinny_k = f.kclass <= 1;
    if (v == GV_64x64) return true;
    if (!f.wide) {
        if (v == GV_256x16 || v == GV_TALL16) return !f.short32 && (v == GV_256x16 || skinny_k);
        if (v == GV_128x32) return true;
        if (v == GV_TALL32) return skinny_k;
        return false;
    }
    if (v == GV_16x256 || v == GV_WIDE16) return !f.short32 && (v == GV_16x256 || skinny_k);
    if (v == GV_32x128) return true;
    if (v == GV_WIDE32) return skinny_k;
    return false;
}

int pick_gemm_tile(int prec, int64_t M, int64_t N, int64_t K, bool a_rows_unit, bool b_cols_unit) {
    const int c = gemm_class(prec, M, N, K, a_rows_unit, b_cols_unit);
    if (c < 0) return GV_64x64;
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_init();
    return g_table[c];
}

void gemm_class_shape(int c, int* prec, int64_t* M, int64_t* N, int64_t* K, bool* a_rows_unit, bool* b_cols_unit) {
    const ClassFields f = fields(c);
    const int64_t s = f.short32 ? 32 : 16;
    const int64_t L = f.kclass == 2 ? 16384 : 65536;
    const int64_t k = f.kclass == 0 ? 2 : f.kclass == 1 ? 32 : 256;
    *prec = f.prec;
    *K = k;
    if (f.wide) {
        *M = s;
        *N = L;
        *a_rows_unit = true;
        *b_cols_unit = f.long_unit != 0;
    } else {
        *M = L;
        *N = s;
        *a_rows_unit = f.long_unit != 0;
        *b_cols_unit = true;
    }
}

}  // namespace tn

using namespace tn;

extern "C" {

tn_status tn_gemm_tiles_get(int32_t* table) {
    if (!table) return TN_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_init();
    for (int c = 0; c < kGemmClasses; ++c) table[c] = g_table[c];
    return TN_OK;
}

tn_status tn_gemm_tiles_set(const int32_t* table) {
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_init();
    if (!table) {
        for (int c = 0; c < kGemmClasses; ++c) g_table[c] = default_variant(c);
        return TN_OK;
    }
    for (int c = 0; c < kGemmClasses; ++c)
        if (!gemm_variant_allowed(c, table[c])) return TN_EINVAL;
    for (int c = 0; c < kGemmClasses; ++c) g_table[c] = table[c];
    return TN_OK;
}

tn_status tn_gemm_tune(int device, int32_t klass, int32_t copies, double* us) {
    if (!us || klass < 0 || klass >= kGemmClasses || copies < 1 || copies > 64) return TN_EINVAL;
    int prec;
    int64_t M, N, K;
    bool a_unit, b_unit;
    gemm_class_shape(klass, &prec, &M, &N, &K, &a_unit, &b_unit);
    const int64_t w = prec == 0 ? 8 : prec == 1 ? 4 : 2;
    const int key0 = prec == 0 ? GEMM_F64 : prec == 1 ? GEMM_F32 : GEMM_BF16;
    for (int v = 0; v < GV_COUNT; ++v) us[v] = -1.0;
    if (hipSetDevice(device) != hipSuccess) return TN_EDEVICE;
    // operands: A (M x K), B (K x N), C (M x N) per copy, one allocation; entries 1/64 (exact in
    // every precision), so the products stay finite
    const int64_t a_el = M * K, b_el = K * N, c_el = M * N;
    const int64_t per = ((a_el + b_el + c_el) * w + 255) / 256 * 256;
    char* mem = nullptr;
    double* aux = nullptr;   // scales (unused: -1) and per-tile maxima
    GemmDesc* dd = nullptr;
    const int64_t max_tiles = (int64_t)copies * ((M + 15) / 16) * ((N + 15) / 16);
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    tn_status st = TN_OK;
    auto hip_ok = [&](hipError_t e) {
        if (e != hipSuccess && st == TN_OK) st = TN_EDEVICE;
        return st == TN_OK;
    };
    if (hip_ok(hipMalloc((void**)&mem, per * copies)) && hip_ok(hipMalloc((void**)&aux, (max_tiles + 8) * 8)) &&
        hip_ok(hipMalloc((void**)&dd, sizeof(GemmDesc) * copies)) && hip_ok(hipStreamCreate(&s)) &&
        hip_ok(hipEventCreate(&e0)) && hip_ok(hipEventCreate(&e1))) {
        std::vector<char> host((size_t)per * copies, 0);
        for (int64_t i = 0; i < copies; ++i) {
            char* base = host.data() + i * per;
            for (int64_t e = 0; e < a_el + b_el; ++e) {
                if (w == 8) ((double*)base)[e] = 1.0 / 64;
                else if (w == 4) ((float*)base)[e] = 1.0f / 64;
                else ((uint16_t*)base)[e] = 0x3c80;   // bfloat16 1/64
            }
        }
        hip_ok(hipMemcpy(mem, host.data(), host.size(), hipMemcpyHostToDevice));
        ViewSpec va, vb;
        va.row_dims = {(int32_t)M};
        va.col_dims = {(int32_t)K};
        va.row_strides = {a_unit ? 1 : K};
        va.col_strides = {a_unit ? M : 1};
        vb.row_dims = {(int32_t)K};
        vb.col_dims = {(int32_t)N};
        vb.row_strides = {b_unit ? N : 1};
        vb.col_strides = {b_unit ? 1 : K};
        for (int v = 0; v < GV_COUNT && st == TN_OK; ++v) {
            if (!gemm_variant_allowed(klass, v)) continue;
            int bm, bn;
            gemm_tile(v, &bm, &bn);
            std::vector<GemmDesc> h(copies);
            int64_t tiles = 0, parts = 0;
            for (int i = 0; i < copies; ++i) {
                GemmDesc& g = h[i];
                std::memset(&g, 0, sizeof(g));
                if (!make_view(va, &g.va).empty() || !make_view(vb, &g.vb).empty()) {
                    st = TN_EINVAL;
                    break;
                }
                char* base = mem + (int64_t)i * per;
                g.A = base;
                g.B = base + a_el * w;
                g.C = base + (a_el + b_el) * w;
                g.M = (int32_t)M;
                g.N = (int32_t)N;
                g.K = (int32_t)K;
                g.mode = GEMM_TENSOR;
                g.tiles_m = (int32_t)((M + bm - 1) / bm);
                g.tiles_n = (int32_t)((N + bn - 1) / bn);
                g.splits = 1;
                g.k_per_split = (int32_t)K;
                g.scale_a = g.scale_b = -1;
                g.maxpart = (int32_t)parts;
                parts += (int64_t)g.tiles_m * g.tiles_n;
                g.tile_begin = tiles;
                tiles += (int64_t)g.tiles_m * g.tiles_n;
            }
            if (st != TN_OK || parts > max_tiles) break;
            if (!hip_ok(hipMemcpy(dd, h.data(), sizeof(GemmDesc) * copies, hipMemcpyHostToDevice))) break;
            const int key = key0 + kGemmVariantStride * v;
            const int warm = 2, reps = 10;
            for (int r = 0; r < warm && st == TN_OK; ++r) hip_ok(launch_gemm(key, dd, copies, tiles, aux, aux + 8, s));
            if (!hip_ok(hipEventRecord(e0, s))) break;
            for (int r = 0; r < reps && st == TN_OK; ++r) hip_ok(launch_gemm(key, dd, copies, tiles, aux, aux + 8, s));
            if (!hip_ok(hipEventRecord(e1, s)) || !hip_ok(hipEventSynchronize(e1))) break;
            float ms = 0.f;
            if (!hip_ok(hipEventElapsedTime(&ms, e0, e1))) break;
            us[v] = 1e3 * ms / reps;
        }
    }
    if (s) (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (dd) (void)hipFree(dd);
    if (aux) (void)hipFree(aux);
    if (mem) (void)hipFree(mem);
    return st;
}

}  // extern "C"
