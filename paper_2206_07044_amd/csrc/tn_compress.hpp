// One bond compression between two dense float64 matrices (see tn_compress.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "tn_internal.hpp"

namespace tn {

// Device descriptors of one compression, uploaded to the start of its workspace.
struct PairDescs {
    GemmDesc gram[2];
    CopyDesc copy[2];
    CoreDesc core;
    GemmDesc absorb[2];
};

// Byte offsets of the parts of a compression's workspace (all 256-byte aligned).
struct PairLayout {
    int64_t ma, D, mb, nw;
    bool gram_a, gram_b;
    int64_t splits_a, splits_b;
    int64_t off_desc, off_side_a, off_side_b, off_work, off_pl, off_pr, off_maxparts, off_stats;
    int64_t n_maxparts;
    int64_t bytes;                // total workspace bytes
};

// Shapes -> workspace layout; "" or an error message (D must be <= 64).
std::string pair_layout(int64_t ma, int64_t D, int64_t mb, int64_t chi, PairLayout* L);
// Enqueue the compression on stream s using workspace ws (device, >= L.bytes, 256-aligned).
// `h` is host storage for the descriptors; it must stay valid until the stream has run the
// upload (callers synchronise before it goes out of scope).  Returns "" or an error message.
std::string pair_enqueue(const PairLayout& L, const double* a, const double* b, double cutoff, int max_sweeps,
                         double* a_out, double* b_out, char* ws, PairDescs* h, hipStream_t s);

}  // namespace tn
