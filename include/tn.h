/*
 * tn.h — C ABI of the MI355X compressed contraction-tree executor.
 *
 * The library evaluates Z, the scalar value of a closed tensor network
 * (Gray & Chan, arXiv:2206.07044, section I, Eq. (tncontract)), along a
 * fixed ordered contraction tree with bond compression: Algorithm 1
 * ("Approximate contraction", section II.F) with early or late compression
 * and tree-gauge distance r >= 0.  Each compression replaces every edge shared by two
 * tensors with one edge of dimension chi' = min(chi, k_A, k_B) using the
 * reduced truncated SVD of section II.C, Eq. (svd), applied through the
 * projectors P_L = R_B V s^-1/2 and P_R = s^-1/2 U^T R_A of SI section B.
 *
 * How the reduced factors are formed (the paper uses Householder QR; the
 * projectors depend on R only through R^T R = A^T A, SI B):
 *   - bonds of size D <= 64 and gradient plans: R from a float64 Gram matrix
 *     A^T A by pivoted Cholesky.  Pivots below 1e-15 of the first one end the
 *     factorisation, so directions of A whose singular value is below about
 *     3e-8 of A's largest are dropped (the Gram squares the spectrum); the
 *     core SVD is a one-sided Jacobi in float64.
 *   - forward plans with D > 64: the leading chi' singular triplets of the
 *     core come from a Krylov method on the same Gram operators (or on A B
 *     directly); eigenvalues of the squared core below 1e-13 of the largest
 *     count as zero, i.e. kept singular values below about 3.2e-7 sigma_1
 *     give zero projector columns.
 * Core singular values at or below 1e-13 sigma_1 always count as zero.
 *
 * Inputs follow the paper's statement of the problem (Algorithm 1, "Input:
 * tensor network T, ordered contraction tree, maximum bond dimension chi,
 * tree gauge distance r, flag compress_late").  All calls return tn_status;
 * on failure tn_last_error(ctx) describes the cause.  A context is used by
 * one host thread at a time; distinct contexts are independent.
 *
 * Memory: every pointer argument marked "host" is read (or written) only
 * during the call and stays owned by the caller.  The context owns its
 * device memory (one arena planned by tn_set_tree) unless a workspace is
 * supplied with tn_set_workspace, which then stays owned by the caller and
 * must outlive every plan made while it was set.
 */
#ifndef TN_H
#define TN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TN_OK = 0,
    TN_EINVAL = 1,    /* invalid graph, tree, option or argument */
    TN_ESTATE = 2,    /* call out of order (e.g. contract before set_tree) */
    TN_ENOMEM = 3,    /* plan exceeds the device budget / allocation failed */
    TN_EDEVICE = 4,   /* HIP runtime error */
    TN_ENUMERIC = 5,  /* non-finite value, or a Jacobi SVD that did not converge */
    TN_ZERO = 6       /* the network evaluates to exactly zero */
} tn_status;

typedef enum {
    TN_FP64 = 0,      /* tensors, contractions and re-absorptions in float64 */
    TN_FP32 = 1,      /* tensors and contractions in float32 on MFMA; Gram, core SVD,
                         projectors and scale exponents in float64 */
    TN_BF16 = 2       /* tensors and projectors stored in bfloat16, contractions on bf16 MFMA with
                         float32 accumulation (rounded to bfloat16 on store); Gram, core SVD and
                         scale exponents in float64 */
} tn_precision;

typedef struct {
    int32_t chi;                 /* maximum bond dimension (>= 1) */
    double cutoff;               /* relative singular-value cutoff: sigma_i < cutoff*sigma_1
                                    contributes a zero column/row (shapes stay static); 0 = none */
    int32_t compress_late;       /* 0: early compression, every bond of a new tensor larger than chi
                                    right after its contraction; 1: late compression (section II.D,
                                    Algorithm 1 with compress_late), before contracting i and j every
                                    other bond of i, then of j, larger than chi; ascending neighbour
                                    id in both */
    int32_t gauge_r;             /* tree-gauge distance r >= 0 (section II.C, SI A).  0: a compression
                                    uses the two bond-adjacent tensors alone.  r >= 1: their R factors
                                    come from the bond placed in the tree gauge of the r-local spanning
                                    tree of live intermediate tensors around it (input tensors are not
                                    spanned; candidates by distance, then larger bond, then smaller ids);
                                    the projectors act on the two tensors themselves.  Computed as
                                    environment metrics (Grams with the children's metrics applied)
                                    on the Gram + core path for every bond size.  Not with grad. */
    int32_t precision;           /* tn_precision */
    int32_t jacobi_max_sweeps;   /* cap on one-sided Jacobi sweeps per core; 0 = default (40) */
    int64_t device_budget_bytes; /* refuse plans whose device arena exceeds this; 0 = no limit */
    int32_t keep_intermediates;  /* 1: never reuse arena memory, so tn_read_tensor can read every
                                    intermediate after an evaluation (element-wise checks) */
    int32_t grad;                /* 1: also plan the reverse pass (tn_grad).  Every compression
                                    takes the Gram + full-spectrum Jacobi core (the adjoint needs
                                    all singular triplets of the core).  What the reverse pass reads
                                    of the forward pass (tensors, core workspaces, projectors) stays
                                    resident unless checkpoint_segments recomputes it; reverse-pass
                                    buffers live from their first to their last reverse level */
    int32_t plain;               /* 1: the plain form: every step (contraction, Gram, core,
                                    re-absorption, scale) is its own kernel launch, issued in order
                                    on the context's stream on every evaluation, with no grouping,
                                    no concurrent streams and no graph replay; same kernels and same
                                    results.  The baseline the grouped, captured form is measured
                                    against.  Needs grad = 0; not accepted by tn_batch_create */
    int32_t checkpoint_segments; /* grad only: recomputation of forward intermediates.  0 or 1: none
                                    (everything the reverse pass reads stays resident).  S >= 2: the
                                    forward levels are cut into S consecutive segments of about
                                    equal produced bytes; only forward buffers live across a
                                    segment boundary (the checkpoints) are kept to the end; the
                                    reverse pass takes the segments last to first and re-runs the
                                    forward launches of each segment but the last before its
                                    reverse levels (a second tn_grad with no evaluation in between
                                    first re-runs the whole forward pass: the re-runs write over
                                    checkpoints).  Same gradient bit for bit (the forward kernels
                                    are deterministic), smaller arena, up to one more forward pass
                                    of work per tn_grad.  -1: the S in
                                    {1,2,3,4,6,8,12,16,24,32} of smallest arena.  tn_batch_grad does
                                    not take contexts planned with S >= 2 (tn_grad per context) */
    int32_t r_factor;            /* tn_r_factor: how the R-factors of a bond's tall sides (more rows
                                    than D) are formed when D <= 64.  TN_RFACTOR_GRAM (0): float64
                                    Gram on MFMA + pivoted Cholesky (pivots below 1e-15 of the first
                                    dropped, i.e. directions under ~3e-8 of the largest).
                                    TN_RFACTOR_TSQR (1): batched Householder TSQR in float64 (row
                                    blocks of 16384 / D rows in LDS, then passes over the stacked
                                    R's), R^T R = the Gram without forming it.  Larger D take the
                                    Gram / Krylov routes either way.  TSQR: grad must be 0; not
                                    accepted by tn_batch_create */
} tn_tree_opts;

typedef enum { TN_RFACTOR_GRAM = 0, TN_RFACTOR_TSQR = 1 } tn_r_factor;

typedef struct tn_ctx tn_ctx;

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t the
 * library enqueues all work on (e.g. torch's current stream); NULL makes the
 * library create its own stream of default priority. */
tn_status tn_create(int device, void* hip_stream, tn_ctx** out);
void tn_destroy(tn_ctx* ctx);
/* Text of the last error on ctx (valid until the next call on ctx). */
const char* tn_last_error(const tn_ctx* ctx);

/* Device workspace for the arena of later tn_set_tree calls (e.g. memory
 * owned by torch: size it with tn_plan_info's arena_bytes of a first plan).
 * dev_ptr: device memory of `bytes` bytes, 256-byte aligned, caller owned; it
 * must stay valid while a plan made with it is in use.  NULL switches back
 * to library allocation.  A plan whose arena exceeds `bytes` fails with
 * TN_ENOMEM before any launch.  The current plan, if any, is unaffected.
 * Errors: TN_EINVAL for a misaligned pointer or zero bytes. */
tn_status tn_set_workspace(tn_ctx* ctx, void* dev_ptr, size_t bytes);

/* Tensor network (section I, Eq. (tncontract); data structure of
 * Fig. "tensor primitives"): n_tensors vertices and n_edges edges
 * (edge_u[e] < edge_v[e], both < n_tensors, edge_dim[e] >= 1; several edges
 * may join the same two tensors).  Tensor v is dense float64, row-major,
 * with one axis per incident edge in ascending edge id; its entries are
 * data[offsets[v] .. offsets[v+1]).  All arrays are host memory.  Replaces
 * any previous graph and tree. */
tn_status tn_load_graph(tn_ctx* ctx, int32_t n_tensors, int32_t n_edges,
                        const int32_t* edge_u, const int32_t* edge_v, const int32_t* edge_dim,
                        const int64_t* offsets, const double* data);

/* New tensor values, same graph and layout (host float64).  Keeps the plan. */
tn_status tn_update_values(tn_ctx* ctx, const double* data);
/* Same, from device memory (float64, same layout); enqueued on the ctx stream. */
tn_status tn_update_values_device(tn_ctx* ctx, const void* dev_data);

/* Ordered contraction tree (section II.A, Algorithm 1 input): n_steps must be
 * n_tensors - 1; step t contracts the live tensors pair_i[t] and pair_j[t]
 * into a new tensor with id n_tensors + t.  Compressions follow from the
 * order (section II.G): after each contraction every bond of the new tensor
 * larger than chi is compressed, neighbours in ascending id.  Host arrays.
 * Plans the device schedule and arena (allocates device memory). */
tn_status tn_set_tree(tn_ctx* ctx, int32_t n_steps, const int32_t* pair_i, const int32_t* pair_j,
                      const tn_tree_opts* opts);

/* Plan summary: device arena bytes, algorithmic forward flops and bytes
 * (SI section D cost model, 2 flops per multiply-add), number of kernel
 * steps.  Any pointer may be NULL. */
tn_status tn_plan_info(const tn_ctx* ctx, int64_t* arena_bytes, double* fwd_flops, double* fwd_bytes,
                       int32_t* n_steps);

/* Evaluate the compressed contraction.  Z = mantissa * 10^log10_exponent
 * with 1 <= |mantissa| < 10 (host outputs).  Synchronises the ctx stream.
 * TN_ZERO: Z == 0 (mantissa 0, exponent -inf). */
tn_status tn_contract_compressed(tn_ctx* ctx, double* mantissa, double* log10_exponent);

/* The last evaluation as sign (+1, -1 or 0) and natural log of |Z|. */
tn_status tn_result(const tn_ctx* ctx, double* sign, double* ln_abs_z);

/* Enqueue an evaluation without synchronising (for timing and batching);
 * tn_fetch synchronises the ctx stream and, when it returns TN_OK or
 * TN_ZERO, makes it the last evaluation (a TN_ENUMERIC evaluation leaves
 * none: tn_result and tn_grad then return TN_ESTATE).
 * The first evaluation after tn_set_tree (or after a change of the
 * tn_profile mask) captures the schedule into a hipGraph on the ctx stream;
 * later ones replay it, so the input values may change between evaluations
 * (tn_update_values*) but not the addresses the plan holds. */
tn_status tn_enqueue(tn_ctx* ctx);
tn_status tn_fetch(tn_ctx* ctx);

/* Per-compression diagnostics of the last evaluation, in schedule order:
 * discarded[c] = sum of discarded sigma^2 / sum sigma^2, tie[c] = 1 when the
 * last kept and first discarded singular values differ by <= 1e-12 sigma_1
 * (several truncations are then equally correct), sweeps[c] = Jacobi sweeps.
 * Arrays hold `cap` entries; *n_out receives the number of compressions. */
tn_status tn_compress_stats(const tn_ctx* ctx, int32_t cap, double* discarded, int32_t* tie,
                            int32_t* sweeps, int32_t* n_out);

/* Kernel kinds for tn_profile: grouped contraction / re-absorption GEMMs, Gram
 * GEMMs, explicit-factor copies, compression cores (LDS-resident, D <= 64, and
 * global-memory), scale finalisation, large-bond Lanczos compressions. */
typedef enum {
    TN_KERNEL_GEMM = 0,
    TN_KERNEL_GRAM = 1,
    TN_KERNEL_COPY = 2,
    TN_KERNEL_CORE_LDS = 3,
    TN_KERNEL_CORE_GLOBAL = 4,
    TN_KERNEL_SCALE = 5,
    TN_KERNEL_LANCZOS = 6,
    TN_KERNEL_BWD_GEMM = 7,      /* reverse pass: adjoint GEMMs and split-K reductions */
    TN_KERNEL_BWD_CORE = 8,      /* reverse pass: per-compression core adjoint */
    TN_KERNEL_RECOMPUTE = 9      /* reverse pass: re-run of one forward segment (all its launches,
                                    timed as one interval; flops and bytes are the segment's) */
} tn_kernel_kind;

/* Time every launch of the kinds in `kind_mask` (bit k = tn_kernel_kind k)
 * during later evaluations, and reset the totals.  Forward launches are timed
 * by device wall-clock stamps (100 MHz) written on the launch's own stream just
 * before and after it (so the duration includes one dispatch gap); reverse-pass
 * launches by HIP events.  Totals are read at tn_fetch: replays enqueued
 * without a fetch in between re-write the same stamps, so fetch after each
 * evaluation for a per-evaluation total.  0 switches timing off. */
tn_status tn_profile(tn_ctx* ctx, uint32_t kind_mask);
/* Totals since tn_profile for one kind: summed launch durations (ms, measured
 * at tn_fetch / tn_contract_compressed), number of launches, and the
 * algorithmic flops and bytes of the steps those launches ran. */
tn_status tn_profile_read(const tn_ctx* ctx, int32_t kind, double* ms, int64_t* launches, double* flops,
                          double* bytes);

/* Tensor `index` of the last evaluation, normalised (divided by its largest
 * absolute entry), as float64 in its axis order.  Indices count tensors in
 * creation order: inputs 0..n-1, then each contraction's result, then the two
 * re-absorbed tensors of each compression.  Needs keep_intermediates = 1 for
 * anything but inputs and the final scalar.  Writes up to `cap` entries to
 * host `out`; *n receives the tensor's size. */
tn_status tn_read_tensor(const tn_ctx* ctx, int32_t index, double* out, int64_t cap, int64_t* n);

/* The projectors of compression `comp` (creation order, as in tn_compress_stats) of the last
 * evaluation (section II.C, Eq. (svd); SI B): P_L (D x chi', row-major) into host `p_left` and
 * P_R (chi' x D, row-major) into host `p_right`, as float64, `cap` >= D * chi' entries each;
 * either may be null.  They are the ones the re-absorption applied (a' = A P_L, b' = P_R B), in
 * the storage precision, computed from the normalised tensors: only the product P_L P_R is
 * scale-free, which is what the explicit projector network T_P of SI B inserts on the bond.
 * The bond: `bond_edges` receives up to `edge_cap` edge ids it bundles, in P_L's row order
 * (slowest first; input edges 0..n_edges-1, then one new edge per compression in creation
 * order); `info` (6 int32) receives D, chi', the new edge's id, the tree nodes a (P_L's side)
 * and b (inputs 0..n-1, step t's result n + t) and the number of bundled edges.  The bond
 * description needs only a tree (no evaluation); the projectors need an evaluation of a tree set
 * with keep_intermediates = 1 (else TN_ESTATE: their memory may have been reused). */
tn_status tn_read_projectors(const tn_ctx* ctx, int32_t comp, double* p_left, double* p_right, int64_t cap,
                             int32_t* bond_edges, int32_t edge_cap, int32_t* info);

/* Reverse pass (no counterpart in the paper, which computes no gradients):
 * d ln|Z| / d data for the last evaluated tree, where data are the input
 * tensor entries of tn_load_graph / tn_update_values.  Written to host
 * float64 `dlnz_ddata` in the same layout as data (n_input entries, caller
 * owned).  Method: reverse mode over the same op order with the scale factors
 * held constant (exact: the result is homogeneous of degree 1 in every
 * tensor); each contraction's adjoint is two GEMMs; each compression's is the
 * adjoint of the rank-chi' truncated SVD of A_mat B_mat (section II.C, Eq.
 * (svd)), computed in the core's singular coordinates from all its singular
 * triplets.  Core singular values at or below 1e-13 sigma_1 count as zero, so
 * this is the derivative of the rank-preserving truncation: exact along
 * perturbations that keep every core's rank (Ising couplings, rescalings).
 * Needs tn_set_tree with opts.grad = 1 and a successful evaluation
 * (TN_ESTATE otherwise); TN_ZERO if Z = 0 (no gradient of ln|Z|). */
tn_status tn_grad(tn_ctx* ctx, double* dlnz_ddata);

/* As tn_grad, writing float64 device memory `dlnz_ddata_dev` (n_input
 * entries, caller owned) on the context's stream without synchronising. */
tn_status tn_grad_device(tn_ctx* ctx, void* dlnz_ddata_dev);

/* Block the host until all work enqueued on the context's stream has finished. */
tn_status tn_sync(tn_ctx* ctx);

/* Ising model of SI F.1 on the loaded graph (every edge of dimension 2):
 * writes the input tensors for couplings J (device float64, one per edge,
 * beta*J_e != 0) into the context, as tn_update_values would.  Each edge's
 * Boltzmann matrix exp(beta J s s') is split as W_lo W_hi with
 * W = H diag(sqrt(cosh beta J), +-sqrt|sinh beta J|) H / sqrt 2 (the sign of
 * sinh on the higher vertex id), and T_v = sum_x prod over v's edges of W[x, :]
 * (axes in ascending edge id).  Runs on the context's stream. */
tn_status tn_ising_values_device(tn_ctx* ctx, double beta, const void* J_dev);

/* Chain rule of the map above: d ln|Z| / d J (device float64, n_edges) from
 * d ln|Z| / d data (device float64, e.g. tn_grad_device's output). */
tn_status tn_ising_coupling_grad_device(tn_ctx* ctx, double beta, const void* J_dev, const void* dlnz_ddata_dev,
                                        void* dlnz_dJ_dev);

/* Backward-plan totals for opts.grad = 1: algorithmic flops and bytes of the
 * reverse pass, its number of levels. */
tn_status tn_grad_info(const tn_ctx* ctx, double* bwd_flops, double* bwd_bytes, int32_t* n_levels);

/* Recomputation totals for opts.grad = 1: the number of segments S (1 = no
 * recomputation), the forward flops re-run by one tn_grad right after an
 * evaluation (every segment but the last that has reverse steps), and the bytes
 * of forward buffers kept across segment boundaries.  TN_ESTATE without a
 * grad plan. */
tn_status tn_grad_checkpoint_info(const tn_ctx* ctx, int32_t* segments, double* recompute_flops,
                                  int64_t* checkpoint_bytes);

/* ---- Batches: independent instances evaluated together ------------------
 * Steps of different instances never depend on each other, so the schedules
 * of several planned contexts are merged level by level (level L of every
 * instance in the same grouped launches) and the whole merged schedule is
 * captured once in a hipGraph; each tn_batch_contract replays it.  Instances
 * may differ in graph, tree, chi and size; they must share the device and the
 * precision.  The contexts stay owned by the caller and must outlive the
 * batch; new values are given with tn_update_values / tn_update_values_device
 * / tn_ising_values_device on the contexts (no recapture).  A batch keeps
 * its own stream, scale and statistics arrays (device memory it owns). */
typedef struct tn_batch tn_batch;

/* Merge and capture.  TN_ESTATE if a context has no plan; TN_EINVAL for
 * mixed devices or precisions or a repeated context. */
tn_status tn_batch_create(int32_t n, tn_ctx* const* ctxs, tn_batch** out);
void tn_batch_destroy(tn_batch* batch);
const char* tn_batch_last_error(const tn_batch* batch);

/* Replay: evaluates every instance; writes n mantissas and log10 exponents
 * (host arrays, may be NULL) and leaves each context as after its own
 * tn_contract_compressed (tn_result, tn_compress_stats and tn_grad work on it).
 * Instances with Z = 0 get mantissa 0 and exponent -inf; the first other
 * failure is returned. */
tn_status tn_batch_contract(tn_batch* batch, double* mantissas, double* log10_exponents);

/* Reverse pass of every instance after tn_batch_contract, into device float64
 * buffers dlnz_ddata_dev[i] (one per instance, layout of its data).  Needs
 * every context planned with opts.grad.  The reverse schedule is captured on
 * the first call and recaptured when the output buffers change. */
tn_status tn_batch_grad(tn_batch* batch, void* const* dlnz_ddata_dev);

/* ---- One bond compression on its own ------------------------------------
 * The compression primitive of section II.C, Eq. (svd) (Fig. "tensor
 * primitives"): two tensors sharing a bond, given as their matricisations
 * A (m_a x D, row-major) and B (D x m_b, row-major), device float64.  Writes
 * a' = A P_L (m_a x chi', row-major) and b' = P_R B (chi' x m_b, row-major)
 * into device float64 buffers a_out (>= m_a * chi' entries) and b_out
 * (>= chi' * m_b), with P_L = R_B V s^-1/2 and P_R = s^-1/2 U^T R_A (SI B), so
 * that a' b' is the rank-chi' truncated SVD of A B; chi' = min(chi, k_A, k_B),
 * k = min(rows, D), goes to *chi_out (host, may be NULL).  `cutoff` zeroes kept
 * triplets with sigma_i < cutoff * sigma_1, as in tn_tree_opts.  The reduced
 * factors come from float64 Grams (or the matrix itself when it has <= D
 * rows) by pivoted Cholesky; the core SVD is a float64 Jacobi.
 * Limits: 1 <= D <= 64, m_a, m_b >= 1, m_a * D and m_b * D below 2^31.
 * Work memory is allocated on the device for the call and freed before it
 * returns; the call runs on ctx's stream and synchronises it.  All buffers
 * stay owned by the caller.  Errors: TN_EINVAL (shapes, null pointers),
 * TN_ENOMEM (work memory), TN_ENUMERIC (Jacobi not converged in 40 sweeps),
 * TN_EDEVICE. */
tn_status tn_compress_pair(tn_ctx* ctx, const double* a_dev, const double* b_dev, int64_t m_a, int32_t D,
                           int64_t m_b, int32_t chi, double cutoff, double* a_out, double* b_out,
                           int32_t* chi_out);

/* Allocation-free variant of tn_compress_pair, for callers that cannot allocate
 * device memory (code that must not call hipMalloc, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, results (bitwise: the
 * same kernels with the same launch shapes) and errors, but the work memory is
 * a fixed 32 MiB device array per GPU, held by the library until the process
 * ends; the call allocates and frees nothing.  32 MiB holds, at D = 64,
 * about 260000 rows per side (float64 Gram partials of 512-row splits; more
 * for smaller D); larger inputs fail with TN_EINVAL before any launch.  All calls on
 * one GPU share that array, and nothing in it needs to start at zero (every
 * word a call reads it has written first), but calls that overlap in time on
 * one GPU (from several threads or contexts) race on it: serialise them.  Runs
 * on ctx's stream and synchronises it before returning. */
tn_status tn_compress_pair_static(tn_ctx* ctx, const double* a_dev, const double* b_dev, int64_t m_a, int32_t D,
                                  int64_t m_b, int32_t chi, double cutoff, double* a_out, double* b_out,
                                  int32_t* chi_out);

/* ---- Tile shapes of the tensor GEMMs (autotuning) ------------------------
 * A contraction or re-absorption GEMM whose short side (M or N) is at most 32
 * while the other exceeds 64 takes the tile shape that a process-wide table
 * holds for its class (other GEMMs take 64 x 64 MFMA tiles).  Class index:
 *   ((((prec * 2 + wide) * 2 + short32) * 3 + kclass) * 2 + long_unit
 * prec: tn_precision; wide: 1 if M is the short side; short32: 1 if the short
 * side is 17..32; kclass: 0 for K <= 4, 1 for K <= 64, 2 above; long_unit: 1 if
 * the long operand's long axis has unit stride.  Entries are tn_gemm_tile
 * values.  The table is read when tn_set_tree plans; plans keep their tiles.
 * Every tile computes the same product (only the summation order differs). */
#define TN_GEMM_CLASSES 72
typedef enum {
    TN_TILE_64x64 = 0,       /* MFMA, 64 x 64 */
    TN_TILE_256x16 = 1,      /* MFMA, tall (short side <= 16) */
    TN_TILE_16x256 = 2,      /* MFMA, wide (short side <= 16) */
    TN_TILE_128x32 = 3,      /* MFMA, tall */
    TN_TILE_32x128 = 4,      /* MFMA, wide */
    TN_TILE_SKINNY_TALL16 = 5,  /* vector FMA, one row of C per thread (N <= 16, K <= 64) */
    TN_TILE_SKINNY_TALL32 = 6,  /* the same, N <= 32 */
    TN_TILE_SKINNY_WIDE16 = 7,  /* vector FMA, one column of C per thread (M <= 16, K <= 64) */
    TN_TILE_SKINNY_WIDE32 = 8   /* the same, M <= 32 */
} tn_gemm_tile;

/* Copy the current table (TN_GEMM_CLASSES int32 entries, host memory). */
tn_status tn_gemm_tiles_get(int32_t* table);
/* Install a table (host memory), or the built-in defaults when table is NULL.
 * TN_EINVAL, leaving the table unchanged, if an entry is not a tile for its
 * class (a tall tile for a wide class, a 16-wide tile for a 32 side, a skinny
 * tile with K > 64).  Not synchronised with concurrent tn_set_tree calls in
 * other threads beyond each call seeing a whole table. */
tn_status tn_gemm_tiles_set(const int32_t* table);
/* Measure one class on device `device`: `copies` GEMMs of the class's
 * representative shape (long side 65536, or 16384 for K > 64; short side 16 or
 * 32; K = 2, 32 or 256) in one grouped launch, 10 timed launches after 2 warm-up
 * ones.  us[t] receives the microseconds per launch of tile t (TN_TILE_*), or -1
 * where the tile does not apply to the class; `us` holds 9 entries.  Allocates
 * and frees its own device memory (up to about 1 GB at copies = 8).  The
 * autotuner (paper_2206_07044_amd/autotune.py) installs the fastest tile of
 * each class with tn_gemm_tiles_set.  TN_EINVAL for a bad class or copies
 * outside 1..64; TN_EDEVICE on a HIP error. */
tn_status tn_gemm_tune(int device, int32_t klass, int32_t copies, double* us);

/* Host-only expansion of Algorithm 1 on shapes (no device use): writes up
 * to `cap` ops as 8 int64 each: (kind, a, b, out, m, n, k, new_dim) with
 * kind 0 = contract: (i, j, new id, free size of i, shared size, free size of
 * j, 0); kind 1 = compress: (tensor, neighbour, new edge id, rows of A_mat,
 * D_AB, columns of B_mat, chi').  *n_ops receives the total count. */
tn_status tn_plan_describe(int32_t n_tensors, int32_t n_edges, const int32_t* edge_u, const int32_t* edge_v,
                           const int32_t* edge_dim, int32_t n_steps, const int32_t* pair_i,
                           const int32_t* pair_j, const tn_tree_opts* opts, int64_t cap, int64_t* ops,
                           int64_t* n_ops);

#ifdef __cplusplus
}
#endif

#endif /* TN_H */
