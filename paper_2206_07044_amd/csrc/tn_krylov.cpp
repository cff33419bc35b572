// Block-Krylov truncated SVD for compressions of a large bond D whose side X has at most D rows
// (section II.C, Eq. (svd), for the bonds that merge two chi-bonds, D ~ chi^2).
//
// With F_X the explicit factor of X (n x D) and Y the matricisation of the other side (m_Y x D,
// read in place through its View), the squared singular values of the core are the eigenvalues
// of S = F_X (Y^T Y) F_X^T (n x n).  S is never formed: a block of vectors Q (n x b) is mapped
// to S Q = F_X (Y^T (Y (F_X^T Q))), two passes over Y as many-workgroup GEMMs.  A block Lanczos
// basis Q of k = s b columns (full reorthogonalisation: two classical Gram-Schmidt passes, then
// CholeskyQR2 of the block) spans the leading eigenvectors; the Rayleigh quotient H = Q^T S Q
// (k x k) goes to the compression core kernel as a Gram matrix against an identity factor, which
// returns its leading eigenvectors V and sigma = sqrt(eig H) as P_L^core = V s^-1/2.  Then
//   P_X = F_X^T Q V s^-1/2            (D x chi'),
//   P_Y = (Y^T Y) P_X s^-1            (D x chi', two more passes over Y),
// and P_L = P_X, P_R = P_Y^T when X is the B side (X = B_mat^T), or P_R = P_X^T, P_L = P_Y when
// X is the A side: A P_L P_R B is then the rank-chi' truncation of A B within the basis.  When n
// is at most the basis size the basis is all of R^n (Q = I) and the result is exact.
#include "tn_krylov.hpp"

#include <algorithm>
#include <cstring>
#include <functional>

#include "tn_kernels.hpp"

namespace tn {

namespace {

std::string dense(int64_t rows, int64_t rs, int64_t cols, int64_t cs, View* v) {
    ViewSpec s;
    s.row_dims = {(int32_t)rows};
    s.row_strides = {rs};
    s.col_dims = {(int32_t)cols};
    s.col_strides = {cs};
    return make_view(s, v);
}

// the passes over Y: Y in the tensor dtype against float64 vectors, formed and kept in float64 (a
// float32 product of the squared operator would lose the small singular values)
int ypass_key(int prec) { return prec == 0 ? GEMM_F64 : prec == 1 ? GEMM_F32_X_F64 : GEMM_BF16_X_F64; }

// An operand: base pointer and dense (rows x cols) layout with element strides, or a View.
struct Opnd {
    const void* p = nullptr;
    int64_t rows = 0, rs = 0, cols = 0, cs = 0;
    const View* view = nullptr;
};
Opnd mat(const void* p, int64_t rows, int64_t rs, int64_t cols, int64_t cs) {
    Opnd o;
    o.p = p;
    o.rows = rows;
    o.rs = rs;
    o.cols = cols;
    o.cs = cs;
    return o;
}
Opnd viewed(const void* p, const View* v) {
    Opnd o;
    o.p = p;
    o.view = v;
    return o;
}

struct Chain {
    const KrylovSink& out;
    std::string err;
    int njobs;

    void fail(const std::string& e) {
        if (err.empty()) err = e;
    }
    void view_of(const Opnd& o, View* v) {
        if (o.view) *v = *o.view;
        else fail(dense(o.rows, o.rs, o.cols, o.cs, v));
    }

    // C = f A B for every job (f: the inverse scales); GEMM_GRAM writes dense split partials at
    // C, GEMM_ADJ writes (or accumulates) through C's layout.
    template <typename F>
    void gemm(int key, int mode, F per_job) {
        KOp op;
        op.kind = KO_GEMM;
        op.key = key;
        op.begin = (int64_t)out.gemm->size();
        op.count = njobs;
        int64_t tiles = 0;
        for (int j = 0; j < njobs; ++j) {
            Opnd A, B, Cm;
            void* C = nullptr;
            int64_t M = 0, N = 0, K = 0;
            int splits = 1, sa = -1, sb = -1, acc = 0;
            per_job(j, A, B, C, Cm, M, N, K, splits, sa, sb, acc);
            GemmDesc g;
            std::memset(&g, 0, sizeof(g));
            view_of(A, &g.va);
            view_of(B, &g.vb);
            if (mode == GEMM_ADJ) view_of(Cm, &g.vc);
            g.A = A.p;
            g.B = B.p;
            g.C = C;
            g.M = (int32_t)M;
            g.N = (int32_t)N;
            g.K = (int32_t)K;
            g.mode = mode;
            g.tiles_m = (int32_t)((M + 63) / 64);
            g.tiles_n = (int32_t)((N + 63) / 64);
            int64_t kps = (K + splits - 1) / splits;
            kps = (kps + 15) / 16 * 16;
            g.splits = (int32_t)((K + kps - 1) / kps);
            g.k_per_split = (int32_t)kps;
            g.scale_a = sa;
            g.scale_b = sb;
            g.accumulate = acc;
            g.tile_begin = tiles;
            tiles += (int64_t)g.tiles_m * g.tiles_n * g.splits;
            out.gemm->push_back(g);
        }
        op.work = tiles;
        out.ops->push_back(op);
    }

    // sum the split partials of a GEMM_GRAM (dense M x N) in place into the first
    template <typename F>
    void reduce(F per_job) {
        KOp op;
        op.kind = KO_REDUCE;
        op.begin = (int64_t)out.reduce->size();
        op.count = njobs;
        int64_t elems = 0;
        for (int j = 0; j < njobs; ++j) {
            double* part = nullptr;
            int64_t M = 0, N = 0;
            int splits = 1;
            per_job(j, part, M, N, splits);
            ReduceDesc r;
            std::memset(&r, 0, sizeof(r));
            fail(dense(M, N, N, 1, &r.vc));
            r.part = part;
            r.out = part;
            r.M = (int32_t)M;
            r.N = (int32_t)N;
            r.splits = splits;
            r.scale_a = r.scale_b = -1;
            r.elem_begin = elems;
            elems += M * N;
            out.reduce->push_back(r);
        }
        op.work = elems;
        out.ops->push_back(op);
    }

    template <typename F>
    void small(int key, F per_job) {
        KOp op;
        op.kind = KO_SMALL;
        op.key = key;
        op.begin = (int64_t)out.small->size();
        op.count = njobs;
        int64_t elems = 0;
        for (int j = 0; j < njobs; ++j) {
            SmallDesc d;
            std::memset(&d, 0, sizeof(d));
            per_job(j, d);
            d.elem_begin = elems;
            elems += (int64_t)d.rows * d.cols;
            out.small->push_back(d);
        }
        op.work = elems;
        out.ops->push_back(op);
    }

    template <typename F>
    void chol(F per_job) {
        KOp op;
        op.kind = KO_CHOL;
        op.begin = (int64_t)out.chol->size();
        op.count = njobs;
        for (int j = 0; j < njobs; ++j) {
            CholInvDesc d;
            std::memset(&d, 0, sizeof(d));
            per_job(j, d);
            out.chol->push_back(d);
        }
        out.ops->push_back(op);
    }
};

SmallDesc small_desc(int op, const double* src, int64_t src_ld, void* dst, int64_t rows, int64_t cols, int64_t dst_ld,
                     int transpose = 0) {
    SmallDesc d;
    std::memset(&d, 0, sizeof(d));
    d.op = op;
    d.src = src;
    d.src_ld = (int32_t)src_ld;
    d.dst = dst;
    d.rows = (int32_t)rows;
    d.cols = (int32_t)cols;
    d.dst_ld = (int32_t)dst_ld;
    d.transpose = transpose;
    return d;
}

}  // namespace

std::string krylov_chain(const KrylovShape& sh, int prec, const std::vector<KrylovJob>& jobs, const KrylovSink& out) {
    const int64_t n = sh.n, D = sh.D, my = sh.my, nw = sh.nw, b = sh.b, k = sh.k;
    const int s = sh.s, full = sh.full;
    const int64_t w = prec == 0 ? 8 : prec == 1 ? 4 : 2;
    const KrylovLayout L = krylov_layout(n, D, my, nw, b, k, full, sh.splits, sh.splits2, w);
    Chain ch{out, "", (int)jobs.size()};
    auto at = [&](int j, int64_t off) -> double* { return (double*)(jobs[j].ws + off); };
    auto raw = [&](int j, int64_t off) -> char* { return jobs[j].ws + off; };
    const int ykey = ypass_key(prec);

    // W (n x b at src) -> orthonormal columns at dst (ld dst_ld): CholeskyQR2 through tmp
    auto cholqr2 = [&](auto src_of, auto tmp_of, auto dst_of, int64_t dst_ld) {
        for (int pass = 0; pass < 2; ++pass) {
            ch.gemm(GEMM_F64, GEMM_GRAM, [&](int j, Opnd& A, Opnd& B, void*& C, Opnd&, int64_t& M, int64_t& N,
                                             int64_t& K, int&, int&, int&, int&) {
                const double* W = pass == 0 ? src_of(j) : tmp_of(j);
                A = mat(W, b, 1, n, b);
                B = mat(W, n, b, b, 1);
                C = at(j, L.g);
                M = b;
                N = b;
                K = n;
            });
            ch.chol([&](int j, CholInvDesc& d) {
                d.g = at(j, L.g);
                d.m = at(j, L.m);
                d.b = (int32_t)b;
            });
            ch.gemm(GEMM_F64, GEMM_ADJ, [&](int j, Opnd& A, Opnd& B, void*& C, Opnd& Cm, int64_t& M, int64_t& N,
                                            int64_t& K, int&, int&, int&, int&) {
                const double* W = pass == 0 ? src_of(j) : tmp_of(j);
                double* dst = pass == 0 ? tmp_of(j) : dst_of(j);
                A = mat(W, n, b, b, 1);
                B = mat(at(j, L.m), b, b, b, 1);
                C = dst;
                Cm = mat(dst, n, pass == 0 ? b : dst_ld, b, 1);
                M = n;
                N = b;
                K = b;
            });
        }
    };

    if (!full) {
        // start block: seeded uniform entries, orthonormalised
        ch.small(0, [&](int j, SmallDesc& d) {
            d = small_desc(SM_RANDOM, nullptr, 0, at(j, L.wo), n, b, b);
            d.seed = (uint32_t)jobs[j].stat + 1u;
        });
        cholqr2([&](int j) { return at(j, L.wo); }, [&](int j) { return at(j, L.wx); },
                [&](int j) { return at(j, L.q); }, k);
    }
    for (int blk = 0; blk < s; ++blk) {
        const int64_t c0 = (int64_t)blk * b;
        const int64_t bj = full ? std::min<int64_t>(b, n - c0) : b;
        // T = F_X^T Q_blk (D x bj) in the tensor dtype: for the full basis Q_blk is a block of the
        // identity, so T is a transposed block of F_X
        std::function<Opnd(int)> tsrc;
        if (full) {
            tsrc = [&, c0, bj](int j) { return mat(jobs[j].fx + c0 * D, D, 1, bj, D); };
        } else {
            ch.gemm(GEMM_F64, GEMM_GRAM, [&, c0](int j, Opnd& A, Opnd& B, void*& C, Opnd&, int64_t& M, int64_t& N,
                                                 int64_t& K, int&, int&, int&, int&) {
                A = mat(jobs[j].fx, D, 1, n, D);
                B = mat(at(j, L.q) + c0, n, k, b, 1);
                C = at(j, L.t1);
                M = D;
                N = b;
                K = n;
            });
            tsrc = [&](int j) { return mat(at(j, L.t1), D, b, b, 1); };
        }
        // U = Y T / s_Y  (m_Y x bj, float64)
        ch.gemm(ykey, GEMM_ADJ, [&, bj](int j, Opnd& A, Opnd& B, void*& C, Opnd& Cm, int64_t& M, int64_t& N,
                                        int64_t& K, int&, int& sa, int&, int&) {
            A = viewed(jobs[j].y, &jobs[j].vy);
            B = tsrc(j);
            C = raw(j, L.u);
            Cm = mat(C, my, bj, bj, 1);
            M = my;
            N = bj;
            K = D;
            sa = jobs[j].y_scale;
        });
        // T2 = Y^T U / s_Y  (D x bj, float64 split partials, summed in place)
        ch.gemm(ykey, GEMM_GRAM, [&, bj](int j, Opnd& A, Opnd& B, void*& C, Opnd&, int64_t& M, int64_t& N,
                                         int64_t& K, int& splits, int& sa, int&, int&) {
            A = viewed(jobs[j].y, &jobs[j].vyt);
            B = mat(raw(j, L.u), my, bj, bj, 1);
            C = at(j, L.t2p);
            M = D;
            N = bj;
            K = my;
            splits = sh.splits;
            sa = jobs[j].y_scale;
        });
        ch.reduce([&, bj](int j, double*& part, int64_t& M, int64_t& N, int& splits) {
            part = at(j, L.t2p);
            M = D;
            N = bj;
            const GemmDesc& g = (*out.gemm)[out.gemm->size() - jobs.size() + j];
            splits = g.splits;
        });
        // S Q_blk = F_X T2 into columns c0.. of WS
        ch.gemm(GEMM_F64, GEMM_ADJ, [&, c0, bj](int j, Opnd& A, Opnd& B, void*& C, Opnd& Cm, int64_t& M,
                                                int64_t& N, int64_t& K, int&, int&, int&, int&) {
            A = mat(jobs[j].fx, n, D, D, 1);
            B = mat(at(j, L.t2p), D, bj, bj, 1);
            C = at(j, L.ws) + c0;
            Cm = mat(C, n, k, bj, 1);
            M = n;
            N = bj;
            K = D;
        });
        if (full || blk == s - 1) continue;
        // next block: S Q_blk orthogonalised against Q_0..Q_blk twice, then CholeskyQR2
        const int64_t kj = c0 + b;
        ch.small(0, [&, c0](int j, SmallDesc& d) {
            d = small_desc(SM_COPY, at(j, L.ws) + c0, k, at(j, L.wo), n, b, b);
        });
        for (int pass = 0; pass < 2; ++pass) {
            ch.gemm(GEMM_F64, GEMM_GRAM, [&, kj](int j, Opnd& A, Opnd& B, void*& C, Opnd&, int64_t& M, int64_t& N,
                                                 int64_t& K, int&, int&, int&, int&) {
                A = mat(at(j, L.q), kj, 1, n, k);
                B = mat(at(j, L.wo), n, b, b, 1);
                C = at(j, L.hc);
                M = kj;
                N = b;
                K = n;
            });
            ch.small(0, [&, kj](int j, SmallDesc& d) {
                d = small_desc(SM_NEG, at(j, L.hc), b, at(j, L.hc), kj, b, b);
            });
            ch.gemm(GEMM_F64, GEMM_ADJ, [&, kj](int j, Opnd& A, Opnd& B, void*& C, Opnd& Cm, int64_t& M, int64_t& N,
                                                int64_t& K, int&, int&, int&, int& acc) {
                A = mat(at(j, L.q), n, k, kj, 1);
                B = mat(at(j, L.hc), kj, b, b, 1);
                C = at(j, L.wo);
                Cm = mat(C, n, b, b, 1);
                M = n;
                N = b;
                K = kj;
                acc = 1;
            });
        }
        cholqr2([&](int j) { return at(j, L.wo); }, [&](int j) { return at(j, L.wx); },
                [&, kj](int j) { return at(j, L.q) + kj; }, k);
    }
    // Rayleigh quotient H = Q^T S Q (k x k), symmetrised; for the full basis H = S
    const int64_t hoff = full ? L.ws : L.h;
    if (!full) {
        ch.gemm(GEMM_F64, GEMM_GRAM, [&](int j, Opnd& A, Opnd& B, void*& C, Opnd&, int64_t& M, int64_t& N,
                                         int64_t& K, int&, int&, int&, int&) {
            A = mat(at(j, L.q), k, 1, n, k);
            B = mat(at(j, L.ws), n, k, k, 1);
            C = at(j, L.h);
            M = k;
            N = k;
            K = n;
        });
    }
    ch.small(0, [&](int j, SmallDesc& d) { d = small_desc(SM_SYM, nullptr, 0, at(j, hoff), k, k, k); });
    ch.small(0, [&](int j, SmallDesc& d) { d = small_desc(SM_IDENTITY, nullptr, 0, at(j, L.ik), k, k, k); });
    // leading eigenpairs of H on the compression core: Gram H against the identity factor
    {
        KOp op;
        op.kind = KO_CORE;
        op.key = k <= kCoreLdsMaxD ? 1 : 0;
        op.begin = (int64_t)out.core->size();
        op.count = (int)jobs.size();
        op.max_d = (int)k;
        for (int j = 0; j < (int)jobs.size(); ++j) {
            CoreDesc cd;
            std::memset(&cd, 0, sizeof(cd));
            cd.gram_a = at(j, hoff);
            cd.splits_a = 1;
            cd.fac_b = at(j, L.ik);
            cd.splits_b = 1;
            cd.rows_b = (int32_t)k;
            cd.D = (int32_t)k;
            cd.chi_new = (int32_t)nw;
            cd.cutoff = jobs[j].cutoff;
            cd.work = at(j, L.core);
            cd.p_left = at(j, L.plc);
            cd.p_right = at(j, L.prc);
            cd.stat = jobs[j].stat;
            cd.kmin = (int32_t)std::min<int64_t>(jobs[j].kmin, k);
            out.core->push_back(cd);
        }
        out.ops->push_back(op);
    }
    // Ritz vectors in the explicit side's row space: QP = Q P_L^core (n x chi')
    const int64_t qpoff = full ? L.plc : L.qp;
    if (!full) {
        ch.gemm(GEMM_F64, GEMM_GRAM, [&](int j, Opnd& A, Opnd& B, void*& C, Opnd&, int64_t& M, int64_t& N,
                                         int64_t& K, int&, int&, int&, int&) {
            A = mat(at(j, L.q), n, k, k, 1);
            B = mat(at(j, L.plc), k, nw, nw, 1);
            C = at(j, L.qp);
            M = n;
            N = nw;
            K = k;
        });
    }
    // P_X = F_X^T QP (D x chi')
    ch.gemm(GEMM_F64, GEMM_GRAM, [&](int j, Opnd& A, Opnd& B, void*& C, Opnd&, int64_t& M, int64_t& N, int64_t& K,
                                     int&, int&, int&, int&) {
        A = mat(jobs[j].fx, D, 1, n, D);
        B = mat(at(j, qpoff), n, nw, nw, 1);
        C = at(j, L.px);
        M = D;
        N = nw;
        K = n;
    });
    const int64_t pxsrc = L.px;
    // P_Y = (Y^T Y) P_X / s_Y^2, then column i divided by sigma_i (= |P_L^core column i|^2)
    ch.gemm(ykey, GEMM_ADJ, [&](int j, Opnd& A, Opnd& B, void*& C, Opnd& Cm, int64_t& M, int64_t& N, int64_t& K, int&,
                                int& sa, int&, int&) {
        A = viewed(jobs[j].y, &jobs[j].vy);
        B = mat(raw(j, pxsrc), D, nw, nw, 1);
        C = raw(j, L.u);
        Cm = mat(C, my, nw, nw, 1);
        M = my;
        N = nw;
        K = D;
        sa = jobs[j].y_scale;
    });
    ch.gemm(ykey, GEMM_GRAM, [&](int j, Opnd& A, Opnd& B, void*& C, Opnd&, int64_t& M, int64_t& N, int64_t& K,
                                 int& splits, int& sa, int&, int&) {
        A = viewed(jobs[j].y, &jobs[j].vyt);
        B = mat(raw(j, L.u), my, nw, nw, 1);
        C = at(j, L.pyp);
        M = D;
        N = nw;
        K = my;
        splits = sh.splits2;
        sa = jobs[j].y_scale;
    });
    ch.reduce([&](int j, double*& part, int64_t& M, int64_t& N, int& splits) {
        part = at(j, L.pyp);
        M = D;
        N = nw;
        const GemmDesc& g = (*out.gemm)[out.gemm->size() - jobs.size() + j];
        splits = g.splits;
    });
    ch.small(0, [&](int j, SmallDesc& d) {
        d = small_desc(SM_COLNORM2, at(j, L.plc), nw, at(j, L.nrm), 1, nw, nw);
        d.src_rows = (int32_t)k;
    });
    ch.small(0, [&](int j, SmallDesc& d) { d = small_desc(SM_COLSCALE, at(j, L.nrm), 0, at(j, L.pyp), D, nw, nw); });
    // convergence: E = F_X P_Y = S Z s^-3/2 against s QP = Z s^1/2, pair by pair
    ch.gemm(GEMM_F64, GEMM_GRAM, [&](int j, Opnd& A, Opnd& B, void*& C, Opnd&, int64_t& M, int64_t& N, int64_t& K,
                                     int&, int&, int&, int&) {
        A = mat(jobs[j].fx, n, D, D, 1);
        B = mat(at(j, L.pyp), D, nw, nw, 1);
        C = at(j, L.e);
        M = n;
        N = nw;
        K = D;
    });
    {
        KOp op;
        op.kind = KO_CHECK;
        op.begin = (int64_t)out.check->size();
        op.count = (int)jobs.size();
        for (int j = 0; j < (int)jobs.size(); ++j) {
            KrylovCheckDesc d;
            std::memset(&d, 0, sizeof(d));
            d.e = at(j, L.e);
            d.qp = at(j, qpoff);
            d.nrm = at(j, L.nrm);
            d.n = (int32_t)n;
            d.nw = (int32_t)nw;
            d.stat = jobs[j].stat;
            d.tol = kKrylovResidualTol;
            out.check->push_back(d);
        }
        out.ops->push_back(op);
    }
    // projectors in the tensor dtype
    ch.small(prec, [&](int j, SmallDesc& d) {
        if (jobs[j].x_is_b) d = small_desc(SM_CAST, at(j, L.px), nw, jobs[j].p_left, D, nw, nw);
        else d = small_desc(SM_CAST, at(j, L.pyp), nw, jobs[j].p_left, D, nw, nw);
    });
    ch.small(prec, [&](int j, SmallDesc& d) {
        if (jobs[j].x_is_b) d = small_desc(SM_CAST, at(j, L.pyp), nw, jobs[j].p_right, nw, D, D, 1);
        else d = small_desc(SM_CAST, at(j, L.px), nw, jobs[j].p_right, nw, D, D, 1);
    });
    return ch.err;
}

}  // namespace tn
