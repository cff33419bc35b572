// Host planner (see tn_plan.hpp).
#include "tn_plan.hpp"

#include <algorithm>
#include <climits>
#include <map>
#include <queue>
#include <set>
#include <tuple>
#include <sstream>

namespace tn {

namespace {

constexpr int64_t kAlign = 256;
constexpr int64_t kMaxElems = (int64_t)INT32_MAX;   // 32-bit element indexing in kernels
constexpr int kGemmTile = 64;
constexpr int kGemmK = 16;
constexpr int64_t kTsqrMaxD = 64;   // TSQR blocks keep a whole D-column width in LDS

struct EdgeLive {
    int64_t dim;
    int32_t end0, end1;
    bool alive;
};

int64_t prod_dims(const std::vector<int32_t>& legs, const std::vector<EdgeLive>& E) {
    int64_t p = 1;
    for (int e : legs) p *= E[e].dim;
    return p;
}

// Strides (in elements) of a tensor's legs, row-major in leg order.
std::vector<int64_t> leg_strides(const TensorVer& t, const std::vector<EdgeLive>& E) {
    std::vector<int64_t> s(t.legs.size());
    int64_t acc = 1;
    for (int a = (int)t.legs.size() - 1; a >= 0; --a) {
        s[a] = acc;
        acc *= E[t.legs[a]].dim;
    }
    return s;
}

ViewSpec tensor_view(const TensorVer& t, const std::vector<int32_t>& rows, const std::vector<int32_t>& cols,
                     const std::vector<EdgeLive>& E) {
    std::vector<int64_t> st = leg_strides(t, E);
    auto pos = [&](int e) {
        for (size_t a = 0; a < t.legs.size(); ++a)
            if (t.legs[a] == e) return (int)a;
        return -1;
    };
    ViewSpec v;
    for (int e : rows) {
        v.row_dims.push_back((int32_t)E[e].dim);
        v.row_strides.push_back(st[pos(e)]);
    }
    for (int e : cols) {
        v.col_dims.push_back((int32_t)E[e].dim);
        v.col_strides.push_back(st[pos(e)]);
    }
    return v;
}

ViewSpec dense_view(int64_t rows, int64_t cols) {
    ViewSpec v;
    v.row_dims = {(int32_t)rows};
    v.row_strides = {cols};
    v.col_dims = {(int32_t)cols};
    v.col_strides = {1};
    return v;
}

std::string make_axis(const std::vector<int32_t>& dims, const std::vector<int64_t>& strides, Axis* ax) {
    // merge adjacent legs that are contiguous in memory, drop unit legs
    std::vector<int64_t> d, s;
    for (size_t i = 0; i < dims.size(); ++i) {
        if (dims[i] == 1) continue;
        if (!d.empty() && s.back() == strides[i] * dims[i]) {
            d.back() *= dims[i];
            s.back() = strides[i];
        } else {
            d.push_back(dims[i]);
            s.push_back(strides[i]);
        }
    }
    if ((int)d.size() > kMaxLegs) return "matricisation needs more than 16 distinct legs";
    ax->n = (int32_t)d.size();
    ax->pad = 0;
    for (int l = 0; l < kMaxLegs; ++l) {
        ax->div[l] = make_fastdiv(1);
        ax->stride[l] = 0;
    }
    for (int l = 0; l < ax->n; ++l) {   // fastest first
        size_t i = d.size() - 1 - l;
        if (d[i] > kMaxElems || s[i] > kMaxElems) return "tensor too large for 32-bit indexing";
        ax->div[l] = make_fastdiv((uint32_t)d[i]);
        ax->stride[l] = (uint32_t)s[i];
    }
    return "";
}

int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Transposed view of a dense row-major (rows x cols) matrix: (cols x rows).
ViewSpec dense_view_t(int64_t rows, int64_t cols) {
    ViewSpec v;
    v.row_dims = {(int32_t)cols};
    v.row_strides = {1};
    v.col_dims = {(int32_t)rows};
    v.col_strides = {cols};
    return v;
}

// Split-K factor for a reduction of length K into an M x N result.
int32_t split_k(int64_t M, int64_t N, int64_t K, int64_t max_bytes) {
    const int64_t tiles = ((M + 63) / 64) * ((N + 63) / 64);
    int64_t s = (K + 255) / 256;
    s = std::min<int64_t>(s, std::max<int64_t>(1, 1024 / tiles));
    s = std::min<int64_t>(s, std::max<int64_t>(1, max_bytes / std::max<int64_t>(1, M * N * 8)));
    return (int32_t)std::max<int64_t>(1, s);
}

// Reverse-pass record of one forward op: its steps carry levels relative to the
// moment the adjoints of all its outputs are complete.
struct BwdOp {
    int32_t outs[2] = {-1, -1};      // tensor versions whose adjoints it reads
    int32_t ins[2] = {-1, -1};       // tensor versions whose adjoints it writes
    int32_t done[2] = {0, 0};        // relative level at which each input adjoint is complete
    std::vector<BStep> steps;
    int32_t comp = -1;
};

// First-fit free list over arena byte offsets; blocks are rounded up to kAlign, and an
// allocation that fits no free block extends the top (taking a free block that touches it).
struct FreeList {
    std::map<int64_t, int64_t> freel;   // offset -> size
    int64_t top;
    explicit FreeList(int64_t base) : top(base) {}
    int64_t alloc(int64_t bytes) {
        bytes = align_up(bytes);
        for (auto it = freel.begin(); it != freel.end(); ++it) {
            if (it->second >= bytes) {
                const int64_t off = it->first;
                const int64_t rest = it->second - bytes;
                freel.erase(it);
                if (rest > 0) freel[off + bytes] = rest;
                return off;
            }
        }
        int64_t off = top;
        if (!freel.empty()) {
            auto it = std::prev(freel.end());
            if (it->first + it->second == top) {
                off = it->first;
                freel.erase(it);
            }
        }
        top = off + bytes;
        return off;
    }
    void release(int64_t off, int64_t bytes) {
        bytes = align_up(bytes);
        auto it = freel.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != freel.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            freel.erase(nx);
        }
        if (it != freel.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                freel.erase(it);
            }
        }
    }
};

// Segment starts for checkpointed recomputation: `want` contiguous ranges of forward levels
// 1..maxl holding about equal bytes of the buffers produced in them (fewer when levels run out).
std::vector<int32_t> segment_starts(const std::vector<Buf>& bufs, int32_t maxl, int32_t want) {
    std::vector<double> at(maxl + 2, 0.0);
    double total = 0;
    for (const Buf& b : bufs)
        if (b.kind != BUF_INPUT && b.kind != BUF_BWD && b.lo >= 1 && b.lo <= maxl) {
            at[b.lo] += (double)b.bytes;
            total += (double)b.bytes;
        }
    std::vector<int32_t> sb{1};
    double cum = 0;
    for (int32_t L = 1; L <= maxl && (int32_t)sb.size() < want; ++L) {
        if (L > sb.back() && cum >= total * (double)sb.size() / want) sb.push_back(L);
        cum += at[L];
    }
    sb.push_back(maxl + 1);
    return sb;
}

}  // namespace

KrylovLayout krylov_layout(int64_t n, int64_t D, int64_t my, int64_t nw, int64_t b, int64_t k, int full,
                           int64_t splits, int64_t splits2, int64_t w) {
    KrylovLayout L{};
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        const int64_t at = off;
        off = align_up(off + std::max<int64_t>(bytes, 8));
        return at;
    };
    L.q = full ? -1 : take(8 * n * k);
    L.ws = take(8 * n * k);
    L.wo = full ? -1 : take(8 * n * b);
    L.wx = full ? -1 : take(8 * n * b);
    L.t1 = full ? -1 : take(8 * D * b);
    L.t1t = -1;
    L.u = take(8 * my * std::max(b, nw));   // float64 whatever the tensor dtype
    L.t2p = take(8 * splits * D * b);
    L.hc = full ? -1 : take(8 * k * b);
    L.g = full ? -1 : take(8 * b * b);
    L.m = full ? -1 : take(8 * b * b);
    L.h = full ? -1 : take(8 * k * k);
    L.ik = take(8 * k * k);
    const int64_t rebuild = (k > 64 && k <= 256) ? 2 * k * k : 0;
    L.core = take(8 * (4 * k * k + 4 * k + 2 * k * nw + rebuild));
    L.plc = take(8 * k * nw);
    L.prc = take(8 * nw * k);
    L.qp = full ? -1 : take(8 * n * nw);
    L.px = take(8 * D * nw);
    L.pxt = -1;
    L.pyp = take(8 * splits2 * D * nw);
    L.nrm = take(8 * nw);
    L.e = take(8 * n * nw);
    L.bytes = off;
    return L;
}

std::string make_view(const ViewSpec& s, View* v) {
    std::string err = make_axis(s.row_dims, s.row_strides, &v->row);
    if (!err.empty()) return err;
    err = make_axis(s.col_dims, s.col_strides, &v->col);
    if (!err.empty()) return err;
    v->row_unit = (v->row.n > 0 && v->row.stride[0] == 1) ? 1 : 0;
    v->col_unit = (v->col.n > 0 && v->col.stride[0] == 1) ? 1 : 0;
    return "";
}

std::string check_graph(const GraphSpec& g) {
    std::ostringstream os;
    if (g.n < 1) return "n_tensors must be >= 1";
    if (g.ne < 0) return "n_edges must be >= 0";
    if ((int)g.eu.size() != g.ne || (int)g.ev.size() != g.ne || (int)g.ed.size() != g.ne)
        return "edge arrays missing";
    std::vector<int64_t> size(g.n, 1);
    for (int e = 0; e < g.ne; ++e) {
        if (g.eu[e] < 0 || g.ev[e] >= g.n || g.eu[e] >= g.ev[e]) {
            os << "edge " << e << " must satisfy 0 <= u < v < n_tensors";
            return os.str();
        }
        if (g.ed[e] < 1) {
            os << "edge " << e << " has dimension < 1";
            return os.str();
        }
        for (int x : {g.eu[e], g.ev[e]}) {
            size[x] *= g.ed[e];
            if (size[x] > kMaxElems) {
                os << "tensor " << x << " exceeds 2^31-1 elements";
                return os.str();
            }
        }
    }
    if ((int)g.offsets.size() != g.n + 1 || g.offsets[0] != 0) return "offsets must hold n_tensors+1 entries starting at 0";
    for (int v = 0; v < g.n; ++v) {
        if (g.offsets[v + 1] - g.offsets[v] != size[v]) {
            os << "tensor " << v << " has " << (g.offsets[v + 1] - g.offsets[v]) << " entries, expected " << size[v];
            return os.str();
        }
    }
    return "";
}

std::string build_plan(const GraphSpec& g, const int32_t* pi, const int32_t* pj, int32_t n_steps,
                       const TreeOpts& o, bool shapes_only, Plan* P) {
    std::ostringstream os;
    *P = Plan();
    P->g = g;
    P->opts = o;
    P->elem_size = o.precision == 1 ? 4 : o.precision == 2 ? 2 : 8;
    const int64_t w = P->elem_size;
    if (o.chi < 1) return "chi must be >= 1";
    if (n_steps != g.n - 1) {
        os << "a tree over " << g.n << " tensors has " << (g.n - 1) << " steps, got " << n_steps;
        return os.str();
    }
    std::vector<EdgeLive> E(g.ne);
    std::vector<std::vector<int32_t>> inc(g.n);
    for (int e = 0; e < g.ne; ++e) {
        E[e] = {g.ed[e], g.eu[e], g.ev[e], true};
        inc[g.eu[e]].push_back(e);
        inc[g.ev[e]].push_back(e);
    }
    const int32_t total_ids = g.n + n_steps;
    std::vector<int32_t> live(total_ids, -1);
    auto new_buf = [&](int64_t bytes, int kind, int lo) {
        Buf b;
        b.bytes = std::max<int64_t>(bytes, 8);
        b.kind = kind;
        b.lo = lo;
        b.hi = lo;
        P->bufs.push_back(b);
        return (int32_t)P->bufs.size() - 1;
    };
    auto touch = [&](int32_t buf, int level) {
        if (buf >= 0) P->bufs[buf].hi = std::max(P->bufs[buf].hi, level);
    };
    for (int v = 0; v < g.n; ++v) {
        TensorVer t;
        t.legs = inc[v];   // ascending edge id by construction
        t.size = prod_dims(t.legs, E);
        t.level = 0;
        if (!shapes_only) t.buf = new_buf(t.size * w, BUF_INPUT, 0);
        P->tens.push_back(t);
        live[v] = v;
    }
    int next_edge = g.ne;
    int32_t last_step_level = 0;
    size_t step_mark = 0;

    auto read_tensor = [&](int32_t ver, int level) {
        TensorVer& t = P->tens[ver];
        t.last_read = std::max(t.last_read, level);
        touch(t.buf, level);
    };

    std::vector<BwdOp> bops;
    auto adj_of = [&](int32_t ver) {
        if ((int32_t)P->adj_buf.size() <= ver) P->adj_buf.resize(ver + 1, -1);
        if (P->adj_buf[ver] < 0) P->adj_buf[ver] = new_buf(P->tens[ver].size * w, BUF_BWD, 0);
        return P->adj_buf[ver];
    };
    // reverse-pass GEMM: C(vc) = [C +] f A(va) B(vb), or split-K float64 partials + a reduction
    // (the reduction reads the partials into C(vc) one level later); returns the levels used
    auto bwd_gemm = [&](BwdOp& op, int rel, int32_t a_buf, int32_t b_buf, int32_t c_buf, const ViewSpec& va,
                        const ViewSpec& vb, const ViewSpec& vc, int64_t M, int64_t N, int64_t K, int32_t sa,
                        int32_t sb, int32_t acc, bool allow_split) {
        BStep g;
        g.kind = BS_GEMM;
        g.level = rel;
        g.a_buf = a_buf;
        g.b_buf = b_buf;
        g.c_buf = c_buf;
        g.va = va;
        g.vb = vb;
        g.vc = vc;
        g.M = M;
        g.N = N;
        g.K = K;
        g.scale_a = sa;
        g.scale_b = sb;
        g.accumulate = acc;
        g.flops = 2.0 * (double)M * N * K;
        g.bytes = (double)w * ((double)M * K + (double)K * N + (double)M * N);
        const int64_t tiles = ((M + 63) / 64) * ((N + 63) / 64);
        if (allow_split && !acc && K > 2048 && tiles < 64) {
            g.partial = 1;
            g.splits = split_k(M, N, K, 64 << 20);
            int64_t kps = (K + g.splits - 1) / g.splits;
            kps = (kps + kGemmK - 1) / kGemmK * kGemmK;
            g.splits = (int32_t)((K + kps - 1) / kps);
            g.k_per_split = (int32_t)kps;
            g.c_buf = new_buf((int64_t)g.splits * M * N * 8, BUF_BWD, 0);
            BStep r;
            r.kind = BS_REDUCE;
            r.level = rel + 1;
            r.a_buf = g.c_buf;
            r.c_buf = c_buf;
            r.vc = vc;
            r.M = M;
            r.N = N;
            r.splits = g.splits;
            r.scale_a = -1;   // the partials already carry the factor
            r.scale_b = -1;
            r.bytes = 8.0 * g.splits * M * N + (double)w * M * N;
            op.steps.push_back(g);
            op.steps.push_back(r);
            return 2;
        }
        g.splits = 1;
        g.k_per_split = (int32_t)K;
        op.steps.push_back(g);
        return 1;
    };

    auto add_gemm_flops = [&](Step& s) {
        s.flops = 2.0 * (double)s.M * (double)s.N * (double)s.K;
        s.bytes = (double)w * ((double)s.M * s.K + (double)s.K * s.N + (double)s.M * s.N);
    };

    for (int t = 0; t < n_steps; ++t) {
        if (o.ordered)
            for (size_t q = step_mark; q < P->steps.size(); ++q) last_step_level = std::max(last_step_level, P->steps[q].level);
        step_mark = P->steps.size();
        const int32_t i = pi[t], j = pj[t];
        if (i < 0 || j < 0 || i >= total_ids || j >= total_ids || i == j || live[i] < 0 || live[j] < 0) {
            os << "step " << t << ": (" << i << ", " << j << ") are not two live tensors";
            return os.str();
        }
        const int32_t k = g.n + t;
        // one bond compression between the live tensors a and b: COMPRESS_TREE_GAUGE of
        // Algorithm 1 at r = 0 (the reduced factors of a and b alone), a's free legs as rows
        auto compress_bond = [&](const int32_t a, const int32_t b) {
            const int32_t va = live[a], vb = live[b];
            const TensorVer Ta = P->tens[va], Tb = P->tens[vb];
            std::vector<int32_t> shared, free_a, free_b;
            for (int e : Ta.legs) {
                if (std::find(Tb.legs.begin(), Tb.legs.end(), e) != Tb.legs.end()) shared.push_back(e);
                else free_a.push_back(e);
            }
            for (int e : Tb.legs)
                if (std::find(shared.begin(), shared.end(), e) == shared.end()) free_b.push_back(e);
            const int64_t D = prod_dims(shared, E);
            const int64_t ma = Ta.size / D, mb = Tb.size / D;
            const int64_t ka = std::min(ma, D), kb = std::min(mb, D);
            const int64_t nw = std::min<int64_t>(o.chi, std::min(ka, kb));
            const int32_t e_new = next_edge++;
            E.push_back({nw, a, b, true});
            P->ops.push_back({1, a, b, e_new, ma, D, mb, nw});
            TensorVer Ta2, Tb2;
            Ta2.legs = free_a;
            Ta2.legs.push_back(e_new);
            Ta2.size = ma * nw;
            Tb2.legs.push_back(e_new);
            Tb2.legs.insert(Tb2.legs.end(), free_b.begin(), free_b.end());
            Tb2.size = nw * mb;
            if (!shapes_only) {
                Compression c{};
                c.a_ver_in = va;
                c.b_ver_in = vb;
                c.node_a = a;
                c.node_b = b;
                c.e_new = e_new;
                c.bond_edges = shared;
                c.ma = ma;
                c.D = D;
                c.mb = mb;
                c.chi_new = (int32_t)nw;
                const int32_t comp_id = (int32_t)P->comps.size();
                // ---- tree gauge (r >= 1): the r-local spanning tree of SI A over the live intermediates
                // around (a, b), then an environment metric for every tree edge, outer tensors first:
                // M_{v->u} = the Gram of v over every leg but its bond to u, with the metrics of v's own
                // children applied on their bonds (the R^T R of the R factor that the inward QR would
                // push into u); the two side Grams take the metrics of a's and b's children the same way
                std::vector<std::pair<int32_t, int32_t>> tau;
                if (o.gauge_r > 0) {
                    auto bonds_of = [&](int32_t x) {
                        std::map<int32_t, int64_t> m;
                        for (int e : P->tens[live[x]].legs) {
                            const int32_t other = (E[e].end0 == x) ? E[e].end1 : E[e].end0;
                            auto it = m.find(other);
                            m[other] = (it == m.end() ? 1 : it->second) * E[e].dim;
                        }
                        return m;
                    };
                    std::set<int32_t> S = {a, b};
                    using Cand = std::tuple<int32_t, int64_t, int32_t, int32_t>;   // distance, -bond, v, u
                    std::priority_queue<Cand, std::vector<Cand>, std::greater<Cand>> pq;
                    for (const int32_t u : {a, b})
                        for (auto& kv : bonds_of(u))
                            if (!S.count(kv.first)) pq.push(Cand{1, -kv.second, kv.first, u});
                    while (!pq.empty()) {
                        const Cand cd = pq.top();
                        pq.pop();
                        const int32_t d = std::get<0>(cd), v = std::get<2>(cd), u = std::get<3>(cd);
                        if (S.count(v) || d > o.gauge_r || v < g.n) continue;   // input tensors are not spanned
                        S.insert(v);
                        tau.push_back({u, v});
                        for (auto& kv : bonds_of(v))
                            if (!S.count(kv.first)) pq.push(Cand{d + 1, -kv.second, kv.first, v});
                    }
                }
                std::map<int32_t, std::vector<int32_t>> gchildren;
                for (auto& pr : tau) gchildren[pr.first].push_back(pr.second);
                struct Metric { int32_t buf, level; std::vector<int32_t> edges; };   // edges: the child's order
                std::map<int32_t, Metric> metrics;
                auto gram_splits = [&](int64_t Dm, int64_t K, int64_t* kps) {
                    const int64_t tiles = ((Dm + 63) / 64) * ((Dm + 63) / 64);
                    int64_t sp = (K + 255) / 256;
                    sp = std::min<int64_t>(sp, std::max<int64_t>(1, 1024 / tiles));
                    sp = std::min<int64_t>(sp, std::max<int64_t>(1, (32 << 20) / (Dm * Dm * 8)));
                    sp = std::max<int64_t>(1, sp);
                    int64_t k = (K + sp - 1) / sp;
                    k = (k + kGemmK - 1) / kGemmK * kGemmK;
                    *kps = k;
                    return (int32_t)((K + k - 1) / k);
                };
                // W = X with the metrics of x's tree children applied on their bonds (x's layout, float64);
                // returns {buffer, level} or {-1, level of x} when x has no children
                auto apply_children = [&](int32_t x) {
                    const int32_t ver = live[x];
                    const TensorVer& Tx = P->tens[ver];
                    int32_t cur = -1, cur_level = Tx.level;
                    auto it = gchildren.find(x);
                    if (it == gchildren.end()) return std::make_pair(cur, cur_level);
                    for (const int32_t wch : it->second) {
                        const Metric& M = metrics.at(wch);
                        std::vector<int32_t> bond, rest;
                        for (int e : Tx.legs)
                            (std::find(M.edges.begin(), M.edges.end(), e) != M.edges.end() ? bond : rest).push_back(e);
                        const int64_t Dm = prod_dims(bond, E);
                        // the metric's index: its edges in the child's order, slowest first
                        ViewSpec vb;
                        for (int e : bond) {
                            int64_t unit = 1;
                            for (size_t q = std::find(M.edges.begin(), M.edges.end(), e) - M.edges.begin() + 1;
                                 q < M.edges.size(); ++q)
                                unit *= E[M.edges[q]].dim;
                            vb.row_dims.push_back((int32_t)E[e].dim);
                            vb.row_strides.push_back(unit * Dm);
                            vb.col_dims.push_back((int32_t)E[e].dim);
                            vb.col_strides.push_back(unit);
                        }
                        Step st;
                        st.kind = ST_GAUGE;
                        st.gauge_mode = GAUGE_APPLY;
                        st.comp = comp_id;
                        st.level = 1 + std::max(cur_level, M.level);
                        st.in_a = cur < 0 ? ver : -1;
                        st.a_buf = cur;
                        st.b_buf = M.buf;
                        st.M = Tx.size / Dm;
                        st.N = Dm;
                        st.K = Dm;
                        st.va = tensor_view(Tx, rest, bond, E);
                        st.vb = vb;
                        st.vc = tensor_view(Tx, rest, bond, E);
                        st.out_buf = new_buf(Tx.size * 8, BUF_FACTOR, st.level);
                        st.flops = 2.0 * (double)st.M * st.N * st.K;
                        st.bytes = (double)(cur < 0 ? w : 8) * st.M * st.K + 8.0 * st.K * st.N + 8.0 * st.M * st.N;
                        if (cur < 0) read_tensor(ver, st.level);
                        else touch(cur, st.level);
                        touch(M.buf, st.level);
                        P->steps.push_back(st);
                        cur = st.out_buf;
                        cur_level = st.level;
                    }
                    return std::make_pair(cur, cur_level);
                };
                // the metric-weighted Gram of x over `rest`, indexed by `bond` (in the order given)
                auto gauge_gram = [&](int32_t x, const std::vector<int32_t>& bond, const std::vector<int32_t>& rest,
                                      int32_t wbuf, int32_t wlevel, int32_t* out_splits) {
                    const int32_t ver = live[x];
                    const TensorVer& Tx = P->tens[ver];
                    const int64_t Dm = prod_dims(bond, E), K = Tx.size / Dm;
                    Step st;
                    st.kind = ST_GAUGE;
                    st.gauge_mode = GAUGE_GRAM;
                    st.comp = comp_id;
                    st.level = 1 + std::max(Tx.level, wlevel);
                    st.in_a = ver;
                    st.b_buf = wbuf;
                    st.M = Dm;
                    st.N = Dm;
                    st.K = K;
                    st.va = tensor_view(Tx, bond, rest, E);
                    st.vb = tensor_view(Tx, rest, bond, E);   // W has x's layout
                    int64_t kps = K;
                    st.splits = gram_splits(Dm, K, &kps);
                    st.k_per_split = (int32_t)kps;
                    st.out_buf = new_buf((int64_t)st.splits * Dm * Dm * 8, BUF_GRAM, st.level);
                    st.flops = 2.0 * (double)Dm * Dm * K;
                    st.bytes = (double)w * Dm * K + 8.0 * Dm * K;
                    read_tensor(ver, st.level);
                    touch(wbuf, st.level);
                    P->steps.push_back(st);
                    *out_splits = st.splits;
                    return std::make_pair(st.out_buf, st.level);
                };
                for (auto it = tau.rbegin(); it != tau.rend(); ++it) {
                    const int32_t u = it->first, v = it->second;
                    const TensorVer& Tv = P->tens[live[v]];
                    const TensorVer& Tu = P->tens[live[u]];
                    std::vector<int32_t> bond, rest;
                    for (int e : Tv.legs)
                        (std::find(Tu.legs.begin(), Tu.legs.end(), e) != Tu.legs.end() ? bond : rest).push_back(e);
                    const std::pair<int32_t, int32_t> wv = apply_children(v);
                    Metric m;
                    m.edges = bond;
                    if (wv.first < 0) {
                        // a leaf of the tree: its plain Gram (the narrow-Gram path for small bonds)
                        const int64_t Dm = prod_dims(bond, E), K = Tv.size / Dm;
                        Step st;
                        st.kind = ST_GRAM;
                        st.comp = comp_id;
                        st.level = Tv.level + 1;
                        st.in_a = live[v];
                        st.M = Dm;
                        st.N = Dm;
                        st.K = K;
                        st.va = tensor_view(Tv, bond, rest, E);
                        st.vb = tensor_view(Tv, rest, bond, E);
                        int64_t kps = K;
                        if (Dm <= kGramNarrowMaxD) {
                            kps = 512;
                            st.splits = (int32_t)((K + kps - 1) / kps);
                        } else {
                            st.splits = gram_splits(Dm, K, &kps);
                        }
                        st.k_per_split = (int32_t)kps;
                        st.out_buf = new_buf((int64_t)st.splits * Dm * Dm * 8, BUF_GRAM, st.level);
                        st.flops = 2.0 * (double)Dm * Dm * K;
                        st.bytes = (double)w * Dm * K;
                        read_tensor(live[v], st.level);
                        P->steps.push_back(st);
                        m.buf = st.out_buf;
                        m.level = st.level;
                    } else {
                        int32_t sp = 1;
                        const std::pair<int32_t, int32_t> gr = gauge_gram(v, bond, rest, wv.first, wv.second, &sp);
                        m.buf = gr.first;
                        m.level = gr.second;
                    }
                    metrics[v] = m;
                }
                const bool gauged = !tau.empty();
                const bool big = D >= kLanczosMinD && !o.grad && !gauged;   // the reverse pass needs the full core spectrum
                const bool xside = ma <= D || mb <= D;
                // one explicit side and a large bond: block Krylov with the other side read in place
                const bool krylov = big && xside && D >= kKrylovMinD;
                const bool glanczos = big && xside && !krylov;
                c.krylov = krylov ? 1 : 0;
                // X = the explicit side (the shorter one when both are explicit)
                const int x_is_b = (mb <= D && (ma > D || mb <= ma)) ? 1 : 0;
                // both sides tall: Gram + block-Jacobi core up to D = 256 (one launch per tournament round over
                // many workgroups); Golub-Kahan-Lanczos on A B (one workgroup) only beyond that
                const bool lanczos = big && !xside && D > kBlockJacobiMaxD && (ma + mb) <= kLanczosMaxRowsPerD * D;
                c.lanczos = lanczos ? 1 : 0;
                c.glanczos = glanczos ? 1 : 0;
                Step core;
                if (lanczos) {
                    // one step: Golub-Kahan-Lanczos truncated SVD of A_mat B_mat read through Views.
                    // The Grams of both sides (float64, D x D) give ||A B||_F^2 = <G_A, G_B> for the
                    // kernel's completeness test; they are not part of the credited work (the QR
                    // terms of both sides are credited with the compression below)
                    int32_t gram_level = 0;
                    for (int side = 0; side < 2; ++side) {
                        const TensorVer& T = side == 0 ? Ta : Tb;
                        const int32_t ver = side == 0 ? va : vb;
                        const std::vector<int32_t>& fr = side == 0 ? free_a : free_b;
                        const int64_t mm = side == 0 ? ma : mb;
                        Step st;
                        st.kind = ST_GRAM;
                        st.level = T.level + 1;
                        st.comp = comp_id;
                        st.in_a = ver;
                        st.M = D;
                        st.N = D;
                        st.K = mm;
                        st.va = tensor_view(T, shared, fr, E);
                        st.vb = tensor_view(T, fr, shared, E);
                        const int64_t tiles = ((D + 63) / 64) * ((D + 63) / 64);
                        int64_t splits = (mm + 255) / 256;
                        splits = std::min<int64_t>(splits, std::max<int64_t>(1, 1024 / tiles));
                        splits = std::min<int64_t>(splits, std::max<int64_t>(1, (32 << 20) / (D * D * 8)));
                        splits = std::max<int64_t>(1, splits);
                        int64_t kps = (mm + splits - 1) / splits;
                        kps = (kps + kGemmK - 1) / kGemmK * kGemmK;
                        splits = (mm + kps - 1) / kps;
                        st.splits = (int32_t)splits;
                        st.k_per_split = (int32_t)kps;
                        st.out_buf = new_buf(splits * D * D * 8, BUF_GRAM, st.level);
                        st.flops = 0.0;
                        st.bytes = (double)w * mm * D;
                        (side == 0 ? c.gram_a : c.gram_b) = 1;
                        (side == 0 ? c.splits_a : c.splits_b) = (int32_t)splits;
                        (side == 0 ? c.side_a_buf : c.side_b_buf) = st.out_buf;
                        read_tensor(ver, st.level);
                        gram_level = std::max(gram_level, st.level);
                        P->steps.push_back(st);
                    }
                    const int64_t r = std::min(std::min(ma, mb), D);
                    c.s_min = (int32_t)std::min<int64_t>(r, 2 * nw + 4);
                    // r + 1: the start vector's component outside the row space of A B adds one
                    // Krylov direction before the range is exhausted; the completeness test may run
                    // the space that far
                    c.s_max = (int32_t)std::min<int64_t>(r + 1, 512);
                    c.s_min = std::min(c.s_min, c.s_max);
                    core.kind = ST_LANCZOS;
                    core.level = 1 + gram_level;
                    touch(c.side_a_buf, core.level + 1);
                    touch(c.side_b_buf, core.level + 1);
                    core.comp = comp_id;
                    core.in_a = va;
                    core.in_b = vb;
                    core.va = tensor_view(Ta, free_a, shared, E);
                    core.vb = tensor_view(Tb, shared, free_b, E);
                    const int64_t sm = c.s_max;
                    const int64_t ls = sm + 1;   // small bidiagonal leading dimension (see the kernel)
                    const int64_t words = ma * sm + mb * (sm + 1) + (ma + mb) * nw + 2 * D + 2 * sm + ls + 2 * ls * ls +
                                          (ls + ma + mb + 2 * D + 1) / 2 + 8;
                    c.work_buf = new_buf(words * 8, BUF_WORK, core.level);
                    read_tensor(va, core.level);
                    read_tensor(vb, core.level);
                } else {
                    int side_level[2];
                    for (int side = 0; side < 2; ++side) {
                        const TensorVer& T = side == 0 ? Ta : Tb;
                        const int32_t ver = side == 0 ? va : vb;
                        const std::vector<int32_t>& fr = side == 0 ? free_a : free_b;
                        const int64_t mm = side == 0 ? ma : mb;
                        if (krylov && side != x_is_b) {   // Y: read in place by the Krylov chain
                            side_level[side] = T.level;
                            (side == 0 ? c.side_a_buf : c.side_b_buf) = -1;
                            continue;
                        }
                        const std::pair<int32_t, int32_t> wside =
                            gauged ? apply_children(side == 0 ? a : b) : std::make_pair(-1, 0);
                        if (wside.first >= 0) {
                            // tree gauge: the side's Gram with its children's metrics applied
                            int32_t sp = 1;
                            const std::pair<int32_t, int32_t> gr =
                                gauge_gram(side == 0 ? a : b, shared, fr, wside.first, wside.second, &sp);
                            (side == 0 ? c.gram_a : c.gram_b) = 1;
                            (side == 0 ? c.splits_a : c.splits_b) = sp;
                            (side == 0 ? c.side_a_buf : c.side_b_buf) = gr.first;
                            side_level[side] = gr.second;
                            continue;
                        }
                        Step st;
                        st.level = T.level + 1;
                        st.comp = comp_id;
                        st.in_a = ver;
                        if (mm > D && o.rfactor == 1 && D <= kTsqrMaxD) {
                            // TSQR: R (D x D) of A_mat (side A) or of B_mat^T (side B), R^T R = the
                            // Gram; passes of row blocks until one block remains.  The core takes R
                            // as an explicit factor of D rows
                            st.kind = ST_TSQR;
                            st.M = D;
                            st.K = mm;
                            st.va = tensor_view(T, fr, shared, E);
                            st.out_buf = new_buf(D * D * 8, BUF_FACTOR, st.level);
                            const int64_t br = tsqr_block_rows((int)D);
                            for (int64_t rows = mm;;) {
                                const int64_t nb = (rows + br - 1) / br;
                                st.tsqr_blocks.push_back((int32_t)nb);
                                if (nb == 1) {
                                    st.tsqr_bufs.push_back(st.out_buf);
                                    break;
                                }
                                st.tsqr_bufs.push_back(new_buf(nb * D * D * 8, BUF_GRAM, st.level));
                                rows = nb * D;
                            }
                            // algorithmic cost of this R-factor: a QR of an (mm x D) matrix (SI section D)
                            st.flops = 2.0 * (double)mm * D * D - 2.0 / 3.0 * (double)D * D * D;
                            st.bytes = (double)w * mm * D;
                            (side == 0 ? c.rows_a : c.rows_b) = (int32_t)D;
                        } else if (mm > D) {
                            // Gram: side A -> A_mat^T A_mat ; side B -> B_mat B_mat^T  (both D x D)
                            st.kind = ST_GRAM;
                            st.M = D;
                            st.N = D;
                            st.K = mm;
                            st.va = tensor_view(T, shared, fr, E);
                            st.vb = tensor_view(T, fr, shared, E);
                            // split-K: short chunks keep each workgroup's serial loop short (the
                            // compressions of one level are few, so latency, not throughput, rules);
                            // about a thousand workgroups per Gram and 32 MiB of partials at most
                            const int64_t tiles = ((D + 63) / 64) * ((D + 63) / 64);
                            int64_t splits, kps;
                            if (D <= kGramNarrowMaxD) {
                                // narrow side (its own kernel, one 512-row range per workgroup)
                                kps = 512;
                                splits = (mm + kps - 1) / kps;
                            } else {
                                splits = (mm + 255) / 256;
                                splits = std::min<int64_t>(splits, std::max<int64_t>(1, 1024 / tiles));
                                splits = std::min<int64_t>(splits, std::max<int64_t>(1, (32 << 20) / (D * D * 8)));
                                splits = std::max<int64_t>(1, splits);
                                kps = (mm + splits - 1) / splits;
                                kps = (kps + kGemmK - 1) / kGemmK * kGemmK;
                                splits = (mm + kps - 1) / kps;
                            }
                            st.splits = (int32_t)splits;
                            st.k_per_split = (int32_t)kps;
                            st.out_buf = new_buf(splits * D * D * 8, BUF_GRAM, st.level);
                            // algorithmic cost of this R-factor: a QR of an (mm x D) matrix (SI section D)
                            st.flops = 2.0 * (double)mm * D * D - 2.0 / 3.0 * (double)D * D * D;
                            st.bytes = (double)w * mm * D;
                            (side == 0 ? c.gram_a : c.gram_b) = 1;
                            (side == 0 ? c.splits_a : c.splits_b) = (int32_t)splits;
                        } else {
                            // explicit factor: side A -> A_mat (ma x D); side B -> B_mat^T (mb x D)
                            st.kind = ST_COPY;
                            st.copy_rows = (int32_t)mm;
                            st.copy_cols = (int32_t)D;
                            st.va = tensor_view(T, fr, shared, E);
                            st.out_buf = new_buf(mm * D * 8, BUF_FACTOR, st.level);
                            st.bytes = (double)(w + 8) * mm * D;
                            (side == 0 ? c.rows_a : c.rows_b) = (int32_t)mm;
                        }
                        (side == 0 ? c.side_a_buf : c.side_b_buf) = st.out_buf;
                        read_tensor(ver, st.level);
                        side_level[side] = st.level;
                        P->steps.push_back(st);
                    }
                    core.kind = ST_CORE;
                    core.level = 1 + std::max(side_level[0], side_level[1]);
                    core.comp = comp_id;
                    touch(c.side_a_buf, core.level);
                    touch(c.side_b_buf, core.level);
                    if (krylov) {
                        core.kind = ST_KRYLOV;
                        c.x_is_b = x_is_b;
                        // Y (m_Y x D) and Y^T through the tensor's own layout
                        const TensorVer& TY = x_is_b ? Ta : Tb;
                        const std::vector<int32_t>& fy = x_is_b ? free_a : free_b;
                        core.in_a = x_is_b ? va : vb;
                        core.va = tensor_view(TY, fy, shared, E);
                        core.vb = tensor_view(TY, shared, fy, E);
                        const int64_t n = x_is_b ? mb : ma, my = x_is_b ? ma : mb;
                        c.kr_n = n;
                        c.kr_my = my;
                        // basis: 4 chi' directions (at most 256, the core kernel's block-Jacobi range),
                        // in blocks of about chi'/2; or all of R^n when n is that small
                        const int64_t kcap = std::min<int64_t>(256, std::max<int64_t>(64, 4 * nw));
                        if (n <= kcap) {
                            c.kr_full = 1;
                            c.kr_k = (int32_t)n;
                            c.kr_b = (int32_t)std::min<int64_t>(64, n);
                            c.kr_s = (int32_t)((n + c.kr_b - 1) / c.kr_b);
                        } else {
                            c.kr_full = 0;
                            const int64_t bb = std::min<int64_t>(64, std::max<int64_t>(8, (nw / 2 + 7) / 8 * 8));
                            c.kr_b = (int32_t)bb;
                            c.kr_s = (int32_t)(kcap / bb);
                            c.kr_k = c.kr_b * c.kr_s;
                        }
                        auto ysplits = [&](int64_t N) {
                            const int64_t tiles = ((D + 63) / 64) * ((N + 63) / 64);
                            int64_t sp = (my + 255) / 256;
                            sp = std::min<int64_t>(sp, std::max<int64_t>(1, 1024 / tiles));
                            sp = std::min<int64_t>(sp, std::max<int64_t>(1, (32 << 20) / (D * N * 8)));
                            return (int32_t)std::max<int64_t>(1, sp);
                        };
                        c.kr_splits = ysplits(c.kr_b);
                        c.kr_splits2 = ysplits(nw);
                        const KrylovLayout L = krylov_layout(n, D, my, nw, c.kr_b, c.kr_k, c.kr_full, c.kr_splits,
                                                             c.kr_splits2, w);
                        c.work_buf = new_buf(L.bytes, BUF_WORK, core.level);
                        // like a core launch, the chain may run on into the next level
                        touch(c.work_buf, core.level + 1);
                        touch(x_is_b ? c.side_b_buf : c.side_a_buf, core.level + 1);
                        read_tensor(x_is_b ? va : vb, core.level + 1);
                    } else if (glanczos) {
                        // X = the explicit side (the shorter one when both are explicit)
                        c.x_is_b = (mb <= D && (ma > D || mb <= ma)) ? 1 : 0;
                        const int64_t n = c.x_is_b ? mb : ma, my = c.x_is_b ? ma : mb;
                        // first convergence check after chi' + 16 steps: a step is one matvec with the
                        // precomputed operator, far cheaper than the tridiagonal eigensolve of a check
                        c.s_min = (int32_t)std::min<int64_t>(n, nw + 16);
                        // up to n steps: the completeness test of the kernel may run the Krylov space
                        // to exhaustion (repeated kept eigenvalues with a heavy discarded tail)
                        c.s_max = (int32_t)std::min<int64_t>(n, 512);
                        const int64_t sm = c.s_max, ls = sm + 1;
                        // T1 = G_Y F_X^T (D x n) when Y has a Gram, else F_X F_Y^T (n x my, my <= D)
                        const int64_t t1 = (my > D ? D : my) * n;
                        const int64_t words = n * n + t1 + n * sm + n * nw + 2 * D + std::max(n, my) +
                                              2 * sm + ls +
                                              2 * ls * ls + 16 * D + 2 * D * nw + std::max(n, my) * nw + ls / 2 +
                                              8;   // 16 = waves of the kernel
                        // the operator S and its half product T1 are formed at the sides' level,
                        // after the side factors (same stream), so the workspace lives from there
                        c.work_buf = new_buf(words * 8, BUF_WORK, core.level - 1);
                        // the executor lets a compression launch run on into the next level (only the
                        // re-absorbing GEMMs wait for it), so what it reads lives one level longer
                        touch(c.work_buf, core.level + 1);
                        touch(c.side_a_buf, core.level + 1);
                        touch(c.side_b_buf, core.level + 1);
                    } else {
                        // R~_A, R~_B, W, V, spectrum; the sorted kept columns of V and W; for the block
                        // Jacobi of 64 < D <= 256, room to rebuild W and V from the transposed problem
                        const int64_t rebuild = (D > 64 && D <= 256) ? 2 * D * D : 0;
                        c.work_buf = new_buf((4 * D * D + 4 * D + 2 * D * nw + rebuild) * 8, BUF_WORK, core.level);
                        // like a Gram-Lanczos launch, a core launch may run on into the next level
                        touch(c.work_buf, core.level + 1);
                        touch(c.side_a_buf, core.level + 1);
                        touch(c.side_b_buf, core.level + 1);
                    }
                }
                c.pl_buf = new_buf(D * nw * w, BUF_PROJ, core.level);
                c.pr_buf = new_buf(nw * D * w, BUF_PROJ, core.level);
                {
                    // algorithmic cost of the compression (SI section D): QR of each tall side,
                    // the R_A R_B core and its SVD; the same whichever kernel computes it
                    double f = 0.0, b = 0.0;
                    for (int64_t mm : {ma, mb})
                        if ((lanczos || krylov) && mm > D) {   // Gram steps carry these terms otherwise
                            f += 2.0 * (double)mm * D * D - 2.0 / 3.0 * (double)D * D * D;
                            b += (double)w * mm * D;
                        }
                    const double p = (double)std::max(ka, kb), q = (double)std::min(ka, kb);
                    f += 2.0 * ka * D * kb + 4.0 * p * q * q - 4.0 / 3.0 * q * q * q;
                    core.flops = f;
                    core.bytes = b;
                }
                c.core_step = (int32_t)P->steps.size();
                P->steps.push_back(core);
                for (int side = 0; side < 2; ++side) {
                    const TensorVer& T = side == 0 ? Ta : Tb;
                    const int32_t ver = side == 0 ? va : vb;
                    Step st;
                    st.kind = ST_ABSORB;
                    st.level = core.level + 1;
                    st.comp = comp_id;
                    st.in_a = ver;
                    st.proj_left = side == 0 ? 1 : 0;
                    st.proj_buf = side == 0 ? c.pl_buf : c.pr_buf;
                    if (side == 0) {   // a' = A_mat . P_L   (ma x D) (D x nw)
                        st.M = ma;
                        st.N = nw;
                        st.K = D;
                        st.va = tensor_view(T, free_a, shared, E);
                        st.vb = dense_view(D, nw);
                    } else {           // b' = P_R . B_mat   (nw x D) (D x mb)
                        st.M = nw;
                        st.N = mb;
                        st.K = D;
                        st.va = dense_view(nw, D);
                        st.vb = tensor_view(T, shared, free_b, E);
                    }
                    add_gemm_flops(st);
                    TensorVer& out = side == 0 ? Ta2 : Tb2;
                    out.level = st.level;
                    out.buf = new_buf(out.size * w, BUF_TENSOR, st.level);
                    P->tens.push_back(out);
                    st.out_t = (int32_t)P->tens.size() - 1;
                    (side == 0 ? c.a_ver_out : c.b_ver_out) = st.out_t;
                    read_tensor(ver, st.level);
                    touch(st.proj_buf, st.level);
                    P->steps.push_back(st);
                }
                P->comps.push_back(c);
                live[a] = c.a_ver_out;
                live[b] = c.b_ver_out;
                if (o.grad) {
                    // a' = A P_L, b' = P_R B depend on (A, B) through K = A B only:
                    //   A_bar = G_a P_L^T + A N_A,   B_bar = P_R^T G_b + N_B B
                    // with H_A = A^T G_a, H_B = B G_b^T and the D x D matrices N_A, N_B from the core
                    BwdOp op;
                    op.comp = comp_id;
                    op.outs[0] = c.a_ver_out;
                    op.outs[1] = c.b_ver_out;
                    op.ins[0] = va;
                    op.ins[1] = vb;
                    const std::vector<int32_t> enew = {e_new};
                    const ViewSpec ga = tensor_view(P->tens[c.a_ver_out], free_a, enew, E);    // ma x nw
                    const ViewSpec gbt = tensor_view(P->tens[c.b_ver_out], free_b, enew, E);   // mb x nw
                    const ViewSpec gb = tensor_view(P->tens[c.b_ver_out], enew, free_b, E);    // nw x mb
                    const ViewSpec out_a = tensor_view(Ta, free_a, shared, E);                 // A's own layout
                    const ViewSpec out_b = tensor_view(Tb, shared, free_b, E);
                    CompBwd cb;
                    auto hsplits = [&](int64_t mm) {
                        int32_t sp = split_k(D, nw, mm, 16 << 20);
                        int64_t kps = (mm + sp - 1) / sp;
                        kps = (kps + kGemmK - 1) / kGemmK * kGemmK;
                        return std::make_pair((int32_t)((mm + kps - 1) / kps), (int32_t)kps);
                    };
                    const auto spa = hsplits(ma), spb = hsplits(mb);
                    cb.splits_a = spa.first;
                    cb.splits_b = spb.first;
                    cb.h_buf = new_buf((int64_t)(spa.first + spb.first) * D * nw * 8, BUF_BWD, 0);
                    cb.na_buf = new_buf(D * D * w, BUF_BWD, 0);
                    cb.nb_buf = new_buf(D * D * w, BUF_BWD, 0);
                    cb.work_buf = new_buf((9 * D * D + 6 * D * nw + 8 * D + 64) * 8, BUF_BWD, 0);
                    P->cbwd.push_back(cb);
                    auto hgemm = [&](int32_t tbuf, const ViewSpec& vt, int32_t gbuf, const ViewSpec& vg, int64_t mm,
                                     std::pair<int32_t, int32_t> sp, int32_t s_t, int32_t s_g, int64_t off) {
                        BStep g;
                        g.kind = BS_GEMM;
                        g.level = 1;
                        g.partial = 1;
                        g.a_buf = tbuf;
                        g.b_buf = gbuf;
                        g.c_buf = cb.h_buf;
                        g.c_off = off;
                        g.va = vt;
                        g.vb = vg;
                        g.M = D;
                        g.N = nw;
                        g.K = mm;
                        g.splits = sp.first;
                        g.k_per_split = sp.second;
                        g.scale_a = s_t;
                        g.scale_b = s_g;
                        g.flops = 2.0 * (double)D * nw * mm;
                        g.bytes = (double)w * (double)mm * (D + nw);
                        op.steps.push_back(g);
                    };
                    // H_A = A^T G_a / (s_A s_a'),  H_B = B G_b^T / (s_B s_b')
                    hgemm(Ta.buf, tensor_view(Ta, shared, free_a, E), adj_of(c.a_ver_out), ga, ma, spa, va,
                          c.a_ver_out, 0);
                    hgemm(Tb.buf, tensor_view(Tb, shared, free_b, E), adj_of(c.b_ver_out), gbt, mb, spb, vb,
                          c.b_ver_out, (int64_t)spa.first * D * nw * 8);
                    // first terms: A_bar = G_a P_L^T / s_a',  B_bar = P_R^T G_b / s_b'
                    bwd_gemm(op, 1, adj_of(c.a_ver_out), c.pl_buf, adj_of(va), ga, dense_view_t(D, nw), out_a, ma, D,
                             nw, c.a_ver_out, -1, 0, false);
                    bwd_gemm(op, 1, c.pr_buf, adj_of(c.b_ver_out), adj_of(vb), dense_view_t(nw, D), gb, out_b, D, mb,
                             nw, -1, c.b_ver_out, 0, false);
                    BStep core_b;
                    core_b.kind = BS_CORE_BWD;
                    core_b.level = 2;
                    core_b.comp = comp_id;
                    {
                        const double r = (double)std::min(ka, kb);
                        core_b.flops = 2.0 * D * r * (double)(ka + kb) + 4.0 * D * r * r + 4.0 * D * D * r;
                    }
                    op.steps.push_back(core_b);
                    // second terms, accumulated: A_bar += A N_A / s_A,  B_bar += N_B B / s_B
                    bwd_gemm(op, 3, Ta.buf, cb.na_buf, adj_of(va), tensor_view(Ta, free_a, shared, E),
                             dense_view(D, D), out_a, ma, D, D, va, -1, 1, false);
                    bwd_gemm(op, 3, cb.nb_buf, Tb.buf, adj_of(vb), dense_view(D, D), tensor_view(Tb, shared, free_b, E),
                             out_b, D, mb, D, -1, vb, 1, false);
                    op.done[0] = op.done[1] = 3;
                    bops.push_back(op);
                }
            } else {
                P->tens.push_back(Ta2);
                live[a] = (int32_t)P->tens.size() - 1;
                P->tens.push_back(Tb2);
                live[b] = (int32_t)P->tens.size() - 1;
            }
            for (int e : shared) E[e].alive = false;
        };
        // neighbour -> shared edges (in x's axis order) of the live tensor x, ascending neighbour id
        auto neighbours = [&](const int32_t x) {
            std::map<int32_t, std::vector<int32_t>> nb;
            for (int e : P->tens[live[x]].legs) nb[(E[e].end0 == x) ? E[e].end1 : E[e].end0].push_back(e);
            return nb;
        };
        if (o.late) {
            // late compression: before contracting i and j, every other bond of i, then of j,
            // larger than chi (Algorithm 1 with compress_late)
            for (const int32_t x : {i, j}) {
                const int32_t partner = x == i ? j : i;
                for (auto& kv : neighbours(x))
                    if (kv.first != partner && prod_dims(kv.second, E) > o.chi) compress_bond(x, kv.first);
            }
        }
        // ---------------------------------------------------------- CONTRACT(i, j) -> k
        {
            const int32_t vi = live[i], vj = live[j];
            const TensorVer Ti = P->tens[vi], Tj = P->tens[vj];
            std::vector<int32_t> shared, free_i, free_j;
            for (int e : Ti.legs) {
                if (std::find(Tj.legs.begin(), Tj.legs.end(), e) != Tj.legs.end()) shared.push_back(e);
                else free_i.push_back(e);
            }
            for (int e : Tj.legs)
                if (std::find(shared.begin(), shared.end(), e) == shared.end()) free_j.push_back(e);
            const int64_t m = prod_dims(free_i, E), s = prod_dims(shared, E), q = prod_dims(free_j, E);
            if (m * q > kMaxElems) {
                os << "step " << t << ": intermediate of " << m * q << " elements exceeds 2^31-1";
                return os.str();
            }
            P->ops.push_back({0, i, j, k, m, s, q, 0});
            TensorVer Tk;
            Tk.legs = free_i;
            Tk.legs.insert(Tk.legs.end(), free_j.begin(), free_j.end());
            Tk.size = m * q;
            if (!shapes_only) {
                Step st;
                st.kind = ST_CONTRACT;
                st.level = 1 + std::max(Ti.level, Tj.level);
                // ordered levelling: a tree step starts no earlier than the last level of the one
                // before it (its compressions included), so independent branches do not all hold
                // their uncompressed intermediates at once: the memory of a sequential run
                if (o.ordered) st.level = std::max(st.level, last_step_level);
                st.in_a = vi;
                st.in_b = vj;
                st.M = m;
                st.N = q;
                st.K = s;
                st.va = tensor_view(Ti, free_i, shared, E);
                st.vb = tensor_view(Tj, shared, free_j, E);
                add_gemm_flops(st);
                Tk.level = st.level;
                Tk.buf = new_buf(Tk.size * w, BUF_TENSOR, st.level);
                P->tens.push_back(Tk);
                st.out_t = (int32_t)P->tens.size() - 1;
                read_tensor(vi, st.level);
                read_tensor(vj, st.level);
                P->steps.push_back(st);
                if (o.grad) {
                    // C = A B:  A_bar = C_bar B^T / (s_C s_B),  B_bar = A^T C_bar / (s_A s_C)
                    BwdOp op;
                    op.outs[0] = st.out_t;
                    op.ins[0] = vi;
                    op.ins[1] = vj;
                    const ViewSpec cbar = tensor_view(P->tens[st.out_t], free_i, free_j, E);
                    op.done[0] = bwd_gemm(op, 1, adj_of(st.out_t), Tj.buf, adj_of(vi), cbar,
                                          tensor_view(Tj, free_j, shared, E), st.va, m, s, q, st.out_t, vj, 0, true);
                    op.done[1] = bwd_gemm(op, 1, Ti.buf, adj_of(st.out_t), adj_of(vj),
                                          tensor_view(Ti, shared, free_i, E), cbar, st.vb, s, q, m, vi, st.out_t, 0,
                                          true);
                    bops.push_back(op);
                }
            } else {
                P->tens.push_back(Tk);
            }
            for (int e : shared) E[e].alive = false;
            for (int e : free_i) (E[e].end0 == i ? E[e].end0 : E[e].end1) = k;
            for (int e : free_j) (E[e].end0 == j ? E[e].end0 : E[e].end1) = k;
            live[i] = live[j] = -1;
            live[k] = (int32_t)P->tens.size() - 1;
        }
        // ---------------------------------------------------------- early compression of k's bonds
        if (!o.late)
            for (auto& kv : neighbours(k))
                if (prod_dims(kv.second, E) > o.chi) compress_bond(k, kv.first);
    }
    int32_t last = -1;
    for (int id = 0; id < total_ids; ++id)
        if (live[id] >= 0) last = live[id];
    P->final_tensor = last;
    if (shapes_only) return "";
    if (P->tens[last].size != 1) return "the tree does not reduce the network to a scalar";

    // ---------------------------------------------------------- levels, per-tile max slots
    int32_t maxl = 0;
    for (auto& s : P->steps) maxl = std::max(maxl, s.level);
    P->n_levels = maxl;
    for (auto& b : P->bufs)
        if (b.kind == BUF_INPUT) b.hi = INT_MAX;
    // the final tensor is read by the result kernel after the last level
    P->bufs[P->tens[last].buf].hi = INT_MAX;

    // ---------------------------------------------------------- reverse pass: what each op reads
    // A reverse op belongs to the forward level of the outputs of its forward op; the forward
    // buffers it reads (operands, core workspace, projectors) are kept at least to that level.
    std::vector<int32_t> bop_level(bops.size(), 0);
    std::vector<uint8_t> bwd_read(P->bufs.size(), 0);
    if (o.grad) {
        for (size_t k = 0; k < bops.size(); ++k) {
            int32_t Lb = 0;
            for (int32_t v : bops[k].outs)
                if (v >= 0) Lb = std::max(Lb, P->tens[v].level);
            bop_level[k] = Lb;
            auto reads = [&](int32_t b) {
                if (b < 0 || P->bufs[b].kind == BUF_BWD) return;
                bwd_read[b] = 1;
                touch(b, Lb);
            };
            for (const BStep& st : bops[k].steps) {
                if (st.kind == BS_GEMM) {
                    reads(st.a_buf);
                    reads(st.b_buf);
                } else if (st.kind == BS_CORE_BWD) {
                    reads(P->comps[bops[k].comp].work_buf);
                }
            }
        }
    }
    std::vector<int32_t> hi0(P->bufs.size());
    for (size_t b = 0; b < P->bufs.size(); ++b) hi0[b] = P->bufs[b].hi;

    // Lay out the arena for `want` segments (grad; 1 = every forward buffer resident) and return
    // its size.  Forward buffers: a buffer live across a segment boundary, or the last level, is
    // kept to the end (a checkpoint); one that lives inside a segment and is read by the reverse
    // pass is kept to the end of its segment; the rest are freed after their last forward read.
    // So at the last level of segment s everything the re-run of s and its reverse ops read is
    // live at once, at disjoint offsets, and a re-run of s writes only over buffers of segment s
    // and of later segments, whose reverse ops are done.  Reverse-pass buffers sit above the
    // forward arena, allocated by reverse level and freed after their last use.
    auto layout = [&](int32_t want) -> int64_t {
        for (size_t b = 0; b < P->bufs.size(); ++b) P->bufs[b].hi = hi0[b];
        P->bsteps.clear();
        P->seg_begin.clear();
        P->seg_bend.clear();
        P->seg_recompute.clear();
        P->recompute_flops = 0;
        P->checkpoint_bytes = 0;
        std::vector<int32_t> sb{1, maxl + 1};
        if (o.grad && want > 1) sb = segment_starts(P->bufs, maxl, want);
        const int32_t S = (int32_t)sb.size() - 1;
        P->n_segments = S;
        auto seg_of = [&](int32_t L) {
            return (int32_t)(std::upper_bound(sb.begin(), sb.end(), L) - sb.begin()) - 1;
        };
        if (o.grad && S == 1) {
            for (auto& b : P->bufs)
                if (b.kind == BUF_TENSOR || b.kind == BUF_WORK || b.kind == BUF_PROJ) b.hi = INT_MAX;
        } else if (o.grad) {
            for (size_t b = 0; b < P->bufs.size(); ++b) {
                Buf& B = P->bufs[b];
                if (B.kind == BUF_INPUT || B.kind == BUF_BWD || B.hi == INT_MAX) continue;
                const int32_t s0 = seg_of(std::max(B.lo, 1));
                if (B.hi > maxl || seg_of(B.hi) > s0) {
                    B.hi = INT_MAX;
                    P->checkpoint_bytes += B.bytes;
                } else if (bwd_read[b]) {
                    B.hi = sb[s0 + 1] - 1;
                }
            }
        }
        // forward arena: allocate by level, free after last use
        std::vector<std::vector<int32_t>> starts(maxl + 1), ends(maxl + 1);
        for (int32_t b = 0; b < (int32_t)P->bufs.size(); ++b) {
            const Buf& B = P->bufs[b];
            if (B.kind == BUF_BWD) continue;
            starts[std::min(B.lo, maxl)].push_back(b);
            if (B.hi != INT_MAX) ends[std::min(B.hi, maxl)].push_back(b);
        }
        FreeList fwd(0);
        for (int L = 0; L <= maxl; ++L) {
            // largest first for less fragmentation
            std::sort(starts[L].begin(), starts[L].end(),
                      [&](int32_t x, int32_t y) { return P->bufs[x].bytes > P->bufs[y].bytes; });
            for (int32_t b : starts[L]) P->bufs[b].off = fwd.alloc(P->bufs[b].bytes);
            if (!o.keep)
                for (int32_t b : ends[L]) fwd.release(P->bufs[b].off, P->bufs[b].bytes);
        }
        if (!o.grad) return fwd.top;
        // reverse levels: segments last to first; inside one, ops in reverse creation order, each
        // as soon as the adjoints of its outputs are complete (consumers come later in creation
        // order and in the same or a later segment)
        std::vector<int32_t> ready(P->tens.size(), 0);
        BStep seed;
        seed.kind = BS_SEED;
        seed.level = 1;
        P->bsteps.push_back(seed);
        ready[last] = 1;
        int32_t maxb = 1;
        P->seg_bend.assign(S, 0);
        P->seg_recompute.assign(S, 0);
        for (int32_t s = S - 1; s >= 0; --s) {
            const int32_t base = s == S - 1 ? 0 : maxb;
            for (size_t k = bops.size(); k-- > 0;) {
                if (seg_of(bop_level[k]) != s) continue;
                const BwdOp& op = bops[k];
                int32_t L0 = base;
                for (int32_t v : op.outs)
                    if (v >= 0) L0 = std::max(L0, ready[v]);
                for (BStep st : op.steps) {
                    st.level += L0;
                    if (st.kind == BS_CORE_BWD) st.comp = op.comp;
                    maxb = std::max(maxb, st.level);
                    P->bsteps.push_back(st);
                }
                for (int t = 0; t < 2; ++t)
                    if (op.ins[t] >= 0) ready[op.ins[t]] = L0 + op.done[t];
                P->seg_recompute[s] = 1;
            }
            P->seg_bend[s] = maxb;
        }
        P->n_blevels = maxb;
        for (auto& st : P->steps)
            if (seg_of(st.level) < S - 1 && P->seg_recompute[seg_of(st.level)]) P->recompute_flops += st.flops;
        P->seg_begin = sb;
        // reverse-pass buffers: live from their first to their last reverse level; adjoints of
        // the inputs are read after the last level (by the gradient copy-out)
        std::vector<int32_t> rlo(P->bufs.size(), INT_MAX), rhi(P->bufs.size(), -1);
        auto use = [&](int32_t b, int32_t L) {
            if (b < 0 || P->bufs[b].kind != BUF_BWD) return;
            rlo[b] = std::min(rlo[b], L);
            rhi[b] = std::max(rhi[b], L);
        };
        for (const BStep& st : P->bsteps) {
            if (st.kind == BS_SEED) {
                use(P->adj_buf[last], st.level);
            } else if (st.kind == BS_CORE_BWD) {
                const CompBwd& cb = P->cbwd[st.comp];
                for (int32_t b : {cb.h_buf, cb.na_buf, cb.nb_buf, cb.work_buf}) use(b, st.level);
            } else {
                use(st.a_buf, st.level);
                use(st.b_buf, st.level);
                use(st.c_buf, st.level);
            }
        }
        for (int v = 0; v < g.n && v < (int)P->adj_buf.size(); ++v)
            if (P->adj_buf[v] >= 0) rhi[P->adj_buf[v]] = INT_MAX;
        std::vector<std::vector<int32_t>> rstarts(maxb + 1), rends(maxb + 1);
        for (int32_t b = 0; b < (int32_t)P->bufs.size(); ++b) {
            if (P->bufs[b].kind != BUF_BWD) continue;
            if (rlo[b] == INT_MAX) rlo[b] = 1;   // never touched: any slot will do
            if (rhi[b] < 0) rhi[b] = rlo[b];
            rstarts[std::min(rlo[b], maxb)].push_back(b);
            if (rhi[b] != INT_MAX) rends[std::min(rhi[b], maxb)].push_back(b);
        }
        FreeList rev(fwd.top);
        for (int L = 0; L <= maxb; ++L) {
            std::sort(rstarts[L].begin(), rstarts[L].end(),
                      [&](int32_t x, int32_t y) { return P->bufs[x].bytes > P->bufs[y].bytes; });
            for (int32_t b : rstarts[L]) P->bufs[b].off = rev.alloc(P->bufs[b].bytes);
            for (int32_t b : rends[L]) rev.release(P->bufs[b].off, P->bufs[b].bytes);
        }
        return rev.top;
    };
    int32_t want = o.grad ? std::max(o.segments, 1) : 1;
    if (o.grad && o.segments < 0) {
        // the candidate count of smallest arena (ties: fewer segments, less re-running)
        int64_t best = -1;
        for (int32_t cand : {1, 2, 3, 4, 6, 8, 12, 16, 24, 32}) {
            if (cand > 1 && cand > maxl) break;
            const int64_t bytes = layout(cand);
            if (best < 0 || bytes < best) {
                best = bytes;
                want = cand;
            }
        }
    }
    int64_t top = layout(want);
    if (o.grad)
        for (auto& st : P->bsteps) {
            P->bwd_flops += st.flops;
            P->bwd_bytes += st.bytes;
        }
    P->arena_bytes = top;

    // ---------------------------------------------------------- totals
    for (auto& s : P->steps) {
        P->fwd_flops += s.flops;
        P->fwd_bytes += s.bytes;
    }
    for (auto& s : P->steps) {
        if (s.kind == ST_CONTRACT || s.kind == ST_ABSORB) {
            // GEMM views are validated here so that errors surface at planning time
            View v;
            std::string err = make_view(s.va, &v);
            if (err.empty()) err = make_view(s.vb, &v);
            if (!err.empty()) return err;
        } else if (s.kind == ST_GRAM || s.kind == ST_COPY || s.kind == ST_TSQR) {
            View v;
            std::string err = make_view(s.va, &v);
            if (err.empty() && s.kind == ST_GRAM) err = make_view(s.vb, &v);
            if (!err.empty()) return err;
        } else if (s.kind == ST_GAUGE) {
            View v;
            std::string err = make_view(s.va, &v);
            if (err.empty()) err = make_view(s.vb, &v);
            if (err.empty() && s.gauge_mode == GAUGE_APPLY) err = make_view(s.vc, &v);
            if (!err.empty()) return err;
        }
    }
    if (o.budget > 0 && P->arena_bytes > o.budget) {
        os << "plan needs " << P->arena_bytes << " device bytes, budget is " << o.budget;
        return os.str();
    }
    return "";
}

}  // namespace tn
