// C-ABI of libphylograd: context, input checks, tree schedule, device
// buffers and the evaluation sequence.  Declarations and the contract of
// every entry point are in include/phylograd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <map>
#include <string>
#include <vector>

#include "pg_internal.h"

using namespace pg;

namespace {

thread_local std::string g_create_error;

struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct pg_ctx {
    int device = 0;
    int precision = PG_FP64;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    std::string err;

    // tree
    bool tree_set = false;
    int n_tips = 0;
    std::vector<int> parent;
    std::vector<int2> children;
    std::vector<int> level_off, level_nodes;
    std::vector<int> height;                  // [2N-1] tips 0, cherries 1, ...

    // patterns
    bool patterns_set = false;
    int S = 0, S_pad = 0, m_pat = 0;
    std::vector<uint8_t> codes;               // [N][S_pad]
    std::vector<unsigned long long> masks;    // [256]
    std::vector<double> weights;              // [S_pad]

    // model
    bool model_set = false;
    int m = 0, K = 0;
    std::vector<double> Q, Q2, pi, rates, catw;
    double qnorm = 0.0;
    // split-BF16 path: eigen-decomposition of Q padded to MP states, and Q
    // as MFMA A operands (three BF16 parts)
    std::vector<double> eV, eVinv, eRe, eIm;
    std::vector<int> eKind;
    bool expm_taylor = false;
    double eig_cond = 0.0, eig_resid = 0.0;
    std::vector<uint16_t> Qop;
    // non-homogeneous model: branch b uses bm_Q[bm_model[b]] (bm_n = 0: off)
    int bm_n = 0;
    std::vector<double> bm_Q, bm_Q2, bm_qnorm;
    std::vector<int> bm_model;

    // device state
    bool dev_stale = true;        // host inputs changed since the last upload
    bool have_partials = false;   // post-order pass results resident
    // partial re-evaluation: host copy of the branch lengths of the resident
    // partials (host-pointer evaluations only) and per-node exponents
    std::vector<double> t_host;
    bool t_host_valid = false;
    bool updates = false;
    void* u_pinned = nullptr;     // pinned staging of one update's inputs
    size_t u_pinned_bytes = 0;
    bool u_inflight = false;      // a copy out of u_pinned may still run
    bool device_pending = false;  // a device-pointer evaluation was enqueued
    std::map<std::string, DevBuf> bufs;
    EvalArgs args{};

    // device allocator (default hipMalloc/hipFree; the serving scheduler
    // supplies a pool so sessions reuse each other's memory)
    DeviceAllocator* allocator = nullptr;

    // timing: event pairs recorded around kernels, read after the stream
    // passes them (no synchronisation between kernels)
    bool timing = false;
    double ms[PG_K_COUNT] = {0};
    int64_t launches[PG_K_COUNT] = {0};
    std::vector<hipEvent_t> ev_pool;
    struct Pending { int kid; hipEvent_t a, b; };
    std::vector<Pending> pending;
};

namespace {

int fail(pg_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

int hip_fail(pg_ctx* c, hipError_t e, const char* where) {
    std::string msg = std::string(where) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory) return fail(c, PG_E_OOM, msg);
    return fail(c, PG_E_DEVICE, msg);
}

#define PG_HIP(c, call)                                     \
    do {                                                    \
        hipError_t _e = (call);                             \
        if (_e != hipSuccess) return hip_fail((c), _e, #call); \
    } while (0)

int ensure_buf(pg_ctx* c, const char* name, size_t bytes) {
    DevBuf& b = c->bufs[name];
    if (b.bytes >= bytes && b.ptr) return PG_OK;
    if (b.ptr) {
        if (c->allocator) {
            c->allocator->release(b.ptr, b.bytes);
        } else {
            hipError_t e = hipFree(b.ptr);
            if (e != hipSuccess) return hip_fail(c, e, "hipFree");
        }
        b.ptr = nullptr;
        b.bytes = 0;
    }
    void* p = nullptr;
    if (c->allocator) {
        p = c->allocator->acquire(std::max<size_t>(bytes, 256));
        if (!p) return fail(c, PG_E_OOM, "device pool allocation failed");
    } else {
        hipError_t e = hipMalloc(&p, std::max<size_t>(bytes, 256));
        if (e != hipSuccess) return hip_fail(c, e, "hipMalloc");
    }
    b.ptr = p;
    b.bytes = std::max<size_t>(bytes, 256);
    return PG_OK;
}

template <typename X>
X* buf(pg_ctx* c, const char* name) {
    return static_cast<X*>(c->bufs[name].ptr);
}

size_t elem_size(int precision) { return precision == PG_FP64 ? 8 : 4; }

// BF16 bits of x, rounded to nearest even (finite x).
uint16_t bf16_bits(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
float bf16_value(uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float x;
    std::memcpy(&x, &u, 4);
    return x;
}

// Split-BF16 model data: eigen-decomposition of Q padded to MP states (the
// padding is identity in V and V^-1 with eigenvalue 0), and Q's MFMA A
// operands [mt][ks][part][lane][j] in three BF16 parts, row 16 mt + lane % 16,
// column 16 (2 ks + j / 4) + 4 (lane / 16) + j % 4 (the kernels' state order
// of the contraction index).
void prepare_split_model(pg_ctx* c) {
    const int m = c->m;
    EigenSystem es;
    const bool ok = eigen_decompose(m, c->Q.data(), es);
    c->eV.assign(MP * MP, 0.0);
    c->eVinv.assign(MP * MP, 0.0);
    c->eRe.assign(MP, 0.0);
    c->eIm.assign(MP, 0.0);
    c->eKind.assign(MP, 0);
    for (int i = 0; i < MP; ++i) c->eV[i * MP + i] = c->eVinv[i * MP + i] = 1.0;
    // one product with a V of condition up to 1e6 keeps F = P - I to about
    // 1e-10 relative, far below what the FP32 path resolves
    c->expm_taylor = !(ok && es.cond <= 1e6 && es.resid <= 1e-11);
    c->eig_cond = ok ? es.cond : INFINITY;
    c->eig_resid = ok ? es.resid : INFINITY;
    if (!c->expm_taylor) {
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                c->eV[i * MP + j] = es.V[i * m + j];
                c->eVinv[i * MP + j] = es.Vinv[i * m + j];
            }
        for (int j = 0; j < m; ++j) {
            c->eRe[j] = es.re[j];
            c->eIm[j] = es.im[j];
            c->eKind[j] = es.kind[j];
        }
    }
    c->Qop.assign(MF_QOP_BYTES / 2, 0);
    for (int mt = 0; mt < 4; ++mt)
        for (int ks = 0; ks < 2; ++ks)
            for (int lane = 0; lane < 64; ++lane)
                for (int j = 0; j < 8; ++j) {
                    const int r = 16 * mt + lane % 16;
                    const int y = 16 * (2 * ks + j / 4) + 4 * (lane / 16) + j % 4;
                    const double v = (r < m && y < m) ? c->Q[r * m + y] : 0.0;
                    const uint16_t hi = bf16_bits((float)v);
                    const double r1 = v - (double)bf16_value(hi);
                    const uint16_t mid = bf16_bits((float)r1);
                    const uint16_t lo = bf16_bits((float)(r1 - (double)bf16_value(mid)));
                    const uint16_t parts[3] = {hi, mid, lo};
                    for (int part = 0; part < 3; ++part)
                        c->Qop[((((mt * 2 + ks) * 3 + part) * 64 + lane) * 8) + j] = parts[part];
                }
}

// Internal nodes grouped by height (tips have height 0); nodes of one level
// have no ancestor relation, so a level is processed in parallel and the
// levels in increasing order form a post-order (decreasing: a pre-order).
void build_levels(pg_ctx* c) {
    const int N = c->n_tips, n_nodes = 2 * N - 1;
    std::vector<int> height(n_nodes, 0);
    // internal nodes: repeat relaxation in label-free order via explicit stack
    std::vector<int> order;
    order.reserve(N - 1);
    std::vector<int> stack{n_nodes - 1};
    std::vector<char> expanded(n_nodes, 0);
    while (!stack.empty()) {
        int v = stack.back();
        if (v < N) { stack.pop_back(); continue; }
        if (!expanded[v]) {
            expanded[v] = 1;
            stack.push_back(c->children[v].x);
            stack.push_back(c->children[v].y);
        } else {
            stack.pop_back();
            height[v] = 1 + std::max(height[c->children[v].x], height[c->children[v].y]);
            order.push_back(v);
        }
    }
    int H = 0;
    for (int v : order) H = std::max(H, height[v]);
    c->level_off.assign(H + 1, 0);
    std::vector<int> count(H + 1, 0);
    for (int v : order) count[height[v]]++;
    // level h (1..H) stored at index h-1
    c->level_off.assign(H + 1, 0);
    for (int h = 1; h <= H; ++h) c->level_off[h] = c->level_off[h - 1] + count[h];
    c->level_nodes.assign(N - 1, 0);
    std::vector<int> fill(c->level_off.begin(), c->level_off.end() - 1);
    // within a level: nodes with two internal children, then one, then none,
    // each group by label.  Consecutive node slots share a wavefront, so the
    // grouping keeps the tip and internal child paths of the kernels from
    // both running in one wavefront for most of the level.
    std::vector<int> sorted(order);
    auto n_tip_children = [&](int v) { return (c->children[v].x < N) + (c->children[v].y < N); };
    std::sort(sorted.begin(), sorted.end(), [&](int u, int v) {
        const int cu = n_tip_children(u), cv = n_tip_children(v);
        return cu != cv ? cu < cv : u < v;
    });
    for (int v : sorted) c->level_nodes[fill[height[v] - 1]++] = v;
    c->height.swap(height);
}

// Traversal schedule of one upload: the level-synchronous part (the top:
// every internal node outside the clades, grouped by height within the top)
// and the clade walks, one list per slot count.
struct Schedule {
    std::vector<int> level_off;       // [H + 1] top levels
    std::vector<int> level_nodes;     // top nodes by level
    std::vector<int4> cl_post, cl_pre;
    std::vector<int> cl_post_off, cl_pre_off;
    int depth = 0;                    // stack blocks per slot
};

// LPT assignment of clades to ns slots (largest clade to the least loaded
// slot); entries slot-major.
void assign_clades(const std::vector<std::vector<int4>>& clades, int ns, std::vector<int4>& out,
                   std::vector<int>& off) {
    std::vector<int> order(clades.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int u, int v) { return clades[u].size() > clades[v].size(); });
    std::vector<size_t> load(ns, 0);
    std::vector<std::vector<int>> bins(ns);
    for (int ci : order) {
        const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[b] += clades[ci].size();
        bins[b].push_back(ci);
    }
    out.clear();
    off.assign(ns + 1, 0);
    for (int b = 0; b < ns; ++b) {
        for (int ci : bins[b]) out.insert(out.end(), clades[ci].begin(), clades[ci].end());
        off[b + 1] = (int)out.size();
    }
}

// cap = 0: no clades (every internal node in the levels).
void build_schedule(const pg_ctx* c, int cap, int ns_post, int ns_pre, Schedule& sc) {
    const int N = c->n_tips, n_nodes = 2 * N - 1, root = n_nodes - 1;
    const auto& ch = c->children;
    // internal nodes in increasing height: children before parents
    const std::vector<int>& up = c->level_nodes;
    std::vector<int> sz(n_nodes, 0);  // internal nodes in the subtree
    for (int v : up) sz[v] = 1 + sz[ch[v].x] + sz[ch[v].y];
    // clade of each internal node (its clade root), -1 for the top
    std::vector<int> clade(n_nodes, -1);
    std::vector<int> roots;
    for (auto it = up.rbegin(); it != up.rend(); ++it) {
        const int v = *it;
        if (v == root) continue;
        const int p = c->parent[v];
        if (clade[p] >= 0) {
            clade[v] = clade[p];
        } else if (sz[v] <= cap) {
            clade[v] = v;
            roots.push_back(v);
        }
    }
    // top levels: height counted over top nodes only
    std::vector<int> th(n_nodes, 0);
    int H = 0;
    for (int v : up) {
        if (clade[v] >= 0) continue;
        int h = 0;
        for (int cc : {ch[v].x, ch[v].y})
            if (cc >= N && clade[cc] < 0) h = std::max(h, th[cc]);
        th[v] = h + 1;
        H = std::max(H, th[v]);
    }
    std::vector<int> count(H + 1, 0), top;
    for (int v : up)
        if (clade[v] < 0) {
            count[th[v]]++;
            top.push_back(v);
        }
    sc.level_off.assign(H + 1, 0);
    for (int h = 1; h <= H; ++h) sc.level_off[h] = sc.level_off[h - 1] + count[h];
    // within a level: nodes with two internal children, then one, then none,
    // each group by label.  Consecutive node slots share a wavefront, so the
    // grouping keeps the tip and internal child paths of the kernels from
    // both running in one wavefront for most of the level.
    auto n_tip_children = [&](int v) { return (ch[v].x < N) + (ch[v].y < N); };
    std::sort(top.begin(), top.end(), [&](int u, int v) {
        const int cu = n_tip_children(u), cv = n_tip_children(v);
        return cu != cv ? cu < cv : u < v;
    });
    sc.level_nodes.assign(top.size(), 0);
    std::vector<int> fill(sc.level_off.begin(), sc.level_off.end() - 1);
    for (int v : top) sc.level_nodes[fill[th[v] - 1]++] = v;
    // clade entries in post order, the child with more internal nodes first
    auto ordered = [&](int v) {
        int f = ch[v].x, g = ch[v].y;
        if (sz[g] > sz[f]) std::swap(f, g);
        return std::make_pair(f, g);
    };
    std::sort(roots.begin(), roots.end());
    std::vector<std::vector<int4>> lists;
    sc.depth = 0;
    for (int r : roots) {
        std::vector<int4> e;
        std::vector<std::pair<int, bool>> st{{r, false}};
        while (!st.empty()) {
            const auto [v, done] = st.back();
            st.pop_back();
            const auto [f, g] = ordered(v);
            if (done) {
                int flags = 0;
                if (v == r) {
                    flags = CL_ROOT;
                } else {
                    const auto [pf, pg2] = ordered(c->parent[v]);
                    if (v == pf && pg2 >= N) flags = CL_STACK;
                }
                e.push_back(make_int4(v, f, g, flags));
                continue;
            }
            st.push_back({v, true});
            if (g >= N) st.push_back({g, false});
            if (f >= N) st.push_back({f, false});
        }
        // stack depth of the walk (pops before pushes within an entry)
        int sp = 0;
        for (const int4& x : e) {
            if (x.y >= N && x.z >= N) --sp;
            if (x.w & CL_STACK) ++sp;
            sc.depth = std::max(sc.depth, sp);
        }
        lists.push_back(std::move(e));
    }
    assign_clades(lists, ns_post, sc.cl_post, sc.cl_post_off);
    assign_clades(lists, ns_pre, sc.cl_pre, sc.cl_pre_off);
}

int check_tree(pg_ctx* c, int32_t N, const int32_t* parent) {
    const int n_nodes = 2 * N - 1;
    const int root = n_nodes - 1;
    if (parent[root] != -1) return fail(c, PG_E_TREE, "parent[2N-2] must be -1 (root last)");
    std::vector<int> nchild(n_nodes, 0);
    std::vector<int2> ch(n_nodes, make_int2(-1, -1));
    for (int v = 0; v < root; ++v) {
        const int p = parent[v];
        if (p < N || p >= n_nodes)
            return fail(c, PG_E_TREE, "node " + std::to_string(v) + " has parent " +
                                          std::to_string(p) + " outside the internal nodes");
        if (nchild[p] == 0) ch[p].x = v;
        else if (nchild[p] == 1) ch[p].y = v;
        nchild[p]++;
    }
    for (int k = N; k < n_nodes; ++k)
        if (nchild[k] != 2)
            return fail(c, PG_E_TREE, "internal node " + std::to_string(k) + " has " +
                                          std::to_string(nchild[k]) + " children (binary tree required)");
    // every node reaches the root: walk up with a step bound (cycle check)
    std::vector<char> ok(n_nodes, 0);
    ok[root] = 1;
    for (int v = 0; v < n_nodes; ++v) {
        std::vector<int> path;
        int u = v;
        int steps = 0;
        while (!ok[u]) {
            path.push_back(u);
            u = parent[u];
            if (++steps > n_nodes) return fail(c, PG_E_TREE, "the parent array has a cycle");
        }
        for (int w : path) ok[w] = 1;
    }
    c->children = ch;
    return PG_OK;
}

int upload(pg_ctx* c) {
    if (!c->tree_set || !c->patterns_set || !c->model_set)
        return fail(c, PG_E_STATE, "tree, patterns and model must all be set before evaluating");
    if (c->m_pat != c->m)
        return fail(c, PG_E_STATE, "patterns have " + std::to_string(c->m_pat) +
                                       " states but the model has " + std::to_string(c->m));
    if (!c->dev_stale) return PG_OK;
    PG_HIP(c, hipSetDevice(c->device));
    const int N = c->n_tips, n_nodes = 2 * N - 1, B = n_nodes - 1;
    const int M = c->m, K = c->K;
    const size_t es = elem_size(c->precision);
    const bool split = c->precision == PG_SPLIT_BF16;
    const int n_pb = c->S_pad / TP;
    const int n_tiles = K * n_pb;
    const size_t vec = (size_t)K * (split ? MP : M) * c->S_pad;
    int r;
    if ((r = ensure_buf(c, "t", sizeof(double) * B))) return r;
    if ((r = ensure_buf(c, "P", split ? MF_SLOT_BYTES * (size_t)B * K : es * (size_t)B * K * M * M))) return r;
    if (split) {
        if ((r = ensure_buf(c, "eV", sizeof(double) * MP * MP))) return r;
        if ((r = ensure_buf(c, "eVinv", sizeof(double) * MP * MP))) return r;
        if ((r = ensure_buf(c, "eRe", sizeof(double) * MP))) return r;
        if ((r = ensure_buf(c, "eIm", sizeof(double) * MP))) return r;
        if ((r = ensure_buf(c, "eKind", sizeof(int) * MP))) return r;
        if ((r = ensure_buf(c, "Qop", MF_QOP_BYTES))) return r;
    }
    if ((r = ensure_buf(c, "msg", es * vec * (N - 1)))) return r;
    if ((r = ensure_buf(c, "qv", es * vec * (N - 1)))) return r;
    if ((r = ensure_buf(c, "codes", (size_t)N * c->S_pad))) return r;
    if ((r = ensure_buf(c, "masks", sizeof(unsigned long long) * 256))) return r;
    // traversal schedule: clades for the small-M FP64 / FP32 kernels, with a
    // smaller cap when a deep clade's stack would not fit CLADE_STACK_MAX
    const int ns_post = split ? node_slots(M) : post_node_slots(M, c->precision);
    const int ns_pre = split ? ns_post : pre_node_slots(M, c->precision);
    // The clade cap is chosen per tree among a few sizes: larger clades mean
    // fewer level-walk iterations above them (each ends at a barrier), but
    // fewer clades to balance over the slots and deeper stacks.  Cost
    // estimate: the busiest pre-order slot's clade entries plus twice the
    // top's level iterations; caps whose stacks exceed CLADE_STACK_MAX are
    // skipped.
    Schedule sc;
    if (!split && M * M <= TP) {
        long best = -1;
        for (int cap : {64, 48, 32, 24, 16}) {
            if (cap > CLADE_CAP) continue;
            Schedule t;
            build_schedule(c, cap, ns_post, ns_pre, t);
            if (es * std::max(ns_post, ns_pre) * t.depth * M * TP > (size_t)CLADE_STACK_MAX) continue;
            long busiest = 0, top_iters = 0;
            for (int b = 0; b < ns_pre; ++b) busiest = std::max<long>(busiest, t.cl_pre_off[b + 1] - t.cl_pre_off[b]);
            for (size_t h = 0; h + 1 < t.level_off.size(); ++h)
                top_iters += (t.level_off[h + 1] - t.level_off[h] + ns_pre - 1) / ns_pre;
            const long cost = busiest + 2 * top_iters;
            if (best < 0 || cost < best) {
                best = cost;
                sc = std::move(t);
            }
        }
        if (best < 0) build_schedule(c, 0, ns_post, ns_pre, sc);
    } else {
        build_schedule(c, 0, ns_post, ns_pre, sc);
    }
    const int n_top = (int)sc.level_nodes.size(), n_cl = (int)sc.cl_post.size();
    const bool one_list = ns_post == ns_pre;
    const size_t n_entries = (size_t)n_top + n_cl * (one_list ? 1 : 2);
    if ((r = ensure_buf(c, "level_off", sizeof(int) * sc.level_off.size()))) return r;
    if ((r = ensure_buf(c, "sched", sizeof(int4) * n_entries))) return r;
    if ((r = ensure_buf(c, "cl_off", sizeof(int) * (ns_post + ns_pre + 2)))) return r;
    if ((r = ensure_buf(c, "Q64", sizeof(double) * M * M))) return r;
    if ((r = ensure_buf(c, "Q2_64", sizeof(double) * M * M))) return r;
    if ((r = ensure_buf(c, "pi64", sizeof(double) * M))) return r;
    if ((r = ensure_buf(c, "rates", sizeof(double) * K))) return r;
    if ((r = ensure_buf(c, "catw", sizeof(double) * K))) return r;
    if ((r = ensure_buf(c, "weights", sizeof(double) * c->S_pad))) return r;
    if ((r = ensure_buf(c, "rootL", sizeof(double) * K * c->S_pad))) return r;
    if ((r = ensure_buf(c, "rootE", sizeof(int) * K * c->S_pad))) return r;
    if ((r = ensure_buf(c, "partial", sizeof(double) * (size_t)n_tiles * B))) return r;
    if ((r = ensure_buf(c, "partial2", sizeof(double) * (size_t)n_tiles * B))) return r;
    if ((r = ensure_buf(c, "logl_part", sizeof(double) * (size_t)n_pb))) return r;
    if ((r = ensure_buf(c, "flag_part", sizeof(int) * (size_t)n_pb))) return r;
    if ((r = ensure_buf(c, "grad", sizeof(double) * B))) return r;
    if ((r = ensure_buf(c, "hess", sizeof(double) * B))) return r;
    if ((r = ensure_buf(c, "logL", sizeof(double) * 2))) return r;
    if ((r = ensure_buf(c, "status", sizeof(int) * 2))) return r;
    if (c->bm_n > 0) {
        if ((r = ensure_buf(c, "bm_Q", sizeof(double) * c->bm_Q.size()))) return r;
        if ((r = ensure_buf(c, "bm_Q2", sizeof(double) * c->bm_Q2.size()))) return r;
        if ((r = ensure_buf(c, "bm_qnorm", sizeof(double) * c->bm_qnorm.size()))) return r;
        if ((r = ensure_buf(c, "bm_model", sizeof(int) * c->bm_model.size()))) return r;
    }

    hipStream_t st = c->stream;
    auto put = [&](const char* name, const void* src, size_t bytes) {
        return hipMemcpyAsync(c->bufs[name].ptr, src, bytes, hipMemcpyHostToDevice, st);
    };
    // pre-order top region: levels from the root down while every level has
    // at most TOP_LEVEL_MAX_NODES nodes and their q vectors fit TOP_LDS_MAX
    const int H = (int)sc.level_off.size() - 1;
    const int top_cap = std::min<int>(255, TOP_LDS_MAX / (int)(es * M * TP));
    int top_level = H, top_nodes = 0;
    for (int h = H - 1; h >= 0 && !split; --h) {
        const int n_h = sc.level_off[h + 1] - sc.level_off[h];
        if (n_h > TOP_LEVEL_MAX_NODES || top_nodes + n_h > top_cap) break;
        top_nodes += n_h;
        top_level = h;
    }
    std::vector<int> region(n_nodes, 0);
    {
        int next = 1;
        for (int i = sc.level_off[top_level]; i < sc.level_off[H]; ++i) region[sc.level_nodes[i]] = next++;
    }
    // [top entries][post clade list][pre clade list unless the same]
    std::vector<int4> sched(n_entries);
    for (int i = 0; i < n_top; ++i) {
        const int k = sc.level_nodes[i];
        // a node with one tip child lists its internal child first, so the
        // first child of every such node takes the same path
        int c0 = c->children[k].x, c1 = c->children[k].y;
        if (c0 < N && c1 >= N) std::swap(c0, c1);
        sched[i] = make_int4(k, c0, c1, region[k] | (region[c0] << 8) | (region[c1] << 16));
    }
    std::copy(sc.cl_post.begin(), sc.cl_post.end(), sched.begin() + n_top);
    if (!one_list) std::copy(sc.cl_pre.begin(), sc.cl_pre.end(), sched.begin() + n_top + n_cl);
    std::vector<int> cl_off(sc.cl_post_off);
    cl_off.insert(cl_off.end(), sc.cl_pre_off.begin(), sc.cl_pre_off.end());
    PG_HIP(c, put("codes", c->codes.data(), c->codes.size()));
    PG_HIP(c, put("masks", c->masks.data(), sizeof(unsigned long long) * 256));
    PG_HIP(c, put("level_off", sc.level_off.data(), sizeof(int) * sc.level_off.size()));
    PG_HIP(c, put("sched", sched.data(), sizeof(int4) * sched.size()));
    PG_HIP(c, put("cl_off", cl_off.data(), sizeof(int) * cl_off.size()));
    PG_HIP(c, put("Q64", c->Q.data(), sizeof(double) * M * M));
    PG_HIP(c, put("Q2_64", c->Q2.data(), sizeof(double) * M * M));
    PG_HIP(c, put("pi64", c->pi.data(), sizeof(double) * M));
    PG_HIP(c, put("rates", c->rates.data(), sizeof(double) * K));
    PG_HIP(c, put("catw", c->catw.data(), sizeof(double) * K));
    PG_HIP(c, put("weights", c->weights.data(), sizeof(double) * c->S_pad));
    if (c->bm_n > 0) {
        PG_HIP(c, put("bm_Q", c->bm_Q.data(), sizeof(double) * c->bm_Q.size()));
        PG_HIP(c, put("bm_Q2", c->bm_Q2.data(), sizeof(double) * c->bm_Q2.size()));
        PG_HIP(c, put("bm_qnorm", c->bm_qnorm.data(), sizeof(double) * c->bm_qnorm.size()));
        PG_HIP(c, put("bm_model", c->bm_model.data(), sizeof(int) * c->bm_model.size()));
    }
    if (split) {
        PG_HIP(c, put("eV", c->eV.data(), sizeof(double) * MP * MP));
        PG_HIP(c, put("eVinv", c->eVinv.data(), sizeof(double) * MP * MP));
        PG_HIP(c, put("eRe", c->eRe.data(), sizeof(double) * MP));
        PG_HIP(c, put("eIm", c->eIm.data(), sizeof(double) * MP));
        PG_HIP(c, put("eKind", c->eKind.data(), sizeof(int) * MP));
        PG_HIP(c, put("Qop", c->Qop.data(), MF_QOP_BYTES));
    }
    // pageable host sources: make sure the copies are done before the vectors move
    PG_HIP(c, hipStreamSynchronize(st));

    EvalArgs& a = c->args;
    a = EvalArgs{};
    a.n_tips = N;
    a.n_nodes = n_nodes;
    a.n_branches = B;
    a.root = n_nodes - 1;
    a.K = K;
    a.M = M;
    a.S = c->S;
    a.S_pad = c->S_pad;
    a.n_pb = n_pb;
    a.n_tiles = n_tiles;
    a.n_levels = H;
    a.qnorm = c->qnorm;
    for (int e = 0; e < 16; ++e) a.Qs[e] = (e < M * M) ? c->Q[e] : 0.0;
    for (int e = 0; e < 16; ++e) a.Q2s[e] = (e < M * M) ? c->Q2[e] : 0.0;
    for (int e = 0; e < 4; ++e) a.pis[e] = (e < M) ? c->pi[e] : 0.0;
    a.t = buf<double>(c, "t");
    a.P = c->bufs["P"].ptr;
    a.msg = c->bufs["msg"].ptr;
    a.qv = c->bufs["qv"].ptr;
    a.codes = buf<uint8_t>(c, "codes");
    a.masks = buf<unsigned long long>(c, "masks");
    a.level_off = buf<int>(c, "level_off");
    a.sched = buf<int4>(c, "sched");
    a.top_level = top_level;
    a.top_nodes = top_nodes;
    a.n_sched = n_top;
    if (n_cl > 0) {
        a.n_cl = n_cl;
        a.cl_depth = sc.depth;
        a.cl_post = a.sched + n_top;
        a.cl_pre = one_list ? a.cl_post : a.cl_post + n_cl;
        a.cl_post_off = buf<int>(c, "cl_off");
        a.cl_pre_off = a.cl_post_off + ns_post + 1;
    }
    // stage the schedule in LDS when it fits and leaves each kernel's total
    // within LDS_BLOCK_MAX
    a.sched_lds = (sizeof(int4) * (size_t)(n_top + n_cl) <= (size_t)SCHED_LDS_MAX) ? 1 : 0;
    if (!split && (post_lds_bytes(a, c->precision) > (size_t)LDS_BLOCK_MAX ||
                   pre_lds_bytes(a, c->precision) > (size_t)LDS_BLOCK_MAX))
        a.sched_lds = 0;
    a.Q64 = buf<double>(c, "Q64");
    a.Q2_64 = buf<double>(c, "Q2_64");
    a.pi64 = buf<double>(c, "pi64");
    a.rates = buf<double>(c, "rates");
    a.catw = buf<double>(c, "catw");
    a.weights = buf<double>(c, "weights");
    a.rootL = buf<double>(c, "rootL");
    a.rootE = buf<int>(c, "rootE");
    a.partial = buf<double>(c, "partial");
    a.partial2 = buf<double>(c, "partial2");
    a.r1 = nullptr;  // allocated by the first Hessian call
    a.logl_part = buf<double>(c, "logl_part");
    a.flag_part = buf<int>(c, "flag_part");
    a.grad_out = buf<double>(c, "grad");
    a.hess_out = buf<double>(c, "hess");
    a.logL_out = buf<double>(c, "logL");
    a.status = buf<int>(c, "status");
    a.n_models = c->bm_n;
    if (c->updates) {
        if ((r = ensure_buf(c, "expo", sizeof(int16_t) * (size_t)(N - 1) * n_tiles * TP))) return r;
        a.expo = buf<int16_t>(c, "expo");
    }
    if (c->bm_n > 0) {
        a.Qm = buf<double>(c, "bm_Q");
        a.Q2m = buf<double>(c, "bm_Q2");
        a.qnorm_m = buf<double>(c, "bm_qnorm");
        a.branch_model = buf<int>(c, "bm_model");
    }
    if (split) {
        a.eV = buf<double>(c, "eV");
        a.eVinv = buf<double>(c, "eVinv");
        a.eRe = buf<double>(c, "eRe");
        a.eIm = buf<double>(c, "eIm");
        a.eKind = buf<int>(c, "eKind");
        a.Qop = c->bufs["Qop"].ptr;
        a.expm_taylor = c->expm_taylor ? 1 : 0;
    }
    c->dev_stale = false;
    c->have_partials = false;
    return PG_OK;
}

hipEvent_t pool_event(pg_ctx* c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Wait for the recorded event pairs, add their durations, recycle them.
int drain_timing(pg_ctx* c) {
    for (auto& p : c->pending) {
        PG_HIP(c, hipEventSynchronize(p.b));
        float ms = 0.f;
        PG_HIP(c, hipEventElapsedTime(&ms, p.a, p.b));
        c->ms[p.kid] += ms;
        c->launches[p.kid] += 1;
        c->ev_pool.push_back(p.a);
        c->ev_pool.push_back(p.b);
    }
    c->pending.clear();
    return PG_OK;
}

// Launch one kernel, bracketed by events when timing is on.
template <typename F>
int timed(pg_ctx* c, int kid, F&& launch) {
    hipEvent_t a = nullptr, b = nullptr;
    if (c->timing) {
        a = pool_event(c);
        b = pool_event(c);
        if (!a || !b) return fail(c, PG_E_DEVICE, "hipEventCreate failed");
        PG_HIP(c, hipEventRecord(a, c->stream));
    }
    hipError_t e = launch();
    if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
    if (c->timing) {
        PG_HIP(c, hipEventRecord(b, c->stream));
        c->pending.push_back({kid, a, b});
    }
    return PG_OK;
}

int check_lengths(pg_ctx* c, const double* t) {
    const int B = 2 * c->n_tips - 2;
    for (int b = 0; b < B; ++b)
        if (!std::isfinite(t[b]) || t[b] < 0.0)
            return fail(c, PG_E_INVALID, "branch length t[" + std::to_string(b) + "] = " +
                                             std::to_string(t[b]) + " is not finite and >= 0");
    return PG_OK;
}

// Enqueue the evaluation on the context's stream.  Branch lengths are read
// from a.t; logL (and the gradient) are written to a.logL_out (a.grad_out).
//   forward only:  pmat, post, logl
//   with gradient: pmat, post, pre, gsum (gsum also reduces logL)
int enqueue_forward(pg_ctx* c, const EvalArgs& a, bool with_logl) {
    int r;
    if ((r = timed(c, PG_K_PMAT, [&] { return launch_pmat(a, c->precision, c->stream); }))) return r;
    if ((r = timed(c, PG_K_POST, [&] { return launch_post(a, c->precision, c->stream); }))) return r;
    if (with_logl && (r = timed(c, PG_K_ROOT, [&] { return launch_logl(a, c->stream); }))) return r;
    return PG_OK;
}

int enqueue_backward(pg_ctx* c, const EvalArgs& a) {
    int r;
    if ((r = timed(c, PG_K_PRE, [&] { return launch_pre(a, c->precision, c->stream, false); }))) return r;
    if ((r = timed(c, PG_K_GSUM, [&] { return launch_gsum(a, c->stream); }))) return r;
    return PG_OK;
}

int status_code(pg_ctx* c, int status) {
    if (status == 1) return fail(c, PG_E_INVALID, "a branch length is not finite and >= 0 (logL is NaN)");
    if (status == 2) return fail(c, PG_E_ZERO_LIK, "a pattern with positive weight has likelihood 0");
    return PG_OK;
}

// Copy logL (and grad) back, wait, and map the device status to a code.
int finish_host(pg_ctx* c, double* logL, double* grad) {
    int status = 0;
    PG_HIP(c, hipMemcpyAsync(&status, c->args.status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    PG_HIP(c, hipMemcpyAsync(logL, c->args.logL_out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (grad)
        PG_HIP(c, hipMemcpyAsync(grad, c->args.grad_out, sizeof(double) * c->args.n_branches,
                                 hipMemcpyDeviceToHost, c->stream));
    PG_HIP(c, hipStreamSynchronize(c->stream));
    int r = drain_timing(c);
    if (r) return r;
    return status_code(c, status);
}

template <typename F>
int guarded(pg_ctx* c, F&& body) {
    try {
        return body();
    } catch (const std::bad_alloc&) {
        return fail(c, PG_E_OOM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(c, PG_E_DEVICE, std::string("internal error: ") + e.what());
    } catch (...) {
        return fail(c, PG_E_DEVICE, "internal error");
    }
}

}  // namespace

namespace pg {

// Device state of a context for the serving scheduler: allocate and upload
// if needed (blocking), then hand out its EvalArgs.
int ctx_prepare(pg_ctx* c) {
    return guarded(c, [&] {
        int r = upload(c);
        if (r == PG_OK) c->have_partials = false;
        return r;
    });
}
EvalArgs ctx_args(const pg_ctx* c) { return c->args; }

// A context without its own stream, events or device query, on `stream`,
// allocating through `alloc` (serving sessions).
pg_ctx* ctx_new_session(int device, int precision, hipStream_t stream, DeviceAllocator* alloc) {
    pg_ctx* c = new pg_ctx();
    c->device = device;
    c->precision = precision;
    c->stream = stream;
    c->allocator = alloc;
    return c;
}
int ctx_precision(const pg_ctx* c) { return c->precision; }
const char* ctx_error(const pg_ctx* c) { return c->err.c_str(); }

}  // namespace pg

extern "C" {

int pg_create(int device, int precision, pg_ctx** out) {
    if (!out) return PG_E_INVALID;
    *out = nullptr;
    if (precision != PG_FP64 && precision != PG_FP32 && precision != PG_SPLIT_BF16) {
        g_create_error = "precision must be PG_FP64, PG_FP32 or PG_SPLIT_BF16";
        return PG_E_UNSUPPORTED;
    }
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || device < 0 || device >= n) {
        g_create_error = "no HIP device " + std::to_string(device) +
                         (e != hipSuccess ? std::string(": ") + hipGetErrorString(e) : std::string());
        return PG_E_DEVICE;
    }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) {
        g_create_error = std::string("hipGetDeviceProperties: ") + hipGetErrorString(e);
        return PG_E_DEVICE;
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        g_create_error = std::string("device is ") + prop.gcnArchName + ", the kernels are built for gfx950";
        return PG_E_DEVICE;
    }
    pg_ctx* c = nullptr;
    try {
        c = new pg_ctx();
    } catch (...) {
        g_create_error = "host allocation failed";
        return PG_E_OOM;
    }
    c->device = device;
    c->precision = precision;
    if ((e = hipSetDevice(device)) != hipSuccess || (e = hipStreamCreate(&c->own_stream)) != hipSuccess) {
        g_create_error = std::string("HIP setup: ") + hipGetErrorString(e);
        pg_destroy(c);
        return PG_E_DEVICE;
    }
    c->stream = c->own_stream;
    *out = c;
    return PG_OK;
}

void pg_destroy(pg_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto& kv : c->bufs)
        if (kv.second.ptr) {
            if (c->allocator) c->allocator->release(kv.second.ptr, kv.second.bytes);
            else (void)hipFree(kv.second.ptr);
        }
    for (auto& p : c->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->u_pinned) (void)hipHostFree(c->u_pinned);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    delete c;
}

const char* pg_last_error(const pg_ctx* c) {
    if (!c) return g_create_error.c_str();
    return c->err.c_str();
}

int pg_set_stream(pg_ctx* c, void* s) {
    if (!c) return PG_E_INVALID;
    return guarded(c, [&] {
        PG_HIP(c, hipStreamSynchronize(c->stream));
        c->stream = s ? static_cast<hipStream_t>(s) : c->own_stream;
        return PG_OK;
    });
}

int pg_set_tree(pg_ctx* c, int32_t N, const int32_t* parent) {
    if (!c) return PG_E_INVALID;
    if (!parent) return fail(c, PG_E_INVALID, "parent is NULL");
    if (N < 2 || N > (1 << 26)) return fail(c, PG_E_INVALID, "need 2 <= n_tips <= 2^26");
    return guarded(c, [&] {
        int r = check_tree(c, N, parent);
        if (r) return r;
        if (c->n_tips != N) {
            c->patterns_set = false;
            c->bm_n = 0;  // branch models are per branch of the old tree
        }
        c->n_tips = N;
        c->parent.assign(parent, parent + 2 * N - 1);
        build_levels(c);
        c->tree_set = true;
        c->dev_stale = true;
        c->have_partials = false;
        return PG_OK;
    });
}

int pg_set_patterns(pg_ctx* c, int32_t S, int32_t m, const uint64_t* tip_masks, const double* weights) {
    if (!c) return PG_E_INVALID;
    if (!c->tree_set) return fail(c, PG_E_STATE, "set the tree before the patterns");
    if (!tip_masks || !weights) return fail(c, PG_E_INVALID, "NULL masks or weights");
    if (S < 1) return fail(c, PG_E_INVALID, "need n_patterns >= 1");
    if (m < 2 || m > 64) return fail(c, PG_E_PATTERNS, "need 2 <= n_states <= 64");
    return guarded(c, [&] {
        const int N = c->n_tips;
        const int S_pad = (S + TP - 1) / TP * TP;
        const unsigned long long full = (m == 64) ? ~0ull : ((1ull << m) - 1);
        std::vector<unsigned long long> table(256, 0);
        for (int x = 0; x < m; ++x) table[x] = 1ull << x;
        table[255] = full;
        std::map<unsigned long long, int> partial_code;
        int next = m;
        std::vector<uint8_t> codes((size_t)N * S_pad, 255);
        for (int v = 0; v < N; ++v)
            for (int s = 0; s < S; ++s) {
                const unsigned long long mk = tip_masks[(size_t)v * S + s];
                if (mk == 0)
                    return fail(c, PG_E_PATTERNS, "empty mask at tip " + std::to_string(v) + ", pattern " +
                                                      std::to_string(s));
                if (mk & ~full)
                    return fail(c, PG_E_PATTERNS, "mask names a state >= n_states at tip " +
                                                      std::to_string(v) + ", pattern " + std::to_string(s));
                uint8_t code;
                if (mk == full) {
                    code = 255;
                } else if ((mk & (mk - 1)) == 0) {
                    code = (uint8_t)__builtin_ctzll(mk);
                } else {
                    auto it = partial_code.find(mk);
                    if (it == partial_code.end()) {
                        if (next >= 255)
                            return fail(c, PG_E_PATTERNS, "more than 255 - n_states distinct ambiguity masks");
                        table[next] = mk;
                        it = partial_code.emplace(mk, next++).first;
                    }
                    code = (uint8_t)it->second;
                }
                codes[(size_t)v * S_pad + s] = code;
            }
        std::vector<double> w(S_pad, 0.0);
        for (int s = 0; s < S; ++s) {
            if (!std::isfinite(weights[s]) || weights[s] < 0.0)
                return fail(c, PG_E_PATTERNS, "pattern weight " + std::to_string(s) + " is not finite and >= 0");
            w[s] = weights[s];
        }
        c->S = S;
        c->S_pad = S_pad;
        c->m_pat = m;
        c->codes.swap(codes);
        c->masks.swap(table);
        c->weights.swap(w);
        c->patterns_set = true;
        c->dev_stale = true;
        c->have_partials = false;
        return PG_OK;
    });
}

int pg_set_model(pg_ctx* c, int32_t m, const double* Q, const double* pi, int32_t K, const double* rates,
                 const double* catw) {
    if (!c) return PG_E_INVALID;
    if (!Q || !pi || !rates || !catw) return fail(c, PG_E_INVALID, "NULL model array");
    if (m < 2 || m > 64) return fail(c, PG_E_MODEL, "need 2 <= n_states <= 64");
    if (K < 1 || K > 64) return fail(c, PG_E_MODEL, "need 1 <= n_cats <= 64");
    if (!kernel_supported(m, c->precision))
        return fail(c, PG_E_UNSUPPORTED, "no kernel compiled for " + std::to_string(m) + " states");
    return guarded(c, [&] {
        double amax = 1.0;
        for (int i = 0; i < m * m; ++i) {
            if (!std::isfinite(Q[i])) return fail(c, PG_E_MODEL, "Q has a non-finite entry");
            amax = std::max(amax, std::fabs(Q[i]));
        }
        double qnorm = 0.0;
        for (int x = 0; x < m; ++x) {
            double row = 0.0, rabs = 0.0;
            for (int y = 0; y < m; ++y) {
                if (x != y && Q[x * m + y] < 0.0)
                    return fail(c, PG_E_MODEL, "Q has a negative off-diagonal rate");
                row += Q[x * m + y];
                rabs += std::fabs(Q[x * m + y]);
            }
            if (std::fabs(row) > 1e-12 * amax * m)
                return fail(c, PG_E_MODEL, "row " + std::to_string(x) + " of Q does not sum to 0");
            qnorm = std::max(qnorm, rabs);
        }
        double ps = 0.0;
        for (int x = 0; x < m; ++x) {
            if (!std::isfinite(pi[x]) || pi[x] < 0.0) return fail(c, PG_E_MODEL, "root frequency < 0 or not finite");
            ps += pi[x];
        }
        if (std::fabs(ps - 1.0) > 1e-12) return fail(c, PG_E_MODEL, "root frequencies do not sum to 1");
        double ws = 0.0;
        for (int l = 0; l < K; ++l) {
            if (!std::isfinite(rates[l]) || rates[l] < 0.0) return fail(c, PG_E_MODEL, "category rate < 0 or not finite");
            if (!std::isfinite(catw[l]) || catw[l] < 0.0) return fail(c, PG_E_MODEL, "category weight < 0 or not finite");
            ws += catw[l];
        }
        if (std::fabs(ws - 1.0) > 1e-12) return fail(c, PG_E_MODEL, "category weights do not sum to 1");
        const int old_m = c->m;
        c->m = m;
        c->K = K;
        c->Q.assign(Q, Q + m * m);
        c->Q2.assign(m * m, 0.0);
        for (int x = 0; x < m; ++x)
            for (int y = 0; y < m; ++y) {
                double acc = 0.0;
                for (int z = 0; z < m; ++z) acc += Q[x * m + z] * Q[z * m + y];
                c->Q2[x * m + y] = acc;
            }
        c->pi.assign(pi, pi + m);
        c->rates.assign(rates, rates + K);
        c->catw.assign(catw, catw + K);
        c->qnorm = qnorm;
        if (c->precision == PG_SPLIT_BF16) prepare_split_model(c);
        if (old_m != m) c->bm_n = 0;  // branch models have the old state count
        c->model_set = true;
        c->dev_stale = true;
        c->have_partials = false;
        return PG_OK;
    });
}

int pg_set_branch_models(pg_ctx* c, int32_t n_models, const double* Q, const int32_t* model_of_branch) {
    if (!c) return PG_E_INVALID;
    if (!c->tree_set || !c->model_set) return fail(c, PG_E_STATE, "set the tree and the model first");
    if (n_models < 0) return fail(c, PG_E_INVALID, "n_models < 0");
    if (n_models > 0 && (!Q || !model_of_branch)) return fail(c, PG_E_INVALID, "NULL Q or model_of_branch");
    if (n_models > 0 && c->precision == PG_SPLIT_BF16)
        return fail(c, PG_E_UNSUPPORTED, "per-branch rate matrices have no split-BF16 kernel");
    return guarded(c, [&] {
        const int m = c->m, B = 2 * c->n_tips - 2;
        std::vector<double> Qs, Q2s, qn;
        std::vector<int> model;
        if (n_models > 0) {
            Qs.assign(Q, Q + (size_t)n_models * m * m);
            Q2s.assign(Qs.size(), 0.0);
            qn.assign(n_models, 0.0);
            for (int k = 0; k < n_models; ++k) {
                const double* Qk = Qs.data() + (size_t)k * m * m;
                double amax = 1.0;
                for (int i = 0; i < m * m; ++i) {
                    if (!std::isfinite(Qk[i])) return fail(c, PG_E_MODEL, "rate matrix has a non-finite entry");
                    amax = std::max(amax, std::fabs(Qk[i]));
                }
                for (int x = 0; x < m; ++x) {
                    double row = 0.0, rabs = 0.0;
                    for (int y = 0; y < m; ++y) {
                        if (x != y && Qk[x * m + y] < 0.0)
                            return fail(c, PG_E_MODEL, "rate matrix " + std::to_string(k) +
                                                           " has a negative off-diagonal rate");
                        row += Qk[x * m + y];
                        rabs += std::fabs(Qk[x * m + y]);
                    }
                    if (std::fabs(row) > 1e-12 * amax * m)
                        return fail(c, PG_E_MODEL, "a row of rate matrix " + std::to_string(k) + " does not sum to 0");
                    qn[k] = std::max(qn[k], rabs);
                }
                double* Q2k = Q2s.data() + (size_t)k * m * m;
                for (int x = 0; x < m; ++x)
                    for (int y = 0; y < m; ++y) {
                        double acc = 0.0;
                        for (int z = 0; z < m; ++z) acc += Qk[x * m + z] * Qk[z * m + y];
                        Q2k[x * m + y] = acc;
                    }
            }
            model.assign(model_of_branch, model_of_branch + B);
            for (int b = 0; b < B; ++b)
                if (model[b] < 0 || model[b] >= n_models)
                    return fail(c, PG_E_INVALID, "model_of_branch[" + std::to_string(b) + "] out of range");
        }
        c->bm_n = n_models;
        c->bm_Q.swap(Qs);
        c->bm_Q2.swap(Q2s);
        c->bm_qnorm.swap(qn);
        c->bm_model.swap(model);
        c->dev_stale = true;
        c->have_partials = false;
        return PG_OK;
    });
}

int pg_logL_update(pg_ctx* c, int32_t n, const int32_t* branches, const double* t_new, double* logL) {
    if (!c) return PG_E_INVALID;
    if (n < 0 || (n > 0 && (!branches || !t_new)) || !logL) return fail(c, PG_E_INVALID, "bad arguments");
    if (c->precision == PG_SPLIT_BF16)
        return fail(c, PG_E_UNSUPPORTED, "partial re-evaluation has no split-BF16 kernel");
    if (!c->have_partials || c->dev_stale || !c->t_host_valid)
        return fail(c, PG_E_STATE, "no resident partials from a host-pointer evaluation");
    return guarded(c, [&] {
        const int N = c->n_tips, B = 2 * N - 2;
        for (int i = 0; i < n; ++i) {
            if (branches[i] < 0 || branches[i] >= B)
                return fail(c, PG_E_INVALID, "branch index " + std::to_string(branches[i]) + " out of range");
            if (!std::isfinite(t_new[i]) || t_new[i] < 0.0)
                return fail(c, PG_E_INVALID, "new length of branch " + std::to_string(branches[i]) +
                                                 " is not finite and >= 0");
        }
        PG_HIP(c, hipSetDevice(c->device));
        std::vector<double> t = c->t_host;
        for (int i = 0; i < n; ++i) t[branches[i]] = t_new[i];
        int r;
        if (!c->updates) {
            // first update: keep per-node exponents from now on, by one
            // full evaluation at the new lengths
            c->updates = true;
            c->dev_stale = true;
            if ((r = upload(c))) return r;
            c->have_partials = false;
            c->t_host_valid = false;
            PG_HIP(c, hipMemcpyAsync((void*)c->args.t, t.data(), sizeof(double) * B, hipMemcpyHostToDevice,
                                     c->stream));
            if ((r = enqueue_forward(c, c->args, true))) return r;
        } else {
            // dirty nodes: each changed internal node (its message changes
            // with its matrix) and every ancestor of a changed branch
            std::vector<char> dirty(2 * N - 1, 0);
            std::vector<int> list;
            for (int i = 0; i < n; ++i) {
                const int b = branches[i];
                if (std::find(list.begin(), list.end(), b) == list.end()) list.push_back(b);
                for (int v = (b >= N) ? b : c->parent[b]; v >= 0 && !dirty[v]; v = c->parent[v]) dirty[v] = 1;
            }
            const int H = (int)c->level_off.size() - 1;
            std::vector<int> off(H + 1, 0);
            std::vector<int4> sched;
            for (int h = 0; h < H; ++h) {
                for (int i = c->level_off[h]; i < c->level_off[h + 1]; ++i) {
                    const int k = c->level_nodes[i];
                    if (dirty[k]) sched.push_back(make_int4(k, c->children[k].x, c->children[k].y, 0));
                }
                off[h + 1] = (int)sched.size();
            }
            // one pinned staging area and one copy: [t][branch list][schedule][level offsets]
            const size_t o_list = sizeof(double) * B;
            const size_t o_sched = (o_list + sizeof(int) * B + 15) & ~size_t(15);
            const size_t o_level = o_sched + sizeof(int4) * (N - 1);
            const size_t bytes = o_level + sizeof(int) * (H + 1);
            if (c->u_pinned_bytes < bytes) {
                if (c->u_pinned) (void)hipHostFree(c->u_pinned);
                c->u_pinned = nullptr;
                c->u_pinned_bytes = 0;
                PG_HIP(c, hipStreamSynchronize(c->stream));
                PG_HIP(c, hipHostMalloc(&c->u_pinned, bytes));
                c->u_pinned_bytes = bytes;
            }
            if ((r = ensure_buf(c, "u_stage", bytes))) return r;
            // a successful call ends with finish_host, which waits for the
            // stream; after an error, wait here before reusing the staging area
            if (c->u_inflight) PG_HIP(c, hipStreamSynchronize(c->stream));
            c->u_inflight = false;
            char* hs = static_cast<char*>(c->u_pinned);
            std::memcpy(hs, t.data(), sizeof(double) * B);
            std::memcpy(hs + o_list, list.data(), sizeof(int) * list.size());
            std::memcpy(hs + o_sched, sched.data(), sizeof(int4) * sched.size());
            std::memcpy(hs + o_level, off.data(), sizeof(int) * off.size());
            char* ds = static_cast<char*>(c->bufs["u_stage"].ptr);
            c->have_partials = false;
            c->t_host_valid = false;
            hipStream_t st = c->stream;
            c->u_inflight = true;
            PG_HIP(c, hipMemcpyAsync(ds, hs, bytes, hipMemcpyHostToDevice, st));
            PG_HIP(c, hipMemcpyAsync((void*)c->args.t, ds, sizeof(double) * B, hipMemcpyDeviceToDevice, st));
            EvalArgs a = c->args;
            if (!list.empty()) {
                a.blist = reinterpret_cast<const int*>(ds + o_list);
                a.n_blist = (int)list.size();
                if ((r = timed(c, PG_K_PMAT, [&] { return launch_pmat(a, c->precision, st); }))) return r;
            }
            EvalArgs p = c->args;
            p.sched = reinterpret_cast<const int4*>(ds + o_sched);
            p.sched_lds = 0;
            p.level_off = reinterpret_cast<const int*>(ds + o_level);
            p.n_levels = H;
            p.n_sched = (int)sched.size();
            p.n_cl = 0;
            p.top_level = p.n_levels;
            p.expo_delta = 1;
            if ((r = timed(c, PG_K_POST, [&] { return launch_post(p, c->precision, st); }))) return r;
            if ((r = timed(c, PG_K_ROOT, [&] { return launch_logl(c->args, st); }))) return r;
        }
        r = finish_host(c, logL, nullptr);
        if (r != PG_E_DEVICE) c->u_inflight = false;
        if (r == PG_E_ZERO_LIK) *logL = -INFINITY;
        if (r == PG_OK) {
            c->have_partials = true;
            c->t_host = t;
            c->t_host_valid = true;
        }
        return r;
    });
}

int pg_logL(pg_ctx* c, const double* t, double* logL) {
    if (!c) return PG_E_INVALID;
    if (!t || !logL) return fail(c, PG_E_INVALID, "NULL t or logL");
    return guarded(c, [&] {
        int r = upload(c);
        if (r) return r;
        if ((r = check_lengths(c, t))) return r;
        PG_HIP(c, hipSetDevice(c->device));
        c->have_partials = false;
        c->t_host_valid = false;
        PG_HIP(c, hipMemcpyAsync((void*)c->args.t, t, sizeof(double) * c->args.n_branches,
                                 hipMemcpyHostToDevice, c->stream));
        if ((r = enqueue_forward(c, c->args, true))) return r;
        r = finish_host(c, logL, nullptr);
        if (r == PG_E_ZERO_LIK) *logL = -INFINITY;
        if (r == PG_OK) {
            c->have_partials = true;
            c->t_host.assign(t, t + c->args.n_branches);
            c->t_host_valid = true;
        }
        return r;
    });
}

int pg_grad(pg_ctx* c, double* grad) {
    if (!c) return PG_E_INVALID;
    if (!grad) return fail(c, PG_E_INVALID, "NULL grad");
    if (!c->have_partials || c->dev_stale)
        return fail(c, PG_E_STATE, "no resident partials: call pg_logL first");
    return guarded(c, [&] {
        PG_HIP(c, hipSetDevice(c->device));
        int r = enqueue_backward(c, c->args);
        if (r) return r;
        double logL = 0.0;
        return finish_host(c, &logL, grad);
    });
}

int pg_logL_and_grad(pg_ctx* c, const double* t, double* logL, double* grad) {
    if (!c) return PG_E_INVALID;
    if (!t || !logL) return fail(c, PG_E_INVALID, "NULL t or logL");
    if (!grad) return pg_logL(c, t, logL);
    return guarded(c, [&] {
        int r = upload(c);
        if (r) return r;
        if ((r = check_lengths(c, t))) return r;
        PG_HIP(c, hipSetDevice(c->device));
        c->have_partials = false;
        c->t_host_valid = false;
        PG_HIP(c, hipMemcpyAsync((void*)c->args.t, t, sizeof(double) * c->args.n_branches,
                                 hipMemcpyHostToDevice, c->stream));
        if ((r = enqueue_forward(c, c->args, false))) return r;
        if ((r = enqueue_backward(c, c->args))) return r;
        r = finish_host(c, logL, grad);
        if (r == PG_E_ZERO_LIK) *logL = -INFINITY;
        if (r == PG_OK) {
            c->have_partials = true;
            c->t_host.assign(t, t + c->args.n_branches);
            c->t_host_valid = true;
        }
        return r;
    });
}

int pg_hessian_diag(pg_ctx* c, double* grad, double* hess) {
    if (!c) return PG_E_INVALID;
    if (!hess) return fail(c, PG_E_INVALID, "NULL hess");
    if (c->precision == PG_SPLIT_BF16)
        return fail(c, PG_E_UNSUPPORTED, "the Hessian diagonal has no split-BF16 kernel");
    if (!c->have_partials || c->dev_stale)
        return fail(c, PG_E_STATE, "no resident partials: call pg_logL first");
    return guarded(c, [&] {
        PG_HIP(c, hipSetDevice(c->device));
        EvalArgs& a = c->args;
        int r;
        if ((r = ensure_buf(c, "r1", sizeof(double) * (size_t)a.n_branches * a.K * a.S_pad))) return r;
        a.r1 = buf<double>(c, "r1");
        if ((r = timed(c, PG_K_PRE, [&] { return launch_pre(a, c->precision, c->stream, true); }))) return r;
        if ((r = timed(c, PG_K_GSUM, [&] { return launch_gsum(a, c->stream); }))) return r;
        if ((r = timed(c, PG_K_GSUM, [&] { return launch_hsum(a, c->stream); }))) return r;
        PG_HIP(c, hipMemcpyAsync(hess, a.hess_out, sizeof(double) * a.n_branches, hipMemcpyDeviceToHost,
                                 c->stream));
        double logL = 0.0;
        return finish_host(c, &logL, grad);
    });
}

int pg_logL_and_grad_device(pg_ctx* c, const double* d_t, double* d_logL, double* d_grad) {
    if (!c) return PG_E_INVALID;
    if (!d_t || !d_logL) return fail(c, PG_E_INVALID, "NULL d_t or d_logL");
    return guarded(c, [&] {
        int r = upload(c);
        if (r) return r;
        PG_HIP(c, hipSetDevice(c->device));
        c->t_host_valid = false;  // lengths of the resident partials are on the device only
        EvalArgs a = c->args;
        a.t = d_t;
        a.logL_out = d_logL;
        if (d_grad) a.grad_out = d_grad;
        if ((r = enqueue_forward(c, a, d_grad == nullptr))) return r;
        if (d_grad && (r = enqueue_backward(c, a))) return r;
        c->have_partials = true;
        c->device_pending = true;
        return PG_OK;
    });
}

int pg_grad_device(pg_ctx* c, double* d_grad) {
    if (!c) return PG_E_INVALID;
    if (!d_grad) return fail(c, PG_E_INVALID, "NULL d_grad");
    if (!c->have_partials || c->dev_stale)
        return fail(c, PG_E_STATE, "no resident partials: evaluate logL first");
    return guarded(c, [&] {
        PG_HIP(c, hipSetDevice(c->device));
        EvalArgs a = c->args;
        a.grad_out = d_grad;
        // the logL reduction of the backward pass goes to the context's own
        // buffer, not to the caller's forward output
        return enqueue_backward(c, a);
    });
}

int pg_status(pg_ctx* c) {
    if (!c) return PG_E_INVALID;
    if (!c->device_pending) return PG_OK;
    return guarded(c, [&] {
        int status = 0;
        PG_HIP(c, hipMemcpyAsync(&status, c->args.status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        PG_HIP(c, hipStreamSynchronize(c->stream));
        return status_code(c, status);
    });
}

int pg_set_timing(pg_ctx* c, int enable) {
    if (!c) return PG_E_INVALID;
    c->timing = enable != 0;
    return PG_OK;
}

int pg_get_timing(pg_ctx* c, double* ms, int64_t* launches) {
    if (!c) return PG_E_INVALID;
    int r = guarded(c, [&] { return drain_timing(c); });
    if (r) return r;
    for (int k = 0; k < PG_K_COUNT; ++k) {
        if (ms) ms[k] = c->ms[k];
        if (launches) launches[k] = c->launches[k];
        c->ms[k] = 0.0;
        c->launches[k] = 0;
    }
    return PG_OK;
}

int64_t pg_device_bytes(const pg_ctx* c) {
    if (!c) return 0;
    int64_t tot = 0;
    for (const auto& kv : c->bufs) tot += (int64_t)kv.second.bytes;
    return tot;
}

int64_t pg_footprint_bytes(int32_t N, int32_t S, int32_t m, int32_t K, int precision) {
    if (N < 2 || S < 1 || m < 2 || K < 1) return -1;
    const bool split = precision == PG_SPLIT_BF16;
    const int64_t es = precision == PG_FP64 ? 8 : 4;
    const int64_t S_pad = (S + TP - 1) / TP * TP;
    const int64_t B = 2 * (int64_t)N - 2;
    const int64_t n_tiles = K * (S_pad / TP);
    const int64_t ms = split ? MP : m;
    int64_t tot = 0;
    tot += 2 * es * (int64_t)K * ms * S_pad * (N - 1);      // msg + qv
    tot += split ? (int64_t)MF_SLOT_BYTES * B * K : es * B * K * m * m;  // P
    tot += (int64_t)N * S_pad;                             // codes
    tot += 8 * (n_tiles * B + (S_pad / TP) * B);           // tile partial sums
    tot += (8 + 8 + 4) * (int64_t)K * S_pad + 8 * S_pad;   // root values, rho, weights
    tot += 8 * 4 * B + 4 * 3 * (int64_t)N + 4096;          // t, grad, hess, schedule
    return tot;
}

int pg_eigensystem(int32_t m, const double* Q, double* V, double* Vinv, double* re, double* im, int32_t* kind,
                   double* cond, double* resid) {
    if (!Q || !V || !Vinv || !re || !im || !kind || !cond || !resid || m < 1 || m > 4096) return PG_E_INVALID;
    try {
        EigenSystem es;
        if (!eigen_decompose(m, Q, es)) return PG_E_MODEL;
        std::copy(es.V.begin(), es.V.end(), V);
        std::copy(es.Vinv.begin(), es.Vinv.end(), Vinv);
        std::copy(es.re.begin(), es.re.end(), re);
        std::copy(es.im.begin(), es.im.end(), im);
        for (int j = 0; j < m; ++j) kind[j] = es.kind[j];
        *cond = es.cond;
        *resid = es.resid;
        return PG_OK;
    } catch (...) {
        return PG_E_OOM;
    }
}

}  // extern "C"
