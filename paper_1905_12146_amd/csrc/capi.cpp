// C-ABI of libphylograd: context, input checks, tree schedule, device
// buffers and the evaluation sequence.  Declarations and the contract of
// every entry point are in include/phylograd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "pg_internal.h"

using namespace pg;

// Device scratch of the allocation-free entry point: every device buffer of
// one of its evaluations, in one array per device, allocated with the code
// object and held until the process ends.  In host code `scratch` names only
// a host-side stand-in: its device address is looked up once per device,
// with that device current (scratch_setup), and only that address is used.
static __device__ __align__(256) unsigned char scratch[PG_NOALLOC_MAX_BYTES];

namespace {

thread_local std::string g_create_error;

struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
};

// A buffer of the allocation-free entry point: its name, size, offset in
// the device scratch and the host data it is uploaded from (or NULL).
struct BufSpecRef {
    const char* name;
    size_t bytes, offset;
    const void* src;
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
    std::vector<Kids> children;               // [2N-1], set for internal nodes
    TreeLevels lv;                            // internal nodes by height

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
    std::vector<uint16_t> Qop, Q2op;
    // non-homogeneous model: branch b uses bm_Q[bm_model[b]] (bm_n = 0: off)
    int bm_n = 0;
    std::vector<double> bm_Q, bm_Q2, bm_qnorm;
    std::vector<int> bm_model;

    // dense-state path: Q and Q^2 as matrix-core fragments (bytes)
    std::vector<uint8_t> qfrag;
    // traversal plan of the tree for the model's state count
    TraversalPlan plan;
    bool plan_stale = true;

    // device state
    bool dev_stale = true;        // host inputs changed since the last upload
    bool host_copies = false;     // copies from the host vectors may be in flight
    // allocation-free evaluation: buffer layout in the device scratch
    bool na_stale = true;
    std::vector<BufSpecRef> na_specs;
    size_t na_total = 0;
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
    size_t granted = std::max<size_t>(bytes, 256);
    if (c->allocator) {
        p = c->allocator->acquire(granted, &granted);
        if (!p) return fail(c, PG_E_OOM, "device pool allocation failed");
    } else {
        hipError_t e = hipMalloc(&p, granted);
        if (e != hipSuccess) return hip_fail(c, e, "hipMalloc");
    }
    b.ptr = p;
    b.bytes = granted;
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
void split_qops(pg_ctx* c);

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
    split_qops(c);
}

// Split-BF16 operands (hi, mid, lo A fragments, [mt][ks][part][lane][8]) of
// Q (gradient) and Q^2 (Hessian): the model's, or with per-branch rate
// matrices one block per matrix, [model][...].
void split_qops(pg_ctx* c) {
    const int m = c->m;
    const int n = c->bm_n > 0 ? c->bm_n : 1;
    auto operands = [&](const double* A, uint16_t* out) {
        for (int mt = 0; mt < 4; ++mt)
            for (int ks = 0; ks < 2; ++ks)
                for (int lane = 0; lane < 64; ++lane)
                    for (int j = 0; j < 8; ++j) {
                        const int r = 16 * mt + lane % 16;
                        const int y = 16 * (2 * ks + j / 4) + 4 * (lane / 16) + j % 4;
                        const double v = (r < m && y < m) ? A[r * m + y] : 0.0;
                        const uint16_t hi = bf16_bits((float)v);
                        const double r1 = v - (double)bf16_value(hi);
                        const uint16_t mid = bf16_bits((float)r1);
                        const uint16_t lo = bf16_bits((float)(r1 - (double)bf16_value(mid)));
                        const uint16_t parts[3] = {hi, mid, lo};
                        for (int part = 0; part < 3; ++part)
                            out[((((mt * 2 + ks) * 3 + part) * 64 + lane) * 8) + j] = parts[part];
                    }
    };
    c->Qop.assign(n * MF_QOP_BYTES / 2, 0);
    c->Q2op.assign(n * MF_QOP_BYTES / 2, 0);
    for (int k = 0; k < n; ++k) {
        const size_t mm = (size_t)k * m * m, o = (size_t)k * MF_QOP_BYTES / 2;
        operands(c->bm_n > 0 ? &c->bm_Q[mm] : c->Q.data(), &c->Qop[o]);
        operands(c->bm_n > 0 ? &c->bm_Q2[mm] : c->Q2.data(), &c->Q2op[o]);
    }
}

// Dense-state path: an eigen-decomposition of Q (m x m) for the transition
// matrices F = P - I = V (exp(B rate t) - I) V^-1, used when it is well
// conditioned enough for the precision (FP64: cond_1(V) <= 1e4 and a
// reconstruction error <= 1e-13, about 1e-12 relative in F; FP32: 1e6 and
// 1e-11); otherwise the kernels use scaling and squaring.
void prepare_dense_model(pg_ctx* c) {
    const int m = c->m;
    EigenSystem es;
    const bool ok = eigen_decompose(m, c->Q.data(), es);
    const bool wide = c->precision == PG_FP64;
    c->expm_taylor = !(ok && es.cond <= (wide ? 1e4 : 1e6) && es.resid <= (wide ? 1e-13 : 1e-11));
    c->eig_cond = ok ? es.cond : INFINITY;
    c->eig_resid = ok ? es.resid : INFINITY;
    c->eV.assign((size_t)m * m, 0.0);
    c->eVinv.assign((size_t)m * m, 0.0);
    c->eRe.assign(m, 0.0);
    c->eIm.assign(m, 0.0);
    c->eKind.assign(m, 0);
    if (!c->expm_taylor) {
        c->eV = es.V;
        c->eVinv = es.Vinv;
        c->eRe = es.re;
        c->eIm = es.im;
        c->eKind = es.kind;
    }
}

int check_tree(pg_ctx* c, int32_t N, const int32_t* parent) {
    const int n_nodes = 2 * N - 1;
    const int root = n_nodes - 1;
    if (parent[root] != -1) return fail(c, PG_E_TREE, "parent[2N-2] must be -1 (root last)");
    std::vector<int> nchild(n_nodes, 0);
    std::vector<Kids> ch(n_nodes, Kids{-1, -1});
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

int check_ready(pg_ctx* c) {
    if (!c->tree_set || !c->patterns_set || !c->model_set)
        return fail(c, PG_E_STATE, "tree, patterns and model must all be set before evaluating");
    if (c->m_pat != c->m)
        return fail(c, PG_E_STATE, "patterns have " + std::to_string(c->m_pat) +
                                       " states but the model has " + std::to_string(c->m));
    return PG_OK;
}

// Host plan of the traversal (schedule, clade lists, top region); rebuilt
// when the tree, patterns or model change.
void ensure_plan(pg_ctx* c) {
    if (!c->plan_stale) return;
    const bool split = c->precision == PG_SPLIT_BF16;
    PlanParams p;
    p.n_states = c->m;
    p.elem_bytes = (int)elem_size(c->precision);
    // clade walks (small M) form 32-bit element offsets: every vector
    // buffer must hold fewer than 2^31 elements, else the level walk serves
    const size_t nodes = 2 * (size_t)c->n_tips - 1, lim = size_t(1) << 31;
    p.clades = !split && c->m * c->m <= TP && nodes * c->K * c->S_pad * c->m < lim && nodes * c->S_pad < lim;
    p.top_region = !split && !dense_states(c->m);
    p.ns_post = split ? node_slots(c->m) : post_node_slots(c->m, c->precision);
    p.ns_pre = split ? p.ns_post : pre_node_slots(c->m, c->precision);
    TraversalPlan plan;
    plan_traversal(c->n_tips, c->parent.data(), c->children.data(), c->lv, p, plan);
    c->plan = std::move(plan);
    c->plan_stale = false;
}

// Sizes of the device buffers of one evaluation.
struct Dims {
    int64_t N = 0, S_pad = 0, M = 0, K = 0;
    int precision = PG_FP64;
    int64_t n_entries = 0, n_level_off = 0, n_cl_off = 0;  // schedule
    int64_t bm_n = 0;                                      // per-branch models
    bool updates = false;                                  // per-node exponents kept
};

struct BufSpec {
    const char* name;
    size_t bytes;
    const void* src = nullptr;  // host data (bytes) to upload, or NULL
};

// Every device buffer of an evaluation.  `lean` leaves out what the
// allocation-free entry point does not use (its caller's t, logL and grad,
// the Hessian's tile sums, the per-node exponents).
std::vector<BufSpec> buffer_specs(const Dims& d, bool lean) {
    const bool split = d.precision == PG_SPLIT_BF16;
    const bool dense = !split && dense_states((int)d.M);
    const size_t es = elem_size(d.precision);
    const size_t N = d.N, B = 2 * d.N - 2, M = d.M, K = d.K, S_pad = d.S_pad;
    const size_t n_pb = S_pad / TP, n_tiles = K * n_pb;
    const size_t vec = K * (split ? MP : dense ? dn_md((int)M) : M) * S_pad;
    std::vector<BufSpec> v;
    auto add = [&](const char* name, size_t bytes) { v.push_back(BufSpec{name, bytes}); };
    if (!lean) add("t", sizeof(double) * B);
    add("P", split ? MF_SLOT_BYTES * B * K : es * B * K * (dense ? dn_slot_elems((int)M) : M * M));
    if (dense) add("Qfrag", es * std::max<size_t>(1, d.bm_n) * dn_qfrag_elems((int)M));
    if (split) {
        add("eV", sizeof(double) * MP * MP);
        add("eVinv", sizeof(double) * MP * MP);
        add("eRe", sizeof(double) * MP);
        add("eIm", sizeof(double) * MP);
        add("eKind", sizeof(int) * MP);
        add("Qop", MF_QOP_BYTES * std::max<size_t>(1, d.bm_n));
        add("Q2op", MF_QOP_BYTES * std::max<size_t>(1, d.bm_n));
    }
    if (dense) {
        add("eV", sizeof(double) * M * M);
        add("eVinv", sizeof(double) * M * M);
        add("eRe", sizeof(double) * M);
        add("eIm", sizeof(double) * M);
        add("eKind", sizeof(int) * M);
    }
    add("msg", es * vec * (N - 1));
    add("qv", es * vec * (N - 1));
    add("codes", N * S_pad);
    add("masks", sizeof(unsigned long long) * 256);
    add("level_off", sizeof(int) * d.n_level_off);
    add("sched", sizeof(int4) * d.n_entries);
    add("cl_off", sizeof(int) * d.n_cl_off);
    add("Q64", sizeof(double) * M * M);
    add("Q2_64", sizeof(double) * M * M);
    add("pi64", sizeof(double) * M);
    add("rates", sizeof(double) * K);
    add("catw", sizeof(double) * K);
    add("weights", sizeof(double) * S_pad);
    add("rootL", sizeof(double) * K * S_pad);
    add("rootE", sizeof(int) * K * S_pad);
    add("partial", sizeof(double) * n_tiles * B);
    // clade walks in launches of their own (small M): their exponent sums
    if (!split && !dense && M * M <= (size_t)TP)
        add("cl_esum", sizeof(int) * (size_t)(post_node_slots((int)M, d.precision) / CW_WAVES) * n_tiles * TP);
    if (!lean) add("partial2", sizeof(double) * n_tiles * B);
    add("logl_part", sizeof(double) * n_pb);
    add("flag_part", sizeof(int) * n_pb);
    if (!lean) {
        add("grad", sizeof(double) * B);
        add("hess", sizeof(double) * B);
        add("logL", sizeof(double) * 2);
    }
    add("status", sizeof(int) * 2);
    if (d.bm_n > 0) {
        add("bm_Q", sizeof(double) * d.bm_n * M * M);
        add("bm_Q2", sizeof(double) * d.bm_n * M * M);
        add("bm_qnorm", sizeof(double) * d.bm_n);
        add("bm_model", sizeof(int) * B);
    }
    if (d.updates && !lean) add("expo", sizeof(int16_t) * (N - 1) * n_tiles * TP);
    return v;
}

Dims ctx_dims(const pg_ctx* c) {
    Dims d;
    d.N = c->n_tips;
    d.S_pad = c->S_pad;
    d.M = c->m;
    d.K = c->K;
    d.precision = c->precision;
    d.n_entries = (int64_t)c->plan.sched.size();
    d.n_level_off = (int64_t)c->plan.level_off.size();
    d.n_cl_off = (int64_t)c->plan.cl_off.size();
    d.bm_n = c->bm_n;
    d.updates = c->updates;
    return d;
}

// The host data each input buffer is uploaded from.
void attach_sources(const pg_ctx* c, std::vector<BufSpec>& specs) {
    static_assert(sizeof(Ent) == sizeof(int4), "schedule entries are uploaded as int4");
    const std::map<std::string, const void*> src = {
        {"eV", c->eV.data()}, {"eVinv", c->eVinv.data()}, {"eRe", c->eRe.data()}, {"eIm", c->eIm.data()},
        {"eKind", c->eKind.data()}, {"Qop", c->Qop.data()}, {"Q2op", c->Q2op.data()}, {"codes", c->codes.data()},
        {"masks", c->masks.data()}, {"level_off", c->plan.level_off.data()}, {"sched", c->plan.sched.data()},
        {"cl_off", c->plan.cl_off.data()}, {"Q64", c->Q.data()}, {"Q2_64", c->Q2.data()},
        {"pi64", c->pi.data()}, {"rates", c->rates.data()}, {"catw", c->catw.data()},
        {"weights", c->weights.data()}, {"bm_Q", c->bm_Q.data()}, {"bm_Q2", c->bm_Q2.data()},
        {"bm_qnorm", c->bm_qnorm.data()}, {"bm_model", c->bm_model.data()}, {"Qfrag", c->qfrag.data()}};
    for (BufSpec& s : specs) {
        auto it = src.find(s.name);
        if (it != src.end()) s.src = it->second;
    }
}

// EvalArgs of the context's plan with buffers at at(name) (NULL for a
// buffer that is not there).
template <typename At>
void fill_args(const pg_ctx* c, At&& at, EvalArgs& a) {
    const TraversalPlan& pl = c->plan;
    const int N = c->n_tips, n_nodes = 2 * N - 1, M = c->m;
    const bool split = c->precision == PG_SPLIT_BF16;
    a = EvalArgs{};
    a.n_tips = N;
    a.n_nodes = n_nodes;
    a.n_branches = n_nodes - 1;
    a.root = n_nodes - 1;
    a.K = c->K;
    a.M = M;
    a.S = c->S;
    a.S_pad = c->S_pad;
    a.n_pb = c->S_pad / TP;
    a.n_tiles = c->K * a.n_pb;
    a.n_levels = pl.n_levels();
    a.qnorm = c->qnorm;
    for (int e = 0; e < 16; ++e) a.Qs[e] = (e < M * M) ? c->Q[e] : 0.0;
    for (int e = 0; e < 16; ++e) a.Q2s[e] = (e < M * M) ? c->Q2[e] : 0.0;
    for (int e = 0; e < 4; ++e) a.pis[e] = (e < M) ? c->pi[e] : 0.0;
    a.t = static_cast<const double*>(at("t"));
    a.P = at("P");
    a.msg = at("msg");
    a.qv = at("qv");
    a.codes = static_cast<const uint8_t*>(at("codes"));
    a.masks = static_cast<const unsigned long long*>(at("masks"));
    a.level_off = static_cast<const int*>(at("level_off"));
    a.sched = static_cast<const int4*>(at("sched"));
    a.top_level = pl.top_level;
    a.top_nodes = pl.top_nodes;
    a.n_sched = pl.n_top;
    if (pl.n_cl > 0) {
        a.n_cl = pl.n_cl;
        a.cl_depth = pl.depth;
        a.cl_post = a.sched + pl.n_top;
        a.cl_pre = pl.one_list ? a.cl_post : a.cl_post + pl.n_cl;
        a.cl_post_off = static_cast<const int*>(at("cl_off"));
        a.cl_pre_off = a.cl_post_off + pl.ns_post + 1;
        a.cl_esum = static_cast<int*>(at("cl_esum"));
    }
    // stage the schedule in LDS when it fits and leaves each kernel's total
    // within LDS_BLOCK_MAX
    a.sched_lds = (sizeof(int4) * (size_t)pl.n_top <= (size_t)SCHED_LDS_MAX) ? 1 : 0;
    if (!split && (post_lds_bytes(a, c->precision) > (size_t)LDS_BLOCK_MAX ||
                   pre_lds_bytes(a, c->precision) > (size_t)LDS_BLOCK_MAX))
        a.sched_lds = 0;
    a.Q64 = static_cast<const double*>(at("Q64"));
    a.Q2_64 = static_cast<const double*>(at("Q2_64"));
    a.pi64 = static_cast<const double*>(at("pi64"));
    a.rates = static_cast<const double*>(at("rates"));
    a.catw = static_cast<const double*>(at("catw"));
    a.weights = static_cast<const double*>(at("weights"));
    a.rootL = static_cast<double*>(at("rootL"));
    a.rootE = static_cast<int*>(at("rootE"));
    a.partial = static_cast<double*>(at("partial"));
    a.partial2 = static_cast<double*>(at("partial2"));
    a.r1 = nullptr;  // allocated by the first Hessian call
    a.logl_part = static_cast<double*>(at("logl_part"));
    a.flag_part = static_cast<int*>(at("flag_part"));
    a.grad_out = static_cast<double*>(at("grad"));
    a.hess_out = static_cast<double*>(at("hess"));
    a.logL_out = static_cast<double*>(at("logL"));
    a.status = static_cast<int*>(at("status"));
    a.expo = static_cast<int16_t*>(at("expo"));
    a.n_models = c->bm_n;
    if (c->bm_n > 0) {
        a.Qm = static_cast<const double*>(at("bm_Q"));
        a.Q2m = static_cast<const double*>(at("bm_Q2"));
        a.qnorm_m = static_cast<const double*>(at("bm_qnorm"));
        a.branch_model = static_cast<const int*>(at("bm_model"));
    }
    if (split || (dense_states(M) && c->precision != PG_SPLIT_BF16)) {
        a.eV = static_cast<const double*>(at("eV"));
        a.eVinv = static_cast<const double*>(at("eVinv"));
        a.eRe = static_cast<const double*>(at("eRe"));
        a.eIm = static_cast<const double*>(at("eIm"));
        a.eKind = static_cast<const int*>(at("eKind"));
        a.Qop = at("Qop");
        a.Q2op = at("Q2op");
        a.expm_taylor = c->expm_taylor ? 1 : 0;
    }
    a.Qfrag = at("Qfrag");
}

// Dense-state path: the A fragments of Q and Q^2 of every rate matrix (the
// model's, or each per-branch matrix) in the vectors' type, [model][Q, Q^2]
// [ob][s][lane] (layout in pg_internal.h).
void prepare_dense_q(pg_ctx* c) {
    const int M = c->m;
    c->qfrag.clear();
    if (c->precision == PG_SPLIT_BF16 || !dense_states(M)) return;
    const int NF = dn_nf(M), KS = dn_ks(M);
    const size_t es = elem_size(c->precision);
    const int n = c->bm_n > 0 ? c->bm_n : 1;
    c->qfrag.assign(es * (size_t)n * dn_qfrag_elems(M), 0);
    for (int k = 0; k < n; ++k)
        for (int which = 0; which < 2; ++which) {
            const double* A = c->bm_n > 0 ? (which ? &c->bm_Q2[(size_t)k * M * M] : &c->bm_Q[(size_t)k * M * M])
                                          : (which ? c->Q2.data() : c->Q.data());
            for (int f = 0; f < NF; ++f)
                for (int L = 0; L < 64; ++L) {
                    const int x = dn_row_state(M, f / KS, L % 16, es == 8),
                              y = dn_col_state(M, f % KS, L / 16, es == 8);
                    const double v = (x >= 0 && y >= 0) ? A[x * M + y] : 0.0;
                    const size_t i = (((size_t)k * 2 + which) * NF + f) * 64 + L;
                    if (es == 8) std::memcpy(&c->qfrag[8 * i], &v, 8);
                    else {
                        const float fv = (float)v;
                        std::memcpy(&c->qfrag[4 * i], &fv, 4);
                    }
                }
        }
}

// Copies made from the context's pageable host vectors by the
// allocation-free entry point may still be in flight: wait for them before
// those vectors change.
int settle_host_copies(pg_ctx* c) {
    if (!c->host_copies) return PG_OK;
    PG_HIP(c, hipStreamSynchronize(c->stream));
    c->host_copies = false;
    return PG_OK;
}

// ---------------------------------------------------------------- device scratch (see `scratch`)
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};
bool g_scratch_done[SCRATCH_MAX_DEVICES] = {};
hipError_t g_scratch_err[SCRATCH_MAX_DEVICES] = {};

// Called by pg_create with `device` current.
void scratch_setup(int device) {
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_done[device]) return;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_ptr[device] = (e == hipSuccess) ? p : nullptr;
    g_scratch_err[device] = e;
    g_scratch_done[device] = true;
}

// This device's scratch address, or NULL (with the reason in c->err).
char* scratch_base(pg_ctx* c) {
    if (c->device < 0 || c->device >= SCRATCH_MAX_DEVICES) {
        fail(c, PG_E_DEVICE, "device index beyond the allocation-free entry point's table");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[c->device]) {
        fail(c, PG_E_DEVICE, std::string("device scratch unavailable: ") +
                                 (g_scratch_done[c->device] ? hipGetErrorString(g_scratch_err[c->device])
                                                            : "not set up"));
        return nullptr;
    }
    return static_cast<char*>(g_scratch_ptr[c->device]);
}

// Layout of the context's buffers in the scratch (256-byte aligned), kept
// until the tree, patterns or model change.
void plan_scratch(pg_ctx* c) {
    if (!c->na_stale) return;
    prepare_dense_q(c);
    std::vector<BufSpec> specs = buffer_specs(ctx_dims(c), true);
    attach_sources(c, specs);
    c->na_specs.clear();
    size_t off = 0;
    for (const BufSpec& s : specs) {
        off = (off + 255) & ~size_t(255);
        c->na_specs.push_back(BufSpecRef{s.name, s.bytes, off, s.src});
        off += s.bytes;
    }
    c->na_total = off;
    c->na_stale = false;
}

// Allocate (or keep) the context's device buffers and upload its inputs.
int upload(pg_ctx* c) {
    int r = check_ready(c);
    if (r) return r;
    if (!c->dev_stale) return PG_OK;
    PG_HIP(c, hipSetDevice(c->device));
    if ((r = settle_host_copies(c))) return r;
    ensure_plan(c);
    prepare_dense_q(c);
    std::vector<BufSpec> specs = buffer_specs(ctx_dims(c), false);
    attach_sources(c, specs);
    for (const BufSpec& s : specs)
        if ((r = ensure_buf(c, s.name, s.bytes))) return r;
    for (const BufSpec& s : specs)
        if (s.src) PG_HIP(c, hipMemcpyAsync(c->bufs[s.name].ptr, s.src, s.bytes, hipMemcpyHostToDevice, c->stream));
    // pageable host sources: make sure the copies are done before the vectors move
    PG_HIP(c, hipStreamSynchronize(c->stream));
    fill_args(c, [&](const char* name) -> void* {
        auto it = c->bufs.find(name);
        return it == c->bufs.end() ? nullptr : it->second.ptr;
    }, c->args);
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

// Device state of a context for the serving scheduler: the host plan (on
// the thread that opens a session), the bytes it will take, and the upload
// (allocate and copy on `stream`, blocking) before its EvalArgs are handed out.
int ctx_plan(pg_ctx* c) {
    return guarded(c, [&] {
        int r = check_ready(c);
        if (r == PG_OK) ensure_plan(c);
        return r;
    });
}

int64_t ctx_need_bytes(pg_ctx* c, size_t granule) {
    ensure_plan(c);
    int64_t tot = 0;
    for (const BufSpec& s : buffer_specs(ctx_dims(c), false))
        tot += (int64_t)((std::max<size_t>(s.bytes, 256) + granule - 1) / granule * granule);
    return tot;
}

int ctx_prepare(pg_ctx* c, hipStream_t stream) {
    return guarded(c, [&] {
        hipStream_t own = c->stream;
        c->stream = stream;
        int r = upload(c);
        c->stream = own;
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
    scratch_setup(device);
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
        int r = settle_host_copies(c);
        if (r) return r;
        if ((r = check_tree(c, N, parent))) return r;
        if (c->n_tips != N) {
            c->patterns_set = false;
            c->bm_n = 0;  // branch models are per branch of the old tree
        }
        c->n_tips = N;
        c->parent.assign(parent, parent + 2 * N - 1);
        build_levels(N, c->children.data(), c->lv);
        c->tree_set = true;
        c->dev_stale = true;
        c->na_stale = true;
        c->plan_stale = true;
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
        if (int r0 = settle_host_copies(c)) return r0;
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
        c->na_stale = true;
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
        if (int r0 = settle_host_copies(c)) return r0;
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
        if (old_m != m) c->bm_n = 0;  // branch models have the old state count
        if (c->precision == PG_SPLIT_BF16) prepare_split_model(c);
        else if (dense_states(m)) prepare_dense_model(c);
        c->model_set = true;
        c->dev_stale = true;
        c->na_stale = true;
        c->plan_stale = true;
        c->have_partials = false;
        return PG_OK;
    });
}

int pg_set_branch_models(pg_ctx* c, int32_t n_models, const double* Q, const int32_t* model_of_branch) {
    if (!c) return PG_E_INVALID;
    if (!c->tree_set || !c->model_set) return fail(c, PG_E_STATE, "set the tree and the model first");
    if (n_models < 0) return fail(c, PG_E_INVALID, "n_models < 0");
    if (n_models > 0 && (!Q || !model_of_branch)) return fail(c, PG_E_INVALID, "NULL Q or model_of_branch");
    return guarded(c, [&] {
        if (int r0 = settle_host_copies(c)) return r0;
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
        if (c->precision == PG_SPLIT_BF16) split_qops(c);
        c->dev_stale = true;
        c->na_stale = true;
        c->have_partials = false;
        return PG_OK;
    });
}

int pg_logL_update(pg_ctx* c, int32_t n, const int32_t* branches, const double* t_new, double* logL) {
    if (!c) return PG_E_INVALID;
    if (n < 0 || (n > 0 && (!branches || !t_new)) || !logL) return fail(c, PG_E_INVALID, "bad arguments");
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
            UpdatePlan up;
            plan_update(N, c->parent.data(), c->children.data(), c->lv, n, branches, up);
            const std::vector<int>& list = up.list;
            const std::vector<Ent>& sched = up.sched;
            const std::vector<int>& off = up.level_off;
            const int H = (int)off.size() - 1;
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
            std::memcpy(hs + o_sched, sched.data(), sizeof(Ent) * sched.size());
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

int pg_logL_and_grad_noalloc(pg_ctx* c, const double* d_t, double* d_logL, double* d_grad) {
    if (!c) return PG_E_INVALID;
    if (!d_t || !d_logL) return fail(c, PG_E_INVALID, "NULL d_t or d_logL");
    return guarded(c, [&] {
        int r = check_ready(c);
        if (r) return r;
        PG_HIP(c, hipSetDevice(c->device));
        if (c->plan_stale || c->na_stale) {
            // host vectors are about to be re-read or replaced
            if ((r = settle_host_copies(c))) return r;
            ensure_plan(c);
            plan_scratch(c);
        }
        if (c->na_total > (size_t)PG_NOALLOC_MAX_BYTES)
            return fail(c, PG_E_INVALID, "the problem needs " + std::to_string(c->na_total) +
                                             " bytes of device scratch; the allocation-free entry point has " +
                                             std::to_string((long long)PG_NOALLOC_MAX_BYTES));
        char* base = scratch_base(c);
        if (!base) return PG_E_DEVICE;
        // inputs from the context's host copies into this device's scratch
        for (const BufSpecRef& s : c->na_specs)
            if (s.src) PG_HIP(c, hipMemcpyAsync(base + s.offset, s.src, s.bytes, hipMemcpyHostToDevice, c->stream));
        c->host_copies = true;
        EvalArgs a;
        fill_args(c, [&](const char* name) -> void* {
            for (const BufSpecRef& s : c->na_specs)
                if (std::strcmp(s.name, name) == 0) return base + s.offset;
            return nullptr;
        }, a);
        a.t = d_t;
        a.logL_out = d_logL;
        a.grad_out = d_grad;
        // no timing events here: creating them may allocate
        const bool timing = c->timing;
        c->timing = false;
        r = enqueue_forward(c, a, d_grad == nullptr);
        if (r == PG_OK && d_grad) r = enqueue_backward(c, a);
        c->timing = timing;
        return r;
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
    // the buffers an evaluation allocates, with the schedule at its largest
    // (top entries plus two clade lists: at most 2 (N - 1) entries, N level
    // offsets, two slot-range tables); each allocation is at least 256 B
    Dims d;
    d.N = N;
    d.S_pad = ((int64_t)S + TP - 1) / TP * TP;
    d.M = m;
    d.K = K;
    d.precision = precision;
    d.n_entries = 2 * ((int64_t)N - 1);
    d.n_level_off = N;
    d.n_cl_off = 2 * (node_slots(2) + 1);
    int64_t tot = 0;
    for (const BufSpec& sp : buffer_specs(d, false)) tot += (int64_t)std::max<size_t>(sp.bytes, 256);
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
