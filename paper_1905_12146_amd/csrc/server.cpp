// Serving scheduler: many independent gradient sessions on one GPU with
// admission by HBM footprint and continuous batching.
//
// A session owns a context (tree, patterns, model, resident partials); its
// host-side planning runs on the thread that opens it.  A session is
// admitted when the device bytes it needs fit the budget next to the
// admitted sessions and a session slot is free; otherwise it waits in
// arrival order.  Admission hands the session to an upload thread, which
// allocates its buffers and copies its inputs on a stream of its own while
// the worker keeps running batches.  The worker thread repeatedly takes, from every admitted
// session with a pending call, its oldest call and runs all of them as one
// batch: one launch each of the transition-matrix, post-order, pre-order and
// reduction kernels, whose blocks are mapped to (call, block-of-that-call).
// A call's blocks, their order and its reductions are the same whether it
// runs alone or in a batch, so its result is bitwise the same.  Calls that
// arrive while a batch runs join the next one.  Closing a session releases
// its device memory and lets waiting sessions in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "pg_internal.h"

using namespace pg;

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Call {
    int64_t session = 0;
    std::vector<double> t;
    bool want_grad = true;
    double logL = 0.0;
    std::vector<double> grad;
    int status = 0;
    int64_t t_submit = 0, t_start = 0, t_done = 0;
    bool done = false;
};

struct Session {
    pg_ctx* ctx = nullptr;
    int64_t reserve = 0;   // bytes reserved for it at admission (pool granularity)
    int64_t charged = 0;   // bytes charged to the budget while admitted
    int n_branches = 0;
    int M = 0;
    enum State { WAITING, UPLOADING, ADMITTED } state = WAITING;
    bool closing = false;
    std::deque<int64_t> pending;
};

// Device memory pool: freed session buffers are kept and handed to later
// sessions, so admission and closing seldom call hipMalloc / hipFree.
// Requests are rounded up to GRANULE; a cached block is reused for a request
// when it is at most 1/8 larger.  Blocks handed out plus blocks cached never
// exceed the budget: cached blocks (largest first) are freed before a new
// allocation would pass it.  Thread-safe.
class Pool : public DeviceAllocator {
public:
    static constexpr size_t GRANULE = 65536;
    explicit Pool(size_t budget) : budget_(budget) {}
    ~Pool() override { trim(0); }
    void* acquire(size_t bytes, size_t* granted) override {
        std::lock_guard<std::mutex> lk(mu_);
        bytes = round(bytes);
        auto it = free_.lower_bound(bytes);
        if (it != free_.end() && it->first <= bytes + bytes / 8) {
            void* p = it->second;
            const size_t sz = it->first;
            cached_ -= sz;
            used_ += sz;
            size_[p] = sz;
            free_.erase(it);
            *granted = sz;
            return p;
        }
        // keep used + cached + bytes within the budget
        trim(budget_ > used_ + bytes ? budget_ - used_ - bytes : 0);
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            trim(0);  // give cached memory back and try once more
            if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        }
        used_ += bytes;
        size_[p] = bytes;
        *granted = bytes;
        return p;
    }
    void release(void* p, size_t) override {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = size_.find(p);
        const size_t bytes = it->second;
        size_.erase(it);
        used_ -= bytes;
        free_.emplace(bytes, p);
        cached_ += bytes;
        trim(budget_ > used_ ? budget_ - used_ : 0);
    }
    // device bytes held: handed out plus cached
    size_t held() {
        std::lock_guard<std::mutex> lk(mu_);
        return used_ + cached_;
    }
    static size_t round(size_t b) { return (b + GRANULE - 1) / GRANULE * GRANULE; }

private:
    void trim(size_t limit) {  // caller holds mu_ (or is the destructor)
        while (cached_ > limit && !free_.empty()) {
            auto it = std::prev(free_.end());
            (void)hipFree(it->second);
            cached_ -= it->first;
            free_.erase(it);
        }
    }
    std::mutex mu_;
    size_t budget_;
    size_t used_ = 0, cached_ = 0;
    std::multimap<size_t, void*> free_;
    std::map<void*, size_t> size_;
};

}  // namespace

struct pg_server {
    int device = 0, precision = PG_FP64;
    int64_t budget = 0, in_use = 0, peak = 0;
    int max_sessions = 0;
    hipStream_t stream = nullptr;
    std::string err;
    Pool* pool = nullptr;

    hipStream_t upload_stream = nullptr;  // session uploads (default priority)

    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_upload;
    std::deque<int64_t> upload_q;          // admitted sessions awaiting their upload
    std::thread uploader;
    bool stop_upload = false;              // set once the worker has ended
    std::map<int64_t, Session> sessions;   // ordered by id = arrival order
    std::deque<int64_t> admit_q;
    std::map<int64_t, Call> calls;
    int64_t next_session = 1, next_ticket = 1;
    bool stop = false;
    std::thread worker;

    // staging: one pinned host buffer and one device buffer per direction
    void* h_in = nullptr;
    void* d_in = nullptr;
    size_t in_cap = 0;
    void* h_out = nullptr;
    void* d_out = nullptr;
    size_t out_cap = 0;

    // statistics
    int64_t steps = 0, calls_done = 0, batched_calls = 0, max_batch = 0, admitted_total = 0;
    int64_t max_waiting = 0;
    int64_t peak_held = 0;                 // largest device bytes held by the pool
};

namespace {

size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

int grow(pg_server* s, void** h, void** d, size_t* cap, size_t need) {
    if (*cap >= need) return PG_OK;
    size_t n = std::max(need, *cap * 2);
    if (*h) (void)hipHostFree(*h);
    if (*d) (void)hipFree(*d);
    *h = nullptr;
    *d = nullptr;
    *cap = 0;
    if (hipHostMalloc(h, n) != hipSuccess) return PG_E_OOM;
    if (hipMalloc(d, n) != hipSuccess) return PG_E_OOM;
    *cap = n;
    (void)s;
    return PG_OK;
}

// Admit waiting sessions in arrival order while they fit: reserve their
// bytes and hand them to the upload thread.  Caller holds mu.
void admit(pg_server* s) {
    int admitted = 0;
    for (auto& kv : s->sessions)
        if (kv.second.state != Session::WAITING) ++admitted;
    while (!s->admit_q.empty()) {
        auto it = s->sessions.find(s->admit_q.front());
        if (it == s->sessions.end()) {
            s->admit_q.pop_front();
            continue;
        }
        Session& ss = it->second;
        if (admitted >= s->max_sessions || s->in_use + ss.reserve > s->budget) break;
        s->admit_q.pop_front();
        ss.state = Session::UPLOADING;
        ss.charged = ss.reserve;
        s->in_use += ss.charged;
        s->peak = std::max(s->peak, s->in_use);
        ++admitted;
        ++s->admitted_total;
        s->upload_q.push_back(it->first);
        s->cv_upload.notify_one();
    }
    s->max_waiting = std::max<int64_t>(s->max_waiting, (int64_t)s->admit_q.size());
}

// Upload thread: allocate and copy each admitted session's device state on
// its own stream, without the lock, while batches keep running.
void upload_loop(pg_server* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        s->cv_upload.wait(lk, [&] { return s->stop_upload || !s->upload_q.empty(); });
        if (s->upload_q.empty()) break;  // the worker has ended and nothing is left
        const int64_t id = s->upload_q.front();
        s->upload_q.pop_front();
        Session& ss = s->sessions.at(id);  // not reaped while UPLOADING
        pg_ctx* ctx = ss.ctx;
        lk.unlock();
        const int r = ctx_prepare(ctx, s->upload_stream);
        const int64_t held = (int64_t)s->pool->held();
        lk.lock();
        s->peak_held = std::max(s->peak_held, held);
        if (r == PG_OK) {
            // charge what the pool actually handed out
            const int64_t got = pg_device_bytes(ctx);
            s->in_use += got - ss.charged;
            ss.charged = got;
            s->peak = std::max(s->peak, s->in_use);
        }
        if (r != PG_OK) {
            // fail every pending call of this session and wake their waiters
            s->err = ctx_error(ctx);
            for (int64_t tk : ss.pending) {
                Call& c = s->calls[tk];
                c.status = r;
                c.done = true;
                c.t_done = now_ns();
            }
            ss.pending.clear();
            ss.closing = true;
            ss.state = Session::ADMITTED;  // reaped with its charge
            s->cv_done.notify_all();
        } else {
            ss.state = Session::ADMITTED;
        }
        s->cv_work.notify_all();
    }
}

// Free sessions that asked to close and have no pending calls.  Caller holds mu.
void reap(pg_server* s) {
    for (auto it = s->sessions.begin(); it != s->sessions.end();) {
        Session& ss = it->second;
        if (ss.closing && ss.pending.empty() && ss.state != Session::UPLOADING) {
            if (ss.state == Session::ADMITTED) s->in_use -= ss.charged;
            pg_destroy(ss.ctx);
            it = s->sessions.erase(it);
        } else {
            ++it;
        }
    }
}

struct Item {
    int64_t ticket;
    Session* sess;
    Call* call;
    EvalArgs args;
};

// Run one batch of calls with the same state count; mu is not held.
int run_group(pg_server* s, std::vector<Item>& items) {
    const int n = (int)items.size();
    // input layout: [t of every call][EvalArgs x n][top-level EvalArgs x n]
    // [pmat map][trav map][gsum map][clade map]
    size_t t_total = 0;
    int pm = 0, tr = 0, gs = 0, cl = 0;
    size_t post_lds = 0, pre_lds = 0, clade_lds = 0, top_lds = 0;
    bool top_kernels = true;
    for (auto& it : items) {
        // a plan with clades always takes the clade launches
        if (it.args.n_cl > 0 && clade_blocks(it.args, s->precision) == 0) return PG_E_DEVICE;
        const EvalArgs top = clade_top_args(it.args, s->precision);
        t_total += it.args.n_branches;
        pm += pmat_blocks(it.args, s->precision);
        tr += traversal_blocks(it.args);
        gs += gsum_total_blocks(it.args);
        cl += clade_blocks(it.args, s->precision);
        post_lds = std::max(post_lds, post_lds_bytes(top, s->precision));
        pre_lds = std::max(pre_lds, pre_lds_bytes(top, s->precision));
        clade_lds = std::max(clade_lds, clade_lds_bytes(it.args, s->precision));
        // the top-level launches serve the batch when they serve every request
        top_kernels = top_kernels && it.args.n_cl > 0 && top_launch_ok(top, s->precision);
        top_lds = std::max(top_lds, top_launch_lds(top, s->precision));
    }
    const size_t off_t = 0;
    const size_t off_args = align16(off_t + sizeof(double) * t_total);
    const size_t off_top = align16(off_args + sizeof(EvalArgs) * n);
    const size_t off_pm = align16(off_top + sizeof(EvalArgs) * n);
    const size_t off_tr = align16(off_pm + sizeof(int2) * pm);
    const size_t off_gs = align16(off_tr + sizeof(int2) * tr);
    const size_t off_cl = align16(off_gs + sizeof(int2) * gs);
    const size_t in_bytes = align16(off_cl + sizeof(int2) * cl);
    // output layout: [logL x n][status x n][grad of every call]
    const size_t o_logl = 0;
    const size_t o_status = align16(sizeof(double) * n);
    const size_t o_grad = align16(o_status + sizeof(int) * n);
    const size_t out_bytes = align16(o_grad + sizeof(double) * t_total);
    int r;
    if ((r = grow(s, &s->h_in, &s->d_in, &s->in_cap, in_bytes))) return r;
    if ((r = grow(s, &s->h_out, &s->d_out, &s->out_cap, out_bytes))) return r;
    char* hi = static_cast<char*>(s->h_in);
    char* di = static_cast<char*>(s->d_in);
    char* dout = static_cast<char*>(s->d_out);
    double* ht = reinterpret_cast<double*>(hi + off_t);
    EvalArgs* ha = reinterpret_cast<EvalArgs*>(hi + off_args);
    EvalArgs* htop = reinterpret_cast<EvalArgs*>(hi + off_top);
    int2* hpm = reinterpret_cast<int2*>(hi + off_pm);
    int2* htr = reinterpret_cast<int2*>(hi + off_tr);
    int2* hgs = reinterpret_cast<int2*>(hi + off_gs);
    int2* hcl = reinterpret_cast<int2*>(hi + off_cl);
    size_t toff = 0;
    int ipm = 0, itr = 0, igs = 0, icl = 0;
    for (int q = 0; q < n; ++q) {
        Item& it = items[q];
        EvalArgs a = it.args;
        std::memcpy(ht + toff, it.call->t.data(), sizeof(double) * a.n_branches);
        a.t = reinterpret_cast<const double*>(di + off_t) + toff;
        a.logL_out = reinterpret_cast<double*>(dout + o_logl) + q;
        a.status = reinterpret_cast<int*>(dout + o_status) + q;
        a.grad_out = reinterpret_cast<double*>(dout + o_grad) + toff;
        ha[q] = a;
        htop[q] = clade_top_args(a, s->precision);
        for (int b = 0, nb = pmat_blocks(a, s->precision); b < nb; ++b) hpm[ipm++] = make_int2(q, b);
        for (int b = 0, nb = traversal_blocks(a); b < nb; ++b) htr[itr++] = make_int2(q, b);
        for (int b = 0, nb = gsum_total_blocks(a); b < nb; ++b) hgs[igs++] = make_int2(q, b);
        for (int b = 0, nb = clade_blocks(a, s->precision); b < nb; ++b) hcl[icl++] = make_int2(q, b);
        toff += a.n_branches;
    }
    hipError_t e;
    if ((e = hipMemcpyAsync(s->d_in, s->h_in, in_bytes, hipMemcpyHostToDevice, s->stream)) != hipSuccess)
        return PG_E_DEVICE;
    BatchLaunch bl{};
    bl.M = items[0].args.M;
    bl.precision = s->precision;
    bl.reqs = reinterpret_cast<const EvalArgs*>(di + off_args);
    bl.reqs_top = reinterpret_cast<const EvalArgs*>(di + off_top);
    bl.pmat_map = reinterpret_cast<const int2*>(di + off_pm);
    bl.trav_map = reinterpret_cast<const int2*>(di + off_tr);
    bl.gsum_map = reinterpret_cast<const int2*>(di + off_gs);
    bl.clade_map = reinterpret_cast<const int2*>(di + off_cl);
    bl.pmat_blocks = pm;
    bl.trav_blocks = tr;
    bl.gsum_blocks = gs;
    bl.clade_blocks = cl;
    bl.post_lds = post_lds;
    bl.pre_lds = pre_lds;
    bl.top_kernels = top_kernels ? 1 : 0;
    bl.top_lds = top_lds;
    bl.clade_lds = clade_lds;
    if ((e = launch_batch(bl, s->stream)) != hipSuccess) return PG_E_DEVICE;
    if ((e = hipMemcpyAsync(s->h_out, s->d_out, out_bytes, hipMemcpyDeviceToHost, s->stream)) != hipSuccess)
        return PG_E_DEVICE;
    if ((e = hipStreamSynchronize(s->stream)) != hipSuccess) return PG_E_DEVICE;
    const char* ho = static_cast<const char*>(s->h_out);
    toff = 0;
    for (int q = 0; q < n; ++q) {
        Call* c = items[q].call;
        c->logL = reinterpret_cast<const double*>(ho + o_logl)[q];
        const int st = reinterpret_cast<const int*>(ho + o_status)[q];
        c->status = st == 1 ? PG_E_INVALID : st == 2 ? PG_E_ZERO_LIK : PG_OK;
        const int B = items[q].args.n_branches;
        if (c->want_grad) {
            const double* g = reinterpret_cast<const double*>(ho + o_grad) + toff;
            c->grad.assign(g, g + B);
        }
        toff += B;
    }
    return PG_OK;
}

void worker_loop(pg_server* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        reap(s);
        admit(s);
        std::vector<Item> batch;
        for (auto& kv : s->sessions) {
            Session& ss = kv.second;
            if (ss.state != Session::ADMITTED || ss.pending.empty()) continue;
            const int64_t tk = ss.pending.front();
            Call& c = s->calls[tk];
            batch.push_back(Item{tk, &ss, &c, ctx_args(ss.ctx)});
        }
        if (batch.empty()) {
            bool uploading = !s->upload_q.empty();
            for (auto& kv : s->sessions) uploading = uploading || kv.second.state == Session::UPLOADING;
            if (s->stop && !uploading) break;
            s->cv_work.wait(lk);
            continue;
        }
        const int64_t t0 = now_ns();
        for (auto& it : batch) it.call->t_start = t0;
        lk.unlock();
        // group by state count (one kernel instantiation per group)
        std::map<int, std::vector<Item>> groups;
        for (auto& it : batch) groups[it.args.M].push_back(it);
        std::map<int64_t, int> result;
        for (auto& g : groups) {
            const int r = run_group(s, g.second);
            for (auto& it : g.second) result[it.ticket] = r;
        }
        lk.lock();
        const int64_t t1 = now_ns();
        for (auto& it : batch) {
            Call& c = *it.call;
            if (result[it.ticket] != PG_OK) c.status = result[it.ticket];
            c.t_done = t1;
            c.done = true;
            it.sess->pending.pop_front();
        }
        ++s->steps;
        s->calls_done += (int64_t)batch.size();
        s->batched_calls += (int64_t)batch.size();
        s->max_batch = std::max<int64_t>(s->max_batch, (int64_t)batch.size());
        s->cv_done.notify_all();
    }
}

}  // namespace

extern "C" {

int pg_server_create(int device, int precision, int64_t hbm_budget, int32_t max_sessions, pg_server** out) {
    if (!out || hbm_budget <= 0 || max_sessions < 1) return PG_E_INVALID;
    *out = nullptr;
    pg_ctx* probe = nullptr;
    int r = pg_create(device, precision, &probe);
    if (r != PG_OK) return r;
    pg_destroy(probe);
    pg_server* s = nullptr;
    try {
        s = new pg_server();
    } catch (...) {
        return PG_E_OOM;
    }
    s->device = device;
    s->precision = precision;
    s->budget = hbm_budget;
    s->max_sessions = max_sessions;
    if (hipSetDevice(device) != hipSuccess || hipStreamCreate(&s->stream) != hipSuccess) {
        delete s;
        return PG_E_DEVICE;
    }
    if (hipStreamCreate(&s->upload_stream) != hipSuccess) {
        (void)hipStreamDestroy(s->stream);
        delete s;
        return PG_E_DEVICE;
    }
    s->pool = new Pool((size_t)hbm_budget);
    try {
        s->worker = std::thread(worker_loop, s);
    } catch (...) {
        delete s->pool;
        (void)hipStreamDestroy(s->upload_stream);
        (void)hipStreamDestroy(s->stream);
        delete s;
        return PG_E_DEVICE;
    }
    try {
        s->uploader = std::thread(upload_loop, s);
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->cv_work.notify_all();
        s->worker.join();
        delete s->pool;
        (void)hipStreamDestroy(s->upload_stream);
        (void)hipStreamDestroy(s->stream);
        delete s;
        return PG_E_DEVICE;
    }
    *out = s;
    return PG_OK;
}

void pg_server_destroy(pg_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (auto& kv : s->sessions) kv.second.closing = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop_upload = true;
    }
    s->cv_upload.notify_all();
    if (s->uploader.joinable()) s->uploader.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto& kv : s->sessions) pg_destroy(kv.second.ctx);
        s->sessions.clear();
    }
    (void)hipSetDevice(s->device);
    if (s->h_in) (void)hipHostFree(s->h_in);
    if (s->h_out) (void)hipHostFree(s->h_out);
    if (s->d_in) (void)hipFree(s->d_in);
    if (s->d_out) (void)hipFree(s->d_out);
    delete s->pool;
    if (s->upload_stream) (void)hipStreamDestroy(s->upload_stream);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

const char* pg_server_last_error(const pg_server* s) { return s ? s->err.c_str() : ""; }

int pg_server_open(pg_server* s, int32_t n_tips, const int32_t* parent, int32_t n_patterns, int32_t n_states,
                   const uint64_t* tip_masks, const double* weights, const double* Q, const double* root_freqs,
                   int32_t n_cats, const double* cat_rates, const double* cat_weights, int64_t* session) {
    if (!s || !session) return PG_E_INVALID;
    pg_ctx* c = nullptr;
    try {
        c = ctx_new_session(s->device, s->precision, s->stream, s->pool);
    } catch (...) {
        return PG_E_OOM;
    }
    int r;
    if ((r = pg_set_tree(c, n_tips, parent)) != PG_OK ||
        (r = pg_set_patterns(c, n_patterns, n_states, tip_masks, weights)) != PG_OK ||
        (r = pg_set_model(c, n_states, Q, root_freqs, n_cats, cat_rates, cat_weights)) != PG_OK) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->err = pg_last_error(c);
        pg_destroy(c);
        return r;
    }
    // host planning here, on the caller's thread; the reservation covers the
    // pool's rounding and its reuse of blocks up to 1/8 larger
    if ((r = ctx_plan(c)) != PG_OK) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->err = pg_last_error(c);
        pg_destroy(c);
        return r;
    }
    const int64_t need = ctx_need_bytes(c, Pool::GRANULE);
    const int64_t reserve = need + need / 8;
    std::lock_guard<std::mutex> lk(s->mu);
    if (reserve > s->budget) {
        s->err = "session needs up to " + std::to_string(reserve) + " device bytes, more than the budget " +
                 std::to_string(s->budget);
        pg_destroy(c);
        return PG_E_OOM;
    }
    const int64_t id = s->next_session++;
    Session& ss = s->sessions[id];
    ss.ctx = c;
    ss.reserve = reserve;
    ss.n_branches = 2 * n_tips - 2;
    ss.M = n_states;
    s->admit_q.push_back(id);
    *session = id;
    s->cv_work.notify_all();
    return PG_OK;
}

int pg_server_submit(pg_server* s, int64_t session, const double* t, int32_t want_grad, int64_t* ticket) {
    if (!s || !t || !ticket) return PG_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->sessions.find(session);
    if (it == s->sessions.end() || it->second.closing) {
        s->err = "unknown or closing session";
        return PG_E_STATE;
    }
    Session& ss = it->second;
    for (int b = 0; b < ss.n_branches; ++b)
        if (!(t[b] >= 0.0) || t[b] == INFINITY) {
            s->err = "branch length " + std::to_string(b) + " is not finite and >= 0";
            return PG_E_INVALID;
        }
    const int64_t tk = s->next_ticket++;
    Call& c = s->calls[tk];
    c.session = session;
    c.t.assign(t, t + ss.n_branches);
    c.want_grad = want_grad != 0;
    c.t_submit = now_ns();
    ss.pending.push_back(tk);
    *ticket = tk;
    s->cv_work.notify_all();
    return PG_OK;
}

int pg_server_wait(pg_server* s, int64_t ticket, double* logL, double* grad, int64_t* latency_ns) {
    if (!s) return PG_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->calls.find(ticket);
    if (it == s->calls.end()) {
        s->err = "unknown ticket";
        return PG_E_STATE;
    }
    s->cv_done.wait(lk, [&] { return it->second.done; });
    Call& c = it->second;
    if (logL) *logL = c.logL;
    if (grad && c.want_grad && !c.grad.empty()) std::memcpy(grad, c.grad.data(), sizeof(double) * c.grad.size());
    if (latency_ns) *latency_ns = c.t_done - c.t_submit;
    const int r = c.status;
    s->calls.erase(it);
    return r;
}

int pg_server_close(pg_server* s, int64_t session) {
    if (!s) return PG_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->sessions.find(session);
    if (it == s->sessions.end()) return PG_E_STATE;
    it->second.closing = true;
    auto q = std::find(s->admit_q.begin(), s->admit_q.end(), session);
    if (q != s->admit_q.end() && it->second.pending.empty()) s->admit_q.erase(q);
    s->cv_work.notify_all();
    return PG_OK;
}

int pg_server_stats(pg_server* s, int64_t* out, int32_t n) {
    if (!s || !out) return PG_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    int64_t admitted = 0;
    for (auto& kv : s->sessions)
        if (kv.second.state != Session::WAITING) ++admitted;
    const int64_t v[PG_SRV_STAT_COUNT] = {s->steps,     s->calls_done, s->max_batch, s->admitted_total,
                                          admitted,     (int64_t)s->admit_q.size(), s->in_use, s->peak,
                                          s->max_waiting, s->peak_held};
    for (int i = 0; i < n && i < PG_SRV_STAT_COUNT; ++i) out[i] = v[i];
    return PG_OK;
}

}  // extern "C"
