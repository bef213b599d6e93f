// Host check of the traversal planners (paper_1905_12146_amd/csrc/plan.cpp).
//
// Built by tests/test_plan.py with g++ and -fsanitize=address,undefined
// together with plan.cpp, and run on trees written by the test:
//
//     plan_check <tree file>         tree file: N, then parent[0..2N-2]
//
// For a grid of kernel configurations (state count, element size, node
// slots, clade walks and top region on or off) it plans the traversal and
// then replays, on the host, the index arithmetic of the kernels' walks:
// every schedule entry read (including the clade walks' reads past the end
// of a list, which reload the last entry), every load address formed (the
// dummy loads of a tip child's message slot and of an internal child's tip
// code, the matrix entries, the q of a clade root), every LDS stack and top
// region slot, and the data flow (a message or q vector is read only after
// the walk that writes it).  It also checks that every internal node is
// scheduled exactly once in each pass, the slot assignment of the top-level
// launches next to the clade launches, and the dirty-path schedules of
// partial re-evaluation for random sets of changed branches.
//
// Exit status 0 when every check passes; otherwise the first failure is
// printed and the status is 1.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "../paper_1905_12146_amd/csrc/plan.h"

using namespace pg;

namespace {

int g_checks = 0;
int g_top_plans = 0;  // plans replayed by check_top_launches

#define CHECK(cond, ...)                                                     \
    do {                                                                     \
        ++g_checks;                                                          \
        if (!(cond)) {                                                       \
            std::fprintf(stderr, "FAIL %s:%d: %s: ", __FILE__, __LINE__, #cond); \
            std::fprintf(stderr, __VA_ARGS__);                               \
            std::fprintf(stderr, "\n");                                      \
            std::exit(1);                                                    \
        }                                                                    \
    } while (0)

struct Tree {
    int N = 0;
    std::vector<int> parent;
    std::vector<Kids> ch;
    TreeLevels lv;
};

bool read_tree(const char* path, Tree& t) {
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    if (std::fscanf(f, "%d", &t.N) != 1 || t.N < 2) return false;
    const int n_nodes = 2 * t.N - 1;
    t.parent.assign(n_nodes, -1);
    for (int v = 0; v < n_nodes; ++v)
        if (std::fscanf(f, "%d", &t.parent[v]) != 1) return false;
    std::fclose(f);
    // children in order of appearance, as the library's tree check fills them
    t.ch.assign(n_nodes, Kids{-1, -1});
    std::vector<int> nchild(n_nodes, 0);
    for (int v = 0; v < n_nodes - 1; ++v) {
        const int p = t.parent[v];
        CHECK(p >= t.N && p < n_nodes, "node %d has parent %d", v, p);
        if (nchild[p] == 0) t.ch[p].x = v;
        else t.ch[p].y = v;
        ++nchild[p];
    }
    for (int k = t.N; k < n_nodes; ++k) CHECK(nchild[k] == 2, "internal node %d has %d children", k, nchild[k]);
    CHECK(t.parent[n_nodes - 1] == -1, "root is not last");
    build_levels(t.N, t.ch.data(), t.lv);
    return true;
}

// The address space of one evaluation's buffers, by node or branch index.
struct Bounds {
    int N, B, n_blocks;  // branches, message / q blocks (internal nodes)
    void msg_block(int node, const char* what) const {
        CHECK(node >= N && node - N < n_blocks, "%s: node %d outside the %d vector blocks", what, node, n_blocks);
    }
    void code_row(int row, const char* what) const { CHECK(row >= 0 && row < N, "%s: tip row %d", what, row); }
    void pmat(int b, const char* what) const { CHECK(b >= 0 && b < B, "%s: branch %d of %d", what, b, B); }
};

// Levels and top-region checks shared by the two passes.
struct Walk {
    const Tree& t;
    const TraversalPlan& pl;
    const PlanParams& pp;
    Bounds bd;
    int root;
    std::vector<char> msg_written, q_hbm, q_lds;

    Walk(const Tree& t_, const TraversalPlan& pl_, const PlanParams& pp_)
        : t(t_), pl(pl_), pp(pp_), root(2 * t_.N - 2) {
        bd = Bounds{t.N, 2 * t.N - 2, t.N - 1};
    }

    const Ent& top_entry(int idx) const {
        CHECK(idx >= 0 && idx < pl.n_top, "top entry %d of %d", idx, pl.n_top);
        return pl.sched[idx];
    }
    // clade list of the post (pre) kernel: entries n_top.. (n_top + n_cl..)
    const Ent& clade_entry(bool pre, int idx) const {
        CHECK(idx >= 0 && idx < pl.n_cl, "clade entry %d of %d", idx, pl.n_cl);
        const size_t base = (size_t)pl.n_top + ((pre && !pl.one_list) ? pl.n_cl : 0);
        CHECK(base + idx < pl.sched.size(), "clade entry beyond the schedule");
        return pl.sched[base + idx];
    }
    int slot_beg(bool pre, int ns) const { return pl.cl_off.at(pre ? pl.ns_post + 1 + ns : ns); }
    int slot_end(bool pre, int ns) const { return pl.cl_off.at(pre ? pl.ns_post + 1 + ns + 1 : ns + 1); }

    // a child's loads in the level walks (child_load)
    void child_load(int c, const char* what) {
        if (c < t.N) {
            bd.code_row(c, what);
            if (pp.clades) bd.pmat(c, what);  // a tip's row-distributed matrix entry
        } else {
            bd.msg_block(c, what);
            CHECK(msg_written[c], "%s: message of node %d read before it is written", what, c);
        }
    }

    // ---------------------------------------------------------------- post-order
    void post() {
        msg_written.assign(2 * t.N - 1, 0);
        std::vector<int> seen(2 * t.N - 1, 0);
        if (pl.n_cl) {
            CHECK(pp.n_states * pp.n_states == TP, "clade walks need row-distributed matrices (M*M = TP)");
            std::vector<char> done = msg_written;  // clades see only their own slot's writes
            for (int ns = 0; ns < pl.ns_post; ++ns) post_clades(ns, seen, done);
            msg_written = done;  // workgroup barrier after the clades
        }
        for (int h = 0; h < pl.n_levels(); ++h) {
            std::vector<char> written = msg_written;
            const int end = pl.level_off[h + 1];
            for (int ns = 0; ns < pl.ns_post; ++ns)
                for (int idx = pl.level_off[h] + ns; idx < end; idx += pl.ns_post) {
                    const Ent& e = top_entry(idx);
                    child_load(e.y, "post level child 0");
                    child_load(e.z, "post level child 1");
                    CHECK(t.ch[e.x].x == e.y || t.ch[e.x].x == e.z, "entry children of node %d", e.x);
                    CHECK((e.y == t.ch[e.x].x && e.z == t.ch[e.x].y) || (e.y == t.ch[e.x].y && e.z == t.ch[e.x].x),
                          "entry children of node %d", e.x);
                    if (e.x != root) {
                        bd.pmat(e.x, "post level own matrix");
                        bd.msg_block(e.x, "post level message write");
                        written[e.x] = 1;
                    }
                    ++seen[e.x];
                }
            msg_written = written;  // workgroup barrier after each level
        }
        for (int k = t.N; k < 2 * t.N - 1; ++k) CHECK(seen[k] == 1, "post-order visits node %d %d times", k, seen[k]);
    }

    void post_clades(int ns, std::vector<int>& seen, std::vector<char>& done) {
        const int beg = slot_beg(false, ns), end = slot_end(false, ns);
        if (beg >= end) return;
        std::vector<char> own(2 * t.N - 1, 0);
        std::vector<int> stack;
        int acc = -1;
        auto entry = [&](int i) { return clade_entry(false, std::min(i, end - 1)); };
        auto load = [&](const Ent& e) {
            bd.code_row(e.y < t.N ? e.y : 0, "post clade code 0");
            bd.code_row(e.z < t.N ? e.z : 0, "post clade code 1");
            bd.pmat(e.y, "post clade child 0 matrix");
            bd.pmat(e.z, "post clade child 1 matrix");
            bd.pmat(e.x, "post clade own matrix");
        };
        Ent nd = entry(beg), nn = entry(beg + 1);
        load(nd);
        for (int i = beg;; ++i) {
            const Ent n2 = entry(i + 2);
            load(nn);
            int m0 = -1, m1 = -1;
            if (nd.y < t.N) {
                m0 = nd.y;
            } else if (nd.z < t.N) {
                m0 = acc;
            } else {
                CHECK(!stack.empty(), "post clade stack underflow at node %d", nd.x);
                m0 = stack.back();
                stack.pop_back();
            }
            m1 = (nd.z < t.N) ? nd.z : acc;
            CHECK(m0 == nd.y, "post clade node %d: first child message is node %d's, not %d's", nd.x, m0, nd.y);
            CHECK(m1 == nd.z, "post clade node %d: second child message is node %d's, not %d's", nd.x, m1, nd.z);
            if (nd.y >= t.N) CHECK(own[nd.y], "post clade: child %d not done before %d", nd.y, nd.x);
            if (nd.z >= t.N) CHECK(own[nd.z], "post clade: child %d not done before %d", nd.z, nd.x);
            CHECK(nd.x != root, "the root is in a clade");
            bd.msg_block(nd.x, "post clade message write");
            own[nd.x] = 1;
            done[nd.x] = 1;
            ++seen[nd.x];
            if (nd.w & CL_STACK) {
                stack.push_back(nd.x);
                CHECK((int)stack.size() <= pl.depth, "post clade stack depth %zu > %d", stack.size(), pl.depth);
            } else {
                acc = nd.x;
            }
            if (i + 1 >= end) break;
            nd = nn;
            nn = n2;
        }
        CHECK(stack.empty(), "post clade stack not empty at the end of slot %d", ns);
    }

    // ---------------------------------------------------------------- pre-order
    void pre() {
        q_hbm.assign(2 * t.N - 1, 0);
        q_lds.assign(pl.top_nodes + 1, 0);
        std::vector<int> seen(2 * t.N - 1, 0);
        const int H = pl.n_levels();
        CHECK(pl.top_level >= 0 && pl.top_level <= H, "top level %d of %d", pl.top_level, H);
        CHECK((size_t)pl.top_nodes * pp.n_states * TP * pp.elem_bytes <= (size_t)TOP_LDS_MAX, "top region LDS");
        int region_count = 0;
        for (int h = H - 1; h >= pl.top_level; --h) {
            const int n_h = pl.level_off[h + 1] - pl.level_off[h];
            CHECK(n_h <= pl.ns_pre, "top region level %d has %d nodes for %d slots", h, n_h, pl.ns_pre);
            region_count += n_h;
            std::vector<char> lds = q_lds;
            for (int ns = 0; ns < pl.ns_pre; ++ns) {
                const int idx = pl.level_off[h] + ns;
                if (idx >= pl.level_off[h + 1]) continue;
                const Ent& e = top_entry(idx);
                if (e.x != root) {
                    const int sl = e.w & 0xff;
                    CHECK(sl >= 1 && sl <= pl.top_nodes, "top region node %d slot %d", e.x, sl);
                    CHECK(q_lds[sl], "top region: q of node %d read from LDS before it is written", e.x);
                }
                pre_children(e, true, lds, seen);
            }
            q_lds = lds;
        }
        CHECK(region_count == pl.top_nodes, "top region holds %d nodes, planned %d", region_count, pl.top_nodes);
        for (int h = pl.top_level - 1; h >= 0; --h) {
            std::vector<char> hbm = q_hbm;
            const int end = pl.level_off[h + 1];
            for (int ns = 0; ns < pl.ns_pre; ++ns)
                for (int idx = pl.level_off[h] + ns; idx < end; idx += pl.ns_pre) {
                    const Ent& e = top_entry(idx);
                    if (e.x != root) {
                        bd.msg_block(e.x, "pre level q read");
                        CHECK(q_hbm[e.x], "pre level: q of node %d read before it is written", e.x);
                    }
                    std::vector<char> unused;
                    pre_children(e, false, unused, seen, &hbm);
                }
            q_hbm = hbm;
        }
        if (pl.n_cl)
            for (int ns = 0; ns < pl.ns_pre; ++ns) pre_clades(ns, seen);
        for (int k = t.N; k < 2 * t.N - 1; ++k) CHECK(seen[k] == 1, "pre-order visits node %d %d times", k, seen[k]);
    }

    // both children of a level-walk entry: loads, gradient partial, q destination
    void pre_children(const Ent& e, bool region, std::vector<char>& lds, std::vector<int>& seen,
                      std::vector<char>* hbm = nullptr) {
        ++seen[e.x];
        const int kids[2] = {e.y, e.z};
        for (int j = 0; j < 2; ++j) {
            const int c = kids[j];
            child_load(c, "pre level child");
            bd.pmat(c, "pre child matrix");
            CHECK(c >= 0 && c < bd.B, "gradient partial of branch %d", c);
            if (c < t.N) continue;
            const int sl = region ? (e.w >> (8 * (j + 1))) & 0xff : 0;
            if (sl) {
                CHECK(sl <= pl.top_nodes, "top region child slot %d", sl);
                lds[sl] = 1;
            } else {
                bd.msg_block(c, "pre q write");
                if (hbm) (*hbm)[c] = 1;
                else q_hbm[c] = 1;  // the region's last level ends with a full barrier
            }
        }
    }

    void pre_clades(int ns, std::vector<int>& seen) {
        const int beg = slot_beg(true, ns), end = slot_end(true, ns), n = end - beg;
        if (n <= 0) return;
        constexpr int DEPTH = 2;  // entries in flight in the kernel's ring
        std::vector<int> stack;
        int acc = -1;
        auto entry = [&](int i) {
            const int idx = end - 1 - std::min(i, n - 1);
            CHECK(idx >= beg && idx < end, "pre clade entry %d outside slot %d's range", idx, ns);
            return clade_entry(true, idx);
        };
        auto load = [&](const Ent& e) {
            bd.msg_block((e.w & CL_ROOT) ? e.x : t.N, "pre clade q");  // offset 0 is block 0 (node N)
            for (int c : {e.y, e.z}) {
                bd.msg_block(c < t.N ? t.N : c, "pre clade child message");
                bd.code_row(c < t.N ? c : 0, "pre clade child code");
                bd.pmat(c, "pre clade child matrix");
            }
        };
        Ent nd[DEPTH];
        for (int j = 0; j < DEPTH; ++j) {
            nd[j] = entry(j);
            load(nd[j]);
        }
        Ent ne = entry(DEPTH);
        for (int i0 = 0; i0 < n; i0 += DEPTH)
            for (int j = 0; j < DEPTH; ++j) {
                if (i0 + j < n) {
                    const Ent& e = nd[j];
                    int q = -1;
                    if (e.w & CL_ROOT) {
                        CHECK(q_hbm[e.x], "clade root %d: q read before it is written", e.x);
                        q = e.x;
                    } else if (e.w & CL_STACK) {
                        CHECK(!stack.empty(), "pre clade stack underflow at node %d", e.x);
                        q = stack.back();
                        stack.pop_back();
                    } else {
                        q = acc;
                    }
                    CHECK(q == e.x, "pre clade node %d gets the q of node %d", e.x, q);
                    ++seen[e.x];
                    const bool in0 = e.y >= t.N, in1 = e.z >= t.N;
                    if (in1) {
                        if (in0) {
                            stack.push_back(e.y);
                            CHECK((int)stack.size() <= pl.depth, "pre clade stack depth %zu > %d", stack.size(),
                                  pl.depth);
                        }
                        acc = e.z;
                    } else if (in0) {
                        acc = e.y;
                    }
                }
                const Ent ne2 = entry(i0 + j + DEPTH + 1);
                nd[j] = ne;
                load(nd[j]);
                ne = ne2;
            }
        CHECK(stack.empty(), "pre clade stack not empty at the end of slot %d", ns);
    }
};

// The top-level launches next to the clade launches (post_top_kernel,
// pre_top_kernel): node i of the top goes to slot i % ns, each slot loads
// its TOP_J nodes (clamped indices) at the start, then takes them level by
// level.  Replays, for every slot, the loads (entries, message blocks, tip
// code rows, matrix entries), the level on which each node is taken, and the
// LDS region slots read and written, and checks that every top node is taken
// exactly once in each pass.  Only plans the launcher sends there.
void check_top_launches(const Tree& t, const TraversalPlan& pl, int ns) {
    if (!(pl.n_cl > 0 && pl.top_level == 0 && pl.n_top >= 1 && pl.top_nodes == pl.n_top &&
          pl.n_top <= TOP_J * ns))
        return;
    ++g_top_plans;
    const int N = t.N, root = 2 * N - 2, H = (int)pl.level_off.size() - 1;
    const Bounds bd{N, 2 * N - 2, N - 1};
    std::vector<char> in_top(2 * N - 1, 0);
    for (int i = 0; i < pl.n_top; ++i) in_top[pl.sched[i].x] = 1;
    for (int h = 0; h < H; ++h)
        CHECK(pl.level_off[h + 1] - pl.level_off[h] <= ns, "top level %d wider than %d slots", h, ns);
    auto slot_of = [&](int w, int which) {
        const int sl = (w >> (8 * which)) & 0xff;
        CHECK(sl >= 0 && sl <= pl.top_nodes, "top region slot %d of %d", sl, pl.top_nodes);
        return sl;
    };
    auto entry = [&](int i) -> const Ent& {
        const int c = std::min(std::max(i, 0), pl.n_top - 1);
        return pl.sched[c];
    };
    auto child_loads = [&](int c, bool msg_from_mem, const char* what) {
        CHECK(c >= 0 && c < 2 * N - 1 && c != root, "%s: child %d", what, c);
        bd.msg_block((c >= N && msg_from_mem) ? c : N, what);
        bd.code_row(c < N ? c : 0, what);
        bd.pmat(c, what);
    };
    // post order: levels upwards, messages of region nodes through LDS
    {
        std::vector<int> taken(pl.n_top, 0), lds_level(pl.top_nodes + 1, -1);
        for (int row = 0; row < ns; ++row) {
            for (int j = 0; j < TOP_J; ++j) {
                const Ent& e = entry(row + j * ns);
                for (int k = 1; k <= 2; ++k) {
                    const int c = k == 1 ? e.y : e.z;
                    const int sl = slot_of(e.w, k);
                    if (c >= N && sl == 0) CHECK(!in_top[c], "post top: top child %d of %d outside the region", c, e.x);
                    child_loads(c, sl == 0, "post top child");
                }
                bd.pmat(e.x == root ? 0 : e.x, "post top own matrix");
            }
        }
        // levels in order; within a level the slots run concurrently, so a
        // region slot written on level h is readable from level h + 1 on
        std::vector<int> next(ns, 0);
        for (int h = 0; h < H; ++h) {
            for (int row = 0; row < ns; ++row) {
                const int i = row + next[row] * ns;
                if (!(next[row] < TOP_J && i < pl.level_off[h + 1])) continue;
                CHECK(i >= pl.level_off[h], "post top: slot %d node %d taken on level %d", row, i, h);
                const Ent& e = pl.sched[i];
                ++taken[i];
                for (int k = 1; k <= 2; ++k)
                    if (const int sl = slot_of(e.w, k))
                        CHECK(lds_level[sl] >= 0 && lds_level[sl] < h, "post top: region slot %d read early", sl);
                if (e.x != root) {
                    const int sl = slot_of(e.w, 0);
                    CHECK(sl >= 1 && lds_level[sl] < 0, "post top: region slot %d of node %d", sl, e.x);
                    lds_level[sl] = h;
                }
                ++next[row];
            }
        }
        for (int i = 0; i < pl.n_top; ++i) CHECK(taken[i] == 1, "post top: node %d taken %d times", i, taken[i]);
    }
    // pre order: levels downwards, q of region nodes through LDS
    {
        std::vector<int> taken(pl.n_top, 0), lds_level(pl.top_nodes + 1, -1), cnt(ns, 0);
        for (int row = 0; row < ns; ++row) {
            const int n = row < pl.n_top ? std::min(TOP_J, (pl.n_top - 1 - row) / ns + 1) : 0;
            cnt[row] = n;
            for (int k = 0; k < TOP_J; ++k) {
                const Ent& e = entry(row + (n - 1 - k) * ns);
                child_loads(e.y, true, "pre top child");
                child_loads(e.z, true, "pre top child");
            }
        }
        for (int h = H - 1; h >= 0; --h) {
            for (int row = 0; row < ns; ++row) {
                const int j = cnt[row] - 1;
                if (!(j >= 0 && row + j * ns >= pl.level_off[h])) continue;
                const int i = row + j * ns;
                CHECK(i < pl.level_off[h + 1], "pre top: slot %d node %d taken on level %d", row, i, h);
                const Ent& e = pl.sched[i];
                ++taken[i];
                if (e.x != root) {
                    const int sl = slot_of(e.w, 0);
                    CHECK(sl >= 1 && lds_level[sl] > h, "pre top: q of node %d (slot %d) read early", e.x, sl);
                }
                for (int k = 1; k <= 2; ++k) {
                    const int c = k == 1 ? e.y : e.z;
                    if (c < N) continue;
                    if (const int sl = slot_of(e.w, k)) {
                        CHECK(lds_level[sl] < 0, "pre top: region slot %d written twice", sl);
                        lds_level[sl] = h;
                    } else {
                        bd.msg_block(c, "pre top q of a clade root");
                        CHECK(!in_top[c], "pre top: top child %d outside the region", c);
                    }
                }
                --cnt[row];
            }
        }
        for (int i = 0; i < pl.n_top; ++i) CHECK(taken[i] == 1, "pre top: node %d taken %d times", i, taken[i]);
    }
}

void check_plan(const Tree& t, const PlanParams& pp) {
    TraversalPlan pl;
    plan_traversal(t.N, t.parent.data(), t.ch.data(), t.lv, pp, pl);
    CHECK(pl.ns_post == pp.ns_post && pl.ns_pre == pp.ns_pre, "slot counts");
    CHECK(pl.one_list == (pp.ns_post == pp.ns_pre), "one list");
    CHECK(pl.cl_off.size() == (size_t)(pp.ns_post + pp.ns_pre + 2), "slot range table size");
    CHECK(pl.sched.size() == (size_t)pl.n_top + (size_t)pl.n_cl * (pl.one_list ? 1 : 2), "schedule size");
    CHECK(pl.level_off.front() == 0 && pl.level_off.back() == pl.n_top, "top level offsets");
    for (size_t h = 0; h + 1 < pl.level_off.size(); ++h) CHECK(pl.level_off[h] <= pl.level_off[h + 1], "levels");
    CHECK(pl.cl_off[pp.ns_post] == pl.n_cl && pl.cl_off.back() == pl.n_cl, "slot ranges cover the lists");
    if (!pp.clades) CHECK(pl.n_cl == 0, "clades without clade walks");
    if (pl.n_cl) {
        CHECK((size_t)pp.elem_bytes * std::max(pp.ns_post, pp.ns_pre) * pl.depth * pp.n_states * TP <=
                  (size_t)CLADE_STACK_MAX, "clade stacks exceed their LDS budget");
        CHECK(pl.cap > 0 && pl.cap <= CLADE_CAP, "clade cap %d", pl.cap);
    }
    // LDS of the traversal workgroups without the schedule (always within
    // the block) and with it (then it must fit SCHED_LDS_MAX)
    const size_t es = pp.elem_bytes, blk = (size_t)pp.n_states * TP * es;
    const size_t stack_b = (size_t)std::max(pp.ns_post, pp.ns_pre) * pl.depth * blk;
    const size_t top_b = (size_t)pl.top_nodes * blk;
    CHECK(std::max(stack_b, top_b) <= (size_t)LDS_BLOCK_MAX, "stack or top region LDS");
    Walk w(t, pl, pp);
    w.post();
    w.pre();
    if (pp.ns_post == pp.ns_pre) check_top_launches(t, pl, pp.ns_pre);
}

void check_updates(const Tree& t, std::mt19937_64& rng) {
    const int N = t.N, B = 2 * N - 2, root = 2 * N - 2;
    for (int trial = 0; trial < 40; ++trial) {
        const int n = 1 + (int)(rng() % (trial < 20 ? 2 : 8));
        std::vector<int> br(n);
        for (int& b : br) b = (int)(rng() % B);
        if (trial % 7 == 0) br.push_back(br[0]);  // a repeated branch
        UpdatePlan up;
        plan_update(N, t.parent.data(), t.ch.data(), t.lv, (int)br.size(), br.data(), up);
        // distinct changed branches, in range
        std::vector<char> inlist(B, 0);
        for (int b : up.list) {
            CHECK(b >= 0 && b < B, "update list branch %d", b);
            CHECK(!inlist[b], "branch %d listed twice", b);
            inlist[b] = 1;
        }
        for (int b : br) CHECK(inlist[b], "changed branch %d not in the list", b);
        // expected dirty set, by definition
        std::vector<char> dirty(2 * N - 1, 0);
        for (int b : br) {
            if (b >= N) dirty[b] = 1;
            for (int v = t.parent[b]; v >= 0; v = t.parent[v]) dirty[v] = 1;
        }
        CHECK(up.level_off.size() == t.lv.level_off.size(), "update level count");
        CHECK(up.level_off.back() == (int)up.sched.size(), "update level offsets");
        // replay the level walk: a clean node's message is valid from the
        // full pass; a dirty one is valid once its level is done
        std::vector<char> valid(2 * N - 1, 1), seen(2 * N - 1, 0);
        for (int k = N; k < 2 * N - 1; ++k)
            if (dirty[k]) valid[k] = 0;
        for (size_t h = 0; h + 1 < up.level_off.size(); ++h) {
            std::vector<char> nv = valid;
            for (int i = up.level_off[h]; i < up.level_off[h + 1]; ++i) {
                const Ent& e = up.sched.at(i);
                CHECK(e.x >= N && e.x <= root, "update node %d", e.x);
                CHECK(dirty[e.x], "clean node %d scheduled", e.x);
                CHECK(!seen[e.x], "node %d scheduled twice", e.x);
                CHECK(t.lv.height[e.x] == (int)h + 1, "node %d at the wrong level", e.x);
                seen[e.x] = 1;
                for (int c : {e.y, e.z}) {
                    CHECK(c >= 0 && c < 2 * N - 1 && t.parent[c] == e.x, "child %d of %d", c, e.x);
                    if (c >= N) CHECK(valid[c], "update reads the stale message of node %d", c);
                }
                nv[e.x] = 1;
            }
            valid = nv;
        }
        for (int k = N; k < 2 * N - 1; ++k) CHECK(seen[k] == dirty[k], "dirty node %d not scheduled", k);
        CHECK(seen[root], "the root is not re-evaluated");
    }
}

// The separate clade launches (small M): workgroup (group g, part q) of
// ns / 4 parts per group runs lists 4q..4q+3, one per wavefront; row r of a
// wavefront takes tile t' = min(4g + r, n_tiles - 1) in pattern-block-major
// order (t' = pb K + l; stored tile l n_pb + pb).  Every tile is walked for
// every list, and the per-workgroup exponent parts cl_esum[q][tile][pattern]
// are all written and inside their buffer.
void check_clade_launch(int ns, int K, int n_pb) {
    const int waves = 4, rows = 4, n_tiles = K * n_pb;
    const int nq = ns / waves, groups = (n_tiles + rows - 1) / rows;
    CHECK(nq * waves == ns, "lists %d not a multiple of the wavefronts per workgroup", ns);
    std::vector<int> walked((size_t)ns * n_tiles, 0);
    std::vector<char> part((size_t)nq * n_tiles, 0);
    for (int g = 0; g < groups; ++g)
        for (int q = 0; q < nq; ++q)
            for (int w = 0; w < waves; ++w)
                for (int r = 0; r < rows; ++r) {
                    const int tp = std::min(g * rows + r, n_tiles - 1);
                    const int pb = tp / K, l = tp % K, tile = l * n_pb + pb;
                    CHECK(pb >= 0 && pb < n_pb && tile >= 0 && tile < n_tiles, "clade launch tile %d", tile);
                    const int list = q * waves + w;
                    CHECK(list < ns, "clade launch list %d of %d", list, ns);
                    walked[(size_t)list * n_tiles + tile] = 1;
                    part[(size_t)q * n_tiles + tile] = 1;
                }
    for (size_t i = 0; i < walked.size(); ++i) CHECK(walked[i], "list %zu of tile %zu not walked", i / n_tiles, i % n_tiles);
    for (size_t i = 0; i < part.size(); ++i) CHECK(part[i], "exponent part %zu not written", i);
}

}  // namespace

int main(int argc, char** argv) {
    if (argc != 2) {
        std::fprintf(stderr, "usage: plan_check <tree file>\n");
        return 2;
    }
    Tree t;
    if (!read_tree(argv[1], t)) {
        std::fprintf(stderr, "cannot read %s\n", argv[1]);
        return 2;
    }
    // levels of the whole tree: every internal node once, children first
    {
        std::vector<int> seen(2 * t.N - 1, 0);
        for (int v : t.lv.level_nodes) {
            CHECK(v >= t.N && v < 2 * t.N - 1, "level node %d", v);
            ++seen[v];
            for (int c : {t.ch[v].x, t.ch[v].y}) CHECK(t.lv.height[c] < t.lv.height[v], "child above parent");
        }
        for (int k = t.N; k < 2 * t.N - 1; ++k) CHECK(seen[k] == 1, "level lists hold node %d %d times", k, seen[k]);
    }
    // kernel configurations: 4 states (row-distributed matrices, clade
    // walks) in FP64 and FP32 with several slot counts; 20 states and the
    // 64-padded split path walk levels only
    struct Cfg { int m, es; bool clades, top; int ns_post, ns_pre; };
    const Cfg cfgs[] = {
        {4, 8, true, true, 16, 16}, {4, 4, true, true, 32, 32}, {4, 8, true, true, 8, 8},
        {4, 8, true, true, 32, 16}, {4, 4, true, true, 16, 32}, {4, 8, false, true, 16, 16},
        {4, 8, true, false, 16, 16}, {20, 8, false, true, 16, 16}, {20, 4, false, true, 16, 16},
        {64, 4, false, false, 16, 16},
    };
    for (const Cfg& c : cfgs) {
        PlanParams p;
        p.n_states = c.m;
        p.elem_bytes = c.es;
        p.clades = c.clades;
        p.top_region = c.top;
        p.ns_post = c.ns_post;
        p.ns_pre = c.ns_pre;
        check_plan(t, p);
    }
    for (int ns : {16, 32})
        for (int K : {1, 2, 3, 4, 5})
            for (int n_pb : {1, 2, 3, 125, 313}) check_clade_launch(ns, K, n_pb);
    std::mt19937_64 rng(12146 + t.N);
    check_updates(t, rng);
    std::printf("plan_check N=%d: %d checks passed (%d plans through the top-level launches)\n", t.N, g_checks,
                g_top_plans);
    return 0;
}
