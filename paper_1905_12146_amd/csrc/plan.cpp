// Host-side planning of the traversal kernels (declarations and the layout
// of what is produced in plan.h).
#include "plan.h"

#include <algorithm>
#include <utility>

namespace pg {

namespace {

// within a level: nodes with two internal children, then one, then none,
// each group by label.  Consecutive node slots share a wavefront, so the
// grouping keeps the tip and internal child paths of the kernels from both
// running in one wavefront for most of the level.
void sort_by_tip_children(int N, const Kids* ch, std::vector<int>& nodes) {
    auto n_tip_children = [&](int v) { return (ch[v].x < N) + (ch[v].y < N); };
    std::sort(nodes.begin(), nodes.end(), [&](int u, int v) {
        const int cu = n_tip_children(u), cv = n_tip_children(v);
        return cu != cv ? cu < cv : u < v;
    });
}

// Top levels and clade lists of one clade cap (0: every internal node in the
// levels).
struct Schedule {
    std::vector<int> level_off;    // [H + 1] top levels
    std::vector<int> level_nodes;  // top nodes by level
    std::vector<Ent> cl_post, cl_pre;
    std::vector<int> cl_post_off, cl_pre_off;
    int depth = 0;                 // stack blocks per slot
};

// LPT assignment of clades to ns slots (largest clade to the least loaded
// slot); entries slot-major.
void assign_clades(const std::vector<std::vector<Ent>>& clades, int ns, std::vector<Ent>& out,
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

void build_schedule(int N, const int* parent, const Kids* ch, const TreeLevels& lv, int cap, int ns_post,
                    int ns_pre, Schedule& sc) {
    const int n_nodes = 2 * N - 1, root = n_nodes - 1;
    // internal nodes in increasing height: children before parents
    const std::vector<int>& up = lv.level_nodes;
    std::vector<int> sz(n_nodes, 0);  // internal nodes in the subtree
    for (int v : up) sz[v] = 1 + sz[ch[v].x] + sz[ch[v].y];
    // clade of each internal node (its clade root), -1 for the top
    std::vector<int> clade(n_nodes, -1);
    std::vector<int> roots;
    for (auto it = up.rbegin(); it != up.rend(); ++it) {
        const int v = *it;
        if (v == root) continue;
        const int p = parent[v];
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
    sort_by_tip_children(N, ch, top);
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
    std::vector<std::vector<Ent>> lists;
    sc.depth = 0;
    for (int r : roots) {
        std::vector<Ent> e;
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
                    const auto [pf, pg2] = ordered(parent[v]);
                    if (v == pf && pg2 >= N) flags = CL_STACK;
                }
                e.push_back(Ent{v, f, g, flags});
                continue;
            }
            st.push_back({v, true});
            if (g >= N) st.push_back({g, false});
            if (f >= N) st.push_back({f, false});
        }
        // stack depth of the walk (pops before pushes within an entry)
        int sp = 0;
        for (const Ent& x : e) {
            if (x.y >= N && x.z >= N) --sp;
            if (x.w & CL_STACK) ++sp;
            sc.depth = std::max(sc.depth, sp);
        }
        lists.push_back(std::move(e));
    }
    assign_clades(lists, ns_post, sc.cl_post, sc.cl_post_off);
    assign_clades(lists, ns_pre, sc.cl_pre, sc.cl_pre_off);
}

}  // namespace

void build_levels(int N, const Kids* ch, TreeLevels& out) {
    const int n_nodes = 2 * N - 1;
    std::vector<int> height(n_nodes, 0);
    // internal nodes in post order via an explicit stack
    std::vector<int> order;
    order.reserve(N - 1);
    std::vector<int> stack{n_nodes - 1};
    std::vector<char> expanded(n_nodes, 0);
    while (!stack.empty()) {
        int v = stack.back();
        if (v < N) { stack.pop_back(); continue; }
        if (!expanded[v]) {
            expanded[v] = 1;
            stack.push_back(ch[v].x);
            stack.push_back(ch[v].y);
        } else {
            stack.pop_back();
            height[v] = 1 + std::max(height[ch[v].x], height[ch[v].y]);
            order.push_back(v);
        }
    }
    int H = 0;
    for (int v : order) H = std::max(H, height[v]);
    std::vector<int> count(H + 1, 0);
    for (int v : order) count[height[v]]++;
    // level h (1..H) stored at index h-1
    out.level_off.assign(H + 1, 0);
    for (int h = 1; h <= H; ++h) out.level_off[h] = out.level_off[h - 1] + count[h];
    out.level_nodes.assign(N - 1, 0);
    std::vector<int> fill(out.level_off.begin(), out.level_off.end() - 1);
    sort_by_tip_children(N, ch, order);
    for (int v : order) out.level_nodes[fill[height[v] - 1]++] = v;
    out.height.swap(height);
}

void plan_traversal(int N, const int* parent, const Kids* ch, const TreeLevels& lv, const PlanParams& p,
                    TraversalPlan& out) {
    const int n_nodes = 2 * N - 1, M = p.n_states;
    const size_t es = (size_t)p.elem_bytes;
    Schedule sc;
    int cap_used = 0;
    if (p.clades) {
        long best = -1;
        for (int cap : {64, 48, 32, 24, 16}) {
            if (cap > CLADE_CAP) continue;
            Schedule t;
            build_schedule(N, parent, ch, lv, cap, p.ns_post, p.ns_pre, t);
            if (es * std::max(p.ns_post, p.ns_pre) * t.depth * M * TP > (size_t)CLADE_STACK_MAX) continue;
            long busiest = 0, top_iters = 0;
            for (int b = 0; b < p.ns_pre; ++b)
                busiest = std::max<long>(busiest, t.cl_pre_off[b + 1] - t.cl_pre_off[b]);
            for (size_t h = 0; h + 1 < t.level_off.size(); ++h)
                top_iters += (t.level_off[h + 1] - t.level_off[h] + p.ns_pre - 1) / p.ns_pre;
            const long cost = busiest + 2 * top_iters;
            if (best < 0 || cost < best) {
                best = cost;
                sc = std::move(t);
                cap_used = cap;
            }
        }
        if (best < 0) build_schedule(N, parent, ch, lv, 0, p.ns_post, p.ns_pre, sc);
    } else {
        build_schedule(N, parent, ch, lv, 0, p.ns_post, p.ns_pre, sc);
    }
    const int n_top = (int)sc.level_nodes.size(), n_cl = (int)sc.cl_post.size();
    const bool one_list = p.ns_post == p.ns_pre;
    // pre-order top region: levels from the root down while every level has
    // at most one node per pre-order node slot (and at most
    // TOP_LEVEL_MAX_NODES) and their q vectors fit TOP_LDS_MAX
    const int H = (int)sc.level_off.size() - 1;
    const int top_cap = std::min<int>(255, TOP_LDS_MAX / (int)(es * M * TP));
    const int top_width = std::min(TOP_LEVEL_MAX_NODES, p.ns_pre);
    int top_level = H, top_nodes = 0;
    for (int h = H - 1; h >= 0 && p.top_region; --h) {
        const int n_h = sc.level_off[h + 1] - sc.level_off[h];
        if (n_h > top_width || top_nodes + n_h > top_cap) break;
        top_nodes += n_h;
        top_level = h;
    }
    std::vector<int> region(n_nodes, 0);
    {
        int next = 1;
        for (int i = sc.level_off[top_level]; i < sc.level_off[H]; ++i) region[sc.level_nodes[i]] = next++;
    }
    out.sched.assign((size_t)n_top + (size_t)n_cl * (one_list ? 1 : 2), Ent{0, 0, 0, 0});
    for (int i = 0; i < n_top; ++i) {
        const int k = sc.level_nodes[i];
        // a node with one tip child lists its internal child first, so the
        // first child of every such node takes the same path
        int c0 = ch[k].x, c1 = ch[k].y;
        if (c0 < N && c1 >= N) std::swap(c0, c1);
        out.sched[i] = Ent{k, c0, c1, region[k] | (region[c0] << 8) | (region[c1] << 16)};
    }
    std::copy(sc.cl_post.begin(), sc.cl_post.end(), out.sched.begin() + n_top);
    if (!one_list) std::copy(sc.cl_pre.begin(), sc.cl_pre.end(), out.sched.begin() + n_top + n_cl);
    out.cl_off = sc.cl_post_off;
    out.cl_off.insert(out.cl_off.end(), sc.cl_pre_off.begin(), sc.cl_pre_off.end());
    out.level_off = std::move(sc.level_off);
    out.n_top = n_top;
    out.n_cl = n_cl;
    out.depth = sc.depth;
    out.cap = n_cl ? cap_used : 0;
    out.ns_post = p.ns_post;
    out.ns_pre = p.ns_pre;
    out.one_list = one_list;
    out.top_level = top_level;
    out.top_nodes = top_nodes;
}

void plan_update(int N, const int* parent, const Kids* ch, const TreeLevels& lv, int n, const int* branches,
                 UpdatePlan& out) {
    std::vector<char> dirty(2 * N - 1, 0);
    out.list.clear();
    out.sched.clear();
    for (int i = 0; i < n; ++i) {
        const int b = branches[i];
        if (std::find(out.list.begin(), out.list.end(), b) == out.list.end()) out.list.push_back(b);
        for (int v = (b >= N) ? b : parent[b]; v >= 0 && !dirty[v]; v = parent[v]) dirty[v] = 1;
    }
    const int H = (int)lv.level_off.size() - 1;
    out.level_off.assign(H + 1, 0);
    for (int h = 0; h < H; ++h) {
        for (int i = lv.level_off[h]; i < lv.level_off[h + 1]; ++i) {
            const int k = lv.level_nodes[i];
            if (dirty[k]) out.sched.push_back(Ent{k, ch[k].x, ch[k].y, 0});
        }
        out.level_off[h + 1] = (int)out.sched.size();
    }
}

}  // namespace pg
