// Monte-Carlo tree search over the SpMV design space (Sec. III-C of the
// paper): selection by exploration + exploitation value, expansion of one
// zero-rollout child, a random rollout whose nodes stay in the tree, and
// min/max backpropagation.  The children of a node are the next tokens of
// its prefix (Prefix::next: DAG-ready vertices bound to canonical streams,
// and the Table III tokens), so the tree covers exactly the enumerated plan
// space and every rollout reaches a plan not benchmarked before.
#include <algorithm>
#include <cmath>
#include <functional>
#include <limits>
#include <random>

#include "spmv_internal.h"

namespace spmv {
namespace {

constexpr double kInf = std::numeric_limits<double>::infinity();

struct Node {
    Prefix::Step step{-1, -1};
    int32_t parent = -1;
    std::vector<Prefix::Step> untried;   // children not created yet, in next() order
    std::vector<int32_t> children;       // created children, in creation order
    bool complete = false, full = false;
    int64_t n = 0;
    double tmin = kInf, tmax = -kInf;
};

struct Draws {
    const uint64_t *rand = nullptr;
    int64_t n_rand = 0, k = 0;
    std::mt19937_64 mt;

    int pick(size_t m, size_t &out)
    {
        uint64_t r;
        if (rand) {
            if (k >= n_rand) return set_error(SPMV_EINVAL, "MCTS ran out of random draws");
            r = rand[k];
        } else {
            r = mt();
        }
        ++k;
        out = size_t(r % uint64_t(m));
        return SPMV_OK;
    }
};

// bench(plan index, seconds out) -> status
using Bench = std::function<int(int64_t, double &)>;

struct Search {
    Prefix pre;
    std::vector<Node> tree;
    double c = 0;

    Node &at(int32_t i) { return tree[size_t(i)]; }

    // children of a fresh node, listed from the current prefix
    void list(int32_t i)
    {
        pre.next(at(i).untried);
        at(i).complete = pre.complete();
    }

    int32_t create(int32_t parent, size_t k)
    {
        Node child;
        child.step = at(parent).untried[k];
        child.parent = parent;
        at(parent).untried.erase(at(parent).untried.begin() + long(k));
        tree.push_back(child);
        const int32_t ci = int32_t(tree.size()) - 1;
        at(parent).children.push_back(ci);
        pre.push(at(ci).step);
        list(ci);
        return ci;
    }

    // exploitation value of child ch under node nd
    static double value(const Node &nd, const Node &ch)
    {
        if (ch.n >= 2 && nd.n >= 2 && nd.tmax > nd.tmin) return (ch.tmax - ch.tmin) / (nd.tmax - nd.tmin);
        return 1.0;
    }

    int iterate(Draws &rng, const Bench &bench, int64_t &index, double &t)
    {
        pre.clear();
        std::vector<int32_t> path{0};
        int32_t cur = 0;
        // selection: descend while every child of the node has rollouts
        while (at(cur).untried.empty() && !at(cur).complete) {
            const Node &nd = at(cur);
            int32_t best = -1;
            double best_score = -kInf;
            for (int32_t ci : nd.children) {
                const Node &ch = at(ci);
                const double explore =
                    ch.full ? -kInf : c * std::sqrt(std::log(double(nd.n)) / double(ch.n));
                const double score = explore + value(nd, ch);
                if (best < 0 || score > best_score) {
                    best = ci;
                    best_score = score;
                }
            }
            if (best < 0 || at(best).full)
                return set_error(SPMV_ESTATE, "MCTS selection reached a fully explored subtree");
            cur = best;
            pre.push(at(cur).step);
            path.push_back(cur);
        }
        // expansion, then the rollout: random children down to a complete plan
        while (!at(cur).complete) {
            size_t k;
            if (int rc = rng.pick(at(cur).untried.size(), k)) return rc;
            cur = create(cur, k);
            path.push_back(cur);
        }
        index = plan_index(pre.multi, pre.n_streams, pre.order, pre.stream);
        if (index < 0) return set_error(SPMV_ESTATE, "MCTS reached a plan outside the space");
        if (int rc = bench(index, t)) return rc;
        // backpropagation, and fully-explored marks from the leaf up
        for (int32_t i : path) {
            Node &nd = at(i);
            ++nd.n;
            nd.tmin = std::min(nd.tmin, t);
            nd.tmax = std::max(nd.tmax, t);
        }
        for (auto it = path.rbegin(); it != path.rend(); ++it) {
            Node &nd = at(*it);
            bool full = nd.complete || nd.untried.empty();
            for (int32_t ci : nd.children) full = full && at(ci).full;
            nd.full = full;
        }
        return SPMV_OK;
    }
};

int options(const spmv_mcts_opts_t *o, spmv_mcts_opts_t &d)
{
    d = spmv_mcts_opts_t{};
    if (o) d = *o;
    if (d.iterations < 0 || d.n_measure < 0 || d.n_streams < 0 ||
        d.n_streams > SPMV_MAX_STREAMS || !(d.c >= 0) || !(d.t_measure >= 0) || d.n_rand < 0 ||
        (d.n_rand > 0 && !d.rand))
        return set_error(SPMV_EINVAL, "MCTS option out of range");
    if (d.c == 0) d.c = std::sqrt(2.0);
    if (d.t_measure == 0) d.t_measure = 0.01;
    if (d.n_measure == 0) d.n_measure = 1;
    if (d.n_streams == 0) d.n_streams = 2;
    return SPMV_OK;
}

int run(int32_t nranks, const spmv_mcts_opts_t &o, const Bench &bench, int64_t *index_out,
        double *time_out, int64_t cap, int64_t *n_out, spmv_mcts_node_t *nodes,
        int64_t node_cap, int64_t *n_nodes)
{
    if (cap < 0 || node_cap < 0) return set_error(SPMV_EINVAL, "negative output capacity");
    Search S;
    S.c = o.c;
    S.pre.init(nranks > 1, o.n_streams);
    S.tree.emplace_back();
    S.list(0);
    Draws rng;
    rng.rand = o.rand;
    rng.n_rand = o.n_rand;
    rng.mt.seed(o.seed);
    int64_t done = 0;
    while ((o.iterations == 0 || done < o.iterations) && !S.tree[0].full) {
        int64_t idx;
        double t;
        if (int rc = S.iterate(rng, bench, idx, t)) return rc;
        if (done < cap) {
            if (index_out) index_out[done] = idx;
            if (time_out) time_out[done] = t;
        }
        ++done;
    }
    *n_out = done;
    if (n_nodes) *n_nodes = int64_t(S.tree.size());
    if (nodes)
        for (int64_t i = 0; i < std::min<int64_t>(node_cap, int64_t(S.tree.size())); ++i) {
            const Node &nd = S.tree[size_t(i)];
            nodes[i] = spmv_mcts_node_t{nd.parent, nd.step.token, nd.step.stream,
                                        nd.full ? 1 : 0,  nd.n,     nd.tmin, nd.tmax};
        }
    return SPMV_OK;
}

}  // namespace
}  // namespace spmv

using namespace spmv;

extern "C" int spmv_mcts_run_table(int32_t nranks, const double *cost, int64_t n_cost,
                                   const spmv_mcts_opts_t *opts, int64_t *index_out,
                                   double *time_out, int64_t cap, int64_t *n_out,
                                   spmv_mcts_node_t *nodes, int64_t node_cap, int64_t *n_nodes)
{
    if (!cost || !n_out || nranks < 1)
        return set_error(SPMV_EINVAL, "bad argument to spmv_mcts_run_table");
    spmv_mcts_opts_t o;
    if (int rc = options(opts, o)) return rc;
    if (n_cost != int64_t(plan_space(nranks > 1, o.n_streams).size()))
        return set_error(SPMV_EINVAL, "cost table must hold one time per plan of the space");
    Bench bench = [&](int64_t i, double &t) {
        t = cost[i];
        return SPMV_OK;
    };
    return run(nranks, o, bench, index_out, time_out, cap, n_out, nodes, node_cap, n_nodes);
}

extern "C" int spmv_mcts_run(spmv_plan_t *const *plans, int32_t n_plans, const double *const *x,
                             double *const *y, void *stream, const spmv_mcts_opts_t *opts,
                             int64_t *index_out, double *time_out, int64_t cap, int64_t *n_out,
                             spmv_mcts_node_t *nodes, int64_t node_cap, int64_t *n_nodes)
{
    if (!plans || n_plans < 1 || !x || !y || !n_out)
        return set_error(SPMV_EINVAL, "bad argument to spmv_mcts_run");
    for (int32_t k = 0; k < n_plans; ++k)
        if (!plans[k]) return set_error(SPMV_EINVAL, "null plan");
    spmv_mcts_opts_t o;
    if (int rc = options(opts, o)) return rc;
    const int32_t nranks = plans[0]->share.nranks;
    for (int32_t k = 1; k < n_plans; ++k)
        if ((plans[k]->share.nranks > 1) != (nranks > 1))
            return set_error(SPMV_EINVAL, "plans of one search must share the DAG");
    const auto &space = plan_space(nranks > 1, o.n_streams);
    std::vector<double> times(size_t(o.n_measure));
    Bench bench = [&](int64_t i, double &t) {
        const PlanEntry &e = space[size_t(i)];
        for (int32_t k = 0; k < n_plans; ++k)
            if (int rc = spmv_plan_reorder(plans[k], e.order.data(), int32_t(e.order.size()),
                                           e.stream, o.n_streams))
                return rc;
        if (int rc = spmv_plan_time(plans, n_plans, x, y, stream, o.t_measure, o.n_measure,
                                    times.data()))
            return rc;
        std::vector<double> s = times;
        std::nth_element(s.begin(), s.begin() + long(s.size() / 2), s.end());
        t = s[s.size() / 2];
        return SPMV_OK;
    };
    return run(nranks, o, bench, index_out, time_out, cap, n_out, nodes, node_cap, n_nodes);
}
