// Monte-Carlo tree search over the SpMV design space (Sec. III-C of the
// paper): selection by exploration + exploitation value, expansion of one
// zero-rollout child, a random rollout whose nodes stay in the tree, and
// min/max backpropagation.  The children of a node are the next tokens of
// its prefix (Prefix::next over the coarse DAG, FinePrefix::next over the
// per-peer DAG: ready vertices bound to canonical streams, and the Table III
// tokens), so the tree covers exactly the plan space of its DAG and every
// rollout reaches a plan not benchmarked before.
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

template <class Pre>
struct Search {
    // bench(complete prefix, seconds out) -> status
    using Bench = std::function<int(const Pre &, double &)>;
    Pre pre;
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

    int iterate(Draws &rng, const Bench &bench, double &t)
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
        if (int rc = bench(pre, t)) return rc;
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

// Runs the search from an initialised empty prefix; bench records each
// rollout's plan where the caller wants it, run() its time.
template <class Pre>
int run(const Pre &root_prefix, const spmv_mcts_opts_t &o,
        const typename Search<Pre>::Bench &bench, double *time_out, int64_t cap, int64_t *n_out,
        spmv_mcts_node_t *nodes, int64_t node_cap, int64_t *n_nodes)
{
    if (cap < 0 || node_cap < 0) return set_error(SPMV_EINVAL, "negative output capacity");
    Search<Pre> S;
    S.c = o.c;
    S.pre = root_prefix;
    S.pre.clear();
    S.tree.emplace_back();
    S.list(0);
    Draws rng;
    rng.rand = o.rand;
    rng.n_rand = o.n_rand;
    rng.mt.seed(o.seed);
    int64_t done = 0;
    while ((o.iterations == 0 || done < o.iterations) && !S.tree[0].full) {
        double t;
        if (int rc = S.iterate(rng, bench, t)) return rc;
        if (done < cap && time_out) time_out[done] = t;
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

// Per-position streams of a complete prefix (-1 for tokens without one).
void seq_streams(const Prefix &p, std::vector<int32_t> &out)
{
    out.clear();
    for (int32_t t : p.order)
        out.push_back(is_vertex(t) && vertex_type(t) == VType::GPU ? p.stream[t] : -1);
}

void seq_streams(const FinePrefix &p, std::vector<int32_t> &out) { out = p.ostream; }

// Median of a measurement set.
double median(std::vector<double> s)
{
    std::nth_element(s.begin(), s.begin() + long(s.size() / 2), s.end());
    return s[s.size() / 2];
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
    Prefix root;
    root.init(nranks > 1, o.n_streams);
    int64_t k = 0;
    Search<Prefix>::Bench bench = [&](const Prefix &p, double &t) {
        const int64_t i = plan_index(p.multi, p.n_streams, p.order, p.stream);
        if (i < 0) return set_error(SPMV_ESTATE, "MCTS reached a plan outside the space");
        if (index_out && k < cap) index_out[k] = i;
        ++k;
        t = cost[i];
        return SPMV_OK;
    };
    return run(root, o, bench, time_out, cap, n_out, nodes, node_cap, n_nodes);
}

namespace {

// Checks shared by the device searches; nranks out.
int check_plans(spmv_plan_t *const *plans, int32_t n_plans, int32_t &nranks)
{
    if (!plans || n_plans < 1) return set_error(SPMV_EINVAL, "need at least one plan");
    for (int32_t k = 0; k < n_plans; ++k)
        if (!plans[k]) return set_error(SPMV_EINVAL, "null plan");
    nranks = plans[0]->share.nranks;
    for (int32_t k = 1; k < n_plans; ++k)
        if ((plans[k]->share.nranks > 1) != (nranks > 1))
            return set_error(SPMV_EINVAL, "plans of one search must share the DAG");
    return SPMV_OK;
}

}  // namespace

extern "C" int spmv_mcts_run(spmv_plan_t *const *plans, int32_t n_plans, const double *const *x,
                             double *const *y, void *stream, const spmv_mcts_opts_t *opts,
                             int64_t *index_out, double *time_out, int64_t cap, int64_t *n_out,
                             spmv_mcts_node_t *nodes, int64_t node_cap, int64_t *n_nodes)
{
    int32_t nranks = 0;
    if (int rc = check_plans(plans, n_plans, nranks)) return rc;
    if (!x || !y || !n_out) return set_error(SPMV_EINVAL, "bad argument to spmv_mcts_run");
    spmv_mcts_opts_t o;
    if (int rc = options(opts, o)) return rc;
    const auto &space = plan_space(nranks > 1, o.n_streams);
    std::vector<double> times(size_t(o.n_measure));
    Prefix root;
    root.init(nranks > 1, o.n_streams);
    int64_t k = 0;
    Search<Prefix>::Bench bench = [&](const Prefix &p, double &t) {
        const int64_t i = plan_index(p.multi, p.n_streams, p.order, p.stream);
        if (i < 0) return set_error(SPMV_ESTATE, "MCTS reached a plan outside the space");
        const PlanEntry &e = space[size_t(i)];
        for (int32_t j = 0; j < n_plans; ++j)
            if (int rc = spmv_plan_reorder(plans[j], e.order.data(), int32_t(e.order.size()),
                                           e.stream, o.n_streams))
                return rc;
        if (int rc = spmv_plan_time(plans, n_plans, x, y, stream, o.t_measure, o.n_measure,
                                    times.data()))
            return rc;
        if (index_out && k < cap) index_out[k] = i;
        ++k;
        t = median(times);
        return SPMV_OK;
    };
    return run(root, o, bench, time_out, cap, n_out, nodes, node_cap, n_nodes);
}

extern "C" int spmv_mcts_run_seq(spmv_plan_t *const *plans, int32_t n_plans,
                                 const double *const *x, double *const *y, void *stream,
                                 int32_t fine, spmv_cost_fn cost, void *user,
                                 const spmv_mcts_opts_t *opts, int32_t *ops_out,
                                 int32_t *streams_out, int32_t max_ops, double *time_out,
                                 int64_t cap, int64_t *n_out, spmv_mcts_node_t *nodes,
                                 int64_t node_cap, int64_t *n_nodes)
{
    int32_t nranks = 0;
    if (int rc = check_plans(plans, n_plans, nranks)) return rc;
    if (!n_out || (!cost && (!x || !y)) || max_ops < 0 || (max_ops > 0 && (!ops_out || !streams_out)))
        return set_error(SPMV_EINVAL, "bad argument to spmv_mcts_run_seq");
    if (fine && nranks < 2) return set_error(SPMV_EINVAL, "a single rank has no fine-grained DAG");
    if (fine)
        for (int32_t k = 1; k < n_plans; ++k)
            if (plans[k]->fdag.tokens != plans[0]->fdag.tokens)
                return set_error(SPMV_EINVAL, "plans of one search must share the DAG");
    spmv_mcts_opts_t o;
    if (int rc = options(opts, o)) return rc;
    std::vector<double> times(size_t(o.n_measure));
    std::vector<int32_t> ss;
    int64_t k = 0;
    // record the rollout, then cost it (callback) or time it on the device
    auto record = [&](const std::vector<int32_t> &order, double &t, auto &&apply) -> int {
        const int32_t n = int32_t(order.size());
        if (k < cap && max_ops > 0) {
            if (n > max_ops) return set_error(SPMV_EINVAL, "max_ops smaller than an order");
            std::copy(order.begin(), order.end(), ops_out + k * max_ops);
            std::copy(ss.begin(), ss.end(), streams_out + k * max_ops);
        }
        ++k;
        if (cost) {
            t = cost(order.data(), ss.data(), n, user);
            return SPMV_OK;
        }
        for (int32_t j = 0; j < n_plans; ++j)
            if (int rc = apply(plans[j])) return rc;
        if (int rc = spmv_plan_time(plans, n_plans, x, y, stream, o.t_measure, o.n_measure,
                                    times.data()))
            return rc;
        t = median(times);
        return SPMV_OK;
    };
    if (!fine) {
        Prefix root;
        root.init(nranks > 1, o.n_streams);
        Search<Prefix>::Bench bench = [&](const Prefix &p, double &t) {
            seq_streams(p, ss);
            return record(p.order, t, [&](spmv_plan_t *q) {
                return spmv_plan_reorder(q, p.order.data(), int32_t(p.order.size()), p.stream,
                                         o.n_streams);
            });
        };
        return run(root, o, bench, time_out, cap, n_out, nodes, node_cap, n_nodes);
    }
    FinePrefix root;
    root.init(&plans[0]->fdag, o.n_streams);
    Search<FinePrefix>::Bench bench = [&](const FinePrefix &p, double &t) {
        seq_streams(p, ss);
        return record(p.order, t, [&](spmv_plan_t *q) {
            return spmv_plan_set_fine(q, p.order.data(), p.ostream.data(), int32_t(p.order.size()),
                                      o.n_streams);
        });
    };
    return run(root, o, bench, time_out, cap, n_out, nodes, node_cap, n_nodes);
}
