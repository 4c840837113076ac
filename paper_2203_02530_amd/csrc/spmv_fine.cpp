// The fine-grained SpMV program (Sec. III-A): instead of one Pack, PostSend,
// WaitSend, PostRecv and WaitRecv for all peers, one of each per peer, so
// that packing for one destination no longer delays sending to another.
//
// Vertices for rank r: start, y_L, y_R, end; per destination q (ranks that
// need some of r's x entries) Pack_q, PostSend_q, WaitSend_q; per source q
// (owners of r's halo entries) PostRecv_q, WaitRecv_q.  Edges: start ->
// {Pack_q, y_L, PostRecv_q}; Pack_q -> PostSend_q -> WaitSend_q -> end;
// PostRecv_q -> WaitRecv_q -> y_R for every source (x_R is assembled by the
// Unpack that runs on y_R's stream right before it); y_L -> end; y_R -> end.
// The only Table III synchronisations are the GPU -> CPU edges Pack_q ->
// PostSend_q: CER-after-Pack_q, CES-b4-PostSend_q (the fine DAG has no
// GPU -> GPU edge across streams, so none depend on the stream map).
//
// Tokens: a vertex of peer q is SPMV_PEER(op, q) = op | (q + 1) << 8; start,
// y_L, y_R, end keep their codes; synchronisation tokens wrap a vertex token
// as in the coarse program.
#include <algorithm>
#include <map>

#include "spmv_internal.h"

namespace spmv {

namespace {

int32_t peer_tok(int32_t op, int32_t q) { return op | ((q + 1) << 8); }

}  // namespace

int32_t tok_op(int32_t t) { return t & 0x0f; }
int32_t tok_kind(int32_t t) { return t & 0x30; }
int32_t tok_peer(int32_t t) { return ((t >> 8) & 0xff) - 1; }

void FineDag::build(const Share &S)
{
    const int32_t P = S.nranks;
    dests.clear();
    srcs.clear();
    for (int32_t q = 0; q < P; ++q) {
        if (q == S.rank) continue;
        if (S.send_off[size_t(q) + 1] > S.send_off[size_t(q)]) dests.push_back(q);
        if (S.recv_off[size_t(q) + 1] > S.recv_off[size_t(q)]) srcs.push_back(q);
    }
    tokens.clear();
    tokens.push_back(SPMV_OP_START);
    tokens.push_back(SPMV_OP_YL);
    tokens.push_back(SPMV_OP_YR);
    tokens.push_back(SPMV_OP_END);
    for (int32_t q : dests) {
        const int32_t pack = peer_tok(SPMV_OP_PACK, q);
        tokens.push_back(pack);
        tokens.push_back(SPMV_CER_AFTER(pack));
        tokens.push_back(SPMV_CES_B4(peer_tok(SPMV_OP_POST_SEND, q)));
        tokens.push_back(peer_tok(SPMV_OP_POST_SEND, q));
        tokens.push_back(peer_tok(SPMV_OP_WAIT_SEND, q));
    }
    for (int32_t q : srcs) {
        tokens.push_back(peer_tok(SPMV_OP_POST_RECV, q));
        tokens.push_back(peer_tok(SPMV_OP_WAIT_RECV, q));
    }
    std::sort(tokens.begin(), tokens.end());
    index.clear();
    for (size_t i = 0; i < tokens.size(); ++i) index[tokens[i]] = int32_t(i);
    // what must precede each token: DAG predecessors and Table III pairs
    need.assign(tokens.size(), {});
    gpu.assign(tokens.size(), false);
    auto at = [&](int32_t t) { return index.at(t); };
    for (size_t i = 0; i < tokens.size(); ++i) {
        const int32_t t = tokens[i];
        std::vector<int32_t> &n = need[i];
        if (t == SPMV_OP_START) continue;
        if (t == SPMV_OP_END) {
            for (size_t j = 0; j < tokens.size(); ++j)
                if (j != i) n.push_back(int32_t(j));
            continue;
        }
        if (tok_kind(t) == SPMV_SYNC_CER) {
            n.push_back(at(t & ~0x30));   // after its GPU vertex
        } else if (tok_kind(t) == SPMV_SYNC_CES) {
            n.push_back(at(SPMV_CER_AFTER(peer_tok(SPMV_OP_PACK, tok_peer(t)))));
        } else {
            n.push_back(at(SPMV_OP_START));
            const int32_t op = tok_op(t), q = tok_peer(t);
            if (op == SPMV_OP_PACK || op == SPMV_OP_YL || op == SPMV_OP_YR) gpu[i] = true;
            if (op == SPMV_OP_POST_SEND) {
                n.push_back(at(peer_tok(SPMV_OP_PACK, q)));
                n.push_back(at(SPMV_CES_B4(t)));
            } else if (op == SPMV_OP_WAIT_SEND) {
                n.push_back(at(peer_tok(SPMV_OP_POST_SEND, q)));
            } else if (op == SPMV_OP_WAIT_RECV) {
                n.push_back(at(peer_tok(SPMV_OP_POST_RECV, q)));
            } else if (op == SPMV_OP_YR) {
                for (int32_t s : srcs) n.push_back(at(peer_tok(SPMV_OP_WAIT_RECV, s)));
            }
        }
    }
}

int FineDag::find(int32_t t) const
{
    auto it = index.find(t);
    return it == index.end() ? -1 : it->second;
}

// ---------------------------------------------------------------- prefixes

void FinePrefix::init(const FineDag *d, int32_t n_streams_)
{
    dag = d;
    n_streams = n_streams_;
    clear();
}

void FinePrefix::clear()
{
    order.clear();
    ostream.clear();
    placed.assign(dag->tokens.size(), false);
    used = 0;
}

bool FinePrefix::ready(int32_t i) const
{
    if (placed[size_t(i)]) return false;
    for (int32_t j : dag->need[size_t(i)])
        if (!placed[size_t(j)]) return false;
    return true;
}

void FinePrefix::next(std::vector<Prefix::Step> &out) const
{
    out.clear();
    for (size_t i = 0; i < dag->tokens.size(); ++i) {
        if (!ready(int32_t(i))) continue;
        if (dag->gpu[i]) {
            const int32_t lim = std::min(used + 1, n_streams);
            for (int32_t s = 0; s < lim; ++s) out.push_back({dag->tokens[i], s});
        } else {
            out.push_back({dag->tokens[i], -1});
        }
    }
}

void FinePrefix::push(Prefix::Step st)
{
    placed[size_t(dag->find(st.token))] = true;
    order.push_back(st.token);
    ostream.push_back(st.stream);
    if (st.stream == used) ++used;
}

// ---------------------------------------------------------------- schedules

int validate_fine(const FineDag &dag, const int32_t *ops, const int32_t *op_stream,
                  int32_t n_ops, int32_t n_streams, FineSchedule &out)
{
    if (n_streams < 1 || n_streams > SPMV_MAX_STREAMS)
        return set_error(SPMV_EINVAL, "n_streams out of range");
    if (!ops || n_ops != int32_t(dag.tokens.size()))
        return set_error(SPMV_EPLAN, "a fine-grained order holds each of the " +
                                         std::to_string(dag.tokens.size()) + " tokens once");
    FinePrefix pre;
    pre.init(&dag, n_streams);
    // streams as given, relabelled by first use
    int32_t relabel[SPMV_MAX_STREAMS];
    std::fill(relabel, relabel + SPMV_MAX_STREAMS, -1);
    int32_t nused = 0;
    out = FineSchedule();
    for (int32_t k = 0; k < n_ops; ++k) {
        const int32_t t = ops[k];
        const int i = dag.find(t);
        if (i < 0) return set_error(SPMV_EPLAN, "token " + std::to_string(t) + " is not in this DAG");
        if (pre.placed[size_t(i)]) return set_error(SPMV_EPLAN, tok_name(t) + " appears twice");
        if (!pre.ready(i))
            return set_error(SPMV_EPLAN, tok_name(t) + " placed before what it depends on");
        int32_t s = -1;
        if (dag.gpu[size_t(i)]) {
            const int32_t g = op_stream ? op_stream[k] : 0;
            if (g < 0 || g >= n_streams)
                return set_error(SPMV_EPLAN, tok_name(t) + " bound to stream out of range");
            if (relabel[g] < 0) relabel[g] = nused++;
            s = relabel[g];
        }
        pre.placed[size_t(i)] = true;
        out.order.push_back(t);
        out.ostream.push_back(s);
    }
    if (out.order.front() != SPMV_OP_START || out.order.back() != SPMV_OP_END)
        return set_error(SPMV_EPLAN, "order must begin with start and end with end");
    out.n_streams_used = nused;
    return SPMV_OK;
}

void fine_default(const FineDag &dag, std::vector<int32_t> &ops, std::vector<int32_t> &streams)
{
    // the coarse default, peer by peer: receives posted first, every Pack
    // and its record on stream 0, y_L on stream 1 before the host waits
    ops.clear();
    streams.clear();
    auto add = [&](int32_t t, int32_t s) {
        ops.push_back(t);
        streams.push_back(s);
    };
    add(SPMV_OP_START, -1);
    for (int32_t q : dag.srcs) add(peer_tok(SPMV_OP_POST_RECV, q), -1);
    for (int32_t q : dag.dests) {
        add(peer_tok(SPMV_OP_PACK, q), 0);
        add(SPMV_CER_AFTER(peer_tok(SPMV_OP_PACK, q)), -1);
    }
    add(SPMV_OP_YL, dag.dests.empty() ? 0 : 1);
    for (int32_t q : dag.dests) {
        add(SPMV_CES_B4(peer_tok(SPMV_OP_POST_SEND, q)), -1);
        add(peer_tok(SPMV_OP_POST_SEND, q), -1);
    }
    for (int32_t q : dag.srcs) add(peer_tok(SPMV_OP_WAIT_RECV, q), -1);
    add(SPMV_OP_YR, dag.dests.empty() ? 0 : 1);
    for (int32_t q : dag.dests) add(peer_tok(SPMV_OP_WAIT_SEND, q), -1);
    add(SPMV_OP_END, -1);
}

int fine_count(const FineDag &dag, int32_t n_streams, double &count)
{
    const size_t n = dag.tokens.size();
    if (n > 40) return set_error(SPMV_EINVAL, "counting is limited to DAGs of 40 tokens");
    // linear extensions by dynamic programming over placed sets
    std::vector<uint64_t> pred(n, 0);
    for (size_t i = 0; i < n; ++i)
        for (int32_t j : dag.need[i]) pred[i] |= uint64_t(1) << j;
    std::map<uint64_t, double> ways;
    ways[0] = 1.0;
    for (size_t step = 0; step < n; ++step) {
        std::map<uint64_t, double> nxt;
        for (const auto &kv : ways)
            for (size_t i = 0; i < n; ++i) {
                const uint64_t b = uint64_t(1) << i;
                if ((kv.first & b) || (pred[i] & ~kv.first)) continue;
                nxt[kv.first | b] += kv.second;
            }
        ways.swap(nxt);
    }
    const double orders = ways.empty() ? 0.0 : ways.begin()->second;
    // canonical stream maps: partitions of the GPU vertices into at most
    // n_streams blocks, sum of Stirling numbers of the second kind
    int32_t g = 0;
    for (bool b : dag.gpu) g += b ? 1 : 0;
    std::vector<std::vector<double>> st(size_t(g) + 1, std::vector<double>(size_t(g) + 1, 0.0));
    st[0][0] = 1.0;
    for (int32_t a = 1; a <= g; ++a)
        for (int32_t k = 1; k <= a; ++k)
            st[size_t(a)][size_t(k)] = double(k) * st[size_t(a) - 1][size_t(k)] + st[size_t(a) - 1][size_t(k) - 1];
    double maps = 0.0;
    for (int32_t k = 1; k <= std::min(g, n_streams); ++k) maps += st[size_t(g)][size_t(k)];
    count = orders * (g ? maps : 1.0);
    return SPMV_OK;
}

}  // namespace spmv

using namespace spmv;

namespace {

int fine_plan(const spmv_plan_t *p)
{
    if (!p) return set_error(SPMV_EINVAL, "plan is NULL");
    if (p->share.nranks < 2) return set_error(SPMV_EINVAL, "a single rank has no fine-grained DAG");
    return SPMV_OK;
}

}  // namespace

extern "C" int spmv_fine_tokens(const spmv_plan_t *p, int32_t *tokens, int32_t cap, int32_t *n)
{
    if (int rc = fine_plan(p)) return rc;
    if (!n || cap < 0 || (cap > 0 && !tokens)) return set_error(SPMV_EINVAL, "bad output");
    const auto &t = p->fdag.tokens;
    std::copy(t.begin(), t.begin() + std::min<size_t>(size_t(cap), t.size()), tokens);
    *n = int32_t(t.size());
    return SPMV_OK;
}

extern "C" int spmv_fine_default(const spmv_plan_t *p, int32_t *ops, int32_t *streams,
                                 int32_t cap, int32_t *n_ops)
{
    if (int rc = fine_plan(p)) return rc;
    if (!n_ops || !ops || !streams) return set_error(SPMV_EINVAL, "bad output");
    std::vector<int32_t> o, st;
    fine_default(p->fdag, o, st);
    if (cap < int32_t(o.size())) return set_error(SPMV_EINVAL, "cap smaller than the order");
    std::copy(o.begin(), o.end(), ops);
    std::copy(st.begin(), st.end(), streams);
    *n_ops = int32_t(o.size());
    return SPMV_OK;
}

extern "C" int spmv_fine_count(const spmv_plan_t *p, int32_t n_streams, double *count)
{
    if (int rc = fine_plan(p)) return rc;
    if (!count || n_streams < 1 || n_streams > SPMV_MAX_STREAMS)
        return set_error(SPMV_EINVAL, "bad argument to spmv_fine_count");
    return fine_count(p->fdag, n_streams, *count);
}

extern "C" int spmv_fine_validate(const spmv_plan_t *p, const int32_t *op_order,
                                  const int32_t *op_stream, int32_t n_ops, int32_t n_streams)
{
    if (int rc = fine_plan(p)) return rc;
    FineSchedule f;
    return validate_fine(p->fdag, op_order, op_stream, n_ops, n_streams, f);
}
