// The SpMV program DAG, the synchronisation rules of Table III, plan
// validation, stream canonicalisation and the enumeration of the design
// space (Sec. III-A to III-C of the paper).
#include <algorithm>
#include <array>
#include <map>
#include <mutex>

#include "spmv_internal.h"

namespace spmv {

namespace {

struct Edge {
    int32_t u, v;
};

// Edges of the SpMV DAG.  start precedes the three independent chains;
// Pack -> PostSend -> WaitSend; PostRecv -> WaitRecv -> Unpack -> y_R (x_R
// must be assembled before the remote product); y_L depends only on start;
// the leaves precede end.
const Edge kMultiEdges[] = {
    {SPMV_OP_START, SPMV_OP_PACK},         {SPMV_OP_START, SPMV_OP_YL},
    {SPMV_OP_START, SPMV_OP_POST_RECV},    {SPMV_OP_PACK, SPMV_OP_POST_SEND},
    {SPMV_OP_POST_SEND, SPMV_OP_WAIT_SEND}, {SPMV_OP_POST_RECV, SPMV_OP_WAIT_RECV},
    {SPMV_OP_WAIT_RECV, SPMV_OP_UNPACK},   {SPMV_OP_UNPACK, SPMV_OP_YR},
    {SPMV_OP_YL, SPMV_OP_END},             {SPMV_OP_YR, SPMV_OP_END},
    {SPMV_OP_WAIT_SEND, SPMV_OP_END},
};
const Edge kSingleEdges[] = {{SPMV_OP_START, SPMV_OP_YL}, {SPMV_OP_YL, SPMV_OP_END}};

const char *kVertexName[SPMV_N_VERTICES] = {"start",    "Pack",     "yL",       "PostSend",
                                            "PostRecv", "WaitSend", "WaitRecv", "Unpack",
                                            "yR",       "end"};

bool in_dag(bool multi, int32_t v)
{
    if (multi) return v >= 0 && v < SPMV_N_VERTICES;
    return v == SPMV_OP_START || v == SPMV_OP_YL || v == SPMV_OP_END;
}

template <class F>
void for_edges(bool multi, F f)
{
    if (multi)
        for (const Edge &e : kMultiEdges) f(e.u, e.v);
    else
        for (const Edge &e : kSingleEdges) f(e.u, e.v);
}

// Table III: the record/wait pair an edge u -> v needs, given the streams of
// GPU vertices.  Returns false when the edge needs none.
bool edge_sync(int32_t u, int32_t v, const int32_t *stream, int32_t &rec, int32_t &wait)
{
    if (v == SPMV_OP_END) return false;                 // end waits for everything
    if (vertex_type(u) == VType::CPU) return false;     // u finished when v starts
    if (vertex_type(v) == VType::CPU) {
        rec = SPMV_CER_AFTER(u);
        wait = SPMV_CES_B4(v);
        return true;
    }
    if (stream[u] == stream[v]) return false;           // same stream: in order
    rec = SPMV_CER_AFTER(u);
    wait = SPMV_CSWE_B4(v);
    return true;
}

}  // namespace

VType vertex_type(int32_t v)
{
    switch (v) {
        case SPMV_OP_PACK:
        case SPMV_OP_YL:
        case SPMV_OP_UNPACK:
        case SPMV_OP_YR: return VType::GPU;
        default: return VType::CPU;
    }
}

bool is_vertex(int32_t t) { return t >= 0 && t < SPMV_N_VERTICES; }

bool is_sync(int32_t t)
{
    int32_t k = t & ~0x0f;
    return (k == SPMV_SYNC_CER || k == SPMV_SYNC_CES || k == SPMV_SYNC_CSWE) &&
           sync_operand(t) < SPMV_N_VERTICES;
}

int op_name(int32_t t, std::string &out)
{
    // peer tokens (fine-grained program): the per-peer vertices, and their
    // synchronisation tokens, with the peer rank in brackets
    if (t >= 0x100) {
        const int32_t peer = ((t >> 8) & 0xff) - 1, base = t & 0xff;
        const int32_t v = base & 0x0f;
        const bool per_peer = v == SPMV_OP_PACK || v == SPMV_OP_POST_SEND ||
                              v == SPMV_OP_POST_RECV || v == SPMV_OP_WAIT_SEND ||
                              v == SPMV_OP_WAIT_RECV;
        if ((t >> 16) != 0 || peer < 0 || !per_peer || op_name(base, out) != SPMV_OK)
            return SPMV_EINVAL;
        out += "[" + std::to_string(peer) + "]";
        return SPMV_OK;
    }
    if (is_vertex(t)) {
        out = kVertexName[t];
        return SPMV_OK;
    }
    if (!is_sync(t)) return SPMV_EINVAL;
    const char *pre = sync_kind(t) == SPMV_SYNC_CER   ? "CER-after-"
                      : sync_kind(t) == SPMV_SYNC_CES ? "CES-b4-"
                                                      : "CSWE-b4-";
    out = std::string(pre) + kVertexName[sync_operand(t)];
    return SPMV_OK;
}

std::string tok_name(int32_t t)
{
    std::string s;
    if (op_name(t, s) != SPMV_OK) s = "token " + std::to_string(t);
    return s;
}

static std::string tok_str(int32_t t) { return tok_name(t); }

int validate_schedule(int32_t nranks, const int32_t *ops, int32_t n_ops,
                      const int32_t *stream_map, int32_t n_streams, Schedule &out)
{
    if (nranks < 1) return set_error(SPMV_EINVAL, "nranks < 1");
    if (n_streams < 1 || n_streams > SPMV_MAX_STREAMS)
        return set_error(SPMV_EINVAL, "n_streams out of range");
    if (!ops || n_ops < 2 || n_ops > SPMV_MAX_OPS)
        return set_error(SPMV_EPLAN, "operation order missing or of bad length");
    const bool multi = nranks > 1;
    out = Schedule();
    out.multi = multi;

    // 1. tokens known, vertices at most once, start first, end last
    int32_t vpos[SPMV_N_VERTICES];
    std::fill(vpos, vpos + SPMV_N_VERTICES, -1);
    std::vector<int32_t> order(ops, ops + n_ops);
    for (int32_t i = 0; i < n_ops; ++i) {
        int32_t t = order[size_t(i)];
        if (is_vertex(t)) {
            if (!in_dag(multi, t))
                return set_error(SPMV_EPLAN, tok_str(t) + " is not a vertex of this DAG");
            if (vpos[t] >= 0) return set_error(SPMV_EPLAN, tok_str(t) + " appears twice");
            vpos[t] = i;
        } else if (!is_sync(t)) {
            return set_error(SPMV_EPLAN, "unknown token " + std::to_string(t));
        }
    }
    if (order.front() != SPMV_OP_START) return set_error(SPMV_EPLAN, "order must begin with start");
    if (order.back() != SPMV_OP_END) return set_error(SPMV_EPLAN, "order must end with end");
    for (int32_t v = 0; v < SPMV_N_VERTICES; ++v) {
        if (!in_dag(multi, v) || vpos[v] >= 0) continue;
        if (v == SPMV_OP_UNPACK) continue;  // may be implied
        return set_error(SPMV_EPLAN, tok_str(v) + " missing from the order");
    }

    // 2. streams of GPU vertices
    for (int32_t v = 0; v < SPMV_N_VERTICES; ++v) out.stream[v] = -1;
    for (int32_t v = 0; v < SPMV_N_VERTICES; ++v) {
        if (vertex_type(v) != VType::GPU || vpos[v] < 0) continue;
        int32_t s = stream_map ? stream_map[v] : 0;
        if (s < 0 || s >= n_streams)
            return set_error(SPMV_EPLAN, tok_str(v) + " bound to stream out of range");
        out.stream[v] = s;
    }

    // 3. implied Unpack: on y_R's stream, immediately before y_R
    if (multi && vpos[SPMV_OP_UNPACK] < 0) {
        out.unpack_implied = true;
        order.insert(order.begin() + vpos[SPMV_OP_YR], SPMV_OP_UNPACK);
        out.stream[SPMV_OP_UNPACK] = out.stream[SPMV_OP_YR];
    }
    std::vector<int32_t> pos(64, -1);   // position of every token code (< 64)
    for (size_t i = 0; i < order.size(); ++i) {
        int32_t t = order[i];
        if (pos[size_t(t)] >= 0)
            return set_error(SPMV_EPLAN, tok_str(t) + " appears twice");
        pos[size_t(t)] = int32_t(i);
    }

    // 4. topological order
    int bad_u = -1, bad_v = -1;
    for_edges(multi, [&](int32_t u, int32_t v) {
        if (bad_u < 0 && pos[size_t(u)] >= pos[size_t(v)]) {
            bad_u = u;
            bad_v = v;
        }
    });
    if (bad_u >= 0)
        return set_error(SPMV_EPLAN, "not topological: " + tok_str(bad_u) + " must precede " +
                                         tok_str(bad_v));

    // 5. Table III synchronisation tokens: exactly the required ones, placed
    //    u < record < wait < v
    std::vector<bool> required(64, false);
    std::string err;
    for_edges(multi, [&](int32_t u, int32_t v) {
        int32_t rec, wait;
        if (!edge_sync(u, v, out.stream, rec, wait)) return;
        required[size_t(rec)] = required[size_t(wait)] = true;
        if (!err.empty()) return;
        if (pos[size_t(rec)] < 0 || pos[size_t(wait)] < 0) {
            err = "edge " + tok_str(u) + " -> " + tok_str(v) + " needs " + tok_str(rec) +
                  " and " + tok_str(wait);
        } else if (!(pos[size_t(u)] < pos[size_t(rec)] && pos[size_t(rec)] < pos[size_t(wait)] &&
                     pos[size_t(wait)] < pos[size_t(v)])) {
            err = "synchronisation for " + tok_str(u) + " -> " + tok_str(v) +
                  " must be placed " + tok_str(u) + " < " + tok_str(rec) + " < " +
                  tok_str(wait) + " < " + tok_str(v);
        }
    });
    if (!err.empty()) return set_error(SPMV_EPLAN, err);
    for (int32_t t : order)
        if (is_sync(t) && !required[size_t(t)])
            return set_error(SPMV_EPLAN, tok_str(t) + " is not required by any edge");

    // 6. canonical streams: relabel by first use along the order
    int32_t relabel[SPMV_MAX_STREAMS];
    std::fill(relabel, relabel + SPMV_MAX_STREAMS, -1);
    int32_t used = 0;
    for (int32_t t : order) {
        if (!is_vertex(t) || vertex_type(t) != VType::GPU) continue;
        int32_t s = out.stream[t];
        if (relabel[s] < 0) relabel[s] = used++;
    }
    for (int32_t v = 0; v < SPMV_N_VERTICES; ++v)
        if (out.stream[v] >= 0) out.stream[v] = relabel[out.stream[v]];
    out.n_streams_used = used;
    out.order = std::move(order);
    return SPMV_OK;
}

void default_order(int32_t nranks, std::vector<int32_t> &ops, int32_t *stream_map)
{
    for (int32_t v = 0; v < SPMV_N_VERTICES; ++v) stream_map[v] = -1;
    if (nranks <= 1) {
        ops = {SPMV_OP_START, SPMV_OP_YL, SPMV_OP_END};
        stream_map[SPMV_OP_YL] = 0;
        return;
    }
    // Post the receive first, launch Pack and y_L on different streams before
    // the host blocks for the send (the fast class of the paper's rules), then
    // y_R behind y_L so it adds into y directly.
    ops = {SPMV_OP_START,
           SPMV_OP_POST_RECV,
           SPMV_OP_PACK,
           SPMV_CER_AFTER(SPMV_OP_PACK),
           SPMV_OP_YL,
           SPMV_CES_B4(SPMV_OP_POST_SEND),
           SPMV_OP_POST_SEND,
           SPMV_OP_WAIT_RECV,
           SPMV_OP_YR,
           SPMV_OP_WAIT_SEND,
           SPMV_OP_END};
    stream_map[SPMV_OP_PACK] = 0;
    stream_map[SPMV_OP_YL] = 1;
    stream_map[SPMV_OP_YR] = 1;
}

// ---------------------------------------------------------------- enumeration
// A program prefix P_k (Sec. III-B): the tokens placed so far and the
// canonical streams of the GPU vertices among them.  The token universe is
// the DAG's vertices without Unpack (implied before y_R) plus the Table III
// tokens whose need does not depend on streams (in this DAG only GPU -> CPU
// edges need synchronisation).

void Prefix::init(bool multi_, int32_t n_streams_)
{
    multi = multi_;
    n_streams = n_streams_;
    tokens.clear();
    if (multi) {
        for (int32_t v = 0; v < SPMV_N_VERTICES; ++v)
            if (v != SPMV_OP_UNPACK) tokens.push_back(v);
        for_edges(true, [&](int32_t u, int32_t v) {
            if (u == SPMV_OP_UNPACK || v == SPMV_OP_UNPACK) return;
            int32_t rec, wait, none[SPMV_N_VERTICES];
            std::fill(none, none + SPMV_N_VERTICES, 0);
            if (edge_sync(u, v, none, rec, wait)) {
                tokens.push_back(rec);
                tokens.push_back(wait);
            }
        });
    } else {
        tokens = {SPMV_OP_START, SPMV_OP_YL, SPMV_OP_END};
    }
    std::sort(tokens.begin(), tokens.end());
    clear();
}

void Prefix::clear()
{
    order.clear();
    std::fill(stream, stream + SPMV_N_VERTICES, -1);
    used = 0;
    placed = 0;
}

// Predecessors of a vertex inside the enumerated DAG (Unpack implied, so y_R
// follows WaitRecv directly).
bool Prefix::preds_done(int32_t v) const
{
    bool ok = true;
    for_edges(multi, [&](int32_t u, int32_t w) {
        if (w == SPMV_OP_UNPACK || u == SPMV_OP_UNPACK) return;
        if (w == v && !(placed & bit(u))) ok = false;
    });
    if (multi && v == SPMV_OP_YR && !(placed & bit(SPMV_OP_WAIT_RECV))) ok = false;
    return ok;
}

bool Prefix::ready(int32_t t) const
{
    if (placed & bit(t)) return false;
    if (is_sync(t)) {
        int32_t k = sync_kind(t), x = sync_operand(t);
        if (k == SPMV_SYNC_CER) return (placed & bit(x)) != 0;
        // a wait is ready once every record it waits on is placed
        bool ok = true;
        for_edges(multi, [&](int32_t u, int32_t v) {
            int32_t rec, wait;
            if (v == x && edge_sync(u, v, stream, rec, wait) && wait == t && !(placed & bit(rec)))
                ok = false;
        });
        return ok;
    }
    if (t == SPMV_OP_END) {
        for (int32_t o : tokens)
            if (o != SPMV_OP_END && !(placed & bit(o))) return false;
        return true;
    }
    if (!preds_done(t)) return false;
    bool ok = true;
    for_edges(multi, [&](int32_t u, int32_t v) {
        int32_t rec, wait;
        if (v == t && edge_sync(u, v, stream, rec, wait) && !(placed & bit(wait))) ok = false;
    });
    return ok;
}

void Prefix::next(std::vector<Step> &out) const
{
    out.clear();
    for (int32_t t : tokens) {
        if (!ready(t)) continue;
        if (is_vertex(t) && vertex_type(t) == VType::GPU) {
            // streams already used, plus one new stream while any is left:
            // children equal under a stream bijection are one child
            const int32_t lim = std::min(used + 1, n_streams);
            for (int32_t s = 0; s < lim; ++s) out.push_back({t, s});
        } else {
            out.push_back({t, -1});
        }
    }
}

void Prefix::push(Step st)
{
    placed |= bit(st.token);
    order.push_back(st.token);
    if (st.stream >= 0) {
        stream[st.token] = st.stream;
        if (st.stream == used) ++used;
    }
}

void Prefix::pop()
{
    const int32_t t = order.back();
    order.pop_back();
    placed &= ~bit(t);
    if (is_vertex(t) && stream[t] >= 0) {   // sync tokens carry no stream
        if (stream[t] == used - 1) {
            bool again = false;   // still used by an earlier vertex?
            for (int32_t o : order)
                if (is_vertex(o) && stream[o] == stream[t] && o != t) again = true;
            if (!again) --used;
        }
        stream[t] = -1;
    }
}

namespace {

void enumerate(Prefix &p, std::vector<PlanEntry> &out)
{
    if (p.complete()) {
        PlanEntry e;
        e.order = p.order;
        std::copy(p.stream, p.stream + SPMV_N_VERTICES, e.stream);
        out.push_back(std::move(e));
        return;
    }
    std::vector<Prefix::Step> kids;
    p.next(kids);
    for (const Prefix::Step &k : kids) {
        p.push(k);
        enumerate(p, out);
        p.pop();
    }
}

}  // namespace

const std::vector<PlanEntry> &plan_space(bool multi, int32_t n_streams)
{
    static std::mutex mu;
    static std::map<std::pair<bool, int32_t>, std::vector<PlanEntry>> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto key = std::make_pair(multi, n_streams);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    Prefix p;
    p.init(multi, n_streams);
    std::vector<PlanEntry> out;
    enumerate(p, out);
    auto &v = cache[key];
    v = std::move(out);
    return v;
}

int64_t plan_index(bool multi, int32_t n_streams, const std::vector<int32_t> &order,
                   const int32_t *stream)
{
    static std::mutex mu;
    static std::map<std::pair<bool, int32_t>, std::map<std::string, int64_t>> cache;
    auto key_of = [](const std::vector<int32_t> &o, const int32_t *s) {
        std::string k(o.begin(), o.end());
        k.push_back(char(-2));
        for (int32_t v = 0; v < SPMV_N_VERTICES; ++v) k.push_back(char(s[v]));
        return k;
    };
    const auto &space = plan_space(multi, n_streams);
    std::lock_guard<std::mutex> lock(mu);
    auto &m = cache[std::make_pair(multi, n_streams)];
    if (m.empty())
        for (size_t i = 0; i < space.size(); ++i) m[key_of(space[i].order, space[i].stream)] = int64_t(i);
    auto f = m.find(key_of(order, stream));
    return f == m.end() ? -1 : f->second;
}

}  // namespace spmv
