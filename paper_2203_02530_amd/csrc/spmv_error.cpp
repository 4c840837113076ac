// Thread-local error messages and small exported helpers of the C ABI.
#include <cstring>
#include <string>

#include "spmv_internal.h"

namespace spmv {

static thread_local std::string g_last_error;

int set_error(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int hip_error(hipError_t e, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
    return e == hipErrorOutOfMemory ? SPMV_ENOMEM : SPMV_EHIP;
}

void clear_error() { g_last_error.clear(); }

}  // namespace spmv

extern "C" const char *spmv_last_error(void) { return spmv::g_last_error.c_str(); }

extern "C" const char *spmv_version(void) { return "spmv-gfx950 0.1"; }

extern "C" int spmv_op_name(int32_t op, char *buf, int32_t cap)
{
    std::string s;
    if (spmv::op_name(op, s) != SPMV_OK)
        return spmv::set_error(SPMV_EINVAL, "unknown token " + std::to_string(op));
    if (buf && cap > 0) {
        size_t n = std::min(size_t(cap - 1), s.size());
        std::memcpy(buf, s.data(), n);
        buf[n] = 0;
    }
    return int(s.size());
}

extern "C" int spmv_plan_validate(int32_t nranks, const int32_t *op_order, int32_t n_ops,
                                  const int32_t *stream_map, int32_t n_streams)
{
    spmv::Schedule sch;
    return spmv::validate_schedule(nranks, op_order, n_ops, stream_map, n_streams, sch);
}

extern "C" int spmv_plan_space_count(int32_t nranks, int32_t n_streams, int64_t *count)
{
    if (!count || nranks < 1 || n_streams < 1 || n_streams > SPMV_MAX_STREAMS)
        return spmv::set_error(SPMV_EINVAL, "bad argument to spmv_plan_space_count");
    *count = int64_t(spmv::plan_space(nranks > 1, n_streams).size());
    return SPMV_OK;
}

extern "C" int spmv_plan_space_get(int32_t nranks, int32_t n_streams, int64_t index,
                                   int32_t *op_order, int32_t *n_ops, int32_t *stream_map)
{
    if (!op_order || !n_ops || !stream_map || nranks < 1 || n_streams < 1 ||
        n_streams > SPMV_MAX_STREAMS)
        return spmv::set_error(SPMV_EINVAL, "bad argument to spmv_plan_space_get");
    const auto &space = spmv::plan_space(nranks > 1, n_streams);
    if (index < 0 || index >= int64_t(space.size()))
        return spmv::set_error(SPMV_EINVAL, "plan index out of range");
    const auto &e = space[size_t(index)];
    std::copy(e.order.begin(), e.order.end(), op_order);
    *n_ops = int32_t(e.order.size());
    std::copy(e.stream, e.stream + SPMV_N_VERTICES, stream_map);
    return SPMV_OK;
}
