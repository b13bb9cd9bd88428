// serve.hip -- real-time serving loop (wh_submit / wh_poll).
#include <hip/hip_runtime.h>

#include "wh_ctx.hpp"

namespace wh {
struct Server {};
void serve_shutdown(wh_ctx* ctx)
{
    delete ctx->server;
    ctx->server = nullptr;
}
} // namespace wh

extern "C" wh_status wh_submit(wh_ctx* ctx, const wh_request* req, uint64_t* ticket)
{
    (void)ctx;
    (void)req;
    (void)ticket;
    return WH_ERR_INVALID;
}

extern "C" wh_status wh_poll(wh_ctx* ctx, uint64_t ticket, wh_result* out)
{
    (void)ctx;
    (void)ticket;
    (void)out;
    return WH_ERR_INVALID;
}
