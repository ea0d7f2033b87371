// Serving loop of the LGCD library: placeholder until the scheduler lands.
#include "dicod_serve.h"

namespace dicod {

struct Server {};

void server_destroy(Server* s) { delete s; }

int server_submit(dicod_ctx* ctx, const float*, int64_t, double, double, int, uint64_t*)
{
    return ctx_fail(ctx, DICOD_ENOTSUP, "dicod_submit: serving is not available in this build");
}

int server_poll(dicod_ctx* ctx, uint64_t, double*, dicod_stats*)
{
    return ctx_fail(ctx, DICOD_ENOREQ, "dicod_poll: unknown request");
}

}  // namespace dicod
