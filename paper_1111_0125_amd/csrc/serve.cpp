// Serving loop (submit / poll with continuous batching).
#include "internal.h"

extern "C" int stag_serve_shutdown_internal(stag_ctx* ctx) {
    (void)ctx;
    return STAG_OK;
}
