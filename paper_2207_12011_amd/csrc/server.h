// server.h -- continuous-batching request loop (internal).
#pragma once

#include "../../include/raypc.h"

namespace raypc {
struct Server;
// Stop the context's server if one runs; finishes queued and running requests first.
void server_shutdown(raypc_ctx* ctx);
}  // namespace raypc
