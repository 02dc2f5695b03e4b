// server.hip -- continuous-batching request loop.
#include "server.h"

namespace raypc {
void server_shutdown(raypc_ctx*) {}
}  // namespace raypc
