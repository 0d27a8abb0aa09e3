// Multi-source batch and serving entry points (being built).
#include "runtime.h"

using namespace bfsmi;

extern "C" {
int bfs_run_batch(bfs_graph*, const int32_t*, int32_t, int8_t*, void*, bfs_stats*)
{
    return fail(BFS_ERR_INVALID, "batch search not built yet");
}
int bfs_server_create(bfs_server**, void*, size_t, const bfs_server_config*)
{
    return fail(BFS_ERR_INVALID, "server not built yet");
}
int bfs_server_add_graph(bfs_server*, bfs_graph*, int32_t*) { return fail(BFS_ERR_INVALID, "server not built yet"); }
int bfs_submit(bfs_server*, int32_t, int32_t, uint64_t*) { return fail(BFS_ERR_INVALID, "server not built yet"); }
int bfs_poll(bfs_server*, uint64_t, int32_t*, bfs_timing*) { return fail(BFS_ERR_INVALID, "server not built yet"); }
int bfs_server_drain(bfs_server*) { return fail(BFS_ERR_INVALID, "server not built yet"); }
int bfs_server_destroy(bfs_server*) { return fail(BFS_ERR_INVALID, "server not built yet"); }
}
