// Entry points whose implementation is not in this build yet: they fail with
// BC_E_INVAL and a message, so a caller never gets a silent result.
#include "graph.h"

using namespace bcpp;

extern "C" {
static int missing(const char* what) { return fail(BC_E_INVAL, std::string(what) + ": not implemented"); }
int bc_server_create(size_t, int32_t, bc_server**) { return missing("bc_server_create"); }
int bc_server_add_graph(bc_server*, const bc_csr*, const int32_t*, int32_t, int32_t*) { return missing("bc_server_add_graph"); }
int bc_query_submit(bc_server*, int32_t, const int32_t*, int32_t, uint32_t, uint64_t*) { return missing("bc_query_submit"); }
int bc_query_poll(bc_server*, uint64_t, double*, int32_t*) { return missing("bc_query_poll"); }
int bc_server_stats_get(bc_server*, bc_server_stats*) { return missing("bc_server_stats_get"); }
void bc_server_destroy(bc_server*) {}
}
