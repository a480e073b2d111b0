// Serving scheduler (placeholder until the scheduler is in place).
#include "khop_impl.h"

extern "C" {
int khop_server_create(int64_t, int32_t, khop_server **) { return KHOP_EINTERNAL; }
int khop_server_add_graph(khop_server *, khop_graph *, int32_t *) { return KHOP_EINTERNAL; }
int khop_server_submit(khop_server *, int32_t, int32_t, int32_t, int64_t, uint64_t *) { return KHOP_EINTERNAL; }
int khop_server_poll(khop_server *, khop_result *, int64_t, int64_t *) { return KHOP_EINTERNAL; }
int khop_server_drain(khop_server *, int64_t) { return KHOP_EINTERNAL; }
int khop_server_destroy(khop_server *) { return KHOP_OK; }
}
