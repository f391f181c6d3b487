// server.cpp -- request server (continuous batching); filled in below.
#include "../../include/rhg.h"

extern "C" rhg_status rhg_server_create(int, uint64_t, rhg_server **) { return RHG_EINVAL; }
extern "C" rhg_status rhg_server_submit(rhg_server *, const rhg_params *, uint64_t *) { return RHG_EINVAL; }
extern "C" rhg_status rhg_server_wait(rhg_server *, uint64_t, int, rhg_graph **, double *) { return RHG_EINVAL; }
extern "C" void rhg_server_destroy(rhg_server *) {}
