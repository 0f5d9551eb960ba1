// Entry points whose implementation lands in later files of this library.
#include "host.h"

using namespace dses;

extern "C" {

dses_status dses_register_batch(const dses_problem *, int32_t, const dses_batch_opts *,
                                dses_result *, dses_status *)
{
    set_error("dses_register_batch: not available in this build");
    return DSES_E_STATE;
}

dses_status dses_server_create(const dses_server_opts *, dses_server **)
{
    set_error("serving: not available in this build");
    return DSES_E_STATE;
}
dses_status dses_server_submit(dses_server *, const dses_target *, const dses_rotset *,
                               const float *, int64_t, float, dses_metric, uint64_t *)
{
    return DSES_E_STATE;
}
dses_status dses_server_wait(dses_server *, uint64_t, int32_t, dses_result *, dses_status *)
{
    return DSES_E_STATE;
}
int32_t dses_server_poll(dses_server *, uint64_t) { return DSES_E_STATE; }
dses_status dses_server_timing(dses_server *, uint64_t, double *, double *) { return DSES_E_STATE; }
dses_status dses_server_destroy(dses_server *) { return DSES_E_STATE; }

}  // extern "C"
