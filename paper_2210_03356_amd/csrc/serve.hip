// Serving entry points (continuous batching) -- placeholder until the
// batched scheduler lands; every call reports SIGN_EINVAL.
#include "driver.hpp"

extern "C" {

int sign_server_create(const sign_server_opts *o, sign_server **s) {
    (void)o;
    if (s) *s = nullptr;
    sfn::set_last_error("serving is not available in this build");
    return SIGN_EINVAL;
}
int sign_serve_submit(sign_server *s, const sign_csr *A, const sign_opts *o, uint64_t *ticket) {
    (void)s; (void)A; (void)o; (void)ticket;
    return SIGN_EINVAL;
}
int sign_serve_poll(sign_server *s, uint64_t ticket, sign_result **out) {
    (void)s; (void)ticket;
    if (out) *out = nullptr;
    return SIGN_EINVAL;
}
int sign_server_stats_get(sign_server *s, sign_server_stats *st) {
    (void)s; (void)st;
    return SIGN_EINVAL;
}
void sign_server_destroy(sign_server *s) { (void)s; }

}  // extern "C"
