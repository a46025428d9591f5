// placeholder: the learned warm start is added in its own step
#include "mgfr_internal.h"
namespace mgfr {
int nn_warm_start(mgfr_ctx *c, const double *delta, double *u, double *t_ms) { (void)c; (void)delta; (void)u; (void)t_ms; return set_error(MGFR_ERR_ARG, "network warm start is not available"); }
void nn_free(mgfr_ctx *c) { (void)c; }
}
