// placeholder: mixed precision is added in its own step
#include "mgfr_internal.h"
namespace mgfr {
int mixed_alloc(mgfr_ctx *c) { (void)c; return set_error(MGFR_ERR_ARG, "mixed precision is not available"); }
int solve_mixed(mgfr_ctx *c, double *u, mgfr_stats *st, double D) { (void)c; (void)u; (void)st; (void)D; return set_error(MGFR_ERR_ARG, "mixed precision is not available"); }
}
