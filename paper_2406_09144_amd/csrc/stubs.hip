// Entry points not implemented yet: they validate nothing and report
// FR_EUNSUPPORTED so the exported symbol set always matches include/frmi.h.
#include "objects.h"

extern "C" {

static int unsupported(const char *name) {
    frmi::set_last_error(std::string(name) + ": not implemented");
    return FR_EUNSUPPORTED;
}


int fr_make_psf_kernel(fr_plan *, const void *, double, fr_psf **out, void *) {
    if (out) *out = nullptr;
    return unsupported("fr_make_psf_kernel");
}
int fr_apply_RNR_exact(fr_plan *, const void *, const void *, void *, int64_t, void *) {
    return unsupported("fr_apply_RNR_exact");
}
int fr_likelihood_grad(fr_plan *, fr_psf *, int, const void *, const void *, const void *, const void *,
                       const void *, int64_t, void *, double *, void *) {
    return unsupported("fr_likelihood_grad");
}
int fr_cg_solve(fr_plan *, fr_psf *, const void *, const void *, const void *, const void *, void *, int, double,
                double *, int *, void *) {
    return unsupported("fr_cg_solve");
}
int fr_query_footprint(const fr_plan *, const fr_psf *, int, int64_t, size_t *, size_t *) {
    return unsupported("fr_query_footprint");
}

}  // extern "C"
