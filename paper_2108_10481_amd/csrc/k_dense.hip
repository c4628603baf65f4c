// Assembled far field and mixed-precision solves.
#include "pbm_internal.h"

namespace pbm {

struct Dense {
    int dummy;
};

bool dense_fits(const DevMesh &) { return false; }
void build_dense(DevMesh &) { fail(PB_E_STATE, "assembled operator mode is not available yet"); }
void destroy_dense(DevMesh &d) { delete d.dense; d.dense = nullptr; }
void dense_apply(DevMesh &, const double *, double *) { fail(PB_E_STATE, "no assembled operator"); }
int mixed_refinement_solve(DevMesh &, const double *, const double *, double *, double *, int *)
{
    fail(PB_E_STATE, "mixed precision needs the assembled operator");
}
pb_status solve_multi(DevMesh &d, int n_sets, const pb_charges *sets, pb_result *out)
{
    pb_status worst = PB_OK;
    for (int k = 0; k < n_sets; ++k) {
        pb_status st = solve_on_mesh(d, &sets[k], &out[k]);
        if (st < 0) return st;
        if (st > worst) worst = st;
    }
    return worst;
}

}  // namespace pbm
