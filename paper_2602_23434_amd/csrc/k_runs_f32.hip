// Run-based step kernels, float32 + cell-offset form.
#include "k_runs_impl.h"

namespace pl {

hipError_t launch_runs_f32(Ctx *c, const ItemDesc *table, const ItemDesc *host, int nitems, int total_units,
                           unsigned sf, unsigned *counter)
{
    return launch_runs_impl<PL_F32_OFFSET>(c, table, host, nitems, total_units, sf, counter);
}


bool runs_plan(const Ctx *c, const ItemDesc *host, int nitems, RunsPlan &pl)
{
    return c->d.prec == PL_F64 ? runs_plan_impl<PL_F64>(c, host, nitems, pl)
                               : runs_plan_impl<PL_F32_OFFSET>(c, host, nitems, pl);
}

}  // namespace pl
