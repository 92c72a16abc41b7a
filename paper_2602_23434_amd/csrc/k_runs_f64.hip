// Run-based step kernels, float64 form.
#include "k_runs_impl.h"

namespace pl {

hipError_t launch_runs_f64(Ctx *c, const ItemDesc *table, const ItemDesc *host, int nitems, int total_units,
                           unsigned sf, unsigned *counter)
{
    return launch_runs_impl<PL_F64>(c, table, host, nitems, total_units, sf, counter);
}

}  // namespace pl
