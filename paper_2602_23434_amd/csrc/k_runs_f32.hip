// Run-based step kernels, float32 + cell-offset form.
#include "k_runs_impl.h"

namespace pl {

hipError_t launch_runs_f32(Ctx *c, const ItemDesc *table, const ItemDesc *host, int nitems, int total_units,
                           unsigned sf, unsigned *counter)
{
    return launch_runs_impl<PL_F32_OFFSET>(c, table, host, nitems, total_units, sf, counter);
}

}  // namespace pl
