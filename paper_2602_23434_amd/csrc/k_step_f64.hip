// Instantiations of the gather -> push -> deposit kernels for the
// float64 particle form.
#include "k_step_impl.h"

namespace pl {

hipError_t launch_group_f64(Ctx *c, const ItemDesc *table, const ItemDesc *host, int nitems, int total_units,
                           unsigned sf, bool push, bool deposit, unsigned *counter)
{
    return launch_group_impl<PL_F64>(c, table, host, nitems, total_units, sf, push, deposit, counter);
}

}  // namespace pl
