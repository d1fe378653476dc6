// Kernel set for 2D grids.
#include "ops_impl.h"

namespace ipmg {
Ops* make_ops2d() { return new OpsImpl<2>(); }
}  // namespace ipmg
