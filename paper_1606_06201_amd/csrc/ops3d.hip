// Kernel set for 3D grids.
#include "ops_impl.h"

namespace ipmg {
Ops* make_ops3d() { return new OpsImpl<3>(); }
}  // namespace ipmg
