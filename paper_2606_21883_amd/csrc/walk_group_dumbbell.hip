// Lane-group walk kernels for the implicit dumbbell of Example 2: the
// instances of walk_group_dev.h for this manifold kind and their host entry
// points.
#include "walk_group_dev.h"

namespace mpwos {

MPWOS_GROUP_KIND_ENTRIES(dumbbell, kDumbbell, MPWOS_GROUP_L)

}  // namespace mpwos
