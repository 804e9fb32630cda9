// Lane-group walk kernels for the hypersphere S^{n-1}_R (n >= 4): the
// instances of walk_group_dev.h for this manifold kind and their host entry
// points.
#include "walk_group_dev.h"

namespace mpwos {

MPWOS_GROUP_KIND_ENTRIES(sphere, kSphere, MPWOS_GROUP_L)

}  // namespace mpwos
