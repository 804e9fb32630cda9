// Lane-group walk kernels for the product manifold of Example 3 (n = 9, one Philox block per lane): the
// instances of walk_group_dev.h for this manifold kind and their host entry
// points.
#include "walk_group_dev.h"

namespace mpwos {

MPWOS_GROUP_KIND_ENTRIES(product, kProduct, MPWOS_GROUP_L1)

}  // namespace mpwos
