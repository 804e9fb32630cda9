// Point-cloud manifolds: placeholder until the kNN / local-fit path lands.
#include <hip/hip_runtime.h>

#include "host_internal.h"

namespace mpwos {

struct CloudState {
  int unused;
};

mpwos_status cloud_create(const mpwos_manifold_desc&, hipStream_t, CloudState**) {
  return fail(MPWOS_EINVAL, "point-cloud manifolds are not available in this build");
}
void cloud_destroy(CloudState* c) { delete c; }
double cloud_spacing_rmax(const CloudState*, const mpwos_options&) { return 0.0; }
void cloud_fill_args(const CloudState*, const mpwos_options&, WalkArgs&) {}
mpwos_status launch_cloud_walks(WalkArgs&, const mpwos_options&, hipStream_t, unsigned long long*) {
  return fail(MPWOS_EINVAL, "point-cloud manifolds are not available in this build");
}
hipError_t launch_cloud_cp(const WalkArgs&, const double*, double*, int64_t, hipStream_t) {
  return hipErrorInvalidValue;
}

}  // namespace mpwos
