// fdtd2d.cpp -- 2D TEz path (placeholder until the 2D kernels land).
#include "host_internal.h"

namespace fdtdp {
struct Host2D { int unused; };
int validate_2d(const fdtd_grid*, const fdtd_profile*, const fdtd_source*) {
  return fail(FDTD_EINVAL, "2D grids are not available in this build");
}
size_t workspace_2d(const fdtd_grid*, const fdtd_profile*, int, int) { return 0; }
Host2D* make_2d(const fdtd_grid*, const fdtd_profile*, const fdtd_source*, int, int, size_t*, size_t*) { return nullptr; }
int upload_2d(Host2D*, char*, hipStream_t, const std::vector<ProbeInfo>&, size_t, int) { return FDTD_EINVAL; }
hipError_t launch_step2d(Host2D*, int64_t, hipStream_t) { return hipErrorInvalidValue; }
int field_size_2d(const Host2D*, int, size_t*) { return FDTD_EINVAL; }
int read_2d(Host2D*, char*, int, int64_t, double*) { return FDTD_EINVAL; }
int check_probe_2d(const Host2D*, int, int, int) { return FDTD_EINVAL; }
double probe_scale_2d(const Host2D*, int) { return 1.0; }
int set_tiling_2d(Host2D*, char*, hipStream_t, int, int) { return FDTD_EINVAL; }
void destroy_2d(Host2D* h) { delete h; }
}  // namespace fdtdp
