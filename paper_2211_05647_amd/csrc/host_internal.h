// host_internal.h -- host-side declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fdtd_plasma.h"

namespace fdtdp {

// CODATA 2018
constexpr double kC0 = 299792458.0;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kQe = 1.602176634e-19;
constexpr double kMe = 9.1093837015e-31;
constexpr double kEta0 = 1.0 / (kEps0 * kC0);   // sqrt(mu0/eps0) with mu0 = 1/(eps0 c^2)

extern thread_local std::string g_last_error;
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
bool is_pow2(int v);

// Velocity grid on +-vmax, cell-centred, and the Maxwellian F0 normalised on it (FP64).
struct VTable {
  int nv = 0;
  double vth = 0, dv = 0, mean_speed = 0, dt = 0;
  int nu_model = 0;
  std::vector<double> v, f;
};
VTable build_vtable(int dims, int nv, double vmax_over_vth, double te_ev, int nu_model,
                    double dt);

// Bump allocator over the workspace (256-byte aligned offsets).
class Carver {
 public:
  size_t take(size_t bytes);
  size_t size() const { return size_; }

 private:
  size_t size_ = 0;
};

struct ProbeInfo {
  int run, field, i, j;
};

struct Host1D {
  int nx = 0, nv = 0, half = 0, ncell = 0;
  int model = 0;      // FDTD_KINETIC_LINEAR / FULL
  int row = 0;        // stored values per plasma node: half (linear) or nv (full)
  double dt = 0;
  VTable vt;
  std::vector<int32_t> cell_node;
  size_t off_E[2] = {0, 0}, off_H[2] = {0, 0}, off_J = 0, off_df = 0;
  size_t off_cell_node = 0, off_tau = 0, off_dens = 0, off_s = 0, off_b = 0, off_w = 0;
  int ntap = 0;
  int64_t tap_cap = 0;
  size_t off_tap = 0, off_chunk = 0;
};

// 1D launch (kernels1d.hip)
template <class T>
hipError_t launch_step1d(const void* runs, const void* tiles, int ntiles, int64_t step,
                         hipStream_t stream, bool full);

hipError_t launch_batch1d_persistent(const void* runs, const int32_t* order, int nruns,
                                     int32_t* queue, int64_t s0, int64_t s1, int groups,
                                     hipStream_t stream);

// Temporally blocked 1D launch (kernels1d_tb.hip): k steps of every tile of one FP32 run.
constexpr int kDefaultTimeBlock = 7;
bool tb_supported(int half);             // stored bins per node the blocked kernel handles
int tb_block();                          // threads per work-group = largest extended range
int tb_max_rows(int half);               // plasma rows one work-group holds
int tb_blocks_per_cu(int k, int half);   // resident work-groups per compute unit
hipError_t launch_step1d_tb(const void* runs, const void* tiles, int ntiles, int64_t step, int k,
                            int half, hipStream_t stream);

// 2D TEz (fdtd2d.cpp / kernels2d.hip)
struct Host2D;
int validate_2d(const fdtd_grid* g, const fdtd_profile* p, const fdtd_source* s);
size_t workspace_2d(const fdtd_grid* g, const fdtd_profile* p, int max_probes, int probe_cap);
Host2D* make_2d(const fdtd_grid* g, const fdtd_profile* p, const fdtd_source* s, int max_probes,
                int probe_cap, size_t* state_bytes, size_t* probe_off);
int upload_2d(Host2D* h, char* ws, hipStream_t stream, const std::vector<ProbeInfo>& probes,
              size_t probe_off, int probe_cap);
hipError_t launch_step2d(Host2D* h, int64_t step, hipStream_t stream);
int field_size_2d(const Host2D* h, int field, size_t* n);
int read_2d(Host2D* h, char* ws, int field, int64_t step, double* dst);
int check_probe_2d(const Host2D* h, int field, int i, int j);
double probe_scale_2d(const Host2D* h, int field);
int set_tiling_2d(Host2D* h, char* ws, hipStream_t stream, int tile, int cells_per_group);
void destroy_2d(Host2D* h);
int closure_counts_2d(const Host2D* h, int64_t* nm, int64_t* nk);

}  // namespace fdtdp
