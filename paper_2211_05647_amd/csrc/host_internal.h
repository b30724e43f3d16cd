// host_internal.h -- host-side declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
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
  int model = 0;      // FDTD_KINETIC_LINEAR / FULL / TWO_TERM
  int row = 0;        // stored values per plasma node: half (linear), nv (full) or
                      // 2 x the padded speed count (two-term)
  double dt = 0;
  VTable vt;
  std::vector<int32_t> cell_node;
  size_t off_E[2] = {0, 0}, off_H[2] = {0, 0}, off_J = 0, off_df = 0;
  size_t off_cell_node = 0, off_tau = 0, off_dens = 0, off_s = 0, off_b = 0, off_w = 0;
  size_t off_c = 0, off_v2h = 0;   // two-term model tables
  int ntap = 0;
  int64_t tap_cap = 0;
  size_t off_tap = 0;
};

// 1D launch (kernels1d.hip)
// cpl: 16-byte chunks per lane of every run in the launch (1, 2, 4; 0 = mixed or unknown),
// streaming: the launch's rows exceed what the Infinity Cache keeps between steps.
template <class T>
hipError_t launch_step1d(const void* runs, const void* tiles, int ntiles, int64_t step,
                         hipStream_t stream, bool full, int cpl = 0, bool streaming = false);

template <class T>
hipError_t launch_step1d_tt(const void* runs, const void* tiles, int ntiles, int64_t step,
                            bool pending, bool flush, hipStream_t stream);


// Temporally blocked 1D launch (kernels1d_tb.hip): k steps of every tile of one FP32 run.
constexpr int kDefaultTimeBlock = 9;
bool tb_supported(int half);             // stored bins per node the blocked kernel handles
int tb_block();                          // threads per work-group = largest extended range
int tb_max_rows(int half);               // plasma rows one work-group holds
int tb_blocks_per_cu(int k, int half);   // resident work-groups per compute unit
// Persistent batch launch (kernels1d_tb.hip): every run of a batch through steps [s0, s1)
// in one launch, (tile, block) items taken in order from a counter.
struct TbQueueTile;              // common.h
struct TbQueueArgs {
  const TbQueueTile* tiles;     // [ntiles] runs with the most blocks first
  const int64_t* seg_start;     // [nseg + 1]
  const int32_t* seg_round;     // [nseg]
  const int32_t* seg_tiles;     // [nseg]
  int32_t* done;                // [ntiles], zero
  unsigned long long* counter;  // zero
  int64_t s0, s1, delta;
  int32_t nseg, k;
};
int tb_queue_blocks_per_cu(int k);
hipError_t launch_batch1d_queue(const void* runs, const TbQueueArgs& a, int groups,
                                hipStream_t stream);
// the same for the two-term model (half = speeds padded to a power of two)
bool tb_tt_supported(int half);
int tb_tt_max_rows(int half);
int tb_tt_blocks_per_cu(int k, int half);
hipError_t launch_step1d_tb_tt(const void* runs, const void* tiles, int ntiles, int64_t step,
                               int k, int half, int64_t in_off, int64_t out_off,
                               hipStream_t stream);
// the same for the full-distribution model (half = Nv / 2)
bool tb_full_supported(int half);
int tb_full_max_rows(int half);
int tb_full_blocks_per_cu(int k, int half);
hipError_t launch_step1d_tb_full(const void* runs, const void* tiles, int ntiles, int64_t step,
                                 int k, int half, int64_t in_off, int64_t out_off,
                                 hipStream_t stream);
// K steps of the tiles; every run's rows are read at df + in_off and written at
// df + out_off (elements), two distinct copies
hipError_t launch_step1d_tb(const void* runs, const void* tiles, int ntiles, int64_t step, int k,
                            int half, int64_t in_off, int64_t out_off, hipStream_t stream);

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
int write_2d(Host2D* h, char* ws, int field, const double* src);
int check_probe_2d(const Host2D* h, int field, int i, int j);
double probe_scale_2d(const Host2D* h, int field);
int set_tiling_2d(Host2D* h, char* ws, hipStream_t stream, int tile, int cells_per_group);
void destroy_2d(Host2D* h);
int closure_counts_2d(const Host2D* h, int64_t* nm, int64_t* nk);

// 3D path (fdtd3d.cpp)
struct Host3D;
int validate_3d(const fdtd_grid* g, const fdtd_profile* p, const fdtd_source* s);
size_t workspace_3d(const fdtd_grid* g, const fdtd_profile* p, int max_probes, int probe_cap);
Host3D* make_3d(const fdtd_grid* g, const fdtd_profile* p, const fdtd_source* s,
                int max_probes, int probe_cap, size_t* state_bytes, size_t* probe_off);
int upload_3d(Host3D* h, char* ws, hipStream_t stream, const std::vector<ProbeInfo>& probes);
int probe_index_3d(const Host3D* h, int field, int i, int j, int k, int32_t* at);
hipError_t launch_step3d(Host3D* h, int64_t step, hipStream_t stream);
int points_3d(const Host3D* h);
int status_3d(Host3D* h, char* ws, int32_t* v);
int field_size_3d(const Host3D* h, int field, size_t* n);
int read_3d(Host3D* h, char* ws, int field, double* dst);
int write_3d(Host3D* h, char* ws, int field, const double* src);
void destroy_3d(Host3D* h);


// CPML coefficients of section 2 (eq. (4) and the grading formulas after it) at depth rho
// into a layer of thickness m dx: b, a (dimensionless: the derivative's dx folded in) and
// 1/kappa.  axis_profile samples them along an axis of n cells with the layer at both
// ends: e side at integer positions 0..n, h side at i + 1/2.
inline void cpml_point(const fdtd_grid& g, double rho, double thick, double dt, double* b, double* a,
                double* rk) {
  if (rho <= 0.0) { *b = 0.0; *a = 0.0; *rk = 1.0; return; }
  const double smax = g.cpml_sigma_factor * (g.cpml_order + 1.0) / (150.0 * M_PI * g.dx);
  const double r = rho / thick;
  const double sig = smax * std::pow(r, g.cpml_order);
  const double kap = 1.0 + (g.cpml_kappa_max - 1.0) * std::pow(r, g.cpml_order);
  const double alp = g.cpml_alpha_min + (g.cpml_alpha_max - g.cpml_alpha_min) * (1.0 - r);
  *b = std::exp(-(sig / kap + alp) * dt / kEps0);
  *a = sig * (*b - 1.0) / (sig * kap + alp * kap * kap);
  *rk = 1.0 / kap;
}

template <class T>
void axis_profile(const fdtd_grid& g, int n, int m, double dt, T* be, T* ae, T* rke, T* bh,
                  T* ah, T* rkh) {
  const double thick = m * g.dx;
  for (int i = 0; i <= n; ++i) {
    double rho = 0.0;
    if (m > 0 && i < m) rho = (m - i) * g.dx;
    if (m > 0 && i > n - m) rho = (i - (n - m)) * g.dx;
    double b, a, rk;
    cpml_point(g, rho, thick, dt, &b, &a, &rk);
    be[i] = (T)b; ae[i] = (T)a; rke[i] = (T)rk;
  }
  for (int i = 0; i < n; ++i) {
    const double x = i + 0.5;
    double rho = 0.0;
    if (m > 0 && x < m) rho = (m - x) * g.dx;
    if (m > 0 && x > n - m) rho = (x - (n - m)) * g.dx;
    double b, a, rk;
    cpml_point(g, rho, thick, dt, &b, &a, &rk);
    bh[i] = (T)b; ah[i] = (T)a; rkh[i] = (T)rk;
  }
}


}  // namespace fdtdp
