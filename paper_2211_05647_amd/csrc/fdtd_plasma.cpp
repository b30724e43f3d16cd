// fdtd_plasma.cpp -- host side of the C ABI declared in include/fdtd_plasma.h.
//
// Validates the problem statement, builds every table in FP64 (velocity grid, the
// frozen Maxwellian F0 and its derivative, collision-frequency shapes, moment weights,
// CPML profiles), rounds each table once to the storage precision, carves the device
// workspace, and enqueues the step kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fdtd_closure.h"
#include "../../include/fdtd_plasma.h"
#include "common.h"
#include "host_internal.h"

using namespace fdtdp;

namespace fdtdp {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(FDTD_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

VTable build_vtable(int dims, int nv, double vmax_over_vth, double te_ev, int nu_model,
                    double dt) {
  VTable t;
  t.nv = nv;
  t.vth = std::sqrt(kQe * te_ev / kMe);
  t.dv = 2.0 * vmax_over_vth * t.vth / nv;
  t.v.resize(nv);
  t.f.resize(nv);
  double norm = 0.0;
  for (int j = 0; j < nv; ++j) {
    t.v[j] = (j - 0.5 * (nv - 1)) * t.dv;
    t.f[j] = std::exp(-t.v[j] * t.v[j] / (2.0 * t.vth * t.vth));
    norm += t.f[j];
  }
  norm *= t.dv;
  for (int j = 0; j < nv; ++j) t.f[j] /= norm;
  // mean speed over the Maxwellian (1V: |v|, 2V: |(vx, vy)|)
  double mean = 0.0;
  if (dims == 1) {
    for (int j = 0; j < nv; ++j) mean += std::fabs(t.v[j]) * t.f[j] * t.dv;
  } else {
    for (int a = 0; a < nv; ++a)
      for (int b = 0; b < nv; ++b)
        mean += std::sqrt(t.v[a] * t.v[a] + t.v[b] * t.v[b]) * t.f[a] * t.f[b] * t.dv * t.dv;
  }
  t.mean_speed = mean;
  t.nu_model = nu_model;
  t.dt = dt;
  return t;
}

size_t Carver::take(size_t bytes) {
  size_t off = (size_ + 255) & ~size_t(255);
  size_ = off + bytes;
  return off;
}

}  // namespace fdtdp

// ----------------------------------------------------------------------------------
// 1D layout: state arrays of every run first (contiguous, saved/loaded as one blob),
// then probe rings, then read-only tables, run descriptors and tiles.
// ----------------------------------------------------------------------------------
namespace {

struct RunSpec1D {
  fdtd_grid g;
  fdtd_profile p;          // p.ne / p.nu_mean point into the owned copies below
  fdtd_source s;
  int64_t steps;
  std::vector<double> ne, nu;
  std::vector<int32_t> taps;   // training-pair tap nodes of this run
};

int validate_1d(const fdtd_grid* g, const fdtd_profile* p, const fdtd_source* s, bool batch) {
  if (!g || !p) return fail(FDTD_EINVAL, "null grid or profile");
  if (g->dims != 1) return fail(FDTD_EINVAL, "dims must be 1 here");
  if (g->nx < 8 || g->nx > (1 << 28)) return fail(FDTD_EINVAL, "nx out of range: %d", g->nx);
  if (!(g->dx > 0.0) || !std::isfinite(g->dx)) return fail(FDTD_EINVAL, "dx must be > 0");
  if (!(g->courant > 0.0) || g->courant > 1.0)
    return fail(FDTD_EINVAL, "1D Courant number must lie in (0, 1], got %g", g->courant);
  if (g->precision != FDTD_FP32 && g->precision != FDTD_FP64)
    return fail(FDTD_EINVAL, "unknown precision %d", g->precision);
  if (batch && g->precision != FDTD_FP32)
    return fail(FDTD_EINVAL, "batched runs are FP32");
  if (g->boundary != FDTD_BC_PEC && g->boundary != FDTD_BC_MUR1)
    return fail(FDTD_EINVAL, "1D boundary must be PEC or MUR1");
  if (p->kinetic == FDTD_KINETIC_TWO_TERM) {
    if (p->nv < 2 || p->nv > 256)
      return fail(FDTD_EINVAL, "two-term speed count nv must lie in [2, 256], got %d", p->nv);
    if (p->f0_model != FDTD_F0_MAXWELL && p->f0_model != FDTD_F0_DRUYVESTEYN)
      return fail(FDTD_EINVAL, "unknown f0_model %d", p->f0_model);
  } else if (!is_pow2(p->nv) || p->nv < 8 || p->nv > 1024) {
    return fail(FDTD_EINVAL, "nv must be a power of two in [8, 1024], got %d", p->nv);
  }
  if (!(p->te_ev > 0.0) || !(p->vmax_over_vth > 0.0))
    return fail(FDTD_EINVAL, "te_ev and vmax_over_vth must be > 0");
  if (p->nu_model != FDTD_NU_HARD_SPHERE && p->nu_model != FDTD_NU_CONST)
    return fail(FDTD_EINVAL, "unknown nu_model %d", p->nu_model);
  if (p->closure != FDTD_CLOSURE_KINETIC)
    return fail(FDTD_EINVAL, "1D runs take the kinetic closure");
  if (p->kinetic != FDTD_KINETIC_LINEAR && p->kinetic != FDTD_KINETIC_FULL &&
      p->kinetic != FDTD_KINETIC_TWO_TERM)
    return fail(FDTD_EINVAL, "unknown kinetic model %d", p->kinetic);
  if (!p->ne || !p->nu_mean) return fail(FDTD_EINVAL, "null ne or nu_mean");
  const int nx = g->nx;
  for (int i = 0; i <= nx; ++i) {
    if (!(p->ne[i] >= 0.0) || !std::isfinite(p->ne[i]))
      return fail(FDTD_EINVAL, "ne[%d] must be finite and >= 0", i);
    if (!(p->nu_mean[i] >= 0.0) || !std::isfinite(p->nu_mean[i]))
      return fail(FDTD_EINVAL, "nu_mean[%d] must be finite and >= 0", i);
  }
  if (p->ne[0] > 0 || p->ne[1] > 0 || p->ne[nx - 1] > 0 || p->ne[nx] > 0)
    return fail(FDTD_EINVAL, "the two end nodes on each side must be vacuum");
  if (s && s->kind != FDTD_SRC_NONE) {
    if (s->kind != FDTD_SRC_POINT_SOFT)
      return fail(FDTD_EINVAL, "1D source must be a point source");
    if (s->i < 2 || s->i > nx - 2) return fail(FDTD_EINVAL, "source node out of [2, nx-2]");
    if (!(s->tau_s > 0.0) || !std::isfinite(s->amplitude) || !std::isfinite(s->f_hz) ||
        !std::isfinite(s->t0_s))
      return fail(FDTD_EINVAL, "bad source parameters");
  }
  return FDTD_OK;
}

template <class T>
size_t sz(size_t n) { return n * sizeof(T); }

int default_tile_1d(int half, int elem, int nx, int ncell) {
  // about 32 KB of F1 per tile, at least 32 nodes, and enough tiles to fill the chip
  int row = half * elem;
  int t = std::max(32, std::min(kMaxTile1D, 32768 / std::max(row, 1)));
  (void)nx;
  (void)ncell;
  int p = 32;
  while (p * 2 <= t) p *= 2;
  return p;
}

}  // namespace

// Owned nodes per blocked tile in a batch (capped by what the extended range allows):
// the wider the tile, the less halo work per owned node.
constexpr int kTbBatchWidth = 512;
// F1 rows beyond this many bytes do not stay in the 256 MB Infinity Cache from one step to
// the next: one-step launches then stream them with nontemporal loads and stores
constexpr size_t kStreamRowBytes = size_t(192) << 20;

// Blocked tiles of one Nv: [off, off + limit.size()) of the blocked tile list, with the
// step limit of each tile's run (non-increasing).
struct TbSeg {
  int half = 0, off = 0;
  std::vector<int64_t> limit;
};

struct fdtd_plasma {
  int dims = 1;
  int precision = FDTD_FP32;
  int nruns = 1;
  int device = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool owns_ws = false;
  int64_t step = 0;
  bool started = false;
  int tile = 0;
  int cells_per_group = 0;
  // state region
  size_t state_off = 0, state_bytes = 0;
  // 1D
  std::vector<RunSpec1D> specs;
  std::vector<Host1D> h1;
  size_t runs_off = 0, tiles_off = 0;
  int ntiles = 0;
  std::vector<int64_t> tile_limit;   // step limit of each tile, non-increasing
  int one_cpl = 0;          // one-step launches: chunks per lane of every run (0: mixed)
  bool one_stream = false;  // one-step launches: rows streamed past the Infinity Cache
  size_t status_off = 0;
  int batch_mode = 1, batch_groups = 0, ntap = 0;   // batch default: K-step launches
  size_t qtiles_off = 0, qdone_off = 0, qstart_off = 0, qround_off = 0, qsegt_off = 0,
         qctr_off = 0;                              // persistent batch launch (mode 0)
  // temporal blocking of a single FP32 1D run: time_block steps per launch (1 = off)
  int time_block = kDefaultTimeBlock;
  size_t tbtiles_off = 0;
  int ntbtiles = 0;
  int64_t tb_rows = 0;     // F1 rows one blocked pass reads (owned plus halo)
  std::vector<TbSeg> tb_seg;
  std::vector<Tile1D> tb_host;   // the blocked tiles (host copy), per Nv group
  // the persistent launch's tables (host copies kept while their uploads may be pending)
  std::vector<TbQueueTile> q_tiles;
  std::vector<int64_t> q_start;
  std::vector<int32_t> q_round, q_segt;
  // A blocked launch reads a run's rows from one copy and writes them to the other, so
  // that no work-group reads halo rows a neighbour of the same launch has already
  // advanced: each run's second copy sits df_delta bytes after its rows (the state
  // region mirrored), df_cur[r] says which copy holds run r's current rows.  One-step
  // launches, readback and saved states use the first copy (moved back when needed).
  size_t df_delta = 0;
  std::vector<uint8_t> df_cur;
  // probes
  int max_probes = 0, probe_cap = 0;
  size_t probe_off = 0;
  std::vector<ProbeInfo> probes;
  // 2D
  Host2D* h2 = nullptr;
  // 3D
  Host3D* h3 = nullptr;
  // timing
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  int64_t last_n = 0;
};

namespace {

int elem_size(int precision) { return precision == FDTD_FP64 ? 8 : 4; }

// Compute the 1D layout; with h != nullptr also fill in device pointers (ws base).
size_t layout_1d(fdtd_plasma* h, const std::vector<RunSpec1D>& specs, int precision,
                 int max_probes, int probe_cap, std::vector<Host1D>* out) {
  Carver cv;
  const int es = elem_size(precision);
  std::vector<Host1D> hs(specs.size());
  for (size_t r = 0; r < specs.size(); ++r) {
    const auto& sp = specs[r];
    Host1D& x = hs[r];
    x.nx = sp.g.nx;
    x.nv = sp.p.nv;
    x.half = sp.p.nv / 2;
    x.model = sp.p.kinetic;
    if (x.model == FDTD_KINETIC_TWO_TERM) {
      // speed bins padded to a power of two of at least one 16-byte vector
      int hp = 16 / es;
      while (hp < sp.p.nv) hp *= 2;
      x.half = hp;
    }
    x.row = x.model == FDTD_KINETIC_LINEAR ? x.half : 2 * x.half;
    x.ncell = 0;
    for (int i = 0; i <= x.nx; ++i) if (sp.p.ne[i] > 0) ++x.ncell;
    for (int b = 0; b < 2; ++b) x.off_E[b] = cv.take((size_t)(x.nx + 1) * es);
    for (int b = 0; b < 2; ++b) x.off_H[b] = cv.take((size_t)(x.nx + 1) * es);
    x.off_J = cv.take((size_t)(x.nx + 1) * es);
    x.off_df = cv.take((size_t)std::max(x.ncell, 1) * x.row * es);
  }
  const size_t state_end = cv.size();
  const size_t mirror_off = cv.take(state_end);   // second copy of the rows (blocked launches)
  const size_t probe_off = cv.take((size_t)std::max(max_probes, 1) * std::max(probe_cap, 1) * es);
  for (size_t r = 0; r < specs.size(); ++r) {
    Host1D& x = hs[r];
    x.ntap = (int)specs[r].taps.size();
    x.tap_cap = specs[r].steps == INT64_MAX ? 0 : specs[r].steps;
    x.off_tap = cv.take((size_t)std::max<int64_t>(x.ntap * x.tap_cap, 1) * 2 * es);
    x.off_cell_node = cv.take(sz<int32_t>(std::max(x.ncell, 1)));
    x.off_tau = cv.take((size_t)std::max(x.ncell, 1) * es);
    x.off_dens = cv.take((size_t)std::max(x.ncell, 1) * es);
    x.off_s = cv.take((size_t)x.half * es);
    x.off_b = cv.take((size_t)x.half * es);
    x.off_c = cv.take((size_t)x.half * es);
    x.off_v2h = cv.take((size_t)x.half * es);
    x.off_w = cv.take(sz<double>(x.half));
  }
  const size_t runs_off = cv.take(specs.size() * (precision == FDTD_FP64 ? sizeof(Run1D<double>)
                                                                          : sizeof(Run1D<float>)));
  // tiles: worst case every node its own 32-node tile
  size_t max_tiles = 0;
  for (auto& x : hs) max_tiles += (size_t)(x.nx + 1 + 31) / 32;
  const size_t tiles_off = cv.take(max_tiles * sizeof(Tile1D));
  // tiles of the temporally blocked kernel (single runs; never narrower than 32 nodes)
  const size_t tbtiles_off = cv.take(max_tiles * sizeof(Tile1D));
  // persistent batch launch: its tile order, per-tile block counts, segment tables, counter
  const size_t qtiles_off = cv.take(max_tiles * sizeof(TbQueueTile));
  const size_t qdone_off = cv.take(sz<int32_t>(max_tiles));
  const size_t qstart_off = cv.take(sz<int64_t>(specs.size() + 1));
  const size_t qround_off = cv.take(sz<int32_t>(specs.size()));
  const size_t qsegt_off = cv.take(sz<int32_t>(specs.size()));
  const size_t qctr_off = cv.take(sz<uint64_t>(1));
  const size_t status_off = cv.take(sz<int32_t>(specs.size()));
  if (h) {
    h->qtiles_off = qtiles_off;
    h->qdone_off = qdone_off;
    h->qstart_off = qstart_off;
    h->qround_off = qround_off;
    h->qsegt_off = qsegt_off;
    h->qctr_off = qctr_off;
    h->status_off = status_off;
    h->state_off = 0;
    h->state_bytes = state_end;
    h->df_delta = mirror_off;
    h->df_cur.assign(specs.size(), 0);
    h->probe_off = probe_off;
    h->runs_off = runs_off;
    h->tiles_off = tiles_off;
    h->tbtiles_off = tbtiles_off;
  }
  if (out) *out = hs;
  return cv.size() + 256;
}

template <class T>
int upload_1d(fdtd_plasma* h) {
  std::vector<Run1D<T>> rd(h->nruns);
  for (int r = 0; r < h->nruns; ++r) {
    const RunSpec1D& sp = h->specs[r];
    Host1D& x = h->h1[r];
    const double dt = sp.g.courant * sp.g.dx / kC0;
    x.dt = dt;
    const int half = x.half;
    std::vector<T> s(half, T(0)), b(half, T(0)), cb(half, T(0)), v2h(half, T(0));
    std::vector<double> w(half, 0.0);
    double kc = 0.0;
    if (x.model == FDTD_KINETIC_TWO_TERM) {
      // speed grid v_k = (k + 1/2) gam on [0, vmax], F0 normalised by 4 pi gam sum v^2 F0
      const int vd = sp.p.nv;
      const double vth = std::sqrt(kQe * sp.p.te_ev / kMe);
      const double gam = sp.p.vmax_over_vth * vth / vd;
      double vd4 = 0.0;
      if (sp.p.f0_model == FDTD_F0_DRUYVESTEYN) {
        const double vd2 = 3.0 * vth * vth * std::tgamma(0.75) / std::tgamma(1.25);
        vd4 = vd2 * vd2;
      }
      std::vector<double> v(vd), F0(vd);
      double norm = 0.0, mean = 0.0;
      for (int k = 0; k < vd; ++k) {
        v[k] = (k + 0.5) * gam;
        F0[k] = sp.p.f0_model == FDTD_F0_DRUYVESTEYN ? std::exp(-std::pow(v[k], 4) / vd4)
                                                     : std::exp(-v[k] * v[k] / (2.0 * vth * vth));
        norm += 4.0 * M_PI * gam * v[k] * v[k] * F0[k];
      }
      for (int k = 0; k < vd; ++k) {
        F0[k] /= norm;
        mean += 4.0 * M_PI * gam * v[k] * v[k] * v[k] * F0[k];
      }
      for (int k = 0; k < vd; ++k) {
        const double dF0 = sp.p.f0_model == FDTD_F0_DRUYVESTEYN
                               ? -4.0 * v[k] * v[k] * v[k] * F0[k] / vd4
                               : -v[k] * F0[k] / (vth * vth);
        const double lo = k * gam, hi = (k + 1) * gam;   // faces of the bin
        const double wk = 0.5 * (lo * lo * lo + (k + 1 < vd ? hi * hi * hi : 0.0));
        s[k] = (T)(sp.p.nu_model == FDTD_NU_HARD_SPHERE ? v[k] / mean : 1.0);
        b[k] = (T)(2.0 * dt * (kQe / kMe) * dF0);
        w[k] = (dt / kEps0) * (-kQe) * (4.0 * M_PI / 3.0) * gam * wk;
        cb[k] = (T)(dt * kQe / (3.0 * kMe) / (v[k] * v[k] * gam));
        v2h[k] = (T)(k + 1 < vd ? 0.5 * hi * hi : 0.0);
      }
      kc = dt * (kQe / kMe) / gam;
    }
    VTable vt;
    if (x.model != FDTD_KINETIC_TWO_TERM) {
      vt = build_vtable(1, sp.p.nv, sp.p.vmax_over_vth, sp.p.te_ev, sp.p.nu_model, dt);
      kc = -(kQe / kMe) * dt / vt.dv;
    }
    x.vt = vt;
    for (int k = 0; k < half && x.model != FDTD_KINETIC_TWO_TERM; ++k) {
      const int j = half + k;  // v_j > 0
      const double g = -vt.v[j] * vt.f[j] / (vt.vth * vt.vth);       // dF0/dv per unit density
      s[k] = (T)(sp.p.nu_model == FDTD_NU_HARD_SPHERE ? std::fabs(vt.v[j]) / vt.mean_speed : 1.0);
      b[k] = (T)(2.0 * dt * (kQe / kMe) * g);
      w[k] = (dt / kEps0) * (-2.0 * kQe * vt.dv) * vt.v[j];
    }
    // full model: velocity CFL number per unit field, and the equilibrium part's face-flux
    // difference per unit density and field, -kc (fhat_{j+1} - fhat_{j-1}) (no flux
    // through +vmax: -kc (-(fhat_{j-1} + fhat_j)) on the last bin)
    if (x.model == FDTD_KINETIC_FULL) {
      for (int k = 0; k < half; ++k) {
        const int j = half + k;
        const double d0 = k + 1 < half ? vt.f[j + 1] - vt.f[j - 1] : -(vt.f[j - 1] + vt.f[j]);
        b[k] = (T)(-kc * d0);
      }
    }
    std::vector<int32_t> cn;
    std::vector<T> tau, dens;
    for (int i = 0; i <= x.nx; ++i) {
      if (sp.p.ne[i] > 0) {
        cn.push_back(i);
        tau.push_back((T)(dt * sp.p.nu_mean[i]));
        dens.push_back((T)sp.p.ne[i]);
      }
    }
    x.cell_node = cn;
    hipError_t e;
    char* base = h->ws;
    if (x.ncell > 0) {
      if ((e = hipMemcpyAsync(base + x.off_cell_node, cn.data(), cn.size() * 4, hipMemcpyHostToDevice, h->stream)) ||
          (e = hipMemcpyAsync(base + x.off_tau, tau.data(), tau.size() * sizeof(T), hipMemcpyHostToDevice, h->stream)) ||
          (e = hipMemcpyAsync(base + x.off_dens, dens.data(), dens.size() * sizeof(T), hipMemcpyHostToDevice, h->stream)))
        return hip_fail(e, "upload cell tables");
    }
    if ((e = hipMemcpyAsync(base + x.off_s, s.data(), half * sizeof(T), hipMemcpyHostToDevice, h->stream)) ||
        (e = hipMemcpyAsync(base + x.off_b, b.data(), half * sizeof(T), hipMemcpyHostToDevice, h->stream)) ||
        (e = hipMemcpyAsync(base + x.off_w, w.data(), half * sizeof(double), hipMemcpyHostToDevice, h->stream)) ||
        (e = hipMemcpyAsync(base + x.off_c, cb.data(), half * sizeof(T), hipMemcpyHostToDevice, h->stream)) ||
        (e = hipMemcpyAsync(base + x.off_v2h, v2h.data(), half * sizeof(T), hipMemcpyHostToDevice, h->stream)))
      return hip_fail(e, "upload velocity tables");

    Run1D<T>& R = rd[r];
    std::memset(&R, 0, sizeof R);
    for (int k = 0; k < 2; ++k) {
      R.E[k] = reinterpret_cast<T*>(base + x.off_E[k]);
      R.H[k] = reinterpret_cast<T*>(base + x.off_H[k]);
    }
    R.J = reinterpret_cast<T*>(base + x.off_J);
    R.df = reinterpret_cast<T*>(base + x.off_df);
    R.cell_node = reinterpret_cast<const int32_t*>(base + x.off_cell_node);
    R.tau = reinterpret_cast<const T*>(base + x.off_tau);
    R.dens = reinterpret_cast<const T*>(base + x.off_dens);
    R.s_bin = reinterpret_cast<const T*>(base + x.off_s);
    R.b_bin = reinterpret_cast<const T*>(base + x.off_b);
    R.w_bin = reinterpret_cast<const double*>(base + x.off_w);
    R.nx = x.nx;
    R.ncell = x.ncell;
    R.half = half;
    R.bc = sp.g.boundary == FDTD_BC_MUR1 ? 1 : 0;
    R.S = (T)sp.g.courant;
    R.q = (T)((sp.g.courant - 1.0) / (sp.g.courant + 1.0));
    R.src_node = (sp.s.kind == FDTD_SRC_POINT_SOFT && sp.s.amplitude != 0.0) ? sp.s.i : -1;
    R.src_amp = sp.s.amplitude;
    R.src_w = 2.0 * M_PI * sp.s.f_hz;
    R.src_tau = sp.s.kind != FDTD_SRC_NONE ? sp.s.tau_s : 1.0;
    R.src_t0 = sp.s.t0_s;
    R.dt = dt;
    R.step_limit = sp.steps;
    R.nprobe = 0;
    R.probe_cap = std::max(h->probe_cap, 1);
    R.probe_buf = reinterpret_cast<T*>(base + h->probe_off);
    R.ntap = x.ntap;
    for (int t = 0; t < x.ntap; ++t) R.tap_node[t] = sp.taps[t];
    R.tap_buf = reinterpret_cast<T*>(base + x.off_tap);
    R.tap_cap = x.tap_cap;
    R.status = reinterpret_cast<int32_t*>(base + h->status_off) + r;
    R.model = x.model;
    R.kc = (T)kc;
    R.c_bin = reinterpret_cast<const T*>(base + x.off_c);
    R.v2h_bin = reinterpret_cast<const T*>(base + x.off_v2h);
  }
  // probes
  for (size_t p = 0; p < h->probes.size(); ++p) {
    const ProbeInfo& pi = h->probes[p];
    Run1D<T>& R = rd[pi.run];
    R.probe_node[R.nprobe] = pi.i;
    R.probe_field[R.nprobe] = pi.field == FDTD_F_E ? 0 : (pi.field == FDTD_F_H ? 1 : 2);
    R.nprobe++;
  }
  // probe rings are per handle: shift each run's buffer to its first probe id
  for (int r = 0; r < h->nruns; ++r) {
    int first = -1;
    for (size_t p = 0; p < h->probes.size(); ++p)
      if (h->probes[p].run == r) { first = (int)p; break; }
    if (first >= 0) rd[r].probe_buf += (size_t)first * rd[r].probe_cap;
  }
  hipError_t e = hipMemcpyAsync(h->ws + h->runs_off, rd.data(), rd.size() * sizeof(Run1D<T>),
                                hipMemcpyHostToDevice, h->stream);
  if (e) return hip_fail(e, "upload run descriptors");
  return FDTD_OK;
}

// Tiles of the temporally blocked kernel: owned ranges of W nodes whose extended range
// (W + 2K nodes, clipped to the line) fits one work-group.  A single run takes W so that
// its tiles fill the device in as few rounds of resident work-groups as possible; in a
// batch every run takes W = kTbBatchWidth (or less if the extended range requires).  Tiles are grouped by Nv (one kernel instance per
// group) and, inside a group, ordered by the run's step limit, longest first, so that
// the tiles of the runs with K steps left are a prefix.  Blocking applies to FP32 runs
// whose Nv the kernel handles; if any run of a batch is not such a run, none is blocked.
int build_tb_tiles(fdtd_plasma* h) {
  h->ntbtiles = 0;
  h->tb_rows = 0;
  h->tb_seg.clear();
  h->tb_host.clear();
  const int k = h->time_block;
  if (k < 3 || h->precision != FDTD_FP32) return FDTD_OK;
  // plasma rows one work-group holds (the two-term kernel keeps two chunks per row)
  auto rows_cap = [](const Host1D& x) {
    return std::min(tb_block(), x.model == FDTD_KINETIC_TWO_TERM ? tb_tt_max_rows(x.half)
                                : x.model == FDTD_KINETIC_FULL   ? tb_full_max_rows(x.half)
                                                                 : tb_max_rows(x.half));
  };
  for (int r = 0; r < h->nruns; ++r) {
    const Host1D& x = h->h1[r];
    const bool ok = x.model == FDTD_KINETIC_LINEAR ? tb_supported(x.half)
                    : x.model == FDTD_KINETIC_TWO_TERM ? tb_tt_supported(x.half)
                    : x.model == FDTD_KINETIC_FULL ? tb_full_supported(x.half) : false;
    if (!ok) return FDTD_OK;
    if (rows_cap(x) - 2 * k < 32) return FDTD_OK;
  }
  int cus = 256;
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device);
  struct Item { int half; int64_t limit; Tile1D t; };
  std::vector<Item> items;
  for (int r = 0; r < h->nruns; ++r) {
    const Host1D& x = h->h1[r];
    const int cap = rows_cap(x);
    const int wmax = cap - 2 * k;
    const int nodes = x.nx + 1;
    int w = std::min(wmax, kTbBatchWidth);
    if (h->nruns == 1) {
      if (nodes < 4 * wmax) return FDTD_OK;   // too short to be worth blocking
      const int per_cu = x.model == FDTD_KINETIC_TWO_TERM ? tb_tt_blocks_per_cu(k, x.half)
                         : x.model == FDTD_KINETIC_FULL   ? tb_full_blocks_per_cu(k, x.half)
                                                          : tb_blocks_per_cu(k, x.half);
      const int conc = std::max(1, cus * per_cu);
      const int rounds = (nodes + conc * wmax - 1) / (conc * wmax);
      w = std::max(32, std::min(wmax, (nodes + rounds * conc - 1) / (rounds * conc)));
    }
    int c0 = 0, c1 = 0;
    for (int n0 = 0; n0 < nodes; n0 += w) {
      Tile1D t;
      t.run = r;
      t.node0 = n0;
      t.node1 = std::min(nodes, n0 + w);
      const int lo = std::max(0, n0 - k), hi = std::min(nodes, t.node1 + k);
      while (c0 < x.ncell && x.cell_node[c0] < lo) ++c0;
      c1 = std::max(c1, c0);
      while (c1 < x.ncell && x.cell_node[c1] < hi) ++c1;
      t.cell0 = c0;
      t.cell1 = c1;
      if (c1 - c0 > cap) return FDTD_OK;   // cannot happen (one cell per node)
      items.push_back({x.half, h->specs[r].steps, t});
    }
  }
  std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) {
    return a.half != b.half ? a.half < b.half : a.limit > b.limit;
  });
  std::vector<Tile1D> tiles;
  for (size_t i = 0; i < items.size(); ++i) {
    if (i == 0 || items[i].half != items[i - 1].half) {
      TbSeg sg;
      sg.half = items[i].half;
      sg.off = (int)i;
      h->tb_seg.push_back(sg);
    }
    h->tb_seg.back().limit.push_back(items[i].limit);
    tiles.push_back(items[i].t);
    h->tb_rows += items[i].t.cell1 - items[i].t.cell0;
  }
  hipError_t e = hipMemcpyAsync(h->ws + h->tbtiles_off, tiles.data(), tiles.size() * sizeof(Tile1D),
                                hipMemcpyHostToDevice, h->stream);
  if (e) return hip_fail(e, "upload blocked tiles");
  h->ntbtiles = (int)tiles.size();
  h->tb_host = std::move(tiles);
  return FDTD_OK;
}

int build_tiles_1d(fdtd_plasma* h) {
  // the one-step launches' form: 16-byte chunks per lane shared by every run (0 if they
  // differ), and whether the rows are streamed (more than the Infinity Cache keeps)
  {
    const int es = elem_size(h->precision), vpl = 16 / es;
    size_t rows_bytes = 0;
    h->one_cpl = -1;
    for (const Host1D& x : h->h1) {
      const int ch = x.half / vpl, cpl = ch < 64 ? 1 : ch / 64;
      h->one_cpl = h->one_cpl < 0 || h->one_cpl == cpl ? cpl : 0;
      rows_bytes += (size_t)x.ncell * x.row * es;
    }
    if (h->one_cpl < 0) h->one_cpl = 0;
    h->one_stream = rows_bytes > kStreamRowBytes;
  }
  std::vector<std::pair<int64_t, Tile1D>> all;
  for (int r = 0; r < h->nruns; ++r) {
    const Host1D& x = h->h1[r];
    const int es = elem_size(h->precision);
    int tile = h->tile > 0 ? h->tile : default_tile_1d(x.row, es, x.nx, x.ncell);
    // two-term rows are short (2 x 32 speeds): 64-node tiles measured fastest on a 65536-node
    // line (7.9 us per step against 9.5 at the 128 the row size alone would give)
    if (h->tile <= 0 && x.model == FDTD_KINETIC_TWO_TERM) tile = std::min(tile, 64);
    tile = std::max(32, std::min(kMaxTile1D, tile));
    int c = 0;
    for (int n0 = 0; n0 <= x.nx; n0 += tile) {
      Tile1D t;
      t.run = r;
      t.node0 = n0;
      t.node1 = std::min(x.nx + 1, n0 + tile);
      t.cell0 = c;
      while (c < x.ncell && x.cell_node[c] < t.node1) ++c;
      t.cell1 = c;
      all.push_back({h->specs[r].steps, t});
    }
  }
  // longest runs first: at batch step s the active tiles are a prefix
  std::stable_sort(all.begin(), all.end(),
                   [](const auto& a, const auto& b) { return a.first > b.first; });
  std::vector<Tile1D> tiles;
  h->tile_limit.clear();
  for (auto& pr : all) {
    tiles.push_back(pr.second);
    h->tile_limit.push_back(pr.first);
  }
  h->ntiles = (int)tiles.size();
  hipError_t e = hipMemcpyAsync(h->ws + h->tiles_off, tiles.data(), tiles.size() * sizeof(Tile1D),
                                hipMemcpyHostToDevice, h->stream);
  if (e) return hip_fail(e, "upload tiles");
  return build_tb_tiles(h);
}

// Work-groups of the persistent batch launch: the set count, else every one that fits.
int batch_groups(const fdtd_plasma* h) {
  if (h->batch_groups > 0) return h->batch_groups;
  int cus = 256;
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device);
  return std::max(1, cus * tb_queue_blocks_per_cu(h->time_block));
}

// The persistent batch launch of steps [s0, s1) (k_batch1d_queue): run r advances
// min(its step count, s1) - s0 steps in blocks of K, then its odd rest as one block or as
// rest - 1 and 1.  Every run's rows must sit in the first copy at the start; afterwards
// run r's rows sit in copy (its block count) & 1.
int run_queue(fdtd_plasma* h, int64_t s0, int64_t s1) {
  const int kb = h->time_block, nr = h->nruns;
  std::vector<int64_t> nblk(nr, 0), full(nr, 0), rest(nr, 0);
  for (int r = 0; r < nr; ++r) {
    const int64_t n = std::max<int64_t>(0, std::min(h->specs[r].steps, s1) - s0);
    full[r] = n / kb;
    rest[r] = n - full[r] * kb;
    nblk[r] = full[r] + (rest[r] == 0 ? 0 : (rest[r] & 1) ? 1 : 2);
  }
  std::vector<int> order;
  for (int r = 0; r < nr; ++r)
    if (nblk[r] > 0) order.push_back(r);
  if (order.empty()) return FDTD_OK;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nblk[a] > nblk[b]; });
  // each run's tiles in node order (the blocked tile list keeps them so), runs most blocks first
  std::vector<std::vector<Tile1D>> per(nr);
  for (const Tile1D& t : h->tb_host) per[t.run].push_back(t);
  h->q_tiles.clear();
  std::vector<int64_t> cum;   // tiles of the runs order[0..k]
  for (int r : order) {
    for (const Tile1D& t : per[r]) {
      TbQueueTile qt;
      qt.tile = t;
      qt.full = (int32_t)full[r];
      qt.rest = (int32_t)rest[r];
      qt.flags = t.node1 < h->h1[r].nx + 1 ? 1 : 0;
      h->q_tiles.push_back(qt);
    }
    cum.push_back((int64_t)h->q_tiles.size());
  }
  // segments in round order: rounds [nblk of order[k + 1], nblk of order[k]) have the
  // tiles of runs order[0..k] active
  h->q_start.clear();
  h->q_round.clear();
  h->q_segt.clear();
  int64_t items = 0;
  for (int k = (int)order.size() - 1; k >= 0; --k) {
    const int64_t lo = k + 1 < (int)order.size() ? nblk[order[k + 1]] : 0, hi = nblk[order[k]];
    if (hi <= lo) continue;
    h->q_start.push_back(items);
    h->q_round.push_back((int32_t)lo);
    h->q_segt.push_back((int32_t)cum[k]);
    items += (hi - lo) * cum[k];
  }
  h->q_start.push_back(items);
  const int ntq = (int)h->q_tiles.size();
  hipError_t e;
  if ((e = hipMemcpyAsync(h->ws + h->qtiles_off, h->q_tiles.data(), ntq * sizeof(TbQueueTile),
                          hipMemcpyHostToDevice, h->stream)) ||
      (e = hipMemcpyAsync(h->ws + h->qstart_off, h->q_start.data(), h->q_start.size() * 8,
                          hipMemcpyHostToDevice, h->stream)) ||
      (e = hipMemcpyAsync(h->ws + h->qround_off, h->q_round.data(), h->q_round.size() * 4,
                          hipMemcpyHostToDevice, h->stream)) ||
      (e = hipMemcpyAsync(h->ws + h->qsegt_off, h->q_segt.data(), h->q_segt.size() * 4,
                          hipMemcpyHostToDevice, h->stream)) ||
      (e = hipMemsetAsync(h->ws + h->qdone_off, 0, (size_t)ntq * 4, h->stream)) ||
      (e = hipMemsetAsync(h->ws + h->qctr_off, 0, 8, h->stream)))
    return hip_fail(e, "upload batch queue");
  TbQueueArgs a;
  a.tiles = reinterpret_cast<const TbQueueTile*>(h->ws + h->qtiles_off);
  a.seg_start = reinterpret_cast<const int64_t*>(h->ws + h->qstart_off);
  a.seg_round = reinterpret_cast<const int32_t*>(h->ws + h->qround_off);
  a.seg_tiles = reinterpret_cast<const int32_t*>(h->ws + h->qsegt_off);
  a.done = reinterpret_cast<int32_t*>(h->ws + h->qdone_off);
  a.counter = reinterpret_cast<unsigned long long*>(h->ws + h->qctr_off);
  a.s0 = s0;
  a.s1 = s1;
  a.delta = (int64_t)(h->df_delta / 4);
  a.nseg = (int32_t)h->q_round.size();
  a.k = kb;
  e = launch_batch1d_queue(h->ws + h->runs_off, a, batch_groups(h), h->stream);
  if (e) return hip_fail(e, "launch persistent batch kernel");
  for (int r : order) h->df_cur[r] = (uint8_t)(nblk[r] & 1);
  return FDTD_OK;
}

int finish_upload(fdtd_plasma* h) {
  int rc;
  if (h->dims == 1) {
    hipError_t ez = hipMemsetAsync(h->ws + h->status_off, 0, sizeof(int32_t) * h->nruns, h->stream);
    if (ez) return hip_fail(ez, "clear run status");
    rc = h->precision == FDTD_FP64 ? upload_1d<double>(h) : upload_1d<float>(h);
    if (rc) return rc;
    rc = build_tiles_1d(h);
    if (rc) return rc;
  } else if (h->dims == 3) {
    rc = upload_3d(h->h3, h->ws, h->stream, h->probes);
    if (rc) return rc;
  } else {
    rc = upload_2d(h->h2, h->ws, h->stream, h->probes, h->probe_off, h->probe_cap);
    if (rc) return rc;
  }
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e) return hip_fail(e, "synchronise after upload");
  return FDTD_OK;
}

int attach_workspace(fdtd_plasma* h, const fdtd_device* dev, size_t need) {
  if (dev->workspace) {
    if (dev->workspace_bytes < need)
      return fail(FDTD_ENOMEM, "workspace has %zu bytes, need %zu", dev->workspace_bytes, need);
    h->ws = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(dev->workspace) + 255) & ~uintptr_t(255));
    h->ws_bytes = dev->workspace_bytes;
    h->owns_ws = false;
  } else {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, need);
    if (e) return fail(FDTD_ENOMEM, "hipMalloc(%zu): %s", need, hipGetErrorString(e));
    h->ws = reinterpret_cast<char*>(p);
    h->ws_bytes = need;
    h->owns_ws = true;
  }
  // zero the evolving state (fields, F1, CPML memory) and the probe rings
  hipError_t e = hipMemsetAsync(h->ws + h->state_off, 0, h->state_bytes, h->stream);
  if (e) return hip_fail(e, "clear state");
  return FDTD_OK;
}

int check_device(const fdtd_device* dev) {
  if (!dev) return fail(FDTD_EINVAL, "null device binding");
  if (dev->max_probes < 0 || dev->max_probes > kMaxProbes)
    return fail(FDTD_EINVAL, "max_probes must lie in [0, %d]", kMaxProbes);
  if (dev->probe_capacity < 0) return fail(FDTD_EINVAL, "probe_capacity < 0");
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e || n <= 0) return fail(FDTD_EDEVICE, "no HIP device");
  if (dev->device < 0 || dev->device >= n) return fail(FDTD_EINVAL, "device %d out of range", dev->device);
  e = hipSetDevice(dev->device);
  if (e) return hip_fail(e, "hipSetDevice");
  return FDTD_OK;
}

int create_1d(int nruns, const fdtd_grid* grids, const fdtd_profile* profiles,
              const fdtd_source* sources, const int64_t* steps, int ntap,
              const int32_t* tap_nodes, const fdtd_device* dev, fdtd_plasma** out,
              bool batch) {
  int rc = check_device(dev);
  if (rc) return rc;
  fdtd_plasma* h = new (std::nothrow) fdtd_plasma();
  if (!h) return fail(FDTD_ENOMEM, "host allocation");
  h->dims = 1;
  h->nruns = nruns;
  h->precision = grids[0].precision;
  h->device = dev->device;
  h->stream = reinterpret_cast<hipStream_t>(dev->hip_stream);
  h->max_probes = dev->max_probes;
  h->probe_cap = dev->probe_capacity;
  h->specs.resize(nruns);
  for (int r = 0; r < nruns; ++r) {
    h->specs[r].g = grids[r];
    h->specs[r].p = profiles[r];
    // inputs are copied: the caller may free its arrays once create returns
    const size_t n = (size_t)grids[r].nx + 1;
    h->specs[r].ne.assign(profiles[r].ne, profiles[r].ne + n);
    h->specs[r].nu.assign(profiles[r].nu_mean, profiles[r].nu_mean + n);
    h->specs[r].p.ne = h->specs[r].ne.data();
    h->specs[r].p.nu_mean = h->specs[r].nu.data();
    fdtd_source none{};
    h->specs[r].s = sources ? sources[r] : none;
    h->specs[r].steps = (batch && steps) ? steps[r] : INT64_MAX;
    for (int t = 0; t < ntap; ++t) h->specs[r].taps.push_back(tap_nodes[(size_t)r * ntap + t]);
  }
  h->ntap = ntap;
  const size_t need = layout_1d(h, h->specs, h->precision, h->max_probes, h->probe_cap, &h->h1);
  rc = attach_workspace(h, dev, need);
  if (!rc) rc = finish_upload(h);
  if (!rc) {
    hipError_t e = hipEventCreate(&h->ev0);
    if (!e) e = hipEventCreate(&h->ev1);
    if (e) rc = hip_fail(e, "hipEventCreate");
  }
  if (rc) {
    fdtd_plasma_destroy(h);
    return rc;
  }
  *out = h;
  return FDTD_OK;
}

}  // namespace

extern "C" {

int fdtd_plasma_workspace_size(const fdtd_grid* grid, const fdtd_profile* profile,
                               const fdtd_device* dev, size_t* bytes) {
  if (!grid || !profile || !bytes) return fail(FDTD_EINVAL, "null argument");
  const int mp = dev ? dev->max_probes : 0, pc = dev ? dev->probe_capacity : 0;
  if (grid->dims == 2) {
    int rc = validate_2d(grid, profile, nullptr);
    if (rc) return rc;
    *bytes = workspace_2d(grid, profile, mp, pc);
    return FDTD_OK;
  }
  if (grid->dims == 3) {
    int rc = validate_3d(grid, profile, nullptr);
    if (rc) return rc;
    *bytes = workspace_3d(grid, profile, mp, pc);
    return FDTD_OK;
  }
  int rc = validate_1d(grid, profile, nullptr, false);
  if (rc) return rc;
  std::vector<RunSpec1D> specs(1);
  specs[0].g = *grid;
  specs[0].p = *profile;
  *bytes = layout_1d(nullptr, specs, grid->precision, mp, pc, nullptr);
  return FDTD_OK;
}

int fdtd_plasma_workspace_size_batch(int32_t nruns, const fdtd_grid* grids,
                                     const fdtd_profile* profiles, const int64_t* steps,
                                     int32_t ntap, const fdtd_device* dev, size_t* bytes) {
  if (nruns <= 0 || !grids || !profiles || !steps || !bytes)
    return fail(FDTD_EINVAL, "bad batch arguments");
  if (ntap < 0 || ntap > kMaxTaps) return fail(FDTD_EINVAL, "ntap must lie in [0, %d]", kMaxTaps);
  std::vector<RunSpec1D> specs(nruns);
  for (int r = 0; r < nruns; ++r) {
    int rc = validate_1d(&grids[r], &profiles[r], nullptr, true);
    if (rc) return rc;
    if (profiles[r].kinetic != profiles[0].kinetic)
      return fail(FDTD_EINVAL, "run %d: the runs of a batch share one kinetic model", r);
    if (steps[r] < 0) return fail(FDTD_EINVAL, "run %d: negative step count", r);
    specs[r].g = grids[r];
    specs[r].p = profiles[r];
    specs[r].steps = steps[r];
    specs[r].taps.assign(ntap, 0);
  }
  *bytes = layout_1d(nullptr, specs, FDTD_FP32, dev ? dev->max_probes : 0,
                     dev ? dev->probe_capacity : 0, nullptr);
  return FDTD_OK;
}

int fdtd_plasma_create(const fdtd_grid* grid, const fdtd_profile* profile,
                       const fdtd_source* source, const fdtd_device* dev, fdtd_plasma** out) {
  if (!grid || !profile || !out) return fail(FDTD_EINVAL, "null argument");
  if (grid->dims == 2) {
    int rc = validate_2d(grid, profile, source);
    if (rc) return rc;
    rc = check_device(dev);
    if (rc) return rc;
    fdtd_plasma* h = new (std::nothrow) fdtd_plasma();
    if (!h) return fail(FDTD_ENOMEM, "host allocation");
    h->dims = 2;
    h->nruns = 1;
    h->precision = grid->precision;
    h->device = dev->device;
    h->stream = reinterpret_cast<hipStream_t>(dev->hip_stream);
    h->max_probes = dev->max_probes;
    h->probe_cap = dev->probe_capacity;
    size_t state_bytes = 0, probe_off = 0;
    h->h2 = make_2d(grid, profile, source, dev->max_probes, dev->probe_capacity, &state_bytes,
                    &probe_off);
    if (!h->h2) {
      delete h;
      return fail(FDTD_ENOMEM, "host allocation (2D)");
    }
    h->state_off = 0;
    h->state_bytes = state_bytes;
    h->probe_off = probe_off;
    int rc2 = attach_workspace(h, dev, workspace_2d(grid, profile, dev->max_probes, dev->probe_capacity));
    if (!rc2) rc2 = finish_upload(h);
    if (!rc2) {
      hipError_t e = hipEventCreate(&h->ev0);
      if (!e) e = hipEventCreate(&h->ev1);
      if (e) rc2 = hip_fail(e, "hipEventCreate");
    }
    if (rc2) {
      fdtd_plasma_destroy(h);
      return rc2;
    }
    *out = h;
    return FDTD_OK;
  }
  if (grid->dims == 3) {
    int rc = validate_3d(grid, profile, source);
    if (rc) return rc;
    rc = check_device(dev);
    if (rc) return rc;
    fdtd_plasma* h = new (std::nothrow) fdtd_plasma();
    if (!h) return fail(FDTD_ENOMEM, "host allocation");
    h->dims = 3;
    h->nruns = 1;
    h->precision = grid->precision;
    h->device = dev->device;
    h->stream = reinterpret_cast<hipStream_t>(dev->hip_stream);
    h->max_probes = dev->max_probes;
    h->probe_cap = dev->probe_capacity;
    size_t state_bytes = 0, probe_off = 0;
    h->h3 = make_3d(grid, profile, source, h->max_probes, h->probe_cap, &state_bytes, &probe_off);
    if (!h->h3) {
      delete h;
      return fail(FDTD_ENOMEM, "host allocation (3D)");
    }
    h->state_off = 0;
    h->state_bytes = state_bytes;
    h->probe_off = probe_off;
    int rc2 = attach_workspace(h, dev, workspace_3d(grid, profile, h->max_probes, h->probe_cap));
    if (!rc2) rc2 = finish_upload(h);
    if (!rc2) {
      hipError_t e = hipEventCreate(&h->ev0);
      if (!e) e = hipEventCreate(&h->ev1);
      if (e) rc2 = hip_fail(e, "hipEventCreate");
    }
    if (rc2) {
      fdtd_plasma_destroy(h);
      return rc2;
    }
    *out = h;
    return FDTD_OK;
  }
  int rc = validate_1d(grid, profile, source, false);
  if (rc) return rc;
  return create_1d(1, grid, profile, source, nullptr, 0, nullptr, dev, out, false);
}

int fdtd_plasma_create_batch(int32_t nruns, const fdtd_grid* grids, const fdtd_profile* profiles,
                             const fdtd_source* sources, const int64_t* steps, int32_t ntap,
                             const int32_t* tap_nodes, const fdtd_device* dev,
                             fdtd_plasma** out) {
  if (nruns <= 0 || !grids || !profiles || !steps || !out)
    return fail(FDTD_EINVAL, "bad batch arguments");
  if (ntap < 0 || ntap > kMaxTaps || (ntap > 0 && !tap_nodes))
    return fail(FDTD_EINVAL, "ntap must lie in [0, %d] with tap_nodes given", kMaxTaps);
  for (int r = 0; r < nruns; ++r) {
    int rc = validate_1d(&grids[r], &profiles[r], sources ? &sources[r] : nullptr, true);
    if (rc) return fail(rc, "run %d: %s", r, g_last_error.c_str());
    if (profiles[r].kinetic != profiles[0].kinetic)
      return fail(FDTD_EINVAL, "run %d: the runs of a batch share one kinetic model", r);
    if (steps[r] < 0) return fail(FDTD_EINVAL, "run %d: negative step count", r);
    for (int t = 0; t < ntap; ++t) {
      const int32_t nd = tap_nodes[(size_t)r * ntap + t];
      if (nd < 0 || nd > grids[r].nx || !(profiles[r].ne[nd] > 0))
        return fail(FDTD_EINVAL, "run %d: tap %d is not a plasma node", r, t);
    }
  }
  return create_1d(nruns, grids, profiles, sources, steps, ntap, tap_nodes, dev, out, true);
}

// Move the rows of the runs whose current rows sit in the second copy back to the first
// (every such run, or with below >= 0 those whose step limit is below `below`), on the
// handle's stream.
static int rows_home(fdtd_plasma* h, int64_t below) {
  const size_t es = h->precision == FDTD_FP64 ? 8 : 4;
  for (int r = 0; r < h->nruns; ++r) {
    if (!h->df_cur[r] || (below >= 0 && h->specs[r].steps >= below)) continue;
    const Host1D& x = h->h1[r];
    const size_t bytes = (size_t)x.ncell * x.row * es;
    if (bytes) {
      hipError_t e = hipMemcpyAsync(h->ws + x.off_df, h->ws + x.off_df + h->df_delta, bytes,
                                    hipMemcpyDeviceToDevice, h->stream);
      if (e) return hip_fail(e, "move rows back");
    }
    h->df_cur[r] = 0;
  }
  return FDTD_OK;
}

int fdtd_plasma_step(fdtd_plasma* h) { return fdtd_plasma_run(h, 1); }

int fdtd_plasma_run(fdtd_plasma* h, int64_t nsteps) {
  if (!h) return fail(FDTD_EINVAL, "null handle");
  if (nsteps < 0) return fail(FDTD_EINVAL, "negative step count");
  hipError_t e = hipSetDevice(h->device);
  if (e) return hip_fail(e, "hipSetDevice");
  h->started = true;
  int64_t nsteps_loop = nsteps;
  if ((e = hipEventRecord(h->ev0, h->stream))) return hip_fail(e, "hipEventRecord");
  if (h->dims == 1 && h->nruns > 1 && h->batch_mode == 0 && h->ntbtiles > 0 &&
      h->h1[0].model == FDTD_KINETIC_LINEAR) {
    // one persistent launch for the whole call
    int rc = rows_home(h, -1);
    if (rc) return rc;
    rc = run_queue(h, h->step, h->step + nsteps);
    if (rc) return rc;
    nsteps_loop = 0;
  }
  int64_t k0 = 0;
  if (h->dims == 1 && h->ntbtiles > 0) {
    // K steps per launch for the runs with at least K steps left; a run that ends inside
    // the pass takes its last steps one launch per step.  Once a batch is down to fewer
    // blocked work-groups than compute units (only its longest runs left), and for the
    // last steps of the call, one step per launch.
    const int kb = h->time_block;
    auto count_ge = [](const std::vector<int64_t>& lim, int64_t v) {   // limits >= v
      return (int)(std::upper_bound(lim.begin(), lim.end(), v,
                                    [](int64_t x, int64_t l) { return x > l; }) -
                   lim.begin());
    };
    const Tile1D* tb = reinterpret_cast<const Tile1D*>(h->ws + h->tbtiles_off);
    const Tile1D* rt = reinterpret_cast<const Tile1D*>(h->ws + h->tiles_off);
    int min_tiles = 256;   // fewer blocked work-groups than compute units: step instead
    hipDeviceGetAttribute(&min_tiles, hipDeviceAttributeMultiprocessorCount, h->device);
    if (h->nruns == 1) min_tiles = 1;
    const int64_t delta = (int64_t)(h->df_delta / 4);   // FP32 elements
    for (; k0 + kb <= nsteps_loop; k0 += kb) {
      const int64_t s = h->step + k0;
      int nblocked = 0;
      for (const TbSeg& sg : h->tb_seg) nblocked += count_ge(sg.limit, s + kb);
      if (nblocked < min_tiles) break;   // the tail of a batch: one step per launch
      // the runs of this pass (step limit >= s + K) have taken every earlier blocked pass,
      // so their rows sit in the same copy
      int cur = -1;
      for (int r = 0; r < h->nruns; ++r) {
        if (h->specs[r].steps < s + kb) continue;
        if (cur >= 0 && cur != h->df_cur[r]) return fail(FDTD_ESTATE, "row copies out of step");
        cur = h->df_cur[r];
      }
      const int64_t in_off = cur == 1 ? delta : 0, out_off = cur == 1 ? 0 : delta;
      // every run of a handle has one model: run 0 decides; a two-term run's blocked
      // kernel leaves F0 complete, so the one-step launches after it start with no l = 0
      // update pending
      const int model = h->h1[0].model;
      for (const TbSeg& sg : h->tb_seg) {
        const int n = count_ge(sg.limit, s + kb);
        if (model == FDTD_KINETIC_TWO_TERM)
          e = launch_step1d_tb_tt(h->ws + h->runs_off, tb + sg.off, n, s, kb, sg.half, in_off,
                                  out_off, h->stream);
        else if (model == FDTD_KINETIC_FULL)
          e = launch_step1d_tb_full(h->ws + h->runs_off, tb + sg.off, n, s, kb, sg.half, in_off,
                                    out_off, h->stream);
        else
          e = launch_step1d_tb(h->ws + h->runs_off, tb + sg.off, n, s, kb, sg.half, in_off,
                               out_off, h->stream);
        if (e) return hip_fail(e, "launch blocked step kernel");
      }
      for (int r = 0; r < h->nruns; ++r)
        if (h->specs[r].steps >= s + kb) h->df_cur[r] ^= 1;
      if (h->nruns > 1) {
        // runs ending inside the pass take their last steps one per launch, in place
        const int rc = rows_home(h, s + kb);
        if (rc) return rc;
        const int p1 = count_ge(h->tile_limit, s + kb), p2 = count_ge(h->tile_limit, s + 1);
        for (int64_t ss = s; p2 > p1 && ss < s + kb; ++ss) {
          if (model == FDTD_KINETIC_TWO_TERM) {
            // the runs still stepping, and those whose last step was ss - 1 (their flush)
            const int n = count_ge(h->tile_limit, ss) - p1;
            e = launch_step1d_tt<float>(h->ws + h->runs_off, rt + p1, n, ss, ss > s, false,
                                        h->stream);
          } else {
            const int n = count_ge(h->tile_limit, ss + 1) - p1;
            e = launch_step1d<float>(h->ws + h->runs_off, rt + p1, n, ss, h->stream,
                                     model == FDTD_KINETIC_FULL, h->one_cpl, h->one_stream);
          }
          if (e) return hip_fail(e, "launch step kernel");
        }
      }
    }
  }
  if (h->dims == 1 && k0 < nsteps_loop) {
    const int rc = rows_home(h, -1);   // one-step launches work in place on the first copy
    if (rc) return rc;
  }
  for (int64_t k = k0; k < nsteps_loop; ++k) {
    const int64_t s = h->step + k;
    if (h->dims == 1) {
      // every run of a handle has one model: run 0 decides
      const int model = h->h1[0].model;
      // active tiles: those whose run still has steps left (limits are non-increasing);
      // two-term runs also those whose last step was s - 1, for their flush
      int n = h->ntiles;
      if (h->nruns > 1) {
        const int64_t lim = model == FDTD_KINETIC_TWO_TERM ? s - 1 : s;
        n = (int)(std::upper_bound(h->tile_limit.begin(), h->tile_limit.end(), lim,
                                   [](int64_t v, int64_t l) { return v >= l; }) -
                  h->tile_limit.begin());
      }
      if (model == FDTD_KINETIC_TWO_TERM) {
        // the l = 0 update of step s - 1 rides on step s (none pending at a call's start)
        const bool pending = k > k0;
        e = h->precision == FDTD_FP64
                ? launch_step1d_tt<double>(h->ws + h->runs_off, h->ws + h->tiles_off, n, s, pending, false, h->stream)
                : launch_step1d_tt<float>(h->ws + h->runs_off, h->ws + h->tiles_off, n, s, pending, false, h->stream);
      } else {
        const bool full = model == FDTD_KINETIC_FULL;
        e = h->precision == FDTD_FP64
                ? launch_step1d<double>(h->ws + h->runs_off, h->ws + h->tiles_off, n, s, h->stream, full,
                                        h->one_cpl, h->one_stream)
                : launch_step1d<float>(h->ws + h->runs_off, h->ws + h->tiles_off, n, s, h->stream, full,
                                       h->one_cpl, h->one_stream);
      }
    } else if (h->dims == 3) {
      e = launch_step3d(h->h3, s, h->stream);
    } else {
      e = launch_step2d(h->h2, s, h->stream);
    }
    if (e) return hip_fail(e, "launch step kernel");
  }
  if (h->dims == 1 && h->h1[0].model == FDTD_KINETIC_TWO_TERM && nsteps_loop > k0) {
    // the last step's l = 0 update, so that the state after the call is complete: the
    // runs that stepped up to the call's end (a run of a batch that stopped earlier took
    // its own flush then)
    const int64_t s = h->step + nsteps_loop;
    int n = h->ntiles;
    if (h->nruns > 1)
      n = (int)(std::upper_bound(h->tile_limit.begin(), h->tile_limit.end(), s - 1,
                                 [](int64_t v, int64_t l) { return v >= l; }) -
                h->tile_limit.begin());
    e = h->precision == FDTD_FP64
            ? launch_step1d_tt<double>(h->ws + h->runs_off, h->ws + h->tiles_off, n, s, true, true, h->stream)
            : launch_step1d_tt<float>(h->ws + h->runs_off, h->ws + h->tiles_off, n, s, true, true, h->stream);
    if (e) return hip_fail(e, "launch l = 0 flush");
  }
  if ((e = hipEventRecord(h->ev1, h->stream))) return hip_fail(e, "hipEventRecord");
  h->step += nsteps;
  h->last_n = nsteps;
  return FDTD_OK;
}

int fdtd_plasma_steps(const fdtd_plasma* h, int64_t* steps) {
  if (!h || !steps) return fail(FDTD_EINVAL, "null argument");
  *steps = h->step;
  return FDTD_OK;
}

int fdtd_plasma_last_run_ms(fdtd_plasma* h, double* ms) {
  if (!h || !ms) return fail(FDTD_EINVAL, "null argument");
  if (h->last_n <= 0) return fail(FDTD_ESTATE, "no run recorded");
  hipError_t e = hipEventSynchronize(h->ev1);
  if (e) return hip_fail(e, "hipEventSynchronize");
  float t = 0.f;
  e = hipEventElapsedTime(&t, h->ev0, h->ev1);
  if (e) return hip_fail(e, "hipEventElapsedTime");
  *ms = (double)t / (double)h->last_n;
  return FDTD_OK;
}

int fdtd_plasma_field_size(const fdtd_plasma* h, int32_t run, int32_t field, size_t* n) {
  if (!h || !n) return fail(FDTD_EINVAL, "null argument");
  if (run < 0 || run >= h->nruns) return fail(FDTD_ERANGE, "run %d out of range", run);
  if (h->dims == 2) return field_size_2d(h->h2, field, n);
  if (h->dims == 3) return field_size_3d(h->h3, field, n);
  const Host1D& x = h->h1[run];
  switch (field) {
    case FDTD_F_E: case FDTD_F_J: *n = x.nx + 1; return FDTD_OK;
    case FDTD_F_H: *n = x.nx; return FDTD_OK;
    case FDTD_F_DF:
      *n = (size_t)x.ncell * x.nv * (x.model == FDTD_KINETIC_TWO_TERM ? 2 : 1);
      return FDTD_OK;
    default: return fail(FDTD_EINVAL, "field %d not defined on a 1D grid", field);
  }
}

int fdtd_plasma_read_fields(fdtd_plasma* h, int32_t run, int32_t field, double* dst,
                            size_t dst_len, int64_t* step_out) {
  size_t n = 0;
  int rc = fdtd_plasma_field_size(h, run, field, &n);
  if (rc) return rc;
  if (!dst) return fail(FDTD_EINVAL, "null destination");
  if (dst_len < n) return fail(FDTD_ERANGE, "destination holds %zu values, need %zu", dst_len, n);
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e) return hip_fail(e, "synchronise");
  if (h->dims == 2) {
    rc = read_2d(h->h2, h->ws, field, h->step, dst);
    if (rc) return rc;
  } else if (h->dims == 3) {
    rc = read_3d(h->h3, h->ws, field, dst);
    if (rc) return rc;
  } else {
    const Host1D& x = h->h1[run];
    const int es = elem_size(h->precision);
    const int64_t srun = std::min<int64_t>(h->step, h->specs[run].steps);
    const int par = (int)(srun & 1);
    size_t off = 0, cnt = 0;
    double scale = 1.0;
    switch (field) {
      case FDTD_F_E: off = x.off_E[par]; cnt = x.nx + 1; break;
      case FDTD_F_H: off = x.off_H[par]; cnt = x.nx; scale = 1.0 / kEta0; break;
      case FDTD_F_J: off = x.off_J; cnt = x.nx + 1; scale = kEps0 / x.dt; break;
      case FDTD_F_DF:
        off = x.off_df + (h->df_cur[run] ? h->df_delta : 0);
        cnt = (size_t)x.ncell * x.row;
        break;
    }
    std::vector<char> buf(std::max<size_t>(cnt, 1) * es);
    if (cnt) {
      e = hipMemcpy(buf.data(), h->ws + off, cnt * es, hipMemcpyDeviceToHost);
      if (e) return hip_fail(e, "copy field");
    }
    auto val = [&](size_t k) -> double {
      return es == 8 ? reinterpret_cast<double*>(buf.data())[k] : reinterpret_cast<float*>(buf.data())[k];
    };
    if (field == FDTD_F_DF && x.model == FDTD_KINETIC_TWO_TERM) {
      // row: F1 then F0 - n F0hat over the padded speed bins
      for (int c = 0; c < x.ncell; ++c)
        for (int k = 0; k < x.nv; ++k) {
          dst[(size_t)c * 2 * x.nv + k] = val((size_t)c * x.row + k);
          dst[(size_t)c * 2 * x.nv + x.nv + k] = val((size_t)c * x.row + x.half + k);
        }
    } else if (field == FDTD_F_DF && x.model == FDTD_KINETIC_FULL) {
      // row: odd half then even half on the v > 0 bins
      for (int c = 0; c < x.ncell; ++c)
        for (int k = 0; k < x.half; ++k) {
          const double o = val((size_t)c * x.nv + k), ev = val((size_t)c * x.nv + x.half + k);
          dst[(size_t)c * x.nv + x.half + k] = ev + o;
          dst[(size_t)c * x.nv + x.half - 1 - k] = ev - o;
        }
    } else if (field == FDTD_F_DF) {
      for (int c = 0; c < x.ncell; ++c)
        for (int k = 0; k < x.half; ++k) {
          const double f = val((size_t)c * x.half + k);
          dst[(size_t)c * x.nv + x.half + k] = f;
          dst[(size_t)c * x.nv + x.half - 1 - k] = -f;
        }
    } else {
      for (size_t k = 0; k < cnt; ++k) dst[k] = val(k) * scale;
    }
    if (step_out) *step_out = srun;
  }
  if (step_out && h->dims != 1) *step_out = h->step;
  for (size_t k = 0; k < n; ++k)
    if (!std::isfinite(dst[k])) return fail(FDTD_ENUMERIC, "non-finite value at index %zu", k);
  return FDTD_OK;
}

int fdtd_plasma_write_fields(fdtd_plasma* h, int32_t run, int32_t field, const double* src,
                             size_t src_len) {
  if (!h || !src) return fail(FDTD_EINVAL, "null argument");
  const bool ok = h->dims == 1   ? (field == FDTD_F_E || field == FDTD_F_H)
                  : h->dims == 2 ? (field == FDTD_F_EX || field == FDTD_F_EY || field == FDTD_F_HZ)
                                 : (field == FDTD_F_EX || field == FDTD_F_EY || field == FDTD_F_EZ ||
                                    field == FDTD_F_HX || field == FDTD_F_HY || field == FDTD_F_HZ);
  if (!ok) return fail(FDTD_EINVAL, "field %d cannot be written on a %dD grid", field, h->dims);
  size_t n = 0;
  int rc = fdtd_plasma_field_size(h, run, field, &n);
  if (rc) return rc;
  if (src_len != n) return fail(FDTD_ERANGE, "source holds %zu values, the field %zu", src_len, n);
  for (size_t k = 0; k < n; ++k)
    if (!std::isfinite(src[k])) return fail(FDTD_EINVAL, "non-finite value at index %zu", k);
  hipError_t e = hipSetDevice(h->device);
  if (e) return hip_fail(e, "hipSetDevice");
  e = hipStreamSynchronize(h->stream);
  if (e) return hip_fail(e, "synchronise");
  if (h->dims == 2) return write_2d(h->h2, h->ws, field, src);
  if (h->dims == 3) return write_3d(h->h3, h->ws, field, src);
  const Host1D& x = h->h1[run];
  const int es = elem_size(h->precision);
  const int64_t srun = std::min<int64_t>(h->step, h->specs[run].steps);
  const int par = (int)(srun & 1);
  const size_t off = field == FDTD_F_E ? x.off_E[par] : x.off_H[par];
  const double scale = field == FDTD_F_E ? 1.0 : kEta0;
  std::vector<char> buf(std::max<size_t>(n, 1) * es);
  for (size_t k = 0; k < n; ++k) {
    if (es == 8) reinterpret_cast<double*>(buf.data())[k] = src[k] * scale;
    else reinterpret_cast<float*>(buf.data())[k] = (float)(src[k] * scale);
  }
  e = hipMemcpy(h->ws + off, buf.data(), n * es, hipMemcpyHostToDevice);
  if (e) return hip_fail(e, "write field");
  return FDTD_OK;
}

int fdtd_plasma_add_probe(fdtd_plasma* h, int32_t run, int32_t field, int32_t i, int32_t j,
                          int32_t* id) {
  if (!h || !id) return fail(FDTD_EINVAL, "null argument");
  if (h->dims == 3) return fail(FDTD_EINVAL, "3D handles take probes through fdtd_plasma_add_probe3d");
  if (h->started) return fail(FDTD_ESTATE, "probes must be added before the first step");
  if ((int)h->probes.size() >= h->max_probes) return fail(FDTD_ERANGE, "no probe slot left");
  if (h->probe_cap <= 0) return fail(FDTD_ERANGE, "probe_capacity is 0");
  if (run < 0 || run >= h->nruns) return fail(FDTD_ERANGE, "run out of range");
  if (h->dims == 1) {
    const Host1D& x = h->h1[run];
    if (field != FDTD_F_E && field != FDTD_F_H && field != FDTD_F_J)
      return fail(FDTD_EINVAL, "1D probes record E, H or J");
    if (i < 0 || i > x.nx || (field == FDTD_F_H && i >= x.nx)) return fail(FDTD_ERANGE, "probe index out of range");
    // a run's probes must be consecutive ids (one ring block per run)
    if (!h->probes.empty() && h->probes.back().run != run) {
      for (auto& p : h->probes)
        if (p.run == run) return fail(FDTD_EINVAL, "add all probes of a run consecutively");
    }
  } else {
    int rc = check_probe_2d(h->h2, field, i, j);
    if (rc) return rc;
  }
  ProbeInfo p{run, field, i, j};
  h->probes.push_back(p);
  *id = (int)h->probes.size() - 1;
  return finish_upload(h) ? FDTD_EDEVICE : FDTD_OK;
}

int fdtd_plasma_add_probe3d(fdtd_plasma* h, int32_t field, int32_t i, int32_t j, int32_t k,
                            int32_t* id) {
  if (!h || !id) return fail(FDTD_EINVAL, "null argument");
  if (h->dims != 3) return fail(FDTD_EINVAL, "fdtd_plasma_add_probe3d takes 3D handles");
  if (h->started) return fail(FDTD_ESTATE, "probes must be added before the first step");
  if ((int)h->probes.size() >= h->max_probes) return fail(FDTD_ERANGE, "no probe slot left");
  if (h->probe_cap <= 0) return fail(FDTD_ERANGE, "probe_capacity is 0");
  int32_t at = 0;
  const int rc = probe_index_3d(h->h3, field, i, j, k, &at);
  if (rc) return rc;
  ProbeInfo p{0, field, at, -1};   // the flat E index
  h->probes.push_back(p);
  *id = (int)h->probes.size() - 1;
  return finish_upload(h) ? FDTD_EDEVICE : FDTD_OK;
}

int fdtd_plasma_read_probe(fdtd_plasma* h, int32_t id, double* dst, size_t dst_len, size_t* n_out) {
  if (!h || !dst) return fail(FDTD_EINVAL, "null argument");
  if (id < 0 || id >= (int)h->probes.size()) return fail(FDTD_ERANGE, "probe id out of range");
  const ProbeInfo& p = h->probes[id];
  int64_t steps = h->step;
  if (h->dims == 1) steps = std::min<int64_t>(steps, h->specs[p.run].steps);
  const size_t n = (size_t)std::min<int64_t>(steps, h->probe_cap);
  if (dst_len < n) return fail(FDTD_ERANGE, "destination holds %zu values, need %zu", dst_len, n);
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e) return hip_fail(e, "synchronise");
  const int es = elem_size(h->precision);
  std::vector<char> buf((size_t)h->probe_cap * es);
  e = hipMemcpy(buf.data(), h->ws + h->probe_off + (size_t)id * h->probe_cap * es,
                buf.size(), hipMemcpyDeviceToHost);
  if (e) return hip_fail(e, "copy probe");
  double scale = 1.0;   // 3D probes record E (V/m)
  if (h->dims == 1) {
    const Host1D& x = h->h1[p.run];
    if (p.field == FDTD_F_H) scale = 1.0 / kEta0;
    if (p.field == FDTD_F_J) scale = kEps0 / x.dt;
  } else if (h->dims == 2) {
    scale = probe_scale_2d(h->h2, p.field);
  }
  for (size_t k = 0; k < n; ++k) {
    const size_t s = (size_t)((steps - (int64_t)n + (int64_t)k) % h->probe_cap);
    dst[k] = scale * (es == 8 ? reinterpret_cast<double*>(buf.data())[s] : reinterpret_cast<float*>(buf.data())[s]);
  }
  if (n_out) *n_out = n;
  return FDTD_OK;
}

int fdtd_plasma_state_size(const fdtd_plasma* h, size_t* bytes) {
  if (!h || !bytes) return fail(FDTD_EINVAL, "null argument");
  *bytes = 16 + h->state_bytes + (size_t)h->max_probes * h->probe_cap * elem_size(h->precision);
  return FDTD_OK;
}

int fdtd_plasma_save_state(fdtd_plasma* h, void* dst, size_t len) {
  size_t need = 0;
  int rc = fdtd_plasma_state_size(h, &need);
  if (rc) return rc;
  if (!dst || len < need) return fail(FDTD_ERANGE, "state buffer holds %zu bytes, need %zu", len, need);
  if (h->dims == 1) {
    rc = rows_home(h, -1);
    if (rc) return rc;
  }
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e) return hip_fail(e, "synchronise");
  char* d = reinterpret_cast<char*>(dst);
  const int64_t magic = 0x46445444504c534dLL;
  std::memcpy(d, &magic, 8);
  std::memcpy(d + 8, &h->step, 8);
  e = hipMemcpy(d + 16, h->ws + h->state_off, h->state_bytes, hipMemcpyDeviceToHost);
  if (!e && need > 16 + h->state_bytes)
    e = hipMemcpy(d + 16 + h->state_bytes, h->ws + h->probe_off, need - 16 - h->state_bytes,
                  hipMemcpyDeviceToHost);
  if (e) return hip_fail(e, "copy state");
  return FDTD_OK;
}

int fdtd_plasma_load_state(fdtd_plasma* h, const void* src, size_t len) {
  size_t need = 0;
  int rc = fdtd_plasma_state_size(h, &need);
  if (rc) return rc;
  if (!src || len != need) return fail(FDTD_ERANGE, "state blob has %zu bytes, need %zu", len, need);
  const char* s = reinterpret_cast<const char*>(src);
  int64_t magic = 0, step = 0;
  std::memcpy(&magic, s, 8);
  std::memcpy(&step, s + 8, 8);
  if (magic != 0x46445444504c534dLL || step < 0) return fail(FDTD_EINVAL, "not a state blob");
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e) return hip_fail(e, "synchronise");
  e = hipMemcpy(h->ws + h->state_off, s + 16, h->state_bytes, hipMemcpyHostToDevice);
  if (!e && need > 16 + h->state_bytes)
    e = hipMemcpy(h->ws + h->probe_off, s + 16 + h->state_bytes, need - 16 - h->state_bytes,
                  hipMemcpyHostToDevice);
  if (e) return hip_fail(e, "copy state");
  h->step = step;
  h->started = true;
  if (h->dims == 1) h->df_cur.assign(h->nruns, 0);
  return FDTD_OK;
}

int fdtd_plasma_set_batch_mode(fdtd_plasma* h, int32_t mode, int32_t groups) {
  if (!h) return fail(FDTD_EINVAL, "null handle");
  if (h->started) return fail(FDTD_ESTATE, "batch mode must be set before the first step");
  if (h->dims != 1) return fail(FDTD_EINVAL, "batch modes apply to 1D handles");
  if (mode != 0 && mode != 1) return fail(FDTD_EINVAL, "mode must be 0 or 1");
  if (groups < 0 || groups > 65536) return fail(FDTD_EINVAL, "groups out of range");
  h->batch_mode = mode;
  h->batch_groups = groups;
  return FDTD_OK;
}

int fdtd_plasma_read_taps(fdtd_plasma* h, int32_t run, double* dst, size_t dst_len, size_t* n_out) {
  if (!h || !dst) return fail(FDTD_EINVAL, "null argument");
  if (h->dims != 1) return fail(FDTD_EINVAL, "taps exist on 1D handles");
  if (run < 0 || run >= h->nruns) return fail(FDTD_ERANGE, "run out of range");
  const Host1D& x = h->h1[run];
  const int64_t steps = std::min<int64_t>(std::min<int64_t>(h->step, h->specs[run].steps), x.tap_cap);
  const size_t n = (size_t)x.ntap * steps * 2;
  if (dst_len < n) return fail(FDTD_ERANGE, "destination holds %zu values, need %zu", dst_len, n);
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e) return hip_fail(e, "synchronise");
  std::vector<float> buf((size_t)std::max<int64_t>(x.ntap * x.tap_cap, 1) * 2);
  if (n) {
    e = hipMemcpy(buf.data(), h->ws + x.off_tap, (size_t)x.ntap * x.tap_cap * 2 * 4, hipMemcpyDeviceToHost);
    if (e) return hip_fail(e, "copy taps");
  }
  const double js = kEps0 / x.dt;
  for (int t = 0; t < x.ntap; ++t)
    for (int64_t s = 0; s < steps; ++s) {
      const size_t src = ((size_t)t * x.tap_cap + s) * 2;
      const size_t d = ((size_t)t * steps + s) * 2;
      dst[d] = buf[src];
      dst[d + 1] = buf[src + 1] * js;
    }
  if (n_out) *n_out = n;
  return FDTD_OK;
}

int fdtd_plasma_tap_buffer(fdtd_plasma* h, int32_t run, const float** dev, int64_t* cap,
                           int32_t* ntap) {
  if (!h || !dev || !cap || !ntap) return fail(FDTD_EINVAL, "null argument");
  if (h->dims != 1 || h->precision != FDTD_FP32) return fail(FDTD_EINVAL, "taps exist on FP32 1D handles");
  if (run < 0 || run >= h->nruns) return fail(FDTD_ERANGE, "run out of range");
  const Host1D& x = h->h1[run];
  *dev = reinterpret_cast<const float*>(h->ws + x.off_tap);
  *cap = x.tap_cap;
  *ntap = x.ntap;
  return FDTD_OK;
}

int fdtd_plasma_closure_counts(fdtd_plasma* h, int64_t* closure_cells, int64_t* kinetic_cells) {
  if (!h || !closure_cells || !kinetic_cells) return fail(FDTD_EINVAL, "null argument");
  if (h->dims == 3) {
    *closure_cells = 0;
    *kinetic_cells = points_3d(h->h3);
    return FDTD_OK;
  }
  if (h->dims != 2) {
    *closure_cells = 0;
    int64_t k = 0;
    for (auto& x : h->h1) k += x.ncell;
    *kinetic_cells = k;
    return FDTD_OK;
  }
  return closure_counts_2d(h->h2, closure_cells, kinetic_cells);
}

int fdtd_plasma_run_status(fdtd_plasma* h, int32_t run, int32_t* status) {
  if (!h || !status) return fail(FDTD_EINVAL, "null argument");
  if (h->dims == 2) { *status = 0; return FDTD_OK; }
  if (run < 0 || run >= h->nruns) return fail(FDTD_ERANGE, "run out of range");
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e) return hip_fail(e, "synchronise");
  int32_t v = 0;
  if (h->dims == 3) {
    const int rc = status_3d(h->h3, h->ws, &v);
    if (rc) return rc;
  } else {
    e = hipMemcpy(&v, h->ws + h->status_off + 4 * (size_t)run, 4, hipMemcpyDeviceToHost);
    if (e) return hip_fail(e, "copy status");
  }
  *status = (v & 4) ? FDTD_ESTATE : v ? FDTD_ENUMERIC : FDTD_OK;
  if (v & 4) fail(FDTD_ESTATE, "run %d: a persistent batch launch gave up waiting for a tile", run);
  else if (v & 2) fail(FDTD_ENUMERIC, "run %d: a field broke the velocity CFL limit", run);
  else if (v & 1) fail(FDTD_ENUMERIC, "run %d: non-finite field", run);
  return FDTD_OK;
}

int fdtd_plasma_set_tiling(fdtd_plasma* h, int32_t tile, int32_t cells_per_group) {
  if (!h) return fail(FDTD_EINVAL, "null handle");
  if (h->started) return fail(FDTD_ESTATE, "tiling must be set before the first step");
  if (tile < 0 || cells_per_group < 0) return fail(FDTD_EINVAL, "negative tiling");
  if (h->dims == 1) {
    if (tile && (tile < 32 || tile > kMaxTile1D))
      return fail(FDTD_EINVAL, "1D tile must lie in [32, %d]", kMaxTile1D);
    if (tile) h->tile = tile;
    if (cells_per_group) h->cells_per_group = cells_per_group;
    int rc = build_tiles_1d(h);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(h->stream);
    return e ? hip_fail(e, "synchronise") : FDTD_OK;
  }
  if (h->dims == 3) return FDTD_OK;   // one fixed launch shape
  return set_tiling_2d(h->h2, h->ws, h->stream, tile, cells_per_group);
}

int fdtd_plasma_set_time_block(fdtd_plasma* h, int32_t steps) {
  if (!h) return fail(FDTD_EINVAL, "null handle");
  if (steps != 1 && steps != 3 && steps != 5 && steps != 7 && steps != 9)
    return fail(FDTD_EINVAL, "steps per pass must be 1, 3, 5, 7 or 9 (got %d)", steps);
  if (h->dims != 1) return FDTD_OK;
  h->time_block = steps;
  int rc = build_tb_tiles(h);
  if (rc) return rc;
  hipError_t e = hipStreamSynchronize(h->stream);
  return e ? hip_fail(e, "synchronise") : FDTD_OK;
}

int fdtd_plasma_time_block(const fdtd_plasma* h, int32_t* steps, int64_t* rows_per_launch) {
  if (!h || !steps) return fail(FDTD_EINVAL, "null argument");
  *steps = h->ntbtiles > 0 ? h->time_block : 1;
  if (rows_per_launch) *rows_per_launch = h->ntbtiles > 0 ? h->tb_rows : 0;
  return FDTD_OK;
}

void fdtd_plasma_destroy(fdtd_plasma* h) {
  if (!h) return;
  hipSetDevice(h->device);
  if (h->stream) hipStreamSynchronize(h->stream);
  if (h->ev0) hipEventDestroy(h->ev0);
  if (h->ev1) hipEventDestroy(h->ev1);
  if (h->owns_ws && h->ws) hipFree(h->ws);
  if (h->h2) destroy_2d(h->h2);
  if (h->h3) destroy_3d(h->h3);
  delete h;
}

const char* fdtd_plasma_strerror(int code) {
  switch (code) {
    case FDTD_OK: return "ok";
    case FDTD_EINVAL: return "invalid argument";
    case FDTD_ENOMEM: return "out of memory or workspace too small";
    case FDTD_EDEVICE: return "HIP device error";
    case FDTD_ERANGE: return "out of range";
    case FDTD_ENUMERIC: return "non-finite value in the fields";
    case FDTD_ESTATE: return "call not allowed in the current state";
    default: return "unknown error";
  }
}

const char* fdtd_plasma_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
