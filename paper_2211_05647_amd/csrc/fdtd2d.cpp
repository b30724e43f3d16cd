// fdtd2d.cpp -- host side of the 2D TEz path: validation, FP64 tables (velocity grid on
// the vy > 0 half plane, Maxwellian F0 and its derivatives, collision shapes, moment
// weights, CPML profiles of section 2), workspace layout, launches and readback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/fdtd_closure.h"
#include "common.h"
#include "host_internal.h"
#include "mlp_common.h"
#include "yee2d.h"

namespace fdtdp {

hipError_t mlp_launch_cells2d(const void* run, const MlpWeights& W, const MlpCells2D& C,
                              int64_t step, hipStream_t st);

struct Host2D {
  fdtd_grid g;
  fdtd_profile p;
  fdtd_source s;
  std::vector<double> ne, nu;
  int nx = 0, ny = 0, m = 0, nv = 0, half = 0, ncell = 0, es = 4;
  double dt = 0;
  int cells_per_block = 0;
  std::vector<int32_t> cell_idx;
  // workspace offsets
  size_t off_Ex = 0, off_Ey = 0, off_Hz = 0, off_phzx = 0, off_phzy = 0, off_pexy = 0,
         off_peyx = 0, off_Jcx = 0, off_Jcy = 0, off_df = 0;
  size_t off_cell = 0, off_tau = 0, off_dens = 0, off_s = 0, off_bx = 0, off_by = 0,
         off_wx = 0, off_wy = 0, off_prof = 0, off_run = 0;
  size_t state_end = 0, probe_off = 0, total = 0;
  char* ws = nullptr;
  int nbk = 0, nbh = 0, nbe = 0, hrows = 1, erows = 1;
  // learned closure (closure cells are not in cell_idx: those hold the kinetic cells)
  bool closure = false;
  std::vector<float> mlp_params;
  std::vector<int32_t> mlp_idx;
  std::vector<float> mlp_coef;     // [n][4] alpha, beta, q1, q2
  size_t off_ring = 0, off_midx = 0, off_mcoef = 0, off_W1 = 0, off_W2 = 0, off_W2T = 0, off_W2P = 0,
         off_mb = 0;
  MlpWeights W{};
  MlpCells2D C{};
};

namespace {

size_t layout(Host2D* h, int max_probes, int probe_cap) {
  Carver cv;
  const int es = h->es, nx = h->nx, ny = h->ny, m = std::max(h->m, 1);
  h->off_Ex = cv.take((size_t)(ny + 1) * nx * es);
  h->off_Ey = cv.take((size_t)ny * (nx + 1) * es);
  h->off_Hz = cv.take((size_t)ny * nx * es);
  h->off_phzx = cv.take((size_t)ny * 2 * m * es);
  h->off_phzy = cv.take((size_t)2 * m * nx * es);
  h->off_pexy = cv.take((size_t)2 * m * nx * es);
  h->off_peyx = cv.take((size_t)ny * 2 * m * es);
  h->off_Jcx = cv.take((size_t)ny * nx * es);
  h->off_Jcy = cv.take((size_t)ny * nx * es);
  h->off_df = cv.take((size_t)std::max(h->ncell, 1) * h->half * es);
  const size_t nm = std::max<size_t>(h->mlp_idx.size(), 1);
  h->off_ring = cv.take(nm * 2 * kHist * 4);
  h->state_end = cv.size();
  h->probe_off = cv.take((size_t)std::max(max_probes, 1) * std::max(probe_cap, 1) * es);
  const size_t nc = std::max(h->ncell, 1);
  h->off_cell = cv.take(nc * 4);
  h->off_tau = cv.take(nc * es);
  h->off_dens = cv.take(nc * es);
  h->off_s = cv.take((size_t)h->half * es);
  h->off_bx = cv.take((size_t)h->half * es);
  h->off_by = cv.take((size_t)h->half * es);
  h->off_wx = cv.take((size_t)h->half * 8);
  h->off_wy = cv.take((size_t)h->half * 8);
  h->off_prof = cv.take((size_t)(6 * (nx + 1) + 6 * (ny + 1)) * es);
  h->off_run = cv.take(std::max(sizeof(Run2D<double>), sizeof(Run2D<float>)));
  h->off_midx = cv.take(nm * 4);
  h->off_mcoef = cv.take(nm * 16);
  h->off_W1 = cv.take(kNH * kK1P * 2);
  h->off_W2 = cv.take(kNH * kK2P * 2);
  h->off_W2T = cv.take(kNH * kK2P * 2);
  h->off_W2P = cv.take(kNH * kK2P * 2);
  h->off_mb = cv.take((3 * kNH + 1) * 4);
  h->total = cv.size() + 256;
  return h->total;
}

// CPML coefficients at depth rho into a layer of thickness `thick` (section 2 formulas):
// b = exp(-(sigma/kappa + alpha) dt / eps0), a = sigma (b - 1) / (sigma kappa + alpha kappa^2)
template <class T>
int upload(Host2D* h, char* ws, hipStream_t st, const std::vector<ProbeInfo>& probes,
           size_t probe_off, int probe_cap) {
  h->ws = ws;
  const int nv = h->nv, half = h->half, nx = h->nx, ny = h->ny, m = h->m;
  const double dt = h->dt;
  VTable vt = build_vtable(2, nv, h->p.vmax_over_vth, h->p.te_ev, h->p.nu_model, dt);
  std::vector<T> s(half), bx(half), by(half);
  std::vector<double> wx(half), wy(half);
  const double vth2 = vt.vth * vt.vth;
  for (int a = 0; a < nv; ++a)
    for (int bb = 0; bb < nv / 2; ++bb) {
      const int q = a * (nv / 2) + bb;
      const int b = nv / 2 + bb;           // vy > 0 half plane
      const double vx = vt.v[a], vy = vt.v[b];
      const double f2 = vt.f[a] * vt.f[b];
      const double sp = std::sqrt(vx * vx + vy * vy);
      s[q] = (T)(h->p.nu_model == FDTD_NU_HARD_SPHERE ? sp / vt.mean_speed : 1.0);
      bx[q] = (T)(2.0 * dt * (kQe / kMe) * (-vx * f2 / vth2));
      by[q] = (T)(2.0 * dt * (kQe / kMe) * (-vy * f2 / vth2));
      wx[q] = (dt / kEps0) * (-2.0 * kQe * vt.dv * vt.dv) * vx;
      wy[q] = (dt / kEps0) * (-2.0 * kQe * vt.dv * vt.dv) * vy;
    }
  std::vector<T> tau, dens;
  for (int c = 0; c < h->ncell; ++c) {
    const int k = h->cell_idx[c];
    tau.push_back((T)(dt * h->nu[k]));
    dens.push_back((T)h->ne[k]);
  }
  std::vector<T> prof(6 * (nx + 1) + 6 * (ny + 1));
  T* px = prof.data();
  T* py = prof.data() + 6 * (nx + 1);
  axis_profile<T>(h->g, nx, m, dt, px, px + (nx + 1), px + 2 * (nx + 1), px + 3 * (nx + 1),
                  px + 4 * (nx + 1), px + 5 * (nx + 1));
  axis_profile<T>(h->g, ny, m, dt, py, py + (ny + 1), py + 2 * (ny + 1), py + 3 * (ny + 1),
                  py + 4 * (ny + 1), py + 5 * (ny + 1));
  hipError_t e;
  auto put = [&](size_t off, const void* src, size_t bytes) {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(ws + off, src, bytes, hipMemcpyHostToDevice, st);
  };
  if ((e = put(h->off_cell, h->cell_idx.data(), h->cell_idx.size() * 4)) ||
      (e = put(h->off_tau, tau.data(), tau.size() * sizeof(T))) ||
      (e = put(h->off_dens, dens.data(), dens.size() * sizeof(T))) ||
      (e = put(h->off_s, s.data(), half * sizeof(T))) ||
      (e = put(h->off_bx, bx.data(), half * sizeof(T))) ||
      (e = put(h->off_by, by.data(), half * sizeof(T))) ||
      (e = put(h->off_wx, wx.data(), half * 8)) || (e = put(h->off_wy, wy.data(), half * 8)) ||
      (e = put(h->off_prof, prof.data(), prof.size() * sizeof(T))))
    return hip_fail(e, "upload 2D tables");

  Run2D<T> R;
  std::memset(&R, 0, sizeof R);
  R.Ex = reinterpret_cast<T*>(ws + h->off_Ex);
  R.Ey = reinterpret_cast<T*>(ws + h->off_Ey);
  R.Hz = reinterpret_cast<T*>(ws + h->off_Hz);
  R.psi_hzx = reinterpret_cast<T*>(ws + h->off_phzx);
  R.psi_hzy = reinterpret_cast<T*>(ws + h->off_phzy);
  R.psi_exy = reinterpret_cast<T*>(ws + h->off_pexy);
  R.psi_eyx = reinterpret_cast<T*>(ws + h->off_peyx);
  R.Jcx = reinterpret_cast<T*>(ws + h->off_Jcx);
  R.Jcy = reinterpret_cast<T*>(ws + h->off_Jcy);
  R.df = reinterpret_cast<T*>(ws + h->off_df);
  R.cell_idx = reinterpret_cast<const int32_t*>(ws + h->off_cell);
  R.tau = reinterpret_cast<const T*>(ws + h->off_tau);
  R.dens = reinterpret_cast<const T*>(ws + h->off_dens);
  R.s_bin = reinterpret_cast<const T*>(ws + h->off_s);
  R.bx_bin = reinterpret_cast<const T*>(ws + h->off_bx);
  R.by_bin = reinterpret_cast<const T*>(ws + h->off_by);
  R.wx_bin = reinterpret_cast<const double*>(ws + h->off_wx);
  R.wy_bin = reinterpret_cast<const double*>(ws + h->off_wy);
  const T* dpx = reinterpret_cast<const T*>(ws + h->off_prof);
  const T* dpy = dpx + 6 * (nx + 1);
  R.bex = dpx; R.aex = dpx + (nx + 1); R.rkex = dpx + 2 * (nx + 1);
  R.bhx = dpx + 3 * (nx + 1); R.ahx = dpx + 4 * (nx + 1); R.rkhx = dpx + 5 * (nx + 1);
  R.bey = dpy; R.aey = dpy + (ny + 1); R.rkey = dpy + 2 * (ny + 1);
  R.bhy = dpy + 3 * (ny + 1); R.ahy = dpy + 4 * (ny + 1); R.rkhy = dpy + 5 * (ny + 1);
  R.nx = nx; R.ny = ny; R.m = m; R.ncell = h->ncell; R.half = half;
  R.cells_per_block = h->cells_per_block;
  R.nbk = h->nbk;
  R.hrows = h->hrows;
  R.erows = h->erows;
  R.S = (T)h->g.courant;
  R.src_kind = (h->s.kind != FDTD_SRC_NONE && h->s.amplitude != 0.0) ? h->s.kind : 0;
  R.src_i = h->s.i; R.src_j = h->s.j;
  R.src_amp = h->s.amplitude; R.src_w = 2.0 * M_PI * h->s.f_hz;
  R.src_tau = R.src_kind ? h->s.tau_s : 1.0; R.src_t0 = h->s.t0_s; R.dt = dt;
  R.probe_cap = std::max(probe_cap, 1);
  R.probe_buf = reinterpret_cast<T*>(ws + probe_off);
  for (const auto& pi : probes) {
    R.probe_field[R.nprobe] = pi.field;
    R.probe_i[R.nprobe] = pi.i;
    R.probe_j[R.nprobe] = pi.j;
    R.nprobe++;
  }
  e = put(h->off_run, &R, sizeof R);
  if (e) return hip_fail(e, "upload 2D run descriptor");
  if (h->closure && !h->mlp_idx.empty()) {
    // bf16 (ties to even) copies of the network weights, padded rows, as the kernels read them
    auto bf = [](float f) {
      uint32_t u;
      std::memcpy(&u, &f, 4);
      u += 0x7FFFu + ((u >> 16) & 1u);
      return (uint16_t)(u >> 16);
    };
    const float* P = h->mlp_params.data();
    std::vector<uint16_t> w1(kNH * kK1P, 0), w2(kNH * kK2P, 0), w2t(kNH * kK2P, 0),
        w2p(kNH * kK2P, 0);
    for (int n = 0; n < kNH; ++n) {
      for (int k = 0; k < kNIn; ++k) w1[n * kK1P + k] = bf(P[kOffW1 + n * kNIn + k]);
      for (int k = 0; k < kNH; ++k) {
        w2[n * kK2P + k] = bf(P[kOffW2 + n * kNH + k]);
        w2t[n * kK2P + k] = bf(P[kOffW2 + k * kNH + n]);
        w2p[n * kK2P + k] = bf(P[kOffW2 + n * kNH + mlp_w2p_col(k)]);
      }
    }
    std::vector<float> mb(3 * kNH + 1);
    for (int n = 0; n < kNH; ++n) {
      mb[n] = P[kOffB1 + n];
      mb[kNH + n] = P[kOffB2 + n];
      const uint32_t u = (uint32_t)bf(P[kOffW3 + n]) << 16;
      std::memcpy(&mb[2 * kNH + n], &u, 4);
    }
    mb[3 * kNH] = P[kOffB3];
    if ((e = put(h->off_midx, h->mlp_idx.data(), h->mlp_idx.size() * 4)) ||
        (e = put(h->off_mcoef, h->mlp_coef.data(), h->mlp_coef.size() * 4)) ||
        (e = put(h->off_W1, w1.data(), w1.size() * 2)) || (e = put(h->off_W2, w2.data(), w2.size() * 2)) ||
        (e = put(h->off_W2T, w2t.data(), w2t.size() * 2)) ||
        (e = put(h->off_W2P, w2p.data(), w2p.size() * 2)) || (e = put(h->off_mb, mb.data(), mb.size() * 4)))
      return hip_fail(e, "upload closure");
    h->W.W1 = reinterpret_cast<uint16_t*>(ws + h->off_W1);
    h->W.W2 = reinterpret_cast<uint16_t*>(ws + h->off_W2);
    h->W.W2T = reinterpret_cast<uint16_t*>(ws + h->off_W2T);
    h->W.W2P = reinterpret_cast<uint16_t*>(ws + h->off_W2P);
    h->W.b1 = reinterpret_cast<float*>(ws + h->off_mb);
    h->W.b2 = h->W.b1 + kNH;
    h->W.w3q = h->W.b1 + 2 * kNH;
    h->W.b3 = h->W.b1 + 3 * kNH;
    h->C.idx = reinterpret_cast<const int32_t*>(ws + h->off_midx);
    h->C.coef = reinterpret_cast<const float*>(ws + h->off_mcoef);
    h->C.ring = reinterpret_cast<float*>(ws + h->off_ring);
    h->C.n = (int)h->mlp_idx.size();
  }
  return FDTD_OK;
}

void set_grid(Host2D* h) {
  h->nbk = h->ncell > 0 ? (h->ncell + h->cells_per_block - 1) / h->cells_per_block : 0;
  h->hrows = field_rows(h->nx, h->ny);
  h->erows = field_rows(h->nx + 1, h->ny + 1);
  h->nbh = ((h->nx + kBlock - 1) / kBlock) * ((h->ny + h->hrows - 1) / h->hrows);
  h->nbe = ((h->nx + kBlock) / kBlock) * ((h->ny + 1 + h->erows - 1) / h->erows);
}

}  // namespace

template <class T>
hipError_t launch_step2d_t(const void* run, int half, int nbk, int nbh, int nbe, int64_t step,
                           hipStream_t stream, bool streaming);
hipError_t launch_step2d_closure(const void* run, int half, int nbk, int nx, int ny, int nbe,
                                 int64_t step, hipStream_t stream, const MlpWeights& W,
                                 const MlpCells2D& C);

int validate_2d(const fdtd_grid* g, const fdtd_profile* p, const fdtd_source* s) {
  if (!g || !p) return fail(FDTD_EINVAL, "null grid or profile");
  if (g->dims != 2) return fail(FDTD_EINVAL, "dims must be 2 here");
  if (g->nx < 8 || g->ny < 8 || g->nx > 32768 || g->ny > 32768)
    return fail(FDTD_EINVAL, "nx, ny must lie in [8, 32768]");
  if (!(g->dx > 0.0) || !std::isfinite(g->dx)) return fail(FDTD_EINVAL, "dx must be > 0");
  if (!(g->courant > 0.0) || g->courant > 1.0 / std::sqrt(2.0))
    return fail(FDTD_EINVAL, "2D Courant number must lie in (0, 1/sqrt(2)], got %g", g->courant);
  if (g->precision != FDTD_FP32 && g->precision != FDTD_FP64)
    return fail(FDTD_EINVAL, "unknown precision %d", g->precision);
  if (g->boundary == FDTD_BC_CPML) {
    if (g->cpml_cells < 1 || 2 * g->cpml_cells + 2 > std::min(g->nx, g->ny))
      return fail(FDTD_EINVAL, "cpml_cells out of range");
    if (!(g->cpml_order > 0) || !(g->cpml_sigma_factor >= 0) || !(g->cpml_kappa_max >= 1) ||
        !(g->cpml_alpha_min >= 0) || !(g->cpml_alpha_max >= 0) ||
        !std::isfinite(g->cpml_order + g->cpml_sigma_factor + g->cpml_kappa_max +
                       g->cpml_alpha_min + g->cpml_alpha_max))
      return fail(FDTD_EINVAL, "bad CPML parameters");
  } else if (g->boundary != FDTD_BC_PEC) {
    return fail(FDTD_EINVAL, "2D boundary must be PEC or CPML");
  }
  if (!is_pow2(p->nv) || p->nv < 8 || p->nv > 32)
    return fail(FDTD_EINVAL, "2D nv must be a power of two in [8, 32], got %d", p->nv);
  if (!(p->te_ev > 0.0) || !(p->vmax_over_vth > 0.0))
    return fail(FDTD_EINVAL, "te_ev and vmax_over_vth must be > 0");
  if (p->nu_model != FDTD_NU_HARD_SPHERE && p->nu_model != FDTD_NU_CONST)
    return fail(FDTD_EINVAL, "unknown nu_model %d", p->nu_model);
  if (p->kinetic != FDTD_KINETIC_LINEAR)
    return fail(FDTD_EINVAL, "2D runs take the linear kinetic model");
  if (p->closure == FDTD_CLOSURE_MLP) {
    if (g->precision != FDTD_FP32) return fail(FDTD_EINVAL, "the learned closure runs in FP32");
    const fdtd_mlp_blob* b = reinterpret_cast<const fdtd_mlp_blob*>(p->mlp);
    if (!b || b->magic != FDTD_MLP_MAGIC || b->version != 1)
      return fail(FDTD_EINVAL, "profile.mlp is not a closure blob");
    for (int i = 0; i < FDTD_CLOSURE_NPARAM; ++i)
      if (!std::isfinite(b->params[i])) return fail(FDTD_EINVAL, "closure parameter %d not finite", i);
    if (!(b->box[1] > b->box[0]) || !(b->box[3] > b->box[2]))
      return fail(FDTD_EINVAL, "closure box is empty");
  } else if (p->closure != FDTD_CLOSURE_KINETIC) {
    return fail(FDTD_EINVAL, "unknown closure %d", p->closure);
  }
  if (!p->ne || !p->nu_mean) return fail(FDTD_EINVAL, "null ne or nu_mean");
  const size_t n = (size_t)g->nx * g->ny;
  for (size_t k = 0; k < n; ++k) {
    if (!(p->ne[k] >= 0.0) || !std::isfinite(p->ne[k]))
      return fail(FDTD_EINVAL, "ne[%zu] must be finite and >= 0", k);
    if (!(p->nu_mean[k] >= 0.0) || !std::isfinite(p->nu_mean[k]))
      return fail(FDTD_EINVAL, "nu_mean[%zu] must be finite and >= 0", k);
  }
  if (s && s->kind != FDTD_SRC_NONE) {
    if (s->kind != FDTD_SRC_LINE_SOFT && s->kind != FDTD_SRC_POINT_SOFT)
      return fail(FDTD_EINVAL, "unknown source kind");
    if (s->i < 1 || s->i > g->nx - 1) return fail(FDTD_EINVAL, "source column out of [1, nx-1]");
    if (s->kind == FDTD_SRC_POINT_SOFT && (s->j < 0 || s->j >= g->ny))
      return fail(FDTD_EINVAL, "source row out of [0, ny)");
    if (!(s->tau_s > 0.0) || !std::isfinite(s->amplitude) || !std::isfinite(s->f_hz) ||
        !std::isfinite(s->t0_s))
      return fail(FDTD_EINVAL, "bad source parameters");
  }
  return FDTD_OK;
}

static Host2D* new_host(const fdtd_grid* g, const fdtd_profile* p, const fdtd_source* s) {
  Host2D* h = new (std::nothrow) Host2D();
  if (!h) return nullptr;
  h->g = *g;
  h->p = *p;
  fdtd_source none{};
  h->s = s ? *s : none;
  h->nx = g->nx;
  h->ny = g->ny;
  h->m = g->boundary == FDTD_BC_CPML ? g->cpml_cells : 0;
  h->nv = p->nv;
  h->half = p->nv * p->nv / 2;
  h->es = g->precision == FDTD_FP64 ? 8 : 4;
  h->dt = g->courant * g->dx / kC0;
  const size_t n = (size_t)g->nx * g->ny;
  h->ne.assign(p->ne, p->ne + n);
  h->nu.assign(p->nu_mean, p->nu_mean + n);
  h->p.ne = h->ne.data();
  h->p.nu_mean = h->nu.data();
  const fdtd_mlp_blob* b = p->closure == FDTD_CLOSURE_MLP
                               ? reinterpret_cast<const fdtd_mlp_blob*>(p->mlp) : nullptr;
  // the network is used only for the kinetic model it was trained on
  h->closure = b && b->dims == 2 && b->nv == p->nv && b->nu_model == p->nu_model &&
               std::fabs(b->te_ev / p->te_ev - 1.0) < 1e-9 &&
               std::fabs(b->vmax_over_vth / p->vmax_over_vth - 1.0) < 1e-9 &&
               std::fabs(b->dt / h->dt - 1.0) < 1e-9;
  double sw = 0.0, swn = 0.0;
  if (h->closure) {
    h->mlp_params.assign(b->params, b->params + FDTD_CLOSURE_NPARAM);
    // single-pole weights: w = vx^2 F0 dv^2 / vth^2 and the nu shape, summed over the grid
    VTable vt = build_vtable(2, p->nv, p->vmax_over_vth, p->te_ev, p->nu_model, h->dt);
    const double vth2 = vt.vth * vt.vth;
    for (int a = 0; a < p->nv; ++a)
      for (int c = 0; c < p->nv; ++c) {
        const double w = vt.v[a] * vt.v[a] * vt.f[a] * vt.f[c] * vt.dv * vt.dv / vth2;
        const double sp = std::sqrt(vt.v[a] * vt.v[a] + vt.v[c] * vt.v[c]);
        sw += w;
        swn += w * (p->nu_model == FDTD_NU_HARD_SPHERE ? sp / vt.mean_speed : 1.0);
      }
  }
  for (size_t k = 0; k < n; ++k) {
    if (!(h->ne[k] > 0)) continue;
    if (h->closure && h->nu[k] > 0) {
      const double wp = std::sqrt(h->ne[k] * kQe * kQe / (kEps0 * kMe));
      const double q1 = 2.0 * (wp * h->dt - b->box[0]) / (b->box[1] - b->box[0]) - 1.0;
      const double q2 = 2.0 * (std::log10(h->nu[k] * h->dt) - b->box[2]) / (b->box[3] - b->box[2]) - 1.0;
      if (q1 >= -1.0 && q1 <= 1.0 && q2 >= -1.0 && q2 <= 1.0) {
        const double nu_eff = h->nu[k] * swn / sw;
        const double wt2 = wp * wp * sw;
        h->mlp_idx.push_back((int32_t)k);
        h->mlp_coef.push_back((float)((2.0 - h->dt * nu_eff) / (2.0 + h->dt * nu_eff)));
        h->mlp_coef.push_back((float)(2.0 * h->dt * h->dt * wt2 / (2.0 + h->dt * nu_eff)));
        h->mlp_coef.push_back((float)q1);
        h->mlp_coef.push_back((float)q2);
        continue;
      }
    }
    h->cell_idx.push_back((int32_t)k);     // kinetic F1 (also the fallback of the closure)
  }
  h->ncell = (int)h->cell_idx.size();
  // about 64 KB of F1 per kinetic work-group
  h->cells_per_block = std::max(4, std::min(256, 65536 / (h->half * h->es)));
  set_grid(h);
  return h;
}

size_t workspace_2d(const fdtd_grid* g, const fdtd_profile* p, int max_probes, int probe_cap) {
  Host2D* h = new_host(g, p, nullptr);
  if (!h) return 0;
  size_t n = layout(h, max_probes, probe_cap);
  delete h;
  return n;
}

Host2D* make_2d(const fdtd_grid* g, const fdtd_profile* p, const fdtd_source* s, int max_probes,
                int probe_cap, size_t* state_bytes, size_t* probe_off) {
  Host2D* h = new_host(g, p, s);
  if (!h) return nullptr;
  layout(h, max_probes, probe_cap);
  *state_bytes = h->state_end;
  *probe_off = h->probe_off;
  return h;
}

int upload_2d(Host2D* h, char* ws, hipStream_t stream, const std::vector<ProbeInfo>& probes,
              size_t probe_off, int probe_cap) {
  return h->es == 8 ? upload<double>(h, ws, stream, probes, probe_off, probe_cap)
                    : upload<float>(h, ws, stream, probes, probe_off, probe_cap);
}

hipError_t launch_step2d(Host2D* h, int64_t step, hipStream_t stream) {
  const void* run = h->ws + h->off_run;
  if (h->es == 8)
    return launch_step2d_t<double>(run, h->half, h->nbk, h->nbh, h->nbe, step, stream, false);
  if (h->C.n > 0)
    return launch_step2d_closure(run, h->half, h->nbk, h->nx, h->ny, h->nbe, step, stream, h->W,
                                 h->C);
  // rows beyond what the 256 MB Infinity Cache keeps between steps are streamed
  const bool streaming = (size_t)h->ncell * h->half * h->es > (size_t(192) << 20);
  return launch_step2d_t<float>(run, h->half, h->nbk, h->nbh, h->nbe, step, stream, streaming);
}

int closure_counts_2d(const Host2D* h, int64_t* nm, int64_t* nk) {
  *nm = (int64_t)h->mlp_idx.size();
  *nk = h->ncell;
  return FDTD_OK;
}

int field_size_2d(const Host2D* h, int field, size_t* n) {
  const size_t nx = h->nx, ny = h->ny;
  switch (field) {
    case FDTD_F_EX: case FDTD_F_JX: *n = (ny + 1) * nx; return FDTD_OK;
    case FDTD_F_EY: case FDTD_F_JY: *n = ny * (nx + 1); return FDTD_OK;
    case FDTD_F_HZ: case FDTD_F_JCX: case FDTD_F_JCY: *n = ny * nx; return FDTD_OK;
    case FDTD_F_DF: *n = (size_t)h->ncell * h->nv * h->nv; return FDTD_OK;
    default: return fail(FDTD_EINVAL, "field %d not defined on a 2D grid", field);
  }
}

int write_2d(Host2D* h, char* ws, int field, const double* src) {
  const int nx = h->nx, ny = h->ny, es = h->es;
  size_t off = 0, cnt = 0;
  double scale = 1.0;
  switch (field) {
    case FDTD_F_EX: off = h->off_Ex; cnt = (size_t)(ny + 1) * nx; break;
    case FDTD_F_EY: off = h->off_Ey; cnt = (size_t)ny * (nx + 1); break;
    case FDTD_F_HZ: off = h->off_Hz; cnt = (size_t)ny * nx; scale = kEta0; break;
    default: return fail(FDTD_EINVAL, "field %d cannot be written on a 2D grid", field);
  }
  std::vector<char> buf(std::max<size_t>(cnt, 1) * es);
  for (size_t k = 0; k < cnt; ++k) {
    if (es == 8) reinterpret_cast<double*>(buf.data())[k] = src[k] * scale;
    else reinterpret_cast<float*>(buf.data())[k] = (float)(src[k] * scale);
  }
  hipError_t e = hipMemcpy(ws + off, buf.data(), cnt * es, hipMemcpyHostToDevice);
  if (e) return hip_fail(e, "write 2D field");
  return FDTD_OK;
}

int read_2d(Host2D* h, char* ws, int field, int64_t, double* dst) {
  const int nx = h->nx, ny = h->ny, es = h->es;
  auto grab = [&](size_t off, size_t cnt, std::vector<double>& out) -> int {
    std::vector<char> buf(std::max<size_t>(cnt, 1) * es);
    if (cnt) {
      hipError_t e = hipMemcpy(buf.data(), ws + off, cnt * es, hipMemcpyDeviceToHost);
      if (e) return hip_fail(e, "copy 2D field");
    }
    out.resize(cnt);
    for (size_t k = 0; k < cnt; ++k)
      out[k] = es == 8 ? reinterpret_cast<double*>(buf.data())[k] : reinterpret_cast<float*>(buf.data())[k];
    return FDTD_OK;
  };
  std::vector<double> v;
  int rc = FDTD_OK;
  const double jscale = kEps0 / h->dt;
  switch (field) {
    case FDTD_F_EX:
      rc = grab(h->off_Ex, (size_t)(ny + 1) * nx, v);
      if (!rc) std::copy(v.begin(), v.end(), dst);
      break;
    case FDTD_F_EY:
      rc = grab(h->off_Ey, (size_t)ny * (nx + 1), v);
      if (!rc) std::copy(v.begin(), v.end(), dst);
      break;
    case FDTD_F_HZ:
      rc = grab(h->off_Hz, (size_t)ny * nx, v);
      if (!rc) for (size_t k = 0; k < v.size(); ++k) dst[k] = v[k] / kEta0;
      break;
    case FDTD_F_JCX:
    case FDTD_F_JCY:
      rc = grab(field == FDTD_F_JCX ? h->off_Jcx : h->off_Jcy, (size_t)ny * nx, v);
      if (!rc) for (size_t k = 0; k < v.size(); ++k) dst[k] = v[k] * jscale;
      break;
    case FDTD_F_JX:
      rc = grab(h->off_Jcx, (size_t)ny * nx, v);
      if (!rc)
        for (int j = 0; j <= ny; ++j)
          for (int i = 0; i < nx; ++i) {
            const double lo = j > 0 ? v[(size_t)(j - 1) * nx + i] : 0.0;
            const double hi = j < ny ? v[(size_t)j * nx + i] : 0.0;
            dst[(size_t)j * nx + i] = 0.5 * (lo + hi) * jscale;
          }
      break;
    case FDTD_F_JY:
      rc = grab(h->off_Jcy, (size_t)ny * nx, v);
      if (!rc)
        for (int j = 0; j < ny; ++j)
          for (int i = 0; i <= nx; ++i) {
            const double lo = i > 0 ? v[(size_t)j * nx + i - 1] : 0.0;
            const double hi = i < nx ? v[(size_t)j * nx + i] : 0.0;
            dst[(size_t)j * (nx + 1) + i] = 0.5 * (lo + hi) * jscale;
          }
      break;
    case FDTD_F_DF: {
      rc = grab(h->off_df, (size_t)h->ncell * h->half, v);
      const int nv = h->nv, hv = nv / 2;
      if (!rc)
        for (int c = 0; c < h->ncell; ++c)
          for (int a = 0; a < nv; ++a)
            for (int bb = 0; bb < hv; ++bb) {
              const double f = v[(size_t)c * h->half + a * hv + bb];
              const int b = hv + bb;
              dst[((size_t)c * nv + a) * nv + b] = f;
              dst[((size_t)c * nv + (nv - 1 - a)) * nv + (nv - 1 - b)] = -f;
            }
      break;
    }
    default:
      return fail(FDTD_EINVAL, "field %d not defined on a 2D grid", field);
  }
  return rc;
}

int check_probe_2d(const Host2D* h, int field, int i, int j) {
  if (field == FDTD_F_EX) {
    if (i < 0 || i >= h->nx || j < 0 || j > h->ny) return fail(FDTD_ERANGE, "Ex probe out of range");
  } else if (field == FDTD_F_EY) {
    if (i < 0 || i > h->nx || j < 0 || j >= h->ny) return fail(FDTD_ERANGE, "Ey probe out of range");
  } else if (field == FDTD_F_HZ) {
    if (i < 0 || i >= h->nx || j < 0 || j >= h->ny) return fail(FDTD_ERANGE, "Hz probe out of range");
  } else {
    return fail(FDTD_EINVAL, "2D probes record Ex, Ey or Hz");
  }
  return FDTD_OK;
}

double probe_scale_2d(const Host2D*, int field) { return field == FDTD_F_HZ ? 1.0 / kEta0 : 1.0; }

int set_tiling_2d(Host2D* h, char* ws, hipStream_t stream, int tile, int cells_per_group) {
  const int cpb = cells_per_group ? cells_per_group : tile;
  if (cpb) {
    if (cpb < 1 || cpb > 4096) return fail(FDTD_EINVAL, "cells per group must lie in [1, 4096]");
    h->cells_per_block = cpb;
    set_grid(h);
    // patch the descriptor's launch fields
    const size_t off = h->es == 8 ? offsetof(Run2D<double>, cells_per_block)
                                  : offsetof(Run2D<float>, cells_per_block);
    int32_t v[2] = {h->cells_per_block, h->nbk};
    hipError_t e = hipMemcpyAsync(ws + h->off_run + off, v, sizeof v, hipMemcpyHostToDevice, stream);
    if (!e) e = hipStreamSynchronize(stream);
    if (e) return hip_fail(e, "update 2D tiling");
  }
  return FDTD_OK;
}

void destroy_2d(Host2D* h) { delete h; }

}  // namespace fdtdp
