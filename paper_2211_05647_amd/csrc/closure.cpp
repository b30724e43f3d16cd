// closure.cpp -- host side of the learned-closure entry points (fdtd_closure_*):
// parameter upload/download, inference on device rows, one training step (forward,
// backward, deterministic gradient reduction, Adam), the isolated 2V replay cells that
// turn recorded field histories into kinetic currents, and training-pair assembly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/fdtd_closure.h"
#include "host_internal.h"
#include "mlp_common.h"

using namespace fdtdp;

namespace fdtdp {
hipError_t mlp_launch_rows(const MlpWeights& W, const float* X, int n, float* Y, hipStream_t st);
hipError_t mlp_launch_grad(const MlpWeights& W, const float* X, const float* T, int n, float* P,
                           float* lossp, float* G, float* loss, hipStream_t st);
hipError_t mlp_launch_adam(float* master, float* m, float* v, const float* G, float lr, float b1,
                           float b2, float eps, float c1, float c2, hipStream_t st);
hipError_t mlp_launch_pack(const float* master, const MlpWeights& W, hipStream_t st);
hipError_t mlp_launch_replay2v(const float* E, int64_t e_stride, int64_t e_series_stride,
                               int nseries, int64_t nsteps, const ReplayCell* cells,
                               const float* s_bin, const float* bx_bin, const double* wx_bin,
                               float* J, int64_t j_series_stride, hipStream_t st);
hipError_t mlp_launch_pairs(const float* E, int64_t e_stride, int64_t e_series_stride,
                            const float* J, int64_t j_series_stride, const PairSeries* ser,
                            const int64_t* idx, int npairs, float* X, float* T, hipStream_t st);
}  // namespace fdtdp

struct fdtd_closure {
  int device = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  bool owns = false;
  int max_rows = 0, max_series = 0;
  float *master = nullptr, *m = nullptr, *v = nullptr, *G = nullptr, *P = nullptr, *lossp = nullptr,
        *loss = nullptr;
  MlpWeights W{};
  ReplayCell* cells = nullptr;
  PairSeries* series = nullptr;
  int64_t* idx = nullptr;
  float *s_bin = nullptr, *bx_bin = nullptr;
  double* wx_bin = nullptr;
  int64_t adam_t = 0;
  bool have_grad = false;
};

namespace {

struct ClosureLayout {
  size_t master, m, v, G, P, lossp, loss, W1, W2, W2T, W2P, b1, b2, w3q, b3, cells, series, idx, s, bx, wx,
      total;
};

ClosureLayout closure_layout(int max_rows, int max_series) {
  Carver cv;
  ClosureLayout L;
  const int nb = (max_rows + 63) / 64;
  L.master = cv.take(kNParam * 4);
  L.m = cv.take(kNParam * 4);
  L.v = cv.take(kNParam * 4);
  L.G = cv.take(kNParam * 4);
  L.P = cv.take((size_t)nb * kNParam * 4);
  L.lossp = cv.take((size_t)nb * 4);
  L.loss = cv.take(4);
  L.W1 = cv.take(kNH * kK1P * 2);
  L.W2 = cv.take(kNH * kK2P * 2);
  L.W2T = cv.take(kNH * kK2P * 2);
  L.W2P = cv.take(kNH * kK2P * 2);
  L.b1 = cv.take(kNH * 4);
  L.b2 = cv.take(kNH * 4);
  L.w3q = cv.take(kNH * 4);
  L.b3 = cv.take(4);
  L.cells = cv.take((size_t)max_series * sizeof(ReplayCell));
  L.series = cv.take((size_t)max_series * sizeof(PairSeries));
  L.idx = cv.take((size_t)max_rows * 8);
  L.s = cv.take(kReplayHalf * 4);
  L.bx = cv.take(kReplayHalf * 4);
  L.wx = cv.take(kReplayHalf * 8);
  L.total = cv.size() + 256;
  return L;
}

int check_rows(const fdtd_closure* c, int n) {
  if (!c) return fail(FDTD_EINVAL, "null closure");
  if (n < 1 || n > c->max_rows) return fail(FDTD_ERANGE, "row count %d outside [1, %d]", n, c->max_rows);
  return FDTD_OK;
}

}  // namespace

extern "C" {

int fdtd_closure_workspace_size(int32_t max_rows, int32_t max_series, size_t* bytes) {
  if (!bytes || max_rows < 64 || max_rows > (1 << 24) || max_series < 1 || max_series > (1 << 20))
    return fail(FDTD_EINVAL, "max_rows must lie in [64, 2^24] and max_series in [1, 2^20]");
  *bytes = closure_layout(max_rows, max_series).total;
  return FDTD_OK;
}

int fdtd_closure_create(const fdtd_device* dev, int32_t max_rows, int32_t max_series,
                        fdtd_closure** out) {
  size_t need = 0;
  int rc = fdtd_closure_workspace_size(max_rows, max_series, &need);
  if (rc) return rc;
  if (!dev || !out) return fail(FDTD_EINVAL, "null argument");
  hipError_t e = hipSetDevice(dev->device);
  if (e) return hip_fail(e, "hipSetDevice");
  fdtd_closure* c = new (std::nothrow) fdtd_closure();
  if (!c) return fail(FDTD_ENOMEM, "host allocation");
  c->device = dev->device;
  c->stream = reinterpret_cast<hipStream_t>(dev->hip_stream);
  c->max_rows = max_rows;
  c->max_series = max_series;
  if (dev->workspace) {
    if (dev->workspace_bytes < need) {
      delete c;
      return fail(FDTD_ENOMEM, "closure workspace has %zu bytes, need %zu", dev->workspace_bytes, need);
    }
    c->ws = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(dev->workspace) + 255) & ~uintptr_t(255));
  } else {
    void* p = nullptr;
    e = hipMalloc(&p, need);
    if (e) {
      delete c;
      return fail(FDTD_ENOMEM, "hipMalloc(%zu)", need);
    }
    c->ws = reinterpret_cast<char*>(p);
    c->owns = true;
  }
  const ClosureLayout L = closure_layout(max_rows, max_series);
  char* b = c->ws;
  c->master = reinterpret_cast<float*>(b + L.master);
  c->m = reinterpret_cast<float*>(b + L.m);
  c->v = reinterpret_cast<float*>(b + L.v);
  c->G = reinterpret_cast<float*>(b + L.G);
  c->P = reinterpret_cast<float*>(b + L.P);
  c->lossp = reinterpret_cast<float*>(b + L.lossp);
  c->loss = reinterpret_cast<float*>(b + L.loss);
  c->W.W1 = reinterpret_cast<uint16_t*>(b + L.W1);
  c->W.W2 = reinterpret_cast<uint16_t*>(b + L.W2);
  c->W.W2T = reinterpret_cast<uint16_t*>(b + L.W2T);
  c->W.W2P = reinterpret_cast<uint16_t*>(b + L.W2P);
  c->W.b1 = reinterpret_cast<float*>(b + L.b1);
  c->W.b2 = reinterpret_cast<float*>(b + L.b2);
  c->W.w3q = reinterpret_cast<float*>(b + L.w3q);
  c->W.b3 = reinterpret_cast<float*>(b + L.b3);
  c->cells = reinterpret_cast<ReplayCell*>(b + L.cells);
  c->series = reinterpret_cast<PairSeries*>(b + L.series);
  c->idx = reinterpret_cast<int64_t*>(b + L.idx);
  c->s_bin = reinterpret_cast<float*>(b + L.s);
  c->bx_bin = reinterpret_cast<float*>(b + L.bx);
  c->wx_bin = reinterpret_cast<double*>(b + L.wx);
  e = hipMemsetAsync(c->ws, 0, L.total - 256, c->stream);
  if (!e) e = hipStreamSynchronize(c->stream);
  if (e) {
    if (c->owns) hipFree(c->ws);
    delete c;
    return hip_fail(e, "clear closure workspace");
  }
  *out = c;
  return FDTD_OK;
}

int fdtd_closure_set_params(fdtd_closure* c, const float* params, size_t n) {
  if (!c || !params) return fail(FDTD_EINVAL, "null argument");
  if (n != (size_t)kNParam) return fail(FDTD_ERANGE, "expected %d parameters", kNParam);
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(params[i])) return fail(FDTD_EINVAL, "parameter %zu is not finite", i);
  hipError_t e = hipMemcpyAsync(c->master, params, n * 4, hipMemcpyHostToDevice, c->stream);
  if (!e) e = hipMemsetAsync(c->m, 0, n * 4, c->stream);
  if (!e) e = hipMemsetAsync(c->v, 0, n * 4, c->stream);
  if (!e) e = mlp_launch_pack(c->master, c->W, c->stream);
  if (!e) e = hipStreamSynchronize(c->stream);
  if (e) return hip_fail(e, "set closure parameters");
  c->adam_t = 0;
  c->have_grad = false;
  return FDTD_OK;
}

int fdtd_closure_get_params(fdtd_closure* c, float* params, size_t n) {
  if (!c || !params) return fail(FDTD_EINVAL, "null argument");
  if (n < (size_t)kNParam) return fail(FDTD_ERANGE, "destination holds %zu values, need %d", n, kNParam);
  hipError_t e = hipStreamSynchronize(c->stream);
  if (!e) e = hipMemcpy(params, c->master, kNParam * 4, hipMemcpyDeviceToHost);
  if (e) return hip_fail(e, "get closure parameters");
  return FDTD_OK;
}

int fdtd_closure_forward(fdtd_closure* c, const float* x_dev, int32_t n, float* y_dev) {
  int rc = check_rows(c, n);
  if (rc) return rc;
  if (!x_dev || !y_dev) return fail(FDTD_EINVAL, "null device pointer");
  hipError_t e = mlp_launch_rows(c->W, x_dev, n, y_dev, c->stream);
  return e ? hip_fail(e, "closure forward") : FDTD_OK;
}

int fdtd_closure_grad(fdtd_closure* c, const float* x_dev, const float* t_dev, int32_t n,
                      float* grad_host, float* loss_host) {
  int rc = check_rows(c, n);
  if (rc) return rc;
  if (!x_dev || !t_dev) return fail(FDTD_EINVAL, "null device pointer");
  hipError_t e = mlp_launch_grad(c->W, x_dev, t_dev, n, c->P, c->lossp, c->G, c->loss, c->stream);
  if (e) return hip_fail(e, "closure gradient");
  c->have_grad = true;
  if (grad_host || loss_host) {
    e = hipStreamSynchronize(c->stream);
    if (!e && grad_host) e = hipMemcpy(grad_host, c->G, kNParam * 4, hipMemcpyDeviceToHost);
    if (!e && loss_host) e = hipMemcpy(loss_host, c->loss, 4, hipMemcpyDeviceToHost);
    if (e) return hip_fail(e, "copy gradient");
  }
  return FDTD_OK;
}

int fdtd_closure_adam(fdtd_closure* c, float lr, float beta1, float beta2, float eps) {
  if (!c) return fail(FDTD_EINVAL, "null closure");
  if (!c->have_grad) return fail(FDTD_ESTATE, "no gradient computed yet");
  if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return fail(FDTD_EINVAL, "bad Adam hyper-parameters");
  c->adam_t += 1;
  const float c1 = (float)(1.0 - std::pow((double)beta1, (double)c->adam_t));
  const float c2 = (float)(1.0 - std::pow((double)beta2, (double)c->adam_t));
  hipError_t e = mlp_launch_adam(c->master, c->m, c->v, c->G, lr, beta1, beta2, eps, c1, c2, c->stream);
  if (!e) e = mlp_launch_pack(c->master, c->W, c->stream);
  return e ? hip_fail(e, "closure Adam step") : FDTD_OK;
}

int fdtd_closure_train_step(fdtd_closure* c, const float* x_dev, const float* t_dev, int32_t n,
                            float lr, float* loss_host) {
  int rc = fdtd_closure_grad(c, x_dev, t_dev, n, nullptr, nullptr);
  if (rc) return rc;
  rc = fdtd_closure_adam(c, lr, 0.9f, 0.999f, 1e-8f);
  if (rc) return rc;
  if (loss_host) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (!e) e = hipMemcpy(loss_host, c->loss, 4, hipMemcpyDeviceToHost);
    if (e) return hip_fail(e, "copy loss");
  }
  return FDTD_OK;
}

int fdtd_closure_single_pole(int32_t dims, int32_t nv, double vmax_over_vth, double te_ev,
                             int32_t nu_model, double ne, double nu_mean, double dt,
                             double* alpha, double* beta) {
  if (!alpha || !beta || (dims != 1 && dims != 2) || !is_pow2(nv) || nv < 8 || !(te_ev > 0) ||
      !(vmax_over_vth > 0) || !(dt > 0) || !(ne >= 0) || !(nu_mean >= 0))
    return fail(FDTD_EINVAL, "bad single-pole arguments");
  VTable vt = build_vtable(dims, nv, vmax_over_vth, te_ev, nu_model, dt);
  // weights of the drive component (x): w = vx^2 F0 dv^d / vth^2; nu shape per bin
  double sw = 0.0, swn = 0.0;
  const double vth2 = vt.vth * vt.vth;
  if (dims == 1) {
    for (int j = 0; j < nv; ++j) {
      const double w = vt.v[j] * vt.v[j] * vt.f[j] * vt.dv / vth2;
      const double s = nu_model == FDTD_NU_HARD_SPHERE ? std::fabs(vt.v[j]) / vt.mean_speed : 1.0;
      sw += w;
      swn += w * s;
    }
  } else {
    for (int a = 0; a < nv; ++a)
      for (int b = 0; b < nv; ++b) {
        const double w = vt.v[a] * vt.v[a] * vt.f[a] * vt.f[b] * vt.dv * vt.dv / vth2;
        const double sp = std::sqrt(vt.v[a] * vt.v[a] + vt.v[b] * vt.v[b]);
        const double s = nu_model == FDTD_NU_HARD_SPHERE ? sp / vt.mean_speed : 1.0;
        sw += w;
        swn += w * s;
      }
  }
  const double nu_eff = nu_mean * swn / sw;
  const double wp2 = ne * kQe * kQe / (kEps0 * kMe) * sw;
  *alpha = (2.0 - dt * nu_eff) / (2.0 + dt * nu_eff);
  *beta = 2.0 * dt * dt * wp2 / (2.0 + dt * nu_eff);
  return FDTD_OK;
}

int fdtd_closure_replay2v(fdtd_closure* c, const float* E_dev, int64_t e_stride,
                          int64_t e_series_stride, int32_t nseries, int64_t nsteps,
                          const double* ne, const double* nu_mean, double te_ev,
                          double vmax_over_vth, int32_t nu_model, double dt, float* J_dev,
                          int64_t j_series_stride) {
  if (!c || !E_dev || !J_dev || !ne || !nu_mean) return fail(FDTD_EINVAL, "null argument");
  if (nseries < 1 || nseries > c->max_series) return fail(FDTD_ERANGE, "nseries out of range");
  if (nsteps < 1 || e_stride < 1 || e_series_stride < 0 || j_series_stride < nsteps)
    return fail(FDTD_EINVAL, "bad replay strides");
  if (!(te_ev > 0) || !(vmax_over_vth > 0) || !(dt > 0) ||
      (nu_model != FDTD_NU_HARD_SPHERE && nu_model != FDTD_NU_CONST))
    return fail(FDTD_EINVAL, "bad replay plasma parameters");
  const int nv = kReplayNv, hv = nv / 2;
  VTable vt = build_vtable(2, nv, vmax_over_vth, te_ev, nu_model, dt);
  std::vector<float> s(kReplayHalf), bx(kReplayHalf);
  std::vector<double> wx(kReplayHalf);
  const double vth2 = vt.vth * vt.vth;
  for (int a = 0; a < nv; ++a)
    for (int bb = 0; bb < hv; ++bb) {
      const int q = a * hv + bb, b = hv + bb;
      const double vx = vt.v[a], vy = vt.v[b], f2 = vt.f[a] * vt.f[b];
      const double sp = std::sqrt(vx * vx + vy * vy);
      s[q] = (float)(nu_model == FDTD_NU_HARD_SPHERE ? sp / vt.mean_speed : 1.0);
      bx[q] = (float)(2.0 * dt * (kQe / kMe) * (-vx * f2 / vth2));
      wx[q] = (dt / kEps0) * (-2.0 * kQe * vt.dv * vt.dv) * vx;
    }
  std::vector<ReplayCell> cells(nseries);
  for (int i = 0; i < nseries; ++i) {
    if (!(ne[i] >= 0) || !(nu_mean[i] >= 0)) return fail(FDTD_EINVAL, "bad series %d", i);
    cells[i].tau = (float)(dt * nu_mean[i]);
    cells[i].dens = (float)ne[i];
  }
  hipError_t e = hipMemcpyAsync(c->s_bin, s.data(), s.size() * 4, hipMemcpyHostToDevice, c->stream);
  if (!e) e = hipMemcpyAsync(c->bx_bin, bx.data(), bx.size() * 4, hipMemcpyHostToDevice, c->stream);
  if (!e) e = hipMemcpyAsync(c->wx_bin, wx.data(), wx.size() * 8, hipMemcpyHostToDevice, c->stream);
  if (!e) e = hipMemcpyAsync(c->cells, cells.data(), cells.size() * sizeof(ReplayCell),
                             hipMemcpyHostToDevice, c->stream);
  if (!e) e = mlp_launch_replay2v(E_dev, e_stride, e_series_stride, nseries, nsteps, c->cells,
                                  c->s_bin, c->bx_bin, c->wx_bin, J_dev, j_series_stride, c->stream);
  if (!e) e = hipStreamSynchronize(c->stream);   // host staging buffers go out of scope
  return e ? hip_fail(e, "replay") : FDTD_OK;
}

int fdtd_closure_make_pairs(fdtd_closure* c, const float* E_dev, int64_t e_stride,
                            int64_t e_series_stride, const float* J_dev, int64_t j_series_stride,
                            int32_t nseries, const float* series4, const int64_t* idx,
                            int32_t npairs, float* X_dev, float* T_dev) {
  int rc = check_rows(c, npairs);
  if (rc) return rc;
  if (!E_dev || !J_dev || !series4 || !idx || !X_dev || !T_dev) return fail(FDTD_EINVAL, "null argument");
  if (nseries < 1 || nseries > c->max_series) return fail(FDTD_ERANGE, "nseries out of range");
  for (int p = 0; p < npairs; ++p) {
    const int64_t si = idx[p] >> 32, n = idx[p] & 0xFFFFFFFFLL;
    if (si < 0 || si >= nseries || n < 0 || n >= j_series_stride)
      return fail(FDTD_ERANGE, "pair %d indexes outside the series", p);
  }
  for (int i = 0; i < nseries; ++i)
    if (!(series4[4 * i + 1] != 0.0f)) return fail(FDTD_EINVAL, "series %d has beta = 0", i);
  hipError_t e = hipMemcpyAsync(c->series, series4, (size_t)nseries * sizeof(PairSeries),
                                hipMemcpyHostToDevice, c->stream);
  if (!e) e = hipMemcpyAsync(c->idx, idx, (size_t)npairs * 8, hipMemcpyHostToDevice, c->stream);
  if (!e) e = mlp_launch_pairs(E_dev, e_stride, e_series_stride, J_dev, j_series_stride, c->series,
                               c->idx, npairs, X_dev, T_dev, c->stream);
  if (!e) e = hipStreamSynchronize(c->stream);
  return e ? hip_fail(e, "make pairs") : FDTD_OK;
}

void fdtd_closure_destroy(fdtd_closure* c) {
  if (!c) return;
  hipSetDevice(c->device);
  if (c->stream) hipStreamSynchronize(c->stream);
  if (c->owns) hipFree(c->ws);
  delete c;
}

}  // extern "C"
