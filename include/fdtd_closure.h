/*
 * fdtd_closure.h -- C ABI of the learned closure of the kinetic-FDTD library.
 *
 * The kinetic model of arXiv 2211.05647 (section 5.2: the F1 equation with elastic
 * collisions nu(v) = N s v, and the current J = -e \int v F d^3v) gives every plasma cell a
 * current that, per velocity bin, obeys a Crank-Nicolson recursion driven by E.  The
 * closure replaces the sum over bins by a single pole (the bins' weighted mean collision
 * rate) and a small network that corrects the drive from the recent field history:
 *
 *     Jn^{n+1/2} = alpha Jn^{n-1/2} + beta (E^n + s y),      Jn = (dt / eps0) J,
 *     y = MLP(E^n/s, ..., E^{n-15}/s, p1, p2),   s = max |E^{n-k}| (k < 16, floor 1e-30),
 *
 * p1 = omega_p dt and p2 = log10(nu_mean dt), each mapped linearly onto [-1, 1] over the
 * training box.  Network: 18 -> 128 (ReLU) -> 128 (ReLU) -> 1, parameters in
 * the order W1[128][18], b1[128], W2[128][128], b2[128], w3[128], b3 (19073 FP32 values).
 * GEMM operands are bfloat16 (round to nearest even), accumulation FP32, master weights FP32.
 * With y = 0 the recursion is exactly the Drude (single-pole) current.
 *
 * Conventions as in fdtd_plasma.h: int return codes (enum fdtd_status), host pointers are
 * host memory, pointers named *_dev are HIP device memory owned by the caller, work is
 * enqueued on the handle's stream.  Calls that return host data synchronise it.
 */
#ifndef FDTD_CLOSURE_H
#define FDTD_CLOSURE_H

#include <stddef.h>
#include <stdint.h>

#include "fdtd_plasma.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdtd_closure fdtd_closure;

#define FDTD_CLOSURE_NPARAM 19073
#define FDTD_CLOSURE_NIN 18
#define FDTD_MLP_MAGIC 0x4d4c5043u

/* A trained closure as fdtd_profile.mlp expects it (2D runs with closure = FDTD_CLOSURE_MLP).
 * The run uses the network only if dims, nv, nu_model, te_ev, vmax_over_vth and dt match
 * the kinetic model it was trained on (dt to 1e-9 relative); a plasma cell uses it only if
 * its (omega_p dt, log10(nu_mean dt)) lies inside box, every other cell keeps the kinetic
 * F1 step (the fallback).  box = (p1 lo, p1 hi, p2 lo, p2 hi). */
typedef struct {
  uint32_t magic;        /* FDTD_MLP_MAGIC */
  uint32_t version;      /* 1 */
  int32_t dims, nv, nu_model, reserved;
  double te_ev, vmax_over_vth, dt;
  double box[4];
  float params[FDTD_CLOSURE_NPARAM];
} fdtd_mlp_blob;

/* Workspace for a trainer/evaluator handling up to max_rows feature rows per call and
 * max_series replay series. */
int fdtd_closure_workspace_size(int32_t max_rows, int32_t max_series, size_t *bytes);
/* Create on dev (workspace semantics as fdtd_device; max_probes ignored). */
int fdtd_closure_create(const fdtd_device *dev, int32_t max_rows, int32_t max_series,
                        fdtd_closure **out);
/* Set the FP32 master parameters (host, FDTD_CLOSURE_NPARAM values, all finite); resets
 * the Adam moments.  Get copies them back. */
int fdtd_closure_set_params(fdtd_closure *c, const float *params, size_t n);
int fdtd_closure_get_params(fdtd_closure *c, float *params, size_t n);
/* y_dev[i] = MLP(x_dev[i][0..17]) for n rows (FP32 in, FP32 out, device memory). */
int fdtd_closure_forward(fdtd_closure *c, const float *x_dev, int32_t n, float *y_dev);
/* Mean squared error of the n rows against t_dev and its gradient (kept on the device for
 * fdtd_closure_adam); optional host copies (NULL to skip). */
int fdtd_closure_grad(fdtd_closure *c, const float *x_dev, const float *t_dev, int32_t n,
                      float *grad_host, float *loss_host);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the gradient fdtd_closure_grad
 * computes, with no handle and no allocation.  params_dev: the FDTD_CLOSURE_NPARAM FP32
 * parameters in device memory (the layout of fdtd_closure_get_params); x_dev [n][18] and
 * t_dev [n]: the rows and targets (device); grad_dev [FDTD_CLOSURE_NPARAM] and loss_dev [1]
 * (device) receive the gradient of the mean squared error and the loss.  The kernels'
 * scratch (bf16 weight copies, per-block partial gradients) is one fixed device array
 * inside the library, about 9.9 MB on each GPU it runs on, held until the process ends;
 * hence n is limited to FDTD_CLOSURE_STATIC_MAX_ROWS (FDTD_ERANGE above it).  Work goes on
 * hip_stream (NULL = the null stream) and nothing synchronises; the results are bitwise
 * those of fdtd_closure_grad with the same parameters.  Every call on one GPU uses that
 * GPU's array, so calls that overlap on one GPU race.  Errors: FDTD_EINVAL for a null
 * pointer or a bad device, FDTD_EDEVICE for a HIP error. */
#define FDTD_CLOSURE_STATIC_MAX_ROWS 8192
int fdtd_closure_grad_static(int32_t device, void *hip_stream, const float *params_dev,
                             const float *x_dev, const float *t_dev, int32_t n,
                             float *grad_dev, float *loss_dev);
/* One Adam step (Kingma & Ba) on the master weights with the last gradient. */
int fdtd_closure_adam(fdtd_closure *c, float lr, float beta1, float beta2, float eps);
/* grad + Adam(lr, 0.9, 0.999, 1e-8); loss_host (optional, synchronises). */
int fdtd_closure_train_step(fdtd_closure *c, const float *x_dev, const float *t_dev, int32_t n,
                            float lr, float *loss_host);
/* Single-pole parameters (alpha, beta) of a dims-V kinetic cell (section 5.2 F1 model on
 * the nv^dims Cartesian grid) for density ne, mean collision rate nu_mean and step dt. */
int fdtd_closure_single_pole(int32_t dims, int32_t nv, double vmax_over_vth, double te_ev,
                             int32_t nu_model, double ne, double nu_mean, double dt,
                             double *alpha, double *beta);
/* Training currents: nseries isolated 2V kinetic cells (32 x 32 bins) driven along x by
 * the recorded fields E_dev[s * e_series_stride + n * e_stride]; writes the normalised
 * current J_dev[s * j_series_stride + n] = (dt/eps0) Jx^{n+1/2}.  ne / nu_mean: host arrays
 * of nseries values. */
int fdtd_closure_replay2v(fdtd_closure *c, const float *E_dev, int64_t e_stride,
                          int64_t e_series_stride, int32_t nseries, int64_t nsteps,
                          const double *ne, const double *nu_mean, double te_ev,
                          double vmax_over_vth, int32_t nu_model, double dt, float *J_dev,
                          int64_t j_series_stride);
/* Training pairs: for idx[p] = (series << 32) | n build the feature row X_dev[p][18] and the
 * target T_dev[p] = ((J^{n+1/2} - alpha J^{n-1/2}) / beta - E^n) / s.  series4: host
 * [nseries][4] = (alpha, beta, p1 scaled, p2 scaled).  idx: host, npairs <= max_rows. */
int fdtd_closure_make_pairs(fdtd_closure *c, const float *E_dev, int64_t e_stride,
                            int64_t e_series_stride, const float *J_dev, int64_t j_series_stride,
                            int32_t nseries, const float *series4, const int64_t *idx,
                            int32_t npairs, float *X_dev, float *T_dev);
void fdtd_closure_destroy(fdtd_closure *c);

/* Plasma cells of a 2D run served by the closure and by the kinetic fallback. */
int fdtd_plasma_closure_counts(fdtd_plasma *h, int64_t *closure_cells, int64_t *kinetic_cells);

/* Device pointer and geometry of a batch run's tap buffer ([ntap][cap][2] FP32:
 * E^n in V/m, normalised (dt/eps0) J^{n+1/2}), for feeding fdtd_closure_replay2v and
 * fdtd_closure_make_pairs without a host round trip. */
int fdtd_plasma_tap_buffer(fdtd_plasma *h, int32_t run, const float **dev, int64_t *cap,
                           int32_t *ntap);

#ifdef __cplusplus
}
#endif
#endif /* FDTD_CLOSURE_H */
