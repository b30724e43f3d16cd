// common.h -- device-side types shared by the kernels of the kinetic-FDTD library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdtdp {

constexpr int kMaxProbes = 16;
constexpr int kBlock = 256;        // threads per work-group of the step kernels
constexpr int kMaxTile1D = 256;    // nodes per 1D tile: one node per thread

// 16-byte vector of the storage type: 4 floats or 2 doubles per lane per chunk.
template <class T> struct Vec;
template <> struct Vec<float> { using type = float4; static constexpr int n = 4; };
template <> struct Vec<double> { using type = double2; static constexpr int n = 2; };

template <class V> __device__ __forceinline__ auto& lane_at(V& v, int k) {
  return reinterpret_cast<typename std::remove_reference<decltype(v.x)>::type*>(&v)[k];
}

// Reciprocal used by the Crank-Nicolson factor 1/(2 + dt nu): the hardware estimate in
// FP32 (the increment it scales is small next to F1 itself), exact division in FP64.
__device__ __forceinline__ float cn_recip(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double cn_recip(double d) { return 1.0 / d; }

// Leap-frog updates, written once so that every thread that recomputes a halo value
// produces the owner's bits exactly.
template <class T> __device__ __forceinline__ T h_update(T h, T s, T e_hi, T e_lo) {
  return fma(s, e_hi - e_lo, h);
}
template <class T> __device__ __forceinline__ T e_update(T e, T s, T h_hi, T h_lo, T j) {
  return fma(s, h_hi - h_lo, e) - j;
}

// Gaussian-modulated sine of the source, evaluated in FP64.
__device__ __forceinline__ double source_wave(double t, double amp, double w, double tau,
                                              double t0) {
  double x = (t - t0) / tau;
  return amp * sin(w * (t - t0)) * exp(-x * x);
}

struct Tile1D {
  int32_t run, node0, node1, cell0, cell1;
};

// One 1D run as the step kernel sees it.  Ping-pong field buffers: at step n the
// current E/H live in buffer (n & 1) and the kernel writes buffer (n & 1) ^ 1.
template <class T> struct Run1D {
  T* E[2];
  T* H[2];
  T* J;            // [nx+1] normalised current dt/eps0 * J at the last half step
  T* df;           // [ncell][half] F1 on v > 0 bins
  const int32_t* cell_node;
  const T* tau;    // [ncell] dt * nu_mean
  const T* dens;   // [ncell] electron density
  const T* s_bin;  // [half] collision-frequency shape
  const T* b_bin;  // [half] 2 dt (e/m) dF0/dv (per unit density)
  const double* w_bin;  // [half] moment weight (dt/eps0)(-2 e dv) v_j
  int32_t nx, ncell, half, bc;
  T S, q;
  int32_t src_node;
  double src_amp, src_w, src_tau, src_t0, dt;
  int64_t step_limit;
  int32_t nprobe, probe_cap;
  int32_t probe_node[kMaxProbes];
  int32_t probe_field[kMaxProbes];
  T* probe_buf;    // [nprobe][probe_cap]
};

}  // namespace fdtdp
