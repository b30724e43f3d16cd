// yee2d.h -- per-point TEz Yee updates with the CPML (arXiv 2211.05647, section 2, eq.
// (2)-(5) and the CPML auxiliary fields of eq. (4)), shared by the 2D step kernels and the
// closure kernel, which runs the H half-step beside the network.
//
// Work is mapped in row segments: a segment is `width` consecutive x points of one row,
// so the row and column of a point come from one wave-uniform division per segment.
#pragma once
#include "common.h"

namespace fdtdp {

template <class T>
__device__ __forceinline__ void record_probe(const Run2D<T>& R, int field, int i, int j, T val,
                                             int64_t step) {
  for (int p = 0; p < R.nprobe; ++p)
    if (R.probe_field[p] == field && R.probe_i[p] == i && R.probe_j[p] == j)
      R.probe_buf[(size_t)p * R.probe_cap + (size_t)(step % R.probe_cap)] = val;
}

// Hz^{n+1/2} at (i+1/2, j+1/2), 0 <= i < nx, 0 <= j < ny, with the H-side psi strips.
template <class T>
__device__ __forceinline__ void h2d_point(const Run2D<T>& R, int i, int j, int64_t step) {
  const int nx = R.nx, ny = R.ny, m = R.m;
  const size_t q = (size_t)j * nx + i;
  const T dEx = R.Ex[q + nx] - R.Ex[q];
  const T dEy = R.Ey[(size_t)j * (nx + 1) + i + 1] - R.Ey[(size_t)j * (nx + 1) + i];
  T acc = dEx * R.rkhy[j] - dEy * R.rkhx[i];
  if (m > 0) {
    if (i < m || i >= nx - m) {
      const int sx = i < m ? i : i - (nx - 2 * m);
      T* p = R.psi_hzx + (size_t)j * (2 * m) + sx;
      const T v = fma(R.bhx[i], *p, R.ahx[i] * dEy);
      *p = v;
      acc -= v;
    }
    if (j < m || j >= ny - m) {
      const int sy = j < m ? j : j - (ny - 2 * m);
      T* p = R.psi_hzy + (size_t)sy * nx + i;
      const T v = fma(R.bhy[j], *p, R.ahy[j] * dEx);
      *p = v;
      acc += v;
    }
  }
  const T hz = fma(R.S, acc, R.Hz[q]);
  R.Hz[q] = hz;
  if (R.nprobe) record_probe(R, 6 /* FDTD_F_HZ */, i, j, hz, step);
}

// E^{n+1} at the point (i, j) of the (nx+1) x (ny+1) node lattice: Ex at (i+1/2, j) when
// i < nx, Ey at (i, j+1/2) when j < ny.  Tangential E on the outer walls stays zero (PEC
// backing of the CPML); the edge current is the mean of the two adjacent cell currents.
template <class T>
__device__ __forceinline__ void e2d_point(const Run2D<T>& R, int i, int j, int64_t step) {
  const int nx = R.nx, ny = R.ny, m = R.m;
  if (i < nx && j >= 1 && j <= ny - 1) {
    const size_t k = (size_t)j * nx + i;
    const T dHz = R.Hz[k] - R.Hz[k - nx];
    T acc = dHz * R.rkey[j];
    if (m > 0 && (j < m || j > ny - m)) {
      const int sy = j < m ? j : j - ny + 2 * m - 1;
      T* p = R.psi_exy + (size_t)sy * nx + i;
      const T v = fma(R.bey[j], *p, R.aey[j] * dHz);
      *p = v;
      acc += v;
    }
    const T jx = T(0.5) * (R.Jcx[k - nx] + R.Jcx[k]);
    const T ex = fma(R.S, acc, R.Ex[k]) - jx;
    R.Ex[k] = ex;
    if (R.nprobe) record_probe(R, 4 /* FDTD_F_EX */, i, j, ex, step);
  }
  if (j < ny && i >= 1 && i <= nx - 1) {
    const size_t k = (size_t)j * (nx + 1) + i;
    const size_t kc = (size_t)j * nx + i;
    const T dHz = R.Hz[kc] - R.Hz[kc - 1];
    T acc = dHz * R.rkex[i];
    if (m > 0 && (i < m || i > nx - m)) {
      const int sx = i < m ? i : i - nx + 2 * m - 1;
      T* p = R.psi_eyx + (size_t)j * (2 * m) + sx;
      const T v = fma(R.bex[i], *p, R.aex[i] * dHz);
      *p = v;
      acc += v;
    }
    const T jy = T(0.5) * (R.Jcy[kc - 1] + R.Jcy[kc]);
    T ey = fma(-R.S, acc, R.Ey[k]) - jy;
    if (R.src_kind != 0 && i == R.src_i && (R.src_kind == 1 || j == R.src_j))
      ey += (T)source_wave((double)(step + 1) * R.dt, R.src_amp, R.src_w, R.src_tau, R.src_t0);
    R.Ey[k] = ey;
    if (R.nprobe) record_probe(R, 5 /* FDTD_F_EY */, i, j, ey, step);
  }
}

// Number of row segments of `width` points covering `rows` rows of `cols` points.
__host__ __device__ inline int row_segments(int cols, int rows, int width) {
  return ((cols + width - 1) / width) * rows;
}

}  // namespace fdtdp
