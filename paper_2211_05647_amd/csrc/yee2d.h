// yee2d.h -- TEz Yee updates with the CPML (arXiv 2211.05647, section 2, eq.
// (2)-(5) and the CPML auxiliary fields of eq. (4)), shared by the 2D step kernels and the
// closure kernel, which runs the H half-step beside the network.
//
// Work is mapped in strips: a work-group (wavefront in the closure kernel) takes a run of
// consecutive columns, one per lane, and 1 or 4 rows, so the strip's row and column come
// from one wave-uniform division and a row shared by two points is read once.
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

// Hz^{n+1/2} at (i+1/2, j+1/2) for rows j0 .. j0 + RR - 1 (those below ny) of column
// i < nx, with the H-side psi strips: every input of the RR points is loaded before any
// arithmetic (RR + 1 Ex, 2 RR Ey and RR Hz values in flight per lane, Ex of a shared row
// read once).
template <int RR, class T>
__device__ __forceinline__ void h2d_rows(const Run2D<T>& R, int i, int j0, int64_t step) {
  const int nx = R.nx, ny = R.ny, m = R.m;
  const T* __restrict__ Ex = R.Ex;
  const T* __restrict__ Ey = R.Ey;
  T* __restrict__ Hz = R.Hz;
  T ex[RR + 1], eyl[RR], eyr[RR], hz[RR];
#pragma unroll
  for (int r = 0; r <= RR; ++r) ex[r] = (j0 + r <= ny) ? Ex[(size_t)(j0 + r) * nx + i] : T(0);
#pragma unroll
  for (int r = 0; r < RR; ++r) {
    const int j = j0 + r;
    const bool in = j < ny;
    eyl[r] = in ? Ey[(size_t)j * (nx + 1) + i] : T(0);
    eyr[r] = in ? Ey[(size_t)j * (nx + 1) + i + 1] : T(0);
    hz[r] = in ? Hz[(size_t)j * nx + i] : T(0);
  }
#pragma unroll
  for (int r = 0; r < RR; ++r) {
    const int j = j0 + r;
    if (j >= ny) break;
    const T dEx = ex[r + 1] - ex[r];
    const T dEy = eyr[r] - eyl[r];
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
    const T h = fma(R.S, acc, hz[r]);
    Hz[(size_t)j * nx + i] = h;
    if (R.nprobe) record_probe(R, 6 /* FDTD_F_HZ */, i, j, h, step);
  }
}

// E^{n+1} at the points (i, j0) .. (i, j0 + RR - 1) (those with j <= ny) of the
// (nx+1) x (ny+1) node lattice: Ex at (i+1/2, j) when i < nx, Ey at (i, j+1/2) when j < ny.
// Tangential E on the outer walls stays zero (PEC backing of the CPML); the edge current
// is the mean of the two adjacent cell currents.  Every input is loaded before any
// arithmetic (Hz and Jcx of a row shared by two points read once).
template <int RR, class T>
__device__ __forceinline__ void e2d_rows(const Run2D<T>& R, int i, int j0, int64_t step) {
  const int nx = R.nx, ny = R.ny, m = R.m;
  const T* __restrict__ Hz = R.Hz;
  const T* __restrict__ Jcx = R.Jcx;
  const T* __restrict__ Jcy = R.Jcy;
  T* __restrict__ Ex = R.Ex;
  T* __restrict__ Ey = R.Ey;
  const bool has_x = i < nx, has_y = i >= 1 && i <= nx - 1;
  // rows j0 - 1 .. j0 + RR - 1 of Hz and Jcx at column i
  T hz[RR + 1], jx[RR + 1], hzl[RR], jyl[RR], jyr[RR], ex[RR], ey[RR];
#pragma unroll
  for (int r = 0; r <= RR; ++r) {
    const int j = j0 - 1 + r;
    const bool in = has_x && j >= 0 && j < ny;
    hz[r] = in ? Hz[(size_t)j * nx + i] : T(0);
    jx[r] = in ? Jcx[(size_t)j * nx + i] : T(0);
  }
#pragma unroll
  for (int r = 0; r < RR; ++r) {
    const int j = j0 + r;
    const bool ix = has_x && j >= 1 && j <= ny - 1;
    const bool iy = has_y && j < ny;
    ex[r] = ix ? Ex[(size_t)j * nx + i] : T(0);
    hzl[r] = iy ? Hz[(size_t)j * nx + i - 1] : T(0);
    jyl[r] = iy ? Jcy[(size_t)j * nx + i - 1] : T(0);
    jyr[r] = iy ? Jcy[(size_t)j * nx + i] : T(0);
    ey[r] = iy ? Ey[(size_t)j * (nx + 1) + i] : T(0);
  }
#pragma unroll
  for (int r = 0; r < RR; ++r) {
    const int j = j0 + r;
    if (j > ny) break;
    if (has_x && j >= 1 && j <= ny - 1) {
      const T dHz = hz[r + 1] - hz[r];
      T acc = dHz * R.rkey[j];
      if (m > 0 && (j < m || j > ny - m)) {
        const int sy = j < m ? j : j - ny + 2 * m - 1;
        T* p = R.psi_exy + (size_t)sy * nx + i;
        const T v = fma(R.bey[j], *p, R.aey[j] * dHz);
        *p = v;
        acc += v;
      }
      const T jv = T(0.5) * (jx[r] + jx[r + 1]);
      const T e = fma(R.S, acc, ex[r]) - jv;
      Ex[(size_t)j * nx + i] = e;
      if (R.nprobe) record_probe(R, 4 /* FDTD_F_EX */, i, j, e, step);
    }
    if (has_y && j < ny) {
      const T dHz = hz[r + 1] - hzl[r];
      T acc = dHz * R.rkex[i];
      if (m > 0 && (i < m || i > nx - m)) {
        const int sx = i < m ? i : i - nx + 2 * m - 1;
        T* p = R.psi_eyx + (size_t)j * (2 * m) + sx;
        const T v = fma(R.bex[i], *p, R.aex[i] * dHz);
        *p = v;
        acc += v;
      }
      const T jv = T(0.5) * (jyl[r] + jyr[r]);
      T e = fma(-R.S, acc, ey[r]) - jv;
      if (R.src_kind != 0 && i == R.src_i && (R.src_kind == 1 || j == R.src_j))
        e += (T)source_wave((double)(step + 1) * R.dt, R.src_amp, R.src_w, R.src_tau, R.src_t0);
      Ey[(size_t)j * (nx + 1) + i] = e;
      if (R.nprobe) record_probe(R, 5 /* FDTD_F_EY */, i, j, e, step);
    }
  }
}

// Rows per thread of the multi-row field updates: 4 once that still leaves about 2048
// work-groups of kBlock columns, else 1.
__host__ __device__ inline int field_rows(int cols, int rows) {
  const int segs = (cols + 255) / 256;
  return segs * ((rows + 3) / 4) >= 2048 ? 4 : 1;
}

}  // namespace fdtdp
