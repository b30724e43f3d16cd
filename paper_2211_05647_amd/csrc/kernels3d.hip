// kernels3d.hip -- one leap-frog step of the 3D Yee cube coupled to the speed-grid F1 of
// every plasma point (arXiv 2211.05647, section 2 in its 3D form and section 5.3).
//
// Three launches per step, in the order of the method:
//   k_h3d    H^{n+1/2} of the three components (one thread per lattice point), with the
//            CPML memory of each derivative inside its layer;
//   k_kin3d  F1 of every plasma point driven by its E component at t^n (Crank-Nicolson in
//            the collision term) and the FP64 moment J = -e (4 pi / 3) gam sum v^3 F1,
//            one lane group per point row;
//   k_e3d    E^{n+1} = E^n + S curl H - J with the CPML memory, the soft source at t^{n+1}
//            (the kinetic launch subtracts J at the plasma points, in place).
// Tangential E on the outer faces is never written (PEC backing of the layer).
#include "common.h"

namespace fdtdp {

namespace {

// Position of a lattice coordinate inside the 2m-wide layer store, or -1 outside the
// layer.  e side (integer positions 0..n): layer where u < m or u > n - m; h side
// (positions u + 1/2, u < n): where u < m or u >= n - m.
__device__ __forceinline__ int layer_e(int u, int n, int m) {
  return u < m ? u : (u > n - m ? u - (n - 2 * m + 1) : -1);
}
__device__ __forceinline__ int layer_h(int u, int n, int m) {
  return u < m ? u : (u >= n - m ? u - (n - 2 * m) : -1);
}

}  // namespace

// The H and E launches map one thread to one lattice point (i, j) of a k plane: the
// plane's (nx+1)(ny+1) points are numbered i fastest and cut into tiles of 256, so every
// lane has work whatever nx is.  Work-groups are dealt to the 8 XCDs round robin
// (work-group b runs on XCD b mod 8); the tiles are renumbered so that each XCD takes a
// contiguous slab of planes, in order: the neighbouring plane a point's curl reads
// (k + 1 for H, k - 1 for E) was then just loaded into that XCD's L2.  (A thread marching
// through a run of planes with that neighbour in a register measured slower: fewer
// threads, a serial chain of loads.)
constexpr int kXcds = 8;

struct PlaneTile {
  int i, j, k;
  bool ok;
};

__device__ __forceinline__ PlaneTile plane_tile(int nx, int ny, int nz) {
  const int tiles = ((nx + 1) * (ny + 1) + 255) / 256;
  const int per_xcd = gridDim.x / kXcds;          // gridDim.x is a multiple of kXcds
  const int b = blockIdx.x;
  const int logical = (b % kXcds) * per_xcd + b / kXcds;
  const int k = logical / tiles, tile = logical - k * tiles;
  const int t = tile * 256 + threadIdx.x;
  PlaneTile p;
  p.ok = k <= nz && t < (nx + 1) * (ny + 1);
  p.j = t / (nx + 1);
  p.i = t - p.j * (nx + 1);
  p.k = k;
  return p;
}

template <class T>
__global__ __launch_bounds__(256) void k_h3d(const Run3D<T> R) {
  const int nx = R.nx, ny = R.ny, nz = R.nz, m = R.m;
  const PlaneTile pt = plane_tile(nx, ny, nz);
  if (!pt.ok) return;
  const int i = pt.i, j = pt.j, k = pt.k;
  const size_t sEx_j = nx, sEx_k = (size_t)(ny + 1) * nx;
  const size_t sEy_j = nx + 1, sEy_k = (size_t)ny * (nx + 1);
  const size_t sEz_j = nx + 1, sEz_k = (size_t)(ny + 1) * (nx + 1);
  const T S = R.S;
  // Hx at (i, j+1/2, k+1/2)
  if (j < ny && k < nz) {
    const size_t q = ((size_t)k * ny + j) * (nx + 1) + i;
    const T dEy_z = R.Ey[(k + 1) * sEy_k + j * sEy_j + i] - R.Ey[k * sEy_k + j * sEy_j + i];
    const T dEz_y = R.Ez[k * sEz_k + (j + 1) * sEz_j + i] - R.Ez[k * sEz_k + j * sEz_j + i];
    T acc = dEy_z * R.rkhz[k] - dEz_y * R.rkhy[j];
    if (m > 0) {
      const int sz = layer_h(k, nz, m), sy = layer_h(j, ny, m);
      if (sz >= 0) {
        T* p = R.p_hxz + ((size_t)sz * ny + j) * (nx + 1) + i;
        const T v = fma(R.bhz[k], *p, R.ahz[k] * dEy_z);
        *p = v;
        acc += v;
      }
      if (sy >= 0) {
        T* p = R.p_hxy + ((size_t)k * 2 * m + sy) * (nx + 1) + i;
        const T v = fma(R.bhy[j], *p, R.ahy[j] * dEz_y);
        *p = v;
        acc -= v;
      }
    }
    R.Hx[q] = fma(S, acc, R.Hx[q]);
  }
  // Hy at (i+1/2, j, k+1/2)
  if (i < nx && k < nz) {
    const size_t q = ((size_t)k * (ny + 1) + j) * nx + i;
    const T dEz_x = R.Ez[k * sEz_k + j * sEz_j + i + 1] - R.Ez[k * sEz_k + j * sEz_j + i];
    const T dEx_z = R.Ex[(k + 1) * sEx_k + j * sEx_j + i] - R.Ex[k * sEx_k + j * sEx_j + i];
    T acc = dEz_x * R.rkhx[i] - dEx_z * R.rkhz[k];
    if (m > 0) {
      const int sx = layer_h(i, nx, m), sz = layer_h(k, nz, m);
      if (sx >= 0) {
        T* p = R.p_hyx + ((size_t)k * (ny + 1) + j) * 2 * m + sx;
        const T v = fma(R.bhx[i], *p, R.ahx[i] * dEz_x);
        *p = v;
        acc += v;
      }
      if (sz >= 0) {
        T* p = R.p_hyz + ((size_t)sz * (ny + 1) + j) * nx + i;
        const T v = fma(R.bhz[k], *p, R.ahz[k] * dEx_z);
        *p = v;
        acc -= v;
      }
    }
    R.Hy[q] = fma(S, acc, R.Hy[q]);
  }
  // Hz at (i+1/2, j+1/2, k)
  if (i < nx && j < ny) {
    const size_t q = ((size_t)k * ny + j) * nx + i;
    const T dEx_y = R.Ex[k * sEx_k + (j + 1) * sEx_j + i] - R.Ex[k * sEx_k + j * sEx_j + i];
    const T dEy_x = R.Ey[k * sEy_k + j * sEy_j + i + 1] - R.Ey[k * sEy_k + j * sEy_j + i];
    T acc = dEx_y * R.rkhy[j] - dEy_x * R.rkhx[i];
    if (m > 0) {
      const int sy = layer_h(j, ny, m), sx = layer_h(i, nx, m);
      if (sy >= 0) {
        T* p = R.p_hzy + ((size_t)k * 2 * m + sy) * nx + i;
        const T v = fma(R.bhy[j], *p, R.ahy[j] * dEx_y);
        *p = v;
        acc += v;
      }
      if (sx >= 0) {
        T* p = R.p_hzx + ((size_t)k * ny + j) * 2 * m + sx;
        const T v = fma(R.bhx[i], *p, R.ahx[i] * dEy_x);
        *p = v;
        acc -= v;
      }
    }
    R.Hz[q] = fma(S, acc, R.Hz[q]);
  }
}

// One row per group of lpc = row / VPL lanes; the wavefront walks its rows together so
// that the moment's shuffles always see whole groups.
template <class T>
__global__ __launch_bounds__(256) void k_kin3d(const Run3D<T> R) {
  using V = typename Vec<T>::type;
  constexpr int VPL = Vec<T>::n;
  const int lane = threadIdx.x & 63;
  const int lpc = R.row / VPL;             // power of two, <= 64
  const int cpw = 64 / lpc;
  const int sub = lane / lpc, li = lane - sub * lpc;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int nwave = (gridDim.x * blockDim.x) >> 6;
  V s = reinterpret_cast<const V*>(R.s_bin)[li];
  V b = reinterpret_cast<const V*>(R.b_bin)[li];
  double w[VPL];
#pragma unroll
  for (int v = 0; v < VPL; ++v) w[v] = R.w_bin[li * VPL + v];
  V* __restrict__ dfv = reinterpret_cast<V*>(R.df);
  const T* E = R.Ex;   // Ex, Ey, Ez are contiguous
  T* Ee = R.Ex;
  T* __restrict__ J = R.Jx;
  for (int base = wave * cpw; base < R.np; base += nwave * cpw) {
    const int p = base + sub;
    const bool live = p < R.np;
    double acc = 0.0;
    int at = 0;
    if (live) {
      at = R.pidx[p];
      const T tau = R.tau[p];
      const T nE = R.dens[p] * E[at];
      const T tau2 = tau + tau;
      V f = dfv[(size_t)p * lpc + li];
#pragma unroll
      for (int v = 0; v < VPL; ++v) {
        // F1' = ((2 - x) F1 + 2 dt (e/m) n dF0/dv E) / (2 + x), x = dt nu_k, as an increment
        const T sv = lane_at(s, v);
        const T r = cn_recip(fma(tau, sv, T(2)));
        const T fv = lane_at(f, v);
        const T t = fma(-(tau2 * sv), fv, lane_at(b, v) * nE);
        const T fn = fma(t, r, fv);
        lane_at(f, v) = fn;
        acc = fma(w[v], (double)fn, acc);
      }
      dfv[(size_t)p * lpc + li] = f;
    }
    double a1[1] = {acc};
    int which = 0;
    const double tot = group_reduce<1>(a1, lpc, li, which);
    if (live && li == 0) {
      // Ampere's law takes -J: applied here, so the E launch reads no current array
      const T jv = (T)tot;
      J[at] = jv;
      Ee[at] = E[at] - jv;
    }
  }
}

// E^{n+1} = E^n + S curl H (the kinetic launch has already taken J^{n+1/2} off E^n at
// the plasma points).
template <class T>
__global__ __launch_bounds__(256) void k_e3d(const Run3D<T> R, int64_t step) {
  const int nx = R.nx, ny = R.ny, nz = R.nz, m = R.m;
  const PlaneTile pt = plane_tile(nx, ny, nz);
  if (!pt.ok) return;
  const int i = pt.i, j = pt.j, k = pt.k;
  const size_t sHx_j = nx + 1, sHx_k = (size_t)ny * (nx + 1);
  const size_t sHy_j = nx, sHy_k = (size_t)(ny + 1) * nx;
  const size_t sHz_j = nx, sHz_k = (size_t)ny * nx;
  const T S = R.S;
  // Ex at (i+1/2, j, k), tangential to the y and z faces
  if (i < nx && j >= 1 && j < ny && k >= 1 && k < nz) {
    const size_t q = ((size_t)k * (ny + 1) + j) * nx + i;
    const T dHz_y = R.Hz[k * sHz_k + j * sHz_j + i] - R.Hz[k * sHz_k + (j - 1) * sHz_j + i];
    const T dHy_z = R.Hy[k * sHy_k + j * sHy_j + i] - R.Hy[(k - 1) * sHy_k + j * sHy_j + i];
    T acc = dHz_y * R.rkey[j] - dHy_z * R.rkez[k];
    if (m > 0) {
      const int sy = layer_e(j, ny, m), sz = layer_e(k, nz, m);
      if (sy >= 0) {
        T* p = R.p_exy + ((size_t)k * 2 * m + sy) * nx + i;
        const T v = fma(R.bey[j], *p, R.aey[j] * dHz_y);
        *p = v;
        acc += v;
      }
      if (sz >= 0) {
        T* p = R.p_exz + ((size_t)sz * (ny + 1) + j) * nx + i;
        const T v = fma(R.bez[k], *p, R.aez[k] * dHy_z);
        *p = v;
        acc -= v;
      }
    }
    T e = fma(S, acc, R.Ex[q]);
    if (R.src_kind != 0 && k == R.src_k && (R.src_kind == 1 || (i == R.src_i && j == R.src_j)))
      e += (T)source_wave((double)(step + 1) * R.dt, R.src_amp, R.src_w, R.src_tau, R.src_t0);
    R.Ex[q] = e;
  }
  // Ey at (i, j+1/2, k), tangential to the x and z faces
  if (i >= 1 && i < nx && j < ny && k >= 1 && k < nz) {
    const size_t q = ((size_t)k * ny + j) * (nx + 1) + i;
    const T dHx_z = R.Hx[k * sHx_k + j * sHx_j + i] - R.Hx[(k - 1) * sHx_k + j * sHx_j + i];
    const T dHz_x = R.Hz[k * sHz_k + j * sHz_j + i] - R.Hz[k * sHz_k + j * sHz_j + i - 1];
    T acc = dHx_z * R.rkez[k] - dHz_x * R.rkex[i];
    if (m > 0) {
      const int sz = layer_e(k, nz, m), sx = layer_e(i, nx, m);
      if (sz >= 0) {
        T* p = R.p_eyz + ((size_t)sz * ny + j) * (nx + 1) + i;
        const T v = fma(R.bez[k], *p, R.aez[k] * dHx_z);
        *p = v;
        acc += v;
      }
      if (sx >= 0) {
        T* p = R.p_eyx + ((size_t)k * ny + j) * 2 * m + sx;
        const T v = fma(R.bex[i], *p, R.aex[i] * dHz_x);
        *p = v;
        acc -= v;
      }
    }
    R.Ey[q] = fma(S, acc, R.Ey[q]);
  }
  // Ez at (i, j, k+1/2), tangential to the x and y faces
  if (i >= 1 && i < nx && j >= 1 && j < ny && k < nz) {
    const size_t q = ((size_t)k * (ny + 1) + j) * (nx + 1) + i;
    const T dHy_x = R.Hy[k * sHy_k + j * sHy_j + i] - R.Hy[k * sHy_k + j * sHy_j + i - 1];
    const T dHx_y = R.Hx[k * sHx_k + j * sHx_j + i] - R.Hx[k * sHx_k + (j - 1) * sHx_j + i];
    T acc = dHy_x * R.rkex[i] - dHx_y * R.rkey[j];
    if (m > 0) {
      const int sx = layer_e(i, nx, m), sy = layer_e(j, ny, m);
      if (sx >= 0) {
        T* p = R.p_ezx + ((size_t)k * (ny + 1) + j) * 2 * m + sx;
        const T v = fma(R.bex[i], *p, R.aex[i] * dHy_x);
        *p = v;
        acc += v;
      }
      if (sy >= 0) {
        T* p = R.p_ezy + ((size_t)k * 2 * m + sy) * (nx + 1) + i;
        const T v = fma(R.bey[j], *p, R.aey[j] * dHx_y);
        *p = v;
        acc -= v;
      }
    }
    R.Ez[q] = fma(S, acc, R.Ez[q]);
  }
}

template <class T>
hipError_t launch_step3d_t(const void* run, int nx, int ny, int nz, int np, int kin_groups,
                           int64_t step, hipStream_t stream) {
  const Run3D<T>& R = *static_cast<const Run3D<T>*>(run);
  const int tiles = ((nx + 1) * (ny + 1) + 255) / 256;
  const int blocks = (tiles * (nz + 1) + kXcds - 1) / kXcds * kXcds;
  const dim3 grid(blocks);
  hipLaunchKernelGGL(k_h3d<T>, grid, dim3(256), 0, stream, R);
  if (np > 0) hipLaunchKernelGGL(k_kin3d<T>, dim3(kin_groups), dim3(256), 0, stream, R);
  hipLaunchKernelGGL(k_e3d<T>, grid, dim3(256), 0, stream, R, step);
  return hipGetLastError();
}

template hipError_t launch_step3d_t<float>(const void*, int, int, int, int, int, int64_t,
                                           hipStream_t);
template hipError_t launch_step3d_t<double>(const void*, int, int, int, int, int, int64_t,
                                            hipStream_t);

}  // namespace fdtdp
