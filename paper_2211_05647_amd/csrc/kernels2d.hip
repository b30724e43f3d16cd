// kernels2d.hip -- one leap-frog step of the 2D TEz Yee grid with CPML (arXiv
// 2211.05647, section 2, eq. (2)-(5) and the CPML of eq. (4)) coupled to the 2V kinetic
// F1 of every plasma cell (section 5.2).
//
// Two launches per step:
//   k_h2d_kin  blocks [0, nbk): F1 update of a range of plasma cells, driven by E^n
//              averaged from the cell's two bounding edges to its centre, and the
//              FP64 moments (Jx, Jy) of the cell;  blocks [nbk, ...): Hz^{n+1/2} with
//              the CPML psi of the H side, one row segment per block.  Both halves only
//              read E^n.
//   k_e2d      E^{n+1} with the CPML psi of the E side, the edge current (mean of the
//              two adjacent cell-centre currents), PEC walls and the soft source.
// With the learned closure, the network and Hz share a launch instead (mlp.hip).
// F1 layout: [cell][vx bin a][vy bin b >= nv/2]: the half plane vy > 0 (F1 is odd under
// v -> -v), one contiguous row of nv*nv/2 values per cell.
#include "common.h"
#include "mlp_common.h"
#include "yee2d.h"

namespace fdtdp {

template <class T, int U>
__device__ __forceinline__ void kinetic2d_block(const Run2D<T>& R, int c0, int c1) {
  using V = typename Vec<T>::type;
  constexpr int VPL = Vec<T>::n;
  constexpr int kWaves = kBlock / 64;
  constexpr int CPL = 4 / U;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ch = R.half / VPL;
  const int lpc = ch < 64 ? ch : 64;
  const int cpl = ch / lpc;
  const int cpw = 64 / lpc;
  const int sub = lane / lpc, li = lane - sub * lpc;
  const int nx = R.nx;

  V s[CPL], bx[CPL], by[CPL];
  double wx[CPL][VPL], wy[CPL][VPL];
#pragma unroll
  for (int m = 0; m < CPL; ++m) {
    if (m < cpl) {
      const int k = li + m * lpc;
      s[m] = reinterpret_cast<const V*>(R.s_bin)[k];
      bx[m] = reinterpret_cast<const V*>(R.bx_bin)[k];
      by[m] = reinterpret_cast<const V*>(R.by_bin)[k];
#pragma unroll
      for (int v = 0; v < VPL; ++v) {
        wx[m][v] = R.wx_bin[k * VPL + v];
        wy[m][v] = R.wy_bin[k * VPL + v];
      }
    }
  }
  V* __restrict__ dfv = reinterpret_cast<V*>(R.df);
  const int stride = kWaves * cpw * U;
  for (int base = c0 + wave * cpw * U; base < c1; base += stride) {
    V f[U][CPL];
    T nex[U], ney[U], tau[U];
    int kk[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = base + u * cpw + sub;
      kk[u] = -1;
      if (c < c1) {
        const int k = R.cell_idx[c];
        const int j = k / nx, i = k - j * nx;
        kk[u] = k;
        const T ne = R.dens[c];
        // E^n averaged from the bounding edges to the cell centre
        nex[u] = ne * (T(0.5) * (R.Ex[(size_t)j * nx + i] + R.Ex[(size_t)(j + 1) * nx + i]));
        ney[u] = ne * (T(0.5) * (R.Ey[(size_t)j * (nx + 1) + i] + R.Ey[(size_t)j * (nx + 1) + i + 1]));
        tau[u] = R.tau[c];
        const V* row = dfv + (size_t)c * ch;
#pragma unroll
        for (int m = 0; m < CPL; ++m)
          if (m < cpl) f[u][m] = row[li + m * lpc];
      }
    }
    double acc[2 * U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc[2 * u] = 0.0;
      acc[2 * u + 1] = 0.0;
      if (kk[u] >= 0) {
#pragma unroll
        for (int m = 0; m < CPL; ++m) {
          if (m < cpl) {
#pragma unroll
            for (int v = 0; v < VPL; ++v) {
              const T x = tau[u] * lane_at(s[m], v);
              const T r = cn_recip(T(2) + x);
              const T fv = lane_at(f[u][m], v);
              const T drive = fma(lane_at(bx[m], v), nex[u], lane_at(by[m], v) * ney[u]);
              const T t = fma(-(x + x), fv, drive);
              const T fn = fma(t, r, fv);
              lane_at(f[u][m], v) = fn;
              acc[2 * u] = fma(wx[m][v], (double)fn, acc[2 * u]);
              acc[2 * u + 1] = fma(wy[m][v], (double)fn, acc[2 * u + 1]);
            }
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (kk[u] >= 0) {
        V* row = dfv + (size_t)(base + u * cpw + sub) * ch;
#pragma unroll
        for (int m = 0; m < CPL; ++m)
          if (m < cpl) row[li + m * lpc] = f[u][m];
      }
    }
    if (lpc < 2 * U) {
#pragma unroll
      for (int q = 0; q < 2 * U; ++q) {
        double sm = acc[q];
        for (int o = lpc >> 1; o > 0; o >>= 1) sm += __shfl_xor(sm, o);
        if (li == 0 && kk[q >> 1] >= 0) ((q & 1) ? R.Jcy : R.Jcx)[kk[q >> 1]] = (T)sm;
      }
    } else {
      int which = 0;
      const double tot = group_reduce<2 * U>(acc, lpc, li, which);
#pragma unroll
      for (int q = 0; q < 2 * U; ++q)
        if (which == q && li == reporter<2 * U>(q, lpc) && kk[q >> 1] >= 0)
          ((q & 1) ? R.Jcy : R.Jcx)[kk[q >> 1]] = (T)tot;
    }
  }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_h2d_kin(const Run2D<T>* __restrict__ rp, int64_t step) {
  const Run2D<T>& R = *rp;
  if ((int)blockIdx.x < R.nbk) {
    const int c0 = blockIdx.x * R.cells_per_block;
    const int c1 = min(R.ncell, c0 + R.cells_per_block);
    const int ch = R.half / Vec<T>::n;
    const int cpl = ch < 64 ? 1 : ch / 64;
    if (cpl == 1) kinetic2d_block<T, 4>(R, c0, c1);
    else if (cpl == 2) kinetic2d_block<T, 2>(R, c0, c1);
    else kinetic2d_block<T, 1>(R, c0, c1);
    return;
  }
  // Hz: one row segment of kBlock points per block
  const int seg = (int)blockIdx.x - R.nbk;
  const int spr = (R.nx + kBlock - 1) / kBlock;
  const int j = seg / spr;
  const int i = (seg - j * spr) * kBlock + (int)threadIdx.x;
  if (j < R.ny && i < R.nx) h2d_point(R, i, j, step);
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_e2d(const Run2D<T>* __restrict__ rp, int64_t step) {
  const Run2D<T>& R = *rp;
  // one row segment of kBlock points of the (nx+1) x (ny+1) lattice per block
  const int spr = (R.nx + kBlock) / kBlock;
  const int j = (int)blockIdx.x / spr;
  const int i = ((int)blockIdx.x - j * spr) * kBlock + (int)threadIdx.x;
  if (j <= R.ny && i <= R.nx) e2d_point(R, i, j, step);
}

template <class T>
hipError_t launch_step2d_t(const void* run, int nbk, int nbh, int nbe, int64_t step,
                           hipStream_t stream) {
  const Run2D<T>* r = static_cast<const Run2D<T>*>(run);
  hipLaunchKernelGGL(k_h2d_kin<T>, dim3(nbk + nbh), dim3(kBlock), 0, stream, r, step);
  hipError_t e = hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(k_e2d<T>, dim3(nbe), dim3(kBlock), 0, stream, r, step);
  return hipGetLastError();
}

hipError_t mlp_launch_cells2d(const void* run, const MlpWeights& W, const MlpCells2D& C,
                              int nx, int ny, int64_t step, hipStream_t st);

// Closure step: kinetic blocks for the fallback cells (if any), then one launch that runs
// the network of every closure cell and the Hz update side by side (both only read E^n,
// and the network's arithmetic hides the field update's memory traffic), then E.
hipError_t launch_step2d_closure(const void* run, int nbk, int nx, int ny, int nbe, int64_t step,
                                 hipStream_t stream, const MlpWeights& W, const MlpCells2D& C) {
  const Run2D<float>* r = static_cast<const Run2D<float>*>(run);
  hipError_t e;
  if (nbk > 0) {
    hipLaunchKernelGGL(k_h2d_kin<float>, dim3(nbk), dim3(kBlock), 0, stream, r, step);
    e = hipGetLastError();
    if (e) return e;
  }
  e = mlp_launch_cells2d(run, W, C, nx, ny, step, stream);
  if (e) return e;
  hipLaunchKernelGGL(k_e2d<float>, dim3(nbe), dim3(kBlock), 0, stream, r, step);
  return hipGetLastError();
}

template hipError_t launch_step2d_t<float>(const void*, int, int, int, int64_t, hipStream_t);
template hipError_t launch_step2d_t<double>(const void*, int, int, int, int64_t, hipStream_t);

}  // namespace fdtdp
