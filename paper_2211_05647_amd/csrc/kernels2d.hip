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

// FP32 2V kinetic step specialised for NV bins per axis (NV = 8, 16 or 32): every size is
// a compile-time constant, so the update of a lane's chunks is straight-line code.
//   A cell's row of NV*NV/2 stored values is CH float4 chunks; L lanes share a cell, lane
//   li owning the C chunks li + L m (m < C), so one load instruction of the wavefront
//   reads L consecutive chunks of each of its G cells.  Chunk li + L m lies in vx row
//   a(li) + m NV/C at the same four vy bins for every m, so the FP64 moment weights are
//   C values of vx and 4 values of vy per lane.
//   FP64 moments: each lane accumulates (Jx, Jy) over its 4 C values; a reduce-scatter
//   over the L lanes leaves Jx on lane 0 and Jy on lane L/2 of the group.
//   The next cell's row and scalars are loaded before the current cell is updated, so
//   every wavefront keeps two rows in flight.
constexpr int kKin2vChunks = 4;       // C: float4 chunks per lane
constexpr bool kKin2vPrefetch = true;

struct Kin2vCell {
  int k;          // grid index of the cell
  float nex, ney, tau;
};

template <int NV, int C, bool S>
__device__ __forceinline__ void kin2v_load(const Run2D<float>& R, int c, bool ok, int li,
                                           float4 (&f)[C], Kin2vCell& q) {
  constexpr int CH = NV * NV / 8, L = CH / C;
  if (ok) {
    const int nx = R.nx;
    const int k = R.cell_idx[c];
    const int j = k / nx, i = k - j * nx;
    const float ne = R.dens[c];
    q.k = k;
    q.nex = ne * (0.5f * (R.Ex[(size_t)j * nx + i] + R.Ex[(size_t)(j + 1) * nx + i]));
    q.ney = ne * (0.5f * (R.Ey[(size_t)j * (nx + 1) + i] + R.Ey[(size_t)j * (nx + 1) + i + 1]));
    q.tau = R.tau[c];
    const float4* row = reinterpret_cast<const float4*>(R.df) + (size_t)c * CH;
#pragma unroll
    for (int m = 0; m < C; ++m) f[m] = row_load<S>(&row[li + L * m]);
  } else {
    q.k = 0;
    q.nex = q.ney = q.tau = 0.f;
#pragma unroll
    for (int m = 0; m < C; ++m) f[m] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

// S: the rows are streamed (more of them than the Infinity Cache keeps between steps), with
// nontemporal loads and stores.
template <int NV, int C, bool PF, bool S>
__device__ __forceinline__ void kinetic2v_f32(const Run2D<float>& R, int c0, int c1) {
  constexpr int CH = NV * NV / 8;
  constexpr int L = CH / C;
  constexpr int G = 64 / L;
  constexpr int kWaves = kBlock / 64;
  static_assert(L >= 2 && L <= 64 && CH % C == 0, "kinetic2v_f32 layout");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane / L, li = lane - g * L;
  float4 s[C], bx[C], by[C];
  double wx[C], wy[4];
#pragma unroll
  for (int m = 0; m < C; ++m) {
    const int k = li + L * m;
    s[m] = reinterpret_cast<const float4*>(R.s_bin)[k];
    bx[m] = reinterpret_cast<const float4*>(R.bx_bin)[k];
    by[m] = reinterpret_cast<const float4*>(R.by_bin)[k];
    wx[m] = R.wx_bin[4 * k];
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) wy[e] = R.wy_bin[4 * li + e];
  float4* __restrict__ dfv = reinterpret_cast<float4*>(R.df);
  int base = c0 + wave * G;
  float4 f[C];
  Kin2vCell q;
  if (PF) kin2v_load<NV, C, S>(R, base + g, base + g < c1, li, f, q);
  for (; base < c1; base += kWaves * G) {
    const int c = base + g;
    const bool ok = c < c1;
    float4 fn_[C];
    Kin2vCell qn;
    if (PF) {
      const int cn = c + kWaves * G;
      kin2v_load<NV, C, S>(R, cn, cn < c1, li, fn_, qn);
    } else {
      kin2v_load<NV, C, S>(R, c, ok, li, f, q);
    }
    double ax = 0.0, ay = 0.0;
#pragma unroll
    for (int m = 0; m < C; ++m) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float x = q.tau * lane_at(s[m], e);
        const float r = cn_recip(2.f + x);
        const float fv = lane_at(f[m], e);
        const float drive = fmaf(lane_at(bx[m], e), q.nex, lane_at(by[m], e) * q.ney);
        const float fn = fmaf(fmaf(-(x + x), fv, drive), r, fv);
        lane_at(f[m], e) = fn;
        ax = fma(wx[m], (double)fn, ax);
        ay = fma(wy[e], (double)fn, ay);
      }
    }
    if (ok) {
      float4* row = dfv + (size_t)c * CH;
#pragma unroll
      for (int m = 0; m < C; ++m) row_store<S>(f[m], &row[li + L * m]);
    }
    // reduce-scatter of (ax, ay) over the L lanes of the group
    const bool hi = (li & (L / 2)) != 0;
    double keep = hi ? ay : ax;
    keep += __shfl_xor(hi ? ax : ay, L / 2);
#pragma unroll
    for (int o = L / 4; o > 0; o >>= 1) keep += __shfl_xor(keep, o);
    if (ok && li == 0) R.Jcx[q.k] = (float)keep;
    if (ok && li == L / 2) R.Jcy[q.k] = (float)keep;
    if (PF) {
#pragma unroll
      for (int m = 0; m < C; ++m) f[m] = fn_[m];
      q = qn;
    }
  }
}

// Work-group b of n renumbered so that the work-groups one XCD runs (the dispatcher deals
// them out to the eight XCDs in turn) take one contiguous range: a field strip's
// neighbouring rows are then read by the same XCD shortly before or after, from its L2,
// instead of again from HBM by another XCD.
__device__ __forceinline__ int xcd_contiguous(int b, int n) {
  const int q = n >> 3, r = n & 7, x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

// NV > 0: FP32 with NV bins per velocity axis (the specialised kinetic path); NV = 0: any
// bin count and precision.
template <class T, int NV, bool S = false>
__global__ __launch_bounds__(kBlock) void k_h2d_kin(const Run2D<T>* __restrict__ rp, int64_t step) {
  const Run2D<T>& R = *rp;
  if ((int)blockIdx.x < R.nbk) {
    const int c0 = blockIdx.x * R.cells_per_block;
    const int c1 = min(R.ncell, c0 + R.cells_per_block);
    if constexpr (NV > 0) {
      kinetic2v_f32<NV, kKin2vChunks, kKin2vPrefetch, S>(R, c0, c1);
    } else {
      const int ch = R.half / Vec<T>::n;
      const int cpl = ch < 64 ? 1 : ch / 64;
      if (cpl == 1) kinetic2d_block<T, 4>(R, c0, c1);
      else if (cpl == 2) kinetic2d_block<T, 2>(R, c0, c1);
      else kinetic2d_block<T, 1>(R, c0, c1);
    }
    return;
  }
  // Hz: kBlock columns by R.hrows (1 or 4) rows per block
  const int seg = xcd_contiguous((int)blockIdx.x - R.nbk, (int)gridDim.x - R.nbk);
  const int spr = (R.nx + kBlock - 1) / kBlock;
  const int strip = seg / spr;
  const int i = (seg - strip * spr) * kBlock + (int)threadIdx.x;
  if (i >= R.nx) return;
  if (R.hrows == 4) h2d_rows<4>(R, i, strip * 4, step);
  else h2d_rows<1>(R, i, strip, step);
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_e2d(const Run2D<T>* __restrict__ rp, int64_t step) {
  const Run2D<T>& R = *rp;
  // kBlock columns by R.erows (1 or 4) rows of the (nx+1) x (ny+1) lattice per block
  const int spr = (R.nx + kBlock) / kBlock;
  const int b = xcd_contiguous((int)blockIdx.x, (int)gridDim.x);
  const int strip = b / spr;
  const int i = (b - strip * spr) * kBlock + (int)threadIdx.x;
  if (i > R.nx) return;
  if (R.erows == 4) e2d_rows<4>(R, i, strip * 4, step);
  else e2d_rows<1>(R, i, strip, step);
}

// H + kinetic launch, picking the kinetic path by the stored bins per cell (and, in FP32,
// streamed rows when `streaming`)
template <class T, int NV>
hipError_t launch_h2d_kin_nv(const Run2D<T>* r, int grid, int64_t step, hipStream_t stream,
                             bool streaming) {
  if (streaming)
    hipLaunchKernelGGL((k_h2d_kin<T, NV, true>), dim3(grid), dim3(kBlock), 0, stream, r, step);
  else
    hipLaunchKernelGGL((k_h2d_kin<T, NV, false>), dim3(grid), dim3(kBlock), 0, stream, r, step);
  return hipGetLastError();
}

template <class T>
hipError_t launch_h2d_kin(const Run2D<T>* r, int half, int grid, int64_t step, hipStream_t stream,
                          bool streaming) {
  if (grid <= 0) return hipSuccess;
  if constexpr (sizeof(T) == 4) {
    if (half == 32) return launch_h2d_kin_nv<T, 8>(r, grid, step, stream, streaming);
    if (half == 128) return launch_h2d_kin_nv<T, 16>(r, grid, step, stream, streaming);
    if (half == 512) return launch_h2d_kin_nv<T, 32>(r, grid, step, stream, streaming);
  }
  hipLaunchKernelGGL((k_h2d_kin<T, 0>), dim3(grid), dim3(kBlock), 0, stream, r, step);
  return hipGetLastError();
}

template <class T>
hipError_t launch_step2d_t(const void* run, int half, int nbk, int nbh, int nbe, int64_t step,
                           hipStream_t stream, bool streaming) {
  const Run2D<T>* r = static_cast<const Run2D<T>*>(run);
  hipError_t e = launch_h2d_kin(r, half, nbk + nbh, step, stream, streaming);
  if (e) return e;
  hipLaunchKernelGGL(k_e2d<T>, dim3(nbe), dim3(kBlock), 0, stream, r, step);
  return hipGetLastError();
}

hipError_t mlp_launch_cells2d(const void* run, const MlpWeights& W, const MlpCells2D& C,
                              int nx, int ny, int64_t step, hipStream_t st);

// Closure step: kinetic blocks for the fallback cells (if any), then one launch that runs
// the network of every closure cell and the Hz update side by side (both only read E^n,
// and the network's arithmetic hides the field update's memory traffic), then E.
hipError_t launch_step2d_closure(const void* run, int half, int nbk, int nx, int ny, int nbe,
                                 int64_t step, hipStream_t stream, const MlpWeights& W,
                                 const MlpCells2D& C) {
  const Run2D<float>* r = static_cast<const Run2D<float>*>(run);
  hipError_t e = launch_h2d_kin(r, half, nbk, step, stream, false);
  if (e) return e;
  e = mlp_launch_cells2d(run, W, C, nx, ny, step, stream);
  if (e) return e;
  hipLaunchKernelGGL(k_e2d<float>, dim3(nbe), dim3(kBlock), 0, stream, r, step);
  return hipGetLastError();
}

template hipError_t launch_step2d_t<float>(const void*, int, int, int, int, int64_t, hipStream_t,
                                           bool);
template hipError_t launch_step2d_t<double>(const void*, int, int, int, int, int64_t, hipStream_t,
                                            bool);

}  // namespace fdtdp
