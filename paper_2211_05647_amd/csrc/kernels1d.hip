// kernels1d.hip -- one leap-frog step of the 1D (Ez, Hy) Yee line coupled to the 1V
// kinetic F1 of every plasma node (arXiv 2211.05647, section 2 and section 5.2).
//
// One work-group owns a tile of E nodes [node0, node1) and the plasma nodes inside
// it [cell0, cell1).  Per step it
//   1. advances F1 of its plasma nodes with E^n (Crank-Nicolson in the collision term,
//      the f_1x update of section 5.2) and reduces the current moment
//      J = -e dv sum_j v_j F1_j in FP64 (half grid: F1 is odd in v, so the sum over
//      v > 0 bins counts twice), keeping the tile's J in LDS;
//   2. updates H^{n+1/2} and E^{n+1} of its nodes (Ampere's law minus J), with the
//      first-order Mur ends and the soft source.
// E and H are double-buffered, so halo values are re-derived from the previous
// buffers and no work-group ever waits for another inside a step.
//
// Memory layout of F1: [cell][v > 0 bin], contiguous in the bin index; a wavefront
// covers one or more cells per pass with 16-byte loads per lane (coalesced rows).
#include "common.h"

namespace fdtdp {

template <class T>
__device__ __forceinline__ void kinetic_tile(const Run1D<T>& R, const T* __restrict__ Ec,
                                             const Tile1D& tile, T* jloc) {
  using V = typename Vec<T>::type;
  constexpr int VPL = Vec<T>::n;
  constexpr int kWaves = kBlock / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ch = R.half / VPL;            // 16-byte chunks per cell row
  const int lpc = ch < 64 ? ch : 64;      // lanes per cell
  const int cpl = ch / lpc;               // chunks per lane (<= 4)
  const int cpw = 64 / lpc;               // cells per wavefront pass
  const int sub = lane / lpc, li = lane - sub * lpc;

  V s[4], b[4];
  double w[4][VPL];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    if (m < cpl) {
      const int k = li + m * lpc;
      s[m] = reinterpret_cast<const V*>(R.s_bin)[k];
      b[m] = reinterpret_cast<const V*>(R.b_bin)[k];
#pragma unroll
      for (int v = 0; v < VPL; ++v) w[m][v] = R.w_bin[k * VPL + v];
    }
  }
  V* __restrict__ dfv = reinterpret_cast<V*>(R.df);
  for (int base = tile.cell0 + wave * cpw; base < tile.cell1; base += kWaves * cpw) {
    const int c = base + sub;
    const bool act = c < tile.cell1;
    double acc = 0.0;
    int node = 0;
    if (act) {
      node = R.cell_node[c];
      const T ne = R.dens[c] * Ec[node];
      const T tau = R.tau[c];
      V* __restrict__ row = dfv + (size_t)c * ch;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        if (m < cpl) {
          V f = row[li + m * lpc];
#pragma unroll
          for (int v = 0; v < VPL; ++v) {
            const T x = tau * lane_at(s[m], v);          // dt * nu_j
            const T r = cn_recip(T(2) + x);
            const T fv = lane_at(f, v);
            // F1' = ((2 - x) F1 + 2 dt (e/m) n dF0/dv E) / (2 + x), as an increment of F1
            const T t = fma(-(x + x), fv, lane_at(b[m], v) * ne);
            const T fn = fma(t, r, fv);
            lane_at(f, v) = fn;
            acc = fma(w[m][v], (double)fn, acc);
          }
          row[li + m * lpc] = f;
        }
      }
    }
    for (int o = lpc >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (act && li == 0) jloc[node - tile.node0] = (T)acc;
  }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_step1d(const Run1D<T>* __restrict__ runs,
                                                   const Tile1D* __restrict__ tiles,
                                                   int64_t step) {
  __shared__ T jloc[kMaxTile1D];
  const Tile1D tile = tiles[blockIdx.x];
  const Run1D<T>& R = runs[tile.run];
  if (step >= R.step_limit) return;
  const int par = (int)(step & 1);
  const T* __restrict__ Ec = R.E[par];
  T* __restrict__ En = R.E[par ^ 1];
  const T* __restrict__ Hc = R.H[par];
  T* __restrict__ Hn = R.H[par ^ 1];
  const int tid = threadIdx.x;
  const int nloc = tile.node1 - tile.node0;
  for (int k = tid; k < nloc; k += kBlock) jloc[k] = T(0);
  __syncthreads();
  if (tile.cell1 > tile.cell0) kinetic_tile<T>(R, Ec, tile, jloc);
  __syncthreads();

  const int nx = R.nx;
  const T S = R.S;
  for (int k = tid; k < nloc; k += kBlock) {
    const int i = tile.node0 + k;
    T en, hn = T(0);
    const T jv = jloc[k];
    if (i == 0) {
      hn = h_update(Hc[0], S, Ec[1], Ec[0]);
      if (R.bc == 1) {
        const T h1 = h_update(Hc[1], S, Ec[2], Ec[1]);
        const T e1 = e_update(Ec[1], S, h1, hn, T(0));
        en = fma(R.q, e1 - Ec[0], Ec[1]);
      } else {
        en = T(0);
      }
      Hn[0] = hn;
    } else if (i == nx) {
      if (R.bc == 1) {
        const T ha = h_update(Hc[nx - 1], S, Ec[nx], Ec[nx - 1]);
        const T hb = h_update(Hc[nx - 2], S, Ec[nx - 1], Ec[nx - 2]);
        const T e = e_update(Ec[nx - 1], S, ha, hb, T(0));
        en = fma(R.q, e - Ec[nx], Ec[nx - 1]);
      } else {
        en = T(0);
      }
    } else {
      const T hm = h_update(Hc[i - 1], S, Ec[i], Ec[i - 1]);
      hn = h_update(Hc[i], S, Ec[i + 1], Ec[i]);
      Hn[i] = hn;
      en = e_update(Ec[i], S, hn, hm, jv);
      if (i == R.src_node)
        en += (T)source_wave((double)(step + 1) * R.dt, R.src_amp, R.src_w, R.src_tau,
                             R.src_t0);
    }
    En[i] = en;
    R.J[i] = jv;
    for (int p = 0; p < R.nprobe; ++p) {
      if (R.probe_node[p] == i) {
        const int f = R.probe_field[p];
        const T val = (f == 0) ? en : (f == 1 ? hn : jv);
        R.probe_buf[(size_t)p * R.probe_cap + (size_t)(step % R.probe_cap)] = val;
      }
    }
  }
}

template <class T>
hipError_t launch_step1d(const void* runs, const void* tiles, int ntiles, int64_t step,
                         hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_step1d<T>, dim3(ntiles), dim3(kBlock), 0, stream,
                     static_cast<const Run1D<T>*>(runs), static_cast<const Tile1D*>(tiles),
                     step);
  return hipGetLastError();
}

template hipError_t launch_step1d<float>(const void*, const void*, int, int64_t, hipStream_t);
template hipError_t launch_step1d<double>(const void*, const void*, int, int64_t, hipStream_t);

}  // namespace fdtdp
