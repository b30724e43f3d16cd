// kernels1d_tb.hip -- K leap-frog steps of the 1D (Ez, Hy) Yee line with the 1V kinetic
// F1 of every plasma node per launch (arXiv 2211.05647, section 2 and section 5.2):
// temporal blocking with halo recomputation.
//
// The kinetic step has no spatial coupling (the model carries no streaming term), so a
// node's state after K steps depends only on the fields and F1 within K nodes of it.  A
// work-group owns nodes [node0, node1) and loads the fields of the extended range
// [node0 - K, node1 + K) (clipped to the line) and the F1 rows of every plasma node in it;
// it then takes all of them through K steps on chip -- fields in LDS, F1 rows in
// registers -- while the range of valid nodes shrinks by one per step and side (not at
// the line's ends, where the Mur update needs only nodes inside the line).  Only the owned
// nodes and their F1 rows are written back.  F1 therefore crosses HBM once per K steps
// (plus the halo rows), instead of once per step.  The rows are read from one copy and
// written to the other (in_off, out_off): a work-group that starts after its neighbour
// has finished still reads that neighbour's rows as they were when the launch began.
//
// Every value is produced by the same arithmetic as the one-step kernel (the same
// update functions, operand order, lane-to-bin mapping and pairing tree of the FP64
// moment), so a blocked run is bitwise the run of K one-step launches.
//
// Requirements (checked on the host): FP32 storage, Nv/2 in {32, 64, 128, 256} stored bins
// per node (one 16-byte chunk per lane, at least 8 lanes per row), K odd (the launch reads
// field buffer step & 1 and writes the other), extended ranges of at most kTbBlock nodes
// and tb_max_rows(Nv/2) plasma nodes.
#include "common.h"
#include "host_internal.h"

namespace fdtdp {

constexpr int kTbBlock = 512;               // threads per work-group (8 wavefronts)
constexpr int kTbWaves = kTbBlock / 64;
constexpr int kTbU = 4;                     // rows per lane group per row slot group
constexpr int kTbIters = 2;                 // row slot groups per lane group: 8 row
                                            // slots with their two Crank-Nicolson
                                            // coefficients per bin (127 VGPRs: two
                                            // work-groups per compute unit; 12 slots
                                            // that recompute them every step measured
                                            // 10% slower)
constexpr int kTbRowsPerGroup = kTbIters * kTbU;

// One sub-step of the fields of a tile's extended range, by the thread of node
// i = x0 + k: H^{n+1/2} on [lo, hi - 1) and E^{n+1} (minus the current Js, plus the soft
// source sample `src`) on the next valid range [nlo, nhi), with the first-order Mur ends;
// the owned nodes also check for non-finite E and feed the probe and tap buffers.  The
// same operations as the one-step kernel's field update.
template <int NW>
__device__ __forceinline__ void tb_fields(const Run1D<float>& R, const Tile1D& tile,
                                          float (*Es)[NW], float (*Hs)[NW],
                                          const float* Js, float src, int k, int i, int p,
                                          int lo, int hi, int nlo, int nhi, int nx, float S,
                                          int bc, float mq, int src_node, int nprobe, int ntap,
                                          int64_t gs) {
  if (i >= lo && i < hi) {
    // every LDS value of the interior update, read in one batch (one LDS round trip on the
    // sub-step's critical path); the clamped neighbours are the ones read only where they
    // exist (k - 1 where E is produced, k + 1 where H is)
    const int km = k > 0 ? k - 1 : 0;
    const int kp = k + 1 < NW ? k + 1 : k;
    const float e0 = Es[p][k], jv = Js[k], ep = Es[p][kp], em = Es[p][km];
    const float h0 = Hs[p][k], hm = Hs[p][km];
    float en = 0.f, hn = 0.f;
    bool has_e = i >= nlo && i < nhi;
    if (i == 0) {
      hn = h_update(h0, S, ep, e0);
      if (bc == 1) {
        const float h1 = h_update(Hs[p][k + 1], S, Es[p][k + 2], ep);
        const float e1 = e_update(ep, S, h1, hn, 0.f);
        en = fmaf(mq, e1 - e0, ep);
      }
      Hs[p ^ 1][k] = hn;
    } else if (i == nx) {
      if (bc == 1) {
        const float ha = h_update(hm, S, e0, em);
        const float hb = h_update(Hs[p][k - 2], S, em, Es[p][k - 2]);
        const float e = e_update(em, S, ha, hb, 0.f);
        en = fmaf(mq, e - e0, em);
      }
    } else {
      if (i < hi - 1) {
        hn = h_update(h0, S, ep, e0);
        Hs[p ^ 1][k] = hn;
      }
      if (has_e) {
        const float hl = h_update(hm, S, e0, em);
        en = e_update(e0, S, hn, hl, jv);
        if (i == src_node) en += src;
      }
    }
    if (has_e) Es[p ^ 1][k] = en;
    if (has_e && i >= tile.node0 && i < tile.node1) {
      if (!isfinite(en))
        __hip_atomic_fetch_or(gptr(R.status), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      for (int q = 0; q < nprobe; ++q) {
        if (gptr(R.probe_node)[q] == i) {
          const int fld = gptr(R.probe_field)[q];
          const float val = (fld == 0) ? en : (fld == 1 ? hn : jv);
          gptr(R.probe_buf)[(size_t)q * R.probe_cap + (size_t)(gs % R.probe_cap)] = val;
        }
      }
      for (int t = 0; t < ntap; ++t) {
        if (gptr(R.tap_node)[t] == i && gs < R.tap_cap) {
          auto dst = gptr(R.tap_buf) + ((size_t)t * R.tap_cap + (size_t)gs) * 2;
          dst[0] = e0;
          dst[1] = jv;
        }
      }
    }
  }
}

// The half of the kinetic update that does not depend on E, F1 + d F1, in place: done
// before the sub-step's E is ready (while wavefront 0 updates the fields).
__device__ __forceinline__ void tb_drive64(float4 (&f)[kTbIters][kTbU],
                                           const float4 (&dd)[kTbIters][kTbU]) {
#pragma unroll
  for (int it = 0; it < kTbIters; ++it)
#pragma unroll
    for (int u = 0; u < kTbU; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float fv = lane_at(f[it][u], v);
        lane_at(f[it][u], v) = fmaf(lane_at(dd[it][u], v), fv, fv);
      }
}

// The kinetic phase of one sub-step for rows of 64 lanes (one row per wavefront slot,
// 4 bins per lane), given f = F1 + d F1 from tb_drive64: F1' = f + c' E -- the same
// operations, in the same order, as F1' = (F1 + d F1) + c' E in one go -- and the FP64
// moment of every slot, the totals
// of the slots whose node holds a valid E (lo <= node < hi) written to Js.  Every slot is
// updated, also rows whose node has dropped out of the valid range: their F1 is never
// written back and their current never reported, and the update stays finite
// (|1 + d| < 1, E finite), so the uniform, branch-free form costs nothing in results.
// The E of the eight slots comes from one LDS read (lane q reads slot q's node,
// tab_loc) and v_readlane; tab_row says whether slot q holds a row.
__device__ __forceinline__ void tb_kinetic64(float4 (&f)[kTbIters][kTbU],
                                             const float4 (&cc)[kTbIters][kTbU],
                                             const double (&w)[4], const float* Esp, float* Js,
                                             int tab_loc, int tab_row, int x0, int lo, int hi,
                                             int li) {
  const float ev = Esp[tab_loc];
#pragma unroll
  for (int it = 0; it < kTbIters; ++it) {
    double acc[kTbU];
#pragma unroll
    for (int u = 0; u < kTbU; ++u) {
      const float E = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ev), it * kTbU + u));
      double a = 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float fn = fmaf(lane_at(cc[it][u], v), E, lane_at(f[it][u], v));
        lane_at(f[it][u], v) = fn;
        a = fma(w[v], (double)fn, a);
      }
      acc[u] = a;
    }
    static_assert(kTbU == 4, "wave_reduce4 sums four rows");
    int which = 0;
    const double tot = wave_reduce4(acc, which);
    // 16-lane row `which` holds the total of slot it * U + which; its first lane reports
    // it if that slot holds a row whose node has a valid E this sub-step
    const int q = it * kTbU + which;
    const int lc = __shfl(tab_loc, q);
    const int has = __shfl(tab_row, q);
    if ((li & 15) == 0 && has && x0 + lc >= lo && x0 + lc < hi) Js[lc] = (float)tot;
  }
}

// Crank-Nicolson coefficients of the eight row slots of a wavefront for rows of 64 lanes:
// d = -2x / (2 + x) and c' = (b / (2 + x)) n per bin, x = dt nu_j (lane q of tab_tau /
// tab_ne holds slot q's dt nu_mean and density; an empty slot has both 0).
__device__ __forceinline__ void tb_coef64(float4 (&dd)[kTbIters][kTbU], float4 (&cc)[kTbIters][kTbU],
                                          const float4& sb, const float4& bb, float tab_tau,
                                          float tab_ne) {
#pragma unroll
  for (int it = 0; it < kTbIters; ++it)
#pragma unroll
    for (int u = 0; u < kTbU; ++u) {
      const float tau = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(tab_tau), it * kTbU + u));
      const float ne = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(tab_ne), it * kTbU + u));
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float r = cn_recip(fmaf(tau, lane_at(sb, v), 2.f));
        lane_at(dd[it][u], v) = -((tau + tau) * lane_at(sb, v)) * r;
        lane_at(cc[it][u], v) = (lane_at(bb, v) * r) * ne;
      }
    }
}

template <int K, int LPC>
__global__ __launch_bounds__(kTbBlock) void k_step1d_tb(const Run1D<float>* __restrict__ runs,
                                                        const Tile1D* __restrict__ tiles,
                                                        int64_t step, int64_t in_off,
    int64_t out_off) {
  __shared__ float Es[2][kTbBlock];
  __shared__ float Hs[2][kTbBlock];
  __shared__ float Js[kTbBlock + 1];        // + a spare slot for rows without a valid E
  __shared__ float tauS[kTbBlock];
  __shared__ float neS[kTbBlock];
  __shared__ int locS[kTbBlock];
  __shared__ float srcS[K];

  const Tile1D tile = tiles[blockIdx.x];
  const Run1D<float>& R = runs[tile.run];
  // source samples of the K sub-steps, evaluated before the F1 rows occupy registers
  if ((int)threadIdx.x < K)
    srcS[threadIdx.x] = (float)source_wave((double)(step + threadIdx.x + 1) * R.dt, R.src_amp,
                                           R.src_w, R.src_tau, R.src_t0);
  const int nx = R.nx;
  const int x0 = tile.node0 - K > 0 ? tile.node0 - K : 0;
  const int x1 = tile.node1 + K < nx + 1 ? tile.node1 + K : nx + 1;
  const int k = threadIdx.x;
  const int i = x0 + k;
  const int par = (int)(step & 1);
  const int ncell = tile.cell1 - tile.cell0;   // plasma nodes of the extended range

  // fields of the extended range, per-cell scalars
  if (i < x1) {
    Es[0][k] = R.E[par][i];
    Hs[0][k] = i < nx ? R.H[par][i] : 0.f;
  }
  Es[1][k] = 0.f;
  Hs[1][k] = 0.f;
  Js[k] = 0.f;
  if (LPC != 64 && k < ncell) {
    const int c = tile.cell0 + k;
    tauS[k] = R.tau[c];
    neS[k] = R.dens[c];
    locS[k] = R.cell_node[c] - x0;
  }

  // F1 rows in registers: lane group `sub` of wavefront `wv`, slot (it, u) holds the row
  // row_slot(it * U + u, wv, sub) of the range
  const int lane = k & 63, wave = k >> 6;
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  constexpr int lpc = LPC;                     // lanes per row (one float4 each)
  constexpr int cpw = 64 / lpc;
  const int sub = lane / lpc, li = lane - sub * lpc;
  // row slot q of lane group `sub` of wavefront w holds plasma row (q * waves + w) * cpw +
  // sub of the range: consecutive rows go to different wavefronts, so every wavefront gets
  // the same number of rows (to one) whatever the range holds
  auto row_slot = [&](int q, int w, int sb) { return (q * kTbWaves + w) * cpw + sb; };
  float4 sb = reinterpret_cast<const float4*>(R.s_bin)[li];
  float4 bb = reinterpret_cast<const float4*>(R.b_bin)[li];
  double w[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) w[v] = R.w_bin[li * 4 + v];
  float4 f[kTbIters][kTbU];
  const float4* __restrict__ dfr = reinterpret_cast<const float4*>(R.df + in_off);
  // one row per wavefront (LPC = 64): lane q of these registers holds the scalars of the
  // wavefront's row slot q, read into scalar registers with v_readlane when needed
  // (an empty slot keeps node 0 of the range, density 0 and no row: its coefficients and
  // F1 stay 0, and it never reports a current)
  int tab_loc = LPC == 64 ? 0 : kTbBlock, tab_row = 0;
  float tab_tau = 0.f, tab_ne = 0.f;
  if constexpr (LPC == 64) {
    if (lane < kTbIters * kTbU) {
      const int cl = row_slot(lane, wv, 0);
      if (cl < ncell) {
        const int c = tile.cell0 + cl;
        tab_loc = R.cell_node[c] - x0;
        tab_tau = R.tau[c];
        tab_ne = R.dens[c];
        tab_row = 1;
      }
    }
  }
#pragma unroll
  for (int it = 0; it < kTbIters; ++it)
#pragma unroll
    for (int u = 0; u < kTbU; ++u) {
      const int cl = row_slot(it * kTbU + u, wv, sub);
      f[it][u] = cl < ncell ? dfr[(size_t)(tile.cell0 + cl) * lpc + li]
                            : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  // Crank-Nicolson coefficients of every row slot, the same for all K steps.  With one
  // row per wavefront: F1' = (F1 + d F1) + c' E, d = -2x / (2 + x), c' = (b / (2 + x)) n
  // (the row's density folded in), both kept; both FMAs update F1 in place.  With shorter rows the per-lane row scalars
  // leave room for one coefficient only (the two would need 141 VGPRs: one work-group
  // per compute unit), and the update keeps the increment form
  // F1 + (b n E - 2x F1) / (2 + x) with 1 / (2 + x) kept.  The one-step kernel takes the
  // same form for the same row length, so the two give the same bits.
  constexpr bool kKeepDC = LPC == 64;
  float4 dd[kTbIters][kTbU], cc[kKeepDC ? kTbIters : 1][kKeepDC ? kTbU : 1];
  if constexpr (kKeepDC) {
    tb_coef64(dd, cc, sb, bb, tab_tau, tab_ne);
    tb_drive64(f, dd);   // the first sub-step's E-independent half
  } else {
#pragma unroll
    for (int it = 0; it < kTbIters; ++it)
#pragma unroll
      for (int u = 0; u < kTbU; ++u) {
        const int cl = row_slot(it * kTbU + u, wv, sub);
        const float tau = cl < ncell ? R.tau[tile.cell0 + cl] : 0.f;
#pragma unroll
        for (int v = 0; v < 4; ++v) lane_at(dd[it][u], v) = cn_recip(fmaf(tau, lane_at(sb, v), 2.f));
      }
  }

  int lo = x0, hi = x1;    // nodes whose E is valid at the start of the sub-step
  const float S = R.S;
  // the run's constants the field phase needs, read once (scalar registers) rather than
  // from the run record in every sub-step
  const int bc = R.bc, src_node = R.src_node, nprobe = R.nprobe, ntap = R.ntap;
  const float mq = R.q;
#pragma unroll 1
  for (int s = 0; s < K; ++s) {
    const int p = s & 1;
    const int64_t gs = step + s;
    __syncthreads();
    if constexpr (LPC == 64) {
      tb_kinetic64(f, cc, w, Es[p], Js, tab_loc, tab_row, x0, lo, hi, li);
    } else {
      // keep the per-row scalars in LDS: re-read each sub-step instead of being hoisted
      // into registers for all rows at once
      asm volatile("" ::: "memory");
      // kinetic update of the rows whose node holds a valid E, FP64 moment -> Js
#pragma unroll
      for (int it = 0; it < kTbIters; ++it) {
        double acc[kTbU];
        int loc[kTbU];
#pragma unroll
        for (int u = 0; u < kTbU; ++u) {
          const int cl = row_slot(it * kTbU + u, wv, sub);
          loc[u] = kTbBlock;            // rows without a valid E report to the spare slot
          bool live = cl < ncell;
          int lc = 0;
          float tau = 0.f, ne = 0.f;
          if (live) {
            lc = locS[cl];
            tau = tauS[cl];
            ne = neS[cl];
            live = x0 + lc >= lo && x0 + lc < hi;
          }
          if (live) {
            loc[u] = lc;
            const float nE = ne * Es[p][lc];
            double a = 0.0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const float fv = lane_at(f[it][u], v);
              // x = dt nu_j; (2 x) = (2 dt nu_mean) s_j exactly
              const float x2 = (tau + tau) * lane_at(sb, v);
              const float t = fmaf(-x2, fv, lane_at(bb, v) * nE);
              const float fn = fmaf(t, lane_at(dd[it][u], v), fv);
              lane_at(f[it][u], v) = fn;
              a = fma(w[v], (double)fn, a);
            }
            acc[u] = a;
          } else {
            acc[u] = 0.0;
          }
        }
        int which = 0;
        const double tot = group_reduce4_dpp<LPC>(acc, which);
#pragma unroll
        for (int u = 0; u < kTbU; ++u)
          if (li == u * (LPC / 4)) Js[loc[u]] = (float)tot;
      }
    }
    __syncthreads();

    // H^{n+1/2} on [lo, hi - 1), E^{n+1} on the next valid range
    const int nlo = lo == 0 ? 0 : lo + 1;
    const int nhi = hi == nx + 1 ? nx + 1 : hi - 1;
    tb_fields(R, tile, Es, Hs, Js, srcS[s], k, i, p, lo, hi, nlo, nhi, nx, S, bc, mq, src_node,
              nprobe, ntap, gs);
    // the next sub-step's E-independent half runs while wavefront 0 updates the fields
    if constexpr (LPC == 64)
      if (s + 1 < K) tb_drive64(f, dd);
    lo = nlo;
    hi = nhi;
  }
  __syncthreads();

  // owned nodes and their F1 rows back to HBM (the other field buffer)
  constexpr int pf = K & 1;
  if (i >= tile.node0 && i < tile.node1) {
    R.E[par ^ 1][i] = Es[pf][k];
    if (i < nx) R.H[par ^ 1][i] = Hs[pf][k];
    R.J[i] = Js[k];
  }
  // the row addresses are formed again here rather than kept live across the K steps
  asm volatile("" ::: "memory");
  float4* __restrict__ dfw = reinterpret_cast<float4*>(R.df + out_off);
#pragma unroll
  for (int it = 0; it < kTbIters; ++it)
#pragma unroll
    for (int u = 0; u < kTbU; ++u) {
      const int cl = row_slot(it * kTbU + u, wv, sub);
      if (cl < ncell) {
        const int node =
            x0 + (LPC == 64 ? __builtin_amdgcn_readlane(tab_loc, it * kTbU + u) : locS[cl]);
        if (node >= tile.node0 && node < tile.node1)
          dfw[(size_t)(tile.cell0 + cl) * lpc + li] = f[it][u];
      }
    }
}

bool tb_supported(int half) { return half == 32 || half == 64 || half == 128 || half == 256; }

int tb_block() { return kTbBlock; }

// Plasma rows one work-group holds for rows of `half` stored bins.
int tb_max_rows(int half) {
  const int lpc = half / 4;
  return kTbWaves * (64 / lpc) * kTbRowsPerGroup;
}

template <int K, int LPC>
int tb_occupancy() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step1d_tb<K, LPC>, kTbBlock, 0) != hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

template <int K>
int tb_occupancy_k(int half) {
  switch (half) {
    case 32: return tb_occupancy<K, 8>();
    case 64: return tb_occupancy<K, 16>();
    case 128: return tb_occupancy<K, 32>();
    default: return tb_occupancy<K, 64>();
  }
}

int tb_blocks_per_cu(int k, int half) {
  switch (k) {
    case 3: return tb_occupancy_k<3>(half);
    case 5: return tb_occupancy_k<5>(half);
    case 7: return tb_occupancy_k<7>(half);
    default: return tb_occupancy_k<9>(half);
  }
}

template <int K>
hipError_t launch_tb_k(const Run1D<float>* r, const Tile1D* t, int ntiles, int64_t step, int half, int64_t in_off, int64_t out_off,
                       hipStream_t stream) {
  switch (half) {
    case 32: hipLaunchKernelGGL((k_step1d_tb<K, 8>), dim3(ntiles), dim3(kTbBlock), 0, stream, r, t, step, in_off, out_off); break;
    case 64: hipLaunchKernelGGL((k_step1d_tb<K, 16>), dim3(ntiles), dim3(kTbBlock), 0, stream, r, t, step, in_off, out_off); break;
    case 128: hipLaunchKernelGGL((k_step1d_tb<K, 32>), dim3(ntiles), dim3(kTbBlock), 0, stream, r, t, step, in_off, out_off); break;
    case 256: hipLaunchKernelGGL((k_step1d_tb<K, 64>), dim3(ntiles), dim3(kTbBlock), 0, stream, r, t, step, in_off, out_off); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// K steps [step, step + K) of the tiles (every tile of one run, half = Nv/2 of that run).
hipError_t launch_step1d_tb(const void* runs, const void* tiles, int ntiles, int64_t step, int k,
                            int half, int64_t in_off, int64_t out_off, hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  const Run1D<float>* r = static_cast<const Run1D<float>*>(runs);
  const Tile1D* t = static_cast<const Tile1D*>(tiles);
  switch (k) {
    case 3: return launch_tb_k<3>(r, t, ntiles, step, half, in_off, out_off, stream);
    case 5: return launch_tb_k<5>(r, t, ntiles, step, half, in_off, out_off, stream);
    case 7: return launch_tb_k<7>(r, t, ntiles, step, half, in_off, out_off, stream);
    case 9: return launch_tb_k<9>(r, t, ntiles, step, half, in_off, out_off, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fdtdp
