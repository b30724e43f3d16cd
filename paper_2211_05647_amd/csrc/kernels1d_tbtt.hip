// kernels1d_tbtt.hip -- K leap-frog steps per launch of the 1D line with the two-term model
// of every plasma node (arXiv 2211.05647, section 5.1 expansion with the l = 0 and l = 1
// equations, section 5.3 speed grid): temporal blocking with halo recomputation, as for
// the linear model (the kinetic step has no spatial coupling, so K steps of a node depend
// on the fields and rows within K nodes of it).
//
// A work-group owns nodes [node0, node1), holds the fields of the range extended by K
// nodes per side in LDS and the [F1 | F0 - n F0hat] rows of its plasma nodes in registers,
// and takes them through K steps.  Each sub-step: the previous sub-step's l = 0 update of
// F0 (E time-centred: E^{n-1} is still in the other LDS buffer), the F1 update (drive with
// the central difference of F0 - n F0hat) and the FP64 moment; then H and E.  After the
// last sub-step its l = 0 update is applied too, so that F0 is complete when the launch
// ends; every update takes the operands of the one-step kernel's (which defers the l = 0
// update the same way, across launches), so a blocked run is bitwise the one-step run.
//
// As in the linear blocked kernel, rows are read from one copy and written to the other
// (in_off, out_off), so that no work-group reads halo rows a neighbour already advanced.
//
// Requirements (checked on the host): FP32 storage, `half` (speeds padded to a power of
// two) 32 or 64 (one 16-byte chunk of F1 and one of F0 per lane, 8 or 16 lanes per row), K
// odd, extended ranges of at most kTtBlock nodes and tb_tt_max_rows(half) plasma nodes, no
// l = 0 update pending at launch.
#include "common.h"
#include "host_internal.h"

namespace fdtdp {

constexpr int kTtBlock = 512;               // threads per work-group (8 wavefronts)
constexpr int kTtWaves = kTtBlock / 64;
constexpr int kTtU = 4;                     // row slots per lane group

template <int K, int LPC>
__global__ __launch_bounds__(kTtBlock) void k_step1d_tb_tt(const Run1D<float>* __restrict__ runs,
                                                           const Tile1D* __restrict__ tiles,
                                                           int64_t step, int64_t in_off,
    int64_t out_off) {
  __shared__ float Es[2][kTtBlock];
  __shared__ float Hs[2][kTtBlock];
  __shared__ float Js[kTtBlock];
  __shared__ float tauS[kTtBlock];
  __shared__ float neS[kTtBlock];
  __shared__ int locS[kTtBlock];
  __shared__ float srcS[K];

  const Tile1D tile = tiles[blockIdx.x];
  const Run1D<float>& R = runs[tile.run];
  if ((int)threadIdx.x < K)
    srcS[threadIdx.x] = (float)source_wave((double)(step + threadIdx.x + 1) * R.dt, R.src_amp,
                                           R.src_w, R.src_tau, R.src_t0);
  const int nx = R.nx;
  const int x0 = tile.node0 - K > 0 ? tile.node0 - K : 0;
  const int x1 = tile.node1 + K < nx + 1 ? tile.node1 + K : nx + 1;
  const int k = threadIdx.x;
  const int i = x0 + k;
  const int par = (int)(step & 1);
  const int ncell = tile.cell1 - tile.cell0;

  if (i < x1) {
    Es[0][k] = R.E[par][i];
    Hs[0][k] = i < nx ? R.H[par][i] : 0.f;
  }
  Es[1][k] = 0.f;
  Hs[1][k] = 0.f;
  Js[k] = 0.f;
  if (k < ncell) {
    const int c = tile.cell0 + k;
    tauS[k] = R.tau[c];
    neS[k] = R.dens[c];
    locS[k] = R.cell_node[c] - x0;
  }

  const int lane = k & 63, wave = k >> 6;
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  constexpr int cpw = 64 / LPC;
  const int sub = lane / LPC, li = lane - sub * LPC;
  const bool first_lane = li == 0, last_lane = li == LPC - 1;
  // slot q of lane group `sub` of wavefront w holds plasma row (q * waves + w) * cpw + sub
  auto row_slot = [&](int q, int w, int sb) { return (q * kTtWaves + w) * cpw + sb; };
  float4 sb = reinterpret_cast<const float4*>(R.s_bin)[li];
  float4 bb = reinterpret_cast<const float4*>(R.b_bin)[li];
  float4 cf = reinterpret_cast<const float4*>(R.c_bin)[li];
  float4 vh = reinterpret_cast<const float4*>(R.v2h_bin)[li];
  double w[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) w[v] = R.w_bin[li * 4 + v];
  const float kd = R.kc;
  float4 f[kTtU], d[kTtU];
  const float4* __restrict__ dfr = reinterpret_cast<const float4*>(R.df + in_off);
#pragma unroll
  for (int u = 0; u < kTtU; ++u) {
    const int cl = row_slot(u, wv, sub);
    const size_t row = (size_t)(tile.cell0 + cl) * (2 * LPC);
    f[u] = cl < ncell ? dfr[row + li] : make_float4(0.f, 0.f, 0.f, 0.f);
    d[u] = cl < ncell ? dfr[row + LPC + li] : make_float4(0.f, 0.f, 0.f, 0.f);
  }

  // l = 0 update of slot u (F1 at n+1/2 in registers): F0 += c_k Ebar (phi_{k+1/2} -
  // phi_{k-1/2}), phi = (v^2/2)(F1_k + F1_{k+1}) on the inner faces, Ebar = (E^n + E^{n+1})
  // / 2 (eb); every lane takes part in the shuffles, `live` rows change
  auto l0_update = [&](int u, bool live, float Eb) {
    // no contraction of v^2 (F1_k + F1_{k+1}) into the flux difference, as in the
    // one-step kernel
#pragma clang fp contract(off)
    const float nf = from_next_lane(f[u].x);
    float ph[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float fr = v < 3 ? lane_at(f[u], v < 3 ? v + 1 : v) : (last_lane ? 0.f : nf);
      ph[v] = lane_at(vh, v) * (lane_at(f[u], v) + fr);   // 0 on the top face
    }
    const float got = from_prev_lane(ph[3]);
    if (live) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float pl = v > 0 ? ph[v > 0 ? v - 1 : 0] : (first_lane ? 0.f : got);
        lane_at(d[u], v) = fmaf(lane_at(cf, v) * Eb, ph[v] - pl, lane_at(d[u], v));
      }
    }
  };

  int lo = x0, hi = x1;
  const float S = R.S;
#pragma unroll 1
  for (int s = 0; s < K; ++s) {
    const int p = s & 1;
    const int64_t gs = step + s;
    __syncthreads();
    asm volatile("" ::: "memory");
    // the previous sub-step's l = 0 update (E^{n-1} is still in the other buffer), then
    // F1^{n+1/2} of the rows whose node holds a valid E^n, FP64 moment -> Js
#pragma unroll
    for (int u = 0; u < kTtU; ++u) {
      const int cl = row_slot(u, wv, sub);
      bool live = cl < ncell;
      int lc = 0;
      float tau = 0.f, ne = 0.f, Ev = 0.f;
      if (live) {
        lc = locS[cl];
        live = x0 + lc >= lo && x0 + lc < hi;
      }
      if (live) {
        tau = tauS[cl];
        ne = neS[cl];
        Ev = Es[p][lc];
      }
      if (s > 0) l0_update(u, live, live ? 0.5f * (Es[p ^ 1][lc] + Ev) : 0.f);
      // d_{k+1} from the next lane, d_{k-1} from the previous one (every lane takes part;
      // DPP row shifts: the values the one-step kernel's lane shuffles fetch)
      const float nd = from_next_lane(d[u].x);
      const float pd = from_prev_lane(d[u].w);
      const float nE = ne * Ev, kE = kd * Ev, tau2 = tau + tau;
      if (live && first_lane && !(fabsf(kE) <= 1.f)) atomicOr(R.status, 2);
      double acc = 0.0;
      if (live) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float dr = v < 3 ? lane_at(d[u], v < 3 ? v + 1 : v) : (last_lane ? 0.f : nd);
          const float dl = v > 0 ? lane_at(d[u], v > 0 ? v - 1 : 0)
                                 : (first_lane ? lane_at(d[u], 0) : pd);   // even at v = 0
          const float sv = lane_at(sb, v);
          const float r = cn_recip(fmaf(tau, sv, 2.f));
          const float fv = lane_at(f[u], v);
          const float drive =
              lane_at(cf, v) != 0.f ? fmaf(kE, dr - dl, lane_at(bb, v) * nE) : 0.f;
          const float t = fmaf(-(tau2 * sv), fv, drive);
          const float fn = fmaf(t, r, fv);
          lane_at(f[u], v) = fn;
          acc = fma(w[v], (double)fn, acc);
        }
      }
      const double tot = group_allreduce_dpp<LPC>(acc);
      if (live && first_lane) Js[lc] = (float)tot;
    }
    __syncthreads();

    // H^{n+1/2} on [lo, hi - 1), E^{n+1} on the next valid range
    const int nlo = lo == 0 ? 0 : lo + 1;
    const int nhi = hi == nx + 1 ? nx + 1 : hi - 1;
    if (i >= lo && i < hi) {
      const float e0 = Es[p][k];
      const float jv = Js[k];
      float en = 0.f, hn = 0.f;
      const bool has_e = i >= nlo && i < nhi;
      if (i == 0) {
        const float ep = Es[p][k + 1], h0 = Hs[p][k];
        hn = h_update(h0, S, ep, e0);
        if (R.bc == 1) {
          const float h1 = h_update(Hs[p][k + 1], S, Es[p][k + 2], ep);
          const float e1 = e_update(ep, S, h1, hn, 0.f);
          en = fmaf(R.q, e1 - e0, ep);
        }
        Hs[p ^ 1][k] = hn;
      } else if (i == nx) {
        if (R.bc == 1) {
          const float em = Es[p][k - 1], hm = Hs[p][k - 1];
          const float ha = h_update(hm, S, e0, em);
          const float hb = h_update(Hs[p][k - 2], S, em, Es[p][k - 2]);
          const float e = e_update(em, S, ha, hb, 0.f);
          en = fmaf(R.q, e - e0, em);
        }
      } else {
        if (i < hi - 1) {
          hn = h_update(Hs[p][k], S, Es[p][k + 1], e0);
          Hs[p ^ 1][k] = hn;
        }
        if (has_e) {
          const float hl = h_update(Hs[p][k - 1], S, e0, Es[p][k - 1]);
          en = e_update(e0, S, hn, hl, jv);
          if (i == R.src_node) en += srcS[s];
        }
      }
      if (has_e) Es[p ^ 1][k] = en;
      if (has_e && i >= tile.node0 && i < tile.node1) {
        if (!isfinite(en)) atomicOr(R.status, 1);
        for (int q = 0; q < R.nprobe; ++q) {
          if (R.probe_node[q] == i) {
            const int fld = R.probe_field[q];
            const float val = (fld == 0) ? en : (fld == 1 ? hn : jv);
            R.probe_buf[(size_t)q * R.probe_cap + (size_t)(gs % R.probe_cap)] = val;
          }
        }
        for (int t = 0; t < R.ntap; ++t) {
          if (R.tap_node[t] == i && gs < R.tap_cap) {
            float* dst = R.tap_buf + ((size_t)t * R.tap_cap + (size_t)gs) * 2;
            dst[0] = e0;
            dst[1] = jv;
          }
        }
      }
    }
    lo = nlo;
    hi = nhi;
  }
  __syncthreads();

  // the last sub-step's l = 0 update: E^{n+K} in buffer pf, E^{n+K-1} in the other
  constexpr int pf = K & 1;
#pragma unroll
  for (int u = 0; u < kTtU; ++u) {
    const int cl = row_slot(u, wv, sub);
    bool live = cl < ncell;
    int lc = 0;
    if (live) {
      lc = locS[cl];
      live = x0 + lc >= lo && x0 + lc < hi;
    }
    l0_update(u, live, live ? 0.5f * (Es[pf ^ 1][lc] + Es[pf][lc]) : 0.f);
  }

  // owned nodes and their rows back to HBM (the other field buffer)
  if (i >= tile.node0 && i < tile.node1) {
    R.E[par ^ 1][i] = Es[pf][k];
    if (i < nx) R.H[par ^ 1][i] = Hs[pf][k];
    R.J[i] = Js[k];
  }
  float4* __restrict__ dfw = reinterpret_cast<float4*>(R.df + out_off);
#pragma unroll
  for (int u = 0; u < kTtU; ++u) {
    const int cl = row_slot(u, wv, sub);
    if (cl < ncell) {
      const int node = x0 + locS[cl];
      if (node >= tile.node0 && node < tile.node1) {
        const size_t row = (size_t)(tile.cell0 + cl) * (2 * LPC);
        dfw[row + li] = f[u];
        dfw[row + LPC + li] = d[u];
      }
    }
  }
}

bool tb_tt_supported(int half) { return half == 32 || half == 64; }

int tb_tt_max_rows(int half) { return kTtWaves * (64 / (half / 4)) * kTtU; }

template <int K, int LPC>
int tb_tt_occupancy() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step1d_tb_tt<K, LPC>, kTtBlock, 0) !=
      hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

int tb_tt_blocks_per_cu(int k, int half) {
  const bool h64 = half == 64;
  switch (k) {
    case 3: return h64 ? tb_tt_occupancy<3, 16>() : tb_tt_occupancy<3, 8>();
    case 5: return h64 ? tb_tt_occupancy<5, 16>() : tb_tt_occupancy<5, 8>();
    case 7: return h64 ? tb_tt_occupancy<7, 16>() : tb_tt_occupancy<7, 8>();
    default: return h64 ? tb_tt_occupancy<9, 16>() : tb_tt_occupancy<9, 8>();
  }
}

template <int K>
hipError_t launch_tb_tt_k(const Run1D<float>* r, const Tile1D* t, int ntiles, int64_t step,
                          int half, int64_t in_off, int64_t out_off, hipStream_t stream) {
  switch (half) {
    case 32: hipLaunchKernelGGL((k_step1d_tb_tt<K, 8>), dim3(ntiles), dim3(kTtBlock), 0, stream, r, t, step, in_off, out_off); break;
    case 64: hipLaunchKernelGGL((k_step1d_tb_tt<K, 16>), dim3(ntiles), dim3(kTtBlock), 0, stream, r, t, step, in_off, out_off); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// K steps [step, step + K) of the tiles of a two-term run, F0 complete before and after.
hipError_t launch_step1d_tb_tt(const void* runs, const void* tiles, int ntiles, int64_t step,
                               int k, int half, int64_t in_off, int64_t out_off, hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  const Run1D<float>* r = static_cast<const Run1D<float>*>(runs);
  const Tile1D* t = static_cast<const Tile1D*>(tiles);
  switch (k) {
    case 3: return launch_tb_tt_k<3>(r, t, ntiles, step, half, in_off, out_off, stream);
    case 5: return launch_tb_tt_k<5>(r, t, ntiles, step, half, in_off, out_off, stream);
    case 7: return launch_tb_tt_k<7>(r, t, ntiles, step, half, in_off, out_off, stream);
    case 9: return launch_tb_tt_k<9>(r, t, ntiles, step, half, in_off, out_off, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fdtdp
