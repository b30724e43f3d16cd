// kernels1d_tbfull.hip -- K leap-frog steps per launch of the 1D line with the
// full-distribution 1V model of every plasma node (the whole f evolves under
// df/dt - (e/m) E df/dv = C(f): arXiv 2211.05647 section 5.1 without the streaming and
// magnetic terms, elastic collisions on the odd part as in section 5.2): temporal blocking
// with halo recomputation, as for the linear and two-term models (the kinetic step has no
// spatial coupling).
//
// A work-group owns nodes [node0, node1), holds the fields of the range extended by K
// nodes per side in LDS and the [odd | even] rows of its plasma nodes in registers (8 row
// slots per lane group), and takes them through K steps.  Each sub-step updates a row with
// the same operations, in the same order, as the one-step kernel's tile (odd pass with the
// Lax-Wendroff corrected faces, even pass from the time-centred odd part, FP64 moment with
// the same DPP reduction tree), then H and E, so that a blocked run is bitwise the one-step
// run.  Rows are read from one copy and written to the other (in_off, out_off), so that no
// work-group reads halo rows a neighbour of the same launch already advanced.
//
// Requirements (checked on the host): FP32 storage, Nv/2 stored bins of each half in
// {32, 64, 128, 256} (one 16-byte chunk of each half per lane), K odd, extended ranges of at
// most kTfBlock nodes and tb_full_max_rows(half) plasma nodes.
#include "common.h"
#include "host_internal.h"

namespace fdtdp {

constexpr int kTfBlock = 512;               // threads per work-group (8 wavefronts)
constexpr int kTfWaves = kTfBlock / 64;
constexpr int kTfSlots = 8;                 // row slots per lane group

template <int K, int LPC>
__global__ __launch_bounds__(kTfBlock) void k_step1d_tb_full(
    const Run1D<float>* __restrict__ runs, const Tile1D* __restrict__ tiles, int64_t step,
    int64_t in_off, int64_t out_off) {
  __shared__ float Es[2][kTfBlock];
  __shared__ float Hs[2][kTfBlock];
  __shared__ float Js[kTfBlock];
  __shared__ float tauS[kTfBlock];
  __shared__ float neS[kTfBlock];
  __shared__ int locS[kTfBlock];
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
  auto row_slot = [&](int q, int w, int sb) { return (q * kTfWaves + w) * cpw + sb; };
  float4 sb = reinterpret_cast<const float4*>(R.s_bin)[li];
  float4 bb = reinterpret_cast<const float4*>(R.b_bin)[li];
  double w[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) w[v] = R.w_bin[li * 4 + v];
  const float kc = R.kc;
  float4 o[kTfSlots], e[kTfSlots];
  const float4* __restrict__ dfr = reinterpret_cast<const float4*>(R.df + in_off);
#pragma unroll
  for (int u = 0; u < kTfSlots; ++u) {
    const int cl = row_slot(u, wv, sub);
    const size_t row = (size_t)(tile.cell0 + cl) * (2 * LPC);
    o[u] = cl < ncell ? dfr[row + li] : make_float4(0.f, 0.f, 0.f, 0.f);
    e[u] = cl < ncell ? dfr[row + LPC + li] : make_float4(0.f, 0.f, 0.f, 0.f);
  }

  int lo = x0, hi = x1;
  const float S = R.S;
#pragma unroll 1
  for (int s = 0; s < K; ++s) {
    const int p = s & 1;
    const int64_t gs = step + s;
    __syncthreads();
    asm volatile("" ::: "memory");
    // the rows whose node holds a valid E^n: odd and even passes, FP64 moment -> Js
#pragma unroll
    for (int u = 0; u < kTfSlots; ++u) {
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
      const float cf = kc * Ev;
      if (live && first_lane && !(fabsf(cf) <= 1.f)) atomicOr(R.status, 2);
      const float ch2 = 0.5f * cf, cc2 = 0.5f * cf * cf, cq = 0.25f * cf;
      const float nE = ne * Ev;
      // odd pass: perturbation face fluxes right of every bin
      float pr[4];
      {
        const float no = next_lane_of_row(o[u].x, LPC);
        const float nev = next_lane_of_row(e[u].x, LPC);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          float orr, er;
          bool outer = false;
          if (v < 3) {
            orr = lane_at(o[u], v < 3 ? v + 1 : v);
            er = lane_at(e[u], v < 3 ? v + 1 : v);
          } else if (!last_lane) {
            orr = no;
            er = nev;
          } else {
            orr = er = 0.f;
            outer = true;
          }
          const float ol = lane_at(o[u], v), el = lane_at(e[u], v);
          pr[v] = outer ? 0.f : fmaf(ch2, el + er, -cc2 * (orr - ol));
        }
      }
      float pl0;
      {
        const float got = prev_lane_of_row(pr[3], LPC);
        const float pc = fmaf(cf, lane_at(e[u], 0), -cf * cf * lane_at(o[u], 0));  // v = 0
        pl0 = !first_lane ? got : pc;
      }
      float4 on;
      float sm[4];
      double acc = 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float pl = v == 0 ? pl0 : pr[v > 0 ? v - 1 : 0];
        const float sv = lane_at(sb, v);
        const float r = cn_recip(fmaf(tau, sv, 2.f));
        const float x2 = (tau + tau) * sv;
        const float ov = lane_at(o[u], v);
        const float t = fmaf(-x2, ov, fmaf(lane_at(bb, v), nE, -2.f * (pr[v] - pl)));
        const float onv = fmaf(t, r, ov);
        lane_at(on, v) = onv;
        sm[v] = ov + onv;
        acc = fma(w[v], (double)onv, acc);
      }
      // even pass: faces of the time-centred odd part
      {
#pragma clang fp contract(off)
        float qr[4];
        const float ns = next_lane_of_row(sm[0], LPC);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          float sr;
          bool outer = false;
          if (v < 3) sr = sm[v < 3 ? v + 1 : v];
          else if (!last_lane) sr = ns;
          else { sr = 0.f; outer = true; }
          qr[v] = outer ? 0.f : cq * (sm[v] + sr);
        }
        const float got = prev_lane_of_row(qr[3], LPC);
        const float ql0 = !first_lane ? got : 0.f;
        if (live) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const float ql = v == 0 ? ql0 : qr[v > 0 ? v - 1 : 0];
            lane_at(e[u], v) = lane_at(e[u], v) - (qr[v] - ql);
          }
          o[u] = on;
        }
      }
      const double tot = row_sum_dpp(acc, LPC, li);
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

  // owned nodes and their rows back to HBM (the other field buffer, the other row copy)
  constexpr int pf = K & 1;
  if (i >= tile.node0 && i < tile.node1) {
    R.E[par ^ 1][i] = Es[pf][k];
    if (i < nx) R.H[par ^ 1][i] = Hs[pf][k];
    R.J[i] = Js[k];
  }
  float4* __restrict__ dfw = reinterpret_cast<float4*>(R.df + out_off);
#pragma unroll
  for (int u = 0; u < kTfSlots; ++u) {
    const int cl = row_slot(u, wv, sub);
    if (cl < ncell) {
      const int node = x0 + locS[cl];
      if (node >= tile.node0 && node < tile.node1) {
        const size_t row = (size_t)(tile.cell0 + cl) * (2 * LPC);
        dfw[row + li] = o[u];
        dfw[row + LPC + li] = e[u];
      }
    }
  }
}

bool tb_full_supported(int half) { return half == 32 || half == 64 || half == 128 || half == 256; }

int tb_full_max_rows(int half) { return kTfWaves * (64 / (half / 4)) * kTfSlots; }

template <int K, int LPC>
int tb_full_occupancy() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step1d_tb_full<K, LPC>, kTfBlock, 0) !=
      hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

template <int K>
int tb_full_occupancy_k(int half) {
  switch (half) {
    case 32: return tb_full_occupancy<K, 8>();
    case 64: return tb_full_occupancy<K, 16>();
    case 128: return tb_full_occupancy<K, 32>();
    default: return tb_full_occupancy<K, 64>();
  }
}

int tb_full_blocks_per_cu(int k, int half) {
  switch (k) {
    case 3: return tb_full_occupancy_k<3>(half);
    case 5: return tb_full_occupancy_k<5>(half);
    case 7: return tb_full_occupancy_k<7>(half);
    default: return tb_full_occupancy_k<9>(half);
  }
}

template <int K>
hipError_t launch_tb_full_k(const Run1D<float>* r, const Tile1D* t, int ntiles, int64_t step,
                            int half, int64_t in_off, int64_t out_off, hipStream_t stream) {
  switch (half) {
    case 32: hipLaunchKernelGGL((k_step1d_tb_full<K, 8>), dim3(ntiles), dim3(kTfBlock), 0, stream, r, t, step, in_off, out_off); break;
    case 64: hipLaunchKernelGGL((k_step1d_tb_full<K, 16>), dim3(ntiles), dim3(kTfBlock), 0, stream, r, t, step, in_off, out_off); break;
    case 128: hipLaunchKernelGGL((k_step1d_tb_full<K, 32>), dim3(ntiles), dim3(kTfBlock), 0, stream, r, t, step, in_off, out_off); break;
    case 256: hipLaunchKernelGGL((k_step1d_tb_full<K, 64>), dim3(ntiles), dim3(kTfBlock), 0, stream, r, t, step, in_off, out_off); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// K steps [step, step + K) of the tiles of a full-distribution run.
hipError_t launch_step1d_tb_full(const void* runs, const void* tiles, int ntiles, int64_t step,
                                 int k, int half, int64_t in_off, int64_t out_off,
                                 hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  const Run1D<float>* r = static_cast<const Run1D<float>*>(runs);
  const Tile1D* t = static_cast<const Tile1D*>(tiles);
  switch (k) {
    case 3: return launch_tb_full_k<3>(r, t, ntiles, step, half, in_off, out_off, stream);
    case 5: return launch_tb_full_k<5>(r, t, ntiles, step, half, in_off, out_off, stream);
    case 7: return launch_tb_full_k<7>(r, t, ntiles, step, half, in_off, out_off, stream);
    case 9: return launch_tb_full_k<9>(r, t, ntiles, step, half, in_off, out_off, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fdtdp
