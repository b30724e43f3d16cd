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

// The source sample of step n + 1 as a real call: inside the persistent launch's item
// loop, an inlined FP64 sin / exp would have its polynomial constants hoisted out of the
// loop and held in some forty registers for the whole launch.
__device__ __attribute__((noinline)) float tb_source_sample(const Run1D<float>& R, int64_t n) {
  return (float)source_wave((double)(n + 1) * R.dt, R.src_amp, R.src_w, R.src_tau, R.src_t0);
}

// On-chip state of one tile (LDS).
template <int K> struct TbLds {
  float Es[2][kTbBlock];
  float Hs[2][kTbBlock];
  float Js[kTbBlock + 1];        // + a spare slot for rows without a valid E
  float tauS[kTbBlock];
  float neS[kTbBlock];
  int locS[kTbBlock];
  float srcS[K];
};

// ns (odd, at most K) steps [step, step + ns) of one tile of run R by the whole work-group:
// the fields and rows of the extended range (halo of K nodes per side) are read, the owned
// nodes' fields go to field buffer (step & 1) ^ 1 and their rows from copy in_off to copy
// out_off.  k is the thread's index in the work-group.  The caller orders LDS use between
// tiles (a barrier before the next tile).
template <int K, int LPC>
__device__ __forceinline__ void tb_tile(const Run1D<float>& R, const Tile1D& tile, int64_t step,
                                        int ns, int64_t in_off, int64_t out_off,
                                        TbLds<K>& L, const int k) {
  auto& Es = L.Es;
  auto& Hs = L.Hs;
  auto& Js = L.Js;
  auto& tauS = L.tauS;
  auto& neS = L.neS;
  auto& locS = L.locS;
  auto& srcS = L.srcS;
  // source samples of the ns sub-steps, evaluated before the F1 rows occupy registers
  if (k < ns) srcS[k] = tb_source_sample(R, step + k);
  const int nx = R.nx;
  const int x0 = tile.node0 - K > 0 ? tile.node0 - K : 0;
  const int x1 = tile.node1 + K < nx + 1 ? tile.node1 + K : nx + 1;
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
  // Crank-Nicolson coefficients of every row slot, the same for all sub-steps.  With one
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
  for (int s = 0; s < ns; ++s) {
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
      if (s + 1 < ns) tb_drive64(f, dd);
    lo = nlo;
    hi = nhi;
  }
  __syncthreads();

  // owned nodes and their F1 rows back to HBM (the other field buffer)
  const int pf = ns & 1;
  if (i >= tile.node0 && i < tile.node1) {
    R.E[par ^ 1][i] = Es[pf][k];
    if (i < nx) R.H[par ^ 1][i] = Hs[pf][k];
    R.J[i] = Js[k];
  }
  // the row addresses are formed again here rather than kept live across the sub-steps
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

template <int K, int LPC>
__global__ __launch_bounds__(kTbBlock) void k_step1d_tb(const Run1D<float>* __restrict__ runs,
                                                        const Tile1D* __restrict__ tiles,
                                                        int64_t step, int64_t in_off,
                                                        int64_t out_off) {
  __shared__ TbLds<K> L;
  const Tile1D tile = tiles[blockIdx.x];
  tb_tile<K, LPC>(runs[tile.run], tile, step, K, in_off, out_off, L, (int)threadIdx.x);
}

// --- persistent batch launch -------------------------------------------------------
// One launch takes every run of a batch through steps [s0, s1) (each run to its own step
// limit).  Work items are (tile, block) pairs: block b of a tile takes its run through
// K steps, and at the run's end through the rest of its steps, as one block if the rest
// is odd, else as rest - 1 steps and then 1 (a block must be odd: it reads field buffer
// step & 1 and writes the other).  Items are numbered round by round -- block b of every
// tile that has one, then block b + 1 -- with the runs of the most blocks first, so the
// tiles of round b are a prefix of the tile array, and rounds with the same number of
// active tiles form a segment (at most one per run).  Work-groups take items in order
// from a counter.  Block b of a tile may start once the tile and its neighbours in the
// same run have finished block b - 1: their outputs are its inputs, and they no longer
// read the field buffer and row copy it writes.  A work-group makes every store of a
// block visible device-wide before it records the block in `done`.  Items are handed out
// in order, so the lowest unfinished item waits on none: the launch drains whatever the
// number of work-groups resident.  A wait longer than kQueueSpinLimit polls gives up: it
// sets bit 2 of the run's status (the batch's results are then void) and moves the
// counter past the last item, so that every work-group leaves after at most its current
// and prefetched items, rather than hang.
struct TbQueue {
  const TbQueueTile* tiles;     // [ntiles] runs with the most blocks first, each in node order
  const int64_t* seg_start;     // [nseg + 1] first item of each segment; [nseg] = all items
  const int32_t* seg_round;     // [nseg] first round of each segment
  const int32_t* seg_tiles;     // [nseg] tiles per round in each segment
  int32_t* done;                // [ntiles] blocks finished per tile (0 at launch)
  unsigned long long* counter;  // next item (0 at launch)
  int64_t s0, s1;               // steps of the launch
  int64_t delta;                // FP32 elements from a run's rows to their second copy
  int32_t nseg;
};

constexpr int kQueueSpinLimit = 1 << 18;
constexpr int kQueueSegLds = 256;   // segment tables up to this size are read from LDS

template <int K>
__global__ __launch_bounds__(kTbBlock, 4) void k_batch1d_queue(const Run1D<float>* __restrict__ runs,
                                                            TbQueue Q) {
  __shared__ TbLds<K> L;
  __shared__ int32_t item_t, item_b, item_ns;
  __shared__ int64_t item_step;
  __shared__ int64_t sg_start[kQueueSegLds + 1];
  __shared__ int32_t sg_round[kQueueSegLds], sg_tiles[kQueueSegLds];
  const bool sg_lds = Q.nseg <= kQueueSegLds;
  if (sg_lds) {
    for (int i = threadIdx.x; i <= Q.nseg; i += kTbBlock) {
      sg_start[i] = Q.seg_start[i];
      if (i < Q.nseg) {
        sg_round[i] = Q.seg_round[i];
        sg_tiles[i] = Q.seg_tiles[i];
      }
    }
  }
  __syncthreads();
  const int64_t total = Q.seg_start[Q.nseg];
  unsigned long long next = 0;   // thread 0: the item after the current one, fetched ahead
  int seg = 0;                   // thread 0: segment of the current item (items only grow)
  if (threadIdx.x == 0) next = atomicAdd(Q.counter, 1ull);
  for (;;) {
    if (threadIdx.x == 0) {
      const int64_t qi = (int64_t)next;
      int b = -1, t = 0, ns = 0;
      int64_t st = 0;
      if (qi < total) {
        next = atomicAdd(Q.counter, 1ull);
        if (sg_lds) {
          while (sg_start[seg + 1] <= qi) ++seg;
        } else {
          while (Q.seg_start[seg + 1] <= qi) ++seg;
        }
        const int64_t off = qi - (sg_lds ? sg_start[seg] : Q.seg_start[seg]);
        const int nt = sg_lds ? sg_tiles[seg] : Q.seg_tiles[seg];
        const int64_t r = off / nt;
        b = (sg_lds ? sg_round[seg] : Q.seg_round[seg]) + (int)r;
        t = (int)(off - r * nt);
        const TbQueueTile qt = Q.tiles[t];
        const int64_t q = qt.full, rest = qt.rest;
        if (b < q) {
          st = Q.s0 + (int64_t)b * K;
          ns = K;
        } else if (rest & 1) {
          st = Q.s0 + q * K;
          ns = (int)rest;
        } else if (b == q) {
          st = Q.s0 + q * K;
          ns = (int)rest - 1;
        } else {
          st = Q.s0 + q * K + rest - 1;
          ns = 1;
        }
        const bool left = qt.tile.node0 > 0, right = (qt.flags & 1) != 0;
        for (int spin = 0;; ++spin) {
          bool ok = __hip_atomic_load(Q.done + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= b;
          if (left)
            ok = ok && __hip_atomic_load(Q.done + t - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= b;
          if (right)
            ok = ok && __hip_atomic_load(Q.done + t + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= b;
          if (ok) break;
          if (spin == kQueueSpinLimit) {
            __hip_atomic_fetch_or(gptr(runs[qt.tile.run].status), 4, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
            atomicMax(Q.counter, 1ull << 62);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        // one acquire for the work-group: the barrier below orders every thread's loads
        // after it (the waves share this compute unit's caches)
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      item_t = t;
      item_b = b;
      item_ns = ns;
      item_step = st;
    }
    __syncthreads();
    const int b = __builtin_amdgcn_readfirstlane(item_b);
    if (b < 0) break;
    const int t = __builtin_amdgcn_readfirstlane(item_t);
    const int ns = __builtin_amdgcn_readfirstlane(item_ns);
    const int64_t st = item_step;
    const Tile1D tile = Q.tiles[t].tile;
    const Run1D<float>& R = runs[tile.run];
    // every run starts the launch with its rows in the first copy: block b reads copy b & 1
    const int64_t in_off = (b & 1) ? Q.delta : 0, out_off = (b & 1) ? 0 : Q.delta;
    // the thread index passed through an empty asm, so that nothing derived from it is
    // hoisted out of the item loop and held in registers across it
    int k = threadIdx.x;
    asm volatile("" : "+v"(k));
    switch (R.half) {
      case 32: tb_tile<K, 8>(R, tile, st, ns, in_off, out_off, L, k); break;
      case 64: tb_tile<K, 16>(R, tile, st, ns, in_off, out_off, L, k); break;
      case 128: tb_tile<K, 32>(R, tile, st, ns, in_off, out_off, L, k); break;
      default: tb_tile<K, 64>(R, tile, st, ns, in_off, out_off, L, k); break;
    }
    // every wave waits for its own stores to complete (vmcnt 0: written to L2), then one
    // release by thread 0 writes them back device-wide before the block is recorded
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_store(Q.done + t, b + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <int K>
int queue_occupancy() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch1d_queue<K>, kTbBlock, 0) != hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

int tb_queue_blocks_per_cu(int k) {
  switch (k) {
    case 3: return queue_occupancy<3>();
    case 5: return queue_occupancy<5>();
    case 7: return queue_occupancy<7>();
    default: return queue_occupancy<9>();
  }
}

hipError_t launch_batch1d_queue(const void* runs, const TbQueueArgs& a, int groups,
                                hipStream_t stream) {
  if (a.nseg <= 0 || groups <= 0) return hipSuccess;
  TbQueue q;
  q.tiles = a.tiles;
  q.seg_start = a.seg_start;
  q.seg_round = a.seg_round;
  q.seg_tiles = a.seg_tiles;
  q.done = a.done;
  q.counter = a.counter;
  q.s0 = a.s0;
  q.s1 = a.s1;
  q.delta = a.delta;
  q.nseg = a.nseg;
  const Run1D<float>* r = static_cast<const Run1D<float>*>(runs);
  switch (a.k) {
    case 3: hipLaunchKernelGGL(k_batch1d_queue<3>, dim3(groups), dim3(kTbBlock), 0, stream, r, q); break;
    case 5: hipLaunchKernelGGL(k_batch1d_queue<5>, dim3(groups), dim3(kTbBlock), 0, stream, r, q); break;
    case 7: hipLaunchKernelGGL(k_batch1d_queue<7>, dim3(groups), dim3(kTbBlock), 0, stream, r, q); break;
    case 9: hipLaunchKernelGGL(k_batch1d_queue<9>, dim3(groups), dim3(kTbBlock), 0, stream, r, q); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
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
