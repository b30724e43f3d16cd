// kernels1d.hip -- one leap-frog step of the 1D (Ez, Hy) Yee line coupled to the 1V
// kinetic F1 of every plasma node (arXiv 2211.05647, section 2 and section 5.2).
//
// A work-group of NT threads owns a tile of at most NT E nodes [node0, node1) and the
// plasma nodes inside it [cell0, cell1).  Per step it
//   1. loads E^n and H^{n-1/2} around its nodes into registers (and E^n into LDS);
//   2. advances F1 of its plasma nodes with E^n (Crank-Nicolson in the collision term,
//      the f_1x update of section 5.2) and reduces the current moment
//      J = -e dv sum_j v_j F1_j in FP64 (half grid: F1 is odd in v, so the sum over
//      v > 0 bins counts twice), keeping the tile's J in LDS;
//   3. updates H^{n+1/2} and E^{n+1} of its nodes (Ampere's law minus J), with the
//      first-order Mur ends and the soft source.
// E and H are double-buffered, so halo values are re-derived from the previous
// buffers and no work-group ever waits for another inside a step.
//
// k_step1d launches it once per step, one work-group per tile (any number of runs;
// tiles of finished runs are left out of the launch); the full-distribution and
// two-term models have launches of their own over the same body.  Blocks of several
// steps per launch, and the persistent batch launch, are in kernels1d_tb.hip.
//
// F1 layout: [cell][v > 0 bin], contiguous in the bin index.  A group of `lpc` lanes
// covers one cell row with 16-byte loads (64 lanes x 16 B = one 1 KB row per wave
// instruction at Nv = 512); each lane group keeps U rows in flight, and the U FP64
// partial moments are reduced with a reduce-scatter butterfly.
#include "common.h"

namespace fdtdp {

template <class T, int U, int NT, bool S = false>
__device__ __forceinline__ void kinetic_tile(const Run1D<T>& R, const T* eloc,
                                             const Tile1D& tile, T* jloc) {
  using V = typename Vec<T>::type;
  constexpr int VPL = Vec<T>::n;
  constexpr int kWaves = NT / 64;
  constexpr int CPL = 4 / U;              // chunks per lane this instance handles
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ch = R.half / VPL;            // 16-byte chunks per cell row
  const int lpc = ch < 64 ? ch : 64;      // lanes per cell
  const int cpl = ch / lpc;               // chunks per lane (<= CPL by dispatch)
  const int cpw = 64 / lpc;               // lane groups per wavefront
  const int sub = lane / lpc, li = lane - sub * lpc;

  V s[CPL], b[CPL];
  double w[CPL][VPL];
#pragma unroll
  for (int m = 0; m < CPL; ++m) {
    if (m < cpl) {
      const int k = li + m * lpc;
      s[m] = reinterpret_cast<const V*>(R.s_bin)[k];
      b[m] = reinterpret_cast<const V*>(R.b_bin)[k];
#pragma unroll
      for (int v = 0; v < VPL; ++v) w[m][v] = R.w_bin[k * VPL + v];
    }
  }
  V* __restrict__ dfv = reinterpret_cast<V*>(R.df);
  const int stride = kWaves * cpw * U;
  for (int base = tile.cell0 + wave * cpw * U; base < tile.cell1; base += stride) {
    V f[U][CPL];
    T ne[U], tau[U];
    int loc[U];
    // issue every load of the U rows before any arithmetic
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = base + u * cpw + sub;
      loc[u] = -1;
      if (c < tile.cell1) {
        loc[u] = R.cell_node[c] - tile.node0;
        tau[u] = R.tau[c];
        ne[u] = R.dens[c];
        const V* row = dfv + (size_t)c * ch;
#pragma unroll
        for (int m = 0; m < CPL; ++m)
          if (m < cpl) f[u][m] = row_load<S>(&row[li + m * lpc]);
      }
    }
    double acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc[u] = 0.0;
      if (loc[u] >= 0) {
        const T Eu = eloc[loc[u]];
        const T nE = ne[u] * Eu;
#pragma unroll
        for (int m = 0; m < CPL; ++m) {
          if (m < cpl) {
#pragma unroll
            for (int v = 0; v < VPL; ++v) {
              // x = dt nu_j; F1' = ((2 - x) F1 + 2 dt (e/m) n dF0/dv E) / (2 + x), with
              // 2 x = (2 dt nu_mean) s_j exactly.  Rows of 64 lanes (the blocked kernel
              // keeps d and c' per row there): (F1 + d F1) + c' E, d = -2x / (2 + x),
              // c' = (b / (2 + x)) n; shorter rows: the increment form
              // F1 + (b n E - 2x F1) / (2 + x).  Each form is the blocked kernel's for
              // that row length, operation for operation, so the two agree to the bit;
              // both keep the damping's relative precision when x is small.
              const T sv = lane_at(s[m], v);
              const T r = cn_recip(fma(tau[u], sv, T(2)));
              const T fv = lane_at(f[u][m], v);
              T fn;
              if (lpc == 64) {
                const T d = -((tau[u] + tau[u]) * sv) * r;
                const T c = (lane_at(b[m], v) * r) * ne[u];
                fn = fma(c, Eu, fma(d, fv, fv));
              } else {
                const T x2 = (tau[u] + tau[u]) * sv;
                const T t = fma(-x2, fv, lane_at(b[m], v) * nE);
                fn = fma(t, r, fv);
              }
              lane_at(f[u][m], v) = fn;
              acc[u] = fma(w[m][v], (double)fn, acc[u]);
            }
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (loc[u] >= 0) {
        const int c = base + u * cpw + sub;
        V* row = dfv + (size_t)c * ch;
#pragma unroll
        for (int m = 0; m < CPL; ++m)
          if (m < cpl) row_store<S>(f[u][m], &row[li + m * lpc]);
      }
    }
    if (U > 1 && lpc < U) {
      // tiny rows (fewer lanes than rows in flight): plain all-reduce per row
#pragma unroll
      for (int u = 0; u < U; ++u) {
        double sm = acc[u];
        for (int o = lpc >> 1; o > 0; o >>= 1) sm += __shfl_xor(sm, o);
        if (li == 0 && loc[u] >= 0) jloc[loc[u]] = (T)sm;
      }
    } else {
      int which = 0;
      bool done = false;
      if constexpr (U == 4) {
        // cross-lane swaps and DPP, no LDS round trips
        double tot = 0.0;
        if (lpc == 64) tot = wave_reduce4(acc, which), done = true;
        else if (lpc == 32) tot = group_reduce4_dpp<32>(acc, which), done = true;
        else if (lpc == 16) tot = group_reduce4_dpp<16>(acc, which), done = true;
        else if (lpc == 8) tot = group_reduce4_dpp<8>(acc, which), done = true;
        if (done) {
          const int step_u = lpc / 4;
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (li == step_u * u && loc[u] >= 0) jloc[loc[u]] = (T)tot;
        }
      }
      if (!done) {
        const double tot = group_reduce<U>(acc, lpc, li, which);
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (which == u && li == reporter<U>(u, lpc) && loc[u] >= 0) jloc[loc[u]] = (T)tot;
      }
    }
  }
}

// Full-distribution model: the whole f of each plasma node evolves under
// df/dt - (e/m) E df/dv = C(f) (section 5.1 without streaming and magnetic terms; elastic
// collisions damp the odd part as in section 5.2).  Row of a plasma node: [odd | even]
// halves of delta = f - n fhat on the v > 0 bins, o_k and e_k (the v < 0 bins are their
// mirrors).  With c = a dt / dv (a = -(e/m) E^n) and zero flux through +-vmax:
//   odd:  p_{k+1/2} = (c/2)(e_k + e_{k+1}) - (c^2/2)(o_{k+1} - o_k)   (perturbation faces;
//         the face at v = 0 carries c e_0 - c^2 o_0), plus the equilibrium part n fhat
//         whose face differences come precomputed in b_bin (times n E);
//         o'_k = o_k + (-2x o_k + b_k n E - 2 (p_{k+1/2} - p_{k-1/2})) / (2 + x);
//   even: q_{k+1/2} = (c/4)(s_k + s_{k+1}), s = o + o' (zero at v = 0 and at vmax);
//         e'_k = e_k - (q_{k+1/2} - q_{k-1/2});
//   J = -e dv sum over both halves of v f = the linear model's moment of o'.
// A lane group of lpc lanes holds a row in 16-byte chunks (chunk li + m lpc of each half);
// the neighbour bins across chunk edges come from the next / previous lane by shuffles.
template <class T, int CPL, int NT, bool S = false>
__device__ __forceinline__ void kinetic_tile_full(const Run1D<T>& R, const T* eloc,
                                                  const Tile1D& tile, T* jloc) {
  using V = typename Vec<T>::type;
  constexpr int VPL = Vec<T>::n;
  constexpr int kWaves = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ch = R.half / VPL;            // chunks per half row
  const int lpc = ch < 64 ? ch : 64;      // lanes per row; ch == CPL * lpc by dispatch
  const int cpw = 64 / lpc;
  const int sub = lane / lpc, li = lane - sub * lpc;
  const bool last_lane = li == lpc - 1, first_lane = li == 0;

  V s[CPL], b[CPL];
  double w[CPL][VPL];
#pragma unroll
  for (int m = 0; m < CPL; ++m) {
    const int k = li + m * lpc;
    s[m] = reinterpret_cast<const V*>(R.s_bin)[k];
    b[m] = reinterpret_cast<const V*>(R.b_bin)[k];
#pragma unroll
    for (int v = 0; v < VPL; ++v) w[m][v] = R.w_bin[k * VPL + v];
  }
  V* __restrict__ dfv = reinterpret_cast<V*>(R.df);
  for (int c0 = tile.cell0 + wave * cpw; c0 < tile.cell1; c0 += kWaves * cpw) {
    const int c = c0 + sub;
    const bool live = c < tile.cell1;   // groups past the end still take part in shuffles
    V o[CPL], e[CPL];
    T ne = T(0), tau = T(0), Ev = T(0);
    int loc = -1;
    if (live) {
      loc = R.cell_node[c] - tile.node0;
      tau = R.tau[c];
      ne = R.dens[c];
      Ev = eloc[loc];
      const V* row = dfv + (size_t)c * (2 * ch);
#pragma unroll
      for (int m = 0; m < CPL; ++m) {
        o[m] = row_load<S>(&row[li + m * lpc]);
        e[m] = row_load<S>(&row[ch + li + m * lpc]);
      }
    } else {
#pragma unroll
      for (int m = 0; m < CPL; ++m)
#pragma unroll
        for (int v = 0; v < VPL; ++v) lane_at(o[m], v) = lane_at(e[m], v) = T(0);
    }
    const T cf = R.kc * Ev;
    if (live && first_lane && !(fabs(cf) <= T(1))) atomicOr(R.status, 2);
    const T ch2 = T(0.5) * cf, cc2 = T(0.5) * cf * cf, cq = T(0.25) * cf;
    const T nE = ne * Ev;
    // odd pass: perturbation face fluxes right of every bin
    T pr[CPL][VPL];
    {
      T no[CPL], nev[CPL];
#pragma unroll
      for (int m = 0; m < CPL; ++m) {
        no[m] = next_lane_of_row(lane_at(o[m], 0), lpc);
        nev[m] = next_lane_of_row(lane_at(e[m], 0), lpc);
      }
#pragma unroll
      for (int m = 0; m < CPL; ++m) {
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
          T orr, er;
          bool outer = false;
          if (v + 1 < VPL) {
            orr = lane_at(o[m], v + 1);
            er = lane_at(e[m], v + 1);
          } else if (!last_lane) {
            orr = no[m];
            er = nev[m];
          } else if (m + 1 < CPL) {
            orr = no[m + 1 < CPL ? m + 1 : m];
            er = nev[m + 1 < CPL ? m + 1 : m];
          } else {
            orr = er = T(0);
            outer = true;
          }
          const T ol = lane_at(o[m], v), el = lane_at(e[m], v);
          pr[m][v] = outer ? T(0) : fma(ch2, el + er, -cc2 * (orr - ol));
        }
      }
    }
    T pl0[CPL];   // face left of element 0 of chunk m
    {
      T got[CPL];
#pragma unroll
      for (int m = 0; m < CPL; ++m) got[m] = prev_lane_of_row(pr[m][VPL - 1], lpc);
      const T pc = fma(cf, lane_at(e[0], 0), -cf * cf * lane_at(o[0], 0));  // face at v = 0
#pragma unroll
      for (int m = 0; m < CPL; ++m)
        pl0[m] = !first_lane ? got[m] : (m > 0 ? got[m > 0 ? m - 1 : 0] : pc);
    }
    V on[CPL];
    T sm[CPL][VPL];
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < CPL; ++m) {
#pragma unroll
      for (int v = 0; v < VPL; ++v) {
        const T pl = v == 0 ? pl0[m] : pr[m][v - 1];
        const T sv = lane_at(s[m], v);
        const T r = cn_recip(fma(tau, sv, T(2)));
        const T x2 = (tau + tau) * sv;
        const T ov = lane_at(o[m], v);
        const T t = fma(-x2, ov, fma(lane_at(b[m], v), nE, T(-2) * (pr[m][v] - pl)));
        const T onv = fma(t, r, ov);
        lane_at(on[m], v) = onv;
        sm[m][v] = ov + onv;
        acc = fma(w[m][v], (double)onv, acc);
      }
    }
    // even pass: faces of the time-centred odd part (no contraction of cq (s_k + s_{k+1})
    // into the face difference, so that the blocked kernel gives the same bits)
    {
#pragma clang fp contract(off)
    T qr[CPL][VPL];
    {
      T ns[CPL];
#pragma unroll
      for (int m = 0; m < CPL; ++m) ns[m] = next_lane_of_row(sm[m][0], lpc);
#pragma unroll
      for (int m = 0; m < CPL; ++m) {
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
          T sr;
          bool outer = false;
          if (v + 1 < VPL) sr = sm[m][v + 1];
          else if (!last_lane) sr = ns[m];
          else if (m + 1 < CPL) sr = ns[m + 1 < CPL ? m + 1 : m];
          else { sr = T(0); outer = true; }
          qr[m][v] = outer ? T(0) : cq * (sm[m][v] + sr);
        }
      }
    }
    {
      T got[CPL];
#pragma unroll
      for (int m = 0; m < CPL; ++m) got[m] = prev_lane_of_row(qr[m][VPL - 1], lpc);
#pragma unroll
      for (int m = 0; m < CPL; ++m) {
        const T ql0 = !first_lane ? got[m] : (m > 0 ? got[m > 0 ? m - 1 : 0] : T(0));
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
          const T ql = v == 0 ? ql0 : qr[m][v - 1];
          lane_at(e[m], v) = lane_at(e[m], v) - (qr[m][v] - ql);
        }
      }
    }
    }
    if (live) {
      V* row = dfv + (size_t)c * (2 * ch);
#pragma unroll
      for (int m = 0; m < CPL; ++m) {
        row_store<S>(on[m], &row[li + m * lpc]);
        row_store<S>(e[m], &row[ch + li + m * lpc]);
      }
    }
    const double tot = row_sum_dpp(acc, lpc, li);   // DPP rounds, as the blocked kernel
    if (live && first_lane) jloc[loc] = (T)tot;
  }
}

// Two-term model on the speed grid (section 5.1 expansion, l = 0 and l = 1 equations,
// section 5.3 speed grid) with the field along the line.  Row of a plasma node:
// [F1 | F0 - n F0hat] over `half` speed bins (the speed count padded to a power of two; the
// padding stays zero).  With `pending`, the l = 0 update of the previous step is applied
// first: F0 += c_k Ebar (phi_{k+1/2} - phi_{k-1/2}), phi = (v^2/2)(F1_k + F1_{k+1}) on the
// inner faces (v2h_bin), zero at v = 0 and vmax, Ebar = (E^{n-1} + E^n)/2 with F1^{n-1/2}
// as stored.  Then (unless `flush`) F1' = F1 + (-2x F1 + E (n b_k + kd (d_{k+1} - d_{k-1})))
// / (2 + x), d = F0 - n F0hat (even across v = 0, zero beyond vmax), and the FP64 moment
// with the face-averaged weights w_k.  Deferring the l = 0 update to the next step lets it
// reuse that step's read of the row; a run ends with a flush launch.
template <class T, int CPL, int NT>
__device__ __forceinline__ void kinetic_tile_tt(const Run1D<T>& R, const T* eloc, const T* eprev,
                                                const Tile1D& tile, T* jloc, bool pending,
                                                bool flush) {
  using V = typename Vec<T>::type;
  constexpr int VPL = Vec<T>::n;
  constexpr int kWaves = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ch = R.half / VPL;
  const int lpc = ch < 64 ? ch : 64;
  const int cpw = 64 / lpc;
  const int sub = lane / lpc, li = lane - sub * lpc;
  const bool last_lane = li == lpc - 1, first_lane = li == 0;

  V s[CPL], b[CPL], cf[CPL], vh[CPL];
  double w[CPL][VPL];
#pragma unroll
  for (int m = 0; m < CPL; ++m) {
    const int k = li + m * lpc;
    s[m] = reinterpret_cast<const V*>(R.s_bin)[k];
    b[m] = reinterpret_cast<const V*>(R.b_bin)[k];
    cf[m] = reinterpret_cast<const V*>(R.c_bin)[k];
    vh[m] = reinterpret_cast<const V*>(R.v2h_bin)[k];
#pragma unroll
    for (int v = 0; v < VPL; ++v) w[m][v] = R.w_bin[k * VPL + v];
  }
  const T kd = R.kc;   // dt (e/m) / gam
  V* __restrict__ dfv = reinterpret_cast<V*>(R.df);
  for (int c0 = tile.cell0 + wave * cpw; c0 < tile.cell1; c0 += kWaves * cpw) {
    const int c = c0 + sub;
    const bool live = c < tile.cell1;
    V f[CPL], d[CPL];
    T ne = T(0), tau = T(0), Ev = T(0), Eb = T(0);
    int loc = -1;
    if (live) {
      loc = R.cell_node[c] - tile.node0;
      tau = R.tau[c];
      ne = R.dens[c];
      Ev = eloc[loc];
      if (pending) Eb = T(0.5) * (eprev[loc] + Ev);
      const V* row = dfv + (size_t)c * (2 * ch);
#pragma unroll
      for (int m = 0; m < CPL; ++m) {
        f[m] = row[li + m * lpc];
        d[m] = row[ch + li + m * lpc];
      }
    } else {
#pragma unroll
      for (int m = 0; m < CPL; ++m)
#pragma unroll
        for (int v = 0; v < VPL; ++v) lane_at(f[m], v) = lane_at(d[m], v) = T(0);
    }
    // the deferred l = 0 update
    if (pending) {
      // no contraction of v^2 (F1_k + F1_{k+1}) into the flux difference, so that the
      // blocked kernel (which forms the same update) gives the same bits
#pragma clang fp contract(off)
      T nf[CPL];
#pragma unroll
      for (int m = 0; m < CPL; ++m) nf[m] = next_lane_of_row(lane_at(f[m], 0), lpc);
      T ph[CPL][VPL];
#pragma unroll
      for (int m = 0; m < CPL; ++m) {
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
          T fr;
          if (v + 1 < VPL) fr = lane_at(f[m], v + 1);
          else if (!last_lane) fr = nf[m];
          else fr = (m + 1 < CPL) ? nf[m + 1 < CPL ? m + 1 : m] : T(0);
          ph[m][v] = lane_at(vh[m], v) * (lane_at(f[m], v) + fr);   // 0 on the top face
        }
      }
      T got[CPL];
#pragma unroll
      for (int m = 0; m < CPL; ++m) got[m] = prev_lane_of_row(ph[m][VPL - 1], lpc);
#pragma unroll
      for (int m = 0; m < CPL; ++m) {
        const T pl0 = !first_lane ? got[m] : (m > 0 ? got[m > 0 ? m - 1 : 0] : T(0));
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
          const T pl = v == 0 ? pl0 : ph[m][v - 1];
          lane_at(d[m], v) = fma(lane_at(cf[m], v) * Eb, ph[m][v] - pl, lane_at(d[m], v));
        }
      }
    }
    double acc = 0.0;
    if (!flush) {
      // neighbours of d: d_{k+1} from the next lane, d_{k-1} from the previous one
      T nd[CPL], pd[CPL];
#pragma unroll
      for (int m = 0; m < CPL; ++m) {
        nd[m] = next_lane_of_row(lane_at(d[m], 0), lpc);
        pd[m] = prev_lane_of_row(lane_at(d[m], VPL - 1), lpc);
      }
      const T nE = ne * Ev, kE = kd * Ev, tau2 = tau + tau;
      // the explicit exchange between F0 and F1 needs (e/m) |E| dt / gam <= 1
      if (live && first_lane && !(fabs(kE) <= T(1))) atomicOr(R.status, 2);
#pragma unroll
      for (int m = 0; m < CPL; ++m) {
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
          T dr, dl;
          if (v + 1 < VPL) dr = lane_at(d[m], v + 1);
          else if (!last_lane) dr = nd[m];
          else dr = (m + 1 < CPL) ? nd[m + 1 < CPL ? m + 1 : m] : T(0);
          if (v > 0) dl = lane_at(d[m], v - 1);
          else if (!first_lane) dl = pd[m];
          else dl = (m > 0) ? pd[m > 0 ? m - 1 : 0] : lane_at(d[m], 0);   // even at v = 0
          const T sv = lane_at(s[m], v);
          const T r = cn_recip(fma(tau, sv, T(2)));
          const T fv = lane_at(f[m], v);
          const T drive =
              lane_at(cf[m], v) != T(0) ? fma(kE, dr - dl, lane_at(b[m], v) * nE) : T(0);
          const T t = fma(-(tau2 * sv), fv, drive);
          const T fn = fma(t, r, fv);
          lane_at(f[m], v) = fn;
          acc = fma(w[m][v], (double)fn, acc);
        }
      }
    }
    if (live) {
      V* row = dfv + (size_t)c * (2 * ch);
#pragma unroll
      for (int m = 0; m < CPL; ++m) {
        if (!flush) row[li + m * lpc] = f[m];
        if (pending) row[ch + li + m * lpc] = d[m];
      }
    }
    if (!flush) {
      // DPP rounds: the tree the blocked kernel uses too
      const double tot = row_sum_dpp(acc, lpc, li);
      if (live && first_lane) jloc[loc] = (T)tot;
    }
  }
}

// One step of one tile by a work-group of NT threads (tile.node1 - tile.node0 <= NT).
// jloc / eloc: LDS arrays of NT values.  The caller synchronises before reusing them.
// C (linear model): 0 = any row length (chosen per run at run time), else the 16-byte
// chunks per lane of every run of the launch (1, 2 or 4), so that only that form is
// compiled and the launch keeps the registers of that form alone; STREAM: streamed rows.
template <class T, int NT, int KIND = 0, int C = 0, bool STREAM = false>
__device__ __forceinline__ void step_tile(const Run1D<T>& R, const Tile1D& tile, int64_t step,
                                          T* jloc, T* eloc, bool pending = false,
                                          bool flush = false) {
  const int par = (int)(step & 1);
  const T* __restrict__ Ec = R.E[par];
  T* __restrict__ En = R.E[par ^ 1];
  const T* __restrict__ Hc = R.H[par];
  T* __restrict__ Hn = R.H[par ^ 1];
  const int k = threadIdx.x;
  const int nloc = tile.node1 - tile.node0;
  const int nx = R.nx;
  const int i = tile.node0 + k;
  const bool own = k < nloc;

  // 1. this thread's node: E^n at i-1, i, i+1 (and i+2 / i-2 at the ends), H^{n-1/2}
  T em = T(0), e0 = T(0), ep = T(0), hm = T(0), h0 = T(0), ex = T(0), hx = T(0);
  if (own) {
    e0 = Ec[i];
    if (i > 0) { em = Ec[i - 1]; hm = Hc[i - 1]; }
    if (i < nx) { ep = Ec[i + 1]; h0 = Hc[i]; }
    if (i == 0) { ex = Ec[2]; hx = Hc[1]; }
    if (i == nx) { ex = Ec[nx - 2]; hx = Hc[nx - 2]; }
    eloc[k] = e0;
    jloc[k] = T(0);
  }
  __syncthreads();

  // 2. kinetic F1 update and FP64 current moment of the tile's plasma nodes
  if (tile.cell1 > tile.cell0) {
    const int ch = R.half / Vec<T>::n;
    const int cpl = ch < 64 ? 1 : ch / 64;
    if constexpr (KIND == 1) {
      if constexpr (C == 1) kinetic_tile_full<T, 1, NT, STREAM>(R, eloc, tile, jloc);
      else if constexpr (C == 2) kinetic_tile_full<T, 2, NT, STREAM>(R, eloc, tile, jloc);
      else if constexpr (C == 4) kinetic_tile_full<T, 4, NT, STREAM>(R, eloc, tile, jloc);
      else if (cpl == 1) kinetic_tile_full<T, 1, NT>(R, eloc, tile, jloc);
      else if (cpl == 2) kinetic_tile_full<T, 2, NT>(R, eloc, tile, jloc);
      else kinetic_tile_full<T, 4, NT>(R, eloc, tile, jloc);
    } else if constexpr (KIND == 2) {
      // E^{n-1} at the tile's nodes, from the buffer this step's E update overwrites
      // after the barrier below (every tile writes only its own nodes)
      const T* eprev = En + tile.node0;
      if (cpl == 1) kinetic_tile_tt<T, 1, NT>(R, eloc, eprev, tile, jloc, pending, flush);
      else kinetic_tile_tt<T, 2, NT>(R, eloc, eprev, tile, jloc, pending, flush);
    } else if constexpr (C == 1) {
      kinetic_tile<T, 4, NT, STREAM>(R, eloc, tile, jloc);
    } else if constexpr (C == 2) {
      kinetic_tile<T, 2, NT, STREAM>(R, eloc, tile, jloc);
    } else if constexpr (C == 4) {
      kinetic_tile<T, 1, NT, STREAM>(R, eloc, tile, jloc);
    } else if (cpl == 1) kinetic_tile<T, 4, NT>(R, eloc, tile, jloc);
    else if (cpl == 2) kinetic_tile<T, 2, NT>(R, eloc, tile, jloc);
    else kinetic_tile<T, 1, NT>(R, eloc, tile, jloc);
  }
  __syncthreads();
  if (flush) return;   // the l = 0 update alone, after a run's last step

  // 3. H^{n+1/2} and E^{n+1}
  if (own) {
    const T S = R.S;
    const T jv = jloc[k];
    T en, hn = T(0);
    if (i == 0) {
      hn = h_update(h0, S, ep, e0);
      if (R.bc == 1) {
        const T h1 = h_update(hx, S, ex, ep);
        const T e1 = e_update(ep, S, h1, hn, T(0));
        en = fma(R.q, e1 - e0, ep);
      } else {
        en = T(0);
      }
      Hn[0] = hn;
    } else if (i == nx) {
      if (R.bc == 1) {
        const T ha = h_update(hm, S, e0, em);
        const T hb = h_update(hx, S, em, ex);
        const T e = e_update(em, S, ha, hb, T(0));
        en = fma(R.q, e - e0, em);
      } else {
        en = T(0);
      }
    } else {
      const T hl = h_update(hm, S, e0, em);
      hn = h_update(h0, S, ep, e0);
      Hn[i] = hn;
      en = e_update(e0, S, hn, hl, jv);
      if (i == R.src_node)
        en += (T)source_wave((double)(step + 1) * R.dt, R.src_amp, R.src_w, R.src_tau,
                             R.src_t0);
    }
    En[i] = en;
    R.J[i] = jv;
    if (!isfinite(en)) atomicOr(R.status, 1);
    for (int p = 0; p < R.nprobe; ++p) {
      if (R.probe_node[p] == i) {
        const int f = R.probe_field[p];
        const T val = (f == 0) ? en : (f == 1 ? hn : jv);
        R.probe_buf[(size_t)p * R.probe_cap + (size_t)(step % R.probe_cap)] = val;
      }
    }
    for (int t = 0; t < R.ntap; ++t) {
      if (R.tap_node[t] == i && step < R.tap_cap) {
        T* dst = R.tap_buf + ((size_t)t * R.tap_cap + (size_t)step) * 2;
        dst[0] = e0;   // E^n, the drive of this step's F1 update
        dst[1] = jv;   // J^{n+1/2}
      }
    }
  }
}

template <class T, int C, bool S>
__global__ __launch_bounds__(kBlock) void k_step1d(const Run1D<T>* __restrict__ runs,
                                                   const Tile1D* __restrict__ tiles,
                                                   int64_t step) {
  __shared__ T jloc[kMaxTile1D];
  __shared__ T eloc[kMaxTile1D];
  const Tile1D tile = tiles[blockIdx.x];
  const Run1D<T>& R = runs[tile.run];
  if (step >= R.step_limit) return;
  step_tile<T, kBlock, 0, C, S>(R, tile, step, jloc, eloc);
}

// The same step for runs of the full-distribution model (a kernel of its own, so the
// linear model's kernels keep their register budget).
template <class T, int C, bool S>
__global__ __launch_bounds__(kBlock) void k_step1d_full(const Run1D<T>* __restrict__ runs,
                                                        const Tile1D* __restrict__ tiles,
                                                        int64_t step) {
  __shared__ T jloc[kMaxTile1D];
  __shared__ T eloc[kMaxTile1D];
  const Tile1D tile = tiles[blockIdx.x];
  const Run1D<T>& R = runs[tile.run];
  if (step >= R.step_limit) return;
  step_tile<T, kBlock, 1, C, S>(R, tile, step, jloc, eloc);
}

// The same step for runs of the two-term model; `pending` applies the previous step's
// l = 0 update first, `flush` applies only that (step = the number of steps done).
template <class T>
__global__ __launch_bounds__(kBlock) void k_step1d_tt(const Run1D<T>* __restrict__ runs,
                                                      const Tile1D* __restrict__ tiles,
                                                      int64_t step, int pending, int flush) {
  __shared__ T jloc[kMaxTile1D];
  __shared__ T eloc[kMaxTile1D];
  const Tile1D tile = tiles[blockIdx.x];
  const Run1D<T>& R = runs[tile.run];
  // a run of a batch whose last step was step - 1 takes only that step's pending l = 0
  // update (its flush), so that its state is complete when it stops
  const bool fl = flush || (pending && step == R.step_limit);
  if (!fl && step >= R.step_limit) return;
  step_tile<T, kBlock, 2>(R, tile, step, jloc, eloc, pending != 0, fl);
}

template <class T>
hipError_t launch_step1d_tt(const void* runs, const void* tiles, int ntiles, int64_t step,
                            bool pending, bool flush, hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_step1d_tt<T>, dim3(ntiles), dim3(kBlock), 0, stream,
                     static_cast<const Run1D<T>*>(runs), static_cast<const Tile1D*>(tiles),
                     step, (int)pending, (int)flush);
  return hipGetLastError();
}

template <class T, int C, bool S>
void launch_k1(const void* runs, const void* tiles, int ntiles, int64_t step, hipStream_t stream,
               bool full) {
  if (full)
    hipLaunchKernelGGL((k_step1d_full<T, C, S>), dim3(ntiles), dim3(kBlock), 0, stream,
                       static_cast<const Run1D<T>*>(runs), static_cast<const Tile1D*>(tiles), step);
  else
    hipLaunchKernelGGL((k_step1d<T, C, S>), dim3(ntiles), dim3(kBlock), 0, stream,
                       static_cast<const Run1D<T>*>(runs), static_cast<const Tile1D*>(tiles), step);
}

template <class T>
hipError_t launch_step1d(const void* runs, const void* tiles, int ntiles, int64_t step,
                         hipStream_t stream, bool full, int cpl, bool streaming) {
  if (ntiles <= 0) return hipSuccess;
  switch (cpl) {
    case 1: streaming ? launch_k1<T, 1, true>(runs, tiles, ntiles, step, stream, full)
                      : launch_k1<T, 1, false>(runs, tiles, ntiles, step, stream, full); break;
    case 2: streaming ? launch_k1<T, 2, true>(runs, tiles, ntiles, step, stream, full)
                      : launch_k1<T, 2, false>(runs, tiles, ntiles, step, stream, full); break;
    case 4: streaming ? launch_k1<T, 4, true>(runs, tiles, ntiles, step, stream, full)
                      : launch_k1<T, 4, false>(runs, tiles, ntiles, step, stream, full); break;
    default: launch_k1<T, 0, false>(runs, tiles, ntiles, step, stream, full); break;
  }
  return hipGetLastError();
}

template hipError_t launch_step1d<float>(const void*, const void*, int, int64_t, hipStream_t,
                                         bool, int, bool);
template hipError_t launch_step1d<double>(const void*, const void*, int, int64_t, hipStream_t,
                                          bool, int, bool);
template hipError_t launch_step1d_tt<float>(const void*, const void*, int, int64_t, bool, bool,
                                            hipStream_t);
template hipError_t launch_step1d_tt<double>(const void*, const void*, int, int64_t, bool, bool,
                                             hipStream_t);

}  // namespace fdtdp
