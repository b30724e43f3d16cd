// kernels3d.hip -- one leap-frog step of the 3D Yee cube coupled to the speed-grid F1 of
// every plasma point (arXiv 2211.05647, section 2 in its 3D form and section 5.3).
//
// Three launches per step (four with F0 evolving), in the order of the method:
//   k_h3d    H^{n+1/2} of the three components (one thread per lattice point), with the
//            CPML memory of each derivative inside its layer;
//   k_kin3d  F1 of every plasma point driven by its E component at t^n (Crank-Nicolson in
//            the collision term) and the FP64 moment J = -e (4 pi / 3) gam sum v^3 F1,
//            one lane group per point row;
//   k_e3d    E^{n+1} = E^n + S curl H - J with the CPML memory, the soft source at t^{n+1}
//            (the kinetic launch subtracts J at the plasma points, in place);
//   k_f0_3d  two-term model only: F0 of every plasma cell from the l = 0 equation (the
//            kinetic launch is then k_kin3d_tt, whose F1 drive includes F0's change).
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

// Rows of a row-per-lane-group launch (grid a multiple of kXcds): work-group b runs on
// XCD b mod 8, so XCD x takes the x-th eighth of the rows and its wavefronts walk that
// range together, cpw rows per wavefront and pass.  Neighbouring rows share cells (and
// cells share edges), so a row's gathers then find what the rows before it loaded in the
// same XCD's L2.
struct RowSpan {
  int first, stride, end;
};

__device__ __forceinline__ RowSpan xcd_rows(int nrows, int cpw) {
  const int per_xcd = gridDim.x / kXcds;
  const int x = blockIdx.x % kXcds;
  const int waves = blockDim.x >> 6;
  const int wave = (blockIdx.x / kXcds) * waves + (threadIdx.x >> 6);
  const int span = (nrows + kXcds - 1) / kXcds;
  const int lo = x * span;
  RowSpan r;
  r.first = lo + wave * cpw;
  r.stride = per_xcd * waves * cpw;
  r.end = min(nrows, lo + span);
  return r;
}

// Every operand of the point's three components is loaded before any arithmetic (the
// stores of one component would otherwise order the loads of the next behind them).
template <class T>
__global__ __launch_bounds__(256) void k_h3d(const Run3D<T> R) {
  const int nx = R.nx, ny = R.ny, nz = R.nz, m = R.m;
  const PlaneTile pt = plane_tile(nx, ny, nz);
  if (!pt.ok) return;
  const int i = pt.i, j = pt.j, k = pt.k;
  const size_t sEx_j = nx, sEx_k = (size_t)(ny + 1) * nx;
  const size_t sEy_j = nx + 1, sEy_k = (size_t)ny * (nx + 1);
  const size_t sEz_j = nx + 1, sEz_k = (size_t)(ny + 1) * (nx + 1);
  const T* __restrict__ Ex = R.Ex;
  const T* __restrict__ Ey = R.Ey;
  const T* __restrict__ Ez = R.Ez;
  // Hx at (i, j+1/2, k+1/2), Hy at (i+1/2, j, k+1/2), Hz at (i+1/2, j+1/2, k)
  const bool vx = j < ny && k < nz, vy = i < nx && k < nz, vz = i < nx && j < ny;
  const size_t qx = ((size_t)k * ny + j) * (nx + 1) + i;
  const size_t qy = ((size_t)k * (ny + 1) + j) * nx + i;
  const size_t qz = ((size_t)k * ny + j) * nx + i;
  const size_t ey = k * sEy_k + j * sEy_j + i, ez = k * sEz_k + j * sEz_j + i,
               ex = k * sEx_k + j * sEx_j + i;
  const T ey0 = (vx || vz) ? Ey[ey] : T(0);
  const T eyk = vx ? Ey[ey + sEy_k] : T(0);
  const T eyi = vz ? Ey[ey + 1] : T(0);
  const T ez0 = (vx || vy) ? Ez[ez] : T(0);
  const T ezj = vx ? Ez[ez + sEz_j] : T(0);
  const T ezi = vy ? Ez[ez + 1] : T(0);
  const T ex0 = (vy || vz) ? Ex[ex] : T(0);
  const T exk = vy ? Ex[ex + sEx_k] : T(0);
  const T exj = vz ? Ex[ex + sEx_j] : T(0);
  const T hx = vx ? R.Hx[qx] : T(0);
  const T hy = vy ? R.Hy[qy] : T(0);
  const T hz = vz ? R.Hz[qz] : T(0);
  const int sx = (m > 0 && i < nx) ? layer_h(i, nx, m) : -1;
  const int sy = (m > 0 && j < ny) ? layer_h(j, ny, m) : -1;
  const int sz = (m > 0 && k < nz) ? layer_h(k, nz, m) : -1;
  T* const p_hxz = (vx && sz >= 0) ? R.p_hxz + ((size_t)sz * ny + j) * (nx + 1) + i : nullptr;
  T* const p_hxy = (vx && sy >= 0) ? R.p_hxy + ((size_t)k * 2 * m + sy) * (nx + 1) + i : nullptr;
  T* const p_hyx = (vy && sx >= 0) ? R.p_hyx + ((size_t)k * (ny + 1) + j) * 2 * m + sx : nullptr;
  T* const p_hyz = (vy && sz >= 0) ? R.p_hyz + ((size_t)sz * (ny + 1) + j) * nx + i : nullptr;
  T* const p_hzy = (vz && sy >= 0) ? R.p_hzy + ((size_t)k * 2 * m + sy) * nx + i : nullptr;
  T* const p_hzx = (vz && sx >= 0) ? R.p_hzx + ((size_t)k * ny + j) * 2 * m + sx : nullptr;
  const T phxz = p_hxz ? *p_hxz : T(0), phxy = p_hxy ? *p_hxy : T(0);
  const T phyx = p_hyx ? *p_hyx : T(0), phyz = p_hyz ? *p_hyz : T(0);
  const T phzy = p_hzy ? *p_hzy : T(0), phzx = p_hzx ? *p_hzx : T(0);
  const T S = R.S;
  if (vx) {
    const T dEy_z = eyk - ey0, dEz_y = ezj - ez0;
    T acc = dEy_z * R.rkhz[k] - dEz_y * R.rkhy[j];
    if (p_hxz) { const T v = fma(R.bhz[k], phxz, R.ahz[k] * dEy_z); *p_hxz = v; acc += v; }
    if (p_hxy) { const T v = fma(R.bhy[j], phxy, R.ahy[j] * dEz_y); *p_hxy = v; acc -= v; }
    R.Hx[qx] = fma(S, acc, hx);
  }
  if (vy) {
    const T dEz_x = ezi - ez0, dEx_z = exk - ex0;
    T acc = dEz_x * R.rkhx[i] - dEx_z * R.rkhz[k];
    if (p_hyx) { const T v = fma(R.bhx[i], phyx, R.ahx[i] * dEz_x); *p_hyx = v; acc += v; }
    if (p_hyz) { const T v = fma(R.bhz[k], phyz, R.ahz[k] * dEx_z); *p_hyz = v; acc -= v; }
    R.Hy[qy] = fma(S, acc, hy);
  }
  if (vz) {
    const T dEx_y = exj - ex0, dEy_x = eyi - ey0;
    T acc = dEx_y * R.rkhy[j] - dEy_x * R.rkhx[i];
    if (p_hzy) { const T v = fma(R.bhy[j], phzy, R.ahy[j] * dEx_y); *p_hzy = v; acc += v; }
    if (p_hzx) { const T v = fma(R.bhx[i], phzx, R.ahx[i] * dEy_x); *p_hzx = v; acc -= v; }
    R.Hz[qz] = fma(S, acc, hz);
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

// Two-term model (section 5.1 expansion with F0 evolving, section 5.3 speed grid): the F1
// drive adds the speed derivative of F0 - n F0hat, taken as the central difference of the
// mean of the four cells around the point's edge (even across v = 0, zero beyond vmax);
// the moment takes the face-averaged weights of w_bin.  E^n is kept for the l = 0 update.
template <class T>
__global__ __launch_bounds__(256) void k_kin3d_tt(const Run3D<T> R) {
  using V = typename Vec<T>::type;
  constexpr int VPL = Vec<T>::n;
  const int lane = threadIdx.x & 63;
  const int lpc = R.row / VPL;             // power of two, <= 64
  const int cpw = 64 / lpc;
  const int sub = lane / lpc, li = lane - sub * lpc;
  const int nxt = sub * lpc + ((li + 1) & (lpc - 1));
  const int prv = sub * lpc + ((li - 1) & (lpc - 1));
  const bool first_lane = li == 0, last_lane = li == lpc - 1;
  V s = reinterpret_cast<const V*>(R.s_bin)[li];
  V b = reinterpret_cast<const V*>(R.b_bin)[li];
  V cf = reinterpret_cast<const V*>(R.c_bin)[li];   // 0 marks the padding
  double w[VPL];
#pragma unroll
  for (int v = 0; v < VPL; ++v) w[v] = R.w_bin[li * VPL + v];
  const T kd = R.kc;
  V* __restrict__ dfv = reinterpret_cast<V*>(R.df);
  const V* __restrict__ d0v = reinterpret_cast<const V*>(R.f0);
  const T* E = R.Ex;   // Ex, Ey, Ez are contiguous
  T* Ee = R.Ex;
  T* __restrict__ J = R.Jx;
  const RowSpan rs = xcd_rows(R.np, cpw);
  for (int base = rs.first; base < rs.end; base += rs.stride) {
    const int p = base + sub;
    const bool live = p < rs.end;
    int at = 0;
    T tau = T(0), ne = T(0), Ev = T(0);
    V f, dm;
#pragma unroll
    for (int v = 0; v < VPL; ++v) lane_at(f, v) = lane_at(dm, v) = T(0);
    if (live) {
      at = R.pidx[p];
      tau = R.tau[p];
      ne = R.dens[p];
      Ev = E[at];
      f = dfv[(size_t)p * lpc + li];
      const int4 c4 = reinterpret_cast<const int4*>(R.pcell)[p];
      V d0 = d0v[(size_t)c4.x * lpc + li], d1 = d0v[(size_t)c4.y * lpc + li];
      V d2 = d0v[(size_t)c4.z * lpc + li], d3 = d0v[(size_t)c4.w * lpc + li];
#pragma unroll
      for (int v = 0; v < VPL; ++v)
        lane_at(dm, v) = T(0.25) * ((lane_at(d0, v) + lane_at(d1, v)) + (lane_at(d2, v) + lane_at(d3, v)));
    }
    const T nd = __shfl(lane_at(dm, 0), nxt);
    const T pd = __shfl(lane_at(dm, VPL - 1), prv);
    const T nE = ne * Ev, kE = kd * Ev, tau2 = tau + tau;
    // the explicit exchange between F0 and F1 needs (e/m) |E| dt / gam <= 1
    if (live && first_lane && !(fabs(kE) <= T(1))) atomicOr(R.status, 2);
    double acc = 0.0;
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
      const T dr = v + 1 < VPL ? lane_at(dm, v + 1 < VPL ? v + 1 : v) : (last_lane ? T(0) : nd);
      const T dl = v > 0 ? lane_at(dm, v > 0 ? v - 1 : 0) : (first_lane ? lane_at(dm, 0) : pd);
      const T sv = lane_at(s, v);
      const T r = cn_recip(fma(tau, sv, T(2)));
      const T fv = lane_at(f, v);
      const T drive = lane_at(cf, v) != T(0) ? fma(kE, dr - dl, lane_at(b, v) * nE) : T(0);
      const T t = fma(-(tau2 * sv), fv, drive);
      const T fn = fma(t, r, fv);
      lane_at(f, v) = fn;
      acc = fma(w[v], (double)fn, acc);
    }
    if (live) dfv[(size_t)p * lpc + li] = f;
    double a1[1] = {acc};
    int which = 0;
    const double tot = group_reduce<1>(a1, lpc, li, which);
    if (live && li == 0) {
      const T jv = (T)tot;
      R.en[p] = Ev;
      J[at] = jv;
      Ee[at] = Ev - jv;
    }
  }
}

// l = 0 update of every plasma cell, after the E launch: G_k = sum over the cell's plasma
// edges of Ebar F1_k / 4 (Ebar = (E^n + E^{n+1}) / 2, F1 at n+1/2), the flux through each
// inner speed face v^2 (G_k + G_{k+1}) / 2 (none through v = 0 or vmax), and
// F0 += dt (e / 3m) (flux above - flux below) / (v_k^2 gam).  Each cell gathers its own
// edges, so the result does not depend on the order work-groups run in.
template <class T>
__global__ __launch_bounds__(256) void k_f0_3d(const Run3D<T> R) {
  using V = typename Vec<T>::type;
  constexpr int VPL = Vec<T>::n;
  const int lane = threadIdx.x & 63;
  const int lpc = R.row / VPL;
  const int cpw = 64 / lpc;
  const int sub = lane / lpc, li = lane - sub * lpc;
  const int nxt = sub * lpc + ((li + 1) & (lpc - 1));
  const int prv = sub * lpc + ((li - 1) & (lpc - 1));
  const bool first_lane = li == 0, last_lane = li == lpc - 1;
  V cf = reinterpret_cast<const V*>(R.c_bin)[li];
  V vh = reinterpret_cast<const V*>(R.v2h_bin)[li];
  const V* __restrict__ dfv = reinterpret_cast<const V*>(R.df);
  V* __restrict__ d0v = reinterpret_cast<V*>(R.f0);
  const T* E = R.Ex;
  const RowSpan rs = xcd_rows(R.nc, cpw);
  for (int base = rs.first; base < rs.end; base += rs.stride) {
    const int c = base + sub;
    const bool live = c < rs.end;
    V g;
#pragma unroll
    for (int v = 0; v < VPL; ++v) lane_at(g, v) = T(0);
    if (live) {
      // (point, E index) of each of the 12 edges, read together
      const int4* ce = reinterpret_cast<const int4*>(R.cedge) + (size_t)c * 6;
      int4 q[6];
#pragma unroll
      for (int u = 0; u < 6; ++u) q[u] = ce[u];
      // every edge's loads issued before any arithmetic (an edge without a plasma point
      // reads point 0's row and the E index 0 and weighs them by zero)
      T eb[12];
      V f[12];
#pragma unroll
      for (int u = 0; u < 12; ++u) {
        const int p = (u & 1) ? q[u >> 1].z : q[u >> 1].x;
        const int at = (u & 1) ? q[u >> 1].w : q[u >> 1].y;
        const int ps = p < 0 ? 0 : p;
        eb[u] = R.en[ps] + E[at];
        if (p < 0) eb[u] = T(0);
        f[u] = dfv[(size_t)ps * lpc + li];
      }
#pragma unroll
      for (int u = 0; u < 12; ++u) {
        const T e8 = T(0.125) * eb[u];
#pragma unroll
        for (int v = 0; v < VPL; ++v) lane_at(g, v) = fma(e8, lane_at(f[u], v), lane_at(g, v));
      }
    }
    const T ng = __shfl(lane_at(g, 0), nxt);
    T ph[VPL];
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
      const T gr = v + 1 < VPL ? lane_at(g, v + 1 < VPL ? v + 1 : v) : (last_lane ? T(0) : ng);
      ph[v] = lane_at(vh, v) * (lane_at(g, v) + gr);   // 0 on the top face and beyond
    }
    const T pl0 = __shfl(ph[VPL - 1], prv);
    if (live) {
      V d = d0v[(size_t)c * lpc + li];
#pragma unroll
      for (int v = 0; v < VPL; ++v) {
        const T pl = v > 0 ? ph[v > 0 ? v - 1 : 0] : (first_lane ? T(0) : pl0);
        lane_at(d, v) = fma(lane_at(cf, v), ph[v] - pl, lane_at(d, v));
      }
      d0v[(size_t)c * lpc + li] = d;
    }
  }
}

// E^{n+1} = E^n + S curl H (the kinetic launch has already taken J^{n+1/2} off E^n at
// the plasma points); every operand loaded before any arithmetic, as in k_h3d.
template <class T>
__global__ __launch_bounds__(256) void k_e3d(const Run3D<T> R, int64_t step) {
  const int nx = R.nx, ny = R.ny, nz = R.nz, m = R.m;
  const PlaneTile pt = plane_tile(nx, ny, nz);
  if (!pt.ok) return;
  const int i = pt.i, j = pt.j, k = pt.k;
  const size_t sHx_j = nx + 1, sHx_k = (size_t)ny * (nx + 1);
  const size_t sHy_j = nx, sHy_k = (size_t)(ny + 1) * nx;
  const size_t sHz_j = nx, sHz_k = (size_t)ny * nx;
  const T* __restrict__ Hx = R.Hx;
  const T* __restrict__ Hy = R.Hy;
  const T* __restrict__ Hz = R.Hz;
  // Ex at (i+1/2, j, k), Ey at (i, j+1/2, k), Ez at (i, j, k+1/2); tangential E on the
  // outer faces is never written
  const bool ik = k >= 1 && k < nz;
  const bool vx = i < nx && j >= 1 && j < ny && ik;
  const bool vy = i >= 1 && i < nx && j < ny && ik;
  const bool vz = i >= 1 && i < nx && j >= 1 && j < ny && k < nz;
  const size_t qx = ((size_t)k * (ny + 1) + j) * nx + i;
  const size_t qy = ((size_t)k * ny + j) * (nx + 1) + i;
  const size_t qz = ((size_t)k * (ny + 1) + j) * (nx + 1) + i;
  const size_t hxo = k * sHx_k + j * sHx_j + i, hyo = k * sHy_k + j * sHy_j + i,
               hzo = k * sHz_k + j * sHz_j + i;
  const T hz0 = (vx || vy) ? Hz[hzo] : T(0);
  const T hzj = vx ? Hz[hzo - sHz_j] : T(0);
  const T hzi = vy ? Hz[hzo - 1] : T(0);
  const T hy0 = (vx || vz) ? Hy[hyo] : T(0);
  const T hyk = vx ? Hy[hyo - sHy_k] : T(0);
  const T hyi = vz ? Hy[hyo - 1] : T(0);
  const T hx0 = (vy || vz) ? Hx[hxo] : T(0);
  const T hxk = vy ? Hx[hxo - sHx_k] : T(0);
  const T hxj = vz ? Hx[hxo - sHx_j] : T(0);
  const T ex = vx ? R.Ex[qx] : T(0);
  const T ey = vy ? R.Ey[qy] : T(0);
  const T ez = vz ? R.Ez[qz] : T(0);
  const int sx = m > 0 ? layer_e(i, nx, m) : -1;
  const int sy = m > 0 ? layer_e(j, ny, m) : -1;
  const int sz = m > 0 ? layer_e(k, nz, m) : -1;
  T* const p_exy = (vx && sy >= 0) ? R.p_exy + ((size_t)k * 2 * m + sy) * nx + i : nullptr;
  T* const p_exz = (vx && sz >= 0) ? R.p_exz + ((size_t)sz * (ny + 1) + j) * nx + i : nullptr;
  T* const p_eyz = (vy && sz >= 0) ? R.p_eyz + ((size_t)sz * ny + j) * (nx + 1) + i : nullptr;
  T* const p_eyx = (vy && sx >= 0) ? R.p_eyx + ((size_t)k * ny + j) * 2 * m + sx : nullptr;
  T* const p_ezx = (vz && sx >= 0) ? R.p_ezx + ((size_t)k * (ny + 1) + j) * 2 * m + sx : nullptr;
  T* const p_ezy = (vz && sy >= 0) ? R.p_ezy + ((size_t)k * 2 * m + sy) * (nx + 1) + i : nullptr;
  const T pexy = p_exy ? *p_exy : T(0), pexz = p_exz ? *p_exz : T(0);
  const T peyz = p_eyz ? *p_eyz : T(0), peyx = p_eyx ? *p_eyx : T(0);
  const T pezx = p_ezx ? *p_ezx : T(0), pezy = p_ezy ? *p_ezy : T(0);
  const T S = R.S;
  if (vx) {
    const T dHz_y = hz0 - hzj, dHy_z = hy0 - hyk;
    T acc = dHz_y * R.rkey[j] - dHy_z * R.rkez[k];
    if (p_exy) { const T v = fma(R.bey[j], pexy, R.aey[j] * dHz_y); *p_exy = v; acc += v; }
    if (p_exz) { const T v = fma(R.bez[k], pexz, R.aez[k] * dHy_z); *p_exz = v; acc -= v; }
    T e = fma(S, acc, ex);
    if (R.src_kind != 0 && k == R.src_k && (R.src_kind == 1 || (i == R.src_i && j == R.src_j)))
      e += (T)source_wave((double)(step + 1) * R.dt, R.src_amp, R.src_w, R.src_tau, R.src_t0);
    R.Ex[qx] = e;
  }
  if (vy) {
    const T dHx_z = hx0 - hxk, dHz_x = hz0 - hzi;
    T acc = dHx_z * R.rkez[k] - dHz_x * R.rkex[i];
    if (p_eyz) { const T v = fma(R.bez[k], peyz, R.aez[k] * dHx_z); *p_eyz = v; acc += v; }
    if (p_eyx) { const T v = fma(R.bex[i], peyx, R.aex[i] * dHz_x); *p_eyx = v; acc -= v; }
    R.Ey[qy] = fma(S, acc, ey);
  }
  if (vz) {
    const T dHy_x = hy0 - hyi, dHx_y = hx0 - hxj;
    T acc = dHy_x * R.rkex[i] - dHx_y * R.rkey[j];
    if (p_ezx) { const T v = fma(R.bex[i], pezx, R.aex[i] * dHy_x); *p_ezx = v; acc += v; }
    if (p_ezy) { const T v = fma(R.bey[j], pezy, R.aey[j] * dHx_y); *p_ezy = v; acc -= v; }
    R.Ez[qz] = fma(S, acc, ez);
  }
}

// E at the probe points after the step (E^{n+1}), into slot `step` mod cap of each
// probe's ring.
template <class T>
__global__ __launch_bounds__(64) void k_probe3d(const T* __restrict__ E,
                                                const int32_t* __restrict__ pix, int nprobe,
                                                T* __restrict__ ring, int cap, int64_t step) {
  const int q = threadIdx.x;
  if (q < nprobe) ring[(size_t)q * cap + (size_t)(step % cap)] = E[pix[q]];
}

template <class T>
hipError_t launch_step3d_t(const void* run, int nx, int ny, int nz, int np, int kin_groups,
                           int nc, int f0_groups, bool two_term, int64_t step,
                           const int32_t* pix, int nprobe, void* ring, int cap,
                           hipStream_t stream) {
  const Run3D<T>& R = *static_cast<const Run3D<T>*>(run);
  const int tiles = ((nx + 1) * (ny + 1) + 255) / 256;
  const int blocks = (tiles * (nz + 1) + kXcds - 1) / kXcds * kXcds;
  const dim3 grid(blocks);
  hipLaunchKernelGGL(k_h3d<T>, grid, dim3(256), 0, stream, R);
  if (np > 0) {
    if (two_term) hipLaunchKernelGGL(k_kin3d_tt<T>, dim3(kin_groups), dim3(256), 0, stream, R);
    else hipLaunchKernelGGL(k_kin3d<T>, dim3(kin_groups), dim3(256), 0, stream, R);
  }
  hipLaunchKernelGGL(k_e3d<T>, grid, dim3(256), 0, stream, R, step);
  if (two_term && nc > 0 && np > 0)
    hipLaunchKernelGGL(k_f0_3d<T>, dim3(f0_groups), dim3(256), 0, stream, R);
  if (nprobe > 0)
    hipLaunchKernelGGL(k_probe3d<T>, dim3(1), dim3(64), 0, stream, R.Ex, pix, nprobe,
                       static_cast<T*>(ring), cap, step);
  return hipGetLastError();
}

template hipError_t launch_step3d_t<float>(const void*, int, int, int, int, int, int, int, bool,
                                           int64_t, const int32_t*, int, void*, int, hipStream_t);
template hipError_t launch_step3d_t<double>(const void*, int, int, int, int, int, int, int, bool,
                                            int64_t, const int32_t*, int, void*, int, hipStream_t);

}  // namespace fdtdp
