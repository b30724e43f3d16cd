// common.h -- device-side types shared by the kernels of the kinetic-FDTD library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdtdp {

constexpr int kMaxProbes = 16;
constexpr int kBlock = 256;        // threads per work-group of the step kernels
constexpr int kMaxTile1D = 256;    // nodes per 1D tile: one node per thread
constexpr int kMaxTaps = 8;        // training-pair taps per 1D run

// 16-byte vector of the storage type: 4 floats or 2 doubles per lane per chunk.
template <class T> struct Vec;
template <> struct Vec<float> { using type = float4; static constexpr int n = 4; };
template <> struct Vec<double> { using type = double2; static constexpr int n = 2; };

template <class V> __device__ __forceinline__ auto& lane_at(V& v, int k) {
  return reinterpret_cast<typename std::remove_reference<decltype(v.x)>::type*>(&v)[k];
}
template <class V> __device__ __forceinline__ auto lane_at(const V& v, int k) {
  using E = typename std::remove_cv<typename std::remove_reference<decltype(v.x)>::type>::type;
  return reinterpret_cast<const E*>(&v)[k];
}

// Reciprocal used by the Crank-Nicolson factor 1/(2 + dt nu): the hardware estimate in
// FP32 (the increment it scales is small next to F1 itself), exact division in FP64.
// A pointer into device global memory with its address space stated, so that accesses
// through it compile to global_* rather than flat_* instructions.  A flat access might
// reach LDS, and the compiler then makes the next LDS access wait for it as well (and
// with it for every global load in flight).
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gptr(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

__device__ __forceinline__ float cn_recip(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double cn_recip(double d) { return 1.0 / d; }

// Leap-frog updates, written once so that every thread that recomputes a halo value
// produces the owner's bits exactly.
template <class T> __device__ __forceinline__ T h_update(T h, T s, T e_hi, T e_lo) {
  return fma(s, e_hi - e_lo, h);
}
template <class T> __device__ __forceinline__ T e_update(T e, T s, T h_hi, T h_lo, T j) {
  return fma(s, h_hi - h_lo, e) - j;
}

// Gaussian-modulated sine of the source, evaluated in FP64.
__device__ __forceinline__ double source_wave(double t, double amp, double w, double tau,
                                              double t0) {
  double x = (t - t0) / tau;
  return amp * sin(w * (t - t0)) * exp(-x * x);
}

// Sum U per-lane values over the lpc lanes of each lane group (lpc >= U).  On return,
// lane `li` of a group holds the total of value index `which`.
template <int U>
__device__ __forceinline__ double group_reduce(double (&a)[U], int lpc, int li, int& which) {
  if constexpr (U == 1) {
    double s = a[0];
    for (int o = lpc >> 1; o > 0; o >>= 1) s += __shfl_xor(s, o);
    which = 0;
    return s;
  } else {
    // requires lpc >= U (the caller handles narrower groups)
    // reduce-scatter rounds: at each round a lane keeps half of its values and sends
    // the other half to its partner
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = a[u];
    int n = U, o = lpc >> 1, sel = 0;
#pragma unroll
    for (int r = 0; (1 << r) < U; ++r) {
      const bool hi = (li & o) != 0;
      const int h = n >> 1;
#pragma unroll
      for (int k = 0; k < U / 2; ++k) {
        if (k < h) {
          const double send = hi ? v[k] : v[k + h];
          const double got = __shfl_xor(send, o);
          v[k] = (hi ? v[k + h] : v[k]) + got;
        }
      }
      sel = sel * 2 + (hi ? 1 : 0);
      n = h;
      o >>= 1;
    }
    double s = v[0];
    for (; o > 0; o >>= 1) s += __shfl_xor(s, o);
    which = sel;
    return s;
  }
}

// Lane index (within a group) that reports value u after group_reduce<U>.
template <int U>
__device__ __forceinline__ int reporter(int u, int lpc) {
  if (U == 1) return u;
  int li = 0, o = lpc >> 1;
  for (int b = U >> 1; b > 0; b >>= 1) {
    if (u & b) li += o;
    o >>= 1;
  }
  return li;
}

// FP64 sums of four rows held by a full wavefront (64 lanes, one partial per row per
// lane), without LDS traffic: two half-wave swaps (v_permlane32_swap, v_permlane16_swap)
// scatter the rows so that 16-lane row r holds row r's partials, then four DPP rounds
// (xor 1, xor 2, mirror within 8, mirror within 16) sum each 16-lane row.  Every lane of
// 16-lane row r returns the total of row r; `which` = lane / 16.  The pairing tree is the
// same on every call, so results are reproducible bit for bit.
__device__ __forceinline__ double f64_join(uint32_t lo, uint32_t hi) {
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ uint32_t f64_lo(double v) { return (uint32_t)__double_as_longlong(v); }
__device__ __forceinline__ uint32_t f64_hi(double v) {
  return (uint32_t)((unsigned long long)__double_as_longlong(v) >> 32);
}
// lanes 0-31 get a[l] + a[l+32], lanes 32-63 get b[l-32] + b[l]
__device__ __forceinline__ double swap32_sum(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane32_swap(f64_lo(a), f64_lo(b), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(f64_hi(a), f64_hi(b), false, false);
  return f64_join(lo[0], hi[0]) + f64_join(lo[1], hi[1]);
}
// even 16-lane rows get a[l] + a[l+16], odd rows get b[l-16] + b[l]
__device__ __forceinline__ double swap16_sum(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane16_swap(f64_lo(a), f64_lo(b), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(f64_hi(a), f64_hi(b), false, false);
  return f64_join(lo[0], hi[0]) + f64_join(lo[1], hi[1]);
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  // every lane reads a lane of its own row, so no lane keeps its old value
  const uint32_t lo = __builtin_amdgcn_mov_dpp(f64_lo(v), CTRL, 0xF, 0xF, true);
  const uint32_t hi = __builtin_amdgcn_mov_dpp(f64_hi(v), CTRL, 0xF, 0xF, true);
  return f64_join(lo, hi);
}
__device__ __forceinline__ double wave_reduce4(const double (&a)[4], int& which) {
  const double s0 = swap32_sum(a[0], a[2]);   // rows 0-1 of the wave: a0, rows 2-3: a2
  const double s1 = swap32_sum(a[1], a[3]);   // rows 0-1: a1, rows 2-3: a3
  double t = swap16_sum(s0, s1);              // row r: a_r
  t += dpp_f64<0xB1>(t);                      // quad_perm [1,0,3,2]
  t += dpp_f64<0x4E>(t);                      // quad_perm [2,3,0,1]
  t += dpp_f64<0x141>(t);                     // row_half_mirror
  t += dpp_f64<0x140>(t);                     // row_mirror
  which = (int)(threadIdx.x & 63) >> 4;
  return t;
}

// FP64 sums of four rows held by lane groups of LPC = 8, 16 or 32 lanes (aligned to LPC),
// one partial per row per lane, without LDS traffic: reduce-scatter rounds that halve the
// rows a lane holds (v_permlane16_swap between the 16-lane halves of a 32-lane group,
// then DPP mirrors across 8-lane halves, quads or lane pairs), then DPP rounds inside the
// part of the group that holds one row.  Every lane returns the total of row `which`;
// lane u * LPC / 4 of the group holds row u.
template <int CTRL>
__device__ __forceinline__ double xchg_sum(bool keep_first, double a, double b) {
  // keep a and send b (keep_first), or keep b and send a; add the partner's sent value
  const double keep = keep_first ? a : b, send = keep_first ? b : a;
  return keep + dpp_f64<CTRL>(send);
}

template <int LPC>
__device__ __forceinline__ double group_reduce4_dpp(const double (&a)[4], int& which) {
  const int li = (int)(threadIdx.x & 63) & (LPC - 1);
  double t;
  if constexpr (LPC == 32) {
    const double s0 = swap16_sum(a[0], a[2]);       // 16-lane half 0: a0, half 1: a2
    const double s1 = swap16_sum(a[1], a[3]);       // half 0: a1, half 1: a3
    t = xchg_sum<0x140>((li & 8) == 0, s0, s1);     // row_mirror across 8-lane halves
    t += dpp_f64<0xB1>(t);                          // xor 1
    t += dpp_f64<0x4E>(t);                          // xor 2
    t += dpp_f64<0x141>(t);                         // row_half_mirror across quads
    which = ((li & 16) ? 2 : 0) + ((li & 8) ? 1 : 0);
  } else if constexpr (LPC == 16) {
    const bool lo = (li & 8) == 0;                  // 8-lane half 0 keeps a0, a1
    const double s0 = xchg_sum<0x140>(lo, a[0], a[2]);
    const double s1 = xchg_sum<0x140>(lo, a[1], a[3]);
    t = xchg_sum<0x141>((li & 4) == 0, s0, s1);     // row_half_mirror across quads
    t += dpp_f64<0xB1>(t);
    t += dpp_f64<0x4E>(t);
    which = ((li & 8) ? 2 : 0) + ((li & 4) ? 1 : 0);
  } else {
    static_assert(LPC == 8, "lane groups of 8, 16 or 32");
    const bool lo = (li & 4) == 0;                  // quad 0 keeps a0, a1
    const double s0 = xchg_sum<0x141>(lo, a[0], a[2]);
    const double s1 = xchg_sum<0x141>(lo, a[1], a[3]);
    t = xchg_sum<0x4E>((li & 2) == 0, s0, s1);      // quad_perm [2,3,0,1] across pairs
    t += dpp_f64<0xB1>(t);
    which = ((li & 4) ? 2 : 0) + ((li & 2) ? 1 : 0);
  }
  return t;
}

// FP64 sum over an aligned lane group of LPC = 8 or 16 lanes, every lane returning the
// total, by DPP rounds without LDS: xor 1, xor 2, then row_half_mirror (after two rounds a
// quad holds one value, so the mirror fetches the other quad's sum) and, for 16 lanes,
// row_mirror across the 8-lane halves.  Additions are commutative, so every lane of the
// group ends with the same bits.
template <int LPC>
__device__ __forceinline__ double group_allreduce_dpp(double s) {
  static_assert(LPC == 8 || LPC == 16, "lane groups of 8 or 16");
  s += dpp_f64<0xB1>(s);                     // quad_perm [1,0,3,2]
  s += dpp_f64<0x4E>(s);                     // quad_perm [2,3,0,1]
  s += dpp_f64<0x141>(s);                    // row_half_mirror
  if constexpr (LPC == 16) s += dpp_f64<0x140>(s);   // row_mirror
  return s;
}

// FP64 sum over an aligned lane group of lpc = 8, 16, 32 or 64 lanes, every lane returning
// the total: group_allreduce_dpp inside each 16-lane row, then v_permlane16_swap joins row
// pairs (32 lanes) and v_permlane32_swap the wave halves (64); each join adds the lower
// lanes' value first on both sides, so every lane of the group ends with the same bits.
// Other group sizes fall back to lane shuffles.
__device__ __forceinline__ double row_sum_dpp(double s, int lpc, int li) {
  if (lpc == 8) return group_allreduce_dpp<8>(s);
  if (lpc == 16) return group_allreduce_dpp<16>(s);
  if (lpc == 32 || lpc == 64) {
    double t = group_allreduce_dpp<16>(s);
    t = swap16_sum(t, t);
    if (lpc == 64) t = swap32_sum(t, t);
    return t;
  }
  double a1[1] = {s};
  int which = 0;
  return group_reduce<1>(a1, lpc, li, which);
}

// A neighbouring lane's value inside a 16-lane row (row_shl:1 -- lane l reads lane l + 1 --
// and row_shr:1 -- lane l reads lane l - 1; 0 past the row's ends), an exact copy.
__device__ __forceinline__ float from_next_lane(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x101, 0xF, 0xF, true));
}
__device__ __forceinline__ float from_prev_lane(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x111, 0xF, 0xF, true));
}

// The next / previous lane's value for rows of lpc lanes: DPP row shifts for rows of up to
// 16 lanes (inside one 16-lane DPP row), wave rotations (wave_rol:1, wave_ror:1) for 32 and
// 64, so that in a 64-lane row holding several chunks per lane the last lane reads lane 0
// (the next chunk's first bin) and lane 0 the last lane; only lanes whose neighbour is in
// their own row, or in the row's next / previous chunk, use the result.
template <class T>
__device__ __forceinline__ T next_lane_of_row(T v, int lpc) {
  if constexpr (sizeof(T) == 4) {
    const int x = __float_as_int(v);
    return __int_as_float(lpc <= 16 ? __builtin_amdgcn_mov_dpp(x, 0x101, 0xF, 0xF, true)
                                    : __builtin_amdgcn_mov_dpp(x, 0x134, 0xF, 0xF, true));
  } else {
    return lpc <= 16 ? dpp_f64<0x101>(v) : dpp_f64<0x134>(v);
  }
}
template <class T>
__device__ __forceinline__ T prev_lane_of_row(T v, int lpc) {
  if constexpr (sizeof(T) == 4) {
    const int x = __float_as_int(v);
    return __int_as_float(lpc <= 16 ? __builtin_amdgcn_mov_dpp(x, 0x111, 0xF, 0xF, true)
                                    : __builtin_amdgcn_mov_dpp(x, 0x13C, 0xF, 0xF, true));
  } else {
    return lpc <= 16 ? dpp_f64<0x111>(v) : dpp_f64<0x13C>(v);
  }
}

// F1 row chunks in and out: plain loads and stores, or (S, for launches whose rows do not
// fit in the Infinity Cache and are streamed through once per step) nontemporal ones that
// do not displace cached data.
template <bool S, class V> __device__ __forceinline__ V row_load(const V* p) {
  if constexpr (S) {
    typedef int i4 __attribute__((ext_vector_type(4)));
    const i4 x = __builtin_nontemporal_load(reinterpret_cast<const i4*>(p));
    return __builtin_bit_cast(V, x);
  } else {
    return *p;
  }
}
template <bool S, class V> __device__ __forceinline__ void row_store(const V& v, V* p) {
  if constexpr (S) {
    typedef int i4 __attribute__((ext_vector_type(4)));
    __builtin_nontemporal_store(__builtin_bit_cast(i4, v), reinterpret_cast<i4*>(p));
  } else {
    *p = v;
  }
}

struct Tile1D {
  int32_t run, node0, node1, cell0, cell1;
};

// A tile of the persistent batch launch with what its items need besides: the run's full
// K-step blocks in the launch and the steps left after them, and flags (bit 0: the tile
// has a right neighbour in its run; a left one exists when node0 > 0).  32 bytes, read in
// one go.
struct alignas(16) TbQueueTile {
  Tile1D tile;
  int32_t full, rest, flags;
};

// One 1D run as the step kernel sees it.  Ping-pong field buffers: at step n the
// current E/H live in buffer (n & 1) and the kernel writes buffer (n & 1) ^ 1.
template <class T> struct Run1D {
  T* E[2];
  T* H[2];
  T* J;            // [nx+1] normalised current dt/eps0 * J at the last half step
  T* df;           // [ncell][half] F1 on v > 0 bins
  const int32_t* cell_node;
  const T* tau;    // [ncell] dt * nu_mean
  const T* dens;   // [ncell] electron density
  const T* s_bin;  // [half] collision-frequency shape
  const T* b_bin;  // [half] 2 dt (e/m) dF0/dv (per unit density)
  const double* w_bin;  // [half] moment weight (dt/eps0)(-2 e dv) v_j
  int32_t nx, ncell, half, bc;
  T S, q;
  int32_t src_node;
  double src_amp, src_w, src_tau, src_t0, dt;
  int64_t step_limit;
  int32_t nprobe, probe_cap;
  int32_t probe_node[kMaxProbes];
  int32_t probe_field[kMaxProbes];
  T* probe_buf;    // [nprobe][probe_cap]
  // training-pair taps: (E^n, J^{n+1/2}) at chosen plasma nodes after every step
  int32_t ntap;
  int32_t tap_node[kMaxTaps];
  T* tap_buf;      // [ntap][tap_cap][2]
  int64_t tap_cap;
  int32_t* status; // bit 0: a non-finite E value was produced
  // kinetic model: 0 linear F1 (df: [ncell][half]); 1 full distribution (df:
  // [ncell][2 half], odd then even half of f - n fhat; b_bin then holds the equilibrium
  // flux differences -(dt/dv)(-e/m)(fhat_{k+1} - fhat_{k-1}) per unit density and field)
  int32_t model;
  T kc;            // full model: -(e/m) dt / dv, the velocity CFL number per unit E;
                   // two-term model: dt (e/m) / gam
  // two-term model (model 2): l = 0 update factor dt e / (3 m v_k^2 gam) and the face
  // weight v_{k+1/2}^2 / 2 of each speed bin (both 0 in the padding, the latter also at vmax)
  const T* c_bin;
  const T* v2h_bin;
};

// One 2D TEz run.  Ex [ny+1][nx] at (i+1/2, j), Ey [ny][nx+1] at (i, j+1/2),
// Hz [ny][nx] at (i+1/2, j+1/2), normalised (E in V/m, Hz scaled by eta0, psi scaled
// to V/m, current by dt/eps0).  CPML memory is stored only in the layer strips.
template <class T> struct Run2D {
  T* Ex;
  T* Ey;
  T* Hz;
  T* psi_hzx;      // [ny][2m]   Hz points inside an x layer
  T* psi_hzy;      // [2m][nx]   Hz points inside a y layer
  T* psi_exy;      // [2m][nx]   Ex points inside a y layer
  T* psi_eyx;      // [ny][2m]   Ey points inside an x layer
  T* Jcx;          // [ny][nx]   cell-centre current (normalised), 0 off plasma
  T* Jcy;
  T* df;           // [ncell][nv][nv/2]  F1 on the vy > 0 half plane
  const int32_t* cell_idx;   // [ncell] j * nx + i
  const T* tau;    // [ncell] dt * nu_mean
  const T* dens;   // [ncell]
  const T* s_bin;  // [nv*nv/2] collision-frequency shape
  const T* bx_bin; // [nv*nv/2] 2 dt (e/m) dF0/dvx per unit density
  const T* by_bin; // [nv*nv/2] 2 dt (e/m) dF0/dvy per unit density
  const double* wx_bin;  // moment weights (dt/eps0)(-2 e dv^2) vx
  const double* wy_bin;  // moment weights (dt/eps0)(-2 e dv^2) vy
  // CPML profiles: b, a (dimensionless), 1/kappa; e side at integer positions, h side
  // at half positions
  const T *bex, *aex, *rkex, *bhx, *ahx, *rkhx;
  const T *bey, *aey, *rkey, *bhy, *ahy, *rkhy;
  int32_t nx, ny, m, ncell, half, cells_per_block, nbk;
  int32_t hrows, erows;   // rows per thread of the Hz and E updates (1 or 4)
  T S;
  int32_t src_kind, src_i, src_j;
  double src_amp, src_w, src_tau, src_t0, dt;
  int32_t nprobe, probe_cap;
  int32_t probe_field[kMaxProbes];
  int32_t probe_i[kMaxProbes];
  int32_t probe_j[kMaxProbes];
  T* probe_buf;
};

// One 3D run (the Yee cube with the CPML on all faces, section 2, and the speed-grid F1
// of section 5.3).  Storage [k][j][i], i fastest: Ex [nz+1][ny+1][nx], Ey [nz+1][ny][nx+1],
// Ez [nz][ny+1][nx+1], Hx [nz][ny][nx+1], Hy [nz][ny+1][nx], Hz [nz+1][ny][nx]; E (and J)
// components contiguous, so a plasma point is one index into Ex..Ez.  Normalised: H by
// eta0, J by dt/eps0, psi by dx.  Each psi array lives only in the layer of its derivative
// axis: that axis's extent is replaced by 2m (first m: the low layer, then the high one).
template <class T> struct Run3D {
  T *Ex, *Ey, *Ez, *Hx, *Hy, *Hz, *Jx, *Jy, *Jz;
  T *p_exy, *p_exz, *p_eyz, *p_eyx, *p_ezx, *p_ezy;
  T *p_hxz, *p_hxy, *p_hyx, *p_hyz, *p_hzy, *p_hzx;
  T* df;                  // [np][row] F1 on the speed grid, row >= vdim (padding stays 0)
  const int32_t* pidx;    // [np] index of the plasma point into the E (and J) arrays
  const T* tau;           // [np] dt * nu_mean
  const T* dens;          // [np] electron density
  const T* s_bin;         // [row] collision-frequency shape (0 in the padding)
  const T* b_bin;         // [row] 2 dt (e/m) dF0/dv per unit density (0 in the padding)
  const double* w_bin;    // [row] (dt/eps0)(-e)(4 pi / 3) gam v^3 (0 in the padding)
  // CPML profiles per axis: e side at integer positions, h side at half positions
  const T *bex, *aex, *rkex, *bhx, *ahx, *rkhx;
  const T *bey, *aey, *rkey, *bhy, *ahy, *rkhy;
  const T *bez, *aez, *rkez, *bhz, *ahz, *rkhz;
  int32_t nx, ny, nz, m, np, row;
  T S;
  int32_t src_kind, src_i, src_j, src_k;
  double src_amp, src_w, src_tau, src_t0, dt;
  // two-term model (F0 evolving per plasma cell); unused by the linear model
  T* f0;                  // [nc][row] F0 - n F0hat of the plasma cells
  T* en;                  // [np] E^n of every plasma point, kept for the l = 0 update
  const int32_t* pcell;   // [np][4] F0 rows of the four cells around the point's edge
  const int32_t* cedge;   // [nc][12][2] (plasma point, its E index) of the cell's edges,
                          // (-1, 0) for an edge without one
  const T* c_bin;         // [row] dt (e / 3m) / (v_k^2 gam) (0 in the padding)
  const T* v2h_bin;       // [row] v_{k+1/2}^2 / 2 on the inner speed faces, else 0
  int32_t* status;        // |= 2 when the field breaks the explicit exchange limit
  T kc;                   // dt (e/m) / gam
  int32_t nc, model;
};

}  // namespace fdtdp
