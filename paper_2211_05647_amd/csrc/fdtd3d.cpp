// fdtd3d.cpp -- host side of the 3D path: validation, FP64 tables (speed grid, isotropic
// F0 -- Maxwellian or Druyvesteyn -- and its derivative, collision shape, moment weights,
// CPML profiles of section 2 per axis), plasma points (and, for the two-term model, plasma
// cells with their edges), workspace layout, launches and readback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"
#include "host_internal.h"

namespace fdtdp {

template <class T>
hipError_t launch_step3d_t(const void* run, int nx, int ny, int nz, int np, int kin_groups,
                           int nc, int f0_groups, bool two_term, int64_t step,
                           const int32_t* pix, int nprobe, void* ring, int cap,
                           hipStream_t stream);

struct Host3D {
  fdtd_grid g;
  fdtd_profile p;
  fdtd_source s;
  std::vector<double> ne, nu;
  int nx = 0, ny = 0, nz = 0, m = 0, vdim = 0, row = 0, np = 0, es = 4;
  bool two_term = false;
  int nc = 0;             // plasma cells (two-term model)
  double dt = 0;
  size_t nE[3] = {0, 0, 0}, nH[3] = {0, 0, 0};
  std::vector<int32_t> pidx;
  std::vector<double> pn, pnu;
  std::vector<int32_t> pcell, cedge;   // [np][4] cell rows, [nc][12][2] edges (two-term)
  std::vector<int32_t> doc;            // readback row of every stored point row
  // workspace offsets
  size_t off_E = 0, off_H = 0, off_J = 0, off_psi[12] = {}, off_df = 0;
  size_t off_f0 = 0, off_en = 0, off_status = 0;
  size_t off_pidx = 0, off_tau = 0, off_dens = 0, off_s = 0, off_b = 0, off_w = 0, off_prof = 0;
  size_t off_pcell = 0, off_cedge = 0, off_c = 0, off_v2h = 0;
  // probes: E index of each probe point, ring of probe_cap samples per probe
  int max_probes = 0, probe_cap = 0, nprobe = 0;
  size_t off_probe = 0, off_pix = 0;
  char* ws = nullptr;
  size_t state_end = 0, total = 0;
  int kin_groups = 1, f0_groups = 1;
  alignas(16) unsigned char run[sizeof(Run3D<double>)];
};

namespace {

// Plasma points: every E point that is updated (not on a face its component is
// tangential to) and whose edge's four cells have a positive mean density -- for the
// two-term model, whose four cells all have a positive density, so that each point's F0
// comes from plasma cells and hands its work back to them.  Order: Ex points, then Ey,
// then Ez, each in storage order (the readback order).  The two-term model then stores
// them by lattice site (k, j, i, component), so that neighbouring rows share cells and a
// cell's 12 edges lie in two planes of sites; `doc` maps a stored row to its readback
// row.  Plasma cells (two-term): ne > 0, in storage order.
void find_points(Host3D* h) {
  const int nx = h->nx, ny = h->ny, nz = h->nz;
  const size_t ncell = (size_t)nx * ny * nz;
  std::vector<int32_t> crow;
  h->nc = 0;
  if (h->two_term) {
    crow.assign(ncell, -1);
    for (size_t q = 0; q < ncell; ++q)
      if (h->ne[q] > 0.0) crow[q] = h->nc++;
  }
  auto cell = [&](int i, int j, int k) { return ((size_t)k * ny + j) * nx + i; };
  auto add = [&](size_t at, size_t c0, size_t c1, size_t c2, size_t c3) {
    const double n = 0.25 * (h->ne[c0] + h->ne[c1] + h->ne[c2] + h->ne[c3]);
    const bool all = h->ne[c0] > 0.0 && h->ne[c1] > 0.0 && h->ne[c2] > 0.0 && h->ne[c3] > 0.0;
    if (h->two_term ? all : n > 0.0) {
      h->pidx.push_back((int32_t)at);
      h->pn.push_back(n);
      h->pnu.push_back(0.25 * (h->nu[c0] + h->nu[c1] + h->nu[c2] + h->nu[c3]));
      if (h->two_term)
        for (size_t c : {c0, c1, c2, c3}) h->pcell.push_back(crow[c]);
    }
  };
  h->pidx.clear();
  h->pn.clear();
  h->pnu.clear();
  h->pcell.clear();
  for (int k = 1; k < nz; ++k)
    for (int j = 1; j < ny; ++j)
      for (int i = 0; i < nx; ++i)
        add(((size_t)k * (ny + 1) + j) * nx + i, cell(i, j - 1, k - 1), cell(i, j, k - 1),
            cell(i, j - 1, k), cell(i, j, k));
  const size_t oy = h->nE[0];
  for (int k = 1; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 1; i < nx; ++i)
        add(oy + ((size_t)k * ny + j) * (nx + 1) + i, cell(i - 1, j, k - 1), cell(i, j, k - 1),
            cell(i - 1, j, k), cell(i, j, k));
  const size_t oz = h->nE[0] + h->nE[1];
  for (int k = 0; k < nz; ++k)
    for (int j = 1; j < ny; ++j)
      for (int i = 1; i < nx; ++i)
        add(oz + ((size_t)k * (ny + 1) + j) * (nx + 1) + i, cell(i - 1, j - 1, k),
            cell(i, j - 1, k), cell(i - 1, j, k), cell(i, j, k));
  h->np = (int)h->pidx.size();
  h->doc.resize(h->np);
  for (int p = 0; p < h->np; ++p) h->doc[p] = p;
  if (h->two_term) {
    // lattice site of each point: E index -> (component, i, j, k)
    std::vector<int64_t> key(h->np);
    const size_t X = nx, Y = ny;
    for (int p = 0; p < h->np; ++p) {
      size_t at = (size_t)h->pidx[p];
      int c = 0;
      size_t i, j, k;
      if (at < h->nE[0]) {
        i = at % X; j = (at / X) % (Y + 1); k = at / (X * (Y + 1));
      } else if (at < h->nE[0] + h->nE[1]) {
        at -= h->nE[0]; c = 1;
        i = at % (X + 1); j = (at / (X + 1)) % Y; k = at / ((X + 1) * Y);
      } else {
        at -= h->nE[0] + h->nE[1]; c = 2;
        i = at % (X + 1); j = (at / (X + 1)) % (Y + 1); k = at / ((X + 1) * (Y + 1));
      }
      key[p] = ((int64_t)((k * (Y + 1) + j) * (X + 1) + i)) * 3 + c;
    }
    std::stable_sort(h->doc.begin(), h->doc.end(), [&](int a, int b) { return key[a] < key[b]; });
    std::vector<int32_t> pidx(h->np), pcell((size_t)4 * h->np);
    std::vector<double> pn(h->np), pnu(h->np);
    for (int q = 0; q < h->np; ++q) {
      const int p = h->doc[q];
      pidx[q] = h->pidx[p];
      pn[q] = h->pn[p];
      pnu[q] = h->pnu[p];
      for (int u = 0; u < 4; ++u) pcell[(size_t)4 * q + u] = h->pcell[(size_t)4 * p + u];
    }
    h->pidx.swap(pidx);
    h->pn.swap(pn);
    h->pnu.swap(pnu);
    h->pcell.swap(pcell);
  }
  h->cedge.assign((size_t)h->nc * 24, 0);
  for (size_t q = 0; q < h->cedge.size(); q += 2) h->cedge[q] = -1;
  if (h->two_term) {
    std::vector<int> fill(h->nc, 0);
    for (int p = 0; p < h->np; ++p)
      for (int q = 0; q < 4; ++q) {
        const int r = h->pcell[(size_t)4 * p + q];
        const size_t at = (size_t)24 * r + 2 * fill[r]++;   // a cell has 12 edges
        h->cedge[at] = p;
        h->cedge[at + 1] = h->pidx[p];
      }
  }
}

void layout(Host3D* h) {
  Carver cv;
  const size_t es = h->es, X = h->nx, Y = h->ny, Z = h->nz, m2 = 2 * (size_t)std::max(h->m, 1);
  h->off_E = cv.take((h->nE[0] + h->nE[1] + h->nE[2]) * es);
  h->off_H = cv.take((h->nH[0] + h->nH[1] + h->nH[2]) * es);
  h->off_J = cv.take((h->nE[0] + h->nE[1] + h->nE[2]) * es);
  // psi strips: ex_y ex_z ey_z ey_x ez_x ez_y hx_z hx_y hy_x hy_z hz_y hz_x
  const size_t sizes[12] = {
      (Z + 1) * m2 * X, m2 * (Y + 1) * X, m2 * Y * (X + 1), (Z + 1) * Y * m2,
      Z * (Y + 1) * m2, Z * m2 * (X + 1), m2 * Y * (X + 1), Z * m2 * (X + 1),
      Z * (Y + 1) * m2, m2 * (Y + 1) * X, (Z + 1) * m2 * X, (Z + 1) * Y * m2};
  for (int q = 0; q < 12; ++q) h->off_psi[q] = cv.take(sizes[q] * es);
  h->off_df = cv.take((size_t)std::max(h->np, 1) * h->row * es);
  h->off_f0 = cv.take((size_t)std::max(h->nc, 1) * h->row * es);
  h->off_en = cv.take((size_t)std::max(h->np, 1) * es);
  h->off_status = cv.take(4);
  h->state_end = cv.size();
  h->off_pidx = cv.take((size_t)std::max(h->np, 1) * 4);
  h->off_tau = cv.take((size_t)std::max(h->np, 1) * es);
  h->off_dens = cv.take((size_t)std::max(h->np, 1) * es);
  h->off_s = cv.take((size_t)h->row * es);
  h->off_b = cv.take((size_t)h->row * es);
  h->off_w = cv.take((size_t)h->row * 8);
  h->off_prof = cv.take((size_t)6 * (X + Y + Z + 3) * es);
  h->off_pcell = cv.take((size_t)std::max(h->np, 1) * 16);
  h->off_cedge = cv.take((size_t)std::max(h->nc, 1) * 96);
  h->off_c = cv.take((size_t)h->row * es);
  h->off_v2h = cv.take((size_t)h->row * es);
  h->off_probe = cv.take((size_t)std::max(h->max_probes, 1) * std::max(h->probe_cap, 1) * es);
  h->off_pix = cv.take((size_t)std::max(h->max_probes, 1) * 4);
  h->total = cv.size() + 256;
}

Host3D* new_host(const fdtd_grid* g, const fdtd_profile* p, const fdtd_source* s,
                 int max_probes, int probe_cap) {
  Host3D* h = new (std::nothrow) Host3D();
  if (!h) return nullptr;
  h->max_probes = max_probes;
  h->probe_cap = probe_cap;
  h->g = *g;
  h->p = *p;
  if (s) h->s = *s; else std::memset(&h->s, 0, sizeof h->s);
  h->nx = g->nx;
  h->ny = g->ny;
  h->nz = g->nz;
  h->m = g->boundary == FDTD_BC_CPML ? g->cpml_cells : 0;
  h->vdim = p->nv;
  h->two_term = p->kinetic == FDTD_KINETIC_TWO_TERM;
  h->es = g->precision == FDTD_FP64 ? 8 : 4;
  const int vpl = 16 / h->es;
  int row = vpl;
  while (row < h->vdim) row *= 2;
  h->row = row;
  h->dt = g->courant * g->dx / kC0;
  const size_t X = h->nx, Y = h->ny, Z = h->nz;
  h->nE[0] = X * (Y + 1) * (Z + 1);
  h->nE[1] = (X + 1) * Y * (Z + 1);
  h->nE[2] = (X + 1) * (Y + 1) * Z;
  h->nH[0] = (X + 1) * Y * Z;
  h->nH[1] = X * (Y + 1) * Z;
  h->nH[2] = X * Y * (Z + 1);
  const size_t nc = X * Y * Z;
  h->ne.assign(p->ne, p->ne + nc);
  h->nu.assign(p->nu_mean, p->nu_mean + nc);
  h->p.ne = h->ne.data();
  h->p.nu_mean = h->nu.data();
  find_points(h);
  layout(h);
  return h;
}

template <class T>
int upload(Host3D* h, char* ws, hipStream_t st, const std::vector<ProbeInfo>& probes) {
  const int nx = h->nx, ny = h->ny, nz = h->nz, m = h->m, vdim = h->vdim, row = h->row;
  const double dt = h->dt;
  // speed grid and F0 (FP64), rounded once
  const double vth = std::sqrt(kQe * h->p.te_ev / kMe);
  const double gam = h->p.vmax_over_vth * vth / vdim;
  std::vector<double> v(vdim), F0(vdim), dF0(vdim);
  double vd4 = 0.0;
  if (h->p.f0_model == FDTD_F0_DRUYVESTEYN) {
    const double vd2 = 3.0 * vth * vth * std::tgamma(0.75) / std::tgamma(1.25);
    vd4 = vd2 * vd2;
  }
  double norm = 0.0, mean = 0.0;
  for (int k = 0; k < vdim; ++k) {
    v[k] = (k + 0.5) * gam;
    const double u = v[k];
    F0[k] = h->p.f0_model == FDTD_F0_DRUYVESTEYN ? std::exp(-u * u * u * u / vd4)
                                                 : std::exp(-u * u / (2.0 * vth * vth));
    norm += 4.0 * M_PI * gam * u * u * F0[k];
  }
  for (int k = 0; k < vdim; ++k) {
    F0[k] /= norm;
    const double u = v[k];
    dF0[k] = h->p.f0_model == FDTD_F0_DRUYVESTEYN ? -4.0 * u * u * u * F0[k] / vd4
                                                  : -u * F0[k] / (vth * vth);
    mean += 4.0 * M_PI * gam * u * u * u * F0[k];
  }
  std::vector<T> s(row, T(0)), b(row, T(0)), cb(row, T(0)), v2h(row, T(0));
  std::vector<double> w(row, 0.0);
  for (int k = 0; k < vdim; ++k) {
    s[k] = (T)(h->p.nu_model == FDTD_NU_HARD_SPHERE ? v[k] / mean : 1.0);
    b[k] = (T)(2.0 * dt * (kQe / kMe) * dF0[k]);
    // linear model: v^3 as section 5.3 prints it; two-term: the mean of v^3 on the two
    // speed faces (none at vmax), the adjoint of the l = 0 flux, so that the work the
    // field does equals the heat the cells gain
    const double lo = k * gam, hi = (k + 1) * gam;
    const double cube = h->two_term ? 0.5 * (lo * lo * lo + (k + 1 < vdim ? hi * hi * hi : 0.0))
                                    : v[k] * v[k] * v[k];
    w[k] = (dt / kEps0) * (-kQe) * (4.0 * M_PI / 3.0) * gam * cube;
    if (h->two_term) {
      cb[k] = (T)(dt * kQe / (3.0 * kMe) / (v[k] * v[k] * gam));
      v2h[k] = (T)(k + 1 < vdim ? 0.5 * hi * hi : 0.0);
    }
  }
  std::vector<T> tau(h->np), dens(h->np);
  for (int q = 0; q < h->np; ++q) {
    tau[q] = (T)(dt * h->pnu[q]);
    dens[q] = (T)h->pn[q];
  }
  std::vector<T> prof((size_t)6 * (nx + ny + nz + 3), T(0));
  T* px = prof.data();
  T* py = px + 6 * (nx + 1);
  T* pz = py + 6 * (ny + 1);
  axis_profile<T>(h->g, nx, m, dt, px, px + (nx + 1), px + 2 * (nx + 1), px + 3 * (nx + 1),
                  px + 4 * (nx + 1), px + 5 * (nx + 1));
  axis_profile<T>(h->g, ny, m, dt, py, py + (ny + 1), py + 2 * (ny + 1), py + 3 * (ny + 1),
                  py + 4 * (ny + 1), py + 5 * (ny + 1));
  axis_profile<T>(h->g, nz, m, dt, pz, pz + (nz + 1), pz + 2 * (nz + 1), pz + 3 * (nz + 1),
                  pz + 4 * (nz + 1), pz + 5 * (nz + 1));
  hipError_t e = hipMemsetAsync(ws, 0, h->state_end, st);
  if (e) return hip_fail(e, "clear 3D state");
  auto put = [&](size_t off, const void* src, size_t bytes) {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(ws + off, src, bytes, hipMemcpyHostToDevice, st);
  };
  if ((e = put(h->off_pidx, h->pidx.data(), h->pidx.size() * 4)) ||
      (e = put(h->off_tau, tau.data(), tau.size() * sizeof(T))) ||
      (e = put(h->off_dens, dens.data(), dens.size() * sizeof(T))) ||
      (e = put(h->off_s, s.data(), row * sizeof(T))) ||
      (e = put(h->off_b, b.data(), row * sizeof(T))) ||
      (e = put(h->off_w, w.data(), row * 8)) ||
      (e = put(h->off_prof, prof.data(), prof.size() * sizeof(T))) ||
      (e = put(h->off_pcell, h->pcell.data(), h->pcell.size() * 4)) ||
      (e = put(h->off_cedge, h->cedge.data(), h->cedge.size() * 4)) ||
      (e = put(h->off_c, cb.data(), row * sizeof(T))) ||
      (e = put(h->off_v2h, v2h.data(), row * sizeof(T))))
    return hip_fail(e, "upload 3D tables");
  // probe points: the E index is kept in ProbeInfo::i
  std::vector<int32_t> pix;
  for (const ProbeInfo& pi : probes) pix.push_back(pi.i);
  h->nprobe = (int)pix.size();
  h->ws = ws;
  if ((e = put(h->off_pix, pix.data(), pix.size() * 4))) return hip_fail(e, "upload 3D probes");

  Run3D<T> R;
  std::memset(&R, 0, sizeof R);
  T* E = reinterpret_cast<T*>(ws + h->off_E);
  T* H = reinterpret_cast<T*>(ws + h->off_H);
  T* J = reinterpret_cast<T*>(ws + h->off_J);
  R.Ex = E; R.Ey = E + h->nE[0]; R.Ez = E + h->nE[0] + h->nE[1];
  R.Hx = H; R.Hy = H + h->nH[0]; R.Hz = H + h->nH[0] + h->nH[1];
  R.Jx = J; R.Jy = J + h->nE[0]; R.Jz = J + h->nE[0] + h->nE[1];
  T** ps[12] = {&R.p_exy, &R.p_exz, &R.p_eyz, &R.p_eyx, &R.p_ezx, &R.p_ezy,
                &R.p_hxz, &R.p_hxy, &R.p_hyx, &R.p_hyz, &R.p_hzy, &R.p_hzx};
  for (int q = 0; q < 12; ++q) *ps[q] = reinterpret_cast<T*>(ws + h->off_psi[q]);
  R.df = reinterpret_cast<T*>(ws + h->off_df);
  R.pidx = reinterpret_cast<const int32_t*>(ws + h->off_pidx);
  R.tau = reinterpret_cast<const T*>(ws + h->off_tau);
  R.dens = reinterpret_cast<const T*>(ws + h->off_dens);
  R.s_bin = reinterpret_cast<const T*>(ws + h->off_s);
  R.b_bin = reinterpret_cast<const T*>(ws + h->off_b);
  R.w_bin = reinterpret_cast<const double*>(ws + h->off_w);
  const T* dx_ = reinterpret_cast<const T*>(ws + h->off_prof);
  const T* dy_ = dx_ + 6 * (nx + 1);
  const T* dz_ = dy_ + 6 * (ny + 1);
  R.bex = dx_; R.aex = dx_ + (nx + 1); R.rkex = dx_ + 2 * (nx + 1);
  R.bhx = dx_ + 3 * (nx + 1); R.ahx = dx_ + 4 * (nx + 1); R.rkhx = dx_ + 5 * (nx + 1);
  R.bey = dy_; R.aey = dy_ + (ny + 1); R.rkey = dy_ + 2 * (ny + 1);
  R.bhy = dy_ + 3 * (ny + 1); R.ahy = dy_ + 4 * (ny + 1); R.rkhy = dy_ + 5 * (ny + 1);
  R.bez = dz_; R.aez = dz_ + (nz + 1); R.rkez = dz_ + 2 * (nz + 1);
  R.bhz = dz_ + 3 * (nz + 1); R.ahz = dz_ + 4 * (nz + 1); R.rkhz = dz_ + 5 * (nz + 1);
  R.nx = nx; R.ny = ny; R.nz = nz; R.m = m; R.np = h->np; R.row = row;
  R.S = (T)h->g.courant;
  const fdtd_source& src = h->s;
  R.src_kind = (src.kind != FDTD_SRC_NONE && src.amplitude != 0.0) ? src.kind : 0;
  R.src_i = src.i; R.src_j = src.j; R.src_k = src.k;
  R.src_amp = src.amplitude;
  R.src_w = 2.0 * M_PI * src.f_hz;
  R.src_tau = src.kind != FDTD_SRC_NONE ? src.tau_s : 1.0;
  R.src_t0 = src.t0_s;
  R.dt = dt;
  R.f0 = reinterpret_cast<T*>(ws + h->off_f0);
  R.en = reinterpret_cast<T*>(ws + h->off_en);
  R.pcell = reinterpret_cast<const int32_t*>(ws + h->off_pcell);
  R.cedge = reinterpret_cast<const int32_t*>(ws + h->off_cedge);
  R.c_bin = reinterpret_cast<const T*>(ws + h->off_c);
  R.v2h_bin = reinterpret_cast<const T*>(ws + h->off_v2h);
  R.status = reinterpret_cast<int32_t*>(ws + h->off_status);
  R.kc = (T)(dt * (kQe / kMe) / gam);
  R.nc = h->nc;
  R.model = h->two_term ? FDTD_KINETIC_TWO_TERM : FDTD_KINETIC_LINEAR;
  std::memcpy(h->run, &R, sizeof R);
  // lane groups of row / VPL lanes, 64 / that many rows per wavefront and pass
  int cus = 256, dev = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int rows_per_block = 4 * (64 / (row / Vec<T>::n));
  h->kin_groups = std::max(1, std::min((h->np + rows_per_block - 1) / rows_per_block, 8 * cus));
  // the two-term launches renumber their work-groups per XCD: a multiple of 8
  h->f0_groups = std::max(1, std::min((h->nc + rows_per_block - 1) / rows_per_block, 8 * cus));
  if (h->two_term) {
    h->kin_groups = (h->kin_groups + 7) / 8 * 8;
    h->f0_groups = (h->f0_groups + 7) / 8 * 8;
  }
  return FDTD_OK;
}

}  // namespace

int validate_3d(const fdtd_grid* g, const fdtd_profile* p, const fdtd_source* s) {
  if (!g || !p) return fail(FDTD_EINVAL, "null grid or profile");
  if (g->nx < 4 || g->ny < 4 || g->nz < 4 || g->nx > 4096 || g->ny > 4096 || g->nz > 4096)
    return fail(FDTD_EINVAL, "3D nx, ny, nz must lie in [4, 4096]");
  if ((double)(g->nx + 1) * (g->ny + 1) * (g->nz + 1) > 2.0e9)
    return fail(FDTD_EINVAL, "3D grid too large for 32-bit point indices");
  if (!(g->dx > 0.0) || !std::isfinite(g->dx)) return fail(FDTD_EINVAL, "dx must be > 0");
  if (!(g->courant > 0.0) || g->courant > 1.0 / std::sqrt(3.0))
    return fail(FDTD_EINVAL, "3D Courant number must lie in (0, 1/sqrt(3)], got %g", g->courant);
  if (g->precision != FDTD_FP32 && g->precision != FDTD_FP64)
    return fail(FDTD_EINVAL, "unknown precision %d", g->precision);
  if (g->boundary == FDTD_BC_CPML) {
    if (g->cpml_cells < 1 || 2 * g->cpml_cells >= std::min(g->nx, std::min(g->ny, g->nz)))
      return fail(FDTD_EINVAL, "cpml_cells out of range");
    if (!(g->cpml_order > 0) || !(g->cpml_sigma_factor >= 0) || !(g->cpml_kappa_max >= 1) ||
        !(g->cpml_alpha_min >= 0) || !(g->cpml_alpha_max >= 0) ||
        !std::isfinite(g->cpml_order + g->cpml_sigma_factor + g->cpml_kappa_max +
                       g->cpml_alpha_min + g->cpml_alpha_max))
      return fail(FDTD_EINVAL, "bad CPML parameters");
  } else if (g->boundary != FDTD_BC_PEC) {
    return fail(FDTD_EINVAL, "3D boundary must be PEC or CPML");
  }
  if (p->nv < 1 || p->nv > 64) return fail(FDTD_EINVAL, "3D nv (speeds) must lie in [1, 64]");
  if (!(p->te_ev > 0.0) || !(p->vmax_over_vth > 0.0))
    return fail(FDTD_EINVAL, "te_ev and vmax_over_vth must be > 0");
  if (p->nu_model != FDTD_NU_HARD_SPHERE && p->nu_model != FDTD_NU_CONST)
    return fail(FDTD_EINVAL, "unknown nu_model %d", p->nu_model);
  if (p->f0_model != FDTD_F0_MAXWELL && p->f0_model != FDTD_F0_DRUYVESTEYN)
    return fail(FDTD_EINVAL, "unknown f0_model %d", p->f0_model);
  if (p->closure != FDTD_CLOSURE_KINETIC) return fail(FDTD_EINVAL, "3D runs take the kinetic closure");
  if (p->kinetic != FDTD_KINETIC_LINEAR && p->kinetic != FDTD_KINETIC_TWO_TERM)
    return fail(FDTD_EINVAL, "3D runs take the linear or the two-term kinetic model");
  if (p->kinetic == FDTD_KINETIC_TWO_TERM && p->nv < 2)
    return fail(FDTD_EINVAL, "the two-term model needs nv >= 2 speeds");
  if (!p->ne || !p->nu_mean) return fail(FDTD_EINVAL, "null ne or nu_mean");
  const size_t n = (size_t)g->nx * g->ny * g->nz;
  for (size_t k = 0; k < n; ++k) {
    if (!(p->ne[k] >= 0.0) || !std::isfinite(p->ne[k]))
      return fail(FDTD_EINVAL, "ne[%zu] must be finite and >= 0", k);
    if (!(p->nu_mean[k] >= 0.0) || !std::isfinite(p->nu_mean[k]))
      return fail(FDTD_EINVAL, "nu_mean[%zu] must be finite and >= 0", k);
  }
  // The two-term point set (E points whose four cells all hold plasma) with plasma inside
  // the x or y absorbing layers carries a mode that grows until the fields overflow (the
  // FP64 reference grows alike), so such a profile is refused rather than run.
  if (p->kinetic == FDTD_KINETIC_TWO_TERM && g->boundary == FDTD_BC_CPML) {
    const int m = g->cpml_cells;
    for (int k = 0; k < g->nz; ++k)
      for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i) {
          const bool side = i < m || i >= g->nx - m || j < m || j >= g->ny - m;
          if (side && p->ne[((size_t)k * g->ny + j) * g->nx + i] > 0.0)
            return fail(FDTD_EINVAL,
                        "3D two-term plasma inside the x/y absorbing layers (cell i=%d j=%d "
                        "k=%d): keep ne = 0 in the outer %d cells of x and y", i, j, k, m);
        }
  }
  if (s && s->kind != FDTD_SRC_NONE) {
    if (s->kind != FDTD_SRC_LINE_SOFT && s->kind != FDTD_SRC_POINT_SOFT)
      return fail(FDTD_EINVAL, "3D source must be a sheet (LINE) or a point");
    if (s->k < 1 || s->k > g->nz - 1) return fail(FDTD_EINVAL, "source plane k out of [1, nz-1]");
    if (s->kind == FDTD_SRC_POINT_SOFT &&
        (s->i < 0 || s->i >= g->nx || s->j < 1 || s->j > g->ny - 1))
      return fail(FDTD_EINVAL, "3D point source must sit on an updated Ex point");
    if (!(s->tau_s > 0.0) || !std::isfinite(s->amplitude) || !std::isfinite(s->f_hz) ||
        !std::isfinite(s->t0_s))
      return fail(FDTD_EINVAL, "bad source parameters");
  }
  return FDTD_OK;
}

size_t workspace_3d(const fdtd_grid* g, const fdtd_profile* p, int max_probes, int probe_cap) {
  Host3D* h = new_host(g, p, nullptr, max_probes, probe_cap);
  if (!h) return 0;
  const size_t n = h->total;
  delete h;
  return n;
}

Host3D* make_3d(const fdtd_grid* g, const fdtd_profile* p, const fdtd_source* s,
                int max_probes, int probe_cap, size_t* state_bytes, size_t* probe_off) {
  Host3D* h = new_host(g, p, s, max_probes, probe_cap);
  if (!h) return nullptr;
  *state_bytes = h->state_end;
  *probe_off = h->off_probe;
  return h;
}

int upload_3d(Host3D* h, char* ws, hipStream_t stream, const std::vector<ProbeInfo>& probes) {
  return h->es == 8 ? upload<double>(h, ws, stream, probes) : upload<float>(h, ws, stream, probes);
}

// Flat E index of the E point (i, j, k) of component `field` (EX, EY, EZ), each in its
// own storage shape.
int probe_index_3d(const Host3D* h, int field, int i, int j, int k, int32_t* at) {
  const size_t X = h->nx, Y = h->ny, Z = h->nz;
  size_t nxc, nyc, nzc, base;
  switch (field) {
    case FDTD_F_EX: nxc = X; nyc = Y + 1; nzc = Z + 1; base = 0; break;
    case FDTD_F_EY: nxc = X + 1; nyc = Y; nzc = Z + 1; base = h->nE[0]; break;
    case FDTD_F_EZ: nxc = X + 1; nyc = Y + 1; nzc = Z; base = h->nE[0] + h->nE[1]; break;
    default: return fail(FDTD_EINVAL, "3D probes record EX, EY or EZ");
  }
  if (i < 0 || j < 0 || k < 0 || (size_t)i >= nxc || (size_t)j >= nyc || (size_t)k >= nzc)
    return fail(FDTD_ERANGE, "probe index (%d, %d, %d) out of range", i, j, k);
  *at = (int32_t)(base + ((size_t)k * nyc + j) * nxc + i);
  return FDTD_OK;
}

hipError_t launch_step3d(Host3D* h, int64_t step, hipStream_t stream) {
  const int32_t* pix = reinterpret_cast<const int32_t*>(h->ws + h->off_pix);
  void* ring = h->ws + h->off_probe;
  if (h->es == 8)
    return launch_step3d_t<double>(h->run, h->nx, h->ny, h->nz, h->np, h->kin_groups, h->nc,
                                   h->f0_groups, h->two_term, step, pix, h->nprobe, ring,
                                   std::max(h->probe_cap, 1), stream);
  return launch_step3d_t<float>(h->run, h->nx, h->ny, h->nz, h->np, h->kin_groups, h->nc,
                                h->f0_groups, h->two_term, step, pix, h->nprobe, ring,
                                std::max(h->probe_cap, 1), stream);
}

int points_3d(const Host3D* h) { return h->np; }

int status_3d(Host3D* h, char* ws, int32_t* v) {
  hipError_t e = hipMemcpy(v, ws + h->off_status, 4, hipMemcpyDeviceToHost);
  return e ? hip_fail(e, "copy 3D status") : FDTD_OK;
}

int field_size_3d(const Host3D* h, int field, size_t* n) {
  switch (field) {
    case FDTD_F_EX: case FDTD_F_JX: *n = h->nE[0]; return FDTD_OK;
    case FDTD_F_EY: case FDTD_F_JY: *n = h->nE[1]; return FDTD_OK;
    case FDTD_F_EZ: case FDTD_F_JZ: *n = h->nE[2]; return FDTD_OK;
    case FDTD_F_HX: *n = h->nH[0]; return FDTD_OK;
    case FDTD_F_HY: *n = h->nH[1]; return FDTD_OK;
    case FDTD_F_HZ: *n = h->nH[2]; return FDTD_OK;
    case FDTD_F_DF: *n = (size_t)(h->np + h->nc) * h->vdim; return FDTD_OK;
    default: return fail(FDTD_EINVAL, "field %d not defined on a 3D grid", field);
  }
}

int write_3d(Host3D* h, char* ws, int field, const double* src) {
  size_t off = 0, cnt = 0;
  double scale = 1.0;
  const size_t es = h->es;
  switch (field) {
    case FDTD_F_EX: off = h->off_E; cnt = h->nE[0]; break;
    case FDTD_F_EY: off = h->off_E + h->nE[0] * es; cnt = h->nE[1]; break;
    case FDTD_F_EZ: off = h->off_E + (h->nE[0] + h->nE[1]) * es; cnt = h->nE[2]; break;
    case FDTD_F_HX: off = h->off_H; cnt = h->nH[0]; scale = kEta0; break;
    case FDTD_F_HY: off = h->off_H + h->nH[0] * es; cnt = h->nH[1]; scale = kEta0; break;
    case FDTD_F_HZ: off = h->off_H + (h->nH[0] + h->nH[1]) * es; cnt = h->nH[2]; scale = kEta0; break;
    default: return fail(FDTD_EINVAL, "field %d cannot be written on a 3D grid", field);
  }
  std::vector<char> buf(std::max<size_t>(cnt, 1) * es);
  for (size_t k = 0; k < cnt; ++k) {
    if (es == 8) reinterpret_cast<double*>(buf.data())[k] = src[k] * scale;
    else reinterpret_cast<float*>(buf.data())[k] = (float)(src[k] * scale);
  }
  hipError_t e = hipMemcpy(ws + off, buf.data(), cnt * es, hipMemcpyHostToDevice);
  if (e) return hip_fail(e, "write 3D field");
  return FDTD_OK;
}

int read_3d(Host3D* h, char* ws, int field, double* dst) {
  size_t off = 0, cnt = 0;
  double scale = 1.0;
  const size_t es = h->es;
  switch (field) {
    case FDTD_F_EX: off = h->off_E; cnt = h->nE[0]; break;
    case FDTD_F_EY: off = h->off_E + h->nE[0] * es; cnt = h->nE[1]; break;
    case FDTD_F_EZ: off = h->off_E + (h->nE[0] + h->nE[1]) * es; cnt = h->nE[2]; break;
    case FDTD_F_HX: off = h->off_H; cnt = h->nH[0]; scale = 1.0 / kEta0; break;
    case FDTD_F_HY: off = h->off_H + h->nH[0] * es; cnt = h->nH[1]; scale = 1.0 / kEta0; break;
    case FDTD_F_HZ: off = h->off_H + (h->nH[0] + h->nH[1]) * es; cnt = h->nH[2]; scale = 1.0 / kEta0; break;
    case FDTD_F_JX: off = h->off_J; cnt = h->nE[0]; scale = kEps0 / h->dt; break;
    case FDTD_F_JY: off = h->off_J + h->nE[0] * es; cnt = h->nE[1]; scale = kEps0 / h->dt; break;
    case FDTD_F_JZ: off = h->off_J + (h->nE[0] + h->nE[1]) * es; cnt = h->nE[2]; scale = kEps0 / h->dt; break;
    case FDTD_F_DF: off = h->off_df; cnt = (size_t)h->np * h->row; break;   // then F0 rows
    default: return fail(FDTD_EINVAL, "field %d not defined on a 3D grid", field);
  }
  std::vector<char> buf(std::max<size_t>(cnt, 1) * es);
  if (cnt) {
    hipError_t e = hipMemcpy(buf.data(), ws + off, cnt * es, hipMemcpyDeviceToHost);
    if (e) return hip_fail(e, "copy 3D field");
  }
  auto val = [&](size_t k) -> double {
    return es == 8 ? reinterpret_cast<double*>(buf.data())[k] : reinterpret_cast<float*>(buf.data())[k];
  };
  if (field == FDTD_F_DF) {
    for (int q = 0; q < h->np; ++q)
      for (int k = 0; k < h->vdim; ++k)
        dst[(size_t)h->doc[q] * h->vdim + k] = val((size_t)q * h->row + k);
    if (h->nc > 0) {
      const size_t n0 = (size_t)h->nc * h->row;
      std::vector<char> b0(n0 * es);
      hipError_t e = hipMemcpy(b0.data(), ws + h->off_f0, n0 * es, hipMemcpyDeviceToHost);
      if (e) return hip_fail(e, "copy 3D F0");
      double* d = dst + (size_t)h->np * h->vdim;
      for (int c = 0; c < h->nc; ++c)
        for (int k = 0; k < h->vdim; ++k) {
          const size_t q = (size_t)c * h->row + k;
          d[(size_t)c * h->vdim + k] =
              es == 8 ? reinterpret_cast<double*>(b0.data())[q] : reinterpret_cast<float*>(b0.data())[q];
        }
    }
  } else {
    for (size_t k = 0; k < cnt; ++k) dst[k] = val(k) * scale;
  }
  return FDTD_OK;
}

void destroy_3d(Host3D* h) { delete h; }

}  // namespace fdtdp
