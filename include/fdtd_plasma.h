/*
 * fdtd_plasma.h -- C ABI of the MI355X (gfx950) kinetic-FDTD plasma library.
 *
 * The library advances Maxwell's curl equations on a Yee grid (arXiv 2211.05647,
 * section 2, eq. (1)-(5); CPML of eq. (4) and the b, a, sigma_max, alpha formulas
 * that follow it), coupled every time step to the two-term kinetic model of the
 * electrons in every plasma cell (section 5.2, eq. for dF1/dt with nu(v) = N s v and
 * J = -e \int v F d^3v, and the Crank-Nicolson style update of f_1x and the Jx sum).
 * The problem is stated the way the paper states it: a grid (cells, cell size,
 * Courant number, absorbing layer), a plasma profile (electron density, collision
 * frequency, temperature, velocity bins), a Gaussian-modulated source (section 5.2
 * table) and a number of time steps.
 *
 * Conventions (all entry points):
 *   - every call returns int: FDTD_OK (0) or a negative fdtd_status; nothing throws
 *     across the ABI.  fdtd_plasma_strerror() names a code; fdtd_plasma_last_error()
 *     gives the thread's last message.
 *   - host pointers are plain host memory; device pointers are HIP device memory.
 *   - input arrays are copied during create; the caller may free them on return.
 *   - if fdtd_device.workspace is non-NULL, the library never allocates device memory:
 *     every device array lives inside that caller-owned buffer, which must stay valid
 *     until fdtd_plasma_destroy.  If it is NULL the library allocates (hipMalloc) and
 *     frees on destroy.
 *   - work is enqueued on fdtd_device.hip_stream (NULL = the null stream); step/run
 *     return once enqueued.  read_* synchronise that stream.
 *   - after k steps, E is at t = k dt while H and J are at t = (k - 1/2) dt.
 *   - a read into a short buffer returns FDTD_ERANGE and writes nothing.
 *   - invalid arguments return FDTD_EINVAL with no side effect; HIP errors return
 *     FDTD_EDEVICE; a non-finite field returns FDTD_ENUMERIC from read_fields.
 *   - handles are not thread-safe; calls on one handle must be serialised.
 */
#ifndef FDTD_PLASMA_H
#define FDTD_PLASMA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdtd_plasma fdtd_plasma;   /* opaque: one run or one batch of runs */

enum fdtd_status {
  FDTD_OK = 0,
  FDTD_EINVAL = -1,   /* bad argument, shape or configuration            */
  FDTD_ENOMEM = -2,   /* workspace too small or allocation failed        */
  FDTD_EDEVICE = -3,  /* HIP runtime error                               */
  FDTD_ERANGE = -4,   /* destination buffer too short / index out of range */
  FDTD_ENUMERIC = -5, /* non-finite value found in the fields            */
  FDTD_ESTATE = -6    /* call not allowed in the handle's current state   */
};

enum fdtd_precision { FDTD_FP64 = 0, FDTD_FP32 = 1 };
enum fdtd_boundary { FDTD_BC_PEC = 0, FDTD_BC_MUR1 = 1, FDTD_BC_CPML = 2 };
enum fdtd_nu_model { FDTD_NU_HARD_SPHERE = 0, FDTD_NU_CONST = 1 };
enum fdtd_closure_kind { FDTD_CLOSURE_KINETIC = 0, FDTD_CLOSURE_MLP = 1 };
enum fdtd_source_kind { FDTD_SRC_NONE = 0, FDTD_SRC_LINE_SOFT = 1, FDTD_SRC_POINT_SOFT = 2 };
enum fdtd_kinetic_model { FDTD_KINETIC_LINEAR = 0, FDTD_KINETIC_FULL = 1,
                          FDTD_KINETIC_TWO_TERM = 2 };
enum fdtd_f0_model { FDTD_F0_MAXWELL = 0, FDTD_F0_DRUYVESTEYN = 1 };

/* Field selectors for read_fields / add_probe.
 * 1D grids (Ez at nodes i = 0..nx, Hy at i + 1/2):
 *   FDTD_F_E  Ez [nx+1] V/m,  FDTD_F_H Hy [nx] A/m,  FDTD_F_J Jz [nx+1] A/m^2,
 *   FDTD_F_DF F1 on the full signed velocity grid, [ncell][nv] (s/m^4), plasma nodes
 *             in increasing order (mirror bins reconstructed from the stored half);
 *             with the full kinetic model, f - ne fhat on that grid.
 * 2D TEz grids (Ex at (i+1/2, j), Ey at (i, j+1/2), Hz at (i+1/2, j+1/2)):
 *   FDTD_F_EX [ny+1][nx], FDTD_F_EY [ny][nx+1], FDTD_F_HZ [ny][nx] (A/m),
 *   FDTD_F_JX [ny+1][nx], FDTD_F_JY [ny][nx+1] (edge currents, A/m^2),
 *   FDTD_F_JCX, FDTD_F_JCY [ny][nx] cell-centre currents (A/m^2, 0 off plasma),
 *   FDTD_F_DF [ncell][nv][nv] (vx index, vy index), the cells that run the kinetic step,
 *             in row-major order (with the learned closure: its fallback cells only).
 * 3D grids (storage [k][j][i], i fastest; H in A/m, J in A/m^2):
 *   FDTD_F_EX [nz+1][ny+1][nx] at (i+1/2, j, k), FDTD_F_EY [nz+1][ny][nx+1] at (i, j+1/2, k),
 *   FDTD_F_EZ [nz][ny+1][nx+1] at (i, j, k+1/2), FDTD_F_HX [nz][ny][nx+1] at (i, j+1/2, k+1/2),
 *   FDTD_F_HY [nz][ny+1][nx] at (i+1/2, j, k+1/2), FDTD_F_HZ [nz+1][ny][nx] at (i+1/2, j+1/2, k),
 *   FDTD_F_JX / JY / JZ shaped like EX / EY / EZ,
 *   FDTD_F_DF [npoint][nv]: F1 on the speed grid (s^3/m^6) of every plasma point, the
 *             Ex points first, then Ey, then Ez, each in storage order; with the TWO_TERM
 *             model followed by [ncell][nv] F0 - ne F0hat of every cell with ne > 0, in
 *             storage order. */
enum fdtd_field {
  FDTD_F_E = 0, FDTD_F_H = 1, FDTD_F_J = 2, FDTD_F_DF = 3,
  FDTD_F_EX = 4, FDTD_F_EY = 5, FDTD_F_HZ = 6, FDTD_F_JX = 7, FDTD_F_JY = 8,
  FDTD_F_JCX = 9, FDTD_F_JCY = 10,
  FDTD_F_EZ = 11, FDTD_F_HX = 12, FDTD_F_HY = 13, FDTD_F_JZ = 14
};

/* Grid (section 2): dims 1 = (Ez, Hy) line, 2 = TEz plane, 3 = Yee cube.  nx, ny, nz in
 * cells (nz read for dims 3 only), dx in metres (dy = dz = dx), courant = c dt / dx
 * (rejected above 1 in 1D, 1/sqrt(2) in 2D, 1/sqrt(3) in 3D).  boundary: 1D takes PEC or
 * MUR1, 2D and 3D take PEC or CPML (3D: the layer on all six faces).  The CPML parameters
 * follow the paper's ranges (thickness 8 cells, order 2-4, sigma factor 0.7-1.5,
 * kappa_max 5-11, alpha_max 0-0.05 S/m). */
typedef struct {
  int32_t dims;
  int32_t nx, ny;
  double dx;
  double courant;
  int32_t precision;
  int32_t boundary;
  int32_t cpml_cells;
  double cpml_order, cpml_sigma_factor, cpml_kappa_max, cpml_alpha_min, cpml_alpha_max;
  int32_t nz;
} fdtd_grid;

/* Plasma profile (section 5.2).  ne / nu_mean: host arrays, 1D: [nx+1] per E node,
 * 2D: [ny][nx] per cell; ne = 0 marks vacuum.  F0 is a Maxwellian at te_ev, F1 starts
 * at zero.  nv bins per velocity axis (a power of two, >= 8), cell-centred on
 * +-vmax_over_vth * v_th.  nu_model HARD_SPHERE: nu(v) = N s |v| scaled so its
 * Maxwellian mean is nu_mean; CONST: nu = nu_mean.  closure: KINETIC, or MLP with the
 * network blob `mlp` (fdtd_mlp_blob) and the kinetic step as fallback.
 * kinetic: LINEAR is the model of section 5.2 (F0 frozen, F1 driven by E dF0/dv).
 * FULL (1D single runs and batches) evolves the whole f of each plasma node under
 * df/dt - (e/m) E df/dv = C(f) (the kinetic equation of section 5.1 without the
 * streaming and magnetic terms): its even part is the l = 0 equation's F0, which heats,
 * its odd part F1.  The velocity derivative is in conservative flux form with zero flux
 * through +-vmax (electron number is kept exactly) and is explicit: each step needs
 * |(e/m) E dt / dv| <= 1, and a step that breaks it sets the run status (see
 * fdtd_plasma_run_status).  Temporally blocked as the LINEAR model is
 * (fdtd_plasma_set_time_block).
 * TWO_TERM (1D single runs and batches, 3D grids): the paper's own representation, section 5.1's
 * expansion F = F0 + (v/|v|).F1 with its l = 0 and l = 1 equations on a speed grid of nv
 * speeds (2..256; the paper uses 31) v_k = (k + 1/2) vmax / nv, F0 (f0_model) evolving
 * under the l = 0 equation without streaming (elastic collisions only: their l = 0 term,
 * of order the electron-to-neutral mass ratio, is dropped), F1 = the z component driven
 * by dF0/dv of the current F0, J = -e (4 pi / 3) gam sum w_k F1_k with w_k the mean of
 * v^3 over the bin's flux-carrying faces, which makes the field energy J removes exactly
 * the electrons' kinetic energy gain.  FDTD_F_DF then gives [ncell][2 nv]: F1, then
 * F0 - ne F0hat.  The exchange between F0 and F1 is explicit: a step with
 * (e/m) |E| dt / (vmax / nv) > 1 sets the run status.  Temporally blocked as the LINEAR
 * model is (fdtd_plasma_set_time_block) for 17..64 speeds.
 * 3D grids (the paper's production model, section 5.3): ne / nu_mean are per cell
 * [nz][ny][nx]; F1 is a vector on a speed grid of nv speeds (1..64; the paper uses 31)
 * v_k = (k + 1/2) vmax / nv, one component at every E point whose edge touches plasma (the
 * point takes the mean ne and nu_mean of the four cells around its edge), updated as
 * in 2D with J = -e (4 pi / 3) (vmax / nv) sum v^3 F1.  f0_model (3D and the 1D TWO_TERM model): MAXWELL, or
 * DRUYVESTEYN, exp(-(v / vD)^4) with the Maxwellian's mean energy (3/2) e te_ev; either
 * normalised by 4 pi (vmax / nv) sum v^2 F0 = 1.  3D runs take the kinetic closure and
 * the LINEAR or the TWO_TERM model.  3D TWO_TERM (nv >= 2): F0 lives in every cell with
 * ne > 0 and F1 only at the E points whose four cells all have ne > 0; an edge's F1
 * drive takes the mean F0 of its four cells, and each cell's l = 0 update takes a
 * quarter of E.F1 from each of its plasma edges (E time-centred), so the field energy
 * J removes is exactly the heat the cells gain; the explicit-exchange limit and the
 * run status are as in 1D.  Four launches per step instead of three.  3D TWO_TERM
 * plasma (ne > 0) must stay out of the x and y absorbing layers (the outer cpml_cells
 * cells of x and y): with plasma inside them this point set carries a mode that grows
 * by tens per thousand steps until the fields overflow, so fdtd_plasma_create refuses
 * such a profile with FDTD_EINVAL. */
typedef struct {
  const double *ne;
  const double *nu_mean;
  double te_ev;
  int32_t nv;
  double vmax_over_vth;
  int32_t nu_model;
  int32_t closure;
  const void *mlp;
  int32_t kinetic;
  int32_t f0_model;
} fdtd_profile;

/* Soft source (section 5.2 table): adds amplitude * sin(2 pi f (t - t0))
 * exp(-((t - t0)/tau)^2) to E at t^{n+1} after each E update.  1D: node i (POINT).
 * 2D: LINE adds to every Ey(i, j + 1/2) of column i; POINT adds to Ey(i, j + 1/2).
 * 3D: LINE adds to every updated Ex(i + 1/2, j, k) of the plane k (a sheet: a plane wave
 * along z), POINT to Ex(i + 1/2, j, k); 0 < k < nz. */
typedef struct {
  int32_t kind;
  int32_t i, j;
  double amplitude, f_hz, tau_s, t0_s;
  int32_t k;
} fdtd_source;

/* Device binding.  hip_stream: a hipStream_t (NULL = null stream).  workspace: device
 * memory of workspace_bytes (see fdtd_plasma_workspace_size) or NULL.  max_probes /
 * probe_capacity reserve room for time-series probes (steps kept per probe). */
typedef struct {
  int32_t device;
  void *hip_stream;
  void *workspace;
  size_t workspace_bytes;
  int32_t max_probes;
  int32_t probe_capacity;
} fdtd_device;

/* Bytes of device workspace a single run needs.  EINVAL on a bad configuration. */
int fdtd_plasma_workspace_size(const fdtd_grid *grid, const fdtd_profile *profile,
                               const fdtd_device *dev, size_t *bytes);

/* Validate, build the FP64 tables on the host (velocity grid, F0 and dF0/dv, collision
 * frequencies, CPML profiles), round them once to the storage precision, copy them and
 * the zero initial state to the device.  *out receives the handle. */
int fdtd_plasma_create(const fdtd_grid *grid, const fdtd_profile *profile,
                       const fdtd_source *source, const fdtd_device *dev, fdtd_plasma **out);

/* Batch of nruns independent 1D FP32 runs of uneven size (arrays of nruns structs), all of
 * one kinetic model (EINVAL otherwise), advanced together; a two-term run that stops takes
 * its last deferred l = 0 update with it, so its state is complete from then on.  steps[r] is the step count of run r: fdtd_plasma_run advances
 * every run to min(its own count, the batch step).  ntap (0..8) training-pair taps per
 * run record (E^n, J^{n+1/2}) at the plasma nodes tap_nodes[r * ntap + k] after every
 * step of that run (NULL when ntap = 0).  Default launch form (batch mode 1): the runs
 * with at least K steps left advance K steps per launch (temporal blocking, K from
 * fdtd_plasma_set_time_block, default 9), one launch per Nv group; runs that end inside
 * such a pass, and the batch's tail once fewer blocked work-groups than compute units
 * remain, take one step per launch over the tiles of the runs still active.  See
 * fdtd_plasma_set_batch_mode for the persistent form.  Workspace size via
 * fdtd_plasma_workspace_size_batch. */
int fdtd_plasma_workspace_size_batch(int32_t nruns, const fdtd_grid *grids,
                                     const fdtd_profile *profiles, const int64_t *steps,
                                     int32_t ntap, const fdtd_device *dev, size_t *bytes);
int fdtd_plasma_create_batch(int32_t nruns, const fdtd_grid *grids,
                             const fdtd_profile *profiles, const fdtd_source *sources,
                             const int64_t *steps, int32_t ntap, const int32_t *tap_nodes,
                             const fdtd_device *dev, fdtd_plasma **out);

/* Batch launch form: mode 1 (default) = K-step blocked launches with one-step launches
 * for the remainders, as described at fdtd_plasma_create_batch; mode 0 = one persistent
 * launch per fdtd_plasma_run: `groups` work-groups (0 = as many as fit on the device) take
 * (tile, K-step block) items of every run in order from a work counter, a block of a tile
 * starting once the tile and its two neighbours have finished the block before; each
 * run's last steps go as one odd block or two.  Mode 0 needs what the blocked path needs
 * (K >= 3, runs of supported Nv) and LINEAR runs; a FULL or TWO_TERM batch takes mode 1's
 * launches, and a batch the blocked path cannot take steps one step per launch.  Both
 * modes give bitwise identical results.  Only before the first step. */
int fdtd_plasma_set_batch_mode(fdtd_plasma *h, int32_t mode, int32_t groups);

/* Copy the taps of run `run`: [ntap][steps taken by that run][2] doubles, (E in V/m,
 * J in A/m^2), oldest first.  FDTD_ERANGE if dst_len is short. */
int fdtd_plasma_read_taps(fdtd_plasma *h, int32_t run, double *dst, size_t dst_len,
                          size_t *n_out);

/* Per-run status after the last run: 0, or FDTD_ENUMERIC if that run produced a
 * non-finite E value (1D; other runs of the batch are unaffected) or, with the FULL or
 * TWO_TERM model (1D and 3D), broke the explicit velocity-exchange limit, or FDTD_ESTATE if
 * a persistent batch launch (batch mode 0) gave up waiting for a neighbouring tile (the
 * batch's results are then void; it does not happen in a correct launch).  2D handles
 * report 0.  Later steps do not clear the flag. */
int fdtd_plasma_run_status(fdtd_plasma *h, int32_t run, int32_t *status);

/* One leap-frog step (H, F1 and J, E, boundary, source), enqueued. */
int fdtd_plasma_step(fdtd_plasma *h);
/* nsteps leap-frog steps, enqueued on the handle's stream. */
int fdtd_plasma_run(fdtd_plasma *h, int64_t nsteps);
/* Steps taken so far (batch: the batch step counter). */
int fdtd_plasma_steps(const fdtd_plasma *h, int64_t *steps);

/* Number of doubles read_fields writes for (run, field). */
int fdtd_plasma_field_size(const fdtd_plasma *h, int32_t run, int32_t field, size_t *n);
/* Synchronise, copy one field of run `run` (0 for a single run) to host as doubles in
 * SI units, layout as documented at enum fdtd_field.  *step_out (optional) receives the
 * step count of that run.  FDTD_ENUMERIC if the copied field holds a NaN or Inf. */
int fdtd_plasma_read_fields(fdtd_plasma *h, int32_t run, int32_t field, double *dst,
                            size_t dst_len, int64_t *step_out);

/* Overwrite a field of the current state with host values in SI units (E in V/m, H in
 * A/m), in the read_fields layout: initial conditions such as the section 4 validation's
 * travelling Gaussian pulse, or a cavity mode.  Writable: 1D FDTD_F_E and FDTD_F_H
 * (E^n and H^{n-1/2} of run `run`), 2D FDTD_F_EX, _EY, _HZ, 3D FDTD_F_EX, _EY, _EZ,
 * _HX, _HY, _HZ.  Values are rounded to the storage precision.  src_len must equal the
 * field's size (FDTD_ERANGE otherwise); a non-finite value or another field gives
 * FDTD_EINVAL and writes nothing.  Synchronises the handle's stream.  The learned
 * closure's field history (2D) and the absorbing-layer memories are not rewritten. */
int fdtd_plasma_write_fields(fdtd_plasma *h, int32_t run, int32_t field, const double *src,
                             size_t src_len);

/* Record `field` at grid index (i, j) after every step (1D: j ignored).  Only before
 * the first step; at most fdtd_device.max_probes.  *id receives the probe id.  3D handles
 * take fdtd_plasma_add_probe3d instead (FDTD_EINVAL here). */
int fdtd_plasma_add_probe(fdtd_plasma *h, int32_t run, int32_t field, int32_t i, int32_t j,
                          int32_t *id);
/* 3D handles: record E component `field` (FDTD_F_EX, _EY or _EZ) at its storage index
 * (i, j, k) (the component's own shape, see enum fdtd_field) after every step, the ports of
 * the paper's reflection and transmission measurement (section 5.3 results).  Rules as
 * for fdtd_plasma_add_probe; FDTD_ERANGE for an index outside the component's array,
 * FDTD_EINVAL for another field or a 1D / 2D handle.  Read with fdtd_plasma_read_probe. */
int fdtd_plasma_add_probe3d(fdtd_plasma *h, int32_t field, int32_t i, int32_t j, int32_t k,
                            int32_t *id);
/* Copy the last min(steps, probe_capacity) samples of probe `id` (oldest first). */
int fdtd_plasma_read_probe(fdtd_plasma *h, int32_t id, double *dst, size_t dst_len,
                           size_t *n_out);

/* Whole evolving state (fields, F1, CPML memory, step counter, probe rings) as an
 * opaque host blob; load requires a handle created with the same configuration and
 * resumes bitwise-identically. */
int fdtd_plasma_state_size(const fdtd_plasma *h, size_t *bytes);
int fdtd_plasma_save_state(fdtd_plasma *h, void *dst, size_t len);
int fdtd_plasma_load_state(fdtd_plasma *h, const void *src, size_t len);

/* Launch shape (autotuner hook): nodes (1D) or cells (2D) per tile, and plasma cells
 * per work-group for the kinetic kernels; 0 keeps the current value.  Only before the
 * first step. */
int fdtd_plasma_set_tiling(fdtd_plasma *h, int32_t tile, int32_t cells_per_group);

/* Temporal blocking of a single 1D run in FP32 storage with the LINEAR or FULL model and Nv
 * in {64, 128, 256, 512}, or the TWO_TERM model with 17..64 speeds (rows padded to 32 or 64):
 * fdtd_plasma_run advances `steps` time steps per kernel launch (each work-group
 * recomputes a halo of `steps` nodes per side, so F1 -- and F0 -- cross HBM once per
 * `steps` steps) and the remainder one step per launch.  steps = 1 turns it off; 3, 5, 7
 * and 9 are accepted.  Results are bitwise those of one-step launches (the kinetic step is
 * local in space, see section 5.2).  The library's default is 9 (the fastest measured on
 * MI355X for the 65,536-node line at Nv = 512 and for a 256-run batch); a caller with a
 * tuning table sets its own.  Batches use K for both launch forms (the persistent one
 * takes K-step blocks too).  Other runs (FP64, 2D, 3D, other speed counts, lines too short
 * to cut into blocks) step one step per launch; the call then only records the value.
 * May be called between runs.  fdtd_plasma_time_block reports the steps per launch in
 * effect (1 when the run is not blocked) and, if rows_per_launch is not NULL, the number of
 * F1 rows one blocked launch reads (owned rows plus the halo rows it recomputes; 0 when
 * not blocked). */
int fdtd_plasma_set_time_block(fdtd_plasma *h, int32_t steps);
int fdtd_plasma_time_block(const fdtd_plasma *h, int32_t *steps, int64_t *rows_per_launch);

/* Average device time per step of the last fdtd_plasma_run, measured with HIP events
 * on the handle's stream (synchronises). */
int fdtd_plasma_last_run_ms(fdtd_plasma *h, double *ms_per_step);

void fdtd_plasma_destroy(fdtd_plasma *h);
const char *fdtd_plasma_strerror(int code);
const char *fdtd_plasma_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FDTD_PLASMA_H */
