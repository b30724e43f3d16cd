/*
 * oracle.c -- plain FP64 CPU oracle of the coupled Yee-FDTD / two-term kinetic
 * plasma model of Dodge, Shafiee & Shokri (arXiv 2211.05647).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant with the
 * HIP library: it builds its own velocity tables, collision frequencies, CPML
 * profiles and source samples from the paper's definitions, in double
 * precision, on the FULL signed velocity grid (the GPU path stores only half
 * of it).  It is deliberately unblocked and unfused: every step is written in
 * the order the method states it, so that it can be checked against the paper
 * by eye.  OpenMP only splits independent loop iterations.
 *
 * Readings of the paper taken here (the paper is silent or garbled):
 *   - Ampere's law subtracts J (Maxwell's equations, eq. (1), second line);
 *     the printed C_J coefficient has no sign, we use -dt/eps0 * J.
 *   - electrons carry charge -e with e > 0; the F1 equation of the numerical
 *     model (section 5.2) is used as printed: dF1/dt - (e/m) E dF0/dv = -nu F1.
 *   - order inside one step: H -> F1 (driven by E^n) -> J -> E -> boundary ->
 *     soft source (the flowchart figure is missing; the F1 update's factor 2*E
 *     puts F1 and J on half-integer time levels, which the E update needs).
 *   - F0 is a Maxwellian at T_e (the workloads fix it), normalised on the
 *     discrete grid; dF0/dv is the analytic derivative -v F0 / v_th^2.
 *   - v_th = sqrt(e T_e / m_e); bins are cell-centred and symmetric,
 *     v_j = (j - (Nv-1)/2) dv, dv = 2 vmax / Nv, with no v = 0 bin.
 *   - the 1V (2V) Cartesian analogue of the current moment of section 5.2 is
 *     J = -e dv sum_j v_j f_j  (J = -e dv^2 sum_ab v_ab f_ab).
 *   - collision frequency nu(v) = N s v with the constant N s fixed so that
 *     the Maxwellian mean of nu equals the prescribed mean frequency
 *     ("hard sphere"), or nu = const (the test mode).
 *   - CPML (section 2, eq. (4) and the b, a, sigma_max, alpha formulas):
 *     psi at the new level is b * psi(old) + a * (field difference); kappa is
 *     graded like sigma with the same power; E-side profiles are sampled at
 *     integer depth, H-side at half-cell depth; the outer wall is PEC.
 *   - 2D TEz: F1 lives at plasma cell centres; E is averaged from the two
 *     bounding edges to the centre and J is averaged back to each edge with
 *     the transposed weights, so field-to-plasma work is exchanged exactly.
 *   - 3D (the paper's production model): F1 is a vector on a speed grid
 *     v_k = (k + 1/2) gam, one component at each E component's point, with
 *     J = -e (4 pi / 3) gam sum v^3 F1 as section 5.3 prints it; F0 Maxwellian
 *     or Druyvesteyn (the paper names the latter without its formula: taken as
 *     exp(-(v/vD)^4) with the Maxwellian's mean energy (3/2) e T_e), normalised
 *     by 4 pi gam sum v^2 F0 = 1; an E point's density and mean collision
 *     frequency are the means over the four cells around its edge; tangential
 *     E on the outer faces stays zero behind the CPML.
 *   - full-distribution model (model = 1, 1V): instead of freezing F0 and
 *     evolving F1 alone, the whole f of each plasma node evolves under
 *     df/dt - (e/m) E df/dv = C(f) (the kinetic equation of section 5.1 with
 *     the streaming and magnetic terms dropped as in section 5.2); in 1V its
 *     even part plays F0 (the l = 0 equation: it heats) and its odd part F1.
 *     Stored: delta = f - n F0hat (zero at start), on the full signed grid.
 *     Velocity derivative in conservative flux form, zero flux through
 *     +-vmax (the electron number is conserved exactly), the odd part first
 *     (central flux with a Lax-Wendroff correction, the collision term with
 *     the linear model's Crank-Nicolson factor), then the even part from the
 *     time-centred odd part; the drive is taken at E^n.  For small fields the
 *     odd part obeys the linear model's update with dF0/dv replaced by a
 *     central difference.
 *   - two-term model on the speed grid (1D line and 3D cube): F0 - n F0hat
 *     evolves under the l = 0 equation in flux form over the speed faces,
 *     the flux through a face the face's v^2 times the mean of the two F1
 *     values beside it times the time-centred E, none through v = 0 or vmax;
 *     the F1 drive adds the central difference of F0 - n F0hat (reflected
 *     evenly below v_0, zero above vmax); the l = 0 collision term (energy
 *     loss to the gas) is left out.  In 3D an edge sees the mean F0 of its
 *     four cells and each cell takes a quarter of every one of its plasma
 *     edges' E.F1; plasma points are the edges with all four cells plasma.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* CODATA 2018 */
static const double K_C0 = 299792458.0;
static const double K_EPS0 = 8.8541878128e-12;
static const double K_QE = 1.602176634e-19;
static const double K_ME = 9.1093837015e-31;
static const double K_PI = 3.14159265358979323846;

static double k_mu0(void) { return 1.0 / (K_EPS0 * K_C0 * K_C0); }

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads the following parallel loops use (n >= 1): lets a caller time the oracle on
 * one core as well as on all of them */
int oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#endif
    (void)n;
    return oracle_threads();
}

int oracle_constants(double *out4)
{
    out4[0] = K_C0; out4[1] = K_EPS0; out4[2] = K_QE; out4[3] = K_ME;
    return 0;
}

/* ---------------------------------------------------------------------------
 * Velocity grid and the frozen isotropic part F0 (section 5.2: F0 is held
 * fixed, F1 starts at zero).  Maxwellian at T_e, discretely normalised so that
 * sum_j fhat_j dv = 1; ghat_j = dfhat/dv = -v_j fhat_j / v_th^2.
 * ------------------------------------------------------------------------- */
int oracle_vgrid(int nv, double vmax_over_vth, double te_ev,
                 double *v, double *fhat, double *ghat,
                 double *dv_out, double *vth_out)
{
    if (nv < 2 || (nv % 2) != 0 || te_ev <= 0.0 || vmax_over_vth <= 0.0)
        return -1;
    double vth = sqrt(K_QE * te_ev / K_ME);
    double dv = 2.0 * vmax_over_vth * vth / (double)nv;
    double norm = 0.0;
    for (int j = 0; j < nv; ++j) {
        v[j] = ((double)j - 0.5 * (double)(nv - 1)) * dv;
        fhat[j] = exp(-v[j] * v[j] / (2.0 * vth * vth));
        norm += fhat[j] * dv;
    }
    for (int j = 0; j < nv; ++j) {
        fhat[j] = fhat[j] / norm;
        ghat[j] = -v[j] * fhat[j] / (vth * vth);
    }
    *dv_out = dv;
    *vth_out = vth;
    return 0;
}

/* Collision-frequency shape s_j with nu_j = nubar * s_j (section 5.2,
 * nu(v) = N s v).  model 0: hard sphere, s_j = |v_j| / <|v|>; model 1: const.
 * dims = 1 uses |v_j|; dims = 2 uses |(vx_a, vy_b)| over the nv*nv grid. */
int oracle_nu_shape(int dims, int nv, const double *v, const double *fhat,
                    double dv, int model, double *s)
{
    if (dims == 1) {
        double mean = 0.0;
        for (int j = 0; j < nv; ++j) mean += fabs(v[j]) * fhat[j] * dv;
        for (int j = 0; j < nv; ++j) s[j] = (model == 0) ? fabs(v[j]) / mean : 1.0;
        return 0;
    }
    if (dims == 2) {
        double mean = 0.0;
        for (int a = 0; a < nv; ++a)
            for (int b = 0; b < nv; ++b)
                mean += sqrt(v[a] * v[a] + v[b] * v[b]) * fhat[a] * fhat[b] * dv * dv;
        for (int a = 0; a < nv; ++a)
            for (int b = 0; b < nv; ++b)
                s[a * nv + b] = (model == 0)
                    ? sqrt(v[a] * v[a] + v[b] * v[b]) / mean : 1.0;
        return 0;
    }
    return -1;
}

/* Elastic collision operator acting on an arbitrary distribution sampled on
 * the signed 1V grid, in mirror form: C(f)_j = -(nu_j / 2) (f_j - f_{mirror j}).
 * Elastic scattering only randomises direction (section 5.1: only elastic
 * collisions), so the isotropic part is untouched and, for the odd part, this
 * reduces to -nu_j f_j, the right-hand side of the F1 equation. */
int oracle_collision1v(int nv, const double *nu, const double *f, double *out)
{
    for (int j = 0; j < nv; ++j)
        out[j] = -0.5 * nu[j] * (f[j] - f[nv - 1 - j]);
    return 0;
}

/* Gaussian-modulated sine (section 5.2 table): A sin(2 pi f (t - t0)) exp(-((t - t0)/tau)^2). */
static double source_wave(double t, double amp, double f, double tau, double t0)
{
    double x = (t - t0) / tau;
    return amp * sin(2.0 * K_PI * f * (t - t0)) * exp(-x * x);
}

/* ---------------------------------------------------------------------------
 * 1D: Ez at integer nodes i = 0..nx, Hy at i + 1/2 (i = 0..nx-1), SI units.
 * bc: 0 = PEC ends, 1 = first-order Mur ends.
 * ne, nubar: [nx+1] electron density (m^-3, 0 = vacuum) and mean collision
 *   frequency (1/s) per E node.  Plasma nodes are those with ne > 0, in
 *   increasing order; df holds their F1 rows, df[c * nv + j].
 * State (in/out): E[nx+1], H[nx], J[nx+1] (J^{n-1/2}), df.
 * Probes: E at probe nodes after every step, probe_E[s * nprobe + p].
 * Snapshots: E after every snap_every-th step, snap_E[k * (nx+1) + i].
 * Returns 0, or -1 on bad arguments.
 * ------------------------------------------------------------------------- */
/* ---------------------------------------------------------------------------
 * One step of the full-distribution model for one plasma node: delta (nv
 * values, f = nf0 + delta) from level n-1/2 to n+1/2 with the acceleration
 * a = -(e/m) E^n, c = a dt / dv; nf0 = n * fhat, nu_j = nubar * sh_j.
 * f splits into its even part fe = nf0 + e and odd part o (o_j = -o_{nv-1-j}).
 * Both parts are advanced in conservative flux form with zero flux through
 * the outer faces of the grid (work: nv + 1 faces in gbuf, nv values in obuf):
 *   odd:  p_{j+1/2} = (c/2)(fe_j + fe_{j+1}) - (c^2/2)(o_{j+1} - o_j),
 *         o'_j = ((2 - dt nu_j) o_j - 2 (p_{j+1/2} - p_{j-1/2})) / (2 + dt nu_j)
 *         (the linear model's Crank-Nicolson collision step with its drive;
 *         the c^2 term is the Lax-Wendroff correction of the advection);
 *   even: q_{j+1/2} = (c/4)(o_j + o'_j + o_{j+1} + o'_{j+1}),
 *         e'_j = e_j - (q_{j+1/2} - q_{j-1/2})
 *         (the odd part time-centred, so that the energy it hands to the even
 *         part is second order in dt also with collisions).
 * ------------------------------------------------------------------------- */
static void full_cell_step(int nv, const double *nf0, const double *sh, double nubar,
                           double dt, double c, double *delta, double *gbuf, double *obuf)
{
    gbuf[0] = 0.0;
    gbuf[nv] = 0.0;
    /* odd part: p on the inner faces */
    for (int j = 0; j + 1 < nv; ++j) {
        int m = nv - 1 - j, mr = nv - 2 - j;           /* mirrors of j and j + 1 */
        double fel = nf0[j] + 0.5 * (delta[j] + delta[m]);
        double fer = nf0[j + 1] + 0.5 * (delta[j + 1] + delta[mr]);
        double ol = 0.5 * (delta[j] - delta[m]), orr = 0.5 * (delta[j + 1] - delta[mr]);
        gbuf[j + 1] = 0.5 * c * (fel + fer) - 0.5 * c * c * (orr - ol);
    }
    for (int j = 0; j < nv; ++j) {
        int m = nv - 1 - j;
        double o = 0.5 * (delta[j] - delta[m]);
        double x = dt * nubar * sh[j];
        obuf[j] = ((2.0 - x) * o - 2.0 * (gbuf[j + 1] - gbuf[j])) / (2.0 + x);
    }
    /* even part: q on the inner faces from the time-centred odd part */
    for (int j = 0; j + 1 < nv; ++j) {
        int m = nv - 1 - j, mr = nv - 2 - j;
        double ol = 0.5 * (delta[j] - delta[m]), orr = 0.5 * (delta[j + 1] - delta[mr]);
        gbuf[j + 1] = 0.25 * c * (ol + obuf[j] + orr + obuf[j + 1]);
    }
    double en[nv];
    for (int j = 0; j < nv; ++j) {
        int m = nv - 1 - j;
        en[j] = 0.5 * (delta[j] + delta[m]) - (gbuf[j + 1] - gbuf[j]);
    }
    for (int j = 0; j < nv; ++j) delta[j] = en[j] + obuf[j];
}

/* Isolated node of the full-distribution model driven by E[n] = E^n: delta
 * (nv values, in/out, f = n fhat + delta) and J[n] = J^{n+1/2} (A/m^2).
 * Returns -1 on bad arguments, -2 if |a dt/dv| > 1 at some step. */
int oracle_full1v(int nv, double vmax_over_vth, double te_ev, int nu_model,
                  double ne, double nubar, double dt, long long nsteps,
                  const double *E, double *delta, double *J)
{
    if (nv < 2 || (nv & 1)) return -1;
    double *v = malloc(sizeof(double) * nv), *fh = malloc(sizeof(double) * nv);
    double *gh = malloc(sizeof(double) * nv), *sh = malloc(sizeof(double) * nv);
    double *nf0 = malloc(sizeof(double) * nv), *g = malloc(sizeof(double) * (nv + 1));
    double *ob = malloc(sizeof(double) * nv);
    double dv, vth;
    int rc = 0;
    if (oracle_vgrid(nv, vmax_over_vth, te_ev, v, fh, gh, &dv, &vth) != 0) {
        rc = -1;
    } else {
        oracle_nu_shape(1, nv, v, fh, dv, nu_model, sh);
        for (int j = 0; j < nv; ++j) nf0[j] = ne * fh[j];
        for (long long n = 0; n < nsteps && rc == 0; ++n) {
            double c = -(K_QE / K_ME) * E[n] * dt / dv;
            if (fabs(c) > 1.0) { rc = -2; break; }
            full_cell_step(nv, nf0, sh, nubar, dt, c, delta, g, ob);
            double acc = 0.0;
            for (int j = 0; j < nv; ++j) acc += v[j] * delta[j];
            J[n] = -K_QE * dv * acc;
        }
    }
    free(v); free(fh); free(gh); free(sh); free(nf0); free(g); free(ob);
    return rc;
}

int oracle_run1d(int nx, double dx, double courant, int bc,
                 int nv, double vmax_over_vth, double te_ev, int nu_model,
                 const double *ne, const double *nubar,
                 int src_node, double src_amp, double src_f, double src_tau, double src_t0,
                 long long step0, long long nsteps,
                 double *E, double *H, double *J, double *df,
                 int nprobe, const int *probe_node, double *probe_E,
                 int snap_every, double *snap_E, int model)
{
    if (nx < 2 || nv < 2 || dx <= 0.0 || courant <= 0.0 || courant > 1.0) return -1;
    if (model != 0 && model != 1) return -1;
    if (ne[0] > 0.0 || ne[nx] > 0.0) return -1;
    double dt = courant * dx / K_C0;

    double *v = malloc(sizeof(double) * nv), *fh = malloc(sizeof(double) * nv);
    double *gh = malloc(sizeof(double) * nv), *sh = malloc(sizeof(double) * nv);
    double dv, vth;
    if (oracle_vgrid(nv, vmax_over_vth, te_ev, v, fh, gh, &dv, &vth) != 0) {
        free(v); free(fh); free(gh); free(sh); return -1;
    }
    oracle_nu_shape(1, nv, v, fh, dv, nu_model, sh);

    int ncell = 0;
    for (int i = 0; i <= nx; ++i) if (ne[i] > 0.0) ++ncell;
    int *cell_node = malloc(sizeof(int) * (ncell > 0 ? ncell : 1));
    for (int i = 0, c = 0; i <= nx; ++i) if (ne[i] > 0.0) cell_node[c++] = i;

    const double ch = dt / (k_mu0() * dx);   /* C_H^E-like coefficient of the H update   */
    const double ce = dt / (K_EPS0 * dx);    /* C_H^E of the E update (sigma = 0)         */
    const double cj = dt / K_EPS0;           /* C_J^E (subtracted, see header)            */
    const double q = (K_C0 * dt - dx) / (K_C0 * dt + dx);   /* Mur-1 coefficient          */

    for (long long s = 0; s < nsteps; ++s) {
        long long n = step0 + s;
        /* 1. Faraday: H^{n+1/2} = H^{n-1/2} + dt/(mu0 dx) (E_{i+1} - E_i) */
        for (int i = 0; i < nx; ++i) H[i] += ch * (E[i + 1] - E[i]);

        /* 2-3. F1 update driven by E^n (section 5.2 update of f_1x), or the
         *      full-distribution step, then the current moment
         *      J^{n+1/2} = -e dv sum_j v_j F1_j (F1: the odd part of delta). */
        int bad = 0;
        #pragma omp parallel for schedule(static) reduction(|:bad)
        for (int c = 0; c < ncell; ++c) {
            int i = cell_node[c];
            double *f = df + (size_t)c * nv;
            double acc = 0.0;
            if (model == 0) {
                for (int j = 0; j < nv; ++j) {
                    double nu = nubar[i] * sh[j];
                    f[j] = ((2.0 - dt * nu) * f[j]
                            + 2.0 * dt * (K_QE / K_ME) * ne[i] * gh[j] * E[i]) / (2.0 + dt * nu);
                }
            } else {
                double nf0[nv], g[nv + 1], ob[nv];
                for (int j = 0; j < nv; ++j) nf0[j] = ne[i] * fh[j];
                double cfl = -(K_QE / K_ME) * E[i] * dt / dv;
                if (fabs(cfl) > 1.0) bad = 1;
                full_cell_step(nv, nf0, sh, nubar[i], dt, cfl, f, g, ob);
            }
            for (int j = 0; j < nv; ++j) acc += v[j] * f[j];
            J[i] = -K_QE * dv * acc;
        }
        if (bad) { free(v); free(fh); free(gh); free(sh); free(cell_node); return -2; }

        /* 4. Ampere: E^{n+1} = E^n + dt/(eps0 dx)(H_{i+1/2} - H_{i-1/2}) - dt/eps0 J^{n+1/2} */
        double e0 = E[0], e1 = E[1], en1 = E[nx - 1], en = E[nx];
        for (int i = 1; i < nx; ++i) E[i] += ce * (H[i] - H[i - 1]) - cj * J[i];

        /* 5. boundaries */
        if (bc == 1) {
            E[0] = e1 + q * (E[1] - e0);
            E[nx] = en1 + q * (E[nx - 1] - en);
        } else {
            E[0] = 0.0; E[nx] = 0.0;
        }

        /* 6. soft source at t^{n+1} */
        if (src_amp != 0.0 && src_node > 0 && src_node < nx)
            E[src_node] += source_wave((double)(n + 1) * dt, src_amp, src_f, src_tau, src_t0);

        for (int p = 0; p < nprobe; ++p) probe_E[s * nprobe + p] = E[probe_node[p]];
        if (snap_every > 0 && ((s + 1) % snap_every) == 0)
            memcpy(snap_E + ((s + 1) / snap_every - 1) * (size_t)(nx + 1), E, sizeof(double) * (nx + 1));
    }
    free(v); free(fh); free(gh); free(sh); free(cell_node);
    return 0;
}

/* ---------------------------------------------------------------------------
 * CPML profile along one axis (section 2, eq. (4) and the following formulas).
 * For each sample point the depth rho into the layer is given; returns b, the
 * coefficient a_raw = a / delta_cell multiplying the raw field difference, and
 * kappa.  Points outside the layer (rho <= 0) get b = 0, a_raw = 0, kappa = 1.
 * ------------------------------------------------------------------------- */
static void cpml_coeff(double rho, double thick, double dx, double dt,
                       double order, double sigma_factor, double kappa_max,
                       double alpha_min, double alpha_max,
                       double *b, double *a_raw, double *kappa)
{
    if (rho <= 0.0) { *b = 0.0; *a_raw = 0.0; *kappa = 1.0; return; }
    double sigma_max = sigma_factor * (order + 1.0) / (150.0 * K_PI * dx);
    double r = rho / thick;
    double sig = sigma_max * pow(r, order);
    double kap = 1.0 + (kappa_max - 1.0) * pow(r, order);
    double alp = alpha_min + (alpha_max - alpha_min) * (1.0 - r);
    double bb = exp(-(sig / kap + alp) * dt / K_EPS0);
    double aa = sig * (bb - 1.0) / (sig * kap + alp * kap * kap);
    *b = bb; *a_raw = aa / dx; *kappa = kap;
}

/* Profiles along an axis with n cells and an ncpml-cell layer at both ends.
 * e-side samples at integer positions 0..n (n+1 values), h-side at i + 1/2
 * (n values). */
int oracle_cpml_profile(int n, int ncpml, double dx, double dt, double order,
                        double sigma_factor, double kappa_max, double alpha_min,
                        double alpha_max,
                        double *be, double *ae, double *ke,
                        double *bh, double *ah, double *kh)
{
    double thick = ncpml * dx;
    for (int i = 0; i <= n; ++i) {
        double rho = 0.0;
        if (i < ncpml) rho = (ncpml - i) * dx;
        if (i > n - ncpml) rho = (i - (n - ncpml)) * dx;
        if (ncpml == 0) rho = 0.0;
        cpml_coeff(rho, thick, dx, dt, order, sigma_factor, kappa_max, alpha_min,
                   alpha_max, &be[i], &ae[i], &ke[i]);
    }
    for (int i = 0; i < n; ++i) {
        double x = i + 0.5, rho = 0.0;
        if (x < ncpml) rho = (ncpml - x) * dx;
        if (x > n - ncpml) rho = (x - (n - ncpml)) * dx;
        if (ncpml == 0) rho = 0.0;
        cpml_coeff(rho, thick, dx, dt, order, sigma_factor, kappa_max, alpha_min,
                   alpha_max, &bh[i], &ah[i], &kh[i]);
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Learned closure of a cell's current (used by oracle_run2d for closure cells):
 * J^{n+1/2} = alpha J^{n-1/2} + beta (E^n + s y), y = MLP([E^n..E^{n-15}]/s, q1, q2),
 * s = max |E window| (floor 1e-30); network 18 -> 128 -> 128 -> 1 with ReLU hidden layers,
 * parameters W1[128][18], b1, W2[128][128], b2, w3, b3.  With bf != 0 the GEMM operands
 * (features, weights, first-layer activations) are rounded to bfloat16 (ties to even).
 * ------------------------------------------------------------------------- */
static double o_bf16(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    u &= 0xFFFF0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

static double o_relu(double x)
{
    return x > 0.0 ? x : 0.0;
}

/* the network on weights already in their working precision (rounded to bfloat16 by
 * mlp_round_weights when bf != 0); features and first-layer activations are rounded here */
static double mlp_eval(const double *p, const double *x, int bf)
{
    const double *W1 = p, *b1 = p + 2304, *W2 = p + 2432, *b2 = p + 18816, *w3 = p + 18944;
    const double b3 = p[19072];
    double xq[18], a1[128];
    for (int k = 0; k < 18; ++k) xq[k] = bf ? o_bf16(x[k]) : x[k];
    for (int n = 0; n < 128; ++n) {
        double z = 0.0;
        for (int k = 0; k < 18; ++k) z += W1[n * 18 + k] * xq[k];
        z += b1[n];
        a1[n] = bf ? o_bf16(o_relu(z)) : o_relu(z);
    }
    double y = 0.0;
    for (int n = 0; n < 128; ++n) {
        double z = 0.0;
        for (int k = 0; k < 128; ++k) z += W2[n * 128 + k] * a1[k];
        z += b2[n];
        y += o_relu(z) * w3[n];
    }
    return y + b3;
}

/* copy of the 19073 parameters with W1, W2 and w3 rounded to bfloat16 when bf != 0
 * (biases stay as they are); the caller frees it */
static double *mlp_round_weights(const double *p, int bf)
{
    double *q = malloc(sizeof(double) * 19073);
    if (!q) return NULL;
    memcpy(q, p, sizeof(double) * 19073);
    if (bf) {
        for (int k = 0; k < 2304; ++k) q[k] = o_bf16(q[k]);
        for (int k = 2432; k < 18816; ++k) q[k] = o_bf16(q[k]);
        for (int k = 18944; k < 19072; ++k) q[k] = o_bf16(q[k]);
    }
    return q;
}

double oracle_mlp(const double *p, const double *x, int bf)
{
    double *q = mlp_round_weights(p, bf);
    if (!q) return NAN;
    const double y = mlp_eval(q, x, bf);
    free(q);
    return y;
}

/* one closure step of one current component; hist[0..15] newest first, shifted in place;
 * params as given by mlp_round_weights */
static double closure_step(double *hist, double e, double jprev, const double *coef,
                           const double *params, int bf)
{
    for (int k = 15; k > 0; --k) hist[k] = hist[k - 1];
    hist[0] = e;
    double s = 0.0;
    for (int k = 0; k < 16; ++k) s = fmax(s, fabs(hist[k]));
    s = fmax(s, 1e-30);
    double x[18];
    for (int k = 0; k < 16; ++k) x[k] = hist[k] / s;
    x[16] = coef[2];
    x[17] = coef[3];
    double y = mlp_eval(params, x, bf);
    return coef[0] * jprev + coef[1] * (e + s * y);
}

/* ---------------------------------------------------------------------------
 * 2D TEz: Ex at (i+1/2, j)   Ex[j*nx + i],      i < nx, j <= ny
 *         Ey at (i, j+1/2)   Ey[j*(nx+1) + i],  i <= nx, j < ny
 *         Hz at (i+1/2,j+1/2) Hz[j*nx + i],     i < nx, j < ny
 * Per-cell inputs ne, nubar [j*nx + i].  Plasma cells are those with ne > 0
 * in increasing linear index; df[(c*nv + a)*nv + b], a = vx bin, b = vy bin.
 * psi: 4 arrays packed back to back: psi_exy (Ex size), psi_eyx (Ey size),
 *      psi_hzx (Hz size), psi_hzy (Hz size).
 * Jx, Jy: edge currents (Ex, Ey sizes).
 * src_kind: 0 none, 1 soft Ey line at column src_i (all j), 2 soft Ey point
 * at (src_i, src_j).  ncpml = 0 gives a closed PEC box.
 * Probes record Ey at probe index (into the Ey array) after every step.
 * ------------------------------------------------------------------------- */
int oracle_run2d(int nx, int ny, double dx, double courant,
                 int ncpml, double cpml_order, double sigma_factor, double kappa_max,
                 double alpha_min, double alpha_max,
                 int nv, double vmax_over_vth, double te_ev, int nu_model,
                 const double *ne, const double *nubar,
                 int src_kind, int src_i, int src_j,
                 double src_amp, double src_f, double src_tau, double src_t0,
                 long long step0, long long nsteps,
                 double *Ex, double *Ey, double *Hz, double *Jx, double *Jy,
                 double *psi, double *df,
                 int nprobe, const int *probe_idx, double *probe_out,
                 const int *cell_mode, const double *clo_coef, const double *mlp_params,
                 int emulate_bf16, double *clo_hist, double *clo_J)
{
    /* cell_mode (per plasma cell, may be NULL): 0 kinetic F1, 1 learned closure with
     * clo_coef[c][4] = (alpha, beta, q1, q2) of that cell, clo_hist[c][2][16] its field
     * history and clo_J[c][2] its normalised current dt/eps0 * J (state, in/out). */
    if (nx < 2 || ny < 2 || nv < 2 || dx <= 0.0) return -1;
    if (courant <= 0.0 || courant > 1.0 / sqrt(2.0)) return -1;
    if (2 * ncpml >= nx || 2 * ncpml >= ny) return -1;
    /* the network's weights in their working precision, rounded once */
    double *mlp_w = NULL;
    if (cell_mode) {
        mlp_w = mlp_round_weights(mlp_params, emulate_bf16);
        if (!mlp_w) return -1;
    }
    const double dt = courant * dx / K_C0;
    const size_t nEx = (size_t)nx * (ny + 1), nEy = (size_t)(nx + 1) * ny, nHz = (size_t)nx * ny;
    double *psi_exy = psi, *psi_eyx = psi + nEx, *psi_hzx = psi + nEx + nEy, *psi_hzy = psi_hzx + nHz;

    /* velocity tables */
    double *v = malloc(sizeof(double) * nv), *fh = malloc(sizeof(double) * nv);
    double *gh = malloc(sizeof(double) * nv), *sh = malloc(sizeof(double) * nv * nv);
    double dv, vth;
    if (oracle_vgrid(nv, vmax_over_vth, te_ev, v, fh, gh, &dv, &vth) != 0) {
        free(v); free(fh); free(gh); free(sh); free(mlp_w); return -1;
    }
    oracle_nu_shape(2, nv, v, fh, dv, nu_model, sh);
    const int nv2 = nv * nv;
    double *gx = malloc(sizeof(double) * nv2), *gy = malloc(sizeof(double) * nv2);
    for (int a = 0; a < nv; ++a)
        for (int b = 0; b < nv; ++b) {
            double f2 = fh[a] * fh[b];
            gx[a * nv + b] = -v[a] * f2 / (vth * vth);
            gy[a * nv + b] = -v[b] * f2 / (vth * vth);
        }

    /* CPML profiles */
    double *bex = malloc(sizeof(double) * (nx + 1)), *aex = malloc(sizeof(double) * (nx + 1)), *kex = malloc(sizeof(double) * (nx + 1));
    double *bhx = malloc(sizeof(double) * nx), *ahx = malloc(sizeof(double) * nx), *khx = malloc(sizeof(double) * nx);
    double *bey = malloc(sizeof(double) * (ny + 1)), *aey = malloc(sizeof(double) * (ny + 1)), *key = malloc(sizeof(double) * (ny + 1));
    double *bhy = malloc(sizeof(double) * ny), *ahy = malloc(sizeof(double) * ny), *khy = malloc(sizeof(double) * ny);
    oracle_cpml_profile(nx, ncpml, dx, dt, cpml_order, sigma_factor, kappa_max, alpha_min, alpha_max, bex, aex, kex, bhx, ahx, khx);
    oracle_cpml_profile(ny, ncpml, dx, dt, cpml_order, sigma_factor, kappa_max, alpha_min, alpha_max, bey, aey, key, bhy, ahy, khy);

    /* plasma cells */
    int ncell = 0;
    for (size_t k = 0; k < nHz; ++k) if (ne[k] > 0.0) ++ncell;
    int *cell_idx = malloc(sizeof(int) * (ncell > 0 ? ncell : 1));
    for (size_t k = 0, c = 0; k < nHz; ++k) if (ne[k] > 0.0) cell_idx[c++] = (int)k;
    double *jbx = calloc(nHz, sizeof(double)), *jby = calloc(nHz, sizeof(double));

    const double ch = dt / k_mu0();
    const double ce = dt / K_EPS0;

    for (long long s = 0; s < nsteps; ++s) {
        long long n = step0 + s;
        /* 1. Hz^{n+1/2} with CPML psi at the H side */
        #pragma omp parallel for schedule(static)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t k = (size_t)j * nx + i;
                double dEx = Ex[(size_t)(j + 1) * nx + i] - Ex[(size_t)j * nx + i];
                double dEy = Ey[(size_t)j * (nx + 1) + i + 1] - Ey[(size_t)j * (nx + 1) + i];
                psi_hzx[k] = bhx[i] * psi_hzx[k] + ahx[i] * dEy;
                psi_hzy[k] = bhy[j] * psi_hzy[k] + ahy[j] * dEx;
                Hz[k] += ch * (dEx / (khy[j] * dx) - dEy / (khx[i] * dx) + psi_hzy[k] - psi_hzx[k]);
            }

        /* 2-3. F1 update with E^n averaged to the cell centre, then the cell
         *      current moments (Jx, Jy)^{n+1/2} */
        #pragma omp parallel for schedule(static)
        for (int c = 0; c < ncell; ++c) {
            int k = cell_idx[c], i = k % nx, j = k / nx;
            double exc = 0.5 * (Ex[(size_t)j * nx + i] + Ex[(size_t)(j + 1) * nx + i]);
            double eyc = 0.5 * (Ey[(size_t)j * (nx + 1) + i] + Ey[(size_t)j * (nx + 1) + i + 1]);
            if (cell_mode && cell_mode[c] == 1) {
                const double *cf = clo_coef + 4 * (size_t)c;
                clo_J[2 * c] = closure_step(clo_hist + 32 * (size_t)c, exc, clo_J[2 * c], cf,
                                            mlp_w, emulate_bf16);
                clo_J[2 * c + 1] = closure_step(clo_hist + 32 * (size_t)c + 16, eyc,
                                                clo_J[2 * c + 1], cf, mlp_w, emulate_bf16);
                jbx[k] = clo_J[2 * c] * K_EPS0 / dt;
                jby[k] = clo_J[2 * c + 1] * K_EPS0 / dt;
                continue;
            }
            double *f = df + (size_t)c * nv2;
            double accx = 0.0, accy = 0.0;
            for (int a = 0; a < nv; ++a)
                for (int b = 0; b < nv; ++b) {
                    int q = a * nv + b;
                    double nu = nubar[k] * sh[q];
                    f[q] = ((2.0 - dt * nu) * f[q]
                            + 2.0 * dt * (K_QE / K_ME) * ne[k] * (gx[q] * exc + gy[q] * eyc))
                           / (2.0 + dt * nu);
                    accx += v[a] * f[q];
                    accy += v[b] * f[q];
                }
            jbx[k] = -K_QE * dv * dv * accx;
            jby[k] = -K_QE * dv * dv * accy;
        }

        /* 4. edge currents: mean of the two adjacent cell-centre currents */
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double lo = (j > 0) ? jbx[(size_t)(j - 1) * nx + i] : 0.0;
                double hi = (j < ny) ? jbx[(size_t)j * nx + i] : 0.0;
                Jx[(size_t)j * nx + i] = 0.5 * (lo + hi);
            }
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                double lo = (i > 0) ? jby[(size_t)j * nx + i - 1] : 0.0;
                double hi = (i < nx) ? jby[(size_t)j * nx + i] : 0.0;
                Jy[(size_t)j * (nx + 1) + i] = 0.5 * (lo + hi);
            }

        /* 5. E^{n+1} with CPML psi at the E side; PEC walls keep the
         *    tangential E on the outer boundary at zero */
        #pragma omp parallel for schedule(static)
        for (int j = 1; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t k = (size_t)j * nx + i;
                double dHz = Hz[(size_t)j * nx + i] - Hz[(size_t)(j - 1) * nx + i];
                psi_exy[k] = bey[j] * psi_exy[k] + aey[j] * dHz;
                Ex[k] += ce * (dHz / (key[j] * dx) + psi_exy[k] - Jx[k]);
            }
        #pragma omp parallel for schedule(static)
        for (int j = 0; j < ny; ++j)
            for (int i = 1; i < nx; ++i) {
                size_t k = (size_t)j * (nx + 1) + i;
                double dHz = Hz[(size_t)j * nx + i] - Hz[(size_t)j * nx + i - 1];
                psi_eyx[k] = bex[i] * psi_eyx[k] + aex[i] * dHz;
                Ey[k] += ce * (-dHz / (kex[i] * dx) - psi_eyx[k] - Jy[k]);
            }

        /* 6. soft source at t^{n+1} */
        if (src_amp != 0.0 && src_kind != 0) {
            double g = source_wave((double)(n + 1) * dt, src_amp, src_f, src_tau, src_t0);
            if (src_kind == 1 && src_i > 0 && src_i < nx)
                for (int j = 0; j < ny; ++j) Ey[(size_t)j * (nx + 1) + src_i] += g;
            if (src_kind == 2 && src_i > 0 && src_i < nx && src_j >= 0 && src_j < ny)
                Ey[(size_t)src_j * (nx + 1) + src_i] += g;
        }
        for (int p = 0; p < nprobe; ++p) probe_out[s * nprobe + p] = Ey[probe_idx[p]];
    }

    free(v); free(fh); free(gh); free(sh); free(gx); free(gy);
    free(bex); free(aex); free(kex); free(bhx); free(ahx); free(khx);
    free(bey); free(aey); free(key); free(bhy); free(ahy); free(khy);
    free(cell_idx); free(jbx); free(jby); free(mlp_w);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Isolated plasma cells driven by a prescribed field (training data for the
 * learned closure and its checks).  The F1 update and current moment are those
 * of the coupled runs above (section 5.2), with E^n taken from the input series
 * instead of a grid.  Returns J^{n+1/2} (SI) for every n.
 * ------------------------------------------------------------------------- */
int oracle_replay1v(int nv, double vmax_over_vth, double te_ev, int nu_model,
                    double ne, double nubar, double dt, long long nsteps,
                    const double *E, double *J)
{
    double *v = malloc(sizeof(double) * nv), *fh = malloc(sizeof(double) * nv);
    double *gh = malloc(sizeof(double) * nv), *sh = malloc(sizeof(double) * nv);
    double *f = calloc(nv, sizeof(double));
    double dv, vth;
    if (oracle_vgrid(nv, vmax_over_vth, te_ev, v, fh, gh, &dv, &vth) != 0) {
        free(v); free(fh); free(gh); free(sh); free(f); return -1;
    }
    oracle_nu_shape(1, nv, v, fh, dv, nu_model, sh);
    for (long long n = 0; n < nsteps; ++n) {
        double acc = 0.0;
        for (int j = 0; j < nv; ++j) {
            double nu = nubar * sh[j];
            f[j] = ((2.0 - dt * nu) * f[j] + 2.0 * dt * (K_QE / K_ME) * ne * gh[j] * E[n])
                   / (2.0 + dt * nu);
            acc += v[j] * f[j];
        }
        J[n] = -K_QE * dv * acc;
    }
    free(v); free(fh); free(gh); free(sh); free(f);
    return 0;
}

int oracle_replay2v(int nv, double vmax_over_vth, double te_ev, int nu_model,
                    double ne, double nubar, double dt, long long nsteps,
                    const double *Ex, const double *Ey, double *Jx, double *Jy)
{
    double *v = malloc(sizeof(double) * nv), *fh = malloc(sizeof(double) * nv);
    double *gh = malloc(sizeof(double) * nv), *sh = malloc(sizeof(double) * nv * nv);
    double *f = calloc((size_t)nv * nv, sizeof(double));
    double dv, vth;
    if (oracle_vgrid(nv, vmax_over_vth, te_ev, v, fh, gh, &dv, &vth) != 0) {
        free(v); free(fh); free(gh); free(sh); free(f); return -1;
    }
    oracle_nu_shape(2, nv, v, fh, dv, nu_model, sh);
    for (long long n = 0; n < nsteps; ++n) {
        double ax = 0.0, ay = 0.0;
        for (int a = 0; a < nv; ++a)
            for (int b = 0; b < nv; ++b) {
                int q = a * nv + b;
                double f2 = fh[a] * fh[b];
                double gx = -v[a] * f2 / (vth * vth), gy = -v[b] * f2 / (vth * vth);
                double nu = nubar * sh[q];
                f[q] = ((2.0 - dt * nu) * f[q]
                        + 2.0 * dt * (K_QE / K_ME) * ne * (gx * Ex[n] + gy * Ey[n])) / (2.0 + dt * nu);
                ax += v[a] * f[q];
                ay += v[b] * f[q];
            }
        Jx[n] = -K_QE * dv * dv * ax;
        Jy[n] = -K_QE * dv * dv * ay;
    }
    free(v); free(fh); free(gh); free(sh); free(f);
    return 0;
}

/* ===========================================================================
 * 3D: the paper's production model.  Yee cube (section 2, eq. (1)-(5) in
 * their 3D form) with the CPML of eq. (4) on all six faces; in every plasma
 * point the anisotropic part F1 of the distribution is a vector on a speed
 * grid (section 5.1 expansion F = F0 + (v/|v|).F1, section 5.3 arrays with
 * v_dim speeds), one component at each E component's point, updated by the
 * section 5.3 Crank-Nicolson form with J = -e (4 pi / 3) gam sum v^3 F1.
 * ======================================================================== */

/* Speed grid v_k = (k + 1/2) gam, k = 0..vdim-1, gam = vmax / vdim, vmax =
 * vmax_over_vth * v_th (v_th = sqrt(e Te / m)).  F0 isotropic, normalised by
 * 4 pi gam sum v_k^2 F0_k = 1:
 *   model 0 Maxwellian  F0 ~ exp(-v^2 / (2 v_th^2)),  dF0/dv = -v F0 / v_th^2;
 *   model 1 Druyvesteyn F0 ~ exp(-(v / vD)^4) with the Maxwellian's mean energy
 *           (3/2) e Te: vD^2 = 3 v_th^2 Gamma(3/4) / Gamma(5/4); dF0/dv = -4 v^3 F0 / vD^4. */
int oracle_sgrid(int vdim, double vmax_over_vth, double te_ev, int f0_model,
                 double *v, double *F0, double *dF0, double *gam_out, double *vth_out)
{
    if (vdim < 1 || te_ev <= 0.0 || vmax_over_vth <= 0.0 || (f0_model != 0 && f0_model != 1))
        return -1;
    double vth = sqrt(K_QE * te_ev / K_ME);
    double gam = vmax_over_vth * vth / (double)vdim;
    double vd4 = 0.0;
    if (f0_model == 1) {
        double vd2 = 3.0 * vth * vth * tgamma(0.75) / tgamma(1.25);
        vd4 = vd2 * vd2;
    }
    double norm = 0.0;
    for (int k = 0; k < vdim; ++k) {
        v[k] = ((double)k + 0.5) * gam;
        double u = v[k];
        F0[k] = (f0_model == 0) ? exp(-u * u / (2.0 * vth * vth)) : exp(-u * u * u * u / vd4);
        norm += 4.0 * K_PI * gam * u * u * F0[k];
    }
    for (int k = 0; k < vdim; ++k) {
        F0[k] /= norm;
        double u = v[k];
        dF0[k] = (f0_model == 0) ? -u * F0[k] / (vth * vth) : -4.0 * u * u * u * F0[k] / vd4;
    }
    *gam_out = gam;
    *vth_out = vth;
    return 0;
}

/* nu_k = nubar * s_k: hard sphere (nu = N s v) s_k = v_k / <v> with the mean
 * speed <v> = 4 pi gam sum v^3 F0; const: s_k = 1. */
int oracle_snu_shape(int vdim, const double *v, const double *F0, double gam, int model,
                     double *s)
{
    double mean = 0.0;
    for (int k = 0; k < vdim; ++k) mean += 4.0 * K_PI * gam * v[k] * v[k] * v[k] * F0[k];
    for (int k = 0; k < vdim; ++k) s[k] = (model == 0) ? v[k] / mean : 1.0;
    return 0;
}

/* Storage (i fastest, then j, then k):
 *   Ex [nz+1][ny+1][nx]  at (i+1/2, j, k)      Hx [nz][ny][nx+1]    at (i, j+1/2, k+1/2)
 *   Ey [nz+1][ny][nx+1]  at (i, j+1/2, k)      Hy [nz][ny+1][nx]    at (i+1/2, j, k+1/2)
 *   Ez [nz][ny+1][nx+1]  at (i, j, k+1/2)      Hz [nz+1][ny][nx]    at (i+1/2, j+1/2, k)
 * E = Ex|Ey|Ez and H = Hx|Hy|Hz concatenated; J like E (SI).  psi: 12 arrays,
 * each the size of its field, in the order ex_y ex_z ey_z ey_x ez_x ez_y
 * hx_z hx_y hy_x hy_z hz_y hz_x.  Tangential E on the outer faces stays zero
 * (PEC backing of the CPML).  ne / nubar per cell [nz][ny][nx]; an E point is
 * a plasma point if it is updated (not on a face its component is tangential
 * to) and the mean density of the four cells that share its edge is > 0; its
 * n and nubar are those means.  df rows (vdim values): the plasma points of
 * Ex, then of Ey, then of Ez, each in storage order.
 * Source kinds: 1 sheet, Ex += g at every updated Ex point of plane k = src_k;
 * 2 point, Ex += g at (src_i + 1/2, src_j, src_k).
 * model 0 is the above with F0 held.  Models 1 and 2 are the two-term model of
 * sections 5.1-5.3 (F0 evolving under the l = 0 equation, or held): a plasma
 * point is then an updated E point whose four cells all have ne > 0, F0 - n F0hat
 * lives in every cell with ne > 0 (df rows after the points' F1 rows, cells in
 * storage order), an edge sees the mean of its four cells' F0 in its F1 drive,
 * and each cell collects a quarter of E.F1 from each of its plasma edges for its
 * l = 0 flux; J takes the weights (v^3 at the lower speed face + v^3 at the upper,
 * zero at vmax) / 2, which makes the exchange of energy between the field and
 * the cells' electrons exact. */
/* One candidate E point at flat index `at` whose edge touches the cells c[0..3]:
 * a plasma point if the mean density is > 0 (strict: if all four cells are
 * plasma, the reading of the two-term model, whose F0 lives in the cells). */
static int o3_point(size_t at, const size_t c[4], const double *ne, const double *nubar,
                    int strict, int np, int *pidx, double *pn, double *pnu, int *pcell)
{
    double n = 0.25 * (ne[c[0]] + ne[c[1]] + ne[c[2]] + ne[c[3]]);
    int ok = strict ? (ne[c[0]] > 0.0 && ne[c[1]] > 0.0 && ne[c[2]] > 0.0 && ne[c[3]] > 0.0)
                    : n > 0.0;
    if (!ok) return np;
    if (pidx) {
        pidx[np] = (int)at;
        pn[np] = n;
        pnu[np] = 0.25 * (nubar[c[0]] + nubar[c[1]] + nubar[c[2]] + nubar[c[3]]);
        if (pcell)
            for (int q = 0; q < 4; ++q) pcell[4 * np + q] = (int)c[q];
    }
    return np + 1;
}

static int o3_plasma_ex(int nx, int ny, int nz, const double *ne, const double *nubar,
                        int strict, int *pidx, double *pn, double *pnu, int *pcell)
{
    int np = 0;
#define CELL(a, b, cc) ((size_t)(cc) * ny * nx + (size_t)(b) * nx + (a))
    for (int k = 1; k < nz; ++k)
        for (int j = 1; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c[4] = {CELL(i, j - 1, k - 1), CELL(i, j, k - 1), CELL(i, j - 1, k), CELL(i, j, k)};
                np = o3_point(((size_t)k * (ny + 1) + j) * nx + i, c, ne, nubar, strict, np,
                              pidx, pn, pnu, pcell);
            }
    size_t offy = (size_t)nx * (ny + 1) * (nz + 1);
    for (int k = 1; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 1; i < nx; ++i) {
                size_t c[4] = {CELL(i - 1, j, k - 1), CELL(i, j, k - 1), CELL(i - 1, j, k), CELL(i, j, k)};
                np = o3_point(offy + ((size_t)k * ny + j) * (nx + 1) + i, c, ne, nubar, strict, np,
                              pidx, pn, pnu, pcell);
            }
    size_t offz = offy + (size_t)(nx + 1) * ny * (nz + 1);
    for (int k = 0; k < nz; ++k)
        for (int j = 1; j < ny; ++j)
            for (int i = 1; i < nx; ++i) {
                size_t c[4] = {CELL(i - 1, j - 1, k), CELL(i, j - 1, k), CELL(i - 1, j, k), CELL(i, j, k)};
                np = o3_point(offz + ((size_t)k * (ny + 1) + j) * (nx + 1) + i, c, ne, nubar, strict,
                              np, pidx, pn, pnu, pcell);
            }
#undef CELL
    return np;
}

static int o3_plasma(int nx, int ny, int nz, const double *ne, const double *nubar,
                     int *pidx, double *pn, double *pnu)
{
    return o3_plasma_ex(nx, ny, nz, ne, nubar, 0, pidx, pn, pnu, NULL);
}

int oracle_plasma3d_count(int nx, int ny, int nz, const double *ne)
{
    return o3_plasma(nx, ny, nz, ne, ne, NULL, NULL, NULL);
}

/* Plasma points of the two-term 3D model (all four cells around the edge are
 * plasma) and plasma cells (ne > 0). */
int oracle_plasma3d_count_strict(int nx, int ny, int nz, const double *ne, int *ncell)
{
    size_t n = (size_t)nx * ny * nz;
    int nc = 0;
    for (size_t q = 0; q < n; ++q) nc += ne[q] > 0.0;
    *ncell = nc;
    return o3_plasma_ex(nx, ny, nz, ne, ne, 1, NULL, NULL, NULL, NULL);
}

/* E index and four cells of every plasma point, in the order df stores them */
int oracle_plasma3d_map(int nx, int ny, int nz, const double *ne, int strict, int *pidx, int *pcell)
{
    int np = o3_plasma_ex(nx, ny, nz, ne, ne, strict, NULL, NULL, NULL, NULL);
    double *tmp = malloc(sizeof(double) * 2 * (np > 0 ? np : 1));
    o3_plasma_ex(nx, ny, nz, ne, ne, strict, pidx, tmp, tmp + (np > 0 ? np : 1), pcell);
    free(tmp);
    return np;
}

int oracle_run3d(int nx, int ny, int nz, double dx, double courant,
                 int ncpml, double cpml_order, double sigma_factor, double kappa_max,
                 double alpha_min, double alpha_max,
                 int vdim, double vmax_over_vth, double te_ev, int nu_model, int f0_model,
                 const double *ne, const double *nubar,
                 int src_kind, int src_i, int src_j, int src_k,
                 double src_amp, double src_f, double src_tau, double src_t0,
                 long long step0, long long nsteps,
                 double *E, double *H, double *J, double *psi, double *df,
                 int nprobe, const int *probe_idx, double *probe_out, int model)
{
    if (nx < 2 || ny < 2 || nz < 2 || vdim < 1 || dx <= 0.0) return -1;
    if (model < 0 || model > 2) return -1;
    if (courant <= 0.0 || courant > 1.0 / sqrt(3.0)) return -1;
    if (2 * ncpml >= nx || 2 * ncpml >= ny || 2 * ncpml >= nz) return -1;
    const double dt = courant * dx / K_C0;
    const size_t NX = nx, NY = ny, NZ = nz;
    const size_t nEx = NX * (NY + 1) * (NZ + 1), nEy = (NX + 1) * NY * (NZ + 1),
                 nEz = (NX + 1) * (NY + 1) * NZ;
    const size_t nHx = (NX + 1) * NY * NZ, nHy = NX * (NY + 1) * NZ, nHz = NX * NY * (NZ + 1);
    double *Ex = E, *Ey = E + nEx, *Ez = E + nEx + nEy;
    double *Hx = H, *Hy = H + nHx, *Hz = H + nHx + nHy;
    double *Jx = J, *Jy = J + nEx, *Jz = J + nEx + nEy;
    double *p_exy = psi, *p_exz = p_exy + nEx, *p_eyz = p_exz + nEx, *p_eyx = p_eyz + nEy;
    double *p_ezx = p_eyx + nEy, *p_ezy = p_ezx + nEz;
    double *p_hxz = p_ezy + nEz, *p_hxy = p_hxz + nHx, *p_hyx = p_hxy + nHx, *p_hyz = p_hyx + nHy;
    double *p_hzy = p_hyz + nHy, *p_hzx = p_hzy + nHz;

    double *v = malloc(sizeof(double) * vdim), *F0 = malloc(sizeof(double) * vdim);
    double *dF0 = malloc(sizeof(double) * vdim), *sh = malloc(sizeof(double) * vdim);
    double gam, vth;
    if (oracle_sgrid(vdim, vmax_over_vth, te_ev, f0_model, v, F0, dF0, &gam, &vth) != 0) {
        free(v); free(F0); free(dF0); free(sh); return -1;
    }
    oracle_snu_shape(vdim, v, F0, gam, nu_model, sh);

    double *pr[3][6];   /* be ae ke bh ah kh per axis */
    int nn[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
        for (int q = 0; q < 6; ++q) pr[a][q] = malloc(sizeof(double) * (nn[a] + 1));
        oracle_cpml_profile(nn[a], ncpml, dx, dt, cpml_order, sigma_factor, kappa_max,
                            alpha_min, alpha_max, pr[a][0], pr[a][1], pr[a][2],
                            pr[a][3], pr[a][4], pr[a][5]);
    }
    const double *bex = pr[0][0], *aex = pr[0][1], *kex = pr[0][2];
    const double *bhx = pr[0][3], *ahx = pr[0][4], *khx = pr[0][5];
    const double *bey = pr[1][0], *aey = pr[1][1], *key = pr[1][2];
    const double *bhy = pr[1][3], *ahy = pr[1][4], *khy = pr[1][5];
    const double *bez = pr[2][0], *aez = pr[2][1], *kez = pr[2][2];
    const double *bhz = pr[2][3], *ahz = pr[2][4], *khz = pr[2][5];

    /* model 0: F1 on every E point with plasma around it, F0 frozen (J weights
     * v^3, as printed); models 1 (F0 evolving) and 2 (held): the two-term model
     * with F0 in the plasma cells, F1 on the points whose four cells are all
     * plasma, face-averaged moment weights (the adjoint of the l = 0 flux form) */
    const int tt = model != 0;
    int np = o3_plasma_ex(nx, ny, nz, ne, nubar, tt, NULL, NULL, NULL, NULL);
    int *pidx = malloc(sizeof(int) * (np > 0 ? np : 1));
    double *pn = malloc(sizeof(double) * (np > 0 ? np : 1));
    double *pnu = malloc(sizeof(double) * (np > 0 ? np : 1));
    int *pcell = malloc(sizeof(int) * 4 * (np > 0 ? np : 1));
    o3_plasma_ex(nx, ny, nz, ne, nubar, tt, pidx, pn, pnu, pcell);
    double *w = malloc(sizeof(double) * vdim);
    for (int k = 0; k < vdim; ++k) {
        double lo = (double)k * gam, hi = (double)(k + 1) * gam;
        w[k] = tt ? 0.5 * (lo * lo * lo + (k + 1 < vdim ? hi * hi * hi : 0.0))
                  : v[k] * v[k] * v[k];
    }
    /* plasma cells (F0 rows after the np F1 rows of df), each cell's edges */
    const size_t ncells = NX * NY * NZ;
    int *crow = malloc(sizeof(int) * ncells);
    int nc = 0;
    for (size_t q = 0; q < ncells; ++q) crow[q] = (tt && ne[q] > 0.0) ? nc++ : -1;
    int *cedge = malloc(sizeof(int) * 12 * (nc > 0 ? nc : 1));
    int *cnt = calloc(nc > 0 ? nc : 1, sizeof(int));
    for (int q = 0; q < 12 * nc; ++q) cedge[q] = -1;
    for (int p = 0; tt && p < np; ++p)
        for (int q = 0; q < 4; ++q) {
            int r = crow[pcell[4 * p + q]];
            cedge[12 * r + cnt[r]++] = p;
        }
    double *d0 = df + (size_t)np * vdim;
    double *estash = malloc(sizeof(double) * (np > 0 ? np : 1));

    const double ch = dt / k_mu0(), ce = dt / K_EPS0;
#define IEX(i, j, k) (((size_t)(k) * (NY + 1) + (j)) * NX + (i))
#define IEY(i, j, k) (((size_t)(k) * NY + (j)) * (NX + 1) + (i))
#define IEZ(i, j, k) (((size_t)(k) * (NY + 1) + (j)) * (NX + 1) + (i))
#define IHX(i, j, k) (((size_t)(k) * NY + (j)) * (NX + 1) + (i))
#define IHY(i, j, k) (((size_t)(k) * (NY + 1) + (j)) * NX + (i))
#define IHZ(i, j, k) (((size_t)(k) * NY + (j)) * NX + (i))
    for (long long s = 0; s < nsteps; ++s) {
        long long n = step0 + s;
        /* 1. H^{n+1/2}: mu dH/dt = -curl E with the CPML-stretched derivatives */
        #pragma omp parallel for schedule(static)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i <= nx; ++i) {
                    size_t q = IHX(i, j, k);
                    double dEy_z = Ey[IEY(i, j, k + 1)] - Ey[IEY(i, j, k)];
                    double dEz_y = Ez[IEZ(i, j + 1, k)] - Ez[IEZ(i, j, k)];
                    p_hxz[q] = bhz[k] * p_hxz[q] + ahz[k] * dEy_z;
                    p_hxy[q] = bhy[j] * p_hxy[q] + ahy[j] * dEz_y;
                    Hx[q] += ch * (dEy_z / (khz[k] * dx) + p_hxz[q] - dEz_y / (khy[j] * dx) - p_hxy[q]);
                }
        #pragma omp parallel for schedule(static)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j <= ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    size_t q = IHY(i, j, k);
                    double dEz_x = Ez[IEZ(i + 1, j, k)] - Ez[IEZ(i, j, k)];
                    double dEx_z = Ex[IEX(i, j, k + 1)] - Ex[IEX(i, j, k)];
                    p_hyx[q] = bhx[i] * p_hyx[q] + ahx[i] * dEz_x;
                    p_hyz[q] = bhz[k] * p_hyz[q] + ahz[k] * dEx_z;
                    Hy[q] += ch * (dEz_x / (khx[i] * dx) + p_hyx[q] - dEx_z / (khz[k] * dx) - p_hyz[q]);
                }
        #pragma omp parallel for schedule(static)
        for (int k = 0; k <= nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    size_t q = IHZ(i, j, k);
                    double dEx_y = Ex[IEX(i, j + 1, k)] - Ex[IEX(i, j, k)];
                    double dEy_x = Ey[IEY(i + 1, j, k)] - Ey[IEY(i, j, k)];
                    p_hzy[q] = bhy[j] * p_hzy[q] + ahy[j] * dEx_y;
                    p_hzx[q] = bhx[i] * p_hzx[q] + ahx[i] * dEy_x;
                    Hz[q] += ch * (dEx_y / (khy[j] * dx) + p_hzy[q] - dEy_x / (khx[i] * dx) - p_hzx[q]);
                }

        /* 2-3. F1 of every plasma point driven by its E component at t^n, and
         *      the current J^{n+1/2} = -e (4 pi / 3) gam sum v^3 F1 (section 5.3) */
        #pragma omp parallel for schedule(static)
        for (int p = 0; p < np; ++p) {
            double *f = df + (size_t)p * vdim;
            double e = E[pidx[p]], acc = 0.0;
            estash[p] = e;
            /* two-term: F0 - n F0hat at the edge = mean over its four cells */
            double dm[vdim > 0 ? vdim : 1];
            for (int k = 0; k < vdim; ++k) {
                dm[k] = 0.0;
                if (tt)
                    for (int q = 0; q < 4; ++q) dm[k] += 0.25 * d0[(size_t)crow[pcell[4 * p + q]] * vdim + k];
            }
            for (int k = 0; k < vdim; ++k) {
                double nu = pnu[p] * sh[k];
                double D = pn[p] * dF0[k];
                if (tt) {
                    double below = k > 0 ? dm[k - 1] : dm[0], above = k + 1 < vdim ? dm[k + 1] : 0.0;
                    D += (above - below) / (2.0 * gam);
                }
                f[k] = ((2.0 - dt * nu) * f[k] + 2.0 * dt * (K_QE / K_ME) * e * D) / (2.0 + dt * nu);
                acc += w[k] * f[k];
            }
            J[pidx[p]] = -K_QE * (4.0 * K_PI / 3.0) * gam * acc;
        }

        /* 4. E^{n+1}: eps dE/dt = curl H - J, interior (tangential) points only */
        #pragma omp parallel for schedule(static)
        for (int k = 1; k < nz; ++k)
            for (int j = 1; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    size_t q = IEX(i, j, k);
                    double dHz_y = Hz[IHZ(i, j, k)] - Hz[IHZ(i, j - 1, k)];
                    double dHy_z = Hy[IHY(i, j, k)] - Hy[IHY(i, j, k - 1)];
                    p_exy[q] = bey[j] * p_exy[q] + aey[j] * dHz_y;
                    p_exz[q] = bez[k] * p_exz[q] + aez[k] * dHy_z;
                    Ex[q] += ce * (dHz_y / (key[j] * dx) + p_exy[q] - dHy_z / (kez[k] * dx) - p_exz[q] - Jx[q]);
                }
        #pragma omp parallel for schedule(static)
        for (int k = 1; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 1; i < nx; ++i) {
                    size_t q = IEY(i, j, k);
                    double dHx_z = Hx[IHX(i, j, k)] - Hx[IHX(i, j, k - 1)];
                    double dHz_x = Hz[IHZ(i, j, k)] - Hz[IHZ(i - 1, j, k)];
                    p_eyz[q] = bez[k] * p_eyz[q] + aez[k] * dHx_z;
                    p_eyx[q] = bex[i] * p_eyx[q] + aex[i] * dHz_x;
                    Ey[q] += ce * (dHx_z / (kez[k] * dx) + p_eyz[q] - dHz_x / (kex[i] * dx) - p_eyx[q] - Jy[q]);
                }
        #pragma omp parallel for schedule(static)
        for (int k = 0; k < nz; ++k)
            for (int j = 1; j < ny; ++j)
                for (int i = 1; i < nx; ++i) {
                    size_t q = IEZ(i, j, k);
                    double dHy_x = Hy[IHY(i, j, k)] - Hy[IHY(i - 1, j, k)];
                    double dHx_y = Hx[IHX(i, j, k)] - Hx[IHX(i, j - 1, k)];
                    p_ezx[q] = bex[i] * p_ezx[q] + aex[i] * dHy_x;
                    p_ezy[q] = bey[j] * p_ezy[q] + aey[j] * dHx_y;
                    Ez[q] += ce * (dHy_x / (kex[i] * dx) + p_ezx[q] - dHx_y / (key[j] * dx) - p_ezy[q] - Jz[q]);
                }

        /* 5. soft source at t^{n+1} */
        if (src_amp != 0.0 && src_kind != 0 && src_k > 0 && src_k < nz) {
            double g = source_wave((double)(n + 1) * dt, src_amp, src_f, src_tau, src_t0);
            if (src_kind == 1)
                for (int j = 1; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) Ex[IEX(i, j, src_k)] += g;
            if (src_kind == 2 && src_i >= 0 && src_i < nx && src_j > 0 && src_j < ny)
                Ex[IEX(src_i, src_j, src_k)] += g;
        }
        /* 6. two-term: F0^{n+1} of every plasma cell from the l = 0 equation, the
         *    flux through each speed face summed over the cell's edges, each edge
         *    handing a quarter of its Ebar F1 to each of its four cells */
        if (model == 1) {
            #pragma omp parallel for schedule(static)
            for (int r = 0; r < nc; ++r) {
                double G[vdim > 0 ? vdim : 1];
                for (int k = 0; k < vdim; ++k) G[k] = 0.0;
                for (int q = 0; q < 12; ++q) {
                    int p = cedge[12 * r + q];
                    if (p < 0) continue;
                    double eb = 0.25 * 0.5 * (estash[p] + E[pidx[p]]);
                    for (int k = 0; k < vdim; ++k) G[k] += eb * df[(size_t)p * vdim + k];
                }
                double phi_lo = 0.0;
                for (int k = 0; k < vdim; ++k) {
                    double vf = (double)(k + 1) * gam;
                    double phi_hi = (k + 1 < vdim) ? vf * vf * 0.5 * (G[k] + G[k + 1]) : 0.0;
                    d0[(size_t)r * vdim + k] += dt * (K_QE / (3.0 * K_ME)) * (phi_hi - phi_lo)
                                                / (v[k] * v[k] * gam);
                    phi_lo = phi_hi;
                }
            }
        }
        for (int p = 0; p < nprobe; ++p) probe_out[s * nprobe + p] = E[probe_idx[p]];
    }
#undef IEX
#undef IEY
#undef IEZ
#undef IHX
#undef IHY
#undef IHZ
    free(v); free(F0); free(dF0); free(sh);
    for (int a = 0; a < 3; ++a)
        for (int q = 0; q < 6; ++q) free(pr[a][q]);
    free(pidx); free(pn); free(pnu); free(pcell); free(w); free(crow); free(cedge); free(cnt);
    free(estash);
    return 0;
}

/* ===========================================================================
 * 1D two-term model on the speed grid: the paper's own representation
 * (section 5.1 expansion F = F0 + (v/|v|).F1, the l = 0 and l = 1 equations,
 * section 5.3 speed grid) in the geometry of its argon experiment, a field
 * E = Ez along the line.  Per plasma node: F1 (the z component) and F0 on the
 * speed grid v_k = (k + 1/2) gam of oracle_sgrid, row = [F1 | F0 - n F0hat].
 * Per step (after H^{n+1/2}):
 *   F1^{n+1/2} = ((2 - dt nu_k) F1 + 2 dt (e/m) E^n D_k) / (2 + dt nu_k),
 *     D_k = n dF0hat/dv (analytic) + centred difference of (F0 - n F0hat),
 *     even across v = 0, zero beyond vmax;
 *   J^{n+1/2} = -e (4 pi / 3) gam sum_k w_k F1_k,
 *     w_k = (v_{k-1/2}^3 + v_{k+1/2}^3) / 2 over the faces of bin k that carry
 *     flux (v_{-1/2} = 0; the face at vmax carries none);
 *   E^{n+1} (Ampere with -J), boundaries, source;
 *   F0^{n+1} = F0^n + dt (e / 3m) Ebar (phi_{k+1/2} - phi_{k-1/2}) / (v_k^2 gam),
 *     phi = v^2 (F1_k + F1_{k+1}) / 2 on the inner faces, 0 at v = 0 and vmax,
 *     Ebar = (E^n + E^{n+1}) / 2   (l = 0 equation without streaming; only
 *     elastic collisions, whose l = 0 term carries the electron-to-neutral
 *     mass ratio and is dropped).
 * The weights w_k make the F0 update exactly the adjoint of the current: the
 * field energy that J^{n+1/2} removes, dt Ebar J, is exactly the kinetic energy
 * (m/2) 4 pi gam sum v_k^4 F0_k gained, and the electron number
 * 4 pi gam sum v_k^2 F0_k is kept.  evolve_f0 = 0 freezes F0 (the linear
 * speed-grid model with these weights).
 * ======================================================================== */
int oracle_run1d_twoterm(int nx, double dx, double courant, int bc,
                         int vdim, double vmax_over_vth, double te_ev, int nu_model, int f0_model,
                         const double *ne, const double *nubar,
                         int src_node, double src_amp, double src_f, double src_tau, double src_t0,
                         long long step0, long long nsteps,
                         double *E, double *H, double *J, double *df,
                         int nprobe, const int *probe_node, double *probe_E, int evolve_f0)
{
    if (nx < 2 || vdim < 2 || dx <= 0.0 || courant <= 0.0 || courant > 1.0) return -1;
    if (ne[0] > 0.0 || ne[nx] > 0.0) return -1;
    const double dt = courant * dx / K_C0;
    double *v = malloc(sizeof(double) * vdim), *F0 = malloc(sizeof(double) * vdim);
    double *dF0 = malloc(sizeof(double) * vdim), *sh = malloc(sizeof(double) * vdim);
    double *w = malloc(sizeof(double) * vdim);
    double gam, vth;
    if (oracle_sgrid(vdim, vmax_over_vth, te_ev, f0_model, v, F0, dF0, &gam, &vth) != 0) {
        free(v); free(F0); free(dF0); free(sh); free(w); return -1;
    }
    oracle_snu_shape(vdim, v, F0, gam, nu_model, sh);
    for (int k = 0; k < vdim; ++k) {
        double lo = (double)k * gam, hi = (double)(k + 1) * gam;      /* faces of bin k */
        w[k] = 0.5 * (lo * lo * lo + (k + 1 < vdim ? hi * hi * hi : 0.0));
    }
    int ncell = 0;
    for (int i = 0; i <= nx; ++i) if (ne[i] > 0.0) ++ncell;
    int *cell_node = malloc(sizeof(int) * (ncell > 0 ? ncell : 1));
    for (int i = 0, c = 0; i <= nx; ++i) if (ne[i] > 0.0) cell_node[c++] = i;
    double *Eold = malloc(sizeof(double) * (nx + 1));

    const double ch = dt / (k_mu0() * dx), ce = dt / (K_EPS0 * dx), cj = dt / K_EPS0;
    const double q = (K_C0 * dt - dx) / (K_C0 * dt + dx);
    const double a0 = K_QE / (3.0 * K_ME);
    for (long long s = 0; s < nsteps; ++s) {
        long long n = step0 + s;
        for (int i = 0; i < nx; ++i) H[i] += ch * (E[i + 1] - E[i]);
        /* F1 driven by E^n and the current F0, then J */
        #pragma omp parallel for schedule(static)
        for (int c = 0; c < ncell; ++c) {
            int i = cell_node[c];
            double *f1 = df + (size_t)c * 2 * vdim, *d0 = f1 + vdim;
            double acc = 0.0;
            for (int k = 0; k < vdim; ++k) {
                double below = k > 0 ? d0[k - 1] : d0[0];
                double above = k + 1 < vdim ? d0[k + 1] : 0.0;
                double D = ne[i] * dF0[k] + (above - below) / (2.0 * gam);
                double x = dt * nubar[i] * sh[k];
                f1[k] = ((2.0 - x) * f1[k] + 2.0 * dt * (K_QE / K_ME) * E[i] * D) / (2.0 + x);
                acc += w[k] * f1[k];
            }
            J[i] = -K_QE * (4.0 * K_PI / 3.0) * gam * acc;
        }
        memcpy(Eold, E, sizeof(double) * (nx + 1));
        double e0 = E[0], e1 = E[1], en1 = E[nx - 1], en = E[nx];
        for (int i = 1; i < nx; ++i) E[i] += ce * (H[i] - H[i - 1]) - cj * J[i];
        if (bc == 1) {
            E[0] = e1 + q * (E[1] - e0);
            E[nx] = en1 + q * (E[nx - 1] - en);
        } else {
            E[0] = 0.0; E[nx] = 0.0;
        }
        if (src_amp != 0.0 && src_node > 0 && src_node < nx)
            E[src_node] += source_wave((double)(n + 1) * dt, src_amp, src_f, src_tau, src_t0);
        /* F0^{n+1} from the l = 0 equation with Ebar = (E^n + E^{n+1}) / 2 */
        if (evolve_f0) {
            #pragma omp parallel for schedule(static)
            for (int c = 0; c < ncell; ++c) {
                int i = cell_node[c];
                double *f1 = df + (size_t)c * 2 * vdim, *d0 = f1 + vdim;
                double eb = 0.5 * (Eold[i] + E[i]);
                double phi_lo = 0.0;
                for (int k = 0; k < vdim; ++k) {
                    double vf = (double)(k + 1) * gam;
                    double phi_hi = (k + 1 < vdim) ? vf * vf * 0.5 * (f1[k] + f1[k + 1]) : 0.0;
                    d0[k] += dt * a0 * eb * (phi_hi - phi_lo) / (v[k] * v[k] * gam);
                    phi_lo = phi_hi;
                }
            }
        }
        for (int p = 0; p < nprobe; ++p) probe_E[s * nprobe + p] = E[probe_node[p]];
    }
    free(v); free(F0); free(dF0); free(sh); free(w); free(cell_node); free(Eold);
    return 0;
}
