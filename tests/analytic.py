"""Closed forms that pin the oracle (and, through it, the HIP path).

None of these re-runs the oracle's time stepping: they are frequency-domain or
analytic solutions of the same discrete (or continuous) equations, computed
independently here with their own constants and velocity tables.
"""
import math

import numpy as np

C0 = 299792458.0
EPS0 = 8.8541878128e-12
QE = 1.602176634e-19
ME = 9.1093837015e-31
MU0 = 1.0 / (EPS0 * C0 ** 2)
ETA0 = math.sqrt(MU0 / EPS0)


def plasma_omega2(ne):
    return np.asarray(ne) * QE ** 2 / (EPS0 * ME)


def velocity_weights(nv, vmax_over_vth, te_ev, nu_model="hard_sphere", dims=1):
    """Per-bin weights w_j = v_j^2 fhat_j dv^d / v_th^2 (component along the drive) and the
    collision-frequency shapes s_j, on the symmetric cell-centred grid."""
    vth = math.sqrt(QE * te_ev / ME)
    dv = 2.0 * vmax_over_vth * vth / nv
    v = (np.arange(nv) - (nv - 1) / 2.0) * dv
    f = np.exp(-v ** 2 / (2 * vth ** 2))
    f /= f.sum() * dv
    if dims == 1:
        w = v ** 2 * f * dv / vth ** 2
        speed = np.abs(v)
        fw = f * dv
    else:
        vx, vy = np.meshgrid(v, v, indexing="ij")
        f2 = np.outer(f, f)
        w = (vx ** 2 * f2 * dv * dv / vth ** 2).ravel()
        speed = np.sqrt(vx ** 2 + vy ** 2).ravel()
        fw = (f2 * dv * dv).ravel()
    if nu_model == "hard_sphere":
        s = speed / np.sum(speed * fw)
    else:
        s = np.ones_like(speed)
    return w, s


def discrete_eps(omega, dt, courant, wp2, nubar, w, s):
    """Effective permittivity of one plasma node of the discrete coupled scheme (leap-frog
    fields, per-bin Crank-Nicolson F1, current at n+1/2), e^{-i omega t} phasors."""
    th = omega * dt / 2.0
    nu = nubar * s
    alpha = (2 - dt * nu) / (2 + dt * nu)
    beta = 2 * dt ** 2 * wp2 * w / (2 + dt * nu)
    return 1.0 + np.sum(1j * beta / (2 * math.sin(th) * (np.exp(-1j * th) - alpha * np.exp(1j * th))))


def discrete_slab_rt(omega, dt, courant, ne_nodes, nubar_nodes, w, s, node_r, node_t,
                     avg_edges=False):
    """Reflection (at node ``node_r``, left of the medium) and transmission (at node
    ``node_t``, right of it) of a right-going discrete plane wave through the medium
    described per E node.  Solves the three-point recurrence exactly by a sweep from the
    outgoing side.  ``avg_edges`` models the 2D scheme seen along a y-invariant slab:
    cell-centre kinetics between nodes i and i+1, E averaged onto them and the current
    averaged back to the nodes."""
    th = omega * dt / 2.0
    K = 2 * math.asin(math.sin(th) / courant)
    nn = len(ne_nodes)
    wp2 = plasma_omega2(ne_nodes)
    sigma = np.zeros(nn, dtype=complex)   # normalised current response chi_i: Jhat_i = chi_i * E_i
    for i in range(nn):
        if ne_nodes[i] > 0:
            sigma[i] = discrete_eps(omega, dt, courant, wp2[i], nubar_nodes[i], w, s) - 1.0
    # recurrence: E_{i+1} + E_{i-1} = 2 E_i - (2 sin th / S)^2 (E_i + P_i)
    # P_i = chi_i E_i (co-located) or 1/4 [chi_{i-1/2}(E_{i-1}+E_i) + chi_{i+1/2}(E_i+E_{i+1})]
    g = (2 * math.sin(th) / courant) ** 2
    N = nn - 1
    E = np.zeros(nn, dtype=complex)
    E[N] = np.exp(1j * K * N)
    E[N - 1] = np.exp(1j * K * (N - 1))
    for i in range(N - 1, 0, -1):
        if not avg_edges:
            E[i - 1] = 2 * E[i] - g * (1 + sigma[i]) * E[i] - E[i + 1]
        else:
            cl, cr = sigma[i - 1], sigma[i]       # cells (i-1, i) and (i, i+1)
            # E_{i+1}(1 + g cr/4) + E_{i-1}(1 + g cl/4) = E_i (2 - g - g (cl + cr)/4)
            E[i - 1] = (E[i] * (2 - g - g * (cl + cr) / 4) - E[i + 1] * (1 + g * cr / 4)) / (1 + g * cl / 4)
    i0 = node_r
    # E_i = I e^{iKi} + R e^{-iKi} for i in the left vacuum region
    A = np.array([[np.exp(1j * K * i0), np.exp(-1j * K * i0)],
                  [np.exp(1j * K * (i0 + 1)), np.exp(-1j * K * (i0 + 1))]])
    I, R = np.linalg.solve(A, E[i0:i0 + 2])
    r = R * np.exp(-1j * K * node_r) / (I * np.exp(1j * K * node_r))
    t = 1.0 / I
    return r, t


def continuous_slab_rt(omega, d, eps):
    """Textbook slab of thickness d and permittivity eps in vacuum, normal incidence."""
    n = np.sqrt(complex(eps))
    if n.imag < 0:
        n = -n
    k = omega / C0
    ph = np.exp(1j * n * k * d)
    den = (1 + n) ** 2 - (1 - n) ** 2 * ph ** 2
    t = 4 * n * ph / den * np.exp(-1j * k * d)
    r = (1 - n ** 2) * (1 - ph ** 2) / den
    return r, t


def continuous_kinetic_eps(omega, wp2, nubar, w, s):
    """Permittivity of the continuous-time kinetic model on the same velocity bins:
    each bin is a Drude term with weight w_j and collision rate nu_j."""
    nu = nubar * s
    return 1.0 - np.sum(wp2 * w / (omega * (omega + 1j * nu)))


def dft(x, omega, dt):
    n = np.arange(len(x))
    return np.sum(np.asarray(x) * np.exp(1j * omega * n * dt))
