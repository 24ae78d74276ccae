"""Plain FP64 CPU oracle for the vdW-DF nonlocal correlation energy and potential, evaluated
in the Roman-Perez--Soler (RPS) form of the libvdwxc paper (arXiv:1703.06999).

TEST INFRASTRUCTURE ONLY.  This module is the independent reference that the GPU library is
checked against.  Only the test-suite, the package's smoke check and the CPU-baseline leg of the
benchmark may import it; the library never does, and it shares no code with the library (it
reads the same seeded inputs and kernel table, nothing else).

It is written for clarity, not speed: every step is the paper's step, in its order and notation,
with numpy / scipy.fft as the only library primitives (the FFT is a library routine; it is pinned
against a naive DFT in the tests).

Steps (Sec. 3, Table 1, and the enumerated procedure of Sec. 3):
  1. q0(n, sigma) with the saturation h_a                       (appendix)
  2. theta_a(r) = n(r) p_a(q0(r))                               (Sec. 2, helper splines)
  3. theta_a(k) by forward 3D FFT                               (Sec. 3, step 2)
  4. per k: phi_ab(|k|) by linear interpolation in k; F_a(k) = sum_b phi_ab theta_b(k);
     energy sum_a theta_a*(k) F_a(k)                            (Sec. 3, steps 3a-3c; eq. enlk)
  5. F_a(r) by inverse FFT                                      (Sec. 3, step 4)
  6. dE/dn, dE/dsigma                                           (Sec. 2, eqs. dedn and dedsigma)
and, beside the nonlocal path, the semilocal LDA correlation E_c^LDA, v_c^LDA of eq. 1's split
(PW92, appendix), and the spin-polarised variant that Sec. 7 announces (q0 from the two spin
densities; steps 2-5 unchanged; the two potentials as the spin-paired one, per spin).

Readings where the paper is silent or garbled (each also listed in the design notes):
  * r_s = (3/(4 pi n))^{1/3}, the Wigner-Seitz radius (the appendix prints r_s^3 = 4 pi n/3,
    which inverts it).
  * The gradient term of q0 is -(Z_ab/36) sigma/(k_F n^2), as printed in the appendix's main
    formula (q0 then carries units of inverse length, like k_F).
  * Helper splines: natural cubic splines (second derivative zero at both ends).
  * q0 below the first mesh point is clamped to it with zero derivatives; q0 equal to the last
    mesh point falls in the last interval.
  * Saturation: for x/a >= 2, exp(-S) underflows to zero in FP64, so h = a and h' = 0 exactly;
    the derivative is set to zero there without forming 0 * (large).
  * n < 1e-30 is a vacuum point: theta = 0 and both partial derivatives are zero.
  * Discrete transforms: theta(m) = sum_j theta(r_j) exp(-2 pi i j.m/N) (unnormalised forward),
    F(r) = (1/N) sum_m F(m) exp(+2 pi i j.m/N), E = Omega/(2 N^2) sum_m sum_a Re[theta_a* F_a];
    this is eq. enlk with integrals replaced by the periodic-grid sums.
  * |G| of a frequency that sits on the Nyquist index of an even axis is ambiguous (+N/2 and
    -N/2 alias).  G is split into the part from the non-Nyquist axes and the part from the
    Nyquist axes (each taken at +N/2), and |G|^2 is the sum of their squared norms: the two are
    added in quadrature, the Nyquist components among themselves are summed as vectors.  With
    one Nyquist index this is the mean of |G|^2 over its two aliases.  It keeps phi(|G|) even in
    G, so F(k) stays Hermitian and F(r) real; for orthogonal cells it is the plain |G|.
  * phi = 0 for |G| >= kmax of the table (callers reject such grids).
  * Potential entry: v = dE/dn - div(2 dE/dsigma grad n), the divergence (and, when no gradient
    is supplied, the gradient) taken spectrally with every Nyquist frequency zeroed.
  * Spin polarisation (Sec. 7 announces it; the paper prints no formula, so this part is pinned
    only through its reductions, limits and finite differences): theta_a = n p_a(q0) with the
    total density n = n_up + n_dn, and q0 = -(4 pi/3) eps_xc^0 with the gradient-corrected LDA
    exchange of the appendix spin-scaled, E_x[n_up, n_dn] = (E_x[2 n_up] + E_x[2 n_dn])/2, and the
    spin-resolved PW92 correlation eps_c(r_s, zeta):
        q0 = sum_s (n_s/n) k_s [1 - (Z_ab/9) sigma_ss / (4 k_s^2 n_s^2)] - (4 pi/3) eps_c(r_s, zeta)
    with k_s = (6 pi^2 n_s)^{1/3} = k_F(2 n_s); at n_up = n_dn, sigma_uu = sigma_dd = sigma/4 it is
    the spin-paired q0.  A spin density below 1e-30 (negative ones included) is taken as zero.
    eps_c(r_s, 1) and the spin stiffness alpha_c(r_s) use Perdew and Wang's published fits (the
    paper prints only the zeta = 0 one).  Saturation, clamp and vacuum as spin-paired.
"""
from __future__ import annotations

import math
import os
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import scipy.fft as sfft

# ---------------------------------------------------------------------------------------------
# constants printed in the paper's appendix
# ---------------------------------------------------------------------------------------------
PW92_A = 0.031091
PW92_ALPHA1 = 0.2137
PW92_BETA = (7.5957, 3.5876, 1.6382, 0.49294)
ZAB = {"DF1": -0.8491, "DF2": -1.887}
# spin-resolved PW92 fits (Perdew and Wang 1992): (A, alpha1, beta1..4) of eps_c(r_s, 1) and of
# -alpha_c(r_s), and f''(0) of the spin interpolation f(zeta); the zeta = 0 set is the appendix's
PW92_FERRO = (0.015545, 0.20548, (14.1189, 6.1977, 3.3662, 0.62517))
PW92_MINUS_ALPHA = (0.016887, 0.11125, (10.357, 3.6231, 0.88026, 0.49671))
PW92_FZZ0 = 1.709921
SATURATION_A = 5.0
SATURATION_TERMS = 12
VACUUM_DENSITY = 1e-30


def _workers():
    """scipy.fft worker threads: the host's cores available to this process, capped by
    OMP_NUM_THREADS when that is set (on a shared host it names this process's share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


WORKERS = _workers()


def _map_chunks(fn, count, chunk):
    """[fn(s, e) for consecutive ranges [s, e) of `chunk` items covering range(count)], the calls
    spread over WORKERS threads (numpy releases the GIL inside its loops).  The ranges are
    independent; the results come back in range order."""
    ranges = [(s, min(s + chunk, count)) for s in range(0, count, chunk)]
    if WORKERS <= 1 or len(ranges) <= 1:
        return [fn(s, e) for s, e in ranges]
    with ThreadPoolExecutor(max_workers=WORKERS) as pool:
        return list(pool.map(lambda r: fn(*r), ranges))


# ---------------------------------------------------------------------------------------------
# 1. q0 (appendix)
# ---------------------------------------------------------------------------------------------

def pw92_correlation(rs):
    """Perdew-Wang LDA correlation energy per particle eps_c(r_s) and d eps_c / d r_s.

    eps_c = -2A (1 + alpha1 r_s) log[1 + 1/(2A sum_{i=1..4} beta_i r_s^{i/2})]   (appendix)
    """
    rs = np.asarray(rs, dtype=np.float64)
    b1, b2, b3, b4 = PW92_BETA
    sq = np.sqrt(rs)
    Q = 2.0 * PW92_A * (b1 * sq + b2 * rs + b3 * rs * sq + b4 * rs * rs)
    dQ = 2.0 * PW92_A * (0.5 * b1 / sq + b2 + 1.5 * b3 * sq + 2.0 * b4 * rs)
    L = np.log1p(1.0 / Q)
    eps = -2.0 * PW92_A * (1.0 + PW92_ALPHA1 * rs) * L
    deps = -2.0 * PW92_A * PW92_ALPHA1 * L + 2.0 * PW92_A * (1.0 + PW92_ALPHA1 * rs) * dQ / (Q * Q + Q)
    return eps, deps


def lda_correlation(n, cell):
    """Semilocal LDA part of the vdW-DF correlation, spin-paired (eq. 1 splits E_c into E_c^LDA +
    E_c^nl; eps_c is the appendix's PW92 form).

    E_c^LDA = int n eps_c(r_s) dr, as the grid sum (Omega/N) sum_j n_j eps_c(r_s(n_j)) with
    r_s = (3/(4 pi n))^{1/3};  v_c^LDA = d(n eps_c)/dn = eps_c + n (d eps_c/d r_s)(d r_s/d n)
    = eps_c - (r_s/3) d eps_c/d r_s.  Vacuum points (n < 1e-30) add nothing and get v = 0.
    Returns (E, v)."""
    n = np.asarray(n, dtype=np.float64)
    cell = np.asarray(cell, dtype=np.float64)
    dV = float(np.linalg.det(cell)) / n.size
    live = n >= VACUUM_DENSITY
    rs = np.where(live, np.cbrt(3.0 / (4.0 * math.pi * np.where(live, n, 1.0))), 1.0)
    eps, deps = pw92_correlation(rs)
    v = np.where(live, eps - (rs / 3.0) * deps, 0.0)
    E = dV * float(np.sum(np.where(live, n * eps, 0.0)))
    return E, v


def pw92_G(rs, A, alpha1, beta):
    """The PW92 form G(r_s) = -2A (1 + alpha1 r_s) log[1 + 1/(2A sum_{i=1..4} beta_i r_s^{i/2})]
    for one parameter set, and dG/dr_s."""
    rs = np.asarray(rs, dtype=np.float64)
    b1, b2, b3, b4 = beta
    sq = np.sqrt(rs)
    Q = 2.0 * A * (b1 * sq + b2 * rs + b3 * rs * sq + b4 * rs * rs)
    dQ = 2.0 * A * (0.5 * b1 / sq + b2 + 1.5 * b3 * sq + 2.0 * b4 * rs)
    L = np.log1p(1.0 / Q)
    G = -2.0 * A * (1.0 + alpha1 * rs) * L
    dG = -2.0 * A * alpha1 * L + 2.0 * A * (1.0 + alpha1 * rs) * dQ / (Q * Q + Q)
    return G, dG


def spin_interpolation(zeta):
    """f(zeta) = [(1+zeta)^{4/3} + (1-zeta)^{4/3} - 2] / (2^{4/3} - 2) and f'(zeta)."""
    z = np.asarray(zeta, dtype=np.float64)
    den = 2.0 ** (4.0 / 3.0) - 2.0
    up, dn = np.cbrt(1.0 + z), np.cbrt(1.0 - z)
    f = ((1.0 + z) * up + (1.0 - z) * dn - 2.0) / den
    df = (4.0 / 3.0) * (up - dn) / den
    return f, df


def pw92_spin_correlation(rs, zeta):
    """Spin-polarised PW92 correlation energy per particle
        eps_c(r_s, zeta) = eps_c(r_s, 0) + alpha_c(r_s) f(zeta)/f''(0) (1 - zeta^4)
                           + [eps_c(r_s, 1) - eps_c(r_s, 0)] f(zeta) zeta^4
    (eps_c(r_s, 0) the appendix's form; eps_c(r_s, 1) and -alpha_c fitted by the same form) and its
    partials in r_s and zeta.  Returns (eps, d eps/d r_s, d eps/d zeta)."""
    rs = np.asarray(rs, dtype=np.float64)
    z = np.asarray(zeta, dtype=np.float64)
    e0, de0 = pw92_correlation(rs)
    e1, de1 = pw92_G(rs, *PW92_FERRO)
    ma, dma = pw92_G(rs, *PW92_MINUS_ALPHA)
    ac, dac = -ma, -dma
    f, df = spin_interpolation(z)
    z4 = z ** 4
    eps = e0 + ac * f / PW92_FZZ0 * (1.0 - z4) + (e1 - e0) * f * z4
    deps_drs = de0 + dac * f / PW92_FZZ0 * (1.0 - z4) + (de1 - de0) * f * z4
    deps_dz = (ac / PW92_FZZ0 * (df * (1.0 - z4) - 4.0 * z ** 3 * f)
               + (e1 - e0) * (df * z4 + 4.0 * z ** 3 * f))
    return eps, deps_drs, deps_dz


def saturation(x, a=SATURATION_A):
    """h_a(x) = a [1 - exp(-sum_{m=1}^{12} (x/a)^m / m)] and its derivative h_a'(x)  (appendix)."""
    x = np.asarray(x, dtype=np.float64)
    t = x / a
    S = np.zeros_like(t)
    dS = np.zeros_like(t)          # dS/dx = (1/a) sum_{m=1}^{12} t^{m-1}
    with np.errstate(over="ignore"):   # huge t only occurs on the saturated branch below
        for m in range(1, SATURATION_TERMS + 1):
            S = S + t ** m / m
            dS = dS + t ** (m - 1)
        e = np.exp(-S)
    h = a * (1.0 - e)
    saturated = t >= 2.0           # exp(-S) == 0 exactly in FP64 there
    hprime = np.where(saturated, 0.0, e * np.where(saturated, 0.0, dS))
    h = np.where(saturated, a, h)
    return h, hprime


def q0_unsaturated(n, sigma, zab):
    """q0 = k_F - (4 pi/3) eps_c^LDA - (Z_ab/36) sigma/(k_F n^2) for n > 0, with its partial
    derivatives in n and sigma (appendix)."""
    n = np.asarray(n, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    kF = np.cbrt(3.0 * math.pi ** 2 * n)
    rs = np.cbrt(3.0 / (4.0 * math.pi * n))
    eps_c, deps_c = pw92_correlation(rs)
    x = kF - (4.0 * math.pi / 3.0) * eps_c - (zab / 36.0) * sigma / (kF * n * n)
    # d kF/dn = kF/(3n); d rs/dn = -rs/(3n)
    dx_dn = (kF / (3.0 * n) + (4.0 * math.pi / 9.0) * (rs / n) * deps_c
             + (7.0 * zab / 108.0) * sigma / (kF * n ** 3))
    dx_dsigma = -(zab / 36.0) / (kF * n * n)
    return x, dx_dn, dx_dsigma


def q0_and_derivatives(n, sigma, qmesh, zab):
    """Saturated q0 = h_5(q0_orig) with dq0/dn, dq0/dsigma and the vacuum mask (n < 1e-30)."""
    n = np.asarray(n, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    vac = ~(n >= VACUUM_DENSITY)
    ns = np.where(vac, 1.0, n)                      # any positive value; masked below
    x, dx_dn, dx_ds = q0_unsaturated(ns, np.where(vac, 0.0, sigma), zab)
    q0, hp = saturation(x)
    dq_dn = np.where(hp == 0.0, 0.0, hp * np.where(hp == 0.0, 0.0, dx_dn))
    dq_ds = np.where(hp == 0.0, 0.0, hp * np.where(hp == 0.0, 0.0, dx_ds))
    below = q0 < qmesh[0]                           # clamp to the first mesh point
    q0 = np.where(below, qmesh[0], q0)
    dq_dn = np.where(below | vac, 0.0, dq_dn)
    dq_ds = np.where(below | vac, 0.0, dq_ds)
    return q0, dq_dn, dq_ds, vac


def q0_spin_unsaturated(n_up, n_dn, s_uu, s_dd, zab):
    """Unsaturated spin-polarised q0 (the reading in the header) for n = n_up + n_dn >= 1e-30, with
    its partials in n_up, n_dn, sigma_uu, sigma_dd.  Spin densities below 1e-30 count as zero (that
    channel drops out; n still moves with it, d n / d n_s = 1).  Returns (x, dx/dn_up, dx/dn_dn,
    dx/dsigma_uu, dx/dsigma_dd)."""
    nu = np.asarray(n_up, dtype=np.float64)
    nd = np.asarray(n_dn, dtype=np.float64)
    su = np.asarray(s_uu, dtype=np.float64)
    sd = np.asarray(s_dd, dtype=np.float64)
    live_u, live_d = nu >= VACUUM_DENSITY, nd >= VACUUM_DENSITY
    nu = np.where(live_u, nu, 0.0)
    nd = np.where(live_d, nd, 0.0)
    n = nu + nd
    # exchange: sum_s (n_s/n) k_s [1 - (Z_ab/9) s_s^2],  s_s^2 = sigma_ss / (4 k_s^2 n_s^2)
    X = np.zeros_like(n)
    dX = []       # d/dn_s of the channel's own term (n held fixed), d/dsigma_ss
    for ns, ss, live in ((nu, su, live_u), (nd, sd, live_d)):
        nsafe = np.where(live, ns, 1.0)
        ks = np.cbrt(6.0 * math.pi ** 2 * nsafe)
        term = ns / n * ks - (zab / 36.0) * ss / (n * nsafe * ks)
        dterm_dns = (4.0 / 3.0) * ks / n + (zab / 27.0) * ss / (n * nsafe ** 2 * ks)
        dterm_dss = -(zab / 36.0) / (n * nsafe * ks)
        X = X + np.where(live, term, 0.0)
        dX.append((np.where(live, dterm_dns, 0.0), np.where(live, dterm_dss, 0.0)))
    # correlation: eps_c(r_s, zeta), r_s = (3/(4 pi n))^{1/3}, zeta = (n_up - n_dn)/n
    rs = np.cbrt(3.0 / (4.0 * math.pi * n))
    zeta = (nu - nd) / n
    ec, dec_drs, dec_dz = pw92_spin_correlation(rs, zeta)
    x = X - (4.0 * math.pi / 3.0) * ec
    drs_dn = -rs / (3.0 * n)
    dx_dnu = dX[0][0] - X / n - (4.0 * math.pi / 3.0) * (dec_drs * drs_dn + dec_dz * (1.0 - zeta) / n)
    dx_dnd = dX[1][0] - X / n - (4.0 * math.pi / 3.0) * (dec_drs * drs_dn - dec_dz * (1.0 + zeta) / n)
    return x, dx_dnu, dx_dnd, dX[0][1], dX[1][1]


def q0_spin_and_derivatives(n_up, n_dn, s_uu, s_dd, qmesh, zab):
    """Saturated spin-polarised q0 with its four partials and the vacuum mask (n_up + n_dn below
    1e-30 after the per-channel cut), saturation and clamp as in q0_and_derivatives."""
    nu = np.asarray(n_up, dtype=np.float64)
    nd = np.asarray(n_dn, dtype=np.float64)
    n = np.where(nu >= VACUUM_DENSITY, nu, 0.0) + np.where(nd >= VACUUM_DENSITY, nd, 0.0)
    vac = ~(n >= VACUUM_DENSITY)
    # vacuum points: any live stand-in (masked below)
    nu_s = np.where(vac, 1.0, nu)
    nd_s = np.where(vac, 1.0, nd)
    zero = lambda a: np.where(vac, 0.0, np.asarray(a, dtype=np.float64))
    x, *dx = q0_spin_unsaturated(nu_s, nd_s, zero(s_uu), zero(s_dd), zab)
    q0, hp = saturation(x)
    dq = [np.where(hp == 0.0, 0.0, hp * np.where(hp == 0.0, 0.0, d)) for d in dx]
    below = q0 < qmesh[0]
    q0 = np.where(below, qmesh[0], q0)
    dq = [np.where(below | vac, 0.0, d) for d in dq]
    return q0, dq, vac, np.where(vac, 0.0, n)


# ---------------------------------------------------------------------------------------------
# 2. helper splines and theta (Sec. 2)
# ---------------------------------------------------------------------------------------------

def spline_coefficients(qmesh):
    """Coefficients a^c_{ab}, c = 0..3, of the helper splines p_a (Sec. 2):

        p_a(q_b + dq) = sum_c a^c_{ab} dq^c,   0 <= dq < q_{b+1} - q_b,

    fixed by p_a(q_b) = delta_ab and continuity of the first two derivatives; the two free end
    conditions are taken natural (p_a'' = 0 at both ends).  Returns an array [4][M][M-1].
    """
    q = np.asarray(qmesh, dtype=np.float64)
    M = q.shape[0]
    h = np.diff(q)
    coeffs = np.zeros((4, M, M - 1))
    for a in range(M):
        y = np.zeros(M)
        y[a] = 1.0
        # second derivatives m_b: tridiagonal system, m_0 = m_{M-1} = 0
        A = np.zeros((M, M))
        rhs = np.zeros(M)
        A[0, 0] = 1.0
        A[M - 1, M - 1] = 1.0
        for b in range(1, M - 1):
            A[b, b - 1] = h[b - 1]
            A[b, b] = 2.0 * (h[b - 1] + h[b])
            A[b, b + 1] = h[b]
            rhs[b] = 6.0 * ((y[b + 1] - y[b]) / h[b] - (y[b] - y[b - 1]) / h[b - 1])
        m = np.linalg.solve(A, rhs)
        for b in range(M - 1):
            coeffs[0, a, b] = y[b]
            coeffs[1, a, b] = (y[b + 1] - y[b]) / h[b] - h[b] * (2.0 * m[b] + m[b + 1]) / 6.0
            coeffs[2, a, b] = m[b] / 2.0
            coeffs[3, a, b] = (m[b + 1] - m[b]) / (6.0 * h[b])
    return coeffs


def spline_interval(qmesh, q0):
    """Interval b with q_b <= q0 < q_{b+1}; q0 equal to the last mesh point uses the last one."""
    M = len(qmesh)
    b = np.searchsorted(qmesh, q0, side="right") - 1
    return np.clip(b, 0, M - 2)


def spline_values(qmesh, coeffs, q0):
    """p_a(q0) and p_a'(q0) for all a: arrays [M][...]."""
    b = spline_interval(qmesh, q0)
    dq = q0 - qmesh[b]
    a0, a1, a2, a3 = (coeffs[c][:, b] for c in range(4))
    p = a0 + a1 * dq + a2 * dq ** 2 + a3 * dq ** 3
    dp = a1 + 2.0 * a2 * dq + 3.0 * a3 * dq ** 2
    return p, dp


def theta_and_derivatives(n, sigma, qmesh, zab):
    """theta_a = n p_a(q0) (Sec. 2) and the factors of the partial derivatives (eqs. dedn,
    dedsigma):  dtheta_a/dn = p_a + n p_a' dq0/dn,  dtheta_a/dsigma = n p_a' dq0/dsigma.
    Vacuum points carry zeros.  Arrays [M][N1][N2][N3].  Every point is independent of the others;
    the points are taken in chunks on the worker threads."""
    n = np.asarray(n, dtype=np.float64)
    sigma = np.broadcast_to(np.asarray(sigma, dtype=np.float64), n.shape)
    coeffs = spline_coefficients(qmesh)
    M = len(qmesh)
    nf, sf = n.reshape(-1), np.ascontiguousarray(sigma).reshape(-1)
    theta = np.empty((M, nf.size))
    dtheta_dn = np.empty((M, nf.size))
    dtheta_ds = np.empty((M, nf.size))

    def points(s, e):
        q0, dq_dn, dq_ds, vac = q0_and_derivatives(nf[s:e], sf[s:e], qmesh, zab)
        p, dp = spline_values(qmesh, coeffs, q0)
        nn = np.where(vac, 0.0, nf[s:e])
        theta[:, s:e] = nn * p
        dtheta_dn[:, s:e] = np.where(vac, 0.0, p + nn * dp * dq_dn)
        dtheta_ds[:, s:e] = nn * dp * dq_ds

    _map_chunks(points, nf.size, 1 << 16)
    shape = (M,) + n.shape
    return theta.reshape(shape), dtheta_dn.reshape(shape), dtheta_ds.reshape(shape)


def theta_and_derivatives_spin(n_up, n_dn, s_uu, s_dd, qmesh, zab):
    """Spin-polarised theta_a = n p_a(q0) (n = n_up + n_dn) and the factors of the four partial
    derivatives: dtheta_a/dn_s = p_a + n p_a' dq0/dn_s, dtheta_a/dsigma_ss = n p_a' dq0/dsigma_ss.
    Returns (theta, [dtheta/dn_up, dtheta/dn_dn, dtheta/dsigma_uu, dtheta/dsigma_dd])."""
    nu = np.asarray(n_up, dtype=np.float64)
    shape = nu.shape
    args = [np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), shape)).reshape(-1)
            for a in (n_up, n_dn, s_uu, s_dd)]
    coeffs = spline_coefficients(qmesh)
    M = len(qmesh)
    size = args[0].size
    theta = np.empty((M, size))
    dtheta = [np.empty((M, size)) for _ in range(4)]

    def points(s, e):
        q0, dq, vac, n = q0_spin_and_derivatives(*(a[s:e] for a in args), qmesh, zab)
        p, dp = spline_values(qmesh, coeffs, q0)
        theta[:, s:e] = n * p
        dtheta[0][:, s:e] = np.where(vac, 0.0, p + n * dp * dq[0])
        dtheta[1][:, s:e] = np.where(vac, 0.0, p + n * dp * dq[1])
        dtheta[2][:, s:e] = n * dp * dq[2]
        dtheta[3][:, s:e] = n * dp * dq[3]

    _map_chunks(points, size, 1 << 16)
    out = (M,) + shape
    return theta.reshape(out), [d.reshape(out) for d in dtheta]


# ---------------------------------------------------------------------------------------------
# grid geometry
# ---------------------------------------------------------------------------------------------

def reciprocal_vectors(cell):
    """Rows b_i with a_i . b_j = 2 pi delta_ij."""
    return 2.0 * math.pi * np.linalg.inv(np.asarray(cell, dtype=np.float64)).T


def signed_frequencies(N):
    """m -> m for m < N/2, m - N above; the Nyquist index N/2 of an even axis is flagged."""
    m = np.arange(N)
    mbar = np.where(m <= N // 2, m, m - N)
    nyq = (N % 2 == 0) & (m == N // 2)
    return mbar.astype(np.float64), nyq


def gvector_norms(grid, cell):
    """|G_m| for every m of the full grid, Nyquist components added in quadrature."""
    B = reciprocal_vectors(cell)
    freq = [signed_frequencies(N) for N in grid]
    regular = np.zeros(tuple(grid) + (3,))
    nyquist = np.zeros(tuple(grid) + (3,))
    for i in range(3):
        f, nyq = freq[i]
        shape = [1, 1, 1]
        shape[i] = grid[i]
        fi = f.reshape(shape)
        ni = nyq.reshape(shape)
        regular += (np.where(ni, 0.0, fi))[..., None] * B[i]
        nyquist += (np.where(ni, fi, 0.0))[..., None] * B[i]
    g2 = np.sum(regular ** 2, axis=-1) + np.sum(nyquist ** 2, axis=-1)
    return np.sqrt(g2)


def gvectors_cartesian(grid, cell):
    """Cartesian G_m (three arrays over the full grid) and the mask of frequencies that touch a
    Nyquist index on any even axis."""
    B = reciprocal_vectors(cell)
    G = np.zeros((3,) + tuple(grid))
    any_nyq = np.zeros(tuple(grid), dtype=bool)
    for i in range(3):
        f, nyq = signed_frequencies(grid[i])
        shape = [1, 1, 1]
        shape[i] = grid[i]
        for c in range(3):
            G[c] += f.reshape(shape) * B[i, c]
        any_nyq |= nyq.reshape(shape)
    return G, any_nyq


# ---------------------------------------------------------------------------------------------
# 3-5. FFTs and the k-space contraction (Sec. 3, steps 2-4; eq. enlk)
# ---------------------------------------------------------------------------------------------

def forward_fft(fields):
    """theta(m) = sum_j theta(r_j) exp(-2 pi i j.m / N) over the last three axes."""
    return sfft.fftn(fields, axes=(-3, -2, -1), workers=WORKERS)


def inverse_fft(fields_k):
    """F(r_j) = (1/N) sum_m F(m) exp(+2 pi i j.m / N), real part."""
    return sfft.ifftn(fields_k, axes=(-3, -2, -1), workers=WORKERS).real


def interpolate_kernel(table, kmax, knorm):
    """phi_ab(k) from the tabulated phi_ab(k_j), k_j = j dk, by linear interpolation in k
    (Sec. 3, step 3a); zero at and beyond kmax.  ``table`` [nk][M][M]; returns [len(k)][M][M]."""
    nk = table.shape[0]
    dk = kmax / (nk - 1)
    s = knorm / dk
    j = np.floor(s).astype(np.int64)
    inside = knorm < kmax
    j = np.where(inside, j, 0)
    w = np.where(inside, s - j, 0.0)
    j1 = np.minimum(j + 1, nk - 1)
    phi = (1.0 - w)[:, None, None] * table[j] + w[:, None, None] * table[j1]
    return np.where(inside[:, None, None], phi, 0.0)


def kspace_contraction(theta_k, knorm, table, kmax, chunk=2048):
    """F_a(m) = sum_b phi_ab(|G_m|) theta_b(m) and the energy sum sum_m sum_a Re[theta_a* F_a]
    (Sec. 3, steps 3a-3c).  theta_k: [M][...] complex; returns (F_k, energy_sum)."""
    M = theta_k.shape[0]
    th = theta_k.reshape(M, -1)
    kn = knorm.reshape(-1)
    F = np.empty_like(th)

    def kpoints(s, e):
        phi = interpolate_kernel(table, kmax, kn[s:e])      # [c][a][b]
        f = np.einsum("cab,bc->ac", phi, th[:, s:e])
        F[:, s:e] = f
        return float(np.sum((np.conj(th[:, s:e]) * f).real))

    esum = 0.0
    for part in _map_chunks(kpoints, kn.shape[0], chunk):   # the chunks' sums in chunk order
        esum += part
    return F.reshape(theta_k.shape), esum


# ---------------------------------------------------------------------------------------------
# the whole evaluation
# ---------------------------------------------------------------------------------------------

def _as_table(kernel):
    return np.asarray(kernel.table, dtype=np.float64), float(kernel.kmax), \
        np.asarray(kernel.qmesh, dtype=np.float64)


def check_inputs(grid, cell, n, sigma):
    if any(int(g) < 1 for g in grid):
        raise ValueError("grid sizes must be >= 1")
    if np.linalg.det(np.asarray(cell, dtype=np.float64)) <= 0.0:
        raise ValueError("cell must have positive volume (right-handed lattice vectors)")
    if not (np.all(np.isfinite(n)) and np.all(np.isfinite(sigma))):
        raise ValueError("density or sigma contains NaN/inf")


class _Steps:
    """Calls ``progress(step_name, seconds)`` after each step, if a callback is given (timing and
    progress reports only; nothing here touches the arithmetic)."""

    def __init__(self, progress):
        self.progress = progress
        self.t = time.perf_counter()

    def done(self, name):
        if self.progress is not None:
            now = time.perf_counter()
            self.progress(name, now - self.t)
            self.t = now


def _nonlocal_fields(theta, knorm, table, kmax, omega, steps):
    """Steps 2-4 of Sec. 3 on the theta fields: forward FFT, contraction with the energy sum,
    inverse FFT.  Returns (E, F(r), theta(k), F(k))."""
    N = theta[0].size
    theta_k = forward_fft(theta)                                                    # step 2
    steps.done("forward FFT")
    F_k, esum = kspace_contraction(theta_k, knorm, table, kmax)                    # step 3
    steps.done("contraction")
    E = omega / (2.0 * N * N) * esum
    F = inverse_fft(F_k)                                                            # step 4
    steps.done("inverse FFT")
    return E, F, theta_k, F_k


def energy_and_partials(n, sigma, cell, kernel, flavour="DF1", return_intermediates=False, progress=None):
    """E_c^nl and the partial derivatives dE/dn, dE/dsigma as fields (Sec. 2, eqs. dedn and
    dedsigma; Sec. 3 procedure).  Returns (E, dedn, dedsigma[, dict]).  ``progress``, if given, is
    called as progress(step, seconds) after each step."""
    steps = _Steps(progress)
    n = np.asarray(n, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    grid = n.shape
    check_inputs(grid, cell, n, sigma)
    table, kmax, qmesh = _as_table(kernel)
    omega = float(np.linalg.det(np.asarray(cell, dtype=np.float64)))
    knorm = gvector_norms(grid, cell)
    if np.max(knorm) >= kmax:
        raise ValueError("grid reaches |G| >= kmax of the kernel table")

    theta, dth_dn, dth_ds = theta_and_derivatives(n, sigma, qmesh, ZAB[flavour])   # step 1
    steps.done("q0 + theta")
    E, F, theta_k, F_k = _nonlocal_fields(theta, knorm, table, kmax, omega, steps)  # steps 2-4
    dedn = np.sum(F * dth_dn, axis=0)                                               # step 5
    dedsigma = np.sum(F * dth_ds, axis=0)
    steps.done("derivatives")
    if return_intermediates:
        return E, dedn, dedsigma, dict(theta=theta, theta_k=theta_k, F_k=F_k, F=F,
                                       dtheta_dn=dth_dn, dtheta_dsigma=dth_ds, knorm=knorm)
    return E, dedn, dedsigma


def energy_and_partials_spin(n_up, n_dn, s_uu, s_dd, cell, kernel, flavour="DF1", progress=None):
    """Spin-polarised E_c^nl (the reading in the header) and its partial derivatives with respect
    to n_up, n_dn, sigma_uu = |grad n_up|^2 and sigma_dd = |grad n_dn|^2 per point, with the
    normalisation of energy_and_partials (dE/d(value at point j) = derivative_j * Omega/N).
    Returns (E, dedn_up, dedn_dn, dedsigma_uu, dedsigma_dd)."""
    steps = _Steps(progress)
    fields = [np.asarray(a, dtype=np.float64) for a in (n_up, n_dn, s_uu, s_dd)]
    grid = fields[0].shape
    check_inputs(grid, cell, fields[0] + fields[1], fields[2] + fields[3])
    table, kmax, qmesh = _as_table(kernel)
    omega = float(np.linalg.det(np.asarray(cell, dtype=np.float64)))
    knorm = gvector_norms(grid, cell)
    if np.max(knorm) >= kmax:
        raise ValueError("grid reaches |G| >= kmax of the kernel table")
    theta, dtheta = theta_and_derivatives_spin(*fields, qmesh, ZAB[flavour])       # step 1
    steps.done("q0 + theta")
    E, F, _, _ = _nonlocal_fields(theta, knorm, table, kmax, omega, steps)         # steps 2-4
    parts = [np.sum(F * d, axis=0) for d in dtheta]                                 # step 5
    steps.done("derivatives")
    return (E, *parts)


def energy_real_space(theta, F, cell):
    """E = (dV/2) sum_j sum_a theta_a(r_j) F_a(r_j): the real-space form of Sec. 2."""
    N = theta[0].size
    dV = float(np.linalg.det(np.asarray(cell, dtype=np.float64))) / N
    return 0.5 * dV * float(np.sum(theta * F))


def spectral_derivative(f, cell, axis):
    """D_i f: derivative along Cartesian axis i by FFT, multiply by i G_i, inverse FFT, with every
    frequency that touches a Nyquist index set to zero.  Real and antisymmetric."""
    G, any_nyq = gvectors_cartesian(f.shape, cell)
    fk = sfft.fftn(f, workers=WORKERS)
    dk = np.where(any_nyq, 0.0, 1j * G[axis] * fk)
    return sfft.ifftn(dk, workers=WORKERS).real


def spectral_gradient(n, cell):
    return np.stack([spectral_derivative(n, cell, i) for i in range(3)])


def potential(n, cell, kernel, grad=None, flavour="DF1", progress=None):
    """v_c^nl = dE/dn|_sigma - div(2 dE/dsigma grad n)  (Sec. 2: v = dE/dn + dE/dsigma dsigma/dn,
    with sigma = |grad n|^2).  ``grad`` [3][...] is the supplied gradient; None means the
    spectral gradient of n.  Returns (E, v, dedn, dedsigma).  ``progress``: as in
    energy_and_partials."""
    steps = _Steps(progress)
    n = np.asarray(n, dtype=np.float64)
    g = spectral_gradient(n, cell) if grad is None else np.asarray(grad, dtype=np.float64)
    sigma = np.sum(g * g, axis=0)
    steps.done("gradient" if grad is None else "sigma")
    E, dedn, dedsigma = energy_and_partials(n, sigma, cell, kernel, flavour, progress=progress)
    steps.t = time.perf_counter()
    div = sum(spectral_derivative(2.0 * dedsigma * g[i], cell, i) for i in range(3))
    steps.done("divergence")
    return E, dedn - div, dedn, dedsigma


def potential_spin(n_up, n_dn, grad_up, grad_dn, cell, kernel, flavour="DF1", progress=None):
    """Spin-polarised potentials v_s = dE/dn_s|_sigma - div(2 dE/dsigma_ss grad n_s), s = up, dn
    (the spin functional of energy_and_partials_spin depends on sigma_ss = |grad n_s|^2 only), with
    the supplied gradients [3][...] and the spectral divergence of ``potential``.
    Returns (E, v_up, v_dn)."""
    steps = _Steps(progress)
    g = [np.asarray(x, dtype=np.float64) for x in (grad_up, grad_dn)]
    sig = [np.sum(x * x, axis=0) for x in g]
    E, dnu, dnd, dsu, dsd = energy_and_partials_spin(n_up, n_dn, sig[0], sig[1], cell, kernel, flavour,
                                                    progress=progress)
    steps.t = time.perf_counter()
    v = [dn - sum(spectral_derivative(2.0 * ds * gs[i], cell, i) for i in range(3))
         for dn, ds, gs in ((dnu, dsu, g[0]), (dnd, dsd, g[1]))]
    steps.done("divergence")
    return E, v[0], v[1]
