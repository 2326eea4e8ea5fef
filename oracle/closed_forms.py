"""Exact potentials of Gaussian densities and other closed forms (Section 4).

These are the checks the method must hit, independent of the method itself:
  * 3D Coulomb of exp(-r^2/sigma^2): sigma^3 sqrt(pi) erf(r/sigma)/(4 r)      (eq. (DensGaus))
  * 3D Coulomb of exp(-sum a_i x_i^2) (any axis scales): the one-dimensional
    integral 1/2 int_0^inf prod_i (t^2+a_i)^(-1/2) exp(-a_i t^2 x_i^2/(t^2+a_i)) dt,
    from the Gaussian integral of 1/r (eq. (GauInte)) and Gaussian convolution;
    a = (1, 1, gamma^2)/sigma^2 gives the anisotropic case of eq. (DensGaus).
  * 2D Coulomb of exp(-r^2/sigma^2): (sqrt(pi) sigma/2) I0(r^2/(2 sigma^2)) exp(-r^2/(2 sigma^2))
  * 2D Coulomb of exp(-(x^2 + gamma^2 y^2)/sigma^2): the integral of eq. (2.5D-clb-exact)
    (its maximum at the origin, and its values anywhere)
  * 2D Poisson of exp(-r^2/sigma^2): -(sigma^2/4)[E1(r^2/sigma^2) + 2 ln r],
    (sigma^2/4)(gamma_e - ln sigma^2) at r = 0                                 (eq. (eg-2d-Exact))
  * Davey-Stewartson potential of pi exp(-pi^2 r^2) (Example 4.5)
  * inverse-power kernel |x|^-beta of exp(-r^2/sigma^2): a 1-D integral, and its value
    at the origin in Gamma functions
  * 3D dipolar of exp(-r^2/sigma^2): -(n.m) rho - 3 n^T D m with the Hessian D
    of the Coulomb potential (Example 4.4)
  * the 1-D factor integral in closed form, (sqrt(pi)/tau) exp(-xi^2/4tau^2)
    Re erf(tau c + i xi/(2 tau)), by mpmath
  * the Coulomb energy of a Gaussian mixture.
Near r = 0 the forms with cancellation switch to their Taylor series.
"""

from __future__ import annotations

import math

import mpmath as mp
import numpy as np
from scipy import special

EULER_GAMMA = 0.57721566490153286061


def coulomb3d_gaussian(r, sigma: float = 1.0):
    r = np.asarray(r, dtype=np.float64)
    out = np.empty_like(r)
    small = r < 1e-3 * sigma
    z = r[~small] / sigma
    out[~small] = sigma ** 3 * math.sqrt(math.pi) * special.erf(z) / (4.0 * r[~small])
    zs = r[small] / sigma
    # erf(z)/z = (2/sqrt(pi))(1 - z^2/3 + z^4/10 - z^6/42)
    out[small] = sigma ** 2 / 2.0 * (1 - zs ** 2 / 3 + zs ** 4 / 10 - zs ** 6 / 42)
    return out


def _tan_nodes(m: int = 400):
    x, w = np.polynomial.legendre.leggauss(m)
    th = (x + 1.0) * (math.pi / 4.0)
    wt = w * (math.pi / 4.0)
    return th, wt


def coulomb3d_triaxial(x, y, z, a=(1.0, 1.0, 1.0), nodes: int = 400):
    """Coulomb potential of exp(-(a1 x^2 + a2 y^2 + a3 z^2)) at the given points.
    Integral over t = tan(theta) on [0, pi/2] by Gauss-Legendre (smooth integrand)."""
    x, y, z = (np.asarray(v, dtype=np.float64).ravel() for v in (x, y, z))
    th, wt = _tan_nodes(nodes)
    out = np.zeros_like(x)
    for t_, w_ in zip(np.tan(th), wt / np.cos(th) ** 2):
        t2 = t_ * t_
        f = w_ * 0.5
        e = 0.0
        for ai, xi in zip(a, (x, y, z)):
            f = f / math.sqrt(t2 + ai)
            e = e + ai * t2 * xi * xi / (t2 + ai)
        out += f * np.exp(-e)
    return out


def coulomb3d_triaxial_mp(x, y, z, a=(1.0, 1.0, 1.0)):
    """Same integral at one point by mpmath quadrature (reference for the above)."""
    with mp.workdps(30):
        def f(t):
            v = mp.mpf(0.5)
            e = mp.mpf(0)
            for ai, xi in zip(a, (x, y, z)):
                v /= mp.sqrt(t * t + ai)
                e += ai * t * t * xi * xi / (t * t + ai)
            return v * mp.exp(-e)
        return float(mp.quad(f, [0, 1, 10, mp.inf]))


def anisotropic3d_max(sigma: float, gamma: float) -> float:
    """max |u| = u(0) for exp(-(x^2+y^2+gamma^2 z^2)/sigma^2):
    (sigma^2/(4 gamma)) int_0^inf dt / ((t+1) sqrt(t + gamma^-2))."""
    with mp.workdps(30):
        g2 = mp.mpf(1) / mp.mpf(gamma) ** 2
        v = mp.quad(lambda t: 1 / ((t + 1) * mp.sqrt(t + g2)), [0, 1, mp.inf])
        return float(mp.mpf(sigma) ** 2 / (4 * mp.mpf(gamma)) * v)


def coulomb2d_gaussian(r, sigma: float = 1.0):
    r = np.asarray(r, dtype=np.float64)
    return math.sqrt(math.pi) * sigma / 2.0 * special.i0e(r * r / (2.0 * sigma * sigma))


def anisotropic2d_max(sigma: float, gamma: float) -> float:
    """max |u| = u(0) for exp(-(x^2+gamma^2 y^2)/sigma^2) (eq. (2.5D-clb-exact) at the origin)."""
    with mp.workdps(30):
        g2 = mp.mpf(1) / mp.mpf(gamma) ** 2
        v = mp.quad(lambda t: 1 / (mp.sqrt(t * t + 1) * mp.sqrt(t * t + g2)), [0, 1, mp.inf])
        return float(mp.mpf(sigma) / (mp.mpf(gamma) * mp.sqrt(mp.pi)) * v)


def coulomb2d_anisotropic(x, y, sigma: float, gamma: float, step: float = 0.1, vmax: float = 45.0):
    """2D Coulomb potential of exp(-(x^2 + gamma^2 y^2)/sigma^2), eq. (2.5D-clb-exact):
    (sigma/(gamma sqrt(pi))) int_0^inf exp(-x^2/(sigma^2(t^2+1)) - y^2/(sigma^2(t^2+gamma^-2)))
    / (sqrt(t^2+1) sqrt(t^2+gamma^-2)) dt.  With t = exp(v) the integrand decays
    exponentially at both ends and is analytic in the strip |Im v| < pi/2, so the
    trapezoidal rule in v converges geometrically (error about exp(-pi^2/step))."""
    x, y = (np.asarray(v, dtype=np.float64).ravel() for v in (x, y))
    g2 = 1.0 / (gamma * gamma)
    out = np.zeros_like(x)
    for k in range(int(round(2.0 * vmax / step)) + 1):
        t = math.exp(-vmax + k * step)          # nodes formed directly: no drift of the spacing
        t2 = t * t
        f = step * t / (math.sqrt(t2 + 1.0) * math.sqrt(t2 + g2))
        out += f * np.exp(-x * x / (sigma * sigma * (t2 + 1.0)) - y * y / (sigma * sigma * (t2 + g2)))
    return out * sigma / (gamma * math.sqrt(math.pi))


def coulomb2d_anisotropic_mp(x: float, y: float, sigma: float, gamma: float) -> float:
    """Same integral at one point by mpmath quadrature (reference for the above)."""
    with mp.workdps(30):
        g2 = mp.mpf(1) / mp.mpf(gamma) ** 2
        s2 = mp.mpf(sigma) ** 2
        f = lambda t: mp.exp(-x * x / (s2 * (t * t + 1)) - y * y / (s2 * (t * t + g2))) / (
            mp.sqrt(t * t + 1) * mp.sqrt(t * t + g2))
        return float(mp.mpf(sigma) / (mp.mpf(gamma) * mp.sqrt(mp.pi)) * mp.quad(f, [0, 1, 10, mp.inf]))


def power_gaussian(r, beta: float, sigma: float, d: int, step: float = 0.05, vmax: float = 90.0):
    """Potential of exp(-|x|^2/sigma^2) under the kernel |x|^-beta (0 < beta < d) at
    distances r: with r^-beta = (2/Gamma(beta/2)) int tau^(beta-1) e^(-r^2 tau^2) dtau and the
    Gaussian convolution, u(r) = (2/Gamma(beta/2)) int_0^inf tau^(beta-1) (pi/(a+tau^2))^(d/2)
    exp(-a tau^2 r^2/(a+tau^2)) dtau, a = 1/sigma^2.  With tau = exp(v) the integrand decays
    exponentially at both ends (rates beta and d-beta) and is analytic in |Im v| < pi/2:
    trapezoidal rule in v."""
    r = np.asarray(r, dtype=np.float64)
    a = 1.0 / (sigma * sigma)
    out = np.zeros_like(r)
    r2 = r * r
    for k in range(int(round(2.0 * vmax / step)) + 1):
        v = -vmax + k * step
        t2 = math.exp(2.0 * v)
        f = step * math.exp(beta * v) * (math.pi / (a + t2)) ** (d / 2.0)
        if f == 0.0:
            continue
        out += f * np.exp(-a * t2 * r2 / (a + t2))
    return out * 2.0 / math.gamma(beta / 2.0)


def power_gaussian_mp(r: float, beta: float, sigma: float, d: int) -> float:
    """Same integral at one distance by mpmath quadrature (reference for the above)."""
    with mp.workdps(30):
        a = 1 / mp.mpf(sigma) ** 2
        f = lambda t: t ** (beta - 1) * (mp.pi / (a + t * t)) ** (mp.mpf(d) / 2) * mp.e ** (-a * t * t * r * r / (a + t * t))
        return float(2 / mp.gamma(mp.mpf(beta) / 2) * mp.quad(f, [0, 1, 10, mp.inf]))


def power_gaussian_origin(beta: float, sigma: float, d: int) -> float:
    """u(0) = |S^(d-1)| int_0^inf r^(d-1-beta) e^(-r^2/sigma^2) dr
            = pi^(d/2) sigma^(d-beta) Gamma((d-beta)/2) / Gamma(d/2)."""
    return math.pi ** (d / 2.0) * sigma ** (d - beta) * math.gamma((d - beta) / 2.0) / math.gamma(d / 2.0)


def davey_stewartson_gaussian(x, y):
    """Davey-Stewartson potential (-ln|x|/(2 pi)) * d_xx rho of rho = pi exp(-pi^2 (x^2+y^2))
    (Example 4.5): -(pi/2) e^{-a} - cos(2 theta) e^{-a} (1 + a - e^a)/(2 pi r^2), a = pi^2 r^2,
    with cos(2 theta) = (x^2 - y^2)/r^2.  Near r = 0, (1 + a - e^a)/r^2 is summed as a series
    (-pi^2 a (1/2 + a/6 + a^2/24 + ...))."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    r2 = x * x + y * y
    a = math.pi ** 2 * r2
    small = a < 0.5
    eq = np.empty_like(a)                              # e^{-a} (1 + a - e^a) / r^2
    big = ~small
    eq[big] = ((1.0 + a[big]) * np.exp(-a[big]) - 1.0) / r2[big]
    asm = a[small]
    ser = np.zeros_like(asm)
    term = np.full_like(asm, 0.5)                      # a^k / (k+2)!
    for k in range(1, 30):
        ser += term
        term = term * asm / (k + 2)
    eq[small] = -math.pi ** 2 * asm * ser * np.exp(-asm)
    with np.errstate(invalid="ignore", divide="ignore"):
        c2t = np.where(r2 > 0, (x * x - y * y) / np.where(r2 > 0, r2, 1.0), 0.0)
    return -(0.5 * math.pi * np.exp(-a) + c2t * eq / (2.0 * math.pi))


def poisson2d_gaussian(r, sigma: float = 1.0):
    r = np.asarray(r, dtype=np.float64)
    out = np.empty_like(r)
    xx = r * r / (sigma * sigma)
    small = xx < 0.5
    big = ~small
    out[big] = -(sigma ** 2 / 4.0) * (special.exp1(xx[big]) + 2.0 * np.log(r[big]))
    # E1(x) + ln x = -gamma_e - sum_{k>=1} (-x)^k / (k k!)
    xs = xx[small]
    ser = np.zeros_like(xs)
    term = np.ones_like(xs)
    for k in range(1, 40):
        term = term * (-xs) / k
        ser += term / k
    # E1(x) + 2 ln r = E1(x) + ln x + ln sigma^2
    out[small] = -(sigma ** 2 / 4.0) * (-EULER_GAMMA - ser + math.log(sigma * sigma))
    return out


def dipolar3d_gaussian(x, y, z, nvec, mvec, sigma: float = 1.0):
    """-(n.m) rho - 3 n^T D m for rho = exp(-r^2/sigma^2), D = Hessian of the
    Coulomb potential phi(r) = sigma^3 sqrt(pi) erf(r/sigma)/(4r)."""
    x, y, z = (np.asarray(v, dtype=np.float64) for v in (x, y, z))
    x, y, z = np.broadcast_arrays(x, y, z)
    r2 = x * x + y * y + z * z
    r = np.sqrt(r2)
    s2 = sigma * sigma
    rho = np.exp(-r2 / s2)
    f1 = np.empty_like(r)        # phi'(r)/r
    f2 = np.empty_like(r)        # (phi'' - phi'/r)/r^2
    small = r < 0.3 * sigma
    big = ~small
    rb = r[big]
    eb = np.exp(-rb * rb / s2)
    erfb = special.erf(rb / sigma)
    f1[big] = s2 / (2.0 * rb ** 2) * eb - sigma ** 3 * math.sqrt(math.pi) / (4.0 * rb ** 3) * erfb
    f2[big] = (-3.0 * s2 / (2.0 * rb ** 4) * eb - eb / rb ** 2
               + 3.0 * sigma ** 3 * math.sqrt(math.pi) / (4.0 * rb ** 5) * erfb)
    # phi = sum_k c_k r^{2k}, c_k = (sigma^2/2)(-1)^k sigma^{-2k} / (k! (2k+1))
    rs2 = r2[small]
    a1 = np.zeros_like(rs2)
    a2 = np.zeros_like(rs2)
    for k in range(1, 30):
        ck = (s2 / 2.0) * (-1.0) ** k / (s2 ** k * math.factorial(k) * (2 * k + 1))
        a1 += 2 * k * ck * rs2 ** (k - 1)
        if k >= 2:
            a2 += 2 * k * (2 * k - 2) * ck * rs2 ** (k - 2)
    f1[small] = a1
    f2[small] = a2
    nx, ny, nz = nvec
    mx, my, mz = mvec
    nm = nx * mx + ny * my + nz * mz
    nx_ = nx * x + ny * y + nz * z
    mx_ = mx * x + my * y + mz * z
    nDm = nm * f1 + nx_ * mx_ * f2
    return -nm * rho - 3.0 * nDm


def factor_mp(tau: float, c: float, k: int, dps: int = 40, p: int = 2) -> float:
    """int_{-c}^{c} exp(-tau^2 y^2) cos(xi y) dy, xi = 2 pi k / (p c), in closed form (mpmath)."""
    with mp.workdps(dps):
        c_ = mp.mpf(c)
        xi = 2 * mp.pi * k / (p * c_)
        if tau == 0.0:
            return float(2 * c_) if k == 0 else float(2 * mp.sin(xi * c_) / xi)
        t = mp.mpf(tau)
        z = mp.mpc(t * c_, xi / (2 * t))
        return float(mp.sqrt(mp.pi) / t * mp.exp(-xi * xi / (4 * t * t)) * mp.re(mp.erf(z)))


def mixture_energy_coulomb3d(a, mu, sigma) -> float:
    """1/2 sum_{c,c'} a_c a_c' pi^3 s_c^3 s_c'^3 erf(R/s)/(4 pi R), s^2 = s_c^2 + s_c'^2."""
    a = np.asarray(a, float)
    mu = np.asarray(mu, float)
    sg = np.asarray(sigma, float)
    E = 0.0
    for i in range(len(a)):
        for j in range(len(a)):
            s = math.sqrt(sg[i] ** 2 + sg[j] ** 2)
            R = float(np.linalg.norm(mu[i] - mu[j]))
            k = (1.0 / (2.0 * math.pi ** 1.5 * s)) if R < 1e-12 else math.erf(R / s) / (4.0 * math.pi * R)
            E += a[i] * a[j] * math.pi ** 3 * sg[i] ** 3 * sg[j] ** 3 * k
    return 0.5 * E


def mixture_potential_coulomb3d(points, a, mu, sigma):
    """sum_c a_c sigma_c^3 sqrt(pi) erf(|x - mu_c|/sigma_c)/(4 |x - mu_c|)."""
    x, y, z = points
    out = 0.0
    for c in range(len(a)):
        r = np.sqrt((x - mu[c][0]) ** 2 + (y - mu[c][1]) ** 2 + (z - mu[c][2]) ** 2)
        out = out + a[c] * coulomb3d_gaussian(r, sigma[c])
    return out
