"""Oracle: FP64 central-loop time-domain EM forward model and Gaussian log-likelihood.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

A plain, slow, CPU implementation written from the paper and from textbook
quasi-static EM.  It shares no code with the HIP path.  Each function names the
passage it follows.  Readings where the paper is silent (the forward model is only
cited, Section 2) are:

* time dependence exp(+i w t); quasi-static, so the air wavenumber is lam;
  mu0 = 4 pi 1e-7 H/m exactly;
* data are -dBz/dt in pT/s at the loop centre for a 1 A step-off current
  (Section 2.3.2: conductive-only data are usually positive);
* a layer property applies below its interface (change-point convention of
  Appendix E.1); the background conductivity is the top segment and the
  background chargeability is zero (Section 2.3.1);
* the frequency-to-time map is the cosine transform of Im(H)/w, spline-interpolated
  in ln w and extended as a constant beyond both ends, averaged over boxcar gates.

Particles are dicts of SoA numpy arrays as produced by the seeded input module.
"""
import numpy as np
from scipy.integrate import quad
from scipy.interpolate import CubicSpline

MU0 = 4.0e-7 * np.pi
LN10 = np.log(10.0)


# --------------------------------------------------------------------------------------
# Minimal forward-mode dual numbers (value + tangents along a trailing axis).  Used only
# for the oracle gradient, which is deliberately a different method from the reverse
# sweep of the HIP path.
# --------------------------------------------------------------------------------------
class Dual:
    __array_ufunc__ = None          # make numpy defer to the reflected operators

    def __init__(self, val, der):
        self.val = np.asarray(val)
        self.der = np.asarray(der)

    @staticmethod
    def lift(x, ndir):
        if isinstance(x, Dual):
            return x
        x = np.asarray(x)
        return Dual(x, np.zeros(x.shape + (ndir,), dtype=x.dtype))

    def _nd(self):
        return self.der.shape[-1]

    def __add__(self, o):
        o = Dual.lift(o, self._nd())
        return Dual(self.val + o.val, self.der + o.der)

    __radd__ = __add__

    def __neg__(self):
        return Dual(-self.val, -self.der)

    def __sub__(self, o):
        return self + (-Dual.lift(o, self._nd()))

    def __rsub__(self, o):
        return Dual.lift(o, self._nd()) - self

    def __mul__(self, o):
        o = Dual.lift(o, self._nd())
        return Dual(self.val * o.val, self.der * o.val[..., None] + o.der * self.val[..., None])

    __rmul__ = __mul__

    def __truediv__(self, o):
        o = Dual.lift(o, self._nd())
        q = self.val / o.val
        return Dual(q, (self.der - q[..., None] * o.der) / o.val[..., None])

    def __rtruediv__(self, o):
        return Dual.lift(o, self._nd()) / self

    def __getitem__(self, idx):
        if not isinstance(idx, tuple):
            idx = (idx,)
        return Dual(self.val[idx], self.der[idx + (slice(None),)])

    @property
    def real(self):
        return Dual(self.val.real, self.der.real)

    @property
    def imag(self):
        return Dual(self.val.imag, self.der.imag)


def _sqrt(x):
    if isinstance(x, Dual):
        v = np.sqrt(x.val)
        return Dual(v, x.der / (2.0 * v)[..., None])
    return np.sqrt(x)


def _exp(x):
    if isinstance(x, Dual):
        v = np.exp(x.val)
        return Dual(v, x.der * v[..., None])
    return np.exp(x)


def _log(x):
    if isinstance(x, Dual):
        return Dual(np.log(x.val), x.der / x.val[..., None])
    return np.log(x)


def _sum(x, axis):
    if isinstance(x, Dual):
        return Dual(x.val.sum(axis=axis), x.der.sum(axis=axis if axis >= 0 else axis - 1))
    return np.sum(x, axis=axis)


def _matvec(K, x):
    """K @ x for x of shape [n] (or a Dual of it)."""
    if isinstance(x, Dual):
        return Dual(K @ x.val, K @ x.der)
    return K @ x


# --------------------------------------------------------------------------------------
# Model parameters of one particle (Section 2.3.1 parameter vector; Fig. 2 direct sum).
# --------------------------------------------------------------------------------------
def particle_params(p, i):
    """Ordered list of (name, row) for the continuous parameters of particle i, in the
    order of the paper's parameter vector: background log10 sigma, layer log10 sigma,
    conductivity depths, chargeabilities, chargeability depths, tau, c."""
    k = int(p["kappa"][i])
    names = [("phi_b", None)] + [("phi", r) for r in range(k)] + [("z_cond", r) for r in range(k)]
    if p["layout"] == 1:
        names += [("m", r) for r in range(k + 1)]
    else:
        lam = int(p["lambda_"][i])
        names += [("m", r) for r in range(lam)] + [("z_charg", r) for r in range(lam)]
    names += [("log10_tau", None), ("c", None)]
    return names


def _value(p, name, row, i):
    return p[name][i] if row is None else p[name][row, i]


def merged_stack(p, i, theta=None):
    """Merged layer stack of particle i (Section 2.1, Fig. 2: the two change-point
    profiles are merged by a direct sum).

    Returns (sigma_inf[L], m[L], thickness[L-1]) as lists of scalars (or Duals when
    theta maps parameter names to Duals).  Layer l spans [Z_l, Z_{l+1}) with Z_0 = 0 and
    Z_1.. the sorted union of both interface sets; a property applies below its
    interface, so a layer takes the segment whose interfaces lie at or above its top.
    The last layer is the infinite basement."""
    def val(name, row):
        if theta is not None:
            return theta[(name, row)]
        return _value(p, name, row, i)

    k = int(p["kappa"][i])
    zc = [(float(_value(p, "z_cond", r, i)), val("z_cond", r)) for r in range(k)]
    if p["layout"] == 1:
        zs = zc
        tops = [(0.0, 0.0)] + zs
        L = k + 1
        phis = [val("phi_b", None)] + [val("phi", r) for r in range(k)]
        ms = [val("m", r) for r in range(L)]
        sig = [_exp(LN10 * ph) for ph in phis]
        thick = [tops[l + 1][1] - tops[l][1] for l in range(L - 1)]
        return sig, ms, thick
    lam = int(p["lambda_"][i])
    zm = [(float(_value(p, "z_charg", r, i)), val("z_charg", r)) for r in range(lam)]
    merged = sorted(zc + zm, key=lambda t: t[0])
    tops = [(0.0, 0.0)] + merged
    L = len(tops)
    zc_vals = [t[0] for t in zc]
    zm_vals = [t[0] for t in zm]
    sig, ms = [], []
    for l in range(L):
        top = tops[l][0]
        ic = sum(1 for z in zc_vals if z <= top)        # conductivity segment index
        im = sum(1 for z in zm_vals if z <= top)        # chargeability segment index
        ph = val("phi_b", None) if ic == 0 else val("phi", ic - 1)
        sig.append(_exp(LN10 * ph))
        ms.append(0.0 if im == 0 else val("m", im - 1))
    thick = [tops[l + 1][1] - tops[l][1] for l in range(L - 1)]
    return sig, ms, thick


# --------------------------------------------------------------------------------------
# Physics (Section 2: Cole-Cole; Ward & Hohmann layered-earth TE reflection, Hankel).
# --------------------------------------------------------------------------------------
def cole_cole(sigma_inf, m, tau, c, omega):
    """Complex conductivity of Section 2: sigma_inf * (1 - m / (1 + (i w tau)^c)),
    principal branch of the power."""
    z = _exp(c * _log(1j * omega * tau))
    return sigma_inf * (1.0 - m / (1.0 + z))


def reflection_te(lam, k2, thick):
    """TE reflection coefficient at the surface of a layered half-space for the
    quasi-static wavenumbers k2[l] = i w mu0 sigma_hat_l (each broadcastable against
    lam) and layer thicknesses thick[l], l = 0..L-2 (the last layer is the basement).

    u_l = sqrt(lam^2 + k2_l) with Re u > 0.  Interface terms
        R_{l,l+1} = (k2_l - k2_{l+1}) / (u_l + u_{l+1})^2   (= (u_l-u_{l+1})/(u_l+u_{l+1}))
        R_air     = -k2_0 / (lam + u_0)^2                    (= (lam-u_0)/(lam+u_0))
    and the bottom-up recursion r_l = (R + r_{l+1} E_{l+1}) / (1 + R r_{l+1} E_{l+1}),
    E_l = exp(-2 u_l h_l), finishing with the air interface."""
    L = len(k2)
    u = [_sqrt(lam * lam + k2[l]) for l in range(L)]
    r = None
    for l in range(L - 2, -1, -1):
        R = (k2[l] - k2[l + 1]) / ((u[l] + u[l + 1]) * (u[l] + u[l + 1]))
        if r is None:
            r = R
        else:
            re = r * _exp(-2.0 * u[l + 1] * thick[l + 1])
            r = (R + re) / (1.0 + R * re)
    R0 = -k2[0] / ((lam + u[0]) * (lam + u[0]))
    if r is None:
        return R0
    re = r * _exp(-2.0 * u[0] * thick[0])
    return (R0 + re) / (1.0 + R0 * re)


def secondary_hz(system, sig, ms, thick, tau, c):
    """Secondary vertical field H_z^s(w) [A/m] at the centre of a horizontal loop of
    radius a at height h (receiver at the transmitter), for every system frequency:

        H_z^s = (I a / 2) int_0^inf r_TE(lam) exp(-2 lam h) lam J1(lam a) dlam
              ~ (I / 2) sum_k w_k lam_k exp(-2 lam_k h) r_TE(lam_k),   lam_k = b_k / a,

    the J1 digital filter applied to the Hankel transform of Section 2."""
    a = system["loop_radius_m"]
    h = system["height_m"]
    I = system["current_a"]
    omega = 2.0 * np.pi * np.asarray(system["freq_hz"])[:, None]          # [nf, 1]
    lam = (np.asarray(system["hankel_b"]) / a)[None, :]                   # [1, nh]
    wts = np.asarray(system["hankel_w"])[None, :]
    k2 = [1j * omega * MU0 * cole_cole(sig[l], ms[l], tau, c, omega) for l in range(len(sig))]
    r = reflection_te(lam, k2, thick)
    return _sum(r * (0.5 * I * wts * lam * np.exp(-2.0 * lam * h)), axis=-1)


def cos_moments(freq_hz, times):
    """mom[m, p, i] = int_{w_m}^{w_{m+1}} (ln w - ln w_m)^p cos(w t_i) dw, p = 0..3,
    by QUADPACK's oscillatory (Clenshaw-Curtis moment) rule."""
    w = 2.0 * np.pi * np.asarray(freq_hz, dtype=np.float64)
    x = np.log(w)
    mom = np.zeros((len(w) - 1, 4, len(times)))
    for m in range(len(w) - 1):
        for pw in range(4):
            for it, t in enumerate(times):
                mom[m, pw, it] = quad(lambda om, xm=x[m], pw=pw: (np.log(om) - xm) ** pw,
                                      w[m], w[m + 1], weight="cos", wvar=t,
                                      epsabs=0.0, epsrel=1e-13, limit=1000)[0]
    return mom


def time_transform_matrix(freq_hz, gate_open_s, gate_close_s):
    """Matrix K [n_gate, n_freq] with y = K @ Im(H_z^s), y in pT/s (-dBz/dt averaged
    over each boxcar gate after a step-off).

    v_j = Im H(w_j) / w_j is interpolated by a natural cubic spline S in x = ln w.  The
    off-time field is B(t) = -(2/pi) mu0 int_0^inf (Im H / w) cos(w t) dw, with
        F(t) = int_{w_1}^{w_n} S(ln w) cos(w t) dw + v_1 sin(w_1 t)/t - v_n sin(w_n t)/t
    (constant Im H / w below w_1 and above w_n, the latter read distributionally), and
        y_g = -(2/pi) mu0 1e12 [F(t_open) - F(t_close)] / (t_close - t_open).
    Each spline piece is integrated against cos(w t) by QUADPACK's oscillatory rule."""
    w = 2.0 * np.pi * np.asarray(freq_hz, dtype=np.float64)
    x = np.log(w)
    n = len(w)
    times = np.concatenate([np.asarray(gate_open_s), np.asarray(gate_close_s)])
    mom = cos_moments(freq_hz, times)
    ng = len(gate_open_s)
    K = np.zeros((ng, n))
    for j in range(n):
        v = np.zeros(n)
        v[j] = 1.0 / w[j]
        S = CubicSpline(x, v, bc_type="natural")
        F = np.zeros(len(times))
        for m in range(n - 1):
            for k in range(4):                    # S.c[k, m] multiplies (x - x_m)^(3-k)
                F += S.c[k, m] * mom[m, 3 - k]
        F += v[0] * np.sin(w[0] * times) / times - v[-1] * np.sin(w[-1] * times) / times
        K[:, j] = -(2.0 / np.pi) * MU0 * 1e12 * (F[:ng] - F[ng:]) / (times[ng:] - times[:ng])
    return K


def gate_response(system, K, sig, ms, thick, tau, c):
    """Gate responses y [n_gate] in pT/s for one merged stack."""
    H = secondary_hz(system, sig, ms, thick, tau, c)
    return _matvec(K, H.imag)


def noise_variance(y, eps_an, eps_mn):
    """Diagonal of the noise covariance of Section 2.3.2: eps_AN^2 + (eps_MN y)^2,
    evaluated at the model response."""
    return np.asarray(eps_an) ** 2 + (eps_mn * y) * (eps_mn * y)


def loglik_from_response(y, d, eps_an, eps_mn):
    """Gaussian log-likelihood of Section 2.3.2 with the model-dependent diagonal
    covariance: -1/2 sum_g [(d_g - y_g)^2 / s_g^2 + ln(2 pi s_g^2)]."""
    s2 = noise_variance(y, eps_an, eps_mn)
    r = np.asarray(d) - y
    terms = r * r / s2 + _log(2.0 * np.pi * s2)
    return -0.5 * np.sum(terms, axis=-1)


# --------------------------------------------------------------------------------------
# Batch drivers.
# --------------------------------------------------------------------------------------
def make_K(system):
    return time_transform_matrix(system["freq_hz"], system["gate_open_s"], system["gate_close_s"])


def forward(p, system, K, idx=None):
    """Gate responses [n, n_gate] for the particles idx (default all)."""
    n = len(p["kappa"])
    idx = range(n) if idx is None else idx
    out = []
    for i in idx:
        sig, ms, thick = merged_stack(p, i)
        tau = 10.0 ** p["log10_tau"][i]
        out.append(gate_response(system, K, sig, ms, thick, tau, p["c"][i]))
    return np.array(out)


def loglik(p, system, K, d, idx=None):
    y = forward(p, system, K, idx)
    s2 = noise_variance(y, system["eps_an"][None, :], system["eps_mn"])
    r = np.asarray(d)[None, :] - y
    return -0.5 * np.sum(r * r / s2 + np.log(2.0 * np.pi * s2), axis=1)


def loglik_grad(p, system, K, d, idx=None):
    """(ll [n], grad dict) by forward-mode tangent propagation through the whole model:
    one tangent per continuous parameter of the particle.  The gradient dict has the
    particle's SoA shapes; slots outside a particle's counts are zero."""
    n = len(p["kappa"])
    idx = list(range(n)) if idx is None else list(idx)
    grad = {k: np.zeros_like(v, dtype=np.float64) for k, v in p.items()
            if k not in ("layout", "kappa", "lambda_")}
    grad = {k: v[..., idx] for k, v in grad.items()}
    lls = np.zeros(len(idx))
    for j, i in enumerate(idx):
        names = particle_params(p, i)
        D = len(names)
        theta = {}
        for q, (name, row) in enumerate(names):
            der = np.zeros(D)
            der[q] = 1.0
            theta[(name, row)] = Dual(np.float64(_value(p, name, row, i)), der)
        sig, ms, thick = merged_stack(p, i, theta)
        tau = _exp(LN10 * theta[("log10_tau", None)])
        y = gate_response(system, K, sig, ms, thick, tau, theta[("c", None)])
        s2 = Dual.lift(np.asarray(system["eps_an"]) ** 2, D) + (system["eps_mn"] * y) * (system["eps_mn"] * y)
        r = Dual.lift(np.asarray(d, dtype=np.float64), D) - y
        terms = r * r / s2 + _log(2.0 * np.pi * s2)
        ll = _sum(terms, axis=0) * (-0.5)
        lls[j] = ll.val
        for q, (name, row) in enumerate(names):
            if row is None:
                grad[name][j] = ll.der[q]
            else:
                grad[name][row, j] = ll.der[q]
    return lls, grad
