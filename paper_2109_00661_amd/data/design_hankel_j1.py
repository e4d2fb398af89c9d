"""Offline design of the 120-point J1 Hankel digital filter used by the forward model.

The forward model evaluates the secondary field of a central loop with a digital
filter for the Hankel transform of order 1 (the paper computes the response with
a Hankel transform, Section 2, without naming a filter).  No published coefficient
table is used: the table is designed here by linear least squares.

A J1 filter approximates

    F(r) = int_0^inf f(lam) J1(lam r) dlam  ~  (1/r) sum_k w_k f(b_k / r),
    b_k = exp(X0 + k*DX),  k = 0..119.

The weights w_k minimise the relative error over transform pairs with closed forms:

    f = lam exp(-p lam)            F = r / (p^2+r^2)^(3/2)
    f = exp(-p lam)                F = (sqrt(p^2+r^2) - p) / (r sqrt(p^2+r^2))
    f = exp(-p lam) / lam          F = (sqrt(p^2+r^2) - p) / r
    f = lam^2 exp(-lam^2)          F = (r/4) exp(-r^2/4)
    f = lam^2 exp(-z u) / u,  u = sqrt(lam^2+q^2), q complex with arg(q) = pi/4
                                   F = r (1 + q R) exp(-q R) / R^3,  R = sqrt(r^2+z^2)

The last pair (the r-derivative of the Sommerfeld identity) carries a second,
complex length scale like the quasi-static wavenumber of a conducting ground, so the
filter resolves the low-induction-number regime where the kernel stays flat down to
lam ~ |k|.  The design targets kernels that carry an exponential height factor with
p/r >= 1 (height/radius >= 1/2); the 30 m / 12.5 m central-loop geometry has 4.8.

Run:  python design_hankel_j1.py  -> writes hankel_j1_120.txt (b_k, w_k; 17 digits).
"""
import os
import numpy as np

N = 120
DX = 0.11
X0 = -10.1
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hankel_j1_120.txt")


def design_rows(b, per_decade=100):
    """Rows of the relative-error least-squares system.  The sampling in r is dense
    (per_decade points per decade, several per filter spacing) so the error is
    controlled between samples and not only at them."""
    rows, rhs = [], []
    for r in np.logspace(-5, 0, 5 * per_decade):           # p = 1, so p/r in [1, 1e5]
        for f, F in ((lambda l: l * np.exp(-l), lambda r: r / (1 + r * r) ** 1.5),
                     (lambda l: np.exp(-l), lambda r: (np.sqrt(1 + r * r) - 1) / (r * np.sqrt(1 + r * r))),
                     (lambda l: np.exp(-l) / l, lambda r: (np.sqrt(1 + r * r) - 1) / r)):
            Fv = F(r)
            rows.append(f(b / r) / r / abs(Fv))
            rhs.append(np.sign(Fv))
    for r in np.logspace(-2, 0.3, int(2.3 * per_decade)):
        Fv = r / 4 * np.exp(-r * r / 4)
        rows.append((b / r) ** 2 * np.exp(-(b / r) ** 2) / r / Fv)
        rhs.append(1.0)
    phase = np.exp(1j * np.pi / 4)
    for z in np.logspace(0, 1, 11):
        for qm in np.logspace(-6, 1, 43):
            q = qm * phase
            u = np.sqrt(b * b + q * q)
            R = np.sqrt(1 + z * z)
            Fv = np.exp(-q * R) * (1 + q * R) / R ** 3
            g = b ** 2 * np.exp(-z * u) / u / abs(Fv)
            t = Fv / abs(Fv)
            rows.append(g.real); rhs.append(t.real)
            rows.append(g.imag); rhs.append(t.imag)
    return np.array(rows), np.array(rhs)


def main():
    b = np.exp(X0 + DX * np.arange(N))
    A, y = design_rows(b)
    w, *_ = np.linalg.lstsq(A, y, rcond=1e-15)
    err = np.abs(A @ w - y).max()
    with open(OUT, "w") as fh:
        fh.write("# 120-point J1 Hankel filter designed by design_hankel_j1.py\n")
        fh.write("# int_0^inf f(lam) J1(lam r) dlam ~ (1/r) sum_k w_k f(b_k/r); b_k = exp(%.17g + %.17g k)\n" % (X0, DX))
        fh.write("# max relative design residual over the closed-form pairs: %.3e\n" % err)
        fh.write("# columns: b_k w_k\n")
        for bk, wk in zip(b, w):
            fh.write("%.17e %.17e\n" % (bk, wk))
    print("wrote %s; max design residual %.3e; max |w| %.3f" % (OUT, err, np.abs(w).max()))


if __name__ == "__main__":
    main()
