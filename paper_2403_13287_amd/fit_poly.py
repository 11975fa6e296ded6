"""Coefficients of the flux kernel's erf and exp (lskum_math.h: lk_erf,
lk_exp), fitted in 50-digit arithmetic (mpmath) by least squares on
Chebyshev nodes, weighted relatively.

erf: erf(x)/x is even and analytic; on [0, 1] it is approximated by a
polynomial P(t) of degree 11 in t = x^2 (4 x 12 nodes in t).

exp: after the reduction x = k ln 2 + r, |r| <= ln(2)/2, e^r = 1 + r +
r^2 Q(r) with Q of degree 9 (coefficients of r^2 .. r^11; 6 x 11 nodes).

The kernel adds the rounding of its FMA steps (a few ulp).

    python -m paper_2403_13287_amd.fit_poly
"""
import mpmath as mp


def _lsq(rows, rhs):
    A = mp.matrix(len(rows), len(rows[0]))
    b = mp.matrix(len(rows), 1)
    for i, (r, v) in enumerate(zip(rows, rhs)):
        for j, a in enumerate(r):
            A[i, j] = a
        b[i] = v
    return mp.lu_solve(A.T * A, A.T * b)


def fit_erf(degree: int = 11, x_max: float = 1.0):
    """erf(x)/x ~ sum_j c_j x^(2j), j = 0..degree, on |x| <= x_max."""
    mp.mp.dps = 50
    T = mp.mpf(x_max) ** 2

    def f(t):
        return mp.erf(mp.sqrt(t)) / mp.sqrt(t) if t > 0 else 2 / mp.sqrt(mp.pi)

    m = 4 * (degree + 1)
    nodes = [T * (1 - mp.cos(mp.pi * (k + mp.mpf(1) / 2) / m)) / 2 for k in range(m)]
    c = _lsq([[t ** j / f(t) for j in range(degree + 1)] for t in nodes], [1] * m)
    grid = [(x_max * k / 2000) ** 2 for k in range(2001)]
    err = max(abs(sum(c[j] * t ** j for j in range(degree + 1)) / f(t) - 1) for t in grid)
    return [c[j] for j in range(degree + 1)], err


def fit_exp(degree: int = 11):
    """e^r ~ 1 + r + sum_{j=2..degree} c_j r^j on |r| <= ln(2)/2."""
    mp.mp.dps = 50
    h = mp.log(2) / 2
    m = 6 * degree
    nodes = [h * mp.cos(mp.pi * (k + mp.mpf(1) / 2) / m) for k in range(m)]
    c = _lsq([[r ** j / mp.exp(r) for j in range(2, degree + 1)] for r in nodes],
             [(mp.exp(r) - 1 - r) / mp.exp(r) for r in nodes])
    grid = [h * (2 * k / 2000 - 1) for k in range(2001)]
    err = max(abs((1 + r + sum(c[j - 2] * r ** j for j in range(2, degree + 1))) / mp.exp(r) - 1)
              for r in grid)
    return [c[j] for j in range(degree - 1)], err


if __name__ == "__main__":
    coeffs, err = fit_erf()
    print(f"erf(x)/x, |x| < 1: max relative fit error {mp.nstr(err, 3)}")
    for j, cj in enumerate(coeffs):
        print(f"  t^{j}: {mp.nstr(cj, 20)}")
    coeffs, err = fit_exp()
    print(f"e^r, |r| <= ln(2)/2: max relative fit error {mp.nstr(err, 3)}")
    for j, cj in enumerate(coeffs):
        print(f"  r^{j + 2}: {mp.nstr(cj, 20)}")
