"""Coefficients of the flux kernel's erf for |x| < 1 (lskum_math.h, lk_erf).

erf(x)/x is an even analytic function; on [0, 1] it is approximated by a
polynomial P(t) of degree 11 in t = x^2, fitted by least squares on 4 x 12
Chebyshev nodes in t, in 50-digit arithmetic (mpmath), weighted relatively.
The fit's relative error on a 2001-point grid is printed; the kernel then
adds the rounding of 11 FMA steps and one product (a few ulp).

    python -m paper_2403_13287_amd.fit_erf
"""
import mpmath as mp

DEGREE = 11


def fit(degree: int = DEGREE, x_max: float = 1.0):
    mp.mp.dps = 50
    T = mp.mpf(x_max) ** 2

    def f(t):
        return mp.erf(mp.sqrt(t)) / mp.sqrt(t) if t > 0 else 2 / mp.sqrt(mp.pi)

    m = 4 * (degree + 1)
    nodes = [T * (1 - mp.cos(mp.pi * (k + mp.mpf(1) / 2) / m)) / 2 for k in range(m)]
    A = mp.matrix(m, degree + 1)
    b = mp.matrix(m, 1)
    for i, t in enumerate(nodes):
        w = 1 / f(t)
        for j in range(degree + 1):
            A[i, j] = w * t ** j
        b[i] = 1
    c = mp.lu_solve(A.T * A, A.T * b)
    err = max(abs(sum(c[j] * (x_max * k / 2000) ** (2 * j) for j in range(degree + 1))
                  / f((x_max * k / 2000) ** 2) - 1) for k in range(2001))
    return [c[j] for j in range(degree + 1)], err


if __name__ == "__main__":
    coeffs, err = fit()
    print(f"max relative fit error {mp.nstr(err, 3)}")
    for j, cj in enumerate(coeffs):
        print(f"t^{j}: {mp.nstr(cj, 20)}")
