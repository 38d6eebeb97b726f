"""Coefficients of the degree-10 polynomial used for 2^f, |f| <= 1/2.

Minimax fit of the relative error of 2^f on [-1/2, 1/2] by the Remez exchange
algorithm, in 40-digit arithmetic (mpmath).  The approximation error is about
2.1e-16 (2.8e-16 with the coefficients rounded to double), the size of one
rounding of the result, so degree 10 is the lowest degree that adds no error
beyond the ~2 ulp of evaluating the polynomial in double by Horner's rule.
Coefficients are printed lowest degree first, rounded to the nearest double;
the output is pasted into common.h (highest degree first).

    python gen_exp2_coeffs.py
"""
import mpmath as mp

mp.mp.dps = 40
DEG = 10


def rel_err(c, x):
    return (mp.polyval(c[::-1], x) - mp.power(2, x)) / mp.power(2, x)


def remez(deg, iters=15, grid_n=4000):
    n = deg + 2
    xs = [mp.mpf(1) / 2 * mp.cos(mp.pi * k / (n - 1)) for k in range(n)]
    grid = [mp.mpf(-0.5) + mp.mpf(k) / grid_n for k in range(grid_n + 1)]
    for _ in range(iters):
        A = mp.matrix(n, n)
        b = mp.matrix(n, 1)
        for i, x in enumerate(xs):
            w = mp.power(2, x)
            for j in range(deg + 1):
                A[i, j] = x ** j
            A[i, deg + 1] = (-1) ** i * w
            b[i] = w
        sol = mp.lu_solve(A, b)
        c = [sol[j] for j in range(deg + 1)]
        vals = [rel_err(c, x) for x in grid]
        ext = [0] + [k for k in range(1, grid_n) if (vals[k] - vals[k - 1]) * (vals[k + 1] - vals[k]) <= 0] + [grid_n]
        if len(ext) > n:
            ext = sorted(sorted(ext, key=lambda k: -abs(vals[k]))[:n])
        if len(ext) < n:
            break
        xs = [grid[k] for k in ext]
    return c, max(abs(v) for v in vals)


if __name__ == "__main__":
    c, err = remez(DEG)
    for k, ck in enumerate(c):
        print("    %r, // f^%d" % (float(ck), k))
    print("max relative approximation error: %s" % mp.nstr(err, 3))
