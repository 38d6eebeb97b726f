"""Print the coefficients of the degree-13 polynomial used for 2^f, |f| <= 1/2.

2^f = e^(f ln 2) = sum_k (ln 2)^k / k! f^k (Taylor series).  The first term
dropped, (ln 2)^14/14! * 2^-14 ~ 4e-18, is below half an ulp of 2^f >= 0.707,
so rounding each coefficient to the nearest double is enough.  Run with mpmath
available; the output is pasted into kernels.hip.
"""
import mpmath as mp

mp.mp.dps = 50
ln2 = mp.log(2)
for k in range(14):
    c = ln2 ** k / mp.factorial(k)
    print("    %r, // (ln 2)^%d / %d!" % (float(c), k, k))
print("drop term bound:", mp.nstr(ln2 ** 14 / mp.factorial(14) * mp.mpf(2) ** -14, 3))
