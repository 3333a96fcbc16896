"""Derive the SSPRK(5,3) Shu-Osher coefficients the oracle uses (TEST INFRASTRUCTURE).

The paper takes the five-stage, third-order SSP Runge-Kutta scheme from a table
that is not reproduced in it.  This script starts from the published 14-digit
coefficients of the optimal SSP(5,3) scheme (SSP coefficient about 2.65), keeps
their sparsity and the alpha entries (row sums made exactly one), and applies
minimal-norm Newton corrections to the nonzero beta entries until the four
third-order conditions  sum b = 1, sum b c = 1/2, sum b c^2 = 1/3,
sum b A c = 1/6  hold to 40 digits.  The corrections are below 4e-10, i.e. the
scheme is the published one, made exactly third order in double precision.

Run:  python oracle/ssprk53_coefficients.py   (prints the table)
"""
import mpmath as mp

mp.mp.dps = 40

ALPHA = {(1, 0): "1", (2, 1): "1", (3, 0): "0.56656131914033", (3, 2): "0.43343868085967",
         (4, 0): "0.09299483444413", (4, 1): "0.00002090369620", (4, 3): "0.90698426185967",
         (5, 0): "0.00736132260920", (5, 1): "0.20127980325145", (5, 2): "0.00182955389682",
         (5, 4): "0.78952932024253"}
BETA = {(1, 0): "0.37726891511710", (2, 1): "0.37726891511710", (3, 2): "0.16352294089771",
        (4, 0): "0.00071997378654", (4, 3): "0.34217696850008", (5, 0): "0.00277719819460",
        (5, 1): "0.00001567934613", (5, 4): "0.29786487010104"}


def butcher(a, b):
    A = [[mp.mpf(0)] * 5 for _ in range(6)]
    for i in range(1, 6):
        for k in range(i):
            for j in range(5):
                A[i][j] += a.get((i, k), 0) * A[k][j]
            A[i][k] += b.get((i, k), 0)
    return A


def residuals(a, b):
    A = butcher(a, b)
    bb, c = A[5], [sum(A[i][:5]) for i in range(5)]
    Ac = [sum(A[i][j] * c[j] for j in range(5)) for i in range(5)]
    return [sum(bb) - 1, sum(bb[i] * c[i] for i in range(5)) - mp.mpf(1) / 2,
            sum(bb[i] * c[i] ** 2 for i in range(5)) - mp.mpf(1) / 3,
            sum(bb[i] * Ac[i] for i in range(5)) - mp.mpf(1) / 6]


def derive():
    a = {k: mp.mpf(v) for k, v in ALPHA.items()}
    b = {k: mp.mpf(v) for k, v in BETA.items()}
    for i in range(1, 6):  # alpha row sums exactly 1 (adjust the largest entry)
        ks = [k for k in a if k[0] == i]
        big = max(ks, key=lambda k: a[k])
        a[big] = 1 - sum(a[k] for k in ks if k != big)
    keys = sorted(b)
    for _ in range(6):
        r = residuals(a, b)
        J = mp.matrix(4, len(keys))
        h = mp.mpf("1e-25")
        for j, k in enumerate(keys):
            b2 = dict(b)
            b2[k] += h
            r2 = residuals(a, b2)
            for i in range(4):
                J[i, j] = (r2[i] - r[i]) / h
        d = J.T * mp.lu_solve(J * J.T, -mp.matrix(r))
        for j, k in enumerate(keys):
            b[k] += d[j]
    return a, b


if __name__ == "__main__":
    a, b = derive()
    print("order-condition residuals:", [mp.nstr(x, 3) for x in residuals(a, b)])
    print("SSP coefficient:", mp.nstr(min(a[k] / b[k] for k in b if k in a), 12))
    for k in sorted(a):
        print("alpha", k, mp.nstr(a[k], 20))
    for k in sorted(b):
        print("beta ", k, mp.nstr(b[k], 20))
