"""Coefficients of the FP64 exp2 polynomial of dev_math.h.

2^f on [-1/2, 1/2] by Chebyshev economization of its Taylor series: the series
of e^(f ln 2) to degree 24 (truncation below 1e-30) is rewritten in Chebyshev
polynomials of x = 2f, the terms of degree 12 and above are dropped (each is
bounded by the absolute value of its coefficient, |T_n| <= 1 on [-1, 1]), and the
rest converted back to powers of f.  Exact rational arithmetic throughout
except ln 2, taken to 60 digits.  Prints the degree-11 coefficients rounded to
FP64 and the bound on the dropped terms."""
from decimal import Decimal, getcontext
from fractions import Fraction

getcontext().prec = 80
LN2 = Fraction(Decimal(2).ln())
DEG_SERIES, DEG = 24, 11


def cheb_monomials(n):
    """T_n(x) as a list of monomial coefficients."""
    t0, t1 = [Fraction(1)], [Fraction(0), Fraction(1)]
    if n == 0:
        return t0
    for _ in range(n - 1):
        t2 = [Fraction(0)] + [2 * c for c in t1]
        for i, c in enumerate(t0):
            t2[i] -= c
        t0, t1 = t1, t2
    return t1


def main():
    # p(f) = sum a_k f^k = sum a_k 2^-k x^k, x = 2f
    fact = Fraction(1)
    a = []
    for k in range(DEG_SERIES + 1):
        if k:
            fact *= k
        a.append(LN2 ** k / fact)
    bx = [a[k] / Fraction(2) ** k for k in range(DEG_SERIES + 1)]   # coefficients in x
    # monomials -> Chebyshev, highest degree first
    cheb = [Fraction(0)] * (DEG_SERIES + 1)
    rest = bx[:]
    for n in range(DEG_SERIES, -1, -1):
        tn = cheb_monomials(n)
        c = rest[n] / tn[n]
        cheb[n] = c
        for i, t in enumerate(tn):
            rest[i] -= c * t
    dropped = sum(abs(c) for c in cheb[DEG + 1:])
    # back to monomials in x up to DEG, then in f
    mono = [Fraction(0)] * (DEG + 1)
    for n in range(DEG + 1):
        for i, t in enumerate(cheb_monomials(n)):
            mono[i] += cheb[n] * t
    coef = [mono[k] * Fraction(2) ** k for k in range(DEG + 1)]
    for k, c in enumerate(coef):
        print(f"    {float(c).hex()},  // c{k}")
    print(f"// dropped terms bound {float(dropped):.3e}")


if __name__ == "__main__":
    main()
