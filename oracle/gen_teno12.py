"""Coefficients of the maximum-order linear reconstruction on the twelve-point
stencil S6 (cells i-5 .. i+6) of TENO12-AA: TEST INFRASTRUCTURE of the oracle.

The paper's framework (Sec. 3.1) adds symmetric large stencils of growing
width; it prints optimised schemes for the 6-, 8- and 10-point stencils only
(Sec. 4.1) and not the optimisation parameters, so the twelve-point stencil
takes the scheme of maximum order: the unique reconstruction
fhat_{i+1/2} = sum_l c_l f_{i-5+l} that is exact, at the face x_{i+1/2}, for
the point value of every polynomial of degree <= 11 given by its cell averages.
Solved here in exact rational arithmetic (fractions, Gaussian elimination) and
rounded once to float64.  ``python gen_teno12.py`` prints the C++ table that
tenoaa_oracle.cpp holds; a test checks that the two agree.
"""
from fractions import Fraction

LO, R = -5, 12


def cell_average_of_power(k, centre):
    """Average of x^k over [centre - 1/2, centre + 1/2]."""
    a, b = Fraction(2 * centre - 1, 2), Fraction(2 * centre + 1, 2)
    return (b ** (k + 1) - a ** (k + 1)) / (k + 1)


def coefficients(lo=LO, r=R):
    # rows: monomials x^k, k = 0..r-1; columns: cells lo..lo+r-1; right side: (1/2)^k
    A = [[cell_average_of_power(k, lo + l) for l in range(r)] + [Fraction(1, 2) ** k] for k in range(r)]
    for col in range(r):
        piv = next(row for row in range(col, r) if A[row][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        for row in range(r):
            if row != col and A[row][col] != 0:
                f = A[row][col] / A[col][col]
                A[row] = [x - f * y for x, y in zip(A[row], A[col])]
    return [A[l][r] / A[l][l] for l in range(r)]


def table():
    return "const double LIN12[12] = {%s};" % ", ".join(repr(float(c)) for c in coefficients())


if __name__ == "__main__":
    print(table())
