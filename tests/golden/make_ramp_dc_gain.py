"""Write ramp_dc_gain.txt: the DC gain H[0] of the band-limited ramp filter.

H[0] = sum_m h[m] over m in [-L/2, L/2).  With h[0] = 1/4 and h[m] = -1/(pi^2 m^2)
for odd m, and sum over all odd m >= 1 of 1/m^2 = pi^2 / 8, the sum equals the
tail (2 / pi^2) * sum_{odd m > L/2} 1/m^2.  This script evaluates that tail
exactly up to M = 10^7 and closes it with the Euler-Maclaurin remainder, in
Python's decimal arithmetic -- a route independent of the oracle's FFT.
"""
from decimal import Decimal, getcontext
import os

getcontext().prec = 40


def pi_decimal():
    # Machin's formula: pi = 16 atan(1/5) - 4 atan(1/239)
    def atan_inv(x):
        x = Decimal(x)
        x2 = x * x
        term = Decimal(1) / x
        total = term
        k = 1
        while True:
            term /= -x2
            t = term / (2 * k + 1)
            if abs(t) < Decimal(10) ** -45:
                break
            total += t
            k += 1
        return total
    return 16 * atan_inv(5) - 4 * atan_inv(239)


def tail_odd_inverse_squares(m0: int, M: int = 200000) -> Decimal:
    """sum over odd m >= m0 of 1/m^2 (m0 odd)."""
    s = Decimal(0)
    m = m0
    stop = m0 + 2 * M
    while m < stop:
        s += Decimal(1) / (Decimal(m) * m)
        m += 2
    # Euler-Maclaurin for sum_{k>=0} f(stop + 2k), f(x) = 1/x^2, step 2:
    # integral/2 + f/2 - (2/12) f' + ...
    x = Decimal(stop)
    s += 1 / (2 * x) + 1 / (2 * x * x) + Decimal(2) / (6 * x ** 3) - Decimal(8) / (30 * x ** 5)
    return s


def main():
    pi = pi_decimal()
    lines = ["# L  H[0] of the band-limited ramp (cycles/pixel), tail series in decimal arithmetic",
             "# written by tests/golden/make_ramp_dc_gain.py"]
    for e in range(3, 15):
        L = 1 << e
        m0 = L // 2 + 1
        if m0 % 2 == 0:
            m0 += 1
        h0 = 2 / (pi * pi) * tail_odd_inverse_squares(m0)
        lines.append(f"{L} {float(h0):.17e}")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ramp_dc_gain.txt")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(path)


if __name__ == "__main__":
    main()
