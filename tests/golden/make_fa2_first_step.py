"""Writes the rows of fa2_first_step.txt: the two-body ForceAtlas2 steps evaluated from
the scalar closed forms in that file's header with 40-digit decimal arithmetic.  Uses
neither the oracle nor the GPU library.

    python tests/golden/make_fa2_first_step.py >> tests/golden/fa2_first_step.txt
"""
from decimal import Decimal as D, getcontext

getcontext().prec = 40


def _sgn(x):
    return D(1) if x > 0 else (D(-1) if x < 0 else D(0))


def two_body(t0, t1, m0, m1, kr, kg, tau, ks, ksmax, iters):
    fp0 = fp1 = D(0)
    s = D(1)
    for _ in range(iters):
        d = t1 - t0
        f0 = -kr * m0 * m1 / d + d - kg * m0 * _sgn(t0)
        f1 = kr * m0 * m1 / d - d - kg * m1 * _sgn(t1)
        sw0, sw1 = abs(f0 - fp0), abs(f1 - fp1)
        S = m0 * sw0 + m1 * sw1
        T = m0 * abs(f0 + fp0) / 2 + m1 * abs(f1 + fp1) / 2
        if S > 0:
            s = min(tau * T / S, D("1.5") * s)
        s0 = ks * s / (1 + s * sw0.sqrt())
        s1 = ks * s / (1 + s * sw1.sqrt())
        if f0 != 0 and s0 > ksmax / abs(f0):
            s0 = ksmax / abs(f0)
        if f1 != 0 and s1 > ksmax / abs(f1):
            s1 = ksmax / abs(f1)
        t0 += s0 * f0
        t1 += s1 * f1
        fp0, fp1 = f0, f1
    return t0, t1, s


ROWS = [
    ("-0.3", "0.3", "2", "2", "1", "1", "1", "0.1", "10", 1, "1", "0"),
    ("-0.3", "0.3", "2", "2", "1", "1", "1", "1", "10", 2, "1", "0"),
    ("-0.3", "0.3", "2", "2", "1", "1", "1", "0.1", "0.05", 1, "1", "0"),
    ("-0.2", "0.5", "1", "3", "1", "1", "1", "1", "10", 2, "1", "0"),
    ("-0.2", "0.5", "1", "3", "1", "1", "0.5", "0.1", "10", 3, "1", "0"),
    ("-0.3", "0.3", "2", "2", "1", "1", "1", "0.1", "10", 1, "0.6", "0.8"),
    ("-0.3", "0.3", "2", "2", "1", "1", "1", "1", "10", 2, "0.6", "0.8"),
    ("-0.2", "0.5", "1", "3", "1", "1", "1", "1", "10", 2, "0.6", "0.8"),
]

if __name__ == "__main__":
    for r in ROWS:
        t0, t1, s = two_body(*[D(v) for v in r[:9]], r[9])
        print(" ".join(str(v) for v in r) + f" {t0:.17e} {t1:.17e} {s:.17e}")
