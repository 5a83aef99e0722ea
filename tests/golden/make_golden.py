"""Writes the stored fixtures of this folder (run: python tests/golden/make_golden.py).

Neither fixture comes from the library or the oracle:

* sersic_bn_erlang.txt: b_n for integer 2n from the Erlang closed form of the regularised
  lower incomplete gamma function, P(a, b) = 1 - exp(-b) sum_{k<a} b^k / k!, solved for
  P(2n, b_n) = 1/2 at 40 significant digits, rounded once (the Sersic profile of the "sersic galaxy model",
  §2.1.1: half the light inside Re).
* point_through_psf.txt: the worked point-source example -- a point source of flux
  10^0.5 on the centre of pixel (2, 3) of a 5 x 7 image through an asymmetric 3 x 3 stamp
  is the stamp times the flux, centred on that pixel (the "psf star model" of §2.1.1 and
  a true convolution, §2.1.3).
"""
import math
import os
import sys

import mpmath

HERE = os.path.dirname(os.path.abspath(__file__))


def erlang_p(a: int, b):
    """P(a, b) = 1 - exp(-b) sum_{k<a} b^k / k! at 40 significant digits."""
    return 1 - mpmath.exp(-b) * sum(b ** k / mpmath.factorial(k) for k in range(a))


def bn_table() -> str:
    lines = [
        "# Sersic b_n for integer 2n, from the Erlang closed form of the regularised lower",
        "# incomplete gamma function: P(a, b) = 1 - exp(-b) * sum_{k<a} b^k / k!, a = 2n.",
        "# b_n is the root of P(2n, b_n) = 1/2 (half the light inside Re; the Sersic profile",
        "# of the \"sersic galaxy model\", §2.1.1).  b_{0.5} = ln 2 exactly.",
        "# Values: roots of the closed form above at 40 significant digits (mpmath), rounded",
        "# once to FP64; independent of any gamma inverse routine (make_golden.py).",
        "# n        b_n",
    ]
    mpmath.mp.dps = 40
    for n in (0.5, 1.0, 1.5, 2.0, 4.0):
        a = int(round(2 * n))
        b = mpmath.findroot(lambda x: erlang_p(a, x) - mpmath.mpf(1) / 2, mpmath.mpf(2 * n - 1.0 / 3.0))
        lines.append(f"{n:<4} {float(b)!r}")
    return "\n".join(lines) + "\n"


def point_table() -> str:
    K = [[0.05, 0.10, 0.05], [0.10, 0.40, 0.15], [0.02, 0.08, 0.05]]
    mpmath.mp.dps = 40
    Fm = mpmath.mpf(10) ** mpmath.mpf("0.5")
    F = float(Fm)
    m = [[0.0] * 7 for _ in range(5)]
    for u in (-1, 0, 1):
        for v in (-1, 0, 1):
            # the exact product of F and the decimal stamp value, rounded once
            m[2 + u][3 + v] = float(Fm * mpmath.mpf(str(K[1 + u][1 + v])))
    lines = [
        "# Worked example: a point source of flux F = 10^0.5 sitting exactly on the centre of",
        "# pixel (i=2, j=3) of a 5x7 image, convolved with the 3x3 stamp K below (not",
        "# symmetric), no sky.  The \"psf star model\" (§2.1.1) is the PSF map shifted to the",
        "# source position, so the model is F*K with its centre on (2, 3), and zero elsewhere.",
        "# Convolution, not correlation: m[2+u, 3+v] = F * K[1+u, 1+v] for u, v in {-1,0,1}.",
        "# K (rows u = -1..1, columns v = -1..1):",
    ]
    lines += [" ".join(f"{x:.2f}" for x in row) for row in K]
    lines.append(f"# expected model rows 0..4 (columns 0..6), F = {F!r}:")
    lines += [" ".join("0" if x == 0.0 else repr(x) for x in row) for row in m]
    return "\n".join(lines) + "\n"


FIXTURES = {"sersic_bn_erlang.txt": bn_table, "point_through_psf.txt": point_table}


def main(check: bool = False) -> int:
    bad = 0
    for name, fn in FIXTURES.items():
        text = fn()
        path = os.path.join(HERE, name)
        if check:
            if open(path).read() != text:
                print(f"{name} differs from what this script writes", file=sys.stderr)
                bad += 1
        else:
            with open(path, "w") as f:
                f.write(text)
    return bad


if __name__ == "__main__":
    sys.exit(main(check="--check" in sys.argv))
