"""Coefficients of the FP32 cutoff polynomial used by the kernels.

fc(t) = (1 + cos(pi sqrt(t))) / 2 on t = r^2 / rc^2 in [0, 1], interpolated at
the Chebyshev points of degree 6 and converted to the monomial basis.  Max
error 5.5e-9 in fc and 5.4e-7 in dfc/dt (FP32 rounding is 6e-8).  Prints the
C++ initialiser pasted into common.h (FcPoly<float>).

    python paper_2002_00054_amd/csrc/gen_cutoff_fp32.py
"""
import numpy as np
from numpy.polynomial import chebyshev as C, polynomial as P

DEG = 6


def main():
    ch = C.Chebyshev.interpolate(lambda x: 0.5 * (1 + np.cos(np.pi * np.sqrt(x))), DEG, domain=[0, 1])
    p = ch.convert(kind=P.Polynomial, domain=[0, 1], window=[0, 1])
    t = np.linspace(0, 1, 100001)
    f = 0.5 * (1 + np.cos(np.pi * np.sqrt(t)))
    print("// max |error| %.2e" % np.max(np.abs(p(t) - f)))
    print("{" + ", ".join("%.17g" % c for c in p.coef) + "}")


if __name__ == "__main__":
    main()
