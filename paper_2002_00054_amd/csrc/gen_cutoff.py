"""Coefficients of the cutoff polynomials used by the kernels.

fc(t) = (1 + cos(pi sqrt(t))) / 2 on t = r^2 / rc^2 in [0, 1], interpolated at
the Chebyshev points and converted to the monomial basis:
  FP32  degree 6:  max error 5.5e-9 in fc and 5.4e-7 in dfc/dt (FP32 rounding 6e-8);
  FP64  degree 10: max error 1.4e-15 in fc and 1.7e-13 in dfc/dt (far below the
        1e-9 relative parity bar of the FP64 form).
Prints the C++ initialisers pasted into common.h (FcPoly<float>, FcPoly<double>).

    python paper_2002_00054_amd/csrc/gen_cutoff.py
"""
import numpy as np
from numpy.polynomial import chebyshev as C, polynomial as P


def fit(deg):
    ch = C.Chebyshev.interpolate(lambda x: 0.5 * (1 + np.cos(np.pi * np.sqrt(x))), deg, domain=[0, 1])
    return ch.convert(kind=P.Polynomial, domain=[0, 1], window=[0, 1])


def main():
    t = np.linspace(0, 1, 100001)
    f = 0.5 * (1 + np.cos(np.pi * np.sqrt(t)))
    for name, deg in (("float", 6), ("double", 10)):
        p = fit(deg)
        print("// FcPoly<%s>: degree %d, max |error| %.2e" % (name, deg, np.max(np.abs(p(t) - f))))
        print("{" + ", ".join("%.17g" % c for c in p.coef) + "}")


if __name__ == "__main__":
    main()
