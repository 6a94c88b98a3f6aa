"""Algorithmic operation counts of the energy+force path, for roofline accounting.

A count is what the formulas of the method require, not what an ISA executes:
every add, multiply, compare and transcendental (exp, cos, sin, sqrt,
reciprocal) is one operation, a fused multiply-add two.  The per-unit figures
below come from writing the terms of Sec. 3.1 step 1 (radial and angular
symmetry functions with the cosine cutoff) and step 3 (their gradients
contracted with dE/dG and scattered onto the atoms) in the contracted form the
kernels evaluate; the units are the work counts the library reports
(``Potential.count_work``): neighbour entries, candidate neighbour pairs,
triplet terms, angular and radial SF-term updates.

Force pass (per unit):
  neighbour entry   34  displacement (3), r^2 (5), sqrt and 1/r (2), cutoff and
                        its derivative (6), per angular eta (2): exp(-eta r^2),
                        g = fc e and dg/dr (7 each = 14), slot force (4)
  radial SF term    10  exp(-eta (r - rs)^2) (4), its r-derivative (4), c * dt (2)
  candidate pair     9  r_jk vector (3), r_jk^2 (5), compare (1)
  triplet term     108  r_jk^2 again (8), cutoff of r_jk and derivative (7),
                        cos theta (7), exp(-eta r_jk^2) for 2 eta (4), per-eta
                        contractions Ua Ub Uc Us (2 x 18 = 36), gradients on j
                        and k (2 x 15 = 30), 8 coefficient products, slot adds (8)
  angular SF term    9  1 + lambda cos (1), P^zeta and P^(zeta-1) (2),
                        c 2^(1-zeta) P^zeta and its zeta lambda P^(zeta-1) partner (4),
                        accumulation into the per-eta sums (2)
SF pass (per unit):
  neighbour entry   20  displacement, r^2, sqrt, 1/r (10), cutoff (4), per angular eta
                        exp and g (3 x 2 = 6)
  radial SF term     6  exp(-eta (r - rs)^2) (4), times fc and accumulate (2)
  candidate pair     9
  triplet term      30  r_jk^2 (8), cutoff of r_jk (5), cos theta (7), exp for
                        2 eta (4), per-eta products g_j g_k e fd (6)
  angular SF term    5  1 + lambda cos (1), P^zeta (1), two products (2), accumulate (1)
"""

FORCE = dict(pairs=34, radial_terms=10, candidates=9, triplets=108, angular_terms=9)
SF = dict(pairs=20, radial_terms=6, candidates=9, triplets=30, angular_terms=5)
#: Network forward + input gradient per atom, unpadded widths n_sf -> 25 -> 25 -> 1:
#: 2 flops per multiply-add of the four matrix-vector products plus tanh and
#: derivative terms.
def mlp_flops(n_sf: int, h1: int = 25, h2: int = 25) -> int:
    mv = 2 * (n_sf * h1 + h1 * h2 + h2)
    return 2 * mv + 4 * (h1 + h2)


def flops(model: dict, counts: dict) -> int:
    """Algorithmic operations of one launch for the given work counts."""
    return int(sum(model[k] * counts[k] for k in model))


#: MI355X peaks used as roofline denominators (published figures).
PEAK_HBM_GBS = 8000.0
PEAK_FP32_VECTOR_TFLOPS = 157.3  # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2 (packed) x 2.4 GHz
PEAK_FP64_VECTOR_TFLOPS = 78.6
