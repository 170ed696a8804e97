"""Isotropic shell weights of the interaction stencils, derived by exact rational algebra.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle; never imported by the product path).

The paper does not print the weights w, p of eq. (FORCE).  It constrains them (Sec.
"Competing interactions", Fig. 1 caption, Appendix B):
  * w lives on the links with |c|^2 <= 4 (links 1..12: shells 1, 2, 4); p on all 24 links
    (shells 1, 2, 4, 5, 8);
  * both sets give isotropic tensors E^(n) (eq. (tensorial)) up to sixth order;
  * the bulk equation of state (BULK) fixes the second moment: the interaction pressure of a
    uniform state is (G/2) psi^2 E2, so (BULK) needs E2 = c_s^2 = 1/3.  (Appendix B writes
    E2 = 1; that normalisation contradicts (BULK) and is not used.)
For w the conditions E2, (4sum), (6sum) have a unique solution on shells {1, 2, 4}.  For p the
same three conditions leave a two-parameter family on five shells; requiring eighth-order
isotropy as well closes it uniquely.  The A-B cross weights t are the D2Q9 weights (shells
{1, 2}, fourth-order isotropic, E2 = 1/3).

Isotropy of E^(2n) in two dimensions (Appendix B): sum_l W c_x^(2a) c_y^(2b) equals
e_2n (2a-1)!! (2b-1)!! for every a + b = n, so all ratios between these moments are fixed.
"""

from fractions import Fraction
from itertools import product

SHELLS = (1, 2, 4, 5, 8)


def shell_links(q):
    """All integer vectors c with |c|^2 == q inside the 5x5 neighbourhood."""
    return [(cx, cy) for cx, cy in product(range(-2, 3), repeat=2) if cx * cx + cy * cy == q]


def moment(q, a, b):
    """sum over the links of shell q of cx^a cy^b (an integer)."""
    return sum(cx ** a * cy ** b for cx, cy in shell_links(q))


def _dfact(n):
    """(n)!! for odd n >= -1, with (-1)!! = 1."""
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


def isotropy_rows(shells, order):
    """Linear conditions (rows over the shell weights) for isotropy of E^(4) .. E^(order)."""
    rows = []
    for n in range(2, order // 2 + 1):
        # m(2a, 2n-2a) * (2n-1)!! == m(2n, 0) * (2a-1)!! (2n-2a-1)!!
        for a in range(1, n // 2 + 1):
            b = n - a
            row = [Fraction(moment(q, 2 * a, 2 * b) * _dfact(2 * n - 1)
                            - moment(q, 2 * n, 0) * _dfact(2 * a - 1) * _dfact(2 * b - 1))
                   for q in shells]
            rows.append(row)
    return rows


def _solve(rows, rhs):
    """Exact Gaussian elimination; requires a unique solution."""
    n = len(rows[0])
    a = [list(r) + [v] for r, v in zip(rows, rhs)]
    piv_row = 0
    pivots = []
    for col in range(n):
        pr = next((i for i in range(piv_row, len(a)) if a[i][col] != 0), None)
        if pr is None:
            continue
        a[piv_row], a[pr] = a[pr], a[piv_row]
        pv = a[piv_row][col]
        a[piv_row] = [v / pv for v in a[piv_row]]
        for i in range(len(a)):
            if i != piv_row and a[i][col] != 0:
                fct = a[i][col]
                a[i] = [vi - fct * vp for vi, vp in zip(a[i], a[piv_row])]
        pivots.append(col)
        piv_row += 1
    if len(pivots) != n:
        raise ValueError("isotropy system does not have a unique solution")
    for i in range(piv_row, len(a)):
        if a[i][n] != 0:
            raise ValueError("isotropy system is inconsistent")
    return [a[i][n] for i in range(n)]


def isotropic_weights(shells, order, e2=Fraction(1, 3)):
    """Weights W(q) for q in shells with E2 = e2 and isotropy up to E^(order)."""
    rows = [[Fraction(moment(q, 2, 0)) for q in shells]]
    rhs = [Fraction(e2)]
    for r in isotropy_rows(shells, order):
        rows.append(r)
        rhs.append(Fraction(0))
    sol = _solve(rows, rhs)
    return dict(zip(shells, sol))


def weights_w():
    """Attractive-belt weights w(q), q in {1, 2, 4}; zero on shells 5 and 8."""
    w = isotropic_weights((1, 2, 4), 6)
    return {q: w.get(q, Fraction(0)) for q in SHELLS}


def weights_p():
    """Repulsive weights p(q) on all five shells (sixth order closed by eighth order)."""
    return isotropic_weights(SHELLS, 8)


def weights_t():
    """A-B cross weights on the first belt (D2Q9 weights), shells {1, 2}."""
    return isotropic_weights((1, 2), 4)


def weights_belt():
    """Alternative reading: D2Q9 weights on belt I (|c|^2 <= 2) for the attractive sum."""
    t = isotropic_weights((1, 2), 4)
    return {q: t.get(q, Fraction(0)) for q in SHELLS}


def e4(W):
    """Fourth-order coefficient, eq. (e4part): sum W cx^2 cy^2."""
    return sum(W[q] * moment(q, 2, 2) for q in SHELLS)


def e6(W):
    """Sixth-order coefficient, eq. (e6part): (1/3) sum W cx^4 cy^2."""
    return sum(W[q] * moment(q, 4, 2) for q in SHELLS) / 3


def as_float_list(W):
    return [float(W.get(q, 0)) for q in SHELLS]


# ----------------------------------------------------------------------------------------
# Three dimensions (the extension of Sec. "Competing interactions"; the paper gives no 3-D
# weights).  The same two belts over the integer vectors of the 5x5x5 cube: the attractive belt
# |c|^2 <= 4 (shells 1, 2, 3, 4) and the repulsive belt |c|^2 <= 8 (shells 1, 2, 3, 4, 5, 6, 8),
# with E2 = 1/3 and isotropy of E^(2n) in three dimensions: sum W cx^(2a) cy^(2b) cz^(2c) equals
# e_2n (2a-1)!! (2b-1)!! (2c-1)!! for every a + b + c = n.  Sixth order fixes w on four shells
# and eighth order fixes p on seven; the A-B weights t are the D3Q19 weights.
# ----------------------------------------------------------------------------------------

SHELLS3 = (1, 2, 3, 4, 5, 6, 8)


def shell_links3(q):
    """All integer vectors c with |c|^2 == q inside the 5x5x5 neighbourhood."""
    return [c for c in product(range(-2, 3), repeat=3) if sum(v * v for v in c) == q]


def moment3(q, a, b, c):
    """sum over the links of shell q of cx^a cy^b cz^c (an integer)."""
    return sum(x ** a * y ** b * z ** c for x, y, z in shell_links3(q))


def isotropy_rows3(shells, order):
    """Linear conditions for isotropy of the 3-D tensors E^(4) .. E^(order): one row per
    partition a >= b >= c of n other than (n, 0, 0), against the (n, 0, 0) moment."""
    rows = []
    for n in range(2, order // 2 + 1):
        for a in range(n, -1, -1):
            for b in range(min(a, n - a), -1, -1):
                c = n - a - b
                if c > b or (a, b, c) == (n, 0, 0):
                    continue
                rows.append([Fraction(moment3(q, 2 * a, 2 * b, 2 * c) * _dfact(2 * n - 1)
                                      - moment3(q, 2 * n, 0, 0) * _dfact(2 * a - 1) * _dfact(2 * b - 1)
                                      * _dfact(2 * c - 1)) for q in shells])
    return rows


def isotropic_weights3(shells, order, e2=Fraction(1, 3)):
    rows = [[Fraction(moment3(q, 2, 0, 0)) for q in shells]]
    rhs = [Fraction(e2)]
    for r in isotropy_rows3(shells, order):
        rows.append(r)
        rhs.append(Fraction(0))
    return dict(zip(shells, _solve(rows, rhs)))


def weights3_w():
    """3-D attractive weights w(q), sixth-order isotropic on shells {1, 2, 3, 4}; zero beyond."""
    w = isotropic_weights3((1, 2, 3, 4), 6)
    return {q: w.get(q, Fraction(0)) for q in SHELLS3}


def weights3_p():
    """3-D repulsive weights p(q), eighth-order isotropic on shells {1, 2, 3, 4, 5, 6, 8}."""
    return isotropic_weights3(SHELLS3, 8)


def weights3_t():
    """3-D A-B cross weights on shells {1, 2} (the D3Q19 weights)."""
    return isotropic_weights3((1, 2), 4)


def as_float_list3(W):
    return [float(W.get(q, 0)) for q in SHELLS3]
