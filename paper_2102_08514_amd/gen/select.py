"""Sub-region selection of Sec. 4.2: Q plane bits q, then sigma(q mod r).

The Q splitting-plane tests give a code q in [0, 2^Q); only the codes of the
K sub-regions occur.  Storing a table over all 2^Q codes is wasteful, so the
paper compresses the range with the smallest modulus r that keeps the
sub-regions' codes apart and looks the sub-region up in a table sigma of r
entries.

Ties.  A query on a plane (or where several meet) must still produce the
code of a sub-region whose closure contains it.  Bit i is therefore taken
as the side of plane i on which the point p + eps (g - p) lies, for one
fixed generic point g inside the fold chamber F (on no splitting plane): a
value exactly on the plane takes g's side.  Since F is convex and p lies in
the closed F, p + eps (g - p) is inside F and on no plane through p, so the
code is that of a real sub-region next to p.  For FP32 queries whose cell
offsets are exact (|x| < 2^23 with the small dyadic plane offsets used
here), the plane tests are exact and only sub-region codes occur.
"""

from fractions import Fraction


def _popcount(v):
    return bin(v).count("1")


def tie_point(planes, chamber_rows, vertices):
    """A rational point strictly inside the chamber and on no splitting plane:
    a weighted mean of the chamber's vertices with distinct generic weights."""
    k = len(vertices)
    for trial in range(1, 200):
        w = [Fraction(1, (j + 2) * trial + j * j + 1) for j in range(k)]
        tot = sum(w)
        g = tuple(sum(w[j] * Fraction(vertices[j][a]) for j in range(k)) / tot for a in range(len(vertices[0])))
        inside = all(sum(Fraction(a) * x for a, x in zip(row, g)) + c > 0 for row, c in chamber_rows)
        generic = all(sum(Fraction(a) * x for a, x in zip(nu, g)) != off for nu, off in planes)
        if inside and generic:
            return g
    raise RuntimeError("no generic interior point found")


def tie_sides(planes, chamber_rows, vertices):
    """Per plane: True if the tie point lies on its >= side (ties set the bit)."""
    g = tie_point(planes, chamber_rows, vertices)
    return [sum(Fraction(a) * x for a, x in zip(nu, g)) > off for nu, off in planes]


def sigma_table(feasible, Q):
    """feasible: {code: sub-region id}.  Returns (r, sigma) with r the smallest
    modulus that keeps the codes apart and sigma[q % r] the sub-region of
    every code q; residues no code reaches repeat a sub-region (unused)."""
    K = len(feasible)
    for r in range(max(K, 1), (1 << Q) + 1):
        res = {}
        for c, k in feasible.items():
            if c % r in res:
                break
            res[c % r] = k
        else:
            return r, [res.get(m, 0) for m in range(r)]
    raise AssertionError("unreachable: r = 2^Q always separates the codes")
