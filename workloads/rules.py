"""Node sets on the standard simplex T0 = {u >= 0, v >= 0, u + v <= 1}.

* ``dunavant6``: the 12-point, degree-6 symmetric rule of Dunavant (1985),
  used as the source quadrature on every skeleton triangle.  The three orbit
  parameters were polished by Gauss-Newton on the 28 moment equations of
  degree <= 6 at 40 digits, so the rule is exact to rounding on that space.
  The paper itself uses Vioreanu-Rokhlin rules (section 4.3, remark on
  Gaussian-like rules); those tables are not reproduced here.
* ``chart_nodes``: the (p+1)(p+2)/2 chart (discretisation) nodes of order p,
  taken as the interior "shrunk" principal lattice: barycentric coordinates
  (i + 1/3, j + 1/3, k + 1/3) / (p + 1), i + j + k = p.  This is an affine
  image of the degree-p principal lattice, hence unisolvent for total degree
  <= p, with every node strictly inside T0.  It stands in for the
  Vioreanu-Rokhlin interpolation nodes of section 3.2, whose tables are not
  available.
"""
import numpy as np

# orbit parameters (barycentric), weights normalised to sum 1 over the triangle
_S21 = ((0.2492867451709104212916386, 0.1167862757263793660252896),
        (0.0630890144915022283403316, 0.05084490637020681692093681))
_S111 = (0.05314504984481694735324967, 0.3103524510337844054166077,
         0.08285107561837357519355346)


def dunavant6():
    """Return an (12, 3) float64 array of (u, v, w) on T0 with sum(w) = 1/2."""
    rows = []
    for a, w in _S21:
        b = 1.0 - 2.0 * a
        for l1, l2, l3 in ((a, a, b), (a, b, a), (b, a, a)):
            rows.append((l2, l3, w))
    b, c, w = _S111
    d = 1.0 - b - c
    for l1, l2, l3 in ((b, c, d), (b, d, c), (c, b, d), (c, d, b), (d, b, c), (d, c, b)):
        rows.append((l2, l3, w))
    r = np.array(rows, dtype=np.float64)
    r[:, 2] *= 0.5          # area of T0
    return r


def chart_nodes(p):
    """Interior shrunk principal lattice of order p: ((p+1)(p+2)/2, 2) (u, v)."""
    pts = []
    for i in range(p + 1):
        for j in range(p + 1 - i):
            k = p - i - j
            l2 = (j + 1.0 / 3.0) / (p + 1)
            l3 = (k + 1.0 / 3.0) / (p + 1)
            pts.append((l2, l3))
    return np.array(pts, dtype=np.float64)


def chart_nodes_45():
    """The 45 order-8 chart nodes."""
    return chart_nodes(8)
