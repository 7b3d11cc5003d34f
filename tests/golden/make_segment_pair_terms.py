"""Write segment_pair_terms.txt from a closed form (no oracle, no library).

Segment j of gamma_1 runs from (-alpha, 0, h) to (alpha, 0, h); segment i of
gamma_2 runs from (0, -beta, 0) to (0, beta, 0).  The set {l - k} of Eq. 4's
Minkowski difference is the rectangle [-alpha, alpha] x [-beta, beta] at
height h, whose solid angle seen from the origin is
4 arcsin(alpha beta / sqrt((alpha^2 + h^2)(beta^2 + h^2))); the segment-pair
term is that solid angle over 4 pi, with the sign of h (Eq. 4 and the
signed-solid-angle reading of Sec. 2.1).
"""
import math
import os

CASES = [(1.0, 1.0, 1.0), (0.5, 2.0, 0.3), (3.0, 0.25, 2.0), (1.0, 1.0, 1e-3), (1.0, 1.0, -0.7),
         (0.1, 0.1, 10.0), (2.0, 5.0, -0.01)]


def main():
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "segment_pair_terms.txt"), "w") as fh:
        fh.write("# Eq. 4 term for perpendicular segments crossing over their midpoints,\n")
        fh.write("# from the rectangle solid-angle closed form (see make_segment_pair_terms.py).\n")
        fh.write("# columns: alpha beta h term\n")
        for a, b, h in CASES:
            v = math.copysign(1.0, h) * math.asin(a * b / math.sqrt((a * a + h * h) * (b * b + h * h))) / math.pi
            fh.write("%r %r %r %.17g\n" % (a, b, h, v))


if __name__ == "__main__":
    main()
