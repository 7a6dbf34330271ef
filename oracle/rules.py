"""Association rules from the frequent itemsets -- TEST INFRASTRUCTURE ONLY
(used by tests/, never by the library; shares no code with it).

The paper names association rule learning as what frequent itemsets serve
(abstract; Section I) and support, confidence and lift as the indicators
evaluated on the mined itemsets (Section IV-A), without defining the latter
two.  This module takes the standard definitions (confidence as in Agrawal,
Imielinski and Swami 1993; lift as in Brin, Motwani, Ullman and Tsur 1997):

  for a frequent itemset Z and a split Z = X + Y with X and Y disjoint and
  non-empty (X the antecedent, Y the consequent),
    conf(X => Y) = supp(Z) / supp(X)
    lift(X => Y) = conf(X => Y) / (supp(Y) / n) = supp(Z) * n / (supp(X) * supp(Y))

Both X and Y are subsets of a frequent set, hence frequent, so their supports
are looked up in F itself.  A rule is reported when conf >= c with the
threshold given exactly as c = min_conf_ppm / 10^6: the test is
supp(Z) * 10^6 >= min_conf_ppm * supp(X) in integers, so no rounding decides
it.  conf and lift are the IEEE double quotients of those integers (each
operand converted to double first).  Order: by the position of Z in the
canonical itemset list, then by X as an ascending tuple, lexicographically
with a prefix before its extensions.
"""
from __future__ import annotations

from itertools import combinations


def rules(F, n: int, min_conf_ppm: int, max_len: int | None = None):
    """F: canonical list of (itemset tuple, support).  Returns a list of
    (z_index, X, Y, supp_x, supp_y, supp_z, conf, lift); itemsets longer than
    max_len (if given) produce no rules."""
    supp = {tuple(x): int(s) for x, s in F}
    out = []
    for zi, (Z, sz) in enumerate(F):
        Z = tuple(Z)
        L = len(Z)
        if L < 2 or (max_len is not None and L > max_len):
            continue
        for k in range(1, L):
            for X in combinations(Z, k):
                Y = tuple(z for z in Z if z not in X)
                sx, sy = supp[X], supp[Y]
                if int(sz) * 1_000_000 >= int(min_conf_ppm) * sx:
                    out.append((zi, X, Y, sx, sy, int(sz), float(sz) / float(sx),
                                float(int(sz) * int(n)) / float(sx * sy)))
    out.sort(key=lambda r: (r[0], r[1]))
    return out
