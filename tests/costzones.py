"""Cost-zone split of a sequence of body costs into G contiguous ranges: range j starts at the
smallest r with G P(r) >= j T, where P(r) is the summed cost of the first r bodies and T = P(n)."""
import numpy as np


def cost_zones_literal(cost, G):
    """The definition read literally, in Python integers (small inputs)."""
    P = [0]
    for c in cost:
        P.append(P[-1] + int(c))
    T = P[-1]
    out = []
    for j in range(G + 1):
        r = 0
        while G * P[r] < j * T:
            r += 1
        out.append(r)
    return np.array(out, dtype=np.int64)


def cost_zones(cost, G):
    """The same split by binary search on the prefix sums (int64; positive costs)."""
    P = np.concatenate([[0], np.cumsum(cost, dtype=np.int64)])
    T = int(P[-1])
    return np.array([np.searchsorted(G * P, j * T, side="left") for j in range(G + 1)], dtype=np.int64)


def group_zones(group_cost, n, G, group=64):
    """The split over walk groups of `group` bodies: group g costs its body count plus
    group_cost[g]; range j starts at min(group x, n) for the smallest group boundary x with
    G P(x) >= j T."""
    counts = np.minimum(group, n - group * np.arange(len(group_cost)))
    x = cost_zones(counts + np.asarray(group_cost, dtype=np.int64), G)
    return np.minimum(group * x, n)
