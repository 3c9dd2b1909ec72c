"""Helpers shared by the GPU tests: task positions in Alg. 4 order and the
per-task comparison with the oracle.  No counting arithmetic here."""
import numpy as np


def alg4_positions(p, tasks):
    """Alg. 4 index of each (i,j,k) row of `tasks` (the plan's order)."""
    base = np.zeros((p, p), np.int64)
    t = 0
    for i in range(p):
        for j in range(i, p):
            base[i, j] = t
            t += p - j
    return base[tasks["i"], tasks["j"]] + (tasks["k"] - tasks["j"])


def in_alg4_order(p, tasks, per):
    """The plan-order per-task vector rearranged into Alg. 4 order."""
    got = np.zeros(len(tasks), np.uint64)
    got[alg4_positions(p, tasks)] = np.asarray(per, dtype=np.uint64)[:len(tasks)]
    return got
