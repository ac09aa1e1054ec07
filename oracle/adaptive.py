"""ORACLE — test infrastructure only.

Zippel reconstruction without known degree bounds: the number of Newton nodes
of each variable is found while sampling.  The paper accepts a result when
further probes reproduce it (Introduction) and leaves the stopping rule of
the univariate interpolation open; this file fixes the reading used by both
sides:

- Stage k samples x_k at its anchor and then at its nodes, one after another
  (in the order of the schedule's node list for x_k).
- After node m, every current term has the divided difference of order m of
  its values at x_0..x_m, the definition
      b_m = sum_{i<=m} f_i / prod_{j<=m, j!=i} (x_i - x_j).
- The stage stops at the first m for which the last `confirm` orders
  (m-confirm+1..m) vanish for every term: the interpolant of degree
  D = m - confirm through x_0..x_D then reproduces the confirming samples.
  Running past cap + confirm nodes (cap = the caller's bound, the schedule's
  node count for x_k minus confirm) is a failure (EPROBE).
- The terms are then lifted by Newton interpolation over x_0..x_D exactly as
  in the fixed-bound reconstruction.

Each stage's solve is the oracle's transposed Vandermonde solve, one node at a
time.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
may use this module; the product library never imports it.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from . import EPROBE, ESINGULAR, OracleError, newton, poly_eval, vandermonde_solve


def divided_difference(p: int, x: Sequence[int], f: Sequence[int]) -> int:
    """Order len(x)-1 divided difference of f at the distinct nodes x (the sum form)."""
    m = len(x)
    acc = 0
    for i in range(m):
        den = 1
        for j in range(m):
            if j != i:
                den = den * (int(x[i]) - int(x[j])) % p
        acc = (acc + int(f[i]) * pow(den, -1, p)) % p
    return acc


def _monomials(p: int, exps: np.ndarray, y: Sequence[int], k: int) -> List[int]:
    out = []
    for l in range(exps.shape[0]):
        m = 1
        for v in range(k):
            m = m * pow(int(y[v]), int(exps[l, v]), p) % p
        out.append(m)
    return out


def adaptive_zippel(p: int, caps: Sequence[int], schedule, box, confirm: int = 1,
                    nprobes=None) -> Tuple[np.ndarray, np.ndarray, List[int]]:
    """(exps, coefs, degrees found per variable).  schedule.nodes[v] must hold
    at least caps[v] + confirm nodes; box is a synth.BlackBox."""
    n = len(caps)
    y = [int(v) for v in schedule.y]
    anchor = [int(v) for v in schedule.anchor]
    exps = np.zeros((1, n), dtype=np.uint16)  # the empty monomial
    coefs = [1]
    found = []
    for kv in range(n):
        k = kv + 1
        X = [anchor[kv]] + [int(v) for v in schedule.nodes[kv][:caps[kv] + confirm]]
        t = exps.shape[0]
        if k == 1:
            rows = [[int(box.eval(1, 1, 1, y, anchor, [X[0]])[0])]]
        else:
            rows = [list(coefs)]
            mono = _monomials(p, exps, y, kv)
            if len(set(mono)) != t or 0 in mono:
                raise OracleError(ESINGULAR, "monomial values collide")
        run, m, D = 0, 0, None
        while D is None:
            m += 1
            if m >= len(X):
                raise OracleError(EPROBE, f"no stop within {len(X) - 1} nodes of x_{k}")
            if k == 1:
                rows.append([int(box.eval(1, 1, 1, y, anchor, [X[m]])[0])])
            else:
                v = box.eval(k, 1, t, y, anchor, [X[m]])
                rows.append([int(a) for a in vandermonde_solve(p, np.array(mono, dtype=np.uint64),
                                                               np.asarray(v, dtype=np.uint64).reshape(1, t))[0]])
            zero = all(divided_difference(p, X[:m + 1], [rows[i][l] for i in range(m + 1)]) == 0
                       for l in range(t))
            run = run + 1 if zero else 0
            if run == confirm:
                D = m - confirm
        found.append(D)
        new_e, new_c = [], []
        for l in range(t):
            g = newton(p, X[:D + 1], [rows[i][l] for i in range(D + 1)])
            for d in range(D + 1):
                if int(g[d]) != 0:
                    e = exps[l].copy()
                    e[kv] = d
                    new_e.append(e)
                    new_c.append(int(g[d]))
        exps = np.array(new_e, dtype=np.uint16).reshape(-1, n)
        coefs = new_c
    c = np.array(coefs, dtype=np.uint64)
    npr = schedule.probes.shape[0] if nprobes is None else nprobes
    for q in range(npr):
        pt = [int(v) for v in schedule.probes[q]]
        want = int(box.at(pt))
        got = poly_eval(p, exps, c, pt) if len(c) else 0
        if want != got:
            raise OracleError(EPROBE, "probe mismatch")
    return exps, c, found
