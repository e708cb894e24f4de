"""Vertex enumeration for tiny LPs with finite boxes (test-side pin).

A bounded LP attains its optimum at a vertex of the feasible polytope. A
vertex is a feasible point where n linearly independent constraints are
active: all equality rows plus n - m_E of the inequalities (>= rows, lower
bounds, upper bounds). Enumerating every such choice and keeping the best
feasible point gives the optimum exactly, up to the linear solves.
"""

import itertools

import numpy as np


def brute_force(lp, feas_tol=1e-9):
    A = lp.csr().toarray()
    n = lp.n
    E = np.flatnonzero(lp.sense == 0)
    I = np.flatnonzero(lp.sense == 1)
    assert np.all(np.isfinite(lp.l)) and np.all(np.isfinite(lp.u))
    # inequality rows as (coefficients, rhs) of  a^T x >= rhs
    ineq = [(A[i], lp.b[i]) for i in I]
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        ineq.append((e, lp.l[j]))
        ineq.append((-e, -lp.u[j]))
    need = n - E.size
    best_obj, best_x, n_vertices = np.inf, None, 0
    for combo in itertools.combinations(range(len(ineq)), need):
        M = np.vstack([A[E]] + [ineq[t][0][None, :] for t in combo]) if need else A[E]
        rhs = np.concatenate([lp.b[E], [ineq[t][1] for t in combo]])
        if abs(np.linalg.det(M)) < 1e-12:
            continue
        x = np.linalg.solve(M, rhs)
        scale = 1.0 + np.abs(x).max()
        if np.any(np.abs(A[E] @ x - lp.b[E]) > feas_tol * scale):
            continue
        if np.any(A[I] @ x - lp.b[I] < -feas_tol * scale):
            continue
        if np.any(x < lp.l - feas_tol * scale) or np.any(x > lp.u + feas_tol * scale):
            continue
        n_vertices += 1
        obj = float(lp.c @ x)
        if obj < best_obj - 1e-12 * (1 + abs(obj)):
            best_obj, best_x = obj, x
    return best_obj, best_x, n_vertices
