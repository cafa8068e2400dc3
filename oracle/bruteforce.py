"""Pure-Python Gauss-Jordan mod p for tiny matrices (test infrastructure only).

A third, independent way to RREF(M): Python integers, lists of lists, the
first remaining nonzero row as pivot, inverse by ``pow(a, -1, p)``.  Used on
matrices of a few dozen entries, exhaustively over small fields.
"""
from __future__ import annotations


def rref_lists(rows: list[list[int]], p: int) -> tuple[list[list[int]], list[int]]:
    """Reduced row echelon form of ``rows`` over F_p.

    Returns (nonzero RREF rows in pivot order, pivot columns)."""
    a = [[x % p for x in r] for r in rows]
    m = len(a)
    n = len(a[0]) if m else 0
    rank, piv = 0, []
    for c in range(n):
        sel = next((i for i in range(rank, m) if a[i][c]), None)
        if sel is None:
            continue
        a[rank], a[sel] = a[sel], a[rank]
        inv = pow(a[rank][c], -1, p)
        a[rank] = [(x * inv) % p for x in a[rank]]
        for i in range(m):
            if i != rank and a[i][c]:
                f = a[i][c]
                a[i] = [(x - f * y) % p for x, y in zip(a[i], a[rank])]
        piv.append(c)
        rank += 1
        if rank == m:
            break
    return a[:rank], piv
