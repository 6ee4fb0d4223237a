"""Task counts and operation-count models of Sections 3.3.3 and 3.4.5
(Tables blr_bch_operations and blr_bh_operations).  Indices are 1-based in
the paper's sums; p = m/b, q = n/b, r the (fixed) low-rank rank."""
from __future__ import annotations


def tiled_task_counts(p: int, q: int) -> dict:
    return {
        "geqrt": q,
        "larfb": q * (q - 1) // 2,
        "tpqrt": sum(p - k for k in range(1, q + 1)),
        "tpmqrt": sum((p - k) * (q - k) for k in range(1, q + 1)),
    }


def t_tiled_sum(m, n, b, r):
    """sum_{k=1}^{q} (p-k+1) b^3 + (p-k+1)(q-k) b^2 r."""
    p, q = m // b, n // b
    return sum((p - k + 1) * b ** 3 + (p - k + 1) * (q - k) * b ** 2 * r
               for k in range(1, q + 1))


def t_tiled_printed(m, n, b, r):
    """The closed form printed under the sum (it does not equal the sum)."""
    return (6 * m * n * b + 3 * n * b ** 2 + 3 * m * n ** 2 * r / b
            - 3 * n ** 2 * b - 5 * n ** 3 * r / b - 3 * m * n * r) / 6


def t_tiled_closed(m, n, b, r):
    """Closed form of the tiled sum, derived here: the b^3 part is
    mnb - n^2 b/2 + n b^2/2 and the b^2 r part is
    r (3mn^2/b - 3mn - n^3/b + 3n^2 - 2nb) / 6."""
    return (m * n * b - n ** 2 * b / 2 + n * b ** 2 / 2
            + r * (3 * m * n ** 2 / b - 3 * m * n - n ** 3 / b + 3 * n ** 2 - 2 * n * b) / 6)


def t_blocked_sum(m, n, b, r):
    """sum_{k=1}^{q} b^3 + p b^2 r + (q-k)(b^2 r + p b r^2)."""
    p, q = m // b, n // b
    return sum(b ** 3 + p * b ** 2 * r + (q - k) * (b ** 2 * r + p * b * r ** 2)
               for k in range(1, q + 1))


def t_blocked_printed(m, n, b, r):
    return (2 * n * b ** 2 + 2 * m * n * r + n ** 2 * r + m * n ** 2 * r ** 2 / b ** 2
            - n * b * r - m * n * r ** 2 / b) / 2
