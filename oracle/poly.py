"""ORACLE — test infrastructure only (never imported by the product library).

Exact integer arithmetic on the tenth-degree polynomial of the second cuboid
conjecture, eq. (1.1) of Gallyamov et al., arXiv:1601.00636:

    Q_pq(t) = t^10 + (2q^2 + p^2)(3q^2 - 2p^2) t^8
            + (q^8 + 10p^2q^6 + 4p^4q^4 - 14p^6q^2 + p^8) t^6
            - p^2q^2 (q^8 - 14p^2q^6 + 4p^4q^4 + 10p^6q^2 + p^8) t^4
            - p^6q^6 (q^2 + 2p^2)(3p^2 - 2q^2) t^2
            - q^10 p^10

Python ints, no modular reduction, no floating point.
"""


def q_coeffs(p: int, q: int) -> list:
    """Coefficients of Q_pq in ascending powers of s = t^2: [c0, c2, c4, c6, c8, 1].

    Eq. (1.1) term by term.
    """
    p, q = int(p), int(q)
    c8 = (2 * q**2 + p**2) * (3 * q**2 - 2 * p**2)
    c6 = q**8 + 10 * p**2 * q**6 + 4 * p**4 * q**4 - 14 * p**6 * q**2 + p**8
    c4 = -(p**2) * q**2 * (q**8 - 14 * p**2 * q**6 + 4 * p**4 * q**4 + 10 * p**6 * q**2 + p**8)
    c2 = -(p**6) * q**6 * (q**2 + 2 * p**2) * (3 * p**2 - 2 * q**2)
    c0 = -(q**10) * p**10
    return [c0, c2, c4, c6, c8, 1]


def q_value(p: int, q: int, t: int) -> int:
    """Q_pq(t) exactly, eq. (1.1)."""
    s = int(t) ** 2
    return sum(c * s**k for k, c in enumerate(q_coeffs(p, q)))


def theorem_1_1_flags(p: int, q: int, t: int) -> int:
    """The four inequalities of Theorem 1.1 as bits 0..3:
    t > p^2, t > pq, t > q^2, (p^2 + t)(pq + t) > 2 t^2."""
    p, q, t = int(p), int(q), int(t)
    f = 0
    if t > p * p:
        f |= 1
    if t > p * q:
        f |= 2
    if t > q * q:
        f |= 4
    if (p * p + t) * (p * q + t) > 2 * t * t:
        f |= 8
    return f
