"""Independent GF(2^p) arithmetic for the tests' brute-force checkers:
carry-less multiplication reduced by the primitive polynomial."""
import numpy as np

POLY = {1: 0b11, 2: 0b111, 3: 0b1011, 4: 0b10011, 5: 0b100101, 6: 0b1000011}


def mul(a: int, b: int, p: int, poly: int | None = None) -> int:
    poly = POLY[p] if poly is None else poly
    r = 0
    for i in range(p):
        if (b >> i) & 1:
            r ^= a << i
    for d in range(2 * p - 2, p - 1, -1):
        if (r >> d) & 1:
            r ^= poly << (d - p)
    return r


def mul_table(p: int) -> np.ndarray:
    q = 1 << p
    return np.array([[mul(a, b, p) for b in range(q)] for a in range(q)], dtype=np.int64)
