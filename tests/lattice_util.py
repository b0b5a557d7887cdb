"""fcc lattice shells by enumeration (test helper, not a test).

The fcc lattice is the set of points (a/2)(i, j, k) with integer i, j, k of
even sum; |R|^2 = a_nn^2 (i^2 + j^2 + k^2) / 2 with a_nn = a / sqrt(2).  The
multiplicity of shell s (|R|^2 = s a_nn^2) is the number of such triples
with i^2 + j^2 + k^2 = 2 s."""
import numpy as np


def fcc_shell_counts(smax):
    """[m_1, ..., m_smax]: lattice vectors of squared length s a_nn^2."""
    b = int(np.ceil(np.sqrt(2 * smax))) + 1
    g = np.arange(-b, b + 1)
    i, j, k = np.meshgrid(g, g, g, indexing="ij")
    even = (i + j + k) % 2 == 0
    q = (i * i + j * j + k * k)[even]
    return [int(np.count_nonzero(q == 2 * s)) for s in range(1, smax + 1)]
