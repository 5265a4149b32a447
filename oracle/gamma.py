"""Euclidean gamma matrices in the chiral basis.

The paper (Sec. 2.1) leaves the basis open; its footnote only says that a
non-relativistic basis would change the flop count.  We fix the chiral basis:
gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] for k = 1,2,3 (mu = 0,1,2 = x,y,z)
and gamma_4 = [[0, 1], [1, 0]] (mu = 3 = t).  Spin index runs 0..3.
"""

import numpy as np

_SIGMA = (
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
)
_I2 = np.eye(2, dtype=np.complex128)
_Z2 = np.zeros((2, 2), dtype=np.complex128)


def gammas() -> np.ndarray:
    """(4, 4, 4) array: gammas()[mu] is gamma_mu."""
    g = np.empty((4, 4, 4), dtype=np.complex128)
    for k in range(3):
        g[k] = np.block([[_Z2, -1j * _SIGMA[k]], [1j * _SIGMA[k], _Z2]])
    g[3] = np.block([[_Z2, _I2], [_I2, _Z2]])
    return g


def gamma5() -> np.ndarray:
    g = gammas()
    return g[0] @ g[1] @ g[2] @ g[3]


def projectors():
    """(1 - gamma_mu) and (1 + gamma_mu) for mu = 0..3."""
    g = gammas()
    one = np.eye(4, dtype=np.complex128)
    return one[None] - g, one[None] + g
