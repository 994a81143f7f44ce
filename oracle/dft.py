"""Dense orthonormal DFT matrices (oracle; test infrastructure only).

Sec. IV writes the 2-D DFT of an N1 x N2 frame as F(X) = F_l X F_r with F_l, F_r
orthonormal symmetric DFT matrices (the text types them as real; they are
complex).  Readings taken here:

* normalisation: unitary, 1/sqrt(N) in both directions, so F^{-1} = F^H;
* sign and origin: forward kernel exp(-2 pi i k n / N), natural order, DC at 0.

The matrix itself is the definition; nothing here is a fast transform.
"""

import numpy as np


def dft_matrix(n):
    """[F_n]_{k,m} = n^{-1/2} exp(-2 pi i k m / n), complex128, symmetric, unitary.

    The exponent is reduced modulo n in exact integer arithmetic before the
    angle is formed, so every entry is accurate to a few ulp of float64.
    """
    k = np.arange(n, dtype=np.int64)
    km = np.outer(k, k) % n
    return np.exp(-2j * np.pi * km.astype(np.float64) / n) / np.sqrt(n)


def fft2_unitary(X, Fl=None, Fr=None):
    """F(X) = F_l X F_r (Sec. IV), by dense matrix products."""
    n1, n2 = X.shape
    Fl = dft_matrix(n1) if Fl is None else Fl
    Fr = dft_matrix(n2) if Fr is None else Fr
    return Fl @ X @ Fr


def ifft2_unitary(K, Fl=None, Fr=None):
    """F^{-1}(K) = F_l^H K F_r^H, the inverse of the unitary map above."""
    n1, n2 = K.shape
    Fl = dft_matrix(n1) if Fl is None else Fl
    Fr = dft_matrix(n2) if Fr is None else Fr
    return Fl.conj().T @ K @ Fr.conj().T
