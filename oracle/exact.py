"""Closed forms of w* = phi_l(h J) v used to pin the oracle (not used by it).

* diagonal J: w*_i = phi_l(h lambda_i) v_i (Sec. 1 definition, elementwise);
* circulant J (periodic advection-diffusion or pure diffusion): J is
  diagonalised by the 2D DFT, w* = IFFT(phi_l(h sigma) FFT(v)) with sigma the
  stencil's Fourier symbol;
* any small J: the Sec. 2.1 theorem -- phi_l(A) b is the top block of the last
  column of exp of the augmented matrix [[A, b, 0], [0, 0, I], [0, 0, 0]] --
  evaluated with scipy's Pade scaling-and-squaring expm (Sec. 1 names Pade and
  scaling-and-squaring as the dense methods).

* pure diffusion with homogeneous Neumann boundaries on a cell-centred grid:
  the 1D second difference with ghost = boundary cell has the DCT-II vectors
  cos(pi k (i + 1/2) / n) as eigenvectors, eigenvalue -(4/dx^2) sin^2(pi k / 2n),
  so w* = IDCT(phi_l(h lambda) DCT(v)) with the orthonormal 2D DCT-II;
Complex phi_l for the Fourier symbol is evaluated through the same theorem on
the scalar (l+1)x(l+1) augmented matrix, so this module does not reuse the
oracle's phi.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def augmented(A: np.ndarray, b: np.ndarray, l: int) -> np.ndarray:
    """(n+l) x (n+l) matrix whose exponential holds phi_l(A) b (Sec. 2.1 theorem).

    With p = l, B = [b, 0, ..., 0] (b in the column paired with phi_l) and the
    shift block K, the last column of exp(A~) starts with phi_l(A) b.
    """
    n = A.shape[0]
    M = np.zeros((n + l, n + l), dtype=np.result_type(A, b, np.float64))
    M[:n, :n] = A
    if l == 0:
        return M
    M[:n, n] = b
    for i in range(l - 1):
        M[n + i, n + i + 1] = 1.0
    return M


def phi_dense(A: np.ndarray, b: np.ndarray, l: int) -> np.ndarray:
    """phi_l(A) b via Pade expm of the augmented matrix."""
    n = A.shape[0]
    if l == 0:
        return scipy.linalg.expm(A) @ b
    E = scipy.linalg.expm(augmented(A, b, l))
    return E[:n, n + l - 1]


def phi_scalar_expm(l: int, z: complex) -> complex:
    """phi_l(z) for one (complex) z from the (l+1)x(l+1) augmented exponential."""
    A = np.array([[z]], dtype=complex)
    return complex(phi_dense(A, np.array([1.0 + 0j]), l)[0])


def diag_closed_form(lam: np.ndarray, v: np.ndarray, l: int, h: float, phi_fn) -> np.ndarray:
    """w*_i = phi_l(h lambda_i) v_i, phi_fn(l, z) a scalar phi evaluator."""
    return np.array([phi_fn(l, h * x) * vi for x, vi in zip(lam, v)])


def advdiff_symbol_at(tx, ty, dx, dy, nu, ax, ay):
    """Fourier symbol of nu*Lap - ax*Dx - ay*Dy (centred, periodic) for the
    mode e^{i(theta_x i + theta_y j)} (theta may be arrays): the second
    difference gives (2 cos theta - 2)/dx^2 and the centred first difference
    i sin(theta)/dx."""
    lap = (2.0 * np.cos(tx) - 2.0) / dx ** 2 + (2.0 * np.cos(ty) - 2.0) / dy ** 2
    adv = 1j * (ax * np.sin(tx) / dx + ay * np.sin(ty) / dy)
    return nu * lap - adv


def advdiff_symbol(nx, ny, dx, dy, nu, ax, ay) -> np.ndarray:
    """Fourier symbol sigma[ky, kx] of every mode of an nx x ny grid."""
    tx = 2.0 * np.pi * np.fft.fftfreq(nx)  # theta_x = 2 pi k / nx
    ty = 2.0 * np.pi * np.fft.fftfreq(ny)
    TX, TY = np.meshgrid(tx, ty, indexing="xy")
    return advdiff_symbol_at(TX, TY, dx, dy, nu, ax, ay)


def fourier_closed_form(sigma: np.ndarray, v: np.ndarray, l: int, h: float) -> np.ndarray:
    """w* = IFFT(phi_l(h sigma) FFT(v)) for a circulant operator with symbol sigma."""
    ny, nx = sigma.shape
    V = np.fft.fft2(np.asarray(v).reshape(ny, nx))
    g = np.empty_like(V)
    for idx, s in np.ndenumerate(sigma):
        g[idx] = phi_scalar_expm(l, h * s)
    w = np.fft.ifft2(g * V)
    return w.real.ravel()


def neumann_diffusion_eigs(nx, ny, dx, dy, alpha) -> np.ndarray:
    """Eigenvalues lam[ky, kx] of alpha Lap (Neumann, cell-centred) on the DCT-II modes."""
    lx = -4.0 / dx ** 2 * np.sin(np.pi * np.arange(nx) / (2.0 * nx)) ** 2
    ly = -4.0 / dy ** 2 * np.sin(np.pi * np.arange(ny) / (2.0 * ny)) ** 2
    return alpha * (ly[:, None] + lx[None, :])


def dct_closed_form(lam: np.ndarray, v: np.ndarray, l: int, h: float) -> np.ndarray:
    """w* = IDCT(phi_l(h lam) DCT(v)) for an operator the 2D DCT-II diagonalises."""
    from scipy.fft import dctn, idctn
    ny, nx = lam.shape
    V = dctn(np.asarray(v, dtype=np.float64).reshape(ny, nx), type=2, norm="ortho")
    g = np.empty_like(V)
    for idx, x in np.ndenumerate(lam):
        g[idx] = phi_scalar_expm(l, h * x).real
    return idctn(g * V, type=2, norm="ortho").ravel()
