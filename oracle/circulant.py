"""Exact equilibrium on circulant graphs (test infrastructure only).

Section 2.1 writes L = U Lambda U^T. For a cycle C_n with every edge of weight
w the Laplacian is circulant, its eigenvectors are the Fourier modes and its
eigenvalues are lambda_k = 2w(1 - cos(2 pi k / n)). Section 2.2 gives Omega the
same eigenvectors with eigenvalues 1/(1 + lambda_k). Hence
  z = IFFT( FFT(s) / (1 + lambda_k) ),
and by Parseval each index of Proposition 1 is a weighted sum of |FFT(s)_k|^2:
  C    = (1/n) sum_k |s^_k|^2 / (1+lambda_k)^2
  D    = (1/n) sum_k lambda_k |s^_k|^2 / (1+lambda_k)^2
  C_I  = (1/n) sum_k lambda_k^2 |s^_k|^2 / (1+lambda_k)^2
  P    = C without the k = 0 term
  I_dc = (1/n) sum_k |s^_k|^2 / (1+lambda_k)
A 2-D torus C_a x C_b is the Cartesian product; its eigenvalues are sums of
the two cycles' eigenvalues over the 2-D Fourier modes.
"""
from __future__ import annotations

import numpy as np


def cycle_eigenvalues(n: int, w: float = 1.0) -> np.ndarray:
    k = np.arange(n)
    return 2.0 * w * (1.0 - np.cos(2.0 * np.pi * k / n))


def torus_eigenvalues(a: int, b: int, w: float = 1.0) -> np.ndarray:
    return cycle_eigenvalues(a, w)[:, None] + cycle_eigenvalues(b, w)[None, :]


def _spectral(shat2, lam, n):
    g = 1.0 / (1.0 + lam)
    c = float(np.sum(shat2 * g * g)) / n
    d = float(np.sum(lam * shat2 * g * g)) / n
    ci = float(np.sum(lam * lam * shat2 * g * g)) / n
    p = c - float((shat2 * g * g).flat[0]) / n
    idc = float(np.sum(shat2 * g)) / n
    return dict(internal_conflict=ci, disagreement=d, polarization=p, controversy=c, dc_index=idc)


def cycle_equilibrium(s: np.ndarray, w: float = 1.0) -> np.ndarray:
    n = s.shape[0]
    return np.real(np.fft.ifft(np.fft.fft(s) / (1.0 + cycle_eigenvalues(n, w))))


def cycle_indices(s: np.ndarray, w: float = 1.0) -> dict:
    n = s.shape[0]
    shat2 = np.abs(np.fft.fft(s)) ** 2
    return _spectral(shat2, cycle_eigenvalues(n, w), n)


def torus_equilibrium(s: np.ndarray, a: int, b: int, w: float = 1.0) -> np.ndarray:
    S = s.reshape(a, b)
    Z = np.real(np.fft.ifft2(np.fft.fft2(S) / (1.0 + torus_eigenvalues(a, b, w))))
    return Z.reshape(-1)


def torus_indices(s: np.ndarray, a: int, b: int, w: float = 1.0) -> dict:
    shat2 = np.abs(np.fft.fft2(s.reshape(a, b))) ** 2
    return _spectral(shat2, torus_eigenvalues(a, b, w), a * b)
