"""Oracle (test infrastructure only): the periodic grid and its discrete
transforms, paper Sec. 2.3.

Real grid: r_n = (n_x L_x/N_x, n_y L_y/N_y, n_z L_z/N_z), n_mu = 0..N_mu-1
(the paper prints the closed range [0, N_mu]; the half-open range is the
periodic grid).  Reciprocal box: k = (m_x/L_x, m_y/L_y, m_z/L_z) with
m_mu in [-N_mu/2+1, N_mu/2] (ordinary frequency, no 2 pi).

Discrete forms of the unitary ordinary-frequency transform pair (their
normalisation fixed by the discretised Hartree energy of Sec. 2.6.4):
    f^(k) = (|Omega|/N_g) sum_r f(r) exp(-2 pi i k.r)
    f(r)  = Re[ (1/|Omega|) sum_{k in box} f^(k) exp(2 pi i k.r) ]
All spectra here live on the FULL box (N_x x N_y x N_z complex), stored in
numpy FFT index order; the Re of the box sum is taken literally.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def box_indices(N: int) -> np.ndarray:
    """Integer m for FFT slot i: m = i for i <= N/2, else i - N (box [-N/2+1, N/2])."""
    i = np.arange(N)
    return np.where(i <= N // 2, i, i - N)


@dataclass
class Grid:
    cell: tuple  # (Lx, Ly, Lz) bohr
    shape: tuple  # (Nx, Ny, Nz)

    def __post_init__(self):
        self.cell = tuple(float(c) for c in self.cell)
        self.shape = tuple(int(n) for n in self.shape)
        for n in self.shape:
            if n % 2:
                raise ValueError("grid sizes must be even")
        self.volume = self.cell[0] * self.cell[1] * self.cell[2]
        self.ng = self.shape[0] * self.shape[1] * self.shape[2]
        self.dv = self.volume / self.ng
        m = [box_indices(n) for n in self.shape]
        self.m = np.meshgrid(*m, indexing="ij")  # integer box indices
        self.k = [self.m[a] / self.cell[a] for a in range(3)]  # ordinary-frequency k
        self.k2 = self.k[0] ** 2 + self.k[1] ** 2 + self.k[2] ** 2
        self.kabs = np.sqrt(self.k2)
        self.nonzero = self.k2 > 0.0

    def points(self) -> np.ndarray:
        """Real-space grid points, shape (Nx, Ny, Nz, 3)."""
        ax = [np.arange(n) * (L / n) for n, L in zip(self.shape, self.cell)]
        X = np.meshgrid(*ax, indexing="ij")
        return np.stack(X, axis=-1)

    # --- transforms (Sec. 2.3) ---
    def forward(self, f: np.ndarray) -> np.ndarray:
        return self.dv * np.fft.fftn(f)

    def inverse(self, F: np.ndarray) -> np.ndarray:
        return np.real(np.fft.ifftn(F) * (self.ng / self.volume))

    def integrate(self, f: np.ndarray) -> float:
        return float(self.dv * np.sum(f))

    def box_sum(self, F: np.ndarray) -> float:
        """(1/|Omega|) Re sum_{k in box} F(k), the discrete form of int dk."""
        return float(np.real(np.sum(F)) / self.volume)
