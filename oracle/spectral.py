"""Spectral grid conventions of the oracle (FP64).

Reading of the modal decomposition (Sec. 3.1, basis equations and the
surface-potential decomposition of Sec. 3.1.2): a real field on the periodic
domain [0,Lx) x [0,Ly) is f(x,y) = sum_k fhat(k) exp(i k.x) over wavevectors
k = (2 pi p / Lx, 2 pi q / Ly), p in [-Nx/2, Nx/2), q in [-Ny/2, Ny/2), with
Hermitian symmetry fhat(-k) = conj(fhat(k)).  Only the half spectrum
p in [0, Nx/2] is stored, as [Ny][Nx/2+1] with x fastest; fhat is the DFT
divided by the number of points; grid spacing is L/N.  Nyquist modes
(p = Nx/2, q = Ny/2) are kept at zero.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def next_5smooth_even(n: int) -> int:
    v = max(2, n + (n & 1))
    while True:
        w = v
        for f in (2, 3, 5):
            while w % f == 0:
                w //= f
        if w == 1:
            return v
        v += 2


def next_2k_or_3x2k(n: int) -> int:
    """Smallest 2^a or 3 2^a (a >= 1) at or above n."""
    best = None
    for b in (2, 6):
        c = b
        while c < n:
            c *= 2
        best = c if best is None else min(best, c)
    return best


@dataclass
class Grid:
    """Mode grid, depth and padding of one realisation."""
    nx: int
    ny: int
    lx: float
    ly: float
    depth: float  # <= 0 means infinite depth
    order_m: int = 3
    dealias: int = 1
    g: float = 1.0
    rho: float = 1.0

    @property
    def dim(self) -> int:
        return 2 if self.ny == 1 else 3

    @property
    def nxh(self) -> int:
        return self.nx // 2 + 1

    @property
    def deep(self) -> bool:
        return not (self.depth > 0)

    def padded(self) -> tuple[int, int]:
        """Product grid: the (M+1)/2 rule, Px >= (M+1) Nx / 2, so products of
        up to M band-limited factors alias nothing into the kept band.  The
        length at or above the rule is a choice (dealias = 1: the next even
        2/3/5-smooth length; 2: the next 2^a or 3 2^a); products with more
        factors than the rule covers alias by amounts that depend on it, so a
        comparison takes the length of the computation it checks."""
        if not self.dealias:
            return self.nx, self.ny
        nxt = next_2k_or_3x2k if self.dealias == 2 else next_5smooth_even
        px = nxt(-(-(self.order_m + 1) * self.nx // 2))
        py = 1 if self.ny == 1 else nxt(-(-(self.order_m + 1) * self.ny // 2))
        return px, py

    # wavenumbers on the half spectrum -------------------------------------------------
    def kx(self) -> np.ndarray:
        return 2 * math.pi * np.arange(self.nxh) / self.lx

    def ky(self) -> np.ndarray:
        q = np.arange(self.ny)
        qs = np.where(q < (self.ny + 1) // 2, q, q - self.ny) if self.ny > 1 else q
        return 2 * math.pi * qs / self.ly

    def kvec(self):
        KX, KY = np.meshgrid(self.kx(), self.ky(), indexing="xy")
        return KX, KY, np.sqrt(KX * KX + KY * KY)

    def dz_symbol(self, j: int) -> np.ndarray:
        """Symbol of the j-th vertical derivative at z = 0 of a mode with the
        cosh(k(z+h))/cosh(kh) basis (Sec. 3.1, basis of the potential):
        k^j tanh(kh) for odd j, k^j for even j; deep water k^j."""
        _, _, K = self.kvec()
        s = K ** j
        if j % 2 == 1 and not self.deep:
            s = s * np.tanh(K * self.depth)
        return s

    def nyquist_mask(self) -> np.ndarray:
        m = np.ones((self.ny, self.nxh))
        m[:, -1] = 0.0 if self.nx % 2 == 0 else 1.0
        if self.ny > 1:
            m[self.ny // 2, :] = 0.0
        return m

    # transforms ---------------------------------------------------------------------
    def to_phys(self, fh: np.ndarray, shape: tuple[int, int] | None = None) -> np.ndarray:
        """Physical values on the (padded) product grid [Py][Px] from a half
        spectrum, by zero-padding the spectrum and an inverse real FFT."""
        px, py = shape if shape is not None else self.padded()
        big = np.zeros((py, px // 2 + 1), dtype=np.complex128)
        hx = self.nx // 2  # keep p in [0, Nx/2) (Nyquist is zero anyway)
        if self.ny == 1:
            big[0, :hx] = fh[0, :hx]
        else:
            hy = self.ny // 2
            big[:hy, :hx] = fh[:hy, :hx]
            big[py - (self.ny - hy - 1):, :hx] = fh[hy + 1:, :hx]
        return np.fft.irfft2(big, s=(py, px)) * (px * py)

    def to_spec(self, f: np.ndarray) -> np.ndarray:
        """Half spectrum of physical values on a product grid, truncated to
        the mode grid; Nyquist modes zeroed."""
        py, px = f.shape
        big = np.fft.rfft2(f) / (px * py)
        out = np.zeros((self.ny, self.nxh), dtype=np.complex128)
        hx = self.nx // 2
        if self.ny == 1:
            out[0, :hx] = big[0, :hx]
        else:
            hy = self.ny // 2
            out[:hy, :hx] = big[:hy, :hx]
            out[hy + 1:, :hx] = big[py - (self.ny - hy - 1):, :hx]
        return out

    def full_spectrum(self, fh: np.ndarray):
        """All modes (signed p, q) with amplitudes, Hermitian-completed.
        Returns (p, q, amp) flat arrays."""
        ps, qs, amps = [], [], []
        q_signed = np.arange(self.ny)
        if self.ny > 1:
            q_signed = np.where(q_signed < self.ny // 2, q_signed, q_signed - self.ny)
        for p in range(self.nx // 2 + 1):
            col = fh[:, p]
            for qi in range(self.ny):
                a = col[qi]
                if a == 0:
                    continue
                ps.append(p); qs.append(q_signed[qi]); amps.append(a)
                if p != 0 and not (2 * p == self.nx):
                    ps.append(-p); qs.append(-q_signed[qi]); amps.append(np.conj(a))
                elif p == 0:
                    pass  # the p = 0 column carries both signs of q already
        return np.array(ps), np.array(qs), np.array(amps)

    def node_coords(self, shape=None):
        px, py = shape if shape is not None else (self.nx, self.ny)
        x = self.lx * np.arange(px) / px
        y = self.ly * np.arange(py) / py if self.ny > 1 else np.zeros(1)
        return x, y

    def integrate(self, f: np.ndarray) -> float:
        """Integral over the domain of physical values on a uniform grid
        (exact for band-limited products that do not alias)."""
        py, px = f.shape
        return float(f.sum() * (self.lx / px) * ((self.ly / py) if self.ny > 1 else 1.0))
