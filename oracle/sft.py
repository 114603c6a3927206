"""Reference of the data preparation (Sec. 2): strain -> Hann-windowed short
Fourier transforms -> normalised power.

TEST INFRASTRUCTURE ONLY: only the tests use this module; it shares no code
with the library.  FP64 throughout.

- Segment j is samples [j N, (j + 1) N) of the strain (no overlap), N = T_sft fs.
- Hann window w_n = 1/2 - 1/2 cos(2 pi n / N), n = 0 .. N-1 (periodic form).
- X_k = sum_n x_n w_n e^{-2 pi i k n / N} (numpy's real FFT as the library
  routine), P_k = |X_k|^2.
- Noise floor: under Gaussian noise P_k is exponential with mean S_k, whose
  median is S_k ln 2, so S_k is estimated as the median of P over the
  `window` bins centred on k divided by ln 2; rho_k = P_k / S_k.
"""
import math

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view


def hann(N):
    n = np.arange(N, dtype=np.float64)
    return 0.5 - 0.5 * np.cos(2.0 * np.pi * n / N)


def power(strain, n_fft):
    """P[j][k] for k = 0 .. n_fft/2 of every whole segment (FP64)."""
    x = np.asarray(strain, np.float64)
    n_seg = x.size // n_fft
    seg = x[:n_seg * n_fft].reshape(n_seg, n_fft) * hann(n_fft)[None, :]
    X = np.fft.rfft(seg, axis=1)
    return X.real * X.real + X.imag * X.imag


def normalise(P, k_lo, n_bins, window):
    """rho[j][b] = P[j][k] ln2 / median(P[j][k - h .. k + h]), k = k_lo + b,
    h = window // 2 (window odd)."""
    assert window % 2 == 1
    h = window // 2
    band = P[:, k_lo - h:k_lo + n_bins + h]
    med = np.median(sliding_window_view(band, window, axis=1), axis=2)
    # a window whose median is 0 (zero strain) carries no noise-floor estimate: rho = 0
    safe = np.where(med > 0.0, med, 1.0)
    return np.where(med > 0.0, P[:, k_lo:k_lo + n_bins] * math.log(2.0) / safe, 0.0)


def normalised_power(strain, n_fft, k_lo, n_bins, window):
    return normalise(power(strain, n_fft), k_lo, n_bins, window)
