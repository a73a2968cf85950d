"""Image-quality metrics of the evaluation (test infrastructure only, like the rest of ``oracle``).

Section 4.1 reports PSNR (and MS-SSIM) of rendered views against ground truth, and training uses
a structural-similarity term. Both are written here plainly in FP64 NumPy:

* PSNR = 10 log10(1 / MSE) over every pixel, channel and view, on images clamped to [0, 1]
  (peak value 1).
* SSIM (Wang, Bovik, Sheikh and Simoncelli, "Image quality assessment: from error visibility to
  structural similarity", 2004): at every position where an 11 x 11 window fits inside the image
  (no padding), with the window weights a normalised Gaussian of standard deviation 1.5 pixels,
    mu_x, mu_y      weighted means,
    s_xx, s_yy      weighted variances E[x^2] - mu_x^2, E[y^2] - mu_y^2,
    s_xy            weighted covariance E[xy] - mu_x mu_y,
    SSIM = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_xx + s_yy + C2)),
  C1 = 0.01^2, C2 = 0.03^2 (K1 = 0.01, K2 = 0.03 with a dynamic range of 1); the result is the
  mean over positions, channels and images.
"""
from __future__ import annotations

import numpy as np

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2


def psnr(a, b) -> float:
    """PSNR in dB of image batches of any matching shape, values clamped to [0, 1]."""
    x = np.clip(np.asarray(a, np.float64), 0.0, 1.0)
    y = np.clip(np.asarray(b, np.float64), 0.0, 1.0)
    mse = float(np.mean((x - y) ** 2))
    return 10.0 * np.log10(1.0 / mse) if mse > 0.0 else float("inf")


def gaussian_window(size: int = WINDOW, sigma: float = SIGMA) -> np.ndarray:
    """Normalised 2-D Gaussian weights (size x size), centred on the middle pixel."""
    r = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    w = np.exp(-(r[:, None] ** 2 + r[None, :] ** 2) / (2.0 * sigma * sigma))
    return w / w.sum()


def _windowed_mean(img: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Weighted mean of every fully contained window of the last two axes."""
    k = w.shape[0]
    view = np.lib.stride_tricks.sliding_window_view(img, (k, k), axis=(-2, -1))
    return np.einsum("...ij,ij->...", view, w)


def ssim_map(a, b) -> np.ndarray:
    """Per-position SSIM of image batches (..., H, W), FP64, over the valid window positions."""
    x = np.asarray(a, np.float64)
    y = np.asarray(b, np.float64)
    w = gaussian_window()
    mx, my = _windowed_mean(x, w), _windowed_mean(y, w)
    sxx = _windowed_mean(x * x, w) - mx * mx
    syy = _windowed_mean(y * y, w) - my * my
    sxy = _windowed_mean(x * y, w) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def ssim(a, b) -> float:
    """Mean SSIM of image batches (N, C, H, W) (or any (..., H, W))."""
    return float(np.mean(ssim_map(a, b)))
