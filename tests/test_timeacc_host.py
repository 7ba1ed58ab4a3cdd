"""Host helpers of the time versus accuracy harness (CPU only)."""
import numpy as np

from paper_1511_05174_amd import timeacc


def test_psnr_definition():
    x = np.array([[1.0, -2.0], [0.5, 0.0]])
    xh = x + np.array([[0.1, 0.0], [0.0, -0.1]])
    mse = 0.02 / 4
    assert np.isclose(timeacc.psnr_db(x, xh), 10 * np.log10(4.0 / mse))


def test_noise_reaches_the_stated_snr():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((4000, 64)) * 3.0
    y = timeacc.add_noise(x, 15.0, np.random.default_rng(1))
    snr = 10 * np.log10(np.mean(x * x) / np.mean((y - x) ** 2))
    assert abs(snr - 15.0) < 0.1
