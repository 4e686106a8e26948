"""The q-weighted loss of the LITE surrogate (the Gamma block weighted in the MSE of
standardised targets, Sec. "Case Study 2: 2D Lid-Driven Cavity") is
realised by the target scaler alone: dividing the Gamma block's scale by sqrt(w) makes
the plain MSE of the re-standardised targets equal to the weighted MSE of the original
ones, for any prediction.  Host-side check of that identity and of scalers_from_stats
(the column statistics themselves come from the library's kernel on the GPU)."""
import math

import numpy as np
import torch

from paper_2606_15622_amd import learned as L


def test_scaler_realises_the_weighted_mse():
    rng = np.random.default_rng(5)
    feats = torch.tensor(rng.standard_normal((500, 32)), dtype=torch.float32)
    tg = torch.tensor(rng.standard_normal((500, 16)) * 3.0 + 1.0, dtype=torch.float32)
    tg[:, 9:] = 0.0
    w = 4.0
    xm, xs = feats.double().mean(0).numpy(), feats.double().std(0).numpy()
    tm, ts = tg.double().mean(0).numpy(), tg.double().std(0).numpy()
    _, _, ym, ys = L.scalers_from_stats(xm, xs, tm, ts)
    _, _, ymw, ysw = L.scalers_from_stats(xm, xs, tm, ts, gamma_weight=w)
    np.testing.assert_allclose(ysw[6:9].numpy(), ys[6:9].numpy() / math.sqrt(w), rtol=1e-6)
    np.testing.assert_array_equal(ysw[:6].numpy(), ys[:6].numpy())
    np.testing.assert_array_equal(ymw.numpy(), ym.numpy())
    y = tg[:, :9].double().numpy()
    pred = y + rng.standard_normal(y.shape)            # any prediction in target units
    m, s, sw = ym[:9].double().numpy(), ys[:9].double().numpy(), ysw[:9].double().numpy()
    weights = np.array([1.0] * 6 + [w] * 3)
    weighted = np.mean(np.sum(weights * ((pred - y) / s) ** 2, 1))
    plain = np.mean(np.sum(((pred - m) / sw - (y - m) / sw) ** 2, 1))
    assert abs(plain - weighted) <= 1e-5 * weighted
