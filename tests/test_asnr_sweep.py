"""The aSNR metric of the Sec. 4.3 quality study and one small point of the sweep."""
import numpy as np
import pytest

import asnr_sweep as S


def test_asnr_metric_closed_form():
    # x_hat = (1 - 10^(-s/20)) x gives SNR_l = s in every channel, whatever x is
    rng = np.random.default_rng(3)
    X = rng.uniform(0.1, 2.0, (4, 8, 8))
    for s in (3.0, 20.0, 41.5):
        assert abs(S.asnr(X, X * (1.0 - 10.0 ** (-s / 20.0))) - s) < 1e-9
    # the mean is over channels, each with its own SNR
    Xh = X.copy()
    Xh[0] *= 1.0 - 10.0 ** (-10.0 / 20.0)
    Xh[1:] *= 1.0 - 10.0 ** (-30.0 / 20.0)
    assert abs(S.asnr(X, Xh) - (10.0 + 3 * 30.0) / 4) < 1e-9


def test_sweep_config_sampling_rate():
    cfg = S.sweep_config(15, 0.05, 40.0, n=256)
    assert cfg.m_per_chan == round(0.05 * 256 * 256) and cfg.L == 15 and cfg.n_src < cfg.L and cfg.n_lines > 0


@pytest.mark.gpu
def test_sweep_point_runs_every_method():
    cfg = S.sweep_config(5, 0.3, 40.0, n=64)
    res = S.run_point(cfg, S.METHODS, iters=120, reweights=2, log=lambda *a: None)
    assert set(res) == set(S.METHODS)
    for m, v in res.items():
        assert np.isfinite(v) and v > 0.0, (m, v)
