"""Pins of the oracle's Gaussian-sum approximation of 1/r (eq. 2.2) and its frozen constants."""
import math

import numpy as np
import pytest

from oracle import constants, sinc
from workloads import configs


@pytest.mark.parametrize("cfg, bound", [(configs.CONFIG1, 3.2e-8), (configs.CONFIG2, 1.3e-9),
                                        (configs.CONFIG4, 1.8e-9)])
def test_radial_sweep_against_closed_form(cfg, bound):
    """1/r = (2/sqrt(pi)) int exp(-r^2 t^2) dt: the folded sum matches 1/r on [1 A, L_s]."""
    t, w = sinc.sinc_table(cfg.M, cfg.h_M, cfg.L_s)
    r = np.geomspace(1.0, cfg.L_s, 4000)
    rel = np.abs(r * sinc.gaussian_sum(r, t, w) - 1.0)
    assert rel.max() <= bound
    # the error is quadrature error, not a loose fit: it is much smaller in the middle of the range
    assert np.median(rel) < bound


def test_fold_matches_unfolded_symmetric_sum():
    """Folding k and -k: the unfolded trapezoid sum over k=-M..M gives the same g(r)."""
    cfg = configs.CONFIG1
    t, w = sinc.sinc_table(cfg.M, cfg.h_M, cfg.L_s)
    k = np.arange(-cfg.M, cfg.M + 1, dtype=float)
    tk = np.sinh(k * cfg.h_M) / cfg.L_s
    ak = cfg.h_M * np.cosh(k * cfg.h_M) / (math.sqrt(math.pi) * cfg.L_s)
    r = np.array([0.5, 1.0, 3.0, 10.0, 40.0])
    unfolded = np.array([np.sum(ak * np.exp(-(tk * rr) ** 2)) for rr in r])
    assert np.allclose(sinc.gaussian_sum(r, t, w), unfolded, rtol=1e-14, atol=0)
    assert t.shape == (cfg.M + 1,) and np.all(w > 0) and np.all(np.diff(t) > 0)


def test_widest_terms_are_long_range():
    """Range separation (eq. 2.4): long terms are the widest, short terms vanish beyond r_c."""
    cfg = configs.CONFIG2
    t, w = sinc.sinc_table(cfg.M, cfg.h_M, cfg.L_s)
    (tl, wl), (ts, ws) = sinc.split(t, w, cfg.K_long)
    assert tl.max() < ts.min()
    r = np.linspace(cfg.r_cut, 3 * cfg.r_cut, 200)
    assert np.all(r * sinc.gaussian_sum(r, ts, ws) <= 1.0000001e-16)
    # just inside the cutoff the short part is still above the threshold
    r_in = cfg.r_cut * (1 - 1e-6)
    assert r_in * sinc.gaussian_sum(np.array([r_in]), ts, ws)[0] > 1e-16 * 0.99


@pytest.mark.slow
@pytest.mark.parametrize("cfg", [configs.CONFIG1, configs.CONFIG2, configs.CONFIG3, configs.CONFIG4])
def test_frozen_constants_rederived(cfg):
    assert cfg.L_s == pytest.approx(2.0 * math.sqrt(3.0) * cfg.b, rel=1e-15)
    assert constants.optimal_step(cfg.M, cfg.b) == cfg.h_M
    assert constants.short_cutoff(cfg.M, cfg.h_M, cfg.L_s, cfg.K_long) == pytest.approx(cfg.r_cut, rel=1e-12)


@pytest.mark.slow
@pytest.mark.parametrize("i", range(len(configs.CONFIG5_PROTEINS)))
def test_serving_constants_rederived(i):
    """Config 5 proteins: box from the radius rule, grid from the size rule, h_M and r_c re-derived."""
    N, b, n, h_M, L_s, r_cut = configs.CONFIG5_PROTEINS[i]
    c = configs.config5_protein(i)
    r_lig = 6.0 * (configs.CONFIG5_L[1] / 50.0) ** (1.0 / 3.0)
    assert b == math.ceil(c.protein_radius + 15.0 + r_lig + 2.0)
    b_max = max(p[1] for p in configs.CONFIG5_PROTEINS)
    assert n == 1 << math.ceil(math.log2(16384 * b / b_max))
    assert L_s == pytest.approx(2.0 * math.sqrt(3.0) * b, rel=1e-15)
    assert constants.optimal_step(32, b) == h_M
    assert constants.short_cutoff(32, h_M, L_s, 22) == pytest.approx(r_cut, rel=1e-12)
