"""Pins of the oracle's particle seeding (Section 2, "Sampling the particles")."""

import math

import numpy as np
import pytest
from scipy import stats

from oracle import seed as sd


@pytest.mark.parametrize("H,W,ppp,n", [(256, 256, 0.02, 1311), (1024, 1024, 0.05, 52429),
                                       (512, 512, 0.05, 13107), (2048, 2048, 0.1, 419430),
                                       (1, 1, 0.49, 0), (1, 1, 0.5, 1), (3, 5, 0.1, 2)])
def test_particle_count_rule(H, W, ppp, n):
    assert sd.particle_count(H, W, ppp) == n


def test_mask_excess_particles_by_zero_intensity():
    P = sd.seed_pair(128, 96, pair_id=3, seed=5, ppp=(0.01, 0.08), d_dist="uniform",
                     d_params=(1.0, 3.0))
    n_max, na = P["n_max"], P["n_active"]
    assert n_max == sd.particle_count(128, 96, 0.08)
    assert na == min(n_max, sd.particle_count(128, 96, P["ppp"]))
    assert 0.01 <= P["ppp"] <= 0.08
    assert np.all(P["I0"][:na] >= 0.8) and np.all(P["I0"][:na] <= 1.0)
    assert np.all(P["I0"][na:] == 0.0)
    assert len(P["x"]) == n_max


def test_ppp_draw_spans_range():
    pp = [sd.pair_scalars(64, 64, 0.005, 0.1, pid, 0)[0] for pid in range(4000)]
    assert min(pp) >= 0.005 and max(pp) <= 0.1
    assert stats.kstest((np.array(pp) - 0.005) / 0.095, "uniform").pvalue > 1e-3


def test_positions_uniform_over_image():
    H, W = 200, 300
    P = sd.seed_pair(H, W, pair_id=1, seed=2, ppp=(0.5, 0.5), d_dist="uniform", d_params=(1, 2))
    x, y = P["x"], P["y"]
    assert x.min() >= 0 and x.max() < W and y.min() >= 0 and y.max() < H
    h, _, _ = np.histogram2d(y, x, bins=(10, 10), range=((0, H), (0, W)))
    assert stats.chisquare(h.reshape(-1)).pvalue > 1e-3


def test_uniform_diameter_and_intensity_moments():
    P = sd.seed_pair(256, 256, 9, 4, ppp=(1.0, 1.0), d_dist="uniform", d_params=(1.5, 3.0),
                     I0=(0.8, 1.0), z=(-1.0, 1.0))
    n = len(P["d"])
    for v, a, b in ((P["d"], 1.5, 3.0), (P["I0"], 0.8, 1.0), (P["z"], -1.0, 1.0)):
        assert abs(v.mean() - (a + b) / 2) < 5 * (b - a) / math.sqrt(12 * n)
        assert abs(v.var() / ((b - a) ** 2 / 12) - 1) < 0.02
        assert v.min() >= a and v.max() < b


def test_clipped_normal_diameter_moments():
    mu, sig, lo, hi = 2.5, 0.5, 1.0, 5.0
    P = sd.seed_pair(512, 512, 2, 8, ppp=(1.0, 1.0), d_dist="normal", d_params=(mu, sig, lo, hi))
    d = P["d"]
    a, b = (lo - mu) / sig, (hi - mu) / sig
    Pa, Pb = stats.norm.cdf(a), stats.norm.cdf(b)
    mean = lo * Pa + hi * (1 - Pb) + mu * (Pb - Pa) + sig * (stats.norm.pdf(a) - stats.norm.pdf(b))
    assert abs(d.mean() - mean) < 5 * sig / math.sqrt(d.size)
    assert d.min() >= lo and d.max() <= hi
    # clipping at 1.0 = mu - 3 sigma takes the lower tail mass
    assert abs(np.mean(d == lo) - Pa) < 5 * math.sqrt(Pa / d.size) + 1e-5


def test_pairs_and_seeds_give_independent_particles():
    A = sd.seed_pair(64, 64, 0, 0, ppp=(0.1, 0.1), d_dist="uniform", d_params=(1, 2))
    B = sd.seed_pair(64, 64, 1, 0, ppp=(0.1, 0.1), d_dist="uniform", d_params=(1, 2))
    C = sd.seed_pair(64, 64, 0, 1, ppp=(0.1, 0.1), d_dist="uniform", d_params=(1, 2))
    assert not np.any(A["x"] == B["x"]) and not np.any(A["x"] == C["x"])


# ----------------------------------------------------------------------- binary32 mirror

def test_ra_exp_accuracy(ra):
    q = np.concatenate([np.linspace(0, 79.9, 20011), np.array([0.0, 1e-7, 0.34657, 0.34658, 18.0])])
    got = np.array([ra.E(float(np.float32(v))) for v in q])
    ref = np.exp(-q.astype(np.float32).astype(np.float64))
    assert ra.E(0.0) == 1.0
    assert np.max(np.abs(got / ref - 1)) < 4e-7
    assert ra.E(80.0) == 0.0 and ra.E(1e30) == 0.0 and ra.E(float("nan")) == 0.0


def test_ra_log_and_cos_accuracy(ra):
    u = (np.arange(1, 2 ** 24, 997, dtype=np.float64) * 2.0 ** -24)
    lg = np.array([ra.ln(float(v)) for v in u])
    assert np.max(np.abs(lg - np.log(u)) / np.maximum(1.0, np.abs(np.log(u)))) < 3e-7
    assert ra.ln(1.0) == 0.0
    c = np.array([ra.cos2pi(float(v)) for v in u])
    assert np.max(np.abs(c - np.cos(2 * np.pi * u))) < 3e-7
    assert ra.cos2pi(0.0) == 1.0 and ra.cos2pi(0.5) == -1.0 and ra.cos2pi(0.25) == 0.0


@pytest.mark.parametrize("d_dist,d_params,W", [("uniform", (1.5, 3.0), 256),
                                               ("normal", (2.5, 0.5, 1.0, 5.0), 1280)])
def test_ra_seed_matches_float64(ra, d_dist, d_params, W):
    H = 96
    P = sd.seed_pair(H, W, 7, 3, ppp=(0.02, 0.05), d_dist=d_dist, d_params=d_params)
    R = ra.seed_pair(H, W, P["n_max"], (0.02, 0.05), 7, 3, d_dist, d_params)
    assert R["n_active"] == P["n_active"] and R["ppp"] == P["ppp"]
    for k in ("x", "y", "z", "d", "I0"):
        ref = P[k]
        tol = 3e-7 * np.maximum(1.0, np.abs(ref))
        if k == "d" and d_dist == "normal":
            tol = 2e-6 * np.maximum(1.0, np.abs(ref))
        assert np.all(np.abs(R[k].astype(np.float64) - ref) <= tol), k
    if W == 256:  # power-of-two size: the binary32 product is exact
        assert np.array_equal(R["x"].astype(np.float64), P["x"])
