"""Seeded generator: determinism, shapes, and the population closed form."""
import hashlib
import math

import numpy as np

import gen


def test_tiny_deterministic_and_shaped():
    a = gen.make_ensemble("tiny", as_torch=False)
    b = gen.make_ensemble("tiny", as_torch=False)
    assert a.shape == (1, 64, 2048) and a.dtype == np.float32
    assert hashlib.sha256(a.tobytes()).hexdigest() == hashlib.sha256(b.tobytes()).hexdigest()
    assert gen.CONFIGS["tiny"].ref_v == 1160
    assert gen.CONFIGS["paper"].ref_v == 924125
    assert gen.CONFIGS["paper"].n_vertices == 1_760_000


def test_two_variable_generator():
    cfg = gen.CONFIGS["tiny"].__class__(**{**gen.CONFIGS["tiny"].__dict__, "n_vars": 2})
    x = gen.make_ensemble(cfg, as_torch=False)
    assert x.shape == (2, 64, 2048)
    assert np.all(np.abs(x[1]) < 1.0 + 1.0)          # tanh + small noise


def test_sample_covariance_converges_to_closed_form():
    cfg = gen.CONFIGS["tiny"].with_members(6000)
    x = gen.make_ensemble(cfg, as_torch=False)[0].astype(np.float64)
    v = np.array([0, 5, 300, 1160, 2047, 1000])
    w = np.array([1, 40, 301, 1160, 2000, 7])
    cov = np.array([np.mean((x[:, a] - x[:, a].mean()) * (x[:, b] - x[:, b].mean()))
                    for a, b in zip(v, w)])
    pop = gen.population_cov(cfg, v, w)
    scale = np.sqrt(gen.population_cov(cfg, v, v) * gen.population_cov(cfg, w, w))
    assert np.all(np.abs(cov - pop) / scale < 6.0 / math.sqrt(cfg.n_members) * 2)


def test_pairs_and_vertices_seeded():
    p = gen.random_pairs(100, 50, seed=1)
    assert p.shape == (50, 2) and p.dtype == np.int64 and p.min() >= 0 and p.max() < 100
    assert np.array_equal(p, gen.random_pairs(100, 50, seed=1))
