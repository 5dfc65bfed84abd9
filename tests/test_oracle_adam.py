"""Pins of the fp64 Adam step and of the serving target generator.

Adam (Kingma and Ba 2015, Algorithm 1): with bias correction, the first step
from zero moments moves every parameter by lr * g / (|g| + eps), i.e. by
exactly lr * sign(g) when eps = 0; a constant gradient keeps the corrected
moments at g and g^2 at every step, so t steps move by t * lr * sign(g). A
dropped bias correction, a swapped beta or a squared/unsquared mix-up breaks
one of these.

SplitMix64 (Steele, Lea and Flood 2014): the published output sequence for
the seed 1234567.
"""
import numpy as np

import oracle
from paper_2401_05345_amd import scenegen as sg


def test_first_step_is_signed_lr():
    rng = np.random.default_rng(0)
    p, g = rng.standard_normal(1000), rng.standard_normal(1000)
    z = np.zeros(1000)
    p1, m1, v1 = oracle.adam_step(p, g, z, z, 1, lr=1e-3, eps=0.0)
    assert np.allclose(p1, p - 1e-3 * np.sign(g), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)


def test_constant_gradient_moves_linearly():
    g = np.array([3.0, -0.5, 1e-3, -7.0])
    p, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    for t in range(1, 51):
        p, m, v = oracle.adam_step(p, g, m, v, t, lr=2e-3, beta1=0.9, beta2=0.999, eps=0.0)
    assert np.allclose(p, -50 * 2e-3 * np.sign(g), rtol=1e-12, atol=1e-14)


def test_eps_and_zero_gradient():
    p = np.array([1.0, 2.0])
    p1, _, _ = oracle.adam_step(p, np.zeros(2), np.zeros(2), np.zeros(2), 1, eps=1e-8)
    assert np.array_equal(p1, p)
    # |g| = eps halves the step
    p1, _, _ = oracle.adam_step(np.zeros(1), np.array([1e-8]), np.zeros(1), np.zeros(1), 1, lr=1.0, eps=1e-8)
    assert np.isclose(p1[0], -0.5, rtol=1e-9)


def test_splitmix64_published_sequence():
    out = sg.splitmix64(1234567, np.arange(5, dtype=np.uint64))
    assert [int(x) for x in out] == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                                      4593380528125082431, 16408922859458223821]


def test_request_target_is_uniform():
    t = sg.request_target(42, 64, 80)
    assert t.shape == (3, 64, 80) and t.dtype == np.float32
    assert t.min() >= 0.0 and t.max() < 1.0
    assert abs(t.mean() - 0.5) < 0.01
    assert np.array_equal(t, sg.request_target(42, 64, 80)) and not np.array_equal(t, sg.request_target(43, 64, 80))
