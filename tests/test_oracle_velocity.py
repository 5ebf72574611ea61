"""Pins of the oracle's IOS velocity codec (section 2.3; the conversion is a
linear reading, see oracle.vel_encode): what the definition fixes by itself.

* the round trip errs by at most s/2 (plus FP64 rounding), s = max deviation
  / 32767, and the largest deviation codes to +-32767 exactly;
* each bulk velocity is the mean of its cell's velocities: the deviations of
  a cell sum to zero (checked with an exactly rounded sum per cell, not the
  oracle's own summation); empty cells hold 0;
* a velocity field constant per bulk cell codes to q = 0 everywhere and
  decodes exactly; scaling every velocity by a power of two leaves the codes
  unchanged and scales the bulk field and the step; shifting every velocity
  by a constant shifts the bulk field by it and leaves the codes unchanged
  (up to rounding at exact ties)."""
import math

import numpy as np

import oracle
import synthetic


def _case(seed, n_fine=32, n=20000):
    x = synthetic.clustered(24, 0.3, 4, 512, 0.5 / n_fine, seed)[:, :n]
    q = oracle.quantize(x, n_fine)
    rng = np.random.default_rng(seed)
    v = (rng.standard_normal(q.shape) * 3.0).astype(np.float32)
    return q, v


def test_round_trip_within_half_a_step():
    q, v = _case(71)
    vq, vb, s, r = oracle.vel_encode(q, v, 32, 2)
    back = oracle.vel_decode(q, vq, vb, s, 32, 2)
    err = np.abs(back - v.astype(np.float64))
    bound = 0.5 * s * (1 + 1e-12) + 1e-12 * np.abs(v).max()
    assert np.all(err <= bound)
    assert np.abs(vq.astype(np.int64)).max() == 32767
    assert np.array_equal(vq, np.rint(r).astype(np.int16))


def test_bulk_is_the_cell_mean():
    q, v = _case(72)
    shift, nb = 3, 4
    _, vb, _, _ = oracle.vel_encode(q, v, 32, shift)
    cell = (q >> 15) >> shift
    key = (cell[2] * nb + cell[1]) * nb + cell[0]
    vbf = vb.reshape(3, -1)
    for c in range(nb ** 3):
        members = np.nonzero(key == c)[0]
        if members.size == 0:
            assert np.all(vbf[:, c] == 0.0)
            continue
        for d in range(3):
            resid = math.fsum(float(v[d, i]) - float(vbf[d, c]) for i in members)
            scale = math.fsum(abs(float(v[d, i])) for i in members)
            assert abs(resid) <= 1e-14 * scale + 1e-300


def test_cellwise_constant_field_codes_to_zero():
    q, _ = _case(73)
    shift, nb = 2, 8
    cell = (q >> 15) >> shift
    key = (cell[2] * nb + cell[1]) * nb + cell[0]
    table = np.arange(3 * nb ** 3, dtype=np.float32).reshape(3, -1) * np.float32(0.25)
    v = table[:, key]
    vq, vb, s, _ = oracle.vel_encode(q, v, 32, shift)
    assert np.all(vq == 0)
    assert np.array_equal(oracle.vel_decode(q, vq, vb, s, 32, shift), v.astype(np.float64))


def test_power_of_two_scaling_keeps_the_codes():
    q, v = _case(75)
    vq, vb, s, _ = oracle.vel_encode(q, v, 32, 2)
    vq2, vb2, s2, _ = oracle.vel_encode(q, v * np.float32(8.0), 32, 2)
    assert np.array_equal(vq, vq2)
    assert np.array_equal(vb * 8.0, vb2)
    assert s2 == 8.0 * s


def test_uniform_shift_moves_only_the_bulk():
    q, v = _case(74)
    vq, vb, s, _ = oracle.vel_encode(q, v, 32, 2)
    vq2, vb2, s2, _ = oracle.vel_encode(q, v + np.float32(8.0), 32, 2)
    full = vb.reshape(3, -1)[0] != 0
    assert np.allclose(vb2.reshape(3, -1)[:, full] - 8.0, vb.reshape(3, -1)[:, full], atol=1e-6)
    assert np.abs(vq2.astype(np.int64) - vq.astype(np.int64)).max() <= 1
