"""The seeded input generators (seeded_inputs.py): deterministic, distinct
streams per operand, the documented value ranges and layouts.  Every parity
test, the benchmark and the oracle checks draw from them, so a drift here
would silently change what is compared."""
import math

import numpy as np
import pytest

import seeded_inputs as si


def test_seed_scheme():
    assert si.seed_for(2, "A") == 2000
    assert si.seed_for(2, "B") == 2001
    assert si.seed_for(4, "W2", 3) == 4036
    seeds = {si.seed_for(c, r, p) for c in range(6) for r in si.ROLE for p in range(50)}
    assert len(seeds) == 6 * len(si.ROLE) * 50          # no two operands share a stream


@pytest.mark.parametrize("gen", [si.uniform, si.log_uniform_signed, si.integers, si.dyadic, si.gaussian])
def test_same_seed_same_bits_other_seed_other_values(gen):
    a = gen((37, 53), 1234)
    b = gen((37, 53), 1234)
    c = gen((37, 53), 1235)
    assert a.dtype == np.float32
    assert a.tobytes() == b.tobytes()
    assert not np.array_equal(a, c)


def test_value_ranges():
    u = si.uniform((4000,), 1)
    assert u.min() >= -1.0 and u.max() <= 1.0 and abs(float(u.mean())) < 0.05
    lu = np.abs(si.log_uniform_signed((4000,), 2).astype(np.float64))
    assert lu.min() >= 1e-3 * (1 - 1e-6) and lu.max() <= 1e3 * (1 + 1e-6)
    assert 0.4 < float(np.mean(si.log_uniform_signed((4000,), 2) < 0)) < 0.6
    it = si.integers((4000,), 3)
    assert set(np.unique(it)) == set(range(-8, 9))
    dy = si.dyadic((4000,), 4).astype(np.float64)
    m, e = np.frexp(dy[dy != 0])
    assert np.all((m * 2 ** 5) == np.round(m * 2 ** 5))   # at most 4 significant bits (+ sign)


def test_float32_rounding_is_round_to_nearest_even_of_the_float64_draw():
    rng = np.random.default_rng(99)
    d = rng.uniform(-1.0, 1.0, size=1000)
    assert np.array_equal(si.uniform((1000,), 99), d.astype(np.float32))


def test_batched_sizes():
    sizes = si.batched_sizes(512, si.seed_for(4, "A"))
    assert sizes == si.batched_sizes(512, si.seed_for(4, "A"))
    flat = np.array(sizes).reshape(-1)
    assert len(sizes) == 512 and flat.min() >= 32 and flat.max() <= 2048
    assert np.all(flat % 8 == 0)
    # log-uniform on [32, 2048]: the median sits near the geometric mean 256
    assert 180 < float(np.median(flat)) < 360
    assert abs(float(np.mean(np.log(flat))) - math.log(256)) < 0.2


def test_store_layouts_and_padding():
    x = np.arange(12, dtype=np.float32).reshape(3, 4)
    buf, ld = si.store(x, "N", 6)
    assert ld == 6 and buf.size == 18
    assert np.array_equal(buf.reshape(3, 6)[:, :4], x) and np.isnan(buf.reshape(3, 6)[:, 4:]).all()
    buf, ld = si.store(x, "T")
    assert ld == 3 and np.array_equal(buf.reshape(4, 3), x.T)
    with pytest.raises(ValueError):
        si.store(x, "N", 3)


def test_sample_indices():
    I, J = si.sample_indices(100, 70, 64, 5)
    I2, J2 = si.sample_indices(100, 70, 64, 5)
    assert np.array_equal(I, I2) and np.array_equal(J, J2)
    assert I.min() >= 0 and I.max() < 100 and J.min() >= 0 and J.max() < 70
    pos = set(zip(I.tolist(), J.tolist()))
    assert len(pos) == len(I) and {(0, 0), (0, 69), (99, 0), (99, 69)} <= pos
