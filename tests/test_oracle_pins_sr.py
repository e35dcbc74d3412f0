"""Pins of the oracle's FP16 storage codes (CPU): the SplitMix64 stream and the two roundings.

Stochastic rounding is pinned by what defines it: the result is one of the two FP16 neighbours, its
expectation over the random integer is the input itself (exactly, for FP16 normal results), values on
the FP16 grid are left alone, and the probability of rounding up grows with the distance from the
lower neighbour.  The generator is pinned by its published first outputs and by the equality of its
counter form with the generator stepped one output at a time.
"""
import numpy as np
import pytest

from oracle import rounding as R


def test_splitmix64_published_outputs_and_counter_form():
    # first outputs of SplitMix64 started at state 0 (Steele, Lea & Flood 2014; the values every
    # implementation of the generator reproduces)
    assert R.splitmix64_sequence(0, 3) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    for seed in (0, 1, 12345, 2 ** 32 - 1, 0xDEADBEEFCAFEF00D):
        seq = R.splitmix64_sequence(seed, 1000)
        at = R.splitmix64_at(seed, np.arange(1000))
        assert [int(v) for v in at] == seq
    # output k far along the stream: the generator stepped k + 1 times
    k = 123456
    assert int(R.splitmix64_at(7, [k])[0]) == R.splitmix64_mix((7 + (k + 1) * R.GAMMA) & R.MASK64)


def test_node_random_ints_are_the_13_bit_fields_of_two_outputs():
    seed, nodes = 99, 70 * 45
    node = np.array([0, 1, 2, nodes - 1, 1234])
    level = np.array([0, 0, 5, 7, 1000])
    r = R.node_random_ints(seed, nodes, node, level)
    assert r.shape == (5, 9) and r.min() >= 0 and r.max() < 2 ** 13
    for n, t, row in zip(node, level, r):
        first = 2 * (int(t) * nodes + int(n))
        lo = R.splitmix64_mix((seed + (first + 1) * R.GAMMA) & R.MASK64)
        hi = R.splitmix64_mix((seed + (first + 2) * R.GAMMA) & R.MASK64)
        v = (hi << 64) | lo
        assert [int(x) for x in row] == [(v >> (13 * i)) & 0x1FFF for i in range(9)]
    # distinct levels and nodes draw distinct integers
    a = R.node_random_ints(seed, nodes, np.arange(nodes), 3)
    b = R.node_random_ints(seed, nodes, np.arange(nodes), 4)
    assert (a != b).mean() > 0.99
    # roughly uniform: each of the 13 bits is set about half the time
    bits = ((a[..., None] >> np.arange(13)) & 1).reshape(-1, 13).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 0.02)


def _fp32_values(rng, n, lo_exp, hi_exp):
    e = rng.uniform(lo_exp, hi_exp, n)
    v = (2.0 ** e * rng.choice([-1.0, 1.0], n)).astype(np.float32)
    return v


def test_stochastic_rounding_expectation_is_the_value_on_fp16_normals():
    rng = np.random.default_rng(1)
    v = _fp32_values(rng, 400, -14, 15.99)
    r = np.arange(2 ** 13)
    for x in v:
        out = R.f16_round_stochastic(np.full(r.size, x), r).astype(np.float64)
        assert np.all(np.isfinite(out))
        # the mean over all 2^13 integers is the FP32 input itself (the sum is exact in FP64)
        assert out.sum() / 2 ** 13 == float(x), x
        # the two FP16 neighbours only, the lower one for the larger integers
        lo, ulp = R.f16_floor_neighbours(np.array([abs(float(x))]))
        mags = np.abs(out)
        assert set(np.unique(mags)) <= {lo[0], lo[0] + ulp[0]}
        up = mags > lo[0]
        assert not np.any(up[1:] & ~up[:-1])  # monotone in r: up exactly for r below a threshold
        assert up.sum() == round((abs(float(x)) - lo[0]) / ulp[0] * 2 ** 13)
        assert np.all(np.sign(out) == np.sign(x))


def test_stochastic_rounding_in_the_fp16_subnormal_range():
    rng = np.random.default_rng(2)
    r = np.arange(2 ** 13)
    for x in list(_fp32_values(rng, 60, -40, -14.01)) + [np.float32(2.0 ** -30 * 3), np.float32(0.0)]:
        out = R.f16_round_stochastic(np.full(r.size, x), r).astype(np.float64)
        lo, ulp = R.f16_floor_neighbours(np.array([abs(float(x))]))
        assert ulp[0] == 2.0 ** -24
        # bias below 2^-12 of the FP16 spacing, exact where the distance is a multiple of 2^-13 spacings
        err = out.sum() / 2 ** 13 - float(x)
        assert abs(err) <= 2.0 ** -24 * 2.0 ** -12
        q = (abs(float(x)) - lo[0]) / ulp[0] * 2 ** 13
        if q == int(q):
            assert err == 0.0
        else:  # the bits below 2^-13 of the spacing are dropped: probability floor(q) / 2^13
            assert (np.abs(out) > lo[0]).sum() == int(q)
    # less than 2^-13 of the spacing above a grid value never rounds up
    x = np.float32(2.0 ** -24 * (5 + 0.3 / 2 ** 13))
    assert np.all(R.f16_round_stochastic(np.full(r.size, x), r).astype(np.float64) == 5 * 2.0 ** -24)


def test_values_on_the_fp16_grid_are_kept_and_round_to_nearest_is_one_neighbour():
    rng = np.random.default_rng(3)
    grid = rng.integers(-30000, 30000, 500).astype(np.float16)
    grid = grid[np.isfinite(grid)]
    r = rng.integers(0, 2 ** 13, grid.size)
    assert np.array_equal(R.f16_round_stochastic(grid.astype(np.float32), r), grid)
    assert np.array_equal(R.f16_round_stochastic(grid.astype(np.float32), np.full(grid.size, 8191)), grid)
    v = _fp32_values(rng, 2000, -20, 15.9)
    rne = R.f16_round_nearest(v).astype(np.float64)
    lo, ulp = R.f16_floor_neighbours(np.abs(v.astype(np.float64)))
    assert np.all((np.abs(rne) == lo) | (np.abs(rne) == lo + ulp))
    # on FP16 normals r = 0 rounds up whenever the value is off the grid, r = 2^13 - 1 never
    normal = np.abs(v.astype(np.float64)) >= 2.0 ** -14
    off = np.abs(v.astype(np.float64)) != lo
    up0 = np.abs(R.f16_round_stochastic(v, np.zeros(v.size, int)).astype(np.float64)) > lo
    assert np.array_equal(up0[normal], off[normal])
    up1 = np.abs(R.f16_round_stochastic(v, np.full(v.size, 8191)).astype(np.float64)) > lo
    assert not up1[normal].any()


def test_overflow_and_signs():
    r = np.arange(2 ** 13)
    x = np.float32(65520.0)  # half-way between 65504 and 65536: infinity for half of the integers
    out = R.f16_round_stochastic(np.full(r.size, x), r)
    assert np.isinf(out).sum() == 2 ** 12 and np.all(out[np.isfinite(out)] == 65504)
    assert np.all(np.isinf(R.f16_round_stochastic(np.full(4, np.float32(70000.0)), np.arange(4))))
    neg = R.f16_round_stochastic(np.full(r.size, np.float32(-1.0001)), r)
    assert np.all(neg < 0) and abs(neg.astype(np.float64).mean() + float(np.float32(1.0001))) < 1e-12
    assert np.signbit(R.f16_round_stochastic(np.array([np.float32(-0.0)]), [5])[0])


def test_f16s_value_and_decode():
    wref = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4) * 0.3
    g = np.linspace(0.0, 0.2, 9 * 6).reshape(9, 6)
    v = R.f16s_value(g, wref, 15)
    want = ((g.astype(np.float32) - wref.astype(np.float32)[:, None]) * np.float32(2 ** 15)).astype(np.float32)
    assert np.array_equal(v, want)
    code = R.f16_round_nearest(v)
    back = R.f16s_decode(code, wref, 15)
    # one decode is within half an FP16 spacing of g (the code is nearest)
    _, ulp = R.f16_floor_neighbours(np.abs(v.astype(np.float64)))
    assert np.all(np.abs(back - g) <= 0.5 * ulp * 2.0 ** -15 + 1e-9 * np.abs(g))
