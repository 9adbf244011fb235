"""The seeded input recipe (CPU only)."""
import numpy as np
import pytest

import synth

MASK = (1 << 64) - 1


def _sequential_splitmix64(seed, count):
    """SplitMix64 as published: add the golden gamma to the state, then
    finalise; plain Python integers, one value at a time."""
    state = seed & MASK
    out = []
    for _ in range(count):
        state = (state + 0x9E3779B97F4A7C15) & MASK
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
        out.append(z ^ (z >> 31))
    return out


def test_counter_form_matches_sequential_generator():
    for seed in (0, 1, 12416, (1 << 64) - 1):
        seq = _sequential_splitmix64(seed, 50)
        ctr = synth.splitmix64_outputs(seed, np.arange(1, 51, dtype=np.uint64))
        assert [int(v) for v in ctr] == seq


def test_uniform_range_and_streams_differ():
    idx = np.arange(100000, dtype=np.uint64)
    a = synth.uniform01(12416, 0, idx)
    b = synth.uniform01(12416, 1, idx)
    assert a.min() >= 0.0 and a.max() < 1.0
    assert abs(a.mean() - 0.5) < 0.01
    assert not np.array_equal(a, b)
    # 53-bit grid: every value times 2^53 is an integer
    assert np.all(np.floor(a * 2.0 ** 53) == a * 2.0 ** 53)


def test_boundary_field_layout():
    n = (5, 4, 3)
    u = synth.boundary_field(n, seed=3)
    assert u.shape == (5, 6, 7)
    assert np.all(u[1:-1, 1:-1, 1:-1] == 0.0)
    flat_idx = np.arange(u.size, dtype=np.uint64).reshape(u.shape)
    ref = synth.uniform01(3, 0, flat_idx.ravel()).reshape(u.shape)
    shell = np.ones(u.shape, bool)
    shell[1:-1, 1:-1, 1:-1] = False
    assert np.array_equal(u[shell], ref[shell])


def test_source_field_and_slabs():
    n = (6, 5, 7)
    b = synth.source_field(n, seed=8)
    assert b.shape == (9, 7, 8)
    inner = b[1:-1, 1:-1, 1:-1]
    assert inner.min() >= -1.0 and inner.max() < 1.0
    shell = np.ones(b.shape, bool)
    shell[1:-1, 1:-1, 1:-1] = False
    assert np.all(b[shell] == 0.0)
    assert np.array_equal(synth.source_slab(n, 2, 6, seed=8), b[2:6])


def test_uneven_cuts_properties():
    for axis in range(3):
        cuts = synth.uneven_cuts(768, 32, 160, seed=12416, axis=axis)
        assert sum(cuts) == 768
        assert all(32 <= c <= 160 for c in cuts)
    assert synth.uneven_cuts(100, 32, 160) == [100]


def test_serving_requests_recipe():
    reqs = synth.serving_requests(200, 10.0, seed=1)
    n = np.array([r["n"] for r in reqs])
    assert n.min() >= 32 and n.max() <= 384
    t = np.array([r["arrival"] for r in reqs])
    assert np.all(np.diff(t) >= 0) and t[0] == 0.0
    assert {r["precision"] for r in reqs} == {"f32", "f64"}


@pytest.mark.parametrize("n", [(7, 5, 4), (16, 9, 12)])
def test_field_box_is_a_slice_of_the_whole_field(n):
    g = synth.boundary_field(n, seed=77)
    b = synth.source_field(n, seed=77)
    P = g.shape
    rng = np.random.default_rng(3)
    for _ in range(6):
        lo = [int(rng.integers(0, P[a] - 1)) for a in range(3)]
        hi = [int(rng.integers(lo[a] + 1, P[a] + 1)) for a in range(3)]
        sl = tuple(slice(l, h) for l, h in zip(lo, hi))
        assert np.array_equal(synth.field_box(n, 0, lo, hi, seed=77), g[sl])
        assert np.array_equal(synth.field_box(n, 1, lo, hi, seed=77), b[sl])
    full = [0, 0, 0], list(P)
    assert np.array_equal(synth.field_box(n, 0, *full, seed=77), g)
    with pytest.raises(ValueError):
        synth.field_box(n, 0, [0, 0, 0], [P[0] + 1, P[1], P[2]])
