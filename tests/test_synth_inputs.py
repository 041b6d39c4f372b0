"""The seeded input generator: published SplitMix64 outputs, determinism,
index-addressability and the normal distribution's first moments."""
import numpy as np

import p2o_synth as S


def test_splitmix64_reference_outputs():
    # SplitMix64 started from state 0 (Steele et al. 2014; Vigna's reference
    # code) yields 0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F.
    z = (np.arange(1, 4, dtype=np.uint64) * S.GOLDEN)
    S._mix64_inplace(z, np.empty_like(z))
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                   0x06C45D188009454F]


def test_entries_are_index_addressable():
    env = S.envelope(6, 3.0, 0.5)
    full = S.blocks(7, 4, 9, 6, env)
    part = S.blocks(7, 4, 9, 6, env, k=[2, 5], s=[3], p=[0, 8])
    np.testing.assert_array_equal(part, full[np.ix_([2, 5], [3], [0, 8])])
    v = S.vector(3, S.ARRAY_M, 50)
    np.testing.assert_array_equal(S.vector(3, S.ARRAY_M, 10, offset=20), v[20:30])


def test_streams_differ_and_are_normal():
    a = S.vector(1, S.ARRAY_M, 200_000)
    b = S.vector(1, S.ARRAY_D, 200_000)
    c = S.vector(2, S.ARRAY_M, 200_000)
    assert not np.array_equal(a, b) and not np.array_equal(a, c)
    for x in (a, b, c):
        assert abs(x.mean()) < 0.01 and abs(x.std() - 1) < 0.01
        assert abs(np.mean(x ** 4) - 3) < 0.1


def test_uniform_ints_range_and_offsets():
    a = S.uniform_ints(4, S.ARRAY_SHAPES, 3000, 50, 600)
    assert a.min() >= 50 and a.max() <= 600 and len(set(a.tolist())) > 400
    np.testing.assert_array_equal(S.uniform_ints(4, S.ARRAY_SHAPES, 10, 50, 600, offset=5), a[5:15])
