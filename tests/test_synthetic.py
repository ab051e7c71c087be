"""The seeded input generators: stream definition and workload recipes."""
import numpy as np

from paper_1704_08907_amd import synthetic as syn


def test_splitmix64_published_vector():
    # first outputs of SplitMix64 seeded with 0 (Steele, Lea and Flood 2014)
    z = syn.SplitMix64(0).next_u64(3)
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_stream_is_counter_based():
    a = syn.SplitMix64(42)
    first = a.next_u64(5)
    rest = a.next_u64(3)
    b = syn.SplitMix64(42).next_u64(8)
    np.testing.assert_array_equal(np.concatenate([first, rest]), b)


def test_uniform_and_normal_ranges():
    r = syn.SplitMix64(7)
    u = r.uniform(100000)
    assert u.min() >= 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.01
    z = syn.SplitMix64(7).normal(100001)
    assert abs(z.mean()) < 0.02 and abs(z.std() - 1.0) < 0.02


def test_positions_inside_half_open_box():
    r = syn.SplitMix64(3)
    x = syn.uniform_positions(r, 20000, [0.0, -1.0], [1e-6, 1.0], "f32")
    assert x.dtype == np.float32
    assert np.all(x[:, 0] >= 0) and np.all(x[:, 0] < np.float32(1e-6))
    assert np.all(x[:, 1] >= -1) and np.all(x[:, 1] < 1)


def test_workload_shapes():
    w = syn.md_square()
    assert w.n == 1000 and w.systems[0].x.dtype == np.float64 and w.systems[0].cutoff == 0.1
    w = syn.spring_cube(4096)
    s = w.systems[0]
    assert s.x.shape == (4096, 3) and s.x.dtype == np.float32 and w.extra["gy"].shape == (4096, 3)
    sizes, _ = syn.batch_sizes()
    assert len(sizes) == 512 and min(sizes) >= 256 and max(sizes) <= 65536
    x, wt, sigma = syn.gaussian_square(1024)
    assert x.shape == (1024, 2) and wt.shape == (1024,) and sigma == 0.1
