"""Host side of streamed batches: chunking by whole segments and the CPU
replica of the device row generator."""
import numpy as np

from paper_1701_08547_amd import streamed, workloads


def test_chunk_bounds_whole_segments():
    seg = np.array([0, 5, 10, 100, 101, 150], np.int64)
    # segments of 5, 5, 90, 1 and 49 evaluations, chunks of at most 20 unless
    # a single segment is longer
    assert streamed.chunk_bounds(seg, 20) == [(0, 2), (2, 3), (3, 4), (4, 5)]
    assert streamed.chunk_bounds(seg, 1000) == [(0, 5)]
    seg = np.array([0, 0, 3, 3], np.int64)  # empty segments ride along
    assert streamed.chunk_bounds(seg, 3) == [(0, 3)]
    assert streamed.chunk_bounds(seg, 2) == [(0, 1), (1, 2), (2, 3)]


def test_replica_values_and_ranges():
    seed = 0x1234ABCD5678EF01
    T, U, R, G = workloads.streamed_rows(seed, np.arange(50000), 304)
    assert set(np.unique(T)) == set(range(64, 1025, 64))
    assert set(np.unique(U)) == set(range(1, 9))
    assert set(np.unique(R)) == set(range(16, 513, 16))
    assert set(np.unique(G)) == {304, 608, 1216, 2432}
    # counter-based: any row can be recomputed on its own
    T2, U2, R2, G2 = workloads.streamed_rows(seed, np.array([49999, 7]), 304)
    assert T2.tolist() == [T[49999], T[7]] and G2.tolist() == [G[49999], G[7]]
    # the finaliser is a bijection of the state: distinct positions differ
    u = workloads.splitmix64_at(seed, np.arange(1 << 16))
    assert np.unique(u).size == 1 << 16


def test_c4_recipe():
    b = workloads.c4()
    assert b.n_var == 100000
    sizes = b.seg[1:] - b.seg[:-1]
    assert sizes.min() >= 256 and sizes.max() <= 1 << 20
    assert 1.2e10 < b.n_evals < 1.35e10
    sub = b.subset([3, 99999])
    assert sub.n_evals == sizes[3] + sizes[99999]


def test_generator_reference_sequence(golden):
    """The counter-based reading of SplitMix64 (output k = state after k + 1
    steps, finalised) reproduces the generator's published sequence."""
    g = golden("splitmix64.json")
    got = workloads.splitmix64_at(g["state"], np.arange(len(g["outputs"])))
    assert [int(x) for x in got] == g["outputs"]
