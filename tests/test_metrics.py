"""The sample count of the benchmark (number of nonzero strip-area weights of A(theta)) against
its definition: the nonzeros of the dense matrix built by polygon clipping, and the device
counter against the host counter (CPU only)."""
import numpy as np
import pytest

from paper_2605_06336_amd import metrics, synth
from tests import brute


@pytest.mark.parametrize("N,nb,V", [(6, 9, 7), (8, 11, 5)])
def test_nnz_matches_clipped_areas(N, nb, V):
    th = np.concatenate([synth.random_angles(V - 3, 11), [0.0, np.pi / 4, np.pi / 2]])
    A = brute.dense_matrix(N, nb, th)
    # areas below 1e-14 are clipping round-off on shared pixel edges, not overlaps
    assert metrics.nnz(N, nb, th) == int(np.sum(A > 1e-14))


def test_nnz_torch_equals_host_count():
    torch = pytest.importorskip("torch")
    th = synth.random_angles(41, 7)
    for N, nb in ((64, 91), (37, 52)):
        assert metrics.nnz_torch(torch, N, nb, th) == metrics.nnz(N, nb, th)
