"""The seeded input generators: the laws they promise and the input order they promise.
CPU only (torch on the CPU for the batched generator)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from datagen.batched import make_batch, zipf_ranks  # noqa: E402


@pytest.mark.parametrize("n,s", [(10, 1.1), (7, 0.5), (50, 1.0), (5, 1.5), (3, 1e-4), (2, 3.0)])
def test_zipf_rejection_inversion_matches_pmf(n, s):
    g = torch.Generator()
    g.manual_seed(7)
    N = 200_000
    k = zipf_ranks(n, s, N, g, "cpu", torch).numpy()
    assert k.min() >= 0 and k.max() < n
    f = np.bincount(k, minlength=n) / N
    p = np.arange(1, n + 1, dtype=np.float64) ** -s
    p /= p.sum()
    # five standard deviations of a binomial frequency
    assert np.all(np.abs(f - p) <= 5 * np.sqrt(p * (1 - p) / N) + 1e-12)


def test_batch_is_seeded_sorted_and_in_range():
    A = make_batch(24, seed=11, orders=(2, 3, 4, 5), nnz_range=(1, 5e3), ext_range=(1, 1e5))
    B = make_batch(24, seed=11, orders=(2, 3, 4, 5), nnz_range=(1, 5e3), ext_range=(1, 1e5))
    for a, b in zip(A, B):
        assert a.extents == b.extents and a.in_order == b.in_order and a.out_order == b.out_order
        for x, y in zip(a.crd, b.crd):
            assert torch.equal(x, y)
        assert torch.equal(a.val, b.val)
        crd = [c.numpy().astype(np.int64) for c in a.crd]
        for m, c in enumerate(crd):
            assert c.min(initial=0) >= 0 and c.max(initial=0) < a.extents[m]
        # lexicographic order of the input order
        if a.nnz > 1:
            keys = np.stack([crd[m] for m in a.in_order])
            order = np.lexsort(keys[::-1])
            assert np.array_equal(keys[:, order], keys)
        assert a.val.dtype == torch.float64 and a.crd[0].dtype == torch.int32
        assert float(a.val.abs().max()) <= 1.0 if a.nnz else True
