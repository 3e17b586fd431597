"""The entry point that allocates nothing (qz_corr_noalloc): the same sums as
qz_corr on consecutive calls, the second and third on smaller lattices (the
library's static scratch keeps the previous call's contents until cleared)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qz():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_12161_amd import binding
    return binding


def test_corr_noalloc_matches_corr(qz):
    cases = [(256, "bit", 20), (128, "bit", 7), (32, "i8", 5), (1024, "bit", 3)]
    for L, layout, n in cases:
        print("corr_noalloc", L, layout, n, flush=True)
        lat = qz.Lattice(L, 900 + L, layout)
        lat.run(n)
        S1, M1 = lat.corr_noalloc()
        S0, M0 = lat.corr()
        assert M1 == M0 and np.array_equal(S1, S0), (L, layout)
        # again on the same state: the previous sums were cleared
        S2, M2 = lat.corr_noalloc()
        assert M2 == M0 and np.array_equal(S2, S0), (L, layout)
        del lat
