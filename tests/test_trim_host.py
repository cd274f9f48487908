"""The library's trimmed layout (host code, no GPU) against the oracle's
enumeration of the bins the reconstruction path reads (Section 2.3)."""
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mj():
    import paper_1504_07038_amd as mj

    mj.lib()
    return mj


@pytest.mark.parametrize("n,Q,P", [(6, 4, 128), (12, 8, 128), (6, 3, 256), (12, 4, 64),
                                   (8, 4, 32), (16, 12, 16), (3, 3, 5), (2, 1, 9)])
def test_trimmed_layout_matches_the_oracle_enumeration(mj, n, Q, P):
    ps = synth.centered_dirs(n)
    words, keep = mj.mojette_trimmed_layout(ps, P, Q)
    assert keep == oracle.kept_bins(ps, P, Q)
    assert words == sum(c for _, c in keep)


def test_trimmed_layout_in_any_direction_order(mj):
    ps = [2, -3, 0, 1, -1, -2]
    words, keep = mj.mojette_trimmed_layout(ps, 128, 4)
    assert words == 773
    assert keep == oracle.kept_bins(ps, 128, 4)


def test_trimmed_layout_argument_errors(mj):
    with pytest.raises(mj.MojetteError):
        mj.mojette_trimmed_layout([0, 1], 16, 3)      # n < Q
    with pytest.raises(mj.MojetteError):
        mj.mojette_trimmed_layout([1, 1, 2], 16, 2)   # repeated direction
