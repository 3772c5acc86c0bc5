"""Host-side logic of the Algorithm 1 driver that needs no GPU (CPU)."""

import pytest

from paper_2412_17617_amd.tree_search import TreeSearch


def test_tree_search_rejects_bad_depths():
    with pytest.raises(ValueError):
        TreeSearch(object(), 2, 16, d_init=3, d_max=2)
    with pytest.raises(ValueError):
        TreeSearch(object(), 2, 16, d_init=1, d_max=3, m_of_depth=(10, 3))


def test_low_rank_tree_search_stays_switched_off():
    # its only GPU run faulted with no cause shown: the option must refuse
    with pytest.raises(NotImplementedError):
        TreeSearch(object(), 2, 16, lowrank=True)
