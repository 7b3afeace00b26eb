"""Host rules of the shipped smoother weights: the per-request weight-set
selection used by the serving benchmark, and the consistency of each
weight file with the network it declares (no GPU needed)."""
import os

import numpy as np
import pytest

from paper_2603_01064_amd.train_weights import load_weights, select_set

WDIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2603_01064_amd", "weights")


def test_select_set_takes_smallest_trained_alpha_at_least_half():
    al = [1e-2, 1e-3, 1e-4, 1e-5]
    assert select_set(al, 1e-2) == 0
    assert select_set(al, 2e-2) == 0      # 1e-2 >= 2e-2 / 2
    assert select_set(al, 3e-2) == 0      # no set reaches 1.5e-2: the largest alpha
    assert select_set(al, 1.9e-3) == 1    # 1e-3 >= 9.5e-4
    assert select_set(al, 2.1e-3) == 0    # 1e-3 < 1.05e-3, so the next larger set
    assert select_set(al, 1e-6) == 3      # below every set: the smallest alpha
    assert select_set([1e-4, 1e-2, 1e-3], 1e-3) == 2  # indices, not positions in a sorted list


@pytest.mark.parametrize("name", sorted(f for f in os.listdir(WDIR) if f.endswith(".npz")))
def test_weight_file_matches_declared_network(name):
    meta, sets = load_weights(os.path.join(WDIR, name))
    ch, ks = meta["channels"], meta["ksize"]
    count = sum(ch[i] * ch[i + 1] * ks ** meta.get("dim", 2) for i in range(len(ch) - 1))
    assert ch[0] == 1 and ch[-1] == 1
    assert len(sets) == len(meta["alphas"]) >= 1
    for lv in sets:
        assert len(lv) == meta["levels"] - 1  # one smoother per level above the coarsest
        for w in lv:
            assert w.dtype == np.float32 and w.shape == (count,) and np.isfinite(w).all()
