"""Host-side FNO weight layout: the packed block has the size the library
expects for 1D and 2D problems, in the documented order."""
import numpy as np

from paper_2603_01064_amd import inputs
from paper_2603_01064_amd.fno import pack_fno_weights
from paper_2603_01064_amd.nmg import Problem


def test_packed_size_matches_problem():
    for dim, arch in ((2, (8, 2, 8, 3)), (1, (6, 3, 16, 5)), (2, (64, 5, 32, 5))):
        C, NL, m, ks = arch
        p = inputs.fno_params(dim, C, NL, m, ks, 1)
        flat = pack_fno_weights(p)
        assert flat.dtype == np.float32
        assert flat.size == Problem(n=63, s=0.04, levels=3, dim=dim, fno=arch).weight_count()


def test_packed_order():
    p = inputs.fno_params(2, 2, 1, 2, 3, 2)
    flat = pack_fno_weights(p)
    C, RM = 2, 2 * 2 * 2 * 2 * 2
    assert np.array_equal(flat[:C], p["lift_w"].astype(np.float32))
    assert np.array_equal(flat[C:2 * C], p["lift_b"].astype(np.float32))
    o = 2 * C
    assert np.array_equal(flat[o:o + RM], p["layers"][0]["R_re"].reshape(-1).astype(np.float32))
    assert np.array_equal(flat[o + RM:o + 2 * RM], p["layers"][0]["R_im"].reshape(-1).astype(np.float32))
    o += 2 * RM
    assert np.array_equal(flat[o:o + C * C * 9], p["layers"][0]["W"].reshape(-1).astype(np.float32))
    assert np.array_equal(flat[-C - 1:-1], p["proj_w"].astype(np.float32))
    assert flat[-1] == np.float32(p["proj_b"])
