"""Group tiling of the exhaustive center (host only; no GPU needed): every
pair a < b of n positions lies in exactly one group, the group count is the
closed form, and planning a million sequences takes no O(n^2) host memory."""
import resource

import numpy as np
import pytest


@pytest.fixture(scope="module")
def H():
    import os
    import paper_1704_00878_amd as H
    if not os.path.exists(H.LIB_PATH):
        pytest.skip("library not built")
    H.lib()
    return H


@pytest.mark.parametrize("step", [64, 128])
@pytest.mark.parametrize("n", [0, 1, 2, 3, 63, 64, 65, 127, 128, 129, 200, 257, 300])
def test_every_pair_once(H, n, step):
    ng = H.halign_exact_tiling(n, step)
    seen = np.zeros((max(n, 1), max(n, 1)), np.int32)
    for g in range(ng):
        _, a, b0 = H.halign_exact_tiling(n, step, g)
        assert 0 <= a < n and b0 % step == 0 and b0 < n
        b = np.arange(b0, min(b0 + step, n))
        b = b[b > a]
        assert len(b) > 0, (g, a, b0)       # no group is idle
        seen[a, b] += 1
    iu = np.triu_indices(n, 1)
    assert (seen[iu] == 1).all()
    assert seen.sum() == n * (n - 1) // 2


def test_groups_in_closed_form_at_a_million(H):
    """n = 1e6: about 3.9e9 groups (more than 2^31), decoded without any
    per-group host data; the process's peak memory does not grow."""
    before = resource.getrusage(resource.RUSAGE_SELF).ru_maxrss
    n, step = 1_000_000, 128
    ng = H.halign_exact_tiling(n, step)
    q = (n + step - 1) // step
    assert ng == step * (q - 1) * q // 2 - (q - 1) + n - 1
    assert ng > 2 ** 31
    rng = np.random.default_rng(0)
    for g in [0, 1, ng - 1, ng - 2] + list(rng.integers(0, ng, 2000)):
        _, a, b0 = H.halign_exact_tiling(n, step, int(g))
        blk = b0 // step
        first = step * blk * (blk + 1) // 2 - blk
        assert a == g - first and 0 <= a < min(b0 + step, n) - 1
    after = resource.getrusage(resource.RUSAGE_SELF).ru_maxrss
    assert after - before < 64 * 1024   # KiB: far below the ~31 GB of a per-group list


def test_out_of_range_group_is_rejected(H):
    ng = H.halign_exact_tiling(100, 64)
    with pytest.raises(H.HalignError):
        H.halign_exact_tiling(100, 64, ng)
