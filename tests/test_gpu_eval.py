"""MSA evaluation on the GPU: the column profile (per-column residue and gap
counts, from which the Results section's avg SP follows) and both SP scores
computed from it, against the oracle."""
import numpy as np
import pytest

import oracle
from paper_1704_00878_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import paper_1704_00878_amd as H
    return H


def _rand_msa(rng, n, w, alpha=24, gap=0.3):
    a = rng.integers(0, alpha, (n, w)).astype(np.uint8)
    a[rng.random((n, w)) < gap] = 255
    return a


@pytest.mark.parametrize("n,w", [(37, 91), (3000, 2500), (1, 1), (5, 1025), (0, 10), (4, 0)])
def test_column_profile(H, n, w):
    import torch
    a = _rand_msa(np.random.default_rng(n * 7 + w), n, w)
    got = H.halign_column_profile(torch.from_numpy(a).cuda()).cpu().numpy()
    assert got.shape == (w, 25)
    assert (got == oracle.column_profile(a, 24)).all()


@pytest.mark.parametrize("slab", ["5", "65535"])
def test_column_profile_slabs(H, slab, monkeypatch):
    """Rows in slabs of 5 (many partial profiles added up) and of 65,535 (a
    16-bit LDS count at its maximum next to its neighbour's half word)."""
    import torch
    monkeypatch.setenv("HALIGN_PROFILE_SLAB", slab)
    rng = np.random.default_rng(5)
    n = 65535 + 7 if slab == "65535" else 301
    a = _rand_msa(rng, n, 1030, alpha=20)
    a[:, 0] = 5          # one residue filling a column (counted in the low half of its word)
    a[:, 256] = 255      # a column of gaps (same word, high half)
    a[:, 1029] = 19
    got = H.halign_column_profile(torch.from_numpy(a).cuda(), alphabet=20).cpu().numpy()
    want = oracle.column_profile(a, 20)
    assert want[0, 5] == n and want[256, 20] == n
    assert (got == want).all()


def test_column_profile_million_rows(H):
    """1e6 rows: the size of the largest MSA workload."""
    import torch
    n, w = 1_000_000, 300
    g = torch.Generator(device="cuda").manual_seed(11)
    d = torch.randint(0, 25, (n, w), dtype=torch.uint8, device="cuda", generator=g)
    d[d == 24] = 255
    got = H.halign_column_profile(d).cpu().numpy()
    a = d.cpu().numpy()
    assert (got == oracle.column_profile(a, 24)).all()


def test_column_profile_rejects_bad_code(H):
    import torch
    a = np.zeros((3, 40), np.uint8)
    a[2, 17] = 24        # not a code of the 24-letter alphabet, not a gap
    with pytest.raises(H.HalignError):
        H.halign_column_profile(torch.from_numpy(a).cuda())
    with pytest.raises(H.HalignError):
        H.halign_sp_score(H.Scoring(), torch.from_numpy(a).cuda())


def test_sp_score_from_profile_large(H):
    """Both SP scores at 5,000 rows: the avg SP numerator against the oracle's
    column count routine, BLOSUM SP against the pair formula over the oracle's
    profile (that formula is pinned against the explicit pair loops on the CPU)."""
    import torch
    from oracle_par import sp_from_profile
    rng = np.random.default_rng(13)
    a = _rand_msa(rng, 5000, 777)
    sp, spb = H.halign_sp_score(H.Scoring(), torch.from_numpy(a).cuda())
    assert sp == oracle.sp_columns(a)
    want_sp, want_bl = sp_from_profile(oracle.column_profile(a, 24), np.asarray(synth.BLOSUM62, np.int8), 1)
    assert sp == want_sp and spb == want_bl
