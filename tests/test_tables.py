"""Scoring-table pins: the BLOSUM62 entered by hand and its background frequencies."""
import numpy as np
from scipy.optimize import brentq

from paper_1704_00878_amd import synth


def test_blosum62_shape_symmetry():
    B = synth.BLOSUM62.astype(int)
    assert B.shape == (24, 24)
    assert (B == B.T).all()


def test_blosum62_published_diagonal():
    # Diagonal of BLOSUM62 as printed by Henikoff & Henikoff (1992).
    diag = dict(A=4, R=5, N=6, D=6, C=9, Q=5, E=5, G=6, H=8, I=4, L=4, K=5, M=5, F=6, P=7,
                S=4, T=5, W=11, Y=7, V=4, B=4, Z=4, X=-1)
    for a, v in diag.items():
        k = synth.ALPHABET.index(a)
        assert synth.BLOSUM62[k, k] == v, a
    assert synth.BLOSUM62[23, 23] == 1
    assert (synth.BLOSUM62[23, :23] == -4).all()


def test_blosum62_diag_dominates():
    # min diagonal 4 > max off-diagonal 3 over the 20 standard residues: this is
    # what makes SW(c, c) the identity alignment with score sum(diag).
    B = synth.BLOSUM62[:20, :20].astype(int)
    off = B[~np.eye(20, dtype=bool)]
    assert np.diag(B).min() == 4 and off.max() == 3
    # S(x, y) <= (S(x,x) + S(y,y)) / 2 for all standard pairs
    d = np.diag(B)
    assert (2 * B <= d[:, None] + d[None, :]).all()


def test_background_and_karlin_altschul():
    p = synth.BACKGROUND
    assert abs(p.sum() - 1.0) < 1e-12 and (p > 0).all()
    B = synth.BLOSUM62[:20, :20].astype(float)
    expected = float(p @ B @ p)
    assert expected < 0  # local alignment statistics need a negative expected score
    lam = brentq(lambda x: float(p @ np.exp(x * B) @ p) - 1.0, 0.05, 2.0)
    # Published ungapped lambda of BLOSUM62 is 0.3176 nats (with slightly different
    # background frequencies); a mistyped entry of more than a few units moves it.
    assert 0.31 < lam < 0.33, lam


def test_encode_decode():
    codes = synth.encode("ARNDCQEGHILKMFPSTWYVBZX*uoJ")
    assert list(codes[:24]) == list(range(24))
    assert codes[24] == synth.ALPHABET.index("C")
    assert codes[25] == synth.ALPHABET.index("K")
    assert codes[26] == synth.ALPHABET.index("X")
    assert synth.decode([0, 255, 17]) == "A-W"


def test_oracle_encode_hand_codes():
    """The oracle's encoding against codes written out by hand from the NCBI
    order A R N D C Q E G H I L K M F P S T W Y V B Z X * (0..23)."""
    import oracle
    oracle.build(force=False)
    got = oracle.encode("MKTAYIAKQR")
    assert list(got) == [12, 11, 16, 0, 18, 9, 0, 11, 5, 1]
    got = oracle.encode("wyv*bzx")                    # lower case and the last letters
    assert list(got) == [17, 18, 19, 23, 20, 21, 22]
    got = oracle.encode("UuOo")                        # U -> C (4), O -> K (11)
    assert list(got) == [4, 4, 11, 11]
    got = oracle.encode(b"J-1 \x00\xff.")              # everything else -> X (22)
    assert list(got) == [22] * 7
    assert list(oracle.encode(b"")) == []
    ascii7 = bytes(range(128))
    assert (oracle.encode(ascii7) == synth.encode(ascii7.decode("ascii"))).all()
    assert (oracle.encode(bytes(range(128, 256))) == 22).all()


def test_generator_deterministic_and_shaped():
    a = synth.generate("plain64")
    b = synth.generate("plain64")
    assert (a.residues == b.residues).all() and (a.offsets == b.offsets).all()
    assert a.n == 64 and a.residues.max() < 20
    L = a.lengths()
    assert 60 <= L.min() and L.max() <= 200
