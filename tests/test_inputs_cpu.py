"""The seeded input generators: reproducible, per-tensor streams (runs without a GPU)."""
import numpy as np

from paper_1912_10024_amd.inputs import CONFIGS, STREAMS, generate, make_nbr


def test_generate_is_reproducible_and_per_tensor():
    d = CONFIGS["tiny"]
    a = generate(d, 0, which=STREAMS)
    b = generate(d, 0, which=("dH", "G<"))
    for name in ("dH", "G<"):
        assert np.array_equal(a[name], b[name])          # a tensor does not depend on which others are drawn
    c = generate(d, 1, which=("G<",))
    assert not np.array_equal(a["G<"], c["G<"])          # the config index changes the stream
    assert not np.array_equal(a["G<"], a["G>"])          # the two components are independent draws


def test_distributions_and_structure():
    d = CONFIGS["tiny"]
    x = generate(d, 0, which=("G<", "dH", "nbr"))
    G = x["G<"]
    assert np.allclose(G, -np.conj(np.swapaxes(G, -1, -2)))   # anti-Hermitian blocks
    nbr = x["nbr"]
    assert nbr.dtype == np.int32 and nbr.shape == (d.na, d.nb)
    for a in range(d.na):
        assert a not in nbr[a] and len(set(nbr[a])) == d.nb  # distinct neighbours, no self-loop
    assert 0.05 < np.std(x["dH"].real) < 0.2                  # N(0, 0.1^2) parts


def test_make_nbr_rejects_too_many_neighbours():
    import pytest
    with pytest.raises(ValueError):
        make_nbr(np.random.default_rng(0), 4, 4)
