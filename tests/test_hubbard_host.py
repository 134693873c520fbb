"""Host-side check of the library's Hubbard operators (Kronecker products of
local dot operators with parity strings) against the oracle's (built entry by
entry from occupation bits): the two constructions agree exactly."""
import numpy as np

from oracle import hubbard as hu
from paper_2511_13330_amd.hubbard import hubbard_operators


def test_library_hubbard_operators_match_oracle():
    for n_dots in (1, 2, 3):
        hs, hc, lj = hubbard_operators(n_dots, 1000.0, 2.0)
        assert np.array_equal(hs, np.array(hu.static_terms(n_dots)))
        if n_dots > 1:
            assert np.array_equal(hc, np.array(hu.hopping_terms(n_dots)))
        assert np.array_equal(lj, np.array(hu.jump_ops(n_dots, 1000.0, 2.0)))
